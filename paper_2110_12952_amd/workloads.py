"""Fractal definitions, workload sizes and seeded input generators.

This module is shared by the tests, the benchmark and the code that drives the
oracle.  It holds *inputs only*: replica offset lists, level/seed/probability
choices and seeded random arrays.  None of the method's arithmetic (membership,
the lambda/nu maps, the automaton, the initial-state generator) lives here.

Replica offsets are (x, y) digit pairs in [0, s)^2, x to the right, y downwards,
origin top-left (paper section 3).  The list order is the replica numbering that
the compact index uses (section 3.1: the replica id of H must agree with the
numbering used by lambda).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

Offsets = Tuple[Tuple[int, int], ...]


@dataclass(frozen=True)
class FractalDef:
    """An NBB fractal F^{k,s}: k replicas, growth ratio s (section 1)."""
    name: str
    s: int
    offsets: Offsets

    @property
    def k(self) -> int:
        return len(self.offsets)

    def flat_offsets(self) -> List[int]:
        out: List[int] = []
        for ox, oy in self.offsets:
            out += [int(ox), int(oy)]
        return out


# Sierpinski triangle F^{3,2}: the paper's case study (section 4.1).
TRIANGLE = FractalDef("triangle", 2, ((0, 0), (1, 0), (0, 1)))
# Sierpinski carpet F^{8,3}: the 3x3 grid without its centre, row-major order.
CARPET = FractalDef("carpet", 3, ((0, 0), (1, 0), (2, 0), (0, 1), (2, 1),
                                  (0, 2), (1, 2), (2, 2)))
# H-fractal F^{7,3}: both full columns plus the centre.
HFRACTAL = FractalDef("hfractal", 3, ((0, 0), (0, 1), (0, 2), (1, 1),
                                      (2, 0), (2, 1), (2, 2)))
# Chandelier-like F^{4,3}: top row plus the centre.
CHANDELIER = FractalDef("chandelier", 3, ((0, 0), (1, 0), (2, 0), (1, 1)))
# Full square F^{4,2}: every cell of the box is a member; the compact order is
# then the Z-order (Morton) curve and the automaton is plain Game of Life.
FULLSQUARE = FractalDef("fullsquare", 2, ((0, 0), (1, 0), (0, 1), (1, 1)))
# Textbook fractals of the same class, used as extra test fractals.
VICSEK = FractalDef("vicsek", 3, ((1, 0), (0, 1), (1, 1), (2, 1), (1, 2)))
XFRACTAL = FractalDef("xfractal", 3, ((0, 0), (2, 0), (1, 1), (0, 2), (2, 2)))
CANTOR_DUST = FractalDef("cantordust", 3, ((0, 0), (2, 0), (0, 2), (2, 2)))
# Cantor set F^{2,3} laid on the first row of its box (Table 1 lists F^{2,3}).
CANTOR = FractalDef("cantor", 3, ((0, 0), (2, 0)))
# A fractal with a single replica: one cell at every level.
SINGLE = FractalDef("single", 2, ((1, 1),))
# s = 4 with 12 replicas in a scrambled order (not one of the paper's pictures).
GRID4 = FractalDef("grid4_12", 4, ((0, 0), (1, 0), (3, 0), (0, 1), (1, 1),
                                   (3, 1), (0, 3), (1, 3), (2, 2), (3, 3),
                                   (2, 3), (3, 2)))

FRACTALS: Dict[str, FractalDef] = {
    f.name: f for f in (TRIANGLE, CARPET, HFRACTAL, CHANDELIER, FULLSQUARE,
                        VICSEK, XFRACTAL, CANTOR_DUST, CANTOR, SINGLE, GRID4)
}

# Game-of-Life rules as (birth counts, survival counts[, neighbourhood]):
# neighbourhood 8 (default) = the Moore neighbourhood, 4 = the four cells
# that share an edge.
RULES = {
    "B3/S23": ((3,), (2, 3)),             # Conway's Game of Life
    "B1357/S1357": ((1, 3, 5, 7), (1, 3, 5, 7)),    # replicator (XOR of neighbours)
    "B1357/S02468": ((1, 3, 5, 7), (0, 2, 4, 6, 8)),  # Fredkin (self XOR neighbours)
    "B36/S23": ((3, 6), (2, 3)),          # HighLife
    "B2/S": ((2,), ()),                   # Seeds
    "B35/S0123456": ((3, 5), (0, 1, 2, 3, 4, 5, 6)),  # every survival count below 7 (table edge cases)
    "vN:B13/S13": ((1, 3), (1, 3), 4),    # 4-neighbour parity (XOR of the four)
    "vN:B13/S024": ((1, 3), (0, 2, 4), 4),  # 4-neighbour Fredkin (self XOR the four)
    "vN:B2/S12": ((2,), (1, 2), 4),       # a 4-neighbour life-like rule
}

VON_NEUMANN = 1 << 31  # rule-word flag: count the four edge neighbours only


def rule_mask(name_or_pair) -> int:
    """Rule word: bit c (0..8) = birth with c live neighbours, bit 16+c =
    survival, bit 31 = four-cell neighbourhood."""
    spec = RULES[name_or_pair] if isinstance(name_or_pair, str) else name_or_pair
    birth, survive = spec[0], spec[1]
    m = VON_NEUMANN if len(spec) > 2 and spec[2] == 4 else 0
    for c in birth:
        m |= 1 << c
    for c in survive:
        m |= 1 << (16 + c)
    return m


def rule_neighbourhood(name_or_pair) -> int:
    spec = RULES[name_or_pair] if isinstance(name_or_pair, str) else name_or_pair
    return spec[2] if len(spec) > 2 else 8


@dataclass(frozen=True)
class Workload:
    """One synthetic automaton run: fractal, level, Bernoulli(p) seed, steps."""
    name: str
    fractal: FractalDef
    r: int
    p: float
    seeds: Tuple[int, ...]
    steps: int
    rule: str = "B3/S23"

    @property
    def n(self) -> int:
        return self.fractal.s ** self.r

    @property
    def cells(self) -> int:
        return self.fractal.k ** self.r


# The workloads of the paper's case study and of the wider evaluation plan.
SMALL_TRIANGLE = Workload("triangle_r10", TRIANGLE, 10, 0.5, (1, 2, 3), 100)
LARGE_TRIANGLE = Workload("triangle_r16", TRIANGLE, 16, 0.3, (12952,), 1000)
CARPET_R9 = Workload("carpet_r9", CARPET, 9, 0.5, (12952,), 200)
HFRACTAL_R10 = Workload("hfractal_r10", HFRACTAL, 10, 0.5, (12952,), 200)

WORKLOADS: Dict[str, Workload] = {
    w.name: w for w in (SMALL_TRIANGLE, LARGE_TRIANGLE, CARPET_R9, HFRACTAL_R10)
}


# Batched workload: 512 independent instances stepped together for 500
# generations.  Each instance draws its fractal uniformly from four types and
# its level uniformly from the levels of that type with k^r in [1e3, 1e7];
# Bernoulli p uniform in [0.2, 0.6]; instance i is initialised from seed i.
BATCH_LEVELS = {"triangle": tuple(range(7, 15)), "carpet": tuple(range(4, 8)),
                "hfractal": tuple(range(4, 9)), "chandelier": tuple(range(5, 12))}


@dataclass(frozen=True)
class BatchItem:
    fractal: FractalDef
    r: int
    p: float
    seed: int

    @property
    def cells(self) -> int:
        return self.fractal.k ** self.r


@dataclass(frozen=True)
class BatchWorkload:
    name: str
    count: int
    steps: int
    draw_seed: int
    levels: Tuple[Tuple[str, Tuple[int, ...]], ...]
    p_range: Tuple[float, float] = (0.2, 0.6)
    rule: str = "B3/S23"

    def items(self) -> List[BatchItem]:
        rng = np.random.default_rng(self.draw_seed)
        out = []
        for i in range(self.count):
            name, lv = self.levels[int(rng.integers(len(self.levels)))]
            r = int(lv[int(rng.integers(len(lv)))])
            p = float(rng.uniform(*self.p_range))
            out.append(BatchItem(FRACTALS[name], r, p, i))
        return out


BATCH512 = BatchWorkload("batch512", 512, 500, 2110, tuple(BATCH_LEVELS.items()))


# Served workload: requests arrive as a Poisson process; each asks for one
# automaton run on a fresh Bernoulli(p) state.  The fractal is uniform over
# `fractals`; log10 of the cell count is uniform in [3, 8] and snapped to the
# nearest level the fractal has among `levels`; the step count is
# log-uniform in [10, 2000].
SERVE_LEVELS = {"carpet": tuple(range(4, 9)), "hfractal": tuple(range(4, 10)),
                "triangle": tuple(range(7, 17)), "chandelier": tuple(range(5, 14))}


@dataclass(frozen=True)
class Request:
    rid: int
    t: float            # arrival time, seconds from the start
    fractal: FractalDef
    r: int
    steps: int
    p: float
    seed: int

    @property
    def cells(self) -> int:
        return self.fractal.k ** self.r


@dataclass(frozen=True)
class ServeWorkload:
    name: str
    rate: float                      # mean arrivals per second
    seconds: float                   # arrival window
    fractals: Tuple[str, ...]
    draw_seed: int
    log10_cells: Tuple[float, float] = (3.0, 8.0)
    steps: Tuple[int, int] = (10, 2000)
    p: float = 0.5
    rule: str = "B3/S23"

    def requests(self, seconds: float = None) -> List[Request]:
        seconds = self.seconds if seconds is None else seconds
        rng = np.random.default_rng(self.draw_seed)
        out, t, rid = [], 0.0, 0
        while True:
            t += float(rng.exponential(1.0 / self.rate))
            if t >= seconds:
                return out
            fd = FRACTALS[self.fractals[int(rng.integers(len(self.fractals)))]]
            u = float(rng.uniform(*self.log10_cells))
            levels = SERVE_LEVELS[fd.name]
            r = min(levels, key=lambda lv: abs(lv * np.log10(fd.k) - u))
            lo, hi = np.log(self.steps[0]), np.log(self.steps[1])
            steps = int(round(float(np.exp(rng.uniform(lo, hi)))))
            out.append(Request(rid, t, fd, int(r), steps, self.p, rid))
            rid += 1


SERVE2000 = ServeWorkload("serve2000", 2000.0, 60.0, ("carpet", "hfractal"), 5)


def random_offsets(rng: np.random.Generator, s: int, k: int) -> Offsets:
    """k distinct digit pairs in [0,s)^2 in random order (a random NBB fractal)."""
    cells = rng.choice(s * s, size=k, replace=False)
    return tuple((int(c % s), int(c // s)) for c in cells)


def random_fractal(seed: int, s_choices: Sequence[int] = (2, 3, 4)) -> FractalDef:
    rng = np.random.default_rng(seed)
    s = int(rng.choice(list(s_choices)))
    k = int(rng.integers(1, s * s + 1))
    return FractalDef(f"random{seed}", s, random_offsets(rng, s, k))


def random_coords(seed: int, count: int, lo: int, hi: int) -> Tuple[np.ndarray, np.ndarray]:
    """count (x, y) pairs uniform in [lo, hi)^2, int32."""
    rng = np.random.default_rng(seed)
    x = rng.integers(lo, hi, size=count, dtype=np.int64).astype(np.int32)
    y = rng.integers(lo, hi, size=count, dtype=np.int64).astype(np.int32)
    return x, y


def random_indices(seed: int, count: int, hi: int) -> np.ndarray:
    """count uint32 indices uniform in [0, hi)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, hi, size=count, dtype=np.int64).astype(np.uint32)


def random_bits(seed: int, count: int, p: float = 0.5) -> np.ndarray:
    """count uint8 values in {0,1}, each 1 with probability p."""
    rng = np.random.default_rng(seed)
    return (rng.random(count) < p).astype(np.uint8)
