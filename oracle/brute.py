"""Pure-Python brute force for tiny levels (test infrastructure only).

A second, independent formulation of the fractal and the automaton, used to pin
the C oracle:

  * the fractal is built by the NBB construction itself (section 1): level 0
    is one cell; level rho+1 is the union of k copies of level rho translated by
    o_j * s^rho.  No digit arithmetic is involved;
  * the compact order is built alongside: the copy made from replica j at the
    step to level rho+1 places its cells after those of replicas 0..j-1, so the
    new (coarsest) replica id is the most significant base-k digit;
  * the automaton counts live neighbours over a Python set of member cells.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Set, Tuple

Cell = Tuple[int, int]


def build_levels(s: int, offsets: Sequence[Cell], r: int) -> List[Cell]:
    """Member cells in compact order: element i is the cell with compact index i."""
    cells: List[Cell] = [(0, 0)]
    for rho in range(r):
        scale = s ** rho
        nxt: List[Cell] = []
        # Replica j of the level-rho fractal; the cell order inside each copy
        # is the level-rho order, so the new replica id is the high digit.
        for (ox, oy) in offsets:
            nxt.extend((x + ox * scale, y + oy * scale) for (x, y) in cells)
        cells = nxt
    return cells


def member_set(s: int, offsets: Sequence[Cell], r: int) -> Set[Cell]:
    return set(build_levels(s, offsets, r))


NEIGHBOURS = {8: [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dx or dy],
              4: [(0, -1), (-1, 0), (1, 0), (0, 1)]}


def gol_step(members: Set[Cell], live: Set[Cell], birth: Sequence[int],
             survive: Sequence[int], neighbourhood: int = 8) -> Set[Cell]:
    """One synchronous generation on the member cells; everything else is
    dead.  neighbourhood 8 = Moore, 4 = the cells sharing an edge."""
    out: Set[Cell] = set()
    for (x, y) in members:
        c = 0
        for dx, dy in NEIGHBOURS[neighbourhood]:
            if (x + dx, y + dy) in live:
                c += 1
        if (x, y) in live:
            if c in survive:
                out.add((x, y))
        elif c in birth:
            out.add((x, y))
    return out


def run_compact(s: int, offsets: Sequence[Cell], r: int, state: Sequence[int],
                birth: Sequence[int], survive: Sequence[int], steps: int,
                neighbourhood: int = 8) -> List[int]:
    """Evolve a compact-order state (list of 0/1) for `steps` generations."""
    order = build_levels(s, offsets, r)
    members = set(order)
    live = {c for c, v in zip(order, state) if v}
    for _ in range(steps):
        live = gol_step(members, live, birth, survive, neighbourhood)
    return [1 if c in live else 0 for c in order]
