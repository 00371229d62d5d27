"""Request loop: automaton runs served from states resident in HBM.

Requests (fractal, level r, step count, Bernoulli p, seed) arrive over time.
An admitted request gets a slot in a device arena (two arenas, the states
alternate between them each generation), is initialised there by the
library's init kernel, and is stepped together with every other admitted
request by the batched step: each round runs up to G generations of all
active requests with one batched call, and a request leaves the batch at
exactly its own step count (per-instance step counts, instances listed by
decreasing remaining steps).  Every generation runs in the library's HIP
kernels; this module only schedules.

Admission (the service is offered more work than the GPU can do).  Every
generation of the batch costs time in proportion to the cells of all active
requests (their footprint C), so at throughput T (cell updates per second,
measured) request j, with R_j generations left, finishes about R_j C / T
from now.  A request is admitted only if
  - its state fits the arena now, and
  - with its cells added to C, every active request and itself still finish
    within `deadline_s` of their arrival:  C' <= T min_j(slack_j / R_j), with
    slack_j the time left before request j's deadline (arrival + deadline_s).
A request that fails either test is rejected at once, with the reason; the
latency percentiles cover completed requests only and are reported beside
the fraction rejected.

The device work goes through an executor (`DeviceExecutor`: the library's
kernels on the current GPU); the loop itself only schedules, so another
executor with the same four methods can stand in for it (the CPU tests run
the loop on one that steps the states on the host).
"""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import nbbfrac as N


class ArenaAllocator:
    """First-fit allocator of 16-byte-aligned ranges in [0, capacity)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity) & ~15
        self._free: List[Tuple[int, int]] = [(0, self.capacity)] if self.capacity else []  # (start, size), sorted
        self._used: Dict[int, int] = {}

    @property
    def used_bytes(self) -> int:
        return sum(self._used.values())

    def alloc(self, nbytes: int) -> Optional[int]:
        size = max(16, (int(nbytes) + 15) & ~15)
        for j, (start, avail) in enumerate(self._free):
            if avail >= size:
                if avail == size:
                    self._free.pop(j)
                else:
                    self._free[j] = (start + size, avail - size)
                self._used[start] = size
                return start
        return None

    def free(self, offset: int) -> None:
        size = self._used.pop(offset)
        j = bisect.bisect_left(self._free, (offset, 0))
        self._free.insert(j, (offset, size))
        # merge with the neighbours
        if j + 1 < len(self._free) and offset + size == self._free[j + 1][0]:
            self._free[j] = (offset, size + self._free[j + 1][1])
            self._free.pop(j + 1)
        if j > 0 and self._free[j - 1][0] + self._free[j - 1][1] == self._free[j][0]:
            self._free[j - 1] = (self._free[j - 1][0], self._free[j - 1][1] + self._free[j][1])
            self._free.pop(j)

    def check(self) -> None:
        """Invariants: free and used ranges tile [0, capacity) without overlap."""
        spans = sorted(list(self._free) + list(self._used.items()))
        pos = 0
        for start, size in spans:
            assert start == pos and size > 0, (start, pos)
            pos += size
        assert pos == self.capacity
        for (a, sa), (b, _) in zip(self._free, self._free[1:]):
            assert a + sa < b  # free neighbours are merged


def plan_round(remaining: Sequence[int], cells: Sequence[int], gen_budget_cells: float,
               max_gens: int) -> Tuple[List[int], int]:
    """Order and length of one round.  Returns (order, G): the active requests
    by decreasing remaining steps, and the number of generations G, chosen so
    that G generations of all of them cost about gen_budget_cells cell
    updates (at least 1, at most max_gens and the largest remaining count)."""
    order = sorted(range(len(remaining)), key=lambda j: -remaining[j])
    total = sum(cells)
    G = int(gen_budget_cells // max(total, 1))
    G = max(1, min(G, max_gens, max(remaining) if remaining else 1))
    return order, G


@dataclass
class _Active:
    req: object
    desc: object
    offset: int
    remaining: int
    admitted: float
    started: Optional[float] = None


@dataclass
class ServeStats:
    offered: int = 0
    admitted: int = 0
    completed: int = 0
    rejected_deadline: int = 0
    rejected_memory: int = 0
    rounds: int = 0
    cell_updates: int = 0
    gpu_seconds: float = 0.0
    wall_seconds: float = 0.0
    latencies: List[float] = field(default_factory=list)
    waits: List[float] = field(default_factory=list)

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        wt = np.array(self.waits) if self.waits else np.zeros(1)
        rejected = self.rejected_deadline + self.rejected_memory
        return {"offered": self.offered, "admitted": self.admitted, "completed": self.completed,
                "rejected_deadline": self.rejected_deadline, "rejected_memory": self.rejected_memory,
                "rejected_frac": rejected / max(self.offered, 1),
                "rounds": self.rounds, "cell_updates": self.cell_updates,
                "cell_updates_per_s": self.cell_updates / max(self.wall_seconds, 1e-9),
                "gpu_busy_frac": self.gpu_seconds / max(self.wall_seconds, 1e-9),
                "wall_s": self.wall_seconds,
                "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
                "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
                "latency_max_ms": float(lat.max() * 1e3),
                "wait_p50_ms": float(np.percentile(wt, 50) * 1e3),
                "wait_p99_ms": float(np.percentile(wt, 99) * 1e3)}


class DeviceExecutor:
    """The loop's device work on the current GPU: two arenas of `arena_bytes`,
    one shared descriptor per (fractal, r), the library's init kernel and its
    batched step with per-instance step counts."""

    def __init__(self, arena_bytes: int, tile_levels: Optional[Dict[str, int]] = None):
        import torch
        self.torch = torch
        dev = torch.device("cuda", torch.cuda.current_device())
        self.arenas = [torch.zeros(arena_bytes, dtype=torch.uint8, device=dev) for _ in range(2)]
        self.tile_levels = dict(tile_levels or {})
        self._desc: Dict[Tuple[str, int], object] = {}
        self._ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        # the batch of the last round, reused while the next round steps the
        # same instances in the same order (building one costs an allocation,
        # table uploads and a synchronisation)
        self._batch = None
        self._batch_key = None
        self.batches_built = 0

    def descriptor(self, fd, r: int):
        """One shared descriptor per (fractal, r).  Instances of a fractal named
        in tile_levels all get that tile level (capped by r), so they share a
        launch; others keep their automatic plan."""
        key = (fd.name, r)
        d = self._desc.get(key)
        if d is None:
            d = N.Fractal(fd.s, fd.offsets, r)
            m = self.tile_levels.get(fd.name)
            inf = d.info()
            if m and inf.strategy != N.STRATEGY_DIRECT:
                d.configure(int(inf.strategy), min(m, r))
            self._desc[key] = d
        return d

    def init(self, desc, seed: int, p: float, arena: int, offset: int, cells: int) -> None:
        desc.init_compact(seed, p, out=self.arenas[arena][offset:offset + cells])

    def step_each(self, descs, offsets, steps, rule: int, arena: int) -> float:
        """Instance j (descs[j] at offsets[j]) takes steps[j] generations from
        arena `arena` (ending in the other one iff steps[j] is odd); returns
        the device time in seconds."""
        torch = self.torch
        stream = torch.cuda.current_stream()
        key = tuple((id(d), int(o)) for d, o in zip(descs, offsets))
        if key != self._batch_key:
            self._batch = None  # frees the old batch's tables first
            self._batch = N.Batch(descs, offsets)
            self._batch_key = key
            self.batches_built += 1
        ev0, ev1 = self._ev
        ev0.record(stream)
        self._batch.step_each(self.arenas[arena], self.arenas[1 - arena], steps, rule)
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) * 1e-3

    def view(self, arena: int, offset: int, cells: int):
        return self.arenas[arena][offset:offset + cells]


class Server:
    """Serves automaton runs from two arenas of `arena_bytes` each (on the
    current GPU unless another executor is given)."""

    def __init__(self, arena_bytes: int, rule: int = N.NBB_RULE_B3S23, deadline_s: float = 1.0,
                 round_s: float = 0.02, max_gens: int = 64, throughput0: float = 1e12,
                 tile_levels: Optional[Dict[str, int]] = None, safety: float = 0.8, executor=None):
        self.exe = executor if executor is not None else DeviceExecutor(arena_bytes, tile_levels)
        self.cur = 0                     # arena holding the active states
        self.alloc = ArenaAllocator(arena_bytes)
        self.rule = int(rule)
        self.deadline_s = float(deadline_s)
        self.round_s = float(round_s)
        self.max_gens = int(max_gens)
        self.throughput = float(throughput0)   # cell updates per second, measured
        self.safety = float(safety)            # fraction of the measured throughput admission counts on

    def run(self, requests: Sequence, on_complete: Optional[Callable] = None, log=None) -> ServeStats:
        exe = self.exe
        st = ServeStats(offered=len(requests))
        active: List[_Active] = []
        footprint = 0          # cells of the active requests
        tightest = float("inf")  # min over active requests of slack / generations left
        i = 0
        t0 = time.perf_counter()
        while i < len(requests) or active:
            now = time.perf_counter() - t0
            # admit what has arrived
            while i < len(requests) and requests[i].t <= now:
                q = requests[i]
                i += 1
                fp = footprint + q.cells
                # the deadline runs from the request's arrival, not from now
                tight = min(tightest, max(0.0, q.t + self.deadline_s - now) / q.steps)
                if fp > self.safety * self.throughput * tight:
                    st.rejected_deadline += 1
                    continue
                off = self.alloc.alloc(q.cells)
                if off is None:
                    st.rejected_memory += 1
                    continue
                d = exe.descriptor(q.fractal, q.r)
                exe.init(d, q.seed, q.p, self.cur, off, q.cells)
                active.append(_Active(q, d, off, q.steps, now))
                footprint, tightest = fp, tight
                st.admitted += 1
            if not active:
                if i < len(requests):
                    time.sleep(max(0.0, requests[i].t - (time.perf_counter() - t0)))
                continue
            # one round: up to G generations of every active request
            rem = [a.remaining for a in active]
            cells = [a.req.cells for a in active]
            order, G = plan_round(rem, cells, self.throughput * self.round_s, self.max_gens)
            active = [active[j] for j in order]
            steps = [min(a.remaining, G) for a in active]
            start = time.perf_counter() - t0
            for a in active:
                if a.started is None:
                    a.started = start
            gpu_s = exe.step_each([a.desc for a in active], [a.offset for a in active], steps, self.rule,
                                  self.cur)
            done_t = time.perf_counter() - t0
            upd = sum(s * c for s, c in zip(steps, (a.req.cells for a in active)))
            st.rounds += 1
            st.gpu_seconds += gpu_s
            st.cell_updates += upd
            if gpu_s > 0 and upd > 0:
                self.throughput = 0.7 * self.throughput + 0.3 * (upd / gpu_s)
            survivors = []
            for a, s_ in zip(active, steps):
                a.remaining -= s_
                if a.remaining:
                    survivors.append(a)
                    continue
                st.completed += 1
                st.latencies.append(done_t - a.req.t)
                st.waits.append(a.started - a.req.t)
                if on_complete is not None:
                    res = 1 - self.cur if (s_ & 1) else self.cur
                    on_complete(a.req, exe.view(res, a.offset, a.req.cells))
                self.alloc.free(a.offset)
            if G & 1:
                self.cur = 1 - self.cur
            active = survivors
            footprint = sum(a.req.cells for a in active)
            tightest = min(((a.req.t + self.deadline_s - done_t) / a.remaining for a in active),
                           default=float("inf"))
            if log and st.rounds % 50 == 0:
                log(f"serve: t={done_t:.1f}s rounds={st.rounds} active={len(active)} done={st.completed} "
                    f"rejected={st.rejected_deadline + st.rejected_memory} {self.throughput:.3e} cell-upd/s")
        st.wall_seconds = time.perf_counter() - t0
        return st
