"""The request loop's scheduling on the CPU: the loop of serve.py driven by an
executor that keeps the arenas in host memory and steps each instance with
the oracle.  What is tested is the loop's own bookkeeping (admission,
arena allocation, rounds of G generations, which arena holds a request's
state after rounds of odd and even length, per-request step counts), so a
request's result must equal a fresh oracle run of its own steps.  Inputs are
seeded and synthetic.
"""
import time

import numpy as np

from oracle import oracle as O
from paper_2110_12952_amd import workloads as W
from paper_2110_12952_amd.serve import Server

B3S23 = W.rule_mask("B3/S23")


class OracleExecutor:
    """Host arenas; instance steps by the oracle's compact step."""

    def __init__(self, arena_bytes):
        self.arenas = [np.full(arena_bytes, 0xEE, np.uint8) for _ in range(2)]
        self._desc = {}
        self.rounds = []   # steps of every round, for the tests

    def descriptor(self, fd, r):
        key = (fd.name, r)
        if key not in self._desc:
            self._desc[key] = O.Fractal(fd.s, fd.offsets, r)
        return self._desc[key]

    def init(self, desc, seed, p, arena, offset, cells):
        self.arenas[arena][offset:offset + cells] = desc.init_compact(seed, p)

    def step_each(self, descs, offsets, steps, rule, arena):
        t0 = time.perf_counter()
        self.rounds.append(list(steps))
        for d, off, s in zip(descs, offsets, steps):
            if s == 0:
                continue
            state = self.arenas[arena][off:off + d.cells].copy()
            self.arenas[(arena + s) & 1][off:off + d.cells] = d.compact_steps(state, rule, s)
        return time.perf_counter() - t0

    def view(self, arena, offset, cells):
        return self.arenas[arena][offset:offset + cells]


SMALL = W.ServeWorkload("serve_host", 300.0, 0.4, ("carpet", "hfractal", "triangle", "chandelier"), 23,
                        log10_cells=(3.0, 3.9), steps=(5, 40))


def _check(results):
    oracles = {}
    for q, got in results:
        key = (q.fractal.name, q.r)
        o = oracles.setdefault(key, O.Fractal(q.fractal.s, q.fractal.offsets, q.r))
        want = o.compact_steps(o.init_compact(q.seed, q.p), B3S23, q.steps)
        np.testing.assert_array_equal(got, want, err_msg=f"request {q.rid} {key} steps={q.steps}")


def test_loop_completes_every_admitted_request_exactly():
    reqs = SMALL.requests()
    assert len(reqs) > 50
    exe = OracleExecutor(1 << 22)
    results = []
    srv = Server(1 << 22, deadline_s=100.0, round_s=0.05, max_gens=7, throughput0=1e9, executor=exe)
    st = srv.run(reqs, on_complete=lambda q, v: results.append((q, v.copy())))
    assert st.offered == len(reqs) == st.admitted == st.completed == len(results)
    _check(results)
    # rounds of odd and of even length both happened, and requests left mid-round
    lengths = {max(r) for r in exe.rounds}
    assert any(g % 2 for g in lengths) and any(g % 2 == 0 for g in lengths)
    assert any(min(r) < max(r) for r in exe.rounds)
    srv.alloc.check()
    assert srv.alloc.used_bytes == 0
    s = st.summary()
    assert s["latency_p99_ms"] >= s["latency_p50_ms"] > 0 and st.cell_updates == sum(q.cells * q.steps for q in reqs)


def test_loop_turns_away_what_does_not_fit():
    reqs = SMALL.requests(0.15)
    big = max(q.cells for q in reqs)
    exe = OracleExecutor(big + 2048)
    results = []
    srv = Server(big + 2048, deadline_s=100.0, round_s=1e-4, max_gens=5, throughput0=1e9, executor=exe)
    st = srv.run(reqs, on_complete=lambda q, v: results.append((q, v.copy())))
    assert st.rejected_memory > 0 and st.completed == st.admitted == len(results) > 0
    assert st.admitted + st.rejected_memory + st.rejected_deadline == st.offered
    _check(results)
    srv.alloc.check()


def test_loop_deadline_admission():
    reqs = SMALL.requests(0.15)
    # at this throughput estimate no request can finish within the deadline
    srv = Server(1 << 22, deadline_s=1e-3, round_s=1e-4, max_gens=5, throughput0=1e3,
                 executor=OracleExecutor(1 << 22))
    st = srv.run(reqs)
    assert st.rejected_deadline == st.offered > 0 and st.rounds == 0
