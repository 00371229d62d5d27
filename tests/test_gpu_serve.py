"""GPU tests of per-instance step counts and of the request loop.

Every request the loop completes is checked against the oracle's compact
step from the same seeded initial state.  Inputs are seeded and synthetic.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_12952_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B3S23 = W.rule_mask("B3/S23")


@pytest.fixture(scope="module")
def N():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2110_12952_amd import nbbfrac
    nbbfrac.lib()
    return nbbfrac


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


SPECS = [("triangle", 6), ("carpet", 3), ("hfractal", 3), ("triangle", 4), ("chandelier", 4),
         ("carpet", 2), ("triangle", 0), ("cantor", 5), ("hfractal", 2), ("triangle", 7)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_step_each_vs_oracle(N, seed):
    rng = np.random.default_rng(seed)
    steps = sorted((int(x) for x in rng.integers(0, 12, size=len(SPECS))), reverse=True)
    frs = [N.Fractal(W.FRACTALS[n].s, W.FRACTALS[n].offsets, r) for n, r in SPECS]
    batch = N.Batch(frs)
    a, b = batch.new_arena(), batch.new_arena()
    a.fill_(0x33)
    b.fill_(0x44)
    for i, f in enumerate(frs):
        f.init_compact(seed * 100 + i, 0.5, out=batch.state(a, i))
    a0 = host(a).copy()
    batch.step_each(a, b, steps)
    ha, hb = host(a), host(b)
    for i, ((name, r), f) in enumerate(zip(SPECS, frs)):
        o = O.Fractal(W.FRACTALS[name].s, W.FRACTALS[name].offsets, r)
        want = o.compact_steps(o.init_compact(seed * 100 + i, 0.5), B3S23, steps[i])
        sl = slice(batch.offsets[i], batch.offsets[i] + f.cells)
        got = hb[sl] if steps[i] & 1 else ha[sl]
        np.testing.assert_array_equal(got, want, err_msg=f"instance {i} {(name, r)} steps={steps[i]}")
        if steps[i] == 0:
            np.testing.assert_array_equal(ha[sl], a0[sl])
            assert (hb[sl] == 0x44).all()


def test_step_each_rejects_increasing_counts(N):
    # the order matters for the per-generation group launches only; the
    # same small instances stepped in LDS take any order
    fd = W.CARPET
    frs = [N.Fractal(fd.s, fd.offsets, 2), N.Fractal(fd.s, fd.offsets, 3)]
    batch = N.Batch(frs, resident=False)
    a, b = batch.new_arena(), batch.new_arena()
    with pytest.raises(N.NbbError, match="increase"):
        batch.step_each(a, b, [3, 5])
    with pytest.raises(ValueError):
        batch.step_each(a, b, [3])
    batch.step_each(a, b, [5, 3])
    res = N.Batch(frs)
    assert res.info().resident == 2
    res.step_each(a, b, [3, 5])


SMALL_SERVE = W.ServeWorkload("serve_small", 400.0, 0.5, ("carpet", "hfractal", "triangle", "chandelier"), 11,
                              log10_cells=(3.0, 4.3), steps=(10, 60))


def _check_completed(results):
    oracles = {}
    for q, got in results:
        key = (q.fractal.name, q.r)
        if key not in oracles:
            oracles[key] = O.Fractal(q.fractal.s, q.fractal.offsets, q.r)
        o = oracles[key]
        want = o.compact_steps(o.init_compact(q.seed, q.p), B3S23, q.steps)
        np.testing.assert_array_equal(got, want, err_msg=f"request {q.rid} {key} steps={q.steps}")


def test_serve_completes_every_admitted_request_exactly(N):
    from paper_2110_12952_amd.serve import Server
    reqs = SMALL_SERVE.requests()
    results = []
    srv = Server(1 << 24, deadline_s=10.0, round_s=0.002, max_gens=16)
    st = srv.run(reqs, on_complete=lambda q, view: results.append((q, view.cpu().numpy().copy())))
    assert st.offered == len(reqs) and st.completed == st.admitted == len(results)
    assert st.rejected_deadline + st.rejected_memory + st.admitted == st.offered
    assert st.admitted > 0.9 * st.offered
    _check_completed(results)
    s = st.summary()
    assert s["latency_p99_ms"] >= s["latency_p50_ms"] > 0
    assert 0.0 <= s["rejected_frac"] < 0.1
    # rounds over an unchanged set of instances reuse the previous round's batch
    assert 0 < srv.exe.batches_built < st.rounds
    srv.alloc.check()
    assert srv.alloc.used_bytes == 0


def test_serve_rejects_what_does_not_fit(N):
    from paper_2110_12952_amd.serve import Server
    reqs = SMALL_SERVE.requests(0.2)
    big = max(q.cells for q in reqs)
    results = []
    # an arena that holds a few states at a time: some requests must be turned away
    srv = Server(big + 4096, deadline_s=10.0, round_s=0.002, max_gens=8)
    st = srv.run(reqs, on_complete=lambda q, view: results.append((q, view.cpu().numpy().copy())))
    assert st.rejected_memory > 0 and st.completed == st.admitted == len(results) > 0
    _check_completed(results)


def test_serve_deadline_admission(N):
    from paper_2110_12952_amd.serve import Server
    reqs = SMALL_SERVE.requests(0.2)
    # a throughput estimate at which no request can finish within the
    # deadline: every request is refused, nothing is run
    srv = Server(1 << 24, deadline_s=1e-3, round_s=0.002, max_gens=8, throughput0=1e3)
    st = srv.run(reqs)
    assert st.rejected_deadline == st.offered > 0
    assert st.completed == st.admitted == st.rounds == 0
