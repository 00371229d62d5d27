"""GPU parity of the temporal-blocking step (several generations per launch,
NBB_STRATEGY_TEMPORAL) through the C ABI: whole states against the oracle's
compact step, over fractals, tile levels, ring depths, rules (Moore and
four-cell), step counts below, at and past the depth (several launches, the
parity launch), and the small triangle workload (r = 10) for its 100
generations.  Inputs are seeded and synthetic; expected values come from
oracle/ only.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_12952_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2110_12952_amd import nbbfrac
    nbbfrac.lib()
    return nbbfrac


def _run(N, fd, r, m, h, rule, steps, seed, p=0.45):
    g = N.Fractal(fd.s, fd.offsets, r)
    g.configure_temporal(m, h)
    inf = g.info()
    assert inf.strategy == N.STRATEGY_TEMPORAL and inf.tiled_form == 3
    if m:
        assert inf.tile_level == m
    if h:
        assert inf.temporal_depth == h
    o = O.Fractal(fd.s, fd.offsets, r)
    init = o.init_compact(seed, p)
    a = torch.from_numpy(init.copy()).cuda()
    b = torch.full_like(a, 7)
    res = g.step_compact(a, b, steps, rule)
    torch.cuda.synchronize()
    assert res.data_ptr() == (b if steps & 1 else a).data_ptr()
    want = o.compact_steps(init, rule, steps)
    np.testing.assert_array_equal(res.cpu().numpy(), want,
                                  err_msg=f"{fd.name} r={r} m={m} h={h} steps={steps} rule={rule:#x}")


CASES = [("triangle", 8, 4, 3), ("triangle", 9, 5, 8), ("triangle", 7, 7, 16), ("triangle", 10, 6, 16),
         ("carpet", 5, 2, 4), ("carpet", 4, 3, 9), ("hfractal", 5, 2, 5), ("hfractal", 4, 3, 2),
         ("chandelier", 6, 3, 6), ("vicsek", 4, 2, 3), ("grid4_12", 3, 2, 8), ("fullsquare", 8, 4, 5),
         ("cantordust", 5, 2, 4)]


@pytest.mark.parametrize("name,r,m,h", CASES)
def test_temporal_vs_oracle(N, name, r, m, h):
    fd = W.FRACTALS[name]
    for i, steps in enumerate((1, h, h + 1, 2 * h + 3)):
        _run(N, fd, r, m, h, W.rule_mask("B3/S23"), steps, 100 + i)


@pytest.mark.parametrize("rule", ["B36/S23", "B1357/S1357", "B1357/S02468", "B2/S", "B35/S0123456",
                                  "vN:B13/S13", "vN:B2/S12"])
def test_temporal_rules(N, rule):
    for name, r, m, h in (("triangle", 8, 4, 5), ("carpet", 4, 2, 4), ("hfractal", 4, 2, 3)):
        _run(N, W.FRACTALS[name], r, m, h, W.rule_mask(rule), 2 * h + 1, 31)


def test_temporal_automatic_plan(N):
    # tile level and depth chosen by the library
    for name, r in (("triangle", 10), ("carpet", 5), ("hfractal", 5), ("chandelier", 7)):
        _run(N, W.FRACTALS[name], r, 0, 0, W.rule_mask("B3/S23"), 37, 5)


def test_temporal_small_triangle_workload(N):
    # the small triangle workload: r = 10, Bernoulli(0.5), 100 generations, each seed
    wl = W.SMALL_TRIANGLE
    for seed in wl.seeds:
        _run(N, wl.fractal, wl.r, 0, 0, W.rule_mask(wl.rule), wl.steps, seed, wl.p)


def test_temporal_zero_steps_and_errors(N):
    fd = W.TRIANGLE
    g = N.Fractal(fd.s, fd.offsets, 6)
    g.configure_temporal(3, 4)
    a = g.init_compact(3, 0.5)
    a0 = a.clone()
    b = torch.full_like(a, 9)
    g.step_compact(a, b, 0)
    torch.cuda.synchronize()
    assert torch.equal(a, a0) and bool((b == 9).all())
    with pytest.raises(N.NbbError):
        g.configure_temporal(3, 9)   # depth beyond the tile side
    with pytest.raises(N.NbbError):
        g.configure_temporal(7, 1)   # level beyond r
    assert g.info().temporal_depth == 4  # the old plan is kept
    # back to the tiled strategy
    g.configure(N.STRATEGY_TILED, 0)
    assert g.info().strategy == N.STRATEGY_TILED and g.info().temporal_depth == 0


def test_temporal_descriptor_in_a_batch(N):
    # a descriptor configured for temporal blocking still steps in a batch
    # through its tile plan
    fd = W.CARPET
    g = N.Fractal(fd.s, fd.offsets, 4)
    g.configure_temporal(2, 3)
    o = O.Fractal(fd.s, fd.offsets, 4)
    batch = N.Batch([g, g], resident=False)
    a, b = batch.new_arena(), batch.new_arena()
    init = [o.init_compact(s_, 0.5) for s_ in (1, 2)]
    for i in range(2):
        batch.state(a, i).copy_(torch.from_numpy(init[i]))
    res = batch.step(a, b, 5)
    torch.cuda.synchronize()
    for i in range(2):
        np.testing.assert_array_equal(batch.state(res, i).cpu().numpy(),
                                      o.compact_steps(init[i], W.rule_mask("B3/S23"), 5))
