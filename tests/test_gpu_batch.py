"""GPU parity of the batched compact step and the autotuner.

Every instance of a batch must end exactly where the oracle's compact step
(and the library's own single-instance step) puts it; bytes of the arenas
outside the instances' ranges must not change.  Inputs are seeded and
synthetic; expected values come from oracle/ only.
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


# An s = 5 fractal: no tiled plan, so its instances take the per-cell step.
PLUS5 = W.FractalDef("plus5", 5, ((2, 0), (0, 2), (2, 2), (4, 2), (2, 4), (1, 1)))

MIXED = [("triangle", 3), ("triangle", 5), ("triangle", 7), ("carpet", 2), ("carpet", 3),
         ("hfractal", 2), ("hfractal", 3), ("chandelier", 3), ("chandelier", 4), ("grid4_12", 3),
         ("cantor", 6), ("triangle", 0), ("vicsek", 3), ("triangle", 6), ("carpet", 3)]


def _mixed(N, with_direct=True, common_level=True):
    fds = [W.FRACTALS[n] for n, _ in MIXED] + ([PLUS5] if with_direct else [])
    rs = [r for _, r in MIXED] + ([2] if with_direct else [])
    frs = [N.Fractal(fd.s, fd.offsets, r) for fd, r in zip(fds, rs)]
    if common_level:
        # one tile level per fractal type, capped by r, so instances group
        for f in frs:
            if f.r >= 1 and f.s <= 4:
                f.configure(N.STRATEGY_TILED, min(f.r, 2))
    return fds, rs, frs


def _spread_offsets(cells, seed):
    """Offsets with random 16-byte-multiple gaps between instances."""
    rng = np.random.default_rng(seed)
    offs, o = [], 0
    for c in cells:
        o += 16 * int(rng.integers(0, 4))
        offs.append(o)
        o += (c + 15) & ~15
    return offs, o + 32


@pytest.mark.parametrize("resident", [True, False])
@pytest.mark.parametrize("rule", ["B3/S23", "B36/S23", "B1357/S02468", "B2/S", "vN:B2/S12"])
@pytest.mark.parametrize("steps", [1, 6])
def test_batch_mixed_vs_oracle(N, rule, steps, resident):
    # every tiled instance here is small: stepped in LDS (resident) or by the
    # per-generation group launches
    fds, rs, frs = _mixed(N)
    offs, total = _spread_offsets([f.cells for f in frs], 7 + steps)
    batch = N.Batch(frs, offs, resident=resident)
    inf = batch.info()
    assert inf.instances == len(frs) and inf.direct >= 2  # triangle r = 0 and the s = 5 fractal
    assert inf.resident == (inf.instances - inf.direct if resident else 0)
    assert (inf.groups == 0) == resident
    a = torch.full((total,), 0xA5, dtype=torch.uint8, device="cuda")
    b = torch.full((total,), 0x5A, dtype=torch.uint8, device="cuda")
    want = []
    for i, (fd, r, f) in enumerate(zip(fds, rs, frs)):
        f.init_compact(100 + i, 0.45, out=batch.state(a, i))
        o = O.Fractal(fd.s, fd.offsets, r)
        want.append(o.compact_steps(o.init_compact(100 + i, 0.45), W.rule_mask(rule), steps))
    res = batch.step(a, b, steps, W.rule_mask(rule))
    assert (res is b) == bool(steps & 1)
    got = host(res)
    for i in range(len(frs)):
        np.testing.assert_array_equal(got[offs[i]:offs[i] + frs[i].cells], want[i],
                                      err_msg=f"instance {i} {MIXED[i] if i < len(MIXED) else 'plus5'}")
    # bytes outside every instance keep their fill in both arenas
    inside = np.zeros(total, bool)
    for o, c in zip(offs, [f.cells for f in frs]):
        inside[o:o + c] = True
    assert (host(a)[~inside] == 0xA5).all() and (host(b)[~inside] == 0x5A).all()


@pytest.mark.parametrize("resident", [True, False])
@pytest.mark.parametrize("rule", ["B3/S23", "B1357/S02468"])
def test_batch_wave_and_workgroup_plans_vs_oracle(N, rule, resident):
    # the same fractals once with one wavefront per tile and once with one
    # work-group per tile, in one batch: separate groups, same results
    specs = [("triangle", 5, 3), ("triangle", 8, 4), ("chandelier", 4, 3), ("carpet", 3, 2),
             ("hfractal", 3, 3), ("grid4_12", 3, 2), ("cantor", 7, 3)]
    frs, want = [], []
    rm = W.rule_mask(rule)
    for j, strategy in enumerate((N.STRATEGY_TILED_WAVE, N.STRATEGY_TILED)):
        for i, (name, r, m) in enumerate(specs):
            fd = W.FRACTALS[name]
            f = N.Fractal(fd.s, fd.offsets, r)
            f.configure(strategy, m)
            assert f.info().strategy == strategy
            frs.append(f)
            o = O.Fractal(fd.s, fd.offsets, r)
            want.append(o.compact_steps(o.init_compact(40 + i, 0.5), rm, 9))
    batch = N.Batch(frs, resident=resident)
    inf = batch.info()
    assert (inf.groups, inf.resident) == ((0, len(frs)) if resident else (2 * len(specs), 0))
    a, b = batch.new_arena(), batch.new_arena()
    for idx, f in enumerate(frs):
        f.init_compact(40 + idx % len(specs), 0.5, out=batch.state(a, idx))
    got = host(batch.step(a, b, 9, rm))
    for idx, f in enumerate(frs):
        np.testing.assert_array_equal(got[batch.offsets[idx]:batch.offsets[idx] + f.cells], want[idx],
                                      err_msg=f"instance {idx}")


def test_batch_groups_by_plan(N):
    _, _, frs = _mixed(N, with_direct=False)
    inf = N.Batch(frs, resident=False).info()
    tiled = [f for f in frs if f.info().strategy != N.STRATEGY_DIRECT]
    kinds = {(f.s, f.offsets, f.info().tile_level, f.info().strategy) for f in tiled}
    assert inf.groups == len(kinds)
    assert inf.tiles == sum(f.info().tiles for f in tiled)
    assert inf.cells == sum(f.cells for f in frs)


def test_batch_default_levels_vs_single(N):
    # descriptors at their automatic levels (different levels, several groups
    # per fractal); every instance must match its own single-instance run
    fds, rs, frs = _mixed(N, common_level=False)
    batch = N.Batch(frs)
    a, b = batch.new_arena(), batch.new_arena()
    singles = []
    for i, f in enumerate(frs):
        f.init_compact(7 * i + 1, 0.5, out=batch.state(a, i))
        s0 = f.init_compact(7 * i + 1, 0.5)
        singles.append(f.step_compact(s0, torch.empty_like(s0), 9))
    res = host(batch.step(a, b, 9))
    for i, f in enumerate(frs):
        np.testing.assert_array_equal(res[batch.offsets[i]:batch.offsets[i] + f.cells], host(singles[i]))


def test_batch_empty_and_single(N):
    e = N.Batch([])
    assert e.info().instances == 0 and e.info().tiles == 0
    a, b = e.new_arena(), e.new_arena()
    assert e.step(a, b, 3) is b
    fd = W.TRIANGLE
    o = O.Fractal(fd.s, fd.offsets, 8)
    f = N.Fractal(fd.s, fd.offsets, 8)
    one = N.Batch([f])
    a, b = one.new_arena(), one.new_arena()
    f.init_compact(5, 0.5, out=one.state(a, 0))
    got = host(one.state(one.step(a, b, 11), 0))
    np.testing.assert_array_equal(got, o.compact_steps(o.init_compact(5, 0.5), B3S23, 11))


def test_batch_zero_steps(N):
    _, _, frs = _mixed(N)
    batch = N.Batch(frs)
    a, b = batch.new_arena(), batch.new_arena()
    a.random_(0, 2)
    b.fill_(3)
    a0 = host(a).copy()
    assert batch.step(a, b, 0) is a
    np.testing.assert_array_equal(host(a), a0)
    assert (host(b) == 3).all()


def test_batch_rejects_bad_arguments(N):
    fd = W.CARPET
    f = N.Fractal(fd.s, fd.offsets, 3)
    g = N.Fractal(fd.s, fd.offsets, 2)
    with pytest.raises(N.NbbError, match="overlap"):
        N.Batch([f, g], [0, 496])          # f holds 512 bytes
    with pytest.raises(N.NbbError, match="multiples of 16"):
        N.Batch([f, g], [0, 520])
    with pytest.raises(N.NbbError) as ei:
        N.Batch([f], [1 << 36])
    assert ei.value.status == N.NBB_E_RANGE
    batch = N.Batch([f, g], [0, 512])
    a = torch.zeros(512 + 64, dtype=torch.uint8, device="cuda")
    short = torch.zeros(512 + 48, dtype=torch.uint8, device="cuda")
    with pytest.raises(N.NbbError, match="shorter"):
        batch.step(short, torch.zeros_like(short), 1)
    with pytest.raises(N.NbbError, match="overlap"):
        batch.step(a, a, 1)
    with pytest.raises(N.NbbError, match="bits outside"):
        batch.step(a, torch.zeros_like(a), 1, rule=1 << 9)
    big = torch.zeros(1200, dtype=torch.uint8, device="cuda")
    with pytest.raises(N.NbbError, match="aligned"):
        batch.step(big[1:577], big[600:1176], 1)


def _c4(N, items):
    return N.shared_descriptors([(it.fractal.s, it.fractal.offsets, it.r) for it in items])


def test_batch512_equals_single_runs_and_oracle(N):
    # the full batched workload, fewer generations: the batch against each
    # instance's own single-instance run (whole states), and the smallest
    # instances against the oracle
    items = W.BATCH512.items()
    frs = _c4(N, items)
    batch = N.Batch(frs)
    inf = batch.info()
    assert inf.groups == 4 and inf.direct == 0
    a, b = batch.new_arena(), batch.new_arena()
    for i, (it, f) in enumerate(zip(items, frs)):
        f.init_compact(it.seed, it.p, out=batch.state(a, i))
    T = 24
    ref = torch.empty_like(a)
    tmp = torch.empty(max(f.cells for f in frs), dtype=torch.uint8, device="cuda")
    for i, (it, f) in enumerate(zip(items, frs)):
        s0 = batch.state(a, i).clone()
        out = f.step_compact(s0, tmp[:f.cells], T)
        batch.state(ref, i).copy_(out)
    res = batch.step(a, b, T)
    got, want = host(res), host(ref)
    for i, f in enumerate(frs):
        sl = slice(batch.offsets[i], batch.offsets[i] + f.cells)
        np.testing.assert_array_equal(got[sl], want[sl], err_msg=f"instance {i}")
    small = sorted(range(len(items)), key=lambda i: items[i].cells)[:4]
    for i in small:
        it = items[i]
        o = O.Fractal(it.fractal.s, it.fractal.offsets, it.r)
        exp = o.compact_steps(o.init_compact(it.seed, it.p), B3S23, T)
        np.testing.assert_array_equal(got[batch.offsets[i]:batch.offsets[i] + frs[i].cells], exp)


def test_batch512_on_a_side_stream_is_ordered_on_it(N):
    # the groups run on streams of the library forked from the caller's and
    # joined back to it: two calls in a row and a copy enqueued after them on
    # the caller's (non-default) stream, waited for on that stream alone, see
    # every group's last generation
    items = W.BATCH512.items()
    frs = _c4(N, items)
    batch = N.Batch(frs)
    assert batch.info().groups == 4
    a, b = batch.new_arena(), batch.new_arena()
    for i, (it, f) in enumerate(zip(items, frs)):
        f.init_compact(it.seed, it.p, out=batch.state(a, i))
    ref = torch.empty_like(a)
    tmp = torch.empty(max(f.cells for f in frs), dtype=torch.uint8, device="cuda")
    for i, f in enumerate(frs):
        out = f.step_compact(batch.state(a, i).clone(), tmp[:f.cells], 7)
        batch.state(ref, i).copy_(out)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        r1 = batch.step(a, b, 3)
        r2 = batch.step(r1, a if r1 is b else b, 4)
        seen = r2.clone()
    side.synchronize()
    got, want = seen.cpu().numpy(), host(ref)
    for i, f in enumerate(frs):
        sl = slice(batch.offsets[i], batch.offsets[i] + f.cells)
        np.testing.assert_array_equal(got[sl], want[sl], err_msg=f"instance {i}")


# ------------------------------------------------------------- autotuner --
@pytest.mark.parametrize("name,r", [("triangle", 10), ("carpet", 5), ("chandelier", 6), ("hfractal", 2)])
def test_autotune_then_step_matches_oracle(N, name, r):
    fd = W.FRACTALS[name]
    f = N.Fractal(fd.s, fd.offsets, r)
    o = O.Fractal(fd.s, fd.offsets, r)
    a, b = f.new_compact(), f.new_compact()
    f.init_compact(3, 0.5, out=a)
    inf = f.autotune(a, b, steps=2)
    assert inf.strategy in (N.STRATEGY_TILED, N.STRATEGY_TILED_WAVE, N.STRATEGY_TEMPORAL, N.STRATEGY_DIRECT)
    got = f.info()
    assert (got.strategy, got.tile_level, got.temporal_depth) == (inf.strategy, inf.tile_level,
                                                                  inf.temporal_depth)
    s0 = f.init_compact(3, 0.5)
    res = host(f.step_compact(s0, torch.empty_like(s0), 13))
    np.testing.assert_array_equal(res, o.compact_steps(o.init_compact(3, 0.5), B3S23, 13))


def test_autotune_rejects_zero_steps(N):
    f = N.Fractal(2, W.TRIANGLE.offsets, 5)
    a, b = f.new_compact(), f.new_compact()
    with pytest.raises(N.NbbError, match="steps"):
        f.autotune(a, b, steps=0)


@pytest.mark.parametrize("resident", [True, False])
@pytest.mark.parametrize("seed", [0, 1])
def test_batch_random_fractals_vs_oracle(N, seed, resident):
    # seeded random NBB fractals (s in 2..4, any k), random levels and plans
    # (automatic, a common level, one wavefront per tile where it fits)
    rng = np.random.default_rng(500 + seed)
    fds, rs, frs = [], [], []
    for i in range(14):
        fd = W.random_fractal(1000 * seed + i)
        r = 1
        while fd.k ** (r + 1) <= 20000 and r < 10:
            r += 1
        r = int(rng.integers(max(1, r - 2), r + 1))
        f = N.Fractal(fd.s, fd.offsets, r)
        choice = int(rng.integers(3))
        if choice == 1 and f.info().strategy != N.STRATEGY_DIRECT:
            f.configure(N.STRATEGY_TILED, max(1, min(r, 2)))
        elif choice == 2 and f.info().strategy != N.STRATEGY_DIRECT:
            try:
                f.configure(N.STRATEGY_TILED_WAVE, max(1, min(r, 2)))
            except N.NbbError:
                pass
        fds.append(fd)
        rs.append(r)
        frs.append(f)
    batch = N.Batch(frs, resident=resident)
    a, b = batch.new_arena(), batch.new_arena()
    rule = W.rule_mask("B36/S23" if seed else "vN:B2/S12")
    want = []
    for i, (fd, r, f) in enumerate(zip(fds, rs, frs)):
        f.init_compact(i, 0.5, out=batch.state(a, i))
        o = O.Fractal(fd.s, fd.offsets, r)
        want.append(o.compact_steps(o.init_compact(i, 0.5), rule, 5))
    got = host(batch.step(a, b, 5, rule))
    for i, f in enumerate(frs):
        np.testing.assert_array_equal(got[batch.offsets[i]:batch.offsets[i] + f.cells], want[i],
                                      err_msg=f"instance {i}: {fds[i]} r={rs[i]}")


# ------------------------------------------------- instances stepped in LDS --
# Instances small enough for one work-group's LDS run all generations in one
# launch on a stream of the batch, beside the per-generation launches of the
# large ones.
LARGE_AND_SMALL = [("triangle", 12, None), ("carpet", 5, None), ("hfractal", 6, None), ("triangle", 9, None),
                   ("triangle", 7, None), ("carpet", 4, None), ("hfractal", 5, None), ("chandelier", 7, None),
                   ("chandelier", 5, None), ("triangle", 3, None), ("vicsek", 4, 2), ("hfractal", 4, 2)]


def _large_and_small(N):
    fds = [W.FRACTALS[n] for n, _, _ in LARGE_AND_SMALL]
    rs = [r for _, r, _ in LARGE_AND_SMALL]
    frs = []
    for fd, (_, r, m) in zip(fds, LARGE_AND_SMALL):
        f = N.Fractal(fd.s, fd.offsets, r)
        if m:
            f.configure(N.STRATEGY_TILED, m)
        frs.append(f)
    return fds, rs, frs


@pytest.mark.parametrize("rule", ["B3/S23", "vN:B13/S13"])
def test_batch_resident_beside_group_launches(N, rule):
    fds, rs, frs = _large_and_small(N)
    offs, total = _spread_offsets([f.cells for f in frs], 3)
    batch = N.Batch(frs, offs, resident=True)
    inf = batch.info()
    # the two largest take the group launches, the small ones LDS
    assert inf.groups >= 1 and len(frs) - 3 <= inf.resident <= len(frs) - 2
    a = torch.full((total,), 0x11, dtype=torch.uint8, device="cuda")
    b = torch.full((total,), 0x22, dtype=torch.uint8, device="cuda")
    rm = W.rule_mask(rule)
    for i, f in enumerate(frs):
        f.init_compact(60 + i, 0.4, out=batch.state(a, i))
    T = 7
    singles = []
    for i, f in enumerate(frs):
        s0 = f.init_compact(60 + i, 0.4)
        singles.append(host(f.step_compact(s0, torch.empty_like(s0), T, rm)))
    got = host(batch.step(a, b, T, rm))
    for i, f in enumerate(frs):
        np.testing.assert_array_equal(got[offs[i]:offs[i] + f.cells], singles[i], err_msg=f"instance {i}")
        if f.cells <= 20000:
            o = O.Fractal(fds[i].s, fds[i].offsets, rs[i])
            np.testing.assert_array_equal(singles[i], o.compact_steps(o.init_compact(60 + i, 0.4), rm, T))
    inside = np.zeros(total, bool)
    for o_, c in zip(offs, [f.cells for f in frs]):
        inside[o_:o_ + c] = True
    assert (host(a)[~inside] == 0x11).all() and (host(b)[~inside] == 0x22).all()


def test_batch_resident_step_each_any_order_vs_oracle(N):
    # per-instance generation counts; resident instances need no order
    fds, rs, frs = _large_and_small(N)
    steps = [9, 6, 4, 0, 1, 2, 3, 5, 8, 13, 7, 10]   # the three largest first, in decreasing order
    batch = N.Batch(frs, resident=True)
    a, b = batch.new_arena(), batch.new_arena()
    a0 = []
    for i, f in enumerate(frs):
        f.init_compact(80 + i, 0.5, out=batch.state(a, i))
        a0.append(host(batch.state(a, i)).copy())
    batch.step_each(a, b, steps)
    ga, gb = host(a), host(b)
    for i, (fd, r, f) in enumerate(zip(fds, rs, frs)):
        got = (gb if steps[i] & 1 else ga)[batch.offsets[i]:batch.offsets[i] + f.cells]
        if steps[i] == 0:
            np.testing.assert_array_equal(got, a0[i])
            continue
        o = O.Fractal(fd.s, fd.offsets, r)
        np.testing.assert_array_equal(got, o.compact_steps(o.init_compact(80 + i, 0.5), B3S23, steps[i]),
                                      err_msg=f"instance {i} steps {steps[i]}")


def test_batch_resident_many_chunks_vs_oracle(N):
    # more small instances than one resident launch takes (several launches
    # per plan), two plans, one shared descriptor per plan
    tri = N.Fractal(2, W.TRIANGLE.offsets, 6)
    car = N.Fractal(3, W.CARPET.offsets, 3)
    frs = [tri if i % 3 else car for i in range(300)]
    batch = N.Batch(frs)
    inf = batch.info()
    assert inf.resident == 300 and inf.groups == 0
    a, b = batch.new_arena(), batch.new_arena()
    for i, f in enumerate(frs):
        f.init_compact(i, 0.5, out=batch.state(a, i))
    got = host(batch.step(a, b, 12))
    ot, oc = O.Fractal(2, W.TRIANGLE.offsets, 6), O.Fractal(3, W.CARPET.offsets, 3)
    for i, f in enumerate(frs):
        o = ot if i % 3 else oc
        np.testing.assert_array_equal(got[batch.offsets[i]:batch.offsets[i] + f.cells],
                                      o.compact_steps(o.init_compact(i, 0.5), B3S23, 12), err_msg=f"instance {i}")
    # per-instance counts (more than one chunk of them), in no order
    steps = [(7 * i) % 11 for i in range(len(frs))]
    for i, f in enumerate(frs):
        f.init_compact(i, 0.5, out=batch.state(a, i))
    batch.step_each(a, b, steps)
    ga, gb = host(a), host(b)
    for i, f in enumerate(frs):
        o = ot if i % 3 else oc
        got = (gb if steps[i] & 1 else ga)[batch.offsets[i]:batch.offsets[i] + f.cells]
        np.testing.assert_array_equal(got, o.compact_steps(o.init_compact(i, 0.5), B3S23, steps[i]),
                                      err_msg=f"instance {i} steps {steps[i]}")


def test_batch_resident_in_graph_replays(N):
    # a captured batch step (fork to the batch's stream and join back inside
    # the capture), replayed with eager work between replays
    fds, rs, frs = _large_and_small(N)
    batch = N.Batch(frs, resident=True)
    assert batch.info().resident >= 9 and batch.info().groups >= 1
    a, b = batch.new_arena(), batch.new_arena()
    for i, f in enumerate(frs):
        f.init_compact(5 + i, 0.5, out=batch.state(a, i))
    a0 = a.clone()
    ref_a, ref_b = batch.new_arena(), batch.new_arena()
    ref_a.copy_(a0)
    batch.step(ref_a, ref_b, 2)        # even: the result is back in ref_a
    want = host(ref_a)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        batch.step(a, b, 1, stream=s)   # warm-up outside capture
        a.copy_(a0)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            batch.step(a, b, 2, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        a.copy_(a0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = host(a)
        for i, f in enumerate(frs):
            sl = slice(batch.offsets[i], batch.offsets[i] + f.cells)
            np.testing.assert_array_equal(got[sl], want[sl], err_msg=f"replay {rep} instance {i}")


def test_batch_resident_default_policy(N):
    # by default small instances go to LDS only when they hold at least 1/8
    # of the tiled cells
    big = N.Fractal(2, W.TRIANGLE.offsets, 12)
    small = [N.Fractal(2, W.TRIANGLE.offsets, 7), N.Fractal(3, W.CARPET.offsets, 3)]
    frs = [big] + small * 4
    assert 8 * sum(f.cells for f in frs[1:]) < sum(f.cells for f in frs)
    inf = N.Batch(frs).info()
    assert inf.resident == 0 and inf.groups == 3
    assert N.Batch(frs, resident=True).info().resident == 8
    assert N.Batch(frs[1:]).info().resident == 8
    assert N.Batch(frs[1:], resident=False).info().resident == 0
    _, _, mixed = _mixed(N)
    inf = N.Batch(mixed).info()
    assert inf.resident == inf.instances - inf.direct and inf.groups == 0


def test_batch_autotune_configures_and_keeps_results(N):
    # plans chosen by timing: every descriptor of a fractal gets the same
    # plan, and the tuned batch still matches the oracle
    specs = [("triangle", 8), ("triangle", 9), ("carpet", 4), ("carpet", 5), ("hfractal", 4), ("triangle", 9)]
    fds = [W.FRACTALS[n] for n, _ in specs]
    frs = N.shared_descriptors([(fd.s, fd.offsets, r) for fd, (_, r) in zip(fds, specs)])
    offsets, length = N.pack_offsets([f.cells for f in frs])
    a = torch.zeros(length, dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    for i, f in enumerate(frs):
        f.init_compact(40 + i, 0.4, out=a[offsets[i]:offsets[i] + f.cells])
    N.batch_autotune(frs, offsets, a, b, steps=3, use_cache=False)
    torch.cuda.synchronize()
    by_fractal = {}
    for (name, _), f in zip(specs, frs):
        inf = f.info()
        by_fractal.setdefault(name, set()).add((inf.strategy, inf.tile_level, inf.tiled_form))
    assert all(len(v) == 1 for v in by_fractal.values()), by_fractal
    # cached: the same choice again without timing
    N.batch_autotune(frs, offsets, a, b, steps=3)
    for (name, _), f in zip(specs, frs):
        inf = f.info()
        assert (inf.strategy, inf.tile_level, inf.tiled_form) in by_fractal[name]
    # the tuned batch against the oracle
    batch = N.Batch(frs, offsets)
    init = []
    for i, f in enumerate(frs):
        f.init_compact(70 + i, 0.5, out=batch.state(a, i))
        init.append(host(batch.state(a, i)).copy())
    res = batch.step(a, b, 7, B3S23)
    for i, ((name, r), fd) in enumerate(zip(specs, fds)):
        o = O.Fractal(fd.s, fd.offsets, r)
        np.testing.assert_array_equal(host(batch.state(res, i)), o.compact_steps(init[i], B3S23, 7),
                                      err_msg=f"instance {i} {name} r={r}")
