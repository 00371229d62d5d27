"""GPU parity: every entry point of libnbbfrac against the CPU oracle, bit-exact.

All inputs are seeded and synthetic; expected values come from oracle/ only.
Small levels are compared element by element over whole states; the full-size
workloads are compared over whole states where the oracle is fast enough and
on sampled cells (light-cone evaluation) where it is not, plus the compact
step against the box step on the GPU for the full step counts.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_12952_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B3S23 = W.rule_mask("B3/S23")
RULES = ["B3/S23", "B36/S23", "B1357/S02468", "B1357/S1357", "B35/S0123456", "B2/S", "vN:B2/S12",
         "vN:B13/S024"]


@pytest.fixture(scope="module")
def N():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2110_12952_amd import nbbfrac
    nbbfrac.lib()  # fails loudly if the HIP library is missing
    return nbbfrac


def pair(name, r, N):
    fd = W.FRACTALS[name]
    return fd, O.Fractal(fd.s, fd.offsets, r), N.Fractal(fd.s, fd.offsets, r)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def box_view(g, box):
    """n x n view of an n x pitch host copy; padding must be zero."""
    b = host(box)
    assert not b[:, g.n:].any()
    return b[:, :g.n]


SMALL = [("triangle", r) for r in (0, 1, 2, 3, 5, 8)] + \
        [("carpet", r) for r in (1, 2, 3, 4)] + [("hfractal", r) for r in (1, 2, 4)] + \
        [("chandelier", r) for r in (2, 5)] + \
        [("fullsquare", 5), ("vicsek", 4), ("xfractal", 3), ("cantordust", 3), ("cantor", 6),
         ("single", 6), ("grid4_12", 3)]


# ---------------------------------------------------------------- the maps --
@pytest.mark.parametrize("name,r", SMALL)
def test_lambda_every_index(N, name, r):
    fd, o, g = pair(name, r, N)
    x, y = g.lam()
    ox, oy = o.lam_many(np.arange(o.cells))
    np.testing.assert_array_equal(host(x), ox)
    np.testing.assert_array_equal(host(y), oy)
    # explicit indices, including ones beyond k^r
    idx = np.concatenate([W.random_indices(r, 1000, o.cells), [o.cells, o.cells + 7, 2**32 - 1]])
    idx = idx.astype(np.uint32)
    x, y = g.lam(dev(idx.view(np.int32)))
    hx, hy = host(x), host(y)
    ok = idx < o.cells
    ox, oy = o.lam_many(idx[ok].astype(np.int64))
    np.testing.assert_array_equal(hx[ok], ox)
    np.testing.assert_array_equal(hy[ok], oy)
    assert (hx[~ok] == -1).all() and (hy[~ok] == -1).all()


@pytest.mark.parametrize("name,r", SMALL)
def test_nu_whole_box_and_ring(N, name, r):
    fd, o, g = pair(name, r, N)
    yy, xx = np.mgrid[-1:o.n + 1, -1:o.n + 1]
    xs, ys = xx.ravel().astype(np.int32), yy.ravel().astype(np.int32)
    got = host(g.nu(dev(xs), dev(ys))).astype(np.int64)
    np.testing.assert_array_equal(got, o.nu_many(xs, ys))
    # far outside, and the int32 extremes
    far = np.array([-2**31, 2**31 - 1, o.n + 5, -7], dtype=np.int32)
    gx, gy = np.repeat(far, 4), np.tile(far, 4)
    assert (host(g.nu(dev(gx), dev(gy))) == -1).all()


@pytest.mark.parametrize("name,r", SMALL)
def test_map_methods_agree(N, name, r):
    # the per-level digit maps and the matrix-core lambda against the oracle
    fd, o, g = pair(name, r, N)
    ox, oy = o.lam_many(np.arange(o.cells))
    methods = [N.MAP_DIGITS] + ([N.MAP_MFMA] if r >= 1 and r * fd.k <= 192 else [])
    for m in methods:
        x, y = g.lam(method=m)
        np.testing.assert_array_equal(host(x), ox, err_msg=f"lambda method {m}")
        np.testing.assert_array_equal(host(y), oy, err_msg=f"lambda method {m}")
        idx = np.concatenate([W.random_indices(r + 5, 777, o.cells), [o.cells, 2**32 - 1]]).astype(np.uint32)
        x, y = g.lam(dev(idx.view(np.int32)), method=m)
        ok = idx < o.cells
        lx, ly = o.lam_many(idx[ok].astype(np.int64))
        np.testing.assert_array_equal(host(x)[ok], lx)
        assert (host(x)[~ok] == -1).all() and (host(y)[~ok] == -1).all()
    yy, xx = np.mgrid[-1:o.n + 1, -1:o.n + 1]
    xs, ys = xx.ravel().astype(np.int32), yy.ravel().astype(np.int32)
    for m in methods:
        np.testing.assert_array_equal(host(g.nu(dev(xs), dev(ys), method=m)).astype(np.int64),
                                      o.nu_many(xs, ys), err_msg=f"nu method {m}")
    if r == 0 or r * fd.k > 192:
        with pytest.raises(N.NbbError):
            g.lam(method=N.MAP_MFMA)
        with pytest.raises(N.NbbError):
            g.nu(dev(xs), dev(ys), method=N.MAP_MFMA)
    else:
        # far outside and the int32 extremes
        far = np.array([-2**31, 2**31 - 1, o.n + 5, -7, 0], dtype=np.int32)
        gx, gy = np.repeat(far, 5), np.tile(far, 5)
        np.testing.assert_array_equal(host(g.nu(dev(gx), dev(gy), method=N.MAP_MFMA)).astype(np.int64),
                                      o.nu_many(gx, gy))
    with pytest.raises(N.NbbError):
        g.nu(dev(xs), dev(ys), method=3)


def test_map_methods_full_size(N):
    fd, o, g = pair("triangle", 16, N)
    x0, y0 = g.lam()
    for m in (N.MAP_DIGITS, N.MAP_MFMA):
        x, y = g.lam(method=m)
        assert torch.equal(x, x0) and torch.equal(y, y0)
    ref = g.nu(x0, y0)
    assert torch.equal(g.nu(x0, y0, method=N.MAP_DIGITS), ref)
    assert torch.equal(g.nu(x0, y0, method=N.MAP_MFMA), ref)
    assert torch.equal(ref.to(torch.int64), torch.arange(g.cells, device="cuda"))


def test_nu_mfma_indices_past_2_28(N):
    # triangle r = 18: indices up to 3^18 - 1 > 2^28 use the fifth 7-bit plane
    fd = W.TRIANGLE
    g = N.Fractal(fd.s, fd.offsets, 18)
    o = O.Fractal(fd.s, fd.offsets, 18)
    idx = np.concatenate([W.random_indices(18, 4096, o.cells), [0, 2**28 - 1, 2**28, o.cells - 1]]).astype(np.uint32)
    x, y = g.lam(dev(idx.view(np.int32)))
    got = host(g.nu(x, y, method=N.MAP_MFMA)).view(np.uint32)
    np.testing.assert_array_equal(got, idx)
    sample = idx[-64:].astype(np.int64)
    ox, oy = o.lam_many(sample)
    np.testing.assert_array_equal(host(x)[-64:], ox)
    np.testing.assert_array_equal(o.nu_many(ox.astype(np.int32), oy.astype(np.int32)), sample)


def test_maps_empty_count(N):
    g = N.Fractal(2, W.TRIANGLE.offsets, 4)
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    x, y = g.lam(count=0)
    assert x.numel() == 0
    assert g.nu(e, e).numel() == 0


@pytest.mark.parametrize("seed", range(6))
def test_maps_random_fractals(N, seed):
    fd = W.random_fractal(100 + seed, s_choices=(2, 3, 4, 5, 7))
    r = 1
    while fd.k ** (r + 1) <= 200000 and fd.s ** (r + 1) <= 4096 and r < 12:
        r += 1
    o = O.Fractal(fd.s, fd.offsets, r)
    g = N.Fractal(fd.s, fd.offsets, r)
    x, y = g.lam()
    ox, oy = o.lam_many(np.arange(o.cells))
    np.testing.assert_array_equal(host(x), ox)
    np.testing.assert_array_equal(host(y), oy)
    cx, cy = W.random_coords(seed, 200000, -2, o.n + 2)
    np.testing.assert_array_equal(host(g.nu(dev(cx), dev(cy))).astype(np.int64), o.nu_many(cx, cy))


def test_maps_full_size_triangle_r16(N):
    # lambda over all 43,046,721 indices; nu(lambda(i)) = i everywhere on the
    # GPU; lambda and nu on sampled points against the oracle.
    fd, o, g = pair("triangle", 16, N)
    x, y = g.lam()
    idx = g.nu(x, y)
    iota = torch.arange(o.cells, dtype=torch.int64, device="cuda")
    assert bool((idx.to(torch.int64) == iota).all())
    assert bool(((x & y) == 0).all())  # members of the triangle
    samp = W.random_indices(16, 300000, o.cells).astype(np.int64)
    ox, oy = o.lam_many(samp)
    np.testing.assert_array_equal(host(x)[samp], ox)
    np.testing.assert_array_equal(host(y)[samp], oy)
    cx, cy = W.random_coords(17, 1000000, -1, o.n + 1)
    np.testing.assert_array_equal(host(g.nu(dev(cx), dev(cy))).astype(np.int64), o.nu_many(cx, cy))


# -------------------------------------------------------------------- init --
@pytest.mark.parametrize("name,r", SMALL)
def test_init_compact_and_box(N, name, r):
    fd, o, g = pair(name, r, N)
    for seed, p in [(1, 0.5), (12952, 0.3), (2**64 - 3, 0.9), (5, 0.0), (6, 1.0)]:
        np.testing.assert_array_equal(host(g.init_compact(seed, p)), o.init_compact(seed, p))
        np.testing.assert_array_equal(box_view(g, g.init_bbox(seed, p)), o.init_bbox(seed, p))


# ------------------------------------------------------------ compact step --
def tile_levels(fd, r):
    """Every tile level the library accepts for this fractal, plus auto and direct."""
    from paper_2110_12952_amd import nbbfrac
    out = [("auto", 0)]
    for m in range(1, r + 1):
        try:
            nbbfrac.plan_tables(fd.s, fd.offsets, r, m)
        except nbbfrac.NbbError:
            continue
        out.append(("tiled", m))  # edge records where the level allows them
        out.append(("box", m))    # byte scatter
        out.append(("wave", m))   # one wavefront per tile, where the tile fits one
    out.append(("direct", 0))
    return out


def configure(N, g, how):
    """Configure g; False if the plan does not fit (wavefront plans only)."""
    kind, m = how
    if kind == "auto":
        g.configure(N.STRATEGY_AUTO, 0)
    elif kind == "tiled":
        g.configure(N.STRATEGY_TILED, m)
        assert g.info().tiled_form in (1, 2)
    elif kind == "box":
        g.configure(N.STRATEGY_TILED_BOX, m)
        assert g.info().strategy == N.STRATEGY_TILED and g.info().tiled_form == 2
    elif kind == "wave":
        try:
            g.configure(N.STRATEGY_TILED_WAVE, m)
        except N.NbbError:
            return False
        assert g.info().strategy == N.STRATEGY_TILED_WAVE
    else:
        g.configure(N.STRATEGY_DIRECT, 0)
    return True


@pytest.mark.parametrize("name,r", SMALL)
def test_step_compact_small(N, name, r):
    fd, o, g = pair(name, r, N)
    st0 = o.init_compact(77 + r, 0.45)
    for how in tile_levels(fd, r):
        if not configure(N, g, how):
            continue
        for rule in RULES:
            rm = W.rule_mask(rule)
            for steps in (1, 2, 7):
                a = dev(st0)
                b = torch.full_like(a, 0xAB)
                res = g.step_compact(a, b, steps, rm)
                np.testing.assert_array_equal(host(res), o.compact_steps(st0, rm, steps),
                                              err_msg=f"{name} r={r} {how} {rule} steps={steps}")


@pytest.mark.parametrize("seed", range(8))
def test_step_compact_random_fractals(N, seed):
    fd = W.random_fractal(200 + seed)
    r = 1
    while fd.k ** (r + 1) <= 300000 and r < 12:
        r += 1
    o = O.Fractal(fd.s, fd.offsets, r)
    g = N.Fractal(fd.s, fd.offsets, r)
    st0 = o.init_compact(seed, 0.5)
    for how in tile_levels(fd, r):
        if not configure(N, g, how):
            continue
        a = dev(st0)
        res = g.step_compact(a, torch.empty_like(a), 5, B3S23)
        np.testing.assert_array_equal(host(res), o.compact_steps(st0, B3S23, 5), err_msg=str((fd, r, how)))


def test_step_compact_zero_steps_and_buffers(N):
    fd, o, g = pair("triangle", 6, N)
    a = dev(o.init_compact(3, 0.5))
    b = torch.full_like(a, 7)
    a0 = host(a).copy()
    assert g.step_compact(a, b, 0) is a
    np.testing.assert_array_equal(host(a), a0)
    assert (host(b) == 7).all()
    res = g.step_compact(a, b, 4)
    assert res is a  # even step count ends in a


def test_step_compact_rejects_bad_arguments(N):
    fd, o, g = pair("triangle", 5, N)
    a = g.new_compact()
    b = g.new_compact()
    big = torch.empty(o.cells + 64, dtype=torch.uint8, device="cuda")
    L = N.lib()
    s = torch.cuda.current_stream().cuda_stream
    assert L.nbb_step_compact(g._h, a.data_ptr(), b.data_ptr(), o.cells - 1, 1, B3S23, None, s) == N.NBB_E_INVALID
    assert L.nbb_step_compact(g._h, a.data_ptr(), a.data_ptr(), o.cells, 1, B3S23, None, s) == N.NBB_E_INVALID
    assert L.nbb_step_compact(g._h, big.data_ptr(), big.data_ptr() + 32, o.cells, 1, B3S23, None, s) == \
        N.NBB_E_INVALID
    assert L.nbb_step_compact(g._h, big.data_ptr() + 1, b.data_ptr(), o.cells, 1, B3S23, None, s) == \
        N.NBB_E_INVALID
    assert L.nbb_step_compact(g._h, a.data_ptr(), b.data_ptr(), o.cells, 1, 1 << 12, None, s) == N.NBB_E_INVALID
    with pytest.raises(N.NbbError):
        g.configure(N.STRATEGY_TILED, 9)
    with pytest.raises(N.NbbError):
        N.Fractal(5, [(0, 0), (4, 4)], 3).configure(N.STRATEGY_TILED, 1)


# ---------------------------------------------------------------- box step --
@pytest.mark.parametrize("name,r", SMALL)
def test_step_bbox_small(N, name, r):
    fd, o, g = pair(name, r, N)
    st0 = o.init_bbox(91 + r, 0.45)
    for rule in RULES:
        rm = W.rule_mask(rule)
        for steps in (1, 2, 7):
            a = g.init_bbox(91 + r, 0.45)
            res = g.step_bbox(a, torch.full_like(a, 0), steps, rm)
            np.testing.assert_array_equal(box_view(g, res), o.bbox_steps(st0, rm, steps),
                                          err_msg=f"{name} r={r} {rule} steps={steps}")


# Levels whose box no longer fits the low-level membership bitmap (n > 1024):
# membership then combines the low bitmap (s^L columns, s^L <= 1024) with the
# high-level byte map, and for s = 3 (SL = 729, not a multiple of 16) a
# 16-column group can straddle two high-level squares.  Every full-size box
# workload runs this form.
BOX_TWO_LEVEL = [("triangle", 11), ("triangle", 12), ("carpet", 7), ("carpet", 8), ("hfractal", 7),
                 ("chandelier", 8)]
BOX_TWO_LEVEL_RULES = ["B3/S23", "B36/S23", "B1357/S02468", "vN:B2/S12"]


@pytest.mark.parametrize("name,r", BOX_TWO_LEVEL)
def test_box_two_level_membership(N, name, r):
    fd, o, g = pair(name, r, N)
    info = g.info()
    assert info.box_high_side > 1 and info.box_low_side * info.box_high_side == o.n
    if fd.s == 3:
        assert info.box_low_side == 729  # 16-column groups straddle high-level squares
    seed, p = 300 + r, 0.45
    st0 = o.init_bbox(seed, p)
    np.testing.assert_array_equal(box_view(g, g.init_bbox(seed, p)), st0, err_msg=f"{name} r={r} init")
    for rule in BOX_TWO_LEVEL_RULES:
        rm = W.rule_mask(rule)
        for steps in (1, 3):
            want = o.bbox_steps(st0, rm, steps)
            a = g.init_bbox(seed, p)
            res = g.step_bbox(a, torch.full_like(a, 0x77), steps, rm)
            np.testing.assert_array_equal(box_view(g, res), want, err_msg=f"{name} r={r} box {rule} {steps}")
            del a, res
            a = g.init_bbox(seed, p)
            res = g.step_lambda(a, torch.full_like(a, 0x5A), steps, rm)
            np.testing.assert_array_equal(box_view(g, res), want, err_msg=f"{name} r={r} lambda {rule} {steps}")
            del a, res


@pytest.mark.parametrize("name,r", SMALL)
def test_step_lambda_small(N, name, r):
    # the lambda approach (threads over fractal cells, state in the box)
    fd, o, g = pair(name, r, N)
    st0 = o.init_bbox(91 + r, 0.45)
    for rule in RULES:
        rm = W.rule_mask(rule)
        for steps in (1, 2, 7):
            a = g.init_bbox(91 + r, 0.45)
            res = g.step_lambda(a, torch.full_like(a, 0x5A), steps, rm)
            np.testing.assert_array_equal(box_view(g, res), o.bbox_steps(st0, rm, steps),
                                          err_msg=f"{name} r={r} {rule} steps={steps}")


def test_step_lambda_matches_box_step(N):
    fd, o, g = pair("hfractal", 5, N)
    pitch = g.pitch + 32
    a = torch.empty((o.n, pitch), dtype=torch.uint8, device="cuda")
    g.init_bbox(6, 0.5, out=a)
    want = g.step_bbox(a.clone(), torch.empty_like(a), 9)
    got = g.step_lambda(a.clone(), torch.full_like(a, 1), 9)
    assert torch.equal(got, want)
    assert g.step_lambda(a, torch.empty_like(a), 0) is a
    with pytest.raises(N.NbbError):
        g.step_lambda(a, a, 1)


@pytest.mark.parametrize("name,r,m", [("triangle", 6, 3), ("triangle", 8, 7), ("carpet", 3, 2), ("hfractal", 3, 2),
                                      ("chandelier", 4, 3), ("grid4_12", 3, 2), ("cantor", 6, 3), ("vicsek", 3, 2),
                                      ("fullsquare", 5, 3), ("triangle", 3, 1)])
def test_blocked_layout(N, name, r, m):
    # the blocked layout: each tile stored as its whole S x S square
    fd, o, g = pair(name, r, N)
    g.configure(N.STRATEGY_TILED, m)
    S, K, T = fd.s ** m, fd.k ** m, fd.k ** (r - m)
    assert g.blocked_bytes() == T * S * S
    st0 = o.init_compact(5 + r, 0.5)
    fm = O.Fractal(fd.s, fd.offsets, m)
    xs, ys = fm.lam_many(np.arange(K))
    i = np.arange(o.cells)
    pos = (i // K) * S * S + ys[i % K] * S + xs[i % K]
    want = np.zeros(T * S * S, np.uint8)
    want[pos] = st0
    member = np.zeros(T * S * S, bool)
    member[pos] = True
    blk = g.to_blocked(dev(st0))
    np.testing.assert_array_equal(host(blk), want)
    np.testing.assert_array_equal(host(g.from_blocked(blk)), st0)
    for rule in RULES:
        rm = W.rule_mask(rule)
        for steps in (1, 4):
            a = g.to_blocked(dev(st0))
            res = g.step_blocked(a, torch.full_like(a, 0xCD), steps, rm)
            got = host(res)
            assert not got[~member].any(), f"{rule}: a position outside the fractal came out alive"
            np.testing.assert_array_equal(got[pos], o.compact_steps(st0, rm, steps),
                                          err_msg=f"{name} r={r} m={m} {rule} steps={steps}")


def test_step_blocked_and_bbox_in_a_captured_graph(N):
    # the blocked-layout and box steps only enqueue kernels too: captured
    # once, replayed with eager work in between, each replay equal to the
    # eager result
    fd, o, g = pair("triangle", 8, N)
    g.configure(N.STRATEGY_TILED, 4)
    st0 = o.init_compact(17, 0.5)
    want = o.compact_steps(st0, B3S23, 5)
    blk0 = g.to_blocked(dev(st0))
    box0 = g.expand(dev(st0))
    a, b = blk0.clone(), torch.empty_like(blk0)
    c, d = box0.clone(), torch.empty_like(box0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.step_blocked(a, b, 2)
        g.step_bbox(c, d, 2)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rk = g.step_blocked(a, b, 5)
        rb = g.step_bbox(c, d, 5)
    assert rk is b and rb is d
    for rep in range(3):
        a.copy_(blk0)
        c.copy_(box0)
        graph.replay()
        g.step_compact(dev(st0), torch.empty(o.cells, dtype=torch.uint8, device="cuda"), 3)  # eager work
        np.testing.assert_array_equal(host(g.from_blocked(rk)), want, err_msg=f"blocked, replay {rep}")
        np.testing.assert_array_equal(host(g.gather(rb)), want, err_msg=f"box, replay {rep}")


def test_blocked_layout_needs_a_tiled_plan(N):
    fd, o, g = pair("carpet", 3, N)
    g.configure(N.STRATEGY_DIRECT)
    assert g.blocked_bytes() == 0
    with pytest.raises(N.NbbError, match="tiled plan"):
        g.to_blocked(g.new_compact(), out=torch.empty(64, dtype=torch.uint8, device="cuda"))


def test_step_bbox_wider_pitch(N):
    fd, o, g = pair("hfractal", 4, N)
    pitch = g.pitch + 48
    a = torch.empty((o.n, pitch), dtype=torch.uint8, device="cuda")
    g.init_bbox(4, 0.5, out=a)
    res = g.step_bbox(a, torch.empty_like(a), 5)
    np.testing.assert_array_equal(box_view(g, res), o.bbox_steps(o.init_bbox(4, 0.5), B3S23, 5))


@pytest.mark.parametrize("name,r", SMALL)
def test_expand_gather(N, name, r):
    fd, o, g = pair(name, r, N)
    st = o.init_compact(8, 0.5)
    box = g.expand(dev(st))
    np.testing.assert_array_equal(box_view(g, box), o.expand(st))
    np.testing.assert_array_equal(host(g.gather(box)), st)


# ------------------------------------------------------- the workload sizes --
def test_small_triangle_workload(N):
    # triangle r = 10 (59,049 cells), Bernoulli(0.5), seeds 1, 2, 3, 100 steps
    w = W.SMALL_TRIANGLE
    fd, o, g = pair("triangle", w.r, N)
    for seed in w.seeds:
        st0 = o.init_compact(seed, w.p)
        a = g.init_compact(seed, w.p)
        np.testing.assert_array_equal(host(a), st0)
        res = g.step_compact(a, torch.empty_like(a), w.steps)
        np.testing.assert_array_equal(host(res), o.compact_steps(st0, B3S23, w.steps))
        box = g.init_bbox(seed, w.p)
        resb = g.step_bbox(box, torch.empty_like(box), w.steps)
        np.testing.assert_array_equal(host(g.gather(resb)), host(res))


def test_workloads_forms(N):
    # the automatic plans of the workloads take the edge-record form where
    # its blocks fill the work-group passes (H r10 at level 4: 343 blocks over
    # two passes of 256 threads takes the byte-scatter form), and either form
    # can be asked for at the same level
    for name, r, form in [("triangle", 16, 1), ("carpet", 9, 1), ("hfractal", 10, 2), ("chandelier", 11, 1),
                          ("triangle", 10, 2)]:  # triangle r10: 9 blocks per tile at its level 4
        fd, o, g = pair(name, r, N)
        inf = g.info()
        assert inf.strategy == N.STRATEGY_TILED and inf.tiled_form == form, name
        g.configure(N.STRATEGY_TILED_BOX, inf.tile_level)
        assert g.info().tiled_form == 2 and g.info().tile_level == inf.tile_level
        g.configure(N.STRATEGY_TILED_EDGE, inf.tile_level)
        assert g.info().tiled_form == 1 and g.info().strategy == N.STRATEGY_TILED
        g.configure(N.STRATEGY_TILED, inf.tile_level)
        assert g.info().tiled_form == form


@pytest.mark.parametrize("name,r,m", [("triangle", 9, 7), ("triangle", 12, 6), ("carpet", 5, 3), ("carpet", 6, 4),
                                      ("hfractal", 6, 3), ("hfractal", 6, 4), ("chandelier", 9, 4),
                                      ("chandelier", 10, 5), ("grid4_12", 4, 3), ("fullsquare", 7, 5),
                                      ("xfractal", 6, 4), ("cantordust", 7, 4)])
def test_edge_form_against_oracle(N, name, r, m):
    # the edge-record form at levels with several tiles, near-end blocks and
    # shared zero rows, over every rule form (B3/S23, tables, bit extract,
    # four-cell), against the oracle and against the byte-scatter form
    fd, o, g = pair(name, r, N)
    g.configure(N.STRATEGY_TILED_EDGE, m)
    assert g.info().tiled_form == 1
    st0 = o.init_compact(808 + r, 0.45)
    for rule in RULES:
        rm = W.rule_mask(rule)
        for steps in (1, 3):
            a = dev(st0)
            res = g.step_compact(a, torch.full_like(a, 0xEE), steps, rm)
            np.testing.assert_array_equal(host(res), o.compact_steps(st0, rm, steps),
                                          err_msg=f"{name} r={r} m={m} {rule} steps={steps}")


def test_large_triangle_workload(N):
    # triangle r = 16 (43,046,721 cells), Bernoulli(0.3), seed 12952: whole
    # state against the oracle after 2 steps; then 1000 steps of the compact
    # step against 1000 steps of the box step on the GPU.
    w = W.LARGE_TRIANGLE
    fd, o, g = pair("triangle", w.r, N)
    st0 = o.init_compact(w.seeds[0], w.p)
    a = g.init_compact(w.seeds[0], w.p)
    np.testing.assert_array_equal(host(a), st0)
    b = torch.empty_like(a)
    res = g.step_compact(a.clone(), b, 2)
    np.testing.assert_array_equal(host(res), o.compact_steps(st0, B3S23, 2))
    res = g.step_compact(a, b, w.steps)
    box = g.init_bbox(w.seeds[0], w.p)
    resb = g.step_bbox(box, torch.empty_like(box), w.steps)
    assert torch.equal(g.gather(resb), res)
    del box, resb


@pytest.mark.parametrize("wname", ["carpet_r9", "hfractal_r10"])
def test_large_carpet_and_h_workloads(N, wname):
    # carpet r = 9 (134M cells) and H r = 10 (282M cells), Bernoulli(0.5):
    # whole initial state and whole state after 2 steps against the oracle,
    # for the compact step and for the box step (its fractal cells equal the
    # oracle's and no other box cell is alive: the box holds bytes, so equal
    # sums leave nothing alive off the fractal); then compact vs box on the
    # GPU for 200 steps.
    w = W.WORKLOADS[wname]
    fd, o, g = pair(w.fractal.name, w.r, N)
    st0 = o.init_compact(w.seeds[0], w.p)
    a = g.init_compact(w.seeds[0], w.p)
    np.testing.assert_array_equal(host(a), st0)
    want2 = o.compact_steps(st0, B3S23, 2)
    b = torch.empty_like(a)
    res = g.step_compact(a.clone(), b, 2)
    np.testing.assert_array_equal(host(res), want2)
    box = g.init_bbox(w.seeds[0], w.p)
    np.testing.assert_array_equal(host(g.gather(box)), st0)
    assert int(box.sum(dtype=torch.int64)) == int(st0.sum(dtype=np.int64))
    resb = g.step_bbox(box.clone(), torch.empty_like(box), 2)
    np.testing.assert_array_equal(host(g.gather(resb)), want2)
    assert int(resb.sum(dtype=torch.int64)) == int(want2.sum(dtype=np.int64))
    del resb, want2
    res = g.step_compact(a, b, w.steps)
    resb = g.step_bbox(box, torch.empty_like(box), w.steps)
    assert torch.equal(g.gather(resb), res)


@pytest.mark.parametrize("name,r,steps", [("triangle", 12, 300), ("carpet", 6, 200), ("hfractal", 7, 200),
                                          ("chandelier", 9, 200), ("grid4_12", 5, 150)])
def test_long_runs_against_oracle(N, name, r, steps):
    # Many generations over many tiles: a result that depends on the order
    # in which work-groups or waves run would show up as a mismatch here.
    fd, o, g = pair(name, r, N)
    st0 = o.init_compact(4242 + r, 0.4)
    want = o.compact_steps(st0, B3S23, steps)
    for rep in range(2):
        a = dev(st0)
        res = g.step_compact(a, torch.empty_like(a), steps)
        np.testing.assert_array_equal(host(res), want, err_msg=f"{name} r={r} repeat {rep}")


def test_triangle_r20_compact(N):
    # the paper's largest level: triangle r = 20 (3,486,784,401 cells, n =
    # 2^20; its box, 2^40 bytes, cannot exist).  Sampled cells against the
    # oracle's light cone from the seeded initial state, and the tiled step
    # against the per-cell step over the whole state.
    fd = W.TRIANGLE
    o = O.Fractal(fd.s, fd.offsets, 20)
    g = N.Fractal(fd.s, fd.offsets, 20)
    assert g.cells == 3 ** 20 and g.info().strategy == N.STRATEGY_TILED
    a = g.init_compact(20, 0.3)
    samp = np.unique(np.concatenate([W.random_indices(5, 4000, g.cells).astype(np.int64),
                                     np.array([0, 1, g.cells - 2, g.cells - 1], np.int64)]))
    sidx = torch.from_numpy(samp).cuda()
    np.testing.assert_array_equal(host(a[sidx]), o.cells_after_seeded(20, 0.3, samp, B3S23, 0))
    b = torch.empty_like(a)
    res = g.step_compact(a.clone(), b, 2)
    np.testing.assert_array_equal(host(res[sidx]), o.cells_after_seeded(20, 0.3, samp, B3S23, 2))
    tiled = res.clone()
    del res
    g.configure(N.STRATEGY_DIRECT)
    res = g.step_compact(a, b, 2)
    assert torch.equal(res, tiled)


@pytest.mark.parametrize("name,r,strategy", [("triangle", 8, "tiled"), ("carpet", 4, "wave"), ("hfractal", 3, "direct")])
def test_step_compact_in_a_captured_graph(N, name, r, strategy):
    # The step entry points only enqueue kernels (no allocation, memset or
    # synchronisation), so a caller can capture them in a HIP graph.  The
    # graph is replayed several times with eager work in between; every
    # replay must give the oracle's result.
    fd, o, g = pair(name, r, N)
    if strategy == "wave":
        g.configure(N.STRATEGY_TILED_WAVE, 2)
    elif strategy == "direct":
        g.configure(N.STRATEGY_DIRECT)
    st0 = o.init_compact(12, 0.5)
    want = o.compact_steps(st0, B3S23, 6)
    a0 = dev(st0)
    a, b = a0.clone(), torch.empty_like(a0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.step_compact(a, b, 2)          # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        res = g.step_compact(a, b, 6)
    assert res is a
    other = dev(o.init_compact(99, 0.5))
    for rep in range(4):
        a.copy_(a0)
        graph.replay()
        g.step_compact(other, torch.empty_like(other), 3)   # eager work between replays
        np.testing.assert_array_equal(host(a), want, err_msg=f"replay {rep}")
