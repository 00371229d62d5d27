"""GPU parity of the bit-packed compact state (one bit per cell).

The packed layout is the byte layout at one bit per cell (cell i = bit i % 8
of byte i / 8, little-endian words); expected values are the oracle's byte
states packed with numpy's packbits, so every bit, the zero bits past the
last cell included, is compared.  Inputs are seeded and synthetic.
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def packed_of(state_bytes):
    """Bit i of the result = byte i of the state; padded to whole 32-bit words."""
    nbytes = (len(state_bytes) + 31) // 32 * 4
    bits = np.packbits(np.asarray(state_bytes, dtype=np.uint8) != 0, bitorder="little")
    out = np.zeros(nbytes, np.uint8)
    out[:len(bits)] = bits
    return out


CASES = [("triangle", 5, None), ("triangle", 8, None), ("triangle", 10, 7), ("triangle", 6, 1), ("triangle", 7, 2),
         ("carpet", 3, None), ("carpet", 5, None), ("carpet", 4, 1), ("hfractal", 4, None), ("hfractal", 5, 2),
         ("chandelier", 5, None), ("chandelier", 6, 3), ("vicsek", 4, None), ("cantor", 8, None),
         ("cantordust", 4, None), ("grid4_12", 3, None), ("xfractal", 4, 2)]


def _fractal(N, name, r, m, strategy=None):
    fd = W.FRACTALS[name]
    f = N.Fractal(fd.s, fd.offsets, r)
    if m is not None or strategy is not None:
        f.configure(strategy or N.STRATEGY_TILED, m or 0)
    return fd, f


@pytest.mark.parametrize("name,r,m", CASES)
def test_pack_unpack_vs_packbits(N, name, r, m):
    fd, f = _fractal(N, name, r, m)
    o = O.Fractal(fd.s, fd.offsets, r)
    s0 = o.init_compact(17, 0.5)
    st = torch.from_numpy(s0).cuda()
    pk = f.pack(st)
    assert pk.numel() == f.packed_bytes() == (f.cells + 31) // 32 * 4
    np.testing.assert_array_equal(host(pk), packed_of(s0))
    np.testing.assert_array_equal(host(f.unpack(pk)), s0)


@pytest.mark.parametrize("rule", ["B3/S23", "B36/S23", "B1357/S02468", "vN:B13/S13"])
@pytest.mark.parametrize("name,r,m", CASES)
def test_step_packed_vs_oracle(N, name, r, m, rule):
    fd, f = _fractal(N, name, r, m)
    o = O.Fractal(fd.s, fd.offsets, r)
    rm = W.rule_mask(rule)
    s0 = o.init_compact(23, 0.45)
    a = f.pack(torch.from_numpy(s0).cuda())
    b = torch.full_like(a, 0xFF)          # stale bits everywhere: every written bit must be set or cleared
    for steps in (1, 6):
        a0 = a.clone()
        res = f.step_packed(a0, b, steps, rm)
        assert (res is b) == bool(steps & 1)
        bits = np.unpackbits(host(res), bitorder="little")
        np.testing.assert_array_equal(bits[:f.cells], o.compact_steps(s0, rm, steps),
                                      err_msg=f"{name} r={r} m={m} steps={steps}")
        # bits past the last cell are never written: 1 where b's fill was, 0 from pack
        assert (bits[f.cells:] == (1 if res is b else 0)).all()


def test_step_packed_wave_plan_and_reconfigure(N):
    # the same descriptor under a wavefront plan, then a work-group plan at
    # another level: the 32-phase table follows the plan
    fd, f = _fractal(N, "triangle", 9, 4, N.STRATEGY_TILED_WAVE)
    o = O.Fractal(fd.s, fd.offsets, 9)
    s0 = o.init_compact(3, 0.5)
    want = packed_of(o.compact_steps(s0, W.rule_mask("B3/S23"), 4))
    for strategy, m in ((N.STRATEGY_TILED_WAVE, 4), (N.STRATEGY_TILED, 7), (N.STRATEGY_TILED, 2)):
        f.configure(strategy, m)
        a = f.pack(torch.from_numpy(s0).cuda())
        res = f.step_packed(a, torch.zeros_like(a), 4)
        np.testing.assert_array_equal(host(res), want, err_msg=f"strategy {strategy} m={m}")


def test_step_packed_triangle_r16_equals_byte_step(N):
    # the full-size triangle: packed and byte steps from the same state agree
    # bit for bit after 5 generations
    wl = W.LARGE_TRIANGLE
    fd = wl.fractal
    f = N.Fractal(fd.s, fd.offsets, wl.r)
    s0 = f.init_compact(wl.seeds[0], wl.p)
    a = f.pack(s0)
    res_p = f.step_packed(a, torch.zeros_like(a), 5)
    res_b = f.step_compact(s0.clone(), torch.empty_like(s0), 5)
    assert torch.equal(f.unpack(res_p), res_b)
    assert torch.equal(f.pack(res_b), res_p)


@pytest.mark.parametrize("name,r", [("triangle", 12), ("carpet", 6), ("hfractal", 6)])
def test_step_packed_random_fractals_and_sizes_vs_byte_step(N, name, r):
    fd = W.FRACTALS[name]
    f = N.Fractal(fd.s, fd.offsets, r)
    s0 = f.init_compact(9, 0.4)
    for rule in ("B3/S23", "vN:B2/S12"):
        rm = W.rule_mask(rule)
        res_p = f.step_packed(f.pack(s0), torch.zeros(f.packed_bytes(), dtype=torch.uint8, device="cuda"), 7, rm)
        res_b = f.step_compact(s0.clone(), torch.empty_like(s0), 7, rm)
        assert torch.equal(f.unpack(res_p), res_b), rule


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_step_packed_random_nbb_fractals_vs_oracle(N, seed):
    fd = W.random_fractal(700 + seed)
    r = 1
    while fd.k ** (r + 1) <= 30000 and r < 10:
        r += 1
    f = N.Fractal(fd.s, fd.offsets, r)
    if f.info().strategy == N.STRATEGY_DIRECT:
        pytest.skip("no tiled plan for this fractal")
    o = O.Fractal(fd.s, fd.offsets, r)
    s0 = o.init_compact(seed, 0.5)
    rm = W.rule_mask("B36/S23")
    res = f.step_packed(f.pack(torch.from_numpy(s0).cuda()), torch.zeros(f.packed_bytes(), dtype=torch.uint8,
                                                                         device="cuda"), 5, rm)
    np.testing.assert_array_equal(host(res), packed_of(o.compact_steps(s0, rm, 5)), err_msg=str(fd))


def test_packed_rejects_bad_arguments(N):
    f = N.Fractal(2, W.TRIANGLE.offsets, 6)
    n = f.packed_bytes()
    a = torch.zeros(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(N.NbbError, match="len"):
        f.step_packed(a[:n - 4], torch.zeros(n - 4, dtype=torch.uint8, device="cuda"), 1)
    with pytest.raises(N.NbbError, match="overlap"):
        f.step_packed(a, a, 1)
    big = torch.zeros(2 * n + 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(N.NbbError, match="aligned"):
        f.step_packed(big[1:n + 1], big[n + 8:2 * n + 8], 1)
    with pytest.raises(N.NbbError, match="bits outside"):
        f.step_packed(a, torch.zeros_like(a), 1, rule=1 << 9)
    d = N.Fractal(5, ((2, 0), (0, 2), (2, 2), (4, 2), (2, 4), (1, 1)), 2)   # no tiled plan (s = 5)
    with pytest.raises(N.NbbError, match="tiled plan"):
        d.pack(d.new_compact(), out=torch.zeros(d.packed_bytes(), dtype=torch.uint8, device="cuda"))
    assert f.step_packed(a, torch.zeros_like(a), 0) is a


@pytest.mark.parametrize("name,r", [("triangle", 8), ("carpet", 4)])
def test_step_packed_in_a_captured_graph(N, name, r):
    # after a first call (which builds the plan's 32-phase table) the packed
    # step only enqueues kernels, so it can be captured; every replay, with
    # eager work in between, must give the oracle's result
    fd = W.FRACTALS[name]
    f = N.Fractal(fd.s, fd.offsets, r)
    o = O.Fractal(fd.s, fd.offsets, r)
    s0 = o.init_compact(31, 0.5)
    want = packed_of(o.compact_steps(s0, W.rule_mask("B3/S23"), 4))
    a0 = f.pack(torch.from_numpy(s0).cuda())
    a, b = a0.clone(), torch.zeros_like(a0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        f.step_packed(a, b, 2)           # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        res = f.step_packed(a, b, 4)
    assert res is a
    other = f.pack(f.init_compact(5, 0.5))
    for rep in range(4):
        a.copy_(a0)
        graph.replay()
        f.step_packed(other, torch.zeros_like(other), 3)   # eager work between replays
        np.testing.assert_array_equal(host(a), want, err_msg=f"replay {rep}")
