"""Host-side checks of libnbbfrac that need no GPU: the library loads and
exports what include/nbbfrac.h declares, argument validation, and the tile
plan tables against the oracle."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_12952_amd import nbbfrac as N
from paper_2110_12952_amd import workloads as W


def test_library_exports_every_declared_symbol():
    L = N.lib()
    names = N.header_symbols()
    assert len(names) >= 17
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    L = N.lib()
    for code, name in N.STATUS_NAMES.items():
        assert L.nbb_status_string(code).decode() == name


def _create(k, s, offsets, r):
    L = N.lib()
    h = ctypes.c_void_p()
    arr = np.ascontiguousarray(offsets, dtype=np.int32) if offsets is not None else None
    st = L.nbb_create(k, s, arr.ctypes.data if arr is not None else None, r, ctypes.byref(h))
    if st == N.NBB_OK:
        L.nbb_destroy(h)
    return st, L.nbb_last_error().decode()


@pytest.mark.parametrize("k,s,offsets,r,why", [
    (0, 2, [0, 0], 3, "k=0"),
    (1, 1, [0, 0], 3, "s<2"),
    (1, 17, [0, 0], 3, "s>16"),
    (5, 2, [0, 0, 1, 0, 0, 1, 1, 1, 0, 0], 3, "k>s^2"),
    (2, 2, [0, 0, 2, 0], 3, "offset out of range"),
    (2, 2, [0, 0, -1, 0], 3, "negative offset"),
    (2, 2, [0, 1, 0, 1], 3, "duplicate offset"),
    (2, 2, None, 3, "null offsets"),
])
def test_create_rejects_invalid(k, s, offsets, r, why):
    st, msg = _create(k, s, offsets, r)
    assert st == N.NBB_E_INVALID, why
    assert msg


@pytest.mark.parametrize("k,s,offsets,r", [
    (3, 2, [0, 0, 1, 0, 0, 1], 21),     # 3^21 > 2^32 - 1
    (1, 2, [1, 1], 31),                 # n = 2^31 does not fit int32 coordinates
    (8, 3, [0, 0, 1, 0, 2, 0, 0, 1, 2, 1, 0, 2, 1, 2, 2, 2], 11),  # 8^11 = 2^33
])
def test_create_rejects_too_large(k, s, offsets, r):
    st, msg = _create(k, s, offsets, r)
    assert st == N.NBB_E_RANGE
    assert "large" in msg


def test_create_null_out():
    L = N.lib()
    arr = np.array([0, 0, 1, 0, 0, 1], dtype=np.int32)
    assert L.nbb_create(3, 2, arr.ctypes.data, 4, None) == N.NBB_E_INVALID


def test_create_without_device_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, msg = _create(3, 2, [0, 0, 1, 0, 0, 1], 4)
    assert st == N.NBB_E_DEVICE


def test_null_descriptor_calls():
    L = N.lib()
    assert L.nbb_query(None, ctypes.byref(N.Info())) == N.NBB_E_INVALID
    assert L.nbb_configure(None, 0, 0) == N.NBB_E_INVALID
    assert L.nbb_step_compact(None, None, None, 0, 1, N.NBB_RULE_B3S23, None, None) == N.NBB_E_INVALID
    assert L.nbb_bbox_pitch(None) == 0
    L.nbb_destroy(None)


# ----------------------------------------------------------------- tile plan --
PLAN_CASES = [("triangle", r) for r in (1, 2, 4, 7, 9)] + \
             [("carpet", r) for r in (1, 2, 4)] + [("hfractal", r) for r in (1, 3, 4)] + \
             [("chandelier", r) for r in (2, 4)] + [("fullsquare", 5), ("vicsek", 3), ("cantor", 4),
                                                    ("single", 5), ("grid4_12", 3), ("xfractal", 3)]


def _plan_levels(name, r):
    f = W.FRACTALS[name]
    levels = [0]
    for m in range(1, r + 1):
        if f.s ** m <= 250:
            levels.append(m)
    return levels


@pytest.mark.parametrize("name,r", PLAN_CASES)
def test_plan_tables_match_oracle(name, r):
    fd = W.FRACTALS[name]
    for m in _plan_levels(name, r):
        p = N.plan_tables(fd.s, fd.offsets, r, m)
        m = p["tile_level"]
        S, Wp, rows = p["tile_side"], p["box_pitch"], p["box_rows"]
        assert S == fd.s ** m and p["tile_cells"] == fd.k ** m and p["tiles"] == fd.k ** (r - m)
        fm = O.Fractal(fd.s, fd.offsets, m)
        xs, ys = fm.lam_many(np.arange(fm.cells))
        np.testing.assert_array_equal(p["lut0"], (ys + 1) * Wp + (xs + 1))
        q, BS = p["block_level"], p["block_side"]
        assert BS == fd.s ** q and q in (1, 2) and q <= m
        fb = O.Fractal(fd.s, fd.offsets, m - q)
        bx, by = fb.lam_many(np.arange(fb.cells))
        np.testing.assert_array_equal(p["lut1"], by * BS * Wp + bx * BS)
        # the box holds every block window (BS+2 rows from row Y*BS, two
        # dwords per row from column (X*BS) & ~3) and nothing beyond
        assert rows == (by * BS + BS + 2).max() and rows <= S + 2
        assert Wp % 4 == 0 and Wp >= ((bx * BS) & ~3).max() + 8 and (ys + 2).max() <= rows
        # halo: every member of each neighbouring level-m copy that lands in
        # the ring [-1, S]^2 around the tile and inside the box, with its
        # local index
        want = set()
        d8 = 0
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == 0 and dy == 0:
                    continue
                for i in range(fm.cells):
                    tx, ty = xs[i] + dx * S, ys[i] + dy * S
                    if -1 <= tx <= S and -1 <= ty <= S and ty + 1 < rows and tx + 1 < Wp:
                        assert fm.nu(xs[i], ys[i]) == i
                        want.add(((d8 << 29) | i, (ty + 1) * Wp + (tx + 1)))
                d8 += 1
        got = set(zip(p["halo_src"].tolist(), p["halo_dst"].tolist()))
        assert got == want
        assert len(got) == p["halo_count"]
        # neighbour tiles: the tile whose block is next to tile t's in direction d
        fc = O.Fractal(fd.s, fd.offsets, r - m)
        cx, cy = fc.lam_many(np.arange(fc.cells))
        dirs = [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dx or dy]
        want_nbr = np.stack([fc.nu_many(cx + dx, cy + dy) for dx, dy in dirs], axis=1).ravel()
        np.testing.assert_array_equal(p["nbr"].astype(np.int64), np.where(want_nbr < 0, 2**32 - 1, want_nbr))


@pytest.mark.parametrize("name", ["triangle", "carpet", "hfractal", "chandelier", "vicsek", "grid4_12"])
def test_tile_decomposition_identity(name):
    # lambda(i) = s^m lambda_{r-m}(i div k^m) + lambda_m(i mod k^m): the fact the
    # tiled step rests on (every aligned run of k^m indices is one level-m copy).
    fd = W.FRACTALS[name]
    r = 4 if fd.s > 2 else 6
    fr = O.Fractal(fd.s, fd.offsets, r)
    xs, ys = fr.lam_many(np.arange(fr.cells))
    for m in range(0, r + 1):
        fm, fc = O.Fractal(fd.s, fd.offsets, m), O.Fractal(fd.s, fd.offsets, r - m)
        i = np.arange(fr.cells)
        cx, cy = fc.lam_many(i // fm.cells)
        lx, ly = fm.lam_many(i % fm.cells)
        np.testing.assert_array_equal(xs, fd.s ** m * cx + lx)
        np.testing.assert_array_equal(ys, fd.s ** m * cy + ly)


def test_plan_rejects_unsupported():
    with pytest.raises(N.NbbError):
        N.plan_tables(5, [(0, 0), (1, 1)], 3)       # s = 5: no tiled step
    with pytest.raises(N.NbbError):
        N.plan_tables(2, [(0, 0), (1, 0), (0, 1)], 4, 5)  # m > r
    with pytest.raises(N.NbbError):
        N.plan_tables(2, [(0, 0), (1, 0), (0, 1)], 10, 8)  # box too large for 16-bit offsets


def test_auto_tile_levels_for_the_workloads():
    got = {w.name: N.plan_tables(w.fractal.s, w.fractal.offsets, w.r)["tile_level"]
           for w in W.WORKLOADS.values()}
    assert got["triangle_r16"] == 7 and got["carpet_r9"] == 4 and got["hfractal_r10"] == 4


def test_batch_workload_items_are_seeded():
    items = W.BATCH512.items()
    assert len(items) == 512 and items == W.BATCH512.items()
    for it in items:
        assert 1e3 <= it.cells <= 1e7 and 0.2 <= it.p <= 0.6
        assert it.r in W.BATCH_LEVELS[it.fractal.name]
    assert [it.seed for it in items] == list(range(512))
    assert {it.fractal.name for it in items} == set(W.BATCH_LEVELS)


def test_pack_offsets():
    offs, total = N.pack_offsets([1, 16, 17, 0, 5])
    assert offs == [0, 16, 32, 64, 64] and total == 80
    assert all(o % 16 == 0 for o in offs)
    assert N.pack_offsets([]) == ([], 16)


def test_batch_create_without_device_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = N.lib()
    h = ctypes.c_void_p()
    assert L.nbb_batch_create(None, None, 0, None, ctypes.byref(h)) == N.NBB_E_DEVICE
    assert L.nbb_batch_create(None, None, 0, None, None) == N.NBB_E_INVALID
    # flags are checked before the device is
    assert L.nbb_batch_create_ex(None, None, 0, N.NBB_BATCH_RESIDENT, None, ctypes.byref(h)) == N.NBB_E_DEVICE
    for bad in (N.NBB_BATCH_RESIDENT | N.NBB_BATCH_NO_RESIDENT, 4, 1 << 31):
        assert L.nbb_batch_create_ex(None, None, 0, bad, None, ctypes.byref(h)) == N.NBB_E_INVALID
    assert "flags" in L.nbb_last_error().decode()
    assert L.nbb_batch_step(None, None, None, 0, 1, N.NBB_RULE_B3S23, None, None) == N.NBB_E_INVALID
    assert L.nbb_batch_query(None, None) == N.NBB_E_INVALID
    L.nbb_batch_destroy(None)
    assert L.nbb_autotune(None, None, None, 0, 1, 0, None, None) == N.NBB_E_INVALID


# ------------------------------------------------------ request-loop host logic --
def test_arena_allocator_first_fit_and_merge():
    from paper_2110_12952_amd.serve import ArenaAllocator
    a = ArenaAllocator(1000)          # rounded down to 992
    assert a.capacity == 992
    x = a.alloc(10)
    y = a.alloc(17)
    z = a.alloc(100)
    assert (x, y, z) == (0, 16, 48) and a.used_bytes == 16 + 32 + 112
    a.free(y)
    assert a.alloc(16) == 16            # first fit reuses the hole
    a.free(16)
    a.free(x)
    a.free(z)
    a.check()
    assert a.alloc(992) == 0 and a.alloc(1) is None


def test_arena_allocator_random_churn():
    from paper_2110_12952_amd.serve import ArenaAllocator
    rng = np.random.default_rng(3)
    a = ArenaAllocator(1 << 16)
    live = {}
    for it in range(3000):
        if live and rng.random() < 0.45:
            off = list(live)[int(rng.integers(len(live)))]
            a.free(off)
            del live[off]
        else:
            n = int(rng.integers(1, 3000))
            off = a.alloc(n)
            if off is not None:
                assert off % 16 == 0 and off + n <= a.capacity
                for o, m in live.items():
                    assert off + n <= o or o + m <= off
                live[off] = n
        if it % 100 == 0:
            a.check()
    for off in list(live):
        a.free(off)
    a.check()
    assert a.used_bytes == 0 and a.alloc(a.capacity) == 0


def test_plan_round():
    from paper_2110_12952_amd.serve import plan_round
    order, G = plan_round([5, 50, 20], [100, 100, 100], 3000, 64)
    assert order == [1, 2, 0] and G == 10
    assert plan_round([5, 50], [100, 100], 1e9, 64)[1] == 50        # capped by the largest remaining
    assert plan_round([500, 500], [100, 100], 1e9, 64)[1] == 64     # and by max_gens
    assert plan_round([500], [10 ** 9], 10, 64)[1] == 1             # at least one generation


def test_serve_workload_requests():
    wl = W.SERVE2000
    rq = wl.requests(5.0)
    assert rq == wl.requests(5.0)
    n = len(rq)
    assert abs(n - 5.0 * wl.rate) < 5 * np.sqrt(5.0 * wl.rate)       # Poisson count
    ts = np.array([q.t for q in rq])
    assert (np.diff(ts) > 0).all() and ts[-1] < 5.0
    gaps = np.diff(ts)
    assert abs(gaps.mean() * wl.rate - 1) < 0.05
    for q in rq[:2000]:
        assert q.fractal.name in wl.fractals and q.r in W.SERVE_LEVELS[q.fractal.name]
        assert 10 <= q.steps <= 2000 and q.p == 0.5 and q.seed == q.rid
    # snapping: every level of each fractal is reachable, and a level is the
    # nearest one to log10 of its cell count
    got = {(q.fractal.name, q.r) for q in rq}
    assert {(f, r) for f in wl.fractals for r in W.SERVE_LEVELS[f]
            if 3 - 0.5 <= r * np.log10(W.FRACTALS[f].k) <= 8 + 0.5} <= got
    st = np.log(np.array([q.steps for q in rq]))
    assert abs(st.mean() - (np.log(10) + np.log(2000)) / 2) < 0.05


def test_binding_fails_loudly_without_the_library(tmp_path):
    # no CPU fallback: with the library missing, every entry point raises
    import os
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2110_12952_amd import nbbfrac as N\n"
            "for call in (N.lib, lambda: N.Fractal(2, ((0, 0), (1, 0), (0, 1)), 4),\n"
            "             lambda: N.plan_tables(2, ((0, 0), (1, 0), (0, 1)), 4)):\n"
            "    try:\n"
            "        call()\n"
            "    except ImportError as e:\n"
            "        assert 'missing' in str(e)\n"
            "    else:\n"
            "        raise SystemExit('no error')\n"
            "print('raised')\n") % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, NBB_LIBRARY=str(tmp_path / "absent.so"))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "raised" in r.stdout, r.stdout + r.stderr
