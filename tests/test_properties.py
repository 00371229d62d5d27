"""Property tests (hypothesis) over random NBB fractals: s in 2..4, k in
1..s^2 distinct replica offsets in random order, small levels.  They check
the oracle against facts that hold for every NBB fractal (section 1: |F_r| =
k^r; section 3: nu inverts lambda on the fractal and rejects every other
point), the tile decomposition the tiled step rests on (a level-m tile is a
copy of F_m at s^m lambda_{r-m}(tile)), and the library's host-side tile plan
(no GPU) against the oracle's lambda.  CPU only.
"""
import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2110_12952_amd import nbbfrac as N  # noqa: E402


@st.composite
def fractals(draw, max_cells=5000):
    s = draw(st.integers(2, 4))
    k = draw(st.integers(1, s * s))
    cells = draw(st.permutations(list(range(s * s))))[:k]
    offsets = tuple((c % s, c // s) for c in cells)
    rmax = 1
    while k ** (rmax + 1) <= max_cells and rmax < 6:
        rmax += 1
    r = draw(st.integers(0, rmax))
    return s, offsets, r


@settings(max_examples=60, deadline=None)
@given(fractals())
def test_member_count_and_maps_are_inverse(f):
    s, offsets, r = f
    o = O.Fractal(s, offsets, r)
    assert o.cells == len(offsets) ** r
    xs, ys = o.lam_many(np.arange(o.cells))
    # lambda lands on distinct members of [0, n)^2
    assert xs.min() >= 0 and ys.min() >= 0 and xs.max() < o.n and ys.max() < o.n
    assert len(set(zip(xs.tolist(), ys.tolist()))) == o.cells
    np.testing.assert_array_equal(o.nu_many(xs, ys), np.arange(o.cells))
    # every other point of the box and its ring is outside
    yy, xx = np.mgrid[-1:o.n + 1, -1:o.n + 1]
    idx = o.nu_many(xx.ravel(), yy.ravel())
    assert (idx >= 0).sum() == o.cells and (idx[idx < 0] == -1).all()


@settings(max_examples=60, deadline=None)
@given(fractals(), st.data())
def test_tile_decomposition(f, data):
    s, offsets, r = f
    if r == 0:
        return
    m = data.draw(st.integers(0, r))
    o, om, oc = O.Fractal(s, offsets, r), O.Fractal(s, offsets, m), O.Fractal(s, offsets, r - m)
    i = np.arange(o.cells)
    K = len(offsets) ** m
    x, y = o.lam_many(i)
    tx, ty = oc.lam_many(i // K)
    lx, ly = om.lam_many(i % K)
    np.testing.assert_array_equal(x, s ** m * tx + lx)
    np.testing.assert_array_equal(y, s ** m * ty + ly)


@settings(max_examples=40, deadline=None)
@given(fractals(max_cells=20000), st.data())
def test_host_tile_plan_places_cells_and_blocks_by_lambda(f, data):
    s, offsets, r = f
    if r == 0:
        return
    m = data.draw(st.integers(1, r))
    try:
        p = N.plan_tables(s, offsets, r, m)
    except N.NbbError:
        return  # a level the tiled step does not take (box or block limits)
    m = p["tile_level"]
    S, Wp = p["tile_side"], p["box_pitch"]
    fm = O.Fractal(s, offsets, m)
    xs, ys = fm.lam_many(np.arange(fm.cells))
    np.testing.assert_array_equal(p["lut0"], (ys + 1) * Wp + (xs + 1))
    q, BS = p["block_level"], p["block_side"]
    fb = O.Fractal(s, offsets, m - q)
    bx, by = fb.lam_many(np.arange(fb.cells))
    np.testing.assert_array_equal(p["lut1"], by * BS * Wp + bx * BS)
    assert S == s ** m and p["tiles"] == len(offsets) ** (r - m)
