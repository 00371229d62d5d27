"""Pins for the CPU oracle: each test checks the oracle against something other
than itself -- values printed in the paper, published known answers, closed
forms, textbook special cases, a library routine (scipy's 2D convolution), an
independent set-based construction (oracle/brute.py) or an exact invariant.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy.signal import convolve2d

from oracle import brute
from oracle import oracle as O
from paper_2110_12952_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
B3S23 = W.rule_mask("B3/S23")

SMALL_FRACTALS = ["triangle", "carpet", "hfractal", "chandelier", "fullsquare", "vicsek",
                  "xfractal", "cantordust", "cantor", "single", "grid4_12"]


def frac(name, r):
    f = W.FRACTALS[name]
    return O.Fractal(f.s, f.offsets, r)


def max_level(name, limit_cells=1 << 14):
    f = W.FRACTALS[name]
    r = 0
    while (f.s ** (r + 1)) ** 2 <= limit_cells * 16 and r < 8:
        r += 1
    return r


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


# ---------------------------------------------------------------- generator --
def test_splitmix64_known_answers():
    rows = read_golden("splitmix64_seed1234567.txt")
    seed = int(rows[0].split()[1])
    for row in rows[1:]:
        key, val = (int(v) for v in row.split())
        assert O.splitmix64(seed, key) == val


def test_threshold_integer():
    assert O.threshold(0.0) == 0
    assert O.threshold(1.0) == 1 << 24
    assert O.threshold(0.5) == 1 << 23
    assert O.threshold(0.3) == 5033164  # floor(0.3 * 16777216) = floor(5033164.8)


# ---------------------------------------------------------- fractal geometry --
def test_table1_hausdorff_dimensions():
    for row in read_golden("table1_hausdorff.txt"):
        name, k, s, printed = row.split()
        f = W.FRACTALS[name]
        assert (f.k, f.s) == (int(k), int(s))
        assert round(math.log(f.k) / math.log(f.s), 2) == float(printed)


@pytest.mark.parametrize("name", SMALL_FRACTALS)
def test_member_count_is_k_pow_r(name):
    # eq. (1): the fractal occupies k^r cells.
    for r in range(0, max_level(name) + 1):
        f = frac(name, r)
        assert int(f.member_mask().sum()) == f.k ** r


def test_triangle_closed_form():
    # Sierpinski triangle with offsets (0,0),(1,0),(0,1): member <=> x & y == 0.
    for r in range(0, 10):
        f = frac("triangle", r)
        y, x = np.mgrid[0:f.n, 0:f.n]
        np.testing.assert_array_equal(f.member_mask(), ((x & y) == 0).astype(np.uint8))


def test_fullsquare_is_whole_box():
    for r in range(0, 7):
        assert frac("fullsquare", r).member_mask().all()


@pytest.mark.parametrize("name", SMALL_FRACTALS)
def test_digit_membership_matches_construction(name):
    # The digit test against the NBB construction of section 1 (replicas of
    # the previous level, translated by o_j s^rho), which uses no digits.
    fd = W.FRACTALS[name]
    for r in range(0, min(max_level(name), 5) + 1):
        f = frac(name, r)
        m = np.zeros((f.n, f.n), dtype=np.uint8)
        for (x, y) in brute.member_set(fd.s, fd.offsets, r):
            m[y, x] = 1
        np.testing.assert_array_equal(f.member_mask(), m)


@pytest.mark.parametrize("seed", range(12))
def test_random_fractals_membership_and_order(seed):
    fd = W.random_fractal(seed)
    r = 1
    while fd.k ** (r + 1) <= 4096 and (fd.s ** (r + 1)) ** 2 <= 1 << 16 and r < 5:
        r += 1
    f = O.Fractal(fd.s, fd.offsets, r)
    order = brute.build_levels(fd.s, fd.offsets, r)
    xs, ys = f.lam_many(np.arange(f.cells))
    assert list(zip(xs.tolist(), ys.tolist())) == order
    assert int(f.member_mask().sum()) == fd.k ** r


# ------------------------------------------------------------------ the maps --
@pytest.mark.parametrize("name", SMALL_FRACTALS)
def test_lambda_follows_construction_order(name):
    fd = W.FRACTALS[name]
    for r in range(0, min(max_level(name), 5) + 1):
        f = frac(name, r)
        xs, ys = f.lam_many(np.arange(f.cells))
        assert list(zip(xs.tolist(), ys.tolist())) == brute.build_levels(fd.s, fd.offsets, r)


def _morton_decode(i):
    # Textbook Z-order decode: even bits -> x, odd bits -> y.
    x = y = 0
    b = 0
    while i >> (2 * b):
        x |= ((i >> (2 * b)) & 1) << b
        y |= ((i >> (2 * b + 1)) & 1) << b
        b += 1
    return x, y


def test_fullsquare_lambda_is_morton():
    for r in range(0, 7):
        f = frac("fullsquare", r)
        xs, ys = f.lam_many(np.arange(f.cells))
        for i in range(f.cells):
            assert (xs[i], ys[i]) == _morton_decode(i)


@pytest.mark.parametrize("name", SMALL_FRACTALS)
def test_nu_inverts_lambda_and_rejects_the_rest(name):
    for r in range(0, min(max_level(name), 4) + 1):
        f = frac(name, r)
        idx = np.arange(f.cells)
        xs, ys = f.lam_many(idx)
        np.testing.assert_array_equal(f.nu_many(xs, ys), idx)  # nu(lambda(i)) = i
        # every coordinate of the box plus the ring around it
        yy, xx = np.mgrid[-1:f.n + 1, -1:f.n + 1]
        nu = f.nu_many(xx.ravel(), yy.ravel())
        inside = (xx.ravel() >= 0) & (yy.ravel() >= 0) & (xx.ravel() < f.n) & (yy.ravel() < f.n)
        mask = np.zeros(nu.shape, dtype=bool)
        mask[inside] = f.member_mask()[yy.ravel()[inside], xx.ravel()[inside]].astype(bool)
        assert (nu[~mask] == -1).all()
        got = nu[mask]
        lx, ly = f.lam_many(got)                 # lambda(nu(p)) = p on members
        np.testing.assert_array_equal(lx, xx.ravel()[mask])
        np.testing.assert_array_equal(ly, yy.ravel()[mask])
        assert sorted(got.tolist()) == list(range(f.cells))


def test_triangle_r2_worked_example():
    f = frac("triangle", 2)
    for row in read_golden("triangle_r2_map.txt"):
        i, x, y, px, py = (int(v) for v in row.split())
        assert f.lam(i) == (x, y)
        assert f.nu(x, y) == i
        assert f.nu_paper2d(x, y) == (px, py)


def test_printed_triangle_H_is_not_injective():
    # Eq. (2) as printed adds the two digit bits, so (1,0) and (0,1) share an
    # id; the oracle instead uses the position of the digit pair in the
    # offset list (the look-up-table form of H that section 3.1 allows).
    def printed_H(x, y, mu):
        return (x % 2 ** (mu + 1)) // 2 ** mu + (y % 2 ** (mu + 1)) // 2 ** mu
    assert printed_H(1, 0, 0) == printed_H(0, 1, 0) == 1
    f = frac("triangle", 1)
    assert f.nu(1, 0) != f.nu(0, 1)


@pytest.mark.parametrize("name", ["triangle", "carpet", "hfractal", "chandelier", "vicsek",
                                  "cantor", "grid4_12"])
def test_paper2d_is_the_unfolding(name):
    # Section 3: the compact space starts as one cell and at each new level
    # the whole current compact space is copied k times, to the right when the
    # new level is odd and downwards when it is even.  Check eqs. (3)-(8)
    # (read with floor(mu/2)) against that recursive description.
    fd = W.FRACTALS[name]
    prev = {(0, 0): (0, 0)}    # level 0: the single cell at compact (0,0)
    W_, H_ = 1, 1
    for r in range(1, min(max_level(name), 5) + 1):
        cur = {}
        scale = fd.s ** (r - 1)
        for j, (ox, oy) in enumerate(fd.offsets):
            for (x, y), (cx, cy) in prev.items():
                if r % 2 == 1:
                    cur[(x + ox * scale, y + oy * scale)] = (cx + j * W_, cy)
                else:
                    cur[(x + ox * scale, y + oy * scale)] = (cx, cy + j * H_)
        if r % 2 == 1:
            W_ *= fd.k
        else:
            H_ *= fd.k
        f = frac(name, r)
        assert (W_, H_) == (fd.k ** ((r + 1) // 2), fd.k ** (r // 2))
        for (x, y), c in cur.items():
            assert f.nu_paper2d(x, y) == c
        assert sorted(cur.values()) == sorted((a, b) for a in range(W_) for b in range(H_))
        prev = cur


def test_paper2d_coincides_with_canonical_up_to_level_2():
    for name in ["triangle", "carpet", "hfractal"]:
        for r in range(0, 3):
            f = frac(name, r)
            Wd = f.k ** ((r + 1) // 2)
            for i in range(f.cells):
                px, py = f.nu_paper2d(*f.lam(i))
                assert py * Wd + px == i
    f = frac("triangle", 3)
    px, py = f.nu_paper2d(*f.lam(3))
    assert (f.lam(3), (px, py), py * 9 + px) == ((2, 0), (0, 1), 9)


# --------------------------------------------------------------- automaton --
def _scipy_step(mask, state, rule):
    ker = np.ones((3, 3), dtype=np.int64)
    ker[1, 1] = 0
    live = (state.astype(np.int64) * mask)
    cnt = convolve2d(live, ker, mode="same", boundary="fill", fillvalue=0)
    idx = cnt + 16 * (live > 0)
    nxt = (rule >> idx) & 1
    return (nxt * mask).astype(np.uint8)


@pytest.mark.parametrize("name", SMALL_FRACTALS)
@pytest.mark.parametrize("rule", ["B3/S23", "B36/S23", "B2/S", "B1357/S02468"])
def test_bbox_step_matches_library_convolution(name, rule):
    fd = W.FRACTALS[name]
    r = min(max_level(name), 5)
    f = frac(name, r)
    mask = f.member_mask()
    st = f.init_bbox(seed=7 + r, p=0.45)
    rm = W.rule_mask(rule)
    ref = st.copy()
    for _ in range(3):
        ref = _scipy_step(mask, ref, rm)
    np.testing.assert_array_equal(f.bbox_steps(st, rm, 3), ref)


def _parse_patterns():
    pats, cur = [], None
    for row in read_golden("gol_patterns.txt"):
        if row.startswith("pattern"):
            parts = row.split()
            cur = {"name": parts[1], "period": int(parts[3]), "rows": [],
                   "shift": (int(parts[5]), int(parts[6])) if "shift" in parts else (0, 0)}
            pats.append(cur)
        else:
            cur["rows"].append(row)
    return pats


@pytest.mark.parametrize("pat", _parse_patterns(), ids=lambda p: p["name"])
def test_fullsquare_textbook_patterns(pat):
    f = frac("fullsquare", 4)  # 16 x 16 box, plain Life with dead border
    box = np.zeros((16, 16), dtype=np.uint8)
    for yy, row in enumerate(pat["rows"]):
        for xx, ch in enumerate(row):
            box[4 + yy, 4 + xx] = ch == "O"
    after = f.expand(f.compact_steps(f.gather(box), B3S23, pat["period"]))
    want = np.roll(np.roll(box, pat["shift"][1], axis=0), pat["shift"][0], axis=1)
    np.testing.assert_array_equal(after, want)
    if pat["period"] > 1:
        assert not np.array_equal(f.bbox_steps(box, B3S23, 1), box)


@pytest.mark.parametrize("name", SMALL_FRACTALS)
@pytest.mark.parametrize("rule", ["B3/S23", "B1357/S1357", "B36/S23", "vN:B2/S12", "vN:B13/S13"])
def test_compact_procedure_matches_box_definition(name, rule):
    # The paper's compact stencil procedure (lambda, neighbour coordinates,
    # nu, read) against the automaton on the box, gathered through lambda.
    r = min(max_level(name), 5)
    f = frac(name, r)
    st = f.init_bbox(seed=99, p=0.4)
    rm = W.rule_mask(rule)
    for steps in (1, 4):
        np.testing.assert_array_equal(f.compact_steps(f.gather(st), rm, steps),
                                      f.gather(f.bbox_steps(st, rm, steps)))


@pytest.mark.parametrize("name", SMALL_FRACTALS)
@pytest.mark.parametrize("rule", ["B3/S23", "vN:B2/S12"])
def test_compact_matches_set_brute_force(name, rule):
    fd = W.FRACTALS[name]
    spec = W.RULES[rule]
    for r in range(0, min(max_level(name), 3) + 1):
        f = frac(name, r)
        st = W.random_bits(seed=r + 3, count=f.cells, p=0.5)
        want = brute.run_compact(fd.s, fd.offsets, r, st.tolist(), spec[0], spec[1], 3,
                                 W.rule_neighbourhood(rule))
        assert f.compact_steps(st, W.rule_mask(rule), 3).tolist() == want


@pytest.mark.parametrize("name,r", [("triangle", 2), ("carpet", 1), ("hfractal", 1),
                                    ("chandelier", 2), ("cantor", 4), ("vicsek", 1),
                                    ("single", 3)])
def test_every_initial_state_one_step(name, r):
    fd = W.FRACTALS[name]
    f = frac(name, r)
    for rule in ("B3/S23", "vN:B2/S12"):
        spec = W.RULES[rule]
        for bits in itertools.product((0, 1), repeat=f.cells):
            st = np.array(bits, dtype=np.uint8)
            want = brute.run_compact(fd.s, fd.offsets, r, list(bits), spec[0], spec[1], 1,
                                     W.rule_neighbourhood(rule))
            assert f.compact_steps(st, W.rule_mask(rule), 1).tolist() == want, rule


@pytest.mark.parametrize("name,r", [("triangle", 6), ("carpet", 3), ("hfractal", 3),
                                    ("chandelier", 4)])
@pytest.mark.parametrize("rule", ["B1357/S1357", "B1357/S02468", "vN:B13/S13", "vN:B13/S024"])
def test_linear_rules_superpose(name, r, rule):
    # Both rules are linear over GF(2), so evolve(A xor B) = evolve(A) xor evolve(B).
    f = frac(name, r)
    rm = W.rule_mask(rule)
    a = W.random_bits(1, f.cells, 0.3)
    b = W.random_bits(2, f.cells, 0.6)
    for steps in (1, 5):
        np.testing.assert_array_equal(f.compact_steps(a ^ b, rm, steps),
                                      f.compact_steps(a, rm, steps) ^ f.compact_steps(b, rm, steps))


@pytest.mark.parametrize("name,r", [("triangle", 5), ("carpet", 3), ("hfractal", 3),
                                    ("chandelier", 3), ("cantor", 4)])
@pytest.mark.parametrize("rule", ["B1357/S1357", "vN:B13/S13"])
def test_single_cell_impulse_under_replicator(name, r, rule):
    f = frac(name, r)
    rm = W.rule_mask(rule)
    four = W.rule_neighbourhood(rule) == 4
    for i in range(0, f.cells, max(1, f.cells // 37)):
        st = np.zeros(f.cells, dtype=np.uint8)
        st[i] = 1
        x, y = f.lam(i)
        want = np.zeros(f.cells, dtype=np.uint8)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dx or dy) and not (four and dx and dy) and f.member(x + dx, y + dy):
                    want[f.nu(x + dx, y + dy)] = 1
        np.testing.assert_array_equal(f.compact_steps(st, rm, 1), want)


@pytest.mark.parametrize("rule,offsets", [
    ("vN:B13/S13", [(1, 0), (-1, 0), (0, 1), (0, -1)]),
    ("B1357/S1357", [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dx or dy])])
def test_parity_rule_doubles_the_neighbourhood(rule, offsets):
    # A parity rule is linear over GF(2) and its neighbourhood operator N
    # satisfies N^2 = N(2x) mod 2 (cross terms pair up), so a single live cell
    # in open space becomes, after 2^j generations, exactly the neighbourhood
    # scaled by 2^j.  Textbook closed form, on the full square far from its
    # edges.
    f = frac("fullsquare", 5)
    c = 16
    box = np.zeros((f.n, f.n), dtype=np.uint8)
    box[c, c] = 1
    st = f.gather(box)
    rm = W.rule_mask(rule)
    for j in range(4):
        out = f.expand(f.compact_steps(st, rm, 2 ** j))
        want = np.zeros_like(box)
        for dx, dy in offsets:
            want[c + dy * 2 ** j, c + dx * 2 ** j] = 1
        np.testing.assert_array_equal(out, want, err_msg=f"{rule} after {2 ** j} generations")


def test_all_dead_stays_dead():
    for name in ["triangle", "carpet", "hfractal"]:
        f = frac(name, 4)
        z = np.zeros(f.cells, dtype=np.uint8)
        assert not f.compact_steps(z, B3S23, 3).any()


# -------------------------------------------------------------------- init --
@pytest.mark.parametrize("name", ["triangle", "carpet", "hfractal", "chandelier", "cantor"])
def test_init_compact_is_gathered_box_init(name):
    f = frac(name, min(max_level(name), 6))
    for seed, p in [(1, 0.5), (12952, 0.3), (2**63 + 5, 0.77)]:
        np.testing.assert_array_equal(f.init_compact(seed, p), f.gather(f.init_bbox(seed, p)))


def test_init_recomputed_cells():
    f = frac("triangle", 6)
    st = f.init_bbox(12952, 0.3)
    thr = O.threshold(0.3)
    for (x, y) in [(0, 0), (5, 2), (17, 40), (63, 0), (1, 62)]:
        alive = ((x & y) == 0) and (O.splitmix64(12952, y * f.n + x) >> 40) < thr
        assert st[y, x] == int(alive)


@pytest.mark.parametrize("p", [0.3, 0.5])
def test_init_live_fraction(p):
    f = frac("triangle", 10)
    st = f.init_compact(3, p)
    n = f.cells
    assert abs(st.mean() - p) < 5 * math.sqrt(p * (1 - p) / n)


def test_init_extremes():
    f = frac("carpet", 4)
    assert not f.init_compact(5, 0.0).any()
    assert f.init_compact(5, 1.0).all()
    assert (f.init_bbox(5, 1.0) == f.member_mask()).all()


def test_init_threshold_boundary():
    # Alive iff top24 < floor(p 2^24): a cell whose draw equals the threshold
    # is dead, one above it alive.
    f = frac("triangle", 3)
    seed = 424242
    for (x, y) in [(0, 0), (3, 4), (7, 0)]:
        top = O.splitmix64(seed, y * f.n + x) >> 40
        assert f.init_bbox(seed, top / 2.0 ** 24)[y, x] == 0
        assert f.init_bbox(seed, (top + 1) / 2.0 ** 24)[y, x] == 1


@pytest.mark.parametrize("name", ["triangle", "carpet", "hfractal", "chandelier", "cantor"])
@pytest.mark.parametrize("rule", ["B3/S23", "vN:B2/S12"])
def test_cells_after_matches_full_steps(name, rule):
    f = frac(name, min(max_level(name), 5))
    st = f.init_compact(31, 0.5)
    rm = W.rule_mask(rule)
    idx = np.arange(0, f.cells, max(1, f.cells // 200))
    for steps in (0, 1, 2, 3):
        np.testing.assert_array_equal(f.cells_after(st, idx, rm, steps),
                                      f.compact_steps(st, rm, steps)[idx])


@pytest.mark.parametrize("name", ["triangle", "carpet", "hfractal", "chandelier"])
def test_cells_after_seeded_matches_full_steps(name):
    # the per-cell initial state is the whole-state init read at that cell,
    # and the light cone from it matches whole-state generations
    f = frac(name, min(max_level(name), 5))
    st = f.init_compact(77, 0.4)
    idx = np.arange(0, f.cells, max(1, f.cells // 300))
    for steps in (0, 1, 2, 3):
        np.testing.assert_array_equal(f.cells_after_seeded(77, 0.4, idx, B3S23, steps),
                                      f.compact_steps(st, B3S23, steps)[idx])
    with pytest.raises(IndexError):
        f.cells_after_seeded(77, 0.4, [f.cells], B3S23, 1)
