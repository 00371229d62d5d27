"""The temporal-blocking plan (several generations per launch), checked on the
CPU.

The plan (box side and pitch, each tile cell's box position, the neighbour
cells within the ring and their positions, the neighbour tiles) is read
through nbb_temporal_plan_build and driven by a numpy model of the kernel's
data movement: per tile, its cells and the ring cells of the neighbour tiles
that exist are placed in a box with a member mask, the rule is applied to the
whole box `gens` times (dead outside the box, non-members forced dead), and
the tile's cells are read back.  For gens <= depth that must equal the
oracle's compact step for every fractal, level, depth and rule here; a wrong
position, a missing ring cell, a wrong neighbour tile or a ring too thin for
the generations fails it.  No GPU is involved.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_12952_amd import nbbfrac as N
from paper_2110_12952_amd import workloads as W

OUT = 0xFFFFFFFF


def box_steps(box, mask, rule, gens):
    """`gens` generations of the rule on a 2-D uint8 box (dead outside it)."""
    four = bool(rule >> 31)
    rule &= 0x1FF01FF
    for _ in range(gens):
        p = np.pad(box.astype(np.int32), 1)
        if four:
            n = p[:-2, 1:-1] + p[2:, 1:-1] + p[1:-1, :-2] + p[1:-1, 2:]
        else:
            n = sum(p[1 + dy:p.shape[0] - 1 + dy, 1 + dx:p.shape[1] - 1 + dx]
                    for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dy or dx)
        idx = n + 16 * box.astype(np.int32)
        box = (((rule >> idx) & 1).astype(np.uint8)) & mask
    return box


def model_step(T, state, rule, gens):
    K, B, P = T["K"], T["B"], T["P"]
    out = np.empty_like(state)
    for t in range(T["tiles"]):
        box = np.zeros(B * P, np.uint8)
        mask = np.zeros(B * P, np.uint8)
        box[T["self"]] = state[t * K:(t + 1) * K]
        mask[T["self"]] = 1
        w, off = T["halo"][0::2], T["halo"][1::2]
        nt = T["nbr"][t * 8 + (w >> 29)]
        ok = nt != OUT
        box[off[ok]] = state[nt[ok].astype(np.int64) * K + (w[ok] & 0x1FFFFFFF)]
        mask[off[ok]] = 1
        box = box_steps(box.reshape(B, P), mask.reshape(B, P), rule, gens).reshape(-1)
        out[t * K:(t + 1) * K] = box[T["self"]]
    return out


CASES = [
    ("triangle", 6, 3, 1), ("triangle", 6, 3, 8), ("triangle", 7, 4, 5), ("triangle", 5, 5, 32),
    ("carpet", 4, 2, 1), ("carpet", 4, 2, 9), ("carpet", 3, 3, 4),
    ("hfractal", 4, 2, 5), ("hfractal", 3, 1, 3),
    ("chandelier", 5, 3, 7), ("chandelier", 4, 2, 2),
    ("vicsek", 4, 2, 6), ("cantordust", 4, 2, 3), ("grid4_12", 3, 2, 4), ("fullsquare", 6, 3, 8),
]
RULES = ["B3/S23", "B36/S23", "B1357/S1357", "B1357/S02468", "B2/S", "B35/S0123456"]


@pytest.mark.parametrize("name,r,m,h", CASES)
def test_model_equals_oracle(name, r, m, h):
    fd = W.FRACTALS[name]
    T = N.temporal_plan_tables(fd.s, fd.offsets, r, m, h)
    assert T["tile_level"] == m and T["depth"] == h
    assert T["B"] == T["tile_side"] + 2 * h and T["P"] % 4 == 0 and T["P"] >= T["B"]
    # positions: the tile's own cells and the ring cells never share a box position
    pos = np.concatenate([T["self"], T["halo"][1::2]])
    assert np.unique(pos).size == pos.size and pos.max() < T["B"] * T["P"]
    o = O.Fractal(fd.s, fd.offsets, r)
    st = o.init_compact(1000 + r + m, 0.45)
    for i, rn in enumerate(RULES):
        rule = W.rule_mask(rn)
        for gens in sorted({1, h}):
            want = o.compact_steps(st, rule, gens)
            got = model_step(T, st, rule, gens)
            np.testing.assert_array_equal(got, want, err_msg=f"{name} r={r} m={m} h={h} {rn} gens={gens}")


@pytest.mark.parametrize("name,r,m,h", [("triangle", 6, 3, 4), ("carpet", 3, 2, 3), ("hfractal", 3, 2, 2)])
def test_four_cell_stencil(name, r, m, h):
    fd = W.FRACTALS[name]
    T = N.temporal_plan_tables(fd.s, fd.offsets, r, m, h)
    o = O.Fractal(fd.s, fd.offsets, r)
    st = o.init_compact(77, 0.5)
    for rn in ("vN:B13/S13", "vN:B2/S12"):
        rule = W.rule_mask(rn)
        np.testing.assert_array_equal(model_step(T, st, rule, h), o.compact_steps(st, rule, h), err_msg=rn)


def test_ring_too_thin_is_detected():
    # the model with more generations than the ring depth must go wrong
    # somewhere (the check above would catch a plan whose ring were too thin)
    fd = W.TRIANGLE
    T = N.temporal_plan_tables(fd.s, fd.offsets, 7, 3, 2)
    o = O.Fractal(fd.s, fd.offsets, 7)
    st = o.init_compact(5, 0.5)
    rule = W.rule_mask("B3/S23")
    assert not np.array_equal(model_step(T, st, rule, 6), o.compact_steps(st, rule, 6))


@pytest.mark.parametrize("m,h,why", [(0, 1, "tile level"), (8, 1, "tile level"), (3, 0, "depth"), (3, 9, "depth"),
                                     (7, 128, "LDS")])
def test_rejected(m, h, why):
    fd = W.TRIANGLE
    with pytest.raises(N.NbbError):
        N.temporal_plan_tables(fd.s, fd.offsets, 7, m, h)
