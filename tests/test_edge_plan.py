"""The edge-record form's host plan, checked on the CPU.

The plan (neighbour records, halo items, v_perm selectors) is read through
nbb_plan_build and driven by a numpy model of the kernel's data movement:
every block's bytes are loaded as the kernel loads them (the aligned 8-byte
window holding them, or the window ending at the state's end, moved down to
the block's first byte; blocks of 4, 8 or 16 cells read whole), turned
into rows and edge records with the plan's selectors, the records numbered
per tile as the kernel numbers them (blocks, then halo items, then one of
zeros), each block's window read back from its own rows and the neighbouring
records named by the plan, and the rule applied to four positions per dword as
the kernel does.  One generation of that model must equal the oracle's step
for every fractal, level and rule here; a wrong neighbour record, a missing
halo block, a bad selector or shift fails it.  No GPU is involved.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_12952_amd import nbbfrac as N
from paper_2110_12952_amd import workloads as W

U32 = np.uint32


def vperm(src0, src1, sel):
    """v_perm_b32 on uint32 arrays: byte i of the result is chosen by byte i
    of sel from the eight bytes src1 (0-3) : src0 (4-7); 8-11 give the sign
    of bytes 1, 3, 5, 7 spread over the byte, 12 gives 0, larger values 0xFF."""
    src0 = np.asarray(src0, np.uint64)
    src1 = np.asarray(src1, np.uint64)
    sel = np.asarray(sel, np.uint64)
    full = (src0 << np.uint64(32)) | src1
    out = np.zeros(np.broadcast(src0, src1, sel).shape, np.uint64)
    for i in range(4):
        s = (sel >> np.uint64(8 * i)) & np.uint64(0xFF)
        byte = (full >> (np.uint64(8) * np.minimum(s, 7))) & np.uint64(0xFF)
        sign_src = np.array([1, 3, 5, 7], np.uint64)[np.clip(s.astype(np.int64) - 8, 0, 3)]
        sign = np.where((full >> (np.uint64(8) * sign_src + np.uint64(7))) & np.uint64(1), np.uint64(0xFF),
                        np.uint64(0))
        v = np.where(s < 8, byte, np.where(s < 12, sign, np.where(s == 12, np.uint64(0), np.uint64(0xFF))))
        out |= v << np.uint64(8 * i)
    return out.astype(U32)


def sel4(a, b, c, d):
    return a | (b << 8) | (c << 16) | (d << 24)


def alignbyte(hi, lo, sh):
    v = (np.asarray(hi, np.uint64) << np.uint64(32)) | np.asarray(lo, np.uint64)
    return ((v >> np.uint64(8 * sh)) & np.uint64(0xFFFFFFFF)).astype(U32)


def window_bytes(p, BS, CB, nsrc):
    """The window the kernel reads a block through: 16 bytes for two source
    dwords and for the form compiled for the triangle's plan (4 x 4 blocks of
    9 cells, selector mask 0x6387), else 24."""
    sel = 0
    for i in range(4):
        sel |= int(p["edge_unpack"][i] != 0x0C0C0C0C) << i
        sel |= int(p["edge_unpack"][4 + i] != 0x0C0C0C0C) << (4 + i)
        sel |= int(p["edge_pack"][i] != 0x0C0C0C0C) << (8 + i)
        sel |= int(p["edge_pack"][4 + i] != 0x0C0C0C0C) << (12 + i)
    return 16 if (nsrc == 2 or (BS == 4 and CB == 9 and sel == 0x6387)) else 24


def load_blocks(state, offs, CB, nsrc, WB):
    """nsrc little-endian dwords of each block at byte offset offs, as the
    kernel assembles them: blocks of 4, 8 or 16 cells whole (the rest zero);
    others from the 8-byte aligned window of WB bytes at or below the block,
    or the window ending
    at the state's end when that one would pass it, moved down to the block's
    first byte (bytes past the window zero).  Every read stays inside the
    state (the state starts 16-byte aligned, so offsets and addresses agree
    modulo 8)."""
    n = offs.size
    out = np.zeros((n, 4 * nsrc), np.uint64)
    if n == 0:
        return np.zeros((0, nsrc), U32)
    if CB in (4, 8, 16):
        assert (offs % CB == 0).all() and offs.max() + CB <= state.size
        out[:, :CB] = state[offs[:, None] + np.arange(CB)[None, :]]
    else:
        s = offs - offs % 8
        s = np.where(s + WB > state.size, state.size - WB, s)
        assert s.min() >= 0 and (s + WB <= state.size).all()
        win = state[s[:, None] + np.arange(WB)[None, :]].astype(np.uint64)
        sh = offs - s
        take = np.minimum(4 * nsrc, WB - sh)
        for i in range(4 * nsrc):
            ok = i < take
            out[ok, i] = win[np.nonzero(ok)[0], sh[ok] + i]
    b = out.reshape(-1, nsrc, 4)
    return (b[..., 0] | (b[..., 1] << 8) | (b[..., 2] << 16) | (b[..., 3] << 24)).astype(U32)


def unpack(p, raw, BS):
    rows = []
    for r in range(BS):
        v = vperm(raw[:, 1], raw[:, 0], p["edge_unpack"][r])
        if p["edge_nsrc"] == 4:
            v |= vperm(raw[:, 3], raw[:, 2], p["edge_unpack"][4 + r])
        rows.append(v)
    return rows


def record(rows, BS):
    if BS == 4:
        l01 = vperm(rows[1], rows[0], sel4(0, 4, 12, 12))
        l23 = vperm(rows[3], rows[2], sel4(0, 4, 12, 12))
        left = vperm(l23, l01, sel4(0, 1, 4, 5))
        r01 = vperm(rows[1], rows[0], sel4(3, 7, 12, 12))
        r23 = vperm(rows[3], rows[2], sel4(3, 7, 12, 12))
        right = vperm(r23, r01, sel4(0, 1, 4, 5))
    else:
        l01 = vperm(rows[1], rows[0], sel4(0, 4, 12, 12))
        left = vperm(rows[BS - 1], l01, sel4(0, 1, 4, 12))
        r01 = vperm(rows[1], rows[0], sel4(2, 6, 12, 12))
        right = vperm(rows[BS - 1], r01, sel4(0, 1, 6, 12))
    return np.stack([rows[0], rows[BS - 1], left, right], axis=-1)


def model_step(fd, r, state, rule, m=0):
    """One generation of the edge-record kernel's data flow at tile level m
    (0: automatic), on the CPU."""
    p = N.plan_tables(fd.s, fd.offsets, r, m)
    assert p["edge_ok"]
    K, BS, nb, T = p["tile_cells"], p["block_side"], p["blocks"], int(p["tiles"])
    CB = fd.k ** p["block_level"]
    nsrc = p["edge_nsrc"]
    assert (BS, nsrc) in ((3, 2), (3, 4), (4, 4))  # the shapes the library instantiates
    assert CB <= 4 * nsrc
    nh = p["edge_halo_count"]
    nrec = p["edge_records"]
    assert nrec == nb + nh + 1 and p["edge_rec_bytes"] == 16 * ((nrec + 3) // 4 * 4)
    blk = p["edge_blk"].reshape(nb, 4)
    # the eight neighbour records: left, right, above, below, above-left,
    # above-right, below-left, below-right
    nbrec = np.stack([blk[:, i // 2] >> (16 * (i % 2)) & 0xFFFF for i in range(8)], axis=1).astype(np.int64)
    assert nbrec.max() < nrec
    rec = np.zeros((T, nrec, 4), U32)  # the last record stays zero
    tiles = np.arange(T)
    # own blocks: loads, rows, records
    off = tiles[:, None] * K + (np.arange(nb) * CB)[None, :]
    WB = window_bytes(p, BS, CB, nsrc)
    raw = load_blocks(state, off.ravel(), CB, nsrc, WB)
    rows = unpack(p, raw, BS)
    rec[np.repeat(tiles, nb), np.tile(np.arange(nb), T)] = record(rows, BS)
    # halo items
    if nh:
        hal = p["edge_halo"].reshape(nh, 2)
        hdir, hlb = hal[:, 0] >> 29, hal[:, 0] & 0x1FFFFFFF
        hslot = hal[:, 1]
        assert (hslot == nb + np.arange(nh)).all()
        nbr = p["nbr"].reshape(T, 8)
        nt = nbr[:, hdir]  # T x nh
        ok = nt != 0xFFFFFFFF
        tt, hh = np.nonzero(ok)
        hoff = nt[tt, hh].astype(np.int64) * K + hlb[hh].astype(np.int64) * CB
        hraw = load_blocks(state, hoff, CB, nsrc, WB)
        rec[tt, hslot[hh]] = record(unpack(p, hraw, BS), BS)
    # the rule per block, read as the kernel reads
    R = rec.reshape(T, nrec * 4)
    ti = np.repeat(tiles, nb)
    rd = lambda i, w: R[ti, 4 * np.tile(nbrec[:, i], T) + w]
    Lc, Rc = rd(0, 3), rd(1, 2)
    aC, bC = rd(2, 1), rd(3, 0)
    aL, aR, bL, bR = rd(4, 1), rd(5, 1), rd(6, 0), rd(7, 0)
    o = rows
    lo = [vperm(o[q], Lc, sel4(q, 4, 5, 6)) for q in range(BS)]
    hi = [vperm(Rc, o[q], sel4(1, 2, 3, 4 + q) if BS == 4 else sel4(1, 2, 4 + q, 12)) for q in range(BS)]
    edge = bool(rule >> 31)
    if edge:
        n = [(aC if q == 0 else o[q - 1]) + (bC if q == BS - 1 else o[q + 1]) + lo[q] + hi[q] for q in range(BS)]
    else:
        if BS == 4:
            H0 = alignbyte(aC, aL, 3) + aC + alignbyte(aR, aC, 1)
            H5 = alignbyte(bC, bL, 3) + bC + alignbyte(bR, bC, 1)
        else:
            H0 = vperm(aC, aL, sel4(2, 4, 5, 6)) + aC + vperm(aR, aC, sel4(1, 2, 4, 12))
            H5 = vperm(bC, bL, sel4(2, 4, 5, 6)) + bC + vperm(bR, bC, sel4(1, 2, 4, 12))
        H = [H0] + [lo[q] + o[q] + hi[q] for q in range(BS)] + [H5]
        n = [H[q] + H[q + 1] + H[q + 2] - o[q] for q in range(BS)]
    nxt = [rule_dword(n[q], o[q], rule) for q in range(BS)]
    while len(nxt) < 4:
        nxt.append(np.zeros_like(nxt[0]))
    out = np.zeros_like(state)
    words = []
    for d in range(4):
        w = vperm(nxt[1], nxt[0], p["edge_pack"][d]) | vperm(nxt[3], nxt[2], p["edge_pack"][4 + d])
        words.append(w)
    by = np.stack([(words[c // 4] >> U32(8 * (c % 4))) & U32(0xFF) for c in range(CB)], axis=-1).astype(np.uint8)
    dst = (ti * K + np.tile(np.arange(nb) * CB, T))[:, None] + np.arange(CB)[None, :]
    out[dst.ravel()] = by.ravel()
    return out


B3S23 = W.rule_mask("B3/S23")


def rule_dword(n, o, rule):
    """Next states of four positions (counts n, states o, one per byte) in
    the kernel's three forms: B3/S23 as one table look-up of (n | o), rules
    without an entry at eight neighbours (or four-cell ones) as birth and
    survival tables selected by o, others bit by bit from the rule word."""
    if rule == B3S23:
        return vperm(np.zeros_like(n), np.full_like(n, 0x01000000), n | o)
    if (rule >> 31) or (rule & ((1 << 8) | (1 << 24))) == 0:
        tb = [sum(((rule >> (base + c + 4 * h)) & 1) << (8 * c) for c in range(4)) for base in (0, 16)
              for h in (0, 1)]
        born = vperm(np.full_like(n, tb[1]), np.full_like(n, tb[0]), n)
        surv = vperm(np.full_like(n, tb[3]), np.full_like(n, tb[2]), n)
        smask = vperm(np.zeros_like(o), np.full_like(o, 0xFF00), o)
        return (surv & smask) | (born & ~smask)
    nq, oq = n.astype(np.uint64), o.astype(np.uint64)
    v = np.zeros_like(nq)
    for c in range(4):
        cnt = (nq >> np.uint64(8 * c)) & np.uint64(0xFF)
        self_ = (oq >> np.uint64(8 * c)) & np.uint64(1)
        bit = (np.uint64(rule) >> (cnt + np.uint64(16) * self_)) & np.uint64(1)
        v |= bit << np.uint64(8 * c)
    return v.astype(U32)


# (fractal, r, tile level): the workloads' levels and tile sizes around them,
# fractals whose blocks need four source dwords (triangle, grid4_12,
# fullsquare) or two, windows that end at the state's end,
# sparse grids whose blocks often border no block (chandelier, cantor dust)
CASES = [("triangle", 7, 7), ("triangle", 9, 7), ("triangle", 10, 5), ("triangle", 12, 6), ("carpet", 4, 4),
         ("carpet", 5, 3), ("carpet", 6, 4), ("hfractal", 5, 4), ("hfractal", 6, 3), ("chandelier", 7, 5),
         ("chandelier", 9, 4), ("vicsek", 5, 3), ("xfractal", 5, 4), ("cantordust", 6, 3),
         ("grid4_12", 3, 2), ("grid4_12", 4, 3), ("fullsquare", 6, 3), ("fullsquare", 6, 5)]
RULES = ["B3/S23", "B36/S23", "B1357/S02468", "B35/S0123456", "B2/S", "vN:B2/S12", "vN:B13/S024"]


@pytest.mark.parametrize("name,r,m", CASES)
def test_edge_model_matches_oracle(name, r, m):
    fd = W.FRACTALS[name]
    p = N.plan_tables(fd.s, fd.offsets, r, m)
    assert p["edge_ok"]
    o = O.Fractal(fd.s, fd.offsets, r)
    st = o.init_compact(31 + r, 0.45)
    for rule in RULES:
        rm = W.rule_mask(rule)
        np.testing.assert_array_equal(model_step(fd, r, st, rm, m), o.compact_steps(st, rm, 1),
                                      err_msg=f"{name} r={r} m={m} {rule}")


def test_edge_plan_refuses_small_tiles():
    # tiles below two load widths keep the byte-scatter form
    fd = W.FRACTALS["hfractal"]
    assert not N.plan_tables(fd.s, fd.offsets, 5, 1)["edge_ok"]  # K = 7
    fd = W.FRACTALS["triangle"]
    assert not N.plan_tables(fd.s, fd.offsets, 5, 2)["edge_ok"]  # K = 9 < 32


@pytest.mark.parametrize("seed", range(6))
def test_edge_model_random_fractals(seed):
    fd = W.random_fractal(500 + seed, s_choices=(2, 3, 4))
    r = 1
    while fd.k ** (r + 1) <= 60000 and r < 12:
        r += 1
    o = O.Fractal(fd.s, fd.offsets, r)
    st = o.init_compact(seed, 0.5)
    ran = 0
    for m in range(1, r + 1):
        try:
            p = N.plan_tables(fd.s, fd.offsets, r, m)
        except N.NbbError:
            continue
        if not p["edge_ok"]:
            continue
        ran += 1
        for rule in ("B3/S23", "B1357/S02468", "vN:B2/S12"):
            rm = W.rule_mask(rule)
            np.testing.assert_array_equal(model_step(fd, r, st, rm, m), o.compact_steps(st, rm, 1),
                                          err_msg=str((fd, r, m, rule)))
    if not ran:
        pytest.skip("the edge form applies at no level of this fractal")


def test_edge_plan_applies_to_the_workloads():
    # the workloads' automatic levels all run in edge form
    for name, r in [("triangle", 16), ("carpet", 9), ("hfractal", 10), ("chandelier", 11)]:
        fd = W.FRACTALS[name]
        p = N.plan_tables(fd.s, fd.offsets, r)
        assert p["edge_ok"], name
        assert p["edge_rec_bytes"] <= 32768, (name, p["edge_rec_bytes"])
        assert p["edge_records"] == p["blocks"] + p["edge_halo_count"] + 1
