"""The batched step that allocates no device memory
(nbb_batch_step_each_noalloc), against the allocating batch
(nbb_batch_create_ex + nbb_batch_step_each) on the same seeded inputs.

Two calls in a row, the second on a smaller batch, so the second call runs on
tables that the first left in the library's static array.  Every instance's
result must equal the allocating batch's bit for bit (and, for a sample of
instances, the oracle's compact step); arena bytes outside the instances'
ranges must not change.  A batch whose tables do not fit the array is refused
before anything is enqueued.  Inputs are seeded and synthetic.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_12952_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B3S23 = W.rule_mask("B3/S23")
SENTINEL = 0xA5


@pytest.fixture(scope="module")
def N():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2110_12952_amd import nbbfrac
    nbbfrac.lib()
    return nbbfrac


# An s = 5 fractal: no tiled plan, so its instance takes the per-cell step.
PLUS5 = W.FractalDef("plus5", 5, ((2, 0), (0, 2), (2, 2), (4, 2), (2, 4), (1, 1)))

# (fractal, level, generations): the first call's batch, then a smaller one
FIRST = [("triangle", 9, 23), ("carpet", 4, 21), ("hfractal", 4, 20), ("triangle", 7, 17), ("chandelier", 6, 16),
         ("hfractal", 3, 13), ("carpet", 3, 12), ("triangle", 9, 9), ("plus5", 3, 8), ("chandelier", 4, 5),
         ("triangle", 5, 4), ("carpet", 2, 0)]
SECOND = [("hfractal", 3, 11), ("triangle", 6, 7), ("carpet", 3, 6), ("triangle", 6, 3)]


def _fd(name):
    return PLUS5 if name == "plus5" else W.FRACTALS[name]


def _setup(N, spec, seed0, gap):
    """Descriptors (one per (fractal, level)), arena offsets with `gap`
    sentinel bytes between instances, the step counts, and two sentinel-filled
    arenas with every instance's initial state at its offset in a."""
    descs, frs, offsets, steps = {}, [], [], []
    off = 64
    for name, r, t in spec:
        key = (name, r)
        if key not in descs:
            fd = _fd(name)
            descs[key] = N.Fractal(fd.s, fd.offsets, r)
        f = descs[key]
        frs.append(f)
        offsets.append(off)
        steps.append(t)
        off += (f.cells + 15) // 16 * 16 + gap
    length = off + 64
    a = torch.full((length,), SENTINEL, dtype=torch.uint8, device="cuda")
    b = torch.full_like(a, SENTINEL)
    for i, (f, o) in enumerate(zip(frs, offsets)):
        f.init_compact(seed0 + i, 0.2 + 0.03 * (i % 10), out=a[o:o + f.cells])
    return descs, frs, offsets, steps, a, b


def _outside_mask(frs, offsets, length):
    m = np.ones(length, dtype=bool)
    for f, o in zip(frs, offsets):
        m[o:o + f.cells] = False
    return m


def _run_and_compare(N, spec, seed0, gap, oracle_sample):
    descs, frs, offsets, steps, a, b = _setup(N, spec, seed0, gap)
    init = a.clone()
    # the allocating batch on copies of the same arenas
    ra, rb = init.clone(), torch.full_like(b, SENTINEL)
    ref = N.Batch(frs, offsets, resident=False)
    ref.step_each(ra, rb, steps)
    # the call under test
    N.batch_step_each_noalloc(frs, offsets, a, b, steps)
    torch.cuda.synchronize()
    ha, hb, hra, hrb = (t.cpu().numpy() for t in (a, b, ra, rb))
    h0 = init.cpu().numpy()
    for i, (f, o, t) in enumerate(zip(frs, offsets, steps)):
        got = (hb if t & 1 else ha)[o:o + f.cells]
        want = (hrb if t & 1 else hra)[o:o + f.cells]
        np.testing.assert_array_equal(got, want, err_msg=f"instance {i} {spec[i]}")
        if t == 0:
            np.testing.assert_array_equal(ha[o:o + f.cells], h0[o:o + f.cells])
    out = _outside_mask(frs, offsets, len(ha))
    assert (ha[out] == SENTINEL).all() and (hb[out] == SENTINEL).all()
    for i in oracle_sample:
        name, r, t = spec[i]
        fd = _fd(name)
        o = O.Fractal(fd.s, fd.offsets, r)
        want = o.compact_steps(h0[offsets[i]:offsets[i] + o.cells].copy(), B3S23, t)
        got = (hb if t & 1 else ha)[offsets[i]:offsets[i] + o.cells]
        np.testing.assert_array_equal(got, want, err_msg=f"instance {i} {spec[i]} vs oracle")
    return ref


def test_noalloc_equals_allocating_batch_two_calls(N):
    # first call: mixed fractals, levels and step counts (decreasing within
    # every group), a per-cell (direct) instance and a zero-step instance
    ref1 = _run_and_compare(N, FIRST, 100, 48, oracle_sample=(0, 4, 8, 10))
    assert ref1.info().groups >= 4 and ref1.info().direct == 1
    # second call: a smaller batch on other offsets; its tables overwrite the
    # first call's in the static array
    _run_and_compare(N, SECOND, 900, 16, oracle_sample=(0, 3))


def test_noalloc_same_stream_back_to_back(N):
    # two calls enqueued on one stream with no synchronisation between them:
    # the second's table build must wait for the first's steps
    spec = [("carpet", 4, 10), ("triangle", 8, 9), ("hfractal", 4, 7)]
    descs, frs, offsets, steps, a, b = _setup(N, spec, 7, 32)
    init = a.clone()
    small = [("triangle", 5, 6)]
    d2, frs2, offs2, steps2, a2, b2 = _setup(N, small, 70, 16)
    init2 = a2.clone()
    N.batch_step_each_noalloc(frs, offsets, a, b, steps)
    N.batch_step_each_noalloc(frs2, offs2, a2, b2, steps2)
    torch.cuda.synchronize()
    for (fr_, of_, st_, aa, bb, i0) in ((frs, offsets, steps, a, b, init), (frs2, offs2, steps2, a2, b2, init2)):
        ra, rb = i0.clone(), torch.full_like(bb, SENTINEL)
        N.Batch(fr_, of_, resident=False).step_each(ra, rb, st_)
        torch.cuda.synchronize()
        for f, o, t in zip(fr_, of_, st_):
            got = (bb if t & 1 else aa)[o:o + f.cells]
            want = (rb if t & 1 else ra)[o:o + f.cells]
            assert torch.equal(got, want)


def test_noalloc_refuses_tables_beyond_the_array(N):
    # triangle r = 12 at tile level 2: 3^10 tiles per instance, 40 table bytes
    # each; eight instances need more than the 16 MiB array holds
    fd = W.TRIANGLE
    f = N.Fractal(fd.s, fd.offsets, 12)
    f.configure(N.STRATEGY_TILED, 2)
    assert f.info().tiles * 8 * 40 > N.NOALLOC_SCRATCH_BYTES
    frs = [f] * 8
    offsets, length = N.pack_offsets([f.cells] * 8)
    a = torch.full((length,), SENTINEL, dtype=torch.uint8, device="cuda")
    b = torch.full_like(a, SENTINEL)
    with pytest.raises(N.NbbError, match="no-allocation scratch"):
        N.batch_step_each_noalloc(frs, offsets, a, b, [3] * 8)
    torch.cuda.synchronize()
    assert bool((a == SENTINEL).all()) and bool((b == SENTINEL).all())
    # half of them fit
    init = torch.zeros_like(a)
    for i in range(4):
        f.init_compact(i, 0.4, out=init[offsets[i]:offsets[i] + f.cells])
    a.copy_(init)
    N.batch_step_each_noalloc(frs[:4], offsets[:4], a, b, [3] * 4)
    ra, rb = init.clone(), torch.empty_like(b)
    N.Batch(frs[:4], offsets[:4], resident=False).step_each(ra, rb, [3] * 4)
    torch.cuda.synchronize()
    for i in range(4):
        o = offsets[i]
        assert torch.equal(b[o:o + f.cells], rb[o:o + f.cells])


def test_noalloc_argument_errors(N):
    fd = W.CARPET
    f = N.Fractal(fd.s, fd.offsets, 3)
    a = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    with pytest.raises(N.NbbError, match="multiples of 16"):
        N.batch_step_each_noalloc([f], [8], a, b, [1])
    with pytest.raises(N.NbbError, match="overlap"):
        N.batch_step_each_noalloc([f, f], [0, 256], a, b, [1, 1])
    with pytest.raises(N.NbbError, match="increase"):
        N.batch_step_each_noalloc([f, f], [0, 512], a, b, [1, 2])
    with pytest.raises(N.NbbError, match="shorter"):
        N.batch_step_each_noalloc([f], [0], a[:256], b[:256], [1])
