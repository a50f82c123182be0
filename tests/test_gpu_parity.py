"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison is exact: extreme slots and their binary64 values, the
filter polygon, the ascending survivor list and the hull index list must be
identical to the oracle's on the same seeded inputs.
"""
import numpy as np
import pytest

import oracle
from paper_1405_3454_amd import inputs
from paper_1405_3454_amd.inputs import to_float

pytestmark = pytest.mark.gpu

KINDS = ["square", "disk", "gaussian", "annulus"]


@pytest.fixture(scope="module")
def H():
    import torch
    from paper_1405_3454_amd.api import Hull
    h = Hull(0)
    yield h
    torch.cuda.synchronize()
    h.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def u32(t):
    from paper_1405_3454_amd.api import as_u32
    return as_u32(t)


def check_all(H, x, y, preset, what=""):
    H.set_directions(preset)
    xt, yt = dev(x), dev(y)
    slots, vals = H.extremes(xt, yt)
    o_slots, o_vals = oracle.extremes(x, y, preset)
    assert np.array_equal(u32(slots), o_slots), (what, u32(slots), o_slots)
    gv = vals.cpu().numpy()
    assert np.array_equal(gv.view(np.uint64)[o_slots != oracle.NONE],
                          o_vals.view(np.uint64)[o_slots != oracle.NONE]), what
    o_verts = oracle.polygon(x, y, o_slots)
    verts = H.polygon(xt, yt, slots)
    assert np.array_equal(u32(verts), o_verts), what
    surv = H.discard(xt, yt, slots)
    o_surv = oracle.discard(x, y, o_verts)
    assert np.array_equal(u32(surv), o_surv), (what, len(surv), len(o_surv))
    hull = H.compute(xt, yt)
    o_hull = oracle.hull_subset(x, y, o_surv)
    assert np.array_equal(u32(hull), o_hull), (what, u32(hull)[:10], o_hull[:10])
    assert np.array_equal(o_hull, oracle.compute(x, y, preset))
    return len(o_surv)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 64, 255, 256, 257, 1023, 1024, 1025, 4099,
                               65536 + 3])
@pytest.mark.parametrize("kind", KINDS)
def test_small_sizes(H, kind, n):
    x, y = inputs.DISTRIBUTIONS[kind](n, 1000 + n)
    check_all(H, x, y, 0, "%s n=%d" % (kind, n))


@pytest.mark.parametrize("preset", [0, 1])
@pytest.mark.parametrize("kind", KINDS)
def test_medium(H, kind, preset):
    x, y = inputs.DISTRIBUTIONS[kind](300_000, 77 + preset)
    check_all(H, x, y, preset, "%s preset=%d" % (kind, preset))


def test_empty(H):
    import torch
    x = torch.zeros(0, dtype=torch.float32, device="cuda:0")
    slots, vals = H.extremes(x, x)
    assert (u32(slots) == oracle.NONE).all()
    assert len(H.compute(x, x)) == 0
    assert len(H.discard(x, x, slots)) == 0


@pytest.mark.parametrize("seed", range(12))
def test_degenerate_grids(H, seed):
    """Tiny lattices: duplicates, ties for every extreme, collinear runs."""
    r = np.random.default_rng(seed)
    n = int(r.integers(1, 5000))
    side = int(r.integers(1, 12))
    x, y = inputs.small_grid(n, side, seed, (int(r.integers(0, 1 << 23)), int(r.integers(0, 1 << 23))))
    check_all(H, x, y, seed % 2, "grid seed=%d n=%d side=%d" % (seed, n, side))


def test_collinear_and_identical(H):
    k = np.arange(5000)
    for x, y in [(to_float(k * 7 % 5000), to_float(np.zeros(5000, np.int64) + 99)),
                 (to_float(np.zeros(5000, np.int64) + 5), to_float(k[::-1])),
                 (to_float(k), to_float(k)),
                 (to_float(np.full(3000, 12345)), to_float(np.full(3000, 54321)))]:
        check_all(H, x, y, 0, "collinear")


def test_regular_polygon(H):
    x, y, m = inputs.regular_polygon(48, 200_000, seed=3)
    check_all(H, x, y, 0, "48-gon")
    check_all(H, x, y, 1, "48-gon cumulative")


@pytest.mark.parametrize("kind", KINDS)
def test_unfiltered_arm(H, kind):
    x, y = inputs.DISTRIBUTIONS[kind](200_000, 5)
    hull = H.compute(dev(x), dev(y), nofilter=True)
    assert np.array_equal(u32(hull), oracle.compute(x, y, nofilter=True))


def test_hull_of_subset(H):
    x, y = inputs.disk(100_000, 9)
    idx = np.sort(np.random.default_rng(1).choice(len(x), 30000, replace=False)).astype(np.uint32)
    import torch
    h = H.hull_of_subset(dev(x), dev(y), torch.from_numpy(idx.view(np.int32)).to("cuda:0"))
    assert np.array_equal(u32(h), oracle.hull_subset(x, y, idx))


@pytest.mark.parametrize("m", [1, 2, 3, 4095, 4096, 4097, 9000])
def test_hull_of_subset_sort_switch(H, m):
    """Subsets around the size where the one-block sort hands over to the
    radix passes: the same hull either way."""
    import torch
    x, y = inputs.disk(20_000, 21)
    idx = np.sort(np.random.default_rng(m).choice(len(x), m, replace=False)).astype(np.uint32)
    h = H.hull_of_subset(dev(x), dev(y), torch.from_numpy(idx.view(np.int32)).to("cuda:0"))
    assert np.array_equal(u32(h), oracle.hull_subset(x, y, idx))


def test_determinism(H):
    x, y = inputs.annulus(500_000, 4)
    xt, yt = dev(x), dev(y)
    a = u32(H.compute(xt, yt))
    default = H.tuning()
    try:
        for bpc in ((2, 2), (16, 16), (8, 8)):
            H.set_tuning(*bpc)
            assert np.array_equal(u32(H.compute(xt, yt)), a)
    finally:
        H.set_tuning(*default)
    assert H.tuning() == default


@pytest.mark.parametrize("preset", [0, 1])
@pytest.mark.parametrize("kind", KINDS)
def test_multi_tile_runs(H, kind, preset):
    """One block per CU for both filter passes (1024 waves) with 3.1M
    points: every wave walks three or four tiles of the set, so the
    extremes pass resolves its ties across the tiles of a run (the per-lane
    best and record-tile logic) for each preset, against the oracle."""
    default = H.tuning()
    H.set_tuning(1, 1)
    try:
        x, y = inputs.DISTRIBUTIONS[kind](3_100_000, 900 + preset)
        check_all(H, x, y, preset, "%s preset=%d q>=3" % (kind, preset))
    finally:
        H.set_tuning(*default)


@pytest.mark.parametrize("preset", [0, 1])
@pytest.mark.parametrize("side", [3, 40])
def test_multi_tile_ties(H, side, preset):
    """Lattices of 3.1M points with 1024 waves: every extreme value is met
    by thousands of points spread over every tile of every run, so the
    lowest index must be found across tiles and runs."""
    default = H.tuning()
    H.set_tuning(1, 1)
    try:
        x, y = inputs.small_grid(3_100_000, side, 60 + side, (5000, 7000))
        check_all(H, x, y, preset, "grid side=%d preset=%d q>=3" % (side, preset))
    finally:
        H.set_tuning(*default)


def test_validate_flag(H):
    from paper_1405_3454_amd._lib import HULL_EDOMAIN, HullError
    x, y = inputs.square(1000, 1)
    xt, yt = dev(x), dev(y)
    assert len(H.compute(xt, yt, validate=True)) > 0
    for v in (np.float32(0.25) + np.float32(2.0 ** -25),   # off the 2^-24 grid
              np.float32(1.0), np.float32(-2.0 ** -24), np.float32(np.nan)):
        bad = x.copy()
        bad[17] = v
        with pytest.raises(HullError) as e:
            H.compute(dev(bad), yt, validate=True)
        assert e.value.code == HULL_EDOMAIN, v


@pytest.mark.parametrize("shift", [1, 2, 3])
@pytest.mark.parametrize("n", [1, 5, 1023, 5000, 70001])
def test_unaligned_inputs(H, shift, n):
    """x, y that start 1-3 floats into a 16-byte block (slices of aligned
    tensors): the tiles align to absolute 16-byte boundaries; every result
    equals the oracle on the same points, indices relative to the slice."""
    H.set_directions(0)
    x, y = inputs.disk(n + 3, 40 + shift)
    xt, yt = dev(x)[shift:], dev(y)[shift:]
    xs, ys = x[shift:][:n], y[shift:][:n]
    xt, yt = xt[:n], yt[:n]
    slots, _ = H.extremes(xt, yt)
    o_slots, _ = oracle.extremes(xs, ys)
    assert np.array_equal(u32(slots), o_slots)
    surv = H.discard(xt, yt, slots)
    o_surv = oracle.discard(xs, ys, oracle.polygon(xs, ys, o_slots))
    assert np.array_equal(u32(surv), o_surv)
    assert np.array_equal(u32(H.compute(xt, yt)), oracle.hull_subset(xs, ys, o_surv))


def test_unaligned_batched_and_mismatched_phase(H):
    from paper_1405_3454_amd._lib import HullError
    H.set_directions(0)
    sizes = [3000, 1, 17, 4096, 999]
    x, y, off, _ = inputs.batch(sizes, 44)
    pad = np.zeros(2, np.float32)
    xt = dev(np.concatenate([pad, x]))[2:]
    yt = dev(np.concatenate([pad, y]))[2:]
    hull, ho = H.compute_batched(xt, yt, dev(off))
    hull, ho = u32(hull), ho.cpu().numpy()
    for s in range(len(sizes)):
        a, b = off[s], off[s + 1]
        want = oracle.hull_subset(x[a:b], y[a:b]).astype(np.int64) + a
        assert np.array_equal(hull[ho[s]:ho[s + 1]].astype(np.int64), want)
    with pytest.raises(HullError):      # x and y at different positions in their blocks
        H.compute(dev(x)[1:len(x) - 1], dev(y)[2:])


@pytest.mark.parametrize("kind", ["disk", "annulus", "gaussian", "square"])
@pytest.mark.parametrize("n", [3, 100, 4096, 200_001])
def test_refinement_keeps_the_hull(H, kind, n):
    """The QuickHull refinement rounds before the sort drop only points
    strictly inside triangles of set points: the hull equals the oracle's and
    the one computed without the rounds."""
    H.set_directions(0)
    x, y = inputs.DISTRIBUTIONS[kind](n, 70 + n % 97)
    xt, yt = dev(x), dev(y)
    want = oracle.compute(x, y, 0)
    assert np.array_equal(u32(H.compute(xt, yt)), want)
    counts = H.candidate_counts()
    slots, _ = oracle.extremes(x, y, 0)
    surv = oracle.discard(x, y, oracle.polygon(x, y, slots))
    assert counts[0] == len(surv)
    # every round keeps the hull's vertices and never adds candidates
    assert all(len(want) <= b <= a for a, b in zip(counts, counts[1:])), counts
    assert np.array_equal(u32(H.compute(xt, yt, refine=False)), want)
    assert H.candidate_counts() == [len(surv)] + [-1] * 4


def test_refinement_degenerate_inputs(H):
    H.set_directions(0)
    for seed in range(6):
        x, y = inputs.small_grid(3000, 1 + seed % 4, seed)
        want = oracle.compute(x, y, 0)
        assert np.array_equal(u32(H.compute(dev(x), dev(y))), want), seed
    x, y, m = inputs.regular_polygon(48, 5000, 3)
    assert np.array_equal(u32(H.compute(dev(x), dev(y))), oracle.compute(x, y, 0))


def test_long_chain(H):
    """8191 strictly convex points on a parabola (every one a lower-hull
    vertex) under 100k random points: the lower chain outgrows what one wave
    stages in LDS, so the merge also walks bridges in global memory."""
    r = np.random.default_rng(77)
    k = np.arange(1, 8192, dtype=np.int64)
    px, py = k * 2048, (k - 4096) ** 2
    qx = r.integers(0, 1 << 24, size=100_000)
    qy = r.integers(0, 1 << 24, size=100_000)
    keep = qy > ((qx / 2048.0 - 4096.0) ** 2) + 4096     # well above the curve
    x = inputs.to_float(np.concatenate([qx[keep][:40_000], px, qx[keep][40_000:]]))
    y = inputs.to_float(np.concatenate([qy[keep][:40_000], py, qy[keep][40_000:]]))
    want = oracle.compute(x, y, 0)
    assert len(want) > 8000
    H.set_directions(0)
    xt, yt = dev(x), dev(y)
    assert np.array_equal(u32(H.compute(xt, yt)), want)
    assert np.array_equal(u32(H.compute(xt, yt, refine=False)), want)
    assert np.array_equal(u32(H.compute(xt, yt, nofilter=True)), oracle.compute(x, y, nofilter=True))
    # two copies in one batch
    n = len(x)
    xb, yb = np.concatenate([x, x]), np.concatenate([y, y])
    hull, ho = H.compute_batched(dev(xb), dev(yb), dev(np.array([0, n, 2 * n], np.int64)))
    hv, ho = u32(hull), ho.cpu().numpy()
    assert np.array_equal(hv[ho[0]:ho[1]], want)
    assert np.array_equal(hv[ho[1]:ho[2]].astype(np.int64), want.astype(np.int64) + n)
