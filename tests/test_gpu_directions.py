"""Direction families beyond the paper's table, on the GPU against the oracle.

Presets 2..7 use G = 1..6 rotation groups at 90 j / G degrees: the min/max
x and y quadrilateral (G = 1, the simplest filter the paper cites in Sec. 1)
up to 24 evenly spaced directions.  Every comparison is exact: slots and
their binary64 values, the filter polygon, the ascending survivors and the
hull index list, for single sets, batches, multi-tile runs (several tiles of
one set per wave, ties resolved across tiles) and the learned slots on top
of the families that leave room for them.
"""
import numpy as np
import pytest

import oracle
from paper_1405_3454_amd import inputs

pytestmark = pytest.mark.gpu

KINDS = ["square", "disk", "gaussian", "annulus"]
EVEN = [2, 3, 4, 5, 6, 7]          # G = preset - 1 groups


@pytest.fixture(scope="module")
def H():
    import torch
    from paper_1405_3454_amd.api import Hull
    h = Hull(0)
    yield h
    torch.cuda.synchronize()
    h.set_directions(0)
    h.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def u32(t):
    from paper_1405_3454_amd.api import as_u32
    return as_u32(t)


def slots_match(g_slots, o_slots, what):
    """The GPU lists max(16, 4G) slot positions; the first 4G are the
    oracle's, the rest are empty."""
    k = len(o_slots)
    assert len(g_slots) == max(16, k), what
    assert np.array_equal(g_slots[:k], o_slots), (what, g_slots[:k], o_slots)
    assert (g_slots[k:] == oracle.NONE).all(), what


def check_preset(H, x, y, preset, what):
    H.set_directions(preset)
    xt, yt = dev(x), dev(y)
    slots, vals = H.extremes(xt, yt)
    gs = u32(slots)
    o_slots, o_vals = oracle.extremes(x, y, preset)
    slots_match(gs, o_slots, what)
    gv = vals.cpu().numpy()[: len(o_slots)]
    ok = o_slots != oracle.NONE
    assert np.array_equal(gv.view(np.uint64)[ok], o_vals.view(np.uint64)[ok]), what
    o_verts = oracle.polygon(x, y, o_slots)
    assert np.array_equal(u32(H.polygon(xt, yt, slots)), o_verts), what
    surv = u32(H.discard(xt, yt, slots))
    o_surv = oracle.discard(x, y, o_verts)
    assert np.array_equal(surv, o_surv), (what, len(surv), len(o_surv))
    o_hull = oracle.hull_subset(x, y, o_surv)
    assert np.array_equal(u32(H.compute(xt, yt)), o_hull), what
    assert np.array_equal(u32(H.compute(xt, yt, refine=False)), o_hull), what
    assert np.array_equal(o_hull, oracle.compute(x, y, preset)), what
    return len(o_surv)


def test_slot_counts(H):
    for p in range(8):
        H.set_directions(p)
        G = len(oracle.preset(p)[0]) if p > 1 else 4
        assert H.slot_count() == max(16, 4 * G)
        if max(16, 4 * G) == 16:
            assert H.slot_count(learned=True) == 24
        else:
            from paper_1405_3454_amd._lib import HullError
            with pytest.raises(HullError):
                H.slot_count(learned=True)
    H.set_directions(0)


def test_library_tables_equal_oracle_tables(H):
    for p in range(8):
        H.set_directions(p)
        c, s = H.direction_table(0)
        oc, os_ = oracle.preset(p)
        assert np.array_equal(c, oc) and np.array_equal(s, os_), p
    H.set_directions(0)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 257, 1023, 1025, 4099, 70001])
@pytest.mark.parametrize("preset", EVEN)
def test_even_presets_small_sizes(H, preset, n):
    kind = KINDS[(n + preset) % 4]
    x, y = inputs.DISTRIBUTIONS[kind](n, 3000 + 10 * n + preset)
    check_preset(H, x, y, preset, "%s n=%d preset=%d" % (kind, n, preset))


@pytest.mark.parametrize("preset", EVEN)
@pytest.mark.parametrize("kind", KINDS)
def test_even_presets_medium(H, kind, preset):
    x, y = inputs.DISTRIBUTIONS[kind](200_000, 91 + preset)
    check_preset(H, x, y, preset, "%s preset=%d" % (kind, preset))


@pytest.mark.parametrize("seed", range(6))
def test_even_presets_degenerate_grids(H, seed):
    r = np.random.default_rng(100 + seed)
    n = int(r.integers(1, 4000))
    side = int(r.integers(1, 10))
    x, y = inputs.small_grid(n, side, seed, (int(r.integers(0, 1 << 23)), int(r.integers(0, 1 << 23))))
    check_preset(H, x, y, EVEN[seed], "grid seed=%d n=%d side=%d" % (seed, n, side))


def test_even_presets_regular_polygon(H):
    x, y, m = inputs.regular_polygon(48, 100_000, seed=5)
    for p in EVEN:
        check_preset(H, x, y, p, "48-gon preset=%d" % p)


@pytest.mark.parametrize("preset", EVEN)
def test_even_presets_multi_tile_runs(H, preset):
    """One block per CU: 1024 waves, so 1.5M points give every wave two or
    more tiles of the set and the cross-tile tie logic runs."""
    k1, k3 = H.tuning()
    try:
        H.set_tuning(1, 1)
        x, y = inputs.disk(1_500_000, 500 + preset)
        # coarse grid: many exact ties in every direction
        x = (np.floor(x * 4096) / 4096).astype(np.float32)
        y = (np.floor(y * 4096) / 4096).astype(np.float32)
        H.set_directions(preset)
        slots, vals = H.extremes(dev(x), dev(y))
        o_slots, o_vals = oracle.extremes(x, y, preset)
        slots_match(u32(slots), o_slots, "preset=%d" % preset)
        gv = vals.cpu().numpy()[: len(o_slots)]
        assert np.array_equal(gv.view(np.uint64), o_vals.view(np.uint64))
        o_verts = oracle.polygon(x, y, o_slots)
        o_surv = oracle.discard(x, y, o_verts)
        assert np.array_equal(u32(H.discard(dev(x), dev(y), slots)), o_surv)
        assert np.array_equal(u32(H.compute(dev(x), dev(y))), oracle.hull_subset(x, y, o_surv))
    finally:
        H.set_tuning(k1, k3)


@pytest.mark.parametrize("preset", EVEN)
def test_even_presets_batched(H, preset):
    r = np.random.default_rng(preset)
    sizes = list(r.integers(0, 5000, size=20)) + [0, 1, 2, 3, 1025, 30000]
    x, y, off, _ = inputs.batch(sizes, 40 + preset)
    H.set_directions(preset)
    xt, yt, ot = dev(x), dev(y), dev(off.astype(np.int64))
    S = len(sizes)
    k = H.slot_count()
    slots = u32(H.extremes_batched(xt, yt, ot)).reshape(S, k)
    surv, so = H.discard_batched(xt, yt, ot, dev(slots.view(np.int32)))
    so, sv = so.cpu().numpy(), u32(surv)
    hull, ho = H.compute_batched(xt, yt, ot)
    ho, hv = ho.cpu().numpy(), u32(hull)
    for s in range(S):
        a, b = int(off[s]), int(off[s + 1])
        xs, ys = x[a:b], y[a:b]
        o_slots, _ = oracle.extremes(xs, ys, preset)
        g = np.where(o_slots == oracle.NONE, oracle.NONE,
                     o_slots.astype(np.int64) + a).astype(np.uint32)
        slots_match(slots[s], g, "set %d" % s)
        o_surv = oracle.discard(xs, ys, oracle.polygon(xs, ys, o_slots))
        assert np.array_equal(sv[so[s]:so[s + 1]].astype(np.int64), o_surv.astype(np.int64) + a), s
        o_hull = oracle.hull_subset(xs, ys, o_surv).astype(np.int64) + a
        assert np.array_equal(hv[ho[s]:ho[s + 1]].astype(np.int64), o_hull), s


def test_learned_slots_on_an_even_family(H):
    """Eight evenly spaced directions (preset 3) plus the eight learned ones:
    fixed slots 0..7, empty 8..15, learned 16..23; survivors and hull exact."""
    from oracle import mlp
    H.set_directions(3)
    H.mlp_set_params(mlp.he_init(33))
    sizes = [4000, 1, 60000, 777]
    x, y, off, _ = inputs.batch(sizes, 17, kinds=("mixture", "ellipse", "disk", "square"))
    xt, yt, ot = dev(x), dev(y), dev(off)
    hb, _ = H.histogram_batched(xt, yt, ot)
    dirs = H.top_directions(H.mlp_forward(hb)).cpu().numpy()
    cd, sd = oracle.direction_table()
    slots = u32(H.extremes_batched(xt, yt, ot, learned=True))
    assert slots.shape == (len(sizes), 24)
    hl, hlo = H.compute_batched(xt, yt, ot, learned=True)
    hl, hlo = u32(hl), hlo.cpu().numpy()
    sv, so = H.discard_batched(xt, yt, ot, dev(slots.view(np.int32)))
    sv, so = u32(sv), so.cpu().numpy()
    for s in range(len(sizes)):
        a, b = int(off[s]), int(off[s + 1])
        xs, ys = x[a:b], y[a:b]
        o_slots, _ = oracle.extremes(xs, ys, 3)
        g = np.where(o_slots == oracle.NONE, oracle.NONE, o_slots.astype(np.int64) + a)
        assert np.array_equal(slots[s, :8].astype(np.int64), g.astype(np.int64)), s
        assert (slots[s, 8:16] == oracle.NONE).all(), s
        es, _ = oracle.extremes_dirs(xs, ys, cd[dirs[s]], sd[dirs[s]])
        assert np.array_equal(slots[s, 16:].astype(np.int64), es.astype(np.int64) + a), s
        local = np.where(slots[s] == oracle.NONE, oracle.NONE,
                         slots[s].astype(np.int64) - a).astype(np.uint32)
        want = oracle.discard(xs, ys, oracle.polygon(xs, ys, local)).astype(np.int64) + a
        assert np.array_equal(sv[so[s]:so[s + 1]].astype(np.int64), want), s
        hw = oracle.hull_subset(xs, ys).astype(np.int64) + a
        assert np.array_equal(hl[hlo[s]:hlo[s + 1]].astype(np.int64), hw), s
    H.set_directions(0)


def test_learned_rejected_past_sixteen_fixed_slots(H):
    import torch
    from paper_1405_3454_amd._lib import HULL_EINVAL, HullError
    from oracle import mlp
    H.mlp_set_params(mlp.he_init(1))
    x, y = inputs.disk(5000, 3)
    for p in (6, 7):
        H.set_directions(p)
        with pytest.raises(HullError) as e:
            H.compute(dev(x), dev(y), learned=True)
        assert e.value.code == HULL_EINVAL
        # the plain method still runs on the same context
        assert np.array_equal(u32(H.compute(dev(x), dev(y))), oracle.compute(x, y, p))
    torch.cuda.synchronize()
    H.set_directions(0)
