"""Pins for the CPU oracle against what the paper and the mathematics fix.

None of these tests calls the GPU library.  Each one is chosen so that a
plausible mistake in the oracle (a wrong sign or slot order, a dropped
collinear case, an off-by-one edge, a non-strict test) fails it.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy.spatial import ConvexHull

import oracle
from paper_1405_3454_amd import inputs
from paper_1405_3454_amd.inputs import to_float, to_grid
from tests import _brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# -- direction constants (Sec. 2 Step 1; Figure 1; Sec. 5) ------------------

def _cr_cos_sin(num, den):
    """Correctly rounded cos/sin of num/den * 2 pi (multiples of 90 deg exact)."""
    mpmath.mp.prec = 300
    if (4 * num) % den == 0:
        q = (4 * num // den) % 4
        return [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][q]
    a = 2 * mpmath.pi * num / den
    return float(mpmath.cos(a)), float(mpmath.sin(a))


@pytest.mark.parametrize("p,angles", [(oracle.PRESET_PAPER, [0, 30, 45, 60]),
                                      (oracle.PRESET_CUMULATIVE, [0, 30, 75, 120])])
def test_preset_constants_correctly_rounded(p, angles):
    c, s = oracle.preset(p)
    for g, deg in enumerate(angles):
        cc, ss = _cr_cos_sin(deg, 360)
        assert c[g] == cc and s[g] == ss, (deg, c[g].hex(), cc.hex(), s[g].hex(), ss.hex())


def test_direction_table_correctly_rounded():
    c, s = oracle.direction_table()
    for d in range(64):
        cc, ss = _cr_cos_sin(d, 64)
        assert c[d] == cc and s[d] == ss, d
        assert not (c[d] == 0 and math.copysign(1, c[d]) < 0)


# -- hull (Andrew's algorithm, erratum to ref. [6]) -------------------------

@pytest.mark.parametrize("seed", range(40))
def test_hull_matches_bruteforce_on_tiny_grids(seed):
    r = np.random.default_rng(seed)
    n = int(r.integers(1, 36))
    side = int(r.integers(1, 7))
    off = (int(r.integers(0, 1000)), int(r.integers(0, 1000)))
    x, y = inputs.small_grid(n, side, seed, off)
    assert list(oracle.hull_subset(x, y)) == _brute.hull(x, y)


@pytest.mark.parametrize("seed", range(5))
def test_hull_matches_qhull_general_position(seed):
    x, y = inputs.disk(2000, 100 + seed)
    ours = oracle.hull_subset(x, y)
    qh = ConvexHull(np.stack([x, y], 1).astype(np.float64))
    v = list(qh.vertices)                       # counter-clockwise in 2D
    k = v.index(int(ours[0]))
    assert list(ours) == v[k:] + v[:k]


def test_hull_degenerate_cases():
    f = to_float
    assert len(oracle.hull_subset(np.zeros(0, np.float32), np.zeros(0, np.float32))) == 0
    assert list(oracle.hull_subset(f([5]), f([7]))) == [0]
    # all identical: lowest index
    assert list(oracle.hull_subset(f([3, 3, 3]), f([4, 4, 4]))) == [0]
    # two distinct points, with a repeat: lowest index of each
    assert list(oracle.hull_subset(f([9, 2, 9, 2]), f([1, 1, 1, 1]))) == [1, 0]
    # collinear horizontal, vertical, diagonal -> the two ends, min first
    assert list(oracle.hull_subset(f([4, 1, 3, 2]), f([0, 0, 0, 0]))) == [1, 0]
    assert list(oracle.hull_subset(f([0, 0, 0, 0]), f([4, 1, 3, 2]))) == [1, 0]
    assert list(oracle.hull_subset(f([2, 0, 1, 3]), f([2, 0, 1, 3]))) == [1, 3]
    # square with midpoints and centre: corners only, CCW from (0,0)
    xs = f([0, 2, 2, 0, 1, 2, 1, 0, 1])
    ys = f([0, 0, 2, 2, 0, 1, 2, 1, 1])
    assert list(oracle.hull_subset(xs, ys)) == [0, 1, 2, 3]


# -- Step 1 extremes: slot order, rotation sign, tie-break ------------------

def _slot_angles(angles):
    """Vertex angle (deg) expected in each slot: u = x cos t - y sin t is the
    projection on direction -t, v = x sin t + y cos t on 90 - t."""
    out = []
    for t in angles:
        out += [(180 - t) % 360, (-t) % 360, (270 - t) % 360, (90 - t) % 360]
    return out


@pytest.mark.parametrize("p,angles", [(oracle.PRESET_PAPER, [0, 30, 45, 60]),
                                      (oracle.PRESET_CUMULATIVE, [0, 30, 75, 120])])
def test_regular_48gon_closed_form(p, angles):
    x, y, m = inputs.regular_polygon(48, 3000, seed=7)
    slots, vals = oracle.extremes(x, y, p)
    want = [a // 7.5 for a in _slot_angles(angles)]
    assert list(slots) == want
    hull = oracle.hull_subset(x, y)
    assert sorted(hull) == list(range(48))
    # the polygon is the distinct slot vertices; interior points all go
    verts = oracle.polygon(x, y, slots)
    assert sorted(verts) == sorted(set(int(s) for s in slots))
    surv = oracle.discard(x, y, verts)
    assert list(surv) == list(range(48))
    assert list(oracle.compute(x, y, p)) == list(hull)


@pytest.mark.parametrize("phase", [0.0, 2.0, -2.5])
def test_extremes_dirs_regular_64gon(phase):
    """Closed form for the learned projection: a regular 64-gon whose vertex
    j sits at angle phase + 360 j / 64 (within half a step of the candidate
    direction 2 pi j / 64), with interior points.  The point of largest
    cos(phi_d) x + sin(phi_d) y is vertex d for every d: a swapped pair of
    constants (s x + c y) picks vertex 16 - d, a sign slip (c x - s y)
    vertex -d, a minimum instead of a maximum vertex d + 32."""
    x, y, m = inputs.regular_polygon(64, 5000, seed=11, phase_deg=phase)
    c, s = oracle.direction_table()
    slots, vals = oracle.extremes_dirs(x, y, c, s)
    assert list(slots) == list(range(64))
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    assert np.array_equal(vals, c * xd[:64] + s * yd[:64])
    # and on a shuffled copy, the slot follows the vertex to its new index
    perm = np.random.default_rng(5).permutation(len(x))
    slots2, _ = oracle.extremes_dirs(x[perm], y[perm], c, s)
    assert list(perm[slots2]) == list(range(64))


def test_extremes_tie_break_lowest_index():
    # points 2, 4, 6 share the minimum x; 1, 5 share the maximum y
    kx = [5, 6, 1, 7, 1, 3, 1]
    ky = [2, 9, 3, 4, 5, 9, 0]
    slots, _ = oracle.extremes(to_float(kx), to_float(ky), oracle.PRESET_PAPER)
    assert slots[0] == 2 and slots[3] == 1 and slots[1] == 3 and slots[2] == 6


def test_extremes_empty_and_single():
    slots, vals = oracle.extremes(np.zeros(0, np.float32), np.zeros(0, np.float32))
    assert (slots == oracle.NONE).all() and np.isnan(vals).all()
    slots, vals = oracle.extremes(to_float([3]), to_float([4]))
    assert (slots == 0).all()


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("p", [0, 1])
def test_extremes_match_numpy_elementwise(seed, p):
    x, y = inputs.DISTRIBUTIONS[["square", "disk", "gaussian", "annulus"][seed % 4]](5000, seed)
    c, s = oracle.preset(p)
    slots, vals = oracle.extremes(x, y, p)
    assert list(slots) == list(_brute.extremes_numpy(x, y, c, s))


@pytest.mark.parametrize("seed", range(4))
def test_cumulative_preset_aliases(seed):
    """With cos120 = -1/2 and sin120 = cos30 exactly, u(120) = -v(30) and
    v(120) = u(30) bit for bit, so slots 12..15 repeat slots 7, 6, 4, 5."""
    x, y = inputs.square(20000, seed)
    slots, vals = oracle.extremes(x, y, oracle.PRESET_CUMULATIVE)
    assert list(slots[12:16]) == [slots[7], slots[6], slots[4], slots[5]]
    assert vals[12] == -vals[7] and vals[15] == vals[5]


# -- Step 2 / Step 3 against the integer brute force -------------------------

@pytest.mark.parametrize("seed", range(12))
def test_polygon_and_discard_bruteforce(seed):
    r = np.random.default_rng(1000 + seed)
    kind = ["square", "disk", "gaussian", "annulus"][seed % 4]
    if seed >= 8:
        x, y = inputs.small_grid(300, int(r.integers(2, 9)), seed, (100, 100))
    else:
        x, y = inputs.DISTRIBUTIONS[kind](300, seed)
    slots, _ = oracle.extremes(x, y, seed % 2)
    verts = oracle.polygon(x, y, slots)
    # polygon == brute hull of the slot points
    uniq = sorted(set(int(s) for s in slots))
    bh = [uniq[j] for j in _brute.hull(x[uniq], y[uniq])]
    assert list(verts) == bh
    vx, vy = _brute.polygon_grid(x, y, verts)
    kx, ky = to_grid(x), to_grid(y)
    want = [i for i in range(len(x)) if not _brute.strictly_inside(int(kx[i]), int(ky[i]), vx, vy)]
    assert list(oracle.discard(x, y, verts)) == want


def test_discard_small_polygons_keep_everything():
    x, y = to_float([1, 5, 3, 3]), to_float([1, 5, 3, 2])
    for verts in ([], [0], [0, 1]):
        assert list(oracle.discard(x, y, np.array(verts, np.uint32))) == [0, 1, 2, 3]


def test_discard_boundary_points_survive():
    # square polygon 0..4, points on edges, at vertices, inside, outside
    x = to_float([0, 4, 4, 0, 2, 4, 2, 1, 5, 0])
    y = to_float([0, 0, 4, 4, 0, 2, 2, 3, 2, 2])
    surv = oracle.discard(x, y, np.array([0, 1, 2, 3], np.uint32))
    assert list(surv) == [0, 1, 2, 3, 4, 5, 8, 9]


# -- invariants of the whole method -----------------------------------------

@pytest.mark.parametrize("kind", ["square", "disk", "gaussian", "annulus"])
@pytest.mark.parametrize("p", [0, 1])
def test_method_invariants(kind, p):
    x, y = inputs.DISTRIBUTIONS[kind](30000, 17)
    hull, surv = oracle.compute(x, y, p, want_survivors=True)
    assert list(hull) == list(oracle.compute(x, y, nofilter=True))
    assert set(hull) <= set(surv)
    kx, ky = to_grid(x), to_grid(y)
    hx, hy = [int(kx[v]) for v in hull], [int(ky[v]) for v in hull]
    sset = set(int(v) for v in surv)
    rng = np.random.default_rng(3)
    disc = [i for i in rng.choice(len(x), 400, replace=False) if i not in sset]
    for i in disc:
        assert _brute.strictly_inside(int(kx[i]), int(ky[i]), hx, hy)
    # every filter vertex lies on the hull boundary
    slots, _ = oracle.extremes(x, y, p)
    verts = oracle.polygon(x, y, slots)
    m = len(hx)
    for v in verts:
        px, py = int(kx[v]), int(ky[v])
        on = False
        for e in range(m):
            ax, ay, bx, by = hx[e], hy[e], hx[(e + 1) % m], hy[(e + 1) % m]
            if (bx - ax) * (py - ay) - (by - ay) * (px - ax) == 0 and \
                    min(ax, bx) <= px <= max(ax, bx) and min(ay, by) <= py <= max(ay, by):
                on = True
                break
        assert on


def test_translation_invariance():
    kx = np.random.default_rng(5).integers(0, 1 << 20, size=(2, 20000))
    x, y = to_float(kx[0]), to_float(kx[1])
    base = oracle.compute(x, y)
    for dx, dy in [(12345, 0), (0, 999999), (1 << 22, 3 << 21)]:
        assert list(oracle.compute(to_float(kx[0] + dx), to_float(kx[1] + dy))) == list(base)


# -- discard statistics: closed forms and the paper's Tables 1-2 ------------

def _remaining_closed_form(dirs_deg):
    d = sorted(set(a % 360 for a in dirs_deg))
    gaps = [(d[(i + 1) % len(d)] - d[i]) % 360 for i in range(len(d))]
    return 1 - sum(math.sin(math.radians(g)) for g in gaps) / (2 * math.pi)


def _dirs(angles):
    return [a for t in angles for a in ((180 - t), -t, 270 - t, 90 - t)]


def test_closed_form_values():
    assert _remaining_closed_form(_dirs([0, 30, 45, 60])) == pytest.approx(0.03384, abs=5e-5)
    assert _remaining_closed_form(_dirs([0, 30, 75, 120])) == pytest.approx(0.06676, abs=5e-5)


@pytest.mark.parametrize("p,angles", [(0, [0, 30, 45, 60]), (1, [0, 30, 75, 120])])
def test_disk_remaining_fraction(p, angles):
    n = 1_000_000
    x, y = inputs.disk(n, 2024)
    _, surv = oracle.compute(x, y, p, want_survivors=True)
    frac = len(surv) / n
    assert frac == pytest.approx(_remaining_closed_form(_dirs(angles)), abs=1.5e-3)
    if p == 0:
        tab = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
        assert frac * 100 == pytest.approx(tab["table2_circle_remaining_percent"]["1000000"], abs=0.15)


@pytest.mark.parametrize("p,angles", [(0, [0, 30, 45, 60]), (1, [0, 30, 75, 120])])
def test_annulus_discard_fraction(p, angles):
    # The extreme points deviate from the ideal directions by ~0.5 degree at
    # 1M points, which moves the annulus fraction by up to ~1 % per set, so
    # average four sets.
    n = 1_000_000
    fr = []
    for seed in range(4):
        x, y = inputs.annulus(n, 2025 + seed)
        _, surv = oracle.compute(x, y, p, want_survivors=True)
        fr.append(1 - len(surv) / n)
    # polygon inscribed in r = 1/2: area (1/2) r^2 sum sin(gap); inner disk r=0.45
    rem = _remaining_closed_form(_dirs(angles))
    a_poly = math.pi * 0.25 * (1 - rem)
    disc = (a_poly - math.pi * 0.2025) / (math.pi * (0.25 - 0.2025))
    assert np.mean(fr) == pytest.approx(disc, abs=3e-3 if p == 0 else 6e-3)


def test_square_remaining_matches_table1():
    tab = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
    fr = []
    for seed in range(4):
        x, y = inputs.square(1_000_000, 300 + seed)
        _, surv = oracle.compute(x, y, want_survivors=True)
        fr.append(len(surv) / 1e6 * 100)
    # Table 1 reports 0.06 % at 1M; more than 99 % discarded (Sec. 3)
    assert np.mean(fr) == pytest.approx(tab["table1_square_remaining_percent"]["1000000"], abs=0.04)
    assert max(fr) < 1.0


# -- learned-proposal helpers -----------------------------------------------

def test_histogram_hand_cases():
    h = oracle.histogram(to_float([0, 99, 0, 99]), to_float([0, 0, 99, 99]))
    want = np.zeros(1024, np.float32)
    for b in (0, 31, 31 * 32, 31 * 32 + 31):
        want[b] = 256.0
    assert (h == want).all()
    h = oracle.histogram(to_float([7] * 10), to_float([9] * 10))
    assert h[0] == 1024.0 and h[1:].sum() == 0
    # runs: n = 64 + 255 * 128 = 32704 -> 256 runs of 64 points starting at
    # multiples of 128, i.e. the points i with i % 128 < 64; every sampled
    # point sits at (0, 0) and every other one at (1000, 1000), so the
    # sampled points alone give a 1 x 1 window and all the mass in bin 0
    i = np.arange(32704)
    kx = np.where(i % 128 < 64, 0, 1000)
    h = oracle.histogram(to_float(kx), to_float(kx))
    assert h[0] == 1024.0 and h[1:].sum() == 0
    # one more point: run r starts at floor(r * 32641 / 255) = 128 r + floor(r / 255),
    # so only the last run moves (to 32641 .. 32704) and point 32704 is sampled
    kx2 = np.concatenate([kx, [1000]])
    kx2[32640] = 1000        # the last run's old first point, now unsampled
    kx2[32641:] = 0
    h = oracle.histogram(to_float(kx2), to_float(kx2))
    assert h[0] == 1024.0 and h[1:].sum() == 0
    # 16384 points or fewer: every point (a 2 x 1 box in a 2 x 2 window: bins 0 and 16)
    kx3 = np.arange(16384) % 2
    h = oracle.histogram(to_float(kx3), to_float(np.zeros(16384, np.int64)))
    assert h.sum() == pytest.approx(1024.0, rel=1e-6) and np.count_nonzero(h) == 2
    # aspect ratio kept: a 3200 x 100 box sits in the middle rows of a
    # 3200 x 3200 window (origin y = -1550): rows 15 and 16 only
    kx = np.array([0, 3199, 1600, 0, 3199], np.int64)
    ky = np.array([0, 99, 50, 99, 0], np.int64)
    h = oracle.histogram(to_float(kx), to_float(ky)).reshape(32, 32)
    assert h.sum() == pytest.approx(1024.0)
    rows = set(np.nonzero(h.sum(1))[0])
    assert rows == {15, 16}
    assert h[15, 0] > 0 and h[15, 31] > 0 and h[16, 0] > 0 and h[16, 31] > 0 and h[16, 16] > 0
    # the same box rotated by 90 degrees: columns 15 and 16 only
    h2 = oracle.histogram(to_float(ky), to_float(kx)).reshape(32, 32)
    assert np.array_equal(h2, h.T)


def test_labels_bruteforce():
    x, y = inputs.mixture(400, 11)
    gain = oracle.labels(x, y, 0)
    c, s = oracle.preset(0)
    slots = _brute.extremes_numpy(x, y, c, s)
    kx, ky = to_grid(x), to_grid(y)
    uniq = sorted(set(int(v) for v in slots))
    base = [uniq[j] for j in _brute.hull(x[uniq], y[uniq])]
    bx, by = [int(kx[v]) for v in base], [int(ky[v]) for v in base]
    surv = [i for i in range(len(x)) if not _brute.strictly_inside(int(kx[i]), int(ky[i]), bx, by)]
    cd, sd = oracle.direction_table()
    w = np.outer(cd, x.astype(np.float64)) + np.outer(sd, y.astype(np.float64))
    for d in range(64):
        e = int(np.argmax(w[d]))
        u2 = sorted(set(uniq) | {e})
        v2 = [u2[j] for j in _brute.hull(x[u2], y[u2])]
        vx, vy = [int(kx[v]) for v in v2], [int(ky[v]) for v in v2]
        cnt = sum(_brute.strictly_inside(int(kx[i]), int(ky[i]), vx, vy) for i in surv)
        assert gain[d] == cnt / len(x), d


def _greedy_bruteforce(x, y, rounds):
    """Greedy joint targets by brute force (exact integer geometry)."""
    c, s = oracle.preset(0)
    slots = _brute.extremes_numpy(x, y, c, s)
    kx, ky = to_grid(x), to_grid(y)
    E = set(int(v) for v in slots)
    cache = {}

    def poly(pts):
        key = frozenset(pts)
        if key not in cache:
            u = sorted(key)
            v = [u[j] for j in _brute.hull(x[u], y[u])]
            cache[key] = ([int(kx[i]) for i in v], [int(ky[i]) for i in v])
        return cache[key]

    bx, by = poly(E)
    surv = [i for i in range(len(x)) if not _brute.strictly_inside(int(kx[i]), int(ky[i]), bx, by)]
    cd, sd = oracle.direction_table()
    w = np.outer(cd, x.astype(np.float64)) + np.outer(sd, y.astype(np.float64))
    ext = [int(np.argmax(w[d])) for d in range(64)]
    order, g0 = [], None
    for r in range(rounds):
        cx, cy = poly(E)
        active = [i for i in surv if not _brute.strictly_inside(int(kx[i]), int(ky[i]), cx, cy)]
        gains = []
        for d in range(64):
            vx, vy = poly(E | {ext[d]})
            gains.append(sum(_brute.strictly_inside(int(kx[i]), int(ky[i]), vx, vy) for i in active))
        if r == 0:
            g0 = gains
        if max(gains) == 0:
            break
        best = gains.index(max(gains))
        order.append(best)
        E = E | {ext[best]}
    gmax = max(g0)
    target = [np.float32(0.5 * (g / gmax)) if gmax > 0 else np.float32(0) for g in g0]
    for r, d in enumerate(order):
        target[d] = np.float32(1.0 - r / (2.0 * rounds))
    return np.array(target, np.float32), order + [-1] * (rounds - len(order))


@pytest.mark.parametrize("kind,seed", [("mixture", 11), ("ellipse", 4)])
def test_label_targets_bruteforce(kind, seed):
    """Greedy joint targets: the oracle equals a brute-force greedy run with
    exact integer geometry, and its first choice is the argmax of the
    (independently pinned) marginal gains."""
    x, y = getattr(inputs, kind)(250, seed)
    t, o = oracle.label_targets(x, y, rounds=8)
    bt, bo = _greedy_bruteforce(x, y, 8)
    assert list(o) == bo
    assert np.array_equal(t, bt)
    gain = oracle.labels(x, y, 0)
    if gain.max() > 0:
        assert o[0] == int(np.argmax(gain))
    # chosen directions rank first, in round order
    chosen = [d for d in o if d >= 0]
    assert list(np.argsort(-t, kind="stable")[:len(chosen)]) == chosen


def test_label_targets_degenerate():
    """No survivors to gain (a triangle's vertices): every target is 0 and the
    sequence is empty; an empty set gives the same."""
    x = np.array([0.25, 0.75, 0.5], np.float32)
    y = np.array([0.25, 0.25, 0.75], np.float32)
    t, o = oracle.label_targets(x, y, rounds=4)
    assert not t.any() and list(o) == [-1] * 4
    t, o = oracle.label_targets(x[:0], y[:0], rounds=4)
    assert not t.any() and list(o) == [-1] * 4


# -- direction families: the min/max quadrilateral (Sec. 1, ref. [3]) and 4G
#    evenly spaced directions ----------------------------------------------

EVEN = sorted(oracle.EVEN_PRESETS.items())       # (preset, directions)


def _even_angles(p):
    G = oracle.EVEN_PRESETS[p] // 4
    return [90.0 * j / G for j in range(G)]


@pytest.mark.parametrize("p,ndir", EVEN)
def test_even_preset_constants_correctly_rounded(p, ndir):
    c, s = oracle.preset(p)
    G = ndir // 4
    assert len(c) == G
    for j in range(G):
        cc, ss = _cr_cos_sin(j, 4 * G)          # 90 j / G degrees = 2 pi j / (4 G)
        assert c[j] == cc and s[j] == ss, (p, j, c[j].hex(), cc.hex(), s[j].hex(), ss.hex())


@pytest.mark.parametrize("p,ndir", EVEN)
def test_even_preset_regular_polygon_closed_form(p, ndir):
    """A regular N-gon whose vertex spacing divides 90/G degrees: slot k of
    group j is the vertex at the slot's direction (slot order and rotation
    sign as for the paper's presets), the filter polygon is the set of those
    vertices, and with G >= 2 its inradius exceeds the interior points'
    radius, so only the N-gon's own vertices survive."""
    G = ndir // 4
    N = 40 if G == 5 else 48
    x, y, m = inputs.regular_polygon(N, 3000, seed=8)
    slots, _ = oracle.extremes(x, y, p)
    assert len(slots) == ndir
    want = [round(a / (360 / N)) % N for a in _slot_angles(_even_angles(p))]
    assert list(slots) == want
    verts = oracle.polygon(x, y, slots)
    assert sorted(verts) == sorted(set(int(s) for s in slots))
    assert len(verts) == ndir
    surv = oracle.discard(x, y, verts)
    if G >= 2:
        assert list(surv) == list(range(N))
    else:       # the quadrilateral's inradius 0.4/sqrt(2) < 0.3: brute force
        vx, vy = _brute.polygon_grid(x, y, verts)
        kx, ky = to_grid(x), to_grid(y)
        want = [i for i in range(len(x)) if not _brute.strictly_inside(int(kx[i]), int(ky[i]), vx, vy)]
        assert list(surv) == want
        assert set(range(N)) <= set(int(v) for v in surv)
    assert list(oracle.compute(x, y, p)) == list(oracle.hull_subset(x, y))


def test_even_closed_form_values():
    # disk remaining with 4 axis directions: 1 - 2/pi; with 16 even ones 2.550 %
    assert _remaining_closed_form(_dirs([0])) == pytest.approx(1 - 2 / math.pi, abs=1e-12)
    assert _remaining_closed_form(_dirs([0])) == pytest.approx(0.3634, abs=5e-5)
    assert _remaining_closed_form(_dirs([0, 22.5, 45, 67.5])) == pytest.approx(0.02550, abs=5e-5)


@pytest.mark.parametrize("p,ndir", EVEN)
def test_even_disk_remaining_fraction(p, ndir):
    n = 1_000_000
    x, y = inputs.disk(n, 2024)
    _, surv = oracle.compute(x, y, p, want_survivors=True)
    frac = len(surv) / n
    assert frac == pytest.approx(_remaining_closed_form(_dirs(_even_angles(p))), abs=1.5e-3)


@pytest.mark.parametrize("p,ndir", EVEN)
def test_even_method_invariants(p, ndir):
    x, y = inputs.DISTRIBUTIONS["gaussian"](20000, 21 + p)
    hull, surv = oracle.compute(x, y, p, want_survivors=True)
    assert list(hull) == list(oracle.compute(x, y, nofilter=True))
    # a family whose directions include another's finds the same extreme
    # points for the shared ones (same constants, same arithmetic), so its
    # polygon contains the other's and it keeps a subset of the survivors:
    # 4 in every family, 8 in 16 and 24, 12 in 24
    supersets = {2: [3, 4, 5, 6, 7], 3: [5, 7], 4: [7]}
    for q in supersets.get(p, []):
        _, s2 = oracle.compute(x, y, q, want_survivors=True)
        assert set(int(v) for v in s2) <= set(int(v) for v in surv), (p, q)
