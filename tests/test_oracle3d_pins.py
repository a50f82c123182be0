"""Pins of the 3D oracle (oracle/hull3d_oracle.c) against facts it does not
compute itself: Caratheodory brute force on tiny lattices, Qhull's vertex
sets on general-position sets, closed forms (cube lattices, flat and
collinear sets), the pinned 2D oracle on sets that lie in a coordinate
plane, and the method's invariants.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import hull3d as o3

G24 = float(1 << 24)


def grid(k):
    return (np.asarray(k, np.float64) / G24).astype(np.float32)


def pts(k):
    k = np.asarray(k, np.int64)
    return grid(k[:, 0]), grid(k[:, 1]), grid(k[:, 2])


def _orient(a, b, c, d):
    ux, uy, uz = b[0] - a[0], b[1] - a[1], b[2] - a[2]
    vx, vy, vz = c[0] - a[0], c[1] - a[1], c[2] - a[2]
    wx, wy, wz = d[0] - a[0], d[1] - a[1], d[2] - a[2]
    return ux * (vy * wz - vz * wy) - uy * (vx * wz - vz * wx) + uz * (vx * wy - vy * wx)


def _in_segment(p, a, b):
    cr = (a[1] - p[1]) * (b[2] - p[2]) - (a[2] - p[2]) * (b[1] - p[1]), \
         (a[2] - p[2]) * (b[0] - p[0]) - (a[0] - p[0]) * (b[2] - p[2]), \
         (a[0] - p[0]) * (b[1] - p[1]) - (a[1] - p[1]) * (b[0] - p[0])
    if any(cr):
        return False
    return all(min(a[i], b[i]) <= p[i] <= max(a[i], b[i]) for i in range(3))


def _in_triangle(p, a, b, c):
    if _orient(a, b, c, p) != 0:
        return False
    # p = a + s (b - a) + t (c - a), s, t >= 0, s + t <= 1, via 2D projections
    n = np.cross(np.array(b) - np.array(a), np.array(c) - np.array(a))
    if not n.any():
        return _in_segment(p, a, b) or _in_segment(p, b, c) or _in_segment(p, a, c)
    drop = int(np.argmax(np.abs(n)))
    keep = [i for i in range(3) if i != drop]
    A, B, C, P = ([q[keep[0]], q[keep[1]]] for q in (a, b, c, p))

    def cr(o, u, v):
        return (u[0] - o[0]) * (v[1] - o[1]) - (u[1] - o[1]) * (v[0] - o[0])
    d1, d2, d3 = cr(A, B, P), cr(B, C, P), cr(C, A, P)
    return (d1 >= 0 and d2 >= 0 and d3 >= 0) or (d1 <= 0 and d2 <= 0 and d3 <= 0)


def _in_tetra(p, a, b, c, d):
    o = _orient(a, b, c, d)
    if o == 0:
        return _in_triangle(p, a, b, c) or _in_triangle(p, a, b, d) or \
            _in_triangle(p, a, c, d) or _in_triangle(p, b, c, d)
    s = [_orient(a, b, c, p), _orient(a, b, p, d), _orient(a, p, c, d), _orient(p, b, c, d)]
    return all(v * o >= 0 for v in s)


def brute_extreme(k):
    """Caratheodory: a point is not extreme iff it lies in a (possibly flat)
    simplex of at most four other distinct points.  Lowest index per repeated
    coordinate triple."""
    P = [tuple(int(v) for v in row) for row in k]
    first = {}
    for i, p in enumerate(P):
        first.setdefault(p, i)
    uniq = sorted(first.items(), key=lambda kv: kv[1])
    out = []
    for p, i in uniq:
        others = [q for q, j in uniq if j != i]
        inside = False
        for r in (1, 2, 3, 4):
            for comb in itertools.combinations(others, r):
                if r == 1:
                    inside = comb[0] == p
                elif r == 2:
                    inside = _in_segment(p, *comb)
                elif r == 3:
                    inside = _in_triangle(p, *comb)
                else:
                    inside = _in_tetra(p, *comb)
                if inside:
                    break
            if inside:
                break
        if not inside:
            out.append(i)
    return np.array(sorted(out), np.uint32)


@pytest.mark.parametrize("seed", range(16))
def test_bruteforce_tiny_lattices(seed):
    r = np.random.default_rng(seed)
    n = int(r.integers(1, 14))
    side = int(r.integers(1, 4))
    k = r.integers(0, side + 1, size=(n, 3)) * 3 + 1000
    if seed % 4 == 0:           # flat: one plane
        k[:, 2] = k[:, 0] + k[:, 1]
    if seed % 8 == 1:           # collinear
        k[:, 1] = k[:, 0]
        k[:, 2] = 2 * k[:, 0]
    x, y, z = pts(k)
    assert np.array_equal(o3.hull_subset(x, y, z), brute_extreme(k)), (seed, k)


@pytest.mark.parametrize("n", [4, 50, 3000])
@pytest.mark.parametrize("shape", ["cube", "ball"])
def test_qhull_general_position(n, shape):
    from scipy.spatial import ConvexHull
    r = np.random.default_rng(n)
    k = r.integers(0, 1 << 24, size=(4 * n, 3))
    if shape == "ball":
        d = (k - (1 << 23)).astype(np.float64)
        k = k[(d ** 2).sum(1) < float(1 << 46)]
    k = k[:n]
    x, y, z = pts(k)
    want = np.sort(ConvexHull(k.astype(np.float64)).vertices).astype(np.uint32)
    assert np.array_equal(o3.hull_subset(x, y, z), want)


def test_cube_lattice_only_corners():
    """3x3x3 lattice of a cube: face centres, edge midpoints and the centre
    lie on the hull or inside it but are not corners."""
    k = np.array([(a, b, c) for a in (0, 4, 8) for b in (0, 4, 8) for c in (0, 4, 8)]) + 77
    order = np.random.default_rng(3).permutation(len(k))
    k = k[order]
    x, y, z = pts(k)
    want = np.sort(np.nonzero(np.all((k - 77) % 8 == 0, axis=1))[0]).astype(np.uint32)
    assert np.array_equal(o3.hull_subset(x, y, z), want)


def test_degenerate_cases():
    x, y, z = pts([[5, 6, 7]])
    assert list(o3.hull_subset(x, y, z)) == [0]
    x, y, z = pts([[5, 6, 7]] * 4)
    assert list(o3.hull_subset(x, y, z)) == [0]
    # collinear: the two ends
    x, y, z = pts([[i, 2 * i, 3 * i] for i in (4, 1, 9, 2)])
    assert list(o3.hull_subset(x, y, z)) == [1, 2]
    # a tilted square with its centre and edge midpoints: four corners
    sq = [[0, 0, 0], [4, 0, 4], [0, 4, 4], [4, 4, 8], [2, 2, 4], [2, 0, 2], [0, 2, 2]]
    x, y, z = pts(np.array(sq) + 10)
    assert list(o3.hull_subset(x, y, z)) == [0, 1, 2, 3]
    assert len(o3.hull_subset(*pts(np.zeros((0, 3), np.int64)))) == 0


@pytest.mark.parametrize("seed", range(4))
def test_extremes_reduce_to_the_2d_oracle(seed):
    """For points in a plane z = const the slots of the rotations about z are
    the 2D oracle's slots of (x, y); likewise (y, z) for x = const about x and
    (z, x) for y = const about y."""
    from paper_1405_3454_amd import inputs
    n = 3000
    a, b = inputs.disk(n, 40 + seed)
    cst = np.full(n, 0.25, np.float32)
    for p in (0, 1, 3):
        G = len(oracle.preset(p)[0])
        for k, (X, Y, Z) in enumerate([(a, b, cst), (cst, a, b), (b, cst, a)]):
            s3, v3 = o3.extremes(X, Y, Z, p)
            s2, v2 = oracle.extremes(a, b, p)
            for g in range(1, G):
                base = 6 + 4 * ((G - 1) * k + g - 1)
                assert np.array_equal(s3[base:base + 4], s2[4 * g:4 * g + 4]), (p, k, g)
                assert np.array_equal(v3[base:base + 4], v2[4 * g:4 * g + 4])
            # the axis slots of the plane's own coordinates
            ax = [(0, 1), (1, 2), (2, 0)][k]
            assert np.array_equal(s3[[2 * ax[0], 2 * ax[0] + 1, 2 * ax[1], 2 * ax[1] + 1]], s2[0:4])


@pytest.mark.parametrize("seed", range(6))
def test_method_invariants(seed):
    """hull(filtered) == hull(all); every discarded point is strictly inside
    the polyhedron's planes and not a corner of the hull; every filter point
    is on the hull's boundary (inside or on, never strictly outside)."""
    r = np.random.default_rng(seed)
    n = 4000
    k = r.integers(0, 1 << 24, size=(3 * n, 3))
    if seed % 2:
        d = (k - (1 << 23)).astype(np.float64)
        k = k[(d ** 2).sum(1) < float(1 << 46)]
    k = k[:n]
    if seed >= 4:
        k = (k >> 18) << 18            # coarse lattice: ties and coplanar points
    x, y, z = pts(k)
    for p in (0, 1, 2, 5):
        h_all = o3.compute(x, y, z, p, nofilter=True)
        h, surv = o3.compute(x, y, z, p, want_survivors=True)
        assert np.array_equal(h, h_all)
        assert np.isin(h, surv).all()
        slots, _ = o3.extremes(x, y, z, p)
        planes = o3.polyhedron(x, y, z, slots)
        disc = np.setdiff1d(np.arange(n), surv)
        # exact products: Python integers (|n . d| reaches 2^75)
        q = k[disc].astype(object)
        ks = k[slots].astype(object)
        for row in planes.astype(object):
            nrm, a = row[:3], row[3:]
            assert ((q - a).dot(nrm) > 0).all()
            # slot points are on the inner side or on the plane
            assert ((ks - a).dot(nrm) >= 0).all()


def test_discard_fraction_ball_and_cube():
    """More directions never keep more points (the polyhedron of a superset
    of extremes contains the smaller one when the sets nest: preset 7's
    directions contain preset 4's and preset 3's)."""
    r = np.random.default_rng(11)
    k = r.integers(0, 1 << 24, size=(60_000, 3))
    d = (k - (1 << 23)).astype(np.float64)
    k = k[(d ** 2).sum(1) < float(1 << 46)][:20_000]
    x, y, z = pts(k)
    kept = {}
    for p in (2, 3, 4, 7):
        _, surv = o3.compute(x, y, z, p, want_survivors=True)
        kept[p] = set(surv.tolist())
    assert kept[7] <= kept[4] <= kept[2]
    assert kept[3] <= kept[2]
