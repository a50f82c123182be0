"""Exact brute-force geometry on Python integers, for pinning the oracle.

Independent of the oracle: hull edges are found by testing every ordered
pair of distinct points against all others (O(n^3)), and strict interiority
uses the triangle-fan area decomposition instead of per-edge signs.
"""
import numpy as np

from paper_1405_3454_amd.inputs import to_grid


def _uniq(kx, ky):
    first = {}
    for i, (a, b) in enumerate(zip(kx, ky)):
        first.setdefault((int(a), int(b)), i)
    return first


def hull(x, y):
    """CCW hull vertex indices from the lexicographic minimum, collinear points
    excluded, lowest index per repeated coordinate."""
    kx, ky = to_grid(x), to_grid(y)
    first = _uniq(kx, ky)
    P = sorted(first)
    if not P:
        return []
    if len(P) == 1:
        return [first[P[0]]]
    nxt = {}
    for a in P:
        for b in P:
            if a == b:
                continue
            ok = True
            ex, ey = b[0] - a[0], b[1] - a[1]
            for c in P:
                cr = ex * (c[1] - a[1]) - ey * (c[0] - a[0])
                if cr < 0:
                    ok = False
                    break
                if cr == 0:
                    d1 = (c[0] - a[0]) * ex + (c[1] - a[1]) * ey
                    d2 = (c[0] - b[0]) * (-ex) + (c[1] - b[1]) * (-ey)
                    if d1 < 0 or d2 < 0:
                        ok = False
                        break
            if ok:
                assert a not in nxt, "two hull edges leave one vertex"
                nxt[a] = b
    out = [P[0]]
    cur = nxt[P[0]]
    while cur != P[0]:
        out.append(cur)
        cur = nxt[cur]
        assert len(out) <= len(P)
    return [first[p] for p in out]


def strictly_inside(px, py, vx, vy):
    """Is the integer point (px, py) strictly inside the convex polygon with
    integer vertices (vx, vy) listed counter-clockwise?  Uses the fan of
    triangles around p: p is strictly inside iff the unsigned fan areas sum
    to the polygon's shoelace area and none of them is zero."""
    m = len(vx)
    if m < 3:
        return False
    area2 = sum(vx[i] * vy[(i + 1) % m] - vx[(i + 1) % m] * vy[i] for i in range(m))
    tot = 0
    for i in range(m):
        ax, ay = vx[i] - px, vy[i] - py
        bx, by = vx[(i + 1) % m] - px, vy[(i + 1) % m] - py
        t = ax * by - ay * bx
        if t == 0:
            return False
        tot += abs(t)
    return tot == abs(area2)


def polygon_grid(x, y, verts):
    kx, ky = to_grid(x), to_grid(y)
    return [int(kx[v]) for v in verts], [int(ky[v]) for v in verts]


def extremes_numpy(x, y, c, s):
    """Slots by numpy elementwise binary64 (each op rounded) + first-index
    argmin/argmax."""
    xd = np.asarray(x, np.float64)
    yd = np.asarray(y, np.float64)
    out = []
    for cg, sg in zip(c, s):
        u = cg * xd - sg * yd
        v = sg * xd + cg * yd
        out += [int(np.argmin(u)), int(np.argmax(u)), int(np.argmin(v)), int(np.argmax(v))]
    return np.array(out, np.uint32)
