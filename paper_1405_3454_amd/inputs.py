"""Seeded synthetic point sets on the 2^-24 grid of [0, 1)^2.

This module only draws input coordinates; it holds none of the hull method's
arithmetic and is the one piece of code that both the GPU path's tests and
the CPU oracle's tests use.  Every coordinate is a float32 k * 2^-24 with
integer 0 <= k < 2^24, so it is exact in float32 and binary64.

The shapes follow the paper's workloads (Sec. 3): uniform points in a square
and in a circle (the paper draws them with Qhull's rbox, which is not used
here).  The Gaussian, annulus, anisotropic mixture and thin-ellipse sets are
this project's additional stress shapes.
"""
import numpy as np

GRID = 1 << 24
HALF = 1 << 23
_SCALE = np.float32(1.0 / GRID)


def to_float(k):
    """Integer grid coordinates -> exact float32 coordinates."""
    return np.asarray(k, dtype=np.float32) * _SCALE


def to_grid(v):
    """float32 grid coordinates -> integers (exact)."""
    return (np.asarray(v, dtype=np.float64) * GRID).astype(np.int64)


def _rng(seed):
    return np.random.default_rng(seed)


def square(n, seed):
    """Uniform in the unit square: kx, ky i.i.d. uniform on [0, 2^24)."""
    r = _rng(seed)
    kx = r.integers(0, GRID, size=n, dtype=np.int32)
    ky = r.integers(0, GRID, size=n, dtype=np.int32)
    return to_float(kx), to_float(ky)


def _reject_int(n, seed, accept):
    """Uniform integer pairs on the grid filtered by accept(dx, dy) where
    dx, dy are offsets from the centre (2^23, 2^23)."""
    r = _rng(seed)
    kx = np.empty(n, np.int32)
    ky = np.empty(n, np.int32)
    got = 0
    while got < n:
        m = max(1024, int((n - got) * 1.35) + 1024)
        a = r.integers(0, GRID, size=m, dtype=np.int32)
        b = r.integers(0, GRID, size=m, dtype=np.int32)
        dx = a.astype(np.int64) - HALF
        dy = b.astype(np.int64) - HALF
        ok = accept(dx, dy)
        a = a[ok]
        b = b[ok]
        t = min(len(a), n - got)
        kx[got:got + t] = a[:t]
        ky[got:got + t] = b[:t]
        got += t
    return kx, ky


def disk(n, seed):
    """Uniform in the disk of radius 1/2 centred at (1/2, 1/2), by integer
    rejection: (kx - 2^23)^2 + (ky - 2^23)^2 < 2^46."""
    kx, ky = _reject_int(n, seed, lambda dx, dy: dx * dx + dy * dy < (1 << 46))
    return to_float(kx), to_float(ky)


ANNULUS_R2_MIN = (2025 * (1 << 48) + 9999) // 10000   # ceil(0.45^2 * 2^48)


def annulus(n, seed):
    """Uniform (in area) in the annulus 0.45 <= r < 0.5 around (1/2, 1/2):
    ceil(0.2025 * 2^48) <= d^2 < 2^46 in grid units."""
    def acc(dx, dy):
        d2 = dx * dx + dy * dy
        return (d2 < (1 << 46)) & (d2 >= ANNULUS_R2_MIN)
    kx, ky = _reject_int(n, seed, acc)
    return to_float(kx), to_float(ky)


def _reject_real(n, r, draw):
    """Draw binary64 pairs with draw(m) until n fall inside [0,1)^2; floor to
    the grid."""
    kx = np.empty(n, np.int32)
    ky = np.empty(n, np.int32)
    got = 0
    while got < n:
        m = max(1024, int((n - got) * 1.2) + 1024)
        px, py = draw(m)
        ok = (px >= 0) & (px < 1) & (py >= 0) & (py < 1)
        a = np.floor(px[ok] * GRID).astype(np.int64)
        b = np.floor(py[ok] * GRID).astype(np.int64)
        ok2 = (a < GRID) & (b < GRID)
        a = a[ok2]
        b = b[ok2]
        t = min(len(a), n - got)
        kx[got:got + t] = a[:t]
        ky[got:got + t] = b[:t]
        got += t
    return to_float(kx), to_float(ky)


def gaussian(n, seed, sigma=0.15):
    """2D Gaussian around (1/2, 1/2), standard deviation sigma, resampled
    (not clamped) into [0, 1)^2."""
    r = _rng(seed)
    return _reject_real(n, r, lambda m: (0.5 + sigma * r.standard_normal(m),
                                         0.5 + sigma * r.standard_normal(m)))


def gaussian_clamped(n, seed, sigma=0.15):
    """Like gaussian() but clamped onto the square's border: a stress input
    with many collinear boundary points."""
    r = _rng(seed)
    px = np.clip(0.5 + sigma * r.standard_normal(n), 0.0, 1.0 - 1.0 / GRID)
    py = np.clip(0.5 + sigma * r.standard_normal(n), 0.0, 1.0 - 1.0 / GRID)
    return (to_float(np.floor(px * GRID).astype(np.int64)),
            to_float(np.floor(py * GRID).astype(np.int64)))


def mixture(n, seed):
    """Anisotropic Gaussian mixture: K ~ U{1..8} components, Dirichlet(1)
    weights, means U[0.25, 0.75]^2, major sigma U[0.02, 0.12], axis ratio
    log-uniform in [1, 50], rotation U[0, pi); resampled into [0, 1)^2."""
    r = _rng(seed)
    K = int(r.integers(1, 9))
    w = r.dirichlet(np.ones(K))
    mu = r.uniform(0.25, 0.75, size=(K, 2))
    smaj = r.uniform(0.02, 0.12, size=K)
    ratio = np.exp(r.uniform(0.0, np.log(50.0), size=K))
    rot = r.uniform(0.0, np.pi, size=K)

    def draw(m):
        comp = r.choice(K, size=m, p=w)
        a = r.standard_normal(m) * smaj[comp]
        b = r.standard_normal(m) * (smaj[comp] / ratio[comp])
        c, s = np.cos(rot[comp]), np.sin(rot[comp])
        return mu[comp, 0] + c * a - s * b, mu[comp, 1] + s * a + c * b
    return _reject_real(n, r, draw)


def ellipse(n, seed):
    """Uniform in a thin rotated ellipse: centre 0.5 +- 0.05, semi-major
    U[0.2, 0.44], axis ratio log-uniform in [20, 200], rotation U[0, pi).  The
    unit disk is sampled by integer rejection, mapped affinely in binary64 and
    floored to the grid."""
    r = _rng(seed)
    cx, cy = r.uniform(0.45, 0.55, size=2)
    a = r.uniform(0.2, 0.44)
    b = a / np.exp(r.uniform(np.log(20.0), np.log(200.0)))
    th = r.uniform(0.0, np.pi)
    c, s = np.cos(th), np.sin(th)
    sub = int(r.integers(0, 2**31))
    kx, ky = _reject_int(n, sub, lambda dx, dy: dx * dx + dy * dy < (1 << 46))
    ux = (kx.astype(np.float64) - HALF) / HALF
    uy = (ky.astype(np.float64) - HALF) / HALF
    px = cx + c * a * ux - s * b * uy
    py = cy + s * a * ux + c * b * uy
    gx = np.clip(np.floor(px * GRID), 0, GRID - 1).astype(np.int64)
    gy = np.clip(np.floor(py * GRID), 0, GRID - 1).astype(np.int64)
    return to_float(gx), to_float(gy)


DISTRIBUTIONS = {
    "square": square,
    "disk": disk,
    "gaussian": gaussian,
    "annulus": annulus,
}


# ---------------------------------------------------------------------------
# Three dimensions (the 3D form of the method): three float32 arrays on the
# grid of [0, 1)^3.

def cube3(n, seed):
    """Uniform in the unit cube."""
    r = _rng(seed)
    k = r.integers(0, GRID, size=(3, n), dtype=np.int32)
    return to_float(k[0]), to_float(k[1]), to_float(k[2])


def _reject3(n, seed, accept, factor):
    r = _rng(seed)
    out = np.empty((3, n), np.int32)
    got = 0
    while got < n:
        m = max(1024, int((n - got) * factor) + 1024)
        k = r.integers(0, GRID, size=(3, m), dtype=np.int32)
        d = k.astype(np.int64) - HALF
        ok = accept(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
        k = k[:, ok]
        t = min(k.shape[1], n - got)
        out[:, got:got + t] = k[:, :t]
        got += t
    return to_float(out[0]), to_float(out[1]), to_float(out[2])


def ball3(n, seed):
    """Uniform in the ball of radius 1/2 about the cube's centre (integer
    rejection: |k - 2^23|^2 < 2^46)."""
    return _reject3(n, seed, lambda d2: d2 < (1 << 46), 2.0)


def shell3(n, seed):
    """Uniform in the spherical shell 0.45 <= r < 0.5 (integer rejection)."""
    lo = int(np.ceil(0.2025 * float(1 << 48)))
    return _reject3(n, seed, lambda d2: (d2 < (1 << 46)) & (d2 >= lo), 8.0)


def gaussian3(n, seed, sigma=0.15):
    """3D normal about the centre, sigma 0.15, resampled into the cube."""
    r = _rng(seed)
    out = np.empty((3, n), np.int64)
    got = 0
    while got < n:
        m = max(1024, int((n - got) * 1.2) + 1024)
        v = 0.5 + sigma * r.standard_normal(size=(3, m))
        ok = np.all((v >= 0.0) & (v < 1.0), axis=0)
        v = v[:, ok]
        t = min(v.shape[1], n - got)
        out[:, got:got + t] = np.floor(v[:, :t] * GRID).astype(np.int64)
        got += t
    return to_float(out[0]), to_float(out[1]), to_float(out[2])


def lattice3(n, side, seed, offset=0):
    """n points of a side^3 integer lattice (duplicates, coplanar and
    collinear points), offset by `offset` grid units."""
    r = _rng(seed)
    k = r.integers(0, side, size=(3, n)) + offset
    return to_float(k[0]), to_float(k[1]), to_float(k[2])


DISTRIBUTIONS3 = {"cube": cube3, "ball": ball3, "shell": shell3, "gaussian": gaussian3}


def set3_torch(kind, n, seed, device="cuda:0"):
    """One 3D set drawn on the device (cube, ball, shell, gaussian)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    if kind == "gaussian":
        out = []
        got = 0
        while got < n:
            v = 0.5 + 0.15 * torch.randn((3, int((n - got) * 1.2) + 1024), generator=g, device=device,
                                         dtype=torch.float64)
            v = v[:, ((v >= 0) & (v < 1)).all(0)]
            out.append(v[:, : n - got])
            got += out[-1].shape[1]
        k = torch.floor(torch.cat(out, 1) * GRID).to(torch.int64)
    else:
        factor = {"cube": 1.0, "ball": 2.0, "shell": 8.0}[kind]
        lo = int(np.ceil(0.2025 * float(1 << 48)))
        out = []
        got = 0
        while got < n:
            k = torch.randint(0, GRID, (3, int((n - got) * factor) + 1024), generator=g, device=device,
                              dtype=torch.int64)
            if kind != "cube":
                d = k - HALF
                d2 = (d * d).sum(0)
                ok = d2 < (1 << 46)
                if kind == "shell":
                    ok &= d2 >= lo
                k = k[:, ok]
            out.append(k[:, : n - got])
            got += out[-1].shape[1]
        k = torch.cat(out, 1)
    f = k.to(torch.float32) * float(_SCALE)
    return f[0].clone(), f[1].clone(), f[2].clone()


def regular_polygon(m, n_interior, seed, radius=0.4, phase_deg=0.0):
    """Vertices of a regular m-gon (radius 0.4 about (1/2, 1/2), vertex j at
    phase + 360 j / m degrees, rounded to the grid) followed by n_interior
    points drawn uniformly inside the disk of radius 0.3.  Returns
    (x, y, vertex_count).  The rounded vertices stay in convex position for
    the sizes used in the tests."""
    j = np.arange(m, dtype=np.float64)
    ang = np.deg2rad(phase_deg + 360.0 * j / m)
    vx = np.rint((0.5 + radius * np.cos(ang)) * GRID).astype(np.int64)
    vy = np.rint((0.5 + radius * np.sin(ang)) * GRID).astype(np.int64)
    kx, ky = _reject_int(n_interior, seed,
                         lambda dx, dy: dx * dx + dy * dy < int((0.3 * GRID) ** 2))
    x = np.concatenate([to_float(vx), to_float(kx)])
    y = np.concatenate([to_float(vy), to_float(ky)])
    return x, y, m


def small_grid(n, side, seed, offset=(0, 0)):
    """n points on a side x side integer lattice (heavy duplicates, ties and
    collinear triples), offset by `offset` grid units."""
    r = _rng(seed)
    kx = r.integers(0, side, size=n) + offset[0]
    ky = r.integers(0, side, size=n) + offset[1]
    return to_float(kx), to_float(ky)


def batch_sizes(S, seed, lo=1_000, hi=1_000_000):
    """S set sizes, log-uniform in [lo, hi], rounded to the nearest integer."""
    r = _rng(seed)
    return np.rint(np.exp(r.uniform(np.log(lo), np.log(hi), size=S))).astype(np.int64)


def batch(sizes, seed, kinds=("square", "disk", "gaussian", "annulus")):
    """Concatenate one set per size, each drawn from a kind chosen uniformly
    at random.  Returns (x, y, offsets[S+1] int64, kind names)."""
    r = _rng(seed)
    sizes = np.asarray(sizes, np.int64)
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    x = np.empty(int(off[-1]), np.float32)
    y = np.empty(int(off[-1]), np.float32)
    names = []
    for i, n in enumerate(sizes):
        k = kinds[int(r.integers(0, len(kinds)))]
        gen = DISTRIBUTIONS[k] if k in DISTRIBUTIONS else globals()[k]
        sx, sy = gen(int(n), int(r.integers(0, 2**31)))
        x[off[i]:off[i + 1]] = sx
        y[off[i]:off[i + 1]] = sy
        names.append(k)
    return x, y, off, names


def mixture_batch_torch(S, n, seed, device="cuda:0", oversample=1.3):
    """S anisotropic Gaussian-mixture sets of n points each, drawn on the
    device with torch (same recipe as mixture(): K ~ U{1..8}, Dirichlet(1)
    weights, means U[0.25, 0.75]^2, major sigma U[0.02, 0.12], axis ratio
    log-uniform [1, 50], rotation U[0, pi)).  Points outside [0, 1)^2 are
    replaced by later draws of the same set; in the rare set that runs out of
    draws the last points are clamped into the square.  Returns float32
    x, y of length S*n (set s = [s*n, (s+1)*n)) on the device."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    K = torch.randint(1, 9, (S,), generator=g, device=device)
    comp_ok = torch.arange(8, device=device)[None, :] < K[:, None]
    e = -torch.log(torch.rand((S, 8), generator=g, device=device, dtype=f64).clamp_min(1e-300))
    w = torch.where(comp_ok, e, torch.zeros_like(e))
    w = w / w.sum(1, keepdim=True)
    mu = 0.25 + 0.5 * torch.rand((S, 8, 2), generator=g, device=device, dtype=f64)
    smaj = 0.02 + 0.10 * torch.rand((S, 8), generator=g, device=device, dtype=f64)
    ratio = torch.exp(torch.rand((S, 8), generator=g, device=device, dtype=f64) * np.log(50.0))
    rot = np.pi * torch.rand((S, 8), generator=g, device=device, dtype=f64)
    m = int(n * oversample) + 16
    comp = torch.multinomial(w.float(), m, replacement=True, generator=g)          # [S, m]
    a = torch.randn((S, m), generator=g, device=device, dtype=f64) * torch.gather(smaj, 1, comp)
    b = torch.randn((S, m), generator=g, device=device, dtype=f64) * \
        torch.gather(smaj / ratio, 1, comp)
    c, s_ = torch.cos(torch.gather(rot, 1, comp)), torch.sin(torch.gather(rot, 1, comp))
    px = torch.gather(mu[:, :, 0], 1, comp) + c * a - s_ * b
    py = torch.gather(mu[:, :, 1], 1, comp) + s_ * a + c * b
    ok = (px >= 0) & (px < 1) & (py >= 0) & (py < 1)
    order = torch.argsort((~ok).to(torch.int8), dim=1, stable=True)[:, :n]
    px = torch.gather(px, 1, order).clamp(0.0, 1.0 - 1.0 / GRID)
    py = torch.gather(py, 1, order).clamp(0.0, 1.0 - 1.0 / GRID)
    kx = torch.floor(px * GRID).clamp(0, GRID - 1)
    ky = torch.floor(py * GRID).clamp(0, GRID - 1)
    scale = 1.0 / GRID
    return ((kx * scale).to(torch.float32).reshape(-1).contiguous(),
            (ky * scale).to(torch.float32).reshape(-1).contiguous())


# ---------------------------------------------------------------------------
# Device-side generators (torch), for the large benchmark workloads.  Same
# recipes as the numpy generators above, different random streams.

def _grid_to_float_t(k):
    import torch
    return (k.to(torch.float64) * (1.0 / GRID)).to(torch.float32)


def _reject_int_t(n, g, device, accept, factor):
    import torch
    kx, ky, got = [], [], 0
    while got < n:
        m = int((n - got) * factor) + 4096
        a = torch.randint(0, GRID, (m,), generator=g, device=device, dtype=torch.int64)
        b = torch.randint(0, GRID, (m,), generator=g, device=device, dtype=torch.int64)
        ok = accept(a - HALF, b - HALF)
        a, b = a[ok][: n - got], b[ok][: n - got]
        kx.append(a)
        ky.append(b)
        got += a.numel()
    return torch.cat(kx), torch.cat(ky)


def _reject_real_t(n, g, device, draw):
    import torch
    kx, ky, got = [], [], 0
    while got < n:
        m = int((n - got) * 1.2) + 4096
        px, py = draw(m)
        ok = (px >= 0) & (px < 1) & (py >= 0) & (py < 1)
        a = torch.floor(px[ok] * GRID).to(torch.int64)
        b = torch.floor(py[ok] * GRID).to(torch.int64)
        ok2 = (a < GRID) & (b < GRID)
        a, b = a[ok2][: n - got], b[ok2][: n - got]
        kx.append(a)
        ky.append(b)
        got += a.numel()
    return torch.cat(kx), torch.cat(ky)


def set_torch(kind, n, seed, device="cuda:0"):
    """One set of n points of the given kind ("square", "disk", "gaussian",
    "annulus", "mixture", "ellipse") drawn on the device; float32 x, y."""
    import torch
    if kind == "mixture":
        return mixture_batch_torch(1, n, seed, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    if n == 0:
        z = torch.zeros(0, dtype=torch.float32, device=device)
        return z, z.clone()
    if kind == "square":
        kx = torch.randint(0, GRID, (n,), generator=g, device=device, dtype=torch.int64)
        ky = torch.randint(0, GRID, (n,), generator=g, device=device, dtype=torch.int64)
    elif kind == "disk":
        kx, ky = _reject_int_t(n, g, device, lambda dx, dy: dx * dx + dy * dy < (1 << 46), 1.35)
    elif kind == "annulus":
        def acc(dx, dy):
            d2 = dx * dx + dy * dy
            return (d2 < (1 << 46)) & (d2 >= ANNULUS_R2_MIN)
        kx, ky = _reject_int_t(n, g, device, acc, 7.0)
    elif kind == "gaussian":
        kx, ky = _reject_real_t(n, g, device, lambda m: (
            0.5 + 0.15 * torch.randn(m, generator=g, device=device, dtype=f64),
            0.5 + 0.15 * torch.randn(m, generator=g, device=device, dtype=f64)))
    elif kind == "ellipse":
        r = _rng(seed)
        cx, cy = r.uniform(0.45, 0.55, size=2)
        a = r.uniform(0.2, 0.44)
        b = a / np.exp(r.uniform(np.log(20.0), np.log(200.0)))
        th = r.uniform(0.0, np.pi)
        c, s = np.cos(th), np.sin(th)
        ux, uy = _reject_int_t(n, g, device, lambda dx, dy: dx * dx + dy * dy < (1 << 46), 1.35)
        ux = (ux.to(f64) - HALF) / HALF
        uy = (uy.to(f64) - HALF) / HALF
        px = cx + c * a * ux - s * b * uy
        py = cy + s * a * ux + c * b * uy
        kx = torch.floor(px * GRID).clamp(0, GRID - 1).to(torch.int64)
        ky = torch.floor(py * GRID).clamp(0, GRID - 1).to(torch.int64)
    else:
        raise ValueError(kind)
    return _grid_to_float_t(kx), _grid_to_float_t(ky)


def batch_torch(sizes, seed, kinds=("square", "disk", "gaussian", "annulus"),
                device="cuda:0", pick=None):
    """Concatenated sets on the device, one per size; set i's kind is
    pick(i) if given, else drawn uniformly from kinds.  Returns
    (x, y, offsets[S+1] int64 on the device, kind names)."""
    import torch
    r = _rng(seed)
    sizes = np.asarray(sizes, np.int64)
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    x = torch.empty(int(off[-1]), dtype=torch.float32, device=device)
    y = torch.empty(int(off[-1]), dtype=torch.float32, device=device)
    names = []
    for i, n in enumerate(sizes):
        k = pick(i) if pick is not None else kinds[int(r.integers(0, len(kinds)))]
        sx, sy = set_torch(k, int(n), int(r.integers(0, 2**31)), device)
        x[off[i]:off[i + 1]] = sx
        y[off[i]:off[i + 1]] = sy
        names.append(k)
    return x, y, torch.from_numpy(off).to(device), names
