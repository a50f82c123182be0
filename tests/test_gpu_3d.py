"""The 3D form of the method on the GPU (hull3_compute) against the 3D oracle.

Exact: the 42 extreme slots, the survivors of the strict-inside test
(ascending) and the hull's extreme points (ascending, lowest index per
repeated coordinate triple), for uniform, ball, shell and Gaussian sets,
sizes across tiles and ragged tails, lattices with ties and coplanar points,
flat and collinear sets, and the unfiltered arm.
"""
import numpy as np
import pytest

from oracle import hull3d as o3
from paper_1405_3454_amd import inputs

pytestmark = pytest.mark.gpu

KINDS = ["cube", "ball", "shell", "gaussian"]


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


def check3(H, x, y, z, preset=0, what="", serial=False):
    H.set_directions(preset)
    slots, surv, hull = H.compute3(dev(x), dev(y), dev(z), serial=serial)
    o_slots, _ = o3.extremes(x, y, z, preset)
    assert np.array_equal(u32(slots), o_slots), (what, u32(slots), o_slots)
    o_hull, o_surv = o3.compute(x, y, z, preset, want_survivors=True)
    assert np.array_equal(u32(surv), o_surv), (what, len(surv), len(o_surv))
    assert np.array_equal(u32(hull), o_hull), (what, len(hull), len(o_hull))
    return len(o_surv), len(o_hull)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 17, 1023, 1025, 4099, 30001])
@pytest.mark.parametrize("kind", KINDS)
def test_sizes(H, kind, n):
    x, y, z = inputs.DISTRIBUTIONS3[kind](n, 500 + n)
    check3(H, x, y, z, 0, "%s n=%d" % (kind, n))


@pytest.mark.parametrize("preset", [0, 1])
@pytest.mark.parametrize("kind", KINDS)
def test_medium(H, kind, preset):
    x, y, z = inputs.DISTRIBUTIONS3[kind](120_000, 77 + preset)
    check3(H, x, y, z, preset, "%s preset %d" % (kind, preset))


@pytest.mark.parametrize("seed", range(8))
def test_lattices(H, seed):
    r = np.random.default_rng(seed)
    n = int(r.integers(1, 6000))
    side = int(r.integers(1, 9))
    x, y, z = inputs.lattice3(n, side, seed, offset=int(r.integers(0, 1 << 20)))
    check3(H, x, y, z, seed % 2, "lattice seed=%d n=%d side=%d" % (seed, n, side))


def test_flat_and_collinear(H):
    k = np.arange(3000)
    r = np.random.default_rng(5)
    a = r.integers(0, 1 << 12, size=3000)
    b = r.integers(0, 1 << 12, size=3000)
    to = inputs.to_float
    cases = [
        (to(a), to(b), to(a + b)),                 # a tilted plane
        (to(a), to(np.full(3000, 77)), to(b)),     # the plane y = const
        (to(k), to(2 * k), to(3 * k)),             # a line
        (to(np.full(50, 9)), to(np.full(50, 8)), to(np.full(50, 7))),   # one point, repeated
    ]
    for x, y, z in cases:
        check3(H, x, y, z, 0, "degenerate")


def test_empty(H):
    import torch
    e = torch.zeros(0, dtype=torch.float32, device="cuda:0")
    slots, surv, hull = H.compute3(e, e.clone(), e.clone())
    assert len(surv) == 0 and len(hull) == 0
    assert (u32(slots) == o3.NONE).all()


@pytest.mark.parametrize("kind", ["ball", "cube"])
def test_unfiltered_arm(H, kind):
    x, y, z = inputs.DISTRIBUTIONS3[kind](40_000, 9)
    _, surv, hull = H.compute3(dev(x), dev(y), dev(z), nofilter=True)
    assert len(surv) == len(x)
    assert np.array_equal(u32(hull), o3.compute(x, y, z, nofilter=True))


def test_repeated_points_lowest_index(H):
    """Every point twice (the copy at a higher index): the hull names the
    first copy."""
    x, y, z = inputs.ball3(5000, 3)
    perm = np.random.default_rng(1).permutation(10000)
    X = np.concatenate([x, x])[perm]
    Y = np.concatenate([y, y])[perm]
    Z = np.concatenate([z, z])[perm]
    check3(H, X, Y, Z, 0, "repeated")


@pytest.mark.parametrize("kind", KINDS)
def test_serial_insertion(H, kind):
    """The one-block insertion form of the hull stage (also the parallel
    rounds' fallback) against the oracle."""
    for n in (5, 4099, 60_000):
        x, y, z = inputs.DISTRIBUTIONS3[kind](n, 31 + n)
        check3(H, x, y, z, 0, "serial %s n=%d" % (kind, n), serial=True)


@pytest.mark.parametrize("seed", range(3))
def test_serial_lattice(H, seed):
    x, y, z = inputs.lattice3(5000, 4 + seed, 70 + seed, offset=1000 * seed)
    check3(H, x, y, z, 0, "serial lattice %d" % seed, serial=True)


@pytest.mark.parametrize("kind,n", [("ball", 400_000), ("shell", 150_000)])
def test_large_parallel_rounds(H, kind, n):
    """Sets whose hull stage runs thousands of proposals per round."""
    x, y, z = inputs.DISTRIBUTIONS3[kind](n, 123)
    check3(H, x, y, z, 0, "large %s" % kind)
