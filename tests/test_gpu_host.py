"""Host-resident input (hull_compute_host) against the CPU oracle.

The set stays in host memory and crosses to the device in chunks; the
extremes are reduced across chunks, each chunk is filtered by the polygon of
the global extremes, and the survivors' hull is taken on the device.  Slots,
survivors (ascending) and hull must equal the oracle's on the whole set,
exactly, whatever the chunk size, the device budget (all chunks streamed
twice, some resident, all resident) and whether the host memory is pinned.
"""
import numpy as np
import pytest

import oracle
from paper_1405_3454_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    from paper_1405_3454_amd.api import Hull
    h = Hull(0)
    yield h
    torch.cuda.synchronize()
    h.set_directions(0)
    h.close()


def u32(t):
    from paper_1405_3454_amd.api import as_u32
    return as_u32(t)


def check_host(H, x, y, preset, chunk, budget, pinned=False, what=""):
    import torch
    H.set_directions(preset)
    if pinned:
        xt = torch.from_numpy(x).pin_memory()
        yt = torch.from_numpy(y).pin_memory()
    else:
        xt, yt = x, y
    slots, surv, hull = H.compute_host(xt, yt, chunk_points=chunk, device_budget=budget)
    torch.cuda.synchronize()
    o_slots, _ = oracle.extremes(x, y, preset)
    gs = u32(slots)
    k = len(o_slots)
    assert np.array_equal(gs[:k], o_slots), (what, gs[:k], o_slots)
    assert (gs[k:] == oracle.NONE).all(), what
    o_surv = oracle.discard(x, y, oracle.polygon(x, y, o_slots))
    assert np.array_equal(u32(surv), o_surv), (what, len(surv), len(o_surv))
    assert np.array_equal(u32(hull), oracle.hull_subset(x, y, o_surv)), what


@pytest.mark.parametrize("n", [0, 1, 5, 1023, 1025, 5000, 70001])
@pytest.mark.parametrize("chunk", [1024, 4096])
def test_small_sets_many_chunks(H, n, chunk):
    kind = ["square", "disk", "gaussian", "annulus"][n % 4]
    x, y = inputs.DISTRIBUTIONS[kind](n, 600 + n) if n else (np.zeros(0, np.float32),) * 2
    for budget in (0, 3 * chunk * 8, 1 << 40):
        check_host(H, x, y, 0, chunk, budget, what="%s n=%d chunk=%d budget=%d" % (kind, n, chunk, budget))


@pytest.mark.parametrize("kind", ["square", "disk", "gaussian", "annulus"])
def test_medium_sets(H, kind):
    x, y = inputs.DISTRIBUTIONS[kind](600_000, 61)
    check_host(H, x, y, 0, 65536, 0, what=kind)
    check_host(H, x, y, 1, 1 << 17, 4 * (1 << 17) * 8, pinned=True, what=kind + " pinned")


@pytest.mark.parametrize("preset", [2, 5, 7])
def test_direction_families(H, preset):
    x, y = inputs.annulus(200_000, 70 + preset)
    check_host(H, x, y, preset, 32768, 0, what="preset %d" % preset)


def test_ties_across_chunks(H):
    """A coarse grid repeats every extreme value in many chunks: the lowest
    index must win across chunk boundaries."""
    x, y = inputs.disk(400_000, 5)
    x = (np.floor(x * 256) / 256).astype(np.float32)
    y = (np.floor(y * 256) / 256).astype(np.float32)
    for preset in (0, 1, 3):
        check_host(H, x, y, preset, 8192, 0, what="grid preset %d" % preset)
        check_host(H, x, y, preset, 8192, 1 << 40, pinned=True, what="grid pinned %d" % preset)


def test_multi_million_points(H):
    x, y = inputs.disk(3_000_000 + 17, 8)
    check_host(H, x, y, 0, 1 << 20, 0, what="3M streamed")
    check_host(H, x, y, 0, 1 << 20, 1 << 40, pinned=True, what="3M resident")


def test_capacity_overflow_reported(H):
    from paper_1405_3454_amd._lib import HULL_EOVERFLOW, HullError
    x, y = inputs.annulus(50_000, 3)
    o_surv = oracle.compute(x, y, want_survivors=True)[1]
    with pytest.raises(HullError) as e:
        H.compute_host(x, y, chunk_points=4096, cap=len(o_surv) - 1)
    assert e.value.code == HULL_EOVERFLOW
    # exactly enough room works
    slots, surv, hull = H.compute_host(x, y, chunk_points=4096, cap=len(o_surv))
    assert np.array_equal(u32(surv), o_surv)
    assert np.array_equal(u32(hull), oracle.compute(x, y))


def test_host_path_matches_device_path(H):
    import torch
    x, y = inputs.gaussian(250_000, 4)
    _, _, hh = H.compute_host(x, y, chunk_points=1 << 15)
    hd = H.compute(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    assert np.array_equal(u32(hh), u32(hd))
