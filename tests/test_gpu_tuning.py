"""Launch shapes and the autotuner: no shape may change any bit.

Every shape of the persistent filter kernels (block size x blocks per CU x
tiles per wave) is run on a single set and on a ragged batch; the extremes,
the ordered survivors and the hulls must equal the oracle's each time.  The
autotuner's table is per size bucket and its choices keep the results.
"""
import itertools

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
    h.set_tuning(3, 4)
    h.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def u32(t):
    from paper_1405_3454_amd.api import as_u32
    return as_u32(t)


SHAPES = list(itertools.product((128, 256, 512), (1, 3, 8), (1, 4, 40)))


@pytest.fixture(scope="module")
def single():
    x, y = inputs.disk(400_000, 321)
    slots, _ = oracle.extremes(x, y)
    surv = oracle.discard(x, y, oracle.polygon(x, y, slots))
    return x, y, slots, surv, oracle.hull_subset(x, y, surv)


@pytest.fixture(scope="module")
def batch():
    sizes = [0, 1, 5, 1023, 1025, 40_000, 3, 250_000, 7777, 0, 65_536]
    x, y, off, _ = inputs.batch(sizes, 77)
    want = []
    for s in range(len(sizes)):
        a, b = int(off[s]), int(off[s + 1])
        want.append(oracle.hull_subset(x[a:b], y[a:b]).astype(np.int64) + a)
    return x, y, off, want


@pytest.mark.parametrize("bs,bpc,tpw", SHAPES)
def test_every_shape_single_set(H, single, bs, bpc, tpw):
    x, y, o_slots, o_surv, o_hull = single
    n = len(x)
    H.set_shape(0, n, 1, bs, bpc, tpw)
    H.set_shape(1, n, 1, bs, bpc, tpw)
    assert H.shape(0, n)[:3] == (bs, bpc, tpw)
    xt, yt = dev(x), dev(y)
    slots, _ = H.extremes(xt, yt)
    assert np.array_equal(u32(slots), o_slots)
    assert np.array_equal(u32(H.discard(xt, yt, slots)), o_surv)
    assert np.array_equal(u32(H.compute(xt, yt)), o_hull)


@pytest.mark.parametrize("bs,bpc,tpw", SHAPES[::2])
def test_every_shape_batch(H, batch, bs, bpc, tpw):
    x, y, off, want = batch
    S = len(off) - 1
    n = len(x)
    H.set_shape(0, n, S, bs, bpc, tpw)
    H.set_shape(1, n, S, bs, bpc, tpw)
    hull, ho = H.compute_batched(dev(x), dev(y), dev(off))
    hv, ho = u32(hull), ho.cpu().numpy()
    for s in range(S):
        assert np.array_equal(hv[ho[s]:ho[s + 1]].astype(np.int64), want[s]), (s, bs, bpc, tpw)


def test_autotune_table_and_results(H, single):
    x, y, o_slots, o_surv, o_hull = single
    H.set_tuning(3, 4)          # clears the table
    assert H.tuning_table() == []
    xt, yt = dev(x), dev(y)
    table = H.autotune(xt, yt)
    kernels = sorted(r["kernel"] for r in table)
    assert kernels == ["discard", "extremes"]
    assert all(r["points"] == "<2^20" and not r["batched"] for r in table)
    assert H.shape(0, len(x))[3] and H.shape(1, len(x))[3]
    # other buckets untouched
    assert not H.shape(0, 100)[3]
    assert np.array_equal(u32(H.compute(xt, yt)), o_hull)
    slots, _ = H.extremes(xt, yt)
    assert np.array_equal(u32(slots), o_slots)


def test_shape_validation(H):
    from paper_1405_3454_amd._lib import HULL_EINVAL, HullError
    for bad in ((64, 1, 1), (256, 0, 1), (256, 17, 1), (256, 1, 0), (1024, 1, 1)):
        with pytest.raises(HullError) as e:
            H.set_shape(0, 1000, 1, *bad)
        assert e.value.code == HULL_EINVAL
