"""Parity at the benchmark's full size: 2^27 points per set, in the launch
configuration bench.py times (default tuning), for each distribution and
both direction presets ({0, 30, 45, 60} and the cumulative {0, 30, 75, 120}).

The oracle runs the whole method on the same arrays (about 10-30 s per set on
one core); extreme slots and values, the survivor list and the hull must be
identical.
"""
import numpy as np
import pytest

import oracle
from paper_1405_3454_amd import inputs

pytestmark = pytest.mark.gpu

N = 1 << 27
SEEDS = {"square": 101, "disk": 102, "gaussian": 103, "annulus": 104}   # bench.py's inputs


_SETS = {}


def _points(kind):
    """The benchmark's set of this kind (drawn once per module)."""
    if kind not in _SETS:
        _SETS[kind] = inputs.DISTRIBUTIONS[kind](N, SEEDS[kind])
    return _SETS[kind]


@pytest.fixture(scope="module")
def H():
    import torch
    from paper_1405_3454_amd.api import Hull
    h = Hull(0)
    yield h
    torch.cuda.synchronize()
    h.close()


@pytest.mark.parametrize("preset", [0, 1])
@pytest.mark.parametrize("kind", ["square", "disk", "gaussian", "annulus"])
def test_full_size(H, kind, preset):
    import torch
    from paper_1405_3454_amd.api import as_u32
    x, y = _points(kind)
    xt = torch.from_numpy(x).to("cuda:0")
    yt = torch.from_numpy(y).to("cuda:0")
    H.set_directions(preset)
    slots, vals = H.extremes(xt, yt)
    surv = H.discard(xt, yt, slots)
    hull = H.compute(xt, yt)
    g_slots, g_vals, g_surv, g_hull = as_u32(slots), vals.cpu().numpy(), as_u32(surv), as_u32(hull)
    del xt, yt
    H.set_directions(0)
    o_slots, o_vals = oracle.extremes(x, y, preset)
    assert np.array_equal(g_slots, o_slots)
    assert np.array_equal(g_vals.view(np.uint64), o_vals.view(np.uint64))
    o_verts = oracle.polygon(x, y, o_slots)
    o_surv = oracle.discard(x, y, o_verts)
    assert len(g_surv) == len(o_surv)
    assert np.array_equal(g_surv, o_surv)
    o_hull = oracle.hull_subset(x, y, o_surv)
    assert np.array_equal(g_hull, o_hull)
    if preset == 0:
        _OHULL[kind] = o_hull


_OHULL = {}
KINDS = ("square", "disk", "gaussian", "annulus")


@pytest.mark.parametrize("tuned", [False, True])
def test_full_size_one_batched_call(H, tuned):
    """The four sets in one batched call of the whole method, the way
    bench.py's main line runs them (tuned: after the autotuner has picked
    the launch shapes on this batch; else the default shapes): each set's
    hull equals the oracle's."""
    import torch
    from paper_1405_3454_amd.api import as_u32
    xs = [_points(k) for k in KINDS]
    xb = torch.from_numpy(np.concatenate([p[0] for p in xs])).to("cuda:0")
    yb = torch.from_numpy(np.concatenate([p[1] for p in xs])).to("cuda:0")
    off = torch.tensor([i * N for i in range(5)], dtype=torch.int64, device="cuda:0")
    hb = torch.empty(4 * N, dtype=torch.int32, device="cuda:0")
    ho = torch.zeros(5, dtype=torch.int64, device="cuda:0")
    H.set_directions(0)
    if tuned:       # the untuned case runs first (parameter order): default shapes
        H.autotune(xb, yb, off)
    H.compute_batched_into(xb, yb, off, hb, ho)
    hoc = ho.cpu().numpy()
    got = as_u32(hb[: int(hoc[-1])]).astype(np.int64)
    del xb, yb, hb
    for i, k in enumerate(KINDS):
        want = _OHULL.get(k)
        if want is None:
            x, y = xs[i]
            want = oracle.compute(x, y, 0)
            _OHULL[k] = want
        g = got[hoc[i]:hoc[i + 1]] - i * N
        assert np.array_equal(g, want.astype(np.int64)), k
