"""The allocation-free Step 1 entry point (hull_extremes_noalloc) against
hull_extremes, through the C ABI.

Two calls in a row on the shared scratch array (the second on a smaller set)
must give exactly hull_extremes' slots and binary64 values, for several
presets; sizes past the scratch limit are refused on the host before any
launch.
"""
import ctypes

import numpy as np
import pytest

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


def _noalloc(H, xt, yt, k):
    import torch
    from paper_1405_3454_amd import _lib
    from paper_1405_3454_amd.api import _ptr, _stream
    slots = torch.full((k,), -7, dtype=torch.int32, device=xt.device)
    vals = torch.full((k,), 3.0, dtype=torch.float64, device=xt.device)
    rc = _lib.lib().hull_extremes_noalloc(H._h, _ptr(xt), _ptr(yt), xt.numel(), _ptr(slots),
                                          _ptr(vals), 0, _stream())
    _lib.check(rc, "hull_extremes_noalloc")
    return slots, vals


def _same(a, b):
    return np.array_equal(a.cpu().numpy().view(np.uint64 if a.dtype.itemsize == 8 else np.uint32),
                          b.cpu().numpy().view(np.uint64 if b.dtype.itemsize == 8 else np.uint32))


@pytest.mark.parametrize("preset", [0, 1, 2, 5, 7])
def test_noalloc_matches_hull_extremes_twice(H, preset):
    import torch
    from paper_1405_3454_amd import inputs
    H.set_directions(preset)
    k = H.slot_count()
    for n, kind, seed in ((3_000_001, "disk", 11 + preset), (70_001, "annulus", 12 + preset)):
        x, y = inputs.DISTRIBUTIONS[kind](n, seed)
        xt = torch.from_numpy(x).to("cuda:0")
        yt = torch.from_numpy(y).to("cuda:0")
        s_ref, v_ref = H.extremes(xt, yt)
        s, v = _noalloc(H, xt, yt, k)
        torch.cuda.synchronize()
        assert _same(s, s_ref), (preset, n)
        assert _same(v, v_ref), (preset, n)
    H.set_directions(0)


def test_noalloc_at_the_size_limit_and_beyond(H):
    import torch
    from paper_1405_3454_amd import _lib, inputs
    from paper_1405_3454_amd.api import _ptr, _stream
    n = _lib.HULL_NOALLOC_MAX_POINTS
    x, y = inputs.square(n, 5)
    xt = torch.from_numpy(x).to("cuda:0")
    yt = torch.from_numpy(y).to("cuda:0")
    s_ref, v_ref = H.extremes(xt, yt)
    s, v = _noalloc(H, xt, yt, 16)
    torch.cuda.synchronize()
    assert _same(s, s_ref) and _same(v, v_ref)
    # one point more: refused on the host, nothing launched (n is only
    # checked against the limit, the buffers are not read)
    slots = torch.empty(16, dtype=torch.int32, device="cuda:0")
    rc = _lib.lib().hull_extremes_noalloc(H._h, _ptr(xt), _ptr(yt), n + 1, _ptr(slots), None, 0,
                                          _stream())
    assert rc == _lib.HULL_ESCRATCH
    # learned slots are not offered here
    rc = _lib.lib().hull_extremes_noalloc(H._h, _ptr(xt), _ptr(yt), 10, _ptr(slots), None,
                                          _lib.HULL_LEARNED, _stream())
    assert rc == _lib.HULL_EINVAL


def test_noalloc_empty_and_tiny(H):
    import torch
    from paper_1405_3454_amd import inputs
    for n in (0, 1, 5):
        x, y = inputs.square(max(n, 1), 9)
        xt = torch.from_numpy(x[:n].copy()).to("cuda:0") if n else torch.zeros(0, device="cuda:0")
        yt = torch.from_numpy(y[:n].copy()).to("cuda:0") if n else torch.zeros(0, device="cuda:0")
        s_ref, v_ref = H.extremes(xt, yt)
        s, v = _noalloc(H, xt, yt, 16)
        torch.cuda.synchronize()
        assert _same(s, s_ref), n
        if n:
            assert _same(v, v_ref), n
