"""Parity at the benchmark's other workloads, at their full shape and in the
launch configuration bench.py times.

 * The batched line: 4096 sets with log-uniform sizes in [1e3, 1e6]
   (about 5.9e8 points), kinds uniform over square/disk/gaussian/annulus,
   drawn on the device exactly as bench.py draws them.  Above 256 sets the
   sort key's set field needs a ninth byte, so the radix sort runs eight
   passes; every set's slots, survivors and hull are compared with the
   oracle run on that set alone, eagerly and from a graph replay.
 * The learned line: 1024 sets of 2^17 points (thin ellipses and mixtures
   alternating) and one thin ellipse of 2^27, with the learned proposal on.
   The 24 slots of every set (16 fixed + 8 along the directions the GPU's
   network picked) are compared with the oracle's extremes along the same
   directions, then the survivors and the hull.  The 2^27 set spans many
   runs of the extremes pass, so the 24-slot run and tie logic is covered at
   the size the benchmark times.

The oracle runs per set on the host, spread over threads (each call is an
independent single-threaded C routine; ctypes releases the interpreter lock
while it runs).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1405_3454_amd import inputs

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def H():
    import torch
    from paper_1405_3454_amd.api import Hull
    h = Hull(0)
    yield h
    torch.cuda.synchronize()
    h.close()


def u32(t):
    from paper_1405_3454_amd.api import as_u32
    return as_u32(t)


def _per_set(fn, S):
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        return list(ex.map(fn, range(S)))


def _shift(v, a):
    return np.where(v == oracle.NONE, oracle.NONE, v.astype(np.int64) + a).astype(np.uint32)


@pytest.mark.timeout(900)
def test_batched_benchmark_batch(H):
    """bench.py's batched workload: batch_sizes(4096, 2024) drawn with seed
    2025 on the device; 8 radix passes; per-set parity, eager and graph."""
    import torch
    S = 4096
    sizes = inputs.batch_sizes(S, 2024)
    xt, yt, ot, names = inputs.batch_torch(sizes, 2025, device="cuda:0")
    x, y, off = xt.cpu().numpy(), yt.cpu().numpy(), ot.cpu().numpy()
    n = len(x)
    print("batched workload: %d sets, %d points" % (S, n), flush=True)
    H.set_directions(0)
    slots = u32(H.extremes_batched(xt, yt, ot)).reshape(S, 16)
    surv, so = H.discard_batched(xt, yt, ot, torch.from_numpy(slots.view(np.int32)).to("cuda:0"))
    sv, so = u32(surv), so.cpu().numpy()
    hull, ho = H.compute_batched(xt, yt, ot)
    hv, ho = u32(hull).copy(), ho.cpu().numpy()
    gh = torch.full((n,), -7, dtype=torch.int32, device="cuda:0")
    gho = torch.zeros(S + 1, dtype=torch.int64, device="cuda:0")
    H.graph_capture(xt, yt, ot, gh, gho)
    H.graph_launch()
    torch.cuda.synchronize()
    assert np.array_equal(gho.cpu().numpy(), ho)
    assert np.array_equal(u32(gh)[: ho[-1]], hv[: ho[-1]])
    del gh, hull, surv
    print("GPU done; oracle per set", flush=True)

    def check(s):
        a, b = int(off[s]), int(off[s + 1])
        xs, ys = x[a:b], y[a:b]
        o_slots, _ = oracle.extremes(xs, ys, 0)
        if not np.array_equal(slots[s], _shift(o_slots, a)):
            return "slots of set %d (%s, n=%d)" % (s, names[s], b - a)
        o_surv = oracle.discard(xs, ys, oracle.polygon(xs, ys, o_slots))
        if not np.array_equal(sv[so[s]:so[s + 1]].astype(np.int64), o_surv.astype(np.int64) + a):
            return "survivors of set %d (%s, n=%d)" % (s, names[s], b - a)
        o_hull = oracle.hull_subset(xs, ys, o_surv)
        if not np.array_equal(hv[ho[s]:ho[s + 1]].astype(np.int64), o_hull.astype(np.int64) + a):
            return "hull of set %d (%s, n=%d)" % (s, names[s], b - a)
        return None

    bad = [e for e in _per_set(check, S) if e]
    assert not bad, bad[:5]


@pytest.mark.timeout(900)
def test_learned_benchmark_batch(H):
    """bench.py's learned inference workload: 1024 x 2^17 + 1 x 2^27 (thin
    ellipses / mixtures, seed 4242) with the learned proposal on."""
    import torch
    H.mlp_set_params(mlp.he_init(77))
    sizes = [1 << 17] * 1024 + [1 << 27]
    S = len(sizes)
    xt, yt, ot, names = inputs.batch_torch(
        sizes, 4242, device="cuda:0",
        pick=lambda i: "ellipse" if (i % 2 == 0 or i == 1024) else "mixture")
    x, y, off = xt.cpu().numpy(), yt.cpu().numpy(), ot.cpu().numpy()
    print("learned workload: %d sets, %d points" % (S, len(x)), flush=True)
    H.set_directions(0)
    hb, _ = H.histogram_batched(xt, yt, ot)
    dirs = H.top_directions(H.mlp_forward(hb)).cpu().numpy()
    slots = u32(H.extremes_batched(xt, yt, ot, learned=True)).reshape(S, 24)
    surv, so = H.discard_batched(xt, yt, ot, torch.from_numpy(slots.view(np.int32)).to("cuda:0"))
    sv, so = u32(surv), so.cpu().numpy()
    hull, ho = H.compute_batched(xt, yt, ot, learned=True)
    hv, ho = u32(hull).copy(), ho.cpu().numpy()
    del surv, hull
    cd, sd = oracle.direction_table()
    print("GPU done; oracle per set", flush=True)

    def check(s):
        a, b = int(off[s]), int(off[s + 1])
        xs, ys = x[a:b], y[a:b]
        o_fixed, _ = oracle.extremes(xs, ys, 0)
        o_dir, _ = oracle.extremes_dirs(xs, ys, cd[dirs[s]], sd[dirs[s]])
        want = np.concatenate([o_fixed, o_dir])
        if not np.array_equal(slots[s], _shift(want, a)):
            return "slots of set %d (%s, n=%d)" % (s, names[s], b - a)
        o_surv = oracle.discard(xs, ys, oracle.polygon(xs, ys, want))
        if not np.array_equal(sv[so[s]:so[s + 1]].astype(np.int64), o_surv.astype(np.int64) + a):
            return "survivors of set %d (%s, n=%d)" % (s, names[s], b - a)
        o_hull = oracle.hull_subset(xs, ys, o_surv)
        if not np.array_equal(hv[ho[s]:ho[s + 1]].astype(np.int64), o_hull.astype(np.int64) + a):
            return "hull of set %d (%s, n=%d)" % (s, names[s], b - a)
        return None

    bad = [e for e in _per_set(check, S) if e]
    assert not bad, bad[:5]
