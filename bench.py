"""Benchmark: hull throughput of the interior-point-discarding method on one
MI355X.

Workload (N=1): four seeded sets of 2^27 points each, coordinates float32
k * 2^-24 -- uniform unit square, uniform disk r = 1/2, Gaussian sigma = 0.15
resampled into [0,1)^2, annulus 0.45 <= r < 0.5.  One step = the whole
method (extremes -> polygon -> strict discard -> sort -> monotone chain ->
index lookup) on each of the four sets, inputs resident in HBM.

Prints one JSON line: throughput in Gpoints/s, the roofline of the dominant
kernel (algorithmic bytes / its mean launch time from HIP events on the
launch stream), per-kernel times, discard fractions, and the CPU oracle timed
on a bounded sample on one host core.
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch at 2^27 points, from two rocprofv3 counter runs
# (FETCH_SIZE scaled by 2.0, WRITE_SIZE by 1.0: the factors a 1 GiB device
# copy gives), averaged over the four sets; reported only while the filter
# kernels' sources hash to the value they had when the counters were taken.
TRAFFIC = {"discard": 1.1824e9, "extremes": 1.1084e9}
TRAFFIC_SOURCES = ("paper_1405_3454_amd/csrc/k_filter.hip", "paper_1405_3454_amd/csrc/hg_common.h",
                   "paper_1405_3454_amd/csrc/hg_device.h")
TRAFFIC_SHA = "e3d576b5bf7a17c1"


def _traffic(kernel, log2n):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != TRAFFIC_SHA or kernel not in TRAFFIC or log2n != 27:
        return None
    return TRAFFIC[kernel]
KINDS = ("square", "disk", "gaussian", "annulus")
SEEDS = {"square": 101, "disk": 102, "gaussian": 103, "annulus": 104}


def _gen(args):
    kind, n, seed = args
    from paper_1405_3454_amd import inputs
    return inputs.DISTRIBUTIONS[kind](n, seed)


def generate(n, kinds=KINDS, workers=4):
    with ProcessPoolExecutor(max_workers=min(workers, len(kinds))) as ex:
        res = list(ex.map(_gen, [(k, n, SEEDS[k]) for k in kinds]))
    return dict(zip(kinds, res))


def cpu_baseline(data, sample):
    """The CPU oracle, single-threaded, on the first `sample` points of each
    of the benchmark's own four sets (a prefix of a seeded random set is a
    random set of the same kind)."""
    import oracle
    oracle.build(force=False)
    pts = 0
    t = 0.0
    for k in KINDS:
        x, y = data[k][0][:sample], data[k][1][:sample]
        t0 = time.perf_counter()
        oracle.compute(x, y)
        t += time.perf_counter() - t0
        pts += len(x)
    return {"value": pts / t / 1e9, "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
            "sample": "first %d points of each of the benchmark's four sets (%s), whole "
                      "method, single thread" % (sample, "/".join(KINDS)),
            "seconds": round(t, 3)}


def _time(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _discard_fraction_batched(H, x, y, off):
    slots = H.extremes_batched(x, y, off)
    _, so = H.discard_batched(x, y, off, slots)
    return 1.0 - float(so[-1].item()) / x.numel()


def bench_batched(args, dev):
    """Batched plain method: 4096 sets, sizes log-uniform in [1e3, 1e6], kinds
    uniform over square/disk/gaussian/annulus.  Per-set calls vs one batched
    call vs the same batched call replayed from a captured hipGraph."""
    import torch
    from paper_1405_3454_amd import inputs
    from paper_1405_3454_amd.api import Hull
    S = args.batch_sets
    sizes = inputs.batch_sizes(S, 2024)
    t0 = time.time()
    x, y, off, names = inputs.batch_torch(sizes, 2025, device=dev)
    torch.cuda.synchronize()
    n = x.numel()
    print("[bench] batched: %d sets, %d points, generated in %.1fs" % (S, n, time.time() - t0),
          file=sys.stderr, flush=True)
    H = Hull(0)
    tuning = H.autotune(x, y, off)
    hull = torch.empty(n, dtype=torch.int32, device=dev)
    ho = torch.zeros(S + 1, dtype=torch.int64, device=dev)
    hcnt = torch.zeros(S, dtype=torch.int64, device=dev)
    offs = off.cpu().numpy()

    def per_set():
        for s in range(S):
            a, b = int(offs[s]), int(offs[s + 1])
            H.compute_into(x[a:b], y[a:b], hull[a:b], hcnt[s:s + 1])

    def batched():
        H.compute_batched_into(x, y, off, hull, ho)

    t_set = _time(per_set, 2, 1)
    t_bat = _time(batched, args.steps, 1)
    H.graph_capture(x, y, off, hull, ho)
    t_graph = _time(H.graph_launch, args.steps, 1)
    disc = _discard_fraction_batched(H, x, y, off)
    H.close()
    res = {"workload": "%d sets, sizes log-uniform [1e3, 1e6], square/disk/gaussian/annulus" % S,
           "points": int(n),
           "per_set_gpts": round(n / t_set / 1e9, 3),
           "batched_gpts": round(n / t_bat / 1e9, 3),
           "graph_gpts": round(n / t_graph / 1e9, 3),
           "ms": {"per_set": round(t_set * 1e3, 3), "batched": round(t_bat * 1e3, 3),
                  "graph": round(t_graph * 1e3, 3)},
           "speedup_graph_vs_per_set": round(t_set / t_graph, 2),
           "discard_fraction": round(disc, 6),
           "tuning": tuning}
    del x, y, hull
    torch.cuda.empty_cache()
    return res


def bench_learned(args, dev):
    """Learned proposal.  Training: mixture sets of 2^16 points, labels,
    histograms, forward/backward and Adam all on the GPU.  Inference: 1024
    sets of 2^17 points (thin ellipses and mixtures alternating) plus one
    thin-ellipse set of 2^27, plain vs learned filter, each replayed from a
    captured hipGraph (histogram, network and top-8 inside the graph)."""
    import torch
    from paper_1405_3454_amd import inputs, train
    from paper_1405_3454_amd.api import Hull
    H = Hull(0)
    t0 = time.perf_counter()
    params, losses = train.train(H, sets=args.train_sets, batch=512, points=1 << 16, lr=1e-3,
                                 seed=7)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    H.close()
    sizes = [1 << 17] * 1024 + [1 << 27]
    t0 = time.time()
    x, y, off, names = inputs.batch_torch(
        sizes, 4242, device=dev, pick=lambda i: "ellipse" if (i % 2 == 0 or i == 1024) else "mixture")
    torch.cuda.synchronize()
    n = x.numel()
    S = len(sizes)
    print("[bench] learned: trained on %d sets in %.1fs; %d points generated in %.1fs"
          % (args.train_sets, t_train, n, time.time() - t0), file=sys.stderr, flush=True)
    out = {}
    hulls = {}
    for name, learned in (("plain", False), ("learned", True)):
        Hc = Hull(0)
        Hc.mlp_set_params(params)
        hull = torch.empty(n, dtype=torch.int32, device=dev)
        ho = torch.zeros(S + 1, dtype=torch.int64, device=dev)
        Hc.graph_capture(x, y, off, hull, ho, learned=learned)
        t = _time(Hc.graph_launch, args.steps, 1)
        slots = Hc.extremes_batched(x, y, off, learned=learned)
        _, so = Hc.discard_batched(x, y, off, slots)
        out[name] = (t, 1.0 - float(so[-1].item()) / n)
        hulls[name] = (ho.cpu(), hull[: int(ho[-1].item())].cpu())
        Hc.close()
        del hull
    same = bool(torch.equal(hulls["plain"][0], hulls["learned"][0]) and
                torch.equal(hulls["plain"][1], hulls["learned"][1]))
    del x, y
    torch.cuda.empty_cache()
    return {"training": {"sets": args.train_sets, "points_per_set": 1 << 16, "batch": 512,
                         "seconds": round(t_train, 2),
                         "sets_per_s": round(args.train_sets / t_train, 1),
                         "loss_first": round(losses[0], 5), "loss_last": round(losses[-1], 5)},
            "workload": "1024 sets x 2^17 (thin ellipses / mixtures) + 1 thin ellipse x 2^27",
            "points": int(n),
            "plain_gpts": round(n / out["plain"][0] / 1e9, 3),
            "learned_gpts": round(n / out["learned"][0] / 1e9, 3),
            "ms": {"plain": round(out["plain"][0] * 1e3, 3),
                   "learned": round(out["learned"][0] * 1e3, 3)},
            "discard_fraction": {"plain": round(out["plain"][1], 6),
                                 "learned": round(out["learned"][1], 6)},
            "speedup_learned_vs_plain": round(out["plain"][0] / out["learned"][0], 3),
            "hulls_identical": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=27)
    ap.add_argument("--preset", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 27,
                    help="points of each set the CPU oracle is timed on")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--batch-sets", type=int, default=4096)
    ap.add_argument("--train-sets", type=int, default=200000)
    ap.add_argument("--skip-extra", action="store_true",
                    help="only the four 2^27 sets (no unfiltered, batched or learned lines)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method runs each point set on a single "
              "device, and this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1405_3454_amd.api import Hull

    n = 1 << args.log2n
    t0 = time.time()
    data = generate(n)
    print("[bench] generated %d x %d points in %.1fs" % (len(KINDS), n, time.time() - t0),
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    X = {k: torch.from_numpy(v[0]).to(dev) for k, v in data.items()}
    Y = {k: torch.from_numpy(v[1]).to(dev) for k, v in data.items()}
    if args.no_cpu:
        del data
    H = Hull(0, preset=args.preset)
    if args.autotune:
        H.autotune(X["disk"], Y["disk"])
    hull = {k: torch.empty(n, dtype=torch.int32, device=dev) for k in KINDS}
    hcnt = {k: torch.zeros(1, dtype=torch.int64, device=dev) for k in KINDS}

    def step():
        for k in KINDS:
            H.compute_into(X[k], Y[k], hull[k], hcnt[k])

    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # timed region: plain step time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps

    # same steps with HIP events around every launch (per-kernel durations)
    H.timing(True)
    H.timing_reset()
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kt = H.timing_read()
    H.timing(False)

    # survivors per set (discard fraction) from one extra discard call each
    disc = {}
    hs = {}
    for k in KINDS:
        slots, _ = H.extremes(X[k], Y[k])
        surv = torch.empty(n, dtype=torch.int32, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        H.discard_into(X[k], Y[k], slots, surv, cnt)
        disc[k] = 1.0 - cnt.item() / n
        hs[k] = int(hcnt[k].item())

    total_pts = len(KINDS) * n
    per_kernel = {name: {"ms_total": round(ms / args.steps, 4), "launches_per_step": c / args.steps,
                         "ms_mean": round(ms / c, 4)} for name, (ms, c) in kt.items()}
    # roofline of the dominant kernel by time per step; algorithmic bytes per
    # launch, averaged over the four sets: the extremes pass reads x and y
    # (8 B per point); the full method's discard pass reads them and writes
    # each survivor's index, key and round-0 edge (4 + 8 + 2 B)
    surv_mean = sum((1.0 - disc[k]) * n for k in KINDS) / len(KINDS)
    alg_bytes = {"extremes": 8.0 * n, "discard": 8.0 * n + 14.0 * surv_mean}
    # categories that time one kernel each (scan and misc group small helpers)
    dom = max(((k, v) for k, v in kt.items() if k not in ("scan", "misc")),
              key=lambda kv: kv[1][0])[0]
    hbm = {}
    for name in ("extremes", "discard"):
        if name in kt:
            ms, c = kt[name]
            hbm[name] = alg_bytes[name] / (ms / c * 1e-3) / 1e9
    rname = dom if dom in alg_bytes else "discard"
    ms, c = kt[rname]
    achieved = alg_bytes[rname] / (ms / c * 1e-3) / 1e9
    roof = {"kernel": rname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _traffic(rname, args.log2n),
            "dominant_by_time": dom}

    out = {
        "metric": "hull Gpoints/s (whole method, plain 16-extreme filter)",
        "value": round(total_pts / dt / 1e9, 3),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "4 sets x 2^%d points (square, disk r=0.5, gaussian s=0.15, "
                               "annulus 0.45..0.5), float32 k*2^-24" % args.log2n,
                   "points_per_step": total_pts,
                   "directions": "0/30/45/60" if args.preset == 0 else "0/30/75/120"},
        "roofline": roof,
        "hbm_gbs": {k: round(v, 1) for k, v in hbm.items()},
        "discard_fraction": {k: round(v, 6) for k, v in disc.items()},
        "hull_vertices": hs,
        "per_kernel": per_kernel,
    }
    if not args.skip_extra:
        # unfiltered arm: the same hull without the filter (sort + chain of all points)
        hull_u = torch.empty(n, dtype=torch.int32, device=dev)
        hu = torch.zeros(1, dtype=torch.int64, device=dev)

        def step_u():
            for k in KINDS:
                H.compute_into(X[k], Y[k], hull_u, hu, nofilter=True)
        t_u = _time(step_u, max(2, args.steps // 2), 1)
        out["unfiltered"] = {"gpts": round(total_pts / t_u / 1e9, 3),
                             "ms_per_step": round(t_u * 1e3, 3),
                             "speedup_of_filter": round(t_u / dt, 3)}
        del hull_u
        H.close()
        del X, Y, hull
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(args, dev)
        out["learned"] = bench_learned(args, dev)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(data, min(n, args.cpu_sample))
    print(json.dumps(out), flush=True)
    if args.skip_extra:
        H.close()


if __name__ == "__main__":
    main()
