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


def cpu_baseline(sample_n):
    """The CPU oracle, single-threaded, on sample_n points of each kind."""
    import oracle
    oracle.build(force=False)
    pts = 0
    t = 0.0
    for k in KINDS:
        x, y = _gen((k, sample_n, SEEDS[k] + 1000))
        t0 = time.perf_counter()
        oracle.compute(x, y)
        t += time.perf_counter() - t0
        pts += sample_n
    return {"value": pts / t / 1e9, "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
            "sample": "%d points of each of %s (seeded), whole method, single thread"
                      % (sample_n, "/".join(KINDS)),
            "seconds": round(t, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=27)
    ap.add_argument("--preset", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=1 << 23)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--autotune", action="store_true")
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
    # roofline of the dominant kernel by time per step; algorithmic bytes per launch
    alg_bytes = {"extremes": 8.0 * n, "discard": 8.0 * n}
    dom = max(kt.items(), key=lambda kv: kv[1][0])[0]
    hbm = {}
    for name in ("extremes", "discard"):
        if name in kt:
            ms, c = kt[name]
            hbm[name] = alg_bytes[name] / (ms / c * 1e-3) / 1e9
    rname = dom if dom in alg_bytes else "discard"
    ms, c = kt[rname]
    achieved = alg_bytes[rname] / (ms / c * 1e-3) / 1e9
    roof = {"kernel": rname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
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
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out), flush=True)
    H.close()


if __name__ == "__main__":
    main()
