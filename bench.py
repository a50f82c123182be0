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

# HBM bytes per launch of the step (one launch over the four 2^27-point
# sets), from two rocprofv3 counter runs (FETCH_SIZE scaled by 2.0,
# WRITE_SIZE by 1.0: the factors a 1 GiB device copy gives); reported only
# while the filter kernels' sources hash to the value they had when the
# counters were taken.
TRAFFIC = {"discard": 4.7457e9, "extremes": 4.3186e9}
TRAFFIC_SOURCES = ("paper_1405_3454_amd/csrc/k_filter.hip", "paper_1405_3454_amd/csrc/hg_common.h",
                   "paper_1405_3454_amd/csrc/hg_device.h")
TRAFFIC_SHA = "b91d2a5274b0d3f5"


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


def host_cpu():
    """Model and thread counts of the host (for the CPU baselines)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable_threads": usable}


def cpu_baseline_batched(xs, ys, offs, workers):
    """The CPU oracle on whole sets of the batched workload: once on one
    thread, once with the sets spread over `workers` threads (the oracle is
    plain single-threaded C; its ctypes calls release the GIL)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build(force=False)
    S = len(offs) - 1
    jobs = [(xs[offs[s]:offs[s + 1]], ys[offs[s]:offs[s + 1]]) for s in range(S)]
    pts = int(offs[-1])
    t0 = time.perf_counter()
    for a, b in jobs:
        oracle.compute(a, b)
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda ab: oracle.compute(ab[0], ab[1]), jobs))
    tn = time.perf_counter() - t0
    return {"one_core": {"value": pts / t1 / 1e9, "unit": "Gpoints/s", "cores": 1,
                         "kind": "oracle", "seconds": round(t1, 3)},
            "all_cores": {"value": pts / tn / 1e9, "unit": "Gpoints/s", "cores": workers,
                          "kind": "oracle", "seconds": round(tn, 3)},
            "sample": "the first %d sets of the batch (%d points), whole method per set" % (S, pts)}


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


def bench_latency(dev, reps=50):
    """One set of 100,000 uniform-square points (about 0.8 MB, cache
    resident): latency of the whole method per call, both presets of the
    paper, eager calls and graph replays; median of `reps`."""
    import torch
    from paper_1405_3454_amd import inputs
    from paper_1405_3454_amd.api import Hull
    x, y = inputs.square(100_000, 100)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    off = torch.tensor([0, len(x)], dtype=torch.int64, device=dev)
    hull = torch.empty(len(x), dtype=torch.int32, device=dev)
    hc = torch.zeros(1, dtype=torch.int64, device=dev)
    ho = torch.zeros(2, dtype=torch.int64, device=dev)
    res = {}
    for preset in (0, 1):
        H = Hull(0, preset=preset)
        out = {}
        for name, fn in (("eager_us", lambda: H.compute_into(xt, yt, hull, hc)),
                         ("graph_us", lambda: H.graph_launch())):
            if name == "graph_us":
                H.graph_capture(xt, yt, off, hull, ho)
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            out[name] = round(float(np.median(ts)) * 1e6, 1)
        H.close()
        res[PRESET_NAMES[preset]] = out
    return {"workload": "one set of 100,000 uniform-square points, float32 k*2^-24",
            "median_of": reps, **res}


PRESET_NAMES = {0: "0/30/45/60 (paper)", 1: "0/30/75/120 (cumulative)", 2: "4 even (quadrilateral)",
                3: "8 even", 4: "12 even", 5: "16 even", 6: "20 even", 7: "24 even"}


def bench_directions(args, xb, yb, offb, X, Y, n):
    """Discard-vs-cost curve of the direction families: the whole method on
    the same four sets under every preset, as the main line runs it (one
    batched call per step, shapes tuned for the batch); the extremes pass
    cost grows with the direction count, the discard fraction with it."""
    import torch
    from paper_1405_3454_amd.api import Hull
    dev = xb.device
    S = offb.numel() - 1
    hb = torch.empty(S * n, dtype=torch.int32, device=dev)
    hob = torch.zeros(S + 1, dtype=torch.int64, device=dev)
    surv = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    steps = max(2, args.steps // 2)
    curve = []
    for preset in range(8):
        H = Hull(0, preset=preset)
        if not args.no_autotune:
            H.autotune(xb, yb, offb)

        def step():
            H.compute_batched_into(xb, yb, offb, hb, hob)
        t = _time(step, steps, 1)
        H.timing(True)
        H.timing_reset()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        kt = H.timing_read()
        H.timing(False)
        disc = {}
        for k in KINDS:
            slots, _ = H.extremes(X[k], Y[k])
            H.discard_into(X[k], Y[k], slots, surv, cnt)
            disc[k] = round(1.0 - cnt.item() / n, 6)
        H.close()
        us = {name: round(ms / c * 1e3, 1) for name, (ms, c) in kt.items()
              if name in ("extremes", "discard", "refine_pass", "polygon")}
        curve.append({"preset": preset, "directions": PRESET_NAMES[preset],
                      "gpts": round(S * n / t / 1e9, 3), "ms_per_step": round(t * 1e3, 3),
                      "us_mean_per_launch": us, "discard_fraction": disc})
    del hb, surv
    return curve


def bench_host(args, X, Y, n):
    """Host-resident input (the paper's setting): the disk set of the main
    workload held in host memory, hull_compute_host with chunks of 2^24
    points; PCIe-inclusive, so it is context, never the headline value."""
    import torch
    from paper_1405_3454_amd.api import Hull
    xh = X["disk"].cpu()
    yh = Y["disk"].cpu()
    xp, yp = xh.pin_memory(), yh.pin_memory()
    H = Hull(0)
    res = {"workload": "disk r=0.5, 2^%d points in host memory, chunks of 2^24" % int(np.log2(n))}
    ref = None
    for name, a, b, budget in (("pageable_streamed_twice", xh, yh, 0),
                               ("pageable_one_crossing", xh, yh, 1 << 40),
                               ("pinned_streamed_twice", xp, yp, 0),
                               ("pinned_one_crossing", xp, yp, 1 << 40)):
        H.compute_host(a, b, chunk_points=1 << 24, device_budget=budget, cap=n // 8)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, surv, hull = H.compute_host(a, b, chunk_points=1 << 24, device_budget=budget,
                                           cap=n // 8)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = min(ts)
        crossings = 1 if budget else 2
        hv = hull.cpu()
        if ref is None:
            ref = hv
        res[name] = {"gpts": round(n / t / 1e9, 3), "ms": round(t * 1e3, 2),
                     "pcie_gbs": round(crossings * 8.0 * n / t / 1e9, 1),
                     "same_hull": bool(torch.equal(ref, hv))}
    H.close()
    return res


def bench_3d(args, dev, log2n=24):
    """The 3D form: one set of 2^24 points per shape (cube, ball, shell,
    Gaussian), the whole method (two extremes passes, polyhedron, discard,
    hull of the survivors by QuickHull rounds); synchronises per round."""
    import torch
    from paper_1405_3454_amd import inputs
    from paper_1405_3454_amd.api import Hull
    n = 1 << log2n
    H = Hull(0)
    res = {"workload": "one set of 2^%d points per shape, float32 k*2^-24 in [0,1)^3" % log2n}
    for kind in ("cube", "ball", "shell", "gaussian"):
        x, y, z = inputs.set3_torch(kind, n, 900 + len(kind), device=dev)
        H.compute3(x, y, z)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, surv, hull = H.compute3(x, y, z)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        H.timing(True)
        H.timing_reset()
        H.compute3(x, y, z)
        torch.cuda.synchronize()
        kt = H.timing_read()
        H.timing(False)
        t = min(ts)
        ext_ms = kt.get("extremes", (0.0, 1))[0]
        disc_ms = kt.get("discard", (0.0, 1))[0]
        res[kind] = {"gpts": round(n / t / 1e9, 3), "ms": round(t * 1e3, 3),
                     "survivors": int(len(surv)), "hull_vertices": int(len(hull)),
                     "discard_fraction": round(1.0 - len(surv) / n, 6),
                     "extremes_us": round(ext_ms * 1e3, 1),
                     "extremes_gbs": round(2 * 12.0 * n / (ext_ms * 1e-3) / 1e9, 1) if ext_ms else None,
                     "discard_us": round(disc_ms * 1e3, 1),
                     "discard_gbs": round(12.0 * n / (disc_ms * 1e-3) / 1e9, 1) if disc_ms else None,
                     "hull_stage_ms": round((kt.get("refine_pass", (0.0, 1))[0] +
                                             kt.get("refine_split", (0.0, 1))[0]), 3)}
        del x, y, z
    H.close()
    torch.cuda.empty_cache()
    return res


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

    # profiling runs (--only) leave out the 4096 per-set calls
    t_set = None if getattr(args, "only", None) else _time(per_set, 2, 1)
    t_bat = _time(batched, args.steps, 1)
    H.graph_capture(x, y, off, hull, ho)
    t_graph = _time(H.graph_launch, args.steps, 1)
    disc = _discard_fraction_batched(H, x, y, off)
    H.close()
    cpu = None
    if not args.no_cpu:
        K = min(S, args.cpu_batch_sets)
        a = int(offs[K])
        cpu = cpu_baseline_batched(x[:a].cpu().numpy(), y[:a].cpu().numpy(), offs[:K + 1],
                                   min(16, host_cpu()["usable_threads"]))
    res = {"workload": "%d sets, sizes log-uniform [1e3, 1e6], square/disk/gaussian/annulus" % S,
           "points": int(n),
           "per_set_gpts": round(n / t_set / 1e9, 3) if t_set else None,
           "batched_gpts": round(n / t_bat / 1e9, 3),
           "graph_gpts": round(n / t_graph / 1e9, 3),
           "ms": {"per_set": round(t_set * 1e3, 3) if t_set else None, "batched": round(t_bat * 1e3, 3),
                  "graph": round(t_graph * 1e3, 3)},
           "speedup_graph_vs_per_set": round(t_set / t_graph, 2) if t_set else None,
           "discard_fraction": round(disc, 6),
           "tuning": tuning}
    if cpu is not None:
        res["cpu_baseline"] = cpu
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
    ap.add_argument("--cpu-batch-sets", type=int, default=1024,
                    help="sets of the batched workload the CPU oracle is timed on")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (no tuning before the timed steps)")
    ap.add_argument("--batch-sets", type=int, default=4096)
    ap.add_argument("--train-sets", type=int, default=200000)
    ap.add_argument("--skip-extra", action="store_true",
                    help="only the four 2^27 sets (no unfiltered, batched or learned lines)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--jsonl", metavar="PATH",
                    help="also append the result line, with its time and arguments, to PATH")
    ap.add_argument("--only", choices=("batched", "3d", "learned"),
                    help="run only this extra line and print its JSON (for profiling; "
                         "not the benchmark's result line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method runs each point set on a single "
              "device, and this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.only:
        import torch
        dev = torch.device("cuda:0")
        fn = {"batched": bench_batched, "3d": bench_3d, "learned": bench_learned}[args.only]
        print(json.dumps({args.only: fn(args, dev)}), flush=True)
        return

    import torch
    from paper_1405_3454_amd.api import Hull

    n = 1 << args.log2n
    t0 = time.time()
    data = generate(n)
    print("[bench] generated %d x %d points in %.1fs" % (len(KINDS), n, time.time() - t0),
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    # the four sets side by side in HBM (CSR offsets); X[k], Y[k] are views
    xb = torch.from_numpy(np.concatenate([data[k][0] for k in KINDS])).to(dev)
    yb = torch.from_numpy(np.concatenate([data[k][1] for k in KINDS])).to(dev)
    offb = torch.tensor([i * n for i in range(len(KINDS) + 1)], dtype=torch.int64, device=dev)
    X = {k: xb[i * n:(i + 1) * n] for i, k in enumerate(KINDS)}
    Y = {k: yb[i * n:(i + 1) * n] for i, k in enumerate(KINDS)}
    if args.no_cpu:
        del data
    H = Hull(0, preset=args.preset)
    # launch shapes tuned for the step (the batch) and for the one-set calls
    # of the diagnostics and the direction-family lines
    tuning = [] if args.no_autotune else H.autotune(xb, yb, offb)
    if not args.no_autotune:
        H.autotune(X["disk"], Y["disk"])
        tuning = H.tuning_table()
    hull = {k: torch.empty(n, dtype=torch.int32, device=dev) for k in KINDS}
    hcnt = {k: torch.zeros(1, dtype=torch.int64, device=dev) for k in KINDS}
    hb = torch.empty(len(KINDS) * n, dtype=torch.int32, device=dev)
    hob = torch.zeros(len(KINDS) + 1, dtype=torch.int64, device=dev)

    def step():
        # the whole method on each of the four sets, in one batched call
        H.compute_batched_into(xb, yb, offb, hb, hob)

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

    # per set: refinement and radix-sort passes against their algorithmic
    # bytes (a refinement round reads its input entries and writes the kept
    # ones, 14 B each; a radix pass reads and writes every key and index,
    # 16 B; up to 4096 keys are sorted in one block and no pass runs)
    passes = {}
    for k in KINDS:
        H.timing(True)
        H.timing_reset()
        for _ in range(args.steps):
            H.compute_into(X[k], Y[k], hull[k], hcnt[k])
        torch.cuda.synchronize()
        kk = H.timing_read()
        H.timing(False)
        cc = H.candidate_counts()
        ref_bytes = sum(14.0 * (cc[r] + cc[r + 1]) for r in range(len(cc) - 1)) if min(cc) >= 0 else 0.0
        keys = cc[-1]
        sort_bytes = 16.0 * keys * 6 if keys > 4096 else 0.0
        row = {"candidates": cc}
        for name, kinds, b in (("refine", ("refine_pass",), ref_bytes),
                               ("sort", ("sort_hist", "sort_scatter"), sort_bytes)):
            ms = sum(kk[c][0] for c in kinds if c in kk) / args.steps
            row[name] = {"us": round(ms * 1e3, 1), "alg_bytes": int(b),
                         "gbs": round(b / (ms * 1e-3) / 1e9, 1) if ms > 0 else None,
                         "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else None}
        passes[k] = row

    total_pts = len(KINDS) * n
    # survivors per set (discard fraction) from one extra discard call each
    disc = {}
    hob_c = hob.cpu().tolist()
    hs = {k: int(hob_c[i + 1] - hob_c[i]) for i, k in enumerate(KINDS)}
    for k in KINDS:
        slots, _ = H.extremes(X[k], Y[k])
        surv = torch.empty(n, dtype=torch.int32, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        H.discard_into(X[k], Y[k], slots, surv, cnt)
        disc[k] = 1.0 - cnt.item() / n
        assert hs[k] == int(hcnt[k].item()), "batched and one-set hulls differ"

    per_kernel = {name: {"ms_total": round(ms / args.steps, 4), "launches_per_step": c / args.steps,
                         "ms_mean": round(ms / c, 4)} for name, (ms, c) in kt.items()}
    # roofline of the dominant kernel by time per step; algorithmic bytes per
    # launch (one launch covers the four sets): the extremes pass reads x and
    # y (8 B per point); the full method's discard pass reads them and writes
    # each survivor's index, key and round-0 edge (4 + 8 + 2 B)
    surv_all = sum((1.0 - disc[k]) * n for k in KINDS)
    alg_bytes = {"extremes": 8.0 * total_pts, "discard": 8.0 * total_pts + 14.0 * surv_all}
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
            "launch": "one launch over the four sets",
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
                   "calls": "one batched call per step (CSR offsets over the four sets)",
                   "directions": PRESET_NAMES[args.preset]},
        "roofline": roof,
        "hbm_gbs": {k: round(v, 1) for k, v in hbm.items()},
        "discard_fraction": {k: round(v, 6) for k, v in disc.items()},
        "hull_vertices": hs,
        # generator seeds of every line (inputs.py draws every point from them)
        "seeds": {"sets": dict(SEEDS), "batched": {"sizes": 2024, "points": 2025},
                  "three_d": {k: 900 + len(k) for k in ("cube", "ball", "shell", "gaussian")},
                  "learned": {"training": 7, "points": 4242}},
        "per_kernel": per_kernel,
        "hull_stage_passes": passes,
        "tuning": tuning,
    }
    out["latency_100k"] = bench_latency(dev)
    if not args.skip_extra:
        # unfiltered arm: the same hull without the filter (sort + chain of
        # all points), the same one batched call per step
        hob_u = torch.zeros(len(KINDS) + 1, dtype=torch.int64, device=dev)

        def step_u():
            H.compute_batched_into(xb, yb, offb, hb, hob_u, nofilter=True)
        t_u = _time(step_u, max(2, args.steps // 2), 1)
        assert hob_u.cpu().tolist() == hob_c, "unfiltered and filtered hulls differ"
        out["unfiltered"] = {"gpts": round(total_pts / t_u / 1e9, 3),
                             "ms_per_step": round(t_u * 1e3, 3),
                             "speedup_of_filter": round(t_u / dt, 3)}
        out["direction_families"] = bench_directions(args, xb, yb, offb, X, Y, n)
        out["host_resident"] = bench_host(args, X, Y, n)
        H.close()
        del X, Y, hull, xb, yb, hb
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(args, dev)
        out["three_d"] = bench_3d(args, dev)
        out["learned"] = bench_learned(args, dev)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(data, min(n, args.cpu_sample))
        out["cpu_baseline"]["host"] = host_cpu()
    print(json.dumps(out), flush=True)
    if args.jsonl:     # the same record, appended with the time it was taken
        rec = dict(out, recorded_utc=time.strftime("%Y-%m-%dT%H:%M:%SZ", time.gmtime()),
                   argv=sys.argv[1:])
        with open(args.jsonl, "a") as f:
            f.write(json.dumps(rec) + "\n")
    if args.skip_extra:
        H.close()


if __name__ == "__main__":
    main()
