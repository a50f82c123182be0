"""Train the learned direction proposal on the GPU with the library's own
kernels (labels, histograms, bf16 MFMA forward/backward, Adam).

Training data: sets of anisotropic Gaussian mixtures drawn on the device
(inputs.mixture_batch_torch).  Targets (default "marginal"): for each of the 64 candidate directions, the
fraction of the set that the 16-extreme filter keeps but the filter with
that direction's extreme point added discards (hull_labels_batched), scaled
per set by its maximum.  Alternative "greedy": joint labels
(hull_label_targets_batched), eight rounds each adding the direction whose
extreme point discards the most of what is still kept.  The picks at
inference are spread out by the direction gap (hull_set_direction_gap), so
the smooth marginal targets serve well.  Loss: mean squared error between
the 64 scores and the targets.

    python -m paper_1405_3454_amd.train --sets 20000 --batch 512 --points 65536 \
        --out paper_1405_3454_amd/weights/proposal.safetensors
"""
import argparse
import os
import sys
import time

import numpy as np

N_PARAMS = 512 * 1024 + 512 + 512 * 512 + 512 + 64 * 512 + 64


def init_params(seed):
    """He-normal weights, zero biases, in the library's parameter layout."""
    r = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((1024, 512), (512, 512), (512, 64)):
        parts.append((r.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def save_params(path, params, meta=None):
    from safetensors.numpy import save_file
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    save_file({"params": np.ascontiguousarray(params, np.float32)}, path,
              metadata={k: str(v) for k, v in (meta or {}).items()})


def load_params(path):
    from safetensors.numpy import load_file
    p = load_file(path)["params"]
    if p.size != N_PARAMS:
        raise ValueError("%s holds %d values, expected %d" % (path, p.size, N_PARAMS))
    return p


def batch_tensors(S, n, seed, device):
    import torch
    from . import inputs
    x, y = inputs.mixture_batch_torch(S, n, seed, device=device)
    off = torch.arange(S + 1, dtype=torch.int64, device=device) * n
    return x, y, off


def train(H, sets, batch, points, lr=1e-3, seed=0, log=None, init=None, targets="marginal"):
    """Train for ceil(sets / batch) Adam steps; returns (params, losses).
    targets: "greedy" (joint greedy targets) or "marginal" (per-direction
    marginal gains, each set scaled by its maximum)."""
    import torch
    dev = H.device
    H.mlp_set_params(init if init is not None else init_params(seed))
    steps = (sets + batch - 1) // batch
    losses = []
    t0 = time.time()
    for k in range(steps):
        x, y, off = batch_tensors(batch, points, 1_000_003 * (seed + 1) + k, dev)
        if targets == "greedy":
            gain, _ = H.label_targets_batched(x, y, off, rounds=8)
        else:
            gain = H.labels_batched(x, y, off)
        hist, _ = H.histogram_batched(x, y, off)
        loss = H.mlp_train_step(hist, gain, lr)
        losses.append(loss)
        if log and (k % 20 == 0 or k == steps - 1):
            log("step %d/%d loss %.5f  (%.1fs)" % (k + 1, steps, float(loss.item()), time.time() - t0))
    torch.cuda.synchronize()
    return H.mlp_get_params(), [float(l.item()) for l in losses]


def evaluate(H, x, y, off):
    """Mean discard fraction of the plain and the learned filter over the sets."""
    import torch
    S = off.numel() - 1
    res = {}
    for name, learned in (("plain", False), ("learned", True)):
        slots = H.extremes_batched(x, y, off, learned=learned)
        _, so = H.discard_batched(x, y, off, slots)
        sizes = (off[1:] - off[:-1]).double()
        kept = (so[1:] - so[:-1]).double()
        res[name] = float((1.0 - kept / sizes.clamp_min(1)).mean().item())
    torch.cuda.synchronize()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--points", type=int, default=1 << 16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights",
                                                   "proposal.safetensors"))
    args = ap.parse_args(argv)
    from .api import Hull
    H = Hull(0)
    params, losses = train(H, args.sets, args.batch, args.points, args.lr, args.seed,
                           log=lambda m: print(m, file=sys.stderr, flush=True))
    x, y, off = batch_tensors(256, args.points, 987654321, H.device)
    ev = evaluate(H, x, y, off)
    save_params(args.out, params, {"sets": args.sets, "batch": args.batch, "points": args.points,
                                   "lr": args.lr, "seed": args.seed,
                                   "final_loss": losses[-1], "eval": ev})
    print({"final_loss": losses[-1], "eval": ev, "out": args.out})


if __name__ == "__main__":
    main()
