"""Python front end of the hull library: torch tensors in, torch tensors out.

Only argument marshalling happens here; every step of the method runs in the
library's HIP kernels (libhullgpu.so).  Indices come back as int32 tensors
holding uint32 values (use ``as_u32`` to view them as numpy uint32).
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (HULL_DIRS_CUMULATIVE, HULL_DIRS_EVEN, HULL_DIRS_PAPER, HULL_DIRS_QUAD,
                   HULL_LEARNED, HULL_NOFILTER, HULL_NOREFINE, HULL_VALIDATE, check, lib)

FIXED_SLOTS = 16
MAX_SLOTS = 24


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def as_u32(t):
    """int32 tensor of uint32 values -> numpy uint32 array."""
    return t.detach().cpu().numpy().view(np.uint32)


def _pts(x, y):
    if x.dtype != torch.float32 or y.dtype != torch.float32:
        raise TypeError("x, y must be float32")
    if not (x.is_cuda and y.is_cuda):
        raise TypeError("x, y must be device tensors")
    if not (x.is_contiguous() and y.is_contiguous()) or x.shape != y.shape or x.dim() != 1:
        raise ValueError("x, y must be contiguous 1-D tensors of equal length")
    return x.numel()


def _flags(nofilter=False, learned=False, validate=False, refine=True):
    return ((HULL_NOFILTER if nofilter else 0) | (HULL_LEARNED if learned else 0) |
            (HULL_VALIDATE if validate else 0) | (0 if refine else HULL_NOREFINE))


class Hull:
    """A library context on one device."""

    def __init__(self, device=0, preset=HULL_DIRS_PAPER):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        check(lib().hull_create(ctypes.byref(h), self.device.index or 0), "hull_create")
        self._h = h
        self.set_directions(preset)

    def close(self):
        if getattr(self, "_h", None):
            lib().hull_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration -----------------------------------------------------
    def set_directions(self, preset):
        check(lib().hull_set_directions(self._h, int(preset)), "hull_set_directions")
        self.preset = preset

    def slot_count(self, learned=False):
        """Slots per set of the extremes calls for the current preset."""
        return check(lib().hull_slot_count(self._h, _flags(learned=learned)), "hull_slot_count")

    def direction_table(self, which=0):
        c = np.zeros(64, np.float64)
        s = np.zeros(64, np.float64)
        n = check(lib().hull_direction_table(self._h, which, c.ctypes.data_as(ctypes.c_void_p),
                                             s.ctypes.data_as(ctypes.c_void_p), 64),
                  "hull_direction_table")
        return c[:n], s[:n]

    def tuning(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        check(lib().hull_tuning(self._h, 1, ctypes.byref(a), ctypes.byref(b)), "hull_tuning")
        return a.value, b.value

    def set_tuning(self, k1, k3):
        a, b = ctypes.c_int(k1), ctypes.c_int(k3)
        check(lib().hull_tuning(self._h, 0, ctypes.byref(a), ctypes.byref(b)), "hull_tuning")

    def shape(self, kernel, n, S=1):
        """(block size, blocks per CU, tiles per wave, tuned) of kernel 0
        (extremes pass) or 1 (discard pass) for n points in S sets."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        t = check(lib().hull_shape(self._h, 1, int(kernel), int(n), int(S), ctypes.byref(a),
                                   ctypes.byref(b), ctypes.byref(c)), "hull_shape")
        return a.value, b.value, c.value, bool(t)

    def set_shape(self, kernel, n, S, block_size, blocks_per_cu, tiles_per_wave):
        a, b, c = ctypes.c_int(block_size), ctypes.c_int(blocks_per_cu), ctypes.c_int(tiles_per_wave)
        check(lib().hull_shape(self._h, 0, int(kernel), int(n), int(S), ctypes.byref(a),
                               ctypes.byref(b), ctypes.byref(c)), "hull_shape")

    BUCKET_LIMITS = ("<2^14", "<2^17", "<2^20", "<2^23", "<2^26", ">=2^26")

    def tuning_table(self):
        """Tuned buckets: list of dicts (kernel, points, batched, shape)."""
        k = check(lib().hull_tuning_table(self._h, None, 0), "hull_tuning_table")
        rows = np.zeros((max(k, 1), 6), np.int32)
        k = check(lib().hull_tuning_table(self._h, rows.ctypes.data_as(ctypes.c_void_p), k),
                  "hull_tuning_table")
        return [{"kernel": ("extremes", "discard")[r[0]], "points": self.BUCKET_LIMITS[r[1]],
                 "batched": bool(r[2]), "block_size": int(r[3]), "blocks_per_cu": int(r[4]),
                 "tiles_per_wave": int(r[5])} for r in rows[:k]]

    def autotune(self, x, y, offsets=None, stream=None):
        n = _pts(x, y)
        S = 0 if offsets is None else offsets.numel() - 1
        check(lib().hull_autotune(self._h, _ptr(x), _ptr(y), _ptr(offsets), S, n, _stream(stream)),
              "hull_autotune")
        return self.tuning_table()

    # -- single set --------------------------------------------------------
    def extremes(self, x, y, learned=False, validate=False, stream=None):
        n = _pts(x, y)
        k = self.slot_count(learned)
        slots = torch.empty(k, dtype=torch.int32, device=x.device)
        vals = torch.empty(k, dtype=torch.float64, device=x.device)
        check(lib().hull_extremes(self._h, _ptr(x), _ptr(y), n, _ptr(slots), _ptr(vals),
                                  _flags(learned=learned, validate=validate), _stream(stream)),
              "hull_extremes")
        return slots, vals

    def polygon(self, x, y, slots, stream=None):
        n = _pts(x, y)
        slots = slots.to(device=x.device, dtype=torch.int32).contiguous()
        verts = torch.empty(max(1, slots.numel()), dtype=torch.int32, device=x.device)
        m = torch.zeros(1, dtype=torch.int32, device=x.device)
        check(lib().hull_polygon(self._h, _ptr(x), _ptr(y), n, _ptr(slots), slots.numel(),
                                 _ptr(verts), _ptr(m), _stream(stream)), "hull_polygon")
        return verts[: int(m.item())]

    def discard_into(self, x, y, slots, surv, n_surv, stream=None):
        """Asynchronous form: survivors to surv (int32[n]), count to n_surv (int64[1])."""
        n = _pts(x, y)
        check(lib().hull_discard(self._h, _ptr(x), _ptr(y), n, _ptr(slots), slots.numel(),
                                 _ptr(surv), _ptr(n_surv), _stream(stream)), "hull_discard")

    def discard(self, x, y, slots, stream=None):
        n = _pts(x, y)
        slots = slots.to(device=x.device, dtype=torch.int32).contiguous()
        surv = torch.empty(max(1, n), dtype=torch.int32, device=x.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=x.device)
        self.discard_into(x, y, slots, surv, cnt, stream)
        return surv[: int(cnt.item())]

    def hull_of_subset(self, x, y, idx, count=None, stream=None):
        n = _pts(x, y)
        idx = idx.to(device=x.device, dtype=torch.int32).contiguous()
        k = torch.tensor([idx.numel()] if count is None else [int(count)], dtype=torch.int64,
                         device=x.device)
        cap = max(1, idx.numel())
        hull = torch.empty(cap, dtype=torch.int32, device=x.device)
        h = torch.zeros(1, dtype=torch.int64, device=x.device)
        check(lib().hull_of_subset(self._h, _ptr(x), _ptr(y), n, _ptr(idx), _ptr(k), idx.numel(),
                                   _ptr(hull), _ptr(h), _stream(stream)), "hull_of_subset")
        return hull[: int(h.item())]

    def compute_into(self, x, y, hull, h, nofilter=False, learned=False, validate=False,
                     stream=None, refine=True):
        """Asynchronous form: hull indices to hull (int32[n]), count to h (int64[1])."""
        n = _pts(x, y)
        check(lib().hull_compute(self._h, _ptr(x), _ptr(y), n, _ptr(hull), _ptr(h),
                                 _flags(nofilter, learned, validate, refine), _stream(stream)),
              "hull_compute")

    def compute(self, x, y, nofilter=False, learned=False, validate=False, stream=None,
                refine=True):
        n = _pts(x, y)
        hull = torch.empty(max(1, n), dtype=torch.int32, device=x.device)
        h = torch.zeros(1, dtype=torch.int64, device=x.device)
        self.compute_into(x, y, hull, h, nofilter, learned, validate, stream, refine)
        return hull[: int(h.item())]

    # -- host-resident input ----------------------------------------------
    def compute_host(self, x, y, chunk_points=0, device_budget=0, cap=None, stream=None):
        """The whole method on a set in host memory: x, y are float32 numpy
        arrays or CPU torch tensors (pinned or not).  Returns (slots,
        survivors, hull) as device int32 tensors; cap bounds the survivors
        (default n)."""
        if isinstance(x, np.ndarray):
            x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
            y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32))
        if x.dtype != torch.float32 or y.dtype != torch.float32 or x.is_cuda or y.is_cuda:
            raise TypeError("x, y must be float32 host arrays")
        if not (x.is_contiguous() and y.is_contiguous()) or x.shape != y.shape or x.dim() != 1:
            raise ValueError("x, y must be contiguous 1-D arrays of equal length")
        n = x.numel()
        cap = n if cap is None else int(cap)
        dev = self.device
        slots = torch.empty(self.slot_count(), dtype=torch.int32, device=dev)
        surv = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
        hull = torch.empty(max(1, cap), dtype=torch.int32, device=dev)
        ns = torch.zeros(1, dtype=torch.int64, device=dev)
        h = torch.zeros(1, dtype=torch.int64, device=dev)
        xp = ctypes.c_void_p(x.data_ptr()) if n else None
        yp = ctypes.c_void_p(y.data_ptr()) if n else None
        check(lib().hull_compute_host(self._h, xp, yp, n, int(chunk_points), int(device_budget),
                                      _ptr(slots), _ptr(surv), _ptr(ns), cap, _ptr(hull), _ptr(h),
                                      0, _stream(stream)), "hull_compute_host")
        return slots, surv[: int(ns.item())], hull[: int(h.item())]

    # -- three dimensions -------------------------------------------------
    def compute3(self, x, y, z, nofilter=False, serial=False, stream=None):
        """The 3D method on device float32 x, y, z (16-byte aligned): returns
        (slots [42], survivors ascending, extreme points ascending) as int32
        device tensors.  serial: the hull stage inserts one point at a time
        in one block.  Synchronises."""
        n = _pts(x, y)
        if z.dtype != torch.float32 or not z.is_cuda or z.shape != x.shape or not z.is_contiguous():
            raise ValueError("z must be a contiguous float32 device tensor like x")
        dev = x.device
        slots = torch.full((_lib.HULL3_SLOTS,), -1, dtype=torch.int32, device=dev)
        surv = torch.empty(max(1, n), dtype=torch.int32, device=dev)
        hull = torch.empty(max(1, n), dtype=torch.int32, device=dev)
        ns = torch.zeros(1, dtype=torch.int64, device=dev)
        h = torch.zeros(1, dtype=torch.int64, device=dev)
        check(lib().hull3_compute(self._h, _ptr(x), _ptr(y), _ptr(z), n, _ptr(slots), _ptr(surv),
                                  _ptr(ns), _ptr(hull), _ptr(h),
                                  (HULL_NOFILTER if nofilter else 0) | (_lib.HULL3_SERIAL if serial else 0),
                                  _stream(stream)), "hull3_compute")
        return slots, surv[: int(ns.item())], hull[: int(h.item())]

    # -- batched -----------------------------------------------------------
    def extremes_batched(self, x, y, offsets, learned=False, validate=False, stream=None):
        n = _pts(x, y)
        S = offsets.numel() - 1
        k = self.slot_count(learned)
        slots = torch.empty(S * k, dtype=torch.int32, device=x.device)
        check(lib().hull_extremes_batched(self._h, _ptr(x), _ptr(y), _ptr(offsets), S, n,
                                          _ptr(slots), _flags(learned=learned, validate=validate),
                                          _stream(stream)), "hull_extremes_batched")
        return slots.view(S, k)

    def discard_batched(self, x, y, offsets, slots, stream=None):
        n = _pts(x, y)
        S = offsets.numel() - 1
        slots = slots.to(device=x.device, dtype=torch.int32).contiguous()
        k = slots.numel() // max(S, 1)
        surv = torch.empty(max(1, n), dtype=torch.int32, device=x.device)
        so = torch.zeros(S + 1, dtype=torch.int64, device=x.device)
        check(lib().hull_discard_batched(self._h, _ptr(x), _ptr(y), _ptr(offsets), S, n,
                                         _ptr(slots), k, _ptr(surv), _ptr(so), _stream(stream)),
              "hull_discard_batched")
        return surv, so

    def compute_batched_into(self, x, y, offsets, hull, hull_offsets, nofilter=False,
                             learned=False, validate=False, stream=None, refine=True):
        n = _pts(x, y)
        S = offsets.numel() - 1
        check(lib().hull_compute_batched(self._h, _ptr(x), _ptr(y), _ptr(offsets), S, n,
                                         _ptr(hull), _ptr(hull_offsets),
                                         _flags(nofilter, learned, validate, refine),
                                         _stream(stream)),
              "hull_compute_batched")

    def compute_batched(self, x, y, offsets, nofilter=False, learned=False, validate=False,
                        stream=None, refine=True):
        n = _pts(x, y)
        S = offsets.numel() - 1
        hull = torch.empty(max(1, n), dtype=torch.int32, device=x.device)
        ho = torch.zeros(S + 1, dtype=torch.int64, device=x.device)
        self.compute_batched_into(x, y, offsets, hull, ho, nofilter, learned, validate, stream,
                                  refine)
        return hull, ho

    def graph_capture(self, x, y, offsets, hull, hull_offsets, nofilter=False, learned=False,
                      stream=None, refine=True):
        n = _pts(x, y)
        S = offsets.numel() - 1
        check(lib().hull_graph_capture(self._h, _ptr(x), _ptr(y), _ptr(offsets), S, n,
                                       _ptr(hull), _ptr(hull_offsets),
                                       _flags(nofilter, learned, refine=refine),
                                       _stream(stream)), "hull_graph_capture")

    def graph_launch(self, stream=None):
        check(lib().hull_graph_launch(self._h, _stream(stream)), "hull_graph_launch")

    # -- learned direction proposal ----------------------------------------
    def mlp_param_count(self):
        return int(lib().hull_mlp_param_count())

    def mlp_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        check(lib().hull_mlp_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size),
              "hull_mlp_set_params")

    def mlp_get_params(self):
        p = np.zeros(self.mlp_param_count(), np.float32)
        check(lib().hull_mlp_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size),
              "hull_mlp_get_params")
        return p

    def mlp_get_state(self):
        """(parameters, Adam first moments, Adam second moments) as one float32
        array of 3 * param_count values, and the step count."""
        st = np.zeros(3 * self.mlp_param_count(), np.float32)
        step = ctypes.c_int64(0)
        check(lib().hull_mlp_get_state(self._h, st.ctypes.data_as(ctypes.c_void_p), st.size,
                                       ctypes.byref(step)), "hull_mlp_get_state")
        return st, int(step.value)

    def mlp_set_state(self, state, step):
        st = np.ascontiguousarray(state, dtype=np.float32)
        check(lib().hull_mlp_set_state(self._h, st.ctypes.data_as(ctypes.c_void_p), st.size,
                                       int(step)), "hull_mlp_set_state")

    def histogram_batched(self, x, y, offsets=None, stream=None):
        """(bf16 bits as int16 [S][1024], float32 [S][1024])"""
        n = _pts(x, y)
        S = 1 if offsets is None else offsets.numel() - 1
        hb = torch.empty((S, 1024), dtype=torch.int16, device=x.device)
        hf = torch.empty((S, 1024), dtype=torch.float32, device=x.device)
        check(lib().hull_histogram_batched(self._h, _ptr(x), _ptr(y), _ptr(offsets), S, n, _ptr(hb),
                                           _ptr(hf), _stream(stream)), "hull_histogram_batched")
        return hb, hf

    def mlp_forward(self, hist, stream=None):
        B = hist.shape[0]
        sc = torch.empty((B, 64), dtype=torch.float32, device=hist.device)
        check(lib().hull_mlp_forward(self._h, _ptr(hist), B, _ptr(sc), _stream(stream)),
              "hull_mlp_forward")
        return sc

    def mlp_backward(self, hist, dscores, stream=None):
        B = hist.shape[0]
        dscores = dscores.to(device=hist.device, dtype=torch.float32).contiguous()
        g = torch.empty(self.mlp_param_count(), dtype=torch.float32, device=hist.device)
        check(lib().hull_mlp_backward(self._h, _ptr(hist), _ptr(dscores), B, _ptr(g),
                                      _stream(stream)), "hull_mlp_backward")
        return g

    def mlp_train_step(self, hist, gain, lr, stream=None):
        B = hist.shape[0]
        gain = gain.to(device=hist.device, dtype=torch.float32).contiguous()
        loss = torch.zeros(1, dtype=torch.float32, device=hist.device)
        check(lib().hull_mlp_train_step(self._h, _ptr(hist), _ptr(gain), B, ctypes.c_float(lr),
                                        _ptr(loss), _stream(stream)), "hull_mlp_train_step")
        return loss

    DEFAULT_DIRECTION_GAP = 2

    def set_direction_gap(self, gap):
        """Minimum spacing (gap + 1 of 64 steps) between the learned picks."""
        check(lib().hull_set_direction_gap(self._h, int(gap)), "hull_set_direction_gap")

    def top_directions(self, scores, stream=None):
        S = scores.shape[0]
        scores = scores.to(dtype=torch.float32).contiguous()
        d = torch.empty((S, 8), dtype=torch.int32, device=scores.device)
        check(lib().hull_top_directions(self._h, _ptr(scores), S, _ptr(d), _stream(stream)),
              "hull_top_directions")
        return d

    def labels_batched(self, x, y, offsets, stream=None):
        n = _pts(x, y)
        S = offsets.numel() - 1
        g = torch.empty((S, 64), dtype=torch.float32, device=x.device)
        check(lib().hull_labels_batched(self._h, _ptr(x), _ptr(y), _ptr(offsets), S, n, _ptr(g),
                                        _stream(stream)), "hull_labels_batched")
        return g

    def label_targets_batched(self, x, y, offsets, rounds=8, stream=None):
        """Greedy joint targets [S, 64] (float32) and the greedy order
        [S, rounds] (int32, -1 after the sequence ends)."""
        n = _pts(x, y)
        S = offsets.numel() - 1
        t = torch.empty((S, 64), dtype=torch.float32, device=x.device)
        o = torch.empty((S, rounds), dtype=torch.int32, device=x.device)
        check(lib().hull_label_targets_batched(self._h, _ptr(x), _ptr(y), _ptr(offsets), S, n,
                                               int(rounds), _ptr(t), _ptr(o), _stream(stream)),
              "hull_label_targets_batched")
        return t, o

    # -- timing ------------------------------------------------------------
    def timing(self, on=True):
        check(lib().hull_timing_enable(self._h, int(bool(on))), "hull_timing_enable")

    def timing_reset(self):
        check(lib().hull_timing_reset(self._h), "hull_timing_reset")

    def candidate_counts(self):
        """Candidates summed over sets at each stage of the last computation:
        [discard survivors, after refinement round 1..4] (-1: round not run)."""
        c = np.full(8, -1, np.int64)
        k = check(lib().hull_candidate_counts(self._h, c.ctypes.data_as(ctypes.c_void_p), 8),
                  "hull_candidate_counts")
        return [int(v) for v in c[:k]]

    def timing_read(self):
        ms = np.zeros(64, np.float64)
        cnt = np.zeros(64, np.int64)
        k = check(lib().hull_timing_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                         cnt.ctypes.data_as(ctypes.c_void_p), 64), "hull_timing_read")
        return {lib().hull_timing_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(k)
                if cnt[i] > 0}


def split_csr(flat, offsets):
    """numpy helper: list of per-set arrays from a CSR pair."""
    off = np.asarray(offsets)
    return [flat[off[i]:off[i + 1]] for i in range(len(off) - 1)]


__all__ = ["Hull", "as_u32", "split_csr", "HULL_DIRS_PAPER", "HULL_DIRS_CUMULATIVE",
           "HULL_DIRS_EVEN", "HULL_DIRS_QUAD",
           "HULL_NOFILTER", "HULL_LEARNED", "HULL_VALIDATE", "HULL_NOREFINE", "_lib"]
