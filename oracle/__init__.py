"""CPU oracle for the interior-point-discarding 2D convex-hull preprocessor.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark import this package.  It
shares no code with the GPU library (``paper_1405_3454_amd``) and never
imports it.

The geometry lives in ``hull_oracle.c`` (plain single-threaded C, binary64,
no contraction); this module builds it with gcc and wraps it with ctypes on
numpy arrays.  The network part of the learned proposal lives in
``oracle/mlp.py``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hull_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NONE = 0xFFFFFFFF

# direction presets (Sec. 2 Step 1, Figure 1, Sec. 5)
PRESET_PAPER = 0       # rotations 0, 30, 45, 60 degrees
PRESET_CUMULATIVE = 1  # 30, 45, 45 read cumulatively: 0, 30, 75, 120 degrees
# presets 2..7: G = p - 1 groups at 90 j / G degrees (4G evenly spaced
# directions); preset 2 is the min/max x and y quadrilateral (Sec. 1, ref. [3])
EVEN_PRESETS = {2: 4, 3: 8, 4: 12, 5: 16, 6: 20, 7: 24}


def build(force=True):
    """Compile hull_oracle.c into liboracle.so (gcc, binary64, no FMA)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
           "-msse2", "-mfpmath=sse", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # HULL_ORACLE_LIB: another build of the same source (the sanitizer test)
        path = os.environ.get("HULL_ORACLE_LIB", _LIB)
        if path == _LIB and not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        L.oracle_preset.argtypes = [I, P, P]
        L.oracle_preset.restype = I
        L.oracle_direction_table.argtypes = [P, P]
        L.oracle_direction_table.restype = None
        L.oracle_extremes.argtypes = [P, P, I64, P, P, I, P, P]
        L.oracle_extremes.restype = None
        L.oracle_extremes_dirs.argtypes = [P, P, I64, P, P, I, P, P]
        L.oracle_extremes_dirs.restype = None
        L.oracle_hull_subset.argtypes = [P, P, P, I64, P, P]
        L.oracle_hull_subset.restype = I
        L.oracle_polygon.argtypes = [P, P, P, I, P, P]
        L.oracle_polygon.restype = I
        L.oracle_discard.argtypes = [P, P, I64, P, I, P, P]
        L.oracle_discard.restype = None
        L.oracle_compute.argtypes = [P, P, I64, P, P, I, I, P, P, P, P]
        L.oracle_compute.restype = I
        L.oracle_histogram.argtypes = [P, P, I64, P]
        L.oracle_histogram.restype = None
        L.oracle_labels.argtypes = [P, P, I64, P, P, I, P, P, I, P]
        L.oracle_labels.restype = I
        L.oracle_label_targets.argtypes = [P, P, I64, P, P, I, P, P, I, I, P, P]
        L.oracle_label_targets.restype = I
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pts(x, y):
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape == y.shape and x.ndim == 1
    return x, y


def preset(p=PRESET_PAPER):
    """(cos, sin) binary64 constants of a direction preset: 4 groups for
    presets 0 and 1, G = p - 1 evenly spaced groups for presets 2..7."""
    c = np.zeros(6, np.float64)
    s = np.zeros(6, np.float64)
    g = lib().oracle_preset(p, _p(c), _p(s))
    if g < 0:
        raise ValueError("unknown preset %r" % p)
    return c[:g], s[:g]


def direction_table():
    """The 64 candidate directions phi_d = 2 pi d / 64 as (cos, sin) arrays."""
    c = np.zeros(64, np.float64)
    s = np.zeros(64, np.float64)
    lib().oracle_direction_table(_p(c), _p(s))
    return c, s


def extremes(x, y, p=PRESET_PAPER, cs=None):
    """Step 1: slots[4G] (argmin u, argmax u, argmin v, argmax v per group) and
    their binary64 values.  cs=(c, s) overrides the preset."""
    x, y = _pts(x, y)
    c, s = cs if cs is not None else preset(p)
    c = np.ascontiguousarray(c, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    G = len(c)
    slots = np.zeros(4 * G, np.uint32)
    vals = np.zeros(4 * G, np.float64)
    lib().oracle_extremes(_p(x), _p(y), len(x), _p(c), _p(s), G, _p(slots), _p(vals))
    return slots, vals


def extremes_dirs(x, y, c, s):
    """Argmax of c*x + s*y per direction (lowest index on ties)."""
    x, y = _pts(x, y)
    c = np.ascontiguousarray(c, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    slots = np.zeros(len(c), np.uint32)
    vals = np.zeros(len(c), np.float64)
    lib().oracle_extremes_dirs(_p(x), _p(y), len(x), _p(c), _p(s), len(c), _p(slots), _p(vals))
    return slots, vals


def hull_subset(x, y, idx=None):
    """Andrew's monotone chain of the listed points: CCW vertex indices from
    the lexicographic minimum, collinear points excluded."""
    x, y = _pts(x, y)
    if idx is None:
        k = len(x)
        ip = None
    else:
        idx = np.ascontiguousarray(idx, np.uint32)
        k = len(idx)
        ip = _p(idx)
    out = np.zeros(max(k, 1), np.uint32)
    h = ctypes.c_int64(0)
    rc = lib().oracle_hull_subset(_p(x), _p(y), ip, k, _p(out), ctypes.byref(h))
    if rc:
        raise MemoryError("oracle_hull_subset")
    return out[: h.value].copy()


def polygon(x, y, slots):
    """Step 2: CCW polygon (vertex indices) of the extreme points."""
    x, y = _pts(x, y)
    slots = np.ascontiguousarray(slots, np.uint32)
    verts = np.zeros(max(len(slots), 1), np.uint32)
    m = ctypes.c_int(0)
    rc = lib().oracle_polygon(_p(x), _p(y), _p(slots), len(slots), _p(verts), ctypes.byref(m))
    if rc:
        raise ValueError("oracle_polygon")
    return verts[: m.value].copy()


def discard(x, y, verts):
    """Step 3: ascending indices of the points not strictly inside verts."""
    x, y = _pts(x, y)
    verts = np.ascontiguousarray(verts, np.uint32)
    surv = np.zeros(max(len(x), 1), np.uint32)
    cnt = ctypes.c_int64(0)
    lib().oracle_discard(_p(x), _p(y), len(x), _p(verts), len(verts), _p(surv), ctypes.byref(cnt))
    return surv[: cnt.value].copy()


def compute(x, y, p=PRESET_PAPER, nofilter=False, cs=None, want_survivors=False):
    """The whole method; returns the hull (and the survivors if asked)."""
    x, y = _pts(x, y)
    c, s = cs if cs is not None else preset(p)
    c = np.ascontiguousarray(c, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    n = len(x)
    hull = np.zeros(max(n, 1), np.uint32)
    h = ctypes.c_int64(0)
    surv = np.zeros(max(n, 1), np.uint32) if want_survivors else None
    cnt = ctypes.c_int64(0)
    rc = lib().oracle_compute(_p(x), _p(y), n, _p(c), _p(s), len(c), int(bool(nofilter)),
                              _p(hull), ctypes.byref(h),
                              _p(surv) if surv is not None else None,
                              ctypes.byref(cnt) if surv is not None else None)
    if rc:
        raise RuntimeError("oracle_compute failed")
    if want_survivors:
        return hull[: h.value].copy(), surv[: cnt.value].copy()
    return hull[: h.value].copy()


def histogram(x, y):
    """32 x 32 occupancy histogram (float32[1024], row by = y bin)."""
    x, y = _pts(x, y)
    h = np.zeros(1024, np.float32)
    lib().oracle_histogram(_p(x), _p(y), len(x), _p(h))
    return h


def labels(x, y, p=PRESET_PAPER, cs=None, dirs=None):
    """Per-direction marginal discard gain (fraction of all points)."""
    x, y = _pts(x, y)
    c, s = cs if cs is not None else preset(p)
    c = np.ascontiguousarray(c, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    cd, sd = dirs if dirs is not None else direction_table()
    cd = np.ascontiguousarray(cd, np.float64)
    sd = np.ascontiguousarray(sd, np.float64)
    gain = np.zeros(len(cd), np.float64)
    rc = lib().oracle_labels(_p(x), _p(y), len(x), _p(c), _p(s), len(c),
                             _p(cd), _p(sd), len(cd), _p(gain))
    if rc:
        raise RuntimeError("oracle_labels failed")
    return gain


def label_targets(x, y, rounds=8, p=PRESET_PAPER, cs=None, dirs=None):
    """Greedy joint training targets (float32 per direction) and the greedy
    order (int32 per round, -1 after the sequence ends)."""
    x, y = _pts(x, y)
    c, s = cs if cs is not None else preset(p)
    c = np.ascontiguousarray(c, np.float64)
    s = np.ascontiguousarray(s, np.float64)
    cd, sd = dirs if dirs is not None else direction_table()
    cd = np.ascontiguousarray(cd, np.float64)
    sd = np.ascontiguousarray(sd, np.float64)
    target = np.zeros(len(cd), np.float32)
    order = np.full(rounds, -1, np.int32)
    rc = lib().oracle_label_targets(_p(x), _p(y), len(x), _p(c), _p(s), len(c), _p(cd), _p(sd),
                                    len(cd), int(rounds), _p(target), _p(order))
    if rc:
        raise RuntimeError("oracle_label_targets failed")
    return target, order
