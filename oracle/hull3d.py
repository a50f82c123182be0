"""CPU oracle for the 3D form of the method (ctypes wrapper of hull3d_oracle.c).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT: only the tests, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the GPU library and never imports it.  The direction constants are the
2D presets' (``oracle.preset``).
"""
import ctypes
import os
import subprocess

import numpy as np

from . import NONE, PRESET_PAPER, preset

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hull3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle3d.so")


def build(force=True):
    """Compile hull3d_oracle.c into liboracle3d.so (gcc, binary64, no FMA)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
           "-msse2", "-mfpmath=sse", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # HULL_ORACLE3D_LIB: another build of the same source (the sanitizer test)
        path = os.environ.get("HULL_ORACLE3D_LIB", _LIB)
        if path == _LIB and not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(path)
        P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.oracle3_slot_count.argtypes = [I]
        L.oracle3_slot_count.restype = I
        L.oracle3_extremes.argtypes = [P, P, P, I64, P, P, I, P, P]
        L.oracle3_extremes.restype = None
        L.oracle3_polyhedron.argtypes = [P, P, P, P, I, P, I]
        L.oracle3_polyhedron.restype = I
        L.oracle3_discard.argtypes = [P, P, P, I64, P, I, P, P]
        L.oracle3_discard.restype = None
        L.oracle3_hull_subset.argtypes = [P, P, P, P, I64, P, P]
        L.oracle3_hull_subset.restype = I
        L.oracle3_compute.argtypes = [P, P, P, I64, P, P, I, I, P, P, P, P]
        L.oracle3_compute.restype = I
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _pts(x, y, z):
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.float32)
    assert x.shape == y.shape == z.shape and x.ndim == 1
    return x, y, z


def _cs(p, cs):
    c, s = cs if cs is not None else preset(p)
    return np.ascontiguousarray(c, np.float64), np.ascontiguousarray(s, np.float64)


def slot_count(p=PRESET_PAPER):
    return lib().oracle3_slot_count(len(preset(p)[0]))


def extremes(x, y, z, p=PRESET_PAPER, cs=None):
    """Step 1: slots (6 + 12 (G - 1)) and their binary64 values."""
    x, y, z = _pts(x, y, z)
    c, s = _cs(p, cs)
    G = len(c)
    ns = lib().oracle3_slot_count(G)
    slots = np.zeros(ns, np.uint32)
    vals = np.zeros(ns, np.float64)
    lib().oracle3_extremes(_p(x), _p(y), _p(z), len(x), _p(c), _p(s), G, _p(slots), _p(vals))
    return slots, vals


def polyhedron(x, y, z, slots):
    """Step 2: the polyhedron's planes as rows (nx, ny, nz, px, py, pz) in
    grid units, normal pointing inside; empty when it has no interior."""
    x, y, z = _pts(x, y, z)
    slots = np.ascontiguousarray(slots, np.uint32)
    cap = 8192
    planes = np.zeros((cap, 6), np.int64)
    nf = lib().oracle3_polyhedron(_p(x), _p(y), _p(z), _p(slots), len(slots), _p(planes), cap)
    assert nf <= cap
    return planes[:nf].copy()


def discard(x, y, z, planes):
    """Step 3: the survivors (ascending indices)."""
    x, y, z = _pts(x, y, z)
    planes = np.ascontiguousarray(planes, np.int64)
    surv = np.zeros(max(len(x), 1), np.uint32)
    cnt = ctypes.c_int64(0)
    lib().oracle3_discard(_p(x), _p(y), _p(z), len(x), _p(planes), len(planes), _p(surv),
                          ctypes.byref(cnt))
    return surv[: cnt.value].copy()


def hull_subset(x, y, z, idx=None):
    """Extreme points of the listed points (all if idx is None), ascending."""
    x, y, z = _pts(x, y, z)
    k = len(x) if idx is None else len(idx)
    idx = None if idx is None else np.ascontiguousarray(idx, np.uint32)
    out = np.zeros(max(k, 1), np.uint32)
    h = ctypes.c_int64(0)
    rc = lib().oracle3_hull_subset(_p(x), _p(y), _p(z), _p(idx), k, _p(out), ctypes.byref(h))
    if rc:
        raise RuntimeError("oracle3_hull_subset failed")
    return out[: h.value].copy()


def compute(x, y, z, p=PRESET_PAPER, nofilter=False, cs=None, want_survivors=False):
    """The whole 3D method: the hull's extreme points (and the survivors)."""
    x, y, z = _pts(x, y, z)
    c, s = _cs(p, cs)
    n = len(x)
    hull = np.zeros(max(n, 1), np.uint32)
    h = ctypes.c_int64(0)
    surv = np.zeros(max(n, 1), np.uint32) if want_survivors else None
    cnt = ctypes.c_int64(0)
    rc = lib().oracle3_compute(_p(x), _p(y), _p(z), n, _p(c), _p(s), len(c), int(bool(nofilter)),
                               _p(hull), ctypes.byref(h), _p(surv),
                               ctypes.byref(cnt) if surv is not None else None)
    if rc:
        raise RuntimeError("oracle3_compute failed")
    if want_survivors:
        return hull[: h.value].copy(), surv[: cnt.value].copy()
    return hull[: h.value].copy()


__all__ = ["build", "lib", "slot_count", "extremes", "polyhedron", "discard", "hull_subset",
           "compute", "NONE"]
