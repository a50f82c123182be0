"""ctypes binding of include/hull.h (argument marshalling only)."""
import ctypes
import os

import torch  # noqa: F401  -- load torch's HIP runtime first so the library shares it

from ._build import LIB

HULL_OK = 0
HULL_EINVAL = -1
HULL_ETOOBIG = -2
HULL_ENOMEM = -3
HULL_EHIP = -4
HULL_EDOMAIN = -5
HULL_ECAPTURE = -6
HULL_ENOMODEL = -7
HULL_ESCRATCH = -8
HULL_EOVERFLOW = -9
HULL_NOALLOC_MAX_POINTS = 1 << 27
HULL_NOALLOC_SCRATCH_BYTES = 40 << 20

HULL_DIRS_PAPER = 0
HULL_DIRS_CUMULATIVE = 1
HULL_NUM_PRESETS = 8


def HULL_DIRS_EVEN(groups):
    """Preset of `groups` rotation groups at 90 j / groups degrees (4 * groups
    evenly spaced directions); groups = 1 is the min/max quadrilateral."""
    return 1 + groups


HULL_DIRS_QUAD = HULL_DIRS_EVEN(1)

HULL_NOFILTER = 1
HULL_LEARNED = 2
HULL_VALIDATE = 4
HULL_NOREFINE = 8

HULL_NONE = 0xFFFFFFFF
HULL_NCOUNTS = 5
HULL_FIXED_SLOTS = 16
HULL_MAX_SLOTS = 24
HULL3_SLOTS = 42
HULL3_SERIAL = 16

P = ctypes.c_void_p
I = ctypes.c_int
I64 = ctypes.c_int64
D = ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "hull_create": (I, [ctypes.POINTER(P), I]),
    "hull_destroy": (I, [P]),
    "hull_set_directions": (I, [P, I]),
    "hull_direction_table": (I, [P, I, P, P, I]),
    "hull_slot_count": (I, [P, I]),
    "hull_strerror": (ctypes.c_char_p, [I]),
    "hull_last_hip_error": (I, [P]),
    "hull_extremes": (I, [P, P, P, I64, P, P, I, P]),
    "hull_extremes_noalloc": (I, [P, P, P, I64, P, P, I, P]),
    "hull_polygon": (I, [P, P, P, I64, P, I, P, P, P]),
    "hull_discard": (I, [P, P, P, I64, P, I, P, P, P]),
    "hull_of_subset": (I, [P, P, P, I64, P, P, I64, P, P, P]),
    "hull_compute": (I, [P, P, P, I64, P, P, I, P]),
    "hull_compute_host": (I, [P, P, P, I64, I64, I64, P, P, P, I64, P, P, I, P]),
    "hull3_compute": (I, [P, P, P, P, I64, P, P, P, P, P, I, P]),
    "hull_extremes_batched": (I, [P, P, P, P, I64, I64, P, I, P]),
    "hull_discard_batched": (I, [P, P, P, P, I64, I64, P, I, P, P, P]),
    "hull_compute_batched": (I, [P, P, P, P, I64, I64, P, P, I, P]),
    "hull_graph_capture": (I, [P, P, P, P, I64, I64, P, P, I, P]),
    "hull_graph_launch": (I, [P, P]),
    "hull_autotune": (I, [P, P, P, P, I64, I64, P]),
    "hull_tuning": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
    "hull_shape": (I, [P, I, I, I64, I64, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
    "hull_tuning_table": (I, [P, P, I]),
    "hull_mlp_param_count": (I64, []),
    "hull_mlp_set_params": (I, [P, P, I64]),
    "hull_mlp_get_params": (I, [P, P, I64]),
    "hull_mlp_get_state": (I, [P, P, I64, P]),
    "hull_mlp_set_state": (I, [P, P, I64, I64]),
    "hull_histogram_batched": (I, [P, P, P, P, I64, I64, P, P, P]),
    "hull_mlp_forward": (I, [P, P, I64, P, P]),
    "hull_mlp_backward": (I, [P, P, P, I64, P, P]),
    "hull_mlp_train_step": (I, [P, P, P, I64, ctypes.c_float, P, P]),
    "hull_top_directions": (I, [P, P, I64, P, P]),
    "hull_labels_batched": (I, [P, P, P, P, I64, I64, P, P]),
    "hull_label_targets_batched": (I, [P, P, P, P, I64, I64, I, P, P, P]),
    "hull_set_direction_gap": (I, [P, I]),
    "hull_timing_enable": (I, [P, I]),
    "hull_timing_read": (I, [P, P, P, I]),
    "hull_candidate_counts": (I, [P, P, I]),
    "hull_timing_name": (ctypes.c_char_p, [I]),
    "hull_timing_reset": (I, [P]),
}

_lib = None


class HullError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        msg = "%s: %s (%d)" % (what, lib().hull_strerror(code).decode(), code)
        super().__init__(msg)


def lib():
    """Load libhullgpu.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError("libhullgpu.so is not built; run paper_1405_3454_amd._build.build() "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code, what):
    if code < 0:
        raise HullError(code, what)
    return code
