"""The C-ABI library loads and exports every symbol include/hull.h declares.

Host-only calls (no kernel launch) are exercised here; compute calls run in
the GPU tests.
"""
import ctypes
import os
import re

import mpmath
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hull.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int64_t|int|const char \*)\s*(hull3?_\w+)\s*\(", txt, re.M)))


def _int_of(expr):
    """Value of a header constant: an integer literal, optionally (1LL << k)
    or (k u << s)."""
    e = expr.strip()
    m = re.fullmatch(r"\(?\s*(\d+)(?:u|U|LL|ll)?\s*<<\s*(\d+)\s*\)?", e)
    if m:
        return int(m.group(1)) << int(m.group(2))
    m = re.fullmatch(r"\(?\s*(-?(?:0x[0-9A-Fa-f]+|\d+))(?:u|U|LL|ll)?\s*\)?", e)
    return int(m.group(1), 0) if m else None


def test_header_constants_match_the_binding():
    from paper_1405_3454_amd import _lib
    txt = open(HEADER).read()
    found = 0
    for name, expr in re.findall(r"^#define\s+(HULL\w*)\s+([^/\n]+?)\s*(?:/\*.*)?$", txt, re.M):
        v = _int_of(expr)
        if v is None or not hasattr(_lib, name):
            continue
        assert getattr(_lib, name) == v, (name, expr)
        found += 1
    assert found >= 25
    assert "hull3_compute" in _declared()


@pytest.fixture(scope="module")
def lib():
    from paper_1405_3454_amd import _build, _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("hull_extremes", "hull_polygon", "hull_discard", "hull_compute",
                 "hull_extremes_batched", "hull_discard_batched", "hull_compute_batched",
                 "hull_of_subset", "hull_graph_capture", "hull_graph_launch"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1405_3454_amd import _lib
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name


def test_strerror(lib):
    from paper_1405_3454_amd import _lib
    for code in (_lib.HULL_OK, _lib.HULL_EINVAL, _lib.HULL_ETOOBIG, _lib.HULL_ENOMEM,
                 _lib.HULL_EHIP, _lib.HULL_EDOMAIN, _lib.HULL_ECAPTURE, _lib.HULL_ENOMODEL):
        assert lib.hull_strerror(code)
    assert lib.hull_strerror(-99) == b"unknown error"


def test_null_arguments_rejected_without_device(lib):
    from paper_1405_3454_amd import _lib
    assert lib.hull_create(None, 0) == _lib.HULL_EINVAL
    assert lib.hull_destroy(None) == _lib.HULL_EINVAL
    assert lib.hull_compute(None, None, None, 0, None, None, 0, None) == _lib.HULL_EINVAL
    assert lib.hull_candidate_counts(None, None, 4) == _lib.HULL_EINVAL
    assert lib.hull_mlp_get_state(None, None, 0, None) == _lib.HULL_EINVAL
    assert lib.hull_mlp_set_state(None, None, 0, 0) == _lib.HULL_EINVAL
    assert lib.hull3_compute(None, None, None, None, 0, None, None, None, None, None, 0,
                             None) == _lib.HULL_EINVAL


def test_candidate_direction_table_correctly_rounded(lib):
    c = np.zeros(64)
    s = np.zeros(64)
    n = lib.hull_direction_table(None, 1, c.ctypes.data_as(ctypes.c_void_p),
                                 s.ctypes.data_as(ctypes.c_void_p), 64)
    assert n == 64
    mpmath.mp.prec = 300
    for d in range(64):
        if d % 16 == 0:
            cc, ss = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][d // 16]
        else:
            a = 2 * mpmath.pi * d / 64
            cc, ss = float(mpmath.cos(a)), float(mpmath.sin(a))
        assert c[d] == cc and s[d] == ss, d


def test_preset_table_matches_paper_angles(lib):
    c = np.zeros(4)
    s = np.zeros(4)
    n = lib.hull_direction_table(None, 0, c.ctypes.data_as(ctypes.c_void_p),
                                 s.ctypes.data_as(ctypes.c_void_p), 4)
    assert n == 4
    mpmath.mp.prec = 300
    for g, deg in enumerate([0, 30, 45, 60]):
        a = mpmath.pi * deg / 180
        assert c[g] == (1.0 if deg == 0 else float(mpmath.cos(a)))
        assert s[g] == (0.0 if deg == 0 else float(mpmath.sin(a)))


@pytest.mark.parametrize("preset", range(8))
def test_every_preset_table_correctly_rounded(lib, preset):
    """The library's own constants for every preset (which = 16 + preset,
    no device needed) against mpmath: presets 0 and 1 at the paper's angles,
    presets 1 + G at 90 j / G degrees."""
    c = np.zeros(8)
    s = np.zeros(8)
    n = lib.hull_direction_table(None, 16 + preset, c.ctypes.data_as(ctypes.c_void_p),
                                 s.ctypes.data_as(ctypes.c_void_p), 8)
    if preset == 0:
        degs = [0, 30, 45, 60]
    elif preset == 1:
        degs = [0, 30, 75, 120]
    else:
        G = preset - 1
        degs = [mpmath.mpf(90) * j / G for j in range(G)]
    assert n == len(degs)
    mpmath.mp.prec = 300
    for g, deg in enumerate(degs):
        a = mpmath.pi * deg / 180
        want_c = 1.0 if deg == 0 else float(mpmath.cos(a))
        want_s = 0.0 if deg == 0 else float(mpmath.sin(a))
        assert c[g] == want_c and s[g] == want_s, (preset, g)


def test_unknown_tables_rejected(lib):
    from paper_1405_3454_amd import _lib
    c = np.zeros(64)
    s = np.zeros(64)
    for which in (2, 15, 24, -1):
        assert lib.hull_direction_table(None, which, c.ctypes.data_as(ctypes.c_void_p),
                                        s.ctypes.data_as(ctypes.c_void_p), 64) == _lib.HULL_EINVAL
    # capacity below the table's size
    assert lib.hull_direction_table(None, 16 + 7, c.ctypes.data_as(ctypes.c_void_p),
                                    s.ctypes.data_as(ctypes.c_void_p), 5) == _lib.HULL_EINVAL
    assert lib.hull_slot_count(None, 0) == _lib.HULL_EINVAL
