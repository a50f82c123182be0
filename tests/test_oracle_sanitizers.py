"""The C oracles under AddressSanitizer and UndefinedBehaviorSanitizer.

Both oracle sources are rebuilt with -fsanitize=address,undefined (no
recovery) into a temporary directory and driven through their Python
wrappers in a child process (the ASan runtime preloaded): every entry point
on small sets, degenerate inputs (empty, one point, repeated, collinear,
flat, lattices with ties) and every preset.  A sanitizer report aborts the
child; its results must also equal the normal build's, which this process
computes.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from oracle import hull3d as o3
from paper_1405_3454_amd import inputs
out = []
G = float(1 << 24)
def grid(k):
    return (np.asarray(k, np.float64) / G).astype(np.float32)
# 2D: every preset, each step and the whole method, over shapes and sizes
for p in range(8):
    for n, kind, seed in ((0, "square", 1), (1, "disk", 2), (5, "gaussian", 3), (3000, "annulus", 4),
                          (2048, "square", 5)):
        if n == 0:
            x = y = np.zeros(0, np.float32)
        else:
            x, y = inputs.DISTRIBUTIONS[kind](n, seed)
        slots, vals = oracle.extremes(x, y, p)
        out.append(slots.tolist())
        out.append(oracle.compute(x, y, p).tolist())
# 2D degenerate: repeated and collinear points
k = np.arange(40) % 7
out.append(oracle.compute(grid(k), grid(2 * k), 0).tolist())
out.append(oracle.compute(grid(np.full(9, 5)), grid(np.full(9, 6)), 1).tolist())
# 3D: sizes, lattices (ties, coplanar points), flat and collinear sets
for n, kind, seed in ((1, "cube", 1), (17, "ball", 2), (2500, "shell", 3), (2500, "gaussian", 4)):
    x, y, z = inputs.DISTRIBUTIONS3[kind](n, seed)
    h, s = o3.compute(x, y, z, 0, want_survivors=True)
    out.append(h.tolist()); out.append(s.tolist())
    out.append(o3.compute(x, y, z, 1, nofilter=True).tolist())
for seed in range(3):
    x, y, z = inputs.lattice3(800, 3 + seed, 50 + seed)
    out.append(o3.compute(x, y, z, seed % 2).tolist())
a = np.arange(300) % 13
out.append(o3.compute(grid(a), grid(2 * a), grid(3 * a)).tolist())
out.append(o3.compute(grid(a), grid(np.full(300, 4)), grid(a * 7 % 11)).tolist())
import json
print(json.dumps(out))
'''


def _have_asan():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
        return p.returncode == 0 and os.path.isabs(p.stdout.strip()) and os.path.exists(p.stdout.strip())
    except OSError:
        return False


@pytest.mark.skipif(not _have_asan(), reason="gcc's AddressSanitizer runtime is not installed")
def test_oracles_clean_under_asan_and_ubsan(tmp_path):
    libs = {}
    for name, src in (("2d", "hull_oracle.c"), ("3d", "hull3d_oracle.c")):
        out = str(tmp_path / ("liboracle_%s_asan.so" % name))
        subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-Wall", "-fsanitize=address,undefined",
                               "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                               "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse", "-fPIC",
                               "-shared", os.path.join(ROOT, "oracle", src), "-o", out])
        libs[name] = out
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               HULL_ORACLE_LIB=libs["2d"], HULL_ORACLE3D_LIB=libs["3d"])
    r = subprocess.run([sys.executable, "-c", DRIVER, ROOT], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    # the same results as the normal build
    r2 = subprocess.run([sys.executable, "-c", DRIVER, ROOT], capture_output=True, text=True,
                        timeout=600)
    assert r2.returncode == 0, r2.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == r2.stdout.strip().splitlines()[-1]
