"""Build the HIP library libhullgpu.so in-tree (hipcc, gfx950)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhullgpu.so")
ARCH = os.environ.get("HULL_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    # every binary64 expression is a sequence of separately rounded
    # operations unless the code calls fma() itself
    "-ffp-contract=off",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".h")))


def build(verbose=False):
    """Compile csrc/hull_lib.hip (which includes the kernel files) into
    libhullgpu.so next to this file.  Always recompiles."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + [os.path.join(CSRC, "hull_lib.hip"), "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
