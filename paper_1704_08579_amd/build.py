"""Build the HIP library (libhsort.so) for gfx950 with hipcc, in place."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhsort.so")

SOURCES = [os.path.join(CSRC, "hs_sort.hip")]
HEADERS = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")] + \
    [os.path.join(INCLUDE, "hsort.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-fvisibility=hidden",
    # hipcc -O3 forms packed fp32 ops by itself; keep them off.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Every atomic here is issued by one lane on purpose.  The atomic
    # optimizer rewrites such an atomic into a wave-combined one whose result
    # is broadcast at once, which makes the partition pass wait for all its
    # in-flight loads right after reserving a tile's slots.
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-I", INCLUDE,
    "-I", CSRC,
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every HIP source into libhsort.so (always, unless force=False
    and the library is newer than all sources)."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
    sys.exit(0)
