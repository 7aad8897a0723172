"""Build libmi.so (the HIP library) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmi.so")

SOURCES = ["mi_kernels.hip", "mi_layout.hip", "mi_sparse.hip", "mi_categorical.hip", "mi_api.hip", "mi_noalloc.hip", "mi_server.cpp"]
HEADERS = ["mi_device.hpp", "mi_internal.hpp", "mi_host.hpp"]

# -packed-fp32-ops: keep hipcc from emitting packed FP32 instructions.
# -ffp-contract=off: the MI epilogue must not be contracted into FMAs, so that
# every kernel variant produces bitwise identical (and symmetric) results.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-pass-failed",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build_library(verbose: bool = False) -> str:
    """Compile every HIP/C++ source of the library into libmi.so; returns its path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, "-I" + INCLUDE, "-I" + CSRC, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout[-4000:] + res.stderr[-8000:])
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(INCLUDE, "mi.h")]
    return any(os.path.exists(d) and os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build_library(verbose=True))
