"""Build step for the HIP library: hipcc for gfx950, in-tree shared object."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsplit_eval.so")
SOURCES = [os.path.join(CSRC, "split_kernels.hip"), os.path.join(CSRC, "split_api.cpp"),
           os.path.join(CSRC, "split_server.cpp"), os.path.join(CSRC, "split_tune.cpp"),
           os.path.join(CSRC, "split_probe.hip"), os.path.join(CSRC, "split_routes.hip"),
           os.path.join(CSRC, "split_variant.hip"), os.path.join(CSRC, "split_minplus.hip"),
           os.path.join(CSRC, "split_search.cpp")]
HEADERS = [os.path.join(INCLUDE, "split_eval.h"), os.path.join(CSRC, "split_internal.h"),
           os.path.join(CSRC, "split_device.h"), os.path.join(CSRC, "window_min_asm.inc"),
           os.path.join(CSRC, "window_argmin_asm.inc"), os.path.join(CSRC, "split_variant.h"),
           os.path.join(CSRC, "split_minplus.h"),
           os.path.join(CSRC, "window_min_multi_asm.inc")]
ARCH = "gfx950"

# Packed FP32 instructions are disabled for every GPU object this library
# builds (none of the kernels use floating point in their hot loops anyway).
HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-pthread",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build_library(out: str = LIB, extra=()) -> str:
    """Compile the kernels and the C ABI into one shared object."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, *extra, "-o", tmp, *SOURCES]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def is_stale(out: str = LIB) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build_library())
