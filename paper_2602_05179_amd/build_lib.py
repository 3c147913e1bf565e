"""Build step for the HIP library: hipcc for gfx950, in-tree shared object."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsplit_eval.so")
SOURCES = [os.path.join(CSRC, "split_kernels.hip"), os.path.join(CSRC, "split_api.cpp"),
           os.path.join(CSRC, "split_server.cpp"), os.path.join(CSRC, "split_tune.cpp"),
           os.path.join(CSRC, "split_probe.hip"), os.path.join(CSRC, "split_routes.hip"),
           os.path.join(CSRC, "split_variant.hip"), os.path.join(CSRC, "split_minplus.hip"),
           os.path.join(CSRC, "split_search.cpp"), os.path.join(CSRC, "split_check.cpp"),
           os.path.join(CSRC, "split_serve.hip"), os.path.join(CSRC, "split_noalloc.hip"),
           os.path.join(CSRC, "split_ou.hip"), os.path.join(CSRC, "split_values.hip"), os.path.join(CSRC, "split_small.hip")]
HEADERS = [os.path.join(INCLUDE, "split_eval.h"), os.path.join(CSRC, "split_internal.h"),
           os.path.join(CSRC, "split_device.h"), os.path.join(CSRC, "window_min_asm.inc"),
           os.path.join(CSRC, "window_argmin_asm.inc"), os.path.join(CSRC, "split_variant.h"),
           os.path.join(CSRC, "split_minplus.h"),
           os.path.join(CSRC, "window_min_multi_asm.inc"), os.path.join(CSRC, "split_check.h"),
           os.path.join(CSRC, "split_serve.h"), os.path.join(CSRC, "split_dp.h"),
           os.path.join(CSRC, "split_values.h"), os.path.join(CSRC, "split_small.h")]
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


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n, len(SOURCES)))


def build_library(out: str = LIB, extra=(), incremental: bool = False) -> str:
    """Compile the kernels and the C ABI into one shared object (one hipcc
    process per source, in parallel, then one link).  `incremental` keeps
    object files and recompiles only sources newer than their object (or
    than any header)."""
    objdir = os.path.join(os.path.dirname(out), "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    newest_header = max(os.path.getmtime(h) for h in HEADERS)

    def compile_one(src):
        if incremental:
            obj = os.path.join(objdir, os.path.basename(src) + ".o")
            if os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(src), newest_header):
                return obj, 0
        else:
            obj = os.path.join(objdir, os.path.basename(src) + ".%d.o" % os.getpid())
        cmd = [hipcc(), *compile_flags, "-I", INCLUDE, "-I", CSRC, *extra, "-c", "-o", obj, src]
        return obj, subprocess.run(cmd).returncode

    with ThreadPoolExecutor(max_workers=_jobs()) as pool:
        results = list(pool.map(compile_one, SOURCES))
    objs = [o for o, _ in results]
    try:
        failed = [os.path.basename(s) for s, (_, rc) in zip(SOURCES, results) if rc != 0]
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc -c " + " ".join(failed))
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.run([hipcc(), *HIPCC_FLAGS, *extra, "-o", tmp, *objs], check=True)
        os.replace(tmp, out)
    finally:
        if not incremental:
            for o in objs:
                if os.path.exists(o):
                    os.remove(o)
    return out


def is_stale(out: str = LIB) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    import sys
    print(build_library(incremental="--incremental" in sys.argv))
