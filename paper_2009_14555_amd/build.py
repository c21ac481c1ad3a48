"""Build libdimp.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdimp.so")
SOURCES = [os.path.join(CSRC, "dimp_kernels.hip"), os.path.join(CSRC, "dimp_patches.hip"),
           os.path.join(CSRC, "dimp_patches_rx.hip"), os.path.join(CSRC, "dimp_patches_n3.hip"),
           os.path.join(CSRC, "dimp_adjoint.hip"), os.path.join(CSRC, "dimp_amr.hip"),
           os.path.join(CSRC, "dimp_velocity.hip"), os.path.join(CSRC, "dimp_sweeps3.hip"),
           os.path.join(CSRC, "dimp_sweeps_n3.hip"),
           os.path.join(CSRC, "dimp_capi.cpp")]
HEADERS = [os.path.join(CSRC, h) for h in ("dimp_device.hpp", "dimp_stencil.hpp", "dimp_lane.hpp", "dimp_sweeps.hpp",
                                              "dimp_internal.hpp", "dimp_pack.hpp", "dimp_patches.hpp", "dimp_adjoint.hpp",
                                              "dimp_amr.hpp")] + [
    os.path.join(ROOT, "include", "dimp.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (plain scalar FP64/FP32 code only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
    "-x", "hip",
]


OBJDIR = os.path.join(HERE, "_build")


def local_includes(path, seen=None):
    """the quoted includes a source reaches, recursively"""
    import re

    seen = set() if seen is None else seen
    for inc in re.findall(r'^\s*#include\s+"([^"]+)"', open(path).read(), re.M):
        f = os.path.normpath(os.path.join(os.path.dirname(path), inc))
        if f not in seen and os.path.exists(f):
            seen.add(f)
            local_includes(f, seen)
    return seen


def build(verbose: bool = False, resource_usage: bool = False, force: bool = True) -> str:
    """compile every source to an object in parallel (each translation unit
    holds its own kernels), then link the shared library; force=False
    recompiles only objects older than their source or a header"""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OBJDIR, exist_ok=True)
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    cflags = [f for f in FLAGS if f != "-shared"]

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        if (not force and not resource_usage and os.path.exists(obj)
                and os.path.getmtime(obj) > max(os.path.getmtime(f) for f in [src, *local_includes(src)])):
            return obj, subprocess.CompletedProcess([], 0, "", "")
        cmd = [HIPCC, *cflags, *extra, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return obj, subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, SOURCES))
    for obj, r in results:
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed")
        if resource_usage:
            sys.stderr.write(r.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in results], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


UNITS_SRC = os.path.join(ROOT, "tests", "adjoint_units.hip")
UNITS_LIB = os.path.join(ROOT, "tests", "libdimp_adjunits.so")


def build_units(verbose: bool = False) -> str:
    """test library: each reverse stage of the adjoint against central
    differences of its forward stage"""
    tmp = UNITS_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-I", CSRC, UNITS_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed (adjoint unit library)")
    os.replace(tmp, UNITS_LIB)
    return UNITS_LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True, resource_usage="--usage" in sys.argv)
    if "--units" in sys.argv:
        build_units(verbose=True)
