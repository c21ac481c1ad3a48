"""Build the CPU oracle shared library (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "oracle.cpp")]

FLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
         "-fopenmp", "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", *FLAGS, *SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


SAN_FLAGS = ["-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-fopenmp",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build_sanitized(out_dir: str, verbose: bool = False) -> str:
    """the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only; any report aborts) into out_dir; a process that loads it
    must preload the sanitizer runtimes (sanitizer_preload())"""
    out = os.path.join(out_dir, "liboracle_san.so")
    cmd = ["g++", *SAN_FLAGS, *SRC, "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


def sanitizer_preload() -> str:
    """LD_PRELOAD value for a process that loads the sanitized oracle"""
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        r = subprocess.run(["g++", "-print-file-name=" + name], capture_output=True, text=True, check=True)
        libs.append(os.path.realpath(r.stdout.strip()))
    return ":".join(libs)


def ensure_built() -> str:
    if not os.path.exists(LIB) or any(os.path.getmtime(s) > os.path.getmtime(LIB)
                                      for s in SRC + [os.path.join(HERE, h) for h in ("oracle.h", "dual.h", "flops.h")]):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
