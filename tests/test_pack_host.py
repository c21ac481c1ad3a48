"""Patch-set work-list packing, checked by a plain C++ build of the packer
(no GPU): coverage, lane bounds, stencil lanes inside their segment, per-patch
separation."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pack_lines(tmp_path):
    exe = tmp_path / "pack_check"
    src = os.path.join(ROOT, "tests", "pack_check.cpp")
    inc = os.path.join(ROOT, "paper_2009_14555_amd", "csrc")
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", inc, src, "-o", str(exe)], capture_output=True,
                       text=True)
    if r.returncode != 0:
        pytest.fail("g++ failed:\n" + r.stderr)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [l for l in r.stdout.splitlines() if l.startswith("OK")]
    assert len(lines) == 6, r.stdout
