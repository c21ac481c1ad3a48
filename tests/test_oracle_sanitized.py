"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a build
of the same source with both (any report aborts the process) runs a set of
small steps that reach every physics branch -- two-gamma Sod with THINC,
the shock/disc with Romenskii plasticity, Johnson-Cook copper, the reactive
slab (3-D, power rate), an LX-17 detonation (JWL, ignition and growth), the
SSP-RK3, the cylindrical source with the axis, the dual-number step -- in a
child process, and must reproduce the plain build's results bit for bit."""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = r'''
import numpy as np
from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P


def run_all():
    out = {}
    cases = [
        ("sod", P.sod_two_gamma(60, thinc=True), "split", 6),
        ("disc", P.shock_disc(20, seed=3), "split", 4),
        ("jc", P.shock_disc_jc(16, seed=2), "split", 3),
        ("slab", P.reactive_slab(8, seed=1), "split", 2),
        ("det", P.detonation_1d(60), "split", 3),
        ("disc_rk3", P.shock_disc(16, seed=4), "rk3", 2),
        ("cyl", P.rate_stick_cyl(8, 16, seed=1), "split", 2),
    ]
    for name, (pb, W), integ, nsteps in cases:
        o = O.Oracle(pb)
        U = o.prim_to_cons(W)
        for k in range(nsteps):
            dt = o.dt_cfl(U)
            U = o.step_rk3(U, dt) if integ == "rk3" else o.step(U, dt, k)
        out[name] = U
        out[name + "_prim"] = o.cons_to_prim(U)
    pb, W = P.plate_impact(12, noise=1e-3, seed=1)
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    rng = np.random.default_rng(0)
    dU = rng.standard_normal((2,) + U.shape) * 1e-3 * np.abs(U)
    dpar = np.zeros((2, 2, 4))
    dpar[1, 1, 3] = 1.0
    U1, T1 = o.step_dual(U, dU, dpar, o.dt_cfl(U), 0)
    out["dual"] = U1
    out["dual_tan"] = T1
    return out
'''


def _child(path, lib, out):
    code = (f"import sys\nsys.path.insert(0, {ROOT!r})\n{CASES}\n"
            f"O.use_library({lib!r})\nO.set_threads(2)\n"
            f"np.savez({out!r}, **run_all())\nprint('sanitized run done', flush=True)\n")
    with open(path, "w") as f:
        f.write(code)


@pytest.mark.slow
def test_oracle_is_clean_under_asan_and_ubsan():
    from oracle import build

    with tempfile.TemporaryDirectory() as tmp:
        lib = build.build_sanitized(tmp)
        script = os.path.join(tmp, "child.py")
        out = os.path.join(tmp, "san.npz")
        _child(script, lib, out)
        env = dict(os.environ)
        env["LD_PRELOAD"] = build.sanitizer_preload()
        # Python's own allocations are not the oracle's: leaks are not checked
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
        env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
        r = subprocess.run([sys.executable, script], env=env, capture_output=True, text=True, timeout=900)
        assert r.returncode == 0 and "sanitized run done" in r.stdout, r.stdout[-3000:] + r.stderr[-6000:]
        assert "runtime error" not in r.stderr, r.stderr[-6000:]
        san = np.load(out)
        ns = {}
        exec(CASES, ns)
        plain = ns["run_all"]()
        for k, v in plain.items():
            assert np.array_equal(np.asarray(san[k]), np.asarray(v), equal_nan=True), k
