"""Floating-point operations per cell-update of the step, counted by the
oracle on operation-counting scalars (measurement infrastructure).

    python -m oracle.count_flops [--out profiles/flops_per_cell.json]

Runs one step of each workload through or_step_flops (split) or
or_step_rk3_flops (the unsplit SSP-RK3) on the seeded inputs
(the same generators the GPU workloads use) and writes, per phase (the
sweep along each axis, the plastic/reactive steps, the wave speed of the
result), the operations per interior cell: add, mul, div, sqrt,
transcendental, comparison, and flops = add + mul + div + sqrt +
transcendental.  Operations on structural zeros are not counted.  The sweep
counts include the oracle's own pencil halo (cells -3..n+2 of each line),
which adds 6/n to the per-cell figure.

Only the non-reactive workload is counted: the oracle finds the reactive
mixture's phase split by plain bisection (64 halvings per cell and call),
which would overstate the work of a method that solves that equation in
closed form.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import pyoracle as O  # noqa: E402
from paper_2009_14555_amd import problems as P  # noqa: E402

COLS = ["add", "mul", "div", "sqrt", "trans", "cmp"]


def count(pb, W, threads: int, pre: int = 0):
    """counts of the step that follows `pre` plain oracle steps"""
    o = O.Oracle(pb)
    O.lib().or_set_threads(threads)
    U = o.prim_to_cons(W)
    for k in range(pre):
        U = o.step(U, o.dt_cfl(U), k)
    dt = o.dt_cfl(U)
    t0 = time.time()
    _, cnt = o.step_flops(U, dt, pre)
    el = time.time() - t0
    nc = int(np.prod(pb.n[: pb.ndim]))
    names = ["sweep_" + "xyz"[d] for d in range(pb.ndim)] + ["sources", "wavespeed"]
    phases = {}
    for name, row in zip(names, cnt):
        per = row / nc
        d = {c: round(float(v), 3) for c, v in zip(COLS, per)}
        d["flops"] = round(float(per[:5].sum()), 3)
        phases[name] = d
    total = round(sum(p["flops"] for p in phases.values()), 3)
    return {"grid": list(pb.n[: pb.ndim]), "cells": nc, "after_steps": pre, "dt": dt, "seconds": round(el, 2),
            "phases": phases, "flops_per_cell_update": total}


def count_rk3(pb, W, threads: int):
    """the SSP-RK3 step: per pass of the GPU's order (y first, x last), one
    evaluation of the direction's part of D(q); the x pass also forms the
    stage (a third of the step's combination work)"""
    o = O.Oracle(pb)
    O.lib().or_set_threads(threads)
    U = o.prim_to_cons(W)
    dt = o.dt_cfl(U)
    t0 = time.time()
    _, cnt = o.step_rk3_flops(U, dt)
    el = time.time() - t0
    nc = int(np.prod(pb.n[: pb.ndim]))
    D = pb.ndim
    rows = {"sweep_" + "xyz"[d]: cnt[d] / nc for d in range(D)}
    rows["sweep_x"] = rows["sweep_x"] + cnt[D] / nc / 3.0
    rows["sources"] = cnt[D + 1] / nc
    rows["wavespeed"] = cnt[D + 2] / nc
    phases = {}
    for name, per in rows.items():
        d = {c: round(float(v), 3) for c, v in zip(COLS, per)}
        d["flops"] = round(float(per[:5].sum()), 3)
        phases[name] = d
    total = 3 * sum(phases["sweep_" + "xyz"[d]]["flops"] for d in range(D)) + phases["sources"]["flops"] + \
        phases["wavespeed"]["flops"]
    return {"grid": list(pb.n[: pb.ndim]), "cells": nc, "integrator": "rk3", "dt": dt, "seconds": round(el, 2),
            "phases": phases, "flops_per_cell_update": round(total, 3)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "flops_per_cell.json"))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--shock-n", type=int, default=2048)
    args = ap.parse_args()
    res = {"command": "python -m oracle.count_flops",
           "convention": "per interior cell; flops = add + mul + div + sqrt + transcendental (one each); "
                         "comparisons listed apart; operations on structural zeros not counted",
           "workloads": {}}
    pb, W = P.shock_disc(args.shock_n, seed=0)
    res["workloads"]["shock_disc_%d" % args.shock_n] = count(pb, W, args.threads)
    print(json.dumps(res["workloads"]["shock_disc_%d" % args.shock_n]), flush=True)
    res["workloads"]["shock_disc_%d_rk3" % args.shock_n] = count_rk3(pb, W, args.threads)
    print(json.dumps(res["workloads"]["shock_disc_%d_rk3" % args.shock_n]), flush=True)
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
