"""Throughput of the FP64 diffuse-interface step on one MI355X.

Default workload: the 2-D shock/elastoplastic-inclusion problem on a
2048 x 2048 grid (stiffened water, Romenskii solid disc with perfect
plasticity, THINC/BVD on, CFL 0.6, seeded +-1% density noise).  One step is
the whole hot path: the two split sweeps (reconstruction, THINC/BVD, Hancock
predictor, HLLC-type flux, conservative + non-conservative update), the
plastic and reactive fractional steps and the CFL max-wave-speed reduction,
whose result sets the next step's dt on the device (no host sync per step).

Output: one JSON line (metric, value = cell-updates/s, roofline of the
dominant kernel measured with HIP events, CPU-oracle baseline on a bounded
sample of the same workload).

Workload patch_set_4096: 4096 independent patches with log-uniform sides in
[16, 128] (same physics, two stored ghost layers each), advanced with one
persistent kernel per sweep and pairs of steps replayed from a HIP graph; the
same kernels launched once per patch and sweep are timed beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 flops (FMA) x 2.4 GHz
FP64_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# VALU issue: one wave64 instruction per SIMD every 4 cycles
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sweeps_shock_disc_2048.json")
VALU_FILES = {"shock_disc_2048": os.path.join(ROOT, "profiles", "valu_sweeps_shock_disc_2048.json"),
              "reactive_slab_256": os.path.join(ROOT, "profiles", "valu_sweeps_reactive_slab_256.json"),
              "rate_stick_800x2000": os.path.join(ROOT, "profiles", "valu_sweeps_rate_stick_800x2000.json")}
FLOPS_FILE = os.path.join(ROOT, "profiles", "flops_per_cell.json")
KERNEL_SOURCES = ["paper_2009_14555_amd/csrc/dimp_device.hpp", "paper_2009_14555_amd/csrc/dimp_stencil.hpp",
                  "paper_2009_14555_amd/csrc/dimp_lane.hpp", "paper_2009_14555_amd/csrc/dimp_sweeps.hpp",
                  "paper_2009_14555_amd/csrc/dimp_kernels.hip", "paper_2009_14555_amd/csrc/dimp_sweeps3.hip",
                  "paper_2009_14555_amd/csrc/dimp_patches.hpp", "paper_2009_14555_amd/csrc/dimp_patches.hip",
                  "paper_2009_14555_amd/csrc/dimp_patches_rx.hip", "paper_2009_14555_amd/csrc/dimp_patches_n3.hip",
                  "paper_2009_14555_amd/csrc/dimp_internal.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def workload(name: str):
    from paper_2009_14555_amd import problems as P

    if name in ("shock_disc_2048", "shock_disc_2048_rk3"):
        pb, W = P.shock_disc(2048, seed=0)
        desc = ("2-D shock on an elastoplastic disc, 2048x2048 FP64, stiffened water + Romenskii solid "
                "(perfect plasticity), THINC/BVD, minmod, CFL 0.6, seed 0")
        if name.endswith("_rk3"):
            desc += "; unsplit operator with the SSP-RK3 of Sec. 3.1"
    elif name == "shock_disc_jc_2048":
        pb, W = P.shock_disc_jc(2048, seed=0)
        desc = ("2-D shock on a Johnson-Cook copper disc (Table 1 Romenskii, Table 5 Johnson-Cook), 2048x2048 "
                "FP64, stiffened water, THINC/BVD, minmod, CFL 0.6, seed 0")
    elif name == "reactive_slab_256":
        pb, W = P.reactive_slab(256, seed=0)
        desc = ("3-D reactive mixture + elastoplastic slab, 256^3 FP64, hot spot 1e10 Pa, THINC/BVD, CFL 0.6, "
                "seed 0")
    elif name == "rate_stick_800x2000":
        pb, W = P.rate_stick(800, 2000, seed=0)
        desc = ("2-D Cartesian LX-17 rate stick in copper, 800x2000 FP64 (the effective resolution of the "
                "100x500 base grid with two factor-2 refinements, full width), JWL reactant/products (Table 3), "
                "ignition and growth (Table 4), Romenskii copper with perfect plasticity 0.4 GPa, 27 GPa booster, "
                "THINC/BVD, CFL 0.6, seed 0")
    elif name == "rate_stick_cyl_400x2000":
        pb, W = P.rate_stick_cyl(400, 2000, seed=0)
        desc = ("cylindrical LX-17 rate stick in copper (Sec. 4.2 geometry: r in [0, 2 r0] with the reflective "
                "axis, z in [0, 10 r0], r0 = 4 mm), 400x2000 FP64 (the paper's effective resolution), JWL "
                "(Table 3), ignition and growth (Table 4), Romenskii copper with perfect plasticity 0.4 GPa, "
                "27 GPa booster, geometric source by Heun's method, THINC/BVD, CFL 0.6, seed 0")
    elif name == "sod_1000":
        pb, W = P.sod_two_gamma(1000)
        desc = "1-D two-material Sod tube, 1000 cells, CFL 0.8"
    elif name == "patch_set_4096":
        tmpl, sizes, prims = P.patch_set(4096, seed=0)
        desc = ("4096 uneven 2-D patches (sides log-uniform in [16,128], 2 ghost layers), stiffened water + "
                "Romenskii solid disc + planar 1e9 Pa shock per patch, THINC/BVD, minmod, CFL 0.6, dx 1/2048, seed 0")
        return tmpl, (sizes, prims), desc
    else:
        raise SystemExit(f"unknown workload {name}")
    return pb, W, desc


def traffic_for(kind_name: str, workload_name: str = "shock_disc_2048"):
    """HBM bytes per launch of a kernel from the committed counter summary,
    only if it was taken on the current kernel sources and this workload"""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("workload", "shock_disc_2048") != workload_name:
        return None
    k = rec.get("kernels", {}).get(kind_name)
    return None if k is None else k.get("bytes_per_launch")


def valu_for(kind_name: str, workload_name: str = "shock_disc_2048"):
    """VALU counters per launch of a kernel (instructions, FP64 flops) from
    the committed counter summary, only if taken on the current sources and
    this workload"""
    try:
        with open(VALU_FILES[workload_name]) as f:
            rec = json.load(f)
    except (KeyError, OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("workload", "shock_disc_2048") != workload_name:
        return None
    return rec.get("kernels", {}).get(kind_name)


def flops_per_cell(workload_name: str):
    """algorithmic flops per cell of each phase (the oracle's operation
    count on the same seeded workload), or None"""
    try:
        with open(FLOPS_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    w = rec.get("workloads", {}).get(workload_name)
    return None if w is None else {k: v["flops"] for k, v in w["phases"].items()}


def with_alu(roof: dict, flops: dict, cells: int, workload_name: str = "shock_disc_2048"):
    """the dominant kernel's HBM roofline (algorithmic bytes per launch over
    its HIP-event duration, against 8 TB/s) with the FP64 view nested beside
    it: algorithmic flops per launch (the sweep along its axis, plus the
    sources and the wave speed when the launch is the fused last sweep) over
    the same duration, against the FP64 vector peak, and the VALU counters of
    the committed profile when it was taken on the current sources"""
    k = roof["kernel"]
    sec = roof["kernels"][k]["avg_us"] / 1e6
    out = dict(roof)
    if flops is not None:
        axis = k.split("_")[1]
        per_cell = flops["sweep_" + axis] + ((flops["sources"] + flops["wavespeed"]) if k.endswith("_fused") else 0.0)
        achieved = per_cell * cells / sec / 1e12
        out["alu"] = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(FP64_PEAK_TFLOPS, 1),
                      "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                      "alg_flops_per_launch": per_cell * cells, "alg_flops_per_cell": round(per_cell, 1)}
    v = valu_for(k, workload_name)
    if v is not None:
        out["valu_counters"] = {
            "issue_frac": round(v["valu_insts_per_launch"] / (VALU_ISSUE_PER_S * sec), 4),
            "f64_tflops_executed": round(v["f64_flops_per_launch"] / sec / 1e12, 2),
            "f64_share_of_valu": round(v["f64_insts_per_launch"] / v["valu_insts_per_launch"], 3)}
    else:
        out["valu_counters"] = None
    return out


def measure_grid(name: str, steps: int = 20, warmup: int = 3, probe_steps: int = 10):
    """a further single-grid workload: ms per step over `steps` device-CFL
    steps after `warmup`, the HBM fraction of the whole step, and the
    per-kernel HIP-event durations with the dominant kernel's roofline"""
    import torch

    from paper_2009_14555_amd import problems as P
    from paper_2009_14555_amd import solver as S

    pb, W, desc = workload(name)
    F, D = P.layout(pb).nfields, pb.ndim
    g = S.Grid(pb, device="cuda:0")
    g.set_primitive(W)
    g.advance_cfl(warmup)
    ms, _ = timed(g.stream, lambda: g.advance_cfl(steps))
    ms_step = ms / steps
    roof = with_alu(kernel_probe(g, probe_steps, pb.ncell, F, D), flops_per_cell(name), pb.ncell, name)
    print(f"[bench] {name}: {ms_step:.4f} ms/step, dominant {roof['kernel']} {roof['frac']:.3f} of HBM",
          file=sys.stderr, flush=True)
    return {"ms_per_step": round(ms_step, 4), "cell_updates_per_s": pb.ncell * steps / (ms / 1e3),
            "hbm_frac_step": round(D * 2 * F * 8 * pb.ncell / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "steps": steps, "warmup": warmup, "roofline": roof, "workload": desc}


def measure_amr3(nsteps: int = 10):
    """three levels, the paper's rate-stick hierarchy (a base grid with two
    factor-2 refinements, 800 x 2000 effective): a 200 x 500 coarse LX-17
    stick, level 1 over the explosive strip, its copper walls and the first
    40% of the stick, level 2 over the strip and the first 30%"""
    import torch

    from paper_2009_14555_amd import problems as P
    from paper_2009_14555_amd import solver as S

    pb0, W0 = P.rate_stick(200, 500, seed=0)
    box0, box1 = (40, 3, 160, 200), (20, 7, 228, 300)
    pb1, W1 = S.patch_prim(pb0, W0, box0)
    pb2, W2 = S.patch_prim(pb1, W1, box1)
    gs = [S.Grid(pb, device="cuda:0") for pb in (pb0, pb1, pb2)]
    for g, w in zip(gs, (W0, W1, W2)):
        g.set_primitive(w)
    outer, inner = S.Hierarchy(gs[0], gs[1], box0), S.Hierarchy(gs[1], gs[2], box1)
    outer.nest(inner)
    for _ in range(3):
        outer.advance(outer.dt())
    dt = outer.dt()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(gs[0].stream)
    for _ in range(nsteps):
        outer.advance(dt)
    ev1.record(gs[0].stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / nsteps
    outer.close()
    inner.close()
    upd = pb0.ncell + 2 * pb1.ncell + 4 * pb2.ncell
    print(f"[bench] three-level rate stick: {ms:.4f} ms per coarse step", file=sys.stderr, flush=True)
    return {"ms_per_coarse_step": round(ms, 4), "cell_updates_per_coarse_step": upd,
            "cell_updates_per_s": upd / (ms / 1e3), "cells": [pb0.ncell, pb1.ncell, pb2.ncell],
            "workload": "three levels (ratio 2, subcycled, refluxed): 200x500 coarse LX-17 rate stick in copper, "
                        "level 1 over coarse cells [40, 160) x [3, 200), level 2 over level-1 cells [20, 228) x "
                        "[7, 300), each stored with 4 ghost layers; fixed dt (the CFL step after 3 steps)"}


def measure_amr_patches(nsteps: int = 20):
    """the 400 x 1000 coarse rate stick with the single patch of the
    two-level case cut in two along the stick (one coarse row between them):
    one level of two patches stepped as a group"""
    import torch

    from paper_2009_14555_amd import problems as P
    from paper_2009_14555_amd import solver as S

    pbc, Wc = P.rate_stick(400, 1000, seed=0)
    boxes = [(90, 3, 310, 150), (90, 151, 310, 300)]
    gc = S.Grid(pbc, device="cuda:0")
    gc.set_primitive(Wc)
    gfs = []
    for b in boxes:
        pbf, Wf = S.patch_prim(pbc, Wc, b)
        g = S.Grid(pbf, device="cuda:0")
        g.set_primitive(Wf)
        gfs.append(g)
    hs = [S.Hierarchy(gc, g, b) for g, b in zip(gfs, boxes)]
    hs[0].group(hs[1])
    for _ in range(3):
        hs[0].advance(hs[0].dt())
    dt = hs[0].dt()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(gc.stream)
    for _ in range(nsteps):
        hs[0].advance(dt)
    ev1.record(gc.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / nsteps
    for h in hs:
        h.close()
    upd = pbc.ncell + 2 * sum(g.pb.ncell for g in gfs)
    print(f"[bench] AMR rate stick, two patches: {ms:.4f} ms per coarse step", file=sys.stderr, flush=True)
    return {"ms_per_coarse_step": round(ms, 4), "cell_updates_per_coarse_step": upd,
            "cell_updates_per_s": upd / (ms / 1e3),
            "workload": "two-level refinement with two patches on the fine level: 400x1000 coarse LX-17 rate stick, "
                        "patches over coarse cells [90, 310) x [3, 150) and [90, 310) x [151, 300), each stored "
                        "with 4 ghost layers; fixed dt (the CFL step after 3 steps)"}


def measure_amr(nsteps: int = 20, integrator: str = "split"):
    """two-level subcycled refinement: a 400 x 1000 coarse LX-17 rate stick
    (the 800 x 2000 workload at half resolution) with one ratio-2 patch over
    the explosive strip and its first 30% (booster and run-up); the fine
    level starts from its coarse parents"""
    import numpy as np
    import torch

    from paper_2009_14555_amd import problems as P
    from paper_2009_14555_amd import solver as S

    pbc, Wc = P.rate_stick(400, 1000, seed=0)
    box = (90, 3, 310, 300)
    pbf, Wf = S.patch_prim(pbc, Wc, box)
    gc, gf = S.Grid(pbc, device="cuda:0"), S.Grid(pbf, device="cuda:0")
    gc.set_primitive(Wc)
    gf.set_primitive(Wf)
    gc.set_integrator(integrator)
    gf.set_integrator(integrator)
    h = S.Hierarchy(gc, gf, box)
    for _ in range(3):
        h.advance(h.dt())
    dts = [h.dt() for _ in range(1)]
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(gc.stream)
    for _ in range(nsteps):
        h.advance(dts[0])
    ev1.record(gc.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / nsteps
    h.close()
    upd = pbc.ncell + 2 * pbf.ncell
    print(f"[bench] AMR rate stick ({integrator}): {ms:.4f} ms per coarse step", file=sys.stderr, flush=True)
    return {"ms_per_coarse_step": round(ms, 4), "cell_updates_per_coarse_step": upd,
            "cell_updates_per_s": upd / (ms / 1e3), "coarse_cells": pbc.ncell, "fine_cells": pbf.ncell,
            "workload": "two-level refinement (ratio 2, two fine steps per coarse step): coarse 400x1000 LX-17 "
                        "rate stick in copper, one patch over coarse cells [90, 310) x [3, 300) stored with 4 "
                        f"ghost layers; fixed dt (the CFL step after 3 steps); {integrator} integrator"}


def cpu_baseline(pb, W, steps: int, rk3: bool = False):
    """the oracle as it stands, on the same workload, all host cores"""
    from oracle import pyoracle as O

    import numpy as np

    nthreads = min(os.cpu_count() or 1, 64)
    O.set_threads(nthreads)
    o = O.Oracle(pb)
    U0 = o.prim_to_cons(W)
    dt = o.dt_cfl(U0)
    U, U1 = U0, None
    t0 = time.perf_counter()
    for k in range(steps):
        U = o.step_rk3(U, dt) if rk3 else o.step(U, dt, k)
        if k == 0:
            U1 = U
    el = time.perf_counter() - t0
    cores = O.get_threads()
    # the first step again on one thread: its rate, and the same bits
    O.set_threads(1)
    t0 = time.perf_counter()
    V = o.step_rk3(U0, dt) if rk3 else o.step(U0, dt, 0)
    el1 = time.perf_counter() - t0
    O.set_threads(nthreads)
    return {"value": pb.ncell * steps / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} full {'RK3 ' if rk3 else ''}step(s) of the same {pb.ncell}-cell workload from its "
                      f"initial state ({el:.1f} s wall)",
            "one_thread": {"value": pb.ncell / el1, "unit": "cell-updates/s", "cores": 1,
                           "sample": f"the first step on one thread ({el1:.1f} s wall)",
                           "bitwise_equal_to_all_cores": bool(np.array_equal(V, U1))}}


def cpu_baseline_patches(tmpl, sizes, prims, npatch: int):
    """the oracle stepping the first npatch patches of the set, one grid each"""
    from oracle import pyoracle as O

    nthreads = min(os.cpu_count() or 1, 64)
    O.set_threads(nthreads)
    cells, el = 0, 0.0
    for (nx, ny), W in list(zip(sizes, prims))[:npatch]:
        o = O.Oracle(tmpl.replace(n=(int(nx), int(ny), 1)))
        U = o.prim_to_cons(W)
        dt = o.dt_cfl(U)
        t0 = time.perf_counter()
        o.step(U, dt, 0)
        el += time.perf_counter() - t0
        cells += int(nx) * int(ny)
    return {"value": cells / el, "unit": "cell-updates/s", "cores": O.get_threads(), "kind": "oracle",
            "sample": f"one step of each of the first {npatch} patches ({cells} interior cells, {el:.1f} s)"}


def kernel_probe(g, probe_steps: int, cells: int, F: int, D: int, io_fields=None):
    """per-kernel durations with HIP events on the bound stream, and the
    roofline entry of the kernel with the largest total; io_fields maps a
    kernel to the state-sized arrays it must read and write (default 2: the
    state in and out)"""
    g.set_kernel_timing(True)
    g.advance_cfl(probe_steps)
    kt = g.kernel_times()
    g.set_kernel_timing(False)
    names = {(d, f): ("sweep_%s%s" % ("xyz"[d], "_fused" if f else "")) for d in range(3) for f in (False, True)}
    per_kernel = {names[k]: {"avg_ms": v[0] / v[1], "launches": v[1], "total_ms": v[0]} for k, v in kt.items()}
    dom = max(per_kernel, key=lambda n: per_kernel[n]["total_ms"])
    alg_bytes_launch = cells * (io_fields or {}).get(dom, 2) * F * 8  # one read and one write of the state per sweep
    achieved = alg_bytes_launch / (per_kernel[dom]["avg_ms"] / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
            "alg_bytes_per_launch": alg_bytes_launch,
            "kernels": {k: {"avg_us": round(v["avg_ms"] * 1e3, 2), "launches": v["launches"]}
                        for k, v in per_kernel.items()}}


def timed(stream, fn):
    import torch

    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1), time.perf_counter() - t0


def measure_batched(tmpl, sizes, prims, steps: int, warmup: int, probe_steps: int = 0, per_patch: bool = True):
    """patch set: batched launches replayed from a graph, the same kernels
    launched per patch and sweep (unless per_patch is False, so that a kernel
    trace holds the batched launches alone), and (optionally) the per-kernel
    probe"""
    import numpy as np

    from paper_2009_14555_amd import problems as P
    from paper_2009_14555_amd import solver as S

    F = P.layout(tmpl).nfields
    cells = int(np.sum(sizes[:, 0] * sizes[:, 1]))
    ps = S.PatchSet(tmpl, sizes, device="cuda:0")
    W = ps.pack(prims)
    ps.set_primitive(W)
    print(f"[bench] patch set: {len(sizes)} patches, {cells} interior cells, {ps.ncell} stored", file=sys.stderr,
          flush=True)
    best = ps.autotune(2)
    print(f"[bench] autotuned launch (row waves per block, tile columns): {best}", file=sys.stderr, flush=True)
    ms_base, nbase = None, 1
    if per_patch:
        # per-patch launches of the same kernels, from the same initial state
        base = S.PatchSet(tmpl, sizes, device="cuda:0")
        base.set_primitive(W)
        base.set_launch(True, *best)
        base.advance_cfl(2)
        nbase = max(2, steps // 10)
        ms_base, _ = timed(base.stream, lambda: base.advance_cfl(nbase))
        print(f"[bench] per-patch launches: {ms_base / nbase:.3f} ms/step over {nbase} steps", file=sys.stderr,
              flush=True)
        del base
    ps.advance_graph(warmup + (warmup % 2))
    ms_total, wall = timed(ps.stream, lambda: ps.advance_graph(steps))
    ms_step = ms_total / steps
    nbad = ps.check_state()
    print(f"[bench] batched graph: {ms_step:.4f} ms/step (wall {wall:.3f} s), bad cells {nbad}", file=sys.stderr,
          flush=True)
    ms_stream, _ = timed(ps.stream, lambda: ps.advance_cfl(steps))
    res = {"patches": int(len(sizes)), "interior_cells": cells, "stored_cells": int(ps.ncell), "launch": list(best),
           "graph_ms_per_step": round(ms_step, 4), "stream_ms_per_step": round(ms_stream / steps, 4),
           "per_patch_ms_per_step": round(ms_base / nbase, 4) if per_patch else None,
           "speedup_vs_per_patch": round((ms_base / nbase) / ms_step, 2) if per_patch else None,
           "cell_updates_per_s": cells * steps / (ms_total / 1e3),
           "hbm_frac_step": round(2 * 2 * F * 8 * cells / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    roof = kernel_probe(ps, probe_steps, cells, F, 2) if probe_steps else None
    return res, roof, F


def measure_adjoint(n: int = 512, nsteps: int = 200, K: int = 20):
    """calibration workload: plate impact, probe-row velocity misfit, the four
    material parameters and the initial velocity field as inputs; time of the
    forward run against forward + checkpointed backward"""
    import torch

    from paper_2009_14555_amd import adjoint as A
    from paper_2009_14555_amd import problems as P
    from paper_2009_14555_amd import solver as S

    pb, W = P.plate_impact(n)
    L = P.layout(pb)
    Wr = W.copy()
    Wr[L.u(0)] = 0.0
    g = S.Grid(pb, device="cuda:0")
    g.set_primitive(Wr)
    U_rest = g.state.clone()
    u0 = torch.tensor(W[L.u(0)], dtype=torch.float64, device="cuda:0")
    v0 = torch.zeros_like(u0)
    sim = A.Differentiable(g, [(0, "gamma"), (0, "pinf"), (1, "G0"), (1, "yield_stress")], K=K)
    th0 = torch.tensor(sim.theta0(), dtype=torch.float64)
    U0 = A.with_velocity(g, U_rest, u0, v0).detach()
    dts = sim.record_dts(U0, th0, nsteps)
    obs = A.probe_velocity(sim.run(U0, th0 * 1.05, dts), L, n // 2).detach()
    ms_fwd, _ = timed(g.stream, lambda: sim.run(U0, th0, dts))
    th = th0.clone().requires_grad_(True)
    u = u0.clone().requires_grad_(True)

    def fwd_adj():
        J = A.misfit(sim.run(A.with_velocity(g, U_rest, u, v0), th, dts), obs, L, n // 2)
        J.backward()

    fwd_adj()  # the first backward binds the adjoint workspace and loads its kernels
    runs = []
    for _ in range(3):
        th.grad = None
        u.grad = None
        runs.append(timed(g.stream, fwd_adj)[0])
    ms_all = sorted(runs)[1]
    ms_fwd = sorted([ms_fwd] + [timed(g.stream, lambda: sim.run(U0, th0, dts))[0] for _ in range(2)])[1]
    # the same gradients with every step's states kept from the forward (no
    # segment replay; 2 states a step in device memory)
    sim_st = A.Differentiable(g, sim.params, K=K, store=True)

    def fwd_adj_st():
        J = A.misfit(sim_st.run(A.with_velocity(g, U_rest, u, v0), th, dts), obs, L, n // 2)
        J.backward()

    runs_st = []
    for _ in range(3):
        th.grad = None
        u.grad = None
        runs_st.append(timed(g.stream, fwd_adj_st)[0])
    ms_st = sorted(runs_st)[1]
    # one step against one step adjoint, same state and dt
    Us = g.state.clone()
    lam = torch.randn_like(Us)
    dp = torch.zeros(12, dtype=torch.float64, device="cuda:0")
    g.adjoint_step(Us, lam, dts[0], 0, dp)
    ms_as, _ = timed(g.stream, lambda: [g.adjoint_step(Us, lam, dts[0], 0, dp) for _ in range(20)])
    # the same with the first sweep kept (as the backward pass runs it)
    g.set_conserved(Us)
    g.set_step_index(0)
    g.advance(dts[0])
    U1 = g.other.clone()
    ms_ak, _ = timed(g.stream, lambda: [g.adjoint_step(Us, lam, dts[0], 0, dp, first_sweep=U1) for _ in range(20)])
    g.set_conserved(Us)
    ms_s, _ = timed(g.stream, lambda: [g.advance(dts[0]) for _ in range(20)])
    print(f"[bench] adjoint: forward {ms_fwd:.1f} ms, forward+backward {ms_all:.1f} ms; step {ms_s / 20 * 1e3:.1f} us, "
          f"step adjoint {ms_as / 20 * 1e3:.1f} us, with the first sweep kept {ms_ak / 20 * 1e3:.1f} us; "
          f"forward+backward with stored states {ms_st:.1f} ms",
          file=sys.stderr, flush=True)
    return {"workload": f"plate impact {n}x{n} FP64, van Albada, THINC/BVD, {nsteps} steps, checkpoint every {K}, "
                        "gradients of a probe-row velocity misfit in (gamma, p_inf, G0, sigma_Y) and the initial "
                        "velocity field",
            "forward_ms": round(ms_fwd, 3), "forward_backward_ms": round(ms_all, 3),
            "timing": "median of 3 runs of each after one untimed forward + backward",
            "ratio_total_to_forward": round(ms_all / ms_fwd, 2),
            "forward_backward_stored_ms": round(ms_st, 3),
            "ratio_stored_total_to_forward": round(ms_st / ms_fwd, 2),
            "step_us": round(ms_s / 20 * 1e3, 2), "step_adjoint_us": round(ms_as / 20 * 1e3, 2),
            "ratio_step_adjoint_to_step": round(ms_as / ms_s, 2),
            "step_adjoint_kept_us": round(ms_ak / 20 * 1e3, 2),
            "ratio_step_adjoint_kept_to_step": round(ms_ak / ms_s, 2),
            "grad_params": [float(x) for x in th.grad.tolist()]}


def run_patches(args, tmpl, sizes, prims, desc) -> int:
    import numpy as np

    cells = int(np.sum(sizes[:, 0] * sizes[:, 1]))
    res, roof, F = measure_batched(tmpl, sizes, prims, args.steps, args.warmup, args.probe_steps,
                                   per_patch=not args.no_per_patch)
    ms_step = res["graph_ms_per_step"]
    out = {
        "metric": "fp64_cell_updates_per_s",
        "value": res["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "patches": res["patches"], "interior_cells": cells,
                   "stored_cells": res["stored_cells"], "fields": F, "launch": res["launch"]},
        "batched": res,
        "hbm_frac_step": res["hbm_frac_step"],
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_patches(tmpl, sizes, prims, 256)
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="shock_disc_2048")
    ap.add_argument("--cpu-steps", type=int, default=15)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe-steps", type=int, default=20, help="steps timed per kernel with HIP events")
    ap.add_argument("--no-per-patch", action="store_true",
                    help="patch-set workload: time the batched graph only (no per-patch launch baseline)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched patch-set and adjoint sections of the default run")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the solver runs on one device: sharding by slabs with a halo exchange is not implemented)",
              file=sys.stderr)
        return 2
    rank = int(os.environ.get("RANK", "0"))

    import torch

    from paper_2009_14555_amd import problems as P
    from paper_2009_14555_amd import solver as S

    if args.workload == "adjoint_plate_512":
        res = measure_adjoint()
        out = {"metric": "fp64_forward_backward_ms", "value": res["forward_backward_ms"], "unit": "ms",
               "n_gpus": 1, "steps": 200, "warmup": 0, "ms_per_step": res["forward_backward_ms"] / 200,
               "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic", "config": {"workload": res["workload"]}, "adjoint": res}
        print(json.dumps(out), flush=True)
        return 0
    if args.workload == "amr_rate_stick":
        res = {"two_levels": measure_amr(), "two_levels_rk3": measure_amr(integrator="rk3"),
               "two_patches": measure_amr_patches(), "three_levels": measure_amr3()}
        two = res["two_levels"]
        out = {"metric": "fp64_cell_updates_per_s", "value": two["cell_updates_per_s"], "unit": "cell-updates/s",
               "n_gpus": 1, "steps": 20, "warmup": 3, "ms_per_step": two["ms_per_coarse_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic", "config": {"workload": two["workload"]}, "amr": res}
        print(json.dumps(out), flush=True)
        return 0
    pb, W, desc = workload(args.workload)
    if args.workload == "patch_set_4096":
        return run_patches(args, pb, W[0], W[1], desc)
    L = P.layout(pb)
    F = L.nfields
    D = pb.ndim
    ncell = pb.ncell
    g = S.Grid(pb, device="cuda:0")
    g.set_primitive(W)
    rk3 = args.workload.endswith("_rk3")
    if rk3:
        g.set_integrator("rk3")
    torch.cuda.synchronize()
    print(f"[bench] {args.workload}: {ncell} cells, {F} fields, warmup {args.warmup}", file=sys.stderr, flush=True)

    # warmup, then the timed region: K whole steps, dt from the device CFL reduction
    g.advance_cfl(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(g.stream)
    g.advance_cfl(args.steps)
    ev1.record(g.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    value = ncell * args.steps / (ms_total / 1e3)
    nbad = g.check_state()
    print(f"[bench] timed {args.steps} steps: {ms_step:.4f} ms/step (wall {wall:.3f} s), bad cells {nbad}",
          file=sys.stderr, flush=True)

    # a plain device copy of the state (known size: F*ncell*8 bytes read and
    # written) that calibrates the HBM byte counters of a profiling run
    cal = g.state.clone()
    torch.cuda.synchronize()
    del cal

    # RK3 passes: y (and z) read the stage state and write a partial sum of
    # D(q) (z also reads the previous one); x reads the stage state, the
    # partial sum and q^n and writes the stage result
    io = {"sweep_x": 4, "sweep_x_fused": 4, "sweep_y": 2, "sweep_z": 3} if rk3 else None
    roof = kernel_probe(g, args.probe_steps, ncell, F, D, io)
    roof["traffic"] = traffic_for(roof["kernel"], args.workload)
    roof = with_alu(roof, flops_per_cell(args.workload), ncell, args.workload)
    # the same K-step region four more times: the median of five
    reps = [ms_step]
    for _ in range(4):
        ms_r, _ = timed(g.stream, lambda: g.advance_cfl(args.steps))
        reps.append(ms_r / args.steps)
    reps_sorted = sorted(reps)
    # algorithmic bytes per cell-update: one read and one write of the state
    # per sweep (split), per RK stage (RK3)
    step_alg_bytes = (3 if rk3 else D) * 2 * F * 8 * ncell
    out = {
        "metric": "fp64_cell_updates_per_s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "grid": list(pb.n[:D]), "fields": F,
                   "alg_bytes_per_cell_update": (3 if rk3 else D) * 2 * F * 8},
        "hbm_frac_step": round(step_alg_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "median_of_5": {"ms_per_step": round(reps_sorted[2], 4), "all_ms_per_step": [round(r, 4) for r in reps],
                        "hbm_frac_step": round(step_alg_bytes / (reps_sorted[2] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roof,
    }
    if not args.no_extras and args.workload == "shock_disc_2048":
        # the 3-D reactive workload (its own configuration)
        out["reactive_slab_256"] = measure_grid("reactive_slab_256")
        # the paper's own integrator on the same workload
        g.set_primitive(W)
        g.set_integrator("rk3")
        g.advance_cfl(3)
        ms_rk, _ = timed(g.stream, lambda: g.advance_cfl(20))
        out["rk3"] = {"ms_per_step": round(ms_rk / 20, 4), "cell_updates_per_s": ncell * 20 / (ms_rk / 1e3),
                      "workload": workload("shock_disc_2048_rk3")[2]}
        print(f"[bench] RK3 integrator: {ms_rk / 20:.4f} ms/step", file=sys.stderr, flush=True)
        # Johnson-Cook copper in place of the perfectly plastic solid
        del g
        pbj, Wj, descj = workload("shock_disc_jc_2048")
        gj = S.Grid(pbj, device="cuda:0")
        gj.set_primitive(Wj)
        gj.advance_cfl(3)
        ms_jc, _ = timed(gj.stream, lambda: gj.advance_cfl(20))
        out["johnson_cook"] = {"ms_per_step": round(ms_jc / 20, 4), "cell_updates_per_s": ncell * 20 / (ms_jc / 1e3),
                               "workload": descj}
        print(f"[bench] Johnson-Cook disc: {ms_jc / 20:.4f} ms/step", file=sys.stderr, flush=True)
        del gj
        # the JWL / ignition-and-growth rate stick
        pbs, Ws, descs = workload("rate_stick_800x2000")
        gs = S.Grid(pbs, device="cuda:0")
        gs.set_primitive(Ws)
        gs.advance_cfl(3)
        ms_rs, _ = timed(gs.stream, lambda: gs.advance_cfl(20))
        Ls = P.layout(pbs)
        st = gs.state
        lam = st[Ls.lam] / torch.clamp(st[Ls.m(0)], min=1e-300)
        mixed = int(((lam > 1e-12) & (lam < 1 - 1e-12)).sum().item())
        out["jwl_rate_stick"] = {"ms_per_step": round(ms_rs / 20, 4),
                                 "cell_updates_per_s": pbs.ncell * 20 / (ms_rs / 1e3),
                                 "cells_mid_reaction_after": mixed, "workload": descs}
        print(f"[bench] JWL rate stick: {ms_rs / 20:.4f} ms/step", file=sys.stderr, flush=True)
        del gs, st, lam
        # the same stick in its own cylindrical geometry (reflective axis, geometric source)
        pbc, Wc, descc = workload("rate_stick_cyl_400x2000")
        gc = S.Grid(pbc, device="cuda:0")
        gc.set_primitive(Wc)
        gc.advance_cfl(3)
        ms_cy, _ = timed(gc.stream, lambda: gc.advance_cfl(20))
        out["jwl_rate_stick_cylindrical"] = {"ms_per_step": round(ms_cy / 20, 4),
                                             "cell_updates_per_s": pbc.ncell * 20 / (ms_cy / 1e3),
                                             "workload": descc}
        print(f"[bench] cylindrical rate stick: {ms_cy / 20:.4f} ms/step", file=sys.stderr, flush=True)
        del gc
        out["amr_rate_stick"] = measure_amr()
        out["amr_rate_stick_rk3"] = measure_amr(integrator="rk3")
        out["amr3_rate_stick"] = measure_amr3()
        out["amr_rate_stick_two_patches"] = measure_amr_patches()
        g = None
        # the batched patch set and the adjoint step, each against its plain counterpart
        tmpl, sizes, prims = P.patch_set(4096, seed=0)
        out["batched"], _, _ = measure_batched(tmpl, sizes, prims, 40, 4)
        out["batched"]["workload"] = workload("patch_set_4096")[2]
        out["adjoint"] = measure_adjoint()
    if rank == 0 and not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pb, W, max(1, args.cpu_steps // 3) if rk3 else args.cpu_steps, rk3)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
