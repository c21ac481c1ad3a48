"""ctypes binding of libdimp.so (the HIP C-ABI of include/dimp.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  Importing this
module loads the library and raises if it is missing -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdimp.so")

OK, EINVAL, EUNSUPPORTED, EHIP, ENOMEM, ENONPHYSICAL, ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS = {0: "OK", -1: "EINVAL", -2: "EUNSUPPORTED", -3: "EHIP", -4: "ENOMEM", -5: "ENONPHYSICAL",
          -6: "ESTATE"}


class dimp_material(C.Structure):
    _fields_ = [("eos", C.c_int32), ("plast", C.c_int32), ("gamma", C.c_double), ("pinf", C.c_double),
                ("eref", C.c_double), ("rho0", C.c_double), ("K0", C.c_double), ("G0", C.c_double),
                ("abar", C.c_double), ("bbar", C.c_double), ("Gamma0", C.c_double), ("cv", C.c_double),
                ("yield_", C.c_double), ("jc", C.c_double * 7), ("jwl", C.c_double * 4)]


class dimp_reactive(C.Structure):
    _fields_ = [("mat", C.c_int32), ("law", C.c_int32), ("reactant", dimp_material),
                ("product", dimp_material), ("Q", C.c_double), ("k", C.c_double), ("n", C.c_double),
                ("pref", C.c_double), ("ig", C.c_double * 17)]


# order of dimp_reactive.ig (ignition-and-growth constants)
IG_ORDER = ("I", "G1", "G2", "a", "b", "c", "d", "e", "g", "x", "y", "z", "Fig", "FG1", "FG2", "rho0", "punit")
RATE_POWER, RATE_IGNITION_GROWTH = 0, 1
EOS_JWL = 3


class dimp_options(C.Structure):
    _fields_ = [("limiter", C.c_int32), ("thinc", C.c_int32), ("beta0", C.c_double), ("delta", C.c_double),
                ("eps", C.c_double), ("va_scale", C.c_double * 6)]


class DimpError(RuntimeError):
    def __init__(self, status, name, msg):
        super().__init__(f"{name} failed: {STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    dp = C.POINTER(C.c_double)
    sig = {
        "dimp_create_grid": [C.c_int, C.POINTER(C.c_int64), dp, C.POINTER(C.c_int32), C.POINTER(H)],
        "dimp_set_materials": [H, C.c_int, C.POINTER(dimp_material), C.POINTER(dimp_reactive)],
        "dimp_set_options": [H, C.POINTER(dimp_options)],
        "dimp_nfields": [H, C.POINTER(C.c_int), C.POINTER(C.c_int64)],
        "dimp_workspace_bytes": [H, C.c_int, C.POINTER(C.c_size_t)],
        "dimp_bind": [H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p],
        "dimp_current": [H, C.POINTER(C.c_int)],
        "dimp_prim_to_cons": [H, C.c_void_p],
        "dimp_cons_to_prim": [H, C.c_void_p],
        "dimp_set_conserved": [H, C.c_void_p],
        "dimp_sweep": [H, C.c_double, C.c_int],
        "dimp_sources": [H, C.c_double],
        "dimp_advance": [H, C.c_double],
        "dimp_advance_static": [H, C.c_double, C.c_void_p],
        "dimp_advance_cfl": [H, C.c_double, C.c_int, C.c_void_p],
        "dimp_set_step_index": [H, C.c_int64],
        "dimp_set_integrator": [H, C.c_int],
        "dimp_set_geometry": [H, C.c_int, C.c_double],
        "dimp_amr_workspace_bytes": [H, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)],
        "dimp_amr_create": [H, H, C.POINTER(C.c_int64), C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)],
        "dimp_amr_dt": [C.c_void_p, C.c_double, C.POINTER(C.c_double)],
        "dimp_amr_advance": [C.c_void_p, C.c_double],
        "dimp_amr_nest": [C.c_void_p, C.c_void_p],
        "dimp_amr_group": [C.c_void_p, C.c_void_p],
        "dimp_amr_destroy": [C.c_void_p],
        "dimp_amr_prolong": [C.c_void_p],
        "dimp_amr_tag": [H, C.c_void_p, C.c_double, C.c_void_p, C.POINTER(C.c_int64)],
        "dimp_max_wavespeed": [H, dp],
        "dimp_max_wavespeed_device": [H, C.c_void_p],
        "dimp_check_state": [H, C.POINTER(C.c_int64)],
        "dimp_set_kernel_timing": [H, C.c_int],
        "dimp_create_patch_set": [C.c_int64, C.POINTER(C.c_int32), dp, C.POINTER(H)],
        "dimp_patch_offsets": [H, C.POINTER(C.c_int64)],
        "dimp_set_patch_launch": [H, C.c_int, C.c_int, C.c_int],
        "dimp_autotune": [H, C.c_int, C.c_double, C.c_void_p, C.POINTER(C.c_int)],
        "dimp_adjoint_sweep": [H, C.c_double, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
        "dimp_adjoint_plastic": [H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
        "dimp_adjoint_step": [H, C.c_double, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
        "dimp_adjoint_step_kept": [H, C.c_double, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p],
        "dimp_adjoint_params": [H, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "dimp_with_velocity": [H, C.c_void_p, C.c_void_p, C.c_void_p],
        "dimp_with_velocity_adjoint": [H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
        "dimp_advance_graph": [H, C.c_double, C.c_int],
        "dimp_kernel_times": [H, dp, C.POINTER(C.c_int64)],
        "dimp_destroy": [H],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.dimp_last_error.argtypes = []
    L.dimp_last_error.restype = C.c_char_p
    return L


lib = _load()

INTEGRATOR_SPLIT, INTEGRATOR_RK3 = 0, 1
WS_RK3, WS_ADJOINT = 1, 2

EXPORTED = ["dimp_create_grid", "dimp_set_materials", "dimp_set_options", "dimp_nfields", "dimp_workspace_bytes",
            "dimp_bind", "dimp_amr_workspace_bytes",
            "dimp_current", "dimp_prim_to_cons", "dimp_cons_to_prim", "dimp_set_conserved", "dimp_sweep", "dimp_sources",
            "dimp_advance", "dimp_advance_static", "dimp_advance_cfl", "dimp_set_step_index", "dimp_set_integrator", "dimp_set_geometry",
            "dimp_max_wavespeed", "dimp_max_wavespeed_device",
            "dimp_check_state", "dimp_set_kernel_timing", "dimp_kernel_times", "dimp_last_error",
            "dimp_destroy", "dimp_create_patch_set", "dimp_patch_offsets", "dimp_set_patch_launch",
            "dimp_autotune", "dimp_advance_graph", "dimp_adjoint_sweep", "dimp_adjoint_plastic",
            "dimp_adjoint_step", "dimp_adjoint_step_kept", "dimp_adjoint_params", "dimp_with_velocity", "dimp_with_velocity_adjoint", "dimp_amr_create", "dimp_amr_dt", "dimp_amr_advance",
            "dimp_amr_nest", "dimp_amr_group", "dimp_amr_destroy", "dimp_amr_prolong", "dimp_amr_tag"]


def call(name, *args):
    rc = getattr(lib, name)(*args)
    if rc != OK:
        raise DimpError(rc, name, lib.dimp_last_error().decode())
    return rc


def material(m) -> dimp_material:
    out = dimp_material(m.eos, m.plast, m.gamma, m.pinf, m.eref, m.rho0, m.K0, m.G0, m.abar, m.bbar,
                        m.Gamma0, m.cv, m.yield_stress)
    jc = getattr(m, "jc_c1", 0.0)
    if jc:
        vals = [m.jc_c1, m.jc_c2, m.jc_c3, m.jc_n, m.jc_m, m.jc_tmelt - m.jc_t0, m.jc_chi0]
        for i, v in enumerate(vals):
            out.jc[i] = v
    if m.eos == EOS_JWL:
        for i, v in enumerate((m.jwl_A, m.jwl_B, m.jwl_R1, m.jwl_R2)):
            out.jwl[i] = v
    return out


def reactive(r) -> dimp_reactive:
    out = dimp_reactive()
    out.mat = r.mat
    if r.mat >= 0:
        out.reactant = material(r.reactant)
        out.product = material(r.product)
        out.Q, out.k, out.n, out.pref = r.Q, r.k, r.n, r.pref
        out.law = getattr(r, "law", RATE_POWER)
        if out.law == RATE_IGNITION_GROWTH:
            for i, k in enumerate(IG_ORDER):
                out.ig[i] = r.ig[k]
    return out


def options(pb) -> dimp_options:
    o = dimp_options()
    o.limiter = pb.limiter
    o.thinc = pb.thinc
    o.beta0, o.delta, o.eps = pb.beta0, pb.delta, pb.eps
    for i in range(6):
        o.va_scale[i] = pb.va_scale[i]
    return o
