"""ctypes wrapper of the CPU oracle (test infrastructure only).

Arrays are numpy float64 of shape (F, *field_shape) in the field order of
oracle.h; the wrapper never touches the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

MAXMAT = 4


class or_mat(C.Structure):
    _fields_ = [("eos", C.c_int32), ("plast", C.c_int32), ("gamma", C.c_double), ("pinf", C.c_double),
                ("eref", C.c_double), ("rho0", C.c_double), ("K0", C.c_double), ("G0", C.c_double),
                ("abar", C.c_double), ("bbar", C.c_double), ("Gamma0", C.c_double), ("cv", C.c_double),
                ("yield_", C.c_double), ("jc_c1", C.c_double), ("jc_c2", C.c_double), ("jc_c3", C.c_double),
                ("jc_n", C.c_double), ("jc_m", C.c_double), ("jc_tmelt", C.c_double), ("jc_t0", C.c_double),
                ("jc_chi0", C.c_double), ("jwl_A", C.c_double), ("jwl_B", C.c_double), ("jwl_R1", C.c_double),
                ("jwl_R2", C.c_double)]


class or_rx(C.Structure):
    _fields_ = [("mat", C.c_int32), ("law", C.c_int32), ("reactant", or_mat), ("product", or_mat),
                ("Q", C.c_double), ("k", C.c_double), ("n", C.c_double), ("pref", C.c_double)] + \
        [("ig_" + k, C.c_double) for k in ("I", "G1", "G2", "a", "b", "c", "d", "e", "g", "x", "y", "z", "Fig",
                                             "FG1", "FG2", "rho0", "punit")]


class or_config(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nmat", C.c_int32), ("n", C.c_int64 * 3), ("dx", C.c_double * 3),
                ("bc", C.c_int32 * 3), ("limiter", C.c_int32), ("thinc", C.c_int32), ("pad", C.c_int32),
                ("beta0", C.c_double), ("delta", C.c_double), ("eps", C.c_double),
                ("va_scale", C.c_double * 6), ("mat", or_mat * MAXMAT), ("rx", or_rx), ("lo", C.c_double * 3),
                ("geom", C.c_int32), ("pad2", C.c_int32)]


_lib = None


def use_library(path: str) -> None:
    """load the oracle from another build of the same source (the sanitized
    build of the tests) before first use"""
    global _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _load(path)


def lib():
    if _lib is None:
        _load(_build.ensure_built())
    return _lib


def _load(path: str):
    global _lib
    if _lib is None:
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        cp = C.POINTER(or_config)
        for name, args in [
            ("or_nfields", [cp]),
            ("or_prim_to_cons", [cp, dp, dp]), ("or_cons_to_prim", [cp, dp, dp]),
            ("or_sweep", [cp, dp, C.c_double, C.c_int]), ("or_plastic", [cp, dp]),
            ("or_plastic_dt", [cp, dp, C.c_double]),
            ("or_reaction", [cp, dp, C.c_double]), ("or_step", [cp, dp, C.c_double, C.c_int64]),
            ("or_geometric", [cp, dp, C.c_double]), ("or_sweep_flux", [cp, dp, C.c_double, C.c_int, dp]),
            ("or_max_wavespeed", [cp, dp, dp]),
            ("or_step_dual", [cp, dp, dp, dp, C.c_double, C.c_int64, C.c_int]),
            ("or_stage_dual", [cp, dp, dp, dp, C.c_double, C.c_int64, C.c_int, C.c_int]),
            ("or_step_flops", [cp, dp, C.c_double, C.c_int64, dp]), ("or_flops_selftest", [dp]),
            ("or_rhs", [cp, dp, dp]), ("or_rhs_dir_flux", [cp, dp, C.c_int, dp, dp]), ("or_step_rk3", [cp, dp, C.c_double]),
            ("or_step_rk3_flops", [cp, dp, C.c_double, dp]),
            ("or_eos", [C.POINTER(or_mat), C.c_double, C.c_double, dp]),
            ("or_thinc", [C.c_double] * 6 + [dp]),
            ("or_youngs_beta", [cp, dp, C.c_int64, C.c_int, dp]),
            ("or_bvd_thinc", [dp, dp]), ("or_phi_edges", [cp, dp, dp, dp]),
            ("or_rx_residual", [cp, dp, C.c_int, dp, dp]), ("or_rx_split", [cp, dp, dp]),
            ("or_strain", [dp, dp, dp]), ("or_pade_exp", [dp, dp]),
            ("or_cell_diag", [cp, dp, dp]), ("or_cell_diag_prim", [cp, dp, dp, dp]),
            ("or_face_flux", [cp, C.c_int, dp, dp, dp, dp]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = None
        L.or_get_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return lib().or_get_threads()


def _mat(m) -> or_mat:
    return or_mat(m.eos, m.plast, m.gamma, m.pinf, m.eref, m.rho0, m.K0, m.G0, m.abar, m.bbar,
                  m.Gamma0, m.cv, m.yield_stress, m.jc_c1, m.jc_c2, m.jc_c3, m.jc_n, m.jc_m, m.jc_tmelt,
                  m.jc_t0, m.jc_chi0, m.jwl_A, m.jwl_B, m.jwl_R1, m.jwl_R2)


def config(pb) -> or_config:
    c = or_config()
    c.ndim = pb.ndim
    c.nmat = pb.nmat
    for d in range(3):
        c.n[d] = int(pb.n[d]) if d < pb.ndim else 1
        c.dx[d] = float(pb.dx[d])
        c.bc[d] = int(pb.bc[d])
        c.lo[d] = float(pb.lo[d])
    c.geom = int(getattr(pb, "geom", 0))
    c.limiter = pb.limiter
    c.thinc = pb.thinc
    c.beta0, c.delta, c.eps = pb.beta0, pb.delta, pb.eps
    for i in range(6):
        c.va_scale[i] = pb.va_scale[i]
    for l, m in enumerate(pb.materials):
        c.mat[l] = _mat(m)
    r = pb.reactive
    c.rx.mat = r.mat
    if r.mat >= 0:
        c.rx.reactant = _mat(r.reactant)
        c.rx.product = _mat(r.product)
        c.rx.Q, c.rx.k, c.rx.n, c.rx.pref = r.Q, r.k, r.n, r.pref
        c.rx.law = r.law
        for k, v in r.ig.items():
            setattr(c.rx, "ig_" + k, float(v))
    return c


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed ({rc})")


class Oracle:
    """Whole-grid oracle operations for one problem description."""

    def __init__(self, pb):
        self.pb = pb
        self.cfg = config(pb)
        self.F = lib().or_nfields(C.byref(self.cfg))
        if self.F < 0:
            raise ValueError("bad problem description")

    def _arr(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape[0] == self.F, (a.shape, self.F)
        return a

    def prim_to_cons(self, W):
        W = self._arr(W)
        U = np.empty_like(W)
        _check(lib().or_prim_to_cons(C.byref(self.cfg), _ptr(W), _ptr(U)), "prim_to_cons")
        return U

    def cons_to_prim(self, U):
        U = self._arr(U)
        W = np.empty_like(U)
        _check(lib().or_cons_to_prim(C.byref(self.cfg), _ptr(U), _ptr(W)), "cons_to_prim")
        return W

    def sweep(self, U, dt, d):
        U = self._arr(U).copy()
        _check(lib().or_sweep(C.byref(self.cfg), _ptr(U), float(dt), int(d)), "sweep")
        return U

    def plastic(self, U, dt=0.0):
        """the plastic step (a Johnson-Cook solid relaxes over dt; perfect
        plasticity is instantaneous)"""
        U = self._arr(U).copy()
        _check(lib().or_plastic_dt(C.byref(self.cfg), _ptr(U), float(dt)), "plastic")
        return U

    def reaction(self, U, dt):
        U = self._arr(U).copy()
        _check(lib().or_reaction(C.byref(self.cfg), _ptr(U), float(dt)), "reaction")
        return U

    def sweep_flux(self, U, dt, d):
        """(the swept state, the face fluxes: the field shape with one more
        face along d)"""
        U = self._arr(U).copy()
        shp = list(U.shape)
        ax = len(shp) - 1 - d
        shp[ax] += 1
        flux = np.zeros(shp)
        _check(lib().or_sweep_flux(C.byref(self.cfg), _ptr(U), float(dt), int(d), _ptr(flux)), "sweep_flux")
        return U, flux

    def geometric(self, U, dt):
        U = self._arr(U).copy()
        _check(lib().or_geometric(C.byref(self.cfg), _ptr(U), float(dt)), "geometric")
        return U

    def step(self, U, dt, step_index=0):
        U = self._arr(U).copy()
        _check(lib().or_step(C.byref(self.cfg), _ptr(U), float(dt), int(step_index)), "step")
        return U

    def step_dual(self, U, dU, dpar, dt, step_index=0, stage=-1):
        """one step with exact tangents: dU (K, F, ...) state directions and
        dpar (K, nmat, 4) directions of each material's (gamma, p_inf, G0,
        yield); returns (U1, dU1).  stage d < ndim: the sweep along d alone;
        stage ndim: the plastic/reactive steps alone"""
        U = self._arr(U).copy()
        dU = np.ascontiguousarray(dU, dtype=np.float64).copy()
        K = dU.shape[0]
        dpar = np.ascontiguousarray(dpar, dtype=np.float64).reshape(K, self.pb.nmat, 4)
        assert dU.shape[1:] == U.shape and K <= 6
        _check(lib().or_stage_dual(C.byref(self.cfg), _ptr(U), _ptr(dU), _ptr(dpar), float(dt), int(step_index), K,
                                   int(stage)), "step_dual")
        return U, dU

    def rhs(self, U):
        """the unsplit spatial operator D(U) (Sec. 3.1)"""
        U = self._arr(U)
        R = np.zeros_like(U)
        _check(lib().or_rhs(C.byref(self.cfg), _ptr(U), _ptr(R)), "rhs")
        return R

    def rhs_flux(self, U):
        """(D(U), {d: face fluxes of direction d}) with D(U) equal to rhs(U)
        bit for bit"""
        U = self._arr(U)
        R = np.zeros_like(U)
        fl = {}
        for d in range(self.pb.ndim):
            shp = list(U.shape)
            shp[len(shp) - 1 - d] += 1
            fl[d] = np.zeros(shp)
            _check(lib().or_rhs_dir_flux(C.byref(self.cfg), _ptr(U), int(d), _ptr(R), _ptr(fl[d])), "rhs_flux")
        return R, fl

    def step_rk3(self, U, dt):
        """one step of the paper's SSP-RK3 on the unsplit operator, then the
        plastic and reactive steps"""
        U = self._arr(U).copy()
        _check(lib().or_step_rk3(C.byref(self.cfg), _ptr(U), float(dt)), "step_rk3")
        return U

    def step_flops(self, U, dt, step_index=0):
        """one step on operation-counting scalars: (U1, counts) with counts
        of shape (ndim + 2, 6): rows = sweep along each axis, plastic /
        reactive steps, wave speed; columns = add, mul, div, sqrt,
        transcendental, comparison, summed over the grid"""
        U = self._arr(U).copy()
        counts = np.zeros((self.pb.ndim + 2, 6))
        _check(lib().or_step_flops(C.byref(self.cfg), _ptr(U), float(dt), int(step_index), _ptr(counts)),
               "step_flops")
        return U, counts

    def step_rk3_flops(self, U, dt):
        """one RK3 step on counting scalars: (U1, counts (ndim + 3, 6)): rows
        = one evaluation of each direction's part of D(q), the stage
        combinations, the sources, the wave speed"""
        U = self._arr(U).copy()
        counts = np.zeros((self.pb.ndim + 3, 6))
        _check(lib().or_step_rk3_flops(C.byref(self.cfg), _ptr(U), float(dt), _ptr(counts)), "step_rk3_flops")
        return U, counts

    def max_wavespeed(self, U):
        U = self._arr(U)
        s = np.zeros(3)
        _check(lib().or_max_wavespeed(C.byref(self.cfg), _ptr(U), _ptr(s)), "max_wavespeed")
        return s[: self.pb.ndim]

    def dt_cfl(self, U, cfl=None):
        cfl = self.pb.cfl if cfl is None else cfl
        s = self.max_wavespeed(U)
        return cfl * min(self.pb.dx[d] / s[d] for d in range(self.pb.ndim))

    def run(self, U, dts, step0=0):
        for k, dt in enumerate(dts):
            U = self.step(U, dt, step0 + k)
        return U

    def cell_diag(self, Ucell):
        Ucell = np.ascontiguousarray(Ucell, dtype=np.float64)
        out = np.zeros(12)
        _check(lib().or_cell_diag(C.byref(self.cfg), _ptr(Ucell), _ptr(out)), "cell_diag")
        keys = ["p", "c2", "cL2", "G", "rho", "s", "rho_a", "rho_b", "T_a", "T_b", "xi", "J2"]
        return dict(zip(keys, out))

    def cell_diag_prim(self, Wcell):
        Wcell = np.ascontiguousarray(Wcell, dtype=np.float64)
        out = np.zeros(12)
        U = np.zeros(self.F)
        _check(lib().or_cell_diag_prim(C.byref(self.cfg), _ptr(Wcell), _ptr(out), _ptr(U)), "diag_prim")
        keys = ["p", "c2", "cL2", "G", "rho", "s", "rho_a", "rho_b", "T_a", "T_b", "xi", "J2"]
        return dict(zip(keys, out)), U

    def face_flux(self, d, WL, WR):
        WL = np.ascontiguousarray(WL, dtype=np.float64)
        WR = np.ascontiguousarray(WR, dtype=np.float64)
        F = np.zeros(self.F)
        ex = np.zeros(4)
        _check(lib().or_face_flux(C.byref(self.cfg), int(d), _ptr(WL), _ptr(WR), _ptr(F), _ptr(ex)), "flux")
        return F, ex

    def phi_edges(self, q, beta):
        """the sweep's volume-fraction edges of the middle cell of the stencil
        q (5 values) with steepness beta (3 values: cells i-1, i, i+1):
        dict(left, right, thinc (bool), vM (4), vT (4), muscl (2), thinc_edges (2))"""
        q = np.ascontiguousarray(q, dtype=np.float64)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        out = np.zeros(16)
        _check(lib().or_phi_edges(C.byref(self.cfg), _ptr(q), _ptr(b), _ptr(out)), "phi_edges")
        return dict(left=out[0], right=out[1], thinc=bool(out[10]), vM=out[2:6].copy(), vT=out[6:10].copy(),
                    muscl=out[11:13].copy(), thinc_edges=out[13:15].copy())

    def rx_residual(self, Ucell, t):
        """the reactive split's residual over t values at one conserved cell:
        (T_b - T_a, p, T_a, T_b) arrays"""
        Ucell = np.ascontiguousarray(Ucell, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.float64)
        out = np.zeros((len(t), 4))
        _check(lib().or_rx_residual(C.byref(self.cfg), _ptr(Ucell), len(t), _ptr(t), _ptr(out)), "rx_residual")
        return out[:, 0], out[:, 1], out[:, 2], out[:, 3]

    def rx_split(self, Ucell) -> float:
        """the split root t the oracle takes at one conserved cell (1: pure)"""
        Ucell = np.ascontiguousarray(Ucell, dtype=np.float64)
        t = C.c_double()
        _check(lib().or_rx_split(C.byref(self.cfg), _ptr(Ucell), C.byref(t)), "rx_split")
        return t.value

    def youngs_beta(self, U, cell, d):
        U = self._arr(U)
        b = C.c_double()
        _check(lib().or_youngs_beta(C.byref(self.cfg), _ptr(U), int(cell), int(d), C.byref(b)), "youngs")
        return b.value


def eos(m, rho, J2=0.0):
    out = np.zeros(6)
    mm = _mat(m)
    _check(lib().or_eos(C.byref(mm), float(rho), float(J2), _ptr(out)), "eos")
    return dict(zip(["Gamma", "pref", "eref", "dpref", "deref", "G"], out))


def bvd_thinc(cand):
    """the BVD choice from the 8 edge candidates (MUSCL R of i-1, THINC R of
    i-1, MUSCL L and R of i, THINC L and R of i, MUSCL L of i+1, THINC L of
    i+1): (THINC chosen, variations for P = MUSCL (4), for P = THINC (4))"""
    c = np.ascontiguousarray(cand, dtype=np.float64)
    v = np.zeros(8)
    r = lib().or_bvd_thinc(_ptr(c), _ptr(v))
    return bool(r), v[:4].copy(), v[4:].copy()


def thinc(qm, q0, qp, beta, eps=1e-20, delta=1e-5):
    out = np.zeros(4)
    lib().or_thinc(qm, q0, qp, beta, eps, delta, _ptr(out))
    return out[0], out[1], out[2], bool(out[3])


def strain(V):
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(9)
    H = np.zeros(9)
    J2 = C.c_double()
    lib().or_strain(_ptr(V), _ptr(H), C.cast(C.byref(J2), C.POINTER(C.c_double)))
    return H.reshape(3, 3), J2.value


def pade_exp(H):
    H = np.ascontiguousarray(H, dtype=np.float64).reshape(9)
    V = np.zeros(9)
    lib().or_pade_exp(_ptr(H), _ptr(V))
    return V.reshape(3, 3)


def flops_selftest():
    out = np.zeros(18)
    _check(lib().or_flops_selftest(_ptr(out)), "flops_selftest")
    return out.reshape(3, 6)
