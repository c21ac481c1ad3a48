"""Hand-written adjoint of the step on the GPU: dot-product tests against
central finite differences of the GPU forward, <w, (S(U+eps v) - S(U-eps v))
/ 2 eps> = <S^T w, v>, for each stage and for a whole step, and the material
parameter adjoints against finite differences in the parameter.

Finite differences need the van Albada epsilon well above the perturbation:
with the default (1e-6 of the field scale) the limiter turns within a few
1e-6 of a flat region, so a central difference of any usable size is no
longer in its quadratic regime.  These tests therefore use an epsilon 1e4
times larger; the exact check at the default epsilon is the dual-number
comparison with the oracle."""
import dataclasses

import numpy as np
import pytest

from paper_2009_14555_amd import problems as P
from tests.parity_util import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_14555_amd import solver

    return solver


VA_SMOOTH = 1e4


def plate_state(S, n=48, steps=12):
    """plate impact (van Albada, THINC/BVD) after a few steps: shocked fluid,
    yielding solid, mixed cells"""
    pb, W = P.plate_impact(n)
    pb = pb.replace(va_scale=tuple(x * VA_SMOOTH for x in pb.va_scale))
    g = S.Grid(pb)
    g.set_primitive(W)
    g.advance_cfl(steps)
    U = to_np(g.state).copy()
    dt = g.dt_cfl()
    return pb, g, U, dt


def directions(U, seed):
    """random perturbation v in the linear regime of every field (volume
    fraction relative to the minor phase, partial densities relative to
    themselves) and random weights w normalised per field"""
    rng = np.random.default_rng(seed)
    F = U.shape[0]
    big = np.abs(U).reshape(F, -1).max(axis=1)[:, None, None]
    scale = np.abs(U) + 1e-3 * big
    scale[0] = np.minimum(U[0], 1.0 - U[0])
    scale[1:3] = np.abs(U[1:3])
    v = rng.standard_normal(U.shape) * scale
    # weights: one over the field's size, at most one (a field that is zero
    # everywhere, such as a shear entry of a state at rest, keeps weight ~1
    # rather than amplifying round-off-sized Jacobian entries)
    w = rng.standard_normal(U.shape) / np.maximum(big, 1.0)
    return v, w


def fd_dot(fwd, U, v, w, eps):
    Sp = fwd(U + eps * v)
    Sm = fwd(U - eps * v)
    return float(np.sum(w * (Sp - Sm)) / (2 * eps))


def dot_check(lhs, rhs, tol, what):
    rel = abs(lhs - rhs) / max(abs(lhs), abs(rhs), 1e-300)
    print(f"{what}: fd {lhs:.12e} adjoint {rhs:.12e} rel {rel:.2e}", flush=True)
    assert rel <= tol, what


def run_sweep(g, U, dt, d):
    g.set_conserved(U)
    g.sweep(dt, d)
    return to_np(g.state).copy()


def run_plastic(g, U):
    g.set_conserved(U)
    g.sources(0.0)
    return to_np(g.state).copy()


def run_step(g, U, dt, k):
    g.set_conserved(U)
    g.set_step_index(k)
    g.advance(dt)
    return to_np(g.state).copy()


@pytest.fixture(scope="module")
def plate(S):
    return plate_state(S)


@pytest.mark.parametrize("d", [0, 1])
def test_sweep_adjoint_dot_product(S, plate, d):
    import torch

    pb, g, U, dt = plate
    v, w = directions(U, 10 + d)
    lhs = fd_dot(lambda X: run_sweep(g, X, dt, d), U, v, w, 1e-7)
    dp = torch.zeros(12, dtype=torch.float64, device="cuda")
    lam = to_np(g.adjoint_sweep(U, w, dt, d, dp))
    dot_check(lhs, float(np.sum(lam * v)), 1e-4, f"sweep {d}")


def test_plastic_adjoint_dot_product(S, plate):
    import torch

    pb, g, U0, dt = plate
    # after the sweeps of a step: the relaxed state of the last step sits on
    # the yield surface, where the relaxation has a kink
    U = run_sweep(g, run_sweep(g, U0, dt, 0), dt, 1)
    v, w = directions(U, 20)
    lhs = fd_dot(lambda X: run_plastic(g, X), U, v, w, 1e-7)
    dp = torch.zeros(12, dtype=torch.float64, device="cuda")
    lam = to_np(g.adjoint_plastic(U, w, dp))
    dot_check(lhs, float(np.sum(lam * v)), 1e-6, "plastic")


def test_smooth_periodic_sweeps(S):
    """a smooth periodic two-material field with THINC/BVD: both sweeps"""
    import torch

    n = (40, 36)
    pb = P.Problem(ndim=2, n=(n[0], n[1], 1), dx=(1 / n[0], 1 / n[1], 1), bc=(P.BC_PERIODIC,) * 3,
                   materials=[P.water_sg(), P.solid_c2()], thinc=1, limiter=P.LIM_VANALBADA)
    pb = pb.replace(va_scale=tuple(x * VA_SMOOTH for x in pb.va_scale))
    g = S.Grid(pb)
    g.set_primitive(P.random_smooth_state(pb, seed=6, solid_strain=3e-3))
    U = to_np(g.state).copy()
    dt = g.dt_cfl()
    for d in (0, 1):
        v, w = directions(U, 50 + d)
        lhs = fd_dot(lambda X: run_sweep(g, X, dt, d), U, v, w, 1e-8)
        dp = torch.zeros(12, dtype=torch.float64, device="cuda")
        lam = to_np(g.adjoint_sweep(U, w, dt, d, dp))
        dot_check(lhs, float(np.sum(lam * v)), 1e-4, f"smooth sweep {d}")


def test_transmissive_small_grids(S):
    """ghost folding at transmissive boundaries, grids down to one cell wide"""
    import torch

    for n in [(7, 5), (1, 9), (3, 1), (60, 2)]:
        pb, W = P.plate_impact(8)
        pb = pb.replace(n=(n[0], n[1], 1), dx=(1 / n[0], 1 / n[1], 1.0),
                        va_scale=tuple(x * VA_SMOOTH for x in pb.va_scale))
        rng = np.random.default_rng(sum(n))
        L = P.layout(pb)
        W = P.blank_prim(pb)
        W[L.phi(0)] = rng.uniform(0.2, 0.8, size=W[0].shape)
        W[L.rho(0)] = 1000.0 * (1 + 0.05 * rng.standard_normal(W[0].shape))
        W[L.rho(1)] = 2700.0 * (1 + 0.05 * rng.standard_normal(W[0].shape))
        W[L.u(0)] = 30.0 * rng.standard_normal(W[0].shape)
        W[L.u(1)] = 30.0 * rng.standard_normal(W[0].shape)
        W[L.p] = 1e8 * (1 + 0.1 * rng.standard_normal(W[0].shape))
        g = S.Grid(pb)
        g.set_primitive(W)
        U = to_np(g.state).copy()
        dt = 0.5 * g.dt_cfl()
        for d in (0, 1):
            v, w = directions(U, 60 + d)
            lhs = fd_dot(lambda X: run_sweep(g, X, dt, d), U, v, w, 1e-8)
            dp = torch.zeros(12, dtype=torch.float64, device="cuda")
            lam = to_np(g.adjoint_sweep(U, w, dt, d, dp))
            dot_check(lhs, float(np.sum(lam * v)), 1e-4, f"grid {n} sweep {d}")


@pytest.mark.parametrize("k", [0, 1])
def test_step_adjoint_dot_product_and_determinism(S, plate, k):
    import torch

    pb, g, U, dt = plate
    v, w = directions(U, 30 + k)
    lhs = fd_dot(lambda X: run_step(g, X, dt, k), U, v, w, 1e-7)
    dp = torch.zeros(12, dtype=torch.float64, device="cuda")
    lam = to_np(g.adjoint_step(U, w, dt, k, dp))
    dot_check(lhs, float(np.sum(lam * v)), 1e-4, f"step {k}")
    dp2 = torch.zeros(12, dtype=torch.float64, device="cuda")
    lam2 = to_np(g.adjoint_step(U, w, dt, k, dp2))
    assert np.array_equal(lam, lam2) and torch.equal(dp, dp2)


@pytest.mark.parametrize("k", [0, 1])
def test_kept_first_sweep_matches_recompute(S, plate, k):
    """after dimp_advance the other bound buffer is the step's first sweep
    (bitwise dimp_sweep of the state), and the adjoint step given it equals
    the one that recomputes it, bit for bit (adjoint and parameter sums)"""
    import torch

    pb, g, U, dt = plate
    d1 = 0 if k % 2 == 0 else 1
    g.set_conserved(U)
    g.sweep(dt, d1)
    U1_ref = g.state.clone()
    g.set_conserved(U)
    g.set_step_index(k)
    g.advance(dt)
    U1 = g.other.clone()
    torch.cuda.synchronize()
    assert torch.equal(U1, U1_ref)
    _, w = directions(U, 70 + k)
    dp = torch.zeros(12, dtype=torch.float64, device="cuda")
    lam = to_np(g.adjoint_step(U, w, dt, k, dp))
    dpk = torch.zeros(12, dtype=torch.float64, device="cuda")
    lamk = to_np(g.adjoint_step(U, w, dt, k, dpk, first_sweep=U1))
    assert np.array_equal(lam, lamk) and torch.equal(dp, dpk)


PARAMS = [(0, "gamma", 1), (0, "pinf", 1), (1, "G0", 2), (1, "yield_stress", 3)]


@pytest.mark.parametrize("mat,name,slot", PARAMS)
def test_parameter_adjoint(S, plate, mat, name, slot):
    import torch

    pb, g, U, dt = plate
    _, w = directions(U, 40)
    base = list(pb.materials)
    th = getattr(base[mat], name)
    h = 1e-6 * abs(th)

    def out(value):
        ms = list(base)
        ms[mat] = dataclasses.replace(base[mat], **{name: value})
        g.set_materials(ms)
        r = run_step(g, U, dt, 0)
        g.set_materials(base)
        return r

    lhs = float(np.sum(w * (out(th + h) - out(th - h))) / (2 * h))
    dp = torch.zeros(12, dtype=torch.float64, device="cuda")
    g.adjoint_step(U, w, dt, 0, dp)
    grad = g.adjoint_params(dp)
    col = {"gamma": 0, "pinf": 1, "G0": 2, "yield_stress": 3}[name]
    dot_check(lhs, float(grad[mat, col]), 1e-5, f"d/d{name}")


def dual_case(S, kind):
    if kind == "plate":
        pb, W = P.plate_impact(40)
        g = S.Grid(pb)
        g.set_primitive(W)
        g.advance_cfl(10)
    else:
        n = (40, 36)
        pb = P.Problem(ndim=2, n=(n[0], n[1], 1), dx=(1 / n[0], 1 / n[1], 1), bc=(P.BC_PERIODIC,) * 3,
                       materials=[P.water_sg(), P.solid_c2(yield_stress=0.05e9)], thinc=1,
                       limiter=P.LIM_VANALBADA)
        g = S.Grid(pb)
        g.set_primitive(P.random_smooth_state(pb, seed=6, solid_strain=3e-3))
    return pb, g


@pytest.mark.parametrize("kind,tol", [("smooth", 1e-7), ("plate", 1e-6)])
@pytest.mark.parametrize("k", [0, 1])
def test_adjoint_matches_oracle_dual_numbers(S, kind, tol, k):
    """exact check at the default van Albada epsilon: the oracle's dual-number
    tangent J v and parameter tangents against the GPU adjoint J^T w.  On a
    smooth periodic field (THINC/BVD, yielding solid) the parameter
    derivatives agree to round-off; the state direction also crosses faces
    where the normal velocity passes through zero (S* ~ 0), where the GPU
    (hardware reciprocals) and the oracle (IEEE division) may round to
    opposite Riemann branches, more so in the quiescent fluid ahead of a
    plate impact, hence the looser bars on that one number"""
    import torch

    from oracle import pyoracle as O

    pb, g = dual_case(S, kind)
    U = to_np(g.state).copy()
    dt = g.dt_cfl()
    v, w = directions(U, 70 + k)
    dpar = np.zeros((5, 2, 4))
    dpar[1, 0, 0] = dpar[2, 0, 1] = dpar[3, 1, 2] = dpar[4, 1, 3] = 1.0
    dU = np.zeros((5,) + U.shape)
    dU[0] = v
    _, T = O.Oracle(pb).step_dual(U, dU, dpar, dt, k)
    dp = torch.zeros(12, dtype=torch.float64, device="cuda")
    lam = to_np(g.adjoint_step(U, w, dt, k, dp))
    grad = g.adjoint_params(dp)
    pairs = [(float(np.sum(w * T[0])), float(np.sum(lam * v)), "state")]
    for j, (mat, col, name) in enumerate([(0, 0, "gamma"), (0, 1, "pinf"), (1, 2, "G0"), (1, 3, "yield")]):
        pairs.append((float(np.sum(w * T[1 + j])), float(grad[mat, col]), name))
    for lhs, rhs, name in pairs:
        rel = abs(lhs - rhs) / max(abs(lhs), abs(rhs), 1e-300)
        print(f"{kind} step {k} {name}: dual {lhs:.12e} adjoint {rhs:.12e} rel {rel:.2e}", flush=True)
        assert rel <= (tol if name == "state" else 1e-9), name
