"""Pins of the oracle's reflective boundaries and the cylindrical geometric
source (Sec. 3, s_g with x = r, y = z):

* a reflective wall is the mirror plane of a symmetric problem: the half
  domain with the wall reproduces the full domain's half bit for bit (1-D
  two-gas slab, 2-D disc cut by the axis with THINC on);
* homologous cylindrical expansion u_r = a r / (1 + a t), rho = rho0 / (1 +
  a t)^2, uniform p (and, for an elastic solid, Vbar = diag((1+at)^(1/3),
  (1+at)^(-2/3), (1+at)^(1/3)) in (r, z, theta)) is an exact solution: the
  step converges to it at first order in dt (the paper's fractional steps),
  which a dropped term, a wrong sign or a wrong theta-row coefficient of s_g
  would break;
* a state at rest with isotropic stress is left exactly unchanged on the
  axis grid.
CPU only."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P


def slab_1d(n, lo, hi, bc):
    pb = P.Problem(ndim=1, n=(n, 1, 1), dx=((hi - lo) / n, 1.0, 1.0), lo=(lo, 0.0, 0.0), bc=(bc, 0, 0),
                   materials=[P.air(1.4), P.air(1.67)], thinc=1, cfl=0.5)
    L = P.layout(pb)
    W = P.blank_prim(pb)
    (x,) = P.cell_centres(pb)
    inside = np.abs(x) < 0.3
    W[L.phi(0)] = np.where(inside, 1 - 1e-6, 1e-6)
    W[L.rho(0)] = 1.0 + 0.2 * np.cos(3 * x)
    W[L.rho(1)] = 0.3 + 0.1 * np.cos(5 * x)
    W[L.u(0)] = -0.8 * np.sin(4 * x)  # odd: flows into the plane x = 0 from both sides
    W[L.p] = 1.0 + 0.3 * np.cos(2 * x)
    return pb, W


def run(pb, W, nsteps, dt=None):
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    dt = 0.4 * pb.dx[0] / 3.0 if dt is None else dt
    for k in range(nsteps):
        U = o.step(U, dt, k)
    return U


def mirrored(pb_half, W_half, pb_full, axis):
    """the full-domain state built as the exact mirror image of the half
    domain's (so the start is symmetric bit for bit)"""
    L = P.layout(pb_half)
    ax = W_half.ndim - 1 - axis  # numpy axis of dimension `axis`
    Wm = np.flip(W_half, axis=ax).copy()
    Wm[L.u(axis)] *= -1
    for q, (i, j) in enumerate(P.vbar_components(pb_half.ndim)):
        if (i == axis) != (j == axis):
            Wm[L.V(q)] *= -1
    return np.concatenate([Wm, W_half], axis=ax)


def test_reflective_wall_is_the_mirror_plane_1d():
    m = 40
    pbh, Wh = slab_1d(m, 0.0, 1.0, P.BC_AXIS)
    pbf, _ = slab_1d(2 * m, -1.0, 1.0, P.BC_TRANSMISSIVE)
    full = run(pbf, mirrored(pbh, Wh, pbf, 0), 12)
    half = run(pbh, Wh, 12)
    np.testing.assert_array_equal(half, full[:, m:])
    # a wall at the far end too: the cells beyond the numerical domain of
    # dependence of that end (3 cells per step) are unchanged
    both = run(*slab_1d(2 * m, 0.0, 2.0, P.BC_REFLECTIVE), 12)
    one = run(*slab_1d(2 * m, 0.0, 2.0, P.BC_AXIS), 12)
    np.testing.assert_array_equal(both[:, :2 * m - 40], one[:, :2 * m - 40])
    assert not np.array_equal(both[:, -4:], one[:, -4:])


def disc_2d(nx, ny, xlo, bc):
    pb = P.Problem(ndim=2, n=(nx, ny, 1), dx=(1.0 / 32, 1.0 / 32, 1.0), lo=(xlo, 0.0, 0.0),
                   bc=(bc, P.BC_TRANSMISSIVE, 0), materials=[P.water_sg(), P.solid_c2()], thinc=1, cfl=0.5)
    L = P.layout(pb)
    W = P.blank_prim(pb)
    x, y = P.cell_centres(pb)
    f = P.disc_fraction(x, y, 0.0, 0.5, 0.25, pb.dx[0], pb.dx[1])
    W[L.phi(0)] = np.clip(1 - f, 1e-6, 1 - 1e-6)
    W[L.rho(0)] = 1000.0 * (1 + 0.01 * np.cos(7 * x) * np.sin(5 * y))
    W[L.rho(1)] = 2700.0
    W[L.u(0)] = -60.0 * np.sin(3 * x)
    W[L.u(1)] = 40.0 * np.cos(2 * x) * np.sin(4 * y)
    W[L.p] = 1e8 * (1 + 0.2 * np.cos(3 * x))
    for q, (i, j) in enumerate(P.vbar_components(2)):
        sgn = -1.0 if (i == 0) != (j == 0) else 1.0
        W[L.V(q)] = (1.0 if i == j else 0.0) + 1e-3 * (np.sin(2 * x) if sgn < 0 else np.cos(2 * x))
    return pb, W


def test_reflective_axis_is_the_mirror_plane_2d():
    pbh, Wh = disc_2d(24, 32, 0.0, P.BC_AXIS)
    pbf, _ = disc_2d(48, 32, -0.75, P.BC_TRANSMISSIVE)
    o = O.Oracle(pbh)
    dt = 0.5 * o.dt_cfl(o.prim_to_cons(Wh))
    full = run(pbf, mirrored(pbh, Wh, pbf, 0), 6, dt)
    half = run(pbh, Wh, 6, dt)
    assert np.all(np.isfinite(half))
    np.testing.assert_array_equal(half, full[:, :, 24:])


def ball_3d(nx, ny, nz, xlo, bcs):
    """a solid ball of radius 0.25 centred at (0, 0.5, 0.5) in water, flows
    odd in x (into the plane x = 0 from both sides), mixed-sign shear of the
    stretch tensor; x in [xlo, xlo + nx/16]"""
    pb = P.Problem(ndim=3, n=(nx, ny, nz), dx=(1.0 / 16,) * 3, lo=(xlo, 0.0, 0.0), bc=bcs,
                   materials=[P.water_sg(), P.solid_c2()], thinc=1, cfl=0.5)
    L = P.layout(pb)
    W = P.blank_prim(pb)
    x, y, z = P.cell_centres(pb)
    r2 = x ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    f = np.clip((0.25 - np.sqrt(r2)) / pb.dx[0] + 0.5, 0.0, 1.0)
    W[L.phi(0)] = np.clip(1 - f, 1e-6, 1 - 1e-6)
    W[L.rho(0)] = 1000.0 * (1 + 0.01 * np.cos(7 * x) * np.sin(5 * y) * np.cos(3 * z))
    W[L.rho(1)] = 2700.0 * (1 + 0.002 * np.cos(4 * x))
    W[L.u(0)] = -60.0 * np.sin(3 * x)
    W[L.u(1)] = 40.0 * np.cos(2 * x) * np.sin(4 * y)
    W[L.u(2)] = 30.0 * np.cos(3 * x) * np.cos(2 * z)
    W[L.p] = 1e8 * (1 + 0.2 * np.cos(3 * x) + 0.05 * np.sin(6 * z))
    for q, (i, j) in enumerate(P.vbar_components(3)):
        odd = (i == 0) != (j == 0)
        W[L.V(q)] = (1.0 if i == j else 0.0) + 1e-3 * (np.sin(2 * x) if odd else np.cos(2 * x + i - j))
    return pb, W


def test_reflective_wall_is_the_mirror_plane_3d():
    """the 3-D sweeps with a wall at x = 0 reproduce the mirror-symmetric
    problem on the doubled domain bit for bit (walls at y and z both ends)"""
    bc_half = (P.BC_AXIS, P.BC_REFLECTIVE, P.BC_REFLECTIVE)
    bc_full = (P.BC_TRANSMISSIVE, P.BC_REFLECTIVE, P.BC_REFLECTIVE)
    pbh, Wh = ball_3d(8, 12, 10, 0.0, bc_half)
    pbf, _ = ball_3d(16, 12, 10, -0.5, bc_full)
    o = O.Oracle(pbh)
    dt = 0.5 * o.dt_cfl(o.prim_to_cons(Wh))
    full = run(pbf, mirrored(pbh, Wh, pbf, 0), 4, dt)
    half = run(pbh, Wh, 4, dt)
    assert np.all(np.isfinite(half))
    np.testing.assert_array_equal(half, full[:, :, :, 8:])


def homologous(n, a, solid=False, T=None):
    """cylindrical grid r in [0, 1] (axis), z periodic (4 cells); uniform
    density and pressure, u_r = a r"""
    if solid:
        mats = [P.water_sg(), dataclasses.replace(P.solid_c2(), plast=P.PLAST_NONE)]
    else:
        mats = [P.air(1.4), P.air(1.4)]
    pb = P.Problem(ndim=2, n=(n, 4, 1), dx=(1.0 / n, 1.0 / n, 1.0), bc=(P.BC_AXIS, P.BC_PERIODIC, 0),
                   materials=mats, thinc=0, cfl=0.5, geom=P.GEOM_CYLINDRICAL)
    L = P.layout(pb)
    W = P.blank_prim(pb)
    r, z = P.cell_centres(pb)
    W[L.phi(0)] = 1e-6 if solid else 0.5
    W[L.rho(0)] = 1000.0 if solid else 1.0
    W[L.rho(1)] = 2700.0 if solid else 1.0
    W[L.u(0)] = a * r
    W[L.p] = 1e8 if solid else 1.0
    return pb, W, r


def homologous_errors(n, solid):
    a = 1000.0 if solid else 0.5
    T = 1e-4 if solid else 0.2
    pb, W, r = homologous(n, a, solid)
    o = O.Oracle(pb)
    L = P.layout(pb)
    U = o.prim_to_cons(W)
    # a fixed dt per resolution (half the CFL step of the start)
    nsteps = int(math.ceil(T / (0.5 * o.dt_cfl(U))))
    dt = T / nsteps
    for k in range(nsteps):
        U = o.step(U, dt, k)
    Wf = o.cons_to_prim(U)
    g = 1 + a * T
    keep = r < 0.3  # the outer boundary's disturbance has not arrived
    rho = U[L.m(0)] + U[L.m(1)]
    rho0 = (1e-6 * 1000.0 + (1 - 1e-6) * 2700.0) if solid else 1.0
    e = {"rho": np.max(np.abs(rho[keep] - rho0 / g ** 2)) / (rho0 / g ** 2),
         "u": np.max(np.abs(Wf[L.u(0)][keep] - a * r[keep] / g)) / (a * 0.3)}
    if solid:
        V = {(i, j): Wf[L.V(q)][keep] for q, (i, j) in enumerate(P.vbar_components(2))}
        e["Vrr"] = np.max(np.abs(V[(0, 0)] - g ** (1 / 3)))
        e["Vzz"] = np.max(np.abs(V[(1, 1)] - g ** (-2 / 3)))
        e["Vtt"] = np.max(np.abs(V[(2, 2)] - g ** (1 / 3)))
        e["Vtt-Vrr"] = np.max(np.abs(V[(2, 2)] - V[(0, 0)]))
    else:
        e["p"] = np.max(np.abs(Wf[L.p][keep] - g ** (-2 * 1.4))) * g ** (2 * 1.4)
    return e


def test_homologous_expansion_of_a_gas_first_order():
    errs = [homologous_errors(n, False) for n in (25, 50, 100)]
    for k in errs[0]:
        e = np.array([x[k] for x in errs])
        order = np.log2(e[:-1] / e[1:])
        # first order in dt (Godunov fractional steps), small in absolute terms
        assert np.all(order > 0.7) and e[-1] < 2e-3, (k, e, order)


def test_homologous_expansion_of_an_elastic_solid():
    """density and velocity converge at first order; the stretch tensor
    follows diag(g^(1/3), g^(-2/3), g^(1/3)) up to the per-step rebuild of
    Vbar from its approximate Hencky strain in the plastic step (an O(J^3)
    change per step whatever dt is: ~3e-5 here, accumulating with the step
    count), with V_tt = V_rr to round-off: a wrong theta-row coefficient of
    the source (or none) would part them by ~0.03-0.1"""
    errs = [homologous_errors(n, True) for n in (25, 50, 100)]
    for k in ("rho", "u"):
        e = np.array([x[k] for x in errs])
        order = np.log2(e[:-1] / e[1:])
        assert np.all(order > 0.5) and e[-1] < 2e-3, (k, e, order)
    for x in errs:
        assert x["Vrr"] < 0.012 and x["Vzz"] < 0.02 and x["Vtt"] < 0.012, x
    d = np.array([x["Vtt-Vrr"] for x in errs])
    assert d[0] < 1e-3 and np.all(np.log2(d[:-1] / d[1:]) > 0.7), d


def test_rest_state_is_exactly_kept_on_the_axis_grid():
    pb, W, r = homologous(20, 0.0, solid=True)
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    U2 = U
    for k in range(4):
        U2 = o.step(U2, 1e-6, k)
    np.testing.assert_array_equal(U2, U)


def test_geometric_step_alone_matches_the_ode():
    """one cell's geometric step is Heun's method on dq/dt = s_g(q): for a
    gas at rest with uniform pressure nothing moves; with u_r the mass obeys
    d(m)/dt = -m u_r / r, which Heun follows to O(dt^3) per step"""
    pb, W, r = homologous(8, 0.5)
    o = O.Oracle(pb)
    L = P.layout(pb)
    U = o.prim_to_cons(W)
    dt = 1e-3
    U1 = o.geometric(U, dt)
    # the momentum equation's pressure terms cancel (sig_rr = sig_tt = -p):
    # d(m)/dt = -m u/r, d(m u)/dt = -(m u) u / r, u = a r: m' = -a m, (m u)' = -a (m u) at t = 0
    m0 = U[L.m(0)]
    assert np.allclose(U1[L.m(0)], m0 * (1 - 0.5 * dt + 0.125 * dt ** 2), rtol=1e-9)
    assert np.all(U1[L.phi(0)] == U[L.phi(0)])
