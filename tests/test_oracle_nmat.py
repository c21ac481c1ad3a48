"""Three materials in the oracle (the model of Sec. 2 takes any number of
solids and fluids): pins independent of the oracle's own three-material
arithmetic.

* Splitting a material in two: a three-material problem whose materials 1 and
  2 are copies of one material, holding fixed shares alpha and 1 - alpha of
  its volume fraction at equal phase densities, is the two-material problem
  with that material; every mixture rule (pressure, sound speeds, shear
  modulus, plastic weights), every minmod-limited slope and every flux is
  linear in the volume fractions and partial densities of the copies, so the
  step of the split problem equals the step of the merged one to round-off
  (THINC off: its profile is not linear in the fraction).
* Relabelling: exchanging the roles of two materials (their stored slots
  and their parameters) exchanges the results, the THINC normal being taken
  from a fraction that the exchange leaves in place."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P


def merged_problem(ndim=2, n=(40, 30), thinc=0, periodic=False):
    nn = tuple(list(n) + [1] * (3 - len(n)))
    bc = (P.BC_PERIODIC if periodic else P.BC_TRANSMISSIVE,) * 3
    pb = P.Problem(ndim=ndim, n=nn, dx=tuple([1.0 / max(n)] * 3), bc=bc,
                   materials=[P.water_sg(), P.solid_c2()], thinc=thinc, cfl=0.5)
    W = P.random_smooth_state(pb, seed=11, solid_strain=2e-3)
    return pb, W


def split_state(pb2, W2, alpha, mats3):
    """the three-material problem and state with material 1 of pb2 split into
    slots 1 and 2 (fractions alpha phi_1 and (1 - alpha) phi_1)"""
    import dataclasses

    pb3 = dataclasses.replace(pb2, materials=mats3)
    L2, L3 = P.layout(pb2), P.layout(pb3)
    W3 = np.zeros((L3.nfields,) + pb2.shape)
    phi_a = W2[L2.phi(0)]
    W3[L3.phi(0)] = phi_a
    W3[L3.phi(1)] = alpha * (1.0 - phi_a)
    W3[L3.rho(0)] = W2[L2.rho(0)]
    W3[L3.rho(1)] = W2[L2.rho(1)]
    W3[L3.rho(2)] = W2[L2.rho(1)]
    for d in range(pb2.ndim):
        W3[L3.u(d)] = W2[L2.u(d)]
    W3[L3.p] = W2[L2.p]
    for q in range(len(P.vbar_components(pb2.ndim))):
        W3[L3.V(q)] = W2[L2.V(q)]
    return pb3, W3


def merge(pb3, U3, pb2):
    """the two-material conserved state of a split one: fractions and partial
    densities of slots 1 and 2 summed"""
    L2, L3 = P.layout(pb2), P.layout(pb3)
    U2 = np.zeros((L2.nfields,) + U3.shape[1:])
    U2[L2.phi(0)] = U3[L3.phi(0)]
    U2[L2.rho(0)] = U3[L3.rho(0)]  # partial densities in conserved form
    U2[L2.rho(1)] = U3[L3.rho(1)] + U3[L3.rho(2)]
    for d in range(pb2.ndim):
        U2[L2.u(d)] = U3[L3.u(d)]
    U2[L2.p] = U3[L3.p]
    for q in range(len(P.vbar_components(pb2.ndim))):
        U2[L2.V(q)] = U3[L3.V(q)]
    return U2


def field_scale_diff(a, b):
    s = np.maximum(np.abs(b).reshape(b.shape[0], -1).max(axis=1), 1e-300)
    return np.abs(a - b).reshape(a.shape[0], -1).max(axis=1) / s


@pytest.mark.parametrize("ndim,n", [(1, (120,)), (2, (40, 30))])
@pytest.mark.parametrize("integrator", ["split", "rk3"])
def test_splitting_a_material_in_two_is_the_merged_problem(ndim, n, integrator):
    pb2, W2 = merged_problem(ndim, n)
    pb3, W3 = split_state(pb2, W2, 0.3, [P.water_sg(), P.solid_c2(), P.solid_c2()])
    o2, o3 = O.Oracle(pb2), O.Oracle(pb3)
    U2, U3 = o2.prim_to_cons(W2), o3.prim_to_cons(W3)
    np.testing.assert_allclose(o3.dt_cfl(U3), o2.dt_cfl(U2), rtol=1e-13)
    for k in range(6):
        dt = o2.dt_cfl(U2)
        U2 = o2.step_rk3(U2, dt) if integrator == "rk3" else o2.step(U2, dt, k)
        U3 = o3.step_rk3(U3, dt) if integrator == "rk3" else o3.step(U3, dt, k)
    d = field_scale_diff(merge(pb3, U3, pb2), U2)
    assert np.all(d < 1e-12), d
    # the copies keep their shares: slot 1 holds alpha of the merged fraction
    L3 = P.layout(pb3)
    phi1 = U3[L3.phi(1)]
    phi12 = 1.0 - U3[L3.phi(0)]
    assert np.max(np.abs(phi1 - 0.3 * phi12)) < 1e-12


def test_relabelling_two_materials_exchanges_the_results():
    """three distinct materials; slots 1 and 2 exchanged (THINC on: its normal
    comes from slot 0, which the exchange leaves in place)"""
    import dataclasses

    pb2, W2 = merged_problem(2, (36, 28), thinc=1)
    mats = [P.water_sg(), P.solid_c2(), P.air(1.4)]
    pb, W = split_state(pb2, W2, 0.4, mats)
    L = P.layout(pb)
    x, y = P.cell_centres(pb)
    W[L.rho(2)] = 1.2 + 0.1 * np.cos(3 * x)  # the air is much lighter
    pbx = dataclasses.replace(pb, materials=[mats[0], mats[2], mats[1]])
    Wx = W.copy()
    phi2 = 1.0 - W[L.phi(0)] - W[L.phi(1)]
    Wx[L.phi(1)] = phi2
    Wx[L.rho(1)], Wx[L.rho(2)] = W[L.rho(2)], W[L.rho(1)]
    o, ox = O.Oracle(pb), O.Oracle(pbx)
    U, Ux = o.prim_to_cons(W), ox.prim_to_cons(Wx)
    for k in range(5):
        dt = o.dt_cfl(U)
        U = o.step(U, dt, k)
        Ux = ox.step(Ux, dt, k)
    swap = Ux.copy()
    swap[L.phi(1)] = 1.0 - Ux[L.phi(0)] - Ux[L.phi(1)]
    swap[L.rho(1)], swap[L.rho(2)] = Ux[L.rho(2)], Ux[L.rho(1)]
    d = field_scale_diff(swap, U)
    assert np.all(d < 1e-12), d


@pytest.mark.parametrize("rk3", [False, True])
def test_splitting_a_material_in_two_under_refinement(rk3):
    """two-level refinement (one patch, subcycled, refluxed) of the split
    three-material problem is the refined merged problem to round-off on both
    levels; on the periodic domain the three-material composite grid conserves
    every partial mass, the momentum and the energy to round-off"""
    from oracle import amr as A
    from tests.test_oracle_amr import prolong_prim

    pb2, W2 = merged_problem(2, (40, 30), periodic=True)
    box = (10, 8, 22, 18)
    mats3 = [P.water_sg(), P.solid_c2(), P.solid_c2()]
    pb3, W3 = split_state(pb2, W2, 0.3, mats3)
    runs = []
    for pbc, Wc in ((pb2, W2), (pb3, W3)):
        pbf = A.fine_problem(pbc, box)
        Wf, _ = prolong_prim(pbc, Wc, pbf, box)
        oc, of = O.Oracle(pbc), O.Oracle(pbf)
        runs.append([pbc, pbf, oc, of, oc.prim_to_cons(Wc), of.prim_to_cons(Wf)])
    L3 = P.layout(pb3)
    cons = list(range(pb3.nmat - 1, L3.V(0)))
    area = pb3.dx[0] * pb3.dx[1]

    def totals(Uc, Uf):
        i0, j0, i1, j1 = box
        out = Uc[cons].sum(axis=(1, 2)) * area - Uc[cons, j0:j1, i0:i1].sum(axis=(1, 2)) * area
        return out + Uf[cons][:, A.interior_mask(box)].sum(axis=1) * (area / 4)

    m0 = totals(runs[1][4], runs[1][5])
    for k in range(4):
        dtk, runs[0][5] = A.dt(runs[0][2], runs[0][3], runs[0][4], runs[0][5], box)
        for r in runs:
            r[4], r[5] = A.step(r[2], r[3], r[4], r[5], box, dtk, k, rk3)
    assert np.all(field_scale_diff(merge(pb3, runs[1][4], pb2), runs[0][4]) < 1e-12)
    assert np.all(field_scale_diff(merge(runs[1][1], runs[1][5], runs[0][1]), runs[0][5]) < 1e-12)
    drift = np.abs(totals(runs[1][4], runs[1][5]) - m0) / np.maximum(np.abs(m0), 1e-3)
    assert np.all(drift < 1e-13), drift
