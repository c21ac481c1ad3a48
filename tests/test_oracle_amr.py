"""Pins of the oracle's two-level subcycled refinement (oracle/amr.py, Sec.
3 with the readings listed there): the ghost fill takes each fine ghost
cell's coarse parent (brute-force index check) at the right time weight;
averaging down is the mean of the four children (a piecewise-constant and a
linear field); a uniform state stays exactly uniform; before a shock reaches
the patch the coarse level is the coarse-only run bit for bit; a smooth wave
crossing the patch is more accurate inside it than the coarse-only run and
no worse outside.  CPU only."""
import math

import numpy as np
import pytest

from oracle import amr as A
from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P


def two_gas(nx, ny, L=1.0):
    return P.Problem(ndim=2, n=(nx, ny, 1), dx=(L / nx, L / ny, 1.0), bc=(P.BC_PERIODIC,) * 3,
                     materials=[P.air(1.4), P.air(1.67)], thinc=0, limiter=P.LIM_VANALBADA, cfl=0.4)


def test_fill_interpolates_inside_the_parents():
    """ghost cells: a linear coarse field (in x and y, and in time) is
    reproduced exactly at the fine centres; a field with a kink is limited
    (no value outside the parent's neighbours); the interior is untouched"""
    box = (4, 3, 8, 6)
    ny, nx = A.fine_shape(box)
    Jc, Ic = np.meshgrid(np.arange(12) + 0.5, np.arange(14) + 0.5, indexing="ij")
    Uc0 = (2.0 * Ic - 3.0 * Jc)[None]
    Uc1 = (4.0 * Ic + 1.0 * Jc)[None]
    rng = np.random.default_rng(0)
    Uf = rng.standard_normal((1, ny, nx))
    for w in (0.0, 0.5):
        out = A.fill(Uc0, Uc1, w, Uf, box)
        for fj in range(ny):
            for fi in range(nx):
                inside = A.G <= fi < nx - A.G and A.G <= fj < ny - A.G
                if inside:
                    assert out[0, fj, fi] == Uf[0, fj, fi]
                else:
                    x = box[0] + (fi - A.G + 0.5) / 2  # fine centre in coarse units
                    y = box[1] + (fj - A.G + 0.5) / 2
                    want = (1 - w) * (2.0 * x - 3.0 * y) + w * (4.0 * x + y)
                    assert abs(out[0, fj, fi] - want) < 1e-12, (fi, fj, w)
    kink = np.abs(Ic - 6.0)[None]  # kink between coarse cells 5 and 6
    out = A.fill(kink, kink, 0.0, Uf, box)
    J, I = A.parents(box)
    ghost = ~A.interior_mask(box)
    lo = np.minimum(np.minimum(kink[0][J, I - 1], kink[0][J, I + 1]), kink[0][J, I])
    hi = np.maximum(np.maximum(kink[0][J, I - 1], kink[0][J, I + 1]), kink[0][J, I])
    assert np.all(out[0][ghost] >= lo[ghost] - 1e-15) and np.all(out[0][ghost] <= hi[ghost] + 1e-15)


def test_average_down_is_the_mean_of_the_children():
    box = (2, 1, 6, 4)
    ny, nx = A.fine_shape(box)
    rng = np.random.default_rng(1)
    Uc = rng.standard_normal((3, 6, 9))
    # piecewise-constant prolongation of Uc into the patch interior
    Uf = np.zeros((3, ny, nx))
    for J in range(box[1], box[3]):
        for I in range(box[0], box[2]):
            fj, fi = A.G + 2 * (J - box[1]), A.G + 2 * (I - box[0])
            Uf[:, fj:fj + 2, fi:fi + 2] = Uc[:, J, I][:, None, None]
    out = A.average_down(np.zeros_like(Uc), Uf, box)
    np.testing.assert_array_equal(out[:, box[1]:box[3], box[0]:box[2]], Uc[:, box[1]:box[3], box[0]:box[2]])
    assert np.all(out[:, :box[1]] == 0) and np.all(out[:, :, :box[0]] == 0)
    # a linear field: the children's mean is the value at the coarse centre
    fx = (np.arange(nx) - A.G + 0.5) / 2
    fy = (np.arange(ny) - A.G + 0.5) / 2
    Uf2 = np.broadcast_to(3.0 * fx[None, :] - 2.0 * fy[:, None], (ny, nx))[None].copy()
    out2 = A.average_down(np.zeros((1, 6, 9)), Uf2, box)
    cx = np.arange(box[2] - box[0]) + 0.5
    cy = np.arange(box[3] - box[1]) + 0.5
    np.testing.assert_allclose(out2[0, box[1]:box[3], box[0]:box[2]], 3.0 * cx[None, :] - 2.0 * cy[:, None],
                               atol=1e-14)


def shock_setup(n=48):
    pbc, W = P.shock_disc(n, seed=1, noise=0.0)
    box = (38, 10, 44, 22)  # right of the disc, the ghost stencil in the uniform water at rest
    pbf = A.fine_problem(pbc, box)
    Wf, _ = prolong_prim(pbc, W, pbf, box)
    return pbc, W, pbf, Wf, box


def prolong_prim(pbc, Wc, pbf, box):
    """fine primitive state: each fine cell takes its coarse parent's (the
    patch's initial data)"""
    J, I = A.parents(box)
    J = np.clip(J, 0, pbc.n[1] - 1)
    I = np.clip(I, 0, pbc.n[0] - 1)
    return Wc[:, J, I].copy(), (J, I)


def run_amr(pbc, Wc, pbf, Wf, box, nsteps):
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    Uc, Uf = oc.prim_to_cons(Wc), of.prim_to_cons(Wf)
    for k in range(nsteps):
        dtk, Uf = A.dt(oc, of, Uc, Uf, box)
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dtk, k)
    return Uc, Uf


def test_uniform_state_stays_uniform():
    pbc = two_gas(24, 20)
    L = P.layout(pbc)
    W = P.blank_prim(pbc)
    W[L.phi(0)] = 0.3
    W[L.rho(0)] = 1.0
    W[L.rho(1)] = 0.5
    W[L.u(0)] = 0.7
    W[L.u(1)] = -0.2
    W[L.p] = 1.0
    box = (6, 5, 14, 13)
    pbf = A.fine_problem(pbc, box)
    Wf, _ = prolong_prim(pbc, W, pbf, box)
    Uc, Uf = run_amr(pbc, W, pbf, Wf, box, 5)
    U0 = O.Oracle(pbc).prim_to_cons(W)
    for f in range(L.nfields):
        assert np.all(Uc[f] == U0[f, 0, 0]), f


def test_coarse_level_untouched_before_the_shock_arrives():
    pbc, W, pbf, Wf, box = shock_setup()
    oc = O.Oracle(pbc)
    Uc, Uf = run_amr(pbc, W, pbf, Wf, box, 3)
    # the same steps on the coarse grid alone (same dt: the patch is at rest)
    U = oc.prim_to_cons(W)
    for k in range(3):
        U = oc.step(U, oc.dt_cfl(U), k)
    np.testing.assert_array_equal(Uc, U)


def wave_setup(nc, box):
    pbc = two_gas(nc, 16)
    L = P.layout(pbc)
    W = P.blank_prim(pbc)
    x, y = P.cell_centres(pbc)
    W[L.phi(0)] = 0.5
    W[L.rho(0)] = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    W[L.rho(1)] = 1.0
    W[L.u(0)] = 1.0
    W[L.p] = 1.0
    pbf = A.fine_problem(pbc, box)
    Lf = P.layout(pbf)
    Wf = P.blank_prim(pbf)
    xf, yf = P.cell_centres(pbf)
    Wf[Lf.phi(0)] = 0.5
    Wf[Lf.rho(0)] = 1.0 + 0.2 * np.sin(2 * np.pi * xf)
    Wf[Lf.rho(1)] = 1.0
    Wf[Lf.u(0)] = 1.0
    Wf[Lf.p] = 1.0
    return pbc, W, pbf, Wf


def test_smooth_wave_through_the_patch():
    """a density wave of material 0 carried at u = 1 through a patch over
    x in [0.25, 0.75): after t = 0.25 the refined cells are closer to the
    exact translation than the coarse-only run, and the rest is no worse
    (within 10%)"""
    nc = 32
    box = (8, 5, 24, 11)
    pbc, W, pbf, Wf = wave_setup(nc, box)
    L = P.layout(pbc)
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    Uc, Uf = oc.prim_to_cons(W), of.prim_to_cons(Wf)
    U = oc.prim_to_cons(W)
    T, t, k = 0.25, 0.0, 0
    while t < T - 1e-14:
        dtk, Uf = A.dt(oc, of, Uc, Uf, box)
        dtk = min(dtk, T - t)
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dtk, k)
        U = oc.step(U, dtk, k)
        t += dtk
        k += 1
    x, y = P.cell_centres(pbc)
    exact = 1.0 + 0.2 * np.sin(2 * np.pi * (x - T))
    rho_amr = oc.cons_to_prim(Uc)[L.rho(0)]
    rho_c = oc.cons_to_prim(U)[L.rho(0)]
    covered = np.zeros_like(x, dtype=bool)
    covered[box[1]:box[3], box[0]:box[2]] = True
    e_amr_in = np.mean(np.abs(rho_amr - exact)[covered])
    e_c_in = np.mean(np.abs(rho_c - exact)[covered])
    e_amr_out = np.mean(np.abs(rho_amr - exact)[~covered])
    e_c_out = np.mean(np.abs(rho_c - exact)[~covered])
    assert e_amr_in < 0.6 * e_c_in, (e_amr_in, e_c_in)
    assert e_amr_out < 1.1 * e_c_out, (e_amr_out, e_c_out)


def tag_brute(pb, W, th):
    """the criterion cell by cell, neighbour by neighbour"""
    L = P.layout(pb)
    N = pb.nmat
    ny, nx = W.shape[1:]
    sc = pb.va_scale

    def variables(j, i):
        phis = [W[L.phi(l), j, i] for l in range(N - 1)]
        last = 1.0
        s = 0.0
        for p_ in phis:
            s += p_
        last = 1.0 - s
        allp = phis + [last]
        out = [(p_, 1e-6 * sc[0]) for p_ in phis]
        out += [(allp[l] * W[L.rho(l), j, i], 1e-6 * sc[1]) for l in range(N)]
        out += [(W[L.u(d), j, i], 1e-6 * sc[3]) for d in range(2)]
        out += [(W[L.p, j, i], 1e-6 * sc[4])]
        return out

    tags = np.zeros((ny, nx), dtype=bool)
    for j in range(ny):
        for i in range(nx):
            for dj, di in ((0, -1), (0, 1), (-1, 0), (1, 0)):
                jn, in_ = j + dj, i + di
                if not (0 <= jn < ny and 0 <= in_ < nx):
                    continue
                for (a, fl), (b, _) in zip(variables(j, i), variables(jn, in_)):
                    if abs(b - a) > th * max(abs(a), abs(b), fl):
                        tags[j, i] = True
    return tags


def test_tag_criterion_against_brute_force():
    pb, W = P.shock_disc(24, seed=3)
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    for k in range(3):
        U = o.step(U, o.dt_cfl(U), k)
    Wp = o.cons_to_prim(U)
    for th in (0.01, 0.1, 0.3):
        tags, bbox = A.tag(pb, Wp, th)
        np.testing.assert_array_equal(tags, tag_brute(pb, Wp, th))
        jj, ii = np.nonzero(tags)
        assert bbox == (ii.min(), jj.min(), ii.max() + 1, jj.max() + 1)


def test_tag_uniform_and_single_cell():
    pbc = two_gas(12, 10).replace(va_scale=(1.0,) * 6)  # floors 1e-6 for an O(1) problem
    L = P.layout(pbc)
    W = P.blank_prim(pbc)
    W[L.phi(0)] = 0.4
    W[L.rho(0)] = 1.0
    W[L.rho(1)] = 2.0
    W[L.u(0)] = 1e-9  # velocities at round-off level fall under the floor
    W[L.p] = 1.0
    tags, bbox = A.tag(pbc, W, 0.05)
    assert not tags.any() and bbox == (0, 0, 0, 0)
    W[L.p, 4, 7] = 1.2
    tags, bbox = A.tag(pbc, W, 0.05)
    want = np.zeros_like(tags)
    for j, i in ((4, 7), (4, 6), (4, 8), (3, 7), (5, 7)):
        want[j, i] = True
    np.testing.assert_array_equal(tags, want)
    assert bbox == (6, 3, 9, 6)
    assert A.regrid_box(bbox, 2, pbc.n) == (4, 3, 9, 7)
    assert A.regrid_box((0, 0, 0, 0), 2, pbc.n) is None


def pulse_setup(nc=32, box=(10, 5, 20, 11)):
    """a two-gas periodic state with a material interface and a pressure
    pulse moving through the patch (density, momentum and energy all cross
    the coarse/fine faces)"""
    pbc = two_gas(nc, 16)
    L = P.layout(pbc)
    x, y = P.cell_centres(pbc)
    W = P.blank_prim(pbc)
    W[L.phi(0)] = np.where(np.abs(x - 0.4) < 0.15, 0.9, 0.1)
    W[L.rho(0)] = 1.0 + 0.2 * np.sin(2 * np.pi * (x + y))
    W[L.rho(1)] = 0.6
    W[L.u(0)] = 0.5
    W[L.u(1)] = 0.2 * np.cos(2 * np.pi * x)
    W[L.p] = 1.0 + 0.5 * np.exp(-80.0 * ((x - 0.3) ** 2 + (y - 0.5) ** 2))
    pbf = A.fine_problem(pbc, box)
    Wf, _ = prolong_prim(pbc, W, pbf, box)
    return pbc, W, pbf, Wf, box


def test_step_with_fluxes_is_the_step():
    """the split step that keeps its face fluxes is the oracle's step bit for
    bit (both sweep orders), and each sweep's update of a conserved component
    is the difference of its face fluxes"""
    pbc, W, _, _, _ = pulse_setup()
    o = O.Oracle(pbc)
    L = P.layout(pbc)
    U = o.prim_to_cons(W)
    dt = o.dt_cfl(U)
    for k in (0, 1):
        Us, fl = A.step_flux(o, U, dt, k)
        np.testing.assert_array_equal(Us, o.step(U, dt, k))
    cons = list(range(pbc.nmat - 1, L.V(0)))
    U1, F = o.sweep_flux(U, dt, 0)
    assert F.shape == (U.shape[0], U.shape[1], U.shape[2] + 1)
    want = U[cons] - dt / pbc.dx[0] * (F[cons, :, 1:] - F[cons, :, :-1])
    np.testing.assert_allclose(U1[cons], want, rtol=0, atol=1e-13)
    U2, F = o.sweep_flux(U, dt, 1)
    assert F.shape == (U.shape[0], U.shape[1] + 1, U.shape[2])
    want = U[cons] - dt / pbc.dx[1] * (F[cons, 1:, :] - F[cons, :-1, :])
    np.testing.assert_allclose(U2[cons], want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("reflux", [True, False])
def test_composite_conservation(reflux, monkeypatch):
    """on a periodic domain the composite grid (the coarse cells outside the
    patch and the patch's interior, each weighted by its area) conserves the
    partial masses, the momentum and the energy to round-off with the flux
    correction; without it the coarse/fine faces leak (the pin fails when
    the correction is dropped)"""
    if not reflux:
        monkeypatch.setattr(A, "reflux", lambda Uc, fc, ff, box, dt, pbc: Uc)
    pbc, W, pbf, Wf, box = pulse_setup()
    L = P.layout(pbc)
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    Uc, Uf = oc.prim_to_cons(W), of.prim_to_cons(Wf)
    cons = list(range(pbc.nmat - 1, L.V(0)))
    area = pbc.dx[0] * pbc.dx[1]
    inner = A.interior_mask(box)

    def totals(Uc, Uf):
        out = Uc[cons].sum(axis=(1, 2)) * area
        i0, j0, i1, j1 = box
        out = out - Uc[cons, j0:j1, i0:i1].sum(axis=(1, 2)) * area
        return out + Uf[cons][:, inner].sum(axis=1) * (area / 4)

    m0 = totals(Uc, Uf)
    for k in range(6):
        dtk, Uf = A.dt(oc, of, Uc, Uf, box)
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dtk, k)
        # averaging down makes the covered coarse cells carry the same totals
        np.testing.assert_allclose(Uc[cons].sum(axis=(1, 2)) * area, totals(Uc, Uf), rtol=1e-13, atol=1e-15)
    drift = np.abs(totals(Uc, Uf) - m0) / np.maximum(np.abs(m0), 1e-3)
    if reflux:
        assert np.all(drift < 1e-13), drift
    else:
        assert np.max(drift) > 1e-8, drift


def three_levels(pbc, Wc, box0, box1):
    """the level problems and initial states of a three-level stack, each
    finer level taking its parents' primitive state"""
    pb1 = A.fine_problem(pbc, box0)
    W1, _ = prolong_prim(pbc, Wc, pb1, box0)
    pb2 = A.fine_problem(pb1, box1)
    W2, _ = prolong_prim(pb1, W1, pb2, box1)
    return [pbc, pb1, pb2], [Wc, W1, W2]


def test_two_level_stack_is_the_two_level_step():
    pbc, W, pbf, Wf, box = pulse_setup()
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    Uc, Uf = oc.prim_to_cons(W), of.prim_to_cons(Wf)
    Us = [Uc, Uf]
    for k in range(3):
        dtk, Uf = A.dt(oc, of, Uc, Uf, box)
        dts, Us = A.dt_levels([oc, of], Us, [box])
        assert dts == dtk
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dtk, k)
        Us, _ = A.step_levels([oc, of], Us, [box], dtk, k)
        np.testing.assert_array_equal(Us[0], Uc)
        np.testing.assert_array_equal(Us[1], Uf)


def test_three_levels_uniform_and_conservative():
    """three nested levels: a uniform state stays exactly uniform on every
    level, and on the periodic pulse the composite grid (coarse cells outside
    the level-1 patch, level-1 interior cells outside the level-2 patch at
    1/4 of the area, level-2 interior cells at 1/16) keeps the partial
    masses, momentum and energy to round-off"""
    box0, box1 = (10, 5, 20, 11), (8, 7, 20, 13)
    pbc = two_gas(32, 16)
    L = P.layout(pbc)
    W = P.blank_prim(pbc)
    W[L.phi(0)] = 0.3
    W[L.rho(0)] = 1.0
    W[L.rho(1)] = 0.5
    W[L.u(0)] = 0.7
    W[L.p] = 1.0
    pbs, Ws = three_levels(pbc, W, box0, box1)
    os_ = [O.Oracle(pb) for pb in pbs]
    Us = [o.prim_to_cons(w) for o, w in zip(os_, Ws)]
    U0 = Us[0][:, 0, 0].copy()
    for k in range(3):
        dtk, Us = A.dt_levels(os_, Us, [box0, box1])
        Us, _ = A.step_levels(os_, Us, [box0, box1], dtk, k)
    for U in Us:
        for f in range(L.nfields):
            assert np.all(U[f] == U0[f]), f

    pbc, W, _, _, _ = pulse_setup(box=box0)
    pbs, Ws = three_levels(pbc, W, box0, box1)
    os_ = [O.Oracle(pb) for pb in pbs]
    Us = [o.prim_to_cons(w) for o, w in zip(os_, Ws)]
    cons = list(range(pbc.nmat - 1, L.V(0)))

    def totals(Us):
        out = np.zeros(len(cons))
        for l, U in enumerate(Us):
            keep = np.ones(U.shape[1:], dtype=bool) if l == 0 else A.interior_mask([box0, box1][l - 1])
            if l + 1 < len(Us):
                i0, j0, i1, j1 = [box0, box1][l]
                keep[j0:j1, i0:i1] = False
            out = out + U[cons][:, keep].sum(axis=1) / 4 ** l
        return out

    m0 = totals(Us)
    for k in range(6):
        dtk, Us = A.dt_levels(os_, Us, [box0, box1])
        Us, _ = A.step_levels(os_, Us, [box0, box1], dtk, k)
    drift = np.abs(totals(Us) - m0) / np.maximum(np.abs(m0), 1.0)
    assert np.all(drift < 1e-13), drift
    assert np.all(np.isfinite(Us[2]))


def test_several_patches():
    """several patches on one level: one patch is the two-level step bit for
    bit; two separated patches keep a uniform state exactly uniform and
    conserve the composite totals of the periodic pulse to round-off (the
    coarse cells between them corrected from both sides)"""
    pbc, W, pbf, Wf, box = pulse_setup()
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    Uc, Uf = oc.prim_to_cons(W), of.prim_to_cons(Wf)
    Vc, Vfs = Uc, [Uf]
    for k in range(2):
        dtk, Uf = A.dt(oc, of, Uc, Uf, box)
        dts, Vfs = A.dt_patches(oc, [of], Vc, Vfs, [box])
        assert dts == dtk
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dtk, k)
        Vc, Vfs = A.step_patches(oc, [of], Vc, Vfs, [box], dtk, k)
        np.testing.assert_array_equal(Vc, Uc)
        np.testing.assert_array_equal(Vfs[0], Uf)

    boxes = [(4, 4, 12, 10), (13, 6, 22, 12)]  # one coarse column between them
    assert A.separated(boxes) and not A.separated([(4, 4, 12, 10), (12, 6, 22, 12)])
    pbc, W, _, _, _ = pulse_setup()
    L = P.layout(pbc)
    oc = O.Oracle(pbc)
    pbfs = [A.fine_problem(pbc, b) for b in boxes]
    ofs = [O.Oracle(pb) for pb in pbfs]
    Uc = oc.prim_to_cons(W)
    Ufs = [o.prim_to_cons(prolong_prim(pbc, W, pb, b)[0]) for o, pb, b in zip(ofs, pbfs, boxes)]
    cons = list(range(pbc.nmat - 1, L.V(0)))

    def totals(Uc, Ufs):
        keep = np.ones(Uc.shape[1:], dtype=bool)
        out = np.zeros(len(cons))
        for Uf, (i0, j0, i1, j1) in zip(Ufs, boxes):
            keep[j0:j1, i0:i1] = False
            out = out + Uf[cons][:, A.interior_mask((i0, j0, i1, j1))].sum(axis=1) / 4
        return out + Uc[cons][:, keep].sum(axis=1)

    m0 = totals(Uc, Ufs)
    for k in range(6):
        dtk, Ufs = A.dt_patches(oc, ofs, Uc, Ufs, boxes)
        Uc, Ufs = A.step_patches(oc, ofs, Uc, Ufs, boxes, dtk, k)
    drift = np.abs(totals(Uc, Ufs) - m0) / np.maximum(np.abs(m0), 1.0)
    assert np.all(drift < 1e-13), drift

    Wu = P.blank_prim(pbc)
    Wu[L.phi(0)] = 0.3
    Wu[L.rho(0)] = 1.0
    Wu[L.rho(1)] = 0.5
    Wu[L.u(1)] = -0.4
    Wu[L.p] = 1.0
    Uc = oc.prim_to_cons(Wu)
    U0 = Uc[:, 0, 0].copy()
    Ufs = [o.prim_to_cons(prolong_prim(pbc, Wu, pb, b)[0]) for o, pb, b in zip(ofs, pbfs, boxes)]
    for k in range(3):
        dtk, Ufs = A.dt_patches(oc, ofs, Uc, Ufs, boxes)
        Uc, Ufs = A.step_patches(oc, ofs, Uc, Ufs, boxes, dtk, k)
    for U in [Uc] + Ufs:
        for f in range(L.nfields):
            assert np.all(U[f] == U0[f]), f


def test_cluster_pins():
    """the oracle's clustering: one blob gives the single-patch regrid box;
    two far blobs give two separated boxes covering every tag; two blobs
    closer than the margin give one box; no tags, no box"""
    n = (48, 40)
    yy, xx = np.mgrid[0:n[1], 0:n[0]]
    one = (xx - 14) ** 2 + (yy - 20) ** 2 < 16
    ext = (int(xx[one].min()), int(yy[one].min()), int(xx[one].max()) + 1, int(yy[one].max()) + 1)
    assert A.cluster(one, 2, n) == [A.regrid_box(ext, 2, n)]
    two = one | ((xx - 36) ** 2 + (yy - 12) ** 2 < 9)
    boxes = A.cluster(two, 2, n)
    assert len(boxes) == 2 and A.separated(boxes)
    for j, i in zip(*np.nonzero(two)):
        assert any(b[0] <= i < b[2] and b[1] <= j < b[3] for b in boxes)
    near = one | ((xx - 22) ** 2 + (yy - 20) ** 2 < 4)  # 3 cells apart, margin 2: grown sets touch
    assert len(A.cluster(near, 2, n)) == 1
    assert A.cluster(np.zeros((n[1], n[0]), dtype=bool), 2, n) == []


def test_rk3_refinement():
    """refinement with the paper's SSP-RK3 on both levels: the flux-keeping
    RK3 step is the oracle's RK3 step bit for bit and its conserved update
    is the difference of its time-weighted fluxes; a uniform state stays
    uniform to round-off; the composite grid conserves the periodic pulse's
    totals to round-off (two levels and three)"""
    pbc, W, pbf, Wf, box = pulse_setup()
    L = P.layout(pbc)
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    U = oc.prim_to_cons(W)
    dt = oc.dt_cfl(U)
    U1, fl = A.step_flux_rk3(oc, U, dt)
    np.testing.assert_array_equal(U1, oc.step_rk3(U, dt))
    cons = list(range(pbc.nmat - 1, L.V(0)))
    want = U[cons] - dt / pbc.dx[0] * (fl[0][cons, :, 1:] - fl[0][cons, :, :-1]) \
        - dt / pbc.dx[1] * (fl[1][cons, 1:, :] - fl[1][cons, :-1, :])
    np.testing.assert_allclose(U1[cons], want, rtol=0, atol=1e-13)

    Uc, Uf = oc.prim_to_cons(W), of.prim_to_cons(Wf)
    area = pbc.dx[0] * pbc.dx[1]
    inner = A.interior_mask(box)
    i0, j0, i1, j1 = box

    def totals(Uc, Uf):
        out = (Uc[cons].sum(axis=(1, 2)) - Uc[cons, j0:j1, i0:i1].sum(axis=(1, 2))) * area
        return out + Uf[cons][:, inner].sum(axis=1) * (area / 4)

    m0 = totals(Uc, Uf)
    for k in range(5):
        dtk, Uf = A.dt(oc, of, Uc, Uf, box)
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dtk, k, rk3=True)
    drift = np.abs(totals(Uc, Uf) - m0) / np.maximum(np.abs(m0), 1e-3)
    assert np.all(drift < 1e-13), drift

    box0, box1 = (10, 5, 20, 11), (8, 7, 20, 13)
    Wu = P.blank_prim(pbc)
    Wu[L.phi(0)] = 0.3
    Wu[L.rho(0)] = 1.0
    Wu[L.rho(1)] = 0.5
    Wu[L.u(0)] = 0.7
    Wu[L.p] = 1.0
    for Wi, uniform in ((Wu, True), (W, False)):
        pbs, Ws = three_levels(pbc, Wi, box0, box1)
        os_ = [O.Oracle(pb) for pb in pbs]
        Us = [o.prim_to_cons(w) for o, w in zip(os_, Ws)]
        U0 = Us[0][:, 0, 0].copy()
        for k in range(3):
            dtk, Us = A.dt_levels(os_, Us, [box0, box1])
            Us, _ = A.step_levels(os_, Us, [box0, box1], dtk, k, rk3=True)
        if uniform:  # up to the stage combinations' rounding (3/4 a + 1/4 a is not a)
            for U_ in Us:
                for f in range(L.nfields):
                    np.testing.assert_allclose(U_[f], U0[f], rtol=1e-14, atol=1e-15)
        assert all(np.all(np.isfinite(U_)) for U_ in Us)


def tree_setup():
    """the pulse's coarse grid with two separated patches, the first refined
    by a patch of its own (four grids, three levels)"""
    pbc, W, _, _, _ = pulse_setup()
    boxes, inner_box = [(4, 4, 12, 10), (13, 6, 22, 12)], (7, 7, 17, 13)
    pbfs = [A.fine_problem(pbc, b) for b in boxes]
    Wfs = [prolong_prim(pbc, W, pb, b)[0] for pb, b in zip(pbfs, boxes)]
    pbi = A.fine_problem(pbfs[0], inner_box)
    Wi = prolong_prim(pbfs[0], Wfs[0], pbi, inner_box)[0]
    return pbc, W, boxes, pbfs, Wfs, inner_box, pbi, Wi


def make_tree(pbc, W, boxes, pbfs, Wfs, inner_box, pbi, Wi):
    oc = O.Oracle(pbc)
    ofs = [O.Oracle(pb) for pb in pbfs]
    oi = O.Oracle(pbi)
    leaf = A.Patch(inner_box, oi, oi.prim_to_cons(Wi))
    kids = [A.Patch(boxes[0], ofs[0], ofs[0].prim_to_cons(Wfs[0]), [leaf]),
            A.Patch(boxes[1], ofs[1], ofs[1].prim_to_cons(Wfs[1]))]
    return oc, oc.prim_to_cons(W), kids


def test_tree_driver():
    """the tree driver is the chain driver (one patch per level) and the
    flat several-patch driver bit for bit, and on a mixed tree (two patches,
    one refined again) the composite totals of the periodic pulse are kept to
    round-off with either integrator"""
    pbc, W, _, _, _ = pulse_setup()
    box0, box1 = (10, 5, 20, 11), (8, 7, 20, 13)
    pbs, Ws = three_levels(pbc, W, box0, box1)
    os_ = [O.Oracle(pb) for pb in pbs]
    Us = [o.prim_to_cons(w) for o, w in zip(os_, Ws)]
    leaf = A.Patch(box1, os_[2], Us[2].copy())
    mid = A.Patch(box0, os_[1], Us[1].copy(), [leaf])
    Ut = Us[0].copy()
    for k in range(3):
        dtk, Us = A.dt_levels(os_, Us, [box0, box1])
        assert A.dt_tree(os_[0], Ut, [mid]) == dtk
        Us, _ = A.step_levels(os_, Us, [box0, box1], dtk, k)
        Ut, _ = A.step_tree(os_[0], Ut, [mid], dtk, k)
        for a, b in zip(Us, [Ut, mid.U, leaf.U]):
            np.testing.assert_array_equal(a, b)

    pbc, W, boxes, pbfs, Wfs, inner_box, pbi, Wi = tree_setup()
    oc, ofs = O.Oracle(pbc), [O.Oracle(pb) for pb in pbfs]
    Uc = oc.prim_to_cons(W)
    Ufs = [o.prim_to_cons(w) for o, w in zip(ofs, Wfs)]
    kids = [A.Patch(b, o, U.copy()) for b, o, U in zip(boxes, ofs, Ufs)]
    Ut = Uc.copy()
    for k in range(3):
        dtk, Ufs = A.dt_patches(oc, ofs, Uc, Ufs, boxes)
        assert A.dt_tree(oc, Ut, kids) == dtk
        Uc, Ufs = A.step_patches(oc, ofs, Uc, Ufs, boxes, dtk, k)
        Ut, _ = A.step_tree(oc, Ut, kids, dtk, k)
        np.testing.assert_array_equal(Ut, Uc)
        for ch, U in zip(kids, Ufs):
            np.testing.assert_array_equal(ch.U, U)

    L = P.layout(pbc)
    cons = list(range(pbc.nmat - 1, L.V(0)))
    for rk3 in (False, True):
        oc, Uc, kids = make_tree(pbc, W, boxes, pbfs, Wfs, inner_box, pbi, Wi)

        def totals():
            keep = np.ones(Uc.shape[1:], dtype=bool)
            out = np.zeros(len(cons))
            for ch in kids:
                i0, j0, i1, j1 = ch.box
                keep[j0:j1, i0:i1] = False
                m = A.interior_mask(ch.box)
                for g in ch.children:
                    a0, b0, a1, b1 = g.box
                    m[b0:b1, a0:a1] = False
                    out = out + g.U[cons][:, A.interior_mask(g.box)].sum(axis=1) / 16
                out = out + ch.U[cons][:, m].sum(axis=1) / 4
            return out + Uc[cons][:, keep].sum(axis=1)

        m0 = totals()
        for k in range(4):
            dtk = A.dt_tree(oc, Uc, kids, rk3)
            Uc, _ = A.step_tree(oc, Uc, kids, dtk, k, rk3)
        drift = np.abs(totals() - m0) / np.maximum(np.abs(m0), 1.0)
        assert np.all(drift < 1e-13), (rk3, drift)


def run_patches(pbc, W, boxes, nsteps, tree=False):
    """nsteps coarse steps of the coarse grid with patches over boxes (each
    starting from its parents' primitive state), by the several-patch driver
    or the tree driver; returns the coarse state, the patch states and the
    time steps"""
    oc = O.Oracle(pbc)
    pbfs = [A.fine_problem(pbc, b) for b in boxes]
    ofs = [O.Oracle(pb) for pb in pbfs]
    Uc = oc.prim_to_cons(W)
    Ufs = [o.prim_to_cons(prolong_prim(pbc, W, pb, b)[0]) for o, pb, b in zip(ofs, pbfs, boxes)]
    kids = [A.Patch(b, o, U) for b, o, U in zip(boxes, ofs, Ufs)]
    dts = []
    for k in range(nsteps):
        if tree:
            dtk = A.dt_tree(oc, Uc, kids)
            Uc, _ = A.step_tree(oc, Uc, kids, dtk, k)
        else:
            dtk, Ufs = A.dt_patches(oc, ofs, Uc, Ufs, boxes)
            Uc, Ufs = A.step_patches(oc, ofs, Uc, Ufs, boxes, dtk, k)
        dts.append(dtk)
    return Uc, ([ch.U for ch in kids] if tree else Ufs), dts


def fine_block(Uf, box, sub):
    """the fine interior cells of patch box that lie in the coarse box sub"""
    return Uf[:, A.G + 2 * (sub[1] - box[1]):A.G + 2 * (sub[3] - box[1]),
              A.G + 2 * (sub[0] - box[0]):A.G + 2 * (sub[2] - box[0])]


@pytest.mark.parametrize("split", ["x", "y"])
def test_touching_patches_split_a_box_exactly(split):
    """fine-to-fine exchange: two touching patches that split a box step
    exactly as one patch over the box (the coarse grid, the fine interiors
    and the time steps bit for bit, both sweep orders), by the several-patch
    and the tree drivers; without the exchange (each patch filling its ghost
    ring from the coarse level only) they do not"""
    pbc, W, _, _, box = pulse_setup()
    i0, j0, i1, j1 = box
    halves = [(i0, j0, 15, j1), (15, j0, i1, j1)] if split == "x" else [(i0, j0, i1, 8), (i0, 8, i1, j1)]
    assert A.disjoint(halves) and not A.separated(halves)
    Uc1, (Uf1,), dts1 = run_patches(pbc, W, [box], 4)
    for tree in (False, True):
        Uc2, Ufs2, dts2 = run_patches(pbc, W, halves, 4, tree)
        assert dts2 == dts1
        np.testing.assert_array_equal(Uc2, Uc1)
        for h, Uf in zip(halves, Ufs2):
            np.testing.assert_array_equal(fine_block(Uf, h, h), fine_block(Uf1, box, h))
    saved = A.exchange
    try:
        A.exchange = lambda Ufs, boxes: Ufs
        Uc3, _, _ = run_patches(pbc, W, halves, 4)
    finally:
        A.exchange = saved
    assert np.max(np.abs(Uc3 - Uc1)) > 1e-6 * np.max(np.abs(Uc1))


def test_exchange_copies_the_other_interiors():
    """every stored cell of a patch grid inside another patch's interior
    holds that patch's value after the exchange (brute force over fine
    positions), every other cell is left as it was"""
    boxes = [(4, 4, 12, 10), (12, 6, 22, 12), (6, 10, 12, 14)]
    rng = np.random.default_rng(3)
    Ufs = [rng.standard_normal((3,) + A.fine_shape(b)) for b in boxes]
    out = A.exchange(Ufs, boxes)
    for p, bp in enumerate(boxes):
        ny, nx = A.fine_shape(bp)
        for fj in range(ny):
            for fi in range(nx):
                X, Y = 2 * bp[0] + fi - A.G, 2 * bp[1] + fj - A.G
                want = Ufs[p][:, fj, fi]
                for q, bq in enumerate(boxes):
                    if q != p and 2 * bq[0] <= X < 2 * bq[2] and 2 * bq[1] <= Y < 2 * bq[3]:
                        want = Ufs[q][:, Y - 2 * bq[1] + A.G, X - 2 * bq[0] + A.G]
                np.testing.assert_array_equal(out[p][:, fj, fi], want)


def test_touching_patches_conserve_and_keep_uniform_states():
    """an L-shaped pair of touching patches (sharing part of a face): the
    composite totals of the periodic pulse are kept to round-off (both sides
    of the shared face compute its flux from the same values; the coarse
    cells beside it are the other patch's average), a uniform state stays
    exactly uniform; overlapping patches and the RK3 on touching patches are
    refused"""
    boxes = [(4, 4, 12, 10), (12, 6, 22, 12)]
    assert A.disjoint(boxes) and not A.separated(boxes)
    assert not A.disjoint([(4, 4, 12, 10), (11, 6, 22, 12)])
    pbc, W, _, _, _ = pulse_setup()
    L = P.layout(pbc)
    cons = list(range(pbc.nmat - 1, L.V(0)))

    def totals(Uc, Ufs):
        keep = np.ones(Uc.shape[1:], dtype=bool)
        out = np.zeros(len(cons))
        for Uf, b in zip(Ufs, boxes):
            keep[b[1]:b[3], b[0]:b[2]] = False
            out = out + Uf[cons][:, A.interior_mask(b)].sum(axis=1) / 4
        return out + Uc[cons][:, keep].sum(axis=1)

    oc = O.Oracle(pbc)
    Uc0 = oc.prim_to_cons(W)
    pbfs = [A.fine_problem(pbc, b) for b in boxes]
    Ufs0 = [O.Oracle(pb).prim_to_cons(prolong_prim(pbc, W, pb, b)[0]) for pb, b in zip(pbfs, boxes)]
    m0 = totals(Uc0, Ufs0)
    Uc, Ufs, _ = run_patches(pbc, W, boxes, 6)
    drift = np.abs(totals(Uc, Ufs) - m0) / np.maximum(np.abs(m0), 1.0)
    assert np.all(drift < 1e-13), drift

    Wu = P.blank_prim(pbc)
    Wu[L.phi(0)] = 0.3
    Wu[L.rho(0)] = 1.0
    Wu[L.rho(1)] = 0.5
    Wu[L.u(0)] = 0.3
    Wu[L.u(1)] = -0.4
    Wu[L.p] = 1.0
    Uc, Ufs, _ = run_patches(pbc, Wu, boxes, 3)
    U0 = oc.prim_to_cons(Wu)[:, 0, 0]
    for U in [Uc] + Ufs:
        for f in range(L.nfields):
            assert np.all(U[f] == U0[f]), f

    ofs = [O.Oracle(pb) for pb in pbfs]
    with pytest.raises(AssertionError):
        A.step_patches(oc, ofs, Uc0, Ufs0, boxes, 1e-4, 0, rk3=True)
