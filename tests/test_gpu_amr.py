"""Two-level subcycled refinement (Sec. 3; the readings are stated in
oracle/amr.py) on the GPU against the oracle's driver over its single-grid
step, element by element on both levels (<= 1e-10 per stored field): a
shock crossing a patch over the elastoplastic disc, a smooth wave crossing a
patch, a two-gas pressure pulse crossing the coarse/fine faces (flux
correction), a shock over a Johnson-Cook disc, and an LX-17 rate stick
refined around its booster, Cartesian and cylindrical; the GPU's dt against
the oracle's; composite conservation on the GPU; and the entry point's error
paths."""
import ctypes as C

import numpy as np
import pytest

from oracle import amr as A
from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P
from tests.parity_util import TOL, assert_parity, to_np
from tests.test_oracle_amr import prolong_prim, pulse_setup, wave_setup

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_14555_amd import solver as S

    return S


def configs():
    out = {}
    pbc, W = P.shock_disc(48, seed=2)
    box = (8, 12, 36, 36)
    pbf = A.fine_problem(pbc, box)
    out["shock_disc"] = (pbc, W, pbf, prolong_prim(pbc, W, pbf, box)[0], box, 8)
    box = (8, 5, 24, 11)
    pbc, W, pbf, Wf = wave_setup(32, box)
    out["wave"] = (pbc, W, pbf, Wf, box, 10)
    pbc, W, pbf, Wf, box = pulse_setup()
    out["pulse"] = (pbc, W, pbf, Wf, box, 8)
    pbc, W = P.shock_disc_jc(48, seed=3)
    box = (8, 12, 36, 36)  # a Johnson-Cook disc: the history slot is refluxed too
    pbf = A.fine_problem(pbc, box)
    out["jc_disc"] = (pbc, W, pbf, prolong_prim(pbc, W, pbf, box)[0], box, 8)
    pbc, W = P.rate_stick(60, 150, seed=4)
    box = (12, 6, 48, 24)  # the strip and its booster's end
    pbf = A.fine_problem(pbc, box)
    out["rate_stick"] = (pbc, W, pbf, prolong_prim(pbc, W, pbf, box)[0], box, 8)
    # off the axis (the patch grid carries its own radii); no density noise:
    # the ghost fill interpolates conserved variables, and across noisy
    # copper at one pressure (+-1% density, bulk modulus ~140 GPa) that
    # makes +-1e7 Pa pulses whose near-zero pressures in the explosive leave
    # the two implementations' rounding to decide the JWL split
    pbc, W = P.rate_stick_cyl(30, 150, seed=5, noise=0.0)
    box = (4, 6, 26, 24)
    pbf = A.fine_problem(pbc, box)
    out["rate_stick_cyl"] = (pbc, W, pbf, prolong_prim(pbc, W, pbf, box)[0], box, 8)
    return out


CONFIGS = configs()


@pytest.mark.parametrize("name", list(CONFIGS))
def test_amr_steps_match_oracle(solver, name):
    pbc, Wc, pbf, Wf, box, nsteps = CONFIGS[name]
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    Uc, Uf = oc.prim_to_cons(Wc), of.prim_to_cons(Wf)
    gc, gf = solver.Grid(pbc), solver.Grid(pbf)
    gc.set_primitive(Wc)
    gf.set_primitive(Wf)
    h = solver.Hierarchy(gc, gf, box)
    for k in range(nsteps):
        dt, Uf = A.dt(oc, of, Uc, Uf, box)
        dt_gpu = h.dt(pbc.cfl)
        assert dt_gpu == pytest.approx(dt, rel=1e-10)
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dt, k)
        h.advance(dt)
    assert np.all(np.isfinite(Uc)) and np.all(np.isfinite(Uf))
    assert_parity(to_np(gc.state), Uc, TOL, f"{name} coarse", P.layout(pbc))
    assert_parity(to_np(gf.state), Uf, TOL, f"{name} fine", P.layout(pbf))
    h.close()


def test_amr_entry_point_errors(solver):
    from paper_2009_14555_amd import dimp as D

    pbc, Wc, pbf, Wf, box, _ = CONFIGS["wave"]
    gc, gf = solver.Grid(pbc), solver.Grid(pbf)
    gc.set_primitive(Wc)
    gf.set_primitive(Wf)
    with pytest.raises(D.DimpError):  # the fine grid does not match the box
        solver.Hierarchy(gc, gf, (box[0], box[1], box[2] + 1, box[3]))
    with pytest.raises(D.DimpError):  # closer than 3 coarse cells to the edge
        solver.Hierarchy(gc, gf, (2, box[1], 2 + box[2] - box[0], box[3]))
    with pytest.raises(D.DimpError):
        solver.Hierarchy(gc, gc, box)
    h = solver.Hierarchy(gc, gf, box)
    with pytest.raises(D.DimpError):
        h.advance(-1.0)
    out = C.c_double()
    with pytest.raises(D.DimpError):
        D.call("dimp_amr_dt", h.h, 0.0, C.byref(out))
    gf.set_integrator("rk3")
    with pytest.raises(D.DimpError):  # the levels step the split integrator
        h.advance(1e-4)
    h.close()


@pytest.mark.parametrize("integrator", ["split", "rk3"])
def test_amr_conserves_on_the_gpu(solver, integrator):
    """the GPU's composite grid (coarse cells outside the patch, the patch's
    interior at a quarter of the area) keeps the partial masses, momentum and
    energy of the periodic pulse to round-off over 12 steps"""
    pbc, Wc, pbf, Wf, box, _ = CONFIGS["pulse"]
    L = P.layout(pbc)
    gc, gf = solver.Grid(pbc), solver.Grid(pbf)
    gc.set_primitive(Wc)
    gf.set_primitive(Wf)
    gc.set_integrator(integrator)
    gf.set_integrator(integrator)
    h = solver.Hierarchy(gc, gf, box)
    cons = list(range(pbc.nmat - 1, L.V(0)))
    inner = A.interior_mask(box)
    i0, j0, i1, j1 = box

    def totals():
        Uc, Uf = to_np(gc.state), to_np(gf.state)
        out = Uc[cons].sum(axis=(1, 2)) - Uc[cons, j0:j1, i0:i1].sum(axis=(1, 2))
        return out + Uf[cons][:, inner].sum(axis=1) / 4

    m0 = totals()
    for _ in range(12):
        h.advance(h.dt(pbc.cfl))
    drift = np.abs(totals() - m0) / np.maximum(np.abs(m0), 1.0)
    assert np.all(drift < 1e-12), drift
    h.close()


def oracle_prim_after(pb, W, nsteps):
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    for k in range(nsteps):
        U = o.step(U, o.dt_cfl(U), k)
    return U, o.cons_to_prim(U)


@pytest.mark.parametrize("name", ["shock_disc", "rate_stick"])
def test_amr_tag_matches_oracle(solver, name):
    """the criterion's decisions from the same primitive state, exactly; and
    the extent from the GPU's own primitive state"""
    import torch

    pbc, Wc = (P.shock_disc(48, seed=2) if name == "shock_disc" else P.rate_stick(60, 150, seed=4))
    U, Wp = oracle_prim_after(pbc, Wc, 4)
    g = solver.Grid(pbc)
    g.set_conserved(U)
    for th in (0.02, 0.1):
        tags_o, bbox_o = A.tag(pbc, Wp, th)
        tags_g, bbox_g = solver.amr_tag_prim(g, torch.tensor(Wp, device=g.device), th)
        np.testing.assert_array_equal(to_np(tags_g).astype(bool), tags_o)
        assert bbox_g == bbox_o
        assert solver.amr_tag(g, th)[1] == bbox_o


def blob(n=32):
    """a dense blob of gas 0 carried at u = 1 through gas 1 (periodic)"""
    pbc = P.Problem(ndim=2, n=(n, n, 1), dx=(1.0 / n, 1.0 / n, 1.0), bc=(P.BC_PERIODIC,) * 3,
                    materials=[P.air(1.4), P.air(1.67)], thinc=1, cfl=0.4, va_scale=(1.0,) * 6)
    L = P.layout(pbc)
    W = P.blank_prim(pbc)
    x, y = P.cell_centres(pbc)
    W[L.phi(0)] = np.clip(np.exp(-((x - 0.3) ** 2 + (y - 0.5) ** 2) / 0.01), 1e-6, 1 - 1e-6)
    W[L.rho(0)] = 2.0
    W[L.rho(1)] = 1.0
    W[L.u(0)] = 1.0
    W[L.p] = 1.0
    return pbc, W


def test_amr_regrid_run_matches_oracle(solver):
    """patch boxes from the criterion every 4 coarse steps (th 0.05, margin
    2), decided on the oracle's state and applied to both sides, around a
    blob that moves"""
    pbc, Wc = blob()
    oc = O.Oracle(pbc)
    Uc = oc.prim_to_cons(Wc)
    box = A.regrid_box(A.tag(pbc, Wc, 0.05)[1], 2, pbc.n)
    of = O.Oracle(A.fine_problem(pbc, box))
    Uf = A.prolong(Uc, box)
    gc = solver.Grid(pbc)
    gc.set_primitive(Wc)
    gf = solver.Grid(A.fine_problem(pbc, box))
    h = solver.Hierarchy(gc, gf, box)
    h.prolong()
    for k in range(16):
        if k > 0 and k % 4 == 0:
            nb = A.regrid_box(A.tag(pbc, oc.cons_to_prim(Uc), 0.05)[1], 2, pbc.n)
            if nb != box:
                box = nb
                of = O.Oracle(A.fine_problem(pbc, box))
                Uf = A.prolong(Uc, box)
                h = h.regrid(box)
        dt, Uf = A.dt(oc, of, Uc, Uf, box)
        assert h.dt(pbc.cfl) == pytest.approx(dt, rel=1e-10)
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dt, k)
        h.advance(dt)
    assert box != A.regrid_box(A.tag(pbc, Wc, 0.05)[1], 2, pbc.n)  # the patch moved with the blob
    assert_parity(to_np(gc.state), Uc, TOL, "regrid coarse", P.layout(pbc))
    assert_parity(to_np(h.fine.state), Uf, TOL, "regrid fine", P.layout(of.pb))
    h.close()


def three_level_stack(solver, pbc, Wc, box0, box1):
    from tests.test_oracle_amr import three_levels

    pbs, Ws = three_levels(pbc, Wc, box0, box1)
    gs = [solver.Grid(pb) for pb in pbs]
    for g, w in zip(gs, Ws):
        g.set_primitive(w)
    outer = solver.Hierarchy(gs[0], gs[1], box0)
    inner = solver.Hierarchy(gs[1], gs[2], box1)
    outer.nest(inner)
    return pbs, Ws, gs, outer, inner


@pytest.mark.parametrize("name", ["pulse", "shock_disc"])
def test_three_levels_match_oracle(solver, name):
    """a three-level stack (level 2 nested in level 1's patch) against the
    oracle's recursive driver on all three levels, and its dt"""
    if name == "pulse":
        pbc, Wc, _, _, _ = pulse_setup(box=(10, 5, 20, 11))
        box0, box1, nsteps = (10, 5, 20, 11), (8, 7, 20, 13), 6
    else:
        # the shock reaches level 2 (its left edge 7 level-1 cells in) by step 3
        pbc, Wc = P.shock_disc(48, seed=2)
        box0, box1, nsteps = (8, 12, 36, 36), (7, 12, 30, 44), 12
    pbs, Ws, gs, outer, inner = three_level_stack(solver, pbc, Wc, box0, box1)
    os_ = [O.Oracle(pb) for pb in pbs]
    Us = [o.prim_to_cons(w) for o, w in zip(os_, Ws)]
    for k in range(nsteps):
        dt, Us = A.dt_levels(os_, Us, [box0, box1])
        assert outer.dt(pbc.cfl) == pytest.approx(dt, rel=1e-10)
        Us, _ = A.step_levels(os_, Us, [box0, box1], dt, k)
        outer.advance(dt)
    for l in range(3):
        assert np.all(np.isfinite(Us[l]))
        assert_parity(to_np(gs[l].state), Us[l], TOL, f"{name} level {l}", P.layout(pbs[l]))
    outer.close()
    inner.close()


def test_three_levels_conserve_and_errors(solver):
    from paper_2009_14555_amd import dimp as D

    box0, box1 = (10, 5, 20, 11), (8, 7, 20, 13)
    pbc, Wc, _, _, _ = pulse_setup(box=box0)
    L = P.layout(pbc)
    pbs, Ws, gs, outer, inner = three_level_stack(solver, pbc, Wc, box0, box1)
    cons = list(range(pbc.nmat - 1, L.V(0)))

    def totals():
        out = np.zeros(len(cons))
        for l, g in enumerate(gs):
            U = to_np(g.state)
            keep = np.ones(U.shape[1:], dtype=bool) if l == 0 else A.interior_mask([box0, box1][l - 1])
            if l < 2:
                i0, j0, i1, j1 = [box0, box1][l]
                keep[j0:j1, i0:i1] = False
            out = out + U[cons][:, keep].sum(axis=1) / 4 ** l
        return out

    m0 = totals()
    for _ in range(8):
        outer.advance(outer.dt(pbc.cfl))
    drift = np.abs(totals() - m0) / np.maximum(np.abs(m0), 1.0)
    assert np.all(drift < 1e-12), drift
    with pytest.raises(D.DimpError):  # the nested hierarchy steps only through the outer one
        inner.advance(1e-4)
    with pytest.raises(D.DimpError):
        outer.nest(inner)  # already nested
    with pytest.raises(D.DimpError):  # grids that do not chain
        inner.nest(outer)
    outer.close()
    inner.close()
    # an inner patch too near the edge of the outer fine grid
    outer2 = solver.Hierarchy(gs[0], gs[1], box0)
    pb_near = A.fine_problem(pbs[1], (5, 7, 17, 13))
    g_near = solver.Grid(pb_near)
    inner2 = solver.Hierarchy(gs[1], g_near, (5, 7, 17, 13))
    with pytest.raises(D.DimpError):
        outer2.nest(inner2)
    outer2.close()
    inner2.close()


def test_several_patches_match_oracle(solver):
    """two separated patches on one level (a group) against the oracle's
    several-patch driver on the coarse grid and both patches, the group's
    dt, composite conservation, and the grouping errors"""
    from paper_2009_14555_amd import dimp as D

    boxes = [(4, 4, 12, 10), (13, 6, 22, 12)]
    pbc, Wc, _, _, _ = pulse_setup()
    L = P.layout(pbc)
    pbfs = [A.fine_problem(pbc, b) for b in boxes]
    Wfs = [prolong_prim(pbc, Wc, pb, b)[0] for pb, b in zip(pbfs, boxes)]
    oc, ofs = O.Oracle(pbc), [O.Oracle(pb) for pb in pbfs]
    Uc, Ufs = oc.prim_to_cons(Wc), [o.prim_to_cons(w) for o, w in zip(ofs, Wfs)]
    gc = solver.Grid(pbc)
    gc.set_primitive(Wc)
    gfs = [solver.Grid(pb) for pb in pbfs]
    for g, w in zip(gfs, Wfs):
        g.set_primitive(w)
    hs = [solver.Hierarchy(gc, g, b) for g, b in zip(gfs, boxes)]
    hs[0].group(hs[1])
    cons = list(range(pbc.nmat - 1, L.V(0)))

    def totals():
        U = to_np(gc.state)
        keep = np.ones(U.shape[1:], dtype=bool)
        out = np.zeros(len(cons))
        for g, (i0, j0, i1, j1) in zip(gfs, boxes):
            keep[j0:j1, i0:i1] = False
            out = out + to_np(g.state)[cons][:, A.interior_mask((i0, j0, i1, j1))].sum(axis=1) / 4
        return out + U[cons][:, keep].sum(axis=1)

    m0 = totals()
    for k in range(8):
        dt, Ufs = A.dt_patches(oc, ofs, Uc, Ufs, boxes)
        assert hs[0].dt(pbc.cfl) == pytest.approx(dt, rel=1e-10)
        Uc, Ufs = A.step_patches(oc, ofs, Uc, Ufs, boxes, dt, k)
        hs[0].advance(dt)
    assert_parity(to_np(gc.state), Uc, TOL, "coarse", L)
    for p in range(2):
        assert_parity(to_np(gfs[p].state), Ufs[p], TOL, f"patch {p}", P.layout(pbfs[p]))
    drift = np.abs(totals() - m0) / np.maximum(np.abs(m0), 1.0)
    assert np.all(drift < 1e-12), drift
    with pytest.raises(D.DimpError):  # members step through the head
        hs[1].advance(1e-4)
    with pytest.raises(D.DimpError):  # already grouped
        hs[0].group(hs[1])
    # a nested patch too near the edge of its outer fine grid
    pb_in = A.fine_problem(pbfs[0], (5, 7, 9, 9))
    g_in = solver.Grid(pb_in)
    h_in = solver.Hierarchy(gfs[0], g_in, (5, 7, 9, 9))
    with pytest.raises(D.DimpError):
        hs[0].nest(h_in)
    h_in.close()
    hs[1].close()  # leaves the group; the head steps alone
    hs[0].advance(1e-5)
    hs[0].close()
    # patches that share a coarse cell
    pb_t = A.fine_problem(pbc, (11, 6, 22, 12))
    g_t = solver.Grid(pb_t)
    h0, h_t = solver.Hierarchy(gc, gfs[0], boxes[0]), solver.Hierarchy(gc, g_t, (11, 6, 22, 12))
    with pytest.raises(D.DimpError):
        h0.group(h_t)
    h0.close()
    h_t.close()


def group_run(solver, pbc, Wc, boxes, nsteps, oracle=True, rk3=False):
    """a coarse grid with a group of patches over boxes, stepped nsteps
    coarse steps on the GPU (and by the oracle's several-patch driver)"""
    pbfs = [A.fine_problem(pbc, b) for b in boxes]
    Wfs = [prolong_prim(pbc, Wc, pb, b)[0] for pb, b in zip(pbfs, boxes)]
    gc = solver.Grid(pbc)
    gc.set_primitive(Wc)
    gfs = [solver.Grid(pb) for pb in pbfs]
    for g, w in zip(gfs, Wfs):
        g.set_primitive(w)
    if rk3:
        for g in [gc] + gfs:
            g.set_integrator("rk3")
    hs = [solver.Hierarchy(gc, g, b) for g, b in zip(gfs, boxes)]
    for h in hs[1:]:
        hs[0].group(h)
    oc, ofs = O.Oracle(pbc), [O.Oracle(pb) for pb in pbfs]
    Uc, Ufs = oc.prim_to_cons(Wc), [o.prim_to_cons(w) for o, w in zip(ofs, Wfs)]
    for k in range(nsteps):
        dt = hs[0].dt(pbc.cfl)
        if oracle:
            dto, Ufs = A.dt_patches(oc, ofs, Uc, Ufs, boxes)
            assert dt == pytest.approx(dto, rel=1e-10)
            Uc, Ufs = A.step_patches(oc, ofs, Uc, Ufs, boxes, dto, k)
        hs[0].advance(dto if oracle else dt)
    return gc, gfs, hs, pbfs, Uc, Ufs


def test_touching_patches_match_oracle(solver):
    """fine-to-fine exchange: an L-shaped pair of touching patches (sharing
    part of a face) against the oracle on the coarse grid and both patches,
    composite conservation; two touching halves of a box step bit for bit as
    one patch over the box; the RK3 on touching patches is refused"""
    from paper_2009_14555_amd import dimp as D

    boxes = [(4, 4, 12, 10), (12, 6, 22, 12)]
    pbc, Wc, _, _, _ = pulse_setup()
    L = P.layout(pbc)
    cons = list(range(pbc.nmat - 1, L.V(0)))
    gc0 = solver.Grid(pbc)
    gc0.set_primitive(Wc)
    Uc0 = to_np(gc0.state)
    gc, gfs, hs, pbfs, Uc, Ufs = group_run(solver, pbc, Wc, boxes, 8)
    assert_parity(to_np(gc.state), Uc, TOL, "coarse", L)
    for p in range(2):
        assert_parity(to_np(gfs[p].state), Ufs[p], TOL, f"patch {p}", L)

    def totals(U, Uf_list):
        keep = np.ones(U.shape[1:], dtype=bool)
        out = np.zeros(len(cons))
        for Uf, b in zip(Uf_list, boxes):
            keep[b[1]:b[3], b[0]:b[2]] = False
            out = out + Uf[cons][:, A.interior_mask(b)].sum(axis=1) / 4
        return out + U[cons][:, keep].sum(axis=1)

    Uf0 = [O.Oracle(pb).prim_to_cons(prolong_prim(pbc, Wc, pb, b)[0]) for pb, b in zip(pbfs, boxes)]
    m0 = totals(Uc0, Uf0)
    drift = np.abs(totals(to_np(gc.state), [to_np(g.state) for g in gfs]) - m0) / np.maximum(np.abs(m0), 1.0)
    assert np.all(drift < 1e-12), drift
    for h in hs[::-1]:
        h.close()

    box = (10, 5, 20, 11)
    gc1, (gf1,), hs1, _, _, _ = group_run(solver, pbc, Wc, [box], 4, oracle=False)
    for halves in ([(10, 5, 15, 11), (15, 5, 20, 11)], [(10, 5, 20, 8), (10, 8, 20, 11)]):
        gc2, gf2, hs2, _, _, _ = group_run(solver, pbc, Wc, halves, 4, oracle=False)
        assert np.array_equal(to_np(gc2.state), to_np(gc1.state))
        F1 = to_np(gf1.state)
        for h, g in zip(halves, gf2):
            y0, x0 = A.G + 2 * (h[1] - box[1]), A.G + 2 * (h[0] - box[0])
            ny, nx = 2 * (h[3] - h[1]), 2 * (h[2] - h[0])
            a = to_np(g.state)[:, A.G:A.G + ny, A.G:A.G + nx]
            assert np.array_equal(a, F1[:, y0:y0 + ny, x0:x0 + nx]), h
        for q in hs2[::-1]:
            q.close()

    gc3, gfs3, hs3, _, _, _ = group_run(solver, pbc, Wc, boxes, 0, oracle=False, rk3=True)
    with pytest.raises(D.DimpError):
        hs3[0].advance(1e-4)
    for h in hs3[::-1]:
        h.close()


def two_blobs(n=48):
    """two compact blobs of gas 0 carried at u = 1 through gas 1 (periodic)"""
    pbc = P.Problem(ndim=2, n=(n, n, 1), dx=(1.0 / n, 1.0 / n, 1.0), bc=(P.BC_PERIODIC,) * 3,
                    materials=[P.air(1.4), P.air(1.67)], thinc=1, cfl=0.4, va_scale=(1.0,) * 6)
    L = P.layout(pbc)
    W = P.blank_prim(pbc)
    x, y = P.cell_centres(pbc)

    def bump(cx, cy, R=0.12):
        r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
        return np.where(r < R, np.cos(0.5 * np.pi * r / R) ** 2, 0.0)

    W[L.phi(0)] = np.clip(bump(0.3, 0.27) + bump(0.3, 0.73), 1e-6, 1 - 1e-6)
    W[L.rho(0)] = 2.0
    W[L.rho(1)] = 1.0
    W[L.u(0)] = 1.0
    W[L.p] = 1.0
    return pbc, W


def test_regrid_into_several_patches_matches_oracle(solver):
    """a level of several patches regridded every 4 coarse steps from the
    criterion (th 0.05, margin 2; boxes clustered from the oracle's tags and
    applied to both sides) around two moving blobs: two patches throughout,
    both levels equal to the oracle's several-patch run"""
    pbc, Wc = two_blobs()
    oc = O.Oracle(pbc)
    Uc = oc.prim_to_cons(Wc)
    boxes = A.cluster(A.tag(pbc, Wc, 0.05)[0], 2, pbc.n)
    assert len(boxes) == 2
    assert solver.cluster_tags(A.tag(pbc, Wc, 0.05)[0], 2, pbc.n) == boxes
    ofs = [O.Oracle(A.fine_problem(pbc, b)) for b in boxes]
    Ufs = [A.prolong(Uc, b) for b in boxes]
    gc = solver.Grid(pbc)
    gc.set_primitive(Wc)
    hs = solver.regrid_patches(gc, [], boxes)
    first = list(boxes)
    for k in range(12):
        if k > 0 and k % 4 == 0:
            nb = A.cluster(A.tag(pbc, oc.cons_to_prim(Uc), 0.05)[0], 2, pbc.n)
            if nb != boxes:
                boxes = nb
                ofs = [O.Oracle(A.fine_problem(pbc, b)) for b in boxes]
                Ufs = [A.prolong(Uc, b) for b in boxes]
                hs = solver.regrid_patches(gc, hs, boxes)
        dt, Ufs = A.dt_patches(oc, ofs, Uc, Ufs, boxes)
        assert hs[0].dt(pbc.cfl) == pytest.approx(dt, rel=1e-10)
        Uc, Ufs = A.step_patches(oc, ofs, Uc, Ufs, boxes, dt, k)
        hs[0].advance(dt)
    assert len(boxes) == 2 and boxes != first  # the patches moved with the blobs
    assert_parity(to_np(gc.state), Uc, TOL, "coarse", P.layout(pbc))
    for p, h in enumerate(hs):
        assert_parity(to_np(h.fine.state), Ufs[p], TOL, f"patch {p}", P.layout(ofs[p].pb))
    for h in hs:
        h.close()


@pytest.mark.parametrize("box", [(6, 5, 7, 6), (3, 3, 29, 13), (3, 3, 4, 13)])
def test_amr_edge_boxes(solver, box):
    """degenerate patches on the 32 x 16 periodic pulse: one coarse cell, the
    largest box the 3-cell margin allows, and a one-cell-wide strip; both
    levels against the oracle after 6 steps"""
    pbc, W, _, _, _ = pulse_setup()
    pbf = A.fine_problem(pbc, box)
    Wf, _ = prolong_prim(pbc, W, pbf, box)
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    Uc, Uf = oc.prim_to_cons(W), of.prim_to_cons(Wf)
    gc, gf = solver.Grid(pbc), solver.Grid(pbf)
    gc.set_primitive(W)
    gf.set_primitive(Wf)
    h = solver.Hierarchy(gc, gf, box)
    for k in range(6):
        dt, Uf = A.dt(oc, of, Uc, Uf, box)
        assert h.dt(pbc.cfl) == pytest.approx(dt, rel=1e-10)
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dt, k)
        h.advance(dt)
    assert_parity(to_np(gc.state), Uc, TOL, f"{box} coarse", P.layout(pbc))
    assert_parity(to_np(gf.state), Uf, TOL, f"{box} fine", P.layout(pbf))
    h.close()


@pytest.mark.parametrize("name", ["pulse", "shock_disc", "rate_stick", "rate_stick_cyl"])
def test_amr_rk3_matches_oracle(solver, name):
    """refinement with the paper's SSP-RK3 on both levels (stage inputs
    refilled at their times, stage-weighted flux correction) against the
    oracle's RK3 driver on both levels"""
    pbc, Wc, pbf, Wf, box, _ = CONFIGS[name]
    oc, of = O.Oracle(pbc), O.Oracle(pbf)
    Uc, Uf = oc.prim_to_cons(Wc), of.prim_to_cons(Wf)
    gc, gf = solver.Grid(pbc), solver.Grid(pbf)
    gc.set_primitive(Wc)
    gf.set_primitive(Wf)
    gc.set_integrator("rk3")
    gf.set_integrator("rk3")
    h = solver.Hierarchy(gc, gf, box)
    for k in range(6):
        dt, Uf = A.dt(oc, of, Uc, Uf, box)
        assert h.dt(pbc.cfl) == pytest.approx(dt, rel=1e-10)
        Uc, Uf = A.step(oc, of, Uc, Uf, box, dt, k, rk3=True)
        h.advance(dt)
    assert_parity(to_np(gc.state), Uc, TOL, f"{name} rk3 coarse", P.layout(pbc))
    assert_parity(to_np(gf.state), Uf, TOL, f"{name} rk3 fine", P.layout(pbf))
    h.close()


def test_three_levels_rk3_match_oracle(solver):
    box0, box1 = (10, 5, 20, 11), (8, 7, 20, 13)
    pbc, Wc, _, _, _ = pulse_setup(box=box0)
    pbs, Ws, gs, outer, inner = three_level_stack(solver, pbc, Wc, box0, box1)
    for g in gs:
        g.set_integrator("rk3")
    os_ = [O.Oracle(pb) for pb in pbs]
    Us = [o.prim_to_cons(w) for o, w in zip(os_, Ws)]
    for k in range(4):
        dt, Us = A.dt_levels(os_, Us, [box0, box1])
        Us, _ = A.step_levels(os_, Us, [box0, box1], dt, k, rk3=True)
        outer.advance(dt)
    for l in range(3):
        assert_parity(to_np(gs[l].state), Us[l], TOL, f"rk3 level {l}", P.layout(pbs[l]))
    outer.close()
    inner.close()


@pytest.mark.parametrize("integrator", ["split", "rk3"])
def test_refinement_tree_matches_oracle(solver, integrator):
    """a refinement tree: two separated patches on the pulse's coarse grid
    (a group), the first refined by a patch of its own (nested); all four
    grids against the oracle's tree driver, and the composite totals"""
    from tests.test_oracle_amr import make_tree, tree_setup

    pbc, W, boxes, pbfs, Wfs, inner_box, pbi, Wi = tree_setup()
    oc, Uc, kids = make_tree(pbc, W, boxes, pbfs, Wfs, inner_box, pbi, Wi)
    gc = solver.Grid(pbc)
    gc.set_primitive(W)
    gfs = [solver.Grid(pb) for pb in pbfs]
    for g, w in zip(gfs, Wfs):
        g.set_primitive(w)
    gi = solver.Grid(pbi)
    gi.set_primitive(Wi)
    for g in [gc, gi] + gfs:
        g.set_integrator(integrator)
    hs = [solver.Hierarchy(gc, g, b) for g, b in zip(gfs, boxes)]
    hi = solver.Hierarchy(gfs[0], gi, inner_box)
    hs[0].group(hs[1])
    hs[0].nest(hi)
    rk3 = integrator == "rk3"
    for k in range(5):
        dt = A.dt_tree(oc, Uc, kids, rk3)
        assert hs[0].dt(pbc.cfl) == pytest.approx(dt, rel=1e-10)
        Uc, _ = A.step_tree(oc, Uc, kids, dt, k, rk3)
        hs[0].advance(dt)
    assert_parity(to_np(gc.state), Uc, TOL, "tree coarse", P.layout(pbc))
    for p in range(2):
        assert_parity(to_np(gfs[p].state), kids[p].U, TOL, f"tree patch {p}", P.layout(pbfs[p]))
    assert_parity(to_np(gi.state), kids[0].children[0].U, TOL, "tree nested patch", P.layout(pbi))
    for h in hs + [hi]:
        h.close()
