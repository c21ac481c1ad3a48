"""Two-level subcycled refinement (Sec. 3) on top of the oracle's single-grid
step (test infrastructure only).

The paper advances each level with the single-grid update over its patches,
the finer level taking r steps of dt/r per coarser step (Berger-Oliger
subcycling, refinement ratio r = 2 here).  What it leaves to its AMReX
platform is read as follows:

* one refined patch over coarse cells [i0, i1) x [j0, j1) of a 2-D grid, at
  least 3 coarse cells from the grid's edges, stored as a grid of its own
  with G = 4 fine ghost layers (the split step's stencil reach of 3 per sweep
  plus the interface normal's transverse neighbour, so that the interior is
  unaffected by the patch grid's own edges);
* fine ghost cells are filled from the coarse level linearly in time
  between the coarse states before and after the coarse step, U_t = U_old +
  w (U_new - U_old) with w = 0 for the first fine step and 1/2 for the second,
  and linearly in space inside their coarse parent: U_t + (+-1/4)(s_x + s_y)
  with minmod-limited slopes of U_t per conserved component (conservative:
  the four children of a cell average to it; no new extrema; piecewise
  constant injection was measured to make the refined cells less accurate
  than the coarse-only run);
* after the fine steps every covered coarse cell becomes the mean of its
  four fine children (conserved variables and Vbar alike);
* flux correction (refluxing, as in the Berger-Colella method the paper's
  platform implements): each split sweep keeps its face fluxes, and after
  averaging down the coarse cells just outside the patch take, on their
  coarse/fine face, the fine fluxes averaged over the face's two fine faces
  and the two fine steps in place of the coarse flux; for the conserved
  components only (the volume fractions and Vbar carry non-conservative
  terms with no flux form), so mass, momentum and energy are conserved over
  the composite grid;
* dt = min(coarse CFL step, 2 x fine CFL step), the fine one over the whole
  patch grid after a ghost fill with the coarse state;
* several patches on one level may touch (share faces) but not overlap.
  With the split integrator the fine level holds one value per fine
  position, the interior value of the patch covering it, else the coarse
  fill: before each fine step every patch grid's stored cells inside another
  patch's interior take that patch's values (fine-to-fine exchange, after
  the coarse fill of every patch; all patches are filled before any steps;
  a patch's ghost layers reach 2 coarse cells, so patches one cell apart
  exchange too).  With G = 4 each patch then computes on its interior what
  one grid over the union would (a box split in two steps as the box), and
  both sides of a shared face compute its flux from the same values.  The
  coarse cells beside a patch face that another patch covers take that
  patch's average, so the flux corrections are applied before averaging
  down.  The SSP-RK3 would need the exchange at every stage input (its
  stages run patch by patch): with it every ghost ring comes from the coarse
  level only and touching patches are refused;
* regridding (tag, regrid_box, prolong): the Sec. 4.2 criterion tags cells
  whose refinement variables jump to a neighbour by more than a fraction;
  the new patch is the tagged extent padded by a margin, and each of its
  cells takes its coarse parent's state (the coarse level holds the averaged
  fine solution; the old fine data are not copied over).
"""
from __future__ import annotations

import numpy as np

G = 4


def fine_shape(box):
    i0, j0, i1, j1 = box
    return 2 * (j1 - j0) + 2 * G, 2 * (i1 - i0) + 2 * G


def parents(box):
    """coarse (J, I) parent of every fine cell of the patch grid"""
    ny, nx = fine_shape(box)
    i0, j0 = box[0], box[1]
    fi = np.arange(nx)
    fj = np.arange(ny)
    I = i0 + np.floor_divide(fi - G, 2)
    J = j0 + np.floor_divide(fj - G, 2)
    return np.meshgrid(J, I, indexing="ij")


def interior_mask(box):
    ny, nx = fine_shape(box)
    m = np.zeros((ny, nx), dtype=bool)
    m[G:ny - G, G:nx - G] = True
    return m


def minmod(a, b):
    return np.where(a * b <= 0.0, 0.0, np.where(np.abs(a) < np.abs(b), a, b))


def fill(Uc_old, Uc_new, w, Uf, box, every=False):
    """fine ghost cells from the coarse level at weight w in time, linear
    with limited slopes inside each coarse parent; every=True: every fine
    cell takes its parent's state (no slopes)"""
    J, I = parents(box)
    ny, nx = fine_shape(box)
    ghost = np.ones((ny, nx), dtype=bool) if every else ~interior_mask(box)
    Jg, Ig = J[ghost], I[ghost]
    # the fine cell's offset from its parent's centre, in coarse cells
    fj, fi = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ox = np.where((fi[ghost] - G) % 2 == 0, -0.25, 0.25)
    oy = np.where((fj[ghost] - G) % 2 == 0, -0.25, 0.25)

    def at(dj, di):
        old = Uc_old[:, Jg + dj, Ig + di]
        return old + w * (Uc_new[:, Jg + dj, Ig + di] - old)

    c = at(0, 0)
    out = Uf.copy()
    if every:
        out[:, ghost] = c
        return out
    sx = minmod(c - at(0, -1), at(0, 1) - c)
    sy = minmod(c - at(-1, 0), at(1, 0) - c)
    out[:, ghost] = c + ox * sx + oy * sy
    return out


def average_down(Uc, Uf, box):
    i0, j0, i1, j1 = box
    out = Uc.copy()
    f = Uf[:, G:G + 2 * (j1 - j0), G:G + 2 * (i1 - i0)]
    out[:, j0:j1, i0:i1] = 0.25 * ((f[:, 0::2, 0::2] + f[:, 0::2, 1::2]) + (f[:, 1::2, 0::2] + f[:, 1::2, 1::2]))
    return out


def dt(oc, of, Uc, Uf, box):
    Uf = fill(Uc, Uc, 0.0, Uf, box)
    return min(oc.dt_cfl(Uc), 2.0 * of.dt_cfl(Uf)), Uf


def step_flux(o, U, dt, k):
    """the oracle's split step (sweeps in the order of step k, then the
    plastic, reactive and geometric steps), keeping each sweep's face
    fluxes"""
    D = o.pb.ndim
    order = range(D) if k % 2 == 0 else reversed(range(D))
    fl = {}
    for d in order:
        U, fl[d] = o.sweep_flux(U, dt, d)
    U = o.plastic(U, dt)
    U = o.reaction(U, dt)
    U = o.geometric(U, dt)
    return U, fl


def step_flux_rk3(o, U, dt, stage_fill=None):
    """the oracle's SSP-RK3 step (its stages bit for bit), keeping the
    time-weighted face fluxes 1/6 F(q^n) + 1/6 F(q^(1)) + 2/3 F(q^(3)) whose
    difference is the step's conservative update; stage_fill(q, c) refills
    the ghost ring of a stage's input at the fraction c of the step (1 for
    q^(1), 1/2 for q^(3))"""
    qn = o._arr(U)
    R, F0 = o.rhs_flux(qn)
    q1 = qn - dt * R
    if stage_fill:
        q1 = stage_fill(q1, 1.0)
    R, F1 = o.rhs_flux(q1)
    q2 = q1 - dt * R
    q3 = 0.75 * qn + 0.25 * q2
    if stage_fill:
        q3 = stage_fill(q3, 0.5)
    R, F2 = o.rhs_flux(q3)
    q4 = q3 - dt * R
    out = (1.0 / 3.0) * qn + (2.0 / 3.0) * q4
    out = o.plastic(out, dt)
    out = o.reaction(out, dt)
    out = o.geometric(out, dt)
    fl = {d: (F0[d] / 6.0 + F1[d] / 6.0) + (2.0 / 3.0) * F2[d] for d in F0}
    return out, fl


def level_step(o, U, dt, k, rk3, Uc_old=None, Uc_new=None, box=None, s=0):
    """one step of a level keeping its fluxes: the split step, or the RK3 step
    whose stage inputs (for a patch: box, the level above's old and new
    states, substep s) take their ghost rings at the stage times"""
    if not rk3:
        return step_flux(o, U, dt, k)
    fill_ = None
    if box is not None:
        def fill_(q, c):
            return fill(Uc_old, Uc_new, 0.5 * (s + c), q, box)
    return step_flux_rk3(o, U, dt, fill_)


def reflux(Uc, fc, ff, box, dt, pbc):
    """flux correction of the coarse cells just outside the patch: on each
    coarse/fine face the coarse flux is replaced by the fine fluxes averaged
    over the face's two fine faces and the two fine steps, for the conserved
    components (partial densities, history slot, momentum, energy; the
    volume fractions and Vbar carry non-conservative terms and are left)"""
    from paper_2009_14555_amd import problems as P

    L = P.layout(pbc)
    cons = list(range(pbc.nmat - 1, L.V(0)))
    i0, j0, i1, j1 = box
    out = Uc.copy()
    lam_x = dt / pbc.dx[0]
    lam_y = dt / pbc.dx[1]
    js = np.arange(j0, j1)
    fj = G + 2 * (js - j0)
    for i_face, i_cell, sgn in ((i0, i0 - 1, -1.0), (i1, i1, 1.0)):
        fi = G + 2 * (i_face - i0)
        fb = 0.25 * ((ff[0][0][:, fj, fi] + ff[0][0][:, fj + 1, fi]) + (ff[1][0][:, fj, fi] + ff[1][0][:, fj + 1, fi]))
        out[cons, j0:j1, i_cell] = out[cons, j0:j1, i_cell] + sgn * (lam_x * (fb[cons] - fc[0][cons, j0:j1, i_face]))
    is_ = np.arange(i0, i1)
    fi = G + 2 * (is_ - i0)
    for j_face, j_cell, sgn in ((j0, j0 - 1, -1.0), (j1, j1, 1.0)):
        fjj = G + 2 * (j_face - j0)
        fb = 0.25 * ((ff[0][1][:, fjj, fi] + ff[0][1][:, fjj, fi + 1]) + (ff[1][1][:, fjj, fi] + ff[1][1][:, fjj, fi + 1]))
        out[cons, j_cell, i0:i1] = out[cons, j_cell, i0:i1] + sgn * (lam_y * (fb[cons] - fc[1][cons, j_face, i0:i1]))
    return out


def step(oc, of, Uc, Uf, box, dt_c, k, rk3=False):
    """one coarse step k of dt_c with two fine steps (2k, 2k + 1) of dt_c/2,
    averaging down and the flux correction (rk3: both levels step the SSP-RK3,
    the fine stage inputs refilled at their stage times)"""
    Uc_old = Uc
    Uc_new, fc = level_step(oc, Uc, dt_c, k, rk3)
    ff = []
    for s in (0, 1):
        Uf = fill(Uc_old, Uc_new, 0.5 * s, Uf, box)
        Uf, fl = level_step(of, Uf, 0.5 * dt_c, 2 * k + s, rk3, Uc_old, Uc_new, box, s)
        ff.append(fl)
    Uc = average_down(Uc_new, Uf, box)
    return reflux(Uc, fc, ff, box, dt_c, oc.pb), Uf


def separated(boxes):
    """True when no two patch boxes overlap or touch: a gap of at least one
    coarse cell between any two (every coarse cell a patch's flux correction
    writes is then outside every patch)"""
    for a in range(len(boxes)):
        for b in range(a + 1, len(boxes)):
            A_, B_ = boxes[a], boxes[b]
            if A_[0] <= B_[2] and B_[0] <= A_[2] and A_[1] <= B_[3] and B_[1] <= A_[3]:
                return False
    return True


def disjoint(boxes):
    """True when no two patch boxes share a coarse cell (they may touch)"""
    for a in range(len(boxes)):
        for b in range(a + 1, len(boxes)):
            A_, B_ = boxes[a], boxes[b]
            if A_[0] < B_[2] and B_[0] < A_[2] and A_[1] < B_[3] and B_[1] < A_[3]:
                return False
    return True


def exchange(Ufs, boxes):
    """fine-to-fine ghost exchange between the patches of one level: every
    stored cell of a patch grid inside another patch's interior takes that
    patch's value.  Patch p's stored cell (fj, fi) sits at the level's fine
    position (2 j0 + fj - G, 2 i0 + fi - G)."""
    out = [U.copy() for U in Ufs]
    for p, bp in enumerate(boxes):
        for q, bq in enumerate(boxes):
            if q == p:
                continue
            # fine positions in q's interior and in p's stored grid
            x0, x1 = max(2 * bq[0], 2 * bp[0] - G), min(2 * bq[2], 2 * bp[2] + G)
            y0, y1 = max(2 * bq[1], 2 * bp[1] - G), min(2 * bq[3], 2 * bp[3] + G)
            if x0 >= x1 or y0 >= y1:
                continue
            out[p][:, y0 - 2 * bp[1] + G:y1 - 2 * bp[1] + G, x0 - 2 * bp[0] + G:x1 - 2 * bp[0] + G] = \
                Ufs[q][:, y0 - 2 * bq[1] + G:y1 - 2 * bq[1] + G, x0 - 2 * bq[0] + G:x1 - 2 * bq[0] + G]
    return out


def cluster(tags, margin, n):
    """several patch boxes from the tags (a regrid into a level of several
    patches): the tagged cells dilated by margin cells (a square of side
    2 margin + 1 around each), the bounding box of each 8-connected component
    of that set, kept 3 cells inside the grid, then any two boxes that are not
    separated replaced by their union until all are; sorted by (j0, i0)"""
    ny, nx = tags.shape
    grown = np.zeros((ny, nx), dtype=bool)
    for j, i in zip(*np.nonzero(tags)):
        grown[max(j - margin, 0):j + margin + 1, max(i - margin, 0):i + margin + 1] = True
    seen = np.zeros((ny, nx), dtype=bool)
    boxes = []
    for j in range(ny):
        for i in range(nx):
            if not grown[j, i] or seen[j, i]:
                continue
            stack = [(j, i)]
            seen[j, i] = True
            i0, j0, i1, j1 = i, j, i + 1, j + 1
            while stack:
                cj, ci = stack.pop()
                i0, j0, i1, j1 = min(i0, ci), min(j0, cj), max(i1, ci + 1), max(j1, cj + 1)
                for dj in (-1, 0, 1):
                    for di in (-1, 0, 1):
                        qj, qi = cj + dj, ci + di
                        if 0 <= qj < ny and 0 <= qi < nx and grown[qj, qi] and not seen[qj, qi]:
                            seen[qj, qi] = True
                            stack.append((qj, qi))
            b = (max(i0, 3), max(j0, 3), min(i1, n[0] - 3), min(j1, n[1] - 3))
            if b[2] > b[0] and b[3] > b[1]:
                boxes.append(b)
    merged = True
    while merged:
        merged = False
        for a in range(len(boxes)):
            for b in range(a + 1, len(boxes)):
                if not separated([boxes[a], boxes[b]]):
                    A_, B_ = boxes[a], boxes[b]
                    boxes[a] = (min(A_[0], B_[0]), min(A_[1], B_[1]), max(A_[2], B_[2]), max(A_[3], B_[3]))
                    del boxes[b]
                    merged = True
                    break
            if merged:
                break
    return sorted(boxes, key=lambda b: (b[1], b[0]))


def dt_patches(oc, ofs, Uc, Ufs, boxes, rk3=False):
    """dt of a coarse grid with several patches: min(coarse CFL step, 2 x every
    patch's CFL step after its ghost fill and, with the split integrator, the
    exchange)"""
    assert disjoint(boxes)
    Ufs = [fill(Uc, Uc, 0.0, Uf, box) for Uf, box in zip(Ufs, boxes)]
    if not rk3:
        Ufs = exchange(Ufs, boxes)
    return min([oc.dt_cfl(Uc)] + [2.0 * of.dt_cfl(Uf) for of, Uf in zip(ofs, Ufs)]), Ufs


def step_patches(oc, ofs, Uc, Ufs, boxes, dt_c, k, rk3=False):
    """one coarse step k of dt_c with several patches on the fine level, each
    a grid of its own (disjoint boxes; touching ones step the split
    integrator only): per substep every patch takes its ghost ring from the
    coarse level, then (split integrator) the fine-to-fine exchange, then
    every patch steps; then every patch's coarse/fine faces are
    flux-corrected and all are averaged down"""
    assert disjoint(boxes)
    assert separated(boxes) or not rk3, "touching patches step the split integrator only"
    Uc_old = Uc
    Uc_new, fc = level_step(oc, Uc, dt_c, k, rk3)
    Ufs = list(Ufs)
    ffs = [[] for _ in boxes]
    for s in (0, 1):
        Ufs = [fill(Uc_old, Uc_new, 0.5 * s, Uf, box) for Uf, box in zip(Ufs, boxes)]
        if not rk3:
            Ufs = exchange(Ufs, boxes)
        for p, box in enumerate(boxes):
            Ufs[p], fl = level_step(ofs[p], Ufs[p], 0.5 * dt_c, 2 * k + s, rk3, Uc_old, Uc_new, box, s)
            ffs[p].append(fl)
    Uc = Uc_new
    for p, box in enumerate(boxes):
        Uc = reflux(Uc, fc, ffs[p], box, dt_c, oc.pb)
    for p, box in enumerate(boxes):
        Uc = average_down(Uc, Ufs[p], box)
    return Uc, Ufs


def dt_levels(os_, Us, boxes):
    """dt of level 0 for a stack of nested levels (level l + 1 refines
    boxes[l] of level l, each taking two steps per step of the level above):
    min over the levels of 2^l times the level's CFL step, each finer level
    after a ghost fill from the level above"""
    Us = list(Us)
    dts = [os_[0].dt_cfl(Us[0])]
    for l in range(1, len(Us)):
        Us[l] = fill(Us[l - 1], Us[l - 1], 0.0, Us[l], boxes[l - 1])
        dts.append(2.0 ** l * os_[l].dt_cfl(Us[l]))
    return min(dts), Us


def step_levels(os_, Us, boxes, dt_, k, l=0, rk3=False, above=None):
    """one step k of level l with dt_ and, recursively, two steps of each
    finer level per step of the level above (Berger-Colella over more than
    two levels): each level's ghost ring is filled from the level above at
    that level's old and new times, the level below is averaged down into it
    and its cells beside that level's patch are flux-corrected after its
    substeps.  Level l + 1 must lie at least G + 3 cells inside level l's
    grid for l >= 1 (its ghost fill then reads only level l's interior).
    Returns the new states and level l's sweep fluxes."""
    Us = list(Us)
    U_old = Us[l]
    if above is None:
        Us[l], fl = level_step(os_[l], Us[l], dt_, k, rk3)
    else:  # (the level above's old and new states, substep)
        Us[l], fl = level_step(os_[l], Us[l], dt_, k, rk3, above[0], above[1], boxes[l - 1], above[2])
    if l + 1 < len(Us):
        ff = []
        for s in (0, 1):
            Us[l + 1] = fill(U_old, Us[l], 0.5 * s, Us[l + 1], boxes[l])
            Us, fsub = step_levels(os_, Us, boxes, 0.5 * dt_, 2 * k + s, l + 1, rk3, (U_old, Us[l], s))
            ff.append(fsub)
        Us[l] = average_down(Us[l], Us[l + 1], boxes[l])
        Us[l] = reflux(Us[l], fl, ff, boxes[l], dt_, os_[l].pb)
    return Us, fl


class Patch:
    """a patch of a refinement tree: its box in the level above, the oracle
    of its grid, its state and its own (disjoint) patches"""

    def __init__(self, box, o, U, children=()):
        self.box, self.o, self.U, self.children = box, o, U, list(children)


def dt_tree(o, U, children, rk3=False):
    """dt of a tree's root level: min(the level's CFL step, 2 x every patch's
    dt, each patch after a ghost fill from the level above and, with the
    split integrator, the exchange among the patches)"""
    boxes = [ch.box for ch in children]
    assert disjoint(boxes)
    Us = [fill(U, U, 0.0, ch.U, ch.box) for ch in children]
    if not rk3:
        Us = exchange(Us, boxes)
    dts = [o.dt_cfl(U)]
    for ch, Uf in zip(children, Us):
        ch.U = Uf
        dts.append(2.0 * dt_tree(ch.o, ch.U, ch.children, rk3))
    return min(dts)


def step_tree(o, U, children, dt_, k, rk3=False, above=None):
    """one step k of a level and, recursively, of its patches (a refinement
    tree: a level of several disjoint patches, any of which is refined by
    patches of its own): per substep every patch's ghost fill from the
    level's old and new states, the exchange among the patches (split
    integrator), and every patch's own recursive step; then every patch corrected beside and
    averaged down.  above: (the level above's old and new states, this
    level's box, substep) for the RK3 stage refills.  Returns the level's new
    state and fluxes; the patches' states are updated in place."""
    boxes = [ch.box for ch in children]
    assert disjoint(boxes)
    assert separated(boxes) or not rk3, "touching patches step the split integrator only"
    U_old = U
    if above is None:
        U_new, fl = level_step(o, U, dt_, k, rk3)
    else:
        U_new, fl = level_step(o, U, dt_, k, rk3, *above)
    ffs = [[] for _ in children]
    for s in (0, 1):
        Us = [fill(U_old, U_new, 0.5 * s, ch.U, ch.box) for ch in children]
        if not rk3:
            Us = exchange(Us, boxes)
        for ch, Uf, ff in zip(children, Us, ffs):
            ch.U, fsub = step_tree(ch.o, Uf, ch.children, 0.5 * dt_, 2 * k + s, rk3, (U_old, U_new, ch.box, s))
            ff.append(fsub)
    for ch, ff in zip(children, ffs):
        U_new = reflux(U_new, fl, ff, ch.box, dt_, o.pb)
    for ch in children:
        U_new = average_down(U_new, ch.U, ch.box)
    return U_new, fl


def fine_problem(pbc, box):
    """the patch grid's problem: same physics, half the cell size, its low
    face at the patch's corner less the ghost layers"""
    ny, nx = fine_shape(box)
    dx = (pbc.dx[0] / 2, pbc.dx[1] / 2, pbc.dx[2])
    lo = (pbc.lo[0] + box[0] * pbc.dx[0] - G * dx[0], pbc.lo[1] + box[1] * pbc.dx[1] - G * dx[1], pbc.lo[2])
    from paper_2009_14555_amd import problems as P

    return pbc.replace(n=(nx, ny, 1), dx=dx, lo=lo, bc=(P.BC_TRANSMISSIVE,) * 3)


def prolong(Uc, box):
    """every fine cell of the patch grid takes its coarse parent's conserved
    state (a new or regridded patch: exactly conservative and no new states;
    the linear ghost-fill slopes, applied to a whole diffuse interface, build
    mixed cells whose phasic densities are far from either parent's and on
    which two round-off-different implementations part at ~1e-6)"""
    ny, nx = fine_shape(box)
    return fill(Uc, Uc, 0.0, np.zeros((Uc.shape[0], ny, nx)), box, every=True)


def tag(pb, W, threshold):
    """Sec. 4.2 refinement criterion on a 2-D primitive state W (F, ny, nx):
    a cell is tagged when a refinement variable (the stored volume
    fractions, phi_l rho_l of every material, u_x, u_y, p) changes to a face
    neighbour inside the grid by more than threshold as a fraction,
    |q_n - q_c| > threshold max(|q_c|, |q_n|, floor), the floor 1e-6 times
    the van Albada scale of the variable's kind.  Returns the tags and the
    tagged extent (i0, j0, i1, j1), all 0 when none."""
    from paper_2009_14555_amd import problems as P

    L = P.layout(pb)
    N = pb.nmat
    sc = pb.va_scale
    phis = [W[L.phi(l)] for l in range(N - 1)]
    s = np.zeros_like(W[0])
    for p_ in phis:
        s = s + p_
    phi_all = phis + [1.0 - s]
    vars_ = [(p_, 1e-6 * sc[0]) for p_ in phis]
    vars_ += [(phi_all[l] * W[L.rho(l)], 1e-6 * sc[1]) for l in range(N)]
    vars_ += [(W[L.u(d)], 1e-6 * sc[3]) for d in range(2)]
    vars_ += [(W[L.p], 1e-6 * sc[4])]
    ny, nx = W.shape[1:]
    tags = np.zeros((ny, nx), dtype=bool)
    for q, fl in vars_:
        def jump(a, b):
            return np.abs(b - a) > threshold * np.maximum(np.maximum(np.abs(a), np.abs(b)), fl)
        jx = jump(q[:, :-1], q[:, 1:])  # between (j, i) and (j, i + 1)
        jy = jump(q[:-1, :], q[1:, :])
        tags[:, :-1] |= jx
        tags[:, 1:] |= jx
        tags[:-1, :] |= jy
        tags[1:, :] |= jy
    if not tags.any():
        return tags, (0, 0, 0, 0)
    jj, ii = np.nonzero(tags)
    return tags, (int(ii.min()), int(jj.min()), int(ii.max()) + 1, int(jj.max()) + 1)


def regrid_box(bbox, margin, n):
    """the patch over the tagged extent padded by margin coarse cells, kept 3
    cells inside the grid; None when nothing is tagged"""
    if bbox[2] <= bbox[0]:
        return None
    i0 = max(bbox[0] - margin, 3)
    j0 = max(bbox[1] - margin, 3)
    i1 = min(bbox[2] + margin, n[0] - 3)
    j1 = min(bbox[3] + margin, n[1] - 3)
    if i1 <= i0 or j1 <= j0:
        return None
    return (i0, j0, i1, j1)
