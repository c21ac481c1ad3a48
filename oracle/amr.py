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
* no flux correction at the coarse/fine faces (the paper names none), so
  conservation holds on each level but not across that boundary;
* dt = min(coarse CFL step, 2 x fine CFL step), the fine one over the whole
  patch grid after a ghost fill with the coarse state.
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


def fill(Uc_old, Uc_new, w, Uf, box):
    """fine ghost cells from the coarse level at weight w in time, linear
    with limited slopes inside each coarse parent"""
    J, I = parents(box)
    ny, nx = fine_shape(box)
    ghost = ~interior_mask(box)
    Jg, Ig = J[ghost], I[ghost]
    # the fine cell's offset from its parent's centre, in coarse cells
    fj, fi = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ox = np.where((fi[ghost] - G) % 2 == 0, -0.25, 0.25)
    oy = np.where((fj[ghost] - G) % 2 == 0, -0.25, 0.25)

    def at(dj, di):
        old = Uc_old[:, Jg + dj, Ig + di]
        return old + w * (Uc_new[:, Jg + dj, Ig + di] - old)

    c = at(0, 0)
    sx = minmod(c - at(0, -1), at(0, 1) - c)
    sy = minmod(c - at(-1, 0), at(1, 0) - c)
    out = Uf.copy()
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


def step(oc, of, Uc, Uf, box, dt_c, k):
    """one coarse step k of dt_c with two fine steps (2k, 2k + 1) of dt_c/2"""
    Uc_old = Uc
    Uc_new = oc.step(Uc, dt_c, k)
    for s in (0, 1):
        Uf = fill(Uc_old, Uc_new, 0.5 * s, Uf, box)
        Uf = of.step(Uf, 0.5 * dt_c, 2 * k + s)
    return average_down(Uc_new, Uf, box), Uf


def fine_problem(pbc, box):
    """the patch grid's problem: same physics, half the cell size, its low
    face at the patch's corner less the ghost layers"""
    ny, nx = fine_shape(box)
    dx = (pbc.dx[0] / 2, pbc.dx[1] / 2, pbc.dx[2])
    lo = (pbc.lo[0] + box[0] * pbc.dx[0] - G * dx[0], pbc.lo[1] + box[1] * pbc.dx[1] - G * dx[1], pbc.lo[2])
    from paper_2009_14555_amd import problems as P

    return pbc.replace(n=(nx, ny, 1), dx=dx, lo=lo, bc=(P.BC_TRANSMISSIVE,) * 3)
