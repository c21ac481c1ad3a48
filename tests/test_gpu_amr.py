"""Two-level subcycled refinement (Sec. 3; the readings are stated in
oracle/amr.py) on the GPU against the oracle's driver over its single-grid
step, element by element on both levels (<= 1e-10 per stored field): a
shock crossing a patch over the elastoplastic disc, a smooth wave crossing a
patch, and an LX-17 rate stick refined around its booster; the GPU's dt
against the oracle's; and the entry point's error paths."""
import ctypes as C

import numpy as np
import pytest

from oracle import amr as A
from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P
from tests.parity_util import TOL, assert_parity, to_np
from tests.test_oracle_amr import prolong_prim, wave_setup

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
    pbc, W = P.rate_stick(60, 150, seed=4)
    box = (12, 6, 48, 24)  # the strip and its booster's end
    pbf = A.fine_problem(pbc, box)
    out["rate_stick"] = (pbc, W, pbf, prolong_prim(pbc, W, pbf, box)[0], box, 8)
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
    h.close()
