"""Reflective boundaries and the cylindrical form (Sec. 3: the geometric
source s_g, x = r, the reflective axis) on the GPU against the oracle,
element by element (<= 1e-10 per stored field): a 1-D two-gas slab against a
wall, a 2-D disc cut by the axis (THINC), a 3-D ball cut by a wall and a 3-D
reactive box between walls, thin and ragged 1-D/2-D/3-D grids between walls,
homologous cylindrical expansion of
a gas and of an elastic solid, the cylindrical LX-17 rate stick (split and
RK3), the device-CFL and graph paths against host-dt steps, the 400 x 2000
cylindrical rate stick; and the entry point's error paths."""
import dataclasses

import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P
from tests.parity_util import TOL, assert_parity, to_np
from tests.test_oracle_cyl import ball_3d, disc_2d, homologous, slab_1d

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
    out["wall_1d"] = slab_1d(60, 0.0, 1.0, P.BC_REFLECTIVE)
    out["axis_disc_2d"] = disc_2d(24, 32, 0.0, P.BC_AXIS)
    pb, W, _ = homologous(40, 0.5)
    out["homologous_gas"] = (pb, W)
    pb, W, _ = homologous(40, 1000.0, solid=True)
    out["homologous_solid"] = (pb, W)
    out["stick_cyl"] = P.rate_stick_cyl(40, 100, seed=3)
    # 3-D: a ball cut by a wall at x = 0, walls at both ends of y and z
    out["ball_3d_walls"] = ball_3d(12, 18, 14, 0.0, (P.BC_AXIS, P.BC_REFLECTIVE, P.BC_REFLECTIVE))
    # 3-D reactive mixture and solid slab between walls (x and z), y periodic;
    # the rate constant scaled with the cell size, as the 24^3 parity case
    pb, W = P.reactive_slab(20, seed=5)
    pb.reactive.k *= 20.0 / 256.0
    out["reactive_box_walls"] = (dataclasses.replace(pb, bc=(P.BC_REFLECTIVE, P.BC_PERIODIC, P.BC_REFLECTIVE)), W)
    return out


CONFIGS = configs()


@pytest.mark.parametrize("integrator", ["split", "rk3"])
@pytest.mark.parametrize("name", list(CONFIGS))
def test_cyl_steps_match_oracle(solver, name, integrator):
    pb, W = CONFIGS[name]
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    g = solver.Grid(pb)
    g.set_primitive(W)
    g.set_integrator(integrator)
    for k in range(10):
        dt = o.dt_cfl(U)
        U = o.step_rk3(U, dt) if integrator == "rk3" else o.step(U, dt, k)
        g.advance(dt)
    assert np.all(np.isfinite(U))
    assert_parity(to_np(g.state), U, TOL, f"{name} {integrator}", P.layout(pb))
    np.testing.assert_allclose(g.max_wavespeed(), o.max_wavespeed(U), rtol=1e-10)


def test_cyl_device_cfl_and_graph_match_host_steps(solver):
    import torch

    pb, W = CONFIGS["stick_cyl"]
    S = solver
    ref = S.Grid(pb)
    ref.set_primitive(W)
    for _ in range(5):
        ref.advance(ref.dt_cfl())
    a = S.Grid(pb)
    a.set_primitive(W)
    a.advance_cfl(5)
    b = S.Grid(pb)
    b.set_primitive(W)
    b.advance_graph(5)
    torch.cuda.synchronize()
    r = to_np(ref.state)
    assert np.array_equal(to_np(a.state), r)
    assert np.array_equal(to_np(b.state), r)


def test_rate_stick_cyl_full_size(solver):
    """400 x 2000, the benchmark's launch configuration: two steps against the
    oracle on every cell"""
    pb, W = P.rate_stick_cyl()
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    g = solver.Grid(pb)
    g.set_primitive(W)
    for k in range(2):
        dt = o.dt_cfl(U)
        U = o.step(U, dt, k)
        g.advance(dt)
    assert_parity(to_np(g.state), U, TOL, "rate_stick_cyl 400x2000", P.layout(pb))


def test_cyl_entry_point_errors(solver):
    import ctypes as C

    import torch

    from paper_2009_14555_amd import dimp as D

    pb, W = CONFIGS["axis_disc_2d"]
    g = solver.Grid(pb)
    g.set_primitive(W)
    with pytest.raises(D.DimpError):
        D.call("dimp_set_geometry", g.h, 5, 0.0)
    with pytest.raises(D.DimpError):
        D.call("dimp_set_geometry", g.h, 1, -1.0)
    D.call("dimp_set_geometry", g.h, 1, 0.0)
    lam = torch.zeros_like(g.state)
    dp = torch.zeros(12, dtype=torch.float64, device=g.state.device)
    with pytest.raises(D.DimpError):  # the adjoint is built for Cartesian grids and open boundaries
        g.adjoint_step(g.state.clone(), lam, 1e-9, 0, dp)
    pb3 = P.Problem(ndim=3, n=(4, 4, 4), dx=(0.25,) * 3, materials=[P.water_sg(), P.solid_c2()])
    g3 = solver.Grid(pb3)
    with pytest.raises(D.DimpError):
        D.call("dimp_set_geometry", g3.h, 1, 0.0)
    h = C.c_void_p()
    with pytest.raises(D.DimpError):
        D.call("dimp_create_grid", 2, (C.c_int64 * 3)(4, 4, 1), (C.c_double * 3)(1.0, 1.0, 1.0),
               (C.c_int32 * 3)(7, 0, 0), C.byref(h))
    # reflective rules on a 3-D grid are accepted (and stepped by the tests above)
    D.call("dimp_create_grid", 3, (C.c_int64 * 3)(4, 4, 4), (C.c_double * 3)(1.0, 1.0, 1.0),
           (C.c_int32 * 3)(2, 3, 2), C.byref(h))
    D.call("dimp_destroy", h)


@pytest.mark.parametrize("n,bcx", [((1,), P.BC_REFLECTIVE), ((2,), P.BC_AXIS), ((5,), P.BC_REFLECTIVE),
                                   ((1, 3), P.BC_AXIS), ((3, 2), P.BC_REFLECTIVE), ((61, 7), P.BC_AXIS),
                                   ((2, 59), P.BC_REFLECTIVE), ((1, 3, 2), P.BC_REFLECTIVE),
                                   ((5, 2, 7), P.BC_AXIS), ((61, 3, 4), P.BC_REFLECTIVE),
                                   ((3, 4, 59), P.BC_AXIS)])
def test_wall_edge_sizes(solver, n, bcx):
    """grids thinner than the stencil (mirror then clamp), a row of one
    segment plus a ragged tail, both integrators"""
    ndim = len(n)
    nn = tuple(list(n) + [1] * (3 - ndim))
    bc = (bcx, P.BC_REFLECTIVE if ndim > 1 else 0, P.BC_REFLECTIVE if ndim > 2 else 0)
    pb = P.Problem(ndim=ndim, n=nn, dx=tuple([1.0 / max(nn)] * 3), bc=bc, materials=[P.water_sg(), P.solid_c2()],
                   thinc=1, cfl=0.5)
    W = P.random_smooth_state(pb, seed=sum(n), solid_strain=2e-3)
    o = O.Oracle(pb)
    for integrator in ("split", "rk3"):
        U = o.prim_to_cons(W)
        g = solver.Grid(pb)
        g.set_primitive(W)
        g.set_integrator(integrator)
        for k in range(3):
            dt = o.dt_cfl(U)
            U = o.step_rk3(U, dt) if integrator == "rk3" else o.step(U, dt, k)
            g.advance(dt)
        # a single cell between two walls keeps round-off momentum only:
        # momentum is compared on the acoustic scale (as for patch sets)
        assert_parity(to_np(g.state), U, TOL, f"n={n} {integrator}", P.layout(pb), acoustic_floor=True)


@pytest.mark.parametrize("nr", [1, 2, 3, 7])
def test_cylindrical_thin_grids(solver, nr):
    pb, W = P.rate_stick_cyl(nr, 24, seed=nr)
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    g = solver.Grid(pb)
    g.set_primitive(W)
    for k in range(4):
        dt = o.dt_cfl(U)
        U = o.step(U, dt, k)
        g.advance(dt)
    assert_parity(to_np(g.state), U, TOL, f"nr={nr}", P.layout(pb), acoustic_floor=True)
