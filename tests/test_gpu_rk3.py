"""The unsplit SSP-RK3 integrator (Sec. 3.1) on the GPU against the oracle's
or_step_rk3, element by element (max relative difference <= 1e-10 per
stored field), on 1-D, 2-D and 3-D inputs with ragged sizes, over several
steps; the device-CFL and graph paths against the host-dt path; the full
2048^2 workload; and the error paths of the entry point."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P
from tests.parity_util import TOL, assert_parity, to_np

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
    out["sod_130"] = P.sod_two_gamma(130, thinc=True)
    pb, W = P.shock_disc(96, seed=3)
    out["shock_disc_96"] = (pb, W)
    pb = P.Problem(ndim=2, n=(70, 45, 1), dx=(1 / 70, 1 / 45, 1), bc=(P.BC_PERIODIC,) * 3,
                   materials=[P.water_sg(), P.solid_c2()], thinc=1, limiter=P.LIM_VANALBADA, cfl=0.5)
    out["strained_2d_va"] = (pb, P.random_smooth_state(pb, seed=6, solid_strain=3e-3))
    pb, W = P.reactive_slab(14, seed=1, noise=0.01)
    out["reactive_14"] = (pb, W)
    pb = P.Problem(ndim=3, n=(13, 11, 9), dx=(1 / 13, 1 / 11, 1 / 9), bc=(P.BC_PERIODIC,) * 3,
                   materials=[P.water_sg(), P.solid_c2()], thinc=1, cfl=0.5)
    out["strained_3d"] = (pb, P.random_smooth_state(pb, seed=5, solid_strain=3e-3))
    return out


CONFIGS = configs()


def pair(S, pb, W):
    o = O.Oracle(pb)
    g = S.Grid(pb)
    g.set_primitive(W)
    g.set_integrator("rk3")
    return o, o.prim_to_cons(W), g


@pytest.mark.parametrize("name", list(CONFIGS))
def test_rk3_steps_match_oracle(solver, name):
    pb, W = CONFIGS[name]
    o, U, g = pair(solver, pb, W)
    cur = g.current()
    for k in range(6):
        dt = o.dt_cfl(U)
        U = o.step_rk3(U, dt)
        g.advance(dt)
        assert_parity(to_np(g.state), U, TOL, f"{name} step {k}", P.layout(pb))
    assert g.current() == cur  # the RK3 step keeps the state in its buffer
    np.testing.assert_allclose(g.max_wavespeed(), o.max_wavespeed(U), rtol=1e-10)


@pytest.mark.parametrize("n", [(1,), (3,), (1, 1), (3, 2), (59, 17), (2, 33), (4, 3, 2), (17, 5, 9)])
def test_rk3_edge_sizes(solver, n):
    ndim = len(n)
    nn = tuple(list(n) + [1] * (3 - ndim))
    pb = P.Problem(ndim=ndim, n=nn, dx=tuple([1.0 / max(nn)] * 3), materials=[P.water_sg(), P.solid_c2()],
                   thinc=1, cfl=0.5)
    W = P.random_smooth_state(pb, seed=sum(n), solid_strain=2e-3)
    o, U, g = pair(solver, pb, W)
    for _ in range(3):
        dt = o.dt_cfl(U)
        U = o.step_rk3(U, dt)
        g.advance(dt)
    assert_parity(to_np(g.state), U, TOL, f"n={n}", P.layout(pb))


def test_rk3_device_cfl_and_graph_match_host_steps(solver):
    """advance_cfl (dt on the device) and advance_graph (pairs of steps from a
    captured graph) give the host-dt result bit for bit"""
    import torch

    pb, W = CONFIGS["shock_disc_96"]
    S = solver
    ref = S.Grid(pb)
    ref.set_primitive(W)
    ref.set_integrator("rk3")
    for _ in range(5):
        ref.advance(ref.dt_cfl())
    a = S.Grid(pb)
    a.set_primitive(W)
    a.set_integrator("rk3")
    a.advance_cfl(5)
    b = S.Grid(pb)
    b.set_primitive(W)
    b.set_integrator("rk3")
    b.advance_graph(5)
    torch.cuda.synchronize()
    r = to_np(ref.state)
    assert np.array_equal(to_np(a.state), r)
    assert np.array_equal(to_np(b.state), r)
    b.advance_graph(4)  # replays of the captured graph
    a.advance_cfl(4)
    assert np.array_equal(to_np(b.state), to_np(a.state))


def test_rk3_full_size_shock_disc_one_step(solver):
    """2048^2, the benchmark's launch configuration: one RK3 step against the
    oracle on every cell"""
    pb, W = P.shock_disc(2048, seed=0)
    o, U, g = pair(solver, pb, W)
    dt = o.dt_cfl(U)
    U = o.step_rk3(U, dt)
    g.advance(dt)
    assert_parity(to_np(g.state), U, TOL, "shock_disc 2048 rk3", P.layout(pb))


def test_rk3_conservation(solver):
    import torch

    pb = P.Problem(ndim=2, n=(160, 144, 1), dx=(1 / 160, 1 / 144, 1), bc=(P.BC_PERIODIC,) * 3,
                   materials=[P.water_sg(), P.solid_c2()], thinc=1, cfl=0.5)
    W = P.random_smooth_state(pb, seed=9, solid_strain=2e-3)
    g = solver.Grid(pb)
    g.set_primitive(W)
    g.set_integrator("rk3")
    L = P.layout(pb)
    idx = [L.m(0), L.m(1), L.mom(0), L.mom(1), L.E]
    before = [float(torch.sum(g.state[f]).item()) for f in idx]
    scale = [float(torch.sum(torch.abs(g.state[f])).item()) for f in idx]
    g.advance_cfl(10)
    after = [float(torch.sum(g.state[f]).item()) for f in idx]
    for a, b, s in zip(before, after, scale):
        assert abs(a - b) <= 1e-13 * s


def test_rk3_entry_point_errors(solver):
    from paper_2009_14555_amd import dimp as D

    pb, W = CONFIGS["strained_2d_va"]
    g = solver.Grid(pb)
    g.set_primitive(W)
    with pytest.raises(ValueError):
        g.set_integrator("rk4")
    with pytest.raises(D.DimpError):
        D.call("dimp_set_integrator", g.h, 7)
    g.set_integrator("rk3")
    import torch

    lam = torch.zeros_like(g.state)
    dp = torch.zeros(12, dtype=torch.float64, device=g.state.device)
    with pytest.raises(D.DimpError):  # the adjoint reverses the split integrator only
        g.adjoint_step(g.state.clone(), lam, 1e-9, 0, dp)
    g.set_integrator("split")
    g.adjoint_step(g.state.clone(), lam, 1e-9, 0, dp)
    tmpl, sizes, prims = P.patch_set(4, seed=0)
    ps = solver.PatchSet(tmpl, sizes)
    with pytest.raises(D.DimpError):
        D.call("dimp_set_integrator", ps.h, 1)
