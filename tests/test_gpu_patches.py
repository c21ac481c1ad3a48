"""Batched patch sets on the GPU: identical bits to per-patch launches and to
graph replay, parity of every sampled patch with the oracle run on that patch
as an independent grid, ghost layers holding the boundary images."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P
from tests.parity_util import TOL, assert_parity, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_14555_amd import solver

    return solver


def small_set(npatch=48, seed=3):
    tmpl, sizes, prims = P.patch_set(npatch, seed=seed, dx=1.0 / 256)
    return tmpl, sizes, prims


def oracle_dt(tmpl, sizes, Us):
    """global dt: CFL over every patch, from the oracle"""
    s = np.zeros(2)
    for (nx, ny), U in zip(sizes, Us):
        o = O.Oracle(tmpl.replace(n=(int(nx), int(ny), 1)))
        s = np.maximum(s, o.max_wavespeed(U))
    return tmpl.cfl * min(tmpl.dx[0] / s[0], tmpl.dx[1] / s[1])


def test_batched_equals_per_patch_launches_bitwise(S):
    tmpl, sizes, prims = small_set()
    a = S.PatchSet(tmpl, sizes)
    b = S.PatchSet(tmpl, sizes)
    a.set_primitive(prims)
    b.set_primitive(prims)
    b.set_launch(per_patch=True)
    a.advance_cfl(5)
    b.advance_cfl(5)
    assert np.array_equal(to_np(a.state), to_np(b.state))


def test_graph_replay_equals_stream_launches_bitwise(S):
    tmpl, sizes, prims = small_set(32, seed=5)
    a = S.PatchSet(tmpl, sizes)
    b = S.PatchSet(tmpl, sizes)
    a.set_primitive(prims)
    b.set_primitive(prims)
    a.advance_graph(7)
    b.advance_cfl(7)
    assert np.array_equal(to_np(a.state), to_np(b.state))
    a.advance_graph(6)  # replays the cached graph
    b.advance_cfl(6)
    assert np.array_equal(to_np(a.state), to_np(b.state))


@pytest.mark.parametrize("cfg", [(1, 4), (2, 8), (4, 8)])
def test_launch_shape_does_not_change_bits(S, cfg):
    tmpl, sizes, prims = small_set(40, seed=7)
    a = S.PatchSet(tmpl, sizes)
    b = S.PatchSet(tmpl, sizes)
    a.set_primitive(prims)
    b.set_primitive(prims)
    b.set_launch(False, *cfg)
    a.advance_cfl(4)
    b.advance_cfl(4)
    assert np.array_equal(to_np(a.state), to_np(b.state))


def test_patches_match_oracle_and_ghosts_are_boundary_images(S):
    tmpl, sizes, prims = small_set(24, seed=11)
    ps = S.PatchSet(tmpl, sizes)
    ps.set_primitive(prims)
    Us = [O.Oracle(tmpl.replace(n=(int(nx), int(ny), 1))).prim_to_cons(W) for (nx, ny), W in zip(sizes, prims)]
    L = P.layout(tmpl)
    for k in range(4):
        dt = oracle_dt(tmpl, sizes, Us)
        Us = [O.Oracle(tmpl.replace(n=(int(nx), int(ny), 1))).step(U, dt, k) for (nx, ny), U in zip(sizes, Us)]
        ps.advance(dt)
    for p in range(len(sizes)):
        G = to_np(ps.patch(p))
        # patches the shock does not cross hold round-off momentum only:
        # momentum is measured against the acoustic scale there
        assert_parity(G[:, 2:-2, 2:-2], Us[p], TOL, f"patch {p}", L, acoustic_floor=True)
        edge = np.pad(G[:, 2:-2, 2:-2], ((0, 0), (2, 2), (2, 2)), mode="edge")
        assert np.array_equal(G, edge), f"ghost layers of patch {p}"


def test_autotune_restores_state_and_picks_a_shape(S):
    tmpl, sizes, prims = small_set(64, seed=2)
    ps = S.PatchSet(tmpl, sizes)
    ps.set_primitive(prims)
    before = to_np(ps.state).copy()
    best = ps.autotune(1)
    assert best[0] in (1, 2, 4) and best[1] in (4, 8)
    assert np.array_equal(to_np(ps.state), before)


def test_graph_on_plain_grid_equals_stream_launches(S):
    pb, W = P.shock_disc(96, seed=1)
    a = S.Grid(pb)
    b = S.Grid(pb)
    a.set_primitive(W)
    b.set_primitive(W)
    a.advance_graph(9)
    b.advance_cfl(9)
    assert np.array_equal(to_np(a.state), to_np(b.state))
