"""Every reverse stage of the adjoint against central differences of its own
forward stage, case by case, on states sampled from a smooth periodic
two-material field and from a plate impact (see tests/adjoint_units.hip)."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2009_14555_amd import problems as P
from tests.parity_util import to_np

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
STAGES = {"c2p": 0, "side": 1, "stress": 2, "face": 3, "star": 4, "edges": 5, "update": 6, "plastic": 7}


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_14555_amd import dimp as D
    from paper_2009_14555_amd import solver as S

    lib = C.CDLL(os.path.join(HERE, "libdimp_adjunits.so"))
    lib.unit_run.restype = C.c_int
    lib.unit_sizes.restype = C.c_int
    states = []
    n = (40, 36)
    pb = P.Problem(ndim=2, n=(n[0], n[1], 1), dx=(1 / n[0], 1 / n[1], 1), bc=(P.BC_PERIODIC,) * 3,
                   materials=[P.water_sg(), P.solid_c2()], thinc=0, limiter=P.LIM_VANALBADA)
    g = S.Grid(pb)
    g.set_primitive(P.random_smooth_state(pb, seed=6, solid_strain=3e-3))
    states.append((pb, to_np(g.state).copy(), to_np(g.primitive()).copy()))
    pb2, W2 = P.plate_impact(48)
    g2 = S.Grid(pb2)
    g2.set_primitive(W2)
    g2.advance_cfl(12)
    states.append((pb2.replace(thinc=0), to_np(g2.state).copy(), to_np(g2.primitive()).copy()))
    return lib, D, states


def scale_of(x, phi_cols=()):
    s = np.abs(x) + 1e-3 * np.abs(x).max(axis=0, keepdims=True) + 1e-300
    for c in phi_cols:
        s[:, c] = np.minimum(x[:, c], 1.0 - x[:, c])
    return s


def inputs(stage, d, U, W, rng, ncase):
    F = U.shape[0]
    Uc = U.reshape(F, *U.shape[1:])
    cells = [(int(rng.integers(1, Uc.shape[1] - 1)), int(rng.integers(1, Uc.shape[2] - 1))) for _ in range(ncase)]

    def w_at(j, i):
        return W[:, j, i]

    def nb(j, i, s):
        return (j, i + s) if d == 0 else (j + s, i)

    X, phi_cols = [], [0]
    for (j, i) in cells:
        if stage == "c2p" or stage == "plastic":
            X.append(U[:, j, i])
        elif stage in ("side", "stress"):
            X.append(w_at(j, i))
        elif stage == "face":
            X.append(np.concatenate([w_at(j, i), w_at(*nb(j, i, 1))]))
            phi_cols = [0, F]
        elif stage == "edges":
            Wm, W0, Wp = w_at(*nb(j, i, -1)), w_at(j, i), w_at(*nb(j, i, 1))
            r = W0[1] * W0[0] + W0[2] * (1 - W0[0])
            X.append(np.concatenate([Wm, W0, Wp, [1.0 / r, 2.2e9]]))
            phi_cols = [0, F, 2 * F]
        elif stage == "star":
            w = w_at(j, i)
            un = w[3 + d]
            rho = w[1] * w[0] + w[2] * (1 - w[0])
            side = [rho, 1e9, 2500.0, w[3], w[4], -w[5], 3e7, 0.0]
            SK = un - 2500.0
            ust = [un + 10.0, w[4 - d] + 5.0]
            X.append(np.concatenate([w, side, [SK, SK - un, 1.0 / (SK - ust[d]), ust[0], ust[1], rho * (SK - un)]]))
        elif stage == "update":
            u = U[:, j, i]
            fa = np.concatenate([u * 50.0, [40.0, 1.0, 0.01]])
            fb = fa * (1.0 + 0.01 * rng.standard_normal(fa.shape))
            X.append(np.concatenate([u, [1.0 / (u[1] + u[2])], fa, fb]))
    X = np.array(X)
    return X, scale_of(X, phi_cols)


def run_stage(lib, D, pb, stage, d, X, V, WY, eps):
    mats = (D.dimp_material * 2)(*[D.material(m) for m in pb.materials])
    opt = D.options(pb)
    dx = (C.c_double * 2)(pb.dx[0], pb.dx[1])
    out = np.zeros(2 * X.shape[0])
    Xc, Vc, Wc = (np.ascontiguousarray(a, dtype=np.float64) for a in (X, V, WY))
    P_ = C.POINTER(C.c_double)
    rc = lib.unit_run(STAGES[stage], d, mats, C.byref(opt), dx, C.c_double(0.3), X.shape[0], Xc.ctypes.data_as(P_),
                      Vc.ctypes.data_as(P_), Wc.ctypes.data_as(P_), C.c_double(eps), out.ctypes.data_as(P_))
    assert rc == 0
    fd, ad = out[0::2], out[1::2]
    return np.abs(fd - ad) / np.maximum(np.maximum(np.abs(fd), np.abs(ad)), 1e-300)


@pytest.mark.parametrize("stage", list(STAGES))
@pytest.mark.parametrize("d", [0, 1])
def test_stage_against_finite_differences(env, stage, d):
    """per case |fd - adjoint| / max(|fd|, |adjoint|); a central difference
    is limited by truncation at large steps (the van Albada limiter turns on
    the scale of its small epsilon) and by round-off at small ones, so each
    stage is judged at the better of two steps: its median error must be
    round-off sized and nine cases in ten must agree to 1e-3"""
    lib, D, states = env
    ni, no = C.c_int(), C.c_int()
    assert lib.unit_sizes(STAGES[stage], C.byref(ni), C.byref(no)) == 0
    for si, (pb, U, W) in enumerate(states):
        rng = np.random.default_rng(100 + si)
        X, sc = inputs(stage, d, U, W, rng, 400)
        assert X.shape[1] == ni.value, (stage, X.shape, ni.value)
        V = rng.standard_normal(X.shape) * sc
        WY = rng.standard_normal((X.shape[0], no.value))
        best = None
        for eps in (1e-7, 1e-9):
            rel = run_stage(lib, D, pb, stage, d, X, V, WY, eps)
            q = (np.median(rel), np.quantile(rel, 0.9))
            print(f"{stage} dir {d} state {si} eps {eps:.0e}: median {q[0]:.1e} p90 {q[1]:.1e} max {rel.max():.1e}",
                  flush=True)
            best = q if best is None or q[0] < best[0] else best
        assert best[0] < 1e-5 and best[1] < 1e-3, (stage, d, si, best)
