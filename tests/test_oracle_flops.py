"""The oracle's operation-counting step (the algorithmic FLOP figure of the
step's roofline): values bit for bit those of the plain step, the counting
rules on fixed expressions, per-line counts affine in the line length, and
the structural-zero rule seen on a real stage (a 1-D sweep costs less than a
2-D one with the same physics)."""
import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P


def test_counting_rules():
    got = O.flops_selftest()
    want = np.array([[2, 1, 1, 1, 0, 0],   # (a + b) * c / d - sqrt(e)
                     [0, 0, 0, 0, 0, 0],   # 0 * a + b, a - 0, 0 / a, -(0 - a)
                     [1, 0, 0, 0, 2, 2]])  # exp(a) + tanh(b), a < b, max(a, b)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("case", ["sod", "disc", "slab"])
def test_counting_step_is_the_plain_step(case):
    if case == "sod":
        pb, W = P.sod_two_gamma(64, thinc=True)
    elif case == "disc":
        pb, W = P.shock_disc(40, seed=2)
    else:
        pb, W = P.reactive_slab(10, seed=1)
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    dt = o.dt_cfl(U)
    for k in range(2):
        U1 = o.step(U, dt, k)
        U2, cnt = o.step_flops(U, dt, k)
        np.testing.assert_array_equal(U1, U2)
        assert cnt.shape == (pb.ndim + 2, 6) and np.all(cnt >= 0)
        U = U1


def uniform_1d(n):
    pb = P.Problem(ndim=1, n=(n, 1, 1), dx=(1.0 / n, 1.0, 1.0), materials=[P.water_sg(), P.solid_c2()],
                   thinc=0, cfl=0.5)
    L = P.layout(pb)
    W = P.blank_prim(pb)
    W[L.phi(0)] = 0.4
    W[L.rho(0)] = 1000.0
    W[L.rho(1)] = 2700.0
    W[L.u(0)] = 10.0
    W[L.p] = 1e8
    return pb, W


def test_sweep_counts_affine_in_line_length():
    """a uniform state takes the same branches everywhere, and a line of n
    cells does its per-cell stages on n + const cells: the sweep count is
    exactly affine in n"""
    c = []
    for n in (8, 16, 24):
        pb, W = uniform_1d(n)
        o = O.Oracle(pb)
        U = o.prim_to_cons(W)
        _, cnt = o.step_flops(U, 1e-7, 0)
        c.append(cnt)
        # the pointwise phases are exactly proportional to n
        np.testing.assert_array_equal(cnt[1:] / n, c[0][1:] / 8)
    np.testing.assert_array_equal(c[2][0] - c[1][0], c[1][0] - c[0][0])


def test_structural_zeros_not_counted():
    """the same physics in 1-D and 2-D: both run the oracle's full 3x3
    tensor algebra, but in 1-D the stretch tensor is diagonal (its six
    off-diagonal entries are the constant 0) and there is one momentum, so
    the counted sweep work per cell is well below the 2-D one (0.77 of it
    for this state)"""
    pb1, W1 = uniform_1d(32)
    o1 = O.Oracle(pb1)
    _, c1 = o1.step_flops(o1.prim_to_cons(W1), 1e-7, 0)
    pb2 = P.Problem(ndim=2, n=(32, 32, 1), dx=(1 / 32, 1 / 32, 1.0), materials=[P.water_sg(), P.solid_c2()],
                    thinc=0, cfl=0.5)
    L = P.layout(pb2)
    W2 = P.blank_prim(pb2)
    W2[L.phi(0)] = 0.4
    W2[L.rho(0)] = 1000.0
    W2[L.rho(1)] = 2700.0
    W2[L.u(0)] = 10.0
    W2[L.p] = 1e8
    for q, (i, j) in enumerate(P.vbar_components(2)):
        W2[L.V(q)] = 1.0 if i == j else 0.0
    o2 = O.Oracle(pb2)
    _, c2 = o2.step_flops(o2.prim_to_cons(W2), 1e-7, 0)
    f1 = c1[0, :5].sum() / 32
    f2 = c2[0, :5].sum() / (32 * 32)
    assert f1 < 0.8 * f2, (f1, f2)


def test_disc_sweep_count_in_expected_range():
    """the 2-D shock/disc sweep: about 1.1-1.3 thousand flops per cell
    (dominated by the face flux and the predictor), the sources a few
    hundred"""
    pb, W = P.shock_disc(96, seed=0)
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    _, cnt = o.step_flops(U, o.dt_cfl(U), 0)
    per = cnt[:, :5].sum(1) / (96 * 96)
    assert 1000 < per[0] < 1500 and 1000 < per[1] < 1500, per
    assert 100 < per[2] < 400 and 100 < per[3] < 300, per


def test_counting_rk3_step_is_the_plain_rk3_step():
    pb, W = P.shock_disc(40, seed=2)
    o = O.Oracle(pb)
    U = o.prim_to_cons(W)
    dt = o.dt_cfl(U)
    U1 = o.step_rk3(U, dt)
    U2, cnt = o.step_rk3_flops(U, dt)
    np.testing.assert_array_equal(U1, U2)
    per = cnt[:, :5].sum(1) / (40 * 40)
    # without the predictor a direction costs less than a split sweep; the
    # three stage combinations are 12 flops per field (11 fields)
    assert 600 < per[0] < 1100 and 600 < per[1] < 1100, per
    assert per[2] == 12 * 11, per
