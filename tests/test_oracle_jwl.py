"""Pins of the oracle's JWL reactive mixture and ignition-and-growth rate
(JWL reference curves of Sec. 2.3, root finding of Appendix B, the rate law
of Sec. 4.2, LX-17 constants of Tables 3 and 4):

* the JWL pair satisfies p_ref = rho^2 de_ref/drho (central differences) and
  its sound speed is the isentropic derivative (brute-force integration);
* Table 3's unreacted LX-17 sits at room temperature at rest (its JWL and
  C_V were fitted so): a check of the transcribed constants;
* the Appendix B split: temperature equality, the specific-volume rule,
  the primitive round trip, and identical components splitting at s = lambda;
* the rate: no ignition below the compression threshold a, ignition switched
  off past F_ig, the second growth term only past F_G2, and the time for a
  growth-only burn at fixed pressure against quadrature of the rate;
* a 1-D LX-17 detonation settling at the Chapman-Jouguet speed computed
  independently from the products' JWL Hugoniot (about 7.6 km/s).
CPU only."""
import dataclasses
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.optimize

from oracle import pyoracle as O
from paper_2009_14555_amd import problems as P
from tests.test_oracle_pointwise import prim_cell


def jwl_np(m, rho):
    """the JWL reference pair written from Sec. 2.3 (test-side copy for the
    independent Hugoniot below)"""
    v = m.rho0 / rho
    xa, xb = math.exp(-m.jwl_R1 * v), math.exp(-m.jwl_R2 * v)
    return m.jwl_A * xa + m.jwl_B * xb, m.jwl_A * xa / (m.jwl_R1 * m.rho0) + m.jwl_B * xb / (m.jwl_R2 * m.rho0)


@pytest.mark.parametrize("which", ["reactant", "product"])
@pytest.mark.parametrize("x", [0.6, 1.0, 1.3, 1.8])
def test_jwl_pref_is_rho2_deref_by_fd(which, x):
    m = getattr(P, "lx17_" + which)()
    rho = x * m.rho0
    h = 1e-5 * rho
    e0, ep, em = O.eos(m, rho), O.eos(m, rho + h), O.eos(m, rho - h)
    de = (ep["eref"] - em["eref"]) / (2 * h)
    dp = (ep["pref"] - em["pref"]) / (2 * h)
    scale = abs(m.jwl_A) * math.exp(-m.jwl_R1 / x) + abs(m.jwl_B) * math.exp(-m.jwl_R2 / x)
    assert abs(rho * rho * de - e0["pref"]) <= 1e-7 * scale
    assert dp == pytest.approx(e0["dpref"], rel=1e-7)
    assert e0["deref"] == pytest.approx(e0["pref"] / rho ** 2, rel=1e-14)
    assert e0["Gamma"] == m.Gamma0 and e0["G"] == 0.0


def test_unreacted_lx17_is_at_room_temperature():
    """T = (p - p_ref)/(rho Gamma C_V) of the Table 3 reactant at rho0 and
    1 atm: 298 K to a tenth of a kelvin"""
    m = P.lx17_reactant()
    e = O.eos(m, m.rho0)
    T = (1.01325e5 - e["pref"]) / (m.rho0 * m.Gamma0 * m.cv)
    assert abs(T - 298.0) < 0.1


def rx_problem(reactive=None):
    return P.Problem(ndim=1, n=(1, 1, 1), dx=(1.0, 1.0, 1.0),
                     materials=[P.placeholder_for_reactive(), P.copper_table1()],
                     reactive=reactive or P.lx17(0))


@pytest.mark.parametrize("which", ["reactant", "product"])
def test_jwl_sound_speed_is_isentropic_derivative(which):
    """a pure component (lambda 1 or 0): c^2 of the cell against dp/drho
    along the isentrope de = p/rho^2 drho (RK4, differenced)"""
    m = getattr(P, "lx17_" + which)()
    lam = 1.0 if which == "reactant" else 0.0
    rho, p = 2200.0, 2e10
    shift = 0.0 if lam == 1.0 else 3.622e6

    def pres(r, e):
        pr, er = jwl_np(m, r)
        return pr + r * m.Gamma0 * (e + shift - er)

    pr, er = jwl_np(m, rho)
    e_spec = (p - pr) / (rho * m.Gamma0) + er - shift

    def isen(r_target, nsteps=200):
        r, e = rho, e_spec
        h = (r_target - rho) / nsteps
        f = lambda rr, ee: pres(rr, ee) / rr ** 2
        for _ in range(nsteps):
            k1 = f(r, e); k2 = f(r + h / 2, e + h / 2 * k1)
            k3 = f(r + h / 2, e + h / 2 * k2); k4 = f(r + h, e + h * k3)
            e += h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            r += h
        return pres(r, e)

    dr = 1e-4 * rho
    c2_fd = (isen(rho + dr) - isen(rho - dr)) / (2 * dr)
    pb = rx_problem()
    d, _ = O.Oracle(pb).cell_diag_prim(prim_cell(pb, [rho, 8930.0], p, phi=[1 - 1e-12, 1e-12], lam=lam))
    # the copper trace (volume fraction 1e-12) moves the mixture by ~1e-12
    assert d["c2"] == pytest.approx(c2_fd, rel=1e-6)


@pytest.mark.parametrize("lam,p,rho", [(0.5, 2e10, 2300.0), (0.9, 3e10, 2500.0), (0.05, 5e9, 1300.0),
                                       (0.98, 1e9, 1950.0), (0.3, 2.7e10, 2450.0)])
def test_lx17_split_constraints(lam, p, rho):
    """Appendix B: at the root T_alpha = T_beta and 1/rho_y = lam/rho_alpha
    + (1-lam)/rho_beta, from the primitive branch (p known) and from the
    conservative branch (energy known), which returns the pressure"""
    pb = rx_problem()
    o = O.Oracle(pb)
    W = prim_cell(pb, [rho, 8930.0], p, phi=[1 - 1e-9, 1e-9], lam=lam)
    dp, U = o.cell_diag_prim(W)
    assert dp["T_a"] == pytest.approx(dp["T_b"], rel=1e-12)
    d = o.cell_diag(U)
    assert d["p"] == pytest.approx(p, rel=1e-11)
    assert d["T_a"] == pytest.approx(d["T_b"], rel=1e-10)
    assert d["T_a"] > 0
    assert lam / d["rho_a"] + (1 - lam) / d["rho_b"] == pytest.approx(1 / rho, rel=1e-13)
    assert d["rho_a"] == pytest.approx(dp["rho_a"], rel=1e-10)


@pytest.mark.parametrize("lam", [0.1, 0.5, 0.93])
def test_identical_components_split_at_lambda(lam):
    """reactant = product (the LX-17 products, Q = 0, one C_V): equal
    temperatures at equal pressure need equal densities, so the split is
    s = lam and the cell is the single JWL material"""
    prod = P.lx17_product()
    rx = dataclasses.replace(P.lx17(0), reactant=prod, product=prod, Q=0.0)
    pb = rx_problem(rx)
    o = O.Oracle(pb)
    L = P.layout(pb)
    rho, p = 2300.0, 2e10
    W = prim_cell(pb, [rho, 8930.0], p, phi=[1 - 1e-12, 1e-12], lam=lam)
    _, U = o.cell_diag_prim(W)
    d = o.cell_diag(U)
    assert d["s"] == pytest.approx(lam, rel=1e-12)
    assert d["rho_a"] == pytest.approx(rho, rel=1e-12) and d["rho_b"] == pytest.approx(rho, rel=1e-12)
    # the same cell with lambda = 1 (no root finding at all)
    U1 = U.copy()
    U1[L.lam] = U[L.m(0)]
    assert o.cell_diag(U1)["p"] == pytest.approx(d["p"], rel=1e-12)


def react(pb, W, dt, nsteps):
    o = O.Oracle(pb)
    L = P.layout(pb)
    _, U = o.cell_diag_prim(W)
    U = U.reshape(-1, 1)
    for _ in range(nsteps):
        U = o.reaction(U, dt)
    return U[L.lam, 0] / U[L.m(0), 0], o.cell_diag(U.reshape(-1))


def lx17_with(**ig):
    rx = P.lx17(0)
    return dataclasses.replace(rx, ig={**rx.ig, **ig})


def test_no_ignition_below_the_compression_threshold():
    """unreacted (F = 0: the growth terms vanish) explosive reacts only when
    compressed past rho0 (1 + a)"""
    pb = rx_problem()
    for rho, burns in [(1905.0 * 1.20, False), (1905.0 * 1.219, False), (1905.0 * 1.30, True)]:
        lam, _ = react(pb, prim_cell(pb, [rho, 8930.0], 3e10, phi=[1 - 1e-9, 1e-9], lam=1.0), 1e-10, 5)
        assert (lam < 1.0) == burns, (rho, lam)


def test_ignition_stops_past_F_ig():
    """with both growth terms off, a strongly compressed cell burns by
    ignition until F passes F_ig = 0.02 and then stops"""
    pb = rx_problem(lx17_with(G1=0.0, G2=0.0))
    W = prim_cell(pb, [1905.0 * 1.5, 8930.0], 3e10, phi=[1 - 1e-9, 1e-9], lam=1.0)
    dt = 2e-12
    lam, _ = react(pb, W, dt, 400)
    F = 1 - lam
    # the last step's increment is below the rate bound I (0.5 - 0.22)^7 dt
    assert 0.02 <= F <= 0.02 + 4e12 * 0.28 ** 7 * dt * 1.01
    lam2, _ = react(pb, W, dt, 800)
    assert lam2 == lam


def test_second_growth_term_only_past_F_G2():
    pb = rx_problem(lx17_with(I=0.0, G1=0.0))
    for F0, burns in [(0.5, False), (0.79, False), (0.81, True)]:
        lam, _ = react(pb, prim_cell(pb, [2400.0, 8930.0], 3e10, phi=[1 - 1e-9, 1e-9], lam=1 - F0), 1e-9, 3)
        assert (lam < 1 - F0) == burns, (F0, lam)


@pytest.mark.parametrize("term", ["G1", "G2"])
def test_growth_burn_time_against_quadrature(term):
    """Q = 0 and identical components keep p fixed while lambda changes, so
    the time from F0 to F1 under one growth term is
    t = int dF / (G (1-F)^c F^d p^y) (quadrature); the oracle's RK4 steps
    reach F1 at that time to the RK4 error"""
    prod = P.lx17_product()
    ig = dict(P.lx17(0).ig)
    if term == "G1":
        ig.update(I=0.0, G2=0.0)
        F0, F1, k, c, d, y = 0.1, 0.6, ig["G1"], ig["c"], ig["d"], ig["y"]
    else:
        ig.update(I=0.0, G1=0.0)
        F0, F1, k, c, d, y = 0.85, 0.97, ig["G2"], ig["e"], ig["g"], ig["z"]
    rx = dataclasses.replace(P.lx17(0), reactant=prod, product=prod, Q=0.0, ig=ig)
    pb = rx_problem(rx)
    p = 3e10
    W = prim_cell(pb, [2400.0, 8930.0], p, phi=[1 - 1e-12, 1e-12], lam=1 - F0)
    rate = lambda F: k * (1 - F) ** c * F ** d * (p / 1e11) ** y
    T = scipy.integrate.quad(lambda F: 1.0 / rate(F), F0, F1, epsabs=0, epsrel=1e-13)[0]
    nsteps = 200
    lam, d1 = react(pb, W, T / nsteps, nsteps)
    assert d1["p"] == pytest.approx(p, rel=1e-12)
    assert 1 - lam == pytest.approx(F1, rel=1e-8)


def cj_speed(rx, rho0=1905.0, p0=1e5):
    """Chapman-Jouguet speed into unreacted explosive at (rho0, p0): the
    products' Hugoniot e_b(v, p) - e0 = (p + p0)(v0 - v)/2 with e_b from
    their JWL lowered by Q, closed form in p for each v; D^2 = v0^2 (p -
    p0)/(v0 - v) minimised over v (tangency of the Rayleigh line)"""
    a, b = rx.reactant, rx.product
    pa, ea = jwl_np(a, rho0)
    e0 = ea + (p0 - pa) / (rho0 * a.Gamma0)
    v0, G = 1 / rho0, b.Gamma0

    def pH(v):
        pr, er = jwl_np(b, 1 / v)
        return (0.5 * p0 * (v0 - v) + pr * v / G - er + rx.Q + e0) / (v / G - 0.5 * (v0 - v))

    D2 = lambda v: v0 * v0 * (pH(v) - p0) / (v0 - v)
    r = scipy.optimize.minimize_scalar(D2, bounds=(v0 / (2 / G + 1) * 1.05, v0 * 0.999), method="bounded",
                                       options={"xatol": 1e-14})
    return math.sqrt(r.fun), pH(r.x)


def test_cj_speed_of_lx17():
    D, p = cj_speed(P.lx17(0))
    assert 7550 < D < 7700 and 2.5e10 < p < 2.8e10, (D, p)


def test_detonation_settles_at_cj_speed():
    """1-D LX-17 column, 50 um cells, ignited by the 27 GPa booster: the
    front (lambda = 1/2) speed over 3-4.8 us is within 0.5% of the CJ speed
    (the ignition-and-growth wave builds up to it from below)"""
    pb, W = P.detonation_1d(800, length=0.04)
    o = O.Oracle(pb)
    L = P.layout(pb)
    U = o.prim_to_cons(W)
    (x,) = P.cell_centres(pb)
    t, k, hist = 0.0, 0, []
    while t < 4.8e-6:
        dt = o.dt_cfl(U)
        U = o.step(U, dt, k)
        t += dt
        k += 1
        if t > 3e-6 and k % 10 == 0:
            lam = o.cons_to_prim(U)[L.lam]
            hist.append((t, x[np.where(lam < 0.5)[0].max()]))
    h = np.array(hist)
    D = np.polyfit(h[:, 0], h[:, 1], 1)[0]
    Dcj, _ = cj_speed(pb.reactive)
    assert abs(D / Dcj - 1) < 0.005, (D, Dcj)
    assert np.all(np.isfinite(U))


def _check_rule_on_cells(o, Uf, cells, z):
    """the oracle's root at each cell equals the root the rule names, found by
    brute force: a dense scan over log-odds z = ln(t/(1-t)) lists the sign
    changes, the one nearest t = 1/2 on the side g(1/2) points to is refined
    by Brent's method; returns how many cells have several roots"""
    t = 1.0 / (1.0 + np.exp(-z))
    i0 = int(np.argmin(np.abs(z)))
    assert z[i0] == 0.0
    multi = 0
    for c in cells:
        Uc = np.ascontiguousarray(Uf[:, c])
        g = o.rx_residual(Uc, t)[0]
        neg = g < 0.0
        ch = np.nonzero(neg[1:] != neg[:-1])[0]
        multi += len(ch) > 1
        up = bool(neg[i0])
        side = ch[ch >= i0] if up else ch[ch < i0]
        assert len(side), "g keeps its sign on the side it points to"
        i = side.min() if up else side.max()
        f = lambda tt: o.rx_residual(Uc, [tt])[0][0]
        want = scipy.optimize.brentq(f, t[i], t[i + 1], xtol=1e-300, rtol=1e-15, maxiter=400)
        got = o.rx_split(Uc)
        assert abs(got - want) <= 1e-12 * min(want, 1.0 - want) + 1e-19, (c, got, want, t[ch])
    return multi


def test_split_root_rule_in_multi_root_cells():
    """App. B fixes the split by temperature equality but not which root
    where there are several (explosive traces, low-density JWL reactant).
    The rule: the first sign change of T_b - T_a met going outward from equal
    densities (t = 1/2) on the side its sign points to.  Checked by brute
    force on every split cell of an air-confined LX-17 stick after 16 steps
    (many with several roots), and on the state after the first sweep of
    step 10, which holds a cell with three roots inside the first bracket of
    the probe ladder (t in (1/2, 3/4)): the rule takes the one nearest 1/2
    there, where plain halving of that bracket lands on the outermost."""
    pb, W = P.rate_stick(48, 100, confined=False, seed=2)
    o = O.Oracle(pb)
    L = P.layout(pb)
    y = pb.reactive.mat
    z = np.linspace(-39.0, 39.0, 6001)  # includes z = 0 (t = 1/2)

    def split_cells(V):
        Vf = V.reshape(V.shape[0], -1)
        lam = Vf[L.lam] / Vf[L.m(y)]
        return Vf, np.nonzero((lam > 1e-12) & (lam < 1.0 - 1e-12))[0]

    U = o.prim_to_cons(W)
    for k in range(16):
        dt = o.dt_cfl(U)
        if k == 10:
            Vf, cells = split_cells(o.sweep(U, dt, 0))
            assert 488 in cells
            Uc = np.ascontiguousarray(Vf[:, 488])
            tb = np.linspace(0.5, 0.75, 2001)
            neg = o.rx_residual(Uc, tb)[0] < 0.0
            roots = tb[1:][neg[1:] != neg[:-1]]
            assert len(roots) == 3 and roots[0] < 0.52 and roots[-1] > 0.74, roots
            assert abs(o.rx_split(Uc) - roots[0]) < 1e-3
            _check_rule_on_cells(o, Vf, cells, z)
        U = o.step(U, dt, k)
    Uf, cells = split_cells(U)
    assert len(cells) > 100
    assert _check_rule_on_cells(o, Uf, cells, z) >= 10
