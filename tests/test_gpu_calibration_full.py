"""The differentiation workload at its own size: plate impact on 512^2 over
200 steps, checkpoint every 20, gradients of the probe-row velocity misfit
with respect to (gamma, p_inf) of the fluid, (G0, sigma_Y) of the solid and
the 512^2 initial velocity field.

* Against the oracle's forward-mode dual numbers (the exact tangent of the
  discrete step; each oracle step linearised at the GPU state of that step so
  both sides differentiate the same branches): the four parameters and one
  seeded random smooth initial-velocity direction.
* Against central finite differences of the GPU forward run over the frozen
  time-step list, at relative steps 1e-4, 1e-5 and 1e-6: the error is
  reported per step; the smallest over the three steps is asserted.
The +-0.1% density/pressure noise keeps faces off the Riemann branch point
S* = 0, where two implementations that round differently could take
different branches."""
import numpy as np
import pytest

from paper_2009_14555_amd import problems as P
from tests.parity_util import to_np

pytestmark = pytest.mark.gpu

PARAMS = [(0, "gamma"), (0, "pinf"), (1, "G0"), (1, "yield_stress")]
SLOTS = {"gamma": 0, "pinf": 1, "G0": 2, "yield_stress": 3}
N, NSTEPS, K = 512, 200, 20


@pytest.fixture(scope="module")
def setup():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_14555_amd import adjoint as A
    from paper_2009_14555_amd import solver as S

    pb, W = P.plate_impact(N, noise=1e-3, seed=4)
    L = P.layout(pb)
    Wr = W.copy()
    Wr[L.u(0)] = 0.0
    g = S.Grid(pb)
    g.set_primitive(Wr)
    U_rest = g.state.clone()
    u0 = torch.tensor(W[L.u(0)], dtype=torch.float64, device="cuda")
    v0 = torch.zeros_like(u0)
    sim = A.Differentiable(g, PARAMS, K=K)
    th0 = torch.tensor(sim.theta0(), dtype=torch.float64)
    U0 = A.with_velocity(g, U_rest, u0, v0).detach()
    dts = sim.record_dts(U0, th0, NSTEPS)
    obs = A.probe_velocity(sim.run(U0, th0 * 1.05, dts), L, N // 2).detach()
    th = th0.clone().requires_grad_(True)
    u = u0.clone().requires_grad_(True)
    v = v0.clone().requires_grad_(True)
    J = A.misfit(sim.run(A.with_velocity(g, U_rest, u, v), th, dts), obs, L, N // 2)
    J.backward()
    du, dv = smooth_direction(0)
    return dict(A=A, pb=pb, L=L, g=g, sim=sim, U_rest=U_rest, u0=u0, v0=v0, th0=th0, dts=dts, obs=obs,
                J=float(J), gth=th.grad.numpy().copy(), gu=to_np(u.grad), gv=to_np(v.grad), du=du, dv=dv)


def smooth_direction(seed):
    """a seeded random smooth initial-velocity direction: random amplitudes
    and phases of the lowest 4 x 4 Fourier modes, normalised to unit rms
    (a cell-by-cell random field would put slopes of the size of the van
    Albada epsilon into the flat regions, where a central difference of any
    usable step leaves the limiter's linear range)"""
    rng = np.random.default_rng(seed)
    x = (np.arange(N) + 0.5) / N
    X, Y = np.meshgrid(x, x)
    out = []
    for _ in range(2):
        f = np.zeros((N, N))
        for kx in range(1, 5):
            for ky in range(1, 5):
                a, px, py = rng.standard_normal(), rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi)
                f += a * np.sin(2 * np.pi * kx * X + px) * np.sin(2 * np.pi * ky * Y + py)
        out.append(f / np.sqrt(np.mean(f * f)))
    return out


def _J(s, theta, du=None, dv=None, h=0.0):
    import torch

    A = s["A"]
    u, v = s["u0"], s["v0"]
    if du is not None:
        u = u + h * torch.tensor(du, device="cuda")
        v = v + h * torch.tensor(dv, device="cuda")
    with torch.no_grad():
        U0 = A.with_velocity(s["g"], s["U_rest"], u, v)
        return float(A.misfit(s["sim"].run(U0, theta, s["dts"]), s["obs"], s["L"], N // 2))


def test_gradients_against_central_differences(setup):
    """G0 and sigma_Y: central differences agree with the adjoint to <= 1e-6
    at the best of the steps.  gamma, p_inf and the velocity direction miss
    1e-6 for a measured reason: the plate's top and bottom faces sit at the
    Riemann branch point S* = 0 (traction equilibrium, broken only by the
    +-0.1% noise), where the HLLC-type flux is continuous with a kink.  At a
    fixed conserved initial state a change of gamma or p_inf shifts the
    water's pressure uniformly (dp/dgamma = rho e - p_inf, 1.8e8 Pa), which
    moves all those faces across the kink once the shift exceeds the noise
    (a relative step of about 1e-6): the map is piecewise smooth with a band
    of kinks at the base point, so a central difference sees the other
    branch's slope for any step above the band and round-off for any step
    below it (measured with the oracle alone on 32^2 x 20 steps: 8.1e-2 for
    steps 1e-3 .. 1e-5, 1.8e-2 at 1e-6, 1.8e-4 at 1e-7, round-off beyond;
    with THINC off the same).  The exact tangent, the oracle's dual numbers,
    agrees with the adjoint to 1e-13 (next test)."""
    s = setup
    th0 = s["th0"]
    best = {}
    for j, (mat, name) in enumerate(PARAMS):
        errs = []
        for hr in (1e-4, 1e-5, 1e-6):
            h = hr * float(th0[j])
            tp, tm = th0.clone(), th0.clone()
            tp[j] += h
            tm[j] -= h
            fd = (_J(s, tp) - _J(s, tm)) / (2 * h)
            errs.append(abs(fd - s["gth"][j]) / abs(s["gth"][j]))
        best[name] = min(errs)
        print(f"d/d{name}: adjoint {s['gth'][j]:.10e}; central differences, rel. error at h_rel "
              f"1e-4/1e-5/1e-6: {errs[0]:.2e} {errs[1]:.2e} {errs[2]:.2e}", flush=True)
    du, dv = s["du"], s["dv"]
    ad = float(np.sum(s["gu"] * du) + np.sum(s["gv"] * dv))
    errs = []
    for hr in (1e-4, 1e-5, 1e-6):
        h = hr * 500.0  # the plate speed sets the scale of the velocity field
        fd = (_J(s, th0, du, dv, h) - _J(s, th0, du, dv, -h)) / (2 * h)
        errs.append(abs(fd - ad) / abs(ad))
    best["u0"] = min(errs)
    print(f"initial-velocity direction: adjoint {ad:.10e}; central differences, rel. error at h_rel "
          f"1e-4/1e-5/1e-6: {errs[0]:.2e} {errs[1]:.2e} {errs[2]:.2e}", flush=True)
    assert best["G0"] <= 1e-6 and best["yield_stress"] <= 1e-6, best
    # measured: gamma 2.8e-5, p_inf 2.1e-4, velocity direction 4.3e-5
    assert max(best.values()) <= 5e-4, best


def test_gradients_against_oracle_dual_numbers(setup):
    import torch

    from oracle import pyoracle as O

    s = setup
    pb, L, g = s["pb"], s["L"], s["g"]
    A = s["A"]
    s["sim"].set_theta(s["th0"])
    U0 = A.with_velocity(g, s["U_rest"], s["u0"], s["v0"]).detach()
    U_rest = to_np(s["U_rest"])
    u0 = to_np(s["u0"])
    rho = U_rest[L.m(0)] + U_rest[L.m(1)]
    du, dv = s["du"], s["dv"]
    T = np.zeros((5,) + U_rest.shape)
    T[0, L.mom(0)] = rho * du
    T[0, L.mom(1)] = rho * dv
    T[0, L.E] = rho * u0 * du
    dpar = np.zeros((5, 2, 4))
    for j, (mat, name) in enumerate(PARAMS):
        dpar[1 + j, mat, SLOTS[name]] = 1.0
    o = O.Oracle(pb)
    g.set_conserved(U0)
    for k, dt in enumerate(s["dts"]):
        Uk = to_np(g.state).copy()
        _, T = o.step_dual(Uk, T, dpar, dt, k)
        g.set_step_index(k)
        g.advance(dt)
        if k % 50 == 49:
            print(f"dual step {k + 1}", flush=True)
    torch.cuda.synchronize()
    U = to_np(g.state)
    row = N // 2
    r = U[L.m(0), row] + U[L.m(1), row]
    up = np.stack([U[L.mom(0), row] / r, U[L.mom(1), row] / r])
    res = up - s["obs"].cpu().numpy()
    assert abs(0.5 * np.sum(res * res) - s["J"]) <= 1e-12 * s["J"]
    dJ = []
    for k in range(5):
        dr = T[k, L.m(0), row] + T[k, L.m(1), row]
        dup = np.stack([(T[k, L.mom(0), row] - up[0] * dr) / r, (T[k, L.mom(1), row] - up[1] * dr) / r])
        dJ.append(float(np.sum(res * dup)))
    ad = float(np.sum(s["gu"] * du) + np.sum(s["gv"] * dv))
    rel = abs(ad - dJ[0]) / abs(dJ[0])
    print(f"initial-velocity direction: dual {dJ[0]:.12e} adjoint {ad:.12e} rel {rel:.2e}", flush=True)
    assert rel <= 1e-9
    for j, (mat, name) in enumerate(PARAMS):
        rel = abs(s["gth"][j] - dJ[1 + j]) / abs(dJ[1 + j])
        print(f"d/d{name}: dual {dJ[1 + j]:.12e} adjoint {s['gth'][j]:.12e} rel {rel:.2e}", flush=True)
        assert rel <= 1e-9, name
