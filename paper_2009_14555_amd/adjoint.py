"""Differentiable simulation: the step's hand-written adjoint behind
torch.autograd, for calibrating material parameters from probe data.

    sim = Differentiable(grid, params=[(0, "gamma"), (0, "pinf"), (1, "G0"), (1, "yield_stress")])
    dts = sim.record_dts(U0, theta, nsteps)          # frozen time steps (CFL of a base run)
    U = sim.run(U0, theta, dts)                       # U0, theta: torch tensors (autograd)
    J = objective(U); J.backward()                    # U0.grad, theta.grad

Every K steps form one segment (a torch.autograd.Function): the forward keeps
only the segment's first state (the checkpoint) and its time steps; the
backward recomputes the K states and applies the step adjoints in reverse,
accumulating the material-parameter adjoints on the device.  Memory: one
checkpoint per segment plus K states during a backward.  The time steps are
inputs (no adjoint flows through dt), so a finite-difference run must replay
the same list.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List, Sequence, Tuple

import torch

from . import dimp as _d
from . import solver as _s

PARAM_COLUMN = {"gamma": 0, "pinf": 1, "G0": 2, "yield_stress": 3}


class Differentiable:
    def __init__(self, grid: _s.Grid, params: Sequence[Tuple[int, str]], K: int = 20, store: bool = False):
        """K: steps per checkpointed segment.  store: the forward keeps every
        step's (state in, first sweep) in device memory (two states a step)
        and the backward uses them instead of replaying each segment; the
        gradients are the same bit for bit (the replay is deterministic)."""
        if K < 1:
            raise ValueError("K must be >= 1")
        for mat, name in params:
            if name not in PARAM_COLUMN:
                raise ValueError(f"unknown parameter {name!r} (one of {sorted(PARAM_COLUMN)})")
            if not 0 <= mat < grid.pb.nmat:
                raise ValueError(f"material index {mat} out of range")
        self.g = grid
        self.params = list(params)
        self.K = K
        self.store = store
        self.base = list(grid.pb.materials)

    # ------------------------------------------------------------ helpers
    def set_theta(self, theta) -> None:
        vals = [float(x) for x in (theta.detach().cpu().tolist() if isinstance(theta, torch.Tensor) else theta)]
        ms = list(self.base)
        for (mat, name), v in zip(self.params, vals):
            ms[mat] = dataclasses.replace(ms[mat], **{name: v})
        self.g.set_materials(ms)

    def theta0(self) -> List[float]:
        return [float(getattr(self.base[mat], name)) for mat, name in self.params]

    def record_dts(self, U0, theta, nsteps: int, cfl: float | None = None) -> List[float]:
        """the CFL time steps of a forward run (one host read per step)"""
        self.set_theta(theta)
        self.g.set_conserved(U0.detach())
        dts = []
        for k in range(nsteps):
            dt = self.g.dt_cfl(cfl)
            dts.append(dt)
            self.g.set_step_index(k)
            self.g.advance(dt)
        return dts

    def forward_steps(self, U0: torch.Tensor, dts: Sequence[float], step0: int, keep: bool = False):
        """keep: every step's (state in, first sweep); the first sweep is the
        bound buffer that does not hold the state after the step"""
        self.g.set_conserved(U0)
        states = []
        for i, dt in enumerate(dts):
            s_in = self.g.state.clone() if keep else None
            self.g.set_step_index(step0 + i)
            self.g.advance(dt)
            if keep:
                states.append((s_in, self.g.other.clone()))
        return self.g.state.clone(), states

    def run(self, U0: torch.Tensor, theta: torch.Tensor, dts: Sequence[float]) -> torch.Tensor:
        U = U0
        for s0 in range(0, len(dts), self.K):
            U = _Segment.apply(U, theta, self, tuple(dts[s0:s0 + self.K]), s0)
        return U


class _Segment(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, theta, sim: Differentiable, dts, step0):
        sim.set_theta(theta)
        U1, states = sim.forward_steps(U0.detach(), dts, step0, keep=sim.store)
        ctx.save_for_backward(U0.detach(), theta.detach())
        ctx.sim, ctx.dts, ctx.step0 = sim, dts, step0
        ctx.states = states if sim.store else None
        return U1

    @staticmethod
    def backward(ctx, lam):
        U0, theta = ctx.saved_tensors
        sim, dts, step0 = ctx.sim, ctx.dts, ctx.step0
        g = sim.g
        sim.set_theta(theta)
        states = ctx.states
        ctx.states = None
        if states is None:
            _, states = sim.forward_steps(U0, dts, step0, keep=True)
        dp = torch.zeros(12, dtype=torch.float64, device=lam.device)
        lam = lam.contiguous()
        for i in range(len(dts) - 1, -1, -1):
            lam = g.adjoint_step(states[i][0], lam, dts[i], step0 + i, dp, first_sweep=states[i][1])
        grad = g.adjoint_params(dp)
        gtheta = torch.tensor([grad[mat, PARAM_COLUMN[name]] for mat, name in sim.params], dtype=theta.dtype,
                              device=theta.device)
        return lam, gtheta, None, None, None


class _WithVelocity(torch.autograd.Function):
    """the library's rest-state-with-velocity map and its adjoint"""

    @staticmethod
    def forward(ctx, U_rest, vel, grid):
        U_rest = U_rest.detach().contiguous()
        vel = vel.detach().contiguous()
        out = torch.empty_like(U_rest)
        _d.call("dimp_with_velocity", grid.h, C.c_void_p(U_rest.data_ptr()), C.c_void_p(vel.data_ptr()),
                C.c_void_p(out.data_ptr()))
        ctx.save_for_backward(U_rest, vel)
        ctx.grid = grid
        return out

    @staticmethod
    def backward(ctx, a_out):
        U_rest, vel = ctx.saved_tensors
        a_out = a_out.contiguous()
        a_rest = torch.empty_like(U_rest)
        a_vel = torch.empty_like(vel)
        _d.call("dimp_with_velocity_adjoint", ctx.grid.h, C.c_void_p(U_rest.data_ptr()), C.c_void_p(vel.data_ptr()),
                C.c_void_p(a_out.data_ptr()), C.c_void_p(a_rest.data_ptr()), C.c_void_p(a_vel.data_ptr()))
        return a_rest, a_vel, None


def with_velocity(grid: _s.Grid, U_rest: torch.Tensor, u: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """conserved state of a rest state given velocity components (u, v),
    computed by the library: momentum rho u and total energy
    E_rest + rho |u|^2 / 2 (differentiable in U_rest, u and v)"""
    return _WithVelocity.apply(U_rest, torch.stack([u, v], 0), grid)


def probe_velocity(U: torch.Tensor, layout, row: int) -> torch.Tensor:
    """(u, v) along one grid row"""
    L = layout
    rho = U[L.m(0), row] + U[L.m(1), row]
    return torch.stack([U[L.mom(0), row] / rho, U[L.mom(1), row] / rho])


def misfit(U: torch.Tensor, obs: torch.Tensor, layout, row: int) -> torch.Tensor:
    """J = 1/2 sum over the probe row of |u - u_obs|^2"""
    d = probe_velocity(U, layout, row) - obs
    return 0.5 * torch.sum(d * d)


__all__ = ["Differentiable", "with_velocity", "probe_velocity", "misfit", "PARAM_COLUMN"]
