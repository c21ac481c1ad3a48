"""An independent textbook solver for the 1-D Euler equations of one ideal
gas: the primitive-variable MUSCL-Hancock method (minmod slopes of (rho, u,
p), the half-step predictor W - (dt/2dx) A(W) dW with the primitive Jacobian
A = [[u, rho, 0], [0, u, 1/rho], [0, rho c^2, u]]) and the HLLC flux with
Davis wave-speed bounds, on a grid with zero-gradient boundaries.  Written
from the textbook method (not from the oracle) so that the oracle's
diffuse-interface step, run on a single material, can be checked against
it.  Test infrastructure only."""
from __future__ import annotations

import numpy as np


def minmod(a, b):
    return np.where(a * b <= 0.0, 0.0, np.where(np.abs(a) < np.abs(b), a, b))


def cons(g, rho, u, p):
    return np.array([rho, rho * u, p / (g - 1.0) + 0.5 * rho * u * u])


def flux(g, rho, u, p):
    E = p / (g - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)])


def hllc(g, WL, WR):
    rl, ul, pl = WL
    rr, ur, pr = WR
    cl = np.sqrt(g * pl / rl)
    cr = np.sqrt(g * pr / rr)
    SL = np.minimum(ul - cl, ur - cr)
    SR = np.maximum(ul + cl, ur + cr)
    S = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur))
    UL, UR = cons(g, rl, ul, pl), cons(g, rr, ur, pr)
    FL, FR = flux(g, rl, ul, pl), flux(g, rr, ur, pr)

    def star(r, u, p, U, SK):
        f = r * (SK - u) / (SK - S)
        return f * np.array([np.ones_like(r), S, U[2] / r + (S - u) * (S + p / (r * (SK - u)))])

    FsL = FL + SL * (star(rl, ul, pl, UL, SL) - UL)
    FsR = FR + SR * (star(rr, ur, pr, UR, SR) - UR)
    return np.where(SL >= 0.0, FL, np.where(S >= 0.0, FsL, np.where(SR > 0.0, FsR, FR)))


def step(g, rho, u, p, dt, dx, hancock=True):
    """one MUSCL-Hancock step of the cell averages (rho, u, p); returns the
    conserved (rho, rho u, rho E) after the step (hancock=False: the faces
    take the unpredicted MUSCL edges)"""
    W = np.array([rho, u, p])
    n = W.shape[1]
    Wg = np.concatenate([W[:, :1]] * 2 + [W] + [W[:, -1:]] * 2, axis=1)  # two ghost cells per side
    d = minmod(Wg[:, 1:-1] - Wg[:, :-2], Wg[:, 2:] - Wg[:, 1:-1])  # slopes of cells -1 .. n
    Wc = Wg[:, 1:-1]
    r, v, q = Wc
    c2 = g * q / r
    dr, dv, dq = d
    inc = np.array([v * dr + r * dv, v * dv + dq / r, r * c2 * dv + v * dq])
    h = 0.5 * (dt / dx) if hancock else 0.0
    WLe = Wc - 0.5 * d - h * inc
    WRe = Wc + 0.5 * d - h * inc
    F = hllc(g, WRe[:, :-1], WLe[:, 1:])  # faces -1/2 .. n-1/2 +1
    U = cons(g, rho, u, p)
    return U - (dt / dx) * (F[:, 1:] - F[:, :-1])
