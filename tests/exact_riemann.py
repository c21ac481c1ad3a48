"""Exact solution of the 1-D Riemann problem for two stiffened gases.

Textbook construction (Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4) with the shifted pressure P = p + p_inf on each side, so an
ideal gas is p_inf = 0.  Independent of both the oracle and the GPU library;
used as a closed-form pin of the whole step.
"""
from __future__ import annotations

import math

import numpy as np


class Side:
    def __init__(self, rho, u, p, gamma, pinf=0.0):
        self.rho, self.u, self.p, self.g, self.pinf = rho, u, p, gamma, pinf
        self.c = math.sqrt(gamma * (p + pinf) / rho)

    def f(self, ps):
        """pressure function f_K(p*) and its derivative"""
        g, P, Ps = self.g, self.p + self.pinf, ps + self.pinf
        if ps > self.p:  # shock
            A = 2.0 / ((g + 1.0) * self.rho)
            B = (g - 1.0) / (g + 1.0) * P
            sq = math.sqrt(A / (Ps + B))
            return (ps - self.p) * sq, sq * (1.0 - 0.5 * (ps - self.p) / (Ps + B))
        r = Ps / P  # rarefaction
        e = (g - 1.0) / (2.0 * g)
        val = 2.0 * self.c / (g - 1.0) * (r ** e - 1.0)
        return val, r ** (-(g + 1.0) / (2.0 * g)) / (self.rho * self.c)


def star(L: Side, R: Side, tol=1e-15):
    pmin = -min(L.pinf, R.pinf) + 1e-12
    p = max(0.5 * (L.p + R.p), pmin)
    for _ in range(200):
        fl, dl = L.f(p)
        fr, dr = R.f(p)
        F = fl + fr + (R.u - L.u)
        dp = F / (dl + dr)
        pn = max(p - dp, pmin)
        if abs(pn - p) <= tol * (abs(p) + 1.0):
            p = pn
            break
        p = pn
    fl, _ = L.f(p)
    fr, _ = R.f(p)
    u = 0.5 * (L.u + R.u) + 0.5 * (fr - fl)
    return p, u


def sample(L: Side, R: Side, x, t, x0=0.5):
    """rho, u, p and a 0/1 material flag (1 = left material) at positions x, time t"""
    ps, us = star(L, R)
    xs = (np.asarray(x, dtype=float) - x0) / t
    rho = np.empty_like(xs)
    u = np.empty_like(xs)
    p = np.empty_like(xs)
    left_mat = xs < us
    for i, s in enumerate(xs):
        if s < us:
            K, sign = L, -1.0
        else:
            K, sign = R, 1.0
        g, P, Ps = K.g, K.p + K.pinf, ps + K.pinf
        if ps > K.p:  # shock on side K
            ratio = ((g + 1) * Ps + (g - 1) * P) / ((g - 1) * Ps + (g + 1) * P)
            rs = K.rho * ratio
            S = K.u + sign * K.c * math.sqrt((g + 1) / (2 * g) * Ps / P + (g - 1) / (2 * g))
            inside = (s > S) if sign < 0 else (s < S)
            if inside:
                rho[i], u[i], p[i] = rs, us, ps
            else:
                rho[i], u[i], p[i] = K.rho, K.u, K.p
        else:  # rarefaction on side K
            rs = K.rho * (Ps / P) ** (1.0 / g)
            cs = K.c * (Ps / P) ** ((g - 1) / (2 * g))
            head = K.u + sign * K.c
            tail = us + sign * cs
            if (sign < 0 and s <= head) or (sign > 0 and s >= head):
                rho[i], u[i], p[i] = K.rho, K.u, K.p
            elif (sign < 0 and s >= tail) or (sign > 0 and s <= tail):
                rho[i], u[i], p[i] = rs, us, ps
            else:
                uf = 2.0 / (g + 1) * (-sign * K.c + (g - 1) / 2 * K.u + s)
                cf = uf - s if sign < 0 else s - uf
                cf = abs(cf)
                Pf = P * (cf / K.c) ** (2 * g / (g - 1))
                rho[i] = K.rho * (Pf / P) ** (1.0 / g)
                u[i] = uf
                p[i] = Pf - K.pinf
    return rho, u, p, left_mat
