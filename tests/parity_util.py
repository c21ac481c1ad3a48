"""Helpers shared by the GPU parity tests (oracle side and comparison)."""
from __future__ import annotations

import numpy as np

TOL = 1e-10  # max relative difference per stored field


def field_groups(nfields: int, layout=None):
    """Normalisation group of each stored field.  Components of the momentum
    vector share one scale (the largest momentum component), and so do the
    entries of the stretch tensor; every other field is its own group.  A
    component that starts at exactly zero (rho v of a y-uniform flow, an
    off-diagonal Vbar) is thus compared against its vector/tensor, not
    against its own round-off."""
    g = list(range(nfields))
    if layout is not None:
        mom = [layout.mom(k) for k in range(layout.ndim)]
        V = [layout.V(q) for q in range(layout.nV)]
        for f in mom:
            g[f] = mom[0]
        for f in V:
            g[f] = V[0]
    return g


def field_rel_diff(a: np.ndarray, b: np.ndarray, layout=None, acoustic_floor: bool = False) -> np.ndarray:
    """per-field max |a-b| / max |b| (max over the field's group).  With
    acoustic_floor the momentum scale is at least sqrt(max rho * max E), the
    momentum of an acoustic disturbance: a region at rest then compares its
    round-off momentum against that, not against itself."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    num = np.max(np.abs(a - b), axis=1)
    own = np.max(np.abs(b), axis=1)
    groups = field_groups(a.shape[0], layout)
    den = np.array([max(own[h] for h in range(len(groups)) if groups[h] == groups[f]) for f in range(len(groups))])
    if acoustic_floor and layout is not None:
        rho = np.sum([b[layout.m(l)] for l in range(layout.nmat)], axis=0)
        scale = np.sqrt(np.max(np.abs(rho)) * np.max(np.abs(b[layout.E])))
        for k in range(layout.ndim):
            den[layout.mom(k)] = max(den[layout.mom(k)], scale)
    den = np.where(den > 0, den, 1.0)
    return num / den


def assert_parity(gpu, ref, tol=TOL, what="", layout=None, acoustic_floor=False):
    d = field_rel_diff(gpu, ref, layout, acoustic_floor)
    bad = np.where(~(d <= tol))[0]
    assert len(bad) == 0, f"{what}: fields {bad.tolist()} differ, rel {d[bad].tolist()} (tol {tol})"
    return d


def to_np(t):
    return t.detach().cpu().numpy()
