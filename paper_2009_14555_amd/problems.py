"""Problem descriptions and seeded synthetic inputs.

This module holds *inputs only*: material constants, grid descriptions and
seeded generators of initial conditions in primitive variables (volume
fraction, phasic densities, reaction progress, velocity, pressure, stretch
tensor).  It contains none of the scheme's arithmetic (no equation of state,
no conversion to conserved variables); each solver converts the primitive
fields itself.

Material constants follow the paper's tables where it gives them:
Table 1 (Romenskii copper, and the exponents alpha-bar = 1, beta-bar = 3,
Gamma = 2 reused for the synthetic solid) and Table 2 (generic explosive:
reactant and product stiffened gases).  The solid and fluid of the 2-D and
batched workloads (rho0 = 2700, K0 = 76 GPa, G0 = 26 GPa, yield 0.3 GPa,
stiffened water gamma = 4.4, p_inf = 6e8) are synthetic stand-ins shaped like
the paper's shock/solid tests (Sec. 4), not data from it.

Primitive slot order (same slots as the conserved state):
  phi_1..phi_{N-1}, rho_1..rho_N, [lambda], u_1..u_D, p, Vbar components
with Vbar components 11,22,33 (1-D), 11,12,21,22,33 (2-D), all nine (3-D).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

EOS_IDEAL, EOS_STIFFENED, EOS_ROMENSKII, EOS_JWL = 0, 1, 2, 3
RATE_POWER, RATE_IG = 0, 1
PLAST_NONE, PLAST_PERFECT, PLAST_JC = 0, 1, 2
# boundary rules per dimension; BC_AXIS: reflective at the low end (the axis
# r = 0 of the cylindrical form), transmissive at the high end
BC_TRANSMISSIVE, BC_PERIODIC, BC_REFLECTIVE, BC_AXIS = 0, 1, 2, 3
GEOM_CARTESIAN, GEOM_CYLINDRICAL = 0, 1
LIM_MINMOD, LIM_VANALBADA = 0, 1

PHI_PURE = 1e-6  # volume fraction of the absent material in a pure region


@dataclass
class Material:
    eos: int = EOS_IDEAL
    gamma: float = 1.4
    pinf: float = 0.0
    eref: float = 0.0
    rho0: float = 0.0
    K0: float = 0.0
    G0: float = 0.0
    abar: float = 1.0
    bbar: float = 3.0
    Gamma0: float = 2.0
    cv: float = 0.0
    plast: int = PLAST_NONE
    yield_stress: float = 0.0
    # Johnson-Cook (PLAST_JC): sigma_Y = (c1 + c2 eps_p^n)(1 - theta^m), rate
    # chi0 exp((s - 1)/c3); theta = (T - T0)/(Tmelt - T0)
    jc_c1: float = 0.0
    jc_c2: float = 0.0
    jc_c3: float = 0.0
    jc_n: float = 1.0
    jc_m: float = 1.0
    jc_tmelt: float = 0.0
    jc_t0: float = 298.0
    jc_chi0: float = 0.0
    # JWL (EOS_JWL): p_ref = A exp(-R1 rho0/rho) + B exp(-R2 rho0/rho), with
    # rho0 and Gamma0 above
    jwl_A: float = 0.0
    jwl_B: float = 0.0
    jwl_R1: float = 1.0
    jwl_R2: float = 1.0


@dataclass
class Reactive:
    mat: int = -1
    reactant: Material = field(default_factory=Material)
    product: Material = field(default_factory=Material)
    Q: float = 0.0
    k: float = 0.0
    n: float = 2.0
    pref: float = 1e10
    # RATE_IG: three-term ignition and growth of F = 1 - lambda
    law: int = RATE_POWER
    ig: dict = field(default_factory=dict)


@dataclass
class Problem:
    ndim: int
    n: Tuple[int, int, int]
    dx: Tuple[float, float, float]
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    bc: Tuple[int, int, int] = (BC_TRANSMISSIVE,) * 3
    materials: List[Material] = field(default_factory=list)
    reactive: Reactive = field(default_factory=Reactive)
    limiter: int = LIM_MINMOD
    thinc: int = 0
    beta0: float = 2.5
    delta: float = 1e-5
    eps: float = 1e-20
    va_scale: Tuple[float, ...] = (1.0, 1e3, 1.0, 1e3, 1e9, 1.0)
    cfl: float = 0.6
    geom: int = GEOM_CARTESIAN  # cylindrical: 2-D, x = r (lo[0] the radius of the low face), y = z

    @property
    def nmat(self) -> int:
        return len(self.materials)

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n[: self.ndim]))

    @property
    def shape(self) -> Tuple[int, ...]:
        """numpy shape of one field, slowest axis first (z, y, x)."""
        return tuple(int(v) for v in reversed(self.n[: self.ndim]))

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------- layout
def vbar_components(ndim: int) -> List[Tuple[int, int]]:
    if ndim == 1:
        return [(0, 0), (1, 1), (2, 2)]
    if ndim == 2:
        return [(0, 0), (0, 1), (1, 0), (1, 1), (2, 2)]
    return [(i, j) for i in range(3) for j in range(3)]


@dataclass(frozen=True)
class Layout:
    ndim: int
    nmat: int
    reactive: bool
    plastic_strain: bool = False  # a Johnson-Cook solid: m_eps in the history slot

    @property
    def extra(self) -> bool:
        return self.reactive or self.plastic_strain

    @property
    def nphi(self) -> int:
        return self.nmat - 1

    def phi(self, l: int) -> int:
        return l

    def rho(self, l: int) -> int:  # phasic density / partial density slot
        return self.nmat - 1 + l

    m = rho

    @property
    def lam(self) -> int:  # the history slot: m_lam (reactive) or m_eps (Johnson-Cook)
        return 2 * self.nmat - 1

    eps = lam

    def u(self, k: int) -> int:
        return 2 * self.nmat - 1 + int(self.extra) + k

    mom = u

    @property
    def p(self) -> int:
        return 2 * self.nmat - 1 + int(self.extra) + self.ndim

    E = p

    def V(self, q: int) -> int:
        return self.p + 1 + q

    @property
    def nV(self) -> int:
        return len(vbar_components(self.ndim))

    @property
    def nfields(self) -> int:
        return self.p + 1 + self.nV

    def vindex(self, i: int, j: int) -> Optional[int]:
        comps = vbar_components(self.ndim)
        if (i, j) in comps:
            return self.V(comps.index((i, j)))
        return None


def layout(pb: Problem) -> Layout:
    return Layout(pb.ndim, pb.nmat, pb.reactive.mat >= 0, any(m.plast == PLAST_JC for m in pb.materials))


def blank_prim(pb: Problem) -> np.ndarray:
    """Primitive array (F, *shape) with identity stretch tensor."""
    L = layout(pb)
    W = np.zeros((L.nfields,) + pb.shape, dtype=np.float64)
    for q, (i, j) in enumerate(vbar_components(pb.ndim)):
        if i == j:
            W[L.V(q)] = 1.0
    return W


def cell_centres(pb: Problem):
    """Cell-centre coordinates, each of numpy field shape."""
    axes = []
    for d in range(pb.ndim):
        axes.append(pb.lo[d] + (np.arange(pb.n[d]) + 0.5) * pb.dx[d])
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(grids))  # x, y, z order


# -------------------------------------------------------------- materials
def air(gamma=1.4) -> Material:
    return Material(eos=EOS_IDEAL, gamma=gamma)


def water_sg() -> Material:
    """Stiffened-gas water (gamma 4.4, p_inf 6e8 Pa)."""
    return Material(eos=EOS_STIFFENED, gamma=4.4, pinf=6e8)


def solid_c2(yield_stress=0.3e9, G0=26e9) -> Material:
    """Elastoplastic solid: Romenskii with rho0 2700, K0 76 GPa, G0 26 GPa and
    the Table 1 exponents (alpha-bar 1, beta-bar 3, Gamma 2), perfect plasticity."""
    return Material(eos=EOS_ROMENSKII, rho0=2700.0, K0=76e9, G0=G0, abar=1.0, bbar=3.0,
                    Gamma0=2.0, plast=PLAST_PERFECT, yield_stress=yield_stress)


def copper_table1() -> Material:
    """Romenskii copper of Table 1 (elastic)."""
    return Material(eos=EOS_ROMENSKII, rho0=8930.0, K0=136.5e9, G0=39.4e9, abar=1.0, bbar=3.0,
                    Gamma0=2.0)


def copper_jc(chi0: float = 1.0) -> Material:
    """Romenskii copper of Table 1 with the Johnson-Cook constants of Table 5
    (c1 0.4 GPa, c2 0.177 GPa, c3 0.025, n 1.0, m 1.09, Tmelt 1358 K, T0 298
    K); the reference rate chi0 (1/s) and the specific heat (390 J/kg/K,
    copper) are not given by the paper."""
    return Material(eos=EOS_ROMENSKII, rho0=8930.0, K0=136.5e9, G0=39.4e9, abar=1.0, bbar=3.0,
                    Gamma0=2.0, cv=390.0, plast=PLAST_JC, jc_c1=0.4e9, jc_c2=0.177e9, jc_c3=0.025, jc_n=1.0,
                    jc_m=1.09, jc_tmelt=1358.0, jc_t0=298.0, jc_chi0=chi0)


def generic_explosive(mat_index: int, k=1e6, n=2.0, pref=1e10) -> Reactive:
    """Table 2 generic explosive: reactant SG (rho0 1600, gamma 4, p_inf 1 GPa,
    C_V 2000), product SG (gamma 3, p_inf 0, C_V 1000, Q 3.68 MJ/kg)."""
    return Reactive(mat=mat_index,
                    reactant=Material(eos=EOS_STIFFENED, gamma=4.0, pinf=1e9, cv=2000.0),
                    product=Material(eos=EOS_STIFFENED, gamma=3.0, pinf=0.0, cv=1000.0),
                    Q=3.68e6, k=k, n=n, pref=pref)


IG_KEYS = ("I", "G1", "G2", "a", "b", "c", "d", "e", "g", "x", "y", "z", "Fig", "FG1", "FG2", "rho0", "punit")


def lx17_reactant() -> Material:
    """unreacted LX-17, JWL of Table 3 (rho0 1905, A 778.1e11 Pa, B -0.0503e11
    Pa, R1 11.3, R2 1.13, Gamma 0.8938, C_V 1305.5)"""
    return Material(eos=EOS_JWL, rho0=1905.0, jwl_A=778.1e11, jwl_B=-0.0503e11, jwl_R1=11.3, jwl_R2=1.13,
                    Gamma0=0.8938, cv=1305.5)


def lx17_product() -> Material:
    """LX-17 detonation products, JWL of Table 3 (A 14.81e11 Pa, B 0.6379e11
    Pa, R1 6.2, R2 2.2, Gamma 0.5, C_V 524.9); the table leaves the products'
    rho0 blank: the reactant's 1905 is used"""
    return Material(eos=EOS_JWL, rho0=1905.0, jwl_A=14.81e11, jwl_B=0.6379e11, jwl_R1=6.2, jwl_R2=2.2,
                    Gamma0=0.5, cv=524.9)


def lx17(mat_index: int) -> Reactive:
    """LX-17 (Tables 3 and 4): JWL reactant and products, Q 3.622 MJ/kg, the
    ignition-and-growth rate (I 4e12 /s, G1 4500e6, G2 30e6 with pressures in
    1e11 Pa; a 0.22, b c e g 0.667, d 1, x 7, y 3, z 1, F_ig 0.02, F_G1 F_G2 0.8)"""
    ig = dict(I=4e12, G1=4500e6, G2=30e6, a=0.22, b=0.667, c=0.667, d=1.0, e=0.667, g=0.667, x=7.0, y=3.0,
              z=1.0, Fig=0.02, FG1=0.8, FG2=0.8, rho0=1905.0, punit=1e11)
    return Reactive(mat=mat_index, reactant=lx17_reactant(), product=lx17_product(), Q=3.622e6, law=RATE_IG,
                    ig=ig)


def placeholder_for_reactive() -> Material:
    """Entry standing in the material list for the reactive mixture."""
    return Material(eos=EOS_STIFFENED, gamma=4.0, pinf=1e9)


# ------------------------------------------------------- stiffened shocks
def sg_shock_state(gamma, pinf, rho0, p0, p1):
    """Post-shock density and particle speed of a right-moving shock into
    stiffened gas at rest (textbook Hugoniot with the shifted pressure p + p_inf)."""
    P0, P1 = p0 + pinf, p1 + pinf
    ratio = ((gamma + 1) * P1 + (gamma - 1) * P0) / ((gamma - 1) * P1 + (gamma + 1) * P0)
    rho1 = rho0 * ratio
    u1 = math.sqrt((p1 - p0) * (rho1 - rho0) / (rho0 * rho1))
    speed = rho1 * u1 / (rho1 - rho0)
    return rho1, u1, speed


# ------------------------------------------------------------ generators
def sod_two_gamma(n: int = 1000, thinc: bool = False, cfl: float = 0.8) -> Tuple[Problem, np.ndarray]:
    """1-D two-material Sod tube on [0,1]: gamma 1.4 | 1.67, interface at 0.5,
    (rho,u,p) = (1,0,1) | (0.125,0,0.1), volume fraction 1-1e-6 | 1e-6."""
    pb = Problem(ndim=1, n=(n, 1, 1), dx=(1.0 / n, 1.0, 1.0), materials=[air(1.4), air(1.67)],
                 thinc=int(thinc), cfl=cfl)
    L = layout(pb)
    W = blank_prim(pb)
    (x,) = cell_centres(pb)
    left = x < 0.5
    W[L.phi(0)] = np.where(left, 1.0 - PHI_PURE, PHI_PURE)
    rho = np.where(left, 1.0, 0.125)
    W[L.rho(0)] = rho
    W[L.rho(1)] = rho
    W[L.p] = np.where(left, 1.0, 0.1)
    return pb, W


def shock_tube(mats: Sequence[Material], left: dict, right: dict, n: int = 400, x0: float = 0.5,
               length: float = 1.0, thinc: bool = False, cfl: float = 0.8) -> Tuple[Problem, np.ndarray]:
    """1-D two-material Riemann problem; left/right dicts give rho, u, p."""
    pb = Problem(ndim=1, n=(n, 1, 1), dx=(length / n, 1.0, 1.0), materials=list(mats),
                 thinc=int(thinc), cfl=cfl)
    L = layout(pb)
    W = blank_prim(pb)
    (x,) = cell_centres(pb)
    lm = x < x0
    W[L.phi(0)] = np.where(lm, 1.0 - PHI_PURE, PHI_PURE)
    W[L.rho(0)] = np.where(lm, left["rho"], right["rho"])
    W[L.rho(1)] = np.where(lm, left["rho"], right["rho"])
    W[L.u(0)] = np.where(lm, left["u"], right["u"])
    W[L.p] = np.where(lm, left["p"], right["p"])
    return pb, W


def disc_fraction(x, y, cx, cy, r, dx, dy, sub=4):
    """Area fraction of a disc inside each cell from sub x sub samples."""
    acc = np.zeros_like(x)
    for a in range(sub):
        for b in range(sub):
            xs = x + ((a + 0.5) / sub - 0.5) * dx
            ys = y + ((b + 0.5) / sub - 0.5) * dy
            acc += ((xs - cx) ** 2 + (ys - cy) ** 2 < r * r)
    return acc / (sub * sub)


def shock_disc(n: int = 2048, seed: int = 0, noise: float = 0.01, thinc: bool = True,
               periodic: bool = False, shock: bool = True, cfl: float = 0.6,
               mirror_y: bool = False) -> Tuple[Problem, np.ndarray]:
    """2-D planar shock in stiffened water (post-shock p = 1e9 Pa) hitting a
    circular elastoplastic inclusion of radius 0.2 centred at (0.5, 0.5) on
    [0,1]^2; seeded +-1% density noise.  Material 0 = water, 1 = solid."""
    bc = (BC_PERIODIC,) * 3 if periodic else (BC_TRANSMISSIVE,) * 3
    pb = Problem(ndim=2, n=(n, n, 1), dx=(1.0 / n, 1.0 / n, 1.0), bc=bc,
                 materials=[water_sg(), solid_c2()], thinc=int(thinc), cfl=cfl)
    L = layout(pb)
    W = blank_prim(pb)
    x, y = cell_centres(pb)
    f = disc_fraction(x, y, 0.5, 0.5, 0.2, pb.dx[0], pb.dx[1])
    phi_w = np.clip(1.0 - f, PHI_PURE, 1.0 - PHI_PURE)
    W[L.phi(0)] = phi_w
    rho_w = np.full(x.shape, 1000.0)
    u = np.zeros(x.shape)
    p = np.full(x.shape, 1e5)
    if shock:
        wat = water_sg()
        rho1, u1, _ = sg_shock_state(wat.gamma, wat.pinf, 1000.0, 1e5, 1e9)
        xs = 0.3 - 8 * pb.dx[0]
        post = x < xs
        rho_w = np.where(post, rho1, rho_w)
        u = np.where(post, u1, u)
        p = np.where(post, 1e9, p)
    fac = np.ones(x.shape)
    if noise:
        rng = np.random.default_rng(seed)
        fac = 1.0 + noise * rng.uniform(-1.0, 1.0, size=x.shape)
        if mirror_y:  # make the noise field symmetric about y = 1/2
            fac = 0.5 * (fac + fac[::-1, :])
    W[L.rho(0)] = rho_w * fac
    W[L.rho(1)] = 2700.0 * fac
    W[L.u(0)] = u
    W[L.p] = p
    return pb, W


def shock_disc_jc(n: int = 2048, seed: int = 0, noise: float = 0.01, thinc: bool = True,
                  periodic: bool = False, cfl: float = 0.6) -> Tuple[Problem, np.ndarray]:
    """shock_disc with a Johnson-Cook copper disc (Table 1 Romenskii copper,
    Table 5 Johnson-Cook constants; rho0 8930) in place of the perfectly
    plastic solid; the plastic strain starts at 0.  Material 0 = water,
    1 = copper."""
    pb0, W0 = shock_disc(n, seed=seed, noise=noise, thinc=thinc, periodic=periodic, cfl=cfl)
    pb = pb0.replace(materials=[water_sg(), copper_jc()])
    L0, L = layout(pb0), layout(pb)
    W = blank_prim(pb)
    for f in range(L0.nfields):
        W[f if f < L0.lam else f + 1] = W0[f]
    W[L.rho(1)] = W0[L0.rho(1)] * (8930.0 / 2700.0)
    W[L.eps] = 0.0
    return pb, W


def reactive_slab(n: int = 256, seed: int = 0, thinc: bool = True, cfl: float = 0.6,
                  noise: float = 0.01) -> Tuple[Problem, np.ndarray]:
    """3-D reactive mixture (generic explosive, lambda = 1, rho 1600, p 1e5)
    below an elastoplastic slab occupying z >= 0.7, ignited by a hot spot of
    radius 10 cells at (0.5, 0.5, 0.35) with p = 1e10 Pa; seeded +-1% density
    noise (a mirror-symmetric start would make results hinge on how exact
    ties at the symmetry planes are broken).
    Material 0 = reactive mixture, 1 = solid."""
    pb = Problem(ndim=3, n=(n, n, n), dx=(1.0 / n,) * 3,
                 materials=[placeholder_for_reactive(), solid_c2()],
                 reactive=generic_explosive(0), thinc=int(thinc), cfl=cfl)
    L = layout(pb)
    W = blank_prim(pb)
    x, y, z = cell_centres(pb)
    dz = pb.dx[2]
    # slab fraction: exact 1-D cell overlap with z >= 0.7
    zlo = z - 0.5 * dz
    fs = np.clip((z + 0.5 * dz - 0.7) / dz, 0.0, 1.0)
    fs = np.where(zlo >= 0.7, 1.0, fs)
    W[L.phi(0)] = np.clip(1.0 - fs, PHI_PURE, 1.0 - PHI_PURE)
    fac = np.ones(x.shape)
    if noise:
        rng = np.random.default_rng(seed)
        fac = 1.0 + noise * rng.uniform(-1.0, 1.0, size=x.shape)
    W[L.rho(0)] = 1600.0 * fac
    W[L.rho(1)] = 2700.0 * fac
    W[L.lam] = 1.0
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.35) ** 2
    hot = r2 < (10 * pb.dx[0]) ** 2
    W[L.p] = np.where(hot, 1e10, 1e5)
    return pb, W


def detonation_1d(n: int = 500, length: float = 0.02, booster: float = 0.002, p_booster: float = 27e9,
                  cfl: float = 0.6, thinc: bool = False) -> Tuple[Problem, np.ndarray]:
    """1-D LX-17 column on [0, length]: unreacted explosive (lambda = 1, rho
    1905, p 1e5) ignited by a booster of products (lambda = 0, rho 1905,
    p 27 GPa) on x < booster (the rate stick's booster of Sec. 4.2), with a
    trace (phi 1e-6) of the Table 1 copper.  Material 0 = reactive mixture."""
    pb = Problem(ndim=1, n=(n, 1, 1), dx=(length / n, 1.0, 1.0),
                 materials=[placeholder_for_reactive(), copper_table1()], reactive=lx17(0), thinc=int(thinc),
                 cfl=cfl)
    L = layout(pb)
    W = blank_prim(pb)
    (x,) = cell_centres(pb)
    W[L.phi(0)] = 1.0 - PHI_PURE
    W[L.rho(0)] = 1905.0
    W[L.rho(1)] = 8930.0
    boost = x < booster
    W[L.lam] = np.where(boost, 0.0, 1.0)
    W[L.p] = np.where(boost, p_booster, 1e5)
    return pb, W


def rate_stick_cyl(nr: int = 400, nz: int = 2000, r0: float = 4e-3, confined: bool = True, seed: int = 0,
                   noise: float = 0.01, p_booster: float = 27e9, cfl: float = 0.6) -> Tuple[Problem, np.ndarray]:
    """The rate stick of Sec. 4.2 in its own geometry: cylindrically symmetric
    (x = r in [0, 2 r0] with the reflective axis at r = 0, y = z in
    [0, 10 r0]), LX-17 for r < r0 inside copper (or air), the booster the
    stick's first r0 in z.  400 x 2000 is the paper's effective resolution
    (100 x 500 base cells with two factor-2 refinements)."""
    pbc, W = rate_stick(2 * nr, nz, r0, confined, seed, noise, p_booster, cfl)
    pb = pbc.replace(n=(nr, nz, 1), lo=(0.0, 0.0, 0.0), bc=(BC_AXIS, BC_TRANSMISSIVE, BC_TRANSMISSIVE),
                     geom=GEOM_CYLINDRICAL)
    return pb, np.ascontiguousarray(W[:, :, nr:])


def rate_stick(nx: int = 800, ny: int = 2000, r0: float = 4e-3, confined: bool = True, seed: int = 0,
               noise: float = 0.01, p_booster: float = 27e9, cfl: float = 0.6) -> Tuple[Problem, np.ndarray]:
    """2-D Cartesian stand-in of the rate stick of Sec. 4.2: an LX-17 strip
    |x| < r0 inside a copper (Table 1, perfect plasticity at 0.4 GPa) or air
    (ideal, gamma 1.4) confiner on x in [-2 r0, 2 r0], y in [0, 10 r0]; the
    booster is the strip's first r0 in y, fully reacted products at 27 GPa;
    everything else at rest at 1e5 Pa.  The default grid is the paper's
    effective resolution (100 x 500 base cells on [0, 2 r0] with two factor-2
    refinements) over the full width.  Seeded +-noise relative density
    perturbation.  Material 0 = reactive mixture, 1 = confiner."""
    conf = dataclasses.replace(copper_table1(), plast=PLAST_PERFECT, yield_stress=0.4e9) if confined else air(1.4)
    pb = Problem(ndim=2, n=(nx, ny, 1), dx=(4 * r0 / nx, 10 * r0 / ny, 1.0), lo=(-2 * r0, 0.0, 0.0),
                 materials=[placeholder_for_reactive(), conf], reactive=lx17(0), thinc=1, cfl=cfl)
    L = layout(pb)
    W = blank_prim(pb)
    x, y = cell_centres(pb)
    dx = pb.dx[0]
    # exact cell overlap with |x| < r0 (cell edges never straddle both sides)
    frac = np.clip((r0 - np.abs(x)) / dx + 0.5, 0.0, 1.0)
    W[L.phi(0)] = np.clip(frac, PHI_PURE, 1.0 - PHI_PURE)
    fac = np.ones(x.shape)
    if noise:
        fac = 1.0 + noise * np.random.default_rng(seed).uniform(-1.0, 1.0, size=x.shape)
    W[L.rho(0)] = 1905.0 * fac
    W[L.rho(1)] = (8930.0 if confined else 1.2) * fac
    boost = (y < r0) & (frac > 0.5)
    W[L.lam] = np.where(boost, 0.0, 1.0)
    W[L.p] = np.where(boost, p_booster, 1e5)
    return pb, W


def plate_impact(n: int = 512, u_plate: float = 500.0, yield_stress=0.3e9, G0=26e9, gamma=4.4,
                 pinf=6e8, noise: float = 0.0, seed: int = 0) -> Tuple[Problem, np.ndarray]:
    """2-D solid plate x in [0.2,0.4], y in [0.25,0.75] moving at +500 m/s
    into stiffened-gas fluid at rest on [0,1]^2; van Albada limiter.
    Material 0 = fluid, 1 = solid.  noise: seeded relative perturbation
    (uniform in +-noise) of the pressure and both densities; without it the
    plate's top and bottom surfaces start in exact traction equilibrium, so
    their contact speed sits exactly at the Riemann solver's branch point."""
    fluid = Material(eos=EOS_STIFFENED, gamma=gamma, pinf=pinf)
    pb = Problem(ndim=2, n=(n, n, 1), dx=(1.0 / n, 1.0 / n, 1.0),
                 materials=[fluid, solid_c2(yield_stress=yield_stress, G0=G0)],
                 limiter=LIM_VANALBADA, thinc=1, cfl=0.6)
    L = layout(pb)
    W = blank_prim(pb)
    x, y = cell_centres(pb)
    inside = (x > 0.2) & (x < 0.4) & (y > 0.25) & (y < 0.75)
    W[L.phi(0)] = np.where(inside, PHI_PURE, 1.0 - PHI_PURE)
    rng = np.random.default_rng(seed)
    fac = [1.0 + noise * rng.uniform(-1.0, 1.0, size=x.shape) for _ in range(3)] if noise else [1.0] * 3
    W[L.rho(0)] = 1000.0 * fac[0]
    W[L.rho(1)] = 2700.0 * fac[1]
    W[L.u(0)] = np.where(inside, u_plate, 0.0)
    W[L.p] = 1e5 * fac[2]
    return pb, W


def patch_sizes(npatch: int = 4096, seed: int = 0, lo: int = 16, hi: int = 128):
    """Interior sizes (nx, ny) per patch, log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    U = rng.uniform(0.0, 1.0, size=(npatch, 2))
    sizes = np.rint(lo * (hi / lo) ** U).astype(np.int64)
    return sizes


def patch_set(npatch: int = 4096, seed: int = 0, dx: float = 1.0 / 2048, kind: str = "plain"):
    """Uneven 2-D patches: each a stiffened-water background at 1e5 Pa with one
    solid disc (random centre, radius U[0.1,0.4] of the smaller side), a planar
    shock (post-shock p = 1e9) in the water upstream of the disc, at a random x
    in [0, cx - r - 2 dx] (no shock when the disc reaches the left edge), and
    +-1% density noise.  The shock starts in water, as in the single-grid disc
    problem: a jump laid across the solid and its mixed cells makes the step
    amplify round-off of 1 - phi by ~1e6 in the first step.
    kind picks the materials (material 0 the background, 1 the disc):
      "plain"    water, perfectly plastic solid (the above);
      "jc"       water, Johnson-Cook copper (Tables 1 and 5; rho 8930, plastic
                 strain 0);
      "reactive" the generic explosive of Table 2 (lambda 1, rho 1600) with a
                 hot region at 1e10 Pa in place of the shocked water, and the
                 perfectly plastic solid;
      "jwl"      LX-17 (Tables 3 and 4; lambda 1, rho 1905) with a booster of
                 products (lambda 0) at 27 GPa in place of the shocked water,
                 and copper with perfect plasticity at 0.4 GPa (the rate-stick
                 confiner; rho 8930);
      "three", "three_reactive", "three_jwl": the "plain", "reactive" and
                 "jwl" patches with a third material, a strip over the top
                 fifth of every patch: Table 1 copper with perfect plasticity
                 at 0.4 GPa (rho 8930) beside water, water beside the
                 explosives.
    Returns (problem template, sizes (npatch,2), list of primitive arrays)."""
    sizes = patch_sizes(npatch, seed)
    rng = np.random.default_rng(seed + 1)
    wat = water_sg()
    rho1, u1, _ = sg_shock_state(wat.gamma, wat.pinf, 1000.0, 1e5, 1e9)
    prims = []
    third = kind.startswith("three")
    base = {"three": "plain", "three_reactive": "reactive", "three_jwl": "jwl"}.get(kind, kind)
    copper = dataclasses.replace(copper_table1(), plast=PLAST_PERFECT, yield_stress=0.4e9)
    if base == "plain":
        mats, rx, back, solid, post_p = [water_sg(), solid_c2()], Reactive(), 1000.0, 2700.0, 1e9
    elif base == "jc":
        mats, rx, back, solid, post_p = [water_sg(), copper_jc()], Reactive(), 1000.0, 8930.0, 1e9
    elif base == "reactive":
        mats, rx = [placeholder_for_reactive(), solid_c2()], generic_explosive(0)
        back, solid, post_p = 1600.0, 2700.0, 1e10
    elif base == "jwl":
        mats, rx, back, solid, post_p = [placeholder_for_reactive(), copper], lx17(0), 1905.0, 8930.0, 27e9
    else:
        raise ValueError(f"unknown patch-set kind {kind!r}")
    if third:
        strip_mat, strip_rho = (copper, 8930.0) if base == "plain" else (water_sg(), 1000.0)
        mats = mats + [strip_mat]
    tmpl = Problem(ndim=2, n=(16, 16, 1), dx=(dx, dx, 1.0), materials=mats, reactive=rx, thinc=1, cfl=0.6)
    for (nx, ny) in sizes:
        pb = tmpl.replace(n=(int(nx), int(ny), 1))
        L = layout(pb)
        W = blank_prim(pb)
        x, y = cell_centres(pb)
        Lx, Ly = nx * dx, ny * dx
        r = rng.uniform(0.1, 0.4) * min(Lx, Ly)
        cx, cy = rng.uniform(0.0, Lx), rng.uniform(0.0, Ly)
        xs = rng.uniform(0.0, 1.0) * max(cx - r - 2 * dx, 0.0)
        if kind == "jc":
            xs = max(cx - r - 2 * dx, 0.0)  # the shock starts at the disc
        f = disc_fraction(x, y, cx, cy, r, dx, dx)
        if third:
            # the strip's exact cell overlap with y > 0.8 Ly; the disc yields to it
            fs = np.clip((y + 0.5 * dx - 0.8 * Ly) / dx, 0.0, 1.0)
            fd = f * (1.0 - fs)
            W[L.phi(1)] = np.clip(fd, PHI_PURE, 1.0 - 2.0 * PHI_PURE)
            W[L.phi(0)] = np.minimum(np.clip(1.0 - fd - fs, PHI_PURE, 1.0 - 2.0 * PHI_PURE),
                                     1.0 - W[L.phi(1)] - PHI_PURE)
            W[L.rho(2)] = strip_rho * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=x.shape))
        else:
            W[L.phi(0)] = np.clip(1.0 - f, PHI_PURE, 1.0 - PHI_PURE)
        post = x < xs
        fac = 1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=x.shape)
        W[L.rho(1)] = solid * fac
        W[L.p] = np.where(post, post_p, 1e5)
        if base in ("plain", "jc"):
            W[L.rho(0)] = np.where(post, rho1, back) * fac
            W[L.u(0)] = np.where(post, u1, 0.0)
        else:
            W[L.rho(0)] = back * fac
            W[L.lam] = np.where(post & (base == "jwl"), 0.0, 1.0)
        if kind == "jc":
            W[L.eps] = 0.0
        prims.append(W)
    return tmpl, sizes, prims


def random_smooth_state(pb: Problem, seed: int = 0, amp: float = 0.02, solid_strain: float = 0.0):
    """Smooth random periodic perturbation of a two-material state (used by
    conservation and shift tests).  Optional small random stretch tensor."""
    rng = np.random.default_rng(seed)
    L = layout(pb)
    W = blank_prim(pb)
    coords = cell_centres(pb)
    phase = rng.uniform(0, 2 * np.pi, size=8)
    wave = np.zeros(pb.shape)
    for d, c in enumerate(coords):
        wave = wave + np.sin(2 * np.pi * c + phase[d])
    blob = 0.5 + 0.5 * np.tanh(4.0 * wave)
    W[L.phi(0)] = np.clip(blob, PHI_PURE, 1.0 - PHI_PURE)
    for l in range(pb.nmat):
        base = pb.materials[l].rho0 if pb.materials[l].eos == EOS_ROMENSKII else 1000.0
        W[L.rho(l)] = base * (1.0 + amp * np.sin(2 * np.pi * coords[0] + phase[2 + l]))
    for k in range(pb.ndim):
        W[L.u(k)] = 50.0 * np.sin(2 * np.pi * coords[(k + 1) % pb.ndim] + phase[4 + k])
    W[L.p] = 1e8 * (1.0 + 0.5 * np.sin(2 * np.pi * coords[-1] + phase[6]))
    if pb.reactive.mat >= 0:
        W[L.lam] = 0.5 + 0.4 * np.sin(2 * np.pi * coords[0] + phase[7])
    if solid_strain:
        for q, (i, j) in enumerate(vbar_components(pb.ndim)):
            W[L.V(q)] = (1.0 if i == j else 0.0) + solid_strain * rng.standard_normal() * np.cos(
                2 * np.pi * coords[0] + phase[q % 8])
    return W
