/*
 * oracle.cpp -- plain CPU reference of the diffuse-interface step.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Slow on purpose: every cell
 * recomputes everything it needs, in the order the paper states it, with no
 * blocking, fusion or reordering.  Built with -O2 -ffp-contract=off and no
 * fast-math.  Templated on the scalar type so the same source can run on
 * forward-mode dual numbers.
 *
 * Paper sections followed (arXiv 2009.14555):
 *   governing system ............ Sec. 2.1 (evolution equations), Sec. 3 (vector form)
 *   Mie-Grueneisen closures ...... Sec. 2.3 (ideal, stiffened, JWL, Romenskii)
 *   mixture rules ................ Sec. 2.2 (mixture rules for rho, rhoE, G, c^2, sigma)
 *   reactive mixture ............. Sec. 2.3.1 and Appendix B (root finding)
 *   hyperbolic update ............ Sec. 3.1 (flux differences, MUSCL on primitives)
 *   THINC / BVD .................. Appendix A
 *   plastic update ............... Sec. 3.2 (relaxation, Bazant log, Pade exp, cofactor)
 *   reactive update .............. Sec. 3.3 (RK4); rates: Sec. 4.1 form, Sec. 4.2
 *                                  ignition and growth (Table 4)
 *   fractional steps ............. Sec. 3 (hyperbolic, then plastic, then reactive)
 * Readings where the paper is silent or garbled are listed in the design notes
 * of the repository; the ones that shape arithmetic are restated inline.
 */
#include "oracle.h"

#include "dual.h"
#include "flops.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

FlopSlot g_flop_slots[256];

namespace {

constexpr int MAXM = OR_MAXMAT;
constexpr int FMAX = 3 * MAXM + 16;

int g_threads = 1;

/* ---------------------------------------------------------------- layout */
struct Lay {
  int D, N, rx, F, nV;
  int ep;  // the Johnson-Cook material (its plastic strain is transported), or -1
  int xf;  // 1 if the extra history slot (m_lam or m_eps) is stored
  int vi[9], vj[9];
  explicit Lay(const or_config& c) {
    D = c.ndim;
    N = c.nmat;
    rx = (c.rx.mat >= 0) ? 1 : 0;
    ep = -1;
    for (int l = N - 1; l >= 0; --l)
      if (c.mat[l].plast == OR_PLAST_JC) ep = l;
    xf = (rx || ep >= 0) ? 1 : 0;
    if (D == 1) {
      nV = 3;
      int a[3] = {0, 1, 2};
      for (int q = 0; q < 3; ++q) { vi[q] = a[q]; vj[q] = a[q]; }
    } else if (D == 2) {
      nV = 5;
      int ii[5] = {0, 0, 1, 1, 2}, jj[5] = {0, 1, 0, 1, 2};
      for (int q = 0; q < 5; ++q) { vi[q] = ii[q]; vj[q] = jj[q]; }
    } else {
      nV = 9;
      for (int q = 0; q < 9; ++q) { vi[q] = q / 3; vj[q] = q % 3; }
    }
    F = (N - 1) + N + xf + D + 1 + nV;
  }
  int phi(int l) const { return l; }
  int m(int l) const { return N - 1 + l; }
  int lam() const { return 2 * N - 1; }  // m_lam or m_eps
  int mom(int k) const { return 2 * N - 1 + xf + k; }
  int E() const { return 2 * N - 1 + xf + D; }
  int V(int q) const { return E() + 1 + q; }
};

int64_t ncell(const or_config& c) {
  int64_t n = 1;
  for (int d = 0; d < c.ndim; ++d) n *= c.n[d];
  return n;
}

/* index along one dimension of integer position x under the dimension's
   boundary rule: transmissive = zero-gradient copy of the nearest interior
   cell, periodic = wrap, reflective = mirror image (x -> -1 - x at the low
   end, 2n - 1 - x at the high end; *flip toggles), then clamped into the grid
   (a grid thinner than the stencil reach) */
int64_t map_index(int bc, int64_t x, int64_t n, bool* flip) {
  if (bc == OR_BC_PERIODIC) {
    x %= n;
    return x < 0 ? x + n : x;
  }
  const bool rlo = (bc == OR_BC_REFLECTIVE || bc == OR_BC_AXIS), rhi = (bc == OR_BC_REFLECTIVE);
  if (x < 0 && rlo) {
    x = -1 - x;
    if (flip) *flip = !*flip;
  } else if (x > n - 1 && rhi) {
    x = 2 * n - 1 - x;
    if (flip) *flip = !*flip;
  }
  if (x < 0) x = 0;
  if (x > n - 1) x = n - 1;
  return x;
}

/* cell index of integer position p (per dimension), with the boundary rule of
   each dimension applied; flip[d] (optional) tells whether the image is
   mirrored in dimension d */
int64_t cell_at(const or_config& c, const int64_t p[3], bool* flip = nullptr) {
  int64_t q[3] = {0, 0, 0};
  for (int d = 0; d < c.ndim; ++d) {
    bool f = false;
    q[d] = map_index(c.bc[d], p[d], c.n[d], &f);
    if (flip) flip[d] = f;
  }
  int64_t n0 = c.n[0], n1 = c.ndim > 1 ? c.n[1] : 1;
  return q[0] + n0 * (q[1] + n1 * q[2]);
}

void pos_of(const or_config& c, int64_t cell, int64_t p[3]) {
  int64_t n0 = c.n[0], n1 = c.ndim > 1 ? c.n[1] : 1;
  p[0] = cell % n0;
  p[1] = (cell / n0) % n1;
  p[2] = cell / (n0 * n1);
  for (int d = c.ndim; d < 3; ++d) p[d] = 0;
}

template <class T> T sq(const T& x) { return x * x; }
template <class T> T tmin(const T& a, const T& b) { return (b < a) ? b : a; }
template <class T> T tmax(const T& a, const T& b) { return (a < b) ? b : a; }
template <class T> T tabs(const T& a) { return (a < T(0)) ? -a : a; }

/* ------------------------------------------------ Mie-Grueneisen closures */
/* Sec. 2.3: every material is p = p_ref + rho*Gamma*(e - e_ref).  Romenskii
   cold energy is read as K0 (x^a - 1)^2 / (2 rho0 a^2), x = rho/rho0, which is
   the form for which rho0 is the zero-pressure density and K0 the bulk modulus
   there (the printed form lacks the square and has rho for rho0).  Shear
   energy G(rho) J^2 / rho with G = G0 x^(b+1) (Sec. 2.2).  Derivatives are in
   rho at fixed J^2. */
template <class T> struct Eos {
  T Gam, pref, eref, dpref, deref, G;
};

/* the material parameters a calibration differentiates (gamma, p_inf of an
   ideal/stiffened gas; G0 and sigma_Y of a Romenskii solid), carried in the
   scalar type so that dual numbers can seed them */
template <class T> struct MatPar {
  T gamma, pinf, G0, yield;
};

template <class T> MatPar<T> mat_par(const or_mat& m) {
  MatPar<T> q;
  q.gamma = T(m.gamma);
  q.pinf = T(m.pinf);
  q.G0 = T(m.G0);
  q.yield = T(m.yield);
  return q;
}

template <class T> Eos<T> eos_eval(const or_mat& m, const MatPar<T>& q, const T& rho, const T& J2) {
  using std::pow;
  Eos<T> e;
  if (m.eos == OR_EOS_IDEAL) {
    e.Gam = q.gamma - 1.0;
    e.pref = T(0); e.eref = T(0); e.dpref = T(0); e.deref = T(0); e.G = T(0);
  } else if (m.eos == OR_EOS_STIFFENED) {
    e.Gam = q.gamma - 1.0;
    e.pref = -q.gamma * q.pinf;
    e.eref = T(m.eref);
    e.dpref = T(0); e.deref = T(0); e.G = T(0);
  } else if (m.eos == OR_EOS_JWL) {
    /* JWL reference curves of Sec. 2.3 with constant Gamma; p_ref = rho^2
       de_ref/drho holds for this pair, so de_ref/drho = p_ref / rho^2 */
    using std::exp;
    T v = m.rho0 / rho;
    T xa = exp(-m.jwl_R1 * v), xb = exp(-m.jwl_R2 * v);
    T pa = m.jwl_A * xa, pb = m.jwl_B * xb;
    e.Gam = T(m.Gamma0);
    e.pref = pa + pb;
    e.eref = pa / (m.jwl_R1 * m.rho0) + pb / (m.jwl_R2 * m.rho0);
    e.dpref = (m.jwl_R1 * pa + m.jwl_R2 * pb) * m.rho0 / (rho * rho);
    e.deref = e.pref / (rho * rho);
    e.G = T(0);
  } else {
    T x = rho / m.rho0;
    T xa = pow(x, m.abar);
    T ec = m.K0 * sq(xa - 1.0) / (2.0 * m.rho0 * m.abar * m.abar);
    T pc = (m.K0 / m.abar) * x * xa * (xa - 1.0);
    T dpc = (m.K0 / (m.abar * m.rho0)) * ((2.0 * m.abar + 1.0) * xa * xa - (m.abar + 1.0) * xa);
    T G = q.G0 * pow(x, m.bbar + 1.0);
    T es = G * J2 / rho;
    T ps = m.bbar * G * J2;
    T dps = m.bbar * (m.bbar + 1.0) * G * J2 / rho;
    e.Gam = T(m.Gamma0);
    e.pref = pc + ps;
    e.eref = ec + es;
    e.dpref = dpc + dps;
    e.deref = e.pref / (rho * rho);
    e.G = G;
  }
  return e;
}

template <class T> Eos<T> eos_eval(const or_mat& m, const T& rho, const T& J2) {
  return eos_eval(m, mat_par<T>(m), rho, J2);
}

/* isentropic sound speed squared of one Mie-Grueneisen material at (rho, p) */
template <class T> T c2_material(const Eos<T>& e, const T& rho, const T& p) {
  return e.dpref - rho * e.Gam * e.deref + ((1.0 + e.Gam) * p - e.pref) / rho;
}

/* -------------------------------------------------- strain (Sec. 3.2) */
template <class T> void mat_mul(const T A[3][3], const T B[3][3], T C[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = A[i][0] * B[0][j];
      s = s + A[i][1] * B[1][j];
      s = s + A[i][2] * B[2][j];
      C[i][j] = s;
    }
}

/* adjugate (transpose of the cofactor matrix) */
template <class T> void adjugate(const T A[3][3], T R[3][3]) {
  R[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  R[0][1] = A[0][2] * A[2][1] - A[0][1] * A[2][2];
  R[0][2] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
  R[1][0] = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  R[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
  R[1][2] = A[0][2] * A[1][0] - A[0][0] * A[1][2];
  R[2][0] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  R[2][1] = A[0][1] * A[2][0] - A[0][0] * A[2][1];
  R[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
}

/* Hencky strain from the stretch tensor: dev H ~ 1/2 H_B^(1)(V V^T) with
   H_B^(m)(X) = (X^m - X^-m)/(2m), so dev H ~ (B - B^-1)/4 with B = V V^T.
   The inverse of the unimodular B is taken as its cofactor matrix (Sec. 3.2),
   and the deviator of the result is used (the approximation alone is not
   trace free).  J^2 = tr(H H^T) (Sec. 2.2). */
template <class T> void strain(const T V[3][3], T H[3][3], T& J2) {
  T Vt[3][3], B[3][3], A[3][3], K[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Vt[i][j] = V[j][i];
  mat_mul(V, Vt, B);
  adjugate(B, A);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K[i][j] = 0.25 * (B[i][j] - A[i][j]);
  T tr = (K[0][0] + K[1][1] + K[2][2]) / 3.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) H[i][j] = (i == j) ? K[i][j] - tr : K[i][j];
  T s = T(0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s = s + H[i][j] * H[i][j];
  J2 = s;
}

/* first Pade approximant of exp: (I - H/2)^-1 (I + H/2), exact inverse */
template <class T> void pade_exp(const T H[3][3], T V[3][3]) {
  T Mm[3][3], Mp[3][3], A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T id = T(i == j ? 1.0 : 0.0);
      Mm[i][j] = id - 0.5 * H[i][j];
      Mp[i][j] = id + 0.5 * H[i][j];
    }
  adjugate(Mm, A);
  T det = Mm[0][0] * A[0][0] + Mm[0][1] * A[1][0] + Mm[0][2] * A[2][0];
  T P[3][3];
  mat_mul(A, Mp, P);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = P[i][j] / det;
}

/* -------------------------------------------------------- cell state */
template <class T> struct Cell {
  T phi[MAXM], rho[MAXM];  // rho[y] is the mixture density of the reactive material
  T lam;
  T eps;  // plastic strain of the Johnson-Cook material
  T u[3];
  T V[3][3];
  T H[3][3], J2;
  Eos<T> e[MAXM];
  // reactive split (Appendix B): s = volume fraction of the reactant inside y
  T s, rho_a, rho_b;
  Eos<T> ea, eb;
  T g[MAXM];  // effective 1/Gamma per unit volume fraction
  T xi, rho_mix, p, rhoe, Gmix, c2, cL2;
  T sig[3][3];
};

template <class T> struct Ctx {
  const or_config& c;
  Lay L;
  int y;  // reactive material or -1
  MatPar<T> mp[MAXM];
  explicit Ctx(const or_config& cc, const MatPar<T>* par = nullptr) : c(cc), L(cc), y(cc.rx.mat) {
    for (int l = 0; l < cc.nmat && l < MAXM; ++l) mp[l] = par ? par[l] : mat_par<T>(cc.mat[l]);
  }
};

template <class T> void kin_and_strain(const Ctx<T>& X, Cell<T>& C) {
  strain(C.V, C.H, C.J2);
  for (int l = 0; l < X.L.N; ++l)
    if (l != X.y) C.e[l] = eos_eval(X.c.mat[l], X.mp[l], C.rho[l], C.J2);
}

/* reactive component closures at the split t = rho_alpha / (rho_alpha +
   rho_beta) (Sec. 2.3.1, Appendix B).  With the specific-volume rule 1/rho_y
   = lam/rho_alpha + (1-lam)/rho_beta, D = lam (1-t) + (1-lam) t gives
   rho_alpha = rho_y D / (1-t), rho_beta = rho_y D / t, and the reactant's
   volume share s = lam rho_y / rho_alpha = lam (1-t) / D (t = 1/2: equal
   densities, s = lam).  Both components are treated as fluids (no shear
   energy); the product reference energy carries -Q.  Pure limits (lam within
   1e-12 of 0 or 1, or t outside (0, 1)) take both at rho_y. */
template <class T> void rx_components(const Ctx<T>& X, Cell<T>& C, const T& t) {
  const or_rx& r = X.c.rx;
  int y = X.y;
  T lam = C.lam;
  bool pure = !(lam > T(1e-12) && lam < T(1.0 - 1e-12)) || !(t > T(0) && t < T(1));
  if (pure) {
    C.rho_a = C.rho[y];
    C.rho_b = C.rho[y];
    C.s = lam;
  } else {
    T D = lam * (1.0 - t) + (1.0 - lam) * t;
    C.rho_a = C.rho[y] * D / (1.0 - t);
    C.rho_b = C.rho[y] * D / t;
    C.s = lam * (1.0 - t) / D;
  }
  C.ea = eos_eval(r.reactant, C.rho_a, T(0));
  C.eb = eos_eval(r.product, C.rho_b, T(0));
  C.eb.eref = C.eb.eref - r.Q;
}

/* pressure function of Appendix B (the equation that gives p from the
   conserved energy), for a given split t of the reactive material */
template <class T> T pressure_from_split(const Ctx<T>& X, Cell<T>& C, const T& rhoe, const T& t) {
  const Lay& L = X.L;
  T den = T(0), num = rhoe;
  for (int l = 0; l < L.N; ++l) {
    if (l == X.y) continue;
    den = den + C.phi[l] / C.e[l].Gam;
    num = num + C.phi[l] * C.rho[l] * (C.e[l].pref / (C.rho[l] * C.e[l].Gam) - C.e[l].eref);
  }
  if (X.y >= 0) {
    int y = X.y;
    rx_components(X, C, t);
    T wa = C.phi[y] * C.rho[y] * C.lam, wb = C.phi[y] * C.rho[y] * (1.0 - C.lam);
    den = den + wa / (C.rho_a * C.ea.Gam) + wb / (C.rho_b * C.eb.Gam);
    num = num + wa * (C.ea.pref / (C.rho_a * C.ea.Gam) - C.ea.eref) +
          wb * (C.eb.pref / (C.rho_b * C.eb.Gam) - C.eb.eref);
  }
  return num / den;
}

/* temperature of a component, T = (p - p_ref) / (rho Gamma C_V) (Appendix B) */
template <class T> T temperature(const Eos<T>& e, const T& rho, const T& p, double cv) {
  return (p - e.pref) / (rho * e.Gam * cv);
}

enum class Known { Energy, Pressure };

/* Appendix B: the split with T_alpha = T_beta, t = rho_alpha / (rho_alpha +
   rho_beta) on (0, 1), a monotone function of the reactant density the paper
   bisects on (the specific-volume rule fixes rho_beta).  For physical states
   the residual g = T_beta - T_alpha grows with t (a denser reactant is colder
   at a given pressure), g(0+) < 0 < g(1-); away from them (traces of the
   explosive in another material, low-density JWL reactant) g can change sign
   several times, and the appendix does not say which root to take.  The rule
   used: the first sign change met going outward from equal densities (t =
   1/2, the split both pure limits take) towards the side g's sign points to,
   i.e. the root nearest equal densities on that side, found on a fixed probe
   sequence:
     1. t = 3/4, 7/8, ... (g < 0 at 1/2) or t = 1/4, 1/8, ... (g >= 0), each
        probe halving the distance left to the end, until g changes sign;
     2. the first bracket so found, crossed from its inner end in RX_SUBSTEPS
        equal steps until g changes sign again;
     3. that sub-bracket halved until its midpoint is one of its ends.
   Where g keeps its sign at every probe of step 1 the ends are taken: t = 1
   (the pure state) once the probes reach 1 in double precision, t = 2^-65
   after 64 probes down.  With the conserved energy known p comes from the
   pressure function; with p known it is used directly.  Pure cells return
   t = 1 (no split). */
constexpr int RX_SUBSTEPS = 8;

template <class T> T rx_solve(const Ctx<T>& X, Cell<T>& C, Known kind, const T& rhoe, const T& p) {
  const or_rx& r = X.c.rx;
  if (!(C.lam > T(1e-12) && C.lam < T(1.0 - 1e-12))) return T(1);
  auto below = [&](const T& t) {
    T pp = (kind == Known::Energy) ? pressure_from_split(X, C, rhoe, t) : p;
    if (kind == Known::Pressure) rx_components(X, C, t);
    return temperature(C.eb, C.rho_b, pp, r.product.cv) - temperature(C.ea, C.rho_a, pp, r.reactant.cv) < T(0);
  };
  // 1. the probe ladder: [lo, hi] ends as the first bracket, `inner` its end
  // nearer 1/2
  const bool up = below(T(0.5));
  T inner = T(0.5), outer = T(0.5);
  bool flipped = false;
  for (int k = 2; k <= 64; ++k) {
    outer = up ? T(0.5) * (inner + T(1)) : T(0.5) * inner;
    if (up && !(outer < T(1))) return T(1);
    if (below(outer) != up) {
      flipped = true;
      break;
    }
    inner = outer;
  }
  if (!flipped) return T(0.5) * inner;  // g >= 0 at every probe down to 2^-64
  // 2. equal steps across the bracket from its inner end
  const T base = inner, w = (outer - inner) / T(RX_SUBSTEPS);
  for (int j = 1; j < RX_SUBSTEPS; ++j) {
    const T t = base + T(double(j)) * w;
    if (below(t) != up) {
      outer = t;
      break;
    }
    inner = t;
  }
  // 3. halve the sub-bracket down to adjacent doubles
  T lo = up ? inner : outer, hi = up ? outer : inner;
  for (int it = 0; it < 200; ++it) {
    const T mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (below(mid))
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* mixture weights, modulus, sound speeds and stress once p is known
   (Sec. 2.2 mixture rules; the sound speed is read as the Allaire form
   sum(Y_l c_l^2 / Gamma_l) / sum(phi_l / Gamma_l), the longitudinal speed as
   c^2 + 4G/(3 rho); stress sigma = -p I + 2 G dev H, i.e. tension positive) */
template <class T> void finish(const Ctx<T>& X, Cell<T>& C) {
  const Lay& L = X.L;
  T rho = T(0);
  for (int l = 0; l < L.N; ++l) rho = rho + C.phi[l] * C.rho[l];
  C.rho_mix = rho;
  T xi = T(0), gnum = T(0), cnum = T(0);
  for (int l = 0; l < L.N; ++l) {
    T cl2, gl;
    if (l == X.y) {
      // reactive mixture sound speed (Sec. 2.3.1), component derivatives at
      // fixed component density with d rho_k / d rho_y = rho_k / rho_y
      T lam = C.lam, p = C.p;
      // volume fractions of the components inside y: lam rho_y / rho_a, (1-lam) rho_y / rho_b
      gl = (lam * C.rho[l] / C.rho_a) / C.ea.Gam + ((1.0 - lam) * C.rho[l] / C.rho_b) / C.eb.Gam;
      T dEdp = lam / (C.rho_a * C.ea.Gam) + (1.0 - lam) / (C.rho_b * C.eb.Gam);
      T dEa = -(p - C.ea.pref) / (C.rho_a * C.rho_a * C.ea.Gam) - C.ea.dpref / (C.rho_a * C.ea.Gam) + C.ea.deref;
      T dEb = -(p - C.eb.pref) / (C.rho_b * C.rho_b * C.eb.Gam) - C.eb.dpref / (C.rho_b * C.eb.Gam) + C.eb.deref;
      T ry = C.rho[l];
      T dEdr = lam * dEa * (C.rho_a / ry) + (1.0 - lam) * dEb * (C.rho_b / ry);
      cl2 = (p / (ry * ry) - dEdr) / dEdp;
    } else {
      gl = 1.0 / C.e[l].Gam;
      cl2 = c2_material(C.e[l], C.rho[l], C.p);
      gnum = gnum + C.phi[l] * C.e[l].G * gl;
    }
    C.g[l] = gl;
    xi = xi + C.phi[l] * gl;
    cnum = cnum + (C.phi[l] * C.rho[l] / rho) * cl2 * gl;
  }
  C.xi = xi;
  C.Gmix = gnum / xi;
  C.c2 = cnum / xi;
  C.cL2 = C.c2 + 4.0 * C.Gmix / (3.0 * rho);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.sig[i][j] = 2.0 * C.Gmix * C.H[i][j] - ((i == j) ? C.p : T(0));
}

/* conserved -> primitive for one cell (U has F entries) */
template <class T> void from_cons(const Ctx<T>& X, const T* U, Cell<T>& C) {
  const Lay& L = X.L;
  T sphi = T(0);
  for (int l = 0; l < L.N - 1; ++l) {
    C.phi[l] = U[L.phi(l)];
    sphi = sphi + C.phi[l];
  }
  C.phi[L.N - 1] = 1.0 - sphi;
  T rho = T(0);
  for (int l = 0; l < L.N; ++l) {
    C.rho[l] = U[L.m(l)] / C.phi[l];
    rho = rho + U[L.m(l)];
  }
  for (int k = 0; k < 3; ++k) C.u[k] = (k < L.D) ? U[L.mom(k)] / rho : T(0);
  C.lam = T(0);
  if (X.y >= 0) C.lam = tmin(tmax(U[L.lam()] / U[L.m(X.y)], T(0)), T(1));
  C.eps = T(0);
  if (L.ep >= 0 && U[L.m(L.ep)] > T(0)) C.eps = U[L.lam()] / U[L.m(L.ep)];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.V[i][j] = T(0);
  for (int q = 0; q < L.nV; ++q) C.V[L.vi[q]][L.vj[q]] = U[L.V(q)];
  kin_and_strain(X, C);
  T uu = T(0);
  for (int k = 0; k < L.D; ++k) uu = uu + C.u[k] * C.u[k];
  T rhoe = U[L.E()] - 0.5 * rho * uu;
  C.rhoe = rhoe;
  if (X.y >= 0) {
    T t = rx_solve(X, C, Known::Energy, rhoe, T(0));
    C.p = pressure_from_split(X, C, rhoe, t);
  } else {
    C.s = T(0);
    C.p = pressure_from_split(X, C, rhoe, T(0));
  }
  finish(X, C);
}

/* primitive -> cell state (W has F entries in primitive slots) */
template <class T> void from_prim(const Ctx<T>& X, const T* W, Cell<T>& C) {
  const Lay& L = X.L;
  T sphi = T(0);
  for (int l = 0; l < L.N - 1; ++l) {
    C.phi[l] = W[L.phi(l)];
    sphi = sphi + C.phi[l];
  }
  C.phi[L.N - 1] = 1.0 - sphi;
  for (int l = 0; l < L.N; ++l) C.rho[l] = W[L.m(l)];
  for (int k = 0; k < 3; ++k) C.u[k] = (k < L.D) ? W[L.mom(k)] : T(0);
  C.lam = T(0);
  if (X.y >= 0) C.lam = tmin(tmax(W[L.lam()], T(0)), T(1));
  C.eps = (L.ep >= 0) ? W[L.lam()] : T(0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.V[i][j] = T(0);
  for (int q = 0; q < L.nV; ++q) C.V[L.vi[q]][L.vj[q]] = W[L.V(q)];
  kin_and_strain(X, C);
  C.p = W[L.E()];
  // rho e = sum phi_l rho_l e_l with e_l = (p - p_ref)/(rho_l Gamma_l) + e_ref
  T rhoe = T(0);
  for (int l = 0; l < L.N; ++l) {
    if (l == X.y) continue;
    rhoe = rhoe + C.phi[l] * ((C.p - C.e[l].pref) / C.e[l].Gam + C.rho[l] * C.e[l].eref);
  }
  C.s = T(0);
  if (X.y >= 0) {
    int y = X.y;
    T t = rx_solve(X, C, Known::Pressure, T(0), C.p);
    rx_components(X, C, t);
    T wa = C.phi[y] * C.rho[y] * C.lam, wb = C.phi[y] * C.rho[y] * (1.0 - C.lam);
    rhoe = rhoe + wa * ((C.p - C.ea.pref) / (C.rho_a * C.ea.Gam) + C.ea.eref) +
           wb * ((C.p - C.eb.pref) / (C.rho_b * C.eb.Gam) + C.eb.eref);
  }
  C.rhoe = rhoe;
  finish(X, C);
}

template <class T> void cell_to_cons(const Ctx<T>& X, const Cell<T>& C, T* U) {
  const Lay& L = X.L;
  for (int l = 0; l < L.N - 1; ++l) U[L.phi(l)] = C.phi[l];
  for (int l = 0; l < L.N; ++l) U[L.m(l)] = C.phi[l] * C.rho[l];
  if (X.y >= 0) U[L.lam()] = C.phi[X.y] * C.rho[X.y] * C.lam;
  if (L.ep >= 0) U[L.lam()] = C.phi[L.ep] * C.rho[L.ep] * C.eps;
  T uu = T(0);
  for (int k = 0; k < L.D; ++k) {
    U[L.mom(k)] = C.rho_mix * C.u[k];
    uu = uu + C.u[k] * C.u[k];
  }
  U[L.E()] = C.rhoe + 0.5 * C.rho_mix * uu;
  for (int q = 0; q < L.nV; ++q) U[L.V(q)] = C.V[L.vi[q]][L.vj[q]];
}

template <class T> void cell_to_prim(const Ctx<T>& X, const Cell<T>& C, T* W) {
  const Lay& L = X.L;
  for (int l = 0; l < L.N - 1; ++l) W[L.phi(l)] = C.phi[l];
  for (int l = 0; l < L.N; ++l) W[L.m(l)] = C.rho[l];
  if (X.y >= 0) W[L.lam()] = C.lam;
  if (L.ep >= 0) W[L.lam()] = C.eps;
  for (int k = 0; k < L.D; ++k) W[L.mom(k)] = C.u[k];
  W[L.E()] = C.p;
  for (int q = 0; q < L.nV; ++q) W[L.V(q)] = C.V[L.vi[q]][L.vj[q]];
}

/* physical flux in direction n (Sec. 3 vector form); the phi slots carry
   phi u_n (the advective part; its source phi div u is handled in the update) */
template <class T> void phys_flux(const Ctx<T>& X, const Cell<T>& C, const T* U, int n, T* Fx) {
  const Lay& L = X.L;
  T un = C.u[n];
  for (int l = 0; l < L.N - 1; ++l) Fx[L.phi(l)] = U[L.phi(l)] * un;
  for (int l = 0; l < L.N; ++l) Fx[L.m(l)] = U[L.m(l)] * un;
  if (L.xf) Fx[L.lam()] = U[L.lam()] * un;
  for (int k = 0; k < L.D; ++k) Fx[L.mom(k)] = U[L.mom(k)] * un - C.sig[k][n];
  T us = T(0);
  for (int k = 0; k < 3; ++k) us = us + C.u[k] * C.sig[k][n];
  Fx[L.E()] = U[L.E()] * un - us;
  for (int q = 0; q < L.nV; ++q) {
    int i = L.vi[q], j = L.vj[q];
    Fx[L.V(q)] = C.V[i][j] * un - C.V[n][j] * C.u[i];
  }
}

/* --------------------------------------------- HLLC-type Riemann solver */
template <class T> struct Face {
  T F[FMAX];
  T ustar;
  T Vn[3];
};

/* Three-wave solver for the whole system.  Wave speeds S_L, S_R are Davis
   bounds on the longitudinal speed.  The single velocity of the model (Sec.
   2.1: one velocity shared by all materials, a 'stick' condition between
   solids) makes the contact carry continuous velocity and traction:
   S* and the tangential star velocity follow from traction continuity,
   star states from the Rankine-Hugoniot conditions across S_K. */
template <class T> void star_flux(const Ctx<T>& X, const Cell<T>& C, const T* U, const T* Fx, int n,
                                  const T& SK, const T& Sst, const T ust[3], const T& mK, T* Fout,
                                  T& ustar_out, T Vn_out[3]) {
  const Lay& L = X.L;
  T un = C.u[n];
  T r = (SK - un) / (SK - Sst);
  T Us[FMAX];
  for (int l = 0; l < L.N - 1; ++l) Us[L.phi(l)] = r * U[L.phi(l)];
  for (int l = 0; l < L.N; ++l) Us[L.m(l)] = r * U[L.m(l)];
  if (L.xf) Us[L.lam()] = r * U[L.lam()];
  T rs = r * C.rho_mix;
  for (int k = 0; k < L.D; ++k) Us[L.mom(k)] = rs * ust[k];
  T sst[3];
  for (int k = 0; k < 3; ++k) sst[k] = C.sig[k][n] - mK * (ust[k] - C.u[k]);
  T usK = T(0), usS = T(0);
  for (int k = 0; k < 3; ++k) {
    usK = usK + C.u[k] * C.sig[k][n];
    usS = usS + ust[k] * sst[k];
  }
  Us[L.E()] = (U[L.E()] * (SK - un) + (usK - usS)) / (SK - Sst);
  for (int q = 0; q < L.nV; ++q) {
    int i = L.vi[q], j = L.vj[q];
    if (i == n)
      Us[L.V(q)] = C.V[i][j];
    else
      Us[L.V(q)] = ((SK - un) * C.V[i][j] - C.V[n][j] * (ust[i] - C.u[i])) / (SK - Sst);
  }
  for (int f = 0; f < L.F; ++f) Fout[f] = Fx[f] + SK * (Us[f] - U[f]);
  ustar_out = un + SK * (r - 1.0);
  // volume-fraction flux written as phi_K u*, the same u* as in its source term
  for (int l = 0; l < L.N - 1; ++l) Fout[L.phi(l)] = U[L.phi(l)] * ustar_out;
  for (int j = 0; j < 3; ++j) Vn_out[j] = C.V[n][j];
}

template <class T> void riemann(const Ctx<T>& X, const Cell<T>& CL, const Cell<T>& CR, int n, Face<T>& out) {
  using std::sqrt;
  const Lay& L = X.L;
  T UL[FMAX], UR[FMAX], FL[FMAX], FR[FMAX];
  cell_to_cons(X, CL, UL);
  cell_to_cons(X, CR, UR);
  phys_flux(X, CL, UL, n, FL);
  phys_flux(X, CR, UR, n, FR);
  T cl = sqrt(CL.cL2), cr = sqrt(CR.cL2);
  T uL = CL.u[n], uR = CR.u[n];
  T SL = tmin(uL - cl, uR - cr);
  T SR = tmax(uL + cl, uR + cr);
  if (SL >= T(0)) {
    for (int f = 0; f < L.F; ++f) out.F[f] = FL[f];
    out.ustar = uL;
    for (int j = 0; j < 3; ++j) out.Vn[j] = CL.V[n][j];
    return;
  }
  if (SR <= T(0)) {
    for (int f = 0; f < L.F; ++f) out.F[f] = FR[f];
    out.ustar = uR;
    for (int j = 0; j < 3; ++j) out.Vn[j] = CR.V[n][j];
    return;
  }
  T mL = CL.rho_mix * (SL - uL);
  T mR = CR.rho_mix * (SR - uR);
  T den = mL - mR;
  T ust[3];
  for (int k = 0; k < 3; ++k)
    ust[k] = ((CL.sig[k][n] - CR.sig[k][n]) + (mL * CL.u[k] - mR * CR.u[k])) / den;
  T Sst = ust[n];
  if (Sst > T(0)) {
    star_flux(X, CL, UL, FL, n, SL, Sst, ust, mL, out.F, out.ustar, out.Vn);
  } else if (Sst < T(0)) {
    star_flux(X, CR, UR, FR, n, SR, Sst, ust, mR, out.F, out.ustar, out.Vn);
  } else {
    Face<T> a, b;
    star_flux(X, CL, UL, FL, n, SL, Sst, ust, mL, a.F, a.ustar, a.Vn);
    star_flux(X, CR, UR, FR, n, SR, Sst, ust, mR, b.F, b.ustar, b.Vn);
    for (int f = 0; f < L.F; ++f) out.F[f] = 0.5 * (a.F[f] + b.F[f]);
    out.ustar = 0.5 * (a.ustar + b.ustar);
    for (int j = 0; j < 3; ++j) out.Vn[j] = 0.5 * (a.Vn[j] + b.Vn[j]);
  }
}

/* ------------------------------------------------ reconstruction pieces */
template <class T> T minmod(const T& a, const T& b) {
  if (a * b <= T(0)) return T(0);
  return (tabs(a) < tabs(b)) ? a : b;
}

template <class T> T vanalbada(const T& a, const T& b, double e2) {
  return (a * (b * b + e2) + b * (a * a + e2)) / (a * a + b * b + 2.0 * e2);
}

template <class T> T sgn(const T& x) { return (x > T(0)) ? T(1) : ((x < T(0)) ? T(-1) : T(0)); }

/* THINC edge values of Appendix A.  The tanh profile is evaluated in the
   orientation where it increases (theta = +1); a decreasing stencil is
   mirrored first and its edges swapped back, which is the same function and
   keeps mirror images exact in floating point. */
template <class T> void thinc_edges(const T& qm, const T& q0, const T& qp, const T& beta, double eps,
                                    T& qL, T& qR, T& C) {
  using std::cosh;
  using std::exp;
  using std::tanh;
  T qmin = tmin(qm, qp);
  T qmax = tmax(qm, qp) - qmin;
  C = (q0 - qmin + eps) / (qmax + eps);
  T theta = sgn(qp - qm);
  T Bv = exp(beta * (2.0 * C - 1.0));
  T tb = tanh(beta);
  T A = (Bv / cosh(beta) - 1.0) / tb;
  T lo = qmin + 0.5 * qmax * (1.0 + A);
  T hi = qmin + 0.5 * qmax * (1.0 + (tb + A) / (1.0 + A * tb));
  if (theta < T(0)) {
    qL = hi;
    qR = lo;
  } else {
    qL = lo;
    qR = hi;
  }
}

/* mixed-cell test of Appendix A: delta < C < 1 - delta and monotone */
template <class T> bool thinc_mixed(const T& qm, const T& q0, const T& qp, const T& C, double delta) {
  return (T(delta) < C) && (C < T(1.0 - delta)) && ((qp - q0) * (q0 - qm) > T(0));
}

/* BVD choice of Appendix A for cell i: TBV^P is the least of the four
   boundary variations that pair P's edges of cell i with the MUSCL or THINC
   edges of the neighbours (MUSCL|MUSCL, THINC|THINC, MUSCL|THINC,
   THINC|MUSCL for the right edge of i-1 and the left edge of i+1); THINC is
   taken only if TBV^THINC < TBV^MUSCL.  Inputs: the right-edge candidates of
   i-1 (mRa, tRa), both candidates of i, the left-edge candidates of i+1
   (mLe, tLe).  v (nullable) receives the four variations for P = MUSCL then
   P = THINC. */
template <class T> bool bvd_thinc(const T& mRa, const T& tRa, const T& mLb, const T& mRb, const T& tLb, const T& tRb,
                                  const T& mLe, const T& tLe, T* v = nullptr) {
  auto tbv = [&](const T& Lp, const T& Rp, T* w) {
    T v1 = tabs(mRa - Lp) + tabs(Rp - mLe);
    T v2 = tabs(tRa - Lp) + tabs(Rp - tLe);
    T v3 = tabs(mRa - Lp) + tabs(Rp - tLe);
    T v4 = tabs(tRa - Lp) + tabs(Rp - mLe);
    if (w) {
      w[0] = v1;
      w[1] = v2;
      w[2] = v3;
      w[3] = v4;
    }
    return tmin(tmin(v1, v2), tmin(v3, v4));
  };
  T tbvM = tbv(mLb, mRb, v);
  T tbvT = tbv(tLb, tRb, v ? v + 4 : nullptr);
  return tbvT < tbvM;
}

/* the MUSCL and THINC edge candidates of one cell of a volume-fraction
   stencil (qm, q0, qp) with limited slope s and steepness beta: MUSCL
   q0 -+ s/2; THINC edges where the cell is mixed, else the MUSCL ones */
template <class T> void phi_candidates(const or_config& c, const T& qm, const T& q0, const T& qp, const T& s,
                                       const T& beta, T& ml, T& mr, T& tl, T& tr) {
  ml = q0 - 0.5 * s;
  mr = q0 + 0.5 * s;
  tl = ml;
  tr = mr;
  if (c.thinc) {
    T ql, qr, C;
    thinc_edges(qm, q0, qp, beta, c.eps, ql, qr, C);
    if (thinc_mixed(qm, q0, qp, C, c.delta)) {
      tl = ql;
      tr = qr;
    }
  }
}

/* Youngs normal component |n_d| from 1-2-1 weighted central differences of
   phi_1 over the 3 (2-D) or 3x3 (3-D) transverse neighbours; symmetric pairs
   are summed first so that mirror images are exact.  1-D: |n| = 1. */
template <class T> T youngs_nd(const Ctx<T>& X, const T* cons, int64_t nc, const int64_t p[3], int d) {
  using std::sqrt;
  const or_config& c = X.c;
  int D = c.ndim;
  if (D == 1) return T(1);
  auto phi = [&](int64_t a, int64_t b, int64_t e) {
    int64_t q[3] = {p[0] + a, p[1] + b, p[2] + e};
    return cons[X.L.phi(0) * nc + cell_at(c, q)];
  };
  T g[3] = {T(0), T(0), T(0)};
  for (int e = 0; e < D; ++e) {
    auto diff = [&](int t1, int t2) {
      // offset +-1 along e, t1 along the first other axis, t2 along the second
      int64_t o[3] = {0, 0, 0}, m[3] = {0, 0, 0};
      int others[2], no = 0;
      for (int a = 0; a < D; ++a)
        if (a != e) others[no++] = a;
      o[e] = 1;
      m[e] = -1;
      if (no > 0) { o[others[0]] += t1; m[others[0]] += t1; }
      if (no > 1) { o[others[1]] += t2; m[others[1]] += t2; }
      return phi(o[0], o[1], o[2]) - phi(m[0], m[1], m[2]);
    };
    T s;
    if (D == 2) {
      s = (diff(-1, 0) + diff(1, 0)) + 2.0 * diff(0, 0);
    } else {
      T corners = (diff(-1, -1) + diff(1, 1)) + (diff(-1, 1) + diff(1, -1));
      T edges = (diff(-1, 0) + diff(1, 0)) + (diff(0, -1) + diff(0, 1));
      s = (corners + 2.0 * edges) + 4.0 * diff(0, 0);
    }
    g[e] = s / c.dx[e];
  }
  T nn = T(0);
  for (int e = 0; e < D; ++e) nn = nn + g[e] * g[e];
  T norm = sqrt(nn);
  if (!(norm > T(0))) return T(1);
  return tabs(g[d]) / norm;
}

/* scale used by the van Albada epsilon for primitive slot f */
double va_scale_of(const Lay& L, const or_config& c, int f) {
  if (f < L.N - 1) return c.va_scale[0];
  if (f < 2 * L.N - 1) return c.va_scale[1];
  if (L.xf && f == L.lam()) return c.va_scale[2];
  if (f < L.E()) return c.va_scale[3];
  if (f == L.E()) return c.va_scale[4];
  return c.va_scale[5];
}

/* ------------------------------------------------------------ one sweep */
/* Dimensionally split MUSCL-Hancock sweep in direction d over the whole grid:
   primitive reconstruction with a limiter, THINC/BVD on the volume fractions,
   a primitive half-step predictor, the HLLC-type face flux and the
   conservative update with the non-conservative terms of phi and Vbar. */
/* rhs != nullptr selects the unsplit form of Sec. 3.1 (the method of lines
   with the SSP-RK3 of eq. (rk)): the edges are the MUSCL/THINC/BVD
   reconstruction alone (no half-step predictor, no clipping), and the
   direction's part of the spatial operator D(q) of eq. (spat_op),
   ((F_{i+1/2} - F_{i-1/2}) - s_non-con) / dx_d, is added to rhs; out and dt
   are then unused. */
/* the mirror image across a wall normal to dimension d: the normal momentum
   and the stretch-tensor entries with exactly one normal index change sign
   (V -> M V M with M the reflection) */
template <class T> void mirror_state(const Lay& L, int d, T* U) {
  U[L.mom(d)] = -U[L.mom(d)];
  for (int q = 0; q < L.nV; ++q)
    if ((L.vi[q] == d) != (L.vj[q] == d)) U[L.V(q)] = -U[L.V(q)];
}

template <class T> void sweep_grid(const or_config& c, const T* in, T* out, T dt, int d,
                                   const MatPar<T>* par = nullptr, T* rhs = nullptr, T* fout = nullptr) {
  Ctx<T> X(c, par);
  const Lay& L = X.L;
  const int F = L.F;
  const int64_t nc = ncell(c);
  const int64_t n = c.n[d];
  const T nu = dt / c.dx[d];
  // enumerate pencils: all cells with coordinate 0 along d
  std::vector<int64_t> starts;
  for (int64_t cell = 0; cell < nc; ++cell) {
    int64_t p[3];
    pos_of(c, cell, p);
    if (p[d] == 0) starts.push_back(cell);
  }
  const int64_t npen = (int64_t)starts.size();
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads)
  for (int64_t ip = 0; ip < npen; ++ip) {
    int64_t p0[3];
    pos_of(c, starts[ip], p0);
    const int64_t G = 3;                  // stencil reach per side
    const int64_t W = n + 2 * G;          // cells -3 .. n+2
    std::vector<Cell<T>> cellv(W);
    std::vector<T> prim(W * F), Uc(W * F);
    std::vector<int64_t> gid(W);
    for (int64_t i = -G; i < n + G; ++i) {
      int64_t p[3] = {p0[0], p0[1], p0[2]};
      p[d] = i;
      bool flip[3] = {false, false, false};
      int64_t id = cell_at(c, p, flip);
      gid[i + G] = id;
      T* U = &Uc[(i + G) * F];
      for (int f = 0; f < F; ++f) U[f] = in[f * nc + id];
      if (flip[d]) mirror_state(L, d, U);
      from_cons(X, U, cellv[i + G]);
      cell_to_prim(X, cellv[i + G], &prim[(i + G) * F]);
    }
    auto Wp = [&](int64_t i) { return &prim[(i + G) * F]; };
    // limited slopes and MUSCL edges for cells -2 .. n+1
    std::vector<T> slope(W * F, T(0));
    for (int64_t i = -G + 1; i < n + G - 1; ++i) {
      for (int f = 0; f < F; ++f) {
        T a = Wp(i)[f] - Wp(i - 1)[f];
        T b = Wp(i + 1)[f] - Wp(i)[f];
        T s;
        if (c.limiter == OR_LIM_VANALBADA) {
          double e = 1e-6 * va_scale_of(L, c, f);
          s = vanalbada(a, b, e * e);
        } else {
          s = minmod(a, b);
        }
        slope[(i + G) * F + f] = s;
      }
    }
    // phi candidates (MUSCL and THINC edges) for cells -2 .. n+1
    const int nphi = L.N - 1;
    std::vector<T> mL(W * MAXM), mR(W * MAXM), tL(W * MAXM), tR(W * MAXM);
    for (int64_t i = -G + 1; i < n + G - 1; ++i) {
      for (int l = 0; l < nphi; ++l) {
        T q0 = Wp(i)[L.phi(l)];
        T s = slope[(i + G) * F + L.phi(l)];
        T qm = Wp(i - 1)[L.phi(l)], qp = Wp(i + 1)[L.phi(l)];
        T beta = T(0);
        if (c.thinc) {
          // interface normal from phi_1; a cell outside the grid sees the grid
          // extended by the boundary rule, like its own values
          int64_t pc[3] = {p0[0], p0[1], p0[2]};
          pc[d] = i;
          T nd = youngs_nd(X, in, nc, pc, d);
          beta = c.beta0 * nd + 0.01;
        }
        T ml, mr, tl, tr;
        phi_candidates(c, qm, q0, qp, s, beta, ml, mr, tl, tr);
        mL[(i + G) * MAXM + l] = ml;
        mR[(i + G) * MAXM + l] = mr;
        tL[(i + G) * MAXM + l] = tl;
        tR[(i + G) * MAXM + l] = tr;
      }
    }
    // edges (with BVD choice) and the predictor, for cells -1 .. n
    std::vector<T> WL(W * F), WR(W * F);
    for (int64_t i = -1; i < n + 1; ++i) {
      T* wl = &WL[(i + G) * F];
      T* wr = &WR[(i + G) * F];
      const T* w = Wp(i);
      for (int f = 0; f < F; ++f) {
        T s = slope[(i + G) * F + f];
        wl[f] = w[f] - 0.5 * s;
        wr[f] = w[f] + 0.5 * s;
      }
      if (c.thinc) {
        for (int l = 0; l < nphi; ++l) {
          int a = (i - 1 + G) * MAXM + l, b = (i + G) * MAXM + l, e = (i + 1 + G) * MAXM + l;
          if (bvd_thinc(mR[a], tR[a], mL[b], mR[b], tL[b], tR[b], mL[e], tL[e])) {
            wl[L.phi(l)] = tL[b];
            wr[L.phi(l)] = tR[b];
          } else {
            wl[L.phi(l)] = mL[b];
            wr[L.phi(l)] = mR[b];
          }
        }
      }
      if (rhs) continue;  // unsplit: the reconstructed edges are the face states
      // primitive predictor: W-bar = W_edge - (nu/2) A(W_i) (W_R - W_L)
      const Cell<T>& Ci = cellv[i + G];
      Cell<T> CeL, CeR;
      from_prim(X, wl, CeL);
      from_prim(X, wr, CeR);
      T dW[FMAX];
      for (int f = 0; f < F; ++f) dW[f] = wr[f] - wl[f];
      T un = Ci.u[d];
      T dun = dW[L.mom(d)];
      T inc[FMAX];
      for (int l = 0; l < nphi; ++l) inc[L.phi(l)] = un * dW[L.phi(l)];
      for (int l = 0; l < L.N; ++l) inc[L.m(l)] = un * dW[L.m(l)] + Ci.rho[l] * dun;
      if (L.xf) inc[L.lam()] = un * dW[L.lam()];
      for (int k = 0; k < L.D; ++k)
        inc[L.mom(k)] = un * dW[L.mom(k)] - (CeR.sig[k][d] - CeL.sig[k][d]) / Ci.rho_mix;
      inc[L.E()] = un * dW[L.E()] + Ci.rho_mix * Ci.c2 * dun;
      for (int q = 0; q < L.nV; ++q) {
        int a = L.vi[q], b = L.vj[q];
        T dua = (a < L.D) ? dW[L.mom(a)] : T(0);
        inc[L.V(q)] = un * dW[L.V(q)] - Ci.V[d][b] * dua + (1.0 / 3.0) * Ci.V[a][b] * dun;
      }
      for (int f = 0; f < F; ++f) {
        wl[f] = wl[f] - 0.5 * nu * inc[f];
        wr[f] = wr[f] - 0.5 * nu * inc[f];
      }
      for (int l = 0; l < nphi; ++l) {
        wl[L.phi(l)] = tmin(tmax(wl[L.phi(l)], T(0)), T(1));
        wr[L.phi(l)] = tmin(tmax(wr[L.phi(l)], T(0)), T(1));
      }
      if (X.y >= 0) {
        wl[L.lam()] = tmin(tmax(wl[L.lam()], T(0)), T(1));
        wr[L.lam()] = tmin(tmax(wr[L.lam()], T(0)), T(1));
      }
    }
    // face fluxes: face f sits between cells f-1 and f, f = 0 .. n
    std::vector<Face<T>> face(n + 1);
    for (int64_t f = 0; f <= n; ++f) {
      Cell<T> CL, CR;
      from_prim(X, &WR[(f - 1 + G) * F], CL);
      from_prim(X, &WL[(f + G) * F], CR);
      riemann(X, CL, CR, d, face[f]);
    }
    if (fout) {
      // the face fluxes of this pencil into the face array (the grid's shape
      // with n_d + 1 faces along d)
      int64_t m[3] = {c.n[0], c.ndim > 1 ? c.n[1] : 1, c.ndim > 2 ? c.n[2] : 1};
      m[d] += 1;
      const int64_t nfaces = m[0] * m[1] * m[2];
      for (int64_t f = 0; f <= n; ++f) {
        int64_t q[3] = {p0[0], p0[1], p0[2]};
        q[d] = f;
        const int64_t idx = q[0] + m[0] * (q[1] + m[1] * q[2]);
        for (int k = 0; k < F; ++k) fout[k * nfaces + idx] = face[f].F[k];
      }
    }
    // update
    for (int64_t i = 0; i < n; ++i) {
      const Face<T>& a = face[i];
      const Face<T>& b = face[i + 1];
      const Cell<T>& Ci = cellv[i + G];
      const T* U = &Uc[(i + G) * F];
      int64_t id = gid[i + G];
      T du = b.ustar - a.ustar;
      T div[FMAX];  // (F_{i+1/2} - F_{i-1/2}) - s_non-con
      for (int l = 0; l < nphi; ++l) {
        int f = L.phi(l);
        div[f] = (b.F[f] - a.F[f]) - Ci.phi[l] * du;
      }
      for (int f = nphi; f < L.V(0); ++f) div[f] = b.F[f] - a.F[f];
      for (int q = 0; q < L.nV; ++q) {
        int f = L.V(q), ii = L.vi[q], jj = L.vj[q];
        T src = (2.0 / 3.0) * Ci.V[ii][jj] * du - Ci.u[ii] * (b.Vn[jj] - a.Vn[jj]);
        div[f] = (b.F[f] - a.F[f]) - src;
      }
      for (int f = 0; f < F; ++f) {
        if (rhs)
          rhs[f * nc + id] = rhs[f * nc + id] + div[f] / c.dx[d];
        else
          out[f * nc + id] = U[f] - nu * div[f];
      }
    }
  }
}

/* ---------------------------------------------------------- plastic step */
/* Sec. 3.2: relax the strain invariant of each material, mix the targets
   with phi/Gamma weights, rescale dev H, and rebuild Vbar = exp(dev H) by the
   first Pade approximant.  Ideal plasticity with an instantaneous rate gives
   the per-material target J*_l = min(J, sigma_Y / (sqrt(6) G_l)); an elastic
   solid keeps J; a fluid (zero shear modulus) relaxes to 0. */
/* Johnson-Cook target of material l (rate law of Sec. 2.3.2, relaxation of
   Sec. 3.2): the root of R(Js) = Js - J + dt chi(Js) on [0, J] by 64
   bisection halvings, with chi = chi0 exp((s - 1)/c3), s = sqrt(6) G Js /
   sigma_Y (sqrt(3/2) |dev sigma| for dev sigma = 2 G dev H), sigma_Y = (c1 +
   c2 eps^n)(1 - theta^m).  The plastic strain gained equals the strain
   invariant relaxed, eps(Js) = eps + (J - Js) (both equations carry the
   same chi); the temperature is that of the state before the relaxation,
   T = T0 + (p - p_ref)/(rho Gamma cv), theta = (T - T0)/(Tmelt - T0) in
   [0, 1]. */
template <class T> T jc_target(const Ctx<T>& X, const Cell<T>& C, int l, const T& J, const T& dt) {
  using std::exp;
  using std::pow;
  using std::sqrt;
  const or_mat& m = X.c.mat[l];
  if (!(dt > T(0))) return J;
  T Tk = m.jc_t0 + (C.p - C.e[l].pref) / (C.rho[l] * C.e[l].Gam * m.cv);
  T theta = tmin(tmax((Tk - m.jc_t0) / (m.jc_tmelt - m.jc_t0), T(0)), T(1));
  T soft = 1.0 - pow(theta, m.jc_m);
  if (!(soft > T(0))) return T(0);  // at or above melt: no strength
  T G6 = sqrt(6.0) * C.e[l].G;
  T lo = T(0), hi = J;
  for (int it = 0; it < 64; ++it) {
    T mid = 0.5 * (lo + hi);
    T ep = tmax(C.eps + (J - mid), T(0));
    T sy = (m.jc_c1 + m.jc_c2 * pow(ep, m.jc_n)) * soft;
    T chi = m.jc_chi0 * exp((G6 * mid / sy - 1.0) / m.jc_c3);
    T R = mid - J + dt * chi;
    if (R < T(0))
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

template <class T> void plastic_cell(const Ctx<T>& X, T* U, const T& dt) {
  using std::sqrt;
  const Lay& L = X.L;
  Cell<T> C;
  from_cons(X, U, C);
  T J = sqrt(C.J2);
  T num = T(0), wsh = T(0);
  T J_ep = J;  // Johnson-Cook target (plastic strain update)
  for (int l = 0; l < L.N; ++l) {
    T Jl = T(0);
    if (l != X.y && X.c.mat[l].eos == OR_EOS_ROMENSKII && X.c.mat[l].G0 > 0.0) {
      Jl = J;
      if (X.c.mat[l].plast == OR_PLAST_PERFECT) {
        T Jy = X.mp[l].yield / (sqrt(6.0) * C.e[l].G);
        Jl = tmin(J, Jy);
      } else if (X.c.mat[l].plast == OR_PLAST_JC) {
        Jl = jc_target(X, C, l, J, dt);
        if (l == L.ep) J_ep = Jl;
      }
      wsh = wsh + C.phi[l] * C.g[l];
    }
    num = num + C.phi[l] * C.g[l] * Jl;
  }
  if (L.ep >= 0 && U[L.m(L.ep)] > T(0)) U[L.lam()] = U[L.m(L.ep)] * (C.eps + (J - J_ep));
  T Jst = num / C.xi;
  /* at J = 0 the factor Jst / J is its limit, the phi/Gamma weight of the
     shear-carrying materials (their targets equal J near 0): the relaxed
     tensor is the identity there either way, and the map stays
     differentiable (its tangent is the limit factor times that of H) */
  T f0 = wsh / C.xi;
  T Hs[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Hs[i][j] = (J > T(0)) ? (Jst / J) * C.H[i][j] : f0 * C.H[i][j];
  T Vn[3][3];
  pade_exp(Hs, Vn);
  for (int q = 0; q < L.nV; ++q) U[L.V(q)] = Vn[L.vi[q]][L.vj[q]];
}

/* --------------------------------------------------------- reaction step */
/* Sec. 3.3: RK4 on d(phi rho lambda)/dt = phi rho lambda-dot with the mass of
   the reactive material and the total energy fixed; each stage re-evaluates
   the pressure from the conserved state at the stage lambda.  Rate (paper
   convention, lambda = 1 reactant): dlambda/dt = -k lambda (max(p,0)/pref)^n. */
/* three-term ignition-and-growth rate of the reacted fraction F = 1 - lam
   (Sec. 4.2, Table 4), rho the mixture material's own density; each term
   holds a positive power of lam = 1 - F, so none acts at lam = 0, and the
   growth terms a positive power of F */
template <class T> T ig_rate(const or_rx& r, const T& lam, const T& rho, const T& p) {
  using std::pow;
  if (!(lam > T(0))) return T(0);
  T F = 1.0 - lam;
  T out = T(0);
  T mu = rho / r.ig_rho0 - 1.0 - r.ig_a;
  if (r.ig_Fig - F > T(0) && mu > T(0)) out = out + r.ig_I * pow(lam, r.ig_b) * pow(mu, r.ig_x);
  T ph = tmax(p, T(0)) / r.ig_punit;
  if (F > T(0)) {
    if (r.ig_FG1 - F > T(0)) out = out + r.ig_G1 * pow(lam, r.ig_c) * pow(F, r.ig_d) * pow(ph, r.ig_y);
    if (F - r.ig_FG2 > T(0)) out = out + r.ig_G2 * pow(lam, r.ig_e) * pow(F, r.ig_g) * pow(ph, r.ig_z);
  }
  return out;
}

template <class T> void reaction_cell(const Ctx<T>& X, T* U, const T& dt) {
  using std::pow;
  const Lay& L = X.L;
  const or_rx& r = X.c.rx;
  int y = X.y;
  T my = U[L.m(y)];
  if (!(my > T(0))) return;
  T lam0 = tmin(tmax(U[L.lam()] / my, T(0)), T(1));
  auto rate = [&](const T& lam) {
    T Uc[FMAX];
    for (int f = 0; f < L.F; ++f) Uc[f] = U[f];
    T lc = tmin(tmax(lam, T(0)), T(1));
    Uc[L.lam()] = my * lc;
    Cell<T> C;
    from_cons(X, Uc, C);
    if (r.law == OR_RATE_IG) return -ig_rate(r, lc, C.rho[y], C.p);
    T pp = tmax(C.p, T(0)) / r.pref;
    return -r.k * lc * pow(pp, r.n);
  };
  T k1 = rate(lam0);
  T k2 = rate(lam0 + 0.5 * dt * k1);
  T k3 = rate(lam0 + 0.5 * dt * k2);
  T k4 = rate(lam0 + dt * k3);
  T lam1 = lam0 + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
  lam1 = tmin(tmax(lam1, T(0)), T(1));
  U[L.lam()] = my * lam1;
}

/* cylindrical geometric source s_g of Sec. 3 at radius r (x = r, y = z, the
   third direction theta): dq/dt = -(1/r) (0 for phi, m_l u_r, the history
   slot times u_r, rho u_r^2 - sig_rr + sig_tt, rho u_z u_r - sig_rz,
   rho E u_r - (u_r sig_rr + u_z sig_zr), (1/3 - delta_{i theta}) Vbar_ij u_r),
   with the mixture stress sig (tension positive) of the state */
template <class T> void geom_rate(const Ctx<T>& X, const T* U, const T& r, T* S) {
  const Lay& L = X.L;
  Cell<T> C;
  from_cons(X, U, C);
  T ur = C.u[0], uz = C.u[1];
  for (int f = 0; f < L.F; ++f) S[f] = T(0);
  for (int l = 0; l < L.N; ++l) S[L.m(l)] = -(U[L.m(l)] * ur) / r;
  if (L.xf) S[L.lam()] = -(U[L.lam()] * ur) / r;
  S[L.mom(0)] = -(U[L.mom(0)] * ur - C.sig[0][0] + C.sig[2][2]) / r;
  S[L.mom(1)] = -(U[L.mom(1)] * ur - C.sig[0][1]) / r;
  S[L.E()] = -(U[L.E()] * ur - (ur * C.sig[0][0] + uz * C.sig[1][0])) / r;
  for (int q = 0; q < L.nV; ++q) {
    double coef = (L.vi[q] == 2) ? (1.0 / 3.0 - 1.0) : 1.0 / 3.0;
    S[L.V(q)] = -(coef * U[L.V(q)] * ur) / r;
  }
}

/* the geometric fractional step over dt by Heun's method (the paper does not
   name the integrator): U + dt/2 (S(U) + S(U + dt S(U))) */
template <class T> void geom_cell(const Ctx<T>& X, T* U, const T& r, const T& dt) {
  const Lay& L = X.L;
  T S0[FMAX], S1[FMAX], U1[FMAX];
  geom_rate(X, U, r, S0);
  for (int f = 0; f < L.F; ++f) U1[f] = U[f] + dt * S0[f];
  geom_rate(X, U1, r, S1);
  for (int f = 0; f < L.F; ++f) U[f] = U[f] + (0.5 * dt) * (S0[f] + S1[f]);
}

template <class T> void gather(const or_config& c, const T* a, int64_t cell, T* U) {
  Lay L(c);
  int64_t nc = ncell(c);
  for (int f = 0; f < L.F; ++f) U[f] = a[f * nc + cell];
}
template <class T> void scatter(const or_config& c, T* a, int64_t cell, const T* U) {
  Lay L(c);
  int64_t nc = ncell(c);
  for (int f = 0; f < L.F; ++f) a[f * nc + cell] = U[f];
}

int check_config(const or_config* c) {
  if (!c) return -1;
  if (c->ndim < 1 || c->ndim > 3) return -1;
  if (c->nmat < 1 || c->nmat > OR_MAXMAT) return -1;
  for (int d = 0; d < c->ndim; ++d)
    if (c->n[d] < 1 || !(c->dx[d] > 0)) return -1;
  if (c->rx.mat >= c->nmat) return -1;
  for (int d = 0; d < c->ndim; ++d)
    if (c->bc[d] < OR_BC_TRANSMISSIVE || c->bc[d] > OR_BC_AXIS) return -1;
  if (c->geom != OR_GEOM_CARTESIAN && c->geom != OR_GEOM_CYLINDRICAL) return -1;
  if (c->geom == OR_GEOM_CYLINDRICAL && (c->ndim != 2 || !(c->lo[0] + 0.5 * c->dx[0] > 0))) return -1;
  if (c->thinc && c->nmat < 2) return -1;
  auto jwl_ok = [](const or_mat& m) {
    return m.eos != OR_EOS_JWL || (m.rho0 > 0 && m.Gamma0 > 0 && m.jwl_R1 > 0 && m.jwl_R2 > 0);
  };
  for (int l = 0; l < c->nmat; ++l)
    if (!jwl_ok(c->mat[l])) return -1;
  if (c->rx.mat >= 0) {
    const or_rx& r = c->rx;
    if (!jwl_ok(r.reactant) || !jwl_ok(r.product)) return -1;
    if (r.law != OR_RATE_POWER && r.law != OR_RATE_IG) return -1;
    if (r.law == OR_RATE_IG &&
        (!(r.ig_rho0 > 0) || !(r.ig_punit > 0) || !(r.ig_I >= 0) || !(r.ig_G1 >= 0) || !(r.ig_G2 >= 0) ||
         !(r.ig_b >= 0) || !(r.ig_c >= 0) || !(r.ig_d > 0) || !(r.ig_e >= 0) || !(r.ig_g > 0) ||
         !(r.ig_x >= 0) || !(r.ig_y >= 0) || !(r.ig_z >= 0)))
      return -1;
  }
  int njc = 0;
  for (int l = 0; l < c->nmat; ++l) {
    const or_mat& m = c->mat[l];
    if (m.plast != OR_PLAST_JC) continue;
    ++njc;
    if (m.eos != OR_EOS_ROMENSKII || !(m.G0 > 0) || !(m.cv > 0) || !(m.jc_c1 > 0) || !(m.jc_c2 >= 0) ||
        !(m.jc_c3 > 0) || !(m.jc_n > 0) || !(m.jc_m > 0) || !(m.jc_tmelt > m.jc_t0) || !(m.jc_chi0 > 0))
      return -1;
  }
  if (njc > 1 || (njc == 1 && c->rx.mat >= 0)) return -1;  // one history slot
  return 0;
}

}  // namespace

/* ================================================================ C API */
extern "C" {

int or_nfields(const or_config* c) {
  if (check_config(c)) return -1;
  return Lay(*c).F;
}

void or_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int or_get_threads(void) { return g_threads; }

int or_prim_to_cons(const or_config* c, const double* prim, double* cons) {
  if (check_config(c)) return -1;
  Ctx<double> X(*c);
  int64_t nc = ncell(*c);
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    double W[FMAX], U[FMAX];
    gather(*c, prim, i, W);
    Cell<double> C;
    from_prim(X, W, C);
    cell_to_cons(X, C, U);
    scatter(*c, cons, i, U);
  }
  return 0;
}

int or_cons_to_prim(const or_config* c, const double* cons, double* prim) {
  if (check_config(c)) return -1;
  Ctx<double> X(*c);
  int64_t nc = ncell(*c);
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    double W[FMAX], U[FMAX];
    gather(*c, cons, i, U);
    Cell<double> C;
    from_cons(X, U, C);
    cell_to_prim(X, C, W);
    scatter(*c, prim, i, W);
  }
  return 0;
}

int or_sweep(const or_config* c, double* cons, double dt, int dir) {
  if (check_config(c) || dir < 0 || dir >= c->ndim) return -1;
  int64_t nc = ncell(*c);
  int F = Lay(*c).F;
  std::vector<double> in(cons, cons + nc * F);
  sweep_grid<double>(*c, in.data(), cons, dt, dir);
  return 0;
}

int or_sweep_flux(const or_config* c, double* cons, double dt, int dir, double* flux) {
  if (check_config(c) || dir < 0 || dir >= c->ndim || !flux) return -1;
  int64_t nc = ncell(*c);
  int F = Lay(*c).F;
  std::vector<double> in(cons, cons + nc * F);
  sweep_grid<double>(*c, in.data(), cons, dt, dir, nullptr, nullptr, flux);
  return 0;
}

int or_plastic_dt(const or_config* c, double* cons, double dt) {
  if (check_config(c) || !(dt >= 0.0)) return -1;
  Ctx<double> X(*c);
  int64_t nc = ncell(*c);
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    double U[FMAX];
    gather(*c, cons, i, U);
    plastic_cell(X, U, dt);
    scatter(*c, cons, i, U);
  }
  return 0;
}

int or_plastic(const or_config* c, double* cons) { return or_plastic_dt(c, cons, 0.0); }

int or_geometric(const or_config* c, double* cons, double dt) {
  if (check_config(c)) return -1;
  if (c->geom != OR_GEOM_CYLINDRICAL) return 0;
  Ctx<double> X(*c);
  int64_t nc = ncell(*c);
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    double U[FMAX];
    gather(*c, cons, i, U);
    const double r = c->lo[0] + ((double)(i % c->n[0]) + 0.5) * c->dx[0];
    geom_cell(X, U, r, dt);
    scatter(*c, cons, i, U);
  }
  return 0;
}

int or_reaction(const or_config* c, double* cons, double dt) {
  if (check_config(c)) return -1;
  if (c->rx.mat < 0) return 0;
  Ctx<double> X(*c);
  int64_t nc = ncell(*c);
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    double U[FMAX];
    gather(*c, cons, i, U);
    reaction_cell(X, U, dt);
    scatter(*c, cons, i, U);
  }
  return 0;
}

/* one full step: the split sweeps (x..z on even steps, z..x on odd steps),
   then the plastic and reactive fractional steps (Sec. 3) */
int or_step(const or_config* c, double* cons, double dt, int64_t step) {
  if (check_config(c)) return -1;
  int D = c->ndim;
  for (int s = 0; s < D; ++s) {
    int d = (step % 2 == 0) ? s : D - 1 - s;
    int rc = or_sweep(c, cons, dt, d);
    if (rc) return rc;
  }
  or_plastic_dt(c, cons, dt);
  or_reaction(c, cons, dt);
  or_geometric(c, cons, dt);
  return 0;
}

int or_step_dual(const or_config* c, double* cons, double* tan, const double* par_tan, double dt,
                 int64_t step, int K) {
  return or_stage_dual(c, cons, tan, par_tan, dt, step, K, -1);
}

int or_stage_dual(const or_config* c, double* cons, double* tan, const double* par_tan, double dt,
                  int64_t step, int K, int stage) {
  using DT = Dual<OR_DUAL_K>;
  if (check_config(c) || c->geom || K < 0 || K > OR_DUAL_K || !cons || (K > 0 && (!tan || !par_tan))) return -1;
  const int64_t nc = ncell(*c);
  const int F = Lay(*c).F;
  const int D = c->ndim;
  const int64_t NF = nc * F;
  std::vector<DT> a(NF), b(NF);
  for (int64_t i = 0; i < NF; ++i) {
    a[i].v = cons[i];
    for (int k = 0; k < K; ++k) a[i].d[k] = tan[k * NF + i];
  }
  MatPar<DT> par[MAXM];
  for (int l = 0; l < c->nmat; ++l) {
    par[l] = mat_par<DT>(c->mat[l]);
    for (int k = 0; k < K; ++k) {
      const double* t = par_tan + (k * c->nmat + l) * 4;
      par[l].gamma.d[k] = t[0];
      par[l].pinf.d[k] = t[1];
      par[l].G0.d[k] = t[2];
      par[l].yield.d[k] = t[3];
    }
  }
  if (stage < -1 || stage > D) return -1;
  for (int s = 0; s < D; ++s) {
    int d = (step % 2 == 0) ? s : D - 1 - s;
    if (stage >= 0 && stage != d) continue;
    sweep_grid<DT>(*c, a.data(), b.data(), DT(dt), d, par);
    a.swap(b);
  }
  Ctx<DT> X(*c, par);
  if (stage < 0 || stage == D) {
#pragma omp parallel for num_threads(g_threads)
    for (int64_t i = 0; i < nc; ++i) {
      DT U[FMAX];
      gather(*c, a.data(), i, U);
      plastic_cell(X, U, DT(dt));
      if (c->rx.mat >= 0) reaction_cell(X, U, DT(dt));
      scatter(*c, a.data(), i, U);
    }
  }
  for (int64_t i = 0; i < NF; ++i) {
    cons[i] = a[i].v;
    for (int k = 0; k < K; ++k) tan[k * NF + i] = a[i].d[k];
  }
  return 0;
}

namespace {
void flop_reset() { std::memset(g_flop_slots, 0, sizeof g_flop_slots); }
void flop_take(double* row) {
  for (int k = 0; k < FC_N; ++k) {
    long long t = 0;
    for (const FlopSlot& sl : g_flop_slots) t += sl.c[k];
    row[k] = (double)t;
  }
}
}  // namespace

/* the spatial operator D(q) of eq. (spat_op): the directions' flux
   differences minus the non-conservative sources, summed x, y, z */
int or_rhs(const or_config* c, const double* cons, double* rhs) {
  if (check_config(c) || !cons || !rhs) return -1;
  const int64_t NF = ncell(*c) * Lay(*c).F;
  for (int64_t i = 0; i < NF; ++i) rhs[i] = 0.0;
  for (int d = 0; d < c->ndim; ++d) sweep_grid<double>(*c, cons, nullptr, 0.0, d, nullptr, rhs);
  return 0;
}

/* direction dir's part of D(cons) added into rhs, and that direction's face
   fluxes (the edges without the predictor, as or_rhs evaluates them) into
   flux (the grid's shape with n_dir + 1 faces along dir, component-major);
   calling it for every direction in order gives or_rhs bit for bit */
int or_rhs_dir_flux(const or_config* c, const double* cons, int dir, double* rhs, double* flux) {
  if (check_config(c) || !cons || !rhs || !flux || dir < 0 || dir >= c->ndim) return -1;
  sweep_grid<double>(*c, cons, nullptr, 0.0, dir, nullptr, rhs, flux);
  return 0;
}

/* one step with the paper's own hyperbolic integrator: the SSP-RK3 of
   eq. (rk) on the unsplit operator D, then the plastic and reactive
   fractional steps (Sec. 3) */
int or_step_rk3(const or_config* c, double* cons, double dt) {
  if (check_config(c) || !cons) return -1;
  const int64_t NF = ncell(*c) * Lay(*c).F;
  std::vector<double> qn(cons, cons + NF), q1(NF), q2(NF), q3(NF), q4(NF), D(NF);
  auto op = [&](const double* q) { or_rhs(c, q, D.data()); };
  op(qn.data());
  for (int64_t i = 0; i < NF; ++i) q1[i] = qn[i] - dt * D[i];
  op(q1.data());
  for (int64_t i = 0; i < NF; ++i) q2[i] = q1[i] - dt * D[i];
  for (int64_t i = 0; i < NF; ++i) q3[i] = 0.75 * qn[i] + 0.25 * q2[i];
  op(q3.data());
  for (int64_t i = 0; i < NF; ++i) q4[i] = q3[i] - dt * D[i];
  for (int64_t i = 0; i < NF; ++i) cons[i] = (1.0 / 3.0) * qn[i] + (2.0 / 3.0) * q4[i];
  or_plastic_dt(c, cons, dt);
  or_reaction(c, cons, dt);
  or_geometric(c, cons, dt);
  return 0;
}

int or_step_flops(const or_config* c, double* cons, double dt, int64_t step, double* counts) {
  if (check_config(c) || !cons || !counts || c->geom) return -1;
  const int64_t nc = ncell(*c);
  const int F = Lay(*c).F;
  const int D = c->ndim;
  const int64_t NF = nc * F;
  std::vector<Flop> a(NF), b(NF);
  for (int64_t i = 0; i < NF; ++i) a[i] = Flop::data(cons[i]);
  const Flop fdt = Flop::data(dt);
  for (int s = 0; s < D; ++s) {
    int d = (step % 2 == 0) ? s : D - 1 - s;
    flop_reset();
    sweep_grid<Flop>(*c, a.data(), b.data(), fdt, d);
    flop_take(counts + d * FC_N);
    a.swap(b);
  }
  Ctx<Flop> X(*c);
  flop_reset();
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    Flop U[FMAX];
    gather(*c, a.data(), i, U);
    plastic_cell(X, U, fdt);
    if (c->rx.mat >= 0) reaction_cell(X, U, fdt);
    scatter(*c, a.data(), i, U);
  }
  flop_take(counts + D * FC_N);
  /* the wave speed of the result, as or_max_wavespeed computes it (the
     maximum itself is a comparison per cell and direction) */
  flop_reset();
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    Flop U[FMAX];
    gather(*c, a.data(), i, U);
    Cell<Flop> C;
    from_cons(X, U, C);
    Flop cl = sqrt(C.cL2);
    for (int d = 0; d < D; ++d) {
      Flop sd = tabs(C.u[d]) + cl;
      (void)sd;
    }
  }
  flop_take(counts + (D + 1) * FC_N);
  for (int64_t i = 0; i < NF; ++i) cons[i] = a[i].v;
  return 0;
}

/* Operations of one SSP-RK3 step (or_step_rk3) on counting scalars: rows
   0..ndim-1 one evaluation of the direction's part of D(q) (on the step's
   initial state), row ndim the three stage combinations, row ndim + 1 the
   plastic and reactive steps, row ndim + 2 the wave speed of the result;
   cons is advanced as by or_step_rk3. */
int or_step_rk3_flops(const or_config* c, double* cons, double dt, double* counts) {
  if (check_config(c) || !cons || !counts || c->geom) return -1;
  const int64_t nc = ncell(*c);
  const int D = c->ndim;
  const int64_t NF = nc * Lay(*c).F;
  std::vector<Flop> qn(NF), q1(NF), q2(NF), q3(NF), q4(NF), R(NF);
  for (int64_t i = 0; i < NF; ++i) qn[i] = Flop::data(cons[i]);
  const Flop fdt = Flop::data(dt);
  std::vector<double> comb(FC_N, 0.0), row(FC_N);
  auto op = [&](const std::vector<Flop>& q, bool count) {
    for (int64_t i = 0; i < NF; ++i) R[i] = Flop(0.0);
    for (int d = 0; d < D; ++d) {
      flop_reset();
      sweep_grid<Flop>(*c, q.data(), nullptr, Flop(0.0), d, nullptr, R.data());
      if (count) flop_take(counts + d * FC_N);
    }
  };
  auto combine = [&](auto&& f) {
    flop_reset();
    for (int64_t i = 0; i < NF; ++i) f(i);
    flop_take(row.data());
    for (int k = 0; k < FC_N; ++k) comb[k] += row[k];
  };
  op(qn, true);
  combine([&](int64_t i) { q1[i] = qn[i] - fdt * R[i]; });
  op(q1, false);
  combine([&](int64_t i) { q2[i] = q1[i] - fdt * R[i]; q3[i] = 0.75 * qn[i] + 0.25 * q2[i]; });
  op(q3, false);
  combine([&](int64_t i) { q4[i] = q3[i] - fdt * R[i]; qn[i] = (1.0 / 3.0) * qn[i] + (2.0 / 3.0) * q4[i]; });
  for (int k = 0; k < FC_N; ++k) counts[D * FC_N + k] = comb[k];
  Ctx<Flop> X(*c);
  flop_reset();
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    Flop U[FMAX];
    gather(*c, qn.data(), i, U);
    plastic_cell(X, U, fdt);
    if (c->rx.mat >= 0) reaction_cell(X, U, fdt);
    scatter(*c, qn.data(), i, U);
  }
  flop_take(counts + (D + 1) * FC_N);
  flop_reset();
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    Flop U[FMAX];
    gather(*c, qn.data(), i, U);
    Cell<Flop> C;
    from_cons(X, U, C);
    Flop cl = sqrt(C.cL2);
    for (int d = 0; d < D; ++d) {
      Flop sd = tabs(C.u[d]) + cl;
      (void)sd;
    }
  }
  flop_take(counts + (D + 2) * FC_N);
  for (int64_t i = 0; i < NF; ++i) cons[i] = qn[i].v;
  return 0;
}

/* the counting rules of Flop on fixed expressions (for tests):
   out[0..5]   (a + b) * c / d - sqrt(e)           : add 2, mul 1, div 1, sqrt 1
   out[6..11]  0 * a + b, a - 0, 0 / a, -(0 - a)   : nothing
   out[12..17] exp(a) + tanh(b), a < b, max(a, b)  : add 1, trans 2, cmp 2 */
int or_flops_selftest(double* out) {
  const int saved = g_threads;
  g_threads = 1;
  Flop a = Flop::data(1.5), b = Flop::data(-2.0), cc = Flop::data(3.0), d = Flop::data(0.25),
       e = Flop::data(2.0), z(0.0);
  flop_reset();
  Flop r = (a + b) * cc / d - sqrt(e);
  flop_take(out);
  flop_reset();
  Flop r2 = z * a + b;
  Flop r3 = a - z;
  Flop r4 = z / a;
  Flop r5 = -(z - a);
  flop_take(out + 6);
  flop_reset();
  Flop r6 = exp(a) + tanh(b);
  bool lt = a < b;
  Flop r7 = tmax(a, b);
  flop_take(out + 12);
  g_threads = saved;
  (void)r; (void)r2; (void)r3; (void)r4; (void)r5; (void)r6; (void)lt; (void)r7;
  return 0;
}

int or_max_wavespeed(const or_config* c, const double* cons, double* smax) {
  if (check_config(c)) return -1;
  Ctx<double> X(*c);
  int64_t nc = ncell(*c);
  int D = c->ndim;
  std::vector<double> part((size_t)nc * 3, 0.0);
#pragma omp parallel for num_threads(g_threads)
  for (int64_t i = 0; i < nc; ++i) {
    double U[FMAX];
    gather(*c, cons, i, U);
    Cell<double> C;
    from_cons(X, U, C);
    double cl = std::sqrt(C.cL2);
    for (int d = 0; d < D; ++d) part[i * 3 + d] = std::fabs(C.u[d]) + cl;
  }
  for (int d = 0; d < 3; ++d) smax[d] = 0.0;
  for (int64_t i = 0; i < nc; ++i)
    for (int d = 0; d < D; ++d) {
      double v = part[i * 3 + d];
      if (v > smax[d] || v != v) smax[d] = v;
    }
  return 0;
}

int or_eos(const or_mat* m, double rho, double J2, double* out) {
  if (!m || !out) return -1;
  Eos<double> e = eos_eval(*m, rho, J2);
  out[0] = e.Gam; out[1] = e.pref; out[2] = e.eref; out[3] = e.dpref; out[4] = e.deref; out[5] = e.G;
  return 0;
}

int or_thinc(double qm, double q0, double qp, double beta, double eps, double delta, double* out) {
  double qL, qR, C;
  thinc_edges(qm, q0, qp, beta, eps, qL, qR, C);
  out[0] = qL; out[1] = qR; out[2] = C;
  out[3] = thinc_mixed(qm, q0, qp, C, delta) ? 1.0 : 0.0;
  return 0;
}

int or_youngs_beta(const or_config* c, const double* cons, int64_t cell, int dir, double* beta) {
  if (check_config(c)) return -1;
  Ctx<double> X(*c);
  int64_t p[3];
  pos_of(*c, cell, p);
  *beta = c->beta0 * youngs_nd(X, cons, ncell(*c), p, dir) + 0.01;
  return 0;
}

int or_bvd_thinc(const double cand[8], double v[8]) {
  return bvd_thinc(cand[0], cand[1], cand[2], cand[3], cand[4], cand[5], cand[6], cand[7], v) ? 1 : 0;
}

int or_phi_edges(const or_config* c, const double q[5], const double beta[3], double out[16]) {
  if (check_config(c)) return -1;
  Lay L(*c);
  double ml[3], mr[3], tl[3], tr[3];
  for (int k = 0; k < 3; ++k) {
    const double a = q[k + 1] - q[k], b = q[k + 2] - q[k + 1];
    double s;
    if (c->limiter == OR_LIM_VANALBADA) {
      const double e = 1e-6 * va_scale_of(L, *c, L.phi(0));
      s = vanalbada(a, b, e * e);
    } else {
      s = minmod(a, b);
    }
    phi_candidates(*c, q[k], q[k + 1], q[k + 2], s, beta[k], ml[k], mr[k], tl[k], tr[k]);
  }
  const bool th = bvd_thinc(mr[0], tr[0], ml[1], mr[1], tl[1], tr[1], ml[2], tl[2], out + 2);
  out[0] = th ? tl[1] : ml[1];
  out[1] = th ? tr[1] : mr[1];
  out[10] = th ? 1.0 : 0.0;
  out[11] = ml[1];
  out[12] = mr[1];
  out[13] = tl[1];
  out[14] = tr[1];
  out[15] = 0.0;
  return 0;
}

/* a conserved cell's state up to the reactive split, as from_cons has it
   before its root; returns rho e */
static double rx_cell_setup(const Ctx<double>& X, const double* U, Cell<double>& C) {
  const Lay& L = X.L;
  double sphi = 0.0;
  for (int l = 0; l < L.N - 1; ++l) {
    C.phi[l] = U[L.phi(l)];
    sphi += C.phi[l];
  }
  C.phi[L.N - 1] = 1.0 - sphi;
  double rho = 0.0;
  for (int l = 0; l < L.N; ++l) {
    C.rho[l] = U[L.m(l)] / C.phi[l];
    rho += U[L.m(l)];
  }
  for (int k = 0; k < 3; ++k) C.u[k] = (k < L.D) ? U[L.mom(k)] / rho : 0.0;
  C.lam = tmin(tmax(U[L.lam()] / U[L.m(X.y)], 0.0), 1.0);
  C.eps = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.V[i][j] = 0.0;
  for (int q = 0; q < L.nV; ++q) C.V[L.vi[q]][L.vj[q]] = U[L.V(q)];
  kin_and_strain(X, C);
  double uu = 0.0;
  for (int k = 0; k < L.D; ++k) uu += C.u[k] * C.u[k];
  return U[L.E()] - 0.5 * rho * uu;
}

int or_rx_split(const or_config* c, const double* U, double* t) {
  if (check_config(c) || c->rx.mat < 0) return -1;
  Ctx<double> X(*c);
  Cell<double> C;
  const double rhoe = rx_cell_setup(X, U, C);
  *t = rx_solve(X, C, Known::Energy, rhoe, 0.0);
  return 0;
}

int or_rx_residual(const or_config* c, const double* U, int n, const double* t, double* out) {
  if (check_config(c) || c->rx.mat < 0) return -1;
  Ctx<double> X(*c);
  Cell<double> C;
  const double rhoe = rx_cell_setup(X, U, C);
  const or_rx& r = c->rx;
  for (int i = 0; i < n; ++i) {
    const double p = pressure_from_split(X, C, rhoe, t[i]);
    const double Ta = temperature(C.ea, C.rho_a, p, r.reactant.cv);
    const double Tb = temperature(C.eb, C.rho_b, p, r.product.cv);
    out[4 * i + 0] = Tb - Ta;
    out[4 * i + 1] = p;
    out[4 * i + 2] = Ta;
    out[4 * i + 3] = Tb;
  }
  return 0;
}

int or_strain(const double* V, double* H, double* J2) {
  double Vm[3][3], Hm[3][3];
  for (int i = 0; i < 9; ++i) Vm[i / 3][i % 3] = V[i];
  strain(Vm, Hm, *J2);
  for (int i = 0; i < 9; ++i) H[i] = Hm[i / 3][i % 3];
  return 0;
}

int or_pade_exp(const double* H, double* V) {
  double Hm[3][3], Vm[3][3];
  for (int i = 0; i < 9; ++i) Hm[i / 3][i % 3] = H[i];
  pade_exp(Hm, Vm);
  for (int i = 0; i < 9; ++i) V[i] = Vm[i / 3][i % 3];
  return 0;
}

static void diag_out(const Cell<double>& C, const or_config& c, double* out) {
  out[0] = C.p; out[1] = C.c2; out[2] = C.cL2; out[3] = C.Gmix; out[4] = C.rho_mix;
  out[5] = C.s; out[6] = C.rho_a; out[7] = C.rho_b;
  out[8] = out[9] = 0.0;
  if (c.rx.mat >= 0) {
    out[8] = temperature(C.ea, C.rho_a, C.p, c.rx.reactant.cv);
    out[9] = temperature(C.eb, C.rho_b, C.p, c.rx.product.cv);
  }
  out[10] = C.xi; out[11] = C.J2;
}

int or_cell_diag(const or_config* c, const double* U, double* out) {
  if (check_config(c)) return -1;
  Ctx<double> X(*c);
  Cell<double> C;
  from_cons(X, U, C);
  diag_out(C, *c, out);
  return 0;
}

int or_cell_diag_prim(const or_config* c, const double* W, double* out, double* U) {
  if (check_config(c)) return -1;
  Ctx<double> X(*c);
  Cell<double> C;
  from_prim(X, W, C);
  diag_out(C, *c, out);
  if (U) cell_to_cons(X, C, U);
  return 0;
}

int or_face_flux(const or_config* c, int dir, const double* WL, const double* WR, double* flux, double* extra) {
  if (check_config(c) || dir < 0 || dir >= c->ndim) return -1;
  Ctx<double> X(*c);
  Cell<double> CL, CR;
  from_prim(X, WL, CL);
  from_prim(X, WR, CR);
  Face<double> fc;
  riemann(X, CL, CR, dir, fc);
  int F = X.L.F;
  for (int f = 0; f < F; ++f) flux[f] = fc.F[f];
  extra[0] = fc.ustar;
  for (int j = 0; j < 3; ++j) extra[1 + j] = fc.Vn[j];
  return 0;
}

}  // extern "C"
