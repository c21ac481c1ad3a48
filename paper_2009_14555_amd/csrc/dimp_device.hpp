// dimp_device.hpp -- device-side physics of the diffuse-interface step (gfx950).
//
// Pointwise pieces of the method of arXiv 2009.14555, written for registers:
//   Mie-Grueneisen closures and mixture rules ....... Sec. 2.2, 2.3
//   reactive mixture (equal p and T split) ........... Sec. 2.3.1, Appendix B
//   strain from the stretch tensor, Pade exp ........ Sec. 3.2
//   HLLC-type flux for the whole system ............. Sec. 3.1 (flux differences)
//   THINC edges, mixed-cell test, BVD ............... Appendix A
//   plastic relaxation, reaction RK4 ................ Sec. 3.2, 3.3
// Layout and arithmetic are specialised at compile time on the dimension D,
// the number of materials N and the presence of a reactive mixture RX, so
// structural zeros of the stretch tensor never reach the FP64 pipes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dimp {

// ------------------------------------------------------------ parameters
struct MatP {
  int eos, plast, shear, abar_one, bbar_three, pad;
  double Gam, invGam;   // Gruneisen coefficient and its inverse
  double pref0, eref0;  // constant reference curves of ideal / stiffened gases
  double inv_rho0, abar, bbar, K0a, ec_coef, dpc_coef, G0;
  double yield_s6;      // sigma_Y / sqrt(6)
  double cv;
  // Johnson-Cook (plast == 2): sigma_Y = (c1 + c2 eps^n)(1 - theta^m), rate
  // chi0 exp((s - 1)/c3), theta = (T - T0)/(Tmelt - T0) in [0, 1]
  double jc_c1, jc_c2, jc_inv_c3, jc_n, jc_m, jc_t0, jc_inv_dT, jc_chi0;
};

// The RX template argument of the layouts and kernels: 0 no history slot;
// 1 a history slot (a reactive mixture of gases, or a Johnson-Cook solid's
// plastic strain); 2 a reactive mixture with a JWL component (the general
// Appendix B split).
// The history slot of the RX layouts holds either the reactive mixture's
// phi_y rho_y lambda (kind RXK_MIX) or the plastic strain phi_y rho_y eps_p
// of a Johnson-Cook solid y (kind RXK_EPS); the slot is transported the same
// way, the closures and sources differ.
constexpr int RXK_MIX = 0, RXK_EPS = 1;
constexpr int LAW_POWER = 0, LAW_IG = 1;
struct RxP {
  int mat, n_is2;
  int kind, gen;  // gen: a component has density-dependent (JWL) reference curves
  int law, pad;   // LAW_POWER or LAW_IG
  int jwl[2];     // component c is JWL
  double Ga, invGa, pa, ea, cva;  // reactant: Gamma, 1/Gamma, constant p_ref, e_ref, C_V
  double Gb, invGb, pb, eb, cvb;  // product (e_ref already lowered by Q)
  double k, n, inv_pref;          // LAW_POWER: -k lam (max(p,0)/pref)^n
  // JWL terms of component c: A, B, R1 rho0, R2 rho0 and 1/(R1 rho0), 1/(R2 rho0)
  double jA[2], jB[2], jR1[2], jR2[2], jiR1[2], jiR2[2];
  // LAW_IG (three-term ignition and growth of F = 1 - lam): I, G1, G2, the
  // exponents b, c, d, e, g, x, y, z, threshold a, switches F_ig, F_G1,
  // F_G2, the reference density and the pressure unit
  double igI, igG1, igG2, ig_a, ig_b, ig_c, ig_d, ig_e, ig_g, ig_x, ig_y, ig_z;
  double igFig, igFG1, igFG2, ig_rho0, ig_punit;
};

// materials the kernels are built for: two or three (the layouts are generic
// in N; the launchers instantiate N = 2 everywhere and N = 3 on 1-D and 2-D
// grids)
constexpr int MAXMAT = 3;

struct Params {
  int64_t n[3];
  int64_t ncell;
  double dx[3];
  int bc[3];
  int limiter, thinc, any_shear, geom;  // geom 1: cylindrical (2-D, x = r, y = z)
  double r_lo;                           // cylindrical: radius of the grid's low x face
  double beta0, delta, eps;
  double va_e2[6];  // squared van Albada epsilon per field kind
  int nmat, pad_nmat;
  MatP mat[MAXMAT];
  RxP rx;
};

constexpr int EOS_IDEAL = 0, EOS_STIFFENED = 1, EOS_ROMENSKII = 2;
constexpr int PLAST_PERFECT = 1, PLAST_JC = 2;

// the RX layout's history slot is the reactive mixture's (closures of
// Appendix B apply to material y)
template <int RX>
__device__ __forceinline__ bool rx_mix(const Params& P) {
  return RX && P.rx.kind == RXK_MIX;
}
constexpr int BC_PERIODIC = 1, BC_REFLECTIVE = 2, BC_AXIS = 3;

// ---------------------------------------------------------------- layout
template <int D, int N, int RX>
struct Lay {
  static constexpr int NPHI = N - 1;
  static constexpr int M0 = N - 1;
  static constexpr int LAM = 2 * N - 1;
  static constexpr int MOM0 = 2 * N - 1 + (RX ? 1 : 0);
  static constexpr int E = MOM0 + D;
  static constexpr int V0 = E + 1;
  static constexpr int NV = (D == 1) ? 3 : (D == 2) ? 5 : 9;
  static constexpr int F = V0 + NV;
  __host__ __device__ static constexpr int vi(int q) {
    return D == 1 ? q : D == 2 ? (q < 2 ? 0 : q < 4 ? 1 : 2) : q / 3;
  }
  __host__ __device__ static constexpr int vj(int q) {
    return D == 1 ? q : D == 2 ? (q == 0 ? 0 : q == 1 ? 1 : q == 2 ? 0 : q == 3 ? 1 : 2) : q % 3;
  }
  // slot of Vbar(i,j) among the stored entries, -1 for a structural zero
  __host__ __device__ static constexpr int vq(int i, int j) {
    return D == 1 ? (i == j ? i : -1)
           : D == 2 ? ((i < 2 && j < 2) ? 2 * i + j : (i == 2 && j == 2) ? 4 : -1)
                    : 3 * i + j;
  }
  // field kind for the van Albada scale: 0 phi, 1 rho, 2 lambda, 3 u, 4 p, 5 Vbar
  __host__ __device__ static constexpr int kind(int f) {
    return f < NPHI ? 0 : f < 2 * N - 1 ? 1 : (RX && f == LAM) ? 2 : f < E ? 3 : f == E ? 4 : 5;
  }
};

// field f changes sign in the mirror image across a wall normal to axis d:
// the normal momentum and the stretch-tensor entries with exactly one
// normal index (V -> M V M, M the reflection)
template <int D, int N, int RX>
__host__ __device__ constexpr bool mirror_odd(int f, int d) {
  using L = Lay<D, N, RX>;
  return f == L::MOM0 + d ||
         (f >= L::V0 && f < L::F && ((L::vi(f - L::V0) == d) != (L::vj(f - L::V0) == d)));
}

// symmetric 3x3 with structural zeros: slots 00,01,02,11,12,22
template <int D>
__host__ __device__ constexpr bool hnz(int i, int j) {
  return D == 3 ? true : D == 2 ? ((i < 2 && j < 2) || (i == 2 && j == 2)) : (i == j);
}
__host__ __device__ constexpr int hs(int i, int j) {
  // not recursive: a recursive form is turned into a runtime loop in some
  // inlined contexts, and the arrays it indexes then go to scratch memory
  const int a = (i < j) ? i : j, b = (i < j) ? j : i;
  return a == 0 ? b : a == 1 ? 2 + b : 5;
}

// Neighbour exchange within a wave: lane i receives the value of lane i - 1
// (from_left) or i + 1 (from_right); lane 0 (from_left) and lane 63
// (from_right), which have no such neighbour, receive 0.  Those are halo
// lanes of every kernel that shifts this way (their results reach no lane
// that is written), and taking 0 lets the move write a fresh register
// instead of first copying the value it would otherwise keep.  Wave-wide DPP
// shifts are plain vector moves, with none of the latency of a permute
// through the LDS crossbar.
__device__ __forceinline__ double from_left(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ double from_right(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}
// the same shifts with lanes 0 and 63 keeping their own value
__device__ __forceinline__ double from_left_keep(double v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
}
__device__ __forceinline__ double from_right_keep(double v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}

// 1/b from the hardware reciprocal refined by two Newton steps: within an ulp
// or two of the correctly rounded quotient, at about half the instructions
// of an IEEE division
__device__ __forceinline__ double frcp(double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  return fma(r, e, r);
}

// a[y] for a runtime index y < M, read with compile-time indices and selects
// so that a register array is never placed in private memory (the empty asm
// keeps the optimiser from folding the selects back into one indexed load)
template <int M>
__device__ __forceinline__ double pick(const double* a, int y) {
  double r = a[0];
#pragma unroll
  for (int l = 1; l < M; ++l) {
    double v = a[l];
    asm volatile("" : "+v"(v));
    r = (l == y) ? v : r;
  }
  return r;
}

template <int D, int N, int RX>
__device__ __forceinline__ double vget(const double* V, int i, int j) {
  using L = Lay<D, N, RX>;
  return L::vq(i, j) >= 0 ? V[L::vq(i, j) >= 0 ? L::vq(i, j) : 0] : 0.0;
}

// ----------------------------------------------------------- closures
struct EosV {
  double Gam, invGam, pref, eref, dpref, deref, G;
};

// Sec. 2.3 closures at phasic density rho (1/rho given) and strain invariant J2
__device__ __forceinline__ EosV eos_eval(const MatP& m, double rho, double irho, double J2) {
  EosV e;
  e.Gam = m.Gam;
  e.invGam = m.invGam;
  if (m.eos != EOS_ROMENSKII) {
    e.pref = m.pref0;
    e.eref = m.eref0;
    e.dpref = 0.0;
    e.deref = 0.0;
    e.G = 0.0;
    return e;
  }
  const double x = rho * m.inv_rho0;
  const double xa = m.abar_one ? x : pow(x, m.abar);
  const double ec = m.ec_coef * (xa - 1.0) * (xa - 1.0);
  const double pc = m.K0a * x * xa * (xa - 1.0);
  const double dpc = m.dpc_coef * ((2.0 * m.abar + 1.0) * xa * xa - (m.abar + 1.0) * xa);
  double G;
  if (m.bbar_three) {
    const double x2 = x * x;
    G = m.G0 * (x2 * x2);
  } else {
    G = m.G0 * pow(x, m.bbar + 1.0);
  }
  const double GJ = G * J2;
  e.pref = pc + m.bbar * GJ;
  e.eref = ec + GJ * irho;
  e.dpref = dpc + m.bbar * (m.bbar + 1.0) * GJ * irho;
  e.deref = e.pref * irho * irho;
  e.G = G;
  return e;
}

// shear modulus only (no reference curves)
__device__ __forceinline__ double shear_modulus(const MatP& m, double rho) {
  if (!m.shear) return 0.0;
  const double x = rho * m.inv_rho0;
  if (m.bbar_three) {
    const double x2 = x * x;
    return m.G0 * (x2 * x2);
  }
  return m.G0 * pow(x, m.bbar + 1.0);
}

__device__ __forceinline__ double c2_mat(const EosV& e, double rho, double irho, double p) {
  return e.dpref - rho * e.Gam * e.deref + ((1.0 + e.Gam) * p - e.pref) * irho;
}

// Hencky strain dev H ~ dev((B - adj B)/4), B = V V^T (Sec. 3.2: Bazant
// approximation with the cofactor standing in for the inverse of the
// unimodular B), and J^2 = tr(H H^T).
template <int D, int N, int RX>
__device__ __forceinline__ void strain(const double* V, double H[6], double& J2) {
  double B[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      double s = 0.0;
      bool first = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (Lay<D, N, RX>::vq(i, k) >= 0 && Lay<D, N, RX>::vq(j, k) >= 0) {
          const double t = vget<D, N, RX>(V, i, k) * vget<D, N, RX>(V, j, k);
          s = first ? t : s + t;
          first = false;
        }
      }
      B[hs(i, j)] = s;
    }
  double A[6];
  if (D == 1) {
    A[0] = B[3] * B[5];
    A[3] = B[0] * B[5];
    A[5] = B[0] * B[3];
    A[1] = A[2] = A[4] = 0.0;
  } else if (D == 2) {
    A[0] = B[3] * B[5];
    A[1] = -B[1] * B[5];
    A[3] = B[0] * B[5];
    A[5] = B[0] * B[3] - B[1] * B[1];
    A[2] = A[4] = 0.0;
  } else {
    A[0] = B[3] * B[5] - B[4] * B[4];
    A[1] = B[2] * B[4] - B[1] * B[5];
    A[2] = B[1] * B[4] - B[2] * B[3];
    A[3] = B[0] * B[5] - B[2] * B[2];
    A[4] = B[2] * B[1] - B[0] * B[4];
    A[5] = B[0] * B[3] - B[1] * B[1];
  }
  double K[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) K[s] = 0.25 * (B[s] - A[s]);
  const double tr = (K[0] + K[3] + K[5]) * (1.0 / 3.0);
  H[0] = K[0] - tr;
  H[3] = K[3] - tr;
  H[5] = K[5] - tr;
  H[1] = K[1];
  H[2] = K[2];
  H[4] = K[4];
  double j2 = H[0] * H[0] + H[3] * H[3] + H[5] * H[5];
  if (D >= 2) j2 += 2.0 * (H[1] * H[1]);
  if (D == 3) j2 += 2.0 * (H[2] * H[2] + H[4] * H[4]);
  J2 = j2;
}

// ------------------------------------------------------ phase densities
// phi_l, rho_l and 1/rho_l of every material.  For two materials one
// division serves both densities and one both inverses.
template <int N>
struct Phases {
  double phi[N], rho[N], irho[N];
};

template <int N>
__device__ __forceinline__ void phases_from_partial(const double* phi_st, const double* m, Phases<N>& Q) {
  double sphi = 0.0;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) {
    Q.phi[l] = phi_st[l];
    sphi += Q.phi[l];
  }
  Q.phi[N - 1] = 1.0 - sphi;
  if (N == 2) {
    const double ip = frcp(Q.phi[0] * Q.phi[1]);
    const double im = frcp(m[0] * m[1]);
    Q.rho[0] = m[0] * (Q.phi[1] * ip);
    Q.rho[1] = m[1] * (Q.phi[0] * ip);
    Q.irho[0] = Q.phi[0] * (m[1] * im);
    Q.irho[1] = Q.phi[1] * (m[0] * im);
  } else {
#pragma unroll
    for (int l = 0; l < N; ++l) {
      Q.rho[l] = m[l] / Q.phi[l];
      Q.irho[l] = Q.phi[l] / m[l];
    }
  }
}

template <int N>
__device__ __forceinline__ void phases_from_prim(const double* phi_st, const double* rho, Phases<N>& Q) {
  double sphi = 0.0;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) {
    Q.phi[l] = phi_st[l];
    sphi += Q.phi[l];
  }
  Q.phi[N - 1] = 1.0 - sphi;
#pragma unroll
  for (int l = 0; l < N; ++l) Q.rho[l] = rho[l];
  if (N == 2) {
    const double ir = frcp(rho[0] * rho[1]);
    Q.irho[0] = rho[1] * ir;
    Q.irho[1] = rho[0] * ir;
  } else {
#pragma unroll
    for (int l = 0; l < N; ++l) Q.irho[l] = 1.0 / rho[l];
  }
}

// ------------------------------------------------------ mixture state
// reference curves of one reactive component at its own density: p_ref,
// e_ref and their density derivatives
struct RxRef {
  double p, e, dp, de;
};

template <int N, int RX>
struct Thermo {
  EosV e[N];
  double xi, ixi;  // sum phi_l / Gamma_l (reactive: effective) and its inverse
  double rho, irho;
  double p, rhoe;
  double Gmix, c2, cL2;
  double rho_a, rho_b;
  RxRef A, B;  // reactive components at rho_a, rho_b
};

// Reference curves of reactive component C (0 reactant, 1 product) at
// density 1/irho: the constant part (a gas's p_ref and e_ref, the product's
// e_ref lowered by Q) plus, for a JWL component (Sec. 2.3),
// A exp(-R1 rho0/rho) + B exp(-R2 rho0/rho) and its energy
// A/(R1 rho0) exp(-R1 rho0/rho) + B/(R2 rho0) exp(-R2 rho0/rho), whose
// density derivative is p_ref/rho^2.
template <int C>
__device__ __forceinline__ RxRef rx_ref(const RxP& r, double irho) {
  RxRef o;
  o.p = C ? r.pb : r.pa;
  o.e = C ? r.eb : r.ea;
  o.dp = 0.0;
  o.de = 0.0;
  if (r.jwl[C]) {
    const double xa = exp(-r.jR1[C] * irho), xb = exp(-r.jR2[C] * irho);
    const double pa = r.jA[C] * xa, pb = r.jB[C] * xb;
    const double i2 = irho * irho;
    o.p = (pa + pb) + o.p;
    o.e = (pa * r.jiR1[C] + pb * r.jiR2[C]) + o.e;
    o.dp = (r.jR1[C] * pa + r.jR2[C] * pb) * i2;
    o.de = (pa + pb) * i2;
  }
  return o;
}

__device__ __forceinline__ RxRef rx_const(double p, double e) {
  RxRef o;
  o.p = p;
  o.e = e;
  o.dp = 0.0;
  o.de = 0.0;
  return o;
}

// Both components at the mixture's own density (a pure cell: no split).  A
// component whose weight is exactly zero keeps its constant part only: its
// terms vanish either way.
__device__ __forceinline__ void rx_pure(const RxP& r, double lam, double ry, double& ra, double& rb, RxRef& A,
                                        RxRef& B) {
  ra = ry;
  rb = ry;
  const double iry = 1.0 / ry;
  A = (lam > 0.0) ? rx_ref<0>(r, iry) : rx_const(r.pa, r.ea);
  B = (lam < 1.0) ? rx_ref<1>(r, iry) : rx_const(r.pb, r.eb);
}

// Appendix B with density-dependent reference curves: a root in (0, 1) of
// g(t) = rho_y (T_b - T_a) in t = rho_a / (rho_a + rho_b), a monotone
// function of the reactant density the paper bisects on; with D = lam (1-t)
// + (1-lam) t the specific-volume rule gives rho_a = rho_y D / (1-t), rho_b
// = rho_y D / t and the volume shares s = lam (1-t) / D, 1 - s = (1-lam) t /
// D.  Away from physical states (explosive traces in another material,
// low-density JWL reactant) g can change sign several times; the root taken
// is the first sign change met going outward from equal densities (t = 1/2,
// the split of the pure limits) towards the side g's sign points to (g < 0:
// above), on a fixed probe sequence: the ladder t = 3/4, 7/8, ... or
// t = 1/4, 1/8, ..., each probe halving the distance left to the end, until
// g changes sign; then RX_SUBSTEPS equal steps across that first bracket
// from its inner end until g changes sign again.  Inside the sub-bracket so
// found Newton steps from the secant point finish, halving whenever a step
// leaves it or is not finite.  Where g keeps its sign at every ladder probe
// the ends are taken: t = 1 (the pure state) once the probes reach 1 in
// double precision, t = 2^-65 after 64 probes down.  KNOWN_P: the pressure p
// is given (primitive branch); otherwise p(t) comes from the pressure
// function with its non-reactive part (num0, den0).
constexpr int RX_SUBSTEPS = 8;

template <bool KNOWN_P>
__device__ __forceinline__ void rx_newton(const RxP& r, double lam, double py, double ry, double p, double num0,
                                          double den0, double& ra, double& rb, RxRef& A, RxRef& B) {
  const double ka = 1.0 / (lam * r.Ga * r.cva), kb = 1.0 / ((1.0 - lam) * r.Gb * r.cvb);
  const double l1 = 1.0 - lam;
  const double la = lam * ry, lb = l1 * ry;
  const double iry = 1.0 / ry;
  double g = 0.0, dg = 1.0;
  // 0 the probe ladder, 3 steps across the first bracket, 1 Newton steps in
  // the sub-bracket, 2 a final midpoint
  int mode = 0;
  auto eval = [&](double t) {
    const double t1 = 1.0 - t;
    const double D = lam * t1 + l1 * t;
    const double iD = 1.0 / D;
    ra = ry * D / t1;
    rb = ry * D / t;
    const double s = lam * t1 * iD, s1 = l1 * t * iD;
    A = rx_ref<0>(r, t1 * iD * iry);
    B = rx_ref<1>(r, t * iD * iry);
    double pp = p, den = 1.0;
    if (!KNOWN_P) {
      const double num = num0 + py * (s * A.p * r.invGa - la * A.e) + py * (s1 * B.p * r.invGb - lb * B.e);
      den = den0 + py * (s * r.invGa + s1 * r.invGb);
      pp = num / den;
    }
    g = kb * (pp - B.p) * s1 - ka * (pp - A.p) * s;
    if (mode == 1) {  // the slope, for Newton steps only: dg/dt = lam (1-lam) / D^2 df/ds
      const double is = 1.0 / s, is1 = 1.0 / s1;
      const double dA = -A.dp * ra * is, dB = B.dp * rb * is1;  // d p_ref / ds
      double dp = 0.0;
      if (!KNOWN_P) {
        const double dnum = py * ((A.p + s * dA) * r.invGa + la * A.de * ra * is +
                                  (s1 * dB - B.p) * r.invGb - lb * B.de * rb * is1);
        dp = (dnum - pp * py * (r.invGa - r.invGb)) / den;
      }
      const double df = ka * ((dp - dA) * s + (pp - A.p)) - kb * ((dp - dB) * s1 - (pp - B.p));
      dg = df * (lam * l1) * (iD * iD);
    }
  };
  // one evaluation site for the four modes
  double lo = 0.0, hi = 1.0, glo = 0.0, ghi = 0.0, t = 0.5;
  double base = 0.5, w = 0.0;  // the first bracket's inner end; its width / RX_SUBSTEPS (signed)
  int probes = 0, sub = 0;
  bool up = false;
  for (int it = 0; it < 160; ++it) {
    eval(t);
    if (mode == 2) break;
    const bool below = g < 0.0;
    if (below) {
      lo = t;
      glo = g;
    } else {
      hi = t;
      ghi = g;
    }
    bool newton = false;
    double tn = 0.0;
    if (mode == 0) {
      ++probes;
      if (probes == 1) up = below;
      if (probes > 1 && below != up) {  // the first bracket: cross it from its inner end
        mode = 3;
        w = (t - base) / RX_SUBSTEPS;
        sub = 1;
        tn = base + w;
      } else {
        base = t;
        tn = up ? 0.5 * (t + 1.0) : 0.5 * t;
        if (up && !(tn < 1.0)) {  // g < 0 at every probe below 1: the pure state
          rx_pure(r, lam, ry, ra, rb, A, B);
          return;
        }
        if (probes == 64) {  // g >= 0 at every probe down to 2^-64
          mode = 2;
          tn = 0.5 * t;
        }
      }
    } else if (mode == 3) {
      if (below != up || sub == RX_SUBSTEPS - 1) {
        newton = true;  // [lo, hi] is the sub-bracket
      } else {
        ++sub;
        tn = base + double(sub) * w;
      }
    } else {
      // the current state is kept once the Newton step is below the
      // resolution the split needs (or below half an ulp of t)
      const double step = g / dg;
      if (g == 0.0 || (isfinite(step) && !(fabs(step) > fmax(1e-14 * fmin(t, 1.0 - t), 0x1p-53 * t)))) break;
      tn = t - step;
      if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);  // NaN steps land here too
    }
    if (newton) {
      mode = 1;
      tn = lo - glo * (hi - lo) / (ghi - glo);
      if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    }
    t = tn;
  }
}

// The split's root rule for two gas components (Appendix B, with the reading
// stated at rx_newton).  Here the residual changes sign at the roots of a
// polynomial of degree <= 2 in the reactant's volume share s (s = lam at
// equal densities t = 1/2; t = lam (1 - s) / (lam (1 - s) + (1 - lam) s)
// decreases with s).  The probe sequence of rx_newton changes sign between
// two probes where an odd number of roots lies between them, so its outcome
// follows from the roots alone: the root nearest t = 1/2 on the side g(1/2)
// points to (t >= 1/2 when g(1/2) < 0, else t <= 1/2), unless the other root
// lies in the same ladder bracket [1 - 2^-(k-1), 1 - 2^-k] (resp. [2^-k,
// 2^-(k-1)]): then both cancel and the ladder runs to its end, t = 1 (the
// pure state; brackets exist for k <= 53) or t = 2^-65 (after the probe
// 2^-64).  Sets s (true) or the end value t_end (false).
__device__ __forceinline__ int rx_bracket(double u) {
  int e;
  frexp(u, &e);  // u in [2^(e-1), 2^e)
  return (1 - e) < 2 ? 2 : 1 - e;
}

__device__ __forceinline__ bool rx_pick(const double* sr, int nr, bool up, double lam, double& s,
                                        double& t_end) {
  // t >= 1/2 exactly where s <= lam, and nearer 1/2 in t is nearer lam in s
  double sa = -1.0, sb = -1.0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (i >= nr) break;
    const double si = sr[i];
    const bool side = up ? (si > 0.0 && si <= lam) : (si >= lam && si < 1.0);
    if (!side) continue;
    if (sa < 0.0 || fabs(si - lam) < fabs(sa - lam)) {
      sb = sa;
      sa = si;
    } else {
      sb = si;
    }
  }
  t_end = up ? 1.0 : 0x1p-65;
  if (sa < 0.0) return false;
  // the distance of the root's t from the end it points to: 1 - t (up) or t
  auto dist = [&](double x) {
    const double a = lam * (1.0 - x), b = (1.0 - lam) * x;
    return (up ? b : a) * frcp(a + b);
  };
  const int ka = rx_bracket(dist(sa));
  if (ka > (up ? 53 : 64)) return false;                         // beyond the last probe
  if (sb >= 0.0 && rx_bracket(dist(sb)) == ka) return false;     // a pair cancels
  s = sa;
  return true;
}

// component densities of the split t (pure outside (0, 1)): with D = lam
// (1 - t) + (1 - lam) t, rho_a = rho_y D / (1 - t), rho_b = rho_y D / t
__device__ __forceinline__ void rx_densities(double lam, double ry, double t, double& ra, double& rb) {
  if (!(t > 0.0 && t < 1.0)) {
    ra = ry;
    rb = ry;
    return;
  }
  const double D = lam * (1.0 - t) + (1.0 - lam) * t;
  ra = ry * D / (1.0 - t);
  rb = ry * D / t;
}

// the densities of a picked share s (lam rho_y / s, (1 - lam) rho_y / (1 - s))
// or of the end value
__device__ __forceinline__ void rx_from_pick(bool picked, double s, double t_end, double lam, double ry, double& ra,
                                             double& rb) {
  if (picked) {
    ra = lam * ry * frcp(s);
    rb = (1.0 - lam) * ry * frcp(1.0 - s);
  } else {
    rx_densities(lam, ry, t_end, ra, rb);
  }
}

// Reactive split from a known pressure (Appendix B, primitive branch).  For
// two gas components temperature equality is linear in t: h(t) = (alpha +
// beta) t - alpha, alpha = (p - p_a)/(Gamma_a C_V,a), beta = (p - p_b)/(Gamma_b
// C_V,b).
template <bool GEN>
__device__ __forceinline__ void rx_split_p(const RxP& r, double lam, double rho_y, double p, double& ra,
                                           double& rb, RxRef& A, RxRef& B) {
  if constexpr (GEN) {
    if (lam >= 1.0 - 1e-12 || lam <= 1e-12)
      rx_pure(r, lam, rho_y, ra, rb, A, B);
    else
      rx_newton<true>(r, lam, 0.0, rho_y, p, 0.0, 0.0, ra, rb, A, B);
    return;
  }
  A = rx_const(r.pa, r.ea);
  B = rx_const(r.pb, r.eb);
  if (lam >= 1.0 - 1e-12 || lam <= 1e-12) {
    ra = rho_y;
    rb = rho_y;
    return;
  }
  // in t the residual is linear, (alpha + beta) t - alpha with alpha = (p -
  // p_a)/(Gamma_a C_V,a), beta = (p - p_b)/(Gamma_b C_V,b): g(1/2) < 0 where
  // beta < alpha, and the root t = alpha/(alpha + beta) lies in (0, 1) on
  // that side exactly where alpha > 0 and beta > 0 (else the ladder runs to
  // its end); the root itself from the share s = kb/(ka + kb), ka = alpha/lam,
  // kb = beta/(1 - lam)
  const double alpha = (p - r.pa) * frcp(r.Ga * r.cva), beta = (p - r.pb) * frcp(r.Gb * r.cvb);
  const bool up = beta < alpha;
  const bool found = alpha > 0.0 && beta > 0.0 &&
                     (up ? beta >= 0x1p-53 * (alpha + beta) : alpha >= 0x1p-64 * (alpha + beta));
  if (found) {
    const double ka = alpha * frcp(lam), kb = beta * frcp(1.0 - lam);
    rx_from_pick(true, kb * frcp(ka + kb), 1.0, lam, rho_y, ra, rb);
  } else {
    rx_densities(lam, rho_y, up ? 1.0 : 0x1p-65, ra, rb);
  }
}

// Reactive split from the conserved energy (Appendix B, conservative
// branch).  With the pressure function linear-fractional in the reactant's
// volume share s, p(s) = (A0 + A1 s)/(B0 + B1 s), and constant reference
// curves, temperature equality is Q(s) = Q2 s^2 + Q1 s + Q0 = 0, with g < 0
// where Q > 0; its roots (stable formula, one Newton polish each) go to the
// rule.
__device__ __forceinline__ void rx_solve_gas(const RxP& r, double lam, double ry, double A0, double A1, double B0,
                                             double B1, double& ra, double& rb) {
  if (lam >= 1.0 - 1e-12 || lam <= 1e-12) {
    ra = ry;
    rb = ry;
    return;
  }
  const double ka = frcp(lam * r.Ga * r.cva);
  const double kb = frcp((1.0 - lam) * r.Gb * r.cvb);
  const double a0 = A0 - r.pa * B0, a1 = A1 - r.pa * B1;
  const double b0 = A0 - r.pb * B0, b1 = A1 - r.pb * B1;
  const double Q2 = ka * a1 + kb * b1;
  const double Q1 = ka * a0 - kb * (b1 - b0);
  const double Q0 = -kb * b0;
  double sr[2];
  int nr = 0;
  if (Q2 == 0.0) {
    if (Q1 != 0.0) sr[nr++] = -Q0 / Q1;
  } else {
    const double disc = Q1 * Q1 - 4.0 * Q2 * Q0;
    if (disc >= 0.0) {
      const double q = -0.5 * (Q1 + copysign(sqrt(disc), Q1));
      if (q != 0.0) {
        sr[nr++] = Q0 / q;
        sr[nr++] = q / Q2;
      } else {
        sr[nr++] = 0.0;
      }
    }
  }
  const bool up = (Q2 * lam + Q1) * lam + Q0 > 0.0;  // g(1/2) < 0
  double sp = 0.0, t_end = 1.0;
  const bool picked = rx_pick(sr, nr, up, lam, sp, t_end);
  if (picked) {
    const double qv = (Q2 * sp + Q1) * sp + Q0, dq = 2.0 * Q2 * sp + Q1;
    if (dq != 0.0) sp = sp - qv * frcp(dq);  // one Newton polish of the root taken
  }
  rx_from_pick(picked, sp, t_end, lam, ry, ra, rb);
}

// The reactive part of the pressure function (Appendix B, conservative
// branch) for a cell whose non-reactive part is (num0, den0): solves the
// split and leaves the full numerator and denominator (xi) of p.
template <bool GEN>
__device__ __forceinline__ void rx_cons(const RxP& r, double py, double ry, double lam, double num0, double den0,
                                        double& ra, double& rb, RxRef& A, RxRef& B, double& num, double& den) {
  if constexpr (GEN) {
    if (lam >= 1.0 - 1e-12 || lam <= 1e-12)
      rx_pure(r, lam, ry, ra, rb, A, B);
    else
      rx_newton<false>(r, lam, py, ry, 0.0, num0, den0, ra, rb, A, B);
  } else {
    A = rx_const(r.pa, r.ea);
    B = rx_const(r.pb, r.eb);
    const double A0 = num0 + py * (r.pb * r.invGb - ry * (lam * r.ea + (1.0 - lam) * r.eb));
    const double A1 = py * (r.pa * r.invGa - r.pb * r.invGb);
    const double B0 = den0 + py * r.invGb;
    const double B1 = py * (r.invGa - r.invGb);
    rx_solve_gas(r, lam, ry, A0, A1, B0, B1, ra, rb);
  }
  const double wa = py * ry * lam, wb = py * ry * (1.0 - lam);
  // the components' volume fractions in the cell, wa / ra and wb / rb
  const double va = wa * frcp(ra), vb = wb * frcp(rb);
  den = den0 + va * r.invGa + vb * r.invGb;
  num = num0 + (va * (A.p * r.invGa) - wa * A.e) + (vb * (B.p * r.invGb) - wb * B.e);
}

template <int N, int RX>
__device__ __forceinline__ void eos_all(const Params& P, const Phases<N>& Q, double J2, Thermo<N, RX>& T) {
#pragma unroll
  for (int l = 0; l < N; ++l) {
    if (rx_mix<RX>(P) && l == P.rx.mat) continue;
    T.e[l] = eos_eval(P.mat[l], Q.rho[l], Q.irho[l], J2);
  }
}

// pressure from the conserved energy (Appendix B pressure function; without
// the reactive terms when RX is false).  Leaves xi and 1/xi in T.
template <int N, int RX>
__device__ __forceinline__ void pressure_from_rhoe(const Params& P, const Phases<N>& Q, double lam,
                                                   Thermo<N, RX>& T) {
  double den = 0.0, num = T.rhoe;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    if (rx_mix<RX>(P) && l == P.rx.mat) continue;
    den += Q.phi[l] * T.e[l].invGam;
    num += Q.phi[l] * (T.e[l].pref * T.e[l].invGam - Q.rho[l] * T.e[l].eref);
  }
  if (rx_mix<RX>(P)) {
    const int y = P.rx.mat;
    const double num0 = num, den0 = den;
    rx_cons<RX == 2>(P.rx, pick<N>(Q.phi, y), pick<N>(Q.rho, y), lam, num0, den0, T.rho_a, T.rho_b, T.A, T.B, num, den);
  }
  T.xi = den;
  T.ixi = frcp(den);
  T.p = num * T.ixi;
}

// mixture modulus and sound speeds (Allaire form of the mixture rule; c_L^2 =
// c^2 + 4G/(3 rho)) once p, the split and (optionally) 1/xi are known
template <int N, int RX>
__device__ __forceinline__ void finish(const Params& P, const Phases<N>& Q, double lam, Thermo<N, RX>& T,
                                       bool have_xi, bool have_rho = false) {
  if (!have_rho) {
    double r = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) r += Q.phi[l] * Q.rho[l];
    T.rho = r;
    T.irho = frcp(r);
  }
  double xi = 0.0, gnum = 0.0, cnum = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    double cl2, gl;
    if (rx_mix<RX>(P) && l == P.rx.mat) {
      const RxP& q = P.rx;
      const double ry = Q.rho[l], ra = T.rho_a, rb = T.rho_b, p = T.p;
      const double ira = frcp(ra), irb = frcp(rb);
      gl = (lam * ry * ira) * q.invGa + ((1.0 - lam) * ry * irb) * q.invGb;
      const double dEdp = lam * q.invGa * ira + (1.0 - lam) * q.invGb * irb;
      // component energy derivatives at fixed pressure, the JWL curves'
      // own slopes included
      const double pa = (RX == 2) ? T.A.p : q.pa, pb = (RX == 2) ? T.B.p : q.pb;
      double dEa = -(p - pa) * q.invGa * (ira * ira);
      double dEb = -(p - pb) * q.invGb * (irb * irb);
      if constexpr (RX == 2) {
        dEa = dEa - T.A.dp * q.invGa * ira + T.A.de;
        dEb = dEb - T.B.dp * q.invGb * irb + T.B.de;
      }
      const double dEdr = (lam * dEa * ra + (1.0 - lam) * dEb * rb) * Q.irho[l];
      cl2 = (p * (Q.irho[l] * Q.irho[l]) - dEdr) * frcp(dEdp);
    } else {
      gl = T.e[l].invGam;
      cl2 = c2_mat(T.e[l], Q.rho[l], Q.irho[l], T.p);
      gnum += Q.phi[l] * T.e[l].G * gl;
    }
    xi += Q.phi[l] * gl;
    cnum += (Q.phi[l] * Q.rho[l] * T.irho) * cl2 * gl;
  }
  if (!have_xi) {
    T.xi = xi;
    T.ixi = frcp(xi);
  }
  T.Gmix = gnum * T.ixi;
  T.c2 = cnum * T.ixi;
  T.cL2 = T.c2 + (4.0 / 3.0) * T.Gmix * T.irho;
}

// conserved -> primitive of one cell; W receives the primitive vector.  FIN
// = false leaves out the mixture's sound speeds and shear modulus (T.c2,
// T.cL2, T.Gmix; the plastic step needs the closures and p only).
template <int D, int N, int RX, bool FIN = true>
__device__ __forceinline__ void cons_to_prim(const Params& P, const double* U, double* W, Thermo<N, RX>& T,
                                             double H[6], double& J2) {
  using L = Lay<D, N, RX>;
  Phases<N> Q;
  phases_from_partial<N>(U, U + L::M0, Q);
  double r = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) r += U[L::M0 + l];
  const double inv_r = frcp(r);
  T.rho = r;
  T.irho = inv_r;
  double lam = 0.0, hist = 0.0;
  if (RX) {
    const double my = pick<N>(U + L::M0, P.rx.mat);
    hist = U[L::LAM] * frcp(my);
    if (P.rx.kind == RXK_MIX)
      lam = fmin(fmax(hist, 0.0), 1.0);
    else
      hist = (my > 0.0) ? hist : 0.0;  // plastic strain
  }
  double uu = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    W[L::MOM0 + k] = U[L::MOM0 + k] * inv_r;
    uu += W[L::MOM0 + k] * W[L::MOM0 + k];
  }
  strain<D, N, RX>(U + L::V0, H, J2);
  eos_all<N, RX>(P, Q, J2, T);
  T.rhoe = U[L::E] - 0.5 * r * uu;
  pressure_from_rhoe<N, RX>(P, Q, lam, T);
  if (FIN) finish<N, RX>(P, Q, lam, T, true, true);
#pragma unroll
  for (int l = 0; l < N - 1; ++l) W[l] = Q.phi[l];
#pragma unroll
  for (int l = 0; l < N; ++l) W[L::M0 + l] = Q.rho[l];
  if (RX) W[L::LAM] = (P.rx.kind == RXK_MIX) ? lam : hist;
  W[L::E] = T.p;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) W[L::V0 + q] = U[L::V0 + q];
}

// primitive -> thermodynamic state (energy from p)
template <int D, int N, int RX>
__device__ __forceinline__ void prim_thermo(const Params& P, const double* W, Thermo<N, RX>& T, double H[6],
                                            double& J2, bool need_energy) {
  using L = Lay<D, N, RX>;
  Phases<N> Q;
  phases_from_prim<N>(W, W + L::M0, Q);
  double lam = 0.0;
  if (RX) lam = fmin(fmax(W[L::LAM], 0.0), 1.0);
  strain<D, N, RX>(W + L::V0, H, J2);
  eos_all<N, RX>(P, Q, J2, T);
  T.p = W[L::E];
  if (rx_mix<RX>(P)) rx_split_p<RX == 2>(P.rx, lam, pick<N>(Q.rho, P.rx.mat), T.p, T.rho_a, T.rho_b, T.A, T.B);
  if (need_energy) {
    double e = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      if (rx_mix<RX>(P) && l == P.rx.mat) continue;
      e += Q.phi[l] * ((T.p - T.e[l].pref) * T.e[l].invGam + Q.rho[l] * T.e[l].eref);
    }
    if (rx_mix<RX>(P)) {
      const RxP& r = P.rx;
      const int y = r.mat;
      const double py = pick<N>(Q.phi, y), ry = pick<N>(Q.rho, y);
      const double wa = py * ry * lam, wb = py * ry * (1.0 - lam);
      if constexpr (RX == 2)
        e += wa * ((T.p - T.A.p) * r.invGa / T.rho_a + T.A.e) + wb * ((T.p - T.B.p) * r.invGb / T.rho_b + T.B.e);
      else
        e += wa * ((T.p - r.pa) * r.invGa / T.rho_a + r.ea) + wb * ((T.p - r.pb) * r.invGb / T.rho_b + r.eb);
    }
    T.rhoe = e;
  }
  finish<N, RX>(P, Q, lam, T, false);
}

// Mixture shear modulus G = sum(phi_l G_l / Gamma_l) / xi and strain of a
// primitive state: all the stress needs besides p
template <int D, int N, int RX>
__device__ __forceinline__ double prim_shear(const Params& P, const double* W, double H[6]) {
  using L = Lay<D, N, RX>;
  double phi[N];
  double sphi = 0.0;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) {
    phi[l] = W[l];
    sphi += phi[l];
  }
  phi[N - 1] = 1.0 - sphi;
  double xi = 0.0, gnum = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    if (rx_mix<RX>(P) && l == P.rx.mat) {
      const RxP& q = P.rx;
      const double lam = fmin(fmax(W[L::LAM], 0.0), 1.0);
      const double ry = W[L::M0 + l];
      double ra, rb;
      RxRef A, B;
      rx_split_p<RX == 2>(q, lam, ry, W[L::E], ra, rb, A, B);
      xi += phi[l] * ((lam * ry / ra) * q.invGa + ((1.0 - lam) * ry / rb) * q.invGb);
    } else {
      const double gl = P.mat[l].invGam;
      xi += phi[l] * gl;
      gnum += phi[l] * shear_modulus(P.mat[l], W[L::M0 + l]) * gl;
    }
  }
  double J2;
  strain<D, N, RX>(W + L::V0, H, J2);
  return gnum * frcp(xi);
}

// ------------------------------------------------ reconstruction pieces
__device__ __forceinline__ double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (fabs(a) < fabs(b)) ? a : b;
}

__device__ __forceinline__ double vanalbada(double a, double b, double e2) {
  return (a * (b * b + e2) + b * (a * a + e2)) / (a * a + b * b + 2.0 * e2);
}

template <int D, int N, int RX>
__device__ __forceinline__ double slope(const Params& P, int f, double wm, double w0, double wp) {
  const double a = w0 - wm, b = wp - w0;
  if (P.limiter == 1) return vanalbada(a, b, P.va_e2[Lay<D, N, RX>::kind(f)]);
  return minmod(a, b);
}

// THINC edge values (Appendix A), evaluated in the increasing orientation and
// swapped back for a decreasing stencil
__device__ __forceinline__ void thinc_edges(double qm, double q0, double qp, double beta, double eps,
                                            double delta, double mL, double mR, double& tL, double& tR) {
  const double qmin = fmin(qm, qp);
  const double qmax = fmax(qm, qp) - qmin;
  const double C = (q0 - qmin + eps) / (qmax + eps);
  tL = mL;
  tR = mR;
  if (!((delta < C) && (C < 1.0 - delta) && ((qp - q0) * (q0 - qm) > 0.0))) return;
  const double Bv = exp(beta * (2.0 * C - 1.0));
  const double tb = tanh(beta);
  const double A = (Bv / cosh(beta) - 1.0) / tb;
  const double lo = qmin + 0.5 * qmax * (1.0 + A);
  const double hi = qmin + 0.5 * qmax * (1.0 + (tb + A) / (1.0 + A * tb));
  if (qp - qm < 0.0) {
    tL = hi;
    tR = lo;
  } else {
    tL = lo;
    tR = hi;
  }
}

// Youngs normal |n_d| from a 3x3 (2-D) stencil phi9[a][b] (a along x, b
// along y, offsets -1..1) or a 3x3x3 stencil phi27[a][b][c]; symmetric pairs
// are summed first.
__device__ __forceinline__ double youngs2(const double s[3][3], const double* dx, int d) {
  const double gx = ((s[2][0] - s[0][0]) + (s[2][2] - s[0][2])) + 2.0 * (s[2][1] - s[0][1]);
  const double gy = ((s[0][2] - s[0][0]) + (s[2][2] - s[2][0])) + 2.0 * (s[1][2] - s[1][0]);
  const double ax = gx / dx[0], ay = gy / dx[1];
  const double nn = sqrt(ax * ax + ay * ay);
  if (!(nn > 0.0)) return 1.0;
  return fabs(d == 0 ? ax : ay) / nn;
}

__device__ __forceinline__ double youngs3(const double s[3][3][3], const double* dx, int d) {
  double g[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    // difference along e at transverse offsets (t1, t2) over the other two axes
    auto df = [&](int t1, int t2) {
      int p[3], m[3];
      const int o1 = (e == 0) ? 1 : 0, o2 = (e == 2) ? 1 : 2;
      p[e] = 2;
      m[e] = 0;
      p[o1] = m[o1] = 1 + t1;
      p[o2] = m[o2] = 1 + t2;
      return s[p[0]][p[1]][p[2]] - s[m[0]][m[1]][m[2]];
    };
    const double corners = (df(-1, -1) + df(1, 1)) + (df(-1, 1) + df(1, -1));
    const double edges = (df(-1, 0) + df(1, 0)) + (df(0, -1) + df(0, 1));
    g[e] = ((corners + 2.0 * edges) + 4.0 * df(0, 0)) / dx[e];
  }
  const double nn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  if (!(nn > 0.0)) return 1.0;
  return fabs(g[d]) / nn;
}

// candidates of the volume fraction edges of one cell: MUSCL (mL, mR) and
// THINC-or-MUSCL (tL, tR)
struct Cand {
  double mL, mR, tL, tR;
};

// the candidates of every stored volume fraction (N - 1 of them), and the
// one of fraction l of either form (a single Cand is fraction 0)
template <int N>
struct CandSet {
  Cand c[N > 1 ? N - 1 : 1];
};
__device__ __forceinline__ const Cand& cand_at(const Cand& c, int) { return c; }
template <int N>
__device__ __forceinline__ const Cand& cand_at(const CandSet<N>& c, int l) {
  return c.c[l];
}

// ------------------------------------------------------- face exchange
template <int D, int N, int RX>
struct FaceV {
  double F[Lay<D, N, RX>::F];  // phi slots carry phi_K u*
  double ustar;
  double Vn[D];                // Vbar*_{n j} for the structurally non-zero j of row n
};

}  // namespace dimp
