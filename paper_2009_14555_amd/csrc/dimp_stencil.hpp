// dimp_stencil.hpp -- per-cell and per-face stages of one split sweep.
//
// One sweep in direction DIR (Sec. 3.1, dimensionally split): primitive
// reconstruction with a limiter, THINC/BVD volume-fraction edges (Appendix
// A), a primitive half-step predictor, the HLLC-type face flux and the
// conservative update with the non-conservative terms of phi and Vbar; the
// fractional source steps (Sec. 3.2, 3.3) and the wave speed are optional
// epilogues of the last sweep.  The kernels that move data call these stages;
// the stages themselves only touch registers.
#pragma once
#include "dimp_device.hpp"

namespace dimp {

// ------------------------------------------------------ THINC candidates
// MUSCL edges (mL, mR) of phi and the THINC-or-MUSCL pair (tL, tR).  The
// interface normal (a sqrt and two divisions) and the three transcendentals
// are only evaluated in mixed cells (Appendix A criterion); cosh and tanh of
// beta come from one exponential.
template <int D, int N, int RX, class Youngs>
__device__ __forceinline__ Cand phi_candidates(const Params& P, double qm, double q0, double qp, Youngs&& nd_of) {
  Cand c;
  const double s = slope<D, N, RX>(P, 0, qm, q0, qp);
  c.mL = q0 - 0.5 * s;
  c.mR = q0 + 0.5 * s;
  c.tL = c.mL;
  c.tR = c.mR;
  if (!P.thinc) return c;
  const double qmin = fmin(qm, qp);
  const double qmax = fmax(qm, qp) - qmin;
  // mixed-cell test delta < C < 1 - delta with C = (q0 - qmin + eps)/(qmax + eps),
  // multiplied through by the non-negative denominator
  const double num = q0 - qmin + P.eps, den = qmax + P.eps;
  if (!((P.delta * den < num) && (num < (1.0 - P.delta) * den) && ((qp - q0) * (q0 - qm) > 0.0))) return c;
  const double C = num / den;
  const double beta = P.beta0 * nd_of() + 0.01;
  const double eb = exp(beta);
  const double ieb = 1.0 / eb;
  const double ch = 0.5 * (eb + ieb);
  const double tb = (eb - ieb) / (eb + ieb);
  const double Bv = exp(beta * (2.0 * C - 1.0));
  const double A = (Bv / ch - 1.0) / tb;
  const double lo = qmin + 0.5 * qmax * (1.0 + A);
  const double hi = qmin + 0.5 * qmax * (1.0 + (tb + A) / (1.0 + A * tb));
  // evaluated in the increasing orientation, swapped back for a decreasing stencil
  const bool dec = (qp - qm) < 0.0;
  c.tL = dec ? hi : lo;
  c.tR = dec ? lo : hi;
  return c;
}

// total boundary variation of the candidate pair (Lp, Rp) of a cell against
// the neighbours' candidates (Appendix A)
__device__ __forceinline__ double tbv(const Cand& m, const Cand& p, double Lp, double Rp) {
  const double v1 = fabs(m.mR - Lp) + fabs(Rp - p.mL);
  const double v2 = fabs(m.tR - Lp) + fabs(Rp - p.tL);
  const double v3 = fabs(m.mR - Lp) + fabs(Rp - p.tL);
  const double v4 = fabs(m.tR - Lp) + fabs(Rp - p.mL);
  return fmin(fmin(v1, v2), fmin(v3, v4));
}

// stress column sigma_{k,DIR} = 2 G dev H - p delta of a primitive state
template <int D, int N, int RX, int DIR>
__device__ __forceinline__ void stress_col(const Params& P, const double* W, double sig[3]) {
  using L = Lay<D, N, RX>;
  if (!P.any_shear) {
#pragma unroll
    for (int k = 0; k < 3; ++k) sig[k] = (k == DIR) ? -W[L::E] : 0.0;
    return;
  }
  double H[6];
  const double G = prim_shear<D, N, RX>(P, W, H);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (hnz<D>(k, DIR))
      sig[k] = 2.0 * G * H[hs(k, DIR)] - ((k == DIR) ? W[L::E] : 0.0);
    else
      sig[k] = 0.0;
  }
}

// Edges of one cell (MUSCL, with the BVD choice for phi) advanced half a
// step by the primitive quasi-linear system frozen at the cell state:
//   phi: u_n dphi     rho_l: u_n drho_l + rho_l du_n     lambda: u_n dlambda
//   u_k: u_n du_k - dsigma_kn / rho     p: u_n dp + rho c^2 du_n
//   Vbar_ij: u_n dV_ij - V_nj du_i + V_ij du_n / 3
// (the last is DVbar/Dt = (grad u) Vbar - div(u) Vbar / 3 of Sec. 2.1).
// MUSCL edges of every primitive component, with the BVD choice for phi
// (C: a Cand, the candidates of the single fraction of two materials, or a
// CandSet<N>, one per stored fraction; of the neighbours' candidates only the
// right edges of cm and the left edges of cp are read)
template <int D, int N, int RX, class C>
__device__ __forceinline__ void edges_muscl(const Params& P, const double* Wm, const double* W0, const double* Wp,
                                            const C& cm, const C& c0, const C& cp, double* WL, double* WR) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const double s = slope<D, N, RX>(P, f, Wm[f], W0[f], Wp[f]);
    WL[f] = W0[f] - 0.5 * s;
    WR[f] = W0[f] + 0.5 * s;
  }
  if (P.thinc) {
#pragma unroll
    for (int l = 0; l < N - 1; ++l) {
      const Cand &a = cand_at(cm, l), &b = cand_at(c0, l), &e = cand_at(cp, l);
      const double tm = tbv(a, e, b.mL, b.mR);
      const double tt = tbv(a, e, b.tL, b.tR);
      const bool th = tt < tm;
      WL[l] = th ? b.tL : b.mL;
      WR[l] = th ? b.tR : b.mR;
    }
  }
}

template <int D, int N, int RX, int DIR, class C>
__device__ __forceinline__ void edges_predict(const Params& P, const double* Wm, const double* W0, const double* Wp,
                                              double irho0, double rc2, const C& cm, const C& c0, const C& cp,
                                              double nu, double* WL, double* WR) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  edges_muscl<D, N, RX>(P, Wm, W0, Wp, cm, c0, cp, WL, WR);
  double sL[3], sR[3];
  stress_col<D, N, RX, DIR>(P, WL, sL);
  stress_col<D, N, RX, DIR>(P, WR, sR);
  double dW[F];
#pragma unroll
  for (int f = 0; f < F; ++f) dW[f] = WR[f] - WL[f];
  const double un = W0[L::MOM0 + DIR];
  const double dun = dW[L::MOM0 + DIR];
  double inc[F];
#pragma unroll
  for (int l = 0; l < N - 1; ++l) inc[l] = un * dW[l];
#pragma unroll
  for (int l = 0; l < N; ++l) inc[L::M0 + l] = un * dW[L::M0 + l] + W0[L::M0 + l] * dun;
  if (RX) inc[L::LAM] = un * dW[L::LAM];
#pragma unroll
  for (int k = 0; k < D; ++k) inc[L::MOM0 + k] = un * dW[L::MOM0 + k] - (sR[k] - sL[k]) * irho0;
  inc[L::E] = un * dW[L::E] + rc2 * dun;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int a = L::vi(q), b = L::vj(q);
    double v = un * dW[L::V0 + q];
    if (a < D && L::vq(DIR, b) >= 0) v -= vget<D, N, RX>(W0 + L::V0, DIR, b) * dW[L::MOM0 + (a < D ? a : 0)];
    v += (1.0 / 3.0) * W0[L::V0 + q] * dun;
    inc[L::V0 + q] = v;
  }
  const double h = 0.5 * nu;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    WL[f] -= h * inc[f];
    WR[f] -= h * inc[f];
  }
#pragma unroll
  for (int l = 0; l < N - 1; ++l) {
    WL[l] = fmin(fmax(WL[l], 0.0), 1.0);
    WR[l] = fmin(fmax(WR[l], 0.0), 1.0);
  }
  if (rx_mix<RX>(P)) {
    WL[L::LAM] = fmin(fmax(WL[L::LAM], 0.0), 1.0);
    WR[L::LAM] = fmin(fmax(WR[L::LAM], 0.0), 1.0);
  }
}

// ----------------------------------------------------------- face flux
template <int D, int N, int RX>
struct Side {
  double rho, E, cl;
  double u[D];
  double sig[3];  // sigma_{k n}
};

template <int D, int N, int RX, int DIR>
__device__ __forceinline__ void side_state(const Params& P, const double* W, Side<D, N, RX>& S) {
  using L = Lay<D, N, RX>;
  Thermo<N, RX> T;
  double H[6], J2;
  prim_thermo<D, N, RX>(P, W, T, H, J2, true);
  S.rho = T.rho;
  double uu = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    S.u[k] = W[L::MOM0 + k];
    uu += S.u[k] * S.u[k];
  }
  S.E = T.rhoe + 0.5 * T.rho * uu;
  S.cl = sqrt(T.cL2);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (hnz<D>(k, DIR))
      S.sig[k] = 2.0 * T.Gmix * H[hs(k, DIR)] - ((k == DIR) ? T.p : 0.0);
    else
      S.sig[k] = 0.0;
  }
}

template <int D, int N, int RX>
__device__ __forceinline__ double m_lambda(const Params& P, const double* W) {
  using L = Lay<D, N, RX>;
  const int y = P.rx.mat;
  double phi_y;
  if (y < N - 1) {
    phi_y = pick<(N > 1 ? N - 1 : 1)>(W, y);
  } else {
    phi_y = 1.0;
#pragma unroll
    for (int l = 0; l < N - 1; ++l) phi_y -= W[l];
  }
  double ry = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l)
    if (l == y) ry = W[L::M0 + l];
  return phi_y * ry * W[L::LAM];
}

// Flux of side K: the physical flux F_K plus S_K (U*_K - U_K), the HLLC-type
// star state with velocity (S*, u*_t) and traction continuous across the
// contact and Rankine-Hugoniot across S_K.  A supersonic face passes SK = 0
// with a = inv = 1, which returns F_K exactly.
template <int D, int N, int RX, int DIR>
__device__ __forceinline__ void star_flux(const Params& P, const double* W, const Side<D, N, RX>& S, double SK,
                                          double a, double inv, const double ust[D], double mK,
                                          FaceV<D, N, RX>& out) {
  using L = Lay<D, N, RX>;
  const double un = S.u[DIR];
  const double r = a * inv;
  const double rm1 = r - 1.0;
  const double us_face = un + SK * rm1;
  double phiN = 1.0;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) {
    phiN -= W[l];
    out.F[l] = W[l] * us_face;  // phi_K u*, the same u* as in the phi source
  }
#pragma unroll
  for (int l = 0; l < N; ++l) {
    const double m = (l < N - 1 ? W[l] : phiN) * W[L::M0 + l];
    out.F[L::M0 + l] = m * un + SK * (rm1 * m);
  }
  if (RX) {
    const double ml = m_lambda<D, N, RX>(P, W);
    out.F[L::LAM] = ml * un + SK * (rm1 * ml);
  }
  const double rs = r * S.rho;
  double usK = 0.0, usS = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double mom = S.rho * S.u[k];
    out.F[L::MOM0 + k] = mom * un - S.sig[k] + SK * (rs * ust[k] - mom);
    const double sst = S.sig[k] - mK * (ust[k] - S.u[k]);
    usK += S.u[k] * S.sig[k];
    usS += ust[k] * sst;
  }
  const double Es = (S.E * a + (usK - usS)) * inv;
  out.F[L::E] = S.E * un - usK + SK * (Es - S.E);
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    const double V = W[L::V0 + q];
    const bool coupled = (i < D) && (L::vq(DIR, j) >= 0);
    const double Vn = coupled ? vget<D, N, RX>(W + L::V0, DIR, j) : 0.0;
    const int ii = i < D ? i : 0;
    double Fx = V * un;
    if (coupled) Fx -= Vn * S.u[ii];
    if (i == DIR) {
      out.F[L::V0 + q] = Fx;  // normal row continuous: U* = U
    } else {
      double Vs = a * V;
      if (coupled) Vs -= Vn * (ust[ii] - S.u[ii]);
      out.F[L::V0 + q] = Fx + SK * (Vs * inv - V);
    }
  }
  out.ustar = us_face;
#pragma unroll
  for (int j = 0; j < D; ++j) out.Vn[j] = vget<D, N, RX>(W + L::V0, DIR, j);
}

template <int D, int N, int RX, int DIR>
__device__ __forceinline__ void face_flux(const Params& P, const double* WL, const double* WR,
                                          FaceV<D, N, RX>& out, bool wall = false) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  Side<D, N, RX> A, B;
  side_state<D, N, RX, DIR>(P, WL, A);
  side_state<D, N, RX, DIR>(P, WR, B);
  const double uL = A.u[DIR], uR = B.u[DIR];
  const double SL = fmin(uL - A.cl, uR - B.cl);
  const double SR = fmax(uL + A.cl, uR + B.cl);
  const double mL = A.rho * (SL - uL);
  const double mR = B.rho * (SR - uR);
  const double iden = frcp(mL - mR);
  double ust[D];
#pragma unroll
  for (int k = 0; k < D; ++k) ust[k] = ((A.sig[k] - B.sig[k]) + (mL * A.u[k] - mR * B.u[k])) * iden;
  // a reflective wall between a cell and its mirror image has S* = 0 exactly
  // (computed so in exact arithmetic; the GPU's round-off is not mirror-exact)
  if (wall) ust[DIR] = 0.0;
  const double Sst = ust[DIR];
  const bool supL = SL >= 0.0, supR = SR <= 0.0;
  const bool sup = supL || supR;
  const bool left = supL || (!supR && Sst > 0.0);
  const bool tie = !sup && (Sst == 0.0);
  // select side K (one star evaluation per face)
  double WK[F];
#pragma unroll
  for (int f = 0; f < F; ++f) WK[f] = left ? WL[f] : WR[f];
  Side<D, N, RX> SK;
  SK.rho = left ? A.rho : B.rho;
  SK.E = left ? A.E : B.E;
  SK.cl = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) SK.u[k] = left ? A.u[k] : B.u[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) SK.sig[k] = left ? A.sig[k] : B.sig[k];
  const double S_K = left ? SL : SR;
  const double m_K = left ? mL : mR;
  const double a = sup ? 1.0 : S_K - SK.u[DIR];
  const double inv = sup ? 1.0 : frcp(S_K - Sst);
  star_flux<D, N, RX, DIR>(P, WK, SK, sup ? 0.0 : S_K, a, inv, ust, m_K, out);
  if (tie) {
    // S* exactly zero: the average of both star fluxes.  A tie is never
    // 'left', so out already holds the right one; only the left one is
    // added.  (Every face between cells of a fluid at rest is a tie.)
    FaceV<D, N, RX> o1;
    const double a1 = SL - A.u[DIR];
    star_flux<D, N, RX, DIR>(P, WL, A, SL, a1, frcp(SL), ust, mL, o1);
#pragma unroll
    for (int f = 0; f < F; ++f) out.F[f] = 0.5 * (o1.F[f] + out.F[f]);
    out.ustar = 0.5 * (o1.ustar + out.ustar);
#pragma unroll
    for (int j = 0; j < D; ++j) out.Vn[j] = 0.5 * (o1.Vn[j] + out.Vn[j]);
  }
}

// ---------------------------------------------------------------- update
// U^{new} = U - nu (F_b - F_a) with phi's source phi div u and Vbar's sources
// (2/3) Vbar div u - u_i beta_j taken with the face velocities u* and the
// upwinded normal rows Vbar*_{n j} (cell-centre coefficients).
template <int D, int N, int RX, int DIR>
__device__ __forceinline__ void update_cell(const double* U, double inv_rho, const FaceV<D, N, RX>& a,
                                            const FaceV<D, N, RX>& b, double nu, double* Un) {
  using L = Lay<D, N, RX>;
  const double du = b.ustar - a.ustar;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) Un[l] = U[l] - nu * ((b.F[l] - a.F[l]) - U[l] * du);
#pragma unroll
  for (int f = N - 1; f < L::V0; ++f) Un[f] = U[f] - nu * (b.F[f] - a.F[f]);
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    double src = (2.0 / 3.0) * U[L::V0 + q] * du;
    if (i < D && j < D) src -= (U[L::MOM0 + (i < D ? i : 0)] * inv_rho) * (b.Vn[j < D ? j : 0] - a.Vn[j < D ? j : 0]);
    Un[L::V0 + q] = U[L::V0 + q] - nu * ((b.F[L::V0 + q] - a.F[L::V0 + q]) - src);
  }
}

// The direction's part of the unsplit operator D(q) of Sec. 3.1: the flux
// difference minus the same non-conservative sources as update_cell, times
// idx = 1/dx.
template <int D, int N, int RX, int DIR>
__device__ __forceinline__ void div_cell(const double* U, double inv_rho, const FaceV<D, N, RX>& a,
                                         const FaceV<D, N, RX>& b, double idx, double* Dd) {
  using L = Lay<D, N, RX>;
  const double du = b.ustar - a.ustar;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) Dd[l] = ((b.F[l] - a.F[l]) - U[l] * du) * idx;
#pragma unroll
  for (int f = N - 1; f < L::V0; ++f) Dd[f] = (b.F[f] - a.F[f]) * idx;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    double src = (2.0 / 3.0) * U[L::V0 + q] * du;
    if (i < D && j < D) src -= (U[L::MOM0 + (i < D ? i : 0)] * inv_rho) * (b.Vn[j < D ? j : 0] - a.Vn[j < D ? j : 0]);
    Dd[L::V0 + q] = ((b.F[L::V0 + q] - a.F[L::V0 + q]) - src) * idx;
  }
}

// --------------------------------------------------------------- sources
// Plastic relaxation (Sec. 3.2): per-material targets of the strain
// invariant (fluid 0, elastic J, ideal plasticity min(J, sigma_Y/(sqrt6 G))),
// mixed with phi/Gamma weights; dev H rescaled; Vbar rebuilt by the first
// Pade approximant with an exact inverse.
// Johnson-Cook target (rate law of Sec. 2.3.2, relaxation of Sec. 3.2): the
// root J* in [0, J] of R(x) = x - J + dt chi(x), chi = chi0 exp(a(x)), a =
// (sqrt6 G x / sigma_Y - 1)/c3, sigma_Y = (c1 + c2 eps^n)(1 - theta^m) with
// the plastic strain eps + (J - x) and the temperature rise (p - p_ref)/(rho
// Gamma cv) of the unrelaxed state.  The paper bisects; here safeguarded
// Newton steps find the same root to rounding in a few evaluations: on R
// from x = J when the relaxation is small (R is increasing and convex there),
// otherwise on the equivalent log(J - x) - log(dt chi0) - a(x) = 0 (nearly
// linear where chi is steep) from the rate-independent estimate a = 0; every
// step stays inside the bracket kept from the signs (bisection otherwise).
struct JcCtx {
  double G6, soft, J, eps;
  __device__ __forceinline__ void at(const MatP& m, double x, double& a, double& da) const {
    const double ep = fmax(eps + (J - x), 0.0);
    const double h = (m.jc_n == 1.0) ? ep : pow(ep, m.jc_n);
    const double isy = frcp((m.jc_c1 + m.jc_c2 * h) * soft);
    // d sigma_Y / dx = -c2 n eps^(n-1) soft (eps decreases as x grows)
    const double dh = (ep > 0.0) ? ((m.jc_n == 1.0) ? 1.0 : m.jc_n * h / ep) : 0.0;
    a = (G6 * x * isy - 1.0) * m.jc_inv_c3;
    da = G6 * isy * (1.0 + x * m.jc_c2 * dh * soft * isy) * m.jc_inv_c3;
  }
};

__device__ __forceinline__ double jc_target(const MatP& m, const EosV& e, double p, double rho, double J,
                                            double eps, double dt) {
  if (!(dt > 0.0) || !(J > 0.0)) return J;
  const double theta = fmin(fmax((p - e.pref) / (rho * e.Gam * m.cv) * m.jc_inv_dT, 0.0), 1.0);
  const double soft = 1.0 - pow(theta, m.jc_m);
  if (!(soft > 0.0)) return 0.0;  // at or above melt: no strength
  const JcCtx c{sqrt(6.0) * e.G, soft, J, eps};
  const double tol = 1e-15 * J;
  double lo = 0.0, hi = J, a, da;
  c.at(m, J, a, da);
  if (a < 700.0 && dt * m.jc_chi0 * exp(a) <= 0.1 * J) {
    double x = J;
    for (int it = 0; it < 60; ++it) {
      c.at(m, x, a, da);
      const double chi = m.jc_chi0 * exp(a);
      const double R = x - J + dt * chi;
      if (R > 0.0)
        hi = x;
      else
        lo = x;
      double xn = x - R / (1.0 + dt * chi * da);
      if (fabs(xn - x) <= tol) return xn;
      if (!(xn >= lo && xn <= hi)) xn = 0.5 * (lo + hi);
      x = xn;
    }
    return x;
  }
  const double L0 = log(dt * m.jc_chi0);
  double x = (m.jc_c1 + m.jc_c2 * (eps + J)) * soft / (c.G6 + m.jc_c2 * soft);  // a = 0 for n = 1
  if (!(x > 0.0 && x < J)) x = 0.5 * J;
  for (int it = 0; it < 60; ++it) {
    c.at(m, x, a, da);
    const double phi = log(J - x) - L0 - a;
    if (phi > 0.0)
      lo = x;
    else
      hi = x;
    double xn = x - phi / (-frcp(J - x) - da);
    if (fabs(xn - x) <= tol) return xn;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    x = xn;
  }
  return x;
}

template <int D, int N, int RX>
__device__ __forceinline__ void plastic_cell(const Params& P, double* U, double dt) {
  using L = Lay<D, N, RX>;
  double W[L::F];
  Thermo<N, RX> T;
  double H[6], J2;
  cons_to_prim<D, N, RX, false>(P, U, W, T, H, J2);
  const double J = sqrt(J2);
  double num = 0.0;
  double phiN = 1.0;
  double J_ep = J;  // target of the Johnson-Cook material (plastic strain update)
#pragma unroll
  for (int l = 0; l < N - 1; ++l) phiN -= W[l];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    if (rx_mix<RX>(P) && l == P.rx.mat) continue;
    const MatP& m = P.mat[l];
    if (!m.shear) continue;
    double Jl = J;
    if (m.plast == PLAST_PERFECT) {
      Jl = fmin(J, m.yield_s6 * frcp(T.e[l].G));
    } else if (RX && m.plast == PLAST_JC) {
      Jl = jc_target(m, T.e[l], T.p, W[L::M0 + l], J, W[L::LAM], dt);
      J_ep = Jl;
    }
    const double phi_l = (l < N - 1) ? W[l] : phiN;
    num += phi_l * T.e[l].invGam * Jl;
  }
  const double fac = (J > 0.0) ? (num * T.ixi) * frcp(J) : 0.0;
  double Hs[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) Hs[s] = (J > 0.0) ? fac * H[s] : 0.0;
  double Mm[6], Mp[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const double id = (s == 0 || s == 3 || s == 5) ? 1.0 : 0.0;
    Mm[s] = id - 0.5 * Hs[s];
    Mp[s] = id + 0.5 * Hs[s];
  }
  double A[6];  // adjugate of M- (symmetric)
  A[0] = Mm[3] * Mm[5] - Mm[4] * Mm[4];
  A[1] = Mm[2] * Mm[4] - Mm[1] * Mm[5];
  A[2] = Mm[1] * Mm[4] - Mm[2] * Mm[3];
  A[3] = Mm[0] * Mm[5] - Mm[2] * Mm[2];
  A[4] = Mm[2] * Mm[1] - Mm[0] * Mm[4];
  A[5] = Mm[0] * Mm[3] - Mm[1] * Mm[1];
  const double det = Mm[0] * A[0] + Mm[1] * A[1] + Mm[2] * A[2];
  const double inv_det = frcp(det);
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (hnz<D>(i, k) && hnz<D>(k, j)) v += A[hs(i, k)] * Mp[hs(k, j)];
    U[L::V0 + q] = v * inv_det;
  }
  if (RX && P.rx.kind == RXK_EPS) {
    // the plastic strain gained equals the strain invariant relaxed
    const double my = pick<N>(U + L::M0, P.rx.mat);
    if (my > 0.0) U[L::LAM] = my * (W[L::LAM] + (J - J_ep));
  }
}

// pressure of a cell whose reactive progress is lam, with the non-reactive
// part of the pressure function (num0, den0) already summed; rho_y is left
// for the rate
template <bool GEN>
__device__ __forceinline__ double rx_pressure(const RxP& r, double phi_y, double rho_y, double lam, double num0,
                                              double den0) {
  double ra, rb, num, den;
  RxRef A, B;
  rx_cons<GEN>(r, phi_y, rho_y, lam, num0, den0, ra, rb, A, B, num, den);
  return num * frcp(den);
}

// Three-term ignition-and-growth rate of the reacted fraction F = 1 - lam
// (Sec. 4.2, Table 4) at the mixture's own density rho and pressure p: each
// term carries a positive power of lam, the growth terms one of F; the
// compression and the pressure are clipped at zero, H(x) = 1 for x > 0 only.
__device__ __forceinline__ double ig_rate(const RxP& r, double lam, double rho, double p) {
  if (!(lam > 0.0)) return 0.0;
  const double F = 1.0 - lam;
  double out = 0.0;
  const double mu = rho / r.ig_rho0 - 1.0 - r.ig_a;
  if (r.igFig - F > 0.0 && mu > 0.0) out = out + r.igI * pow(lam, r.ig_b) * pow(mu, r.ig_x);
  const double ph = fmax(p, 0.0) / r.ig_punit;
  if (F > 0.0) {
    if (r.igFG1 - F > 0.0) out = out + r.igG1 * pow(lam, r.ig_c) * pow(F, r.ig_d) * pow(ph, r.ig_y);
    if (F - r.igFG2 > 0.0) out = out + r.igG2 * pow(lam, r.ig_e) * pow(F, r.ig_g) * pow(ph, r.ig_z);
  }
  return out;
}

// Cylindrical geometric source s_g of Sec. 3 at radius r (2-D, x = r, y = z,
// theta the third direction): dq/dt = -(1/r) (0 for phi, m_l u_r, the history
// slot times u_r, rho u_r^2 - sig_rr + sig_tt, rho u_z u_r - sig_rz,
// rho E u_r - (u_r sig_rr + u_z sig_zr), (1/3 - delta_{i theta}) Vbar_ij u_r)
// with the mixture stress sig = -p I + 2 G dev H
template <int D, int N, int RX>
__device__ __forceinline__ void geom_rate(const Params& P, const double* U, double r, double* S) {
  using L = Lay<D, N, RX>;
  double W[L::F], H[6], J2;
  Thermo<N, RX> T;
  cons_to_prim<D, N, RX>(P, U, W, T, H, J2);
  const double ur = W[L::MOM0], uz = W[L::MOM0 + 1];
  const double g2 = 2.0 * T.Gmix;
  const double srr = g2 * H[0] - T.p, stt = g2 * H[5] - T.p, srz = g2 * H[1];
#pragma unroll
  for (int f = 0; f < L::F; ++f) S[f] = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) S[L::M0 + l] = -(U[L::M0 + l] * ur) / r;
  if (RX) S[L::LAM] = -(U[L::LAM] * ur) / r;
  S[L::MOM0] = -(U[L::MOM0] * ur - srr + stt) / r;
  S[L::MOM0 + 1] = -(U[L::MOM0 + 1] * ur - srz) / r;
  S[L::E] = -(U[L::E] * ur - (ur * srr + uz * srz)) / r;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const double coef = (L::vi(q) == 2) ? (1.0 / 3.0 - 1.0) : 1.0 / 3.0;
    S[L::V0 + q] = -(coef * U[L::V0 + q] * ur) / r;
  }
}

// the geometric fractional step over dt by Heun's method
template <int D, int N, int RX>
__device__ __forceinline__ void geom_cell(const Params& P, double* U, double r, double dt) {
  using L = Lay<D, N, RX>;
  double S0[L::F], S1[L::F], U1[L::F];
  geom_rate<D, N, RX>(P, U, r, S0);
#pragma unroll
  for (int f = 0; f < L::F; ++f) U1[f] = U[f] + dt * S0[f];
  geom_rate<D, N, RX>(P, U1, r, S1);
#pragma unroll
  for (int f = 0; f < L::F; ++f) U[f] = U[f] + (0.5 * dt) * (S0[f] + S1[f]);
}

// Reaction (Sec. 3.3): RK4 on lambda at fixed mass and total energy, the
// pressure re-evaluated at every stage; rate -k lam (max(p,0)/pref)^n or
// the ignition-and-growth law.  WS: also the per-direction wave speed of the
// result (the last step of the fused epilogue), from the same phase
// densities, velocity and non-reactive closures with the split at the new
// lambda.
template <int D, int N, int RX, bool WS = false>
__device__ __forceinline__ void reaction_cell(const Params& P, double* U, double dt, double* s = nullptr);

// per-direction |u_d| + c_L of one cell
template <int D, int N, int RX>
__device__ __forceinline__ void wavespeed_cell(const Params& P, const double* U, double s[D]);

template <int D, int N, int RX, bool WS>
__device__ __forceinline__ void reaction_cell(const Params& P, double* U, double dt, double* s) {
  using L = Lay<D, N, RX>;
  const RxP& r = P.rx;
  const int y = r.mat;
  const double my = rx_mix<RX>(P) ? pick<N>(U + L::M0, y) : 0.0;
  if (!rx_mix<RX>(P) || !(my > 0.0)) {
    if (WS) wavespeed_cell<D, N, RX>(P, U, s);
    return;
  }
  Phases<N> Q;
  phases_from_partial<N>(U, U + L::M0, Q);
  double rt = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) rt += U[L::M0 + l];
  const double irt = frcp(rt);
  double u[D], uu = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    u[k] = U[L::MOM0 + k] * irt;
    uu += u[k] * u[k];
  }
  double H[6], J2;
  strain<D, N, RX>(U + L::V0, H, J2);
  Thermo<N, RX> T;
  eos_all<N, RX>(P, Q, J2, T);  // the non-reactive materials
  const double rhoe = U[L::E] - 0.5 * rt * uu;
  double num0 = rhoe, den0 = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    if (l == y) continue;
    den0 += Q.phi[l] * T.e[l].invGam;
    num0 += Q.phi[l] * (T.e[l].pref * T.e[l].invGam - Q.rho[l] * T.e[l].eref);
  }
  double phi_y = 0.0, rho_y = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l)
    if (l == y) {
      phi_y = Q.phi[l];
      rho_y = Q.rho[l];
    }
  auto rate = [&](double lam) {
    const double lc = fmin(fmax(lam, 0.0), 1.0);
    const double p = rx_pressure<RX == 2>(r, phi_y, rho_y, lc, num0, den0);
    if (r.law == LAW_IG) return -ig_rate(r, lc, rho_y, p);
    const double x = fmax(p, 0.0) * r.inv_pref;
    const double xn = r.n_is2 ? x * x : pow(x, r.n);
    return -r.k * lc * xn;
  };
  const double l0 = fmin(fmax(U[L::LAM] * frcp(my), 0.0), 1.0);
  const double k1 = rate(l0);
  double l1 = l0;
  // no rate at the start (an unreacted cell below the ignition threshold, a
  // fully burnt one): every later stage evaluates the same lambda and gives
  // 0 again, so the result is l0 exactly
  if (k1 != 0.0) {
    const double k2 = rate(l0 + 0.5 * dt * k1);
    const double k3 = rate(l0 + 0.5 * dt * k2);
    const double k4 = rate(l0 + dt * k3);
    l1 = l0 + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
    l1 = fmin(fmax(l1, 0.0), 1.0);
  }
  U[L::LAM] = my * l1;
  if (WS) {
    double num, den;
    rx_cons<RX == 2>(r, phi_y, rho_y, l1, num0, den0, T.rho_a, T.rho_b, T.A, T.B, num, den);
    T.rho = rt;
    T.irho = irt;
    T.xi = den;
    T.ixi = frcp(den);
    T.p = num * T.ixi;
    T.rhoe = rhoe;
    finish<N, RX>(P, Q, l1, T, true, true);
    const double cl = sqrt(T.cL2);
#pragma unroll
    for (int k = 0; k < D; ++k) s[k] = fabs(u[k]) + cl;
  }
}

template <int D, int N, int RX>
__device__ __forceinline__ void wavespeed_cell(const Params& P, const double* U, double s[D]) {
  using L = Lay<D, N, RX>;
  double W[L::F];
  Thermo<N, RX> T;
  double H[6], J2;
  cons_to_prim<D, N, RX>(P, U, W, T, H, J2);
  const double cl = sqrt(T.cL2);
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = fabs(W[L::MOM0 + k]) + cl;
}

// The last sweep's epilogue on the new conserved state: plastic relaxation,
// reaction, and the per-direction wave speed of the result.  Without a
// reactive mixture the plastic weights phi_l/Gamma_l need no pressure, so the
// phase densities and velocity are computed once and only the strain-
// dependent closures are evaluated again for the wave speed.
template <int D, int N, int RX>
__device__ __forceinline__ void epilogue_cell(const Params& P, double* U, double dt, double s[D]) {
  if (RX) {
    plastic_cell<D, N, RX>(P, U, dt);
    reaction_cell<D, N, RX, true>(P, U, dt, s);
    return;
  }
  using L = Lay<D, N, RX>;
  Phases<N> Q;
  phases_from_partial<N>(U, U + L::M0, Q);
  double r = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) r += U[L::M0 + l];
  const double inv_r = frcp(r);
  double u[D], uu = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    u[k] = U[L::MOM0 + k] * inv_r;
    uu += u[k] * u[k];
  }
  // plastic step (Sec. 3.2)
  double H[6], J2;
  strain<D, N, RX>(U + L::V0, H, J2);
  const double J = sqrt(J2);
  double xi = 0.0, num = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    const MatP& m = P.mat[l];
    const double wl = Q.phi[l] * m.invGam;
    xi += wl;
    if (!m.shear) continue;
    double Jl = J;
    if (m.plast == PLAST_PERFECT) Jl = fmin(J, m.yield_s6 * frcp(shear_modulus(m, Q.rho[l])));
    num += wl * Jl;
  }
  const double fac = (J > 0.0) ? (num * frcp(xi)) * frcp(J) : 0.0;
  double Mm[6], Mp[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double id = (q == 0 || q == 3 || q == 5) ? 1.0 : 0.0;
    const double hq = (J > 0.0) ? fac * H[q] : 0.0;
    Mm[q] = id - 0.5 * hq;
    Mp[q] = id + 0.5 * hq;
  }
  double A[6];
  A[0] = Mm[3] * Mm[5] - Mm[4] * Mm[4];
  A[1] = Mm[2] * Mm[4] - Mm[1] * Mm[5];
  A[2] = Mm[1] * Mm[4] - Mm[2] * Mm[3];
  A[3] = Mm[0] * Mm[5] - Mm[2] * Mm[2];
  A[4] = Mm[2] * Mm[1] - Mm[0] * Mm[4];
  A[5] = Mm[0] * Mm[3] - Mm[1] * Mm[1];
  const double inv_det = frcp(Mm[0] * A[0] + Mm[1] * A[1] + Mm[2] * A[2]);
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (hnz<D>(i, k) && hnz<D>(k, j)) v += A[hs(i, k)] * Mp[hs(k, j)];
    U[L::V0 + q] = v * inv_det;
  }
  // wave speed of the relaxed state
  strain<D, N, RX>(U + L::V0, H, J2);
  Thermo<N, RX> T;
  T.rho = r;
  T.irho = inv_r;
  eos_all<N, RX>(P, Q, J2, T);
  T.rhoe = U[L::E] - 0.5 * r * uu;
  pressure_from_rhoe<N, RX>(P, Q, 0.0, T);
  finish<N, RX>(P, Q, 0.0, T, true, true);
  const double cl = sqrt(T.cL2);
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = fabs(u[k]) + cl;
}

// --------------------------------------------------- wave max reduction
// Non-negative doubles order like their bit patterns (a NaN, positive here,
// orders above every finite value).  The wave maximum is pushed with an
// atomic only when it exceeds the value last seen at the destination: the
// destination only grows, so a stale read can only cause an extra atomic.
__device__ __forceinline__ void wave_max_atomic(double v, unsigned long long* dst) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = (o > v || o != o) ? o : v;
  }
  if ((threadIdx.x & 63) == 0) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned long long seen = __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (b > seen) atomicMax(dst, b);
  }
}

// The wave maximum of v written by lane 0 to its own slot (no atomics: one
// slot per wave, reduced afterwards in a fixed order).
__device__ __forceinline__ void wave_max_store(double v, double* dst) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = (o > v || o != o) ? o : v;
  }
  if ((threadIdx.x & 63) == 0) *dst = v;
}

// ------------------------------------------------------------- indexing
// index along one axis under its boundary rule: periodic wrap, otherwise
// clamped (transmissive; also a reflective axis's transverse neighbour, where
// the mirror image of cell -1 is cell 0)
__device__ __forceinline__ int64_t bc_map(int64_t i, int64_t n, int bc) {
  if (bc == BC_PERIODIC) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

// along a sweep axis with reflective ends (both, or the low end for
// BC_AXIS): the mirror image -1 - i or 2n - 1 - i, then clamped (a grid
// thinner than the stencil)
__device__ __forceinline__ int64_t bc_map_wall(int64_t i, int64_t n, int bc) {
  if (i < 0) i = -1 - i;
  else if (i > n - 1 && bc == BC_REFLECTIVE) i = 2 * n - 1 - i;
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

// whether position i along an axis with rule bc reads a mirror image
__device__ __forceinline__ bool bc_mirrored(int64_t i, int64_t n, int bc) {
  return (i < 0 && (bc == BC_REFLECTIVE || bc == BC_AXIS)) || (i > n - 1 && bc == BC_REFLECTIVE);
}

}  // namespace dimp
