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

// ---------------------------------------------------------- candidates
template <int D, int N, bool RX>
__device__ __forceinline__ Cand phi_candidates(const Params& P, double qm, double q0, double qp, double nd) {
  Cand c;
  const double s = slope<D, N, RX>(P, 0, qm, q0, qp);
  c.mL = q0 - 0.5 * s;
  c.mR = q0 + 0.5 * s;
  c.tL = c.mL;
  c.tR = c.mR;
  if (P.thinc) {
    const double beta = P.beta0 * nd + 0.01;
    thinc_edges(qm, q0, qp, beta, P.eps, P.delta, c.mL, c.mR, c.tL, c.tR);
  }
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

// stress column sigma_{k,DIR} = 2 G dev H - p delta from a primitive state
template <int D, int N, bool RX, int DIR>
__device__ __forceinline__ void stress_col(const Params& P, const double* W, double sig[3]) {
  using L = Lay<D, N, RX>;
  if (!P.any_shear) {
#pragma unroll
    for (int k = 0; k < 3; ++k) sig[k] = (k == DIR) ? -W[L::E] : 0.0;
    return;
  }
  Thermo<N, RX> T;
  double H[6], J2;
  prim_thermo<D, N, RX>(P, W, T, H, J2, false);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (hnz<D>(k, DIR))
      sig[k] = 2.0 * T.Gmix * H[hs(k, DIR)] - ((k == DIR) ? T.p : 0.0);
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
template <int D, int N, bool RX, int DIR>
__device__ __forceinline__ void edges_predict(const Params& P, const double* Wm, const double* W0, const double* Wp,
                                              double rho0, double rc2, const Cand& cm, const Cand& c0,
                                              const Cand& cp, double nu, double* WL, double* WR) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const double s = slope<D, N, RX>(P, f, Wm[f], W0[f], Wp[f]);
    WL[f] = W0[f] - 0.5 * s;
    WR[f] = W0[f] + 0.5 * s;
  }
  if (P.thinc) {
    // N = 2: one stored volume fraction
    const double tm = tbv(cm, cp, c0.mL, c0.mR);
    const double tt = tbv(cm, cp, c0.tL, c0.tR);
    if (tt < tm) {
      WL[0] = c0.tL;
      WR[0] = c0.tR;
    } else {
      WL[0] = c0.mL;
      WR[0] = c0.mR;
    }
  }
  double sL[3], sR[3];
  stress_col<D, N, RX, DIR>(P, WL, sL);
  stress_col<D, N, RX, DIR>(P, WR, sR);
  double dW[F];
#pragma unroll
  for (int f = 0; f < F; ++f) dW[f] = WR[f] - WL[f];
  const double un = W0[L::MOM0 + DIR];
  const double dun = dW[L::MOM0 + DIR];
  const double inv_rho = 1.0 / rho0;
  double inc[F];
#pragma unroll
  for (int l = 0; l < N - 1; ++l) inc[l] = un * dW[l];
#pragma unroll
  for (int l = 0; l < N; ++l) inc[L::M0 + l] = un * dW[L::M0 + l] + W0[L::M0 + l] * dun;
  if (RX) inc[L::LAM] = un * dW[L::LAM];
#pragma unroll
  for (int k = 0; k < D; ++k) inc[L::MOM0 + k] = un * dW[L::MOM0 + k] - (sR[k] - sL[k]) * inv_rho;
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
  if (RX) {
    WL[L::LAM] = fmin(fmax(WL[L::LAM], 0.0), 1.0);
    WR[L::LAM] = fmin(fmax(WR[L::LAM], 0.0), 1.0);
  }
}

// ----------------------------------------------------------- face flux
template <int D, int N, bool RX>
struct Side {
  double rho, E, cl;
  double u[D];
  double sig[3];  // sigma_{k n}
};

template <int D, int N, bool RX, int DIR>
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

// conserved vector and physical flux of one side, written straight into the
// face result (used for supersonic faces)
template <int D, int N, bool RX, int DIR>
__device__ __forceinline__ void side_flux(const double* W, const Side<D, N, RX>& S, FaceV<D, N, RX>& out) {
  using L = Lay<D, N, RX>;
  const double un = S.u[DIR];
#pragma unroll
  for (int l = 0; l < N - 1; ++l) out.F[l] = W[l] * un;
  double phiN = 1.0;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) phiN -= W[l];
#pragma unroll
  for (int l = 0; l < N; ++l) out.F[L::M0 + l] = ((l < N - 1 ? W[l] : phiN) * W[L::M0 + l]) * un;
  if (RX) out.F[L::LAM] = 0.0;  // filled by the caller that knows phi_y
  double us = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    out.F[L::MOM0 + k] = (S.rho * S.u[k]) * un - S.sig[k];
    us += S.u[k] * S.sig[k];
  }
  out.F[L::E] = S.E * un - us;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    double v = W[L::V0 + q] * un;
    if (i < D && L::vq(DIR, j) >= 0) v -= vget<D, N, RX>(W + L::V0, DIR, j) * S.u[i];
    out.F[L::V0 + q] = v;
  }
  out.ustar = un;
#pragma unroll
  for (int j = 0; j < D; ++j) out.Vn[j] = vget<D, N, RX>(W + L::V0, DIR, j);
}

template <int D, int N, bool RX>
__device__ __forceinline__ double m_lambda(const Params& P, const double* W) {
  using L = Lay<D, N, RX>;
  const int y = P.rx.mat;
  double phi_y;
  if (y < N - 1) {
    phi_y = W[y];
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

// HLLC-type star flux of side K: Rankine-Hugoniot across S_K with velocity
// (S*, u*_t) and traction continuous across the contact
template <int D, int N, bool RX, int DIR>
__device__ __forceinline__ void star_flux(const Params& P, const double* W, const Side<D, N, RX>& S, double SK,
                                          double Sst, const double ust[D], double mK, FaceV<D, N, RX>& out) {
  using L = Lay<D, N, RX>;
  side_flux<D, N, RX, DIR>(W, S, out);
  const double un = S.u[DIR];
  const double a = SK - un;
  const double inv = 1.0 / (SK - Sst);
  const double r = a * inv;
  const double rm1 = r - 1.0;
  double phiN = 1.0;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) phiN -= W[l];
  // mass-like components: U* - U = (r - 1) U
#pragma unroll
  for (int l = 0; l < N; ++l)
    out.F[L::M0 + l] += SK * (rm1 * ((l < N - 1 ? W[l] : phiN) * W[L::M0 + l]));
  if (RX) {
    const double ml = m_lambda<D, N, RX>(P, W);
    out.F[L::LAM] = ml * un + SK * (rm1 * ml);
  }
  const double rs = r * S.rho;
  double sst[3];
  double usK = 0.0, usS = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    out.F[L::MOM0 + k] += SK * (rs * ust[k] - S.rho * S.u[k]);
    sst[k] = S.sig[k] - mK * (ust[k] - S.u[k]);
    usK += S.u[k] * S.sig[k];
    usS += ust[k] * sst[k];
  }
  const double Es = (S.E * a + (usK - usS)) * inv;
  out.F[L::E] += SK * (Es - S.E);
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    if (i == DIR) continue;  // normal row is continuous: U* = U
    const double V = W[L::V0 + q];
    double Vs = a * V;
    if (i < D && L::vq(DIR, j) >= 0) Vs -= vget<D, N, RX>(W + L::V0, DIR, j) * (ust[i < D ? i : 0] - S.u[i < D ? i : 0]);
    Vs *= inv;
    out.F[L::V0 + q] += SK * (Vs - V);
  }
  const double us_face = un + SK * rm1;
  out.ustar = us_face;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) out.F[l] = W[l] * us_face;
}

template <int D, int N, bool RX, int DIR>
__device__ __forceinline__ void face_flux(const Params& P, const double* WL, const double* WR,
                                          FaceV<D, N, RX>& out) {
  using L = Lay<D, N, RX>;
  Side<D, N, RX> A, B;
  side_state<D, N, RX, DIR>(P, WL, A);
  side_state<D, N, RX, DIR>(P, WR, B);
  const double uL = A.u[DIR], uR = B.u[DIR];
  const double SL = fmin(uL - A.cl, uR - B.cl);
  const double SR = fmax(uL + A.cl, uR + B.cl);
  if (SL >= 0.0) {
    side_flux<D, N, RX, DIR>(WL, A, out);
    if (RX) out.F[L::LAM] = m_lambda<D, N, RX>(P, WL) * uL;
    return;
  }
  if (SR <= 0.0) {
    side_flux<D, N, RX, DIR>(WR, B, out);
    if (RX) out.F[L::LAM] = m_lambda<D, N, RX>(P, WR) * uR;
    return;
  }
  const double mL = A.rho * (SL - uL);
  const double mR = B.rho * (SR - uR);
  const double den = mL - mR;
  double ust[D];
#pragma unroll
  for (int k = 0; k < D; ++k) ust[k] = ((A.sig[k] - B.sig[k]) + (mL * A.u[k] - mR * B.u[k])) / den;
  const double Sst = ust[DIR];
  if (Sst > 0.0) {
    star_flux<D, N, RX, DIR>(P, WL, A, SL, Sst, ust, mL, out);
  } else if (Sst < 0.0) {
    star_flux<D, N, RX, DIR>(P, WR, B, SR, Sst, ust, mR, out);
  } else {
    FaceV<D, N, RX> o2;
    star_flux<D, N, RX, DIR>(P, WL, A, SL, Sst, ust, mL, out);
    star_flux<D, N, RX, DIR>(P, WR, B, SR, Sst, ust, mR, o2);
#pragma unroll
    for (int f = 0; f < L::F; ++f) out.F[f] = 0.5 * (out.F[f] + o2.F[f]);
    out.ustar = 0.5 * (out.ustar + o2.ustar);
#pragma unroll
    for (int j = 0; j < D; ++j) out.Vn[j] = 0.5 * (out.Vn[j] + o2.Vn[j]);
  }
}

// ---------------------------------------------------------------- update
// U^{new} = U - nu (F_b - F_a) with phi's source phi div u and Vbar's sources
// (2/3) Vbar div u - u_i beta_j taken with the face velocities u* and the
// upwinded normal rows Vbar*_{n j} (cell-centre coefficients).
template <int D, int N, bool RX, int DIR>
__device__ __forceinline__ void update_cell(const double* U, const FaceV<D, N, RX>& a, const FaceV<D, N, RX>& b,
                                            double nu, double* Un) {
  using L = Lay<D, N, RX>;
  const double du = b.ustar - a.ustar;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) Un[l] = U[l] - nu * ((b.F[l] - a.F[l]) - U[l] * du);
#pragma unroll
  for (int f = N - 1; f < L::V0; ++f) Un[f] = U[f] - nu * (b.F[f] - a.F[f]);
  double rho = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) rho += U[L::M0 + l];
  const double inv_rho = 1.0 / rho;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    double src = (2.0 / 3.0) * U[L::V0 + q] * du;
    if (i < D && j < D) src -= (U[L::MOM0 + (i < D ? i : 0)] * inv_rho) * (b.Vn[j < D ? j : 0] - a.Vn[j < D ? j : 0]);
    Un[L::V0 + q] = U[L::V0 + q] - nu * ((b.F[L::V0 + q] - a.F[L::V0 + q]) - src);
  }
}

// --------------------------------------------------------------- sources
// Plastic relaxation (Sec. 3.2): per-material targets of the strain
// invariant (fluid 0, elastic J, ideal plasticity min(J, sigma_Y/(sqrt6 G))),
// mixed with phi/Gamma weights; dev H rescaled; Vbar rebuilt by the first
// Pade approximant with an exact inverse.
template <int D, int N, bool RX>
__device__ __forceinline__ void plastic_cell(const Params& P, double* U) {
  using L = Lay<D, N, RX>;
  double W[L::F];
  Thermo<N, RX> T;
  double H[6], J2;
  cons_to_prim<D, N, RX>(P, U, W, T, H, J2);
  const double J = sqrt(J2);
  double num = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    if (RX && l == P.rx.mat) continue;
    const MatP& m = P.mat[l];
    if (!m.shear) continue;
    double Jl = J;
    if (m.plast) Jl = fmin(J, m.yield_s6 / T.e[l].G);
    const double phi_l = (l < N - 1) ? W[l] : 1.0 - [&] {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < N - 1; ++k) s += W[k];
      return s;
    }();
    num += phi_l * T.e[l].invGam * Jl;
  }
  const double fac = (J > 0.0) ? (num / T.xi) / J : 0.0;
  double Hs[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) Hs[s] = (J > 0.0) ? fac * H[s] : 0.0;
  // M- = I - H*/2, M+ = I + H*/2 (symmetric)
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
  const double inv_det = 1.0 / det;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    const double v = A[hs(i, 0)] * Mp[hs(0, j)] + A[hs(i, 1)] * Mp[hs(1, j)] + A[hs(i, 2)] * Mp[hs(2, j)];
    U[L::V0 + q] = v * inv_det;
  }
}

// pressure of a cell whose reactive progress is lam, with the non-reactive
// part of the pressure function (num0, den0) already summed
__device__ __forceinline__ double rx_pressure(const RxP& r, double phi_y, double rho_y, double lam, double num0,
                                              double den0) {
  const double A0 = num0 + phi_y * (r.pb * r.invGb - rho_y * (lam * r.ea + (1.0 - lam) * r.eb));
  const double A1 = phi_y * (r.pa * r.invGa - r.pb * r.invGb);
  const double B0 = den0 + phi_y * r.invGb;
  const double B1 = phi_y * (r.invGa - r.invGb);
  const double s = rx_solve_s(r, lam, A0, A1, B0, B1);
  double ra, rb;
  if (s >= 1.0 || s <= 0.0) {
    ra = rho_y;
    rb = rho_y;
  } else {
    ra = lam * rho_y / s;
    rb = (1.0 - lam) * rho_y / (1.0 - s);
  }
  const double wa = phi_y * rho_y * lam, wb = phi_y * rho_y * (1.0 - lam);
  const double den = den0 + wa * r.invGa / ra + wb * r.invGb / rb;
  const double num = num0 + wa * (r.pa * r.invGa / ra - r.ea) + wb * (r.pb * r.invGb / rb - r.eb);
  return num / den;
}

// Reaction (Sec. 3.3): RK4 on lambda at fixed mass and total energy, the
// pressure re-evaluated at every stage; rate -k lam (max(p,0)/pref)^n.
template <int D, int N, bool RX>
__device__ __forceinline__ void reaction_cell(const Params& P, double* U, double dt) {
  if (!RX) return;
  using L = Lay<D, N, RX>;
  const RxP& r = P.rx;
  const int y = r.mat;
  const double my = U[L::M0 + y];
  if (!(my > 0.0)) return;
  double phi[N], rho[N];
  double sphi = 0.0;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) {
    phi[l] = U[l];
    sphi += phi[l];
  }
  phi[N - 1] = 1.0 - sphi;
  double rt = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    rho[l] = U[L::M0 + l] / phi[l];
    rt += U[L::M0 + l];
  }
  double uu = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double uk = U[L::MOM0 + k] / rt;
    uu += uk * uk;
  }
  double H[6], J2;
  strain<D, N, RX>(U + L::V0, H, J2);
  double num0 = U[L::E] - 0.5 * rt * uu, den0 = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    if (l == y) continue;
    const EosV e = eos_eval(P.mat[l], rho[l], J2);
    den0 += phi[l] * e.invGam;
    num0 += phi[l] * (e.pref * e.invGam - rho[l] * e.eref);
  }
  double phi_y = 0.0, rho_y = 0.0;
#pragma unroll
  for (int l = 0; l < N; ++l)
    if (l == y) {
      phi_y = phi[l];
      rho_y = rho[l];
    }
  auto rate = [&](double lam) {
    const double lc = fmin(fmax(lam, 0.0), 1.0);
    const double p = rx_pressure(r, phi_y, rho_y, lc, num0, den0);
    const double x = fmax(p, 0.0) * r.inv_pref;
    const double xn = r.n_is2 ? x * x : pow(x, r.n);
    return -r.k * lc * xn;
  };
  const double l0 = fmin(fmax(U[L::LAM] / my, 0.0), 1.0);
  const double k1 = rate(l0);
  const double k2 = rate(l0 + 0.5 * dt * k1);
  const double k3 = rate(l0 + 0.5 * dt * k2);
  const double k4 = rate(l0 + dt * k3);
  double l1 = l0 + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
  l1 = fmin(fmax(l1, 0.0), 1.0);
  U[L::LAM] = my * l1;
}

// per-direction |u_d| + c_L of one cell
template <int D, int N, bool RX>
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

// --------------------------------------------------- wave max reduction
// non-negative doubles order like their bit patterns; NaN (positive) wins
__device__ __forceinline__ void wave_max_atomic(double v, unsigned long long* dst) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = (o > v || o != o) ? o : v;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

// ------------------------------------------------------------- indexing
__device__ __forceinline__ int64_t bc_map(int64_t i, int64_t n, int bc) {
  if (bc == BC_PERIODIC) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

}  // namespace dimp
