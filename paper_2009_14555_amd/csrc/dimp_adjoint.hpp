// dimp_adjoint.hpp -- hand-written reverse (vector-Jacobian) stages of the
// split step, for 2-D, two materials, no reactive mixture.
//
// Each *_bwd function takes the inputs of its forward stage and the adjoints
// ("bars") of the stage outputs, recomputes the forward intermediates it
// needs, and accumulates the adjoints of the stage inputs.  Non-smooth
// operations (min/max, clamps, the Riemann branch, BVD, the THINC mixed-cell
// test and the yield min) are differentiated along the branch the forward
// takes; the smooth limiter of the adjoint mode is van Albada.  At S* = 0
// exactly the face flux is the mean of the two star fluxes (as in the
// forward), and its adjoint is the mean of the two branch adjoints.
//
// Material-parameter adjoints are accumulated per material in the packed
// form (Gamma, 1/Gamma, p_ref, e_ref, G0, sigma_Y/sqrt6); the host maps them
// to (gamma, p_inf, G0, sigma_Y).  `own` gates the parameter accumulation so
// that every stage instance is counted by exactly one wave.
#pragma once
#include "dimp_stencil.hpp"

namespace dimp {
namespace adj {

using L2 = Lay<2, 2, false>;
constexpr int F2 = L2::F;  // 11

enum { PB_GAM = 0, PB_IGAM, PB_PREF, PB_EREF, PB_G0, PB_Y, PB_N };

struct PBar {
  double v[2][PB_N];
};

// add v to a parameter adjoint only on the wave that owns the stage
// instance (a select, so a discarded lane's value never reaches the sum)
__device__ __forceinline__ void pacc(double& dst, bool own, double v) { dst = own ? dst + v : dst; }

__device__ __forceinline__ void pbar_zero(PBar& b) {
#pragma unroll
  for (int l = 0; l < 2; ++l)
#pragma unroll
    for (int k = 0; k < PB_N; ++k) b.v[l][k] = 0.0;
}

struct EosB {
  double Gam, invGam, pref, eref, dpref, deref, G;
};

__device__ __forceinline__ EosB eosb_zero() {
  EosB b;
  b.Gam = b.invGam = b.pref = b.eref = b.dpref = b.deref = b.G = 0.0;
  return b;
}

// ---------------------------------------------------------------- closures
// adjoint of eos_eval at (rho, irho, J2): rho, irho and J2 are independent
// inputs of the closure (as in the forward, which is handed both densities)
__device__ __forceinline__ void eos_bwd(const MatP& m, int l, double rho, double irho, double J2, const EosB& b,
                                        double& rb, double& ib, double& jb, PBar& pb, bool own) {
  pacc(pb.v[l][PB_GAM], own, b.Gam);
  pacc(pb.v[l][PB_IGAM], own, b.invGam);
  if (m.eos != EOS_ROMENSKII) {
    pacc(pb.v[l][PB_PREF], own, b.pref);
    pacc(pb.v[l][PB_EREF], own, b.eref);
    return;
  }
  const double a = m.abar, bb = m.bbar;
  const double x = rho * m.inv_rho0;
  const double xa = pow(x, a);
  const double xb1 = pow(x, bb + 1.0);
  const double G = m.G0 * xb1;
  const double GJ = G * J2;
  const double pc = m.K0a * x * xa * (xa - 1.0);
  const double pref = pc + bb * GJ;
  // deref = pref irho^2
  const double prefb = b.pref + b.deref * irho * irho;
  ib += b.deref * 2.0 * pref * irho;
  // pref = pc + bb GJ; eref = ec + GJ irho; dpref = dpc + bb(bb+1) GJ irho
  const double GJb = prefb * bb + b.eref * irho + b.dpref * bb * (bb + 1.0) * irho;
  ib += b.eref * GJ + b.dpref * bb * (bb + 1.0) * GJ;
  const double pcb = prefb, ecb = b.eref, dpcb = b.dpref;
  const double Gb = b.G + GJb * J2;
  jb += GJb * G;
  pacc(pb.v[l][PB_G0], own, Gb * xb1);
  double xbar = Gb * m.G0 * (bb + 1.0) * pow(x, bb);
  xbar += pcb * m.K0a * xa * (xa - 1.0);
  double xab = pcb * m.K0a * x * (2.0 * xa - 1.0);
  xab += ecb * m.ec_coef * 2.0 * (xa - 1.0);
  xab += dpcb * m.dpc_coef * (2.0 * (2.0 * a + 1.0) * xa - (a + 1.0));
  xbar += xab * a * pow(x, a - 1.0);
  rb += xbar * m.inv_rho0;
}

// adjoint of shear_modulus(m, rho) = G0 x^(b+1)
__device__ __forceinline__ void shear_bwd(const MatP& m, int l, double rho, double Gb, double& rb, PBar& pb,
                                          bool own) {
  if (!m.shear) return;
  const double x = rho * m.inv_rho0;
  pacc(pb.v[l][PB_G0], own, Gb * pow(x, m.bbar + 1.0));
  rb += Gb * m.G0 * (m.bbar + 1.0) * pow(x, m.bbar) * m.inv_rho0;
}

// adjoint of c2_mat(e, rho, irho, p)
__device__ __forceinline__ void c2mat_bwd(const EosV& e, double rho, double irho, double p, double cb, EosB& eb,
                                          double& rb, double& ib, double& pbar) {
  eb.dpref += cb;
  rb -= cb * e.Gam * e.deref;
  eb.Gam += cb * (-rho * e.deref + p * irho);
  eb.deref -= cb * rho * e.Gam;
  pbar += cb * (1.0 + e.Gam) * irho;
  eb.pref -= cb * irho;
  ib += cb * ((1.0 + e.Gam) * p - e.pref);
}

// ------------------------------------------------------------------ strain
// 2-D stretch tensor slots V00, V01, V10, V11, V22; symmetric slots of B, A,
// H: 0 = 00, 1 = 01, 3 = 11, 5 = 22 (02 and 12 vanish)
__device__ __forceinline__ void strain_bwd(const double* V, const double* Hb_in, double J2b, double* Vb) {
  const double V00 = V[0], V01 = V[1], V10 = V[2], V11 = V[3], V22 = V[4];
  const double B0 = V00 * V00 + V01 * V01, B1 = V00 * V10 + V01 * V11, B3 = V10 * V10 + V11 * V11, B5 = V22 * V22;
  const double A0 = B3 * B5, A1 = -B1 * B5, A3 = B0 * B5, A5 = B0 * B3 - B1 * B1;
  const double K0 = 0.25 * (B0 - A0), K1 = 0.25 * (B1 - A1), K3 = 0.25 * (B3 - A3), K5 = 0.25 * (B5 - A5);
  const double tr = (K0 + K3 + K5) * (1.0 / 3.0);
  const double H0 = K0 - tr, H1 = K1, H3 = K3 - tr, H5 = K5 - tr;
  const double Hb0 = Hb_in[0] + 2.0 * J2b * H0, Hb1 = Hb_in[1] + 4.0 * J2b * H1;
  const double Hb3 = Hb_in[3] + 2.0 * J2b * H3, Hb5 = Hb_in[5] + 2.0 * J2b * H5;
  const double mb = (Hb0 + Hb3 + Hb5) * (1.0 / 3.0);
  const double Kb0 = Hb0 - mb, Kb1 = Hb1, Kb3 = Hb3 - mb, Kb5 = Hb5 - mb;
  double Bb0 = 0.25 * Kb0, Bb1 = 0.25 * Kb1, Bb3 = 0.25 * Kb3, Bb5 = 0.25 * Kb5;
  const double Ab0 = -0.25 * Kb0, Ab1 = -0.25 * Kb1, Ab3 = -0.25 * Kb3, Ab5 = -0.25 * Kb5;
  Bb3 += Ab0 * B5 + Ab5 * B0;
  Bb5 += Ab0 * B3 - Ab1 * B1 + Ab3 * B0;
  Bb1 += -Ab1 * B5 - 2.0 * Ab5 * B1;
  Bb0 += Ab3 * B5 + Ab5 * B3;
  Vb[0] += 2.0 * Bb0 * V00 + Bb1 * V10;
  Vb[1] += 2.0 * Bb0 * V01 + Bb1 * V11;
  Vb[2] += Bb1 * V00 + 2.0 * Bb3 * V10;
  Vb[3] += Bb1 * V01 + 2.0 * Bb3 * V11;
  Vb[4] += 2.0 * Bb5 * V22;
}

// --------------------------------------------------- conserved -> primitive
// Outputs of the forward used downstream in a sweep: W (all 11), irho0 =
// 1/(m0+m1) and rc2 = rho c^2.  Ub accumulates.
__device__ __forceinline__ void c2p_bwd(const Params& P, const double* U, const double* Wb, double irb_out,
                                        double rc2b, double* Ub, PBar& pb, bool own) {
  using L = L2;
  const double phi[2] = {U[0], 1.0 - U[0]};
  const double m[2] = {U[L::M0], U[L::M0 + 1]};
  double rho[2], irho[2];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    rho[l] = m[l] / phi[l];
    irho[l] = phi[l] / m[l];
  }
  const double r = m[0] + m[1];
  const double ir = 1.0 / r;
  double u[2], uu = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    u[k] = U[L::MOM0 + k] * ir;
    uu += u[k] * u[k];
  }
  double H[6], J2;
  strain<2, 2, false>(U + L::V0, H, J2);
  EosV e[2];
#pragma unroll
  for (int l = 0; l < 2; ++l) e[l] = eos_eval(P.mat[l], rho[l], irho[l], J2);
  const double rhoe = U[L::E] - 0.5 * r * uu;
  double xi = 0.0, num = rhoe;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    xi += phi[l] * e[l].invGam;
    num += phi[l] * (e[l].pref * e[l].invGam - rho[l] * e[l].eref);
  }
  const double ixi = 1.0 / xi;
  const double p = num * ixi;
  double cl2[2], cnum = 0.0;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    cl2[l] = c2_mat(e[l], rho[l], irho[l], p);
    cnum += (phi[l] * rho[l] * ir) * cl2[l] * e[l].invGam;
  }
  const double c2 = cnum * ixi;
  // ---- reverse
  double phib[2] = {Wb[0], 0.0};
  double rhob[2] = {Wb[L::M0], Wb[L::M0 + 1]};
  double irhob[2] = {0.0, 0.0};
  double ub[2] = {Wb[L::MOM0], Wb[L::MOM0 + 1]};
  double pbar = Wb[L::E];
  double rb = 0.0, irb = irb_out;
  EosB eb[2] = {eosb_zero(), eosb_zero()};
  // rc2 = r c2, c2 = cnum ixi
  rb += rc2b * c2;
  const double c2b = rc2b * r;
  const double cnumb = c2b * ixi;
  double ixib = c2b * cnum;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    const double g = e[l].invGam;
    const double w = phi[l] * rho[l] * ir;
    phib[l] += cnumb * rho[l] * ir * cl2[l] * g;
    rhob[l] += cnumb * phi[l] * ir * cl2[l] * g;
    irb += cnumb * phi[l] * rho[l] * cl2[l] * g;
    eb[l].invGam += cnumb * w * cl2[l];
    const double clb = cnumb * w * g;
    c2mat_bwd(e[l], rho[l], irho[l], p, clb, eb[l], rhob[l], irhob[l], pbar);
  }
  // p = num ixi
  const double numb = pbar * ixi;
  ixib += pbar * num;
  const double xib = -ixib * ixi * ixi;
  double rhoeb = numb;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    phib[l] += xib * e[l].invGam;
    eb[l].invGam += xib * phi[l];
    phib[l] += numb * (e[l].pref * e[l].invGam - rho[l] * e[l].eref);
    eb[l].pref += numb * phi[l] * e[l].invGam;
    eb[l].invGam += numb * phi[l] * e[l].pref;
    rhob[l] -= numb * phi[l] * e[l].eref;
    eb[l].eref -= numb * phi[l] * rho[l];
  }
  // rhoe = E - r uu / 2
  Ub[L::E] += rhoeb;
  rb -= 0.5 * rhoeb * uu;
#pragma unroll
  for (int k = 0; k < 2; ++k) ub[k] -= rhoeb * r * u[k];
  double J2b = 0.0;
#pragma unroll
  for (int l = 0; l < 2; ++l) eos_bwd(P.mat[l], l, rho[l], irho[l], J2, eb[l], rhob[l], irhob[l], J2b, pb, own);
  double Hb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double Vb[5] = {Wb[L::V0], Wb[L::V0 + 1], Wb[L::V0 + 2], Wb[L::V0 + 3], Wb[L::V0 + 4]};
  strain_bwd(U + L::V0, Hb, J2b, Vb);
#pragma unroll
  for (int q = 0; q < 5; ++q) Ub[L::V0 + q] += Vb[q];
  // u_k = mom_k / r
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    Ub[L::MOM0 + k] += ub[k] * ir;
    irb += ub[k] * U[L::MOM0 + k];
  }
  rb -= irb * ir * ir;
  double mb[2] = {rb, rb};
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    mb[l] += rhob[l] / phi[l] - irhob[l] * irho[l] / m[l];
    phib[l] += -rhob[l] * rho[l] / phi[l] + irhob[l] / m[l];
  }
  Ub[0] += phib[0] - phib[1];
  Ub[L::M0] += mb[0];
  Ub[L::M0 + 1] += mb[1];
}

// --------------------------------------------------------- limiter, THINC
// d vanalbada / d(a, b)
__device__ __forceinline__ void vanalbada_bwd(double a, double b, double e2, double sb, double& ab, double& bb) {
  const double Nn = a * (b * b + e2) + b * (a * a + e2);
  const double Dd = a * a + b * b + 2.0 * e2;
  const double iD = 1.0 / Dd;
  const double dNa = b * b + e2 + 2.0 * a * b, dNb = a * a + e2 + 2.0 * a * b;
  ab += sb * (dNa * Dd - Nn * 2.0 * a) * iD * iD;
  bb += sb * (dNb * Dd - Nn * 2.0 * b) * iD * iD;
}

// adjoint of youngs2(s, dx, d) into sb[3][3] (indices [x][y])
__device__ __forceinline__ void youngs2_bwd(const double s[3][3], const double* dx, int d, double nb,
                                            double sb[3][3]) {
  const double gx = ((s[2][0] - s[0][0]) + (s[2][2] - s[0][2])) + 2.0 * (s[2][1] - s[0][1]);
  const double gy = ((s[0][2] - s[0][0]) + (s[2][2] - s[2][0])) + 2.0 * (s[1][2] - s[1][0]);
  const double ax = gx / dx[0], ay = gy / dx[1];
  const double nn = sqrt(ax * ax + ay * ay);
  if (!(nn > 0.0)) return;
  const double ad = d == 0 ? ax : ay;
  const double ao = d == 0 ? ay : ax;
  const double sg = ad > 0.0 ? 1.0 : (ad < 0.0 ? -1.0 : 0.0);
  const double in3 = 1.0 / (nn * nn * nn);
  const double adb = nb * (sg / nn - fabs(ad) * ad * in3);
  const double aob = nb * (-fabs(ad) * ao * in3);
  const double axb = d == 0 ? adb : aob, ayb = d == 0 ? aob : adb;
  const double gxb = axb / dx[0], gyb = ayb / dx[1];
  sb[2][0] += gxb; sb[0][0] -= gxb; sb[2][2] += gxb; sb[0][2] -= gxb; sb[2][1] += 2.0 * gxb; sb[0][1] -= 2.0 * gxb;
  sb[0][2] += gyb; sb[0][0] -= gyb; sb[2][2] += gyb; sb[2][0] -= gyb; sb[1][2] += 2.0 * gyb; sb[1][0] -= 2.0 * gyb;
}

// Adjoint of phi_candidates: cb = bars of (mL, mR, tL, tR); accumulates the
// bars of (qm, q0, qp) and of the normal's stencil st[x][y].  The forward
// decisions are re-taken with the forward's own expressions.
template <int DIR>
__device__ __forceinline__ void cand_bwd(const Params& P, double qm, double q0, double qp, const double st[3][3],
                                         const double cb[4], double& qmb, double& q0b, double& qpb,
                                         double stb[3][3]) {
  const double a = q0 - qm, b = qp - q0;
  // MUSCL pair: mL = q0 - s/2, mR = q0 + s/2
  double sbar = 0.5 * (cb[1] - cb[0]);
  q0b += cb[0] + cb[1];
  double tLb = cb[2], tRb = cb[3];
  bool thinc_taken = false;
  if (P.thinc) {
    const double qmin = fmin(qm, qp);
    const double qmax = fmax(qm, qp) - qmin;
    const double num = q0 - qmin + P.eps, den = qmax + P.eps;
    if ((P.delta * den < num) && (num < (1.0 - P.delta) * den) && ((qp - q0) * (q0 - qm) > 0.0)) {
      thinc_taken = true;
      const double C = num / den;
      const double nd = youngs2(st, P.dx, DIR);
      const double beta = P.beta0 * nd + 0.01;
      const double eb = exp(beta);
      const double ieb = 1.0 / eb;
      const double ch = 0.5 * (eb + ieb), sh = 0.5 * (eb - ieb);
      const double tb = (eb - ieb) / (eb + ieb);
      const double Bv = exp(beta * (2.0 * C - 1.0));
      const double A = (Bv / ch - 1.0) / tb;
      const double den2 = 1.0 + A * tb;
      const double g = (tb + A) / den2;
      const bool dec = (qp - qm) < 0.0;
      const double lob = dec ? tRb : tLb;
      const double hib = dec ? tLb : tRb;
      double qminb = lob + hib;
      double qmaxb = 0.5 * (1.0 + A) * lob + 0.5 * (1.0 + g) * hib;
      const double gb = 0.5 * qmax * hib;
      double Ab = 0.5 * qmax * lob + gb * (1.0 - tb * tb) / (den2 * den2);
      double tbb = gb * (1.0 - A * A) / (den2 * den2);
      // A = (Bv/ch - 1)/tb
      const double Bvb = Ab / (ch * tb);
      const double chb = -Ab * Bv / (ch * ch * tb);
      tbb += -Ab * A / tb;
      // Bv = exp(beta (2C - 1))
      double betab = Bvb * Bv * (2.0 * C - 1.0);
      const double Cb = Bvb * Bv * 2.0 * beta;
      betab += chb * sh + tbb * (1.0 - tb * tb);
      // C = num / den
      q0b += Cb / den;
      qminb += -Cb / den;
      qmaxb += -Cb * C / den;
      youngs2_bwd(st, P.dx, DIR, betab * P.beta0, stb);
      // qmax = max(qm, qp) - qmin, qmin = min(qm, qp)
      if (qm <= qp) {
        qmb += qminb - qmaxb;
        qpb += qmaxb;
      } else {
        qpb += qminb - qmaxb;
        qmb += qmaxb;
      }
    }
  }
  if (!thinc_taken) {
    // (tL, tR) are the MUSCL pair
    sbar += 0.5 * (tRb - tLb);
    q0b += tLb + tRb;
  }
  double ab = 0.0, bb = 0.0;
  vanalbada_bwd(a, b, P.va_e2[0], sbar, ab, bb);
  qmb -= ab;
  q0b += ab - bb;
  qpb += bb;
}

// ---------------------------------------------------------------- stress
// adjoint of stress_col<2,2,false,DIR>(W) for a primitive state W
template <int DIR>
__device__ __forceinline__ void stress_bwd(const Params& P, const double* W, const double sigb[3], double* Wb,
                                           PBar& pb, bool own) {
  using L = L2;
  Wb[L::E] -= sigb[DIR];
  if (!P.any_shear) return;
  const double phi[2] = {W[0], 1.0 - W[0]};
  double Gl[2], xi = 0.0, gnum = 0.0;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    Gl[l] = shear_modulus(P.mat[l], W[L::M0 + l]);
    xi += phi[l] * P.mat[l].invGam;
    gnum += phi[l] * Gl[l] * P.mat[l].invGam;
  }
  const double G = gnum / xi;
  double H[6], J2;
  strain<2, 2, false>(W + L::V0, H, J2);
  double Gb = 0.0, Hb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    Gb += 2.0 * sigb[k] * H[hs(k, DIR)];
    Hb[hs(k, DIR)] += 2.0 * G * sigb[k];
  }
  const double gnumb = Gb / xi;
  const double xib = -Gb * G / xi;
  double phib[2] = {0.0, 0.0};
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    const double g = P.mat[l].invGam;
    phib[l] += gnumb * Gl[l] * g + xib * g;
    pacc(pb.v[l][PB_IGAM], own, (gnumb * phi[l] * Gl[l] + xib * phi[l]));
    double rb = 0.0;
    shear_bwd(P.mat[l], l, W[L::M0 + l], gnumb * phi[l] * g, rb, pb, own);
    Wb[L::M0 + l] += rb;
  }
  Wb[0] += phib[0] - phib[1];
  double Vb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  strain_bwd(W + L::V0, Hb, 0.0, Vb);
#pragma unroll
  for (int q = 0; q < 5; ++q) Wb[L::V0 + q] += Vb[q];
}

// ----------------------------------------------------- edges (predictor)
// Adjoint of edges_predict<2,2,false,DIR>: WLb, WRb are the bars of the
// returned edges.  Accumulates the bars of Wm, W0, Wp, irho0, rc2 and of the
// cell's own candidates (mL, mR, tL, tR).
template <int DIR>
__device__ __forceinline__ void edges_bwd(const Params& P, const double* Wm, const double* W0, const double* Wp,
                                          double irho0, double rc2, const Cand& cm, const Cand& c0, const Cand& cp,
                                          double nu, const double* WLb_in, const double* WRb_in, double* Wmb,
                                          double* W0b, double* Wpb, double& irho0b, double& rc2b, double cb[4],
                                          PBar& pb, bool own) {
  using L = L2;
  constexpr int F = F2;
  double s[F], WL[F], WR[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    s[f] = slope<2, 2, false>(P, f, Wm[f], W0[f], Wp[f]);
    WL[f] = W0[f] - 0.5 * s[f];
    WR[f] = W0[f] + 0.5 * s[f];
  }
  bool th = false;
  if (P.thinc) {
    const double tm = tbv(cm, cp, c0.mL, c0.mR);
    const double tt = tbv(cm, cp, c0.tL, c0.tR);
    th = tt < tm;
    WL[0] = th ? c0.tL : c0.mL;
    WR[0] = th ? c0.tR : c0.mR;
  }
  double sL[3], sR[3];
  stress_col<2, 2, false, DIR>(P, WL, sL);
  stress_col<2, 2, false, DIR>(P, WR, sR);
  double dW[F];
#pragma unroll
  for (int f = 0; f < F; ++f) dW[f] = WR[f] - WL[f];
  const double un = W0[L::MOM0 + DIR];
  const double dun = dW[L::MOM0 + DIR];
  double inc[F];
  inc[0] = un * dW[0];
#pragma unroll
  for (int l = 0; l < 2; ++l) inc[L::M0 + l] = un * dW[L::M0 + l] + W0[L::M0 + l] * dun;
#pragma unroll
  for (int k = 0; k < 2; ++k) inc[L::MOM0 + k] = un * dW[L::MOM0 + k] - (sR[k] - sL[k]) * irho0;
  inc[L::E] = un * dW[L::E] + rc2 * dun;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int a = L::vi(q), b = L::vj(q);
    double v = un * dW[L::V0 + q];
    if (a < 2 && L::vq(DIR, b) >= 0) v -= vget<2, 2, false>(W0 + L::V0, DIR, b) * dW[L::MOM0 + (a < 2 ? a : 0)];
    v += (1.0 / 3.0) * W0[L::V0 + q] * dun;
    inc[L::V0 + q] = v;
  }
  const double h = 0.5 * nu;
  // ---- reverse: clamps of phi
  double WLb[F], WRb[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    WLb[f] = WLb_in[f];
    WRb[f] = WRb_in[f];
  }
  {
    const double l0 = WL[0] - h * inc[0], r0 = WR[0] - h * inc[0];
    if (!(l0 > 0.0 && l0 < 1.0)) WLb[0] = 0.0;
    if (!(r0 > 0.0 && r0 < 1.0)) WRb[0] = 0.0;
  }
  double incb[F];
#pragma unroll
  for (int f = 0; f < F; ++f) incb[f] = -h * (WLb[f] + WRb[f]);
  double dWb[F];
#pragma unroll
  for (int f = 0; f < F; ++f) dWb[f] = 0.0;
  double unb = 0.0, dunb = 0.0;
  double sLb[3] = {0.0, 0.0, 0.0}, sRb[3] = {0.0, 0.0, 0.0};
  unb += incb[0] * dW[0];
  dWb[0] += incb[0] * un;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    const double ib = incb[L::M0 + l];
    unb += ib * dW[L::M0 + l];
    dWb[L::M0 + l] += ib * un;
    W0b[L::M0 + l] += ib * dun;
    dunb += ib * W0[L::M0 + l];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double ib = incb[L::MOM0 + k];
    unb += ib * dW[L::MOM0 + k];
    dWb[L::MOM0 + k] += ib * un;
    sRb[k] -= ib * irho0;
    sLb[k] += ib * irho0;
    irho0b -= ib * (sR[k] - sL[k]);
  }
  {
    const double ib = incb[L::E];
    unb += ib * dW[L::E];
    dWb[L::E] += ib * un;
    rc2b += ib * dun;
    dunb += ib * rc2;
  }
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int a = L::vi(q), b = L::vj(q);
    const double ib = incb[L::V0 + q];
    unb += ib * dW[L::V0 + q];
    dWb[L::V0 + q] += ib * un;
    if (a < 2 && L::vq(DIR, b) >= 0) {
      const int qn = L::vq(DIR, b) >= 0 ? L::vq(DIR, b) : 0;
      W0b[L::V0 + qn] -= ib * dW[L::MOM0 + (a < 2 ? a : 0)];
      dWb[L::MOM0 + (a < 2 ? a : 0)] -= ib * W0[L::V0 + qn];
    }
    W0b[L::V0 + q] += (1.0 / 3.0) * ib * dun;
    dunb += (1.0 / 3.0) * ib * W0[L::V0 + q];
  }
  dWb[L::MOM0 + DIR] += dunb;
  W0b[L::MOM0 + DIR] += unb;
  // dW = WR - WL (WL/WR here are the pre-predictor edges)
#pragma unroll
  for (int f = 0; f < F; ++f) {
    WRb[f] += dWb[f];
    WLb[f] -= dWb[f];
  }
  stress_bwd<DIR>(P, WL, sLb, WLb, pb, own);
  stress_bwd<DIR>(P, WR, sRb, WRb, pb, own);
  // edges from slopes (phi: from the BVD choice)
  double sbar[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    W0b[f] += WLb[f] + WRb[f];
    sbar[f] = 0.5 * (WRb[f] - WLb[f]);
  }
  cb[0] = cb[1] = cb[2] = cb[3] = 0.0;
  if (P.thinc) {
    // phi edges came from the candidates, not from the slope above
    W0b[0] -= WLb[0] + WRb[0];
    sbar[0] = 0.0;
    if (th) {
      cb[2] = WLb[0];
      cb[3] = WRb[0];
    } else {
      cb[0] = WLb[0];
      cb[1] = WRb[0];
    }
  }
#pragma unroll
  for (int f = 0; f < F; ++f) {
    double ab = 0.0, bb = 0.0;
    vanalbada_bwd(W0[f] - Wm[f], Wp[f] - W0[f], P.va_e2[L::kind(f)], sbar[f], ab, bb);
    Wmb[f] -= ab;
    W0b[f] += ab - bb;
    Wpb[f] += bb;
  }
}

// -------------------------------------------------------------- face flux
struct SideB {
  double rho, E, cl, u[2], sig[3];
};

__device__ __forceinline__ SideB sideb_zero() {
  SideB b;
  b.rho = b.E = b.cl = 0.0;
  b.u[0] = b.u[1] = 0.0;
  b.sig[0] = b.sig[1] = b.sig[2] = 0.0;
  return b;
}

// adjoint of side_state<2,2,false,DIR>(W)
template <int DIR>
__device__ __forceinline__ void side_bwd(const Params& P, const double* W, const SideB& Sb, double* Wb, PBar& pb,
                                         bool own) {
  using L = L2;
  const double phi[2] = {W[0], 1.0 - W[0]};
  double rho[2], irho[2];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    rho[l] = W[L::M0 + l];
    irho[l] = 1.0 / rho[l];
  }
  double H[6], J2;
  strain<2, 2, false>(W + L::V0, H, J2);
  EosV e[2];
#pragma unroll
  for (int l = 0; l < 2; ++l) e[l] = eos_eval(P.mat[l], rho[l], irho[l], J2);
  const double p = W[L::E];
  double rhoe = 0.0, rhom = 0.0, xi = 0.0, gnum = 0.0;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    rhoe += phi[l] * ((p - e[l].pref) * e[l].invGam + rho[l] * e[l].eref);
    rhom += phi[l] * rho[l];
    xi += phi[l] * e[l].invGam;
    gnum += phi[l] * e[l].G * e[l].invGam;
  }
  const double irhom = 1.0 / rhom, ixi = 1.0 / xi;
  double cl2[2], cnum = 0.0;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    cl2[l] = c2_mat(e[l], rho[l], irho[l], p);
    cnum += (phi[l] * rho[l] * irhom) * cl2[l] * e[l].invGam;
  }
  const double Gmix = gnum * ixi, c2 = cnum * ixi;
  const double cL2 = c2 + (4.0 / 3.0) * Gmix * irhom;
  const double cl = sqrt(cL2);
  const double u[2] = {W[L::MOM0], W[L::MOM0 + 1]};
  const double uu = u[0] * u[0] + u[1] * u[1];
  // ---- reverse
  double phib[2] = {0.0, 0.0}, rhob[2] = {0.0, 0.0}, irhob[2] = {0.0, 0.0};
  double ub[2] = {Sb.u[0], Sb.u[1]};
  double pbar = 0.0;
  double Hb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  EosB eb[2] = {eosb_zero(), eosb_zero()};
  const double cL2b = Sb.cl * 0.5 / cl;
  double Gmixb = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    Gmixb += 2.0 * Sb.sig[k] * H[hs(k, DIR)];
    Hb[hs(k, DIR)] += 2.0 * Gmix * Sb.sig[k];
  }
  pbar -= Sb.sig[DIR];
  double rhoeb = Sb.E;
  double rhomb = 0.5 * Sb.E * uu + Sb.rho;
#pragma unroll
  for (int k = 0; k < 2; ++k) ub[k] += Sb.E * rhom * u[k];
  const double c2b = cL2b;
  Gmixb += cL2b * (4.0 / 3.0) * irhom;
  double irhomb = cL2b * (4.0 / 3.0) * Gmix;
  const double cnumb = c2b * ixi;
  const double gnumb = Gmixb * ixi;
  const double ixib = c2b * cnum + Gmixb * gnum;
  const double xib = -ixib * ixi * ixi;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    const double g = e[l].invGam;
    const double w = phi[l] * rho[l] * irhom;
    phib[l] += cnumb * rho[l] * irhom * cl2[l] * g;
    rhob[l] += cnumb * phi[l] * irhom * cl2[l] * g;
    irhomb += cnumb * phi[l] * rho[l] * cl2[l] * g;
    eb[l].invGam += cnumb * w * cl2[l];
    c2mat_bwd(e[l], rho[l], irho[l], p, cnumb * w * g, eb[l], rhob[l], irhob[l], pbar);
    phib[l] += gnumb * e[l].G * g;
    eb[l].G += gnumb * phi[l] * g;
    eb[l].invGam += gnumb * phi[l] * e[l].G;
    phib[l] += xib * g;
    eb[l].invGam += xib * phi[l];
  }
  rhomb -= irhomb * irhom * irhom;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    const double g = e[l].invGam;
    phib[l] += rhomb * rho[l];
    rhob[l] += rhomb * phi[l];
    phib[l] += rhoeb * ((p - e[l].pref) * g + rho[l] * e[l].eref);
    pbar += rhoeb * phi[l] * g;
    eb[l].pref -= rhoeb * phi[l] * g;
    eb[l].invGam += rhoeb * phi[l] * (p - e[l].pref);
    rhob[l] += rhoeb * phi[l] * e[l].eref;
    eb[l].eref += rhoeb * phi[l] * rho[l];
  }
  double J2b = 0.0;
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    eos_bwd(P.mat[l], l, rho[l], irho[l], J2, eb[l], rhob[l], irhob[l], J2b, pb, own);
    rhob[l] -= irhob[l] * irho[l] * irho[l];
  }
  double Vb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  strain_bwd(W + L::V0, Hb, J2b, Vb);
  Wb[0] += phib[0] - phib[1];
#pragma unroll
  for (int l = 0; l < 2; ++l) Wb[L::M0 + l] += rhob[l];
#pragma unroll
  for (int k = 0; k < 2; ++k) Wb[L::MOM0 + k] += ub[k];
  Wb[L::E] += pbar;
#pragma unroll
  for (int q = 0; q < 5; ++q) Wb[L::V0 + q] += Vb[q];
}

struct FaceB {
  double F[F2];
  double ustar;
  double Vn[2];
};

// adjoint of star_flux<2,2,false,DIR>: accumulates the bars of W_K (phi,
// densities, stretch tensor), of the side S_K, and of SK, a, inv, ust, mK
template <int DIR>
__device__ __forceinline__ void star_bwd(const double* W, const Side<2, 2, false>& S, double SK, double a,
                                         double inv, const double ust[2], double mK, const FaceB& Ob, double* Wb,
                                         SideB& Sb, double& SKb, double& ab, double& invb, double ustb[2],
                                         double& mKb) {
  using L = L2;
  const double un = S.u[DIR];
  const double r = a * inv;
  const double rm1 = r - 1.0;
  const double usf = un + SK * rm1;
  const double phiN = 1.0 - W[0];
  const double m0 = W[0] * W[L::M0], m1 = phiN * W[L::M0 + 1];
  const double rs = r * S.rho;
  double usK = 0.0, usS = 0.0, sst[2], mom[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    mom[k] = S.rho * S.u[k];
    sst[k] = S.sig[k] - mK * (ust[k] - S.u[k]);
    usK += S.u[k] * S.sig[k];
    usS += ust[k] * sst[k];
  }
  const double Es = (S.E * a + (usK - usS)) * inv;
  // ---- reverse
  double usfb = Ob.ustar + Ob.F[0] * W[0] + Ob.F[L::M0] * m0 + Ob.F[L::M0 + 1] * m1;
  Wb[0] += Ob.F[0] * usf;
  const double m0b = Ob.F[L::M0] * usf, m1b = Ob.F[L::M0 + 1] * usf;
  Wb[0] += m0b * W[L::M0] - m1b * W[L::M0 + 1];
  Wb[L::M0] += m0b * W[0];
  Wb[L::M0 + 1] += m1b * phiN;
  double unb = 0.0, rsb = 0.0, rb = 0.0;
  double usKb = 0.0, usSb = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double Fb = Ob.F[L::MOM0 + k];
    const double momb = Fb * (un - SK);
    unb += Fb * mom[k];
    Sb.sig[k] -= Fb;
    SKb += Fb * (rs * ust[k] - mom[k]);
    rsb += Fb * SK * ust[k];
    ustb[k] += Fb * SK * rs;
    Sb.rho += momb * S.u[k];
    Sb.u[k] += momb * S.rho;
  }
  {
    const double Fb = Ob.F[L::E];
    Sb.E += Fb * (un - SK);
    unb += Fb * S.E;
    usKb -= Fb;
    SKb += Fb * (Es - S.E);
    const double Esb = Fb * SK;
    Sb.E += Esb * a * inv;
    ab += Esb * S.E * inv;
    usKb += Esb * inv;
    usSb -= Esb * inv;
    invb += Esb * (S.E * a + (usK - usS));
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    Sb.u[k] += usKb * S.sig[k];
    Sb.sig[k] += usKb * S.u[k];
    ustb[k] += usSb * sst[k];
    const double sstb = usSb * ust[k];
    Sb.sig[k] += sstb;
    mKb -= sstb * (ust[k] - S.u[k]);
    ustb[k] -= sstb * mK;
    Sb.u[k] += sstb * mK;
  }
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    const double V = W[L::V0 + q];
    const bool coupled = (i < 2) && (L::vq(DIR, j) >= 0);
    const int qn = coupled ? L::vq(DIR, j) : 0;
    const double Vn = coupled ? W[L::V0 + qn] : 0.0;
    const int ii = i < 2 ? i : 0;
    const double Fb = Ob.F[L::V0 + q];
    Wb[L::V0 + q] += Fb * un;
    unb += Fb * V;
    if (coupled) {
      Wb[L::V0 + qn] -= Fb * S.u[ii];
      Sb.u[ii] -= Fb * Vn;
    }
    if (i != DIR) {
      double Vs = a * V;
      if (coupled) Vs -= Vn * (ust[ii] - S.u[ii]);
      SKb += Fb * (Vs * inv - V);
      const double Vsb = Fb * SK * inv;
      invb += Fb * SK * Vs;
      Wb[L::V0 + q] -= Fb * SK;
      ab += Vsb * V;
      Wb[L::V0 + q] += Vsb * a;
      if (coupled) {
        Wb[L::V0 + qn] -= Vsb * (ust[ii] - S.u[ii]);
        ustb[ii] -= Vsb * Vn;
        Sb.u[ii] += Vsb * Vn;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int qn = L::vq(DIR, j);
    if (qn >= 0) Wb[L::V0 + (qn >= 0 ? qn : 0)] += Ob.Vn[j];
  }
  unb += usfb;
  SKb += usfb * rm1;
  rb += usfb * SK;
  rb += rsb * S.rho;
  Sb.rho += rsb * r;
  ab += rb * inv;
  invb += rb * a;
  Sb.u[DIR] += unb;
}

// Adjoint of face_flux<2,2,false,DIR>(WLf, WRf): accumulates the bars of the
// left and right states.
template <int DIR>
__device__ __forceinline__ void face_bwd(const Params& P, const double* WLf, const double* WRf, const FaceB& Ob,
                                         double* WLb, double* WRb, PBar& pb, bool own) {
  using SD = Side<2, 2, false>;
  SD A, B;
  side_state<2, 2, false, DIR>(P, WLf, A);
  side_state<2, 2, false, DIR>(P, WRf, B);
  const double uL = A.u[DIR], uR = B.u[DIR];
  const double SL = fmin(uL - A.cl, uR - B.cl);
  const double SR = fmax(uL + A.cl, uR + B.cl);
  const double mL = A.rho * (SL - uL);
  const double mR = B.rho * (SR - uR);
  const double iden = 1.0 / (mL - mR);
  double ust[2], unum[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    unum[k] = (A.sig[k] - B.sig[k]) + (mL * A.u[k] - mR * B.u[k]);
    ust[k] = unum[k] * frcp(mL - mR);
  }
  const double Sst = ust[DIR];
  const bool supL = SL >= 0.0, supR = SR <= 0.0;
  const bool sup = supL || supR;
  const bool left = supL || (!supR && Sst > 0.0);
  const bool tie = !sup && (Sst == 0.0);
  SideB Ab = sideb_zero(), Bb = sideb_zero();
  double SLb = 0.0, SRb = 0.0, mLb = 0.0, mRb = 0.0, ustb[2] = {0.0, 0.0};
  if (!tie) {
    const SD& SK = left ? A : B;
    const double* WK = left ? WLf : WRf;
    double* WKb = left ? WLb : WRb;
    SideB& SKbar = left ? Ab : Bb;
    const double S_K = left ? SL : SR;
    const double m_K = left ? mL : mR;
    const double a = sup ? 1.0 : S_K - SK.u[DIR];
    const double inv = sup ? 1.0 : 1.0 / (S_K - Sst);
    double SKb = 0.0, abar = 0.0, invb = 0.0, mKb = 0.0;
    star_bwd<DIR>(WK, SK, sup ? 0.0 : S_K, a, inv, ust, m_K, Ob, WKb, SKbar, SKb, abar, invb, ustb, mKb);
    if (!sup) {
      // a = S_K - u_K,n ; inv = 1/(S_K - S*)
      double S_Kb = SKb + abar - invb * inv * inv;
      SKbar.u[DIR] -= abar;
      ustb[DIR] += invb * inv * inv;
      if (left) {
        SLb += S_Kb;
        mLb += mKb;
      } else {
        SRb += S_Kb;
        mRb += mKb;
      }
    }
  } else {
    FaceB half;
#pragma unroll
    for (int f = 0; f < F2; ++f) half.F[f] = 0.5 * Ob.F[f];
    half.ustar = 0.5 * Ob.ustar;
    half.Vn[0] = 0.5 * Ob.Vn[0];
    half.Vn[1] = 0.5 * Ob.Vn[1];
    {
      const double a = SR - B.u[DIR], inv = 1.0 / (SR - Sst);
      double SKb = 0.0, abar = 0.0, invb = 0.0, mKb = 0.0;
      star_bwd<DIR>(WRf, B, SR, a, inv, ust, mR, half, WRb, Bb, SKb, abar, invb, ustb, mKb);
      SRb += SKb + abar - invb * inv * inv;
      Bb.u[DIR] -= abar;
      ustb[DIR] += invb * inv * inv;
      mRb += mKb;
    }
    {
      const double a = SL - A.u[DIR], inv = 1.0 / (SL - Sst);
      double SKb = 0.0, abar = 0.0, invb = 0.0, mKb = 0.0;
      star_bwd<DIR>(WLf, A, SL, a, inv, ust, mL, half, WLb, Ab, SKb, abar, invb, ustb, mKb);
      SLb += SKb + abar - invb * inv * inv;
      Ab.u[DIR] -= abar;
      ustb[DIR] += invb * inv * inv;
      mLb += mKb;
    }
  }
  // ust_k = unum_k / (mL - mR)
  double idenb = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    Ab.sig[k] += ustb[k] * iden;
    Bb.sig[k] -= ustb[k] * iden;
    mLb += ustb[k] * A.u[k] * iden;
    Ab.u[k] += ustb[k] * mL * iden;
    mRb -= ustb[k] * B.u[k] * iden;
    Bb.u[k] -= ustb[k] * mR * iden;
    idenb += ustb[k] * unum[k];
  }
  mLb -= idenb * iden * iden;
  mRb += idenb * iden * iden;
  // mL = rhoL (SL - uL), mR = rhoR (SR - uR)
  Ab.rho += mLb * (SL - uL);
  SLb += mLb * A.rho;
  Ab.u[DIR] -= mLb * A.rho;
  Bb.rho += mRb * (SR - uR);
  SRb += mRb * B.rho;
  Bb.u[DIR] -= mRb * B.rho;
  // SL = min(uL - clL, uR - clR), SR = max(uL + clL, uR + clR)
  if (uL - A.cl <= uR - B.cl) {
    Ab.u[DIR] += SLb;
    Ab.cl -= SLb;
  } else {
    Bb.u[DIR] += SLb;
    Bb.cl -= SLb;
  }
  if (uL + A.cl >= uR + B.cl) {
    Ab.u[DIR] += SRb;
    Ab.cl += SRb;
  } else {
    Bb.u[DIR] += SRb;
    Bb.cl += SRb;
  }
  side_bwd<DIR>(P, WLf, Ab, WLb, pb, own);
  side_bwd<DIR>(P, WRf, Bb, WRb, pb, own);
}

// ------------------------------------------------------------------ update
// adjoint of update_cell<2,2,false,DIR>: lam = bar of Un.  Accumulates the
// bars of U, inv_rho and of both faces.
__device__ __forceinline__ void update_bwd(const double* U, double inv_rho, const FaceV<2, 2, false>& a,
                                           const FaceV<2, 2, false>& b, double nu, const double* lam, double* Ub,
                                           double& irb, FaceB& ab, FaceB& bb) {
  using L = L2;
  const double du = b.ustar - a.ustar;
  double dub = 0.0;
  Ub[0] += lam[0] * (1.0 + nu * du);
  bb.F[0] -= nu * lam[0];
  ab.F[0] += nu * lam[0];
  dub += nu * lam[0] * U[0];
#pragma unroll
  for (int f = 1; f < L::V0; ++f) {
    Ub[f] += lam[f];
    bb.F[f] -= nu * lam[f];
    ab.F[f] += nu * lam[f];
  }
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    const double lv = lam[L::V0 + q];
    Ub[L::V0 + q] += lv;
    bb.F[L::V0 + q] -= nu * lv;
    ab.F[L::V0 + q] += nu * lv;
    const double srcb = nu * lv;
    Ub[L::V0 + q] += srcb * (2.0 / 3.0) * du;
    dub += srcb * (2.0 / 3.0) * U[L::V0 + q];
    if (i < 2 && j < 2) {
      const int ii = i < 2 ? i : 0, jj = j < 2 ? j : 0;
      const double dv = b.Vn[jj] - a.Vn[jj];
      const double t = U[L::MOM0 + ii] * inv_rho;
      Ub[L::MOM0 + ii] -= srcb * inv_rho * dv;
      irb -= srcb * U[L::MOM0 + ii] * dv;
      bb.Vn[jj] -= srcb * t;
      ab.Vn[jj] += srcb * t;
    }
  }
  bb.ustar += dub;
  ab.ustar -= dub;
}

// ----------------------------------------------------------------- plastic
// Adjoint of the plastic relaxation of the non-reactive epilogue at the
// pre-relaxation state U.  lam: bar of the relaxed state; Ub receives the
// bar of U (every field: the untouched fields pass their bar through).
__device__ __forceinline__ void plastic_bwd(const Params& P, const double* U, const double* lam, double* Ub,
                                            PBar& pb, bool own) {
  using L = L2;
#pragma unroll
  for (int f = 0; f < L::V0; ++f) Ub[f] = lam[f];
#pragma unroll
  for (int q = 0; q < L::NV; ++q) Ub[L::V0 + q] = 0.0;
  const double phi[2] = {U[0], 1.0 - U[0]};
  const double m[2] = {U[L::M0], U[L::M0 + 1]};
  double rho[2];
#pragma unroll
  for (int l = 0; l < 2; ++l) rho[l] = m[l] / phi[l];
  double H[6], J2;
  strain<2, 2, false>(U + L::V0, H, J2);
  const double J = sqrt(J2);
  double xi = 0.0, num = 0.0, wsh = 0.0, Jl[2] = {0.0, 0.0}, Gl[2] = {0.0, 0.0};
  bool yl[2] = {false, false};
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    const MatP& mt = P.mat[l];
    const double wl = phi[l] * mt.invGam;
    xi += wl;
    if (!mt.shear) continue;
    Jl[l] = J;
    if (mt.plast == PLAST_PERFECT) {
      Gl[l] = shear_modulus(mt, rho[l]);
      const double Jy = mt.yield_s6 * (1.0 / Gl[l]);
      if (!(J <= Jy)) {
        Jl[l] = Jy;
        yl[l] = true;
      }
    }
    num += wl * Jl[l];
    wsh += wl;
  }
  const bool pos = J > 0.0;
  const double fac = pos ? (num / xi) / J : wsh / xi;  // J = 0: the limit of num/(xi J)
  // full 3x3 forms of Mm = I - fac H / 2, Mp = I + fac H / 2
  double Hf[3][3], Mm[3][3], Mp[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Hf[i][j] = H[hs(i, j)];
      const double id = (i == j) ? 1.0 : 0.0;
      Mm[i][j] = id - 0.5 * fac * Hf[i][j];
      Mp[i][j] = id + 0.5 * fac * Hf[i][j];
    }
  double A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      A[i][j] = Mm[(j + 1) % 3][(i + 1) % 3] * Mm[(j + 2) % 3][(i + 2) % 3] -
                Mm[(j + 1) % 3][(i + 2) % 3] * Mm[(j + 2) % 3][(i + 1) % 3];
  const double det = Mm[0][0] * A[0][0] + Mm[0][1] * A[1][0] + Mm[0][2] * A[2][0];
  const double idet = 1.0 / det;
  double X[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) s += A[i][k] * Mp[k][j];
      X[i][j] = s;
    }
  // ---- reverse: Vnew(i,j) = X(i,j)/det on the stored slots
  double Xb[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Xb[i][j] = 0.0;
  double detb = 0.0;
#pragma unroll
  for (int q = 0; q < L::NV; ++q) {
    const int i = L::vi(q), j = L::vj(q);
    Xb[i][j] += lam[L::V0 + q] * idet;
    detb -= lam[L::V0 + q] * X[i][j] * idet * idet;
  }
  double Ab[3][3], Mpb[3][3], Mmb[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double sa = 0.0, sp = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sa += Xb[i][k] * Mp[j][k];
        sp += A[k][i] * Xb[k][j];
      }
      Ab[i][j] = sa;
      Mpb[i][j] = sp;
      Mmb[i][j] = 0.0;
    }
  // det: d det / d Mm(i,j) = A(j,i)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Mmb[i][j] += detb * A[j][i];
  // adjugate by cyclic cofactors
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int r1 = (j + 1) % 3, r2 = (j + 2) % 3, c1 = (i + 1) % 3, c2 = (i + 2) % 3;
      const double g = Ab[i][j];
      Mmb[r1][c1] += g * Mm[r2][c2];
      Mmb[r2][c2] += g * Mm[r1][c1];
      Mmb[r1][c2] -= g * Mm[r2][c1];
      Mmb[r2][c1] -= g * Mm[r1][c2];
    }
  // Mm = I - fac Hf/2, Mp = I + fac Hf/2 (Hf symmetric in the slots of H)
  double Hb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double facb = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double hb = 0.5 * (Mpb[i][j] - Mmb[i][j]);
      Hb[hs(i, j)] += hb * fac;
      facb += hb * Hf[i][j];
    }
  double J2b = 0.0;
  double phib[2] = {0.0, 0.0}, rhob[2] = {0.0, 0.0};
  if (pos) {
    // fac = num / (xi J)
    const double numb = facb / (xi * J);
    const double xib = -facb * fac / xi;
    double Jb = -facb * fac / J;
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const MatP& mt = P.mat[l];
      phib[l] += xib * mt.invGam;
      pacc(pb.v[l][PB_IGAM], own, xib * phi[l]);
      if (!mt.shear) continue;
      const double wl = phi[l] * mt.invGam;
      const double wlb = numb * Jl[l];
      phib[l] += wlb * mt.invGam;
      pacc(pb.v[l][PB_IGAM], own, wlb * phi[l]);
      const double Jlb = numb * wl;
      if (yl[l]) {
        // Jl = Y6 / G_l
        pacc(pb.v[l][PB_Y], own, Jlb / Gl[l]);
        const double Gb = -Jlb * Jl[l] / Gl[l];
        shear_bwd(mt, l, rho[l], Gb, rhob[l], pb, own);
      } else {
        Jb += Jlb;
      }
    }
    J2b += Jb * 0.5 / J;
  }
  double Vb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  strain_bwd(U + L::V0, Hb, J2b, Vb);
#pragma unroll
  for (int q = 0; q < 5; ++q) Ub[L::V0 + q] += Vb[q];
  // rho_l = m_l / phi_l
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    Ub[L::M0 + l] += rhob[l] / phi[l];
    phib[l] -= rhob[l] * rho[l] / phi[l];
  }
  Ub[0] += phib[0] - phib[1];
}

}  // namespace adj
}  // namespace dimp
