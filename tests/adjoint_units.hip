// Test library: each hand-written reverse stage of the adjoint against central
// differences of its own forward stage, case by case on the GPU.  For a case
// with input x, direction v and output weights w it returns
//   fd  = <w, (f(x + eps v) - f(x - eps v)) / (2 eps)>   (forward stage)
//   adj = <f^T w, v>                                      (reverse stage)
// Parameters are packed here from the public material/option structs, the
// same way the library packs them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../include/dimp.h"
#include "dimp_adjoint.hpp"

using namespace dimp;
using adj::F2;

namespace {

MatP pack(const dimp_material& m) {
  MatP q;
  std::memset(&q, 0, sizeof q);
  q.eos = m.eos;
  q.plast = m.plast;
  q.cv = m.cv;
  if (m.eos == DIMP_EOS_ROMENSKII) {
    q.Gam = m.Gamma0;
    q.inv_rho0 = 1.0 / m.rho0;
    q.abar = m.abar;
    q.bbar = m.bbar;
    q.K0a = m.K0 / m.abar;
    q.ec_coef = m.K0 / (2.0 * m.rho0 * m.abar * m.abar);
    q.dpc_coef = m.K0 / (m.abar * m.rho0);
    q.G0 = m.G0;
    q.abar_one = (m.abar == 1.0);
    q.bbar_three = (m.bbar == 3.0);
    q.shear = (m.G0 > 0.0);
    q.yield_s6 = m.yield / std::sqrt(6.0);
  } else {
    q.Gam = m.gamma - 1.0;
    q.pref0 = (m.eos == DIMP_EOS_STIFFENED) ? -m.gamma * m.pinf : 0.0;
    q.eref0 = (m.eos == DIMP_EOS_STIFFENED) ? m.eref : 0.0;
  }
  q.invGam = 1.0 / q.Gam;
  return q;
}

Params make_params(const dimp_material* mats, const dimp_options* o, const double* dx) {
  Params P;
  std::memset(&P, 0, sizeof P);
  for (int d = 0; d < 3; ++d) {
    P.n[d] = 1;
    P.dx[d] = d < 2 ? dx[d] : 1.0;
  }
  P.ncell = 1;
  P.limiter = o->limiter;
  P.thinc = o->thinc;
  P.beta0 = o->beta0;
  P.delta = o->delta;
  P.eps = o->eps;
  for (int i = 0; i < 6; ++i) {
    const double e = 1e-6 * o->va_scale[i];
    P.va_e2[i] = e * e;
  }
  for (int l = 0; l < 2; ++l) {
    P.mat[l] = pack(mats[l]);
    if (P.mat[l].shear) P.any_shear = 1;
  }
  P.rx.mat = -1;
  return P;
}

struct FaceIO {
  __device__ static void put(const FaceV<2, 2, false>& f, double* y) {
    for (int k = 0; k < F2; ++k) y[k] = f.F[k];
    y[F2] = f.ustar;
    y[F2 + 1] = f.Vn[0];
    y[F2 + 2] = f.Vn[1];
  }
  __device__ static void get(const double* y, FaceV<2, 2, false>& f) {
    for (int k = 0; k < F2; ++k) f.F[k] = y[k];
    f.ustar = y[F2];
    f.Vn[0] = y[F2 + 1];
    f.Vn[1] = y[F2 + 2];
  }
  __device__ static adj::FaceB bar(const double* y) {
    adj::FaceB b;
    for (int k = 0; k < F2; ++k) b.F[k] = y[k];
    b.ustar = y[F2];
    b.Vn[0] = y[F2 + 1];
    b.Vn[1] = y[F2 + 2];
    return b;
  }
};

// ------------------------------------------------------------- the stages
struct StC2P {
  static constexpr int NI = F2, NO = F2 + 2;
  __device__ static void fwd(const Params& P, double, const double* x, double* y) {
    Thermo<2, false> T;
    double H[6], J2;
    cons_to_prim<2, 2, false>(P, x, y, T, H, J2);
    y[F2] = T.irho;
    y[F2 + 1] = T.rho * T.c2;
  }
  __device__ static void bwd(const Params& P, double, const double* x, const double* yb, double* xb) {
    adj::PBar pb;
    adj::pbar_zero(pb);
    adj::c2p_bwd(P, x, yb, yb[F2], yb[F2 + 1], xb, pb, true);
  }
};

template <int DIR>
struct StSide {
  static constexpr int NI = F2, NO = 8;
  __device__ static void fwd(const Params& P, double, const double* x, double* y) {
    Side<2, 2, false> S;
    side_state<2, 2, false, DIR>(P, x, S);
    y[0] = S.rho; y[1] = S.E; y[2] = S.cl; y[3] = S.u[0]; y[4] = S.u[1];
    y[5] = S.sig[0]; y[6] = S.sig[1]; y[7] = S.sig[2];
  }
  __device__ static void bwd(const Params& P, double, const double* x, const double* yb, double* xb) {
    adj::PBar pb;
    adj::pbar_zero(pb);
    adj::SideB b;
    b.rho = yb[0]; b.E = yb[1]; b.cl = yb[2]; b.u[0] = yb[3]; b.u[1] = yb[4];
    b.sig[0] = yb[5]; b.sig[1] = yb[6]; b.sig[2] = yb[7];
    adj::side_bwd<DIR>(P, x, b, xb, pb, true);
  }
};

template <int DIR>
struct StStress {
  static constexpr int NI = F2, NO = 3;
  __device__ static void fwd(const Params& P, double, const double* x, double* y) {
    stress_col<2, 2, false, DIR>(P, x, y);
  }
  __device__ static void bwd(const Params& P, double, const double* x, const double* yb, double* xb) {
    adj::PBar pb;
    adj::pbar_zero(pb);
    adj::stress_bwd<DIR>(P, x, yb, xb, pb, true);
  }
};

template <int DIR>
struct StFace {
  static constexpr int NI = 2 * F2, NO = F2 + 3;
  __device__ static void fwd(const Params& P, double, const double* x, double* y) {
    FaceV<2, 2, false> f;
    face_flux<2, 2, false, DIR>(P, x, x + F2, f);
    FaceIO::put(f, y);
  }
  __device__ static void bwd(const Params& P, double, const double* x, const double* yb, double* xb) {
    adj::PBar pb;
    adj::pbar_zero(pb);
    adj::face_bwd<DIR>(P, x, x + F2, FaceIO::bar(yb), xb, xb + F2, pb, true);
  }
};

// star flux with given side quantities: x = W(11), side(8), SK, a, inv, ust(2), mK
template <int DIR>
struct StStar {
  static constexpr int NI = F2 + 8 + 6, NO = F2 + 3;
  __device__ static void side(const double* x, Side<2, 2, false>& S) {
    const double* s = x + F2;
    S.rho = s[0]; S.E = s[1]; S.cl = s[2]; S.u[0] = s[3]; S.u[1] = s[4];
    S.sig[0] = s[5]; S.sig[1] = s[6]; S.sig[2] = s[7];
  }
  __device__ static void fwd(const Params& P, double, const double* x, double* y) {
    Side<2, 2, false> S;
    side(x, S);
    const double* r = x + F2 + 8;
    const double ust[2] = {r[3], r[4]};
    FaceV<2, 2, false> f;
    star_flux<2, 2, false, DIR>(P, x, S, r[0], r[1], r[2], ust, r[5], f);
    FaceIO::put(f, y);
  }
  __device__ static void bwd(const Params& P, double, const double* x, const double* yb, double* xb) {
    Side<2, 2, false> S;
    side(x, S);
    const double* r = x + F2 + 8;
    const double ust[2] = {r[3], r[4]};
    adj::SideB Sb = adj::sideb_zero();
    double SKb = 0.0, ab = 0.0, invb = 0.0, ustb[2] = {0.0, 0.0}, mKb = 0.0;
    adj::star_bwd<DIR>(x, S, r[0], r[1], r[2], ust, r[5], FaceIO::bar(yb), xb, Sb, SKb, ab, invb, ustb, mKb);
    double* sb = xb + F2;
    sb[0] += Sb.rho; sb[1] += Sb.E; sb[2] += Sb.cl; sb[3] += Sb.u[0]; sb[4] += Sb.u[1];
    sb[5] += Sb.sig[0]; sb[6] += Sb.sig[1]; sb[7] += Sb.sig[2];
    double* rb = xb + F2 + 8;
    rb[0] += SKb; rb[1] += ab; rb[2] += invb; rb[3] += ustb[0]; rb[4] += ustb[1]; rb[5] += mKb;
  }
};

// edges without THINC: x = Wm, W0, Wp, irho0, rc2
template <int DIR>
struct StEdges {
  static constexpr int NI = 3 * F2 + 2, NO = 2 * F2;
  __device__ static void fwd(const Params& P, double nu, const double* x, double* y) {
    auto nd = []() { return 1.0; };
    const Cand c0 = phi_candidates<2, 2, false>(P, x[0], x[F2], x[2 * F2], nd);
    edges_predict<2, 2, false, DIR>(P, x, x + F2, x + 2 * F2, x[3 * F2], x[3 * F2 + 1], c0, c0, c0, nu, y, y + F2);
  }
  __device__ static void bwd(const Params& P, double nu, const double* x, const double* yb, double* xb) {
    auto nd = []() { return 1.0; };
    const Cand c0 = phi_candidates<2, 2, false>(P, x[0], x[F2], x[2 * F2], nd);
    adj::PBar pb;
    adj::pbar_zero(pb);
    double cb[4];
    adj::edges_bwd<DIR>(P, x, x + F2, x + 2 * F2, x[3 * F2], x[3 * F2 + 1], c0, c0, c0, nu, yb, yb + F2, xb,
                        xb + F2, xb + 2 * F2, xb[3 * F2], xb[3 * F2 + 1], cb, pb, true);
    double st[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, stb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    adj::cand_bwd<DIR>(P, x[0], x[F2], x[2 * F2], st, cb, xb[0], xb[F2], xb[2 * F2], stb);
  }
};

// update: x = U(11), inv_rho, face a (14), face b (14)
template <int DIR>
struct StUpdate {
  static constexpr int NI = F2 + 1 + 2 * (F2 + 3), NO = F2;
  __device__ static void fwd(const Params& P, double nu, const double* x, double* y) {
    FaceV<2, 2, false> a, b;
    FaceIO::get(x + F2 + 1, a);
    FaceIO::get(x + F2 + 1 + F2 + 3, b);
    update_cell<2, 2, false, DIR>(x, x[F2], a, b, nu, y);
  }
  __device__ static void bwd(const Params& P, double nu, const double* x, const double* yb, double* xb) {
    FaceV<2, 2, false> a, b;
    FaceIO::get(x + F2 + 1, a);
    FaceIO::get(x + F2 + 1 + F2 + 3, b);
    adj::FaceB ab, bb;
    for (int k = 0; k < F2; ++k) ab.F[k] = bb.F[k] = 0.0;
    ab.ustar = bb.ustar = 0.0;
    ab.Vn[0] = ab.Vn[1] = bb.Vn[0] = bb.Vn[1] = 0.0;
    adj::update_bwd(x, x[F2], a, b, nu, yb, xb, xb[F2], ab, bb);
    double* pa = xb + F2 + 1;
    double* pbp = pa + F2 + 3;
    for (int k = 0; k < F2; ++k) {
      pa[k] += ab.F[k];
      pbp[k] += bb.F[k];
    }
    pa[F2] += ab.ustar; pa[F2 + 1] += ab.Vn[0]; pa[F2 + 2] += ab.Vn[1];
    pbp[F2] += bb.ustar; pbp[F2 + 1] += bb.Vn[0]; pbp[F2 + 2] += bb.Vn[1];
  }
};

struct StPlastic {
  static constexpr int NI = F2, NO = F2;
  __device__ static void fwd(const Params& P, double, const double* x, double* y) {
    for (int k = 0; k < F2; ++k) y[k] = x[k];
    plastic_cell<2, 2, false>(P, y, 0.0);  // perfect plasticity: instantaneous, no dt
  }
  __device__ static void bwd(const Params& P, double, const double* x, const double* yb, double* xb) {
    adj::PBar pb;
    adj::pbar_zero(pb);
    adj::plastic_bwd(P, x, yb, xb, pb, true);
  }
};

template <class S>
__global__ void k_unit(Params P, double nu, int n, const double* X, const double* V, const double* WY, double eps,
                       double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double x[S::NI], xp[S::NI], xm[S::NI], xb[S::NI], y1[S::NO], y2[S::NO], w[S::NO];
  for (int i = 0; i < S::NI; ++i) {
    x[i] = X[(size_t)c * S::NI + i];
    const double v = V[(size_t)c * S::NI + i];
    xp[i] = x[i] + eps * v;
    xm[i] = x[i] - eps * v;
    xb[i] = 0.0;
  }
  for (int k = 0; k < S::NO; ++k) w[k] = WY[(size_t)c * S::NO + k];
  S::fwd(P, nu, xp, y1);
  S::fwd(P, nu, xm, y2);
  double fd = 0.0;
  for (int k = 0; k < S::NO; ++k) fd += w[k] * (y1[k] - y2[k]);
  fd /= 2.0 * eps;
  S::bwd(P, nu, x, w, xb);
  double ad = 0.0;
  for (int i = 0; i < S::NI; ++i) ad += xb[i] * V[(size_t)c * S::NI + i];
  out[2 * c] = fd;
  out[2 * c + 1] = ad;
}

template <class S>
int run(const Params& P, double nu, int n, const double* X, const double* V, const double* WY, double eps,
        double* out) {
  double *dX = nullptr, *dV = nullptr, *dW = nullptr, *dO = nullptr;
  const size_t ni = (size_t)n * S::NI * sizeof(double), no = (size_t)n * S::NO * sizeof(double);
  if (hipMalloc(&dX, ni) || hipMalloc(&dV, ni) || hipMalloc(&dW, no) || hipMalloc(&dO, 2 * n * sizeof(double)))
    return 1;
  hipMemcpy(dX, X, ni, hipMemcpyHostToDevice);
  hipMemcpy(dV, V, ni, hipMemcpyHostToDevice);
  hipMemcpy(dW, WY, no, hipMemcpyHostToDevice);
  hipLaunchKernelGGL(k_unit<S>, dim3((n + 63) / 64), dim3(64), 0, 0, P, nu, n, dX, dV, dW, eps, dO);
  int rc = hipDeviceSynchronize() != hipSuccess;
  hipMemcpy(out, dO, 2 * n * sizeof(double), hipMemcpyDeviceToHost);
  hipFree(dX);
  hipFree(dV);
  hipFree(dW);
  hipFree(dO);
  return rc;
}

}  // namespace

extern "C" {

// sizes (inputs, outputs) of a stage; -1 for an unknown stage
int unit_sizes(int stage, int* ni, int* no) {
  switch (stage) {
    case 0: *ni = StC2P::NI; *no = StC2P::NO; return 0;
    case 1: *ni = StSide<0>::NI; *no = StSide<0>::NO; return 0;
    case 2: *ni = StStress<0>::NI; *no = StStress<0>::NO; return 0;
    case 3: *ni = StFace<0>::NI; *no = StFace<0>::NO; return 0;
    case 4: *ni = StStar<0>::NI; *no = StStar<0>::NO; return 0;
    case 5: *ni = StEdges<0>::NI; *no = StEdges<0>::NO; return 0;
    case 6: *ni = StUpdate<0>::NI; *no = StUpdate<0>::NO; return 0;
    case 7: *ni = StPlastic::NI; *no = StPlastic::NO; return 0;
  }
  return -1;
}

// run stage (0 c2p, 1 side, 2 stress, 3 face, 4 star, 5 edges, 6 update,
// 7 plastic) along dir on n host cases; out[2c] = fd, out[2c+1] = adjoint
int unit_run(int stage, int dir, const dimp_material* mats, const dimp_options* opt, const double* dx, double nu,
             int n, const double* X, const double* V, const double* WY, double eps, double* out) {
  const Params P = make_params(mats, opt, dx);
#define DIMP_UNIT(S0, S1) return dir == 0 ? run<S0>(P, nu, n, X, V, WY, eps, out) : run<S1>(P, nu, n, X, V, WY, eps, out)
  switch (stage) {
    case 0: DIMP_UNIT(StC2P, StC2P);
    case 1: DIMP_UNIT(StSide<0>, StSide<1>);
    case 2: DIMP_UNIT(StStress<0>, StStress<1>);
    case 3: DIMP_UNIT(StFace<0>, StFace<1>);
    case 4: DIMP_UNIT(StStar<0>, StStar<1>);
    case 5: DIMP_UNIT(StEdges<0>, StEdges<1>);
    case 6: DIMP_UNIT(StUpdate<0>, StUpdate<1>);
    case 7: DIMP_UNIT(StPlastic, StPlastic);
  }
#undef DIMP_UNIT
  return -1;
}

}  // extern "C"
