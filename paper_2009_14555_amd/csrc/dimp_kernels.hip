// dimp_kernels.hip -- gfx950 kernels of the split diffuse-interface step:
// the 1-D and 2-D sweeps (instantiated from dimp_sweeps.hpp; the 3-D ones
// live in dimp_sweeps3.hip) and the pointwise kernels (primitive <->
// conserved, sources, wave speed, state check, the CFL step).
#include <hip/hip_runtime.h>

#include "dimp_sweeps.hpp"

namespace dimp {

// ------------------------------------------------------ pointwise kernels
template <int D, int N, int RX>
__global__ __launch_bounds__(256) void k_prim_to_cons(Params P, const double* __restrict__ W, double* __restrict__ U) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  const int64_t nc = P.ncell;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double w[F];
#pragma unroll
    for (int f = 0; f < F; ++f) w[f] = W[f * nc + c];
    Thermo<N, RX> T;
    double H[6], J2;
    prim_thermo<D, N, RX>(P, w, T, H, J2, true);
    double phiN = 1.0;
#pragma unroll
    for (int l = 0; l < N - 1; ++l) {
      U[l * nc + c] = w[l];
      phiN -= w[l];
    }
#pragma unroll
    for (int l = 0; l < N; ++l) U[(L::M0 + l) * nc + c] = (l < N - 1 ? w[l] : phiN) * w[L::M0 + l];
    if (RX) {
      const int y = P.rx.mat;
      double py = phiN, ry = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l)
        if (l == y) {
          py = (l < N - 1) ? w[l] : phiN;
          ry = w[L::M0 + l];
        }
      U[L::LAM * nc + c] = py * ry * (P.rx.kind == RXK_MIX ? fmin(fmax(w[L::LAM], 0.0), 1.0) : w[L::LAM]);
    }
    double uu = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      U[(L::MOM0 + k) * nc + c] = T.rho * w[L::MOM0 + k];
      uu += w[L::MOM0 + k] * w[L::MOM0 + k];
    }
    U[L::E * nc + c] = T.rhoe + 0.5 * T.rho * uu;
#pragma unroll
    for (int q = 0; q < L::NV; ++q) U[(L::V0 + q) * nc + c] = w[L::V0 + q];
  }
}

template <int D, int N, int RX>
__global__ __launch_bounds__(256) void k_cons_to_prim(Params P, const double* __restrict__ U, double* __restrict__ W) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  const int64_t nc = P.ncell;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double u[F], w[F];
#pragma unroll
    for (int f = 0; f < F; ++f) u[f] = U[f * nc + c];
    Thermo<N, RX> T;
    double H[6], J2;
    cons_to_prim<D, N, RX>(P, u, w, T, H, J2);
#pragma unroll
    for (int f = 0; f < F; ++f) W[f * nc + c] = w[f];
  }
}

template <int D, int N, int RX>
__global__ __launch_bounds__(256) void k_sources(Params P, double* __restrict__ U, double dt_arg,
                                                const double* __restrict__ dtp) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  const int64_t nc = P.ncell;
  const double dt = dtp ? dtp[0] : dt_arg;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double u[F];
#pragma unroll
    for (int f = 0; f < F; ++f) u[f] = U[f * nc + c];
    plastic_cell<D, N, RX>(P, u, dt);
    reaction_cell<D, N, RX>(P, u, dt);
    if (D == 2 && P.geom) geom_cell<D, N, RX>(P, u, P.r_lo + ((double)(c % P.n[0]) + 0.5) * P.dx[0], dt);
#pragma unroll
    for (int f = 0; f < F; ++f) U[f * nc + c] = u[f];
  }
}

template <int D, int N, int RX>
__global__ __launch_bounds__(256) void k_wavespeed(Params P, const double* __restrict__ U,
                                                   unsigned long long* __restrict__ smax) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  const int64_t nc = P.ncell;
  double s[D];
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double u[F], sc[D];
#pragma unroll
    for (int f = 0; f < F; ++f) u[f] = U[f * nc + c];
    wavespeed_cell<D, N, RX>(P, u, sc);
#pragma unroll
    for (int k = 0; k < D; ++k) s[k] = (sc[k] > s[k] || sc[k] != sc[k]) ? sc[k] : s[k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) wave_max_atomic(s[k], smax + k);
}

template <int D, int N, int RX>
__global__ __launch_bounds__(256) void k_check(Params P, const double* __restrict__ U,
                                               unsigned long long* __restrict__ nbad) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  const int64_t nc = P.ncell;
  unsigned long long bad = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double u[F], w[F];
    bool ok = true;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      u[f] = U[f * nc + c];
      ok = ok && isfinite(u[f]);
    }
    if (ok) {
      Thermo<N, RX> T;
      double H[6], J2;
      cons_to_prim<D, N, RX>(P, u, w, T, H, J2);
      double sphi = 0.0;
#pragma unroll
      for (int l = 0; l < N - 1; ++l) {
        ok = ok && (w[l] >= 0.0) && (w[l] <= 1.0);
        sphi += w[l];
      }
      ok = ok && (sphi <= 1.0);
#pragma unroll
      for (int l = 0; l < N; ++l) ok = ok && (w[L::M0 + l] > 0.0);
      ok = ok && (T.c2 > 0.0) && isfinite(T.p);
    }
    bad += ok ? 0 : 1;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(nbad, bad);
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void k_u64_to_f64(const unsigned long long* p, double* out, int n) {
  const int i = threadIdx.x;
  if (i < n) out[i] = __longlong_as_double((long long)p[i]);
}

// CFL time step from the per-direction max wave speed (bit patterns):
// dt = cfl * min_d dx_d / smax_d; also appended to a caller log if given.  A
// step that is not finite and positive (a zero or NaN wave speed) is replaced
// by dt = 0 and flagged in the status word smax[5], which the state check
// reports.
__device__ __forceinline__ void cfl_dt_from(const double s[3], unsigned long long* smax, double cfl, double dx0,
                                            double dx1, double dx2, int D, double* dt, double* log, int64_t idx) {
  const double dxs[3] = {dx0, dx1, dx2};
  double m = 0.0;
  bool first = true;
  for (int d = 0; d < D; ++d) {
    const double v = dxs[d] / s[d];
    m = first ? v : fmin(m, v);
    first = false;
  }
  double r = cfl * m;
  if (!(r > 0.0 && r <= 1.79769313486231570e308)) {
    r = 0.0;
    smax[5] = 1ull;
  }
  dt[0] = r;
  if (log) log[idx] = r;
}

__global__ void k_cfl_dt(unsigned long long* __restrict__ smax, double cfl, double dx0, double dx1, double dx2,
                         int D, double* __restrict__ dt, double* __restrict__ log, int64_t idx) {
  if (threadIdx.x != 0) return;
  double s[3];
  for (int d = 0; d < 3; ++d) s[d] = __longlong_as_double((long long)smax[d]);
  cfl_dt_from(s, smax, cfl, dx0, dx1, dx2, D, dt, log, idx);
}

// Max over the per-wave slots of the last fused sweep, in two fixed-order
// stages (deterministic): block b reduces the contiguous chunk b of the slots
// into out[b]; a single block then reduces those into the wave-speed words
// read by k_cfl_dt and the host query (bit patterns of non-negative doubles;
// a NaN wins) and, when req.dt is set, turns them into the next step's dt by
// the k_cfl_dt rule.  (One launch whose last block, found by a ticket counter,
// does the second stage took 24 us at 2048^2 against 9.5 us for the two:
// 288 returning atomics on one word.)
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

template <bool FINAL>
__global__ __launch_bounds__(256) void k_reduce_smax(const double* __restrict__ part, int64_t nslots, int64_t chunk,
                                                     int D, double* __restrict__ out,
                                                     unsigned long long* __restrict__ smax, DtReq req) {
  __shared__ double red[3][4];
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < nslots ? lo + chunk : nslots;
  double m[3] = {0.0, 0.0, 0.0};
  for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x)
    for (int k = 0; k < D; ++k) m[k] = nanmax(m[k], part[t * 3 + k]);
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m[k] = nanmax(m[k], __shfl_xor(m[k], off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 3; ++k) red[k][w] = m[k];
  __syncthreads();
  if (!FINAL) {
    if (threadIdx.x < 3) {
      const int k = threadIdx.x;
      out[(int64_t)blockIdx.x * 3 + k] = nanmax(nanmax(red[k][0], red[k][1]), nanmax(red[k][2], red[k][3]));
    }
    return;
  }
  if (threadIdx.x == 0) {
    double s[3];
    for (int k = 0; k < 3; ++k) {
      const double v = nanmax(nanmax(red[k][0], red[k][1]), nanmax(red[k][2], red[k][3]));
      s[k] = (k < D) ? v : 0.0;
      smax[k] = (k < D) ? (unsigned long long)__double_as_longlong(v) : 0ull;
    }
    if (req.dt) cfl_dt_from(s, smax, req.cfl, req.dx0, req.dx1, req.dx2, D, req.dt, req.log, req.idx);
  }
}

// ---------------------------------------------------------------- launch
hipError_t launch_sweep(const Params& P, int D, int rx, const double* in, double* out, double dt,
                        const double* dtp, int dir, bool fuse, double* part, int S, hipStream_t st) {
#define DIMP_SWEEP_RX(DD)                                                                  \
  return rx == 2 ? launch_sweep_t<DD, 2, 2>(P, in, out, dt, dtp, dir, fuse, part, S, st)   \
         : rx    ? launch_sweep_t<DD, 2, 1>(P, in, out, dt, dtp, dir, fuse, part, S, st)   \
                 : launch_sweep_t<DD, 2, 0>(P, in, out, dt, dtp, dir, fuse, part, S, st)
  if (P.nmat == 3) return launch_sweep_n3(P, D, rx, in, out, dt, dtp, dir, fuse, part, S, st);
  if (P.nmat != 2) return hipErrorInvalidValue;
  if (D == 1) DIMP_SWEEP_RX(1);
  if (D == 2) DIMP_SWEEP_RX(2);
  return launch_sweep3(P, rx, in, out, dt, dtp, dir, fuse, part, S, st);
#undef DIMP_SWEEP_RX
}

hipError_t launch_rk_sweep(const Params& P, int D, int rx, int dir, int mode, int stage, bool fuse,
                           const double* in, double* out, const double* Rin, const double* qn, double dt,
                           const double* dtp, double* part, hipStream_t st) {
  if (mode < M_RK_FIRST || mode > M_RK_LAST || stage < 1 || stage > 3) return hipErrorInvalidValue;
#define DIMP_RK_RX(DD)                                                                              \
  return rx == 2 ? launch_rk_t<DD, 2, 2>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st)   \
         : rx    ? launch_rk_t<DD, 2, 1>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st)   \
                 : launch_rk_t<DD, 2, 0>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st)
  if (P.nmat == 3) return launch_rk_sweep_n3(P, D, rx, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st);
  if (P.nmat != 2) return hipErrorInvalidValue;
  if (D == 1) DIMP_RK_RX(1);
  if (D == 2) DIMP_RK_RX(2);
  return launch_rk_sweep3(P, rx, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st);
#undef DIMP_RK_RX
}

int64_t sweep_slots(const Params& P, int D, int dir) {
  if (dir == 0) return ((P.n[0] + 57) / 58) * P.n[1] * P.n[2];
  const int oa = (dir == 1) ? 2 : 1;
  const int64_t no = (D == 3) ? P.n[oa] : 1;
  return ((P.n[0] + TILE_COLUMNS - 1) / TILE_COLUMNS) * no * ((P.n[dir] + 57) / 58) * TILE_COLUMNS;
}

hipError_t launch_reduce_smax(const double* part, int64_t nslots, int D, double* scratch,
                              unsigned long long* smax, hipStream_t st, const DtReq* req) {
  const int64_t nb = reduce_smax_blocks(nslots);
  const int64_t chunk = (nslots + nb - 1) / nb;
  const DtReq none{};
  hipLaunchKernelGGL(k_reduce_smax<false>, dim3((unsigned)nb), dim3(256), 0, st, part, nslots, chunk, D, scratch,
                     smax, none);
  hipLaunchKernelGGL(k_reduce_smax<true>, dim3(1), dim3(256), 0, st, scratch, nb, nb, D, nullptr, smax,
                     req ? *req : none);
  return hipGetLastError();
}

// one slot per thread of the first stage up to 1024 blocks (a chunk of 2048
// slots per block left 36 blocks at 2048^2, each waiting for 8 rounds of
// loads: 8.4 us for 73728 slots)
int64_t reduce_smax_blocks(int64_t nslots) {
  const int64_t nb = (nslots + 255) / 256;
  return nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
}

// pointwise kernels: D in 1..3 and two materials, or D in 1..2 and three
#define DIMP_DISPATCH_D(DD, NN, RX, KERNEL, ...)                                          \
  do {                                                                                      \
    if (RX == 2) hipLaunchKernelGGL((KERNEL<DD, NN, 2>), __VA_ARGS__);                      \
    else if (RX) hipLaunchKernelGGL((KERNEL<DD, NN, 1>), __VA_ARGS__);                      \
    else hipLaunchKernelGGL((KERNEL<DD, NN, 0>), __VA_ARGS__);                              \
  } while (0)
#define DIMP_DISPATCH(D, RX, KERNEL, ...)                                                   \
  do {                                                                                      \
    if (P.nmat == 3) {                                                                      \
      if (D == 1) DIMP_DISPATCH_D(1, 3, RX, KERNEL, __VA_ARGS__);                           \
      else if (D == 2) DIMP_DISPATCH_D(2, 3, RX, KERNEL, __VA_ARGS__);                      \
      else return hipErrorInvalidValue;                                                     \
    } else if (D == 1) DIMP_DISPATCH_D(1, 2, RX, KERNEL, __VA_ARGS__);                      \
    else if (D == 2) DIMP_DISPATCH_D(2, 2, RX, KERNEL, __VA_ARGS__);                        \
    else DIMP_DISPATCH_D(3, 2, RX, KERNEL, __VA_ARGS__);                                    \
  } while (0)

hipError_t launch_prim_to_cons(const Params& P, int D, int rx, const double* W, double* U, hipStream_t st) {
  const int grid = grid_for(P.ncell, 256);
  DIMP_DISPATCH(D, rx, k_prim_to_cons, dim3(grid), dim3(256), 0, st, P, W, U);
  return hipGetLastError();
}

hipError_t launch_cons_to_prim(const Params& P, int D, int rx, const double* U, double* W, hipStream_t st) {
  const int grid = grid_for(P.ncell, 256);
  DIMP_DISPATCH(D, rx, k_cons_to_prim, dim3(grid), dim3(256), 0, st, P, U, W);
  return hipGetLastError();
}

hipError_t launch_sources(const Params& P, int D, int rx, double* U, double dt, const double* dtp,
                          hipStream_t st) {
  const int grid = grid_for(P.ncell, 256);
  DIMP_DISPATCH(D, rx, k_sources, dim3(grid), dim3(256), 0, st, P, U, dt, dtp);
  return hipGetLastError();
}

hipError_t launch_wavespeed(const Params& P, int D, int rx, const double* U, unsigned long long* smax,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, smax, 3);
  const int64_t want = P.ncell < 256LL * 2048 ? P.ncell : 256LL * 2048;
  const int grid = grid_for(want, 256);
  DIMP_DISPATCH(D, rx, k_wavespeed, dim3(grid), dim3(256), 0, st, P, U, smax);
  return hipGetLastError();
}

hipError_t launch_check(const Params& P, int D, int rx, const double* U, unsigned long long* nbad, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, nbad, 1);
  const int grid = grid_for(P.ncell, 256);
  DIMP_DISPATCH(D, rx, k_check, dim3(grid), dim3(256), 0, st, P, U, nbad);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_cfl_dt(const Params& P, int D, unsigned long long* smax, double cfl, double* dt,
                         double* log, int64_t idx, hipStream_t st) {
  hipLaunchKernelGGL(k_cfl_dt, dim3(1), dim3(64), 0, st, smax, cfl, P.dx[0], P.dx[1], P.dx[2], D, dt, log, idx);
  return hipGetLastError();
}

hipError_t launch_u64_to_f64(const unsigned long long* p, double* out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_u64_to_f64, dim3(1), dim3(64), 0, st, p, out, n);
  return hipGetLastError();
}

}  // namespace dimp
