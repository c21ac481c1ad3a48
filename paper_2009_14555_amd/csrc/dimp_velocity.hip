// dimp_velocity.hip -- a state at rest given a velocity field, and its
// vector-Jacobian product.
//
// The calibration runs of the adjoint differentiate with respect to the
// initial velocity: the conserved state is the rest state with the momentum
// rho u and the total energy E_rest + rho |u|^2 / 2 (E = e + |u|^2/2 of Sec.
// 2.2 with rho the mixture density sum_l phi_l rho_l).  Pointwise kernels,
// one cell per thread, HBM-bound.
#include <hip/hip_runtime.h>

#include "dimp_internal.hpp"

namespace dimp {

template <int D, int N, int RX>
__global__ __launch_bounds__(256) void k_with_velocity(int64_t nc, const double* __restrict__ rest,
                                                       const double* __restrict__ vel, double* __restrict__ out) {
  using L = Lay<D, N, RX>;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double rho = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) rho += rest[(L::M0 + l) * nc + c];
    double uu = 0.0;
#pragma unroll
    for (int f = 0; f < L::F; ++f) {
      if (f >= L::MOM0 && f < L::MOM0 + D) {
        const double v = vel[(f - L::MOM0) * nc + c];
        out[f * nc + c] = rho * v;
        uu += v * v;
      } else if (f != L::E) {
        out[f * nc + c] = rest[f * nc + c];
      }
    }
    out[L::E * nc + c] = rest[L::E * nc + c] + 0.5 * rho * uu;
  }
}

// adjoints: a_rest = dJ/d(rest state), a_vel = dJ/d(velocity), given a_out =
// dJ/d(out); the rest state's momentum is overwritten, so its adjoint is 0
template <int D, int N, int RX>
__global__ __launch_bounds__(256) void k_with_velocity_adj(int64_t nc, const double* __restrict__ rest,
                                                           const double* __restrict__ vel,
                                                           const double* __restrict__ a_out,
                                                           double* __restrict__ a_rest, double* __restrict__ a_vel) {
  using L = Lay<D, N, RX>;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double rho = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) rho += rest[(L::M0 + l) * nc + c];
    const double aE = a_out[L::E * nc + c];
    double uu = 0.0, drho = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double v = vel[k * nc + c];
      const double am = a_out[(L::MOM0 + k) * nc + c];
      uu += v * v;
      drho += am * v;
      a_vel[k * nc + c] = rho * (am + aE * v);
    }
    drho += 0.5 * aE * uu;
#pragma unroll
    for (int f = 0; f < L::F; ++f) {
      double a = a_out[f * nc + c];
      if (f >= L::M0 && f < L::M0 + N) a += drho;
      if (f >= L::MOM0 && f < L::MOM0 + D) a = 0.0;
      a_rest[f * nc + c] = a;
    }
  }
}

static int vel_grid(int64_t nc) {
  int64_t g = (nc + 255) / 256;
  if (g > 65535LL * 16) g = 65535LL * 16;
  return (int)(g < 1 ? 1 : g);
}

#define DIMP_VEL_DISPATCH(KERNEL, ...)                                                       \
  do {                                                                                       \
    const dim3 g_(vel_grid(nc)), b_(256);                                                    \
    if (D == 1) {                                                                            \
      if (rx) hipLaunchKernelGGL((KERNEL<1, 2, 1>), g_, b_, 0, st, __VA_ARGS__);             \
      else hipLaunchKernelGGL((KERNEL<1, 2, 0>), g_, b_, 0, st, __VA_ARGS__);                \
    } else if (D == 2) {                                                                     \
      if (rx) hipLaunchKernelGGL((KERNEL<2, 2, 1>), g_, b_, 0, st, __VA_ARGS__);             \
      else hipLaunchKernelGGL((KERNEL<2, 2, 0>), g_, b_, 0, st, __VA_ARGS__);                \
    } else {                                                                                 \
      if (rx) hipLaunchKernelGGL((KERNEL<3, 2, 1>), g_, b_, 0, st, __VA_ARGS__);             \
      else hipLaunchKernelGGL((KERNEL<3, 2, 0>), g_, b_, 0, st, __VA_ARGS__);                \
    }                                                                                        \
  } while (0)

hipError_t launch_with_velocity(int D, bool rx, int64_t nc, const double* rest, const double* vel, double* out,
                                hipStream_t st) {
  DIMP_VEL_DISPATCH(k_with_velocity, nc, rest, vel, out);
  return hipGetLastError();
}

hipError_t launch_with_velocity_adj(int D, bool rx, int64_t nc, const double* rest, const double* vel,
                                    const double* a_out, double* a_rest, double* a_vel, hipStream_t st) {
  DIMP_VEL_DISPATCH(k_with_velocity_adj, nc, rest, vel, a_out, a_rest, a_vel);
  return hipGetLastError();
}

}  // namespace dimp
