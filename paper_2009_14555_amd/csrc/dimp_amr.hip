// dimp_amr.hip -- kernels of the two-level subcycled refinement (Sec. 3):
// the coarse-to-fine ghost fill and the fine-to-coarse averaging.  Both are
// pointwise over the cells they write (HBM-bound, small next to the sweeps).
#include "dimp_amr.hpp"

namespace dimp {
namespace {

__device__ __forceinline__ double amr_minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (fabs(a) < fabs(b)) ? a : b;
}

// one thread per fine cell of the ghost ring (the interior is skipped)
__global__ __launch_bounds__(256) void k_amr_fill(AmrBox b, const double* __restrict__ cold,
                                                  const double* __restrict__ cnew, double w,
                                                  double* __restrict__ fine, int all) {
  const int64_t nf = b.nxf * b.nyf, nc = b.nxc * b.nyc;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nf; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t fi = t % b.nxf, fj = t / b.nxf;
    const bool inside = fi >= b.G && fi < b.nxf - b.G && fj >= b.G && fj < b.nyf - b.G;
    if (inside && !all) continue;
    // parent (floor division of the offset from the patch corner) and the
    // fine centre's offset from the parent's, in coarse cells
    const int64_t di = fi - b.G, dj = fj - b.G;
    const int64_t I = b.i0 + (di >= 0 ? di / 2 : -((1 - di) / 2));
    const int64_t J = b.j0 + (dj >= 0 ? dj / 2 : -((1 - dj) / 2));
    const double ox = ((di & 1) == 0) ? -0.25 : 0.25;
    const double oy = ((dj & 1) == 0) ? -0.25 : 0.25;
    const int64_t c0 = J * b.nxc + I;
    for (int f = 0; f < b.F; ++f) {
      const double* o = cold + f * nc;
      const double* n = cnew + f * nc;
      auto at = [&](int64_t c) { return o[c] + w * (n[c] - o[c]); };
      const double c = at(c0);
      if (all) {  // a new patch: every cell takes its parent's state
        fine[f * nf + t] = c;
        continue;
      }
      const double sx = amr_minmod(c - at(c0 - 1), at(c0 + 1) - c);
      const double sy = amr_minmod(c - at(c0 - b.nxc), at(c0 + b.nxc) - c);
      fine[f * nf + t] = c + ox * sx + oy * sy;
    }
  }
}

// one thread per covered coarse cell
__global__ __launch_bounds__(256) void k_amr_average(AmrBox b, const double* __restrict__ fine,
                                                     double* __restrict__ coarse) {
  const int64_t pw = b.i1 - b.i0, ph = b.j1 - b.j0;
  const int64_t nf = b.nxf * b.nyf, nc = b.nxc * b.nyc;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < pw * ph; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t I = b.i0 + t % pw, J = b.j0 + t / pw;
    const int64_t fi = b.G + 2 * (I - b.i0), fj = b.G + 2 * (J - b.j0);
    const int64_t f00 = fj * b.nxf + fi;
    for (int f = 0; f < b.F; ++f) {
      const double* q = fine + f * nf;
      coarse[f * nc + J * b.nxc + I] = 0.25 * ((q[f00] + q[f00 + 1]) + (q[f00 + b.nxf] + q[f00 + b.nxf + 1]));
    }
  }
}

// fractional change of a refinement variable between two cells, against the
// larger magnitude with the kind's floor
__device__ __forceinline__ bool amr_jump(double a, double b, double fl, double th) {
  return fabs(b - a) > th * fmax(fmax(fabs(a), fabs(b)), fl);
}

// one thread per coarse cell; neighbours across the grid's edge are absent
__global__ __launch_bounds__(256) void k_amr_tag(TagLayout L, const double* __restrict__ W, double th,
                                                 unsigned char* __restrict__ tags,
                                                 unsigned long long* __restrict__ bbox) {
  const int64_t nc = L.nx * L.ny;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = c % L.nx, j = c / L.nx;
    bool tag = false;
    const int64_t nb[4] = {i > 0 ? c - 1 : -1, i < L.nx - 1 ? c + 1 : -1, j > 0 ? c - L.nx : -1,
                           j < L.ny - 1 ? c + L.nx : -1};
    for (int k = 0; k < 4; ++k) {
      const int64_t n = nb[k];
      if (n < 0) continue;
      double sa = 0.0, sb = 0.0;  // the last volume fraction is 1 - sum
      for (int l = 0; l < L.nphi; ++l) {
        const double a = W[l * nc + c], b = W[l * nc + n];
        tag = tag || amr_jump(a, b, L.floor_phi, th);
        sa += a;
        sb += b;
      }
      for (int l = 0; l < L.nmat; ++l) {  // phi_l rho_l
        const double pa = (l < L.nphi) ? W[l * nc + c] : 1.0 - sa;
        const double pb = (l < L.nphi) ? W[l * nc + n] : 1.0 - sb;
        tag = tag || amr_jump(pa * W[(L.rho0 + l) * nc + c], pb * W[(L.rho0 + l) * nc + n], L.floor_rho, th);
      }
      for (int d = 0; d < L.ndim; ++d)
        tag = tag || amr_jump(W[(L.u0 + d) * nc + c], W[(L.u0 + d) * nc + n], L.floor_u, th);
      tag = tag || amr_jump(W[L.p * nc + c], W[L.p * nc + n], L.floor_p, th);
    }
    tags[c] = tag ? 1 : 0;
    if (tag) {
      atomicMin(bbox + 0, (unsigned long long)i);
      atomicMin(bbox + 1, (unsigned long long)j);
      atomicMax(bbox + 2, (unsigned long long)i);
      atomicMax(bbox + 3, (unsigned long long)j);
    }
  }
}

int amr_grid(int64_t work) {
  int64_t g = (work + 255) / 256;
  if (g > 65535LL * 16) g = 65535LL * 16;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t launch_amr_fill(const AmrBox& b, const double* cold, const double* cnew, double w, double* fine,
                           hipStream_t st, bool all) {
  hipLaunchKernelGGL(k_amr_fill, dim3(amr_grid(b.nxf * b.nyf)), dim3(256), 0, st, b, cold, cnew, w, fine,
                     all ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_amr_tag(const TagLayout& t, const double* prim, double threshold, unsigned char* tags,
                          unsigned long long* bbox, hipStream_t st) {
  hipLaunchKernelGGL(k_amr_tag, dim3(amr_grid(t.nx * t.ny)), dim3(256), 0, st, t, prim, threshold, tags, bbox);
  return hipGetLastError();
}

hipError_t launch_amr_average(const AmrBox& b, const double* fine, double* coarse, hipStream_t st) {
  hipLaunchKernelGGL(k_amr_average, dim3(amr_grid((b.i1 - b.i0) * (b.j1 - b.j0))), dim3(256), 0, st, b, fine,
                     coarse);
  return hipGetLastError();
}

}  // namespace dimp
