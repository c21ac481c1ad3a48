// dimp_amr.hip -- kernels of the two-level subcycled refinement (Sec. 3):
// the coarse-to-fine ghost fill, the fine-to-coarse averaging, the fluxes
// through the coarse/fine boundary and the flux correction of the coarse
// cells beside it.  All are small next to the sweeps.
#include <algorithm>

#include "dimp_amr.hpp"
#include "dimp_lane.hpp"

namespace dimp {
namespace {

__device__ __forceinline__ double amr_minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return (fabs(a) < fabs(b)) ? a : b;
}

// number of fine cells the fill writes: the ghost ring, or every cell
__host__ __device__ inline int64_t amr_fill_count(const AmrBox& b, int all) {
  return all ? b.nxf * b.nyf : b.nxf * b.nyf - (b.nxf - 2 * b.G) * (b.nyf - 2 * b.G);
}

// one thread per fine cell written: with all, cell t of the grid; else the
// t-th cell of the ring (its G bottom rows, its G top rows, then G cells at
// each end of every row between)
__global__ __launch_bounds__(256) void k_amr_fill(AmrBox b, const double* __restrict__ cold,
                                                  const double* __restrict__ cnew, double w,
                                                  double* __restrict__ fine, int all) {
  const int64_t nf = b.nxf * b.nyf, nc = b.nxc * b.nyc;
  const int64_t count = amr_fill_count(b, all), band = b.G * b.nxf;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < count; u += (int64_t)gridDim.x * blockDim.x) {
    int64_t fi, fj;
    if (all || u < band) {
      fi = u % b.nxf;
      fj = u / b.nxf;
    } else if (u < 2 * band) {
      fi = (u - band) % b.nxf;
      fj = b.nyf - b.G + (u - band) / b.nxf;
    } else {
      const int64_t v = u - 2 * band, c = v % (2 * b.G);
      fj = b.G + v / (2 * b.G);
      fi = c < b.G ? c : b.nxf - 2 * b.G + c;
    }
    const int64_t t = fj * b.nxf + fi;
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

// fine-to-fine exchange: the level's fine positions [x0, x0 + w) x [y0, y0 +
// h) (fine index 2 I + a inside coarse cell I) lie in patch q's interior and
// in patch p's stored grid; p's stored cells there <- q's values, all fields
__global__ __launch_bounds__(256) void k_amr_exchange(AmrBox p, AmrBox q, int64_t x0, int64_t y0, int64_t w,
                                                      int64_t h, const double* __restrict__ src,
                                                      double* __restrict__ dst) {
  const int64_t nfp = p.nxf * p.nyf, nfq = q.nxf * q.nyf;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < w * h; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t X = x0 + t % w, Y = y0 + t / w;
    const int64_t cp = (Y - 2 * p.j0 + p.G) * p.nxf + (X - 2 * p.i0 + p.G);
    const int64_t cq = (Y - 2 * q.j0 + q.G) * q.nxf + (X - 2 * q.i0 + q.G);
    for (int f = 0; f < p.F; ++f) dst[f * nfp + cp] = src[f * nfq + cq];
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

// Ten faces per wave: lanes 6k .. 6k + 5 hold the cells pos - 3 .. pos + 2
// along DIR of face k (lanes 60..63 idle).  The flux through the left face of
// a segment's fourth cell depends on the segment's six cells only (3 before
// the face, 2 after; the cross-lane shifts never carry a value from the next
// segment into that result), so each segment's lane 3 stores its face's flux
// as the sweep computes it (the same stages, lane_face): the split sweep's
// (MUSCL-Hancock edges, time step dt) or, with RK, the unsplit operator's
// (edges without the predictor); times wgt, added to what is stored with acc.
constexpr int FLUX_SEG = 6, FLUX_PER_WAVE = 10;

template <int N, int RX, int DIR, bool RK>
__global__ __launch_bounds__(256) void k_amr_flux(Params P, FaceSet fs, const double* __restrict__ in, double dt,
                                                  double* __restrict__ flux, double wgt, int acc) {
  constexpr int D = 2;
  constexpr int F = Lay<D, N, RX>::F;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wave * FLUX_PER_WAVE >= 2 * fs.len) return;  // uniform per wave
  const int seg = lane / FLUX_SEG, l = lane - seg * FLUX_SEG;
  int64_t face = wave * FLUX_PER_WAVE + seg;
  const bool live = seg < FLUX_PER_WAVE && face < 2 * fs.len;
  if (!live) face = 0;  // any valid face; nothing is stored
  const int side = face >= fs.len ? 1 : 0;
  const int64_t t = face - side * fs.len;
  const int64_t na = P.n[DIR];
  int64_t a = fs.pos[side] - 3 + l;
  a = a < 0 ? 0 : (a >= na ? na - 1 : a);
  const int64_t tr = fs.t0 + t;
  auto at = [&](int64_t along, int64_t across) { return DIR == 0 ? across * P.n[0] + along : along * P.n[0] + across; };
  const int64_t nc = P.ncell, cell = at(a, tr);
  auto load_U = [&](double* U) {
#pragma unroll
    for (int f = 0; f < F; ++f) U[f] = in[f * nc + cell];
  };
  double phi_t[3][3] = {};
  if (P.thinc) {
#pragma unroll
    for (int b = 0; b < 3; ++b) phi_t[b][1] = in[at(a, tr + b - 1)];
  }
  FaceV<D, N, RX> fa;
  double irho0;
  lane_face<D, N, RX, DIR, RK>(P, load_U, phi_t, RK ? 1.0 / P.dx[DIR] : dt / P.dx[DIR], fa, irho0, false);
  (void)irho0;
  if (live && l == 3) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      double* q = flux + ((int64_t)f * 2 + side) * fs.len + t;
      *q = acc ? *q + wgt * fa.F[f] : wgt * fa.F[f];
    }
  }
}

// One thread per coarse face of the patch's boundary (x faces first); each
// corrects the one coarse cell outside the patch beside it, so no two threads
// write the same cell.
__global__ __launch_bounds__(256) void k_amr_reflux(AmrBox b, int c0, int c1, double lamx, double lamy,
                                                    const double* __restrict__ fcx, const double* __restrict__ fcy,
                                                    const double* __restrict__ fx0, const double* __restrict__ fy0,
                                                    const double* __restrict__ fx1, const double* __restrict__ fy1,
                                                    double* __restrict__ coarse) {
  const int64_t pw = b.i1 - b.i0, ph = b.j1 - b.j0;
  const int64_t nc = b.nxc * b.nyc;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 2 * (pw + ph);
       t += (int64_t)gridDim.x * blockDim.x) {
    const bool xf = t < 2 * ph;
    const int64_t len = xf ? ph : pw;
    const int64_t u = xf ? t : t - 2 * ph;
    const int side = u >= len ? 1 : 0;
    const int64_t r = u - side * len;
    int64_t cell;
    if (xf)
      cell = (b.j0 + r) * b.nxc + (side ? b.i1 : b.i0 - 1);
    else
      cell = (side ? b.j1 : b.j0 - 1) * b.nxc + b.i0 + r;
    const double* fc = xf ? fcx : fcy;
    const double* f0 = xf ? fx0 : fy0;
    const double* f1 = xf ? fx1 : fy1;
    const double lam = xf ? lamx : lamy;
    const double sgn = side ? 1.0 : -1.0;
    for (int f = c0; f < c1; ++f) {
      const int64_t q = ((int64_t)f * 2 + side) * (2 * len) + 2 * r;  // the two fine faces
      const double fb = 0.25 * ((f0[q] + f0[q + 1]) + (f1[q] + f1[q + 1]));
      const double fcc = fc[((int64_t)f * 2 + side) * len + r];
      coarse[f * nc + cell] += sgn * (lam * (fb - fcc));
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
  hipLaunchKernelGGL(k_amr_fill, dim3(amr_grid(amr_fill_count(b, all ? 1 : 0))), dim3(256), 0, st, b, cold, cnew, w,
                     fine, all ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_amr_tag(const TagLayout& t, const double* prim, double threshold, unsigned char* tags,
                          unsigned long long* bbox, hipStream_t st) {
  hipLaunchKernelGGL(k_amr_tag, dim3(amr_grid(t.nx * t.ny)), dim3(256), 0, st, t, prim, threshold, tags, bbox);
  return hipGetLastError();
}

hipError_t launch_amr_flux(const Params& P, int rx, int dir, const FaceSet& fs, const double* in, double dt,
                           double* flux, hipStream_t st, bool rk, double wgt, bool acc) {
  if (dir < 0 || dir > 1 || fs.len < 1) return hipErrorInvalidValue;
  const int64_t na = P.n[dir], nt = P.n[1 - dir];
  for (int s = 0; s < 2; ++s)
    if (fs.pos[s] < 3 || fs.pos[s] + 2 > na - 1) return hipErrorInvalidValue;
  if (fs.t0 < 1 || fs.t0 + fs.len > nt - 1) return hipErrorInvalidValue;
  const int64_t waves = (2 * fs.len + FLUX_PER_WAVE - 1) / FLUX_PER_WAVE;
  const int grid = (int)((waves + 3) / 4);
  const int a = acc ? 1 : 0;
#define DIMP_AMR_FLUX(NV, RXV, DIRV)                                                                           \
  do {                                                                                                         \
    if (rk)                                                                                                    \
      hipLaunchKernelGGL((k_amr_flux<NV, RXV, DIRV, true>), dim3(grid), dim3(256), 0, st, P, fs, in, dt, flux,   \
                         wgt, a);                                                                              \
    else                                                                                                       \
      hipLaunchKernelGGL((k_amr_flux<NV, RXV, DIRV, false>), dim3(grid), dim3(256), 0, st, P, fs, in, dt, flux,  \
                         wgt, a);                                                                              \
  } while (0)
#define DIMP_AMR_FLUX_RX(NV, DIRV)          \
  do {                                      \
    if (rx == 2) DIMP_AMR_FLUX(NV, 2, DIRV); \
    else if (rx) DIMP_AMR_FLUX(NV, 1, DIRV); \
    else DIMP_AMR_FLUX(NV, 0, DIRV);         \
  } while (0)
  if (P.nmat == 3) {
    if (dir == 0) DIMP_AMR_FLUX_RX(3, 0);
    else DIMP_AMR_FLUX_RX(3, 1);
  } else if (P.nmat == 2) {
    if (dir == 0) DIMP_AMR_FLUX_RX(2, 0);
    else DIMP_AMR_FLUX_RX(2, 1);
  } else {
    return hipErrorInvalidValue;
  }
#undef DIMP_AMR_FLUX_RX
#undef DIMP_AMR_FLUX
  return hipGetLastError();
}

hipError_t launch_amr_reflux(const AmrBox& b, int c0, int c1, const double lam[2], const double* const fc[2],
                             const double* const ff0[2], const double* const ff1[2], double* coarse,
                             hipStream_t st) {
  const int64_t nface = 2 * ((b.i1 - b.i0) + (b.j1 - b.j0));
  hipLaunchKernelGGL(k_amr_reflux, dim3(amr_grid(nface)), dim3(256), 0, st, b, c0, c1, lam[0], lam[1], fc[0], fc[1],
                     ff0[0], ff0[1], ff1[0], ff1[1], coarse);
  return hipGetLastError();
}

hipError_t launch_amr_exchange(const AmrBox& p, const AmrBox& q, const double* src, double* dst, hipStream_t st) {
  if (p.F != q.F || p.G != q.G || p.nxc != q.nxc || p.nyc != q.nyc) return hipErrorInvalidValue;
  const int64_t x0 = std::max(2 * q.i0, 2 * p.i0 - p.G), x1 = std::min(2 * q.i1, 2 * p.i1 + p.G);
  const int64_t y0 = std::max(2 * q.j0, 2 * p.j0 - p.G), y1 = std::min(2 * q.j1, 2 * p.j1 + p.G);
  if (x0 >= x1 || y0 >= y1) return hipSuccess;
  hipLaunchKernelGGL(k_amr_exchange, dim3(amr_grid((x1 - x0) * (y1 - y0))), dim3(256), 0, st, p, q, x0, y0, x1 - x0,
                     y1 - y0, src, dst);
  return hipGetLastError();
}

hipError_t launch_amr_average(const AmrBox& b, const double* fine, double* coarse, hipStream_t st) {
  hipLaunchKernelGGL(k_amr_average, dim3(amr_grid((b.i1 - b.i0) * (b.j1 - b.j0))), dim3(256), 0, st, b, fine,
                     coarse);
  return hipGetLastError();
}

}  // namespace dimp
