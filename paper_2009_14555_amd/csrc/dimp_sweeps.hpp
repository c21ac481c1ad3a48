// dimp_sweeps.hpp -- the sweep kernels (row and tile) and their launch templates.
//
//  * sweep_row: sweep along x, the contiguous axis.  One cell per lane: a
//    wave covers 64 consecutive cells of a row, 3 on each side being halo,
//    so 58 cells are written per wave.  Stencil neighbours along x come from
//    cross-lane shuffles; no LDS, no barriers.  Loads and stores are
//    coalesced 512-byte rows per field.
//  * sweep_tile: sweep along y or z.  The same one-cell-per-lane stages on a
//    tile of TILE_COLUMNS x columns by 64 cells, staged through LDS so that
//    HBM sees contiguous row segments; XCD-aware block order.
// The last sweep of a step can fuse the plastic and reactive fractional steps
// and the wave-speed reduction into its epilogue (FUSE), so a 2-D step reads
// and writes the state exactly twice.  Included by the translation units that
// instantiate the sweeps: dimp_kernels.hip (1-D and 2-D grids) and
// dimp_sweeps3.hip (3-D grids), compiled in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "dimp_internal.hpp"
#include "dimp_lane.hpp"

namespace dimp {

#ifndef TILE_COLUMNS
#define TILE_COLUMNS 4
#endif
// waves per SIMD the sweep kernels are built for (launch bound): three in 1-D
// and 2-D (<= 168 VGPRs, no or a few spilled dwords); the 3-D sweeps (nine
// stretch entries, up to 17 fields) need 200-250 VGPRs and run two without
// spilling, and so do the sweeps of a JWL mixture (its Newton split inlined)
// and of three materials (two more fields and a second set of THINC/BVD
// candidates: 30-90 spilled bytes a lane at three waves)
template <int D, int N, int RX, bool FUSE>
constexpr int sweep_waves() {
  return (D == 3 || RX == 2 || N > 2) ? 2 : 3;
}

// Output modes of the sweep kernels.  M_SPLIT: the split sweep, out = the
// updated state.  The unsplit SSP-RK3 of Sec. 3.1 evaluates D(q) direction
// by direction, y (and z) first through the tile kernel, x last through the
// row kernel, and builds the stage as it goes.  A stage is
//   a qn + b (q - dt D(q)),  (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3)
// for stages 1, 2, 3 (eq. (rk) with q^(2) and q^(4) folded in): M_RK_FIRST
// writes a qn + b (q - dt D_dir); M_RK_MID and M_RK_LAST write
// Rin - b dt D_dir (in 1-D the x pass is the first); the last pass of stage 3
// fuses the sources and the wave speed (FUSE).  The partial results differ
// from summing D first only by rounding.
enum { M_SPLIT = 0, M_RK_FIRST = 1, M_RK_MID = 2, M_RK_LAST = 3 };

__device__ __forceinline__ double rk_a(int stage) { return stage == 1 ? 0.0 : stage == 2 ? 0.75 : 1.0 / 3.0; }
__device__ __forceinline__ double rk_b(int stage) { return stage == 1 ? 1.0 : stage == 2 ? 0.25 : 2.0 / 3.0; }

// ----------------------------------------------------------- row sweep
// Sweep along x.  Each wave: one 64-cell segment of one row, loaded and
// stored straight from HBM (512-byte rows per field).
template <int D, int N, int RX, bool FUSE, int MODE = M_SPLIT, bool WALL = false>
__global__ __launch_bounds__(256, (sweep_waves<D, N, RX, FUSE>())) void sweep_row(Params P, const double* __restrict__ in, double* __restrict__ out,
                                                  double dt_arg, const double* __restrict__ dtp,
                                                  double* __restrict__ part, const double* __restrict__ Rin,
                                                  const double* qn, int stage) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  const double dt = dtp ? dtp[0] : dt_arg;
  const int lane = threadIdx.x & 63;
  const int64_t nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int64_t nseg = (nx + 57) / 58;
  // XCD-aware block order: consecutive logical blocks (the same and the
  // neighbouring rows, whose volume fractions the THINC normals read) run on
  // one XCD and share its L2
  const int64_t nblocks = (nseg * ny * nz + 3) / 4;
  const int64_t per = (nblocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (lb >= nblocks) return;  // uniform per block
  const int64_t wave = lb * 4 + (threadIdx.x >> 6);
  const int64_t row = wave / nseg;
  if (row >= ny * nz) return;  // uniform per wave
  const int64_t seg = wave - row * nseg;
  const int64_t x = seg * 58 + lane - 3;
  // WALL instances: reflective ends along x (mirror images, the wall's tie)
  const bool xflip = WALL && bc_mirrored(x, nx, P.bc[0]);
  const int64_t xm = WALL ? bc_map_wall(x, nx, P.bc[0]) : bc_map(x, nx, P.bc[0]);
  const int64_t yj = row % ny, zk = row / ny;
  const int64_t nc = P.ncell;
  const int64_t cell = row * nx + xm;
  // the conserved state is read from HBM once and parked in LDS (each lane
  // only touches its own slots) until the update needs it again
  __shared__ double stash[F * 256];
  bool first = true;
  auto load_U = [&](double* U) {
    if (first) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        U[f] = in[f * nc + cell];
        if (WALL && mirror_odd<D, N, RX>(f, 0) && xflip) U[f] = -U[f];  // a wall's mirror image
        stash[f * 256 + threadIdx.x] = U[f];
      }
      first = false;
    } else {
      asm volatile("" ::: "memory");  // re-read LDS rather than keep U live in registers
#pragma unroll
      for (int f = 0; f < F; ++f) U[f] = stash[f * 256 + threadIdx.x];
    }
  };
  double phi_t[3][3];
  if (P.thinc && D >= 2) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (D == 2 && c != 1) continue;
        if (b == 1 && c == 1) {
          phi_t[b][c] = in[cell];
          continue;
        }
        const int64_t yy = bc_map(yj + b - 1, ny, P.bc[1]);
        const int64_t zz = (D == 3) ? bc_map(zk + c - 1, nz, P.bc[2]) : 0;
        phi_t[b][c] = in[(zz * ny + yy) * nx + xm];
      }
  }
  const bool writer = (lane >= 3) && (lane < 61) && (x < nx);
  // the face on this lane's left is a reflective wall
  const bool wall = WALL && ((x == 0 && (P.bc[0] == BC_REFLECTIVE || P.bc[0] == BC_AXIS)) ||
                             (x == nx && P.bc[0] == BC_REFLECTIVE));
  double Un[F], s[D];
  if (MODE == M_SPLIT) {
    lane_sweep<D, N, RX, 0, FUSE>(P, load_U, phi_t, dt / P.dx[0], dt, writer, Un, s, wall);
  } else {
    lane_sweep<D, N, RX, 0, false, true>(P, load_U, phi_t, 1.0 / P.dx[0], dt, writer, Un, s, wall);
    if (writer) {
      const double b = rk_b(stage);
      if (D > 1) {
        // the y (and z) passes have formed a qn + b (q - dt D_y ...)
#pragma unroll
        for (int f = 0; f < F; ++f) Un[f] = Rin[f * nc + cell] - (b * dt) * Un[f];
      } else {
        double U[F];
        load_U(U);
        const double a = rk_a(stage);
#pragma unroll
        for (int f = 0; f < F; ++f) {
          const double q = U[f] - dt * Un[f];
          Un[f] = (stage == 1) ? q : a * qn[f * nc + cell] + b * q;
        }
      }
      if (FUSE) epilogue_cell<D, N, RX>(P, Un, dt, s);
    }
  }
  if (writer) {
#pragma unroll
    for (int f = 0; f < F; ++f) out[f * nc + cell] = Un[f];
  }
  if (FUSE) {
#pragma unroll
    for (int k = 0; k < D; ++k) wave_max_store(s[k], part + wave * 3 + k);
  }
}

// ---------------------------------------------------------- tile sweep
// Sweep along y or z.  A block of CW waves covers CW consecutive x columns
// and 64 cells along the sweep axis; the tile is staged through LDS so that
// HBM sees rows of CW doubles, while each wave holds one column with one cell
// per lane and runs the same stages as the row sweep.  Block indices are
// remapped so that neighbouring x chunks (which share L2 lines) run on the
// same XCD at about the same time.
template <int CW>
struct TileGeom {
  // element (f, r, c) of a [F][64][CW] tile: the column index is XOR-swizzled
  // by the row so that both access patterns are free of LDS bank conflicts:
  // the coalesced copies (16 lanes = 16/CW rows x CW columns) and the
  // per-wave column reads (16 lanes = 16 rows of one column)
  static constexpr int RS = 16 / CW;
  __device__ static constexpr int at(int f, int r, int c) { return (f * 64 + r) * CW + (c ^ ((r / RS) & (CW - 1))); }
  static constexpr int PP = CW + 3;  // phi tile row: CW + 2 columns (x halo of one), padded to an odd pitch
  // the results get a tile of their own (no barrier between the last read of
  // the input tile and the first write of a result) where both fit in 64 KB
  // of LDS; otherwise they overwrite the input tile after a barrier
  template <int F, int NPL>
  static constexpr bool separate() { return (2 * F * 64 * CW + NPL * 64 * PP) * 8 <= 65536; }
  template <int F, int NPL>
  static constexpr int lds_doubles() { return (separate<F, NPL>() ? 2 : 1) * F * 64 * CW + NPL * 64 * PP; }
};

template <int D, int N, int RX, int DIR, bool FUSE, int CW, int MODE = M_SPLIT, bool WALL = false>
__global__ __launch_bounds__(64 * CW, (sweep_waves<D, N, RX, FUSE>())) void sweep_tile(Params P, const double* __restrict__ in,
                                                       double* __restrict__ out, double dt_arg,
                                                       const double* __restrict__ dtp,
                                                       double* __restrict__ part, int64_t nblocks,
                                                       const double* __restrict__ Rin, const double* qn,
                                                       int stage) {
  using L = Lay<D, N, RX>;
  using G = TileGeom<CW>;
  constexpr int F = L::F;
  constexpr int PP = G::PP;
  constexpr int NPL = (D == 3) ? 3 : 1;      // phi planes along the other transverse axis
  constexpr bool SEP = G::template separate<F, NPL>();
  extern __shared__ double lds[];
  double* tileU = lds;                               // [F][64][CW] input state
  double* tileO = SEP ? lds + F * 64 * CW : tileU;   // [F][64][CW] results
  double* tileP = lds + (SEP ? 2 : 1) * F * 64 * CW; // [NPL][64][PP]
  const double dt = dtp ? dtp[0] : dt_arg;

  // XCD-aware logical block index
  const int64_t per = (nblocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (lb >= nblocks) return;  // uniform per block, before any barrier
  const int64_t nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int64_t nm = P.n[DIR];
  const int oa = (DIR == 1) ? 2 : 1;  // the other transverse axis (3-D)
  const int64_t no = (D == 3) ? P.n[oa] : 1;
  const int64_t nxc = (nx + CW - 1) / CW;
  const int64_t xc = lb % nxc;
  int64_t rest = lb / nxc;
  const int64_t o = rest % no;
  const int64_t seg = rest / no;
  const int64_t x0 = xc * CW;
  const int64_t j0 = seg * 58 - 3;
  const int64_t sx = 1, sm = (DIR == 1) ? nx : nx * ny, so = (oa == 1) ? nx : nx * ny;
  const int64_t nc = P.ncell;
  const int tid = threadIdx.x;

  // load the tile: thread t -> row r (sweep axis), column c (x)
  for (int t = tid; t < 64 * CW; t += 64 * CW) {
    const int r = t / CW, c = t % CW;
    const int64_t xx = bc_map(x0 + c, nx, P.bc[0]);
    const int64_t jj = WALL ? bc_map_wall(j0 + r, nm, P.bc[DIR]) : bc_map(j0 + r, nm, P.bc[DIR]);
    const int64_t cell = xx * sx + jj * sm + o * so;
#pragma unroll
    for (int f = 0; f < F; ++f) tileU[G::at(f, r, c)] = in[f * nc + cell];
    // WALL instances: a wall's mirror image
    if (WALL && bc_mirrored(j0 + r, nm, P.bc[DIR])) {
#pragma unroll
      for (int f = 0; f < F; ++f)
        if (mirror_odd<D, N, RX>(f, DIR)) tileU[G::at(f, r, c)] = -tileU[G::at(f, r, c)];
    }
  }
  if (P.thinc && D >= 2) {
    for (int t = tid; t < 64 * (CW + 2) * NPL; t += 64 * CW) {
      const int pl = t / (64 * (CW + 2));
      const int rem = t - pl * 64 * (CW + 2);
      const int r = rem / (CW + 2), c = rem % (CW + 2);
      const int64_t xx = bc_map(x0 + c - 1, nx, P.bc[0]);
      const int64_t jj = bc_map(j0 + r, nm, P.bc[DIR]);
      const int64_t oo = (D == 3) ? bc_map(o + pl - 1, no, P.bc[oa]) : 0;
      tileP[(pl * 64 + r) * PP + c] = in[xx * sx + jj * sm + oo * so];
    }
  }
  __syncthreads();
  const int w = tid >> 6, lane = tid & 63;
  auto load_U = [&](double* U) {
    asm volatile("" ::: "memory");  // re-read LDS rather than keep U live in registers
#pragma unroll
    for (int f = 0; f < F; ++f) U[f] = tileU[G::at(f, lane, w)];
  };
  // transverse phi offsets: b along x, c along the other axis (3-D)
  double phi_t[3][3];
  if (P.thinc && D >= 2) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (D == 2 && c != 1) continue;
        const int pl = (D == 3) ? c : 0;
        phi_t[b][c] = tileP[(pl * 64 + lane) * PP + w + b];
      }
  }
  // lane_sweep orders the transverse offsets over the other two axes in
  // increasing axis order: for DIR = 1 that is (x, z), for DIR = 2 (x, y)
  const bool writer = (lane >= 3) && (lane < 61) && (j0 + lane < nm) && (x0 + w < nx);
  const int64_t jl = j0 + lane;
  const bool wall = WALL && ((jl == 0 && (P.bc[DIR] == BC_REFLECTIVE || P.bc[DIR] == BC_AXIS)) ||
                             (jl == nm && P.bc[DIR] == BC_REFLECTIVE));
  double Un[F], s[D];
  if (MODE == M_SPLIT)
    lane_sweep<D, N, RX, DIR, FUSE>(P, load_U, phi_t, dt / P.dx[DIR], dt, writer, Un, s, wall);
  else
    lane_sweep<D, N, RX, DIR, false, true>(P, load_U, phi_t, 1.0 / P.dx[DIR], dt, writer, Un, s, wall);
  if (MODE == M_RK_FIRST && writer) {
    // q - dt D_y(q) (the input tile still holds q)
    double U[F];
    load_U(U);
#pragma unroll
    for (int f = 0; f < F; ++f) Un[f] = U[f] - dt * Un[f];
  }
  if (!SEP) __syncthreads();  // everyone has read its column of the input tile
  if (writer) {
#pragma unroll
    for (int f = 0; f < F; ++f) tileO[G::at(f, lane, w)] = Un[f];
  }
  __syncthreads();
  for (int t = tid; t < 64 * CW; t += 64 * CW) {
    const int r = t / CW, c = t % CW;
    const int64_t xx = x0 + c, jj = j0 + r;
    if (r >= 3 && r < 61 && xx < nx && jj < nm) {
      const int64_t cell = xx * sx + jj * sm + o * so;
      if (MODE == M_SPLIT) {
#pragma unroll
        for (int f = 0; f < F; ++f) out[f * nc + cell] = tileO[G::at(f, r, c)];
      } else {
        // the stage's partial result: the tile holds D_z (mid) or
        // q - dt D_y (first)
        const double a = rk_a(stage), b = rk_b(stage);
#pragma unroll
        for (int f = 0; f < F; ++f) {
          const double d = tileO[G::at(f, r, c)];
          double v;
          if (MODE == M_RK_MID)
            v = Rin[f * nc + cell] - (b * dt) * d;
          else
            v = (stage == 1) ? d : a * qn[f * nc + cell] + b * d;
          out[f * nc + cell] = v;
        }
      }
    }
  }
  if (FUSE && MODE == M_SPLIT) {
    const int64_t slot = lb * CW + (tid >> 6);
#pragma unroll
    for (int k = 0; k < D; ++k) wave_max_store(s[k], part + slot * 3 + k);
  }
}

// ---------------------------------------------------------------- launch
static inline int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g > 65535LL * 64) g = 65535LL * 64;
  return (int)(g < 1 ? 1 : g);
}

template <int D, int N, int RX, int DIR, bool FUSE, int MODE = M_SPLIT>
static void launch_tile(const Params& P, const double* in, double* out, double dt, const double* dtp,
                        double* part, hipStream_t st, const double* Rin = nullptr, const double* qn = nullptr,
                        int stage = 0) {
  const bool walls = P.bc[DIR] >= BC_REFLECTIVE;
  constexpr int CW = TILE_COLUMNS;
  using L = Lay<D, N, RX>;
  const int oa = (DIR == 1) ? 2 : 1;
  const int64_t no = (D == 3) ? P.n[oa] : 1;
  const int64_t nblocks = ((P.n[0] + CW - 1) / CW) * no * ((P.n[DIR] + 57) / 58);
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  const size_t lds = sizeof(double) * TileGeom<CW>::template lds_doubles<L::F, (D == 3) ? 3 : 1>();
  if (walls) {
    hipLaunchKernelGGL((sweep_tile<D, N, RX, DIR, FUSE, CW, MODE, true>), dim3((unsigned)grid), dim3(64 * CW), lds,
                       st, P, in, out, dt, dtp, part, nblocks, Rin, qn, stage);
    return;
  }
  hipLaunchKernelGGL((sweep_tile<D, N, RX, DIR, FUSE, CW, MODE>), dim3((unsigned)grid), dim3(64 * CW), lds, st, P,
                     in, out, dt, dtp, part, nblocks, Rin, qn, stage);
}

static inline int row_grid(const Params& P) {
  const int64_t nseg = (P.n[0] + 57) / 58;
  const int64_t waves = nseg * P.n[1] * P.n[2];
  const int64_t nblocks = (waves * 64 + 255) / 256;  // four waves a block
  return (int)(((nblocks + 7) / 8) * 8);
}

template <int D, int N, int RX>
static hipError_t launch_rk_t(const Params& P, int dir, int mode, int stage, bool fuse, const double* in,
                              double* out, const double* Rin, const double* qn, double dt, const double* dtp,
                              double* part, hipStream_t st) {
  if (dir == 0) {
    if (mode != M_RK_LAST) return hipErrorInvalidValue;
    if (P.bc[0] >= BC_REFLECTIVE) {
      if (fuse)
        hipLaunchKernelGGL((sweep_row<D, N, RX, true, M_RK_LAST, true>), dim3(row_grid(P)), dim3(256), 0, st, P, in,
                           out, dt, dtp, part, Rin, qn, stage);
      else
        hipLaunchKernelGGL((sweep_row<D, N, RX, false, M_RK_LAST, true>), dim3(row_grid(P)), dim3(256), 0, st, P,
                           in, out, dt, dtp, part, Rin, qn, stage);
      return hipGetLastError();
    }
    if (fuse)
      hipLaunchKernelGGL((sweep_row<D, N, RX, true, M_RK_LAST>), dim3(row_grid(P)), dim3(256), 0, st, P, in, out, dt,
                         dtp, part, Rin, qn, stage);
    else
      hipLaunchKernelGGL((sweep_row<D, N, RX, false, M_RK_LAST>), dim3(row_grid(P)), dim3(256), 0, st, P, in, out,
                         dt, dtp, part, Rin, qn, stage);
    return hipGetLastError();
  }
  if constexpr (D >= 2) {
    if (dir == 1 && mode == M_RK_FIRST) {
      launch_tile<D, N, RX, 1, false, M_RK_FIRST>(P, in, out, dt, dtp, part, st, nullptr, qn, stage);
      return hipGetLastError();
    }
    if constexpr (D == 3) {
      if (dir == 2 && mode == M_RK_MID) {
        launch_tile<D, N, RX, 2, false, M_RK_MID>(P, in, out, dt, dtp, part, st, Rin, qn, stage);
        return hipGetLastError();
      }
    }
  }
  return hipErrorInvalidValue;
}

template <int D, int N, int RX>
static hipError_t launch_sweep_t(const Params& P, const double* in, double* out, double dt, const double* dtp,
                                 int dir, bool fuse, double* part, int S, hipStream_t st) {
  (void)S;
  const int block = 256;
  if (dir == 0) {
    const int grid = row_grid(P);
    if (P.bc[0] >= BC_REFLECTIVE) {
      if (fuse)
        hipLaunchKernelGGL((sweep_row<D, N, RX, true, M_SPLIT, true>), dim3(grid), dim3(block), 0, st, P, in, out,
                           dt, dtp, part, nullptr, nullptr, 0);
      else
        hipLaunchKernelGGL((sweep_row<D, N, RX, false, M_SPLIT, true>), dim3(grid), dim3(block), 0, st, P, in, out,
                           dt, dtp, part, nullptr, nullptr, 0);
      return hipGetLastError();
    }
    if (fuse)
      hipLaunchKernelGGL((sweep_row<D, N, RX, true>), dim3(grid), dim3(block), 0, st, P, in, out, dt, dtp, part,
                         nullptr, nullptr, 0);
    else
      hipLaunchKernelGGL((sweep_row<D, N, RX, false>), dim3(grid), dim3(block), 0, st, P, in, out, dt, dtp, part,
                         nullptr, nullptr, 0);
    return hipGetLastError();
  }
  if constexpr (D >= 2) {
    if (dir == 1) {
      if (fuse) launch_tile<D, N, RX, 1, true>(P, in, out, dt, dtp, part, st);
      else launch_tile<D, N, RX, 1, false>(P, in, out, dt, dtp, part, st);
      return hipGetLastError();
    }
    if constexpr (D == 3) {
      if (fuse) launch_tile<D, N, RX, 2, true>(P, in, out, dt, dtp, part, st);
      else launch_tile<D, N, RX, 2, false>(P, in, out, dt, dtp, part, st);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace dimp
