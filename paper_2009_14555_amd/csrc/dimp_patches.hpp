// dimp_patches.hpp -- split sweeps over a set of independent 2-D patches.
//
// AMR-style patch sets (the paper's AMR platform applies the single-grid
// update to every patch of a level in turn, Sec. 3): many small rectangular
// patches of different sizes, each stored with two ghost layers, all advanced
// with one global dt.  Instead of one launch per patch and sweep, one launch
// per sweep covers a precomputed task list of the whole set:
//  * psweep_row: a work item is one wave (one cell per lane, as in
//    sweep_row) holding segments of interior rows;
//  * psweep_tile: a work item is a CW-column x 64-row tile staged through LDS
//    (as in sweep_tile) holding segments of column chunks.
// Segments carry their own 3-lane halos, so short lines of different patches
// share a wave: a writer lane reads lanes within 3 of itself only, all inside
// its own segment, and the packing cannot change any result bit.
// Each wave/block takes one work item (a grid-stride persistent loop was
// measured first: its carried state pushed the sweep body into VGPR spills).
// Boundaries are transmissive per patch: halo reads are clamped into the
// patch interior, and every sweep also writes the ghost copies of the
// boundary cells it updates, so the stored ghost layers always hold the
// boundary images.  Per-patch launches run the same kernels on the task
// range of one patch, so both modes produce identical bits.
#pragma once
#include <hip/hip_runtime.h>

#include "dimp_internal.hpp"
#include "dimp_lane.hpp"

namespace dimp {

constexpr int PD = 2;
// waves per SIMD of the patch sweeps: 2 with a JWL mixture (its split holds
// more live state) or three materials, else 3
template <int N, int RX>
constexpr int patch_waves() {
  return (RX == 2 || N > 2) ? 2 : 3;
}

// write a value of interior cell (i, j) and, for boundary cells, its ghost
// images (the cell itself on the interior rows/columns it borders)
__device__ __forceinline__ void put_row(double* o, int64_t r, int i, int nx, double v) {
  o[r + i] = v;
  if (i == 0) {
    o[r - 1] = v;
    o[r - 2] = v;
  }
  if (i == nx - 1) {
    o[r + nx] = v;
    o[r + nx + 1] = v;
  }
}

__device__ __forceinline__ void write_with_ghosts(const PatchGeo& g, double* out, int64_t E, int f, int i, int j,
                                                  double v) {
  const int64_t pitch = g.nx + 2 * PATCH_GHOST;
  double* o = out + f * E + g.off + PATCH_GHOST;
  put_row(o, (j + PATCH_GHOST) * pitch, i, g.nx, v);
  if (j == 0) {
    put_row(o, (PATCH_GHOST - 1) * pitch, i, g.nx, v);
    put_row(o, (PATCH_GHOST - 2) * pitch, i, g.nx, v);
  }
  if (j == g.ny - 1) {
    put_row(o, (g.ny + PATCH_GHOST) * pitch, i, g.nx, v);
    put_row(o, (g.ny + PATCH_GHOST + 1) * pitch, i, g.nx, v);
  }
}

// XCD-aware block order: the hardware deals consecutive blocks round-robin
// to the 8 XCDs; remapping gives each XCD a contiguous run of tasks, so
// neighbouring rows/tiles of one patch share that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t per = nb >> 3;
  const int64_t xcd = b & 7, k = b >> 3;
  return (b < (per << 3)) ? xcd * per + k : b;
}

// segment of lane (or tile row) r among segments [sb, se): the last one
// whose first lane is <= r
__device__ __forceinline__ int4 segment_of(const int4* __restrict__ seg, int sb, int se, int r) {
  int4 sg = seg[sb];
  for (int k = sb + 1; k < se; ++k) {
    const int4 c = seg[k];
    if (r >= (c.w & 255)) sg = c;
  }
  return sg;
}

template <int N, int RX, bool FUSE, int WPB>
__global__ __launch_bounds__(64 * WPB, (patch_waves<N, RX>())) void psweep_row(
    Params P, const PatchGeo* __restrict__ geo, WorkList wl, int64_t w0, int64_t nwork, const double* __restrict__ in,
    double* __restrict__ out, double dt_arg, const double* __restrict__ dtp, double* __restrict__ part) {
  constexpr int F = Lay<PD, N, RX>::F;
  const int lane = threadIdx.x & 63;
  const int64_t wv = xcd_block(blockIdx.x, gridDim.x) * WPB + (threadIdx.x >> 6);
  if (wv >= nwork) return;  // whole waves only: a work item is one wave
  const double dt = dtp ? dtp[0] : dt_arg;
  const double nu = dt / P.dx[0];
  const int64_t E = P.ncell;
  __shared__ double stash[F * 64 * WPB];
  const int sb = wl.beg[w0 + wv], se = wl.beg[w0 + wv + 1];
  const int4 sg = segment_of(wl.seg, sb, se, lane);  // {patch, row, first x, lane0 | n << 8}
  const PatchGeo g = geo[sg.x];
  const int j = sg.y;
  const int q = lane - (sg.w & 255), ncl = sg.w >> 8;
  const int x = sg.z + q - SEG_HALO;
  const int xm = x < 0 ? 0 : (x > g.nx - 1 ? g.nx - 1 : x);
  const int64_t pitch = g.nx + 2 * PATCH_GHOST;
  const int64_t cell = g.off + (int64_t)(j + PATCH_GHOST) * pitch + PATCH_GHOST + xm;
  bool first = true;
  auto load_U = [&](double* U) {
    if (first) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        U[f] = in[f * E + cell];
        stash[f * 64 * WPB + threadIdx.x] = U[f];
      }
      first = false;
    } else {
      asm volatile("" ::: "memory");
#pragma unroll
      for (int f = 0; f < F; ++f) U[f] = stash[f * 64 * WPB + threadIdx.x];
    }
  };
  double phi_t[3][3];
  if (P.thinc) {
    // rows j-1, j+1 clamped into the patch (stored ghost values are never read)
    phi_t[0][1] = in[j > 0 ? cell - pitch : cell];
    phi_t[1][1] = in[cell];
    phi_t[2][1] = in[j < g.ny - 1 ? cell + pitch : cell];
  }
  const bool writer = (q >= SEG_HALO) && (q < ncl + SEG_HALO);
  double Un[F], s[PD];
  lane_sweep<PD, N, RX, 0, FUSE>(P, load_U, phi_t, nu, dt, writer, Un, s);
  if (writer) {
#pragma unroll
    for (int f = 0; f < F; ++f) write_with_ghosts(g, out, E, f, x, j, Un[f]);
  }
  if (FUSE) {
#pragma unroll
    for (int k = 0; k < PD; ++k) wave_max_store(s[k], part + (w0 + wv) * 3 + k);
  }
}

template <int N, int RX, bool FUSE, int CW>
__global__ __launch_bounds__(64 * CW, (patch_waves<N, RX>())) void psweep_tile(
    Params P, const PatchGeo* __restrict__ geo, WorkList wl, int64_t w0, int64_t nwork, const double* __restrict__ in,
    double* __restrict__ out, double dt_arg, const double* __restrict__ dtp, double* __restrict__ part) {
  constexpr int F = Lay<PD, N, RX>::F;
  constexpr int PITCH = CW + 1;
  constexpr int PP = CW + 2;
  extern __shared__ double lds[];
  double* tileU = lds;
  double* tileP = lds + F * 64 * PITCH;
  const int64_t t = xcd_block(blockIdx.x, gridDim.x);
  if (t >= nwork) return;  // whole block: a work item is one tile
  const double dt = dtp ? dtp[0] : dt_arg;
  const double nu = dt / P.dx[1];
  const int64_t E = P.ncell;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int sb = wl.beg[w0 + t], se = wl.beg[w0 + t + 1];
  // this thread's tile element (row r, column c) for the load and the store
  const int r = tid / CW, c = tid % CW;
  const int4 sr = segment_of(wl.seg, sb, se, r);  // {patch, x0, first y, lane0 | n << 8}
  const PatchGeo gr = geo[sr.x];
  const int64_t pr = gr.nx + 2 * PATCH_GHOST;
  const int qr = r - (sr.w & 255);
  const int xr = sr.y + c, jr = sr.z + qr - SEG_HALO;
  {
    const int xc = xr > gr.nx - 1 ? gr.nx - 1 : xr;
    const int jc = jr < 0 ? 0 : (jr > gr.ny - 1 ? gr.ny - 1 : jr);
    const int64_t cell = gr.off + (jc + PATCH_GHOST) * pr + PATCH_GHOST + xc;
#pragma unroll
    for (int f = 0; f < F; ++f) tileU[(f * 64 + r) * PITCH + c] = in[f * E + cell];
  }
  if (P.thinc) {
    for (int qq = tid; qq < 64 * PP; qq += 64 * CW) {
      const int rr = qq / PP, cc = qq % PP;
      const int4 sg = segment_of(wl.seg, sb, se, rr);
      const PatchGeo g = geo[sg.x];
      const int xx = sg.y + cc - 1, jj = sg.z + rr - (sg.w & 255) - SEG_HALO;
      const int xc = xx < 0 ? 0 : (xx > g.nx - 1 ? g.nx - 1 : xx);
      const int jc = jj < 0 ? 0 : (jj > g.ny - 1 ? g.ny - 1 : jj);
      tileP[rr * PP + cc] = in[g.off + (jc + PATCH_GHOST) * (int64_t)(g.nx + 2 * PATCH_GHOST) + PATCH_GHOST + xc];
    }
  }
  __syncthreads();
  auto load_U = [&](double* U) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int f = 0; f < F; ++f) U[f] = tileU[(f * 64 + lane) * PITCH + w];
  };
  double phi_t[3][3];
  if (P.thinc) {
#pragma unroll
    for (int b = 0; b < 3; ++b) phi_t[b][1] = tileP[lane * PP + w + b];
  }
  bool writer;
  {
    const int4 sl = segment_of(wl.seg, sb, se, lane);
    const int ql = lane - (sl.w & 255);
    writer = (ql >= SEG_HALO) && (ql < (sl.w >> 8) + SEG_HALO) && (sl.y + w < geo[sl.x].nx);
  }
  double Un[F], s[PD];
  lane_sweep<PD, N, RX, 1, FUSE>(P, load_U, phi_t, nu, dt, writer, Un, s);
  __syncthreads();
  if (writer) {
#pragma unroll
    for (int f = 0; f < F; ++f) tileU[(f * 64 + lane) * PITCH + w] = Un[f];
  }
  __syncthreads();
  if (qr >= SEG_HALO && qr < (sr.w >> 8) + SEG_HALO && xr < gr.nx) {
#pragma unroll
    for (int f = 0; f < F; ++f) write_with_ghosts(gr, out, E, f, xr, jr, tileU[(f * 64 + r) * PITCH + c]);
  }
  if (FUSE) {
#pragma unroll
    for (int k = 0; k < PD; ++k) wave_max_store(s[k], part + ((w0 + t) * CW + w) * 3 + k);
  }
}

template <int N, int RX, int CW>
size_t tile_lds_bytes() {
  return sizeof(double) * (Lay<PD, N, RX>::F * 64 * (CW + 1) + 64 * (CW + 2));
}

// one sweep of a patch set with N materials and the RX layout (the
// launch_patch_sweep contract)
template <int N, int RX>
hipError_t launch_patch_t(const Params& P, const PatchGeo* geo, WorkList wl, int64_t w0, int64_t nwork,
                          const double* in, double* out, double dt, const double* dtp, int dir, bool fuse,
                          double* part, int row_wpb, int cw, hipStream_t st) {
  if (nwork <= 0) return hipSuccess;
  if (dir == 0) {
    const dim3 grid((unsigned)((nwork + row_wpb - 1) / row_wpb));
    const dim3 block(64 * row_wpb);
#define DIMP_ROW(W)                                                                                              \
  if (fuse)                                                                                                     \
    hipLaunchKernelGGL((psweep_row<N, RX, true, W>), grid, block, 0, st, P, geo, wl, w0, nwork, in, out, dt, dtp,  \
                       part);                                                                                   \
  else                                                                                                          \
    hipLaunchKernelGGL((psweep_row<N, RX, false, W>), grid, block, 0, st, P, geo, wl, w0, nwork, in, out, dt, dtp, \
                       part);
    if (row_wpb == 1) {
      DIMP_ROW(1)
    } else if (row_wpb == 2) {
      DIMP_ROW(2)
    } else {
      DIMP_ROW(4)
    }
#undef DIMP_ROW
    return hipGetLastError();
  }
  const dim3 grid((unsigned)nwork);
  if (cw == 8) {
    const size_t lds = tile_lds_bytes<N, RX, 8>();
    if (fuse)
      hipLaunchKernelGGL((psweep_tile<N, RX, true, 8>), grid, dim3(512), lds, st, P, geo, wl, w0, nwork, in, out, dt,
                         dtp, part);
    else
      hipLaunchKernelGGL((psweep_tile<N, RX, false, 8>), grid, dim3(512), lds, st, P, geo, wl, w0, nwork, in, out, dt,
                         dtp, part);
  } else {
    const size_t lds = tile_lds_bytes<N, RX, 4>();
    if (fuse)
      hipLaunchKernelGGL((psweep_tile<N, RX, true, 4>), grid, dim3(256), lds, st, P, geo, wl, w0, nwork, in, out, dt,
                         dtp, part);
    else
      hipLaunchKernelGGL((psweep_tile<N, RX, false, 4>), grid, dim3(256), lds, st, P, geo, wl, w0, nwork, in, out, dt,
                         dtp, part);
  }
  return hipGetLastError();
}

}  // namespace dimp
