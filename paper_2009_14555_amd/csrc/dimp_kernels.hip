// dimp_kernels.hip -- gfx950 kernels of the split diffuse-interface step.
//
// Data movement (the physics lives in dimp_device.hpp / dimp_stencil.hpp):
//  * sweep_row: sweep along x, the contiguous axis.  One cell per lane: a
//    wave covers 64 consecutive cells of a row, 3 on each side being halo,
//    so 58 cells are written per wave.  Stencil neighbours along x come from
//    cross-lane shuffles; no LDS, no barriers.  Loads and stores are
//    coalesced 512-byte rows per field.
//  * sweep_col: sweep along y or z.  Lanes run across x (coalesced), each
//    thread marches S cells along the sweep axis keeping the stencil window
//    (primitive states, THINC candidates, the last predicted edge and the
//    last face flux) in registers; 6 halo cells per S are recomputed.
//  * pointwise kernels: primitive <-> conserved, sources, wave speed, state
//    check.
// The last sweep of a step can fuse the plastic and reactive fractional steps
// and the wave-speed reduction into its epilogue (FUSE), so a 2-D step reads
// and writes the state exactly twice.
#include <hip/hip_runtime.h>

#include "dimp_internal.hpp"
#include "dimp_stencil.hpp"

namespace dimp {

// ----------------------------------------------------------- row sweep
template <int D, int N, bool RX, bool FUSE>
__global__ __launch_bounds__(256) void sweep_row(Params P, const double* __restrict__ in, double* __restrict__ out,
                                                  double dt, unsigned long long* __restrict__ smax) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  constexpr int DIR = 0;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int64_t nseg = (nx + 57) / 58;
  const int64_t row = wave / nseg;
  if (row >= ny * nz) return;  // uniform per wave
  const int64_t seg = wave - row * nseg;
  const int64_t x = seg * 58 + lane - 3;
  const int64_t xm = bc_map(x, nx, P.bc[0]);
  const int64_t yj = row % ny, zk = row / ny;
  const int64_t nc = P.ncell;
  const int64_t cell = row * nx + xm;
  const double nu = dt / P.dx[0];

  double U[F];
#pragma unroll
  for (int f = 0; f < F; ++f) U[f] = in[f * nc + cell];
  double W[F];
  double rho0, rc2;
  {
    Thermo<N, RX> T;
    double H[6], J2;
    cons_to_prim<D, N, RX>(P, U, W, T, H, J2);
    rho0 = T.rho;
    rc2 = T.rho * T.c2;
  }
  double Wm[F], Wp[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    Wm[f] = __shfl_up(W[f], 1, 64);
    Wp[f] = __shfl_down(W[f], 1, 64);
  }
  // Youngs normal stencil of phi_1 around this cell
  double nd = 1.0;
  if (P.thinc && D >= 2) {
    if (D == 2) {
      double col[3];
      col[1] = W[0];
      col[0] = in[bc_map(yj - 1, ny, P.bc[1]) * nx + xm];
      col[2] = in[bc_map(yj + 1, ny, P.bc[1]) * nx + xm];
      double s[3][3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        s[0][b] = __shfl_up(col[b], 1, 64);
        s[1][b] = col[b];
        s[2][b] = __shfl_down(col[b], 1, 64);
      }
      nd = youngs2(s, P.dx, DIR);
    } else {
      double col[3][3];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int64_t yy = bc_map(yj + b - 1, ny, P.bc[1]);
          const int64_t zz = bc_map(zk + c - 1, nz, P.bc[2]);
          col[b][c] = (b == 1 && c == 1) ? W[0] : in[(zz * ny + yy) * nx + xm];
        }
      double s[3][3][3];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          s[0][b][c] = __shfl_up(col[b][c], 1, 64);
          s[1][b][c] = col[b][c];
          s[2][b][c] = __shfl_down(col[b][c], 1, 64);
        }
      nd = youngs3(s, P.dx, DIR);
    }
  }
  const Cand c0 = phi_candidates<D, N, RX>(P, Wm[0], W[0], Wp[0], nd);
  Cand cm, cp;
  cm.mL = __shfl_up(c0.mL, 1, 64);
  cm.mR = __shfl_up(c0.mR, 1, 64);
  cm.tL = __shfl_up(c0.tL, 1, 64);
  cm.tR = __shfl_up(c0.tR, 1, 64);
  cp.mL = __shfl_down(c0.mL, 1, 64);
  cp.mR = __shfl_down(c0.mR, 1, 64);
  cp.tL = __shfl_down(c0.tL, 1, 64);
  cp.tR = __shfl_down(c0.tR, 1, 64);
  double WL[F], WR[F];
  edges_predict<D, N, RX, DIR>(P, Wm, W, Wp, rho0, rc2, cm, c0, cp, nu, WL, WR);
  // face on the left of this cell: right edge of the left neighbour | my left edge
  double WRm[F];
#pragma unroll
  for (int f = 0; f < F; ++f) WRm[f] = __shfl_up(WR[f], 1, 64);
  FaceV<D, N, RX> fa, fb;
  face_flux<D, N, RX, DIR>(P, WRm, WL, fa);
#pragma unroll
  for (int f = 0; f < F; ++f) fb.F[f] = __shfl_down(fa.F[f], 1, 64);
  fb.ustar = __shfl_down(fa.ustar, 1, 64);
#pragma unroll
  for (int j = 0; j < D; ++j) fb.Vn[j] = __shfl_down(fa.Vn[j], 1, 64);
  const bool writer = (lane >= 3) && (lane < 61) && (x < nx);
  double Un[F];
  update_cell<D, N, RX, DIR>(U, fa, fb, nu, Un);
  double s[D];
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = 0.0;
  if (FUSE && writer) {
    plastic_cell<D, N, RX>(P, Un);
    reaction_cell<D, N, RX>(P, Un, dt);
    wavespeed_cell<D, N, RX>(P, Un, s);
  }
  if (writer) {
#pragma unroll
    for (int f = 0; f < F; ++f) out[f * nc + cell] = Un[f];
  }
  if (FUSE) {
#pragma unroll
    for (int k = 0; k < D; ++k) wave_max_atomic(s[k], smax + k);
  }
}

// -------------------------------------------------------- column sweep
template <int D, int N, bool RX, int DIR>
struct ColGeom {
  int64_t base;    // cell index of march coordinate 0 at this thread's transverse position
  int64_t stride;  // cell stride along the march
  int64_t nmarch;
  int bc;
};

// phi_1 at transverse offsets around march coordinate j: 3 values (2-D,
// offsets in x) or 9 (3-D, offsets in the two transverse axes)
template <int D, int DIR>
struct PhiRow {
  double v[D == 2 ? 3 : 9];
};

template <int D, int N, bool RX, int DIR, bool FUSE>
__global__ __launch_bounds__(256) void sweep_col(Params P, const double* __restrict__ in, double* __restrict__ out,
                                                  double dt, unsigned long long* __restrict__ smax, int S) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  const int64_t nx = P.n[0], ny = P.n[1], nz = P.n[2];
  const int64_t nc = P.ncell;
  const int64_t nm = P.n[DIR];
  const int64_t nseg = (nm + S - 1) / S;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // transverse coordinates: x (fastest, coalesced) and the other axis
  const int64_t x = t % nx;
  int64_t rest = t / nx;
  int64_t o2 = 0, seg;
  if (D == 3) {
    const int64_t n2 = (DIR == 1) ? nz : ny;
    o2 = rest % n2;
    rest /= n2;
  }
  seg = rest;
  const bool active = seg < nseg;
  if (!active) seg = nseg - 1;  // keep the wave's control flow uniform; no writes
  const int64_t stride = (DIR == 1) ? nx : nx * ny;
  int64_t base;
  if (D == 2)
    base = x;
  else if (DIR == 1)
    base = o2 * nx * ny + x;  // o2 = z
  else
    base = o2 * nx + x;       // o2 = y
  const int bcm = P.bc[DIR];
  const int64_t j0 = seg * S;
  const double nu = dt / P.dx[DIR];

  auto load_phirow = [&](int64_t jm, PhiRow<D, DIR>& r, double self) {
    if (!P.thinc) return;
    if (D == 2) {
      const int64_t xm = bc_map(x - 1, nx, P.bc[0]), xp = bc_map(x + 1, nx, P.bc[0]);
      r.v[0] = in[jm * stride + xm];
      r.v[1] = self;
      r.v[2] = in[jm * stride + xp];
    } else {
      // transverse axes: x and the other one (a = x offset, c = other offset)
      const int oa = (DIR == 1) ? 2 : 1;
      const int64_t no = P.n[oa];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (a == 1 && c == 1) {
            r.v[3 * a + c] = self;
            continue;
          }
          const int64_t xx = bc_map(x + a - 1, nx, P.bc[0]);
          const int64_t oo = bc_map(o2 + c - 1, no, P.bc[oa]);
          const int64_t cidx = (DIR == 1) ? (oo * nx * ny + jm * nx + xx) : (oo * nx + jm * nx * ny + xx);
          r.v[3 * a + c] = in[cidx];
        }
    }
  };

  // windows: W and cell scalars for cells j-2, j-1, j (w0,w1,w2) and the
  // previous cell j-3 (wq), candidates for j-3, j-2 (ca, cb), phi rows
  double w0[F], w1[F], w2[F], wq[F];
  double r0 = 0, r1 = 0, r2 = 0, rq = 0, k0 = 0, k1 = 0, k2 = 0, kq = 0;  // rho and rho c^2
  PhiRow<D, DIR> p0, p1, p2;
  Cand ca, cb, cc;
  double wbR[F];  // right predicted edge of cell j-3
  FaceV<D, N, RX> fprev;
  double s[D];
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = 0.0;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    w0[f] = w1[f] = w2[f] = wq[f] = wbR[f] = 0.0;
  }
  ca = cb = cc = Cand{0, 0, 0, 0};

  for (int k = -3; k < S + 3; ++k) {
    const int64_t j = j0 + k;
    // rotate: (wq <- w0 <- w1 <- w2), candidates (ca <- cb <- cc)
#pragma unroll
    for (int f = 0; f < F; ++f) {
      wq[f] = w0[f];
      w0[f] = w1[f];
      w1[f] = w2[f];
    }
    rq = r0; r0 = r1; r1 = r2;
    kq = k0; k0 = k1; k1 = k2;
    p0 = p1;
    p1 = p2;
    ca = cb;
    cb = cc;
    // 1. ingest cell j
    {
      const int64_t jm = bc_map(j, nm, bcm);
      const int64_t cell = base + jm * stride;
      double U[F];
#pragma unroll
      for (int f = 0; f < F; ++f) U[f] = in[f * nc + cell];
      Thermo<N, RX> T;
      double H[6], J2;
      cons_to_prim<D, N, RX>(P, U, w2, T, H, J2);
      r2 = T.rho;
      k2 = T.rho * T.c2;
      load_phirow(jm, p2, w2[0]);
    }
    // 2. candidates of cell j-1
    if (k >= -1) {
      double nd = 1.0;
      if (P.thinc) {
        if (D == 2) {
          double st[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            st[a][0] = p0.v[a];
            st[a][1] = p1.v[a];
            st[a][2] = p2.v[a];
          }
          nd = youngs2(st, P.dx, DIR);
        } else {
          double st[3][3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const double v0 = p0.v[3 * a + c], v1 = p1.v[3 * a + c], v2 = p2.v[3 * a + c];
              if (DIR == 1) {  // axes (x, y=march, z)
                st[a][0][c] = v0;
                st[a][1][c] = v1;
                st[a][2][c] = v2;
              } else {         // axes (x, y=other, z=march)
                st[a][c][0] = v0;
                st[a][c][1] = v1;
                st[a][c][2] = v2;
              }
            }
          nd = youngs3(st, P.dx, DIR);
        }
      }
      cc = phi_candidates<D, N, RX>(P, w0[0], w1[0], w2[0], nd);
    }
    // 3. edges and predictor of cell j-2; 4. face between j-3 and j-2;
    // 5. update of cell j-3
    if (k >= 1) {
      double WL[F], WR[F];
      edges_predict<D, N, RX, DIR>(P, wq, w0, w1, r0, k0, ca, cb, cc, nu, WL, WR);
      if (k >= 2) {
        FaceV<D, N, RX> fcur;
        face_flux<D, N, RX, DIR>(P, wbR, WL, fcur);
        if (k >= 3) {
          const int64_t jc = j - 3;
          const int64_t cell = base + jc * stride;  // jc is inside [j0, j0+S) here
          if (active && jc < nm) {
            double U[F], Un[F];
#pragma unroll
            for (int f = 0; f < F; ++f) U[f] = in[f * nc + cell];
            update_cell<D, N, RX, DIR>(U, fprev, fcur, nu, Un);
            if (FUSE) {
              plastic_cell<D, N, RX>(P, Un);
              reaction_cell<D, N, RX>(P, Un, dt);
              double sc[D];
              wavespeed_cell<D, N, RX>(P, Un, sc);
#pragma unroll
              for (int q = 0; q < D; ++q) s[q] = (sc[q] > s[q] || sc[q] != sc[q]) ? sc[q] : s[q];
            }
#pragma unroll
            for (int f = 0; f < F; ++f) out[f * nc + cell] = Un[f];
          }
        }
        fprev = fcur;
      }
#pragma unroll
      for (int f = 0; f < F; ++f) wbR[f] = WR[f];
    }
  }
  if (FUSE) {
#pragma unroll
    for (int q = 0; q < D; ++q) wave_max_atomic(s[q], smax + q);
  }
}

// ------------------------------------------------------ pointwise kernels
template <int D, int N, bool RX>
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
      U[L::LAM * nc + c] = py * ry * fmin(fmax(w[L::LAM], 0.0), 1.0);
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

template <int D, int N, bool RX>
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

template <int D, int N, bool RX>
__global__ __launch_bounds__(256) void k_sources(Params P, double* __restrict__ U, double dt) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  const int64_t nc = P.ncell;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
    double u[F];
#pragma unroll
    for (int f = 0; f < F; ++f) u[f] = U[f * nc + c];
    plastic_cell<D, N, RX>(P, u);
    reaction_cell<D, N, RX>(P, u, dt);
#pragma unroll
    for (int f = 0; f < F; ++f) U[f * nc + c] = u[f];
  }
}

template <int D, int N, bool RX>
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

template <int D, int N, bool RX>
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

// ---------------------------------------------------------------- launch
static int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g > 65535LL * 64) g = 65535LL * 64;
  return (int)(g < 1 ? 1 : g);
}

template <int D, bool RX>
static hipError_t launch_sweep_t(const Params& P, const double* in, double* out, double dt, int dir, bool fuse,
                                 unsigned long long* smax, int S, hipStream_t st) {
  constexpr int N = 2;
  const int block = 256;
  if (dir == 0) {
    const int64_t nseg = (P.n[0] + 57) / 58;
    const int64_t waves = nseg * P.n[1] * P.n[2];
    const int grid = (int)((waves * 64 + block - 1) / block);
    if (fuse)
      hipLaunchKernelGGL((sweep_row<D, N, RX, true>), dim3(grid), dim3(block), 0, st, P, in, out, dt, smax);
    else
      hipLaunchKernelGGL((sweep_row<D, N, RX, false>), dim3(grid), dim3(block), 0, st, P, in, out, dt, smax);
    return hipGetLastError();
  }
  if constexpr (D >= 2) {
    const int64_t nm = P.n[dir];
    const int64_t nseg = (nm + S - 1) / S;
    const int64_t threads = P.ncell / nm * nseg;
    const int grid = (int)((threads + block - 1) / block);
    if (dir == 1) {
      if (fuse)
        hipLaunchKernelGGL((sweep_col<D, N, RX, 1, true>), dim3(grid), dim3(block), 0, st, P, in, out, dt, smax, S);
      else
        hipLaunchKernelGGL((sweep_col<D, N, RX, 1, false>), dim3(grid), dim3(block), 0, st, P, in, out, dt, smax, S);
      return hipGetLastError();
    }
    if constexpr (D == 3) {
      if (fuse)
        hipLaunchKernelGGL((sweep_col<D, N, RX, 2, true>), dim3(grid), dim3(block), 0, st, P, in, out, dt, smax, S);
      else
        hipLaunchKernelGGL((sweep_col<D, N, RX, 2, false>), dim3(grid), dim3(block), 0, st, P, in, out, dt, smax, S);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep(const Params& P, int D, bool rx, const double* in, double* out, double dt, int dir,
                        bool fuse, unsigned long long* smax, int S, hipStream_t st) {
  if (D == 1) return rx ? launch_sweep_t<1, true>(P, in, out, dt, dir, fuse, smax, S, st)
                        : launch_sweep_t<1, false>(P, in, out, dt, dir, fuse, smax, S, st);
  if (D == 2) return rx ? launch_sweep_t<2, true>(P, in, out, dt, dir, fuse, smax, S, st)
                        : launch_sweep_t<2, false>(P, in, out, dt, dir, fuse, smax, S, st);
  return rx ? launch_sweep_t<3, true>(P, in, out, dt, dir, fuse, smax, S, st)
            : launch_sweep_t<3, false>(P, in, out, dt, dir, fuse, smax, S, st);
}

#define DIMP_DISPATCH(D, RX, KERNEL, ...)                                                   \
  do {                                                                                      \
    if (D == 1) {                                                                           \
      if (RX) hipLaunchKernelGGL((KERNEL<1, 2, true>), __VA_ARGS__);                        \
      else hipLaunchKernelGGL((KERNEL<1, 2, false>), __VA_ARGS__);                          \
    } else if (D == 2) {                                                                    \
      if (RX) hipLaunchKernelGGL((KERNEL<2, 2, true>), __VA_ARGS__);                        \
      else hipLaunchKernelGGL((KERNEL<2, 2, false>), __VA_ARGS__);                          \
    } else {                                                                                \
      if (RX) hipLaunchKernelGGL((KERNEL<3, 2, true>), __VA_ARGS__);                        \
      else hipLaunchKernelGGL((KERNEL<3, 2, false>), __VA_ARGS__);                          \
    }                                                                                       \
  } while (0)

hipError_t launch_prim_to_cons(const Params& P, int D, bool rx, const double* W, double* U, hipStream_t st) {
  const int grid = grid_for(P.ncell, 256);
  DIMP_DISPATCH(D, rx, k_prim_to_cons, dim3(grid), dim3(256), 0, st, P, W, U);
  return hipGetLastError();
}

hipError_t launch_cons_to_prim(const Params& P, int D, bool rx, const double* U, double* W, hipStream_t st) {
  const int grid = grid_for(P.ncell, 256);
  DIMP_DISPATCH(D, rx, k_cons_to_prim, dim3(grid), dim3(256), 0, st, P, U, W);
  return hipGetLastError();
}

hipError_t launch_sources(const Params& P, int D, bool rx, double* U, double dt, hipStream_t st) {
  const int grid = grid_for(P.ncell, 256);
  DIMP_DISPATCH(D, rx, k_sources, dim3(grid), dim3(256), 0, st, P, U, dt);
  return hipGetLastError();
}

hipError_t launch_wavespeed(const Params& P, int D, bool rx, const double* U, unsigned long long* smax,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, smax, 3);
  const int64_t want = P.ncell < 256LL * 2048 ? P.ncell : 256LL * 2048;
  const int grid = grid_for(want, 256);
  DIMP_DISPATCH(D, rx, k_wavespeed, dim3(grid), dim3(256), 0, st, P, U, smax);
  return hipGetLastError();
}

hipError_t launch_check(const Params& P, int D, bool rx, const double* U, unsigned long long* nbad, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, nbad, 1);
  const int grid = grid_for(P.ncell, 256);
  DIMP_DISPATCH(D, rx, k_check, dim3(grid), dim3(256), 0, st, P, U, nbad);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_u64_to_f64(const unsigned long long* p, double* out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_u64_to_f64, dim3(1), dim3(64), 0, st, p, out, n);
  return hipGetLastError();
}

}  // namespace dimp
