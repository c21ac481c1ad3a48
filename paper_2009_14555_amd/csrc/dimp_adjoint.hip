// dimp_adjoint.hip -- vector-Jacobian products of the split step (2-D, two
// materials, no reactive mixture, van Albada limiter).
//
// Sweep adjoint: one wave per 54-cell segment of a line along the sweep axis,
// one cell per lane at positions seg*54 + lane - 5.  Every lane recomputes the
// forward sweep exactly as the forward kernels do (same stage functions, same
// decisions), then the reverse runs stage by stage, exchanging adjoints with
// the neighbouring lanes by shuffles:
//   update -> faces (the left face of a lane is its own; the right face's
//   adjoint comes from the next lane) -> edges -> slopes, candidates ->
//   primitive state -> conserved state.
// An output depends on the cells within 2 of it, and the forward is exact on
// lanes 3..60, so the adjoints of lanes 5..58 are complete: those lanes own
// their cells, write them once, and count the parameter contributions of
// their stage instances once (no atomics; the result is deterministic).
// Transmissive boundaries: ghost positions carry no output adjoint, and the
// adjoints that reach them (clamped copies of the boundary cell) are folded
// into the boundary cell.  The interface normal's transverse neighbours get
// their adjoint through two per-cell buffers and a gather pass.
#include <hip/hip_runtime.h>

#include "dimp_adjoint.hpp"
#include "dimp_internal.hpp"

namespace dimp {

namespace {

using adj::F2;
using adj::L2;
using adj::PBar;
using adj::PB_N;
constexpr int AOUT = 54, AHALO = 5;

template <int DIR>
__device__ __forceinline__ int64_t cell_at(const Params& P, int64_t along, int64_t trans) {
  return DIR == 0 ? trans * P.n[0] + along : along * P.n[0] + trans;
}

__device__ __forceinline__ double shup(double v, int d) { return d == 1 ? from_left_keep(v) : __shfl_up(v, d, 64); }
__device__ __forceinline__ double shdn(double v, int d) { return d == 1 ? from_right_keep(v) : __shfl_down(v, d, 64); }

// sum the 12 parameter adjoints over the block into part[blockIdx][12]
__device__ __forceinline__ void block_param_sum(const PBar& pb, double* part) {
  __shared__ double red[4][12];
  double v[12];
#pragma unroll
  for (int l = 0; l < 2; ++l)
#pragma unroll
    for (int k = 0; k < 6; ++k) v[6 * l + k] = pb.v[l][k];
#pragma unroll
  for (int k = 0; k < 12; ++k)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 12; ++k) red[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x < 12) {
    const int nw = blockDim.x >> 6;
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q][threadIdx.x];
    part[(int64_t)blockIdx.x * 12 + threadIdx.x] = s;
  }
}

// Three phases, so that no forward intermediate stays live across the
// reverse (the whole forward + reverse in one live range needed ~700 doubles
// per lane and spilled to scratch memory):
//   1. forward to the faces: primitive state, candidates, edges, face flux
//      of the lane's left face (the conserved state is parked in LDS);
//   2. face reverse: update and face-flux adjoints, giving the bars of the
//      edge states; the conserved-state bar of the update and the parameter
//      bars so far go to LDS;
//   3. cell reverse: the primitive state and the candidates are recomputed
//      from the parked conserved state (a compiler barrier keeps them from
//      being merged with phase 1's), then edges -> candidates -> primitive
//      -> conserved.
template <int DIR>
__global__ __launch_bounds__(256) void k_sweep_adj(Params P, const double* __restrict__ U_in,
                                                   const double* __restrict__ lam_out, double* __restrict__ lam_in,
                                                   double* __restrict__ tang, double* __restrict__ part, double nu,
                                                   int64_t nseg, int64_t nwaves) {
  using L = L2;
  constexpr int F = F2;
  constexpr int TD = 1 - DIR;
  __shared__ double sU[F * 256];        // conserved state
  __shared__ double sUb[(F + 1) * 256];  // conserved-state bar of the update, and irho0's bar
  __shared__ double sPb[2 * PB_N * 256];  // parameter bars of phase 2
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // y: blocks are dealt round-robin over the 8 XCDs (each with its own L2);
  // within every full run of 32 blocks, the four blocks on one XCD take
  // consecutive virtual ids, so one segment of 16 adjacent lines (the 16
  // doubles of a cache line) is read through one L2 (221 -> 183 us on a
  // 512x512 grid).  A last partial run keeps the identity (the map stays
  // one-to-one).  The same placement in x measured no change.
  int64_t vb = blockIdx.x;
  if (DIR == 1 && vb < (int64_t)(gridDim.x / 32) * 32) {
    const int64_t j = vb % 32;
    vb = vb - j + (j % 8) * 4 + j / 8;
  }
  const int64_t wv = (vb * blockDim.x + tid) >> 6;
  const bool live = wv < nwaves;  // whole waves; every thread still joins the block sum
  PBar pb;
  adj::pbar_zero(pb);
  if (live) {
    const int64_t nA = P.n[DIR], nT = P.n[TD];
    const bool periodic = P.bc[DIR] == BC_PERIODIC;
    // x: a block's four waves are four segments of one line (contiguous).
    // y: sixteen consecutive waves (four virtual blocks) are one segment of
    // sixteen adjacent lines (columns), so their loads share cache lines; a
    // last group of fewer than sixteen lines takes its g lines the same way
    // (a one-to-one map of wv onto (line, seg) in both cases)
    int64_t line, seg;
    if (DIR == 0) {
      line = wv / nseg;
      seg = wv % nseg;
    } else {
      constexpr int64_t G = 16;
      const int64_t grp = wv / (G * nseg), base = grp * G;
      const int64_t g = nT - base < G ? nT - base : G;
      const int64_t rem = wv - grp * G * nseg;
      seg = rem / g;
      line = base + rem % g;
    }
    const int64_t x = seg * AOUT + lane - AHALO;
    const bool inside = x >= 0 && x < nA;
    const int64_t xm = bc_map(x, nA, P.bc[DIR]);
    const int64_t E = P.ncell;
    const int64_t cell = cell_at<DIR>(P, xm, line);
    double phi_t[3];
    phi_t[0] = U_in[cell_at<DIR>(P, xm, bc_map(line - 1, nT, P.bc[TD]))];
    phi_t[2] = U_in[cell_at<DIR>(P, xm, bc_map(line + 1, nT, P.bc[TD]))];
    // the interface normal's stencil st[x][y] from phi_t and its neighbours
    auto stencil = [&](double st[3][3]) {
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double v0 = from_left_keep(phi_t[b]), v2 = from_right_keep(phi_t[b]);
        if (DIR == 0) {
          st[0][b] = v0; st[1][b] = phi_t[b]; st[2][b] = v2;
        } else {
          st[b][0] = v0; st[b][1] = phi_t[b]; st[b][2] = v2;
        }
      }
    };
    // primitive state, its neighbours and the candidates of the lane and
    // its neighbours, from the parked conserved state
    auto forward_cells = [&](double* W, double* Wm, double* Wp, double& irho0, double& rc2, Cand& cm, Cand& c0,
                             Cand& cp, double st[3][3]) {
      double U[F];
      asm volatile("" ::: "memory");  // re-read LDS; recompute rather than keep phase-1 values live
#pragma unroll
      for (int f = 0; f < F; ++f) U[f] = sU[f * 256 + tid];
      Thermo<2, false> T;
      double H[6], J2;
      cons_to_prim<2, 2, false>(P, U, W, T, H, J2);
      irho0 = T.irho;
      rc2 = T.rho * T.c2;
#pragma unroll
      for (int f = 0; f < F; ++f) {
        Wm[f] = from_left_keep(W[f]);
        Wp[f] = from_right_keep(W[f]);
      }
      stencil(st);
      auto normal = [&]() -> double { return youngs2(st, P.dx, DIR); };
      c0 = phi_candidates<2, 2, false>(P, Wm[0], W[0], Wp[0], normal);
      cm.mL = from_left_keep(c0.mL); cm.mR = from_left_keep(c0.mR); cm.tL = from_left_keep(c0.tL); cm.tR = from_left_keep(c0.tR);
      cp.mL = from_right_keep(c0.mL); cp.mR = from_right_keep(c0.mR); cp.tL = from_right_keep(c0.tL); cp.tR = from_right_keep(c0.tR);
    };
    // ownership
    const bool window = lane >= AHALO && lane < AHALO + AOUT;
    bool own;
    if (periodic)
      own = window && inside;
    else
      own = (window && inside) || (x >= -2 && x < 0) || (x >= nA && x < nA + 2);
    const bool own_face = periodic ? (window && inside) : ((window && inside) || x == nA);

    // ------------------------------------------------ 1. forward to the faces
    {
      double U[F];
#pragma unroll
      for (int f = 0; f < F; ++f) {
        U[f] = U_in[f * E + cell];
        sU[f * 256 + tid] = U[f];
      }
      phi_t[1] = U[0];
    }
    double WL[F], WRm[F], irho0;
    FaceV<2, 2, false> fa;
    {
      double W[F], Wm[F], Wp[F], rc2, st[3][3];
      Cand cm, c0, cp;
      forward_cells(W, Wm, Wp, irho0, rc2, cm, c0, cp, st);
      double WR[F];
      edges_predict<2, 2, false, DIR>(P, Wm, W, Wp, irho0, rc2, cm, c0, cp, nu, WL, WR);
#pragma unroll
      for (int f = 0; f < F; ++f) WRm[f] = from_left_keep(WR[f]);
      face_flux<2, 2, false, DIR>(P, WRm, WL, fa);
    }
    // ---------------------------------------------------- 2. face reverse
    double WLb[F], WRb[F];
    {
      FaceV<2, 2, false> fb;
#pragma unroll
      for (int f = 0; f < F; ++f) fb.F[f] = 0.0;  // the update adjoint reads u* and the normal rows only
      fb.ustar = from_right_keep(fa.ustar);
#pragma unroll
      for (int j = 0; j < 2; ++j) fb.Vn[j] = from_right_keep(fa.Vn[j]);
      double U[F], lam[F], Ub[F];
      asm volatile("" ::: "memory");
#pragma unroll
      for (int f = 0; f < F; ++f) {
        U[f] = sU[f * 256 + tid];
        lam[f] = (inside || periodic) ? lam_out[f * E + cell] : 0.0;
        Ub[f] = 0.0;
      }
      double irb = 0.0;
      adj::FaceB fab, fbb;
#pragma unroll
      for (int f = 0; f < F; ++f) fab.F[f] = fbb.F[f] = 0.0;
      fab.ustar = fbb.ustar = 0.0;
      fab.Vn[0] = fab.Vn[1] = fbb.Vn[0] = fbb.Vn[1] = 0.0;
      adj::update_bwd(U, irho0, fa, fb, nu, lam, Ub, irb, fab, fbb);
#pragma unroll
      for (int f = 0; f < F; ++f) {
        sUb[f * 256 + tid] = Ub[f];
        fab.F[f] += from_left_keep(fbb.F[f]);
      }
      sUb[F * 256 + tid] = irb;
      fab.ustar += from_left_keep(fbb.ustar);
#pragma unroll
      for (int j = 0; j < 2; ++j) fab.Vn[j] += from_left_keep(fbb.Vn[j]);
      double WRmb[F];
#pragma unroll
      for (int f = 0; f < F; ++f) WRmb[f] = WLb[f] = 0.0;
      adj::face_bwd<DIR>(P, WRm, WL, fab, WRmb, WLb, pb, own_face);
#pragma unroll
      for (int f = 0; f < F; ++f) WRb[f] = from_right_keep(WRmb[f]);
#pragma unroll
      for (int l = 0; l < 2; ++l)
#pragma unroll
        for (int k = 0; k < PB_N; ++k) {
          sPb[(l * PB_N + k) * 256 + tid] = pb.v[l][k];
          pb.v[l][k] = 0.0;
        }
    }
    // ---------------------------------------------------- 3. cell reverse
    double W[F], Wm[F], Wp[F], irho0c, rc2, st[3][3];
    Cand cm, c0, cp;
    forward_cells(W, Wm, Wp, irho0c, rc2, cm, c0, cp, st);
    double Wmb[F], W0b[F], Wpb[F];
#pragma unroll
    for (int f = 0; f < F; ++f) Wmb[f] = W0b[f] = Wpb[f] = 0.0;
    double irbe = 0.0, rc2b = 0.0, cb[4];
    adj::edges_bwd<DIR>(P, Wm, W, Wp, irho0c, rc2, cm, c0, cp, nu, WLb, WRb, Wmb, W0b, Wpb, irbe, rc2b, cb, pb, own);
    double qmb = 0.0, q0b = 0.0, qpb = 0.0;
    double stb[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) stb[a][b] = 0.0;
    adj::cand_bwd<DIR>(P, Wm[0], W[0], Wp[0], st, cb, qmb, q0b, qpb, stb);
    // stencil adjoint in (along offset a, transverse offset b) order
    double sab[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) sab[a][b] = (DIR == 0) ? stb[a][b] : stb[b][a];
    // gather the primitive adjoint of my cell from the lanes that used it
#pragma unroll
    for (int f = 0; f < F; ++f) W0b[f] += shup(Wpb[f], 1) + shdn(Wmb[f], 1);
    W0b[0] += q0b + shup(qpb, 1) + shdn(qmb, 1);
    W0b[0] += sab[1][1] + shup(sab[2][1], 1) + shdn(sab[0][1], 1);
    double Tm = sab[1][0] + shup(sab[2][0], 1) + shdn(sab[0][0], 1);
    double Tp = sab[1][2] + shup(sab[2][2], 1) + shdn(sab[0][2], 1);
    double U[F], Ub[F];
    asm volatile("" ::: "memory");
#pragma unroll
    for (int f = 0; f < F; ++f) {
      U[f] = sU[f * 256 + tid];
      Ub[f] = sUb[f * 256 + tid];
    }
    const double irb = sUb[F * 256 + tid];
    adj::c2p_bwd(P, U, W0b, irb + irbe, rc2b, Ub, pb, own);
    // transmissive: fold the ghost positions into the boundary cells
    if (!periodic) {
      double fold[F], tm2 = 0.0, tp2 = 0.0;
#pragma unroll
      for (int f = 0; f < F; ++f) fold[f] = 0.0;
#pragma unroll
      for (int d = 1; d <= 2; ++d) {
        const bool left = (x == 0);
        const bool right = (x == nA - 1);
#pragma unroll
        for (int f = 0; f < F; ++f) {
          const double a = shup(Ub[f], d), b = shdn(Ub[f], d);
          fold[f] += (left ? a : 0.0) + (right ? b : 0.0);
        }
        const double ta = shup(Tm, d), tb = shdn(Tm, d), pa = shup(Tp, d), pbv = shdn(Tp, d);
        tm2 += (left ? ta : 0.0) + (right ? tb : 0.0);
        tp2 += (left ? pa : 0.0) + (right ? pbv : 0.0);
      }
#pragma unroll
      for (int f = 0; f < F; ++f) Ub[f] += fold[f];
      Tm += tm2;
      Tp += tp2;
    }
    if (window && inside) {
#pragma unroll
      for (int f = 0; f < F; ++f) lam_in[f * E + cell] = Ub[f];
      tang[cell] = Tm;
      tang[E + cell] = Tp;
    }
#pragma unroll
    for (int l = 0; l < 2; ++l)
#pragma unroll
      for (int k = 0; k < PB_N; ++k) pb.v[l][k] += sPb[(l * PB_N + k) * 256 + tid];
  }
  block_param_sum(pb, part);
}

// lam_in[phi] += the interface-normal adjoints written by the transverse
// neighbours: Tm(s) targets the cell at s - 1, Tp(s) the cell at s + 1
template <int DIR>
__global__ void k_tang_gather(Params P, const double* __restrict__ tang, double* __restrict__ lam_in) {
  constexpr int TD = 1 - DIR;
  const int64_t E = P.ncell;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= E) return;
  const int64_t i = c % P.n[0], j = c / P.n[0];
  const int64_t along = DIR == 0 ? i : j, t = DIR == 0 ? j : i;
  const int64_t nT = P.n[TD];
  const int bc = P.bc[TD];
  int64_t src[3];
  int ns = 0;
  for (int d = -1; d <= 1; ++d) {
    int64_t s = t + d;
    if (bc == BC_PERIODIC) {
      s = bc_map(s, nT, bc);
    } else if (s < 0 || s >= nT) {
      continue;
    }
    bool dup = false;
    for (int q = 0; q < ns; ++q) dup = dup || (src[q] == s);
    if (!dup) src[ns++] = s;
  }
  double acc = 0.0;
  for (int q = 0; q < ns; ++q) {
    const int64_t s = src[q];
    const int64_t cs = cell_at<DIR>(P, along, s);
    if (bc_map(s - 1, nT, bc) == t) acc += tang[cs];
    if (bc_map(s + 1, nT, bc) == t) acc += tang[E + cs];
  }
  lam_in[c] += acc;
}

__global__ __launch_bounds__(256) void k_plastic_adj(Params P, const double* __restrict__ U_pre,
                                                     const double* __restrict__ lam_out,
                                                     double* __restrict__ lam_in, double* __restrict__ part) {
  constexpr int F = F2;
  const int64_t E = P.ncell;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  PBar pb;
  adj::pbar_zero(pb);
  if (c < E) {
    double U[F], lam[F], Ub[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      U[f] = U_pre[f * E + c];
      lam[f] = lam_out[f * E + c];
    }
    adj::plastic_bwd(P, U, lam, Ub, pb, true);
#pragma unroll
    for (int f = 0; f < F; ++f) lam_in[f * E + c] = Ub[f];
  }
  block_param_sum(pb, part);
}

// dparams[k] += sum over blocks of part[b][k].  The partial sums are read as
// one flat array, element e = 12 b + k: thread t takes e = t, t + 768, ...
// (coalesced; 768 is a multiple of 12, so every element a thread reads is
// parameter t % 12), sixteen loads in flight into sixteen accumulators (one
// block is latency bound: a 512x512 step's 43k partial sums take four rounds
// of loads), summed pairwise; then thread k adds, in thread order, the 64
// threads' sums of parameter k.  The grouping is fixed: the result is the
// same on every run.
__global__ __launch_bounds__(768) void k_param_total(const double* __restrict__ part, int64_t nblk,
                                                     double* __restrict__ dparams) {
  constexpr int T = 768, U = 16;
  __shared__ double red[T];
  const int t = threadIdx.x;
  const int64_t ne = nblk * 12;
  double a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = 0.0;
  // unconditional loads at clamped (in-range) positions, so all sixteen are
  // issued before the first wait; positions past the end add zero
  for (int64_t e = t; e < ne; e += (int64_t)U * T) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = part[min(e + (int64_t)u * T, ne - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] += (e + (int64_t)u * T < ne) ? v[u] : 0.0;
  }
#pragma unroll
  for (int w = U / 2; w >= 1; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) a[u] += a[u + w];
  red[t] = a[0];
  __syncthreads();
  if (t < 12) {
    double s = 0.0;
    for (int q = t; q < T; q += 12) s += red[q];
    dparams[t] += s;
  }
}

}  // namespace

int64_t adjoint_sweep_blocks(const Params& P, int dir) {
  const int64_t nA = P.n[dir], nT = P.n[1 - dir];
  const int64_t nseg = (nA + AOUT - 1) / AOUT;
  return (nT * nseg + 3) / 4;
}

int64_t adjoint_cell_blocks(const Params& P) { return (P.ncell + 255) / 256; }

hipError_t launch_sweep_adjoint(const Params& P, int dir, const double* U_in, const double* lam_out,
                                double* lam_in, double* tang, double* part, double* dparams, double dt,
                                hipStream_t st) {
  const int64_t nA = P.n[dir], nT = P.n[1 - dir];
  const int64_t nseg = (nA + AOUT - 1) / AOUT;
  const int64_t nwaves = nT * nseg;
  const int64_t nblk = (nwaves + 3) / 4;
  const double nu = dt / P.dx[dir];
  if (dir == 0)
    hipLaunchKernelGGL(k_sweep_adj<0>, dim3((unsigned)nblk), dim3(256), 0, st, P, U_in, lam_out, lam_in, tang, part,
                       nu, nseg, nwaves);
  else
    hipLaunchKernelGGL(k_sweep_adj<1>, dim3((unsigned)nblk), dim3(256), 0, st, P, U_in, lam_out, lam_in, tang, part,
                       nu, nseg, nwaves);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned g = (unsigned)((P.ncell + 255) / 256);
  if (dir == 0)
    hipLaunchKernelGGL(k_tang_gather<0>, dim3(g), dim3(256), 0, st, P, tang, lam_in);
  else
    hipLaunchKernelGGL(k_tang_gather<1>, dim3(g), dim3(256), 0, st, P, tang, lam_in);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return dparams ? launch_param_total(part, nblk, dparams, st) : hipSuccess;
}

hipError_t launch_plastic_adjoint(const Params& P, const double* U_pre, const double* lam_out, double* lam_in,
                                  double* part, double* dparams, hipStream_t st) {
  const int64_t nblk = (P.ncell + 255) / 256;
  hipLaunchKernelGGL(k_plastic_adj, dim3((unsigned)nblk), dim3(256), 0, st, P, U_pre, lam_out, lam_in, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return dparams ? launch_param_total(part, nblk, dparams, st) : hipSuccess;
}

hipError_t launch_param_total(const double* part, int64_t nblk, double* dparams, hipStream_t st) {
  hipLaunchKernelGGL(k_param_total, dim3(1), dim3(768), 0, st, part, nblk, dparams);
  return hipGetLastError();
}

}  // namespace dimp
