// dimp_lane.hpp -- the stages of one sweep for a wave holding one cell per lane.
#pragma once
#include "dimp_stencil.hpp"

namespace dimp {

// ------------------------------------------------- lane-per-cell sweep
// The stages of one sweep for a wave whose 64 lanes hold 64 consecutive cells
// along the sweep axis (3 halo cells on each side, lanes 3..60 are written).
// U: the lane's conserved state; phi_t[b][c]: phi_1 of the lane's cell at
// transverse offsets (b, c) in {-1,0,1}^2 (2-D uses c = 1 only), with the
// offset along the sweep axis supplied by shuffles.
// U is read twice through load_U (for the primitive state and for the
// update) rather than kept in registers across the face computation.
// RK = false: the split MUSCL-Hancock sweep, Un = the updated state (and, with
// FUSE, the source steps and the wave speed s of the result).  RK = true: the
// direction's part of the unsplit operator of Sec. 3.1, Un = D_dir(q) with
// nu = 1/dx (edges without the predictor; FUSE is left to the caller).
//
// lane_face: the stages up to the flux through the face on the left of the
// lane's cell (fa; wall: that face is a reflective wall), and the cell's
// 1 / (sum of partial densities); it depends on the cells 3 to the left and
// 2 to the right.  lane_sweep adds the update.
template <int D, int N, int RX, int DIR, bool RK, class LoadU>
__device__ __forceinline__ void lane_face(const Params& P, LoadU&& load_U, const double (&phi_t)[3][3], double nu,
                                          FaceV<D, N, RX>& fa, double& irho0, bool wall) {
  using L = Lay<D, N, RX>;
  constexpr int F = L::F;
  double W[F];
  double rc2;
  {
    double U[F];
    load_U(U);
    Thermo<N, RX> T;
    double H[6], J2;
    cons_to_prim<D, N, RX>(P, U, W, T, H, J2);
    irho0 = T.irho;  // 1 / sum of partial densities
    rc2 = T.rho * T.c2;
  }
  double Wm[F], Wp[F];
#pragma unroll
  for (int f = 0; f < F; ++f) {
    Wm[f] = from_left(W[f]);
    Wp[f] = from_right(W[f]);
  }
  // phi stencil along the sweep axis for the interface normal (all lanes
  // shuffle; the normal itself is only evaluated in mixed cells)
  double sm[3][3], sp[3][3];
  if (P.thinc && D >= 2) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (D == 2 && c != 1) continue;
        sm[b][c] = from_left(phi_t[b][c]);
        sp[b][c] = from_right(phi_t[b][c]);
      }
  }
  auto normal = [&]() -> double {
    if (D == 1) return 1.0;
    if (D == 2) {
      // axes (x, y): the sweep axis DIR and the transverse offset b
      double st[3][3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double v0 = sm[b][1], v1 = phi_t[b][1], v2 = sp[b][1];
        if (DIR == 0) {
          st[0][b] = v0; st[1][b] = v1; st[2][b] = v2;
        } else {
          st[b][0] = v0; st[b][1] = v1; st[b][2] = v2;
        }
      }
      return youngs2(st, P.dx, DIR);
    }
    // 3-D: transverse offsets (b, c) run over the two other axes in order
    double st[3][3][3];
    constexpr int o1 = (DIR == 0) ? 1 : 0, o2 = (DIR == 2) ? 1 : 2;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v[3] = {sm[b][c], phi_t[b][c], sp[b][c]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          int idx[3];
          idx[DIR] = a;
          idx[o1] = b;
          idx[o2] = c;
          st[idx[0]][idx[1]][idx[2]] = v[a];
        }
      }
    return youngs3(st, P.dx, DIR);
  };
  // candidates of every stored volume fraction, all with the normal of the
  // first; the neighbours' right (left) edge candidates by shifts
  CandSet<N> c0, cm, cp;
#pragma unroll
  for (int l = 0; l < N - 1; ++l) {
    c0.c[l] = phi_candidates<D, N, RX>(P, Wm[l], W[l], Wp[l], normal);
    cm.c[l].mR = from_left(c0.c[l].mR);
    cm.c[l].tR = from_left(c0.c[l].tR);
    cp.c[l].mL = from_right(c0.c[l].mL);
    cp.c[l].tL = from_right(c0.c[l].tL);
  }
  double WL[F], WR[F];
  if (RK) {
    (void)rc2;
    edges_muscl<D, N, RX>(P, Wm, W, Wp, cm, c0, cp, WL, WR);
  } else {
    edges_predict<D, N, RX, DIR>(P, Wm, W, Wp, irho0, rc2, cm, c0, cp, nu, WL, WR);
  }
  // face on the left of this cell: right edge of the left neighbour | my left edge
  double WRm[F];
#pragma unroll
  for (int f = 0; f < F; ++f) WRm[f] = from_left(WR[f]);
  face_flux<D, N, RX, DIR>(P, WRm, WL, fa, wall);
}

template <int D, int N, int RX, int DIR, bool FUSE, bool RK = false, class LoadU>
__device__ __forceinline__ void lane_sweep(const Params& P, LoadU&& load_U, const double (&phi_t)[3][3], double nu,
                                           double dt, bool writer, double* Un, double* s, bool wall = false) {
  constexpr int F = Lay<D, N, RX>::F;
  FaceV<D, N, RX> fa, fb;
  double irho0;
  lane_face<D, N, RX, DIR, RK>(P, load_U, phi_t, nu, fa, irho0, wall);
#pragma unroll
  for (int f = 0; f < F; ++f) fb.F[f] = from_right(fa.F[f]);
  fb.ustar = from_right(fa.ustar);
#pragma unroll
  for (int j = 0; j < D; ++j) fb.Vn[j] = from_right(fa.Vn[j]);
  {
    double U[F];
    load_U(U);
    if (RK)
      div_cell<D, N, RX, DIR>(U, irho0, fa, fb, nu, Un);
    else
      update_cell<D, N, RX, DIR>(U, irho0, fa, fb, nu, Un);
  }
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = 0.0;
  if (FUSE && !RK && writer) epilogue_cell<D, N, RX>(P, Un, dt, s);
}

}  // namespace dimp
