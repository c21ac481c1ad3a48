// dimp_amr.hpp -- launchers of the two-level refinement kernels (coarse to
// fine ghost fill, the exchange between touching patches, averaging down,
// the fluxes through the coarse/fine boundary and the flux correction); see
// dimp_amr.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dimp_device.hpp"

namespace dimp {

// A refined patch over coarse cells [i0, i1) x [j0, j1) of a 2-D coarse grid
// (nxc x nyc), stored as a fine grid of (2 (i1 - i0) + 2 G) x (2 (j1 - j0) +
// 2 G) cells with G ghost layers; field-major arrays, x fastest.
struct AmrBox {
  int64_t i0, j0, i1, j1;
  int64_t nxc, nyc, nxf, nyf;
  int G, F;
};

// fine ghost cells <- coarse level at time weight w (old + w (new - old)),
// linear inside the parent with minmod-limited slopes; with all set, every
// fine cell <- its parent's state (a new patch)
hipError_t launch_amr_fill(const AmrBox& b, const double* cold, const double* cnew, double w, double* fine,
                           hipStream_t st, bool all = false);

// Field slots of a primitive state for the refinement criterion: volume
// fractions [0, nphi), phasic densities [rho0, rho0 + nmat), velocities
// [u0, u0 + ndim), pressure p; floors per kind (phi, rho, u, p).
struct TagLayout {
  int nphi, rho0, nmat, u0, ndim, p;
  int64_t nx, ny;
  double floor_phi, floor_rho, floor_u, floor_p;
};
// tags[c] = 1 where a refinement variable changes by more than threshold (as
// a fraction) to a face neighbour; bbox (4 unsigned: min i, min j, max i,
// max j, preset by the caller) receives the tagged cells' extent
hipError_t launch_amr_tag(const TagLayout& t, const double* prim, double threshold, unsigned char* tags,
                          unsigned long long* bbox, hipStream_t st);
// fine-to-fine exchange between two patches of one level (same coarse grid,
// disjoint boxes): the stored cells of patch p (state dst) that lie in patch
// q's interior <- q's values (state src); nothing where they do not meet
hipError_t launch_amr_exchange(const AmrBox& p, const AmrBox& q, const double* src, double* dst, hipStream_t st);
// covered coarse cells <- mean of their four fine children
hipError_t launch_amr_average(const AmrBox& b, const double* fine, double* coarse, hipStream_t st);


// Faces of a level normal to one axis: those at index pos[0] and pos[1]
// along the axis (face k is the left face of cell k) for the transverse cells
// t0 .. t0 + len - 1.  Their fluxes are stored field-major as [F][2][len].
struct FaceSet {
  int64_t pos[2];
  int64_t t0, len;
};
// The fluxes of the split sweep along dir (MUSCL-Hancock with time step dt,
// the state in) through the faces of fs, on a 2-D grid of two or three materials (rx:
// the kernel variant of the reactive model); with rk, those of the unsplit
// operator's direction dir (edges without the predictor).  Stored times wgt,
// or added to the stored values with acc.  Each face's stencil (3 cells
// before it, 2 after, 1 across) must lie inside the grid:
// hipErrorInvalidValue otherwise.
hipError_t launch_amr_flux(const Params& P, int rx, int dir, const FaceSet& fs, const double* in, double dt,
                           double* flux, hipStream_t st, bool rk = false, double wgt = 1.0, bool acc = false);
// Flux correction of the coarse cells sharing a face with the patch: for the
// fields [c0, c1), U += -/+ (dt / dx) (Fbar - Fc) on the low/high side, Fc
// the coarse flux and Fbar the mean of the two fine faces' fluxes over the two
// fine steps (fc[dir]: [F][2][len] over the patch's coarse faces, ff[s][dir]:
// over its fine faces in fine step s)
hipError_t launch_amr_reflux(const AmrBox& b, int c0, int c1, const double lam[2], const double* const fc[2],
                             const double* const ff0[2], const double* const ff1[2], double* coarse,
                             hipStream_t st);

}  // namespace dimp
