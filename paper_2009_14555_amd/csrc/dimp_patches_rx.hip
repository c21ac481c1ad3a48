// dimp_patches_rx.hip -- the two-material patch-set sweeps with a history
// slot: a gas mixture or a Johnson-Cook solid (RX = 1) and a JWL mixture
// (RX = 2).
#include "dimp_patches.hpp"

namespace dimp {

hipError_t launch_patch_sweep_rx(const Params& P, int rx, const PatchGeo* geo, WorkList wl, int64_t w0,
                                 int64_t nwork, const double* in, double* out, double dt, const double* dtp, int dir,
                                 bool fuse, double* part, int row_wpb, int cw, hipStream_t st) {
  if (rx == 1) return launch_patch_t<2, 1>(P, geo, wl, w0, nwork, in, out, dt, dtp, dir, fuse, part, row_wpb, cw, st);
  if (rx == 2) return launch_patch_t<2, 2>(P, geo, wl, w0, nwork, in, out, dt, dtp, dir, fuse, part, row_wpb, cw, st);
  return hipErrorInvalidValue;
}

}  // namespace dimp
