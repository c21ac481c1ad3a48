// dimp_patches_n3.hip -- the patch-set sweeps of three materials, with and
// without a history slot.
#include "dimp_patches.hpp"

namespace dimp {

hipError_t launch_patch_sweep_n3(const Params& P, int rx, const PatchGeo* geo, WorkList wl, int64_t w0,
                                 int64_t nwork, const double* in, double* out, double dt, const double* dtp, int dir,
                                 bool fuse, double* part, int row_wpb, int cw, hipStream_t st) {
  if (rx == 0) return launch_patch_t<3, 0>(P, geo, wl, w0, nwork, in, out, dt, dtp, dir, fuse, part, row_wpb, cw, st);
  if (rx == 1) return launch_patch_t<3, 1>(P, geo, wl, w0, nwork, in, out, dt, dtp, dir, fuse, part, row_wpb, cw, st);
  if (rx == 2) return launch_patch_t<3, 2>(P, geo, wl, w0, nwork, in, out, dt, dtp, dir, fuse, part, row_wpb, cw, st);
  return hipErrorInvalidValue;
}

}  // namespace dimp
