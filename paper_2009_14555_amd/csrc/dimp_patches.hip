// dimp_patches.hip -- the patch-set sweeps of two materials without a history
// slot, and the dispatch over the layouts (the RX = 1, 2 instances live in
// dimp_patches_rx.hip, the three-material ones in dimp_patches_n3.hip).
#include "dimp_patches.hpp"

namespace dimp {

hipError_t launch_patch_sweep(const Params& P, int rx, const PatchGeo* geo, WorkList wl, int64_t w0, int64_t nwork,
                              const double* in, double* out, double dt, const double* dtp, int dir, bool fuse,
                              double* part, int row_wpb, int cw, hipStream_t st) {
  if (P.nmat == 3)
    return launch_patch_sweep_n3(P, rx, geo, wl, w0, nwork, in, out, dt, dtp, dir, fuse, part, row_wpb, cw, st);
  if (P.nmat != 2) return hipErrorInvalidValue;
  if (rx == 0)
    return launch_patch_t<2, 0>(P, geo, wl, w0, nwork, in, out, dt, dtp, dir, fuse, part, row_wpb, cw, st);
  return launch_patch_sweep_rx(P, rx, geo, wl, w0, nwork, in, out, dt, dtp, dir, fuse, part, row_wpb, cw, st);
}

}  // namespace dimp
