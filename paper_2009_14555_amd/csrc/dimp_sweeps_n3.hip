// dimp_sweeps_n3.hip -- the sweeps of 1-D and 2-D grids holding three
// materials (instantiated from dimp_sweeps.hpp in a unit of their own, compiled
// in parallel with the two-material ones).
#include <hip/hip_runtime.h>

#include "dimp_sweeps.hpp"

namespace dimp {

hipError_t launch_sweep_n3(const Params& P, int D, int rx, const double* in, double* out, double dt,
                           const double* dtp, int dir, bool fuse, double* part, int S, hipStream_t st) {
#define DIMP_SWEEP3_RX(DD)                                                                 \
  return rx == 2 ? launch_sweep_t<DD, 3, 2>(P, in, out, dt, dtp, dir, fuse, part, S, st)   \
         : rx    ? launch_sweep_t<DD, 3, 1>(P, in, out, dt, dtp, dir, fuse, part, S, st)   \
                 : launch_sweep_t<DD, 3, 0>(P, in, out, dt, dtp, dir, fuse, part, S, st)
  if (D == 1) DIMP_SWEEP3_RX(1);
  if (D == 2) DIMP_SWEEP3_RX(2);
#undef DIMP_SWEEP3_RX
  return hipErrorInvalidValue;
}

hipError_t launch_rk_sweep_n3(const Params& P, int D, int rx, int dir, int mode, int stage, bool fuse,
                              const double* in, double* out, const double* Rin, const double* qn, double dt,
                              const double* dtp, double* part, hipStream_t st) {
#define DIMP_RK3_RX(DD)                                                                                      \
  return rx == 2 ? launch_rk_t<DD, 3, 2>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st)     \
         : rx    ? launch_rk_t<DD, 3, 1>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st)     \
                 : launch_rk_t<DD, 3, 0>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st)
  if (D == 1) DIMP_RK3_RX(1);
  if (D == 2) DIMP_RK3_RX(2);
#undef DIMP_RK3_RX
  return hipErrorInvalidValue;
}

}  // namespace dimp
