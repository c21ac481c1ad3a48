// dimp_sweeps3.hip -- the sweeps of 3-D grids (instantiated from
// dimp_sweeps.hpp in a unit of their own so that the 1-D/2-D and 3-D kernels
// compile in parallel).
#include <hip/hip_runtime.h>

#include "dimp_sweeps.hpp"

namespace dimp {

hipError_t launch_sweep3(const Params& P, int rx, const double* in, double* out, double dt, const double* dtp,
                         int dir, bool fuse, double* part, int S, hipStream_t st) {
  return rx == 2 ? launch_sweep_t<3, 2, 2>(P, in, out, dt, dtp, dir, fuse, part, S, st)
         : rx    ? launch_sweep_t<3, 2, 1>(P, in, out, dt, dtp, dir, fuse, part, S, st)
                 : launch_sweep_t<3, 2, 0>(P, in, out, dt, dtp, dir, fuse, part, S, st);
}

hipError_t launch_rk_sweep3(const Params& P, int rx, int dir, int mode, int stage, bool fuse, const double* in,
                            double* out, const double* Rin, const double* qn, double dt, const double* dtp,
                            double* part, hipStream_t st) {
  return rx == 2 ? launch_rk_t<3, 2, 2>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st)
         : rx    ? launch_rk_t<3, 2, 1>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st)
                 : launch_rk_t<3, 2, 0>(P, dir, mode, stage, fuse, in, out, Rin, qn, dt, dtp, part, st);
}

}  // namespace dimp
