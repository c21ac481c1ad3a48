// dimp_internal.hpp -- launchers shared by the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "dimp_device.hpp"
#include "dimp_pack.hpp"

namespace dimp {

// march length of the column sweeps (unused by the tile kernels)
constexpr int COL_SEGMENT = 16;

// patch sets: ghost layers stored around every patch, and the patch table
constexpr int PATCH_GHOST = 2;
struct PatchGeo {
  int64_t off;     // element index of cell (-PATCH_GHOST, -PATCH_GHOST)
  int32_t nx, ny;  // interior cells
};

// Packed work list of a patch set on the device (segments packed by
// pack_lines): work item k (one wave of the x sweep, one tile of the y sweep)
// holds segments [beg[k], beg[k+1]).
struct WorkList {
  const int4* seg;
  const int32_t* beg;
};

// part: per-item wave-speed slots, indexed by the global work item (x) or
// item * cw + wave (y), so per-patch launches of sub-ranges never collide
// rx: the layout's history slot (0 none, 1 a gas mixture or a Johnson-Cook
// solid, 2 a JWL mixture)
hipError_t launch_patch_sweep(const Params& P, int rx, const PatchGeo* geo, WorkList wl, int64_t w0, int64_t nwork,
                              const double* in, double* out, double dt, const double* dtp, int dir, bool fuse,
                              double* part, int row_wpb, int cw, hipStream_t st);
// the three-material instances (dimp_patches_n3.hip)
hipError_t launch_patch_sweep_n3(const Params& P, int rx, const PatchGeo* geo, WorkList wl, int64_t w0,
                                 int64_t nwork, const double* in, double* out, double dt, const double* dtp, int dir,
                                 bool fuse, double* part, int row_wpb, int cw, hipStream_t st);
// the two-material rx = 1, 2 instances (dimp_patches_rx.hip)
hipError_t launch_patch_sweep_rx(const Params& P, int rx, const PatchGeo* geo, WorkList wl, int64_t w0,
                                 int64_t nwork, const double* in, double* out, double dt, const double* dtp, int dir,
                                 bool fuse, double* part, int row_wpb, int cw, hipStream_t st);

// adjoint (2-D, two materials, no reactive mixture): blocks of the sweep and
// cell kernels (sizes of the per-block parameter partial sums), launchers
int64_t adjoint_sweep_blocks(const Params& P, int dir);
int64_t adjoint_cell_blocks(const Params& P);
hipError_t launch_sweep_adjoint(const Params& P, int dir, const double* U_in, const double* lam_out,
                                double* lam_in, double* tang, double* part, double* dparams, double dt,
                                hipStream_t st);
hipError_t launch_plastic_adjoint(const Params& P, const double* U_pre, const double* lam_out, double* lam_in,
                                  double* part, double* dparams, hipStream_t st);
// the sweep and plastic launchers add their blocks' parameter partial sums
// (12 doubles a block) to dparams, or leave them in part when dparams is
// null; this adds nblk blocks' partial sums to dparams (fixed order)
hipError_t launch_param_total(const double* part, int64_t nblk, double* dparams, hipStream_t st);

// the 3-D sweeps (dimp_sweeps3.hip), called by launch_sweep and
// launch_rk_sweep for D = 3
hipError_t launch_sweep3(const Params& P, int rx, const double* in, double* out, double dt, const double* dtp,
                         int dir, bool fuse, double* part, int S, hipStream_t st);
hipError_t launch_rk_sweep3(const Params& P, int rx, int dir, int mode, int stage, bool fuse, const double* in,
                            double* out, const double* Rin, const double* qn, double dt, const double* dtp,
                            double* part, hipStream_t st);
// three materials on 1-D and 2-D grids (dimp_sweeps_n3.hip), called by
// launch_sweep and launch_rk_sweep when P.nmat is 3
hipError_t launch_sweep_n3(const Params& P, int D, int rx, const double* in, double* out, double dt,
                           const double* dtp, int dir, bool fuse, double* part, int S, hipStream_t st);
hipError_t launch_rk_sweep_n3(const Params& P, int D, int rx, int dir, int mode, int stage, bool fuse,
                              const double* in, double* out, const double* Rin, const double* qn, double dt,
                              const double* dtp, double* part, hipStream_t st);
hipError_t launch_sweep(const Params& P, int D, int rx, const double* in, double* out, double dt,
                        const double* dtp, int dir, bool fuse, double* part, int S, hipStream_t st);
// One directional pass of stage `stage` (1..3) of the unsplit SSP-RK3
// (Sec. 3.1), the stage being a qn + b (in - dt D(in)) with qn the step's
// initial state.  mode 1 (y, the first direction): out = a qn + b (in - dt
// D_y(in)); mode 2 (z): out = Rin - b dt D_z(in); mode 3 (x, last): out =
// Rin - b dt D_x(in) (in 1-D the whole stage); fuse (stage 3): the sources and
// the wave-speed slots of the result.
hipError_t launch_rk_sweep(const Params& P, int D, int rx, int dir, int mode, int stage, bool fuse,
                           const double* in, double* out, const double* Rin, const double* qn, double dt,
                           const double* dtp, double* part, hipStream_t st);
// per-wave wave-speed slots a fused sweep along dir writes (3 doubles each),
// and their fixed-order reduction into the wave-speed words
int64_t sweep_slots(const Params& P, int D, int dir);
// (two fixed-order stages; scratch holds reduce_smax_blocks(nslots) * 3 doubles)
// With req (dt set) the reduction also writes the next step's dt (the
// launch_cfl_dt rule, log[idx] when log is set).
struct DtReq {
  double cfl = 0.0, dx0 = 0.0, dx1 = 0.0, dx2 = 0.0;
  double* dt = nullptr;
  double* log = nullptr;
  int64_t idx = 0;
};
hipError_t launch_reduce_smax(const double* part, int64_t nslots, int D, double* scratch,
                              unsigned long long* smax, hipStream_t st, const DtReq* req = nullptr);
int64_t reduce_smax_blocks(int64_t nslots);
// dt from the wave-speed words smax[0..D-1]; a step that is not finite and
// positive becomes 0 and sets the status word smax[5]
hipError_t launch_cfl_dt(const Params& P, int D, unsigned long long* smax, double cfl, double* dt,
                         double* log, int64_t idx, hipStream_t st);
hipError_t launch_prim_to_cons(const Params& P, int D, int rx, const double* W, double* U, hipStream_t st);
hipError_t launch_cons_to_prim(const Params& P, int D, int rx, const double* U, double* W, hipStream_t st);
hipError_t launch_sources(const Params& P, int D, int rx, double* U, double dt, const double* dtp, hipStream_t st);
hipError_t launch_wavespeed(const Params& P, int D, int rx, const double* U, unsigned long long* smax,
                            hipStream_t st);
hipError_t launch_check(const Params& P, int D, int rx, const double* U, unsigned long long* nbad, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
// a rest state given a velocity field (D arrays): momentum rho u, energy
// E_rest + rho |u|^2 / 2, every other field copied; and its adjoint
hipError_t launch_with_velocity(int D, bool rx, int64_t nc, const double* rest, const double* vel, double* out,
                                hipStream_t st);
hipError_t launch_with_velocity_adj(int D, bool rx, int64_t nc, const double* rest, const double* vel,
                                    const double* a_out, double* a_rest, double* a_vel, hipStream_t st);
hipError_t launch_u64_to_f64(const unsigned long long* p, double* out, int n, hipStream_t st);

}  // namespace dimp
