// dimp_internal.hpp -- launchers shared by the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "dimp_device.hpp"

namespace dimp {

// march length of the column sweeps (cells per thread along y or z)
constexpr int COL_SEGMENT = 16;

hipError_t launch_sweep(const Params& P, int D, bool rx, const double* in, double* out, double dt,
                        const double* dtp, int dir, bool fuse, unsigned long long* smax, int S, hipStream_t st);
hipError_t launch_cfl_dt(const Params& P, int D, const unsigned long long* smax, double cfl, double* dt,
                         double* log, int64_t idx, hipStream_t st);
hipError_t launch_prim_to_cons(const Params& P, int D, bool rx, const double* W, double* U, hipStream_t st);
hipError_t launch_cons_to_prim(const Params& P, int D, bool rx, const double* U, double* W, hipStream_t st);
hipError_t launch_sources(const Params& P, int D, bool rx, double* U, double dt, hipStream_t st);
hipError_t launch_wavespeed(const Params& P, int D, bool rx, const double* U, unsigned long long* smax,
                            hipStream_t st);
hipError_t launch_check(const Params& P, int D, bool rx, const double* U, unsigned long long* nbad, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
hipError_t launch_u64_to_f64(const unsigned long long* p, double* out, int n, hipStream_t st);

}  // namespace dimp
