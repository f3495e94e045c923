// Host-side launch interface of the solver kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "lsfft_internal.hpp"

namespace lsfft {

struct LaunchArgs {
  dim3 grid;
  size_t lds;
  hipStream_t stream;
  const InstDesc* desc;
  InstState* state;
  const WorkItem* items;
  const int* count;       // device pointer to the number of items
  const double* lame;     // device Lame table, pairs (lambda, mu)
  const void* tw;         // device twiddle table in the plan precision
};

// kind 0: x pass (len = nx); kind 1: strided pass (len = ny or nz).
// Returns the LDS bytes of one work item (0 if unsupported) and the rows or
// pencils per tile.
size_t query_geometry(bool f64, int kind, int len, int* per_tile);

hipError_t launch_xpass_f32(const LaunchArgs& a, int mode);
hipError_t launch_xpass_f64(const LaunchArgs& a, int mode);
hipError_t launch_ypass_f32(const LaunchArgs& a, int dir, int which, int extra, int gate);
hipError_t launch_ypass_f64(const LaunchArgs& a, int dir, int which, int extra, int gate);
hipError_t launch_green_f32(const LaunchArgs& a, int mode);
hipError_t launch_green_f64(const LaunchArgs& a, int mode);

hipError_t launch_xpass(bool f64, const LaunchArgs& a, int mode);
hipError_t launch_ypass(bool f64, const LaunchArgs& a, int dir, int which, int extra, int gate);
hipError_t launch_green(bool f64, const LaunchArgs& a, int mode);
hipError_t launch_cg_update(bool f64, const LaunchArgs& a);
hipError_t launch_reduce(const LaunchArgs& a, const int* inst_list, int ninst, int mode);
hipError_t launch_phase_max(const uint8_t* phase, long long n, int* out, hipStream_t s);
hipError_t launch_accumulate(bool f64, int dim, const LaunchArgs& a, const GroupDesc* groups, int g, long long nvox);
hipError_t launch_scale(double* a, long long n, double s, hipStream_t st);

}  // namespace lsfft
