// Host-side launch interface of the solver kernels.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "lsfft_internal.hpp"

namespace lsfft {

struct LaunchArgs {
  dim3 grid;
  int block;              // threads per workgroup (precision dependent)
  size_t lds;
  hipStream_t stream;
  const InstDesc* desc;
  InstState* state;
  const WorkItem* items;
  const int* count;       // device pointer to the number of items
  const double* lame;     // device Lame table, pairs (lambda, mu)
  const void* tw;         // device twiddle table in the plan precision
  hipEvent_t ev0 = nullptr, ev1 = nullptr;   // if set: timestamps of the kernel's own start and end
  // y pass only: solves whose stopping rule the launch applies first (device
  // list and device count), or null
  const int* red_inst = nullptr;
  const int* red_n = nullptr;
};

// Launch through LaunchArgs `a`: with timing events the runtime stamps them
// at the kernel's start and end (not around the dispatch packets).
#define LSFFT_LAUNCH(K, GRID, BLOCK, LDS, STREAM, ...)                                                 \
  do {                                                                                                 \
    if (a.ev0) hipExtLaunchKernelGGL(K, GRID, dim3(BLOCK), LDS, STREAM, a.ev0, a.ev1, 0, __VA_ARGS__);  \
    else hipLaunchKernelGGL(K, GRID, BLOCK, LDS, STREAM, __VA_ARGS__);                                 \
  } while (0)

// kind 0: x pass (len = nx); kind 1: y pass (len = ny); kind 2: outer pass
// (len = nz in 3D, ny in 2D).  Returns the LDS bytes of one work item (0 if
// unsupported) and the rows or pencils per tile.
size_t query_geometry(bool f64, int kind, int len, int* per_tile);
int threads_per_block(bool f64);
int threads_per_block_green(bool f64);

// Launchers of one pass family for one precision T, dimension DIM (x and
// outer pass) and length group (outer pass: LONG = lengths from 32 on); each
// specialization below is built in its own translation unit from k_pass.hip.
template <typename T, int DIM> hipError_t launch_x(const LaunchArgs& a, int mode, int len);
template <typename T> hipError_t launch_y(const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len);
template <typename T, int DIM, bool LONG> hipError_t launch_g(const LaunchArgs& a, int mode, int len);
template <> hipError_t launch_x<float, 2>(const LaunchArgs&, int, int);
template <> hipError_t launch_x<float, 3>(const LaunchArgs&, int, int);
template <> hipError_t launch_x<double, 2>(const LaunchArgs&, int, int);
template <> hipError_t launch_x<double, 3>(const LaunchArgs&, int, int);
template <> hipError_t launch_y<float>(const LaunchArgs&, int, int, int, int, int);
template <> hipError_t launch_y<double>(const LaunchArgs&, int, int, int, int, int);
template <> hipError_t launch_g<float, 2, false>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<float, 2, true>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<float, 3, false>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<float, 3, true>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<double, 2, false>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<double, 2, true>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<double, 3, false>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<double, 3, true>(const LaunchArgs&, int, int);

// dispatch on (precision, dimension, transform length)
hipError_t launch_xpass(bool f64, const LaunchArgs& a, int mode, int dim, int len);
hipError_t launch_ypass(bool f64, const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len);
hipError_t launch_green(bool f64, const LaunchArgs& a, int mode, int dim, int len);
hipError_t launch_cg_update(bool f64, const LaunchArgs& a);
hipError_t launch_reduce(const LaunchArgs& a, const int* inst_list, const int* d_ninst, int ninst, int mode);
hipError_t launch_phase_max(const uint8_t* phase, long long n, int* out, hipStream_t s);
hipError_t launch_accumulate(bool f64, int dim, const LaunchArgs& a, const GroupDesc* groups, int g, long long nvox);
hipError_t launch_scale(double* a, long long n, double s, hipStream_t st);
constexpr int kRveBinsMax = 1024;   // bins of launch_radial_max
hipError_t launch_radial_max(int dim, const double* avg, const int n[3], const double h[3], const double c[3],
                             double dr, int nbins, unsigned long long* bins, hipStream_t st);
// Fixed device scratch of the allocation-free RVE entry point: two rows of
// kRveBinsMax bin maxima.  rve_scratch_init looks up the calling process's
// copy on `device` (once per device; the plan constructor calls it);
// rve_scratch_ptr returns it, or null if the lookup failed or never ran.
constexpr int kRveScratchWords = 2 * kRveBinsMax;
hipError_t rve_scratch_init(int device);
unsigned long long* rve_scratch_ptr(int device);
hipError_t launch_zero_u64(unsigned long long* a, long long n, hipStream_t st);

// mixed-precision defect correction; `inst` lists `count` solves, `max_pc`
// is the largest half spectrum among them
hipError_t launch_widen(const float* src, double* dst, long long n, hipStream_t st);
hipError_t launch_defect(const InstDesc* d64, const InstState* s64, const InstDesc* d32, const int* inst, int count,
                         long long max_pc, hipStream_t st);
hipError_t launch_correct(const InstDesc* d64, const InstState* s64, const InstDesc* d32, const InstState* s32,
                          const int* inst, int count, bool cg, long long max_pc, hipStream_t st);
hipError_t launch_narrow(const InstDesc* d64, const InstState* s64, const InstDesc* d32, const int* inst, int count,
                         long long max_pc, hipStream_t st);

}  // namespace lsfft
