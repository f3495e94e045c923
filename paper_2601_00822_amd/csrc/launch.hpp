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
// (len = nz in 3D, ny in 2D); kind 3: the x pass of the iteration.  Returns
// the LDS bytes of one work item of schedule variant `var` (0 if
// unsupported) and the rows or pencils per tile.
size_t query_geometry(bool f64, int kind, int len, int var, int* per_tile);
int threads_per_block(bool f64);

// Launchers of one pass family for one precision T, dimension DIM (x and
// outer pass), length group (outer pass: LONG = lengths from 32 on) and
// schedule variant V (see GSched, YSched, XSched; variants other than 0 are
// built for FP32 3D and lengths from 32 on only); each specialization below
// is built in its own translation unit from k_pass.hip.
template <typename T, int DIM, int V> hipError_t launch_x(const LaunchArgs& a, int mode, int len);
template <typename T, int V> hipError_t launch_y(const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len);
template <typename T, int DIM, bool LONG, int V> hipError_t launch_g(const LaunchArgs& a, int mode, int len);
template <> hipError_t launch_x<float, 2, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_x<float, 3, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_x<float, 3, 1>(const LaunchArgs&, int, int);
template <> hipError_t launch_x<float, 3, 2>(const LaunchArgs&, int, int);
template <> hipError_t launch_x<double, 2, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_x<double, 3, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_y<float, 0>(const LaunchArgs&, int, int, int, int, int);
template <> hipError_t launch_y<float, 1>(const LaunchArgs&, int, int, int, int, int);
template <> hipError_t launch_y<float, 2>(const LaunchArgs&, int, int, int, int, int);
template <> hipError_t launch_y<double, 0>(const LaunchArgs&, int, int, int, int, int);
template <> hipError_t launch_g<float, 2, false, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<float, 2, true, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<float, 3, false, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<float, 3, true, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<float, 3, true, 1>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<float, 3, true, 2>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<double, 2, false, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<double, 2, true, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<double, 3, false, 0>(const LaunchArgs&, int, int);
template <> hipError_t launch_g<double, 3, true, 0>(const LaunchArgs&, int, int);

// Schedule variants: kind 0 x pass, 1 y pass, 2 outer pass.  The number of
// variants a (precision, dimension, kind, length) has (1 = the default only).
int schedule_variants(bool f64, int dim, int kind, int len);

// dispatch on (precision, dimension, transform length, schedule variant)
hipError_t launch_xpass(bool f64, const LaunchArgs& a, int mode, int dim, int len, int var);
hipError_t launch_ypass(bool f64, const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len, int var);
hipError_t launch_green(bool f64, const LaunchArgs& a, int mode, int dim, int len, int var);
hipError_t launch_cg_update(bool f64, const LaunchArgs& a);
hipError_t launch_reduce(const LaunchArgs& a, const int* inst_list, const int* d_ninst, int ninst, int mode);
hipError_t launch_phase_max(const uint8_t* phase, long long n, int* out, hipStream_t s);
hipError_t launch_accumulate(bool f64, int dim, const LaunchArgs& a, const GroupDesc* groups, int g, long long nvox);
hipError_t launch_scale(double* a, long long n, double s, hipStream_t st);
// data kernels of the surrogate's dataset (see k_block_mean, k_sample_norms,
// k_bump_forces)
hipError_t launch_block_mean(bool f64_in, bool f64_out, const void* in, void* out, long long nfield, int nx, int ny,
                             int nz, int fct, double scale, hipStream_t st);
hipError_t launch_sample_norms(bool f64, const void* y, const void* t, int nsample, long long len, double* res,
                               hipStream_t st);
hipError_t launch_bump_forces(bool f64, void* const* fs, const int* first, const double* bumps, int nforce, int nx,
                              int ny, int nz, int dim, hipStream_t st);
// Nonlocal kernel regression (see k_nl_gram, k_nl_gram1, k_nl_apply,
// k_nl_apply1).  Offsets of the horizon are given as index deltas in the
// LDS box of a tile (nl_box: its extent (lx, ly, lz) for halo R; one_voxel
// names the tiles of the matrix-form normal equations), sorted by shell:
// shell q holds offsets first[q] .. first[q + 1] - 1; ee holds the direction
// products e_a e_b of every offset at ee[(o 3 + b) 3 + a].  form 0 is the
// scalar kernel, form 1 the matrix kernel K1 I + K2 e e^T.
// launch_nl_gram writes to `out` for form 0 kNlAccWords doubles (the upper
// triangle of G row by row for degree kNlMaxDegree, entries beyond `deg`
// zero, then g, then Gamma . Gamma) and for form 1 kNlAccWords1 doubles (the
// upper triangle for nf = 2 (deg + 1) features row by row, then g, then
// Gamma . Gamma, then zeros); W is [deg + 1][nshell] and `partial` holds
// kNlGramSlots x kNlAccWords1 doubles.  launch_nl_apply writes
// sum_q kw1[q] (S_q - n_q u) per component, plus the kw2 terms for form 1.
constexpr int kNlMaxDegree = 8, kNlMaxHalo = 6, kNlAccWords = 55, kNlGramSlots = 2048;
constexpr int kNlMaxHalo1 = 4, kNlAccWords1 = 190;
void nl_box(int dim, int R, bool one_voxel, int box[3]);
hipError_t launch_nl_gram(bool f64, int dim, const int n[3], int R, int deg, int form, int nsample, const void* u,
                          const void* gam, const int* offs, const int* first, const double* ee, int nshell,
                          const double* W, double* partial, double* out, hipStream_t st);
hipError_t launch_nl_apply(bool f64, int dim, const int n[3], int R, int form, int nsample, const void* u,
                           const int* offs, const int* first, const double* ee, int nshell, const double* kw1,
                           const double* kw2, void* out, hipStream_t st);
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
