// Small kernels (reductions, validation, averaging) and the dispatch of the
// precision-specific pass launchers.
#define LSFFT_MISC_TU 1
#include "kernels_impl.hpp"
#include "launch.hpp"

#include <mutex>

namespace lsfft {

template <typename T>
static size_t geom_query(int kind, int len, int* per_tile) {
  size_t bytes = 0;
  int q = 0;
  switch (len) {
#define X(L)                                                                    \
  case L:                                                                       \
    if (kind == 0) { bytes = lds_x<T, L>(); q = XGeom<T, L / 2>::MR; }          \
    else if (kind == 3) { bytes = lds_xi<T, L>(); q = XGeom<T, L / 2>::MR; }    \
    else if (kind == 1) { bytes = lds_y<T, L>(); q = SGeom<T, L>::MP; }         \
    else { bytes = lds_g<T, L>(); q = SGeom<T, L>::MPG; }                        \
    break;
    LSFFT_LEN_CASES(X)
#undef X
    default: return 0;
  }
  if (per_tile) *per_tile = q;
  return bytes;
}

size_t query_geometry(bool f64, int kind, int len, int* per_tile) {
  return f64 ? geom_query<double>(kind, len, per_tile) : geom_query<float>(kind, len, per_tile);
}

int threads_per_block(bool f64) { return f64 ? Cfg<double>::NTH : Cfg<float>::NTH; }
int threads_per_block_green(bool f64) { return f64 ? Cfg<double>::NTH_G : Cfg<float>::NTH_G; }

hipError_t launch_xpass(bool f64, const LaunchArgs& a, int mode, int dim, int len) {
  if (f64) return dim == 3 ? launch_x<double, 3>(a, mode, len) : launch_x<double, 2>(a, mode, len);
  return dim == 3 ? launch_x<float, 3>(a, mode, len) : launch_x<float, 2>(a, mode, len);
}

hipError_t launch_ypass(bool f64, const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len) {
  return f64 ? launch_y<double>(a, dir, which, ncomp, gate, len) : launch_y<float>(a, dir, which, ncomp, gate, len);
}

hipError_t launch_green(bool f64, const LaunchArgs& a, int mode, int dim, int len) {
  const bool lng = len >= 32;
  if (f64) {
    if (dim == 3) return lng ? launch_g<double, 3, true>(a, mode, len) : launch_g<double, 3, false>(a, mode, len);
    return lng ? launch_g<double, 2, true>(a, mode, len) : launch_g<double, 2, false>(a, mode, len);
  }
  if (dim == 3) return lng ? launch_g<float, 3, true>(a, mode, len) : launch_g<float, 3, false>(a, mode, len);
  return lng ? launch_g<float, 2, true>(a, mode, len) : launch_g<float, 2, false>(a, mode, len);
}

hipError_t launch_cg_update(bool f64, const LaunchArgs& a) {
  if (f64)
    LSFFT_LAUNCH((k_cg_update<double>), a.grid, Cfg<double>::NTH, sizeof(double) * 16, a.stream, a.desc, a.state,
                 a.items, a.count);
  else
    LSFFT_LAUNCH((k_cg_update<float>), a.grid, Cfg<float>::NTH, sizeof(double) * 16, a.stream, a.desc, a.state,
                 a.items, a.count);
  return hipGetLastError();
}

hipError_t launch_reduce(const LaunchArgs& a, const int* inst_list, const int* d_ninst, int ninst, int mode) {
  if (ninst <= 0) return hipSuccess;
  // the block size of the plan's y pass (a.block): the same summation order
  // as the stopping rule run inside that pass
  if (a.block == Cfg<double>::NTH)
    LSFFT_LAUNCH(k_reduce<Cfg<double>::NTH>, dim3(ninst), Cfg<double>::NTH, 0, a.stream, a.desc, a.state, inst_list,
                 d_ninst, mode);
  else
    LSFFT_LAUNCH(k_reduce<Cfg<float>::NTH>, dim3(ninst), Cfg<float>::NTH, 0, a.stream, a.desc, a.state, inst_list,
                 d_ninst, mode);
  return hipGetLastError();
}

hipError_t launch_phase_max(const uint8_t* phase, long long n, int* out, hipStream_t s) {
  long long blocks = (n + NTR - 1) / NTR;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_phase_max, dim3((unsigned)blocks), NTR, 0, s, phase, n, out);
  return hipGetLastError();
}

hipError_t launch_accumulate(bool f64, int dim, const LaunchArgs& a, const GroupDesc* groups, int g, long long nvox) {
  long long blocks = (nvox + NTR - 1) / NTR;
  if (blocks > 4096) blocks = 4096;
  const dim3 grid((unsigned)blocks);
  if (f64) {
    if (dim == 3) hipLaunchKernelGGL((k_accumulate<double, 3>), grid, NTR, 0, a.stream, a.desc, groups, g, a.lame);
    else hipLaunchKernelGGL((k_accumulate<double, 2>), grid, NTR, 0, a.stream, a.desc, groups, g, a.lame);
  } else {
    if (dim == 3) hipLaunchKernelGGL((k_accumulate<float, 3>), grid, NTR, 0, a.stream, a.desc, groups, g, a.lame);
    else hipLaunchKernelGGL((k_accumulate<float, 2>), grid, NTR, 0, a.stream, a.desc, groups, g, a.lame);
  }
  return hipGetLastError();
}

hipError_t launch_radial_max(int dim, const double* avg, const int n[3], const double h[3], const double c[3],
                             double dr, int nbins, unsigned long long* bins, hipStream_t st) {
  if (nbins < 1 || nbins > kRveMaxBins) return hipErrorInvalidValue;
  const long long nvox = (long long)n[0] * n[1] * n[2];
  long long blocks = (nvox + NTR - 1) / NTR;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  if (dim == 3)
    hipLaunchKernelGGL((k_radial_max<3>), dim3((unsigned)blocks), NTR, 0, st, avg, n[0], n[1], n[2], h[0], h[1], h[2],
                       c[0], c[1], c[2], dr, nbins, bins);
  else
    hipLaunchKernelGGL((k_radial_max<2>), dim3((unsigned)blocks), NTR, 0, st, avg, n[0], n[1], 1, h[0], h[1], 1.0,
                       c[0], c[1], 0.0, dr, nbins, bins);
  return hipGetLastError();
}

// ---- fixed device scratch of the allocation-free RVE entry point ----------
// The radial maxima of lsfft_rve_identify_noalloc live in this array (one
// copy per GPU, held until the process ends).  Host code never passes the
// array's name to a kernel: it stands for a host-side shadow, not a device
// address.  Each device's address is looked up once, with that device
// current, and kept in rve_scratch_dev.
static_assert(kRveMaxBins == kRveBinsMax, "radial-maxima bin limits must agree");
static __device__ __align__(256) unsigned long long rve_scratch[kRveScratchWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex rve_scratch_mu;
int rve_scratch_state[kMaxDevices] = {0};                  // 0 untried, 1 ready, -1 failed
unsigned long long* rve_scratch_dev[kMaxDevices] = {nullptr};
}  // namespace

hipError_t rve_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(rve_scratch_mu);
  if (rve_scratch_state[device] == 1) return hipSuccess;
  if (rve_scratch_state[device] == -1) return hipErrorInvalidDevice;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != device) e = hipSetDevice(device);
  void* ptr = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(rve_scratch));
  if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || ptr == nullptr) {
    rve_scratch_state[device] = -1;
    return e != hipSuccess ? e : hipErrorInvalidSymbol;
  }
  rve_scratch_dev[device] = static_cast<unsigned long long*>(ptr);
  rve_scratch_state[device] = 1;
  return hipSuccess;
}

unsigned long long* rve_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(rve_scratch_mu);
  return rve_scratch_state[device] == 1 ? rve_scratch_dev[device] : nullptr;
}

hipError_t launch_zero_u64(unsigned long long* a, long long n, hipStream_t st) {
  long long blocks = (n + NTR - 1) / NTR;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)blocks), NTR, 0, st, a, n);
  return hipGetLastError();
}

hipError_t launch_scale(double* a, long long n, double s, hipStream_t st) {
  long long blocks = (n + NTR - 1) / NTR;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), NTR, 0, st, a, n, s);
  return hipGetLastError();
}

// grid.x strides over the half spectrum of one solve, grid.y = solve slot
// (callers keep count <= 65535)
static dim3 spectrum_grid(long long max_pc, int count, int dims) {
  long long bx = (max_pc * dims + NTR - 1) / NTR;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  return dim3((unsigned)bx, (unsigned)count);
}

hipError_t launch_widen(const float* src, double* dst, long long n, hipStream_t st) {
  long long blocks = (n + NTR - 1) / NTR;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)blocks), NTR, 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_defect(const InstDesc* d64, const InstState* s64, const InstDesc* d32, const int* inst, int count,
                         long long max_pc, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_defect, spectrum_grid(max_pc, count, 1), NTR, 0, st, d64, s64, d32, inst);
  return hipGetLastError();
}

hipError_t launch_correct(const InstDesc* d64, const InstState* s64, const InstDesc* d32, const InstState* s32,
                          const int* inst, int count, bool cg, long long max_pc, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_correct, spectrum_grid(max_pc, count, 3), NTR, 0, st, d64, s64, d32, s32, inst, cg ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_narrow(const InstDesc* d64, const InstState* s64, const InstDesc* d32, const int* inst, int count,
                         long long max_pc, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_narrow, spectrum_grid(max_pc, count, 3), NTR, 0, st, d64, s64, d32, inst);
  return hipGetLastError();
}

}  // namespace lsfft
