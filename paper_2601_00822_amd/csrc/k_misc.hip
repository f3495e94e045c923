// Small kernels (reductions, validation, averaging) and the dispatch of the
// precision-specific pass launchers.
#define LSFFT_MISC_TU 1
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

template <typename T>
static size_t geom_query(int kind, int len, int* per_line) {
  size_t bytes = 0;
  int q = 0;
  switch (len) {
#define X(L)                                                                    \
  case L:                                                                       \
    if (kind == 0) { bytes = lds_x<T, L>(); q = RowGeom<T, L / 2>::MR; }        \
    else { bytes = lds_strided<T, L>(); q = StridedGeom<T, L>::MP; }            \
    break;
    LSFFT_LEN_CASES(X)
#undef X
    default: return 0;
  }
  if (per_line) *per_line = q;
  return bytes;
}

size_t query_geometry(bool f64, int kind, int len, int* per_tile) {
  return f64 ? geom_query<double>(kind, len, per_tile) : geom_query<float>(kind, len, per_tile);
}

hipError_t launch_xpass(bool f64, const LaunchArgs& a, int mode) {
  return f64 ? launch_xpass_f64(a, mode) : launch_xpass_f32(a, mode);
}

hipError_t launch_ypass(bool f64, const LaunchArgs& a, int dir, int which, int extra, int gate) {
  return f64 ? launch_ypass_f64(a, dir, which, extra, gate) : launch_ypass_f32(a, dir, which, extra, gate);
}

hipError_t launch_green(bool f64, const LaunchArgs& a, int mode) {
  return f64 ? launch_green_f64(a, mode) : launch_green_f32(a, mode);
}

hipError_t launch_cg_update(bool f64, const LaunchArgs& a) {
  if (f64) hipLaunchKernelGGL((k_cg_update<double>), a.grid, NT, sizeof(double) * 8, a.stream, a.desc, a.state, a.items, a.count);
  else hipLaunchKernelGGL((k_cg_update<float>), a.grid, NT, sizeof(double) * 8, a.stream, a.desc, a.state, a.items, a.count);
  return hipGetLastError();
}

hipError_t launch_reduce(const LaunchArgs& a, const int* inst_list, int ninst, int mode) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(ninst), NT, 0, a.stream, a.desc, a.state, inst_list, ninst, mode);
  return hipGetLastError();
}

hipError_t launch_phase_max(const uint8_t* phase, long long n, int* out, hipStream_t s) {
  long long blocks = (n + NT - 1) / NT;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_phase_max, dim3((unsigned)blocks), NT, 0, s, phase, n, out);
  return hipGetLastError();
}

hipError_t launch_accumulate(bool f64, int dim, const LaunchArgs& a, const GroupDesc* groups, int g, long long nvox) {
  long long blocks = (nvox + NT - 1) / NT;
  if (blocks > 4096) blocks = 4096;
  const dim3 grid((unsigned)blocks);
  if (f64) {
    if (dim == 3) hipLaunchKernelGGL((k_accumulate<double, 3>), grid, NT, 0, a.stream, a.desc, groups, g, a.lame);
    else hipLaunchKernelGGL((k_accumulate<double, 2>), grid, NT, 0, a.stream, a.desc, groups, g, a.lame);
  } else {
    if (dim == 3) hipLaunchKernelGGL((k_accumulate<float, 3>), grid, NT, 0, a.stream, a.desc, groups, g, a.lame);
    else hipLaunchKernelGGL((k_accumulate<float, 2>), grid, NT, 0, a.stream, a.desc, groups, g, a.lame);
  }
  return hipGetLastError();
}

hipError_t launch_scale(double* a, long long n, double s, hipStream_t st) {
  long long blocks = (n + NT - 1) / NT;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), NT, 0, st, a, n, s);
  return hipGetLastError();
}

}  // namespace lsfft
