// Small kernels (reductions, validation, averaging) and the dispatch of the
// precision-specific pass launchers.
#define LSFFT_MISC_TU 1
#include "kernels_impl.hpp"
#include "launch.hpp"

#include <mutex>

namespace lsfft {

template <typename T, int V>
static size_t geom_query_v(int kind, int len, int* per_tile) {
  size_t bytes = 0;
  int q = 0;
  switch (len) {
#define X(L)                                                                          \
  case L:                                                                             \
    if (kind == 0) { bytes = lds_x<T, L, V>(); q = XGeom<T, L / 2, XSched<V>::EX_DIV>::MR; } \
    else if (kind == 3) { bytes = lds_xi<T, L, V>(); q = XGeom<T, L / 2, XSched<V>::EX_DIV>::MR; } \
    else if (kind == 1) { bytes = lds_y<T, L, V>(); q = YSched<T, L, V>::MP; }         \
    else { bytes = lds_g<T, L, V>(); q = GSched<T, L, V>::MP; }                        \
    break;
    LSFFT_LEN_CASES(X)
#undef X
    default: return 0;
  }
  if (per_tile) *per_tile = q;
  return bytes;
}

int schedule_variants(bool f64, int dim, int kind, int len) {
  if (f64 || dim != 3 || len < 32) return 1;
  return kind == 2 ? kVarG : kind == 1 ? kVarY : kVarX;
}

size_t query_geometry(bool f64, int kind, int len, int var, int* per_tile) {
  if (f64) return var == 0 ? geom_query_v<double, 0>(kind, len, per_tile) : 0;
  switch (var) {
    case 0: return geom_query_v<float, 0>(kind, len, per_tile);
    case 1: return geom_query_v<float, 1>(kind, len, per_tile);
    case 2: return geom_query_v<float, 2>(kind, len, per_tile);
    default: return 0;
  }
}

int threads_per_block(bool f64) { return f64 ? Cfg<double>::NTH : Cfg<float>::NTH; }

hipError_t launch_xpass(bool f64, const LaunchArgs& a, int mode, int dim, int len, int var) {
  if (f64) {
    if (var != 0) return hipErrorInvalidValue;
    return dim == 3 ? launch_x<double, 3, 0>(a, mode, len) : launch_x<double, 2, 0>(a, mode, len);
  }
  if (dim != 3) return var == 0 ? launch_x<float, 2, 0>(a, mode, len) : hipErrorInvalidValue;
  switch (var) {
    case 0: return launch_x<float, 3, 0>(a, mode, len);
    case 1: return launch_x<float, 3, 1>(a, mode, len);
    case 2: return launch_x<float, 3, 2>(a, mode, len);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ypass(bool f64, const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len, int var) {
  if (f64) return var == 0 ? launch_y<double, 0>(a, dir, which, ncomp, gate, len) : hipErrorInvalidValue;
  switch (var) {
    case 0: return launch_y<float, 0>(a, dir, which, ncomp, gate, len);
    case 1: return launch_y<float, 1>(a, dir, which, ncomp, gate, len);
    case 2: return launch_y<float, 2>(a, dir, which, ncomp, gate, len);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_green(bool f64, const LaunchArgs& a, int mode, int dim, int len, int var) {
  const bool lng = len >= 32;
  if (f64) {
    if (var != 0) return hipErrorInvalidValue;
    if (dim == 3) return lng ? launch_g<double, 3, true, 0>(a, mode, len) : launch_g<double, 3, false, 0>(a, mode, len);
    return lng ? launch_g<double, 2, true, 0>(a, mode, len) : launch_g<double, 2, false, 0>(a, mode, len);
  }
  if (dim != 3) {
    if (var != 0) return hipErrorInvalidValue;
    return lng ? launch_g<float, 2, true, 0>(a, mode, len) : launch_g<float, 2, false, 0>(a, mode, len);
  }
  if (!lng) return var == 0 ? launch_g<float, 3, false, 0>(a, mode, len) : hipErrorInvalidValue;
  switch (var) {
    case 0: return launch_g<float, 3, true, 0>(a, mode, len);
    case 1: return launch_g<float, 3, true, 1>(a, mode, len);
    case 2: return launch_g<float, 3, true, 2>(a, mode, len);
    default: return hipErrorInvalidValue;
  }
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

static unsigned grid_for(long long n, long long cap) {
  long long b = (n + NTR - 1) / NTR;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_block_mean(bool f64_in, bool f64_out, const void* in, void* out, long long nfield, int nx, int ny,
                             int nz, int fct, double scale, hipStream_t st) {
  const long long ncoarse = (long long)(nx / fct) * (ny / fct) * (nz > 1 ? nz / fct : 1);
  const dim3 grid(grid_for(nfield * ncoarse, 8192));
#define LSFFT_BM(TI, TO)                                                                                      \
  hipLaunchKernelGGL((k_block_mean<TI, TO>), grid, NTR, 0, st, static_cast<const TI*>(in), static_cast<TO*>(out), \
                     nfield, nx, ny, nz, fct, scale)
  if (f64_in) {
    if (f64_out) LSFFT_BM(double, double);
    else LSFFT_BM(double, float);
  } else {
    if (f64_out) LSFFT_BM(float, double);
    else LSFFT_BM(float, float);
  }
#undef LSFFT_BM
  return hipGetLastError();
}

hipError_t launch_sample_norms(bool f64, const void* y, const void* t, int nsample, long long len, double* res,
                               hipStream_t st) {
  if (nsample <= 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(k_sample_norms<double>, dim3((unsigned)nsample), NTR, 0, st, static_cast<const double*>(y),
                       static_cast<const double*>(t), len, res);
  else
    hipLaunchKernelGGL(k_sample_norms<float>, dim3((unsigned)nsample), NTR, 0, st, static_cast<const float*>(y),
                       static_cast<const float*>(t), len, res);
  return hipGetLastError();
}

hipError_t launch_bump_forces(bool f64, void* const* fs, const int* first, const double* bumps, int nforce, int nx,
                              int ny, int nz, int dim, hipStream_t st) {
  if (nforce <= 0) return hipSuccess;
  const dim3 grid(grid_for((long long)nx * ny * nz, 2048), (unsigned)nforce);
  if (f64)
    hipLaunchKernelGGL(k_bump_forces<double>, grid, NTR, 0, st, reinterpret_cast<double* const*>(fs), first, bumps,
                       nx, ny, nz, dim);
  else
    hipLaunchKernelGGL(k_bump_forces<float>, grid, NTR, 0, st, reinterpret_cast<float* const*>(fs), first, bumps, nx,
                       ny, nz, dim);
  return hipGetLastError();
}

static_assert(kNlMaxDegree == kNlMaxDeg && kNlMaxHalo == kNlMaxR && kNlAccWords == kNlAcc &&
                  kNlGramSlots == kNlGramBlocks && kNlMaxHalo1 == kNlMaxR1 && kNlAccWords1 == kNlAcc1,
              "nonlocal constants of the launcher and the kernels must agree");

// tiles of the nonlocal kernels: two voxels per thread (8 x 8 x 8 in 3D,
// 16 x 32 in 2D), or one (8 x 8 x 4, 16 x 16: the matrix-form normal
// equations)
static NlGeom nl_geom(int dim, const int n[3], int R, int nshell, int deg, bool one_voxel) {
  NlGeom G;
  G.nx = n[0];
  G.ny = n[1];
  G.nz = (dim == 3) ? n[2] : 1;
  G.dim = dim;
  G.vpt = one_voxel ? 1 : 2;
  G.tx = (dim == 3) ? kNlTX : kNlTX2;
  G.ty = (dim == 3) ? kNlTY : (one_voxel ? kNlTY21 : kNlTY2);
  G.tz = (dim == 3) ? (one_voxel ? kNlTZ1 : kNlTZ) : 1;
  G.ntx = (G.nx + G.tx - 1) / G.tx;
  G.nty = (G.ny + G.ty - 1) / G.ty;
  G.ntz = (G.nz + G.tz - 1) / G.tz;
  G.R = R;
  G.lx = G.tx + 2 * R;
  G.ly = G.ty + 2 * R;
  G.lz = (dim == 3) ? G.tz + 2 * R : 1;
  G.nshell = nshell;
  G.deg = deg;
  return G;
}

void nl_box(int dim, int R, bool one_voxel, int box[3]) {
  const int n[3] = {1, 1, 1};
  const NlGeom G = nl_geom(dim, n, R, 0, 0, one_voxel);
  box[0] = G.lx;
  box[1] = G.ly;
  box[2] = G.lz;
}

static size_t nl_box_bytes(const NlGeom& G, bool f64) { return (size_t)G.lx * G.ly * G.lz * (f64 ? 8 : 4); }

static size_t nl_lds_bytes(const NlGeom& G, bool f64) {
  const size_t box = nl_box_bytes(G, f64);
  const size_t red = (size_t)kNlAcc * (NTR / 64) * sizeof(double);
  return box > red ? box : red;
}

hipError_t launch_nl_gram(bool f64, int dim, const int n[3], int R, int deg, int form, int nsample, const void* u,
                          const void* gam, const int* offs, const int* first, const double* ee, int nshell,
                          const double* W, double* partial, double* out, hipStream_t st) {
  if (deg < 0 || deg > kNlMaxDeg || R < 0 || nsample < 1 || nshell < 0 || (form != 0 && form != 1))
    return hipErrorInvalidValue;
  if (R > (form == 1 && dim == 3 ? kNlMaxR1 : kNlMaxR)) return hipErrorInvalidValue;
  const NlGeom G = nl_geom(dim, n, R, nshell, deg, form == 1);
  const long long items = (long long)nsample * G.ntx * G.nty * G.ntz;
  const unsigned grid = (unsigned)(items < kNlGramBlocks ? items : kNlGramBlocks);
  if (form == 0) {
    const size_t lds = nl_lds_bytes(G, f64);
    if (f64)
      hipLaunchKernelGGL(k_nl_gram<double>, dim3(grid), NTR, lds, st, G, static_cast<const double*>(u),
                         static_cast<const double*>(gam), nsample, offs, first, W, partial);
    else
      hipLaunchKernelGGL(k_nl_gram<float>, dim3(grid), NTR, lds, st, G, static_cast<const float*>(u),
                         static_cast<const float*>(gam), nsample, offs, first, W, partial);
  } else {
    const size_t lds = sizeof(double) * ((size_t)kNlF1 * kNlFeatPitch + NTR) + nl_box_bytes(G, f64);
    if (lds > 65536) return hipErrorInvalidValue;
    if (f64)
      hipLaunchKernelGGL(k_nl_gram1<double>, dim3(grid), NTR, lds, st, G, static_cast<const double*>(u),
                         static_cast<const double*>(gam), nsample, offs, first, ee, W, partial);
    else
      hipLaunchKernelGGL(k_nl_gram1<float>, dim3(grid), NTR, lds, st, G, static_cast<const float*>(u),
                         static_cast<const float*>(gam), nsample, offs, first, ee, W, partial);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int stride = form == 0 ? kNlAcc : kNlAcc1;
  hipLaunchKernelGGL(k_nl_gram_sum, dim3(1), NTR, 0, st, partial, (int)grid, stride, stride, out);
  return hipGetLastError();
}

hipError_t launch_nl_apply(bool f64, int dim, const int n[3], int R, int form, int nsample, const void* u,
                           const int* offs, const int* first, const double* ee, int nshell, const double* kw1,
                           const double* kw2, void* out, hipStream_t st) {
  if (R < 0 || R > kNlMaxR || nsample < 1 || nshell < 0 || (form != 0 && form != 1)) return hipErrorInvalidValue;
  const NlGeom G = nl_geom(dim, n, R, nshell, 0, false);
  const long long items = (long long)nsample * G.ntx * G.nty * G.ntz;
  if (items > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = nl_lds_bytes(G, f64);
  if (form == 0) {
    if (f64)
      hipLaunchKernelGGL(k_nl_apply<double>, dim3((unsigned)items), NTR, lds, st, G, static_cast<const double*>(u),
                         nsample, offs, first, kw1, static_cast<double*>(out));
    else
      hipLaunchKernelGGL(k_nl_apply<float>, dim3((unsigned)items), NTR, lds, st, G, static_cast<const float*>(u),
                         nsample, offs, first, kw1, static_cast<float*>(out));
  } else {
    if (f64)
      hipLaunchKernelGGL(k_nl_apply1<double>, dim3((unsigned)items), NTR, lds, st, G, static_cast<const double*>(u),
                         nsample, offs, first, ee, kw1, kw2, static_cast<double*>(out));
    else
      hipLaunchKernelGGL(k_nl_apply1<float>, dim3((unsigned)items), NTR, lds, st, G, static_cast<const float*>(u),
                         nsample, offs, first, ee, kw1, kw2, static_cast<float*>(out));
  }
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
