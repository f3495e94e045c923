// Launchers of the pass kernels: one switch over the supported transform
// lengths (LSFFT_LEN_CASES*) and the pass modes per kernel family.  The build
// compiles this file once per combination of
//   LSFFT_PASS  0 x pass, 1 y pass, 2 outer pass
//   LSFFT_F64   0 float, 1 double
//   LSFFT_DIM   2 or 3 (x and outer pass)
//   LSFFT_LONG  outer pass: 0 lengths below 32, 1 lengths from 32 on
//   LSFFT_VARIANT  schedule variant (0 when undefined); variants other than 0
//               exist for FP32 3D only and cover the lengths from 32 on
// so that every kernel specialization is compiled once and the translation
// units build in parallel.
#include "kernels_impl.hpp"
#include "launch.hpp"

#if !defined(LSFFT_PASS) || !defined(LSFFT_F64)
#error "k_pass.hip is built once per pass family: define LSFFT_PASS and LSFFT_F64"
#endif
#ifndef LSFFT_VARIANT
#define LSFFT_VARIANT 0
#endif

namespace lsfft {
namespace {
#if LSFFT_F64
using T = double;
#else
using T = float;
#endif
}  // namespace

#if LSFFT_PASS == 0
// ---- x pass: C2R, Hooke's law, R2C along x ---------------------------------
namespace {
template <int L>
hipError_t x_modes(const LaunchArgs& a, int mode) {
  const T* tw = static_cast<const T*>(a.tw);
  switch (mode) {
#define M(MODE)                                                                                                \
  case MODE:                                                                                                   \
    LSFFT_LAUNCH((k_xpass<T, L, LSFFT_DIM, MODE, LSFFT_VARIANT>), a.grid, Cfg<T>::NTH_X, a.lds, a.stream, a.desc, \
                 a.state, a.items, a.count, a.lame, tw);                                                       \
    return hipGetLastError();
    M(M_FT) M(M_ITER) M(M_MAT)
#undef M
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

template <>
hipError_t launch_x<T, LSFFT_DIM, LSFFT_VARIANT>(const LaunchArgs& a, int mode, int len) {
  switch (len) {
#define X(L) case L: return x_modes<L>(a, mode);
#if LSFFT_VARIANT == 0
    LSFFT_LEN_CASES(X)
#else
    LSFFT_LEN_CASES_LONG(X)
#endif
#undef X
    default: return hipErrorInvalidValue;
  }
}

#elif LSFFT_PASS == 1
// ---- y pass (3D): one component of a tile per work unit --------------------
namespace {
template <int L>
hipError_t y_dirs(const LaunchArgs& a, int dir, int which, int ncomp, int gate) {
  const T* tw = static_cast<const T*>(a.tw);
  if (dir < 0)
    LSFFT_LAUNCH((k_ypass<T, L, -1, LSFFT_VARIANT>), a.grid, Cfg<T>::NTH, a.lds, a.stream, a.desc, a.state, a.items,
                 a.count, tw,
                 which, ncomp, gate, a.red_inst, a.red_n);
  else
    LSFFT_LAUNCH((k_ypass<T, L, +1, LSFFT_VARIANT>), a.grid, Cfg<T>::NTH, a.lds, a.stream, a.desc, a.state, a.items,
                 a.count, tw,
                 which, ncomp, gate, a.red_inst, a.red_n);
  return hipGetLastError();
}
}  // namespace

template <>
hipError_t launch_y<T, LSFFT_VARIANT>(const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len) {
  switch (len) {
#define X(L) case L: return y_dirs<L>(a, dir, which, ncomp, gate);
#if LSFFT_VARIANT == 0
    LSFFT_LEN_CASES(X)
#else
    LSFFT_LEN_CASES_LONG(X)
#endif
#undef X
    default: return hipErrorInvalidValue;
  }
}

#elif LSFFT_PASS == 2
// ---- outer pass: transforms along the outermost axis with the Green update --
namespace {
template <int L>
hipError_t g_modes(const LaunchArgs& a, int mode) {
  const T* tw = static_cast<const T*>(a.tw);
  switch (mode) {
#define M(MODE)                                                                                                 \
  case MODE:                                                                                                    \
    LSFFT_LAUNCH((k_green<T, L, LSFFT_DIM, MODE, LSFFT_VARIANT>), a.grid, (GSched<T, L, LSFFT_VARIANT>::NTH),  \
                 a.lds, a.stream, a.desc, a.state, a.items, a.count, tw);                                      \
    return hipGetLastError();
    M(M_FT) M(M_INIT) M(M_ITER) M(M_MAT) M(M_CG_INIT) M(M_CG_AP) M(M_CG_DIR) M(M_AA_RES) M(M_AA_UPD) M(M_KCONV)
#undef M
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

template <>
hipError_t launch_g<T, LSFFT_DIM, (LSFFT_LONG != 0), LSFFT_VARIANT>(const LaunchArgs& a, int mode, int len) {
  switch (len) {
#define X(L) case L: return g_modes<L>(a, mode);
#if LSFFT_LONG
    LSFFT_LEN_CASES_LONG(X)
#else
    LSFFT_LEN_CASES_SHORT(X)
#endif
#undef X
    default: return hipErrorInvalidValue;
  }
}
#else
#error "LSFFT_PASS must be 0, 1 or 2"
#endif

}  // namespace lsfft
