// x-pass kernels: float, 3D.
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

hipError_t launch_xpass_f32_3d(const LaunchArgs& a, int mode, int len) {
  const float* tw = static_cast<const float*>(a.tw);
  switch (len) {
    case 4:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 4, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 4, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 4, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 6:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 6, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 6, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 6, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 8:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 8, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 8, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 8, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 12:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 12, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 12, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 12, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 16:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 16, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 16, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 16, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 24:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 24, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 24, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 24, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 32:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 32, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 32, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 32, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 48:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 48, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 48, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 48, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 64:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 64, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 64, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 64, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 96:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 96, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 96, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 96, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 128:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 128, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 128, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 128, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 256:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<float, 256, 3, M_FT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<float, 256, 3, M_ITER>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<float, 256, 3, M_MAT>), a.grid, Cfg<float>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lsfft
