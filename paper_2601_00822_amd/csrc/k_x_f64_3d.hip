// x-pass kernels: double, 3D.
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

hipError_t launch_xpass_f64_3d(const LaunchArgs& a, int mode, int len) {
  const double* tw = static_cast<const double*>(a.tw);
  switch (len) {
    case 4:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 4, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 4, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 4, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 6:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 6, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 6, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 6, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 8:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 8, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 8, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 8, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 12:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 12, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 12, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 12, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 16:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 16, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 16, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 16, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 24:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 24, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 24, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 24, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 32:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 32, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 32, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 32, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 48:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 48, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 48, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 48, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 64:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 64, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 64, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 64, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 96:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 96, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 96, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 96, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 128:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 128, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 128, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 128, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 256:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_xpass<double, 256, 3, M_FT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_xpass<double, 256, 3, M_ITER>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_xpass<double, 256, 3, M_MAT>), a.grid, Cfg<double>::NTH_X, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lsfft
