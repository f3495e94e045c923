// Outer-axis (Green/body-force) pass kernels: double, 2D, lengths [4, 6, 8, 12, 16, 24].
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

hipError_t launch_green_f64_2d_s(const LaunchArgs& a, int mode, int len) {
  const double* tw = static_cast<const double*>(a.tw);
  switch (len) {
    case 4:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<double, 4, 2, M_FT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<double, 4, 2, M_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<double, 4, 2, M_ITER>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<double, 4, 2, M_MAT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<double, 4, 2, M_CG_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<double, 4, 2, M_CG_AP>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<double, 4, 2, M_CG_DIR>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 6:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<double, 6, 2, M_FT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<double, 6, 2, M_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<double, 6, 2, M_ITER>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<double, 6, 2, M_MAT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<double, 6, 2, M_CG_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<double, 6, 2, M_CG_AP>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<double, 6, 2, M_CG_DIR>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 8:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<double, 8, 2, M_FT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<double, 8, 2, M_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<double, 8, 2, M_ITER>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<double, 8, 2, M_MAT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<double, 8, 2, M_CG_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<double, 8, 2, M_CG_AP>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<double, 8, 2, M_CG_DIR>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 12:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<double, 12, 2, M_FT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<double, 12, 2, M_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<double, 12, 2, M_ITER>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<double, 12, 2, M_MAT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<double, 12, 2, M_CG_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<double, 12, 2, M_CG_AP>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<double, 12, 2, M_CG_DIR>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 16:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<double, 16, 2, M_FT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<double, 16, 2, M_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<double, 16, 2, M_ITER>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<double, 16, 2, M_MAT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<double, 16, 2, M_CG_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<double, 16, 2, M_CG_AP>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<double, 16, 2, M_CG_DIR>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 24:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<double, 24, 2, M_FT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<double, 24, 2, M_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<double, 24, 2, M_ITER>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<double, 24, 2, M_MAT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<double, 24, 2, M_CG_INIT>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<double, 24, 2, M_CG_AP>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<double, 24, 2, M_CG_DIR>), a.grid, Cfg<double>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lsfft
