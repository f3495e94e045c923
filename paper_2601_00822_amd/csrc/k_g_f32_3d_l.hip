// Outer-axis (Green/body-force) pass kernels: float, 3D, lengths [32, 48, 64, 96, 128, 256].
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

hipError_t launch_green_f32_3d_l(const LaunchArgs& a, int mode, int len) {
  const float* tw = static_cast<const float*>(a.tw);
  switch (len) {
    case 32:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<float, 32, 3, M_FT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<float, 32, 3, M_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<float, 32, 3, M_ITER>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<float, 32, 3, M_MAT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<float, 32, 3, M_CG_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<float, 32, 3, M_CG_AP>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<float, 32, 3, M_CG_DIR>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 48:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<float, 48, 3, M_FT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<float, 48, 3, M_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<float, 48, 3, M_ITER>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<float, 48, 3, M_MAT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<float, 48, 3, M_CG_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<float, 48, 3, M_CG_AP>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<float, 48, 3, M_CG_DIR>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 64:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<float, 64, 3, M_FT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<float, 64, 3, M_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<float, 64, 3, M_ITER>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<float, 64, 3, M_MAT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<float, 64, 3, M_CG_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<float, 64, 3, M_CG_AP>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<float, 64, 3, M_CG_DIR>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 96:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<float, 96, 3, M_FT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<float, 96, 3, M_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<float, 96, 3, M_ITER>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<float, 96, 3, M_MAT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<float, 96, 3, M_CG_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<float, 96, 3, M_CG_AP>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<float, 96, 3, M_CG_DIR>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 128:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<float, 128, 3, M_FT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<float, 128, 3, M_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<float, 128, 3, M_ITER>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<float, 128, 3, M_MAT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<float, 128, 3, M_CG_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<float, 128, 3, M_CG_AP>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<float, 128, 3, M_CG_DIR>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    case 256:
      switch (mode) {
        case M_FT: LSFFT_LAUNCH((k_green<float, 256, 3, M_FT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_INIT: LSFFT_LAUNCH((k_green<float, 256, 3, M_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_ITER: LSFFT_LAUNCH((k_green<float, 256, 3, M_ITER>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_MAT: LSFFT_LAUNCH((k_green<float, 256, 3, M_MAT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_INIT: LSFFT_LAUNCH((k_green<float, 256, 3, M_CG_INIT>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_AP: LSFFT_LAUNCH((k_green<float, 256, 3, M_CG_AP>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError();
        case M_CG_DIR: LSFFT_LAUNCH((k_green<float, 256, 3, M_CG_DIR>), a.grid, Cfg<float>::NTH_G, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); return hipGetLastError(); default: return hipErrorInvalidValue; }
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lsfft
