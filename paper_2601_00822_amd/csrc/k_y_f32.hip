// y-pass kernels: float.
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

hipError_t launch_ypass_f32(const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len) {
  const float* tw = static_cast<const float*>(a.tw);
  switch (len) {
    case 4:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 4, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 4, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 6:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 6, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 6, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 8:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 8, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 8, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 12:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 12, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 12, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 16:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 16, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 16, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 24:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 24, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 24, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 32:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 32, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 32, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 48:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 48, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 48, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 64:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 64, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 64, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 96:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 96, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 96, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 128:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 128, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 128, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 256:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<float, 256, -1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<float, 256, +1>), a.grid, Cfg<float>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lsfft
