// y-pass kernels: double.
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

hipError_t launch_ypass_f64(const LaunchArgs& a, int dir, int which, int ncomp, int gate, int len) {
  const double* tw = static_cast<const double*>(a.tw);
  switch (len) {
    case 4:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 4, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 4, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 6:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 6, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 6, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 8:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 8, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 8, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 12:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 12, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 12, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 16:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 16, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 16, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 24:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 24, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 24, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 32:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 32, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 32, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 48:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 48, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 48, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 64:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 64, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 64, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 96:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 96, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 96, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 128:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 128, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 128, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    case 256:
      if (dir < 0) LSFFT_LAUNCH((k_ypass<double, 256, -1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      else LSFFT_LAUNCH((k_ypass<double, 256, +1>), a.grid, Cfg<double>::NTH, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, ncomp, gate, a.red_inst, a.red_n);
      return hipGetLastError();
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lsfft
