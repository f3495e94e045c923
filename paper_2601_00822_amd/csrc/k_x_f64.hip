// x-pass kernels, double instantiation.
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

template <typename T>
static hipError_t launch_x_t(const LaunchArgs& a, int mode) {
  const T* tw = static_cast<const T*>(a.tw);
  switch (mode) {
    case M_FT: hipLaunchKernelGGL((k_xpass<T, M_FT>), a.grid, NT, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); break;
    case M_ITER: hipLaunchKernelGGL((k_xpass<T, M_ITER>), a.grid, NT, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); break;
    case M_MAT: hipLaunchKernelGGL((k_xpass<T, M_MAT>), a.grid, NT, a.lds, a.stream, a.desc, a.state, a.items, a.count, a.lame, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_xpass_f64(const LaunchArgs& a, int mode) { return launch_x_t<double>(a, mode); }

}  // namespace lsfft
