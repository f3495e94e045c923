// y-pass kernels, float instantiation.
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

template <typename T>
static hipError_t launch_y_t(const LaunchArgs& a, int dir, int which, int extra, int gate) {
  const T* tw = static_cast<const T*>(a.tw);
  if (dir < 0)
    hipLaunchKernelGGL((k_ypass<T, -1>), a.grid, NT, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, extra, gate);
  else
    hipLaunchKernelGGL((k_ypass<T, +1>), a.grid, NT, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw, which, extra, gate);
  return hipGetLastError();
}

hipError_t launch_ypass_f32(const LaunchArgs& a, int dir, int which, int extra, int gate) {
  return launch_y_t<float>(a, dir, which, extra, gate);
}

}  // namespace lsfft
