// Green/body-force outer-pass kernels, double instantiation.
#include "kernels_impl.hpp"
#include "launch.hpp"

namespace lsfft {

template <typename T>
static hipError_t launch_g_t(const LaunchArgs& a, int mode) {
  const T* tw = static_cast<const T*>(a.tw);
  switch (mode) {
#define G(MODE_) case MODE_: hipLaunchKernelGGL((k_green<T, MODE_>), a.grid, NT, a.lds, a.stream, a.desc, a.state, a.items, a.count, tw); break;
    G(M_FT) G(M_INIT) G(M_ITER) G(M_MAT) G(M_CG_INIT) G(M_CG_AP) G(M_CG_DIR)
#undef G
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_green_f64(const LaunchArgs& a, int mode) { return launch_g_t<double>(a, mode); }

}  // namespace lsfft
