// Launchers of the node-parallel FP64 stage for large half-range velocity sets.
#include "large_kernels.hpp"

namespace hhlb {

// One RK stage: the cell phase, then the node phase (same stream).
void launch_large(const LargeArgs &a, int adv, int H, hipStream_t s) {
  const int groups = 2 * ((H + kLargeNG - 1) / kLargeNG);
  if (adv == 0) {
    hipLaunchKernelGGL(large_cell_kernel<0>, dim3(a.nwin), dim3(192), 0, s, a);
    hipLaunchKernelGGL((large_node_kernel<0, kLargeNG>), dim3(a.nwin, groups), dim3(64), 0, s, a);
  } else {
    hipLaunchKernelGGL(large_cell_kernel<1>, dim3(a.nwin), dim3(192), 0, s, a);
    hipLaunchKernelGGL((large_node_kernel<1, kLargeNG>), dim3(a.nwin, groups), dim3(64), 0, s, a);
  }
}

}  // namespace hhlb
