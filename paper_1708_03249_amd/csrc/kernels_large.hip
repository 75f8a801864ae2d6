// Launchers of the node-parallel FP64 stage for large half-range velocity sets.
#include "large_kernels.hpp"

namespace hhlb {

// One RK stage: the cell phase, then the node phase (same stream).
void launch_large(const LargeArgs &a, int adv, int H, hipStream_t s) {
  const dim3 cgrid(a.nwin * (kCellGroups + 1)), ngrid(a.nwin * 2 * ((H + kTileNodes - 1) / kTileNodes));
  if (adv == 0) {
    hipLaunchKernelGGL(large_cell_kernel<0>, cgrid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(large_node_kernel<0>, ngrid, dim3(64 * kNodeWaves), 0, s, a);
  } else {
    hipLaunchKernelGGL(large_cell_kernel<1>, cgrid, dim3(256), 0, s, a);
    hipLaunchKernelGGL(large_node_kernel<1>, ngrid, dim3(64 * kNodeWaves), 0, s, a);
  }
}

}  // namespace hhlb
