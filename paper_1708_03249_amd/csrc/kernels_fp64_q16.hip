// The FP64 half-range two-wave stage kernel at Q = 16 (the large workload's
// kernel), in a translation unit of its own: build.py compiles it with the
// backend's ILP-first instruction scheduler, which at this order leaves
// less register spill and runs faster; the other kernels keep the default
// scheduler, under which they run faster.
#include "launch.hpp"

namespace hhlb {
namespace {

template <int NF, int ADV>
void launch_q16(const StageArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((stage_kernel_half<16, NF, ADV>), dim3(a.nwin), dim3(128), 0, s, a, a.tb, a.chans, a.wins,
                     a.inv_dx, a.gw, (const double *)a.in_f, (const double *)a.in_c);
}

}  // namespace

void register_fp64_q16(LaunchMap &m) {
  m[{0, 16, 1, 0, 0, 2}] = launch_q16<1, 0>;
  m[{0, 16, 1, 1, 0, 2}] = launch_q16<1, 1>;
  m[{0, 16, 2, 0, 0, 2}] = launch_q16<2, 0>;
  m[{0, 16, 2, 1, 0, 2}] = launch_q16<2, 1>;
}

}  // namespace hhlb
