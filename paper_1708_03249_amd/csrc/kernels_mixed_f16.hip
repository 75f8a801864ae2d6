// Mixed-precision half-range stage kernels, force block in F16 form.
#include "launch.hpp"
#include "mixed_kernels.hpp"

namespace hhlb {
namespace {

template <int Q, int NF, int ADV>
void launch_stage(const StageArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((stage_kernel_mixed<Q, NF, ADV, kPrecF16>), dim3(a.nwin), dim3(128), 0, s, a, a.tb,
                     a.chans, a.wins, a.inv_dx, a.gw, (const float *)a.base_f, (const float *)a.base_c,
                     (const float *)a.in_f, (const float *)a.in_c);
}

template <int Q>
void add(LaunchMap &m) {
  m[{0, Q, 1, 0, kPrecF16, 2}] = launch_stage<Q, 1, 0>;
  m[{0, Q, 1, 1, kPrecF16, 2}] = launch_stage<Q, 1, 1>;
  m[{0, Q, 2, 0, kPrecF16, 2}] = launch_stage<Q, 2, 0>;
  m[{0, Q, 2, 1, kPrecF16, 2}] = launch_stage<Q, 2, 1>;
}

}  // namespace

void register_mixed_f16(LaunchMap &m) {
  add<1>(m); add<2>(m); add<3>(m); add<4>(m); add<6>(m); add<8>(m); add<12>(m); add<16>(m);
}

}  // namespace hhlb
