// FP64 stage kernels: half-range (two waves per window) and full-range; the
// fused-step kernel of the half-range model.
#include "fused_kernels.hpp"
#include "launch.hpp"

namespace hhlb {
namespace {

template <int QUAD, int Q, int NF, int ADV>
void launch_stage(const StageArgs &a, hipStream_t s) {
  if constexpr (QUAD == 0)
    hipLaunchKernelGGL((stage_kernel_half<Q, NF, ADV>), dim3(a.nwin), dim3(128), 0, s, a, a.tb, a.chans,
                       a.wins, a.inv_dx, a.gw, (const double *)a.in_f, (const double *)a.in_c);
  else
    hipLaunchKernelGGL((stage_kernel<QUAD, Q, NF, ADV>), dim3(a.nwin), dim3(64), 0, s, a);
}

template <int Q, int ADV>
void launch_quarter(const StageArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((stage_kernel_quarter<Q, ADV>), dim3(a.nwin), dim3(256), 0, s, a, a.tb, a.chans, a.wins,
                     a.inv_dx, a.gw, (const double *)a.in_f, (const double *)a.in_c);
}

template <int Q, int NF, int ADV>
void launch_fused(const StageArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((fused_kernel_half<Q, NF, ADV>), dim3(a.nwin), dim3(128), 0, s, a, a.tb, a.chans,
                     reinterpret_cast<const DevFusedWindow *>(a.wins), a.inv_dx, a.gw, (const double *)a.in_f,
                     (const double *)a.in_c);
}

template <int QUAD, int Q>
void add(LaunchMap &m) {
  // the half-range two-wave kernel at Q = 16 has a translation unit of its
  // own (kernels_fp64_q16.hip, built with another instruction scheduler)
  if constexpr (!(QUAD == 0 && Q == 16)) {
    m[{QUAD, Q, 1, 0, 0, 2}] = launch_stage<QUAD, Q, 1, 0>;
    m[{QUAD, Q, 1, 1, 0, 2}] = launch_stage<QUAD, Q, 1, 1>;
    m[{QUAD, Q, 2, 0, 0, 2}] = launch_stage<QUAD, Q, 2, 0>;
    m[{QUAD, Q, 2, 1, 0, 2}] = launch_stage<QUAD, Q, 2, 1>;
  }
  if constexpr (QUAD == 0) {   // four waves per window: f and chi, half range
    m[{QUAD, Q, 2, 0, 0, 4}] = launch_quarter<Q, 0>;
    m[{QUAD, Q, 2, 1, 0, 4}] = launch_quarter<Q, 1>;
  }
  if constexpr (QUAD == 0 && Q <= kQmaxFused) {   // one launch per RK-3 step
    m[{QUAD, Q, 1, 0, 0, 1}] = launch_fused<Q, 1, 0>;
    m[{QUAD, Q, 1, 1, 0, 1}] = launch_fused<Q, 1, 1>;
    m[{QUAD, Q, 2, 0, 0, 1}] = launch_fused<Q, 2, 0>;
    m[{QUAD, Q, 2, 1, 0, 1}] = launch_fused<Q, 2, 1>;
  }
}

}  // namespace

void register_fp64(LaunchMap &m) {
  add<0, 1>(m); add<0, 2>(m); add<0, 3>(m); add<0, 4>(m);
  add<0, 6>(m); add<0, 8>(m); add<0, 12>(m); add<0, 16>(m);
  add<1, 2>(m); add<1, 4>(m); add<1, 8>(m); add<1, 16>(m);
}

}  // namespace hhlb
