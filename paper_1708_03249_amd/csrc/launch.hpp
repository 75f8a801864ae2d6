// Registry of the stage-kernel launchers, keyed by model shape and arithmetic
// form.  Each kernel family is instantiated in its own translation unit.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <tuple>

#include "step_kernels.hpp"

namespace hhlb {

using Launcher = void (*)(const StageArgs &, hipStream_t);
// (quadrature kind, Q, functions (1 = f, 2 = f and chi), advection, precision,
//  shape: 2 = the two-wave stage kernels, 4 = the four-wave FP64 stage kernel,
//  1 = the fused kernel of a whole RK-3 step, 3 = the FP64 stage kernel across
//  classes, keyed by the largest order it holds)
using LaunchKey = std::tuple<int, int, int, int, int, int>;
using LaunchMap = std::map<LaunchKey, Launcher>;

void register_fp64(LaunchMap &m);
void register_fp64_q16(LaunchMap &m);
void register_mixed_f32(LaunchMap &m);
void register_mixed_bf16(LaunchMap &m);
void register_mixed_f16(LaunchMap &m);
void register_classes(LaunchMap &m);

// The node-parallel FP64 stage of large half-range classes (Q > 16):
// kernels_large.hip.
struct LargeArgs;
void launch_large(const LargeArgs &a, int adv, int H, hipStream_t s);

// The mixed-quadrature (App. A) velocity-space stage: kernels_multi.hip.
struct MultiArgs;
void launch_multi(const MultiArgs &a, hipStream_t s, int V, int k_doubles, int n_max);

}  // namespace hhlb
