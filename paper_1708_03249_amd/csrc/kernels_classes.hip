// FP64 stage kernels that take the windows of several half-range model
// classes in one launch per stage (one block per window, or persistent
// blocks that take windows in turn).
#include <algorithm>

#include "launch.hpp"

namespace hhlb {
namespace {

template <int QTOP, int NF, int ADV>
void launch_classes(const StageArgs &a, hipStream_t s) {
  const auto *w = reinterpret_cast<const DevClassWindow *>(a.wins);
  if (a.nblocks < 0) {
    // persistent: as many blocks as the current device holds at once
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_kernel_classes<QTOP, NF, ADV, true>, 128, 0);
    const int blocks = std::max(1, std::min(a.nwin, cus * per_cu));
    hipLaunchKernelGGL((stage_kernel_classes<QTOP, NF, ADV, true>), dim3(blocks), dim3(128), 0, s, a, a.tb,
                       a.chans, w, a.inv_dx, a.gw, (const double *)a.in_f, (const double *)a.in_c);
  } else {
    hipLaunchKernelGGL((stage_kernel_classes<QTOP, NF, ADV, false>), dim3(a.nwin), dim3(128), 0, s, a, a.tb,
                       a.chans, w, a.inv_dx, a.gw, (const double *)a.in_f, (const double *)a.in_c);
  }
}

template <int QTOP>
void add(LaunchMap &m) {
  m[{0, QTOP, 1, 0, 0, 3}] = launch_classes<QTOP, 1, 0>;
  m[{0, QTOP, 1, 1, 0, 3}] = launch_classes<QTOP, 1, 1>;
  m[{0, QTOP, 2, 0, 0, 3}] = launch_classes<QTOP, 2, 0>;
  m[{0, QTOP, 2, 1, 0, 3}] = launch_classes<QTOP, 2, 1>;
}

}  // namespace

void register_classes(LaunchMap &m) {
  add<8>(m); add<12>(m); add<16>(m);
}

}  // namespace hhlb
