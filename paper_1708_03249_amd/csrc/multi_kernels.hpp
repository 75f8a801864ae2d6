// Mixed-quadrature velocity space in d = 2 or 3 dimensions (App. A) for a
// spatially homogeneous gas: the right-hand side of Eq. (boltz_multi_k)
// without the advection term,
//   L_v = - sum_a F_a (K_a f)_v - (f_v - feq_v) n / Kn,
// on the direct-product velocity set (App. A.1), with feq = n g_x g_y [g_z]
// from the point's n, u, T (App. A.2) and one 1-D contraction per axis for
// the force (App. A.3); one RK-3 stage per launch (Eq. rk3).
//
// The kernel itself is in kernels_multi.hip.  W lanes per point: 16 (four
// points per wave) for V <= 128, else 64 (one point per wave); four waves
// per block.  f is point-major (V doubles per point, velocity
// v = (i V_y + j) V_z + k, x slowest), so a point's populations are one
// contiguous run; lane s of a point's segment holds velocities s + W t and
// the populations sit in LDS for the contractions.  The per-axis
// equilibrium coefficients come from axis_coeffs (the same wave-level code
// as the 1-D large-velocity-set path).
#pragma once
#include "large_kernels.hpp"

namespace hhlb {

constexpr int kMultiAxes = 3;
constexpr int kMultiVaxis = 32;    // velocities per axis
constexpr int kMultiVmax = 512;    // velocities of the product set
constexpr int kMultiWaves = 4;     // points per block

// The kernel stages each K_a in LDS with its rows padded by zeros to a
// multiple of HHLB_MULTI_GROUP columns, and contracts a row that many columns
// at a time (the loads of a group issue together, one LDS wait per group).
#ifndef HHLB_MULTI_GROUP
#define HHLB_MULTI_GROUP 4
#endif
constexpr int kMultiGroup = HHLB_MULTI_GROUP;
static_assert(kMultiGroup >= 1 && kMultiVaxis % kMultiGroup == 0, "group width");
// 1: the kernel loads y^n with the populations; 0: just before the contractions.
#ifndef HHLB_MULTI_YN_EARLY
#define HHLB_MULTI_YN_EARLY 0
#endif
// Waves per SIMD the compiler must fit the registers of the instances for
// orders <= 7 to (0: its own choice).  Five fit the LDS of a block; the
// W = 16 instance then keeps 96 VGPRs with a 12-byte spill.
#ifndef HHLB_MULTI_OCC
#define HHLB_MULTI_OCC 5
#endif
__host__ __device__ inline int multi_kcols(int Va) { return (Va + kMultiGroup - 1) / kMultiGroup * kMultiGroup; }

// Tables of one product set.  The trailing doubles hold, per axis a, the
// momenta p_a[V_a] at p_off[a], the 1-D matrix K_a[V_a][V_a] (row-major) at
// k_off[a] and the equilibrium table HWs_a[H_a][N_a + 1] at hw_off[a]; after
// them (idx_off doubles in) V int32 words, byte a of word v the axis-a
// index of velocity v.
struct DevMulti {
  int32_t d, V;
  int32_t Va[kMultiAxes], stride[kMultiAxes];
  int32_t p_off[kMultiAxes], k_off[kMultiAxes], hw_off[kMultiAxes];
  int32_t idx_off;
  DevLarge ax[kMultiAxes];
};

struct MultiArgs {
  const DevMulti *tm;
  const double *tab;               // the trailing doubles
  const double *in, *base;         // stage state, y^n
  double *out;
  int64_t npts;
  double F[kMultiAxes];            // acceleration (m = 1)
  double inv_Kn, dt, a_base, b_stage;
  int32_t rhs_only;                // 1: out = L[in]
};

}  // namespace hhlb
