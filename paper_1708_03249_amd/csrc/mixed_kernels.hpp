// gfx950 kernel for one TVD RK-3 stage of the half-range model in mixed
// precision.  The populations are kept as phi_k = f_k / w_k (and
// chi_k / w_k), which keeps every stored value of order one whatever the
// node weight.  Advection (WENO-5 / upwind-3), collision, the force
// contraction and the RK-3 combination run in FP32 arithmetic; the moment
// sums, the wall-density flux balance of Eq. (nplus_def) and the
// equilibrium coefficients stay in FP64.
//
// Storage.  A state rounded to FP32 at every step would lose the part of
// each step's increment below half an ulp, the same part every step once the
// flow is nearly steady: the slow modes then settle off the FP64 solution by
// about eps / (dt lambda) and the conserved mass drifts linearly.  So
//  * y^n is stored as an FP32 value hi plus a 16-bit correction word lo,
//    a fixed-point fraction of hi's ulp (y = hi + lo 2^(e-39) for
//    hi = m 2^e, m in [1/2, 1)), which carries y^n to about 2^-39;
//  * the two RK stage buffers hold increments, d1 = y1 - y^n and
//    d2 = y2 - y^n, in FP32, so their rounding is relative to the increment;
//  * the last stage adds (2/3)(d2 + dt L[y2]) to (hi, lo) with an exact
//    two-sum and writes the new (hi, lo) to the other copy of a ping-pong
//    pair (its stencil still reads the neighbours' hi).
// With the increments, stage s computes d_out = (1 - a_s)(d_in + dt L[y_s]),
// y_s = hi + d_in, a_s = 0, 3/4, 1/3 the weights of y^n in Eq. (rk3).  The force block -F (K y) is
// contracted on the matrix cores: FP32 MFMA (16 x 16 x 4) for the FP32 form
// at Q = 16, BF16 or FP16 MFMA (16 x 16 x 16, FP32 accumulation) for those
// forms at every Q (zero-padded to 16), and FP32 VALU otherwise.
//
// Thread mapping as in the FP64 half-range kernel: one 128-thread block per
// 64-cell window, wave 0 = p > 0 half, wave 1 = p < 0 half, one cell per lane.
#pragma once
#include "step_kernels.hpp"

// Launch shape of the mixed kernel (measured on the large workload):
// the moment partials share the tiles' LDS (17 KB per block instead of 23),
// four waves per SIMD (128 registers), y^n operands six node-functions ahead.
#ifndef HHLB_MIXED_ALIAS
#define HHLB_MIXED_ALIAS 1
#endif
#ifndef HHLB_PREFETCH_MIXED
#define HHLB_PREFETCH_MIXED 10
#endif
#ifndef HHLB_MIXED_WAVES
#define HHLB_MIXED_WAVES 4
#endif
// 1: keep the prologue's stage increments in registers for the combination
// instead of loading them again in pass 2
#ifndef HHLB_MIXED_KEEP_D
#define HHLB_MIXED_KEEP_D 0
#endif

namespace hhlb {

enum { kPrecF32 = 1, kPrecBF16 = 2, kPrecF16 = 3 };

__device__ __forceinline__ float dpp_shr1f(float x) {  // lane l <- lane l-1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_shl1f(float x) {  // lane l <- lane l+1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float readlane_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// WENO-5 face value in FP32: the construction of the FP64 form (product-form
// weights after an exact power-of-two rescaling, the limits of Table (weno)
// when sigmas vanish), with thresholds for the FP32 range.  After rescaling
// the largest q lies in [1/4, 1); a q below 1e-17 counts as vanishing, and
// the products are regular above 1e-37, which the pairs of non-vanishing q
// always exceed.
__device__ __forceinline__ float weno5f(float a, float b, float c, float d, float e) {
  const float k13 = 13.0f / 12.0f;
  float t1 = a - 2.0f * b + c, t2 = a - 4.0f * b + 3.0f * c;
  const float s1 = k13 * t1 * t1 + 0.25f * t2 * t2;
  t1 = b - 2.0f * c + d; t2 = b - d;
  const float s2 = k13 * t1 * t1 + 0.25f * t2 * t2;
  t1 = c - 2.0f * d + e; t2 = 3.0f * c - 4.0f * d + e;
  const float s3 = k13 * t1 * t1 + 0.25f * t2 * t2;
  const float F1 = 2.0f * a - 7.0f * b + 11.0f * c;
  const float F2 = -b + 5.0f * c + 2.0f * d;
  const float F3 = 2.0f * c + 5.0f * d - e;
  const int ex = __builtin_amdgcn_frexp_expf(fmaxf(s1, fmaxf(s2, s3)));
  const float r1 = ldexpf(s1, -ex), r2 = ldexpf(s2, -ex), r3 = ldexpf(s3, -ex);
  const float q1s = r1 * r1, q2s = r2 * r2, q3s = r3 * r3;
  const float p1 = 0.1f * q2s * q3s, p2 = 0.6f * q1s * q3s, p3 = 0.3f * q1s * q2s;
  float n1 = p1, n2 = p2, n3 = p3, dd = p1 + p2 + p3;
  if (!(dd > 1e-37f)) {   // limit rule, as in the FP64 form
    const float tiny = 1e-17f;
    n1 = q1s < tiny ? 0.1f : 0.0f;
    n2 = q2s < tiny ? 0.6f : 0.0f;
    n3 = q3s < tiny ? 0.3f : 0.0f;
    dd = n1 + n2 + n3;
  }
  // 1/6 of the candidate stencils folded into the normalisation
  return (n1 * F1 + n2 * F2 + n3 * F3) * __builtin_amdgcn_rcpf(6.0f * dd);
}

// Correction word of y = hi + lo: lo counts 2^-15 ulps of hi (|lo| <= 2^14).
__device__ __forceinline__ float lo_value(float hi, int16_t lo) {
  return ldexpf((float)lo, __builtin_amdgcn_frexp_expf(hi) - 39);
}
// y^n + delta -> (hi', lo'): the FP32 sum, and its exact rounding error
// (two-sum) stored as the correction word.
__device__ __forceinline__ void add_to_state(float hi, int16_t lo, float delta, float &hi_out, int16_t &lo_out) {
  const float t = lo_value(hi, lo) + delta;
  const float s = hi + t;
  const float bb = s - hi;
  const float e = (hi - (s - bb)) + (t - bb);
  hi_out = s;
  // |e| <= ulp(s)/2 gives |lo| <= 2^14 for normal s; the clamp only guards
  // denormal sums
  const float q = __builtin_rintf(ldexpf(e, 39 - __builtin_amdgcn_frexp_expf(s)));
  lo_out = (int16_t)fminf(fmaxf(q, -32767.0f), 32767.0f);
}

// Lane-parallel WENO-5 in FP32: the triple decomposition of weno5_lanes
// (FaceCoef) with the power-of-two rescaling of weno5f, which the FP32 range
// needs in smooth flow (unscaled products of four sigmas underflow there).
struct FaceCoefF {
  float dl, dc, dr, el, gl, ec, er, gr;
};
__device__ __forceinline__ FaceCoefF face_coef_f(int hw) {
  const FaceCoef c = face_coef(hw);
  return FaceCoefF{(float)c.dl, (float)c.dc, (float)c.dr, (float)c.el, (float)c.gl,
                   (float)c.ec, (float)c.er, (float)c.gr};
}
__device__ __forceinline__ float weno5f_lanes(float y, const FaceCoefF &c, bool used) {
  const float ym = dpp_shr1f(y), yp = dpp_shl1f(y);
  const float D2 = fmaf(-2.0f, y, ym) + yp;
  const float E = (float)kHalfKappa * (yp - ym);
  const float A = D2 * D2;
  const float bC = fmaf(E, E, A);
  const float tL = fmaf((float)kKappa, D2, E), tR = fmaf((float)kKappa, D2, -E);
  const float bL = fmaf(tL, tL, A), bR = fmaf(tR, tR, A);
  const float fL = fmaf(c.gl, D2, fmaf(c.el, E, y));
  const float fC = fmaf(1.0f / 12.0f, D2, fmaf(c.ec, E, y));
  const float fR = fmaf(c.gr, D2, fmaf(c.er, E, y));
  const float sL = dpp_shr1f(bL), FL = dpp_shr1f(fL);
  const float sR = dpp_shl1f(bR), FR = dpp_shl1f(fR);
  const int ex = __builtin_amdgcn_frexp_expf(fmaxf(sL, fmaxf(bC, sR)));
  const float rL = ldexpf(sL, -ex), rC = ldexpf(bC, -ex), rR = ldexpf(sR, -ex);
  const float qL = rL * rL, qC = rC * rC, qR = rR * rR;
  float wL = c.dl * (qC * qR), wC = c.dc * (qL * qR), wR = c.dr * (qL * qC);
  float dd = wL + wC + wR;
  if (!(dd > 1e-37f) && used) {   // limit rule, as in weno5f
    const float tiny = 1e-17f;
    wL = qL < tiny ? c.dl : 0.0f;
    wC = qC < tiny ? c.dc : 0.0f;
    wR = qR < tiny ? c.dr : 0.0f;
    dd = wL + wC + wR;
  }
  return fmaf(wL, FL, fmaf(wC, fC, wR * FR)) * __builtin_amdgcn_rcpf(dd);
}
// The same face values as deviations from the upwind cell's own value:
// returns fv - y (exact arithmetic), with dm = y_{i-1} - y_i and
// dp = y_{i+1} - y_i.  Every candidate and smoothness indicator is formed
// from these neighbour differences, which are exact in FP32 for neighbours
// within a factor two of each other, instead of from the values themselves:
// the rounding then scales with the differences rather than with y, and the
// flux difference the stage needs, v (y_i - y_{i-+1}) + v (dev_i - dev_{i-+1}),
// inherits that accuracy.
__device__ __forceinline__ float weno5f_lanes_dev(float y, const FaceCoefF &c, bool used, float &dm, float &dp) {
  const float ym = dpp_shr1f(y), yp = dpp_shl1f(y);
  dm = ym - y;
  dp = yp - y;
  const float D2 = dm + dp;
  const float E = (float)kHalfKappa * (dp - dm);
  const float A = D2 * D2;
  const float bC = fmaf(E, E, A);
  const float tL = fmaf((float)kKappa, D2, E), tR = fmaf((float)kKappa, D2, -E);
  const float bL = fmaf(tL, tL, A), bR = fmaf(tR, tR, A);
  // candidates of this lane's triple as deviations from the value of the
  // lane they are shifted to: y_m - y_{m+1} = -dp (to the right neighbour),
  // y_m - y_{m-1} = -dm (to the left one)
  const float fL = fmaf(c.gl, D2, fmaf(c.el, E, -dp));
  const float fC = fmaf(1.0f / 12.0f, D2, c.ec * E);
  const float fR = fmaf(c.gr, D2, fmaf(c.er, E, -dm));
  const float sL = dpp_shr1f(bL), FL = dpp_shr1f(fL);
  const float sR = dpp_shl1f(bR), FR = dpp_shl1f(fR);
  const int ex = __builtin_amdgcn_frexp_expf(fmaxf(sL, fmaxf(bC, sR)));
  const float rL = ldexpf(sL, -ex), rC = ldexpf(bC, -ex), rR = ldexpf(sR, -ex);
  const float qL = rL * rL, qC = rC * rC, qR = rR * rR;
  float wL = c.dl * (qC * qR), wC = c.dc * (qL * qR), wR = c.dr * (qL * qC);
  float dd = wL + wC + wR;
  if (!(dd > 1e-37f) && used) {   // limit rule, as in weno5f
    const float tiny = 1e-17f;
    wL = qL < tiny ? c.dl : 0.0f;
    wC = qC < tiny ? c.dc : 0.0f;
    wR = qR < tiny ? c.dr : 0.0f;
    dd = wL + wC + wR;
  }
  return fmaf(wL, FL, fmaf(wC, fC, wR * FR)) * __builtin_amdgcn_rcpf(dd);
}
__device__ __forceinline__ float upwind3f_lanes_dev(float y, const FaceCoefF &c, float &dm, float &dp) {
  const float ym = dpp_shr1f(y), yp = dpp_shl1f(y);
  dm = ym - y;
  dp = yp - y;
  const float D2 = dm + dp;
  const float E = (float)kHalfKappa * (dp - dm);
  return fmaf(1.0f / 12.0f, D2, c.ec * E);
}
template <int ADV>
__device__ __forceinline__ float face_dev_f_lanes(float y, const FaceCoefF &c, bool used, float &dm, float &dp) {
  if constexpr (ADV == 0) return weno5f_lanes_dev(y, c, used, dm, dp);
  else return upwind3f_lanes_dev(y, c, dm, dp);
}

__device__ __forceinline__ float upwind3f_lanes(float y, const FaceCoefF &c) {
  const float ym = dpp_shr1f(y), yp = dpp_shl1f(y);
  const float D2 = fmaf(-2.0f, y, ym) + yp;
  const float E = (float)kHalfKappa * (yp - ym);
  return fmaf(1.0f / 12.0f, D2, fmaf(c.ec, E, y));
}
template <int ADV>
__device__ __forceinline__ float face_value_f_lanes(float y, const FaceCoefF &c, bool used) {
  if constexpr (ADV == 0) return weno5f_lanes(y, c, used);
  else return upwind3f_lanes(y, c);
}

template <int ADV>
__device__ __forceinline__ float face_value_f(float a, float b, float c, float d, float e) {
  if constexpr (ADV == 0) return weno5f(a, b, c, d, e);
  else return (-b + 5.0f * c + 2.0f * d) * (1.0f / 6.0f);
}

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short bfx4 __attribute__((ext_vector_type(4)));
typedef _Float16 hfx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) { return __builtin_bit_cast(short, (__bf16)x); }
__device__ __forceinline__ float bf16_value(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }
// The value an operand has once rounded for the matrix cores.
template <int PREC>
__device__ __forceinline__ float operand_value(float x) {
  if constexpr (PREC == kPrecBF16) return __uint_as_float((uint32_t)(uint16_t)to_bf16(x) << 16);
  else if constexpr (PREC == kPrecF16) return (float)(_Float16)x;
  else return x;
}

// FP16 low parts are formed 2^11 times larger than the remainder they stand
// for: the remainder of an entry below FP16's normal range (2^-14) would
// otherwise fall into its subnormals, which keep only an absolute 2^-24.
// The products of the low parts are scaled back in FP32 before the product
// of the high parts is added.  BF16 has the FP32 exponent range: no scale.
constexpr float kF16LoScale = 2048.0f, kF16LoUnscale = 1.0f / 2048.0f;

// The value the matrix cores see for the low part of x (x = xh + remainder).
template <int PREC>
__device__ __forceinline__ float low_value(float x, float xh) {
  if constexpr (PREC == kPrecF16) return (float)(_Float16)((x - xh) * kF16LoScale) * kF16LoUnscale;
  else return operand_value<PREC>(x - xh);
}

// A operand of the force block for the matrix cores, built once per wave
// from the FP32 table Ks (H x H, row-major), zero outside the H x H block.
// Register layouts (checked on the GPU):
//   16x16x4 f32:        A[i][k] in lane i + 16 k (k < 4 per instruction)
//   16x16x16 bf16/f16:  A[i][k] in lane i + 16 (k / 4), element k % 4
//   both:               B[k][j] like A with j for i; D[i][j] in lane
//                       j + 16 (i / 4), accumulator register i % 4
template <int PREC>
struct ForceA;
template <>
struct ForceA<kPrecF32> {
  float v[4];
  template <int H>
  __device__ __forceinline__ void load(const float *Ks, int lane) {
    const int i = lane & 15;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int k = 4 * kc + (lane >> 4);
      v[kc] = (i < H && k < H) ? Ks[(i < H ? i : 0) * H + (k < H ? k : 0)] : 0.0f;
    }
  }
};
// BF16 / FP16: the table as a high part v (the entry rounded to the operand
// format) plus a low part lo (the remainder, exact in FP32, rounded again),
// so that the products carry about twice the operand precision.
template <>
struct ForceA<kPrecBF16> {
  bfx4 v, lo;
  template <int H>
  __device__ __forceinline__ void load(const float *Ks, int lane) {
    const int i = lane & 15;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = 4 * (lane >> 4) + t;
      const float x = (i < H && k < H) ? Ks[(i < H ? i : 0) * H + (k < H ? k : 0)] : 0.0f;
      v[t] = to_bf16(x);
      lo[t] = to_bf16(x - bf16_value(v[t]));
    }
  }
};
template <>
struct ForceA<kPrecF16> {   // loaded from the row-scaled table Ks16
  hfx4 v, lo;
  template <int H>
  __device__ __forceinline__ void load(const float *Ks, int lane) {
    const int i = lane & 15;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = 4 * (lane >> 4) + t;
      const float x = (i < H && k < H) ? Ks[(i < H ? i : 0) * H + (k < H ? k : 0)] : 0.0f;
      v[t] = (_Float16)x;
      lo[t] = (_Float16)((x - (float)v[t]) * kF16LoScale);
    }
  }
};

// OUT[i] = sum_k M[i][k] X[k] (i, k < H) for the 64 cells of the wave (one
// per lane), as four 16-cell products on the matrix cores.  The cell-major
// values go through the wave's padded LDS tile T (64 x 17 floats) into the
// B layout and back.
template <int PREC, int H>
__device__ __forceinline__ void mfma_force(const ForceA<PREC> &aM, const float X[H], float OUT[H], float *T,
                                           int lane) {
  constexpr int S = 17;
#pragma unroll
  for (int k = 0; k < H; ++k) T[lane * S + k] = X[k];
  __builtin_amdgcn_wave_barrier();
  flt4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    acc[cb] = flt4{0.0f, 0.0f, 0.0f, 0.0f};
    const float *row = T + (16 * cb + (lane & 15)) * S;
    if constexpr (PREC == kPrecF32) {
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int k = 4 * kc + (lane >> 4);
        const float b = k < H ? row[k < H ? k : 0] : 0.0f;
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aM.v[kc], b, acc[cb], 0, 0, 0);
      }
    } else {
      float bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 4 * (lane >> 4) + t;
        bv[t] = k < H ? row[k < H ? k : 0] : 0.0f;
      }
      // hi/lo split of both operands: Kh yh + Kh yl + Kl yh, the small
      // products first (the dropped Kl yl is below 2^-16 of |K||y| in BF16,
      // 2^-22 in FP16; the FP16 low parts come scaled by kF16LoScale)
      if constexpr (PREC == kPrecBF16) {
        bfx4 bh, bl;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          bh[t] = to_bf16(bv[t]);
          bl[t] = to_bf16(bv[t] - bf16_value(bh[t]));
        }
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aM.lo, bh, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aM.v, bl, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aM.v, bh, acc[cb], 0, 0, 0);
      } else {
        hfx4 bh, bl;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          bh[t] = (_Float16)bv[t];
          bl[t] = (_Float16)((bv[t] - (float)bh[t]) * kF16LoScale);
        }
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(aM.lo, bh, acc[cb], 0, 0, 0);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(aM.v, bl, acc[cb], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[cb][r] *= kF16LoUnscale;   // exact: a power of two
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16f16(aM.v, bh, acc[cb], 0, 0, 0);
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * cb + (lane & 15)) * S + 4 * (lane >> 4) + r] = acc[cb][r];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int k = 0; k < H; ++k) OUT[k] = T[lane * S + k];
  __builtin_amdgcn_wave_barrier();
}

template <int Q, int NFUN, int ADV, int PREC>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(HHLB_MIXED_WAVES))) void stage_kernel_mixed(
    StageArgs A, const DevTables *__restrict__ tb, const DevChannel *__restrict__ chans,
    const DevWindow *__restrict__ wins, const double *__restrict__ inv_dx,
    const double *__restrict__ gw, const float *__restrict__ hi_f, const float *__restrict__ hi_c,
    const float *__restrict__ d_f, const float *__restrict__ d_c) {
  constexpr int H = Q;
  constexpr int NC = NFUN;
  constexpr bool kMfmaEq = HHLB_MFMA && (H == 16);                          // FP64 equilibrium table
  constexpr bool kMfmaK = PREC != kPrecF32 || (HHLB_MFMA && H == 16);       // force block
  __shared__ double s_nw[2];
  // per-wave transpose tiles: 64 x 17 doubles for the FP64 equilibrium
  // table, 64 x 17 floats when only the force block uses the matrix cores
  constexpr int kTile = kMfmaEq ? 2 * 64 * 17 : (kMfmaK ? 64 * 17 : 1);
#if HHLB_MIXED_ALIAS
  // the moment partials share the tiles' memory (a barrier separates them)
  constexpr int kLds = kTile > 2 * 6 * 64 ? kTile : 2 * 6 * 64;
  __shared__ double s_lds[kLds];
  double (*s_part)[6][64] = reinterpret_cast<double (*)[6][64]>(s_lds);
  double *s_T = s_lds;
#else
  __shared__ double s_part[2][6][64];
  __shared__ double s_T[kTile];
#endif
  const int hw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int w = A.xcd_map ? xcd_window(blockIdx.x, A.nwin) : (int)blockIdx.x;
  const DevWindow win = wins[w];
  const DevChannel C = chans[win.ch];
  const int Nx = C.Nx;
  const int i = win.i0 - kHalo + lane;
  const bool inside = i >= 0 && i < Nx;
  const int kb0 = hw * H;
  const float sg = hw ? -1.0f : 1.0f;
  // stage value y_s = hi + d_in (d_in = 0 in the first stage)
  const bool has_d = A.stage != 0;
  const int64_t rbase = C.off + (int64_t)kb0 * Nx;
  float yf[H], yc[NC > 1 ? H : 1];
#if HHLB_MIXED_KEEP_D
  // the stage increments stay in registers for the combination of pass 2
  float kdf[H], kdc[NC > 1 ? H : 1];
#endif
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const int64_t o = rbase + (int64_t)j * Nx + i;
    const float dv = inside && has_d ? d_f[o] : 0.0f;
    yf[j] = inside ? hi_f[o] + dv : 0.0f;
#if HHLB_MIXED_KEEP_D
    kdf[j] = dv;
#endif
  }
  if constexpr (NC > 1) {
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int64_t o = rbase + (int64_t)j * Nx + i;
      const float dv = inside && has_d ? d_c[o] : 0.0f;
      yc[j] = inside ? hi_c[o] + dv : 0.0f;
#if HHLB_MIXED_KEEP_D
      kdc[j] = dv;
#endif
    }
  }

  // ---- closure, part 1: incoming ghosts (quadratic extrapolation) and the
  // wall density from the incoming wall-face fluxes, balanced in FP64 ----
  const bool needL = win.i0 < kHalo;
  const bool needR = win.i0 - kHalo + 63 >= Nx;
  double nw_mine = 0.0;
  if ((hw == 1 && needL) || (hw == 0 && needR)) {
    const bool left = hw == 1;
    const int l0 = left ? kHalo : Nx - 1 - (win.i0 - kHalo);
    const int dl = left ? 1 : -1;
    const int gi = left ? -i : i - Nx + 1;
    const float c0 = gi == 1 ? 3.0f : (gi == 2 ? 6.0f : 10.0f);
    const float c1 = gi == 1 ? -3.0f : (gi == 2 ? -8.0f : -15.0f);
    const float c2 = gi == 1 ? 1.0f : (gi == 2 ? 3.0f : 6.0f);
    const bool is_ghost = gi >= 1 && gi <= 3;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const float y0 = readlane_f(yf[j], l0), y1 = readlane_f(yf[j], l0 + dl),
                  y2 = readlane_f(yf[j], l0 + 2 * dl);
      if (lane == j) { a0 = y0; a1 = y1; a2 = y2; }
      if (is_ghost) yf[j] = c0 * y0 + c1 * y1 + c2 * y2;
      if constexpr (NC > 1) {
        const float x0 = readlane_f(yc[j], l0), x1 = readlane_f(yc[j], l0 + dl),
                    x2 = readlane_f(yc[j], l0 + 2 * dl);
        if (is_ghost) yc[j] = c0 * x0 + c1 * x1 + c2 * x2;
      }
    }
    const double d0 = a0, d1 = a1, d2 = a2;
    const double g1 = 3.0 * d0 - 3.0 * d1 + d2, g2 = 6.0 * d0 - 8.0 * d1 + 3.0 * d2;
    const double fv = face_value<ADV>(d2, d1, d0, g1, g2);
    // flux p_k f_k = (w_k p_k) phi_k, with the FP32 velocities of the
    // advection so that the balance holds for the fluxes the stage applies
    const double acc = wave_sum(lane < H ? tb->wpfq[kb0 + (lane < H ? lane : 0)] * fv : 0.0);
    nw_mine = -acc * (left ? C.inv_DL : C.inv_DR);
  }

  // ---- partial moments of this half (FP64) and the rank-1 projections ----
  double pn = 0.0, pm = 0.0, ps = 0.0, pc = 0.0, pbf = 0.0, pbc = 0.0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double y = yf[j];
    pn += tb->wq[j] * y;
    pm += tb->wpq[kb0 + j] * y;
    ps += tb->wp2q[kb0 + j] * y;
    pbf += tb->kbs[j] * y;
    if constexpr (NC > 1) {
      const double x = yc[j];
      pc += tb->wq[j] * x;
      pbc += tb->kbs[j] * x;
    }
  }
  s_part[hw][0][lane] = pn;
  s_part[hw][1][lane] = pm;
  s_part[hw][2][lane] = ps;
  s_part[hw][3][lane] = pc;
  s_part[hw][4][lane] = pbf;
  s_part[hw][5][lane] = pbc;
  if (lane == 0) s_nw[hw] = nw_mine;
  __syncthreads();
  double n = s_part[0][0][lane] + s_part[1][0][lane];
  double mom = s_part[0][1][lane] + s_part[1][1][lane];
  const double s2 = s_part[0][2][lane] + s_part[1][2][lane];
  const double ech = s_part[0][3][lane] + s_part[1][3][lane];
  const float bf = (float)(s_part[0][4][lane] + s_part[1][4][lane]);
  const float bc = (float)(s_part[0][5][lane] + s_part[1][5][lane]);
#if HHLB_MIXED_ALIAS
  __syncthreads();   // the tiles below overwrite the partials
#endif
  const double nL = s_nw[1], nR = s_nw[0];

  // ---- closure, part 2: emergent ghosts phi = n_w g^w_k / w_k ----
  if (hw == 0 && i < 0) {
    const double *gwL = gw + C.gw_off;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double ph = nL * gwL[j] * tb->iwq[j];
      yf[j] = (float)ph;
      if constexpr (NC > 1) yc[j] = (float)(C.half_Dt * C.TL * ph);
    }
  }
  if (hw == 1 && i >= Nx && i <= Nx + 2) {
    const double *gwR = gw + C.gw_off + 2 * H + H;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double ph = nR * gwR[j] * tb->iwq[j];
      yf[j] = (float)ph;
      if constexpr (NC > 1) yc[j] = (float)(C.half_Dt * C.TR * ph);
    }
  }
  if (A.nwall && A.stage == 2 && lane == 0) {
    if (hw == 1 && win.i0 == 0) A.nwall[2 * win.ch] = nL;
    if (hw == 0 && win.i0 <= Nx - 1 && Nx - 1 < win.i0 + kWin) A.nwall[2 * win.ch + 1] = nR;
  }

  // ---- moments (Eq. fmoms), FP64 ----
  if (!inside) n = 1.0, mom = 0.0;
  const double u = mom / n;
  double T = (s2 - u * mom + 2.0 * ech) * C.inv_1pDt / n;
  if (!inside) T = 1.0;

  // ---- equilibrium coefficients of this half (FP64, as in the FP64 form) ----
  double G[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) G[l] = 0.0;
  const bool collide = C.inv_Kn != 0.0;
  bool wide_wave = false;   // the correction rule lay beyond the calibrated ladder
  if (collide) {
    const double sT = sqrt(T);
    const double ub = (hw ? -u : u) * tb->inv_p0, s = sT * tb->inv_p0, y0 = -u / sT;
    auto accum = [&](double x, double wt) {
      double qm = 1.0, q = x - tb->a[0];
      G[0] += wt;
      if (Q > 1) G[1] += wt * q;
#pragma unroll
      for (int l = 1; l + 1 < Q; ++l) {
        const double qn = (x - tb->a[l]) * q - tb->mb[l] * qm;
        qm = q; q = qn;
        G[l + 1] += wt * q;
      }
    };
#pragma unroll 1
    for (int j = 0; j < tb->nm; ++j) accum(ub + s * tb->zm[j], tb->wm[j]);
    const double ymax = wave_max(inside ? fabs(y0) : 0.0);
    if (ymax > 0.0) {
      const int li = ladder_entry(tb, ymax);
      const int nc = tb->lad_n[li], o = tb->lad_off[li];
      const double sgd = hw ? -1.0 : 1.0;
      wide_wave = nc > tb->lad_n[kLadder - 1];
      for (int j = 0; j < nc; ++j) {
        const double t = tb->ltau[o + j];
        const double yt = y0 * t;
        const double e = y0 * tb->llamw[o + j] * exp(-0.5 * yt * yt);
        accum(ub * (1.0 - t), -sgd * e);
      }
    }
  }

  const bool out_lane = lane >= kHalo && lane < kHalo + kWin && inside;
  const int ic = inside ? i : 0;
  const float dx_inv = (float)inv_dx[C.cell_off + ic];
  const int64_t obase = C.off + (int64_t)kb0 * Nx;
  const float gforce = (float)C.g, dt = (float)C.dt;
  // lane i forms the face value at i+1/2 (hw = 0) or i-1/2 (hw = 1); the
  // other face of its cell comes from the neighbouring lane
  const FaceCoefF fcoef = face_coef_f(hw);
  const bool face_used = inside && lane >= kHalo - 1 + hw && lane < kHalo + kWin + hw;
  const bool wall_face = hw == 0 ? (i == -1) : (i == Nx);
  const float sdx = hw == 0 ? -dx_inv : dx_inv;   // L = sdx (F - F_other) + source

  // pass 1: local sources in FP32: -F (K y)_k - (y_k - y^eq_k)/tau
  float srcf[H], srcc[NC > 1 ? H : 1];
  {
    // BGK term (y_k - y^eq_k)/tau formed in FP64 and rounded once: a rounded
    // y^eq would bias the collision's mass, momentum and energy by one
    // rounding of the equilibrium per step, the same each step in a steady
    // state, while this keeps the error relative to y - y^eq
    float colf[H], colc[NC > 1 ? H : 1];
    const double itau = n * C.inv_Kn, eqc = C.half_Dt * T;
    auto bgk = [&](int j, double geq) {
      const double fe = n * geq;
      colf[j] = (float)(((double)yf[j] - fe) * itau);
      if constexpr (NC > 1) colc[j] = (float)(((double)yc[j] - eqc * fe) * itau);
    };
    if constexpr (kMfmaEq) {
      double aH[4];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) aH[kc] = tb->HWss[(lane & 15) * Q + 4 * kc + (lane >> 4)];
      double geq[H];
      mfma_contract16(aH, G, geq, s_T + hw * 64 * 17, lane);
#pragma unroll
      for (int j = 0; j < H; ++j) bgk(j, geq[j]);
    } else {
#pragma unroll
      for (int j = 0; j < H; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < Q; ++l) acc += tb->HWss[j * Q + l] * G[l];
        bgk(j, acc);
      }
    }
    float ky[H];
    if constexpr (kMfmaK) {
      ForceA<PREC> aK;
      aK.template load<H>(PREC == kPrecF16 ? tb->Ks16 : tb->Ks, lane);
      float *Tw = (float *)s_T + hw * (kMfmaEq ? 2 : 1) * 64 * 17;
#pragma unroll
      for (int fn = 0; fn < NC; ++fn) {
        const float *y = fn == 0 ? yf : yc;
        if constexpr (PREC == kPrecF32) {
          mfma_force<PREC, H>(aK, y, ky, Tw, lane);
        } else {
          // FP16: scale the cell by a power of two so that max |y| < 1
          float sc = 1.0f, isc = 1.0f;
          if constexpr (PREC == kPrecF16) {
            float m = 0.0f;
#pragma unroll
            for (int j = 0; j < H; ++j) m = fmaxf(m, fabsf(y[j]));
            const int e = __builtin_amdgcn_frexp_expf(m);
            sc = ldexpf(1.0f, -e);
            isc = ldexpf(1.0f, e);
          }
          float ys[H];
          // mass defect of the split product Kh (yh + yl) + Kl yh:
          // sum_j crs_j (yh_j + yl_j) + crs_lo_j yh_j (yh + yl is exact in FP32)
          float d = 0.0f;
#pragma unroll
          for (int j = 0; j < H; ++j) {
            ys[j] = y[j] * sc;
            const float yh = operand_value<PREC>(ys[j]), yl = low_value<PREC>(ys[j], yh);
            d = fmaf(tb->crs[j], yh + yl, fmaf(tb->crs_lo[j], yh, d));
          }
          mfma_force<PREC, H>(aK, ys, ky, Tw, lane);
          const float dc = d * isc * tb->iwh;
#pragma unroll
          for (int j = 0; j < H; ++j) {
            const float o = PREC == kPrecF16 ? ky[j] * tb->irsc[j] : ky[j];
            ky[j] = o * isc - dc;
          }
        }
        const float bb = fn == 0 ? bf : bc;
#pragma unroll
        for (int j = 0; j < H; ++j) {
          if (fn == 0) srcf[j] = -gforce * sg * (ky[j] + tb->kas[j] * bb) - colf[j];
          else if constexpr (NC > 1) srcc[j] = -gforce * sg * (ky[j] + tb->kas[j] * bb) - colc[j];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < H; ++j) {
        float kf = 0.0f, kc = 0.0f;
#pragma unroll
        for (int jj = 0; jj < H; ++jj) {
          const float kv = tb->Ks[j * H + jj];
          kf += kv * yf[jj];
          if constexpr (NC > 1) kc += kv * yc[jj];
        }
        srcf[j] = -gforce * sg * (kf + tb->kas[j] * bf) - colf[j];
        if constexpr (NC > 1) srcc[j] = -gforce * sg * (kc + tb->kas[j] * bc) - colc[j];
      }
    }
  }
  // keep the finished sources in registers: without this fence the compiler
  // sinks their terms into pass 2 and holds several values per node
#pragma unroll
  for (int j = 0; j < H; ++j) {
    asm volatile("" : "+v"(srcf[j]));
    if constexpr (NC > 1) asm volatile("" : "+v"(srcc[j]));
  }

  // pass 2: advection and the RK-3 combination, FP32, in increment form.
  // The stage increment (and, in the last stage, hi and lo of y^n) are
  // loaded HHLB_PREFETCH_MIXED node-functions ahead of their use.
  const bool last = A.stage == 2;
  constexpr int NSEC = H * NC;
  constexpr int PD = HHLB_PREFETCH_MIXED < NSEC ? HHLB_PREFETCH_MIXED : NSEC;
  // uniform base of population row r of an array, opaque at its point of
  // use: otherwise the compiler precomputes the bases of every row up front
  // and spills them
  auto row = [&](auto *base, int r) {
    auto *p = base + obase + (int64_t)r * Nx;
    asm volatile("" : "+s"(p));
    return p;
  };
  float dq[PD], hq[PD];
  int16_t lq[PD];
  auto fetch = [&](int sec, int slot) {
    const int r = sec / NC;
    const bool f0 = (sec % NC) == 0;
#if HHLB_MIXED_KEEP_D
    dq[slot] = 0.0f;
#else
    dq[slot] = has_d ? row(f0 ? d_f : d_c, r)[ic] : 0.0f;
#endif
    if (last) {
      hq[slot] = row(f0 ? hi_f : hi_c, r)[ic];
      lq[slot] = row(f0 ? A.lo_in_f : A.lo_in_c, r)[ic];
    } else {
      hq[slot] = 0.0f;
      lq[slot] = 0;
    }
  };
#pragma unroll
  for (int d = 0; d < PD; ++d) fetch(d, d);
  const float b_inc = (float)A.b_stage;   // 1 - a_s
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const float v = tb->pf[kb0 + j];
#pragma unroll
    for (int fn = 0; fn < NC; ++fn) {
      const int sec = j * NC + fn;
#if HHLB_MIXED_KEEP_D
      const float din = fn == 0 ? kdf[j] : kdc[NC > 1 ? j : 0];
#else
      const float din = dq[sec % PD];
#endif
      const float hi = hq[sec % PD];
      const int16_t lo = lq[sec % PD];
      if (sec + PD < NSEC) fetch(sec + PD, sec % PD);
      const float y0v = fn == 0 ? yf[j] : yc[j];
      const float src = fn == 0 ? srcf[j] : srcc[j];
      // flux difference from the face values' deviations: F_i - F_other =
      // v (y_i - y_other) + v (dev_i - dev_other), the other face's lane being
      // i-1 (hw = 0) or i+1 (hw = 1); the wall face's value is imposed as the
      // ghost itself (deviation 0)
      float dm, dp;
      float dev = face_dev_f_lanes<ADV>(y0v, fcoef, face_used, dm, dp);
      if (wall_face) dev = 0.0f;
      const float Fd = v * dev;
      const float Fdo = hw == 0 ? dpp_shr1f(Fd) : dpp_shl1f(Fd);
      const float L = fmaf(sdx, fmaf(v, hw == 0 ? -dm : -dp, Fd - Fdo), src);
      const float inc = b_inc * (din + dt * L);
      if (!last) {
        if (out_lane) row((float *)(fn == 0 ? A.out_f : A.out_c), j)[ic] = inc;
      } else {
        float hn;
        int16_t ln;
        add_to_state(hi, lo, inc, hn, ln);
        if (out_lane) {
          row((float *)(fn == 0 ? A.out_f : A.out_c), j)[ic] = hn;
          row(fn == 0 ? A.lo_out_f : A.lo_out_c, j)[ic] = ln;
        }
      }
      // a scheduling fence after every HHLB_SCHED_GROUP node-functions:
      // interleaving more unrolled WENO evaluations exceeds the register file
      if ((j * NC + fn + 1) % HHLB_SCHED_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
    }
  }
  // waves whose correction lay beyond the calibrated ladder, counted once the
  // registers of the step are free
  if (wide_wave && lane == 0 && A.wide) atomicAdd(A.wide, 1ull);
}

}  // namespace hhlb
