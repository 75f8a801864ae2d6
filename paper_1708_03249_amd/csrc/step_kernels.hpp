// gfx950 kernels for one TVD RK-3 stage of the half-range (HHLB) and
// full-range (HLB) lattice Boltzmann models with a force term.
//
// Mapping: one 64-lane wavefront per "window" of 64 consecutive cells of one
// channel; lanes 3..60 own the 58 output cells, lanes 0..2 and 61..63 are the
// 3-cell halo of the WENO-5 stencil.  Each lane keeps every velocity node of
// its cell in registers (structure-of-arrays loads, one coalesced row per
// node), so the per-cell algebra (moments, equilibrium, force matrix, BGK) is
// lane-local and the x-neighbours of the stencil come from DPP wave shifts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hhlb {

constexpr int kQmaxDev = 16;   // largest per-half order with a kernel
constexpr int kNc = 8;         // Gauss-Legendre points of the full-range kernel's correction
constexpr int kLadder = 8;     // calibrated correction point counts the half-range kernel chooses from
constexpr int kComposite = 6;  // beyond them: the top count on 2, 4, .., 64 panels
constexpr int kLadderAll = kLadder + kComposite;
constexpr int kLadderTop = 16; // the top calibrated count
constexpr int kLadderPts = 64 + kLadderTop * (2 + 4 + 8 + 16 + 32 + 64);   // points over all entries
constexpr int kWin = 58;       // output cells per wavefront

// Build-time tuning switches of the half-range kernel: matrix cores for the
// two 16 x 16 contractions (Q = 16), the moment partials sharing the
// transpose tiles' LDS, and the occupancy target.
#ifndef HHLB_MFMA
#define HHLB_MFMA 1
#endif
#ifndef HHLB_HALF_ALIAS
#define HHLB_HALF_ALIAS 1
#endif
#ifndef HHLB_HALF_WAVES
#define HHLB_HALF_WAVES 3
#endif
#ifndef HHLB_QUARTER_WAVES
#define HHLB_QUARTER_WAVES 4
#endif
// node-functions per scheduling section in the advection pass
#ifndef HHLB_SCHED_GROUP
#define HHLB_SCHED_GROUP 1
#endif
// how many node-functions ahead the advection pass loads the values of y^n
// (the mixed kernel has its own distance, HHLB_PREFETCH_MIXED)
#ifndef HHLB_PREFETCH
#define HHLB_PREFETCH 16
#endif
constexpr int kHalo = 3;

// Per model class (quadrature, Q, N, p0): uploaded once.
struct DevTables {
  double p[2 * 256];                      // p_k / m (every node, also of the large-Q classes)
  double z[kQmaxDev], w[kQmaxDev];        // positive nodes (units of p0), weights
  double a[kQmaxDev + 2];                 // recurrence: sqrt(b_{l+1}) h_{l+1} = (z-a_l) h_l - sqrt(b_l) h_{l-1}
  double sb[kQmaxDev + 3];                // sqrt(b_l)
  double isb[kQmaxDev + 3];               // 1/sqrt(b_l)
  double Kin[kQmaxDev * kQmaxDev];        // half: + half within block (H x H); full: dense V x V
  double ka[kQmaxDev], kb[kQmaxDev];      // half: rank-1 cross term
  double HW[2 * kQmaxDev * kQmaxDev];     // half: H x Q; full: V x Q (zero beyond N)
  double tau[kNc], lamw[kNc];             // GL nodes in (0,1), weights * 1/sqrt(2 pi)
  double inv_p0;
  // half-range kernel: monic recurrence q_{l+1} = (x - a_l) q_l - b_l q_{l-1}
  double mb[kQmaxDev + 2];                // b_l
  double HWs[kQmaxDev * kQmaxDev];        // H x Q: w_k h_l(z_k) / sqrt(b_0 .. b_l) (zero beyond N)
  // correction ladder: count lad_n[j] is exact enough up to |y0| <= lad_y[j];
  // entries kLadder.. are composite rules of the top count (2^(j-kLadder+1)
  // panels over [y0, 0], each panel within the top count's reach)
  int lad_n[kLadderAll], lad_off[kLadderAll];
  double lad_y[kLadderAll];
  double ltau[kLadderPts], llamw[kLadderPts];
  // main-part rule of the equilibrium: the M-point half-range Gauss rule,
  // M = ceil((N+1)/2), exact for the degree-N integrands
  int nm;
  double zm[kQmaxDev], wm[kQmaxDev];
  // mixed-precision form: the state is kept as phi_k = f_k / w_k, so the
  // half-range tables are rescaled by the node weights
  double wq[kQmaxDev], iwq[kQmaxDev];     // w_k, 1/w_k of a half
  double wpq[2 * kQmaxDev];               // w_k p_k/m (both halves)
  double wpfq[2 * kQmaxDev];              // w_k (p_k/m rounded to FP32): the wall-flux balance uses
                                          // the velocities the FP32 advection uses
  double wp2q[2 * kQmaxDev];              // w_k (p_k/m)^2
  double kbs[kQmaxDev];                   // kb_j w_j
  double HWss[kQmaxDev * kQmaxDev];       // HWs[k][l] / w_k
  float Ks[kQmaxDev * kQmaxDev];          // Kin[k][j] w_j / w_k
  float kas[kQmaxDev];                    // ka_k / w_k
  float pf[2 * kQmaxDev];                 // p_k/m
  // reduced-precision force operands (BF16 / FP16 forms): the FP16 table is
  // Ks with row k scaled by rsc_k (a power of two, |row| <= 1) and irsc_k =
  // 1/rsc_k.  The matrix cores see the table as a high part Kh (the operand
  // rounding of it) plus a low part Kl (the rounding of the remainder);
  // crs_j = sum_k w_k Kh_kj and crs_lo_j = sum_k w_k Kl_kj are their weighted
  // column sums exactly as rounded, whose mass defect the kernel removes;
  // iwh = 1 / sum over a half of w_k
  float Ks16[kQmaxDev * kQmaxDev];
  float irsc[kQmaxDev];
  float crs[kQmaxDev];
  float crs_lo[kQmaxDev];                 // the same sums for the table's low part (hi/lo split)
  float iwh;
};

// Per channel.
struct DevChannel {
  int64_t off;        // offset (doubles) of this channel in each state array
  int32_t Nx;
  int32_t cell_off;   // offset of this channel's cells in per-cell arrays
  int32_t gw_off;     // offset of the wall equilibria (2V doubles: left, right)
  int32_t pad;
  double g;           // acceleration (F = m g)
  double inv_Kn;      // 1/Kn (0 when collisionless)
  double dt;
  double TL, TR;      // wall temperatures
  double inv_DL;      // 1 / sum_{p_k>0} (p_k/m) gwL_k  (mixed form: p_k/m rounded to FP32)
  double inv_DR;      // 1 / sum_{p_k<0} (p_k/m) gwR_k
  double half_Dt;     // Dt/2
  double inv_1pDt;    // 1/(1+Dt)
};

// Window: channel id and first output cell.
struct DevWindow {
  int32_t ch;
  int32_t i0;
};

struct StageArgs {
  const DevTables *tb;
  const DevChannel *chans;
  const DevWindow *wins;
  int32_t nwin;
  int32_t stage;             // 0, 1, 2 (only stage 2 writes the wall densities)
  int32_t xcd_map;           // 1: XCD-aware block -> window mapping, 0: identity
  int32_t nblocks;           // launch across classes: blocks (0: one per window)
  const double *inv_dx;      // per cell
  const double *gw;          // wall equilibria
  // state arrays: double (FP64 form) or float (mixed form)
  const void *in_f, *in_c;   // stage state
  const void *base_f, *base_c;  // y^n (pointwise)
  void *out_f, *out_c;
  double a_base, b_stage;    // out = a_base * y^n + b_stage * (y_s + dt L[y_s])
  double *nwall;             // 2 per channel (may be null)
  // count of waves whose equilibrium needed more than one correction panel
  // (|y0| beyond the calibrated range of the ladder; may be null)
  unsigned long long *wide;
  // mixed form only: 16-bit correction words of y^n (read in the last stage)
  // and of y^{n+1} (written there)
  const int16_t *lo_in_f, *lo_in_c;
  int16_t *lo_out_f, *lo_out_c;
};

__device__ __forceinline__ double dpp_shr1(double x) {  // lane l <- lane l-1
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_shl1(double x) {  // lane l <- lane l+1
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_readlane(lo, l);
  hi = __builtin_amdgcn_readlane(hi, l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// 1/x for normal, finite x > 0: the hardware estimate refined by two
// Newton-Raphson steps (within an ulp or so; the weights it scales are
// renormalised anyway).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// WENO-5 face value (Eqs. weno5_flux, weno5_omega, weno_sigma) for the
// upwind-ordered stencil (a..e) = (f_{i-2}, .., f_{i+2}), with the limits of
// Table (weno) when smoothness indicators vanish.  The weights are formed as
// delta_q prod_{r!=q} sigma_r^2 (mathematically delta_q/sigma_q^2 times the
// common factor prod_r sigma_r^2) after an exact power-of-two rescaling of
// the sigmas; when that product underflows the limit rule is applied.
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e) {
  const double k13 = 13.0 / 12.0;
  double t1 = a - 2.0 * b + c, t2 = a - 4.0 * b + 3.0 * c;
  const double s1 = k13 * t1 * t1 + 0.25 * t2 * t2;
  t1 = b - 2.0 * c + d; t2 = b - d;
  const double s2 = k13 * t1 * t1 + 0.25 * t2 * t2;
  t1 = c - 2.0 * d + e; t2 = 3.0 * c - 4.0 * d + e;
  const double s3 = k13 * t1 * t1 + 0.25 * t2 * t2;
  const double F1 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
  const double F2 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
  const double F3 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
  // exact power-of-two rescaling so that the largest sigma lies in [0.5, 1)
  // (all-zero sigmas stay zero and fall through to the limit rule)
  const int ex = __builtin_amdgcn_frexp_exp(fmax(s1, fmax(s2, s3)));
  const double r1 = ldexp(s1, -ex), r2 = ldexp(s2, -ex), r3 = ldexp(s3, -ex);
  const double q1s = r1 * r1, q2s = r2 * r2, q3s = r3 * r3;
  const double p1 = 0.1 * q2s * q3s, p2 = 0.6 * q1s * q3s, p3 = 0.3 * q1s * q2s;
  double n1 = p1, n2 = p2, n3 = p3, dd = p1 + p2 + p3;
  if (!(dd > 1e-250)) {
    // limit of Table (weno): ideal weights restricted to the vanishing
    // sigmas (a branch no lane takes in smooth flow, so the common path
    // carries no selects)
    const double tiny = 1e-125;
    n1 = q1s < tiny ? 0.1 : 0.0;
    n2 = q2s < tiny ? 0.6 : 0.0;
    n3 = q3s < tiny ? 0.3 : 0.0;
    dd = n1 + n2 + n3;
  }
  return (n1 * F1 + n2 * F2 + n3 * F3) * recip(dd);
}

// Lane-parallel WENO-5 of the half-range kernels: lane i holds cell i.
// Every smoothness indicator and candidate value of Eqs. (weno_sigma) and
// (weno5_flux) depends on one triple of consecutive cells.  With
// D2 = y_{m-1} - 2 y_m + y_{m+1} and D1 = y_{m+1} - y_{m-1} of the triple
// centred on cell m:
//   sigma: 13/12 D2^2 + (D2 + D1/2)^2,  13/12 D2^2 + (D1/2)^2,  13/12 D2^2 + (D2 - D1/2)^2
//   F:     y_m + a D1 + b D2, (a, b) in {(+-3/4, 13/12), (+-1/4, 1/12)}.
// Each lane evaluates them once for its own triple; the candidates of the
// triples centred on i-1 and i+1 arrive by one DPP shift each.  The sigmas
// are all scaled by 12/13 (a common factor cancels in the weights), which
// leaves D2^2 + (kappa (D2 +- D1/2))^2 with kappa = sqrt(12/13).
//   hw = 0 (p > 0): value at the face i+1/2 from cells i-2..i+2;
//   hw = 1 (p < 0): value at the face i-1/2 from cells i+2..i-2 (mirrored).
// The ideal weights (0.1, 0.6, 0.3) of the upwind-ordered candidates then
// belong to the triples (i-1, i, i+1) for hw = 0 and (i+1, i, i-1) for hw = 1.
struct FaceCoef {
  double dl, dc, dr;   // ideal weights of the triples centred on i-1, i, i+1
  double el, gl;       // candidate of triple i-1: y + el E + gl D2 (E = kappa D1 / 2)
  double ec;           // candidate of triple i:   y + ec E + D2 / 12
  double er, gr;       // candidate of triple i+1
};
constexpr double kKappa = 0.9607689228305228;         // sqrt(12/13)
constexpr double kHalfKappa = 0.4803844614152614;     // sqrt(12/13) / 2
__device__ __forceinline__ FaceCoef face_coef(int hw) {
  const double h = 1.0 / (2.0 * kKappa);   // a = 1/4 in units of E
  if (hw == 0) return FaceCoef{0.1, 0.6, 0.3, 3.0 * h, 13.0 / 12.0, h, -h, 1.0 / 12.0};
  return FaceCoef{0.3, 0.6, 0.1, h, 1.0 / 12.0, -h, -3.0 * h, 13.0 / 12.0};
}

// The face value of the lane's cell (see FaceCoef).  `used` marks lanes whose
// value is consumed: only they may send the wave into the rescaling branch.
// The product-form weights delta_q prod_{r!=q} sigma_r^2 are formed directly;
// when their sum leaves [1e-290, 1e290] the sigmas are rescaled by an exact
// power of two and, if the sum still underflows, the limit of Table (weno)
// applies (as in weno5).
__device__ __forceinline__ double weno5_lanes(double y, const FaceCoef &c, bool used) {
  const double ym = dpp_shr1(y), yp = dpp_shl1(y);
  const double D2 = fma(-2.0, y, ym) + yp;
  const double E = kHalfKappa * (yp - ym);
  const double A = D2 * D2;
  const double bC = fma(E, E, A);
  const double tL = fma(kKappa, D2, E), tR = fma(kKappa, D2, -E);
  const double bL = fma(tL, tL, A), bR = fma(tR, tR, A);
  const double fL = fma(c.gl, D2, fma(c.el, E, y));
  const double fC = fma(1.0 / 12.0, D2, fma(c.ec, E, y));
  const double fR = fma(c.gr, D2, fma(c.er, E, y));
  const double sL = dpp_shr1(bL), FL = dpp_shr1(fL);
  const double sR = dpp_shl1(bR), FR = dpp_shl1(fR);
  double qL = sL * sL, qC = bC * bC, qR = sR * sR;
  double wL = c.dl * (qC * qR), wC = c.dc * (qL * qR), wR = c.dr * (qL * qC);
  double dd = wL + wC + wR;
  if (!(dd > 1e-290 && dd < 1e290) && used) {
    const int ex = __builtin_amdgcn_frexp_exp(fmax(sL, fmax(bC, sR)));
    const double rL = ldexp(sL, -ex), rC = ldexp(bC, -ex), rR = ldexp(sR, -ex);
    qL = rL * rL; qC = rC * rC; qR = rR * rR;
    wL = c.dl * (qC * qR); wC = c.dc * (qL * qR); wR = c.dr * (qL * qC);
    dd = wL + wC + wR;
    if (!(dd > 1e-250)) {
      const double tiny = 1e-125;
      wL = qL < tiny ? c.dl : 0.0;
      wC = qC < tiny ? c.dc : 0.0;
      wR = qR < tiny ? c.dr : 0.0;
      dd = wL + wC + wR;
    }
  }
  return fma(wL, FL, fma(wC, fC, wR * FR)) * recip(dd);
}

// Third-order upwind value of the lane's cell in the same orientation:
// (-y_{i-1} + 5 y_i + 2 y_{i+1})/6 (hw = 0), (2 y_{i-1} + 5 y_i - y_{i+1})/6
// (hw = 1), i.e. the central candidate y + ec E + D2/12.
__device__ __forceinline__ double upwind3_lanes(double y, const FaceCoef &c) {
  const double ym = dpp_shr1(y), yp = dpp_shl1(y);
  const double D2 = fma(-2.0, y, ym) + yp;
  const double E = kHalfKappa * (yp - ym);
  return fma(1.0 / 12.0, D2, fma(c.ec, E, y));
}

template <int ADV>
__device__ __forceinline__ double face_value_lanes(double y, const FaceCoef &c, bool used) {
  if constexpr (ADV == 0) return weno5_lanes(y, c, used);
  else return upwind3_lanes(y, c);
}

// Third-order upwind-biased face value (-f_{i-1} + 5 f_i + 2 f_{i+1})/6.
__device__ __forceinline__ double upwind3(double b, double c, double d) {
  return (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
}

template <int ADV>
__device__ __forceinline__ double face_value(double a, double b, double c, double d, double e) {
  if constexpr (ADV == 0) return weno5(a, b, c, d, e);
  else return upwind3(b, c, d);
}

// Map a block index to a window so that consecutive windows (which share
// halo cells) are dispatched to the same XCD (blocks go round-robin over 8).
__device__ __forceinline__ int xcd_window(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = b & 7, pos = b >> 3;
  return x * q + (x < r ? x : r) + pos;
}

// The correction rule of a wave whose largest |y0| is ymax (a scalar): the
// first ladder entry, calibrated or composite, whose reach covers it; the
// last (64 panels of the top count) when none does, also for a non-finite
// ymax.  Entries beyond the calibrated ones hold more points than the top
// count, which is how the kernels count such waves.
__device__ __forceinline__ int ladder_entry(const DevTables *tb, double ymax) {
  int li = kLadderAll - 1;
  for (int j = 1; j < kLadderAll; ++j)
    if (tb->lad_y[j] >= ymax) { li = j; break; }
  return li;
}

// Wall density of Eq. (nplus_def): n_w = -sum_in F_k / sum_out (p_k/m) g^w_k,
// with the incoming fluxes reconstructed from ghosts extrapolated
// quadratically from the first three interior cells (Sec. IV.C.3).
// left: incoming nodes k >= H use cells 0,1,2; right: nodes k < H use
// cells Nx-1, Nx-2, Nx-3.  Lane j handles incoming node j.
template <int V, int ADV>
__device__ __forceinline__ double wall_density(const DevTables *tb, const double *fin, int Nx,
                                               bool left, double inv_D) {
  constexpr int H = V / 2;
  const int lane = threadIdx.x;
  double contrib = 0.0;
  if (lane < H) {
    const int k = left ? H + lane : lane;
    const double *row = fin + (int64_t)k * Nx;
    double y0, y1, y2;  // nearest, second, third interior cell from the wall
    if (left) { y0 = row[0]; y1 = row[1]; y2 = row[2]; }
    else { y0 = row[Nx - 1]; y1 = row[Nx - 2]; y2 = row[Nx - 3]; }
    double gh1 = 3.0 * y0 - 3.0 * y1 + y2;        // first ghost
    double gh2 = 6.0 * y0 - 8.0 * y1 + 3.0 * y2;  // second ghost
    // upwind-ordered stencil for the wall face (flow towards the wall)
    double fv = face_value<ADV>(y2, y1, y0, gh1, gh2);
    contrib = tb->p[k] * fv;
  }
  return -wave_sum(contrib) * inv_D;
}

template <int QUAD, int Q, int NFUN, int ADV>
__global__ __launch_bounds__(64) void stage_kernel(StageArgs A) {
  constexpr int V = QUAD == 0 ? 2 * Q : Q;
  constexpr int H = V / 2;
  constexpr int NC = NFUN;
  const int w = A.xcd_map ? xcd_window(blockIdx.x, A.nwin) : (int)blockIdx.x;
  const DevWindow win = A.wins[w];
  const DevChannel C = A.chans[win.ch];
  const DevTables *__restrict__ tb = A.tb;
  const int lane = threadIdx.x;
  const int Nx = C.Nx;
  const int i = win.i0 - kHalo + lane;
  const bool inside = i >= 0 && i < Nx;
  const double *fin = (const double *)A.in_f + C.off;
  const double *cin = NC > 1 ? (const double *)A.in_c + C.off : nullptr;

  double yf[V], yc[NC > 1 ? V : 1];
#pragma unroll
  for (int k = 0; k < V; ++k) yf[k] = inside ? fin[(int64_t)k * Nx + i] : 0.0;
  if constexpr (NC > 1) {
#pragma unroll
    for (int k = 0; k < V; ++k) yc[k] = inside ? cin[(int64_t)k * Nx + i] : 0.0;
  }

  // ---- diffuse-reflection closure (windows whose halo reaches a wall) ----
  const bool needL = win.i0 - kHalo < 0;
  const bool needR = win.i0 - kHalo + 63 >= Nx;
  const double *gwL = A.gw + C.gw_off, *gwR = gwL + V;
  double nL = 0.0, nR = 0.0;
  if (needL) nL = wall_density<V, ADV>(tb, fin, Nx, true, C.inv_DL);
  if (needR) nR = wall_density<V, ADV>(tb, fin, Nx, false, C.inv_DR);
  if (i < 0) {  // left ghosts: emergent p > 0 from the wall, incoming extrapolated
    const int gi = -i;  // 1, 2, 3
    const double c0 = gi == 1 ? 3.0 : (gi == 2 ? 6.0 : 10.0);
    const double c1 = gi == 1 ? -3.0 : (gi == 2 ? -8.0 : -15.0);
    const double c2 = gi == 1 ? 1.0 : (gi == 2 ? 3.0 : 6.0);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      if (k < H) {
        yf[k] = nL * gwL[k];
        if constexpr (NC > 1) yc[k] = C.half_Dt * C.TL * yf[k];
      } else {
        const double *r = fin + (int64_t)k * Nx;
        yf[k] = c0 * r[0] + c1 * r[1] + c2 * r[2];
        if constexpr (NC > 1) {
          const double *rc = cin + (int64_t)k * Nx;
          yc[k] = c0 * rc[0] + c1 * rc[1] + c2 * rc[2];
        }
      }
    }
  } else if (i >= Nx && i <= Nx + 2) {  // right ghosts
    const int gi = i - Nx + 1;
    const double c0 = gi == 1 ? 3.0 : (gi == 2 ? 6.0 : 10.0);
    const double c1 = gi == 1 ? -3.0 : (gi == 2 ? -8.0 : -15.0);
    const double c2 = gi == 1 ? 1.0 : (gi == 2 ? 3.0 : 6.0);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      if (k >= H) {
        yf[k] = nR * gwR[k];
        if constexpr (NC > 1) yc[k] = C.half_Dt * C.TR * yf[k];
      } else {
        const double *r = fin + (int64_t)k * Nx;
        yf[k] = c0 * r[Nx - 1] + c1 * r[Nx - 2] + c2 * r[Nx - 3];
        if constexpr (NC > 1) {
          const double *rc = cin + (int64_t)k * Nx;
          yc[k] = c0 * rc[Nx - 1] + c1 * rc[Nx - 2] + c2 * rc[Nx - 3];
        }
      }
    }
  }
  if (A.nwall && A.stage == 2) {
    if (win.i0 == 0 && lane == 0) A.nwall[2 * win.ch] = nL;
    if (win.i0 <= Nx - 1 && Nx - 1 < win.i0 + kWin && lane == 0) A.nwall[2 * win.ch + 1] = nR;
  }

  // ---- moments (Eq. fmoms; chi adds the transverse energy) ----
  double n = 0.0, mom = 0.0;
#pragma unroll
  for (int k = 0; k < V; ++k) { n += yf[k]; mom += tb->p[k] * yf[k]; }
  if (!inside) n = 1.0, mom = 0.0;
  const double u = mom / n;
  double e2 = 0.0, ech = 0.0;
#pragma unroll
  for (int k = 0; k < V; ++k) {
    const double dp = tb->p[k] - u;
    e2 += dp * dp * yf[k];
    if constexpr (NC > 1) ech += yc[k];
  }
  double T = (e2 + 2.0 * ech) * C.inv_1pDt / n;
  if (!inside) T = 1.0;
  const double inv_tau = n * C.inv_Kn;

  // ---- truncated equilibrium g_k(u, T) ----
  double geq[V];
  if (C.inv_Kn != 0.0) {
    if constexpr (QUAD == 0) {
      // exact change of variables (see the host builder for the derivation)
      double Gp[Q], Gm[Q];
#pragma unroll
      for (int l = 0; l < Q; ++l) Gp[l] = Gm[l] = 0.0;
      const double sT = sqrt(T);
      const double ub = u * tb->inv_p0, s = sT * tb->inv_p0, y0 = -u / sT;
      auto accum = [&](double x, double wt, double *G) {
        double hm = 0.0, h = tb->isb[0];
        G[0] += wt * h;
#pragma unroll
        for (int l = 0; l + 1 < Q; ++l) {
          const double hn = ((x - tb->a[l]) * h - tb->sb[l] * hm) * tb->isb[l + 1];
          hm = h; h = hn;
          G[l + 1] += wt * h;
        }
      };
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        accum(ub + s * tb->z[j], tb->w[j], Gp);
        accum(-ub + s * tb->z[j], tb->w[j], Gm);
      }
      if (y0 != 0.0) {
#pragma unroll
        for (int j = 0; j < kNc; ++j) {
          const double yt = y0 * tb->tau[j];
          const double e = y0 * tb->lamw[j] * exp(-0.5 * yt * yt);
          const double xc = ub * (1.0 - tb->tau[j]);
          accum(xc, -e, Gp);
          accum(-xc, e, Gm);
        }
      }
#pragma unroll
      for (int k = 0; k < H; ++k) {
        double ap = 0.0, am = 0.0;
#pragma unroll
        for (int l = 0; l < Q; ++l) { ap += tb->HW[k * Q + l] * Gp[l]; am += tb->HW[k * Q + l] * Gm[l]; }
        geq[k] = ap; geq[H + k] = am;
      }
    } else {
      double G[Q];
      const double aa = T * tb->inv_p0 * tb->inv_p0 - 1.0, bb = u * tb->inv_p0;
      G[0] = 1.0;
      if (Q > 1) G[1] = bb;
#pragma unroll
      for (int l = 1; l + 1 < Q; ++l) G[l + 1] = bb * G[l] + (double)l * aa * G[l - 1];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < Q; ++l) acc += tb->HW[k * Q + l] * G[l];
        geq[k] = acc;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) geq[k] = 0.0;
  }

  // ---- force: (K y)_k ----
  double bf = 0.0, bc = 0.0;
  if constexpr (QUAD == 0) {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      bf += tb->kb[k % H] * yf[k];
      if constexpr (NC > 1) bc += tb->kb[k % H] * yc[k];
    }
  }

  const bool out_lane = lane >= kHalo && lane < kHalo + kWin && inside;
  const double dx_inv = inside ? A.inv_dx[C.cell_off + i] : 0.0;
  const double *bfp = (const double *)A.base_f + C.off;
  double *ofp = (double *)A.out_f + C.off;
  const double *bcp = NC > 1 ? (const double *)A.base_c + C.off : nullptr;
  double *ocp = NC > 1 ? (double *)A.out_c + C.off : nullptr;
  const double gforce = C.g, dt = C.dt;
  const bool lwall_face = (i == -1), rwall_face = (i == Nx - 1);

#pragma unroll
  for (int k = 0; k < V; ++k) {
    const double v = tb->p[k];
#pragma unroll
    for (int fn = 0; fn < NC; ++fn) {
      const double *y = fn == 0 ? yf : yc;
      // force
      double ky = 0.0;
      if constexpr (QUAD == 0) {
        const int kk = k % H, hb = k < H ? 0 : H;
        const double sg = k < H ? 1.0 : -1.0;
#pragma unroll
        for (int j = 0; j < H; ++j) ky += tb->Kin[kk * H + j] * y[hb + j];
        ky = sg * (ky + tb->ka[kk] * (fn == 0 ? bf : bc));
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) ky += tb->Kin[k * V + j] * y[j];
      }
      // advection: face value at i+1/2, neighbours by wave shifts
      const double yc0 = y[k];
      const double ym1 = dpp_shr1(yc0), yp1 = dpp_shl1(yc0);
      double fv;
      if (k < H) {
        const double ym2 = dpp_shr1(ym1), yp2 = dpp_shl1(yp1);
        fv = face_value<ADV>(ym2, ym1, yc0, yp1, yp2);
      } else {
        const double yp2 = dpp_shl1(yp1), yp3 = dpp_shl1(yp2);
        fv = face_value<ADV>(yp3, yp2, yp1, yc0, ym1);
      }
      double F = v * fv;
      // emergent wall-face fluxes are v_k times the wall Maxwellian (Eq. weno_flux_eq)
      if (k < H && lwall_face) F = v * yc0;
      if (k >= H && rwall_face) F = v * yp1;
      const double Fl = dpp_shr1(F);
      double L = -(F - Fl) * dx_inv - gforce * ky;
      if (C.inv_Kn != 0.0) {
        const double eq = fn == 0 ? n * geq[k] : C.half_Dt * T * n * geq[k];
        L -= (yc0 - eq) * inv_tau;
      }
      if (out_lane) {
        const int64_t o = (int64_t)k * Nx + i;
        const double *bp = fn == 0 ? bfp : bcp;
        double *op = fn == 0 ? ofp : ocp;
        const double base = A.a_base != 0.0 ? bp[o] : 0.0;
        op[o] = A.a_base * base + A.b_stage * (yc0 + dt * L);
      }
    }
  }
}

// Maximum over the wave (all lanes active).  After the butterfly every lane
// holds the same value; it is returned through the first lane as a scalar,
// so that what depends on it (the ladder entry, the loop counts of the
// correction) stays in scalar registers and scalar branches.
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Register layout of v_mfma_f64_16x16x4f64 (checked on the GPU):
//   A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
//   D[i][j] in lane j + 16 (i % 4), accumulator register i / 4.
// OUT[i][cell] = sum_k M[i][k] X[k][cell] for the 16 x 16 table M (held as
// four A operands, aM[kc] = M[lane % 16][4 kc + lane / 16]) and the 16
// values X[0..15] each lane (= cell) holds.  The cell-major data are
// transposed into the B layout and back through a padded LDS tile T of
// 64 x 17 doubles owned by this wavefront.
__device__ __forceinline__ void mfma_contract16(const double aM[4], const double X[16], double OUT[16],
                                                double *T, int lane) {
  constexpr int S = 17;
#pragma unroll
  for (int k = 0; k < 16; ++k) T[lane * S + k] = X[k];
  __builtin_amdgcn_wave_barrier();
  dbl4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    acc[cb] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const double b = T[(16 * cb + (lane & 15)) * S + 4 * kc + (lane >> 4)];
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aM[kc], b, acc[cb], 0, 0, 0);
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * cb + (lane & 15)) * S + 4 * r + (lane >> 4)] = acc[cb][r];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int k = 0; k < 16; ++k) OUT[k] = T[lane * S + k];
  __builtin_amdgcn_wave_barrier();
}

// mfma_contract16 without the read-back: OUT[i] of cell `lane` is left in
// T[lane * 17 + i] for the caller.  Each block of 16 cells reads and writes
// only its own 16 rows of T, so the blocks run one after another with one
// accumulator (the caller holds many live values at this point).
__device__ __forceinline__ void mfma_contract16_keep(const double aM[4], const double X[16], double *T,
                                                     int lane) {
  constexpr int S = 17;
#pragma unroll
  for (int k = 0; k < 16; ++k) T[lane * S + k] = X[k];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const double b = T[(16 * cb + (lane & 15)) * S + 4 * kc + (lane >> 4)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aM[kc], b, acc, 0, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * cb + (lane & 15)) * S + 4 * r + (lane >> 4)] = acc[r];
    __builtin_amdgcn_wave_barrier();
  }
}

// Half-range kernel: the two momentum halves of a window run in the two
// wavefronts of a 128-thread block (wave 0: p > 0, wave 1: p < 0).  Each lane
// holds the Q nodes of its half for f and chi; the only coupling between the
// halves -- moment sums, the rank-1 cross term of the force matrix and the
// wall densities -- goes through 6 KB of LDS and one barrier.
// LDS of one window (doubles): the moment partials of the two halves and,
// at Q = 16, the transpose tiles of the matrix-core contractions, which the
// partials share when HHLB_HALF_ALIAS is set (a barrier separates them).
template <int Q>
constexpr int half_lds_doubles() {
  constexpr int tiles = (HHLB_MFMA && Q == 16) ? 2 * 64 * 17 : 0, parts = 2 * 6 * 64;
  return HHLB_HALF_ALIAS ? (tiles > parts ? tiles : parts) : tiles + parts;
}

// One window of the half-range stage, run by a block of two waves (one per
// momentum half); s_lds holds half_lds_doubles<Q>() doubles and s_nw two.
template <int Q, int NFUN, int ADV>
__device__ __forceinline__ void stage_half_window(
    const StageArgs &A, const DevTables *__restrict__ tb, const DevChannel *__restrict__ chans,
    const DevWindow win, const double *__restrict__ inv_dx, const double *__restrict__ gw,
    const double *__restrict__ in_f, const double *__restrict__ in_c, double *s_lds, double *s_nw) {
  constexpr int H = Q;
  constexpr int NC = NFUN;
  constexpr bool kMfma = HHLB_MFMA && (H == 16);   // matrix cores for the 16 x 16 contractions
  double (*s_part)[6][64] = reinterpret_cast<double (*)[6][64]>(s_lds);
  double *s_T = HHLB_HALF_ALIAS ? s_lds : s_lds + 2 * 6 * 64;
  const int hw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const DevChannel C = chans[win.ch];
  const int Nx = C.Nx;
  const int i = win.i0 - kHalo + lane;
  const bool inside = i >= 0 && i < Nx;
  const int kb0 = hw * H;
  const double sg = hw ? -1.0 : 1.0;
  const double *fin = in_f + C.off + (int64_t)kb0 * Nx;
  const double *cin = NC > 1 ? in_c + C.off + (int64_t)kb0 * Nx : nullptr;

  double yf[H], yc[NC > 1 ? H : 1];
#pragma unroll
  for (int j = 0; j < H; ++j) yf[j] = inside ? fin[(int64_t)j * Nx + i] : 0.0;
  if constexpr (NC > 1) {
#pragma unroll
    for (int j = 0; j < H; ++j) yc[j] = inside ? cin[(int64_t)j * Nx + i] : 0.0;
  }

  // ---- closure, part 1: ghosts of the nodes flowing into a wall are
  // extrapolated quadratically from the three nearest cells (Sec. IV.C.3) and
  // their wall-face fluxes give the wall density (Eq. nplus_def).
  const bool needL = win.i0 < kHalo;
  const bool needR = win.i0 - kHalo + 63 >= Nx;
  double nw_mine = 0.0;
  if ((hw == 1 && needL) || (hw == 0 && needR)) {
    const bool left = hw == 1;
    const int l0 = left ? kHalo : Nx - 1 - (win.i0 - kHalo);   // lane of the wall cell
    const int dl = left ? 1 : -1;
    const int gi = left ? -i : i - Nx + 1;                      // ghost order 1..3 (else <= 0)
    const double c0 = gi == 1 ? 3.0 : (gi == 2 ? 6.0 : 10.0);
    const double c1 = gi == 1 ? -3.0 : (gi == 2 ? -8.0 : -15.0);
    const double c2 = gi == 1 ? 1.0 : (gi == 2 ? 3.0 : 6.0);
    const bool is_ghost = gi >= 1 && gi <= 3;
    // lane j gathers node j's three wall-adjacent values; ghost lanes
    // extrapolate every node of this half
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double y0 = readlane_d(yf[j], l0), y1 = readlane_d(yf[j], l0 + dl),
                   y2 = readlane_d(yf[j], l0 + 2 * dl);
      if (lane == j) { a0 = y0; a1 = y1; a2 = y2; }
      if (is_ghost) yf[j] = c0 * y0 + c1 * y1 + c2 * y2;
      if constexpr (NC > 1) {
        const double x0 = readlane_d(yc[j], l0), x1 = readlane_d(yc[j], l0 + dl),
                     x2 = readlane_d(yc[j], l0 + 2 * dl);
        if (is_ghost) yc[j] = c0 * x0 + c1 * x1 + c2 * x2;
      }
    }
    // incoming wall-face flux of node `lane`, all nodes in parallel
    const double g1 = 3.0 * a0 - 3.0 * a1 + a2, g2 = 6.0 * a0 - 8.0 * a1 + 3.0 * a2;
    const double fv = face_value<ADV>(a2, a1, a0, g1, g2);
    const double acc = wave_sum(lane < H ? tb->p[kb0 + (lane < H ? lane : 0)] * fv : 0.0);
    nw_mine = -acc * (left ? C.inv_DL : C.inv_DR);
  }

  // ---- partial moments of this half and the rank-1 force projections ----
  double pn = 0.0, pm = 0.0, ps = 0.0, pc = 0.0, pbf = 0.0, pbc = 0.0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double v = tb->p[kb0 + j];
    pn += yf[j];
    pm += v * yf[j];
    ps += v * v * yf[j];
    pbf += tb->kb[j] * yf[j];
    if constexpr (NC > 1) { pc += yc[j]; pbc += tb->kb[j] * yc[j]; }
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
  const double bf = s_part[0][4][lane] + s_part[1][4][lane];
  const double bc = s_part[0][5][lane] + s_part[1][5][lane];
  const double nL = s_nw[1], nR = s_nw[0];
#if HHLB_HALF_ALIAS
  __syncthreads();   // the tiles below overwrite the partials
#endif

  // ---- closure, part 2: emergent ghosts n_w g^w_k in all three cells ----
  if (hw == 0 && i < 0) {
    const double *gwL = gw + C.gw_off;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      yf[j] = nL * gwL[j];
      if constexpr (NC > 1) yc[j] = C.half_Dt * C.TL * yf[j];
    }
  }
  if (hw == 1 && i >= Nx && i <= Nx + 2) {
    const double *gwR = gw + C.gw_off + 2 * H + H;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      yf[j] = nR * gwR[j];
      if constexpr (NC > 1) yc[j] = C.half_Dt * C.TR * yf[j];
    }
  }
  if (A.nwall && A.stage == 2 && lane == 0) {
    if (hw == 1 && win.i0 == 0) A.nwall[2 * win.ch] = nL;
    if (hw == 0 && win.i0 <= Nx - 1 && Nx - 1 < win.i0 + kWin) A.nwall[2 * win.ch + 1] = nR;
  }

  // ---- moments (Eq. fmoms) ----
  if (!inside) n = 1.0, mom = 0.0;
  const double u = mom / n;
  double T = (s2 - u * mom + 2.0 * ech) * C.inv_1pDt / n;
  if (!inside) T = 1.0;
  const double inv_tau = n * C.inv_Kn;

  // ---- equilibrium coefficients of this half (monic recurrence; the
  // normalisation is folded into HWs) ----
  double G[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) G[l] = 0.0;
  const bool collide = C.inv_Kn != 0.0;
  bool wide_wave = false;   // the correction rule lay beyond the calibrated ladder
  if (collide) {
    const double sT = sqrt(T);
    const double ub = sg * u * tb->inv_p0, s = sT * tb->inv_p0, y0 = -u / sT;
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
    // correction over [y0, 0]: the smallest ladder entry that covers the wave
    const double ymax = wave_max(inside ? fabs(y0) : 0.0);
    if (ymax > 0.0) {
      const int li = ladder_entry(tb, ymax);
      const int nc = tb->lad_n[li], o = tb->lad_off[li];
      wide_wave = nc > tb->lad_n[kLadder - 1];
      for (int j = 0; j < nc; ++j) {
        const double t = tb->ltau[o + j];
        const double yt = y0 * t;
        const double e = y0 * tb->llamw[o + j] * exp(-0.5 * yt * yt);
        accum(ub * (1.0 - t), -sg * e);
      }
    }
  }

  const bool out_lane = lane >= kHalo && lane < kHalo + kWin && inside;
  const int ic = inside ? i : 0;   // clamped cell index: loads stay in bounds
  const double dx_inv = inv_dx[C.cell_off + ic];
  const int64_t obase = C.off + (int64_t)kb0 * Nx;
  const double gforce = C.g, dt = C.dt;

  // pass 1: local source -F (K y)_k - (y_k - y^eq_k)/tau for f and chi,
  // with the equilibrium population g_k of this half
  double srcf[H], srcc[(NC > 1 && !kMfma) ? H : 1];
  const double eqc = C.half_Dt * T;
  if constexpr (kMfma) {
    // (K_in y) and (HWs G) as 16 x 16 x 64-cell products on the matrix cores
    double *Tw = s_T + hw * 64 * 17;
    double aK[4], aH[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      aK[kc] = tb->Kin[(lane & 15) * H + 4 * kc + (lane >> 4)];
      aH[kc] = tb->HWs[(lane & 15) * Q + 4 * kc + (lane >> 4)];
    }
    double geq[H], ky[H];
    mfma_contract16(aH, G, geq, Tw, lane);
    mfma_contract16(aK, yf, ky, Tw, lane);
#pragma unroll
    for (int j = 0; j < H; ++j) {
      srcf[j] = -gforce * sg * (ky[j] + tb->ka[j] * bf) - (yf[j] - n * geq[j]) * inv_tau;
      // keep the finished source in a register: without this fence the
      // compiler sinks its terms into pass 2 and holds three values per node
      asm volatile("" : "+v"(srcf[j]));
    }
    if constexpr (NC > 1) {
      // the chi source stays in the lane's row of the tile until pass 2
      // reads it, which keeps 16 values out of the register file
      mfma_contract16_keep(aK, yc, Tw, lane);
#pragma unroll
      for (int j = 0; j < H; ++j)
        Tw[lane * 17 + j] = -gforce * sg * (Tw[lane * 17 + j] + tb->ka[j] * bc) - (yc[j] - eqc * n * geq[j]) * inv_tau;
    }
  } else {
    double geq[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) acc += tb->HWs[j * Q + l] * G[l];
      geq[j] = acc;
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
      double kf = 0.0, kc = 0.0;
#pragma unroll
      for (int jj = 0; jj < H; ++jj) {
        const double kv = tb->Kin[j * H + jj];
        kf += kv * yf[jj];
        if constexpr (NC > 1) kc += kv * yc[jj];
      }
      kf = sg * (kf + tb->ka[j] * bf);
      const double feq = n * geq[j];
      srcf[j] = -gforce * kf - (yf[j] - feq) * inv_tau;   // inv_tau = 0 when collisionless
      if constexpr (NC > 1) {
        kc = sg * (kc + tb->ka[j] * bc);
        srcc[j] = -gforce * kc - (yc[j] - eqc * feq) * inv_tau;
      }
    }
  }
  // pass 2: advection (WENO-5 / upwind-3 face fluxes, Sec. IV.C.2) and the
  // RK-3 combination.  The y^n values the combination needs are loaded
  // HHLB_PREFETCH node-functions ahead of their use, so that the memory
  // latency overlaps the WENO arithmetic of the nodes in between.  Lane i
  // forms the face value at i+1/2 (hw = 0) or i-1/2 (hw = 1); the other face
  // of its cell comes from the neighbouring lane.
  constexpr int NSEC = H * NC;
  constexpr int PD = HHLB_PREFETCH < NSEC ? HHLB_PREFETCH : NSEC;
  const bool need_base = A.a_base != 0.0;
  auto base_ptr = [&](int sec) {
    return (const double *)((sec % NC) == 0 ? A.base_f : A.base_c) + obase + (int64_t)(sec / NC) * Nx + ic;
  };
  const FaceCoef fcoef = face_coef(hw);
  const bool face_used = inside && lane >= kHalo - 1 + hw && lane < kHalo + kWin + hw;
  const bool wall_face_l = hw == 0 ? (i == -1) : (i == Nx);
  const double sdx = hw == 0 ? -dx_inv : dx_inv;   // L = sdx (F - F_other) + source
  double bq[PD];
#pragma unroll
  for (int d = 0; d < PD; ++d) bq[d] = need_base ? *base_ptr(d) : 0.0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double v = tb->p[kb0 + j];
#pragma unroll
    for (int fn = 0; fn < NC; ++fn) {
      const int sec = j * NC + fn;
      const double base = bq[sec % PD];
      if (sec + PD < NSEC) bq[sec % PD] = need_base ? *base_ptr(sec + PD) : 0.0;
      const double y0v = fn == 0 ? yf[j] : yc[j];
      double src;
      if constexpr (kMfma && NC > 1) src = fn == 0 ? srcf[j] : s_T[hw * 64 * 17 + lane * 17 + j];
      else src = fn == 0 ? srcf[j] : srcc[j];
      double fv = face_value_lanes<ADV>(y0v, fcoef, face_used);
      if (wall_face_l) fv = y0v;
      const double F = v * fv;
      const double Fo = hw == 0 ? dpp_shr1(F) : dpp_shl1(F);
      const double L = fma(sdx, F - Fo, src);
      const int64_t o = obase + (int64_t)j * Nx + ic;
      double *op = (double *)(fn == 0 ? A.out_f : A.out_c);
      const double yn = A.a_base * base + A.b_stage * (y0v + dt * L);
      if (out_lane) op[o] = yn;
      // a scheduling fence after every HHLB_SCHED_GROUP node-functions:
      // interleaving more unrolled WENO evaluations exceeds the register file
      if ((j * NC + fn + 1) % HHLB_SCHED_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
    }
  }
  // waves whose correction lay beyond the calibrated ladder, counted once the
  // registers of the step are free
  if (wide_wave && lane == 0 && A.wide) atomicAdd(A.wide, 1ull);
}

template <int Q, int NFUN, int ADV>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(HHLB_HALF_WAVES))) void stage_kernel_half(
    StageArgs A, const DevTables *__restrict__ tb, const DevChannel *__restrict__ chans,
    const DevWindow *__restrict__ wins, const double *__restrict__ inv_dx,
    const double *__restrict__ gw, const double *__restrict__ in_f,
    const double *__restrict__ in_c) {
  __shared__ double s_lds[half_lds_doubles<Q>()];
  __shared__ double s_nw[2];
  const int w = A.xcd_map ? xcd_window(blockIdx.x, A.nwin) : (int)blockIdx.x;
  stage_half_window<Q, NFUN, ADV>(A, tb, chans, wins[w], inv_dx, gw, in_f, in_c, s_lds, s_nw);
}

// One launch per stage for the windows of several half-range model classes
// that share the functions and the scheme (FP64).  Record b names the window
// and its class; the class's order Q, the same for the whole block, selects
// the per-order window code (orders up to QTOP with a kernel of their own).
// Persistent form: with fewer blocks than windows each block takes windows
// b, b + gridDim.x, .. in turn.
struct DevClassWindow {
  int32_t ch, i0;   // as DevWindow
  int32_t cls, Q;   // model class (index of its tables) and its order
};

template <int QTOP, int NFUN, int ADV, bool PERSIST>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(QTOP <= 8 ? 4 : HHLB_HALF_WAVES))) void stage_kernel_classes(
    StageArgs A, const DevTables *__restrict__ tbs, const DevChannel *__restrict__ chans,
    const DevClassWindow *__restrict__ wins, const double *__restrict__ inv_dx,
    const double *__restrict__ gw, const double *__restrict__ in_f,
    const double *__restrict__ in_c) {
  __shared__ double s_lds[half_lds_doubles<QTOP>()];
  __shared__ double s_nw[2];
  for (int b = blockIdx.x; b < A.nwin; b += gridDim.x) {
    if (PERSIST && b != (int)blockIdx.x) __syncthreads();   // the last window's LDS reads are done
    const int w = A.xcd_map ? xcd_window(b, A.nwin) : b;
    const DevClassWindow cw = wins[w];
    const DevWindow win{cw.ch, cw.i0};
    const DevTables *tb = tbs + __builtin_amdgcn_readfirstlane(cw.cls);
    switch (__builtin_amdgcn_readfirstlane(cw.Q)) {
#define HHLB_CLASS_CASE(q)                                                                   \
  case q:                                                                                    \
    if constexpr (q <= QTOP)                                                                 \
      stage_half_window<q, NFUN, ADV>(A, tb, chans, win, inv_dx, gw, in_f, in_c, s_lds, s_nw); \
    break;
      HHLB_CLASS_CASE(1) HHLB_CLASS_CASE(2) HHLB_CLASS_CASE(3) HHLB_CLASS_CASE(4)
      HHLB_CLASS_CASE(6) HHLB_CLASS_CASE(8) HHLB_CLASS_CASE(12) HHLB_CLASS_CASE(16)
#undef HHLB_CLASS_CASE
      default: break;
    }
    if constexpr (!PERSIST) break;   // one window per block
  }
}

// The contraction of mfma_contract16 through an unpadded 64 x 16 tile whose
// columns are XOR-swizzled by the row (column c of row r at c ^ (r & 15)):
// the row writes, the B-operand reads and the D writes then spread over the
// LDS banks as with the padded tile, in 8 KB instead of 8.5 KB per wave.
__device__ __forceinline__ void mfma_contract16_sw(const double aM[4], const double X[16], double OUT[16],
                                                   double *T, int lane) {
  const int sw = lane & 15;
#pragma unroll
  for (int k = 0; k < 16; ++k) T[lane * 16 + (k ^ sw)] = X[k];
  __builtin_amdgcn_wave_barrier();
  dbl4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    acc[cb] = dbl4{0.0, 0.0, 0.0, 0.0};
    const double *row = T + (16 * cb + sw) * 16;   // row r = 16 cb + (lane & 15): r & 15 = sw
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const double b = row[(4 * kc + (lane >> 4)) ^ sw];
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aM[kc], b, acc[cb], 0, 0, 0);
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * cb + sw) * 16 + ((4 * r + (lane >> 4)) ^ sw)] = acc[cb][r];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int k = 0; k < 16; ++k) OUT[k] = T[lane * 16 + (k ^ sw)];
  __builtin_amdgcn_wave_barrier();
}

// Half-range kernel with four waves per window: wave w handles momentum
// half (w & 1) of function (w >> 1), f or chi, so each lane keeps Q nodes of
// one function.  Compared with the two-wave kernel this halves the state
// held per wave (no register spill at Q = 16, four waves per SIMD) at the
// price of computing the equilibrium coefficients of a half in both of its
// waves.  Coupling through LDS and one barrier as in the two-wave kernel.
template <int Q, int ADV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HHLB_QUARTER_WAVES))) void stage_kernel_quarter(
    StageArgs A, const DevTables *__restrict__ tb, const DevChannel *__restrict__ chans,
    const DevWindow *__restrict__ wins, const double *__restrict__ inv_dx,
    const double *__restrict__ gw, const double *__restrict__ in_f,
    const double *__restrict__ in_c) {
  constexpr int H = Q;
  constexpr bool kMfma = HHLB_MFMA && (H == 16);
  __shared__ double s_part[2][6][64];
  __shared__ double s_nw[2];
  __shared__ double s_T[kMfma ? 4 * 64 * 16 : 1];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int hw = wv & 1, fn = wv >> 1;
  const int lane = threadIdx.x & 63;
  const int w = A.xcd_map ? xcd_window(blockIdx.x, A.nwin) : (int)blockIdx.x;
  const DevWindow win = wins[w];
  const DevChannel C = chans[win.ch];
  const int Nx = C.Nx;
  const int i = win.i0 - kHalo + lane;
  const bool inside = i >= 0 && i < Nx;
  const int kb0 = hw * H;
  const double sg = hw ? -1.0 : 1.0;
  const double *yin = (fn == 0 ? in_f : in_c) + C.off + (int64_t)kb0 * Nx;

  double y[H];
#pragma unroll
  for (int j = 0; j < H; ++j) y[j] = inside ? yin[(int64_t)j * Nx + i] : 0.0;

  // ---- closure, part 1: incoming ghosts of this wave's function; the f
  // waves also balance the wall flux (Eq. nplus_def) ----
  const bool needL = win.i0 < kHalo;
  const bool needR = win.i0 - kHalo + 63 >= Nx;
  double nw_mine = 0.0;
  if ((hw == 1 && needL) || (hw == 0 && needR)) {
    const bool left = hw == 1;
    const int l0 = left ? kHalo : Nx - 1 - (win.i0 - kHalo);
    const int dl = left ? 1 : -1;
    const int gi = left ? -i : i - Nx + 1;
    const double c0 = gi == 1 ? 3.0 : (gi == 2 ? 6.0 : 10.0);
    const double c1 = gi == 1 ? -3.0 : (gi == 2 ? -8.0 : -15.0);
    const double c2 = gi == 1 ? 1.0 : (gi == 2 ? 3.0 : 6.0);
    const bool is_ghost = gi >= 1 && gi <= 3;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double y0 = readlane_d(y[j], l0), y1 = readlane_d(y[j], l0 + dl),
                   y2 = readlane_d(y[j], l0 + 2 * dl);
      if (lane == j) { a0 = y0; a1 = y1; a2 = y2; }
      if (is_ghost) y[j] = c0 * y0 + c1 * y1 + c2 * y2;
    }
    if (fn == 0) {
      const double g1 = 3.0 * a0 - 3.0 * a1 + a2, g2 = 6.0 * a0 - 8.0 * a1 + 3.0 * a2;
      const double fv = face_value<ADV>(a2, a1, a0, g1, g2);
      const double acc = wave_sum(lane < H ? tb->p[kb0 + (lane < H ? lane : 0)] * fv : 0.0);
      nw_mine = -acc * (left ? C.inv_DL : C.inv_DR);
    }
  }

  // ---- partial moments: f waves n, n u, sum p^2 f and kb.f; chi waves
  // sum chi and kb.chi ----
  if (fn == 0) {
    double pn = 0.0, pm = 0.0, ps = 0.0, pb = 0.0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double v = tb->p[kb0 + j];
      pn += y[j];
      pm += v * y[j];
      ps += v * v * y[j];
      pb += tb->kb[j] * y[j];
    }
    s_part[hw][0][lane] = pn;
    s_part[hw][1][lane] = pm;
    s_part[hw][2][lane] = ps;
    s_part[hw][4][lane] = pb;
    if (lane == 0) s_nw[hw] = nw_mine;
  } else {
    double pc = 0.0, pb = 0.0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      pc += y[j];
      pb += tb->kb[j] * y[j];
    }
    s_part[hw][3][lane] = pc;
    s_part[hw][5][lane] = pb;
  }
  __syncthreads();
  double n = s_part[0][0][lane] + s_part[1][0][lane];
  double mom = s_part[0][1][lane] + s_part[1][1][lane];
  const double s2 = s_part[0][2][lane] + s_part[1][2][lane];
  const double ech = s_part[0][3][lane] + s_part[1][3][lane];
  const double bproj = s_part[0][4 + fn][lane] + s_part[1][4 + fn][lane];
  const double nL = s_nw[1], nR = s_nw[0];

  // ---- closure, part 2: emergent ghosts ----
  const double fscale_L = fn == 0 ? 1.0 : C.half_Dt * C.TL;
  const double fscale_R = fn == 0 ? 1.0 : C.half_Dt * C.TR;
  if (hw == 0 && i < 0) {
    const double *gwL = gw + C.gw_off;
#pragma unroll
    for (int j = 0; j < H; ++j) y[j] = fscale_L * nL * gwL[j];
  }
  if (hw == 1 && i >= Nx && i <= Nx + 2) {
    const double *gwR = gw + C.gw_off + 2 * H + H;
#pragma unroll
    for (int j = 0; j < H; ++j) y[j] = fscale_R * nR * gwR[j];
  }
  if (fn == 0 && A.nwall && A.stage == 2 && lane == 0) {
    if (hw == 1 && win.i0 == 0) A.nwall[2 * win.ch] = nL;
    if (hw == 0 && win.i0 <= Nx - 1 && Nx - 1 < win.i0 + kWin) A.nwall[2 * win.ch + 1] = nR;
  }

  // ---- moments (Eq. fmoms) ----
  if (!inside) n = 1.0, mom = 0.0;
  const double u = mom / n;
  double T = (s2 - u * mom + 2.0 * ech) * C.inv_1pDt / n;
  if (!inside) T = 1.0;
  const double inv_tau = n * C.inv_Kn;

  // ---- equilibrium coefficients of this half (as in the two-wave kernel) ----
  double G[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) G[l] = 0.0;
  bool wide_wave = false;   // the correction rule lay beyond the calibrated ladder
  if (C.inv_Kn != 0.0) {
    const double sT = sqrt(T);
    const double ub = sg * u * tb->inv_p0, s = sT * tb->inv_p0, y0 = -u / sT;
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
      wide_wave = nc > tb->lad_n[kLadder - 1];
      for (int j = 0; j < nc; ++j) {
        const double t = tb->ltau[o + j];
        const double yt = y0 * t;
        const double e = y0 * tb->llamw[o + j] * exp(-0.5 * yt * yt);
        accum(ub * (1.0 - t), -sg * e);
      }
    }
  }

  const bool out_lane = lane >= kHalo && lane < kHalo + kWin && inside;
  const int ic = inside ? i : 0;
  const double dx_inv = inv_dx[C.cell_off + ic];
  const int64_t obase = C.off + (int64_t)kb0 * Nx;
  const double gforce = C.g, dt = C.dt;
  const bool wall_face = hw == 0 ? (i == -1) : (i == Nx - 1);
  const double eqc = fn == 0 ? 1.0 : C.half_Dt * T;

  // pass 1: local source -F (K y)_k - (y_k - y^eq_k)/tau
  double src[H];
  if constexpr (kMfma) {
    double *Tw = s_T + wv * 64 * 16;
    double aK[4], aH[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      aK[kc] = tb->Kin[(lane & 15) * H + 4 * kc + (lane >> 4)];
      aH[kc] = tb->HWs[(lane & 15) * Q + 4 * kc + (lane >> 4)];
    }
    double geq[H], ky[H];
    mfma_contract16_sw(aH, G, geq, Tw, lane);
    mfma_contract16_sw(aK, y, ky, Tw, lane);
#pragma unroll
    for (int j = 0; j < H; ++j)
      src[j] = -gforce * sg * (ky[j] + tb->ka[j] * bproj) - (y[j] - eqc * n * geq[j]) * inv_tau;
  } else {
#pragma unroll
    for (int j = 0; j < H; ++j) {
      double acc = 0.0, kf = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) acc += tb->HWs[j * Q + l] * G[l];
#pragma unroll
      for (int jj = 0; jj < H; ++jj) kf += tb->Kin[j * H + jj] * y[jj];
      src[j] = -gforce * sg * (kf + tb->ka[j] * bproj) - (y[j] - eqc * n * acc) * inv_tau;
    }
  }

  // pass 2: advection and the RK-3 combination, y^n prefetched
  constexpr int PD = HHLB_PREFETCH < H ? HHLB_PREFETCH : H;
  const bool need_base = A.a_base != 0.0;
  const double *bptr = (const double *)(fn == 0 ? A.base_f : A.base_c) + obase + ic;
  double *optr = (double *)(fn == 0 ? A.out_f : A.out_c) + obase + ic;
  double bq[PD];
#pragma unroll
  for (int d = 0; d < PD; ++d) bq[d] = need_base ? bptr[(int64_t)d * Nx] : 0.0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double v = tb->p[kb0 + j];
    const double base = bq[j % PD];
    if (j + PD < H) bq[j % PD] = need_base ? bptr[(int64_t)(j + PD) * Nx] : 0.0;
    const double y0v = y[j];
    double F;
    if (hw == 0) {
      const double ym1 = dpp_shr1(y0v), ym2 = dpp_shr1(ym1);
      const double yp1 = dpp_shl1(y0v), yp2 = dpp_shl1(yp1);
      F = v * face_value<ADV>(ym2, ym1, y0v, yp1, yp2);
      if (wall_face) F = v * y0v;
    } else {
      const double ym1 = dpp_shr1(y0v);
      const double yp1 = dpp_shl1(y0v), yp2 = dpp_shl1(yp1), yp3 = dpp_shl1(yp2);
      F = v * face_value<ADV>(yp3, yp2, yp1, y0v, ym1);
      if (wall_face) F = v * yp1;
    }
    const double Fl = dpp_shr1(F);
    const double L = -(F - Fl) * dx_inv + src[j];
    const double yn = A.a_base * base + A.b_stage * (y0v + dt * L);
    if (out_lane) optr[(int64_t)j * Nx] = yn;
    if ((j + 1) % HHLB_SCHED_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
  }
  // waves whose correction lay beyond the calibrated ladder, counted once the
  // registers of the step are free
  if (wide_wave && lane == 0 && A.wide) atomicAdd(A.wide, 1ull);
}

}  // namespace hhlb
