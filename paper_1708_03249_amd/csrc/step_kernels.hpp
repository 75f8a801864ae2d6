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
constexpr int kNc = 8;         // Gauss-Legendre points of the equilibrium correction
constexpr int kWin = 58;       // output cells per wavefront
constexpr int kHalo = 3;

// Per model class (quadrature, Q, N, p0): uploaded once.
struct DevTables {
  double p[2 * kQmaxDev];                 // p_k / m
  double z[kQmaxDev], w[kQmaxDev];        // positive nodes (units of p0), weights
  double a[kQmaxDev + 2];                 // recurrence: sqrt(b_{l+1}) h_{l+1} = (z-a_l) h_l - sqrt(b_l) h_{l-1}
  double sb[kQmaxDev + 3];                // sqrt(b_l)
  double isb[kQmaxDev + 3];               // 1/sqrt(b_l)
  double Kin[kQmaxDev * kQmaxDev];        // half: + half within block (H x H); full: dense V x V
  double ka[kQmaxDev], kb[kQmaxDev];      // half: rank-1 cross term
  double HW[2 * kQmaxDev * kQmaxDev];     // half: H x Q; full: V x Q (zero beyond N)
  double tau[kNc], lamw[kNc];             // GL nodes in (0,1), weights * 1/sqrt(2 pi)
  double inv_p0;
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
  double inv_DL;      // 1 / sum_{p_k>0} (p_k/m) gwL_k
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
  const double *inv_dx;      // per cell
  const double *gw;          // wall equilibria
  const double *in_f, *in_c; // stage state
  const double *base_f, *base_c;  // y^n (pointwise)
  double *out_f, *out_c;
  double a_base, b_stage;    // out = a_base * y^n + b_stage * (y_s + dt L[y_s])
  double *nwall;             // 2 per channel (may be null)
};

__device__ __forceinline__ double dpp_shr1(double x) {  // lane l <- lane l-1
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_shl1(double x) {  // lane l <- lane l+1
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
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
  double s1 = k13 * t1 * t1 + 0.25 * t2 * t2;
  t1 = b - 2.0 * c + d; t2 = b - d;
  double s2 = k13 * t1 * t1 + 0.25 * t2 * t2;
  t1 = c - 2.0 * d + e; t2 = 3.0 * c - 4.0 * d + e;
  double s3 = k13 * t1 * t1 + 0.25 * t2 * t2;
  double F1 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
  double F2 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
  double F3 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
  double smax = fmax(s1, fmax(s2, s3));
  double q1 = 0.1, q2 = 0.6, q3 = 0.3;
  if (smax > 0.0) {
    int ex = 0;
    (void)frexp(smax, &ex);
    double r1 = ldexp(s1, -ex), r2 = ldexp(s2, -ex), r3 = ldexp(s3, -ex);
    r1 *= r1; r2 *= r2; r3 *= r3;
    double p1 = 0.1 * r2 * r3, p2 = 0.6 * r1 * r3, p3 = 0.3 * r1 * r2;
    double den = p1 + p2 + p3;
    if (den > 1e-250) {
      double inv = 1.0 / den;
      q1 = p1 * inv; q2 = p2 * inv; q3 = p3 * inv;
    } else {
      // limit: ideal weights restricted to the (relatively) vanishing sigmas
      double tiny = 1e-125;
      double z1 = r1 < tiny ? 0.1 : 0.0, z2 = r2 < tiny ? 0.6 : 0.0, z3 = r3 < tiny ? 0.3 : 0.0;
      double zs = z1 + z2 + z3;
      q1 = z1 / zs; q2 = z2 / zs; q3 = z3 / zs;
    }
  }
  return q1 * F1 + q2 * F2 + q3 * F3;
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
  const int w = xcd_window(blockIdx.x, A.nwin);
  const DevWindow win = A.wins[w];
  const DevChannel C = A.chans[win.ch];
  const DevTables *__restrict__ tb = A.tb;
  const int lane = threadIdx.x;
  const int Nx = C.Nx;
  const int i = win.i0 - kHalo + lane;
  const bool inside = i >= 0 && i < Nx;
  const double *fin = A.in_f + C.off;
  const double *cin = NC > 1 ? A.in_c + C.off : nullptr;

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
  const double *bfp = A.base_f + C.off;
  double *ofp = A.out_f + C.off;
  const double *bcp = NC > 1 ? A.base_c + C.off : nullptr;
  double *ocp = NC > 1 ? A.out_c + C.off : nullptr;
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

}  // namespace hhlb
