// gfx950 kernel for one whole TVD RK-3 step (the three stages of Eq. rk3)
// of the half-range model per launch, FP64: step fusion with a 9-cell halo.
//
// The per-stage kernels read the stage state and y^n and write the next
// stage: 8 array passes per function and step.  Here a window keeps y^n and
// the stage state of its 64 cells in registers through the three stages and
// touches memory twice per function: y^n in, y^{n+1} out.
//
// Window geometry.  Lane l holds cell c0 + l.  Each stage's WENO-5 stencil
// reaches 3 cells, so a lane's value stays exact for one stage less per 3
// lanes from an edge of the window that is not a wall: a window whose edges
// are interior keeps 9 halo lanes on each side and writes at most the 46
// cells of lanes 9..54.  At a wall the closure (Sec. IV.C.3) rebuilds the
// ghosts from the current stage every stage, exactly as the per-stage kernel
// does, so nothing is lost there.  The faces the method needs read the first
// two ghosts only, so a wall may sit where just two ghost lanes fit (cell 0
// at lane 2 or 3; cell Nx-1 at lane 61 or below).  The host builds each
// channel's windows (fused_windows) so that every window edge is either such
// a wall or lies inside the channel with its whole halo.
//
// Per stage the arithmetic is that of stage_kernel_half: the same closure,
// moments, equilibrium, force block, BGK, face values and combination
// y_{s+1} = a_s y^n + b_s (y_s + dt L[y_s]), with y^n from registers.  Lanes
// outside the stage's exact range compute values that are never used; they
// are kept out of the wave-wide decisions (the equilibrium ladder and the
// WENO rescaling branch).
#pragma once
#include "step_kernels.hpp"

// occupancy target: three waves per SIMD while y^n and the stage state of
// both functions fit beside the working set (Q <= 4), two above
#ifndef HHLB_FUSED_WAVES_SMALL
#define HHLB_FUSED_WAVES_SMALL 3
#endif
#ifndef HHLB_FUSED_WAVES_LARGE
#define HHLB_FUSED_WAVES_LARGE 2
#endif

namespace hhlb {

constexpr int kFusedHalo = 3 * kHalo;   // halo lanes of an interior window edge
// largest per-half order with a fused-step kernel: y^n and the stage state of
// both functions stay in registers, 4Q doubles per lane
#ifndef HHLB_FUSED_QMAX
#define HHLB_FUSED_QMAX 16
#endif
constexpr int kQmaxFused = HHLB_FUSED_QMAX;

// One window of the fused kernel: channel, first output cell, cell of lane
// 0 and the number of output cells (lanes i0 - c0 .. i0 - c0 + nout - 1).
struct DevFusedWindow {
  int32_t ch, i0, c0, nout;
};

template <int Q, int NFUN, int ADV>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(
    Q <= 4 ? HHLB_FUSED_WAVES_SMALL : HHLB_FUSED_WAVES_LARGE))) void fused_kernel_half(
    StageArgs A, const DevTables *__restrict__ tb, const DevChannel *__restrict__ chans,
    const DevFusedWindow *__restrict__ wins, const double *__restrict__ inv_dx,
    const double *__restrict__ gw, const double *__restrict__ in_f,
    const double *__restrict__ in_c) {
  constexpr int H = Q;
  constexpr int NC = NFUN;
  __shared__ double s_nw[2];
  constexpr bool kMfma = HHLB_MFMA && (H == 16);
  constexpr int kLds = (kMfma ? 2 * 64 * 17 : 1) > 2 * 6 * 64 ? 2 * 64 * 17 : 2 * 6 * 64;
  __shared__ double s_lds[kLds];
  double (*s_part)[6][64] = reinterpret_cast<double (*)[6][64]>(s_lds);
  double *s_T = s_lds;
  const int hw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int w = A.xcd_map ? xcd_window(blockIdx.x, A.nwin) : (int)blockIdx.x;
  const DevFusedWindow win = wins[w];
  const DevChannel C = chans[win.ch];
  const int Nx = C.Nx;
  const int c0 = win.c0;                             // cell of lane 0
  const int hl = win.i0 - c0, nout = win.nout;       // output lanes hl .. hl + nout - 1
  const bool needL = c0 < 0;                         // the walls inside the window
  const bool needR = Nx - 1 - c0 <= 61;
  const int i = c0 + lane;
  const bool inside = i >= 0 && i < Nx;
  const int ic = inside ? i : 0;                     // clamped cell index: loads stay in bounds
  const int kb0 = hw * H;
  const double sg = hw ? -1.0 : 1.0;
  const int64_t obase = C.off + (int64_t)kb0 * Nx;

  double yf[H], yc[NC > 1 ? H : 1], nf[H], nc[NC > 1 ? H : 1];
#pragma unroll
  for (int j = 0; j < H; ++j) nf[j] = inside ? in_f[obase + (int64_t)j * Nx + ic] : 0.0;
  if constexpr (NC > 1) {
#pragma unroll
    for (int j = 0; j < H; ++j) nc[j] = inside ? in_c[obase + (int64_t)j * Nx + ic] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < H; ++j) {
    yf[j] = nf[j];
    if constexpr (NC > 1) yc[j] = nc[j];
  }

  const double dx_inv = inv_dx[C.cell_off + ic];
  const double gforce = C.g, dt = C.dt;
  const FaceCoef fcoef = face_coef(hw);
  const bool wall_face_l = hw == 0 ? (i == -1) : (i == Nx);
  const double sdx = hw == 0 ? -dx_inv : dx_inv;   // L = sdx (F - F_other) + source
  const double *gwL = gw + C.gw_off, *gwR = gw + C.gw_off + 2 * H + H;

#pragma unroll 1
  for (int st = 0; st < 3; ++st) {
    // Eq. (rk3): y_{s+1} = a_s y^n + b_s (y_s + dt L[y_s])
    const double a_s = st == 0 ? 0.0 : (st == 1 ? 0.75 : 1.0 / 3.0);
    const double b_s = st == 0 ? 1.0 : (st == 1 ? 0.25 : 2.0 / 3.0);
    // lanes whose stage result is still exact: 3 fewer per stage at each
    // window edge that is not a wall
    const int lo = needL ? 0 : kHalo * (st + 1);
    const int hi = needR ? 63 : 60 - kHalo * st;
    const bool live = lane >= lo && lane <= hi;
    if (st > 0) __syncthreads();   // the previous stage's tiles are read before the partials overwrite them

    // ---- closure, part 1: incoming ghosts extrapolated from the three
    // nearest cells, and the wall density from their wall-face fluxes ----
    double nw_mine = 0.0;
    if ((hw == 1 && needL) || (hw == 0 && needR)) {
      const bool left = hw == 1;
      const int l0 = left ? -c0 : Nx - 1 - c0;     // lane of the wall cell
      const int dl = left ? 1 : -1;
      const int gi = left ? -i : i - Nx + 1;       // ghost order 1..3 (else <= 0)
      const double e0 = gi == 1 ? 3.0 : (gi == 2 ? 6.0 : 10.0);
      const double e1 = gi == 1 ? -3.0 : (gi == 2 ? -8.0 : -15.0);
      const double e2 = gi == 1 ? 1.0 : (gi == 2 ? 3.0 : 6.0);
      const bool is_ghost = gi >= 1 && gi <= 3;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const double y0 = readlane_d(yf[j], l0), y1 = readlane_d(yf[j], l0 + dl),
                     y2 = readlane_d(yf[j], l0 + 2 * dl);
        if (lane == j) { a0 = y0; a1 = y1; a2 = y2; }
        if (is_ghost) yf[j] = e0 * y0 + e1 * y1 + e2 * y2;
        if constexpr (NC > 1) {
          const double x0 = readlane_d(yc[j], l0), x1 = readlane_d(yc[j], l0 + dl),
                       x2 = readlane_d(yc[j], l0 + 2 * dl);
          if (is_ghost) yc[j] = e0 * x0 + e1 * x1 + e2 * x2;
        }
      }
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
    __syncthreads();   // the tiles below overwrite the partials

    // ---- closure, part 2: emergent ghosts n_w g^w_k in all three cells ----
    if (hw == 0 && i < 0) {
#pragma unroll
      for (int j = 0; j < H; ++j) {
        yf[j] = nL * gwL[j];
        if constexpr (NC > 1) yc[j] = C.half_Dt * C.TL * yf[j];
      }
    }
    if (hw == 1 && i >= Nx && i <= Nx + 2) {
#pragma unroll
      for (int j = 0; j < H; ++j) {
        yf[j] = nR * gwR[j];
        if constexpr (NC > 1) yc[j] = C.half_Dt * C.TR * yf[j];
      }
    }
    if (A.nwall && st == 2 && lane == 0) {
      if (hw == 1 && needL) A.nwall[2 * win.ch] = nL;
      if (hw == 0 && needR) A.nwall[2 * win.ch + 1] = nR;
    }

    // ---- moments (Eq. fmoms) ----
    if (!inside) n = 1.0, mom = 0.0;
    const double u = mom / n;
    double T = (s2 - u * mom + 2.0 * ech) * C.inv_1pDt / n;
    if (!inside) T = 1.0;
    const double inv_tau = n * C.inv_Kn;

    // ---- equilibrium coefficients of this half ----
    double G[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) G[l] = 0.0;
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
      const double ymax = wave_max(inside && live ? fabs(y0) : 0.0);
      if (ymax > 0.0) {
        const int li = ladder_entry(tb, ymax);
        const int ncor = tb->lad_n[li], o = tb->lad_off[li];
        if (ncor > tb->lad_n[kLadder - 1] && lane == 0 && A.wide) atomicAdd(A.wide, 1ull);
        for (int j = 0; j < ncor; ++j) {
          const double t = tb->ltau[o + j];
          const double yt = y0 * t;
          const double e = y0 * tb->llamw[o + j] * exp(-0.5 * yt * yt);
          accum(ub * (1.0 - t), -sg * e);
        }
      }
    }

    // pass 1: local source -F (K y)_k - (y_k - y^eq_k)/tau for f and chi
    double srcf[H], srcc[(NC > 1 && !kMfma) ? H : 1];
    const double eqc = C.half_Dt * T;
    if constexpr (kMfma) {
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
        asm volatile("" : "+v"(srcf[j]));
      }
      if constexpr (NC > 1) {
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
        double kf = 0.0, kcc = 0.0;
#pragma unroll
        for (int jj = 0; jj < H; ++jj) {
          const double kv = tb->Kin[j * H + jj];
          kf += kv * yf[jj];
          if constexpr (NC > 1) kcc += kv * yc[jj];
        }
        kf = sg * (kf + tb->ka[j] * bf);
        const double feq = n * geq[j];
        srcf[j] = -gforce * kf - (yf[j] - feq) * inv_tau;
        if constexpr (NC > 1) {
          kcc = sg * (kcc + tb->ka[j] * bc);
          srcc[j] = -gforce * kcc - (yc[j] - eqc * feq) * inv_tau;
        }
      }
    }

    // pass 2: advection and the RK-3 combination into the registers; the
    // face values of node j read only node j's values, so y[j] is replaced
    // once its flux difference is formed
    // faces the exact lanes need: lane i forms the face at i+1/2 (hw = 0) or
    // i-1/2 (hw = 1), and L of lane i also takes its neighbour's
    const bool face_used = inside && lane >= lo - 1 + hw && lane <= hi + hw;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double v = tb->p[kb0 + j];
#pragma unroll
      for (int fn = 0; fn < NC; ++fn) {
        const double y0v = fn == 0 ? yf[j] : yc[j];
        double src;
        if constexpr (kMfma && NC > 1) src = fn == 0 ? srcf[j] : s_T[hw * 64 * 17 + lane * 17 + j];
        else src = fn == 0 ? srcf[j] : srcc[j];
        double fv = face_value_lanes<ADV>(y0v, fcoef, face_used);
        if (wall_face_l) fv = y0v;
        const double F = v * fv;
        const double Fo = hw == 0 ? dpp_shr1(F) : dpp_shl1(F);
        const double L = fma(sdx, F - Fo, src);
        const double yb = fn == 0 ? nf[j] : nc[j];
        const double yn = a_s * yb + b_s * (y0v + dt * L);
        if (fn == 0) yf[j] = yn;
        else if constexpr (NC > 1) yc[j] = yn;
        if ((j * NC + fn + 1) % HHLB_SCHED_GROUP == 0) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  // ---- y^{n+1} of the window's output cells ----
  const bool out_lane = lane >= hl && lane < hl + nout;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const int64_t o = obase + (int64_t)j * Nx + ic;
    if (out_lane) {
      ((double *)A.out_f)[o] = yf[j];
      if constexpr (NC > 1) ((double *)A.out_c)[o] = yc[j];
    }
  }
}

}  // namespace hhlb
