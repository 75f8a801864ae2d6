// Node-parallel FP64 stage for large velocity sets, equilibrium order
// N <= 20: the half-range model with 17 <= Q <= 256 nodes per half and the
// full-range model with 18 <= Q <= 512 nodes, the paper's HHLB(20;Q) and
// HLB(20;Q) models of the ballistic study (Sec. V.E).  The nodes of a half
// no longer fit a lane's registers, so one stage runs as two kernels:
//   large_cell_kernel: one wave per cell, lanes over nodes and then over
//     quadrature points: the moments (Eq. fmoms), 1/tau, the rank-1 force
//     projections and the equilibrium coefficients of both halves (half
//     range: Sec. IV.B.3 by the change of variables of stage_kernel_half;
//     full range: the closed form of Sec. IV.A.3); per channel, the wall
//     densities (Eq. nplus_def).
//   large_node_kernel: per window and tile of 16 nodes of one half, the
//     force -F (K y)_k contracted on FP64 MFMA tiles (half range: the
//     within-half block of Eq. hh_Kk_hh plus the rank-1 cross term; full
//     range: the dense matrix of Eq. H_Kk), the wall ghosts (Sec. IV.C.3),
//     BGK towards the synthesised equilibrium, WENO-5 / upwind-3 advection
//     (the lane-parallel face values of stage_kernel_half) and the RK-3
//     combination.  The lanes of the node phase hold cells, as in
//     stage_kernel_half.
#pragma once
#include "step_kernels.hpp"

namespace hhlb {

constexpr int kQmaxLarge = 256;   // nodes per half
constexpr int kNmaxLarge = 20;    // equilibrium order
constexpr int kCellStride = 48;   // doubles per cell in the cell-phase output

// Tables of one large model class.  Half range: the transposed within-half
// block KinT[j * H + k] = Kin[k][j]; full range (full = 1): the transposed
// dense matrix KT[j * V + k] = K[k][j].  Then HWs[k * (N+1) + l] for the H
// nodes with p > 0.
struct DevLarge {
  int32_t H, N, nm, full;
  double inv_p0;
  double sq[kNmaxLarge + 2];                       // sqrt(l), full range
  double ka[kQmaxLarge], kb[kQmaxLarge];
  double a[kNmaxLarge + 2], mb[kNmaxLarge + 2];   // monic recurrence
  double zm[kQmaxDev], wm[kQmaxDev];               // main rule (half-range Gauss-Hermite)
  int32_t lad_n[kLadderAll], lad_off[kLadderAll];   // calibrated entries, then composite ones
  double lad_y[kLadderAll];
  double ltau[kLadderPts], llamw[kLadderPts];
};

struct LargeArgs {
  const DevLarge *tl;
  const double *KinT, *HWs, *p;   // KinT: KT in the full range; p: V momenta
  const DevChannel *chans;
  const DevWindow *wins;
  int32_t nwin, stage;
  const double *inv_dx, *gw;
  const double *in_f, *in_c;      // stage state
  const double *base_f, *base_c;  // y^n
  double *out_f, *out_c;
  double a_base, b_stage;
  double *cell;                   // cell-phase output, kCellStride per cell
  double *lnw;                    // wall densities of this stage, 2 per channel
  double *nwall;                  // diagnostics copy (written in stage 2)
  unsigned long long *wide;       // cells whose equilibrium needed several correction panels
  int32_t nfun;
  int32_t xcd_map;                // 1: the blocks of a window run on one XCD
};

// Sum over aligned segments of W lanes (W = 64: the whole wave).
template <int W>
__device__ __forceinline__ double seg_sum(double x) {
#pragma unroll
  for (int off = W / 2; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Equilibrium coefficients of one axis at (u, T) for a segment of W lanes
// (every lane of the segment returns the same G^+_l and G^-_l, l <= N;
// lane = the lane's index within its segment): Sec. IV.B.3 by the change of
// variables, the main rule and the correction spread over the lanes and
// collected by segment sums; for the full range the closed-form recurrence
// of Sec. IV.A.3.  Called by every lane of the wave; W >= 16 holds the main
// rule (at most 11 points for N <= 20) and the largest correction (16).
// NM bounds the order N (the register arrays' size).  Returns whether the
// correction took a composite rule (|y0| beyond the ladder's calibrated
// range).
template <int W = 64, int NM = kNmaxLarge>
__device__ __forceinline__ bool axis_coeffs(const DevLarge *tl, double u, double T, int lane,
                                            double (&Gp)[NM + 1], double (&Gm)[NM + 1]) {
  const int N = tl->N;
#pragma unroll
  for (int l = 0; l <= NM; ++l) Gp[l] = Gm[l] = 0.0;
  if (tl->full) {
    // full range (Sec. IV.A.3): G_l = E[He_l(X)], X ~ N(m u/p0, m T/p0^2),
    // obeys G_{l+1} = ub G_l + l a G_{l-1} with a = m T/p0^2 - 1; kept as
    // G_l / sqrt(l!) against HWs = w_k h_l(z_k) (h_l = He_l / sqrt(l!)).
    // The mirrored half has h_l(-z) = (-1)^l h_l(z).
    const double ub = u * tl->inv_p0, aa = T * tl->inv_p0 * tl->inv_p0 - 1.0;
    Gp[0] = 1.0;
    if (N >= 1) Gp[1] = ub;
#pragma unroll
    for (int l = 1; l < NM; ++l)
      if (l + 1 <= N) Gp[l + 1] = (ub * Gp[l] + tl->sq[l] * aa * Gp[l - 1]) / tl->sq[l + 1];
#pragma unroll
    for (int l = 0; l <= NM; ++l) Gm[l] = (l & 1) ? -Gp[l] : Gp[l];
    return false;
  }
  const double sT = sqrt(T), s = sT * tl->inv_p0, y0 = -u / sT;
  auto accum = [&](double (&G)[NM + 1], double x, double wt) {
    double qm = 1.0, q = x - tl->a[0];
    G[0] += wt;
    if (N >= 1) G[1] += wt * q;
#pragma unroll
    for (int l = 1; l < NM; ++l) {
      if (l + 1 <= N) {
        const double qn = (x - tl->a[l]) * q - tl->mb[l] * qm;
        qm = q;
        q = qn;
        G[l + 1] += wt * q;
      }
    }
  };
  if (lane < tl->nm) {
    accum(Gp, u * tl->inv_p0 + s * tl->zm[lane], tl->wm[lane]);
    accum(Gm, -u * tl->inv_p0 + s * tl->zm[lane], tl->wm[lane]);
  }
  const double ymax = fabs(y0);
  bool wide = false;
  if (ymax > 0.0) {
    // the first entry, calibrated or composite, whose reach covers |y0|
    // (the last when none does, also for a non-finite |y0|)
    int li = kLadderAll - 1;
    for (int j = 1; j < kLadderAll; ++j)
      if (tl->lad_y[j] >= ymax) { li = j; break; }
    const int nc = tl->lad_n[li], o = tl->lad_off[li];
    wide = nc > tl->lad_n[kLadder - 1];
    // the segment's lanes take the entry's points W at a time: one pass
    // for a calibrated count (nc <= 16 <= W), more for a composite rule
    const int passes = (nc + W - 1) / W;
    for (int rr = 0; rr < passes; ++rr) {
      const int q = rr * W + lane;
      if (q < nc) {
        const double t = tl->ltau[o + q], yt = y0 * t;
        const double e = y0 * tl->llamw[o + q] * exp(-0.5 * yt * yt);
        accum(Gp, u * tl->inv_p0 * (1.0 - t), -e);
        accum(Gm, -u * tl->inv_p0 * (1.0 - t), e);
      }
    }
  }
#pragma unroll
  for (int l = 0; l <= NM; ++l) {
    if (l <= N) {
      Gp[l] = seg_sum<W>(Gp[l]);
      Gm[l] = seg_sum<W>(Gm[l]);
    }
  }
  return wide;
}

// Cell phase: a 1-D grid of nwin x (kCellGroups + 1) blocks; block b maps to
// window w and group y (with xcd_map, the groups of a window run on one
// XCD, so the cache lines its cells share stay in one L2).  For y <
// kCellGroups each wave takes one cell, i0 + 4 y + wave: its lanes run over
// the V nodes for the moments and projections, then over the quadrature
// points of the equilibrium (the main rule and the correction), and wave
// sums collect both.  Group kCellGroups: wave 0 the left-wall density if the
// window holds cell 0, wave 1 the right-wall one if it holds cell Nx-1
// (lanes over the incoming nodes).
constexpr int kCellGroups = (kWin + 3) / 4;

template <int ADV>
__global__ __launch_bounds__(256) void large_cell_kernel(LargeArgs A) {
  constexpr int G = kCellGroups + 1;
  const int lb = A.xcd_map ? xcd_window(blockIdx.x, A.nwin * G) : (int)blockIdx.x;
  const int gy = lb % G;
  const DevWindow win = A.wins[lb / G];
  const DevChannel C = A.chans[win.ch];
  const DevLarge *tl = A.tl;
  const int H = tl->H, V = 2 * H, N = tl->N, Nx = C.Nx;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double *yf = A.in_f + C.off, *yc = A.nfun > 1 ? A.in_c + C.off : nullptr;
  if (gy < kCellGroups) {
    const int r = 4 * gy + wave;
    const int i = win.i0 + r;
    if (r >= kWin || i >= Nx) return;   // wave-uniform
    // V <= 2 kQmaxLarge = 8 x 64: a fixed trip count and unconditional loads
    // (clamped index, the surplus terms selected away), so they issue at once
    constexpr int KT = 2 * kQmaxLarge / 64;
    double yv[KT], xv[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const int k = lane + 64 * t, kk = k < V ? k : V - 1;
      yv[t] = yf[(int64_t)kk * Nx + i];
      xv[t] = yc ? yc[(int64_t)kk * Nx + i] : 0.0;
    }
    double n = 0, mom = 0, s2 = 0, ech = 0, bf = 0, bc = 0;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const int k = lane + 64 * t, kk = k < V ? k : V - 1;
      const double v = A.p[kk], kbv = tl->kb[kk < H ? kk : kk - H];
      const double y = k < V ? yv[t] : 0.0, x = k < V ? xv[t] : 0.0;
      n += y;
      mom += v * y;
      s2 += v * v * y;
      bf += kbv * y;
      ech += x;
      bc += kbv * x;
    }
    n = wave_sum(n);
    mom = wave_sum(mom);
    s2 = wave_sum(s2);
    bf = wave_sum(bf);
    if (yc) {
      ech = wave_sum(ech);
      bc = wave_sum(bc);
    }
    const double u = mom / n;
    const double T = (s2 - u * mom + 2.0 * ech) * C.inv_1pDt / n;
    double Gp[kNmaxLarge + 1], Gm[kNmaxLarge + 1];
#pragma unroll
    for (int l = 0; l <= kNmaxLarge; ++l) Gp[l] = Gm[l] = 0.0;
    if (C.inv_Kn != 0.0) {
      const bool wide = axis_coeffs(tl, u, T, lane, Gp, Gm);
      if (wide && lane == 0 && A.wide) atomicAdd(A.wide, 1ull);
    }
    if (lane == 0) {
      double *out = A.cell + (int64_t)(C.cell_off + i) * kCellStride;
      out[0] = n;
      out[1] = T;
      out[2] = n * C.inv_Kn;
      out[3] = bf;
      out[4] = bc;
#pragma unroll
      for (int l = 0; l <= kNmaxLarge; ++l) {
        if (l <= N) {
          out[5 + l] = Gp[l];
          out[5 + kNmaxLarge + 1 + l] = Gm[l];
        }
      }
    }
    return;
  }
  // wall densities from the incoming wall-face fluxes of f (Eq. nplus_def):
  // ghosts extrapolated quadratically from the three nearest cells
  if (wave > 1) return;
  const bool left = wave == 0;
  if (left ? win.i0 != 0 : !(win.i0 <= Nx - 1 && Nx - 1 < win.i0 + kWin)) return;
  double acc = 0.0;
  for (int j = lane; j < H; j += 64) {
    const int k = left ? H + j : j;
    const double *row = yf + (int64_t)k * Nx;
    const double y0 = left ? row[0] : row[Nx - 1], y1 = left ? row[1] : row[Nx - 2],
                 y2 = left ? row[2] : row[Nx - 3];
    const double g1 = 3.0 * y0 - 3.0 * y1 + y2, g2 = 6.0 * y0 - 8.0 * y1 + 3.0 * y2;
    acc += A.p[k] * face_value<ADV>(y2, y1, y0, g1, g2);
  }
  const double nw = -wave_sum(acc) * (left ? C.inv_DL : C.inv_DR);
  if (lane == 0) {
    A.lnw[2 * win.ch + (left ? 0 : 1)] = nw;
    if (A.stage == 2 && A.nwall) A.nwall[2 * win.ch + (left ? 0 : 1)] = nw;
  }
}

// Node phase: a 1-D grid of nwin x 2 ceil(H/16) blocks; block b maps to a
// window and a tile of 16 nodes of one half (tiles never straddle the
// halves), four waves.  With xcd_map the tiles of a window run on one XCD:
// they all read the window's rows, which then stay in that XCD's L2.  The within-half force
// block is a contraction over the half's H rows, D[node][cell] =
// sum_j Kin[node][j] y_j[cell], run on FP64 MFMA 16x16x4 tiles: the rows are
// split over the four waves in steps of 4, the A operand (the transposed
// table) and the B operand (the rows of f or chi for the window's 64 cells)
// load straight from memory in the MFMA layout, and the four partial tiles
// are summed through LDS.  After that wave w owns nodes kt0 + 4w .. kt0 + 4w
// + 3, lane = cell i0 - kHalo + lane as in stage_kernel_half.
#ifndef HHLB_LARGE_WAVES
#define HHLB_LARGE_WAVES 4   // waves per node-phase block (the rows split over them)
#endif
#ifndef HHLB_LARGE_OCC
#define HHLB_LARGE_OCC 2     // waves per SIMD the node phase is compiled for
#endif
constexpr int kNodeWaves = HHLB_LARGE_WAVES;
constexpr int kTileNodes = 16;
constexpr int kStepsPerWave = (kQmaxLarge / 4 + kNodeWaves - 1) / kNodeWaves;   // per chunk

template <int ADV>
__global__ __launch_bounds__(64 * kNodeWaves) __attribute__((amdgpu_waves_per_eu(HHLB_LARGE_OCC))) void large_node_kernel(LargeArgs A) {
  constexpr int NG = kTileNodes / kNodeWaves;   // nodes per wave after the reduction
  constexpr int S = 65;                         // padded LDS row: 64 cells
  __shared__ double s_red[kNodeWaves * kTileNodes * S];
  __shared__ double s_hw[kTileNodes * (kNmaxLarge + 1)];   // HWs rows of the tile
  const DevLarge *tl = A.tl;
  const int H = tl->H, N = tl->N;
  const int gph = (H + kTileNodes - 1) / kTileNodes, ntile = 2 * gph;
  const int lb = A.xcd_map ? xcd_window(blockIdx.x, A.nwin * ntile) : (int)blockIdx.x;
  const int ty = lb % ntile;
  const DevWindow win = A.wins[lb / ntile];
  const DevChannel C = A.chans[win.ch];
  const int Nx = C.Nx;
  const int hw = ty / gph;                               // 0: p > 0, 1: p < 0
  const int kt0 = (ty % gph) * kTileNodes;               // first node of the tile
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = win.i0 - kHalo + lane;
  const bool inside = i >= 0 && i < Nx;
  const int ic = inside ? i : (i < 0 ? 0 : Nx - 1);      // clamped: loads stay in bounds
  const bool nfc = A.nfun > 1;
  const bool full = tl->full != 0;
  const double sg = full ? 1.0 : (hw ? -1.0 : 1.0);      // K = blockdiag(Kin, -Kin) + cross (half)
  const int64_t rowh = C.off + (int64_t)hw * H * Nx;     // first row of this half
  const double *fin = A.in_f + rowh, *cin = nfc ? A.in_c + rowh : nullptr;
  // rows of the contraction: the half's H rows, or all V = 2H (full range)
  const int nrows = full ? 2 * H : H;
  const double *rf = full ? A.in_f + C.off : fin;
  const double *rc = full ? (nfc ? A.in_c + C.off : nullptr) : cin;

  // the tile's equilibrium rows HWs[k][0..N] (read after the first barrier)
  for (int t = threadIdx.x; t < kTileNodes * (kNmaxLarge + 1); t += 64 * kNodeWaves) {
    const int q = t / (kNmaxLarge + 1), l = t % (kNmaxLarge + 1), k = kt0 + q;
    s_hw[t] = (k < H && l <= N) ? A.HWs[(int64_t)k * (N + 1) + l] : 0.0;
  }

  // force: MFMA contraction over this wave's share of the rows
  const int nsteps = (nrows + 3) / 4, spw = (nsteps + kNodeWaves - 1) / kNodeWaves;
  const int s0 = wave * spw;
  const int nsw = nsteps - s0 < 0 ? 0 : (nsteps - s0 < spw ? nsteps - s0 : spw);
  const int kr = lane >> 4, jl = lane & 15;
  const int an = kt0 + jl;                               // A row: node within the half
  const int acol = full ? hw * H + an : an;              // its column of the table
  int bcell[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int il = win.i0 - kHalo + 16 * c + jl;
    bcell[c] = il < 0 ? 0 : (il >= Nx ? Nx - 1 : il);
  }
  // chunks of kStepsPerWave steps (one chunk for the half range, Q <= 256;
  // two for a full-range V up to 512), every load of a chunk issued before
  // its first MFMA
  auto contract = [&](const double *src, dbl4 acc[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int t0 = 0; t0 < nsw; t0 += kStepsPerWave) {   // wave-uniform
      double av[kStepsPerWave], bv[kStepsPerWave][4];
#pragma unroll
      for (int t = 0; t < kStepsPerWave; ++t) {
        const int row = 4 * (s0 + t0 + t) + kr;
        const bool ok = t0 + t < nsw && row < nrows;
        const bool oka = ok && an < H;
        av[t] = A.KinT[oka ? (int64_t)row * nrows + acol : 0];
        if (!oka) av[t] = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[t][c] = ok ? src[(int64_t)row * Nx + bcell[c]] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < kStepsPerWave; ++t) {
        if (t0 + t >= nsw) break;   // wave-uniform: MFMA runs with every lane active
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t][c], acc[c], 0, 0, 0);
      }
    }
  };
  // D[node 4r + kr][cell 16c + jl] sits in acc[c][r]; partial tiles to LDS,
  // then wave w sums its NG nodes over the four partials
  auto reduce = [&](const dbl4 acc[4], double out[NG]) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) s_red[(wave * kTileNodes + 4 * r + kr) * S + 16 * c + jl] = acc[c][r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < kNodeWaves; ++w) v += s_red[(w * kTileNodes + wave * NG + q) * S + lane];
      out[q] = v;
    }
    __syncthreads();
  };
  double kf[NG], kc[NG];
  {
    dbl4 accf[4];
    contract(rf, accf);
    reduce(accf, kf);
  }
#pragma unroll
  for (int q = 0; q < NG; ++q) kc[q] = 0.0;
  if (nfc) {   // uniform over the block
    dbl4 accc[4];
    contract(rc, accc);
    reduce(accc, kc);
  }
  const int k0 = kt0 + wave * NG;                        // first node of this wave
  const int ng = H - k0 < NG ? H - k0 : NG;              // may be <= 0 in the last tile
  if (ng <= 0) return;   // wave-uniform, after the last barrier

  double yf[NG], yc[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int j = q < ng ? k0 + q : k0;
    yf[q] = inside ? fin[(int64_t)j * Nx + i] : 0.0;
    yc[q] = (inside && nfc) ? cin[(int64_t)j * Nx + i] : 0.0;
  }
  // wall ghosts (Sec. IV.C.3): incoming nodes extrapolated quadratically
  // from the three nearest cells, emergent nodes n_w g^w_k in all three
  const bool needL = win.i0 < kHalo, needR = win.i0 - kHalo + 63 >= Nx;
  if ((hw == 1 && needL) || (hw == 0 && needR)) {
    const bool lw = hw == 1;
    const int l0 = lw ? kHalo : Nx - 1 - (win.i0 - kHalo);
    const int dl = lw ? 1 : -1;
    const int gi = lw ? -i : i - Nx + 1;
    const double c0 = gi == 1 ? 3.0 : (gi == 2 ? 6.0 : 10.0);
    const double c1 = gi == 1 ? -3.0 : (gi == 2 ? -8.0 : -15.0);
    const double c2 = gi == 1 ? 1.0 : (gi == 2 ? 3.0 : 6.0);
    const bool ghost = gi >= 1 && gi <= 3;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const double y0 = readlane_d(yf[q], l0), y1 = readlane_d(yf[q], l0 + dl), y2 = readlane_d(yf[q], l0 + 2 * dl);
      const double x0 = readlane_d(yc[q], l0), x1 = readlane_d(yc[q], l0 + dl), x2 = readlane_d(yc[q], l0 + 2 * dl);
      if (ghost) {
        yf[q] = c0 * y0 + c1 * y1 + c2 * y2;
        yc[q] = c0 * x0 + c1 * x1 + c2 * x2;
      }
    }
  }
  const double nL = A.lnw[2 * win.ch], nR = A.lnw[2 * win.ch + 1];
  if (hw == 0 && i < 0) {
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const int k = q < ng ? k0 + q : k0;
      yf[q] = nL * A.gw[C.gw_off + k];
      yc[q] = nfc ? C.half_Dt * C.TL * yf[q] : 0.0;
    }
  }
  if (hw == 1 && i >= Nx && i <= Nx + 2) {
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const int k = q < ng ? k0 + q : k0;
      yf[q] = nR * A.gw[C.gw_off + 2 * H + H + k];
      yc[q] = nfc ? C.half_Dt * C.TR * yf[q] : 0.0;
    }
  }

  const double *cd = A.cell + (int64_t)(C.cell_off + ic) * kCellStride;
  const double n = cd[0], T = cd[1], inv_tau = cd[2], bf = cd[3], bc = cd[4];
  const double *Gp = cd + 5 + (hw ? kNmaxLarge + 1 : 0);
  double G[kNmaxLarge + 1];   // fixed trip count: the loads issue together
#pragma unroll
  for (int l = 0; l <= kNmaxLarge; ++l) G[l] = l <= N ? Gp[l] : 0.0;
  const double eqc = C.half_Dt * T;
  double srcf[NG], srcc[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int k = q < ng ? k0 + q : k0;
    const double *hwr = s_hw + (wave * NG + (q < ng ? q : 0)) * (kNmaxLarge + 1);
    double geq = 0.0;
    if (inv_tau != 0.0) {
#pragma unroll
      for (int l = 0; l <= kNmaxLarge; ++l) geq = fma(hwr[l], G[l], geq);
    }
    srcf[q] = -C.g * sg * (kf[q] + tl->ka[k] * bf) - (yf[q] - n * geq) * inv_tau;
    srcc[q] = -C.g * sg * (kc[q] + tl->ka[k] * bc) - (yc[q] - eqc * n * geq) * inv_tau;
  }

  // advection (lane-parallel face values) and the RK-3 combination
  const FaceCoef fcoef = face_coef(hw);
  const bool face_used = inside && lane >= kHalo - 1 + hw && lane < kHalo + kWin + hw;
  const bool wall_face = hw == 0 ? (i == -1) : (i == Nx);
  const bool out_lane = lane >= kHalo && lane < kHalo + kWin && inside;
  const double dx_inv = A.inv_dx[C.cell_off + ic];
  const double sdx = hw == 0 ? -dx_inv : dx_inv;
  const bool need_base = A.a_base != 0.0;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    if (q >= ng) break;
    const int k = k0 + q;
    const double v = A.p[hw * H + k];
    const int64_t o = rowh + (int64_t)k * Nx + ic;
#pragma unroll
    for (int fn = 0; fn < 2; ++fn) {
      if (fn == 1 && !nfc) break;
      const double y0v = fn == 0 ? yf[q] : yc[q];
      double fv = face_value_lanes<ADV>(y0v, fcoef, face_used);
      if (wall_face) fv = y0v;
      const double F = v * fv;
      const double Fo = hw == 0 ? dpp_shr1(F) : dpp_shl1(F);
      const double L = fma(sdx, F - Fo, fn == 0 ? srcf[q] : srcc[q]);
      const double base = need_base ? (fn == 0 ? A.base_f : A.base_c)[o] : 0.0;
      const double yn = A.a_base * base + A.b_stage * (y0v + C.dt * L);
      if (out_lane) (fn == 0 ? A.out_f : A.out_c)[o] = yn;
    }
  }
}

}  // namespace hhlb
