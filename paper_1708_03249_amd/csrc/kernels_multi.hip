// The mixed-quadrature (App. A) velocity-space stage kernel and its launcher.
#include "multi_kernels.hpp"

namespace hhlb {

// W lanes per point: W = 64 (one point per wave, V <= 512) or W = 16 (four
// points per wave, V <= 128); each lane holds velocities sub + W t, t < 8.
// NM bounds the axes' equilibrium orders (7 or 20: the size of the register
// arrays of the coefficients).
#if HHLB_MULTI_OCC
#define HHLB_MULTI_ATTR __attribute__((amdgpu_waves_per_eu(NM <= 7 ? HHLB_MULTI_OCC : 1)))
#else
#define HHLB_MULTI_ATTR
#endif
template <int W, int NM>
__global__ __launch_bounds__(64 * kMultiWaves) HHLB_MULTI_ATTR void multi_kernel(MultiArgs A) {
  constexpr int P = 64 / W;                 // points per wave
  constexpr int VW = 8 * W;                 // largest V for this width
  constexpr int KT = VW / W;
  __shared__ double s_f[kMultiWaves][P * VW];
  __shared__ double s_g[kMultiWaves][P * kMultiAxes * kMultiVaxis];
  extern __shared__ double s_K[];   // the axes' K_a, row-major, rows padded to multi_kcols(V_a), back to back
  __shared__ double s_p[kMultiAxes * kMultiVaxis];
  __shared__ int32_t s_idx[kMultiVmax];   // packed per-axis indices of each velocity
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int seg = lane / W, sub = lane % W;
  const DevMulti *tm = A.tm;
  const int d = tm->d, V = tm->V;
  // the block stages the axes' tables (every wave takes this barrier)
  int ko[kMultiAxes] = {0, 0, 0};   // offset of K_a in s_K
  int va[kMultiAxes] = {1, 1, 1}, kc[kMultiAxes] = {1, 1, 1}, st[kMultiAxes] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < kMultiAxes; ++a) {
    if (a >= d) break;
    const int Va = tm->Va[a], c = multi_kcols(Va);
    va[a] = Va;
    kc[a] = c;
    st[a] = tm->stride[a];
    if (a + 1 < kMultiAxes) ko[a + 1] = ko[a] + Va * c;
    for (int t = threadIdx.x; t < Va * c; t += 64 * kMultiWaves) {
      const int r = t / c, col = t - r * c;
      s_K[ko[a] + t] = col < Va ? A.tab[tm->k_off[a] + r * Va + col] : 0.0;
    }
    if ((int)threadIdx.x < Va) s_p[a * kMultiVaxis + threadIdx.x] = A.tab[tm->p_off[a] + threadIdx.x];
  }
  {
    const int32_t *gi = (const int32_t *)(A.tab + tm->idx_off);
    for (int t = threadIdx.x; t < V; t += 64 * kMultiWaves) s_idx[t] = gi[t];
  }
  __syncthreads();
  // a point past the end computes on the last point's data and stores nothing
  const int64_t pt0 = ((int64_t)blockIdx.x * kMultiWaves + wave) * P + seg;
  const bool valid = pt0 < A.npts;
  const int64_t pt = valid ? pt0 : A.npts - 1;
  const double *y = A.in + pt * V;
  double *sf = s_f[wave] + seg * VW, *sg = s_g[wave] + seg * kMultiAxes * kMultiVaxis;
  // per-axis indices of this lane's velocities (v = (i V_y + j) V_z + k)
  int ia[KT][kMultiAxes];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int v = sub + W * t, w = v < V ? s_idx[v] : 0;
#pragma unroll
    for (int a = 0; a < kMultiAxes; ++a) ia[t][a] = (w >> (8 * a)) & 0xff;
  }

  // populations (fixed trip count: the loads issue together) and moments
  double fv[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int v = sub + W * t;
    fv[t] = v < V ? y[v] : 0.0;
  }
  // y^n of the stages that combine with it, in one fixed-trip pass so that
  // the loads issue together: here (HHLB_MULTI_YN_EARLY, latency hidden behind
  // the moments and the equilibrium, 16 more live VGPRs) or, by default, just
  // before the contractions
  const bool use_base = !A.rhs_only && A.a_base != 0.0;
  double bv[KT];
#if HHLB_MULTI_YN_EARLY
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int v = sub + W * t;
    bv[t] = use_base && v < V ? A.base[pt * V + v] : 0.0;
  }
#endif
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int v = sub + W * t;
    if (v < V) sf[v] = fv[t];
  }
  double n = 0.0, mom[kMultiAxes] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int v = sub + W * t;
    if (v < V) {
      n += fv[t];
#pragma unroll
      for (int a = 0; a < kMultiAxes; ++a)
        if (a < d) mom[a] += s_p[a * kMultiVaxis + ia[t][a]] * fv[t];
    }
  }
  n = seg_sum<W>(n);
  double u[kMultiAxes] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < kMultiAxes; ++a)
    if (a < d) u[a] = seg_sum<W>(mom[a]) / n;
  double c2 = 0.0;
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int v = sub + W * t;
    if (v < V) {
      double q = 0.0;
#pragma unroll
      for (int a = 0; a < kMultiAxes; ++a)
        if (a < d) {
          const double c = s_p[a * kMultiVaxis + ia[t][a]] - u[a];
          q += c * c;
        }
      c2 += q * fv[t];
    }
  }
  const double T = seg_sum<W>(c2) / (d * n);

  // per-axis 1-D equilibrium factors g_a[i] (App. A.2) into LDS; a runtime
  // loop over the axes keeps one inlined copy of axis_coeffs (code size)
  if (A.inv_Kn != 0.0) {
#pragma unroll 1
    for (int a = 0; a < d; ++a) {
      const double ua = a == 0 ? u[0] : (a == 1 ? u[1] : u[2]);
      double Gp[NM + 1], Gm[NM + 1];
      axis_coeffs<W, NM>(&tm->ax[a], ua, T, sub, Gp, Gm);
      const int Va = tm->Va[a], H = Va / 2, N = tm->ax[a].N;
      for (int i = sub; i < Va; i += W) {
        const int k = i < H ? i : i - H;
        const double *hw = A.tab + tm->hw_off[a] + k * (N + 1);
        double gp = 0.0, gm = 0.0;
#pragma unroll
        for (int l = 0; l <= NM; ++l)
          if (l <= N) {
            gp = fma(hw[l], Gp[l], gp);
            gm = fma(hw[l], Gm[l], gm);
          }
        sg[a * kMultiVaxis + i] = i < H ? gp : gm;
      }
    }
  }
  __builtin_amdgcn_wave_barrier();

#if !HHLB_MULTI_YN_EARLY
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int v = sub + W * t;
    bv[t] = use_base && v < V ? A.base[pt * V + v] : 0.0;
  }
#endif

  // force contractions, BGK and the RK-3 combination (the populations come
  // back from LDS).  A row of K_a is taken kMultiGroup columns at a time; the
  // zero columns past V_a pair with the axis' last population, so the sum is
  // the plain one over i' < V_a in the same order.
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int v = sub + W * t;
    if (v >= V) continue;
    const double fvv = sf[v];
    const int w = s_idx[v];
    double force = 0.0, g = n;
#pragma unroll
    for (int a = 0; a < kMultiAxes; ++a) {
      if (a < d) {
        const int i = (w >> (8 * a)) & 0xff;
        const double *K = s_K + ko[a] + i * kc[a];
        const double *fa = sf + (v - i * st[a]);   // the populations along axis a through v
        double acc = 0.0;
        for (int ip = 0; ip < kc[a]; ip += kMultiGroup) {
          double kk[kMultiGroup], ff[kMultiGroup];
#pragma unroll
          for (int u = 0; u < kMultiGroup; ++u) {
            const int j = ip + u < va[a] ? ip + u : va[a] - 1;
            kk[u] = K[ip + u];
            ff[u] = fa[j * st[a]];
          }
#pragma unroll
          for (int u = 0; u < kMultiGroup; ++u) acc = fma(kk[u], ff[u], acc);
        }
        force = fma(A.F[a], acc, force);
        g *= sg[a * kMultiVaxis + i];
      }
    }
    double L = -force;
    if (A.inv_Kn != 0.0) L -= (fvv - g) * (n * A.inv_Kn);
    const int64_t o = pt * V + v;
    if (valid) A.out[o] = A.rhs_only ? L : A.a_base * bv[t] + A.b_stage * (fvv + A.dt * L);
  }
}

template <int W, int NM>
void launch_w(const MultiArgs &a, hipStream_t s, size_t shm) {
  const int64_t pts_per_block = (int64_t)(64 / W) * kMultiWaves;
  const int64_t blocks = (a.npts + pts_per_block - 1) / pts_per_block;
  hipLaunchKernelGGL((multi_kernel<W, NM>), dim3((unsigned)blocks), dim3(64 * kMultiWaves), shm, s, a);
}

void launch_multi(const MultiArgs &a, hipStream_t s, int V, int k_doubles, int n_max) {
  if (a.npts <= 0) return;
  const size_t shm = sizeof(double) * (size_t)k_doubles;   // the K_a tables
  const bool small_n = n_max <= 7;
  if (V <= 8 * 16) {   // four points per wave
    if (small_n) launch_w<16, 7>(a, s, shm);
    else launch_w<16, kNmaxLarge>(a, s, shm);
  } else {
    if (small_n) launch_w<64, 7>(a, s, shm);
    else launch_w<64, kNmaxLarge>(a, s, shm);
  }
}

}  // namespace hhlb
