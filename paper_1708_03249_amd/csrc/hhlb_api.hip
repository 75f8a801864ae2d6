// C ABI of the half-range lattice Boltzmann step library (declared in
// include/hhlb.h): argument checking, host tables, workspace layout, and the
// launch sequence of the three RK-3 stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hhlb.h"
#include "fused_kernels.hpp"
#include "large_kernels.hpp"
#include "launch.hpp"
#include "multi_kernels.hpp"
#include "step_kernels.hpp"
#include "tables.hpp"

namespace {

thread_local std::string g_err;

hhlb_status fail(hhlb_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return fail(HHLB_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

using hhlb::Launcher;

const hhlb::LaunchMap &launchers() {
  static hhlb::LaunchMap m = [] {
    hhlb::LaunchMap t;
    hhlb::register_fp64(t);
    hhlb::register_fp64_q16(t);
    hhlb::register_mixed_f32(t);
    hhlb::register_mixed_bf16(t);
    hhlb::register_mixed_f16(t);
    hhlb::register_classes(t);
    return t;
  }();
  return m;
}

// ---- auxiliary kernels ---------------------------------------------------

// Node weight that converts stored values to populations: w_k for the
// mixed form (phi_k = f_k / w_k), 1 for the FP64 form.
__device__ __forceinline__ double node_scale(const hhlb::DevTables *tb, int V, int k, int scaled) {
  return scaled ? tb->w[k % (V / 2)] : 1.0;
}

// Stored value at index j: the FP64 value, or the mixed form's FP32 value
// plus its 16-bit correction word.
__device__ __forceinline__ double stored(const double *y, const int16_t *, int64_t j) { return y[j]; }
__device__ __forceinline__ double stored(const float *y, const int16_t *lo, int64_t j) {
  const float hi = y[j];
  return (double)hi + (double)ldexpf((float)lo[j], __builtin_amdgcn_frexp_expf(hi) - 39);
}

template <typename S>
__global__ void moments_kernel(const hhlb::DevTables *tbs, const int32_t *ch_class,
                               const hhlb::DevChannel *chans, const int32_t *ch_V, int n_ch, int scaled,
                               const S *f, const int16_t *flo, const S *c, const int16_t *clo, int has_chi,
                               double *n_out, double *u_out, double *T_out) {
  const int ch = blockIdx.y;
  if (ch >= n_ch) return;
  const hhlb::DevChannel C = chans[ch];
  const hhlb::DevTables *tb = tbs + ch_class[ch];
  const int V = ch_V[ch];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < C.Nx; i += gridDim.x * blockDim.x) {
    double n = 0, mom = 0;
    for (int k = 0; k < V; ++k) {
      double y = node_scale(tb, V, k, scaled) * stored(f, flo, C.off + (int64_t)k * C.Nx + i);
      n += y;
      mom += tb->p[k] * y;
    }
    double u = mom / n, e2 = 0, ech = 0;
    for (int k = 0; k < V; ++k) {
      const double sc = node_scale(tb, V, k, scaled);
      double dp = tb->p[k] - u;
      e2 += dp * dp * sc * stored(f, flo, C.off + (int64_t)k * C.Nx + i);
      if (has_chi && C.half_Dt != 0.0) ech += sc * stored(c, clo, C.off + (int64_t)k * C.Nx + i);
    }
    n_out[C.cell_off + i] = n;
    u_out[C.cell_off + i] = u;
    T_out[C.cell_off + i] = (e2 + 2 * ech) * C.inv_1pDt / n;
  }
}

// Mass sum_i dx_i n_i per channel (Eq. Ndef) and the count of non-finite
// stored values (added to nonfinite[0] and flag[0]).
template <typename S>
__global__ void mass_kernel(const hhlb::DevTables *tbs, const int32_t *ch_class, const hhlb::DevChannel *chans,
                            const int32_t *ch_V, int n_ch, int scaled, const S *f, const int16_t *flo, const S *c,
                            int has_chi, const double *dx, double *mass, int32_t *nonfinite, int32_t *flag) {
  const int ch = blockIdx.x;
  if (ch >= n_ch) return;
  const hhlb::DevChannel C = chans[ch];
  const hhlb::DevTables *tb = tbs + ch_class[ch];
  const int V = ch_V[ch];
  __shared__ double part[256];
  double acc = 0;
  int bad = 0;
  for (int i = threadIdx.x; i < C.Nx; i += blockDim.x) {
    double n = 0;
    for (int k = 0; k < V; ++k) {
      const int64_t j = C.off + (int64_t)k * C.Nx + i;
      const double y = stored(f, flo, j);
      n += node_scale(tb, V, k, scaled) * y;
      if (!isfinite(y)) ++bad;
      if (has_chi && C.half_Dt != 0.0 && !isfinite((double)c[j])) ++bad;
    }
    acc += dx[C.cell_off + i] * n;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && mass) mass[ch] = part[0];
  if (bad) {
    if (nonfinite) atomicAdd(nonfinite, bad);
    atomicAdd(flag, bad);
  }
}

// Residual per channel: max over f (and chi) of ||y1 - y||_inf / (dt ||y||_inf)
// with y1 = y + dt L[y] one forward-Euler stage from the current state.
// d1 holds y1 (FP64 form) or the increment y1 - y (mixed form).
template <typename S>
__global__ void residual_kernel(const hhlb::DevTables *tbs, const int32_t *ch_class,
                                const hhlb::DevChannel *chans, const int32_t *ch_V, int n_ch, int scaled,
                                int increment, const S *f, const S *f1, const S *c, const S *c1, int has_chi,
                                double *res) {
  const int ch = blockIdx.x;
  if (ch >= n_ch) return;
  const hhlb::DevChannel C = chans[ch];
  const hhlb::DevTables *tb = tbs + ch_class[ch];
  const int V = ch_V[ch];
  const bool chi = has_chi && C.half_Dt != 0.0;
  __shared__ double part[4][256];
  double df = 0, nf = 0, dc = 0, nc = 0;
  const int64_t total = (int64_t)V * C.Nx;
  for (int64_t j = threadIdx.x; j < total; j += blockDim.x) {
    const double sc = node_scale(tb, V, (int)(j / C.Nx), scaled);
    const double y = (double)f[C.off + j], y1 = (double)f1[C.off + j];
    df = fmax(df, sc * fabs(increment ? y1 : y1 - y));
    nf = fmax(nf, sc * fabs(y));
    if (chi) {
      const double x = (double)c[C.off + j], x1 = (double)c1[C.off + j];
      dc = fmax(dc, sc * fabs(increment ? x1 : x1 - x));
      nc = fmax(nc, sc * fabs(x));
    }
  }
  part[0][threadIdx.x] = df; part[1][threadIdx.x] = nf;
  part[2][threadIdx.x] = dc; part[3][threadIdx.x] = nc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 4; ++q) part[q][threadIdx.x] = fmax(part[q][threadIdx.x], part[q][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double r = part[0][0] / (C.dt * part[1][0]);
    if (chi) r = fmax(r, part[2][0] / (C.dt * part[3][0]));
    res[ch] = r;
  }
}

// Store a population value: FP64 as is; mixed form as FP32 value plus the
// correction word of the rounding error.
__device__ __forceinline__ void put(double *y, int16_t *, int64_t j, double v) { y[j] = v; }
__device__ __forceinline__ void put(float *y, int16_t *lo, int64_t j, double v) {
  const float hi = (float)v;
  y[j] = hi;
  const double q = rint(ldexp(v - (double)hi, 39 - __builtin_amdgcn_frexp_expf(hi)));
  lo[j] = (int16_t)fmin(fmax(q, -32767.0), 32767.0);
}

// f_k = feq_k in every cell (chi = (Dt/2) T0 f), in the stored form.
template <typename S>
__global__ void fill_kernel(const hhlb::DevTables *tbs, const int32_t *ch_class, const hhlb::DevChannel *chans,
                            const int32_t *ch_V, int n_ch, int scaled, const double *feq, const int32_t *feq_off,
                            double T0, S *f, int16_t *flo, S *c, int16_t *clo) {
  const int ch = blockIdx.y;
  if (ch >= n_ch) return;
  const hhlb::DevChannel C = chans[ch];
  const hhlb::DevTables *tb = tbs + ch_class[ch];
  const int V = ch_V[ch];
  const int64_t total = (int64_t)V * C.Nx;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(j / C.Nx);
    const double y = feq[feq_off[ch] + k] / node_scale(tb, V, k, scaled);
    put(f, flo, C.off + j, y);
    if (c) put(c, clo, C.off + j, C.half_Dt * T0 * y);
  }
}

// Boundary conversion between FP64 populations and the stored form:
// to_state: stored = pop / w_k; else pop = w_k * stored.
template <typename S>
__global__ void convert_kernel(const hhlb::DevTables *tbs, const int32_t *ch_class, const hhlb::DevChannel *chans,
                               const int32_t *ch_V, int n_ch, int scaled, int to_state, double *pop, S *st,
                               int16_t *lo) {
  const int ch = blockIdx.y;
  if (ch >= n_ch) return;
  const hhlb::DevChannel C = chans[ch];
  const hhlb::DevTables *tb = tbs + ch_class[ch];
  const int V = ch_V[ch];
  const int64_t total = (int64_t)V * C.Nx;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total;
       j += (int64_t)gridDim.x * blockDim.x) {
    const double sc = node_scale(tb, V, (int)(j / C.Nx), scaled);
    if (to_state) put(st, lo, C.off + j, pop[C.off + j] / sc);
    else pop[C.off + j] = sc * stored(st, lo, C.off + j);
  }
}

__global__ void zero_kernel(int32_t *p) { *p = 0; }

// chi of the channels without transverse degrees of freedom (Dt = 0): the
// kernels never advance it, so the boundary reports it as zero.
__global__ void zero_chi_kernel(const hhlb::DevChannel *chans, const int32_t *ch_V, int n_ch, double *chi) {
  const int ch = blockIdx.y;
  if (ch >= n_ch) return;
  const hhlb::DevChannel C = chans[ch];
  if (C.half_Dt != 0.0) return;
  const int64_t total = (int64_t)ch_V[ch] * C.Nx;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x)
    chi[C.off + j] = 0.0;
}

}  // namespace

// ---- solver ---------------------------------------------------------------

struct ModelClass {
  int quad, Q, N, adv, Dt;
  double p0;
  hhlb::Rule rule;
  hhlb::DevTables dev;
  Launcher launch = nullptr;    // two waves per window
  Launcher launch4 = nullptr;   // four waves per window (FP64, f and chi), if built
  Launcher fused = nullptr;     // one launch per RK-3 step (FP64 half range), if built
  std::vector<hhlb::DevWindow> windows;
  size_t win_off = 0;  // byte offset in workspace
  std::vector<hhlb::DevFusedWindow> fwindows;   // the fused kernel's windows (9-cell halos)
  size_t fwin_off = 0;
  // Q > 16 (half-range Hermite, FP64): the node-parallel stage, whose tables
  // (DevLarge, then KinT and HWs) live in their own workspace block
  bool large = false;
  std::vector<char> lblob;
  size_t lbl_off = 0;
};

struct hhlb_solver {
  std::vector<hhlb_channel> ch;
  std::vector<int> ch_class;
  std::vector<ModelClass> classes;
  std::vector<hhlb::DevChannel> dch;
  std::vector<int64_t> off;     // state offsets (elements), n_ch+1
  std::vector<int32_t> cell_off;
  std::vector<double> dx, inv_dx, gw, dts;
  std::vector<int32_t> Vs;
  int64_t total_state = 0, total_cells = 0;
  bool has_chi = false;
  bool any_dt0 = false;   // some channel has Dt = 0 (no chi of its own)
  int precision = HHLB_FP64;
  size_t esize = sizeof(double);   // bytes per stored population
  hipStream_t stream = nullptr;
  // workspace layout (byte offsets)
  size_t o_tables = 0, o_chans = 0, o_chclass = 0, o_V = 0, o_dx = 0, o_invdx = 0, o_gw = 0,
         o_nwall = 0, o_feq = 0, o_feqoff = 0, o_flag = 0, o_wide = 0, o_state = 0, bytes = 0;
  // large classes: per-cell output of the cell phase and the stage's wall densities
  size_t o_cell = 0, o_lnw = 0;
  bool any_large = false;
  char *ws = nullptr;
  // stored state.  FP64 form: hi[0] = y^n (the last stage updates it in
  // place), B and C = RK stage values.  Mixed form: hi[par] + lo[par] = y^n
  // as FP32 value and 16-bit correction word (a ping-pong pair, par flips
  // every step), B and C = stage increments y_s - y^n in FP32.
  void *hiF[2] = {nullptr, nullptr}, *hiC[2] = {nullptr, nullptr};
  int16_t *loF[2] = {nullptr, nullptr}, *loC[2] = {nullptr, nullptr};
  void *fB = nullptr, *fC = nullptr, *cB = nullptr, *cC = nullptr;
  int par = 0;
  void *fA() const { return hiF[par]; }
  void *cA() const { return hiC[par]; }
  int16_t *lA() const { return loF[par]; }
  int16_t *lcA() const { return loC[par]; }
  // non-finite count of the last hhlb_diagnostics, read back by the next hhlb_step
  int32_t *flag_host = nullptr;
  hipEvent_t ev_flag = nullptr;
  bool flag_pending = false;
  // launch configuration (hhlb_set_tuning / hhlb_autotune): direct launches,
  // classes one after the other, XCD-aware window mapping by default
  hhlb_tuning tuning = {0, 0, 1, 2, 0, 0, 0.0f};
  // launches across classes (hhlb_tuning.merge_classes): FP64 half-range
  // classes with the same functions and scheme take one launch per stage
  struct MergeGroup {
    Launcher launch = nullptr;
    int qtop = 0;
    std::vector<size_t> members;
    std::vector<hhlb::DevClassWindow> wins;
    size_t win_off = 0;
  };
  std::vector<MergeGroup> groups;
  std::vector<int> class_group;        // group of each class, -1: launched alone
  std::vector<hipStream_t> cstreams;   // one per model class (class_streams)
  std::vector<hipEvent_t> cjoin;
  hipEvent_t cfork = nullptr;
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gexec_k[2] = {nullptr, nullptr}, gexec_1[2] = {nullptr, nullptr};  // per starting parity
  bool has_graphs() const {
    for (int p = 0; p < 2; ++p)
      if (gexec_k[p] || gexec_1[p]) return true;
    return false;
  }
  // Wait until nothing the solver enqueued is in flight: the caller's
  // stream (graph replays are joined back into it), the replay stream and
  // the class streams.
  void quiesce() {
    (void)hipStreamSynchronize(stream);
    if (gstream) (void)hipStreamSynchronize(gstream);
    for (hipStream_t st : cstreams) (void)hipStreamSynchronize(st);
  }
  // Graph executables are destroyed only once no replay of them can still
  // be queued or running.
  void drop_graphs() {
    if (!has_graphs()) return;
    quiesce();
    for (int p = 0; p < 2; ++p) {
      if (gexec_k[p]) (void)hipGraphExecDestroy(gexec_k[p]);
      if (gexec_1[p]) (void)hipGraphExecDestroy(gexec_1[p]);
      gexec_k[p] = gexec_1[p] = nullptr;
    }
  }
  ~hhlb_solver() {
    quiesce();
    drop_graphs();
    for (hipEvent_t e : cjoin) (void)hipEventDestroy(e);
    for (hipStream_t st : cstreams) (void)hipStreamDestroy(st);
    if (cfork) (void)hipEventDestroy(cfork);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (ev_flag) (void)hipEventDestroy(ev_flag);
    if (flag_host) (void)hipHostFree(flag_host);
  }
  bool mixed() const { return precision != HHLB_FP64; }
};

namespace {

hhlb_status check_channel(const hhlb_channel &c, int idx) {
  auto bad = [&](const char *what) {
    return fail(HHLB_E_ARG, "channel " + std::to_string(idx) + ": " + what);
  };
  if (c.quad != HHLB_HALF_HERMITE && c.quad != HHLB_FULL_HERMITE && c.quad != HHLB_HALF_LAGUERRE)
    return bad("unknown quadrature");
  if (c.Q < 1) return bad("Q must be >= 1");
  if (c.quad == HHLB_FULL_HERMITE && (c.Q % 2)) return bad("full-range Q must be even");
  int N = c.N < 0 ? std::min(20, c.Q - 1) : c.N;
  if (N >= c.Q) return bad("N must satisfy 0 <= N < Q");
  if (c.Nx < 8) return bad("Nx must be >= 8");
  if (c.adv != HHLB_WENO5 && c.adv != HHLB_UPWIND3) return bad("unknown advection scheme");
  if (c.transverse_dof != 0 && c.transverse_dof != 2) return bad("transverse_dof must be 0 or 2");
  if (!(c.L > 0) || !std::isfinite(c.L)) return bad("L must be positive");
  if (!(c.stretch_A >= 0 && c.stretch_A < 1)) return bad("stretch_A must be in [0,1)");
  if (!(c.Kn > 0)) return bad("Kn must be > 0 (INFINITY for collisionless)");
  if (!std::isfinite(c.g)) return bad("g must be finite");
  if (!(c.T_left > 0) || !(c.T_right > 0) || !std::isfinite(c.T_left) || !std::isfinite(c.T_right))
    return bad("wall temperatures must be positive");
  if (!(c.p0 > 0) || !std::isfinite(c.p0)) return bad("p0 must be positive");
  if (!(c.dt != 0) || !std::isfinite(c.dt)) return bad("dt must be non-zero and finite");
  return HHLB_OK;
}

// Grid of Eqs. (x_eta) and (etai): the cell widths
// dx_i = x(eta_{i+1/2}) - x(eta_{i-1/2}).  On the stretched grid the
// difference of the two faces is taken in closed form,
// tanh a - tanh b = sinh(a - b) / (cosh a cosh b), which keeps full relative
// accuracy for the thin cells next to the walls (the difference of faces near
// +-L/2 would cancel).
void make_grid(const hhlb_channel &c, std::vector<double> &dx) {
  const int Nx = c.Nx;
  dx.resize(Nx);
  if (c.stretch_A == 0.0) {
    for (int i = 0; i < Nx; ++i) dx[i] = (double)((long double)c.L / Nx);
  } else {
    const long double A = c.stretch_A, deta = 2.0L / Nx * atanhl(A), sd = sinhl(deta);
    for (int i = 0; i < Nx; ++i) {
      const long double a = (i + 1 - Nx / 2.0L) * deta, b = (i - Nx / 2.0L) * deta;   // faces i+1/2, i-1/2
      dx[i] = (double)((long double)c.L / (2 * A) * sd / (coshl(a) * coshl(b)));
    }
  }
}

// Round-to-nearest-even conversions of FP32 values, as the matrix-core
// operands see them (finite values of normal range).
float round_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  float y;
  std::memcpy(&y, &u, 4);
  return y;
}
float round_f16(float x) { return (float)(_Float16)x; }

// Windows of the fused-step kernel for one channel of Nx cells.  A window's
// edge is a wall whose first two ghosts fit in the 64 lanes, or lies inside
// the channel with its whole 9-lane halo (lane 63 at a cell).
//  - Nx <= 58: one window, both walls, three ghosts each (c0 = -3);
//    Nx = 59, 60: one window with two ghosts per wall (c0 = -2);
//  - else a left-wall window (c0 = -3, 52 cells on lanes 3..54), interior
//    windows of 46 cells (c0 = first cell - 9), and a right-wall window
//    once at most 53 cells remain (cell Nx-1 at lane <= 61).
//  An interior edge needs at least 55 remaining cells after the window's
//  first output; a window takes one cell less whenever the remainder would
//  be exactly 54, which neither kind of window can start from.
void fused_windows(int ch, int Nx, std::vector<hhlb::DevFusedWindow> &w) {
  if (Nx <= 60) {
    w.push_back({ch, 0, Nx <= 58 ? -3 : -2, Nx});
    return;
  }
  int o = 0;
  bool first = true;
  for (;;) {
    const int R = Nx - o;
    if (!first && R <= 53) {
      w.push_back({ch, o, o - 9, R});
      return;
    }
    int m = first ? 52 : 46;
    if (R - m == 54) --m;
    w.push_back({ch, o, first ? -3 : o - 9, m});
    o += m;
    first = false;
  }
}

// Device tables of one model class (quadrature, Q, N, p0).
// Correction rules beyond the calibrated ladder (entries kLadder..): the top
// count on 2, 4, .., 64 equal panels of [y0, 0], each panel within the top
// count's reach, so the composite rule reaches that many times as far (the
// nodes (p + tau_q)/P, the weights lambda_q/P), tabulated after the
// calibrated points from offset o.  Without a calibrated top reach the
// entries repeat the top one.  T is DevTables or DevLarge.
template <class T>
void add_composite_entries(T &d, int o, double ytop, long double inv_s2pi) {
  static_assert(hhlb::kLadderTop * (2 + 4 + 8 + 16 + 32 + 64) + 64 <= hhlb::kLadderPts, "ladder points");
  std::vector<long double> tt, lt;
  hhlb::gauss_legendre01(hhlb::kLadderTop, tt, lt);
  for (int c = 0; c < hhlb::kComposite; ++c) {
    const int j = hhlb::kLadder + c, P = 2 << c;
    if (!(ytop > 0.0)) {
      d.lad_n[j] = d.lad_n[hhlb::kLadder - 1];
      d.lad_off[j] = d.lad_off[hhlb::kLadder - 1];
      d.lad_y[j] = ytop;
      continue;
    }
    d.lad_n[j] = hhlb::kLadderTop * P;
    d.lad_off[j] = o;
    d.lad_y[j] = ytop * P;
    for (int pnl = 0; pnl < P; ++pnl)
      for (int q = 0; q < hhlb::kLadderTop; ++q) {
        d.ltau[o + pnl * hhlb::kLadderTop + q] = (double)((pnl + tt[q]) / P);
        d.llamw[o + pnl * hhlb::kLadderTop + q] = (double)(lt[q] / P * inv_s2pi);
      }
    o += hhlb::kLadderTop * P;
  }
}

hhlb_status make_tables(const hhlb_channel &h, int N, int precision, const hhlb::Rule &r, hhlb::DevTables &d) {
  std::memset(&d, 0, sizeof(d));
  for (int k = 0; k < r.V; ++k) d.p[k] = r.p[k];
  for (int k = 0; k < r.H; ++k) { d.z[k] = (double)r.z[k]; d.w[k] = (double)r.w[k]; }
  for (int l = 0; l < h.Q + 1 && l < (int)r.a.size(); ++l) d.a[l] = (double)r.a[l];
  for (int l = 0; l < h.Q + 2 && l < (int)r.b.size(); ++l) {
    d.sb[l] = (double)sqrtl(r.b[l]);
    d.isb[l] = (double)(1.0L / sqrtl(r.b[l]));
  }
  if (hhlb::half_range(h.quad)) {
    for (int j = 0; j < r.H * r.H; ++j) d.Kin[j] = r.Kin[j];
    for (int k = 0; k < r.H; ++k) { d.ka[k] = r.ka[k]; d.kb[k] = r.kb[k]; }
    for (int k = 0; k < r.H; ++k)
      for (int l = 0; l < h.Q; ++l) d.HW[k * h.Q + l] = l <= N ? r.HW[(size_t)k * h.Q + l] : 0.0;
  } else {
    for (int j = 0; j < r.V * r.V; ++j) d.Kin[j] = r.K[j];
    for (int k = 0; k < r.V; ++k)
      for (int l = 0; l < h.Q; ++l) d.HW[k * h.Q + l] = l <= N ? r.HW[(size_t)k * h.Q + l] : 0.0;
  }
  std::vector<long double> tau, lam;
  hhlb::gauss_legendre01(hhlb::kNc, tau, lam);
  const long double inv_s2pi = 1.0L / sqrtl(2 * 3.141592653589793238462643383279502884L);
  for (int j = 0; j < hhlb::kNc; ++j) { d.tau[j] = (double)tau[j]; d.lamw[j] = (double)(lam[j] * inv_s2pi); }
  d.inv_p0 = 1.0 / h.p0;
  // monic recurrence and the normalisation folded into the contraction
  std::vector<long double> HWs((size_t)r.H * h.Q, 0.0L);
  {
    long double prod = 1;
    for (int l = 0; l < h.Q + 1 && l < (int)r.b.size(); ++l) d.mb[l] = (double)r.b[l];
    std::vector<long double> inv_norm(h.Q);
    for (int l = 0; l < h.Q; ++l) { prod *= r.b[l]; inv_norm[l] = 1.0L / sqrtl(prod); }
    if (hhlb::half_range(h.quad))
      for (int k = 0; k < r.H; ++k)
        for (int l = 0; l < h.Q; ++l) {
          HWs[(size_t)k * h.Q + l] = l <= N ? (long double)r.HW[(size_t)k * h.Q + l] * inv_norm[l] : 0.0L;
          d.HWs[k * h.Q + l] = (double)HWs[(size_t)k * h.Q + l];
        }
  }
  if (hhlb::half_range(h.quad)) {
    // main rule of the half-range equilibrium: M = ceil((N+1)/2) points
    // (a half-range Gauss-Hermite rule for either half-range kind)
    const int M = (N + 2) / 2;
    hhlb::Rule rm;
    std::string err2;
    int st2 = hhlb::build_rule(HHLB_HALF_HERMITE, M, 1.0, rm, err2);
    if (st2) return fail(st2, "equilibrium rule: " + err2);
    d.nm = M;
    for (int j = 0; j < M; ++j) { d.zm[j] = (double)rm.z[j]; d.wm[j] = (double)rm.w[j]; }
    // tables of the scaled (phi = f / w) mixed-precision form
    for (int k = 0; k < r.H; ++k) {
      const long double wk = r.w[k];
      d.wq[k] = (double)wk;
      d.iwq[k] = (double)(1.0L / wk);
      d.kbs[k] = (double)((long double)r.kb[k] * wk);
      d.kas[k] = (float)((long double)r.ka[k] / wk);
      for (int j = 0; j < r.H; ++j) d.Ks[k * r.H + j] = (float)((long double)r.Kin[k * r.H + j] * r.w[j] / wk);
      for (int l = 0; l < h.Q; ++l) d.HWss[k * h.Q + l] = (double)(HWs[(size_t)k * h.Q + l] / wk);
    }
    for (int k = 0; k < r.V; ++k) {
      const long double wk = r.w[k % r.H], pk = r.p[k];
      d.wpq[k] = (double)(wk * pk);
      d.wpfq[k] = (double)(wk * (long double)(float)r.p[k]);
      d.wp2q[k] = (double)(wk * pk * pk);
      d.pf[k] = (float)r.p[k];
    }
    // reduced-precision operands: FP16 row scales, and the weighted column
    // sums of the block exactly as the matrix cores round it
    long double wsum = 0;
    for (int k = 0; k < r.H; ++k) wsum += r.w[k];
    d.iwh = (float)(1.0L / wsum);
    for (int k = 0; k < r.H; ++k) {
      float m = 0.0f;
      for (int j = 0; j < r.H; ++j) m = std::max(m, std::fabs(d.Ks[k * r.H + j]));
      int e = 0;
      std::frexp(m, &e);
      const float rs = std::ldexp(1.0f, -e);
      d.irsc[k] = std::ldexp(1.0f, e);
      for (int j = 0; j < r.H; ++j) d.Ks16[k * r.H + j] = d.Ks[k * r.H + j] * rs;
    }
    // the operands' high part rounds the table entry, the low part rounds
    // the (exactly representable) remainder
    for (int j = 0; j < r.H; ++j) {
      long double c = 0, cl = 0;
      for (int k = 0; k < r.H; ++k) {
        float kh = d.Ks[k * r.H + j], kl = 0.0f;
        if (precision == HHLB_MIXED_BF16) {
          kh = round_bf16(d.Ks[k * r.H + j]);
          kl = round_bf16(d.Ks[k * r.H + j] - kh);
        } else if (precision == HHLB_MIXED_F16) {
          // the low part as the kernel forms it: the remainder rounded to
          // FP16 at 2^11 times its size, then scaled back (exact)
          const float x = d.Ks16[k * r.H + j], xh = round_f16(x);
          kh = xh * d.irsc[k];
          kl = round_f16((x - xh) * 2048.0f) / 2048.0f * d.irsc[k];
        }
        c += r.w[k] * (long double)kh;
        cl += r.w[k] * (long double)kl;
      }
      d.crs[j] = (float)c;
      d.crs_lo[j] = (float)cl;
    }
  }
  // correction ladder (half range): point counts and the |y0| each covers
  static constexpr int counts[hhlb::kLadder] = {0, 2, 3, 4, 6, 8, 12, 16};
  double limits[hhlb::kLadder] = {0};
  if (hhlb::half_range(h.quad)) hhlb::correction_limits(r, N, counts, hhlb::kLadder, 3e-16, limits);
  int o = 0;
  for (int j = 0; j < hhlb::kLadder; ++j) {
    d.lad_n[j] = counts[j];
    d.lad_off[j] = o;
    d.lad_y[j] = limits[j];
    if (counts[j] > 0) {
      std::vector<long double> t2, l2;
      hhlb::gauss_legendre01(counts[j], t2, l2);
      for (int q = 0; q < counts[j]; ++q) {
        d.ltau[o + q] = (double)t2[q];
        d.llamw[o + q] = (double)(l2[q] * inv_s2pi);
      }
    }
    o += counts[j];
  }
  add_composite_entries(d, o, limits[hhlb::kLadder - 1], inv_s2pi);
  return HHLB_OK;
}

// The device tables of a model class, built once per process: the
// correction-ladder calibration evaluates the equilibrium thousands of times
// (about 0.1 s per class), and solvers (e.g. one per channel) often repeat
// the same classes.
hhlb_status cached_tables(const hhlb_channel &h, int N, int precision, const hhlb::Rule &r, hhlb::DevTables &d) {
  using Key = std::tuple<int, int, int, double, int>;
  static std::mutex mu;
  static std::map<Key, hhlb::DevTables> cache;
  const Key key{h.quad, h.Q, N, h.p0, precision};
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      d = it->second;
      return HHLB_OK;
    }
  }
  hhlb_status st = make_tables(h, N, precision, r, d);
  if (st) return st;
  std::lock_guard<std::mutex> lock(mu);
  cache.emplace(key, d);
  return HHLB_OK;
}

// Tables of a large class (Q > 16): the momenta in DevTables (the aux
// kernels read them there) and the node-parallel stage's block.
hhlb_status make_large_tables(const hhlb_channel &h, int N, const hhlb::Rule &r, hhlb::DevTables &d,
                              std::vector<char> &blob) {
  std::memset(&d, 0, sizeof(d));
  for (int k = 0; k < r.V; ++k) d.p[k] = r.p[k];
  d.inv_p0 = 1.0 / h.p0;
  const int H = r.H, Q = h.Q, V = r.V;
  const bool full = h.quad == HHLB_FULL_HERMITE;
  const int rows = full ? V : H;
  const size_t nK = (size_t)rows * rows, nW = (size_t)H * (N + 1);
  blob.assign(sizeof(hhlb::DevLarge) + sizeof(double) * (nK + nW), 0);
  hhlb::DevLarge &L = *(hhlb::DevLarge *)blob.data();
  double *KinT = (double *)(blob.data() + sizeof(hhlb::DevLarge));
  double *HWs = KinT + nK;
  L.H = H;
  L.N = N;
  L.inv_p0 = 1.0 / h.p0;
  if (full) {
    // Eq. (H_Kk), transposed: KT[j V + k] = K[k][j]; no cross term.  HWs in
    // the orthonormal form w_k h_l(z_k) = w_k He_l(z_k) / l! * sqrt(l!)
    // (the table holds w_k He_l(z_k) / l!) for the H nodes with p > 0.
    L.full = 1;
    for (int l = 0; l <= hhlb::kNmaxLarge + 1; ++l) L.sq[l] = std::sqrt((double)l);
    for (int j = 0; j < V; ++j)
      for (int k = 0; k < V; ++k) KinT[(size_t)j * V + k] = r.K[(size_t)k * V + j];
    long double sf = 1;
    for (int l = 0; l <= N; ++l) {
      if (l > 0) sf *= sqrtl((long double)l);
      for (int k = 0; k < H; ++k)
        HWs[(size_t)k * (N + 1) + l] = (double)((long double)r.HW[(size_t)k * Q + l] * sf);
    }
    return HHLB_OK;
  }
  for (int k = 0; k < H; ++k) { L.ka[k] = r.ka[k]; L.kb[k] = r.kb[k]; }
  for (int l = 0; l <= N + 1 && l < (int)r.a.size(); ++l) { L.a[l] = (double)r.a[l]; L.mb[l] = (double)r.b[l]; }
  for (int j = 0; j < H; ++j)
    for (int k = 0; k < H; ++k) KinT[(size_t)j * H + k] = r.Kin[(size_t)k * H + j];
  // monic recurrence: the normalisation 1/sqrt(b_0 .. b_l) folds into HWs
  long double prod = 1;
  std::vector<long double> inv_norm(N + 1);
  for (int l = 0; l <= N; ++l) { prod *= r.b[l]; inv_norm[l] = 1.0L / sqrtl(prod); }
  for (int k = 0; k < H; ++k)
    for (int l = 0; l <= N; ++l) HWs[(size_t)k * (N + 1) + l] = (double)((long double)r.HW[(size_t)k * Q + l] * inv_norm[l]);
  // main rule of the equilibrium integral: M = ceil((N+1)/2) half-range points
  const int M = (N + 2) / 2;
  hhlb::Rule rm;
  std::string err2;
  int st2 = hhlb::build_rule(HHLB_HALF_HERMITE, M, 1.0, rm, err2);
  if (st2) return fail(st2, "equilibrium rule: " + err2);
  L.nm = M;
  for (int j = 0; j < M; ++j) { L.zm[j] = (double)rm.z[j]; L.wm[j] = (double)rm.w[j]; }
  static constexpr int counts[hhlb::kLadder] = {0, 2, 3, 4, 6, 8, 12, 16};
  static_assert(hhlb::kLadderTop == counts[hhlb::kLadder - 1], "top ladder count");
  double limits[hhlb::kLadder] = {0};
  hhlb::correction_limits(r, N, counts, hhlb::kLadder, 3e-16, limits);
  const long double inv_s2pi = 1.0L / sqrtl(2 * 3.141592653589793238462643383279502884L);
  int o = 0;
  for (int j = 0; j < hhlb::kLadder; ++j) {
    L.lad_n[j] = counts[j];
    L.lad_off[j] = o;
    L.lad_y[j] = limits[j];
    if (counts[j] > 0) {
      std::vector<long double> t2, l2;
      hhlb::gauss_legendre01(counts[j], t2, l2);
      for (int q = 0; q < counts[j]; ++q) {
        L.ltau[o + q] = (double)t2[q];
        L.llamw[o + q] = (double)(l2[q] * inv_s2pi);
      }
    }
    o += counts[j];
  }
  add_composite_entries(L, o, limits[hhlb::kLadder - 1], inv_s2pi);
  return HHLB_OK;
}

// Kernel launch arguments shared by the aux kernels.
struct AuxArgs {
  const hhlb::DevTables *tbs;
  const int32_t *ch_class;
  const hhlb::DevChannel *chans;
  const int32_t *ch_V;
  int n_ch, scaled;
};

AuxArgs aux(const hhlb_solver *s) {
  return AuxArgs{(const hhlb::DevTables *)(s->ws + s->o_tables), (const int32_t *)(s->ws + s->o_chclass),
                 (const hhlb::DevChannel *)(s->ws + s->o_chans), (const int32_t *)(s->ws + s->o_V),
                 (int)s->ch.size(), s->mixed() ? 1 : 0};
}

dim3 state_grid(const hhlb_solver *s) {
  int64_t maxlen = 0;
  for (size_t c = 0; c + 1 < s->off.size(); ++c) maxlen = std::max<int64_t>(maxlen, s->off[c + 1] - s->off[c]);
  return dim3((unsigned)std::min<int64_t>((maxlen + 255) / 256, 4096), (unsigned)s->ch.size());
}

template <typename S>
void launch_convert(const hhlb_solver *s, int to_state, double *pop, void *st, int16_t *lo) {
  const AuxArgs a = aux(s);
  hipLaunchKernelGGL(convert_kernel<S>, state_grid(s), dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans, a.ch_V,
                     a.n_ch, a.scaled, to_state, pop, (S *)st, lo);
}

// pop (FP64, boundary layout) <-> stored state of function fn (0 = f, 1 = chi)
void convert(const hhlb_solver *s, int to_state, double *pop, int fn) {
  void *st = fn == 0 ? s->fA() : s->cA();
  if (s->mixed()) launch_convert<float>(s, to_state, pop, st, fn == 0 ? s->lA() : s->lcA());
  else launch_convert<double>(s, to_state, pop, st, nullptr);
}

}  // namespace

extern "C" {

const char *hhlb_last_error(void) { return g_err.c_str(); }

hhlb_status hhlb_nodes(int32_t quad, int32_t Q, double p0, double *p_out, double *w_out) {
  if (!p_out || !w_out) return fail(HHLB_E_ARG, "null output pointer");
  try {
    hhlb::Rule r;
    std::string err;
    int st = hhlb::build_rule(quad, Q, p0, r, err);
    if (st) return fail(st, err);
    std::memcpy(p_out, r.p.data(), sizeof(double) * r.V);
    std::memcpy(w_out, r.wv.data(), sizeof(double) * r.V);
  } catch (...) {
    return fail(HHLB_E_NOMEM, "allocation failed");
  }
  return HHLB_OK;
}

hhlb_status hhlb_force_matrix(int32_t quad, int32_t Q, double p0, double *K_out) {
  if (!K_out) return fail(HHLB_E_ARG, "null output pointer");
  try {
    hhlb::Rule r;
    std::string err;
    int st = hhlb::build_rule(quad, Q, p0, r, err);
    if (st) return fail(st, err);
    std::memcpy(K_out, r.K.data(), sizeof(double) * r.V * r.V);
  } catch (...) {
    return fail(HHLB_E_NOMEM, "allocation failed");
  }
  return HHLB_OK;
}

hhlb_status hhlb_equilibrium(int32_t quad, int32_t Q, int32_t N, double p0, double n, double u,
                             double T, double *feq_out) {
  if (!feq_out) return fail(HHLB_E_ARG, "null output pointer");
  if (N < 0 || N >= Q) return fail(HHLB_E_ARG, "N must satisfy 0 <= N < Q");
  if (!(T > 0) || !std::isfinite(u) || !std::isfinite(n)) return fail(HHLB_E_ARG, "need T > 0, finite n, u");
  try {
    hhlb::Rule r;
    std::string err;
    int st = hhlb::build_rule(quad, Q, p0, r, err);
    if (st) return fail(st, err);
    hhlb::equilibrium(r, N, u, T, feq_out);
    for (int k = 0; k < r.V; ++k) feq_out[k] *= n;
  } catch (...) {
    return fail(HHLB_E_NOMEM, "allocation failed");
  }
  return HHLB_OK;
}

hhlb_status hhlb_create(const hhlb_channel *channels, int32_t n_ch, int32_t precision,
                        void *hip_stream, hhlb_solver **out) {
  if (!channels || !out || n_ch < 1) return fail(HHLB_E_ARG, "need channels, n_ch >= 1 and out");
  if (precision < HHLB_FP64 || precision > HHLB_MIXED_F16) return fail(HHLB_E_ARG, "unknown precision");
  for (int c = 0; c < n_ch; ++c) {
    hhlb_status st = check_channel(channels[c], c);
    if (st) return st;
    if (precision != HHLB_FP64 && channels[c].quad != HHLB_HALF_HERMITE)
      return fail(HHLB_E_UNSUPPORTED, "channel " + std::to_string(c) +
                                          ": the mixed-precision forms cover the half-range Hermite model only");
  }
  std::unique_ptr<hhlb_solver> s;
  try {
    s.reset(new hhlb_solver());
    s->stream = (hipStream_t)hip_stream;
    s->precision = precision;
    s->esize = precision == HHLB_FP64 ? sizeof(double) : sizeof(float);
    s->ch.assign(channels, channels + n_ch);
    std::map<std::tuple<int, int, int, int, int, double>, int> cls;
    s->off.assign(n_ch + 1, 0);
    s->cell_off.assign(n_ch, 0);
    for (int c = 0; c < n_ch; ++c) {
      const hhlb_channel &h = channels[c];
      int N = h.N < 0 ? std::min(20, h.Q - 1) : h.N;
      auto key = std::make_tuple(h.quad, h.Q, N, h.adv, h.transverse_dof, h.p0);
      auto it = cls.find(key);
      int id;
      if (it == cls.end()) {
        ModelClass mc;
        mc.quad = h.quad; mc.Q = h.Q; mc.N = N; mc.adv = h.adv; mc.Dt = h.transverse_dof; mc.p0 = h.p0;
        std::string err;
        const bool large = h.Q > hhlb::kQmaxDev;
        if (large) {
          // the node-parallel stage: FP64, N <= 20, half-range Gauss-Hermite
          // with Q <= 256 per half or full-range Gauss-Hermite with Q <= 512
          const bool ok_kind = (h.quad == HHLB_HALF_HERMITE && h.Q <= hhlb::kQmaxLarge) ||
                               (h.quad == HHLB_FULL_HERMITE && h.Q <= 2 * hhlb::kQmaxLarge);
          if (!ok_kind || precision != HHLB_FP64 || N > hhlb::kNmaxLarge)
            return fail(HHLB_E_UNSUPPORTED, "channel " + std::to_string(c) + ": Q > " +
                                                std::to_string(hhlb::kQmaxDev) +
                                                " runs in FP64 with N <= 20: the half-range Hermite model with Q <= " +
                                                std::to_string(hhlb::kQmaxLarge) +
                                                " or the full-range Hermite model with Q <= " +
                                                std::to_string(2 * hhlb::kQmaxLarge));
        }
        int st = hhlb::build_rule(h.quad, h.Q, h.p0, mc.rule, err);
        if (st) return fail(st, "channel " + std::to_string(c) + ": " + err);
        const int nf = h.transverse_dof > 0 ? 2 : 1;
        if (large) {
          mc.large = true;
          s->any_large = true;
          st = make_large_tables(h, N, mc.rule, mc.dev, mc.lblob);
          if (st) return st;
        } else {
          // both half-range kinds run the half-range kernels (tables differ)
          const int kq = hhlb::half_range(h.quad) ? HHLB_HALF_HERMITE : HHLB_FULL_HERMITE;
          auto lk = launchers().find({kq, h.Q, nf, h.adv, precision, 2});
          if (lk == launchers().end())
            return fail(HHLB_E_UNSUPPORTED, "channel " + std::to_string(c) + ": no kernel for quad=" +
                                                std::to_string(h.quad) + " Q=" + std::to_string(h.Q));
          mc.launch = lk->second;
          auto lk4 = launchers().find({kq, h.Q, nf, h.adv, precision, 4});
          if (lk4 != launchers().end()) mc.launch4 = lk4->second;
          auto lkf = launchers().find({kq, h.Q, nf, h.adv, precision, 1});
          if (lkf != launchers().end() && kq == HHLB_HALF_HERMITE) mc.fused = lkf->second;
          st = cached_tables(h, N, precision, mc.rule, mc.dev);
          if (st) return st;
        }
        id = (int)s->classes.size();
        s->classes.push_back(std::move(mc));
        cls[key] = id;
      } else {
        id = it->second;
      }
      s->ch_class.push_back(id);
      const ModelClass &mc = s->classes[id];
      const int V = mc.rule.V;
      s->Vs.push_back(V);
      s->off[c + 1] = s->off[c] + (int64_t)V * h.Nx;
      s->cell_off[c] = (int32_t)s->total_cells;
      s->total_cells += h.Nx;
      if (h.transverse_dof > 0) s->has_chi = true;
      else s->any_dt0 = true;
    }
    s->total_state = s->off[n_ch];
    if (s->total_cells > INT32_MAX / 2) return fail(HHLB_E_UNSUPPORTED, "too many cells");
    // per channel: grid, dt, wall equilibria, denominators, windows
    for (int c = 0; c < n_ch; ++c) {
      const hhlb_channel &h = channels[c];
      ModelClass &mc = s->classes[s->ch_class[c]];
      const hhlb::Rule &r = mc.rule;
      std::vector<double> dx;
      make_grid(h, dx);
      double dxmin = dx[0];
      for (double d : dx) dxmin = std::min(dxmin, d);
      for (double d : dx) { s->dx.push_back(d); s->inv_dx.push_back(1.0 / d); }
      double vmax = 0;
      for (double p : r.p) vmax = std::max(vmax, std::fabs(p));
      double dt = h.dt;
      if (dt < 0) {
        dt = -dt * dxmin / vmax;
        if (std::isfinite(h.Kn)) dt = std::min(dt, 0.5 * h.Kn);
      }
      s->dts.push_back(dt);
      std::vector<double> gL(r.V), gR(r.V);
      hhlb::equilibrium(r, mc.N, 0.0L, (long double)h.T_left, gL.data());
      hhlb::equilibrium(r, mc.N, 0.0L, (long double)h.T_right, gR.data());
      long double DL = 0, DR = 0;
      for (int k = 0; k < r.V; ++k) {
        // the mixed form's FP32 advection moves the emergent populations with
        // the FP32-rounded velocities
        const long double pk = s->mixed() ? (long double)(float)r.p[k] : (long double)r.p[k];
        if (k < r.H) DL += pk * gL[k];
        else DR += pk * gR[k];
      }
      hhlb::DevChannel d;
      std::memset(&d, 0, sizeof(d));
      d.off = s->off[c];
      d.Nx = h.Nx;
      d.cell_off = s->cell_off[c];
      d.gw_off = (int32_t)s->gw.size();
      for (double v : gL) s->gw.push_back(v);
      for (double v : gR) s->gw.push_back(v);
      d.g = h.g;
      d.inv_Kn = std::isfinite(h.Kn) ? 1.0 / h.Kn : 0.0;
      d.dt = dt;
      d.TL = h.T_left;
      d.TR = h.T_right;
      d.inv_DL = (double)(1.0L / DL);
      d.inv_DR = (double)(1.0L / DR);
      d.half_Dt = 0.5 * h.transverse_dof;
      d.inv_1pDt = 1.0 / (1.0 + h.transverse_dof);
      s->dch.push_back(d);
      for (int i0 = 0; i0 < h.Nx; i0 += hhlb::kWin) mc.windows.push_back({c, i0});
      if (mc.fused) fused_windows(c, h.Nx, mc.fwindows);
    }
    // classes that can share a launch per stage: FP64 half-range classes of
    // the per-stage window kernels, grouped by functions and scheme
    s->class_group.assign(s->classes.size(), -1);
    if (precision == HHLB_FP64) {
      std::map<std::pair<int, int>, std::vector<size_t>> by;
      for (size_t ci = 0; ci < s->classes.size(); ++ci) {
        const ModelClass &mc = s->classes[ci];
        if (!mc.large && hhlb::half_range(mc.quad) && mc.launch) by[{mc.Dt > 0 ? 2 : 1, mc.adv}].push_back(ci);
      }
      for (auto &kv : by) {
        if (kv.second.size() < 2) continue;
        int qmax = 0;
        for (size_t ci : kv.second) qmax = std::max(qmax, s->classes[ci].Q);
        const int qtop = qmax <= 8 ? 8 : (qmax <= 12 ? 12 : 16);
        auto lk = launchers().find({HHLB_HALF_HERMITE, qtop, kv.first.first, kv.first.second, HHLB_FP64, 3});
        if (lk == launchers().end()) continue;
        hhlb_solver::MergeGroup g;
        g.launch = lk->second;
        g.qtop = qtop;
        g.members = kv.second;
        for (size_t ci : kv.second) {
          const ModelClass &mc = s->classes[ci];
          for (const auto &w : mc.windows) g.wins.push_back({w.ch, w.i0, (int32_t)ci, (int32_t)mc.Q});
          s->class_group[ci] = (int)s->groups.size();
        }
        s->groups.push_back(std::move(g));
      }
    }
    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r0 = o; o = align256(o + bytes); return r0; };
    s->o_tables = take(sizeof(hhlb::DevTables) * s->classes.size());
    s->o_chans = take(sizeof(hhlb::DevChannel) * n_ch);
    s->o_chclass = take(sizeof(int32_t) * n_ch);
    s->o_V = take(sizeof(int32_t) * n_ch);
    for (auto &mc : s->classes) {
      mc.win_off = take(sizeof(hhlb::DevWindow) * mc.windows.size());
      mc.fwin_off = take(sizeof(hhlb::DevFusedWindow) * mc.fwindows.size());
    }
    for (auto &g : s->groups) g.win_off = take(sizeof(hhlb::DevClassWindow) * g.wins.size());
    s->o_dx = take(sizeof(double) * s->total_cells);
    s->o_invdx = take(sizeof(double) * s->total_cells);
    s->o_gw = take(sizeof(double) * s->gw.size());
    s->o_nwall = take(sizeof(double) * 2 * n_ch);
    int64_t feq_total = 0;
    for (int c = 0; c < n_ch; ++c) feq_total += s->Vs[c];
    s->o_feq = take(sizeof(double) * feq_total);
    s->o_feqoff = take(sizeof(int32_t) * n_ch);
    s->o_flag = take(sizeof(int32_t));
    s->o_wide = take(sizeof(unsigned long long));
    for (auto &mc : s->classes)
      if (mc.large) mc.lbl_off = take(mc.lblob.size());
    if (s->any_large) {
      s->o_cell = take(sizeof(double) * hhlb::kCellStride * s->total_cells);
      s->o_lnw = take(sizeof(double) * 2 * n_ch);
    }
    s->o_state = o;
    // per function: FP64 form 3 copies of 8 bytes; mixed form 4 copies of
    // 4 bytes (hi x 2, B, C) and 2 copies of 2 bytes (lo x 2)
    const int nfun = s->has_chi ? 2 : 1;
    for (int j = 0; j < nfun * (s->mixed() ? 4 : 3); ++j) take(s->esize * s->total_state);
    if (s->mixed())
      for (int j = 0; j < nfun * 2; ++j) take(sizeof(int16_t) * s->total_state);
    s->bytes = o;
  } catch (...) {
    return fail(HHLB_E_NOMEM, "host allocation failed");
  }
  *out = s.release();
  return HHLB_OK;
}

hhlb_status hhlb_workspace_bytes(const hhlb_solver *s, size_t *bytes) {
  if (!s || !bytes) return fail(HHLB_E_ARG, "null argument");
  *bytes = s->bytes;
  return HHLB_OK;
}

hhlb_status hhlb_bind_workspace(hhlb_solver *s, void *dev_ptr) {
  if (!s || !dev_ptr) return fail(HHLB_E_ARG, "null argument");
  if (((uintptr_t)dev_ptr) & 255) return fail(HHLB_E_ARG, "workspace must be 256-byte aligned");
  char *ws = (char *)dev_ptr;
  const int n_ch = (int)s->ch.size();
  std::vector<hhlb::DevTables> tabs;
  for (auto &mc : s->classes) tabs.push_back(mc.dev);
  std::vector<int32_t> feq_off(n_ch);
  int64_t acc = 0;
  for (int c = 0; c < n_ch; ++c) { feq_off[c] = (int32_t)acc; acc += s->Vs[c]; }
  HIP_TRY(hipMemcpyAsync(ws + s->o_tables, tabs.data(), sizeof(hhlb::DevTables) * tabs.size(),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(ws + s->o_chans, s->dch.data(), sizeof(hhlb::DevChannel) * n_ch,
                         hipMemcpyHostToDevice, s->stream));
  std::vector<int32_t> chclass(s->ch_class.begin(), s->ch_class.end());
  HIP_TRY(hipMemcpyAsync(ws + s->o_chclass, chclass.data(), sizeof(int32_t) * n_ch,
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(ws + s->o_V, s->Vs.data(), sizeof(int32_t) * n_ch, hipMemcpyHostToDevice,
                         s->stream));
  for (auto &mc : s->classes) {
    HIP_TRY(hipMemcpyAsync(ws + mc.win_off, mc.windows.data(), sizeof(hhlb::DevWindow) * mc.windows.size(),
                           hipMemcpyHostToDevice, s->stream));
    if (!mc.fwindows.empty())
      HIP_TRY(hipMemcpyAsync(ws + mc.fwin_off, mc.fwindows.data(),
                             sizeof(hhlb::DevFusedWindow) * mc.fwindows.size(), hipMemcpyHostToDevice, s->stream));
    if (mc.large)
      HIP_TRY(hipMemcpyAsync(ws + mc.lbl_off, mc.lblob.data(), mc.lblob.size(), hipMemcpyHostToDevice, s->stream));
  }
  for (auto &g : s->groups)
    HIP_TRY(hipMemcpyAsync(ws + g.win_off, g.wins.data(), sizeof(hhlb::DevClassWindow) * g.wins.size(),
                           hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(ws + s->o_dx, s->dx.data(), sizeof(double) * s->total_cells,
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(ws + s->o_invdx, s->inv_dx.data(), sizeof(double) * s->total_cells,
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(ws + s->o_gw, s->gw.data(), sizeof(double) * s->gw.size(),
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(ws + s->o_feqoff, feq_off.data(), sizeof(int32_t) * n_ch,
                         hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemsetAsync(ws + s->o_nwall, 0, sizeof(double) * 2 * n_ch, s->stream));
  HIP_TRY(hipMemsetAsync(ws + s->o_flag, 0, sizeof(int32_t), s->stream));
  HIP_TRY(hipMemsetAsync(ws + s->o_wide, 0, sizeof(unsigned long long), s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->ws = ws;
  s->flag_pending = false;
  s->drop_graphs();
  s->par = 0;
  char *st = ws + s->o_state;
  const size_t stride = align256(s->esize * s->total_state);
  auto next = [&](size_t bytes) { char *p = st; st += align256(bytes); return (void *)p; };
  const size_t vb = s->esize * s->total_state, lb = sizeof(int16_t) * s->total_state;
  // FP64: y^n ping-pongs between A and B (every step writes the other copy)
  // and C holds the second stage; mixed: (hi, lo) ping-pong, B and C the
  // stage increments
  s->hiF[0] = next(vb); s->fB = next(vb); s->fC = next(vb);
  s->hiF[1] = s->mixed() ? next(vb) : s->fB;
  if (s->has_chi) {
    s->hiC[0] = next(vb); s->cB = next(vb); s->cC = next(vb);
    s->hiC[1] = s->mixed() ? next(vb) : s->cB;
  } else {
    s->hiC[0] = s->hiC[1] = s->cB = s->cC = nullptr;
  }
  if (s->mixed()) {
    s->loF[0] = (int16_t *)next(lb); s->loF[1] = (int16_t *)next(lb);
    if (s->has_chi) { s->loC[0] = (int16_t *)next(lb); s->loC[1] = (int16_t *)next(lb); }
  }
  (void)stride;
  return HHLB_OK;
}

hhlb_status hhlb_state_offsets(const hhlb_solver *s, int64_t *off) {
  if (!s || !off) return fail(HHLB_E_ARG, "null argument");
  std::memcpy(off, s->off.data(), sizeof(int64_t) * s->off.size());
  return HHLB_OK;
}

hhlb_status hhlb_time_steps(const hhlb_solver *s, double *dt_out) {
  if (!s || !dt_out) return fail(HHLB_E_ARG, "null argument");
  std::memcpy(dt_out, s->dts.data(), sizeof(double) * s->dts.size());
  return HHLB_OK;
}

hhlb_status hhlb_set_state(hhlb_solver *s, const double *f_dev, const double *chi_dev) {
  if (!s || !f_dev) return fail(HHLB_E_ARG, "null argument");
  if (!s->ws) return fail(HHLB_E_STATE, "no workspace bound");
  if (s->has_chi && !chi_dev) return fail(HHLB_E_ARG, "chi is required when a channel has Dt > 0");
  if (!s->mixed()) {
    HIP_TRY(hipMemcpyAsync(s->fA(), f_dev, sizeof(double) * s->total_state, hipMemcpyDeviceToDevice, s->stream));
    if (s->has_chi)
      HIP_TRY(hipMemcpyAsync(s->cA(), chi_dev, sizeof(double) * s->total_state, hipMemcpyDeviceToDevice, s->stream));
  } else {
    convert(s, 1, const_cast<double *>(f_dev), 0);
    if (s->has_chi) convert(s, 1, const_cast<double *>(chi_dev), 1);
    HIP_TRY(hipGetLastError());
  }
  return HHLB_OK;
}

hhlb_status hhlb_get_state(const hhlb_solver *s, double *f_dev, double *chi_dev) {
  if (!s || !f_dev) return fail(HHLB_E_ARG, "null argument");
  if (!s->ws) return fail(HHLB_E_STATE, "no workspace bound");
  if (!s->mixed()) {
    HIP_TRY(hipMemcpyAsync(f_dev, s->fA(), sizeof(double) * s->total_state, hipMemcpyDeviceToDevice, s->stream));
    if (chi_dev && s->has_chi)
      HIP_TRY(hipMemcpyAsync(chi_dev, s->cA(), sizeof(double) * s->total_state, hipMemcpyDeviceToDevice, s->stream));
  } else {
    convert(s, 0, f_dev, 0);
    if (chi_dev && s->has_chi) convert(s, 0, chi_dev, 1);
    HIP_TRY(hipGetLastError());
  }
  if (chi_dev && !s->has_chi) HIP_TRY(hipMemsetAsync(chi_dev, 0, sizeof(double) * s->total_state, s->stream));
  if (chi_dev && s->has_chi && s->any_dt0) {
    const AuxArgs a = aux(s);
    hipLaunchKernelGGL(zero_chi_kernel, state_grid(s), dim3(256), 0, s->stream, a.chans, a.ch_V, a.n_ch, chi_dev);
    HIP_TRY(hipGetLastError());
  }
  return HHLB_OK;
}

hhlb_status hhlb_init_equilibrium(hhlb_solver *s, double n0, double u0, double T0) {
  if (!s) return fail(HHLB_E_ARG, "null solver");
  if (!s->ws) return fail(HHLB_E_STATE, "no workspace bound");
  if (!(T0 > 0) || !std::isfinite(n0) || !std::isfinite(u0)) return fail(HHLB_E_ARG, "need T0 > 0, finite n0, u0");
  const int n_ch = (int)s->ch.size();
  std::vector<double> feq;
  for (int c = 0; c < n_ch; ++c) {
    const ModelClass &mc = s->classes[s->ch_class[c]];
    std::vector<double> g(mc.rule.V);
    hhlb::equilibrium(mc.rule, mc.N, u0, T0, g.data());
    for (double v : g) feq.push_back(n0 * v);
  }
  HIP_TRY(hipMemcpyAsync(s->ws + s->o_feq, feq.data(), sizeof(double) * feq.size(), hipMemcpyHostToDevice,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const AuxArgs a = aux(s);
  const double *fq = (const double *)(s->ws + s->o_feq);
  const int32_t *fo = (const int32_t *)(s->ws + s->o_feqoff);
  if (s->mixed())
    hipLaunchKernelGGL(fill_kernel<float>, state_grid(s), dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans,
                       a.ch_V, a.n_ch, a.scaled, fq, fo, T0, (float *)s->fA(), s->lA(), (float *)s->cA(),
                       s->lcA());
  else
    hipLaunchKernelGGL(fill_kernel<double>, state_grid(s), dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans,
                       a.ch_V, a.n_ch, a.scaled, fq, fo, T0, (double *)s->fA(), (int16_t *)nullptr,
                       (double *)s->cA(), (int16_t *)nullptr);
  HIP_TRY(hipGetLastError());
  return HHLB_OK;
}

}  // extern "C"

namespace {

// Enqueue one RK stage of model class ci.
void enqueue_class_stage(hhlb_solver *s, size_t ci, int stage, const void *inf, const void *inc, void *outf,
                         void *outc, double a_base, double b_stage, hipStream_t stream,
                         const int16_t *lo_in_f = nullptr, const int16_t *lo_in_c = nullptr,
                         int16_t *lo_out_f = nullptr, int16_t *lo_out_c = nullptr) {
  ModelClass &mc = s->classes[ci];
  if (mc.large) {
    hhlb::LargeArgs la;
    la.tl = (const hhlb::DevLarge *)(s->ws + mc.lbl_off);
    la.KinT = (const double *)(s->ws + mc.lbl_off + sizeof(hhlb::DevLarge));
    const size_t rows = mc.quad == HHLB_FULL_HERMITE ? (size_t)mc.rule.V : (size_t)mc.rule.H;
    la.HWs = la.KinT + rows * rows;
    la.p = ((const hhlb::DevTables *)(s->ws + s->o_tables) + ci)->p;
    la.chans = (const hhlb::DevChannel *)(s->ws + s->o_chans);
    la.wins = (const hhlb::DevWindow *)(s->ws + mc.win_off);
    la.nwin = (int32_t)mc.windows.size();
    la.stage = stage;
    la.inv_dx = (const double *)(s->ws + s->o_invdx);
    la.gw = (const double *)(s->ws + s->o_gw);
    la.in_f = (const double *)inf; la.in_c = (const double *)inc;
    la.base_f = (const double *)s->fA(); la.base_c = (const double *)s->cA();
    la.out_f = (double *)outf; la.out_c = (double *)outc;
    la.a_base = a_base;
    la.b_stage = b_stage;
    la.cell = (double *)(s->ws + s->o_cell);
    la.lnw = (double *)(s->ws + s->o_lnw);
    la.nwall = (double *)(s->ws + s->o_nwall);
    la.wide = (unsigned long long *)(s->ws + s->o_wide);
    la.nfun = mc.Dt > 0 ? 2 : 1;
    la.xcd_map = s->tuning.xcd_map;
    hhlb::launch_large(la, mc.adv, mc.rule.H, stream);
    return;
  }
  hhlb::StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.tb = (const hhlb::DevTables *)(s->ws + s->o_tables) + ci;
  a.chans = (const hhlb::DevChannel *)(s->ws + s->o_chans);
  a.wins = (const hhlb::DevWindow *)(s->ws + mc.win_off);
  a.nwin = (int32_t)mc.windows.size();
  a.stage = stage;
  a.xcd_map = s->tuning.xcd_map;
  a.inv_dx = (const double *)(s->ws + s->o_invdx);
  a.gw = (const double *)(s->ws + s->o_gw);
  a.in_f = inf; a.in_c = inc;
  a.base_f = s->fA(); a.base_c = s->cA();
  a.out_f = outf; a.out_c = outc;
  a.a_base = a_base;
  a.b_stage = b_stage;
  a.nwall = (double *)(s->ws + s->o_nwall);
  a.wide = (unsigned long long *)(s->ws + s->o_wide);
  a.lo_in_f = lo_in_f; a.lo_in_c = lo_in_c;
  a.lo_out_f = lo_out_f; a.lo_out_c = lo_out_c;
  (s->tuning.waves_per_window == 4 && mc.launch4 ? mc.launch4 : mc.launch)(a, stream);
}

// One whole RK-3 step of model class ci in one launch (FP64 half-range
// classes with a fused-step kernel): y^n from (inf, inc), y^{n+1} to (outf, outc).
void enqueue_class_fused(hhlb_solver *s, size_t ci, const void *inf, const void *inc, void *outf, void *outc,
                         hipStream_t stream) {
  ModelClass &mc = s->classes[ci];
  hhlb::StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.tb = (const hhlb::DevTables *)(s->ws + s->o_tables) + ci;
  a.chans = (const hhlb::DevChannel *)(s->ws + s->o_chans);
  a.wins = (const hhlb::DevWindow *)(s->ws + mc.fwin_off);   // DevFusedWindow records
  a.nwin = (int32_t)mc.fwindows.size();
  a.stage = 2;
  a.xcd_map = s->tuning.xcd_map;
  a.inv_dx = (const double *)(s->ws + s->o_invdx);
  a.gw = (const double *)(s->ws + s->o_gw);
  a.in_f = inf; a.in_c = inc;
  a.out_f = outf; a.out_c = outc;
  a.nwall = (double *)(s->ws + s->o_nwall);
  a.wide = (unsigned long long *)(s->ws + s->o_wide);
  mc.fused(a, stream);
}

// One RK stage of the classes of merge group gi in one launch (FP64).
void enqueue_group_stage(hhlb_solver *s, size_t gi, int stage, const void *inf, const void *inc, void *outf,
                         void *outc, double a_base, double b_stage, hipStream_t stream) {
  const auto &g = s->groups[gi];
  hhlb::StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.tb = (const hhlb::DevTables *)(s->ws + s->o_tables);   // the classes' tables, indexed by class
  a.chans = (const hhlb::DevChannel *)(s->ws + s->o_chans);
  a.wins = (const hhlb::DevWindow *)(s->ws + g.win_off);    // DevClassWindow records
  a.nwin = (int32_t)g.wins.size();
  a.nblocks = s->tuning.merge_classes == 2 ? -1 : 0;
  a.stage = stage;
  a.xcd_map = s->tuning.xcd_map;
  a.inv_dx = (const double *)(s->ws + s->o_invdx);
  a.gw = (const double *)(s->ws + s->o_gw);
  a.in_f = inf; a.in_c = inc;
  a.base_f = s->fA(); a.base_c = s->cA();
  a.out_f = outf; a.out_c = outc;
  a.a_base = a_base;
  a.b_stage = b_stage;
  a.nwall = (double *)(s->ws + s->o_nwall);
  a.wide = (unsigned long long *)(s->ws + s->o_wide);
  g.launch(a, stream);
}

// One RK-3 step of merge group gi (FP64, the per-stage buffers of
// enqueue_class_steps) from the solver's current parity (left unchanged).
void enqueue_group_step(hhlb_solver *s, size_t gi, hipStream_t stream) {
  const int p = s->par, q = p ^ 1;
  enqueue_group_stage(s, gi, 0, s->hiF[p], s->hiC[p], s->hiF[q], s->hiC[q], 0.0, 1.0, stream);
  enqueue_group_stage(s, gi, 1, s->hiF[q], s->hiC[q], s->fC, s->cC, 0.75, 0.25, stream);
  enqueue_group_stage(s, gi, 2, s->fC, s->cC, s->hiF[q], s->hiC[q], 1.0 / 3.0, 2.0 / 3.0, stream);
}

// One RK stage of every class on one stream.
void enqueue_stage(hhlb_solver *s, int stage, const void *inf, const void *inc, void *outf, void *outc,
                   double a_base, double b_stage, hipStream_t stream) {
  for (size_t ci = 0; ci < s->classes.size(); ++ci)
    enqueue_class_stage(s, ci, stage, inf, inc, outf, outc, a_base, b_stage, stream);
}

// n_steps RK-3 steps (Eq. rk3) of class ci on one stream, starting from the
// solver's current state parity (left unchanged).
//  FP64, y^n in copy p of the pair (A, B), q = 1 - p: stage 1 p -> q,
//        stage 2 (q, p) -> C, stage 3 (C, p) -> q (y1 in q is dead by then);
//        or, with step fusion, one launch p -> q.
//  Mixed: stage 1 hi -> d1 (B), stage 2 (hi, d1) -> d2 (C), stage 3
//        (hi, lo, d2) -> the other (hi, lo) copy.
// Every step moves y^n to the other copy: the parity flips.
void enqueue_class_steps(hhlb_solver *s, size_t ci, int64_t n_steps, hipStream_t stream) {
  const int par0 = s->par;
  for (int64_t step = 0; step < n_steps; ++step) {
    const int p = s->par, q = p ^ 1;
    if (!s->mixed()) {
      if (s->tuning.step_fusion && s->classes[ci].fused) {
        enqueue_class_fused(s, ci, s->hiF[p], s->hiC[p], s->hiF[q], s->hiC[q], stream);
      } else {
        enqueue_class_stage(s, ci, 0, s->hiF[p], s->hiC[p], s->hiF[q], s->hiC[q], 0.0, 1.0, stream);
        enqueue_class_stage(s, ci, 1, s->hiF[q], s->hiC[q], s->fC, s->cC, 0.75, 0.25, stream);
        enqueue_class_stage(s, ci, 2, s->fC, s->cC, s->hiF[q], s->hiC[q], 1.0 / 3.0, 2.0 / 3.0, stream);
      }
      s->par = q;
    } else {
      enqueue_class_stage(s, ci, 0, nullptr, nullptr, s->fB, s->cB, 0.0, 1.0, stream);
      enqueue_class_stage(s, ci, 1, s->fB, s->cB, s->fC, s->cC, 0.75, 0.25, stream);
      enqueue_class_stage(s, ci, 2, s->fC, s->cC, s->hiF[q], s->hiC[q], 1.0 / 3.0, 2.0 / 3.0, stream,
                          s->loF[p], s->loC[p], s->loF[q], s->loC[q]);
      s->par = q;
    }
  }
  s->par = par0;
}

// n_steps steps of every class.  With one stream the classes run one after
// the other within each step; with class streams (direct launches only) each
// class runs its whole step sequence on a stream of its own (classes touch
// disjoint channels, so nothing orders them), forked from and joined back
// into `stream` by events.  Graph capture always takes the one-stream form,
// so the fork/join events are never part of a captured graph.  The state
// parity advances by n_steps.
hhlb_status enqueue_steps(hhlb_solver *s, int64_t n_steps, hipStream_t stream, bool capturing = false) {
  const size_t nc = s->classes.size();
  if (capturing || !s->tuning.class_streams || nc < 2) {
    const int par0 = s->par;
    const bool merge = s->tuning.merge_classes != 0;
    for (int64_t step = 0; step < n_steps; ++step) {
      if (merge)
        for (size_t gi = 0; gi < s->groups.size(); ++gi) enqueue_group_step(s, gi, stream);
      for (size_t ci = 0; ci < nc; ++ci)
        if (!merge || s->class_group[ci] < 0) enqueue_class_steps(s, ci, 1, stream);
      s->par ^= 1;
    }
    (void)par0;
    return HHLB_OK;
  }
  // one stream and one join event per class, created and kept in pairs
  while (s->cstreams.size() < nc) {
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(st);
      return fail(HHLB_E_HIP, std::string("hipEventCreateWithFlags: ") + hipGetErrorString(e));
    }
    s->cstreams.push_back(st);
    s->cjoin.push_back(ev);
  }
  if (!s->cfork) HIP_TRY(hipEventCreateWithFlags(&s->cfork, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(s->cfork, stream));
  for (size_t ci = 0; ci < nc; ++ci) {
    HIP_TRY(hipStreamWaitEvent(s->cstreams[ci], s->cfork, 0));
    enqueue_class_steps(s, ci, n_steps, s->cstreams[ci]);
    HIP_TRY(hipEventRecord(s->cjoin[ci], s->cstreams[ci]));
  }
  for (size_t ci = 0; ci < nc; ++ci) HIP_TRY(hipStreamWaitEvent(stream, s->cjoin[ci], 0));
  if (n_steps & 1) s->par ^= 1;
  return HHLB_OK;
}

// Capture `steps` steps starting from the current parity (the parity the
// capture advanced is restored: nothing ran yet).
hhlb_status make_graph(hhlb_solver *s, int64_t steps, hipGraphExec_t *out) {
  hipGraph_t g = nullptr;
  const int par0 = s->par;
  HIP_TRY(hipStreamBeginCapture(s->gstream, hipStreamCaptureModeThreadLocal));
  hhlb_status st = enqueue_steps(s, steps, s->gstream, true);
  s->par = par0;
  hipError_t e = hipStreamEndCapture(s->gstream, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(HHLB_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(HHLB_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return HHLB_OK;
}

hhlb_status run_steps(hhlb_solver *s, int64_t n_steps) {
  if (s->tuning.graph_steps <= 0) {
    hhlb_status st = enqueue_steps(s, n_steps, s->stream);
    if (st) return st;
    HIP_TRY(hipGetLastError());
    return HHLB_OK;
  }
  // graph replay on an internal stream, ordered after the caller's stream
  // and before whatever the caller enqueues next
  if (!s->ev_in) HIP_TRY(hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
  if (!s->ev_out) HIP_TRY(hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
  if (!s->gstream) HIP_TRY(hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking));
  const int64_t K = s->tuning.graph_steps;
  const int64_t full = n_steps / K, rest = n_steps % K;
  // every step flips the state parity: one graph per starting parity, all
  // captured before the first launch
  for (int p = 0; p < 2; ++p) {
    const int par0 = s->par;
    s->par = p;
    hhlb_status st = HHLB_OK;
    if (full && !s->gexec_k[p]) st = make_graph(s, K, &s->gexec_k[p]);
    if (!st && rest && !s->gexec_1[p]) st = make_graph(s, 1, &s->gexec_1[p]);
    s->par = par0;
    if (st) return st;
  }
  HIP_TRY(hipEventRecord(s->ev_in, s->stream));
  HIP_TRY(hipStreamWaitEvent(s->gstream, s->ev_in, 0));
  for (int64_t r = 0; r < full; ++r) {
    HIP_TRY(hipGraphLaunch(s->gexec_k[s->par], s->gstream));
    if (K & 1) s->par ^= 1;
  }
  for (int64_t r = 0; r < rest; ++r) {
    HIP_TRY(hipGraphLaunch(s->gexec_1[s->par], s->gstream));
    s->par ^= 1;
  }
  HIP_TRY(hipEventRecord(s->ev_out, s->gstream));
  HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_out, 0));
  return HHLB_OK;
}

hhlb_status check_flag(hhlb_solver *s) {
  if (s->flag_pending) {
    // the non-finite count of the last hhlb_diagnostics
    HIP_TRY(hipEventSynchronize(s->ev_flag));
    s->flag_pending = false;
    if (*s->flag_host > 0)
      return fail(HHLB_E_NUMERIC, std::to_string(*s->flag_host) + " non-finite populations in the state");
  }
  return HHLB_OK;
}

}  // namespace

extern "C" hhlb_status hhlb_step(hhlb_solver *s, int64_t n_steps) {
  if (!s) return fail(HHLB_E_ARG, "null solver");
  if (n_steps < 0) return fail(HHLB_E_ARG, "n_steps must be >= 0");
  if (!s->ws) return fail(HHLB_E_STATE, "no workspace bound");
  hhlb_status st = check_flag(s);
  if (st) return st;
  if (n_steps == 0) return HHLB_OK;
  return run_steps(s, n_steps);
}

extern "C" hhlb_status hhlb_set_graph_steps(hhlb_solver *s, int32_t steps_per_graph) {
  if (!s || steps_per_graph < 0) return fail(HHLB_E_ARG, "need a solver and steps_per_graph >= 0");
  s->drop_graphs();
  s->tuning.graph_steps = steps_per_graph;
  return HHLB_OK;
}

extern "C" hhlb_status hhlb_set_tuning(hhlb_solver *s, const hhlb_tuning *t) {
  if (!s || !t) return fail(HHLB_E_ARG, "null argument");
  if (t->graph_steps < 0 || (t->class_streams != 0 && t->class_streams != 1) || (t->xcd_map != 0 && t->xcd_map != 1) ||
      (t->waves_per_window != 2 && t->waves_per_window != 4) || (t->step_fusion != 0 && t->step_fusion != 1) ||
      t->merge_classes < 0 || t->merge_classes > 2)
    return fail(HHLB_E_ARG, "graph_steps >= 0, class_streams, xcd_map and step_fusion 0 or 1, "
                            "waves_per_window 2 or 4, merge_classes 0, 1 or 2");
  if (t->merge_classes && (t->class_streams || t->step_fusion || t->waves_per_window != 2))
    return fail(HHLB_E_ARG, "merge_classes needs class_streams 0, step_fusion 0 and waves_per_window 2");
  s->drop_graphs();
  s->tuning.graph_steps = t->graph_steps;
  s->tuning.class_streams = t->class_streams;
  s->tuning.xcd_map = t->xcd_map;
  s->tuning.waves_per_window = t->waves_per_window;
  s->tuning.step_fusion = t->step_fusion;
  s->tuning.merge_classes = t->merge_classes;
  return HHLB_OK;
}

extern "C" hhlb_status hhlb_get_tuning(const hhlb_solver *s, hhlb_tuning *t) {
  if (!s || !t) return fail(HHLB_E_ARG, "null argument");
  *t = s->tuning;
  return HHLB_OK;
}

extern "C" hhlb_status hhlb_autotune(hhlb_solver *s, int32_t trial_steps, hhlb_tuning *best_out) {
  if (!s || trial_steps < 1) return fail(HHLB_E_ARG, "need a solver and trial_steps >= 1");
  if (!s->ws) return fail(HHLB_E_STATE, "no workspace bound");
  hhlb_status st = check_flag(s);
  if (st) return st;
  const bool multi = s->classes.size() > 1;
  bool has4 = false, hasf = false;
  for (auto &mc : s->classes) {
    has4 = has4 || mc.launch4 != nullptr;
    hasf = hasf || mc.fused != nullptr;
  }
  std::vector<hhlb_tuning> cands;
  for (int sf : {0, 1})
    for (int wpw : {2, 4})
      for (int gs : {0, 16})
        for (int cs : {0, 1})
          for (int xm : {1, 0})
            for (int mg : {0, 1, 2}) {
              if (cs && (!multi || gs > 0)) continue;   // class streams apply to direct launches
              if (wpw == 4 && !has4) continue;
              if (sf && !hasf) continue;
              if (mg && (s->groups.empty() || cs || sf || wpw != 2)) continue;
              hhlb_tuning t{};
              t.graph_steps = gs;
              t.class_streams = cs;
              t.xcd_map = xm;
              t.waves_per_window = wpw;
              t.step_fusion = sf;
              t.merge_classes = mg;
              cands.push_back(t);
            }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const hhlb_tuning saved = s->tuning;
  hhlb_tuning best = saved;
  float best_ms = 0.0f;
  bool have = false;
  for (hhlb_tuning &t : cands) {
    s->drop_graphs();
    s->tuning = t;
    // one untimed step builds graphs and streams, then the timed trial
    st = run_steps(s, 1);
    if (st) break;
    hipError_t e = hipEventRecord(e0, s->stream);
    if (e == hipSuccess) st = run_steps(s, trial_steps);
    if (!st && e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (!st && e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (!st && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) st = fail(HHLB_E_HIP, std::string("autotune timing: ") + hipGetErrorString(e));
    if (st) break;
    t.ms_per_step = ms / trial_steps;
    if (!have || t.ms_per_step < best_ms) { best = t; best_ms = t.ms_per_step; have = true; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->drop_graphs();
  if (st) {
    s->tuning = saved;
    return st;
  }
  s->tuning = best;
  if (best_out) *best_out = best;
  return HHLB_OK;
}

extern "C" {

hhlb_status hhlb_moments(const hhlb_solver *s, double *n_dev, double *u_dev, double *T_dev) {
  if (!s || !n_dev || !u_dev || !T_dev) return fail(HHLB_E_ARG, "null argument");
  if (!s->ws) return fail(HHLB_E_STATE, "no workspace bound");
  int maxNx = 0;
  for (auto &c : s->ch) maxNx = std::max(maxNx, c.Nx);
  dim3 grid((maxNx + 255) / 256, (unsigned)s->ch.size());
  const AuxArgs a = aux(s);
  const int hc = s->has_chi ? 1 : 0;
  if (s->mixed())
    hipLaunchKernelGGL(moments_kernel<float>, grid, dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans, a.ch_V,
                       a.n_ch, a.scaled, (const float *)s->fA(), (const int16_t *)s->lA(), (const float *)s->cA(),
                       (const int16_t *)s->lcA(), hc, n_dev, u_dev, T_dev);
  else
    hipLaunchKernelGGL(moments_kernel<double>, grid, dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans, a.ch_V,
                       a.n_ch, a.scaled, (const double *)s->fA(), (const int16_t *)nullptr, (const double *)s->cA(),
                       (const int16_t *)nullptr, hc, n_dev, u_dev, T_dev);
  HIP_TRY(hipGetLastError());
  return HHLB_OK;
}

hhlb_status hhlb_diagnostics(hhlb_solver *s, double *n_wall_dev, double *mass_dev, double *residual_dev,
                             int32_t *nonfinite_dev) {
  if (!s) return fail(HHLB_E_ARG, "null solver");
  if (!s->ws) return fail(HHLB_E_STATE, "no workspace bound");
  const int n_ch = (int)s->ch.size();
  const AuxArgs a = aux(s);
  const int hc = s->has_chi ? 1 : 0;
  if (n_wall_dev)
    HIP_TRY(hipMemcpyAsync(n_wall_dev, s->ws + s->o_nwall, sizeof(double) * 2 * n_ch, hipMemcpyDeviceToDevice,
                           s->stream));
  if (residual_dev) {
    // one forward-Euler stage from the current state into the C copies; the
    // state (A) and the wall densities are left untouched
    if (s->mixed()) {
      enqueue_stage(s, 0, nullptr, nullptr, s->fC, s->cC, 0.0, 1.0, s->stream);
      hipLaunchKernelGGL(residual_kernel<float>, dim3(n_ch), dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans,
                         a.ch_V, a.n_ch, a.scaled, 1, (const float *)s->fA(), (const float *)s->fC,
                         (const float *)s->cA(), (const float *)s->cC, hc, residual_dev);
    } else {
      enqueue_stage(s, 0, s->fA(), s->cA(), s->fC, s->cC, 0.0, 1.0, s->stream);
      hipLaunchKernelGGL(residual_kernel<double>, dim3(n_ch), dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans,
                         a.ch_V, a.n_ch, a.scaled, 0, (const double *)s->fA(), (const double *)s->fC,
                         (const double *)s->cA(), (const double *)s->cC, hc, residual_dev);
    }
    HIP_TRY(hipGetLastError());
  }
  // mass and the non-finite count (always taken: hhlb_step reports it)
  if (!s->flag_host) {
    HIP_TRY(hipHostMalloc((void **)&s->flag_host, sizeof(int32_t), hipHostMallocDefault));
    *s->flag_host = 0;
    HIP_TRY(hipEventCreateWithFlags(&s->ev_flag, hipEventDisableTiming));
  }
  int32_t *flag = (int32_t *)(s->ws + s->o_flag);
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(1), 0, s->stream, flag);
  if (nonfinite_dev) hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(1), 0, s->stream, nonfinite_dev);
  const double *dx = (const double *)(s->ws + s->o_dx);
  if (s->mixed())
    hipLaunchKernelGGL(mass_kernel<float>, dim3(n_ch), dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans, a.ch_V,
                       a.n_ch, a.scaled, (const float *)s->fA(), (const int16_t *)s->lA(), (const float *)s->cA(),
                       hc, dx, mass_dev, nonfinite_dev, flag);
  else
    hipLaunchKernelGGL(mass_kernel<double>, dim3(n_ch), dim3(256), 0, s->stream, a.tbs, a.ch_class, a.chans, a.ch_V,
                       a.n_ch, a.scaled, (const double *)s->fA(), (const int16_t *)nullptr, (const double *)s->cA(),
                       hc, dx, mass_dev, nonfinite_dev, flag);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(s->flag_host, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipEventRecord(s->ev_flag, s->stream));
  s->flag_pending = true;
  return HHLB_OK;
}

hhlb_status hhlb_launch_info(const hhlb_solver *s, int32_t *launches_per_stage, int64_t *windows_total) {
  if (!s) return fail(HHLB_E_ARG, "null solver");
  if (launches_per_stage) {
    int32_t n = 0;
    const bool merge = s->tuning.merge_classes != 0;
    for (size_t ci = 0; ci < s->classes.size(); ++ci)
      if (!merge || s->class_group[ci] < 0) n += s->classes[ci].large ? 2 : 1;   // large: cell and node phase
    if (merge) n += (int32_t)s->groups.size();
    *launches_per_stage = n;
  }
  if (windows_total) {
    int64_t t = 0;
    for (auto &mc : s->classes) t += (int64_t)mc.windows.size();
    *windows_total = t;
  }
  return HHLB_OK;
}

hhlb_status hhlb_equilibrium_ladder(const hhlb_solver *s, int32_t channel, int32_t *counts, double *reach) {
  if (!s || !counts || !reach) return fail(HHLB_E_ARG, "null argument");
  if (channel < 0 || channel >= (int32_t)s->ch.size()) return fail(HHLB_E_ARG, "channel out of range");
  const ModelClass &mc = s->classes[s->ch_class[channel]];
  if (!hhlb::half_range(mc.quad)) return fail(HHLB_E_UNSUPPORTED, "the full-range equilibrium has no ladder");
  for (int j = 0; j < hhlb::kLadder; ++j) {
    counts[j] = mc.large ? ((const hhlb::DevLarge *)mc.lblob.data())->lad_n[j] : mc.dev.lad_n[j];
    reach[j] = mc.large ? ((const hhlb::DevLarge *)mc.lblob.data())->lad_y[j] : mc.dev.lad_y[j];
  }
  return HHLB_OK;
}

hhlb_status hhlb_wide_equilibrium_count(const hhlb_solver *s, int64_t *count) {
  if (!s || !count) return fail(HHLB_E_ARG, "null argument");
  if (!s->ws) return fail(HHLB_E_STATE, "no workspace bound");
  unsigned long long c = 0;
  HIP_TRY(hipMemcpyAsync(&c, s->ws + s->o_wide, sizeof c, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  *count = (int64_t)c;
  return HHLB_OK;
}

hhlb_status hhlb_destroy(hhlb_solver *s) {
  delete s;
  return HHLB_OK;
}

}  // extern "C"

// ---- mixed-quadrature velocity space (App. A), homogeneous gas ------------

namespace {

// Tables of one product set: DevMulti and its trailing doubles, built once
// per set of axes and kept for the life of the process (the uploads read
// them asynchronously).
struct MultiSet {
  std::vector<char> blob;
  int d = 0, V = 0;
  int kdoubles = 0;   // sum of V_a multi_kcols(V_a): the padded K_a tables the kernel stages in LDS
  int nmax = 0;       // the largest equilibrium order of the axes
};

std::mutex g_multi_mu;
std::map<std::string, std::shared_ptr<const MultiSet>> g_multi_cache;

hhlb_status multi_set(const hhlb_axis *axes, int32_t d, std::shared_ptr<const MultiSet> &out) {
  if (!axes) return fail(HHLB_E_ARG, "null axes");
  if (d < 2 || d > hhlb::kMultiAxes) return fail(HHLB_E_ARG, "d must be 2 or 3");
  std::string key = std::to_string(d);
  for (int a = 0; a < d; ++a) {
    char b[96];
    std::snprintf(b, sizeof b, "|%d,%d,%d,%a", axes[a].quad, axes[a].Q, axes[a].N, axes[a].p0);
    key += b;
  }
  {
    std::lock_guard<std::mutex> lk(g_multi_mu);
    auto it = g_multi_cache.find(key);
    if (it != g_multi_cache.end()) { out = it->second; return HHLB_OK; }
  }
  try {
    std::vector<hhlb::Rule> rules(d);
    int V = 1;
    for (int a = 0; a < d; ++a) {
      const hhlb_axis &x = axes[a];
      const std::string ax = "axis " + std::to_string(a) + ": ";
      if (x.quad != HHLB_HALF_HERMITE && x.quad != HHLB_FULL_HERMITE && x.quad != HHLB_HALF_LAGUERRE)
        return fail(HHLB_E_ARG, ax + "unknown quadrature");
      if (x.N < 0 || x.N >= x.Q) return fail(HHLB_E_ARG, ax + "N must satisfy 0 <= N < Q");
      std::string err;
      int st = hhlb::build_rule(x.quad, x.Q, x.p0, rules[a], err);
      if (st) return fail(st, ax + err);
      if (x.N > hhlb::kNmaxLarge || rules[a].V > hhlb::kMultiVaxis)
        return fail(HHLB_E_UNSUPPORTED, ax + "needs N <= 20 and at most 32 velocities");
      V *= rules[a].V;
    }
    if (V > hhlb::kMultiVmax) return fail(HHLB_E_UNSUPPORTED, "the product set has more than 512 velocities");
    hhlb::DevMulti hdr;
    std::memset(&hdr, 0, sizeof hdr);
    hdr.d = d;
    hdr.V = V;
    std::vector<double> tail;
    int stride = V;
    for (int a = 0; a < d; ++a) {
      const hhlb::Rule &r = rules[a];
      stride /= r.V;
      hdr.Va[a] = r.V;
      hdr.stride[a] = stride;
      hdr.p_off[a] = (int32_t)tail.size();
      tail.insert(tail.end(), r.p.begin(), r.p.end());
      hdr.k_off[a] = (int32_t)tail.size();
      tail.insert(tail.end(), r.K.begin(), r.K.end());
      // the axis' equilibrium tables: those of the 1-D large-velocity-set path
      hhlb_channel h;
      std::memset(&h, 0, sizeof h);
      h.quad = axes[a].quad;
      h.Q = axes[a].Q;
      h.p0 = axes[a].p0;
      hhlb::DevTables dt;
      std::vector<char> lb;
      int st = make_large_tables(h, axes[a].N, r, dt, lb);
      if (st) return st;
      std::memcpy(&hdr.ax[a], lb.data(), sizeof(hhlb::DevLarge));
      const size_t rows = axes[a].quad == HHLB_FULL_HERMITE ? (size_t)r.V : (size_t)r.H;
      const double *hws = (const double *)(lb.data() + sizeof(hhlb::DevLarge)) + rows * rows;
      hdr.hw_off[a] = (int32_t)tail.size();
      tail.insert(tail.end(), hws, hws + (size_t)r.H * (axes[a].N + 1));
    }
    // packed per-axis indices of every velocity (v = (i V_y + j) V_z + k)
    hdr.idx_off = (int32_t)tail.size();
    std::vector<int32_t> idx(V, 0);
    for (int v = 0; v < V; ++v)
      for (int a = 0; a < d; ++a) idx[v] |= ((v / hdr.stride[a]) % hdr.Va[a]) << (8 * a);
    auto ms = std::make_shared<MultiSet>();
    ms->blob.resize(sizeof hdr + sizeof(double) * tail.size() + sizeof(int32_t) * V);
    std::memcpy(ms->blob.data(), &hdr, sizeof hdr);
    std::memcpy(ms->blob.data() + sizeof hdr, tail.data(), sizeof(double) * tail.size());
    std::memcpy(ms->blob.data() + sizeof hdr + sizeof(double) * tail.size(), idx.data(), sizeof(int32_t) * V);
    ms->d = d;
    ms->V = V;
    for (int a = 0; a < d; ++a) {
      ms->kdoubles += hdr.Va[a] * hhlb::multi_kcols(hdr.Va[a]);
      ms->nmax = std::max(ms->nmax, (int)axes[a].N);
    }
    std::lock_guard<std::mutex> lk(g_multi_mu);
    out = g_multi_cache.emplace(key, ms).first->second;
  } catch (...) {
    return fail(HHLB_E_NOMEM, "allocation failed");
  }
  return HHLB_OK;
}

size_t multi_state_bytes(int64_t npts, int V) { return align256((size_t)npts * (size_t)V * sizeof(double)); }

hhlb_status multi_launch_checks(const MultiSet &ms, const void *f, int64_t npts, const double *F, double Kn,
                                const void *work, size_t work_bytes, size_t need) {
  if (npts < 0) return fail(HHLB_E_ARG, "npts must be >= 0");
  if ((!f && npts > 0) || !F || !work) return fail(HHLB_E_ARG, "null pointer");
  if (!(Kn > 0)) return fail(HHLB_E_ARG, "Kn must be > 0 (+INFINITY: no collisions)");
  for (int a = 0; a < ms.d; ++a)
    if (!std::isfinite(F[a])) return fail(HHLB_E_ARG, "F must be finite");
  if (work_bytes < need) return fail(HHLB_E_ARG, "workspace too small");
  return HHLB_OK;
}

hhlb::MultiArgs multi_args(const MultiSet &ms, void *work, int64_t npts, const double *F, double Kn) {
  hhlb::MultiArgs a;
  std::memset(&a, 0, sizeof a);
  a.tm = (const hhlb::DevMulti *)work;
  a.tab = (const double *)((const char *)work + sizeof(hhlb::DevMulti));
  a.npts = npts;
  for (int k = 0; k < ms.d; ++k) a.F[k] = F[k];
  a.inv_Kn = std::isinf(Kn) ? 0.0 : 1.0 / Kn;
  return a;
}

// The scratch of hhlb_multi_step_noalloc: the tables and the two RK stage
// copies of the homogeneous system live in this file-scope device array
// instead of a caller-provided workspace.  Each GPU holds its own copy until
// the process ends.  Host code never uses the array's name as an address:
// the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kMultiScratchBytes = size_t(32) << 20;

}  // namespace

static __device__ __align__(256) char scratch[kMultiScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

hhlb_status scratch_address(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HHLB_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HHLB_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return HHLB_OK;
}

hhlb_status multi_steps(const MultiSet &ms, double *f_dev, int64_t npts, const double *F, double Kn, double dt,
                        int32_t n_steps, void *work_dev, hipStream_t s);

}  // namespace

extern "C" {

hhlb_status hhlb_multi_nodes(const hhlb_axis *axes, int32_t d, double *p_out, double *w_out) {
  if (!p_out || !w_out) return fail(HHLB_E_ARG, "null output pointer");
  std::shared_ptr<const MultiSet> ms;
  int st = multi_set(axes, d, ms);
  if (st) return st;
  const hhlb::DevMulti &h = *(const hhlb::DevMulti *)ms->blob.data();
  const double *tab = (const double *)(ms->blob.data() + sizeof(hhlb::DevMulti));
  for (int v = 0; v < h.V; ++v) {
    w_out[v] = 1.0;
    for (int a = 0; a < d; ++a) p_out[(size_t)a * h.V + v] = tab[h.p_off[a] + (v / h.stride[a]) % h.Va[a]];
  }
  // the product of the axis weights
  try {
    for (int a = 0; a < d; ++a) {
      hhlb::Rule r;
      std::string err;
      st = hhlb::build_rule(axes[a].quad, axes[a].Q, axes[a].p0, r, err);
      if (st) return fail(st, err);
      for (int v = 0; v < h.V; ++v) w_out[v] *= r.wv[(v / h.stride[a]) % h.Va[a]];
    }
  } catch (...) {
    return fail(HHLB_E_NOMEM, "allocation failed");
  }
  return HHLB_OK;
}

hhlb_status hhlb_multi_workspace_bytes(const hhlb_axis *axes, int32_t d, int64_t npts, size_t *bytes) {
  if (!bytes) return fail(HHLB_E_ARG, "null output pointer");
  if (npts < 0) return fail(HHLB_E_ARG, "npts must be >= 0");
  std::shared_ptr<const MultiSet> ms;
  int st = multi_set(axes, d, ms);
  if (st) return st;
  *bytes = align256(ms->blob.size()) + 2 * multi_state_bytes(npts, ms->V);
  return HHLB_OK;
}

hhlb_status hhlb_multi_rhs(const hhlb_axis *axes, int32_t d, const double *f_dev, int64_t npts,
                           const double *F, double Kn, double *L_dev, void *work_dev, size_t work_bytes,
                           void *hip_stream) {
  std::shared_ptr<const MultiSet> ms;
  int st = multi_set(axes, d, ms);
  if (st) return st;
  st = multi_launch_checks(*ms, f_dev, npts, F, Kn, work_dev, work_bytes, align256(ms->blob.size()));
  if (st) return st;
  if (!L_dev && npts > 0) return fail(HHLB_E_ARG, "null pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  HIP_TRY(hipMemcpyAsync(work_dev, ms->blob.data(), ms->blob.size(), hipMemcpyHostToDevice, s));
  hhlb::MultiArgs a = multi_args(*ms, work_dev, npts, F, Kn);
  a.in = f_dev;
  a.out = L_dev;
  a.rhs_only = 1;
  hhlb::launch_multi(a, s, ms->V, ms->kdoubles, ms->nmax);
  HIP_TRY(hipGetLastError());
  return HHLB_OK;
}

hhlb_status hhlb_multi_step(const hhlb_axis *axes, int32_t d, double *f_dev, int64_t npts, const double *F,
                            double Kn, double dt, int32_t n_steps, void *work_dev, size_t work_bytes,
                            void *hip_stream) {
  std::shared_ptr<const MultiSet> ms;
  int st = multi_set(axes, d, ms);
  if (st) return st;
  const size_t tb = align256(ms->blob.size()), sb = multi_state_bytes(npts, ms->V);
  st = multi_launch_checks(*ms, f_dev, npts, F, Kn, work_dev, work_bytes, tb + 2 * sb);
  if (st) return st;
  if (n_steps < 0 || !(dt > 0) || !std::isfinite(dt)) return fail(HHLB_E_ARG, "need n_steps >= 0 and dt > 0");
  return multi_steps(*ms, f_dev, npts, F, Kn, dt, n_steps, work_dev, (hipStream_t)hip_stream);
}

hhlb_status hhlb_multi_step_noalloc(const hhlb_axis *axes, int32_t d, double *f_dev, int64_t npts,
                                    const double *F, double Kn, double dt, int32_t n_steps, void *hip_stream) {
  std::shared_ptr<const MultiSet> ms;
  int st = multi_set(axes, d, ms);
  if (st) return st;
  if (npts < 0) return fail(HHLB_E_ARG, "npts must be >= 0");
  const size_t tb = align256(ms->blob.size()), sb = multi_state_bytes(npts, ms->V);
  if (tb + 2 * sb > kMultiScratchBytes)
    return fail(HHLB_E_ARG, "npts = " + std::to_string(npts) + " needs " + std::to_string(tb + 2 * sb) +
                                " bytes of scratch; the static scratch holds " +
                                std::to_string(kMultiScratchBytes) + " (use hhlb_multi_step with a workspace)");
  void *work = nullptr;
  st = scratch_address(&work);
  if (st) return st;
  st = multi_launch_checks(*ms, f_dev, npts, F, Kn, work, kMultiScratchBytes, tb + 2 * sb);
  if (st) return st;
  if (n_steps < 0 || !(dt > 0) || !std::isfinite(dt)) return fail(HHLB_E_ARG, "need n_steps >= 0 and dt > 0");
  return multi_steps(*ms, f_dev, npts, F, Kn, dt, n_steps, work, (hipStream_t)hip_stream);
}

}  // extern "C"

namespace {

hhlb_status multi_steps(const MultiSet &msr, double *f_dev, int64_t npts, const double *F, double Kn, double dt,
                        int32_t n_steps, void *work_dev, hipStream_t s) {
  const MultiSet *ms = &msr;
  const size_t tb = align256(ms->blob.size()), sb = multi_state_bytes(npts, ms->V);
  HIP_TRY(hipMemcpyAsync(work_dev, ms->blob.data(), ms->blob.size(), hipMemcpyHostToDevice, s));
  double *y1 = (double *)((char *)work_dev + tb), *y2 = (double *)((char *)work_dev + tb + sb);
  hhlb::MultiArgs a = multi_args(*ms, work_dev, npts, F, Kn);
  a.dt = dt;
  for (int k = 0; k < n_steps; ++k) {
    // Eq. (rk3): y1 = y + dt L[y]; y2 = 3/4 y + 1/4 (y1 + dt L[y1]);
    // y+ = 1/3 y + 2/3 (y2 + dt L[y2])
    a.in = f_dev; a.base = nullptr; a.out = y1; a.a_base = 0.0; a.b_stage = 1.0;
    hhlb::launch_multi(a, s, ms->V, ms->kdoubles, ms->nmax);
    a.in = y1; a.base = f_dev; a.out = y2; a.a_base = 0.75; a.b_stage = 0.25;
    hhlb::launch_multi(a, s, ms->V, ms->kdoubles, ms->nmax);
    a.in = y2; a.base = f_dev; a.out = f_dev; a.a_base = 1.0 / 3.0; a.b_stage = 2.0 / 3.0;
    hhlb::launch_multi(a, s, ms->V, ms->kdoubles, ms->nmax);
  }
  HIP_TRY(hipGetLastError());
  return HHLB_OK;
}

}  // namespace
