// Drives the library's host code through the C ABI, built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host side (device code unchanged):
//
//   solver_lifecycle host <channels.txt>   no GPU call: the velocity sets, force
//       matrices and equilibria of every model kind, solver construction for
//       every kind of channel and for a batch of channels of uneven size and
//       order in each arithmetic form (tables, class grouping, launch groups
//       across classes, workspace layout), the launch-configuration checks and
//       the argument-error paths; then destruction.
//   solver_lifecycle gpu <channels.txt>    on a GPU: the autotuner's candidate
//       loop twice on one solver, launch configurations switched back to back
//       with steps queued and no synchronisation by the caller, solvers
//       destroyed with work in flight, in each arithmetic form.
//
// channels.txt holds one channel of the batched workload per line:
// Q Nx Kn g T_right.  Prints "OK" and exits 0 when every call returned what
// it should; any sanitizer report ends the process with a non-zero status.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hhlb.h"

namespace {

int g_checks = 0;
const auto g_t0 = std::chrono::steady_clock::now();

void phase(const char *what) {
  const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - g_t0).count();
  std::printf("[lifecycle] %6.1f s  %s\n", t, what);
  std::fflush(stdout);
}

void expect(hhlb_status got, hhlb_status want, const char *what, int line) {
  ++g_checks;
  if (got == want) return;
  std::printf("FAIL line %d: %s returned %d, expected %d (%s)\n", line, what, got, want, hhlb_last_error());
  std::fflush(stdout);
  std::exit(3);
}
#define EXPECT(call, want) expect((call), (want), #call, __LINE__)
#define OK(call) expect((call), HHLB_OK, #call, __LINE__)

void hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  std::printf("HIP FAIL %s: %s\n", what, hipGetErrorString(e));
  std::fflush(stdout);
  std::exit(4);
}

hhlb_channel base_channel() {
  hhlb_channel c;
  std::memset(&c, 0, sizeof(c));
  c.quad = HHLB_HALF_HERMITE; c.Q = 4; c.N = 3; c.Nx = 64; c.adv = HHLB_WENO5; c.transverse_dof = 2;
  c.L = 1.0; c.stretch_A = 0.0; c.Kn = 0.1; c.g = -0.1; c.T_left = 1.0; c.T_right = 1.0; c.p0 = 1.0;
  c.dt = -0.5;
  return c;
}

std::vector<hhlb_channel> load(const char *path) {
  std::vector<hhlb_channel> v;
  FILE *fh = std::fopen(path, "r");
  if (!fh) {
    std::printf("cannot open %s\n", path);
    std::exit(2);
  }
  int Q, Nx;
  double Kn, g, Tr;
  while (std::fscanf(fh, "%d %d %lf %lf %lf", &Q, &Nx, &Kn, &g, &Tr) == 5) {
    hhlb_channel c = base_channel();
    c.Q = Q; c.N = Q - 1; c.Nx = Nx; c.Kn = Kn; c.g = g; c.T_right = Tr;
    v.push_back(c);
  }
  std::fclose(fh);
  if (v.empty()) {
    std::printf("no channels in %s\n", path);
    std::exit(2);
  }
  return v;
}

// Host tables of one model: nodes, weights, force matrix and equilibria.
void tables(int quad, int Q) {
  const int V = quad == HHLB_FULL_HERMITE ? Q : 2 * Q;
  std::vector<double> p(V), w(V), K((size_t)V * V), feq(V);
  OK(hhlb_nodes(quad, Q, 1.0, p.data(), w.data()));
  OK(hhlb_force_matrix(quad, Q, 0.7, K.data()));
  const int N = Q - 1 < 20 ? Q - 1 : 20;
  const double uT[][2] = {{0.0, 1.0}, {0.3, 1.7}, {-0.9, 0.5}, {2.5, 0.8}};
  for (const auto &x : uT) OK(hhlb_equilibrium(quad, Q, N, 1.0, 1.2, x[0], x[1], feq.data()));
  for (int k = 0; k < V; ++k)
    if (!std::isfinite(p[k]) || !(w[k] >= 0) || !std::isfinite(feq[k])) {
      std::printf("FAIL: quad %d Q %d entry %d: p %g w %g feq %g\n", quad, Q, k, p[k], w[k], feq[k]);
      std::exit(3);
    }
}

// Everything a solver answers on the host, then destruction.
void inspect_and_destroy(hhlb_solver *s, int n_ch, bool half_range) {
  size_t bytes = 0;
  OK(hhlb_workspace_bytes(s, &bytes));
  std::vector<int64_t> off(n_ch + 1);
  OK(hhlb_state_offsets(s, off.data()));
  std::vector<double> dt(n_ch);
  OK(hhlb_time_steps(s, dt.data()));
  for (int c = 0; c < n_ch; ++c)
    if (!(dt[c] > 0) || off[c + 1] <= off[c]) {
      std::printf("FAIL: channel %d dt %g offsets %lld %lld\n", c, dt[c], (long long)off[c], (long long)off[c + 1]);
      std::exit(3);
    }
  int32_t lps = 0;
  int64_t wins = 0;
  OK(hhlb_launch_info(s, &lps, &wins));
  int32_t counts[8];
  double reach[8];
  for (int c : {0, n_ch / 2, n_ch - 1})
    EXPECT(hhlb_equilibrium_ladder(s, c, counts, reach), half_range ? HHLB_OK : HHLB_E_UNSUPPORTED);
  EXPECT(hhlb_equilibrium_ladder(s, n_ch, counts, reach), HHLB_E_ARG);
  // the calls that need device memory refuse without a workspace
  EXPECT(hhlb_step(s, 1), HHLB_E_STATE);
  EXPECT(hhlb_init_equilibrium(s, 1.0, 0.0, 1.0), HHLB_E_STATE);
  EXPECT(hhlb_autotune(s, 2, nullptr), HHLB_E_STATE);
  // launch configurations: the valid ones are taken, the rest refused
  hhlb_tuning t, back;
  OK(hhlb_get_tuning(s, &t));
  const hhlb_tuning good[] = {{16, 0, 1, 2, 0, 0, 0.f}, {0, 1, 0, 4, 1, 0, 0.f}, {16, 0, 1, 2, 0, 2, 0.f},
                              {3, 0, 0, 2, 0, 1, 0.f}};
  for (const hhlb_tuning &g : good) {
    OK(hhlb_set_tuning(s, &g));
    OK(hhlb_get_tuning(s, &back));
    if (back.graph_steps != g.graph_steps || back.merge_classes != g.merge_classes) {
      std::printf("FAIL: tuning not kept\n");
      std::exit(3);
    }
  }
  const hhlb_tuning bad[] = {{-1, 0, 1, 2, 0, 0, 0.f}, {0, 2, 1, 2, 0, 0, 0.f}, {0, 0, 1, 3, 0, 0, 0.f},
                             {0, 0, 1, 2, 0, 3, 0.f},  {0, 1, 1, 2, 0, 1, 0.f}, {0, 0, 1, 4, 0, 2, 0.f},
                             {0, 0, 1, 2, 1, 1, 0.f}};
  for (const hhlb_tuning &b : bad) EXPECT(hhlb_set_tuning(s, &b), HHLB_E_ARG);
  EXPECT(hhlb_set_graph_steps(s, -1), HHLB_E_ARG);
  OK(hhlb_set_graph_steps(s, 8));
  OK(hhlb_destroy(s));
}

void host_mode(const std::vector<hhlb_channel> &batch) {
  // velocity sets of every kind (the large-Q ones are built by the solvers below)
  for (int Q : {1, 2, 3, 4, 6, 8, 12, 16, 40}) tables(HHLB_HALF_HERMITE, Q);
  for (int Q : {2, 4, 8, 16, 64}) tables(HHLB_FULL_HERMITE, Q);
  for (int Q : {1, 2, 3, 4, 8, 16}) tables(HHLB_HALF_LAGUERRE, Q);
  std::vector<double> buf(4096);
  EXPECT(hhlb_nodes(HHLB_HALF_HERMITE, 4, 1.0, nullptr, buf.data()), HHLB_E_ARG);
  EXPECT(hhlb_nodes(HHLB_FULL_HERMITE, 3, 1.0, buf.data(), buf.data() + 8), HHLB_E_ARG);
  EXPECT(hhlb_nodes(7, 4, 1.0, buf.data(), buf.data() + 8), HHLB_E_ARG);
  EXPECT(hhlb_equilibrium(HHLB_HALF_HERMITE, 4, 4, 1.0, 1.0, 0.0, 1.0, buf.data()), HHLB_E_ARG);
  EXPECT(hhlb_equilibrium(HHLB_HALF_HERMITE, 4, 3, 1.0, 1.0, 0.0, -1.0, buf.data()), HHLB_E_ARG);
  EXPECT(hhlb_force_matrix(HHLB_HALF_HERMITE, 4, 1.0, nullptr), HHLB_E_ARG);

  phase("velocity sets");
  // the batch in every arithmetic form
  const int n = (int)batch.size();
  for (int prec : {HHLB_FP64, HHLB_MIXED_F32, HHLB_MIXED_BF16, HHLB_MIXED_F16}) {
    hhlb_solver *s = nullptr;
    OK(hhlb_create(batch.data(), n, prec, nullptr, &s));
    inspect_and_destroy(s, n, true);
  }
  phase("batch solvers");
  // one solver per kind of channel, and the structured-kernel kinds in one solver
  std::vector<hhlb_channel> kinds;
  hhlb_channel c = base_channel();
  kinds.push_back(c);
  c.stretch_A = 0.9; c.adv = HHLB_UPWIND3; c.Nx = 100; kinds.push_back(c);
  c = base_channel(); c.transverse_dof = 0; c.Q = 16; c.N = 15; c.Nx = 513; kinds.push_back(c);
  c = base_channel(); c.quad = HHLB_FULL_HERMITE; c.Q = 16; c.N = 15; c.T_right = 1.5; kinds.push_back(c);
  c = base_channel(); c.quad = HHLB_HALF_LAGUERRE; c.Q = 8; c.N = 4; c.p0 = 0.5; kinds.push_back(c);
  c = base_channel(); c.Q = 12; c.N = 11; c.Nx = 8; kinds.push_back(c);
  std::vector<hhlb_channel> large;   // the node-parallel stage: HHLB(20;200), HLB(20;500)
  c = base_channel(); c.Q = 200; c.N = 20; c.Nx = 24; c.Kn = INFINITY; c.transverse_dof = 0; c.dt = 1e-4;
  large.push_back(c);
  c.quad = HHLB_FULL_HERMITE; c.Q = 500; large.push_back(c);
  for (const auto *set : {&kinds, &large})
    for (const hhlb_channel &k : *set) {
      hhlb_solver *s = nullptr;
      OK(hhlb_create(&k, 1, HHLB_FP64, nullptr, &s));
      inspect_and_destroy(s, 1, k.quad != HHLB_FULL_HERMITE);
    }
  {
    hhlb_solver *s = nullptr;
    OK(hhlb_create(kinds.data(), (int)kinds.size(), HHLB_FP64, nullptr, &s));
    int32_t counts[8];
    double reach[8];
    OK(hhlb_equilibrium_ladder(s, 0, counts, reach));
    EXPECT(hhlb_equilibrium_ladder(s, 3, counts, reach), HHLB_E_UNSUPPORTED);
    OK(hhlb_destroy(s));
  }
  phase("solvers of every kind");
  // construction errors, each reported before anything is built
  hhlb_solver *s = nullptr;
  c = base_channel();
  EXPECT(hhlb_create(nullptr, 1, HHLB_FP64, nullptr, &s), HHLB_E_ARG);
  EXPECT(hhlb_create(&c, 0, HHLB_FP64, nullptr, &s), HHLB_E_ARG);
  EXPECT(hhlb_create(&c, 1, 9, nullptr, &s), HHLB_E_ARG);
  EXPECT(hhlb_create(&c, 1, HHLB_FP64, nullptr, nullptr), HHLB_E_ARG);
  struct Bad { const char *what; void (*edit)(hhlb_channel &); hhlb_status want; };
  const Bad bads[] = {
      {"Nx", [](hhlb_channel &x) { x.Nx = 7; }, HHLB_E_ARG},
      {"N", [](hhlb_channel &x) { x.N = x.Q; }, HHLB_E_ARG},
      {"Kn", [](hhlb_channel &x) { x.Kn = 0.0; }, HHLB_E_ARG},
      {"T", [](hhlb_channel &x) { x.T_right = -1.0; }, HHLB_E_ARG},
      {"A", [](hhlb_channel &x) { x.stretch_A = 1.0; }, HHLB_E_ARG},
      {"dt", [](hhlb_channel &x) { x.dt = NAN; }, HHLB_E_ARG},
      {"Dt", [](hhlb_channel &x) { x.transverse_dof = 1; }, HHLB_E_ARG},
      {"adv", [](hhlb_channel &x) { x.adv = 5; }, HHLB_E_ARG},
      {"odd full-range Q", [](hhlb_channel &x) { x.quad = HHLB_FULL_HERMITE; x.Q = 5; x.N = 4; }, HHLB_E_ARG},
      {"Q = 300", [](hhlb_channel &x) { x.Q = 300; x.N = 20; }, HHLB_E_UNSUPPORTED},
  };
  for (const Bad &b : bads) {
    hhlb_channel x = base_channel();
    b.edit(x);
    s = nullptr;
    expect(hhlb_create(&x, 1, HHLB_FP64, nullptr, &s), b.want, b.what, __LINE__);
    if (s) {
      std::printf("FAIL: a solver came back for %s\n", b.what);
      std::exit(3);
    }
  }
  c = base_channel();
  c.quad = HHLB_HALF_LAGUERRE;
  EXPECT(hhlb_create(&c, 1, HHLB_MIXED_F32, nullptr, &s), HHLB_E_UNSUPPORTED);
  // the mixed-quadrature velocity space: product sets of two and three axes
  const hhlb_axis ax3[3] = {{HHLB_HALF_HERMITE, 4, 3, 1.0}, {HHLB_FULL_HERMITE, 4, 3, 1.0},
                            {HHLB_FULL_HERMITE, 4, 3, 1.0}};
  std::vector<double> pm(3 * 128), wm(128);
  OK(hhlb_multi_nodes(ax3, 3, pm.data(), wm.data()));
  OK(hhlb_multi_nodes(ax3, 2, pm.data(), wm.data()));
  size_t mb = 0;
  OK(hhlb_multi_workspace_bytes(ax3, 3, 1000000, &mb));
  EXPECT(hhlb_multi_nodes(ax3, 4, pm.data(), wm.data()), HHLB_E_ARG);
  OK(hhlb_destroy(nullptr));
}

void gpu_cycle(const std::vector<hhlb_channel> &ch, int prec, bool tune, hipStream_t stream) {
  hhlb_solver *s = nullptr;
  OK(hhlb_create(ch.data(), (int)ch.size(), prec, stream, &s));
  size_t bytes = 0;
  OK(hhlb_workspace_bytes(s, &bytes));
  void *ws = nullptr;
  hip_ok(hipMalloc(&ws, bytes), "hipMalloc");
  OK(hhlb_bind_workspace(s, ws));
  OK(hhlb_init_equilibrium(s, 1.0, 0.0, 1.0));
  if (tune) {
    hhlb_tuning best;
    OK(hhlb_autotune(s, 10, &best));
    std::printf("[lifecycle] form %d: autotune chose graph %d streams %d xcd %d waves %d fusion %d merge %d "
                "(%.3f ms/step)\n", prec, best.graph_steps, best.class_streams, best.xcd_map,
                best.waves_per_window, best.step_fusion, best.merge_classes, best.ms_per_step);
    std::fflush(stdout);
    OK(hhlb_autotune(s, 4, nullptr));
  }
  const hhlb_tuning cfgs[] = {
      {16, 0, 1, 2, 0, 0, 0.f}, {0, 1, 1, 2, 0, 0, 0.f}, {16, 0, 0, 4, 0, 0, 0.f}, {0, 0, 1, 2, 1, 0, 0.f},
      {16, 0, 1, 2, 0, 1, 0.f}, {16, 0, 1, 2, 0, 2, 0.f}, {0, 1, 0, 4, 1, 0, 0.f}, {16, 0, 1, 2, 1, 0, 0.f},
  };
  for (int r = 0; r < 2; ++r)
    for (const hhlb_tuning &t : cfgs) {
      OK(hhlb_set_tuning(s, &t));
      OK(hhlb_step(s, 3 + r * 17));
      OK(hhlb_set_graph_steps(s, r ? 5 : 16));
      OK(hhlb_step(s, 7));
    }
  int64_t wide = 0;
  OK(hhlb_wide_equilibrium_count(s, &wide));
  OK(hhlb_step(s, 9));
  OK(hhlb_destroy(s));   // with steps still queued
  hip_ok(hipStreamSynchronize(stream), "hipStreamSynchronize");
  hip_ok(hipFree(ws), "hipFree");
}

void gpu_mode(const std::vector<hhlb_channel> &batch) {
  hipStream_t stream;
  hip_ok(hipStreamCreate(&stream), "hipStreamCreate");
  gpu_cycle(batch, HHLB_FP64, true, stream);
  gpu_cycle(batch, HHLB_MIXED_F32, true, stream);
  gpu_cycle(batch, HHLB_MIXED_BF16, false, nullptr);
  gpu_cycle(batch, HHLB_FP64, false, stream);
  hip_ok(hipStreamDestroy(stream), "hipStreamDestroy");
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 3 || (std::strcmp(argv[1], "host") && std::strcmp(argv[1], "gpu"))) {
    std::printf("usage: %s host|gpu channels.txt\n", argv[0]);
    return 2;
  }
  const std::vector<hhlb_channel> batch = load(argv[2]);
  std::printf("[lifecycle] %s mode, %zu channels\n", argv[1], batch.size());
  std::fflush(stdout);
  if (!std::strcmp(argv[1], "host")) host_mode(batch);
  else gpu_mode(batch);
  std::printf("[lifecycle] %d checks OK\n", g_checks);
  return 0;
}
