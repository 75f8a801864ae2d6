// Host table builder for the half-range (Sec. IV.B) and full-range
// (Sec. IV.A) Gauss-Hermite and the half-range Gauss-Laguerre lattice
// Boltzmann models.
//
// Half-range Hermite polynomials are generated from their three-term
// recurrence (Appendix B), whose coefficients come from a discretised
// Stieltjes procedure on a fine composite Gauss-Legendre grid of [0, 40];
// Laguerre polynomials from their exact recurrence;
// nodes are the eigenvalues of the Jacobi matrix (Eq. hh_A_matrix; found by
// Sturm-sequence bisection) and weights the Christoffel numbers
// 1 / sum_{l<Q} h_l(z_k)^2.  Everything is evaluated in long double through
// the recurrence (never through monomial coefficients) and rounded once.
#include "tables.hpp"

#include <cfloat>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include "../../include/hhlb.h"

namespace hhlb {

namespace {

using ld = long double;
const ld kPi = 3.141592653589793238462643383279502884L;

// Legendre P_n and derivative at x by recurrence.
void legendre(int n, ld x, ld &p, ld &dp) {
  ld p0 = 1, p1 = x;
  if (n == 0) { p = 1; dp = 0; return; }
  for (int k = 2; k <= n; ++k) {
    ld p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1);
}

// Orthonormal polynomial values h_0..h_n at x from the recurrence.
void ortho_values(const Rule &r, int n, ld x, ld *h) {
  h[0] = 1 / sqrtl(r.b[0]);
  if (n >= 1) h[1] = (x - r.a[0]) * h[0] / sqrtl(r.b[1]);
  for (int l = 1; l < n; ++l) h[l + 1] = ((x - r.a[l]) * h[l] - sqrtl(r.b[l]) * h[l - 1]) / sqrtl(r.b[l + 1]);
}

// Number of eigenvalues of the n x n Jacobi matrix below x (Sturm count).
int sturm_count(const Rule &r, int n, ld x) {
  int cnt = 0;
  ld d = 1;
  for (int i = 0; i < n; ++i) {
    ld off2 = (i == 0) ? 0 : r.b[i];
    ld dn = (r.a[i] - x) - (i == 0 ? 0 : off2 / d);
    if (dn == 0) dn = -LDBL_MIN;
    if (dn < 0) ++cnt;
    d = dn;
  }
  return cnt;
}

// Discretised Stieltjes procedure for omega(z) = exp(-z^2/2)/sqrt(2 pi) on
// [0, inf): returns a[0..n-1], b[0..n] of the monic recurrence
// pi_{l+1} = (z - a_l) pi_l - b_l pi_{l-1}, b_0 = int omega.
void stieltjes_half(int n, std::vector<ld> &a, std::vector<ld> &b) {
  // 48-point Gauss-Legendre panels of width 1/8 on [0, 50]: near z = 0 the
  // squared degree-l family oscillates with half-wavelength about
  // pi / (4 sqrt(l)) (0.05 at l = 258), which these panels resolve to long
  // double rounding; wider panels lose digits above degree 150
  const int panels = 400, per = 48;
  const ld width = 0.125L;
  std::vector<ld> gx(per), gw(per);
  {
    std::vector<ld> tau, lam;
    gauss_legendre01(per, tau, lam);
    for (int i = 0; i < per; ++i) { gx[i] = tau[i]; gw[i] = lam[i]; }
  }
  const int M = panels * per;
  std::vector<ld> x(M), wt(M), pk(M), pkm1(M, 0), tmp(M);
  for (int pnl = 0; pnl < panels; ++pnl)
    for (int i = 0; i < per; ++i) {
      ld zz = (pnl + gx[i]) * width;
      x[pnl * per + i] = zz;
      wt[pnl * per + i] = gw[i] * width * expl(-zz * zz / 2) / sqrtl(2 * kPi);
    }
  a.assign(n, 0);
  b.assign(n + 1, 0);
  // normalised (Lanczos) form: q_l = pi_l / ||pi_l||
  ld nrm = 0;
  for (int j = 0; j < M; ++j) nrm += wt[j];
  b[0] = nrm;
  for (int j = 0; j < M; ++j) pk[j] = 1 / sqrtl(nrm);
  for (int l = 0; l < n; ++l) {
    ld al = 0;
    for (int j = 0; j < M; ++j) al += wt[j] * x[j] * pk[j] * pk[j];
    a[l] = al;
    ld sb = (l == 0) ? 0 : sqrtl(b[l]);
    for (int j = 0; j < M; ++j) tmp[j] = (x[j] - al) * pk[j] - sb * pkm1[j];
    ld nn = 0;
    for (int j = 0; j < M; ++j) nn += wt[j] * tmp[j] * tmp[j];
    b[l + 1] = nn;
    ld inv = 1 / sqrtl(nn);
    for (int j = 0; j < M; ++j) { pkm1[j] = pk[j]; pk[j] = tmp[j] * inv; }
  }
}

// Eigenvalues of the leading n x n Jacobi matrix by bisection.
void jacobi_eigenvalues(const Rule &r, int n, ld lo, ld hi, std::vector<ld> &ev) {
  ev.resize(n);
  for (int k = 0; k < n; ++k) {
    ld a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      ld m = (a + b) / 2;
      if (m <= a || m >= b) break;
      if (sturm_count(r, n, m) > k) b = m; else a = m;
    }
    ev[k] = (a + b) / 2;
  }
}

}  // namespace

static void compute_gauss_legendre01(int n, std::vector<ld> &tau, std::vector<ld> &lam) {
  tau.resize(n);
  lam.resize(n);
  for (int i = 0; i < n; ++i) {
    ld x = cosl(kPi * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      ld p, dp;
      legendre(n, x, p, dp);
      ld dx = p / dp;
      x -= dx;
      if (fabsl(dx) < 1e-22L) break;
    }
    ld p, dp;
    legendre(n, x, p, dp);
    // map [-1,1] -> [0,1]: weights 2/((1-x^2) P_n'(x)^2) halve
    tau[i] = (x + 1) / 2;
    lam[i] = 1 / ((1 - x * x) * dp * dp);
  }
  // sort ascending
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (tau[j] < tau[i]) { std::swap(tau[i], tau[j]); std::swap(lam[i], lam[j]); }
}

// The rules are built once per point count and process: the equilibrium's
// correction-ladder calibration asks for the same few counts thousands of
// times.
void gauss_legendre01(int n, std::vector<ld> &tau, std::vector<ld> &lam) {
  static std::mutex mu;
  static std::map<int, std::pair<std::vector<ld>, std::vector<ld>>> memo;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = memo.find(n);
    if (it != memo.end()) {
      tau = it->second.first;
      lam = it->second.second;
      return;
    }
  }
  compute_gauss_legendre01(n, tau, lam);
  std::lock_guard<std::mutex> lock(mu);
  memo.emplace(n, std::make_pair(tau, lam));
}

int build_rule(int quad, int Q, double p0, Rule &r, std::string &err) {
  // V <= 2 kQmaxTables: Q per half for the half-range kinds, Q in all for the full range
  if (Q < 1 || Q > (quad == kFull ? 2 * kQmaxTables : kQmaxTables)) { err = "Q out of range"; return HHLB_E_ARG; }
  if (!(p0 > 0) || !std::isfinite(p0)) { err = "p0 must be positive"; return HHLB_E_ARG; }
  if (quad == kFull && (Q % 2)) { err = "full-range Q must be even (no node at p = 0)"; return HHLB_E_ARG; }
  if (quad != kHalf && quad != kFull && quad != kHalfLag) { err = "unknown quadrature"; return HHLB_E_ARG; }
  r = Rule();
  r.quad = quad; r.Q = Q; r.p0 = p0;
  r.V = half_range(quad) ? 2 * Q : Q;
  r.H = r.V / 2;
  const int V = r.V, H = r.H;
  const ld lp0 = p0;
  if (quad == kHalf) {
    stieltjes_half(Q + 2, r.a, r.b);
  } else if (quad == kHalfLag) {
    // omega = exp(-z): monic recurrence pi_{l+1} = (z - (2l+1)) pi_l - l^2 pi_{l-1},
    // b_0 = int omega = 1
    r.a.assign(Q + 2, 0);
    r.b.assign(Q + 3, 0);
    for (int l = 0; l < Q + 2; ++l) r.a[l] = 2 * l + 1;
    r.b[0] = 1;
    for (int l = 1; l <= Q + 2; ++l) r.b[l] = (ld)l * l;
  } else {
    // probabilists' Hermite: monic recurrence with a_l = 0, b_l = l, b_0 = 1
    r.a.assign(Q + 2, 0);
    r.b.assign(Q + 3, 0);
    r.b[0] = 1;
    for (int l = 1; l <= Q + 2; ++l) r.b[l] = l;
  }
  // nodes and Christoffel weights
  std::vector<ld> ev;
  // node envelopes: 2.5 sqrt(Q) (Hermite families), 4Q (Laguerre)
  ld hi = quad == kHalfLag ? 4 * (ld)Q + 8 : 8 + 4 * sqrtl((ld)Q);
  jacobi_eigenvalues(r, Q, quad == kFull ? -hi : 0, hi, ev);
  std::vector<ld> h(Q + 2);
  std::vector<ld> zall(Q), wall(Q);
  for (int k = 0; k < Q; ++k) {
    ortho_values(r, Q - 1, ev[k], h.data());
    ld s = 0;
    for (int l = 0; l < Q; ++l) s += h[l] * h[l];
    zall[k] = ev[k];
    wall[k] = 1 / s;
  }
  r.z.resize(H);
  r.w.resize(H);
  if (half_range(quad)) {
    for (int k = 0; k < H; ++k) { r.z[k] = zall[k]; r.w[k] = wall[k]; }
  } else {
    for (int k = 0; k < H; ++k) { r.z[k] = zall[H + k]; r.w[k] = wall[H + k]; }
  }
  // self-check: exactness for degree <= 2Q-1 against the weight's moments
  {
    std::vector<ld> mu(2 * Q + 1);
    if (quad == kHalfLag) {
      mu[0] = 1;   // int z^s exp(-z) = s!
      for (int s = 1; s <= 2 * Q; ++s) mu[s] = s * mu[s - 1];
    } else {
      if (quad == kHalf) {
        mu[0] = 0.5L;
        mu[1] = 1 / sqrtl(2 * kPi);
      } else {
        mu[0] = 1;
        mu[1] = 0;
      }
      for (int s = 2; s <= 2 * Q; ++s) mu[s] = (s - 1) * mu[s - 2];
    }
    for (int s = 0; s < 2 * Q; ++s) {
      ld acc = 0;
      for (int k = 0; k < Q; ++k) acc += wall[k] * powl(zall[k], s);
      ld ref = mu[s];
      ld scale = 0;
      for (int k = 0; k < Q; ++k) scale += wall[k] * powl(fabsl(zall[k]), s);
      if (fabsl(acc - ref) > 1e-15L * scale) {
        err = "quadrature self-check failed";
        return HHLB_E_NUMERIC;
      }
    }
  }
  r.p.resize(V);
  r.wv.resize(V);
  for (int k = 0; k < V; ++k) {
    int kk = k % H;
    r.p[k] = (double)((k < H ? 1 : -1) * lp0 * r.z[kk]);
    r.wv[k] = (double)r.w[kk];
  }
  r.K.assign((size_t)V * V, 0.0);
  r.HW.assign((size_t)(half_range(quad) ? H : V) * Q, 0.0);
  if (half_range(quad)) {
    // Eq. (hh_Kk) through the recurrence.  The within-half block needs the
    // expansion coefficients of the derivative, phi_s' = sum_{l<s} c_{s,l} phi_l;
    // integrating by parts on [0, inf),
    //   c_{s,l} = -omega(0) phi_s(0) phi_l(0) - int phi_s omega' phi_l.
    // Hermite (omega' = -z omega): the integral is sqrt(b_s) for l = s-1
    // (Eq. hh_Kk_hh, h_{l,l}/h_{l+1,l+1} = sqrt(b_{l+1})); Laguerre
    // (omega' = -omega): it vanishes for l < s (Eq. hh_Kk_L).
    // Phi^Q_0(z_k) = sum_{s<Q} phi_s(0) phi_s(z_k) (Eq. Phi_def).
    std::vector<ld> h0(Q + 1);
    ortho_values(r, Q, 0.0L, h0.data());
    std::vector<std::vector<ld>> hz(H, std::vector<ld>(Q + 1));
    for (int k = 0; k < H; ++k) ortho_values(r, Q, r.z[k], hz[k].data());
    const bool lag = quad == kHalfLag;
    const ld s2pi = lag ? 1.0L : sqrtl(2 * kPi);   // 1 / omega(0)
    std::vector<ld> Phi0(H);
    for (int k = 0; k < H; ++k) {
      ld acc = 0;
      for (int s = 0; s < Q; ++s) acc += h0[s] * hz[k][s];
      Phi0[k] = acc;
    }
    std::vector<ld> inner((size_t)H * H);
    for (int k = 0; k < H; ++k)
      for (int kp = 0; kp < H; ++kp) {
        ld acc = 0;
        for (int l = 0; l <= Q - 2; ++l) {
          ld tail = 0;
          for (int s = l + 1; s <= Q - 1; ++s) tail += h0[s] * hz[k][s];
          acc += hz[kp][l] * (h0[l] / s2pi * tail - (lag ? 0.0L : sqrtl(r.b[l + 1]) * hz[k][l + 1]));
        }
        inner[(size_t)k * H + kp] = acc;
      }
    r.Kin.assign((size_t)H * H, 0.0);
    r.ka.assign(H, 0.0);
    r.kb.assign(H, 0.0);
    for (int k = 0; k < H; ++k) {
      r.ka[k] = (double)(-(r.w[k] / lp0) * Phi0[k] / (2 * s2pi));
      r.kb[k] = (double)Phi0[k];
      for (int kp = 0; kp < H; ++kp) r.Kin[(size_t)k * H + kp] = (double)(r.w[k] / lp0 * inner[(size_t)k * H + kp]);
    }
    for (int k = 0; k < V; ++k)
      for (int kp = 0; kp < V; ++kp) {
        int kk = k % H, kq = kp % H;
        ld sk = k < H ? 1 : -1, skp = kp < H ? 1 : -1;
        ld within = (k < H) == (kp < H) ? sk * r.w[kk] / lp0 * inner[(size_t)kk * H + kq] : 0;
        ld cross = -(sk * r.w[kk] / lp0) * Phi0[kk] * Phi0[kq] / (2 * s2pi);
        r.K[(size_t)k * V + kp] = (double)(within + cross);
      }
    for (int k = 0; k < H; ++k)
      for (int l = 0; l < Q; ++l) r.HW[(size_t)k * Q + l] = (double)(r.w[k] * hz[k][l]);
    if (lag) {
      Rule rh;
      std::string e2;
      int st = build_rule(kHalf, Q, 1.0, rh, e2);
      if (st) { err = "equilibrium rule: " + e2; return st; }
      r.zm = rh.z;
      r.wm = rh.w;
    }
  } else {
    // Eq. (H_Kk) with He_l = sqrt(l!) h_l (orthonormal h_l):
    // He_{l+1}(z_k) He_l(z_k')/l! = sqrt(l+1) h_{l+1}(z_k) h_l(z_k').
    std::vector<std::vector<ld>> hz(V, std::vector<ld>(Q + 1));
    std::vector<ld> zz(V);
    for (int k = 0; k < V; ++k) {
      zz[k] = (k < H ? 1 : -1) * r.z[k % H];
      ortho_values(r, Q, zz[k], hz[k].data());
    }
    for (int k = 0; k < V; ++k)
      for (int kp = 0; kp < V; ++kp) {
        ld acc = 0;
        for (int l = 0; l <= Q - 2; ++l) acc += sqrtl((ld)(l + 1)) * hz[k][l + 1] * hz[kp][l];
        r.K[(size_t)k * V + kp] = (double)(-(r.w[k % H] / lp0) * acc);
      }
    // He_l(z)/l! = h_l(z)/sqrt(l!)
    for (int k = 0; k < V; ++k) {
      ld fact = 1;
      for (int l = 0; l < Q; ++l) {
        if (l > 0) fact *= l;
        r.HW[(size_t)k * Q + l] = (double)(r.w[k % H] * hz[k][l] / sqrtl(fact));
      }
    }
  }
  return HHLB_OK;
}

// Half-range equilibrium by an exact change of variables.  With
// p = m u + sqrt(m T) y the Maxwellian becomes the standard normal density,
// so the coefficient G^+_l = int_0^inf dp g h_l(p/p0) of Sec. IV.B.3 is
//   int_{y0}^inf omega(y) h_l(ub + s y) dy,   ub = m u/p0, s = sqrt(mT)/p0,
// y0 = -u sqrt(m/T): the part on [0, inf) is a polynomial of degree <= N
// against the half-range Gaussian weight, integrated exactly by a Q-point
// half-range Gauss-Hermite rule (the rule itself for HHLB, an auxiliary one
// for the Laguerre model); the remainder over [y0, 0] is a short
// Gauss-Legendre integral.
// G^-_l follows with u -> -u.  Then g_k = w_k sum_{l<=N} G^sigma_l h_l(z_k).
// Full range (Sec. IV.A.3): G_l = E[He_l(X)], X ~ N(ub, mT/p0^2), from
// G_{l+1} = ub G_l + l (mT/p0^2 - 1) G_{l-1}; g_k = w_k sum G_l He_l(z_k)/l!.
void equilibrium_nc(const Rule &r, int N, ld u, ld T, int nc, ld *g) {
  const int Q = r.Q, H = r.H;
  const ld m = 1, p0 = r.p0;
  if (r.quad == kFull) {
    ld a = m * T / (p0 * p0) - 1, bb = m * u / p0;
    std::vector<ld> G(N + 1);
    G[0] = 1;
    if (N >= 1) G[1] = bb;
    for (int l = 1; l < N; ++l) G[l + 1] = bb * G[l] + l * a * G[l - 1];
    std::vector<ld> h(Q + 1);
    for (int k = 0; k < r.V; ++k) {
      ld z = (k < H ? 1 : -1) * r.z[k % H];
      ortho_values(r, N, z, h.data());
      ld acc = 0, fact = 1;
      for (int l = 0; l <= N; ++l) {
        if (l > 0) fact *= l;
        acc += G[l] * h[l] / sqrtl(fact);
      }
      g[k] = r.w[k % H] * acc;
    }
    return;
  }
  std::vector<ld> tau, lam;
  if (nc > 0) gauss_legendre01(nc, tau, lam);
  ld ub = m * u / p0, s = sqrtl(m * T) / p0, y0 = -u * sqrtl(m / T);
  std::vector<ld> h(Q + 1), Gp(N + 1, 0), Gm(N + 1, 0);
  // main part: a half-range Gauss-Hermite rule (the rule itself, or the
  // auxiliary one of a Laguerre rule)
  const std::vector<ld> &zr = r.zm.empty() ? r.z : r.zm;
  const std::vector<ld> &wr = r.wm.empty() ? r.w : r.wm;
  for (size_t j = 0; j < zr.size(); ++j) {
    ortho_values(r, N, ub + s * zr[j], h.data());
    for (int l = 0; l <= N; ++l) Gp[l] += wr[j] * h[l];
    ortho_values(r, N, -ub + s * zr[j], h.data());
    for (int l = 0; l <= N; ++l) Gm[l] += wr[j] * h[l];
  }
  if (y0 != 0) {
    for (int i = 0; i < nc; ++i) {
      ld e = y0 * lam[i] * expl(-(y0 * tau[i]) * (y0 * tau[i]) / 2) / sqrtl(2 * kPi);
      ortho_values(r, N, ub * (1 - tau[i]), h.data());
      for (int l = 0; l <= N; ++l) Gp[l] -= e * h[l];
      ortho_values(r, N, -ub * (1 - tau[i]), h.data());
      for (int l = 0; l <= N; ++l) Gm[l] += e * h[l];
    }
  }
  for (int k = 0; k < H; ++k) {
    ortho_values(r, N, r.z[k], h.data());
    ld ap = 0, am = 0;
    for (int l = 0; l <= N; ++l) { ap += Gp[l] * h[l]; am += Gm[l] * h[l]; }
    g[k] = r.w[k] * ap;
    g[H + k] = r.w[k] * am;
  }
}

void equilibrium(const Rule &r, int N, ld u, ld T, double *g) {
  std::vector<ld> gl(r.V);
  equilibrium_nc(r, N, u, T, 32, gl.data());
  for (int k = 0; k < r.V; ++k) g[k] = (double)gl[k];
}

double correction_limit(const Rule &r, int N, int nc, double tol) {
  double out = 0.0;
  correction_limits(r, N, &nc, 1, tol, &out);
  return out;
}

void correction_limits(const Rule &r, int N, const int *ncs, int n, double tol, double *out) {
  for (int j = 0; j < n; ++j) out[j] = 0.0;
  if (!half_range(r.quad)) return;
  const ld Ts[4] = {0.5L, 1.0L, 2.0L, 3.0L};
  std::vector<ld> g(r.V), gr(r.V);
  std::vector<bool> active(n);
  int n_active = 0;
  for (int j = 0; j < n; ++j) {
    active[j] = ncs[j] > 0;
    n_active += active[j];
  }
  // the grid 1e-6 .. 1 of |y0|; a count keeps the last y0 of an unbroken run
  // of passes; the 40-point reference is shared by every count.  A count
  // passes when its difference from the reference is below tol max|g| or
  // below 8 times the evaluation's own rounding noise (the 40- against the
  // 48-point reference): an ill-conditioned equilibrium (the Laguerre rule at
  // the hot end of the range) otherwise fails every count on noise alone.
  std::vector<ld> g2(r.V);
  for (int e = 0; e <= 96 && n_active > 0; ++e) {
    const ld y = 1e-6L * powl(10.0L, e / 16.0L);
    std::vector<bool> ok(n, true);
    for (ld T : Ts)
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const ld u = sgn * y * sqrtl(T);
        equilibrium_nc(r, N, u, T, 40, gr.data());
        equilibrium_nc(r, N, u, T, 48, g2.data());
        ld mx = 0, noise = 0;
        for (int k = 0; k < r.V; ++k) {
          mx = std::max(mx, fabsl(gr[k]));
          noise = std::max(noise, fabsl(g2[k] - gr[k]));
        }
        const ld bound = std::max((ld)tol * mx, 8 * noise);
        for (int j = 0; j < n; ++j) {
          if (!active[j] || !ok[j]) continue;
          equilibrium_nc(r, N, u, T, ncs[j], g.data());
          ld err = 0;
          for (int k = 0; k < r.V; ++k) err = std::max(err, fabsl(g[k] - gr[k]));
          if (err > bound) ok[j] = false;
        }
      }
    for (int j = 0; j < n; ++j) {
      if (!active[j]) continue;
      if (ok[j]) out[j] = (double)y;
      else { active[j] = false; --n_active; }
    }
  }
}

}  // namespace hhlb
