// Host-side tables of the half-range / full-range Gauss-Hermite and the
// half-range Gauss-Laguerre models,
// built in long double and rounded to double once.
#pragma once
#include <string>
#include <vector>

namespace hhlb {

constexpr int kHalf = 0, kFull = 1, kHalfLag = 2;   // half Hermite, full Hermite, half Laguerre
// half-range kinds share the kernels' split force matrix and equilibrium form
inline bool half_range(int quad) { return quad != kFull; }
constexpr int kQmaxTables = 256;  // largest Q the host builder accepts (twice that for the full range)

struct Rule {
  int quad = 0, Q = 0, V = 0, H = 0;
  double p0 = 1.0;
  // orthonormal three-term recurrence of the weight omega(z):
  //   sqrt(b[l+1]) h_{l+1}(z) = (z - a[l]) h_l(z) - sqrt(b[l]) h_{l-1}(z),
  //   h_0 = 1/sqrt(b[0]),  b[0] = int omega.
  std::vector<long double> a, b;
  std::vector<long double> z, w;     // H positive nodes (ascending) and weights
  std::vector<double> p, wv;         // V momenta p_k (m = 1) and weights
  std::vector<double> K;             // V x V force matrix, row-major
  // half-range only: K = blockdiag(Kin, -Kin) + ka (x) kb (rank-1 cross term)
  std::vector<double> Kin, ka, kb;   // H x H, H, H
  // HW[k][l] = w_k h_l(z_k) (half, H x Q) or w_k He_l(z_k)/l! (full, V x Q)
  std::vector<double> HW;
  // half-range Laguerre: a Q-point half-range Gauss-Hermite rule for the main
  // part of the equilibrium coefficients (the Maxwellian becomes the normal
  // density there, which the Laguerre weight does not integrate exactly)
  std::vector<long double> zm, wm;
};

// Builds the rule; returns 0 or a negative hhlb_status and an error text.
int build_rule(int quad, int Q, double p0, Rule &r, std::string &err);

// Discrete equilibrium g_k(u, T) of order N (V values, n = 1), long double.
void equilibrium(const Rule &r, int N, long double u, long double T, double *g);

// Same, with the half-range correction integral taken with nc Gauss-Legendre
// points (the form the kernels evaluate); g in long double.
void equilibrium_nc(const Rule &r, int N, long double u, long double T, int nc, long double *g);

// Largest |y0| = |u| sqrt(m/T) for which nc correction points keep the
// half-range equilibrium within tol of max|g| (T in [0.5, 3]).
double correction_limit(const Rule &r, int N, int nc, double tol);
// The same for n point counts at once (out[j] for ncs[j]; 0 for ncs[j] <= 0).
void correction_limits(const Rule &r, int N, const int *ncs, int n, double tol, double *out);

// Gauss-Legendre nodes tau_i in (0,1) and weights lam_i (sum 1), n points.
void gauss_legendre01(int n, std::vector<long double> &tau, std::vector<long double> &lam);

}  // namespace hhlb
