/*
 * hhlb_oracle.c -- plain, slow CPU oracle for the time step of the half-range
 * Gauss-Hermite lattice Boltzmann model with a force term (Ambrus, Sofonea,
 * Fournier, Blanco, "Implementation of the force term in half-range lattice
 * Boltzmann models", arXiv:1708.03249).
 *
 * TEST INFRASTRUCTURE.  This file is the reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU library; the library must never call it.
 *
 * Conventions (non-dimensional units, as in the paper's Sec. I end):
 *   m = 1; the momentum scale p0 is a parameter; the force is F = m*g where g is
 *   the acceleration along x (the paper writes F = -m g_p, so g = -g_p);
 *   the velocity set has V nodes, index k < V/2 positive momenta in ascending
 *   order, index k >= V/2 the mirrored negative momenta p_k = -p_{k-V/2}.
 *   Half-range (HHLB(N;Q)): V = 2Q.  Full-range (HLB(N;Q), Q even): V = Q.
 *   A reduced transverse-energy function chi with Dt transverse degrees of
 *   freedom travels with f (Dt = 0 reproduces the paper's 1-D model).
 *
 * Precision: every quadrature, force-matrix and equilibrium table is built
 * in __float128 from the defining formulas and rounded to double once; the
 * equilibrium coefficients are evaluated in __float128 because the monomial
 * form of the half-range polynomials cancels heavily (coefficients grow like
 * 1e5 at Q = 16).  The time step itself runs in plain double loops, in the
 * order the paper describes them.
 *
 * Parity is pinned against closed forms and invariants in the CPU tests;
 * no function here is unpinned except where its header comment says so.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 qf;

#define ORC_QMAX 256           /* largest quadrature order the tables accept  */
#define ORC_VMAX (2 * ORC_QMAX)
#define ORC_NEQ 21             /* equilibrium orders N <= 20 (the paper's largest) */
#define ORC_QMONO 16           /* half-range Hermite: monomial construction up to
                                  this Q, the three-term recurrence beyond it   */
#define ORC_QLAG 32            /* largest half-range Laguerre order            */
#define ORC_QFMONO 64          /* full-range Hermite: monomial construction up to
                                  this Q, the three-term recurrence beyond it
                                  (up to Q = ORC_VMAX)                         */
#define ORC_CMAX (ORC_QLAG + 2)  /* monomial rows kept: Laguerre l <= Q+1, and
                                    the recurrence rules' h_0 .. h_21          */

enum { ORC_HALF = 0, ORC_FULL = 1, ORC_HALF_LAGUERRE = 2 };
enum { ORC_WENO5 = 0, ORC_UPWIND3 = 1 };

/* One channel: the paper's statement of the problem (Sec. IV.D and V). */
typedef struct {
  int32_t quad;   /* ORC_HALF (HHLB), ORC_FULL (HLB) or ORC_HALF_LAGUERRE    */
  int32_t Q;      /* quadrature order                                          */
  int32_t N;      /* equilibrium expansion order, 0 <= N < Q                   */
  int32_t Nx;     /* number of cells                                           */
  int32_t adv;    /* ORC_WENO5 or ORC_UPWIND3                                  */
  int32_t Dt;     /* transverse degrees of freedom carried by chi (0 or 2)     */
  double L;       /* channel width; walls at x = -L/2 (left) and +L/2 (right)  */
  double A;       /* tanh stretching parameter, 0 = uniform grid               */
  double Kn;      /* Knudsen number, tau = Kn/n; +inf = collisionless          */
  double g;       /* acceleration along x, F = m g                             */
  double T_left, T_right; /* wall temperatures                                 */
  double p0;      /* momentum scale                                            */
  double dt;      /* time step                                                 */
} orc_channel;

/* ------------------------------------------------------------------------ */
/* Tables                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int quad, Q, V, H;             /* H = V/2 nodes per half                    */
  double p0;
  qf z[ORC_QMAX];                /* positive nodes z_k (ascending), H of them */
  qf w[ORC_QMAX];                /* their weights                             */
  /* half-range: monomial coefficients c[l][s] of the orthonormal h_l
   * (l <= Q+1 up to ORC_QMONO; l <= 21, the equilibrium's range, beyond)  */
  qf c[ORC_CMAX][ORC_CMAX];
  /* half-range Hermite beyond ORC_QMONO: orthonormal recurrence
   * sqrt(b_{l+1}) h_{l+1} = (z - a_l) h_l - sqrt(b_l) h_{l-1}, h_0 = 1/sqrt(b_0) */
  int rec;
  qf ra[ORC_VMAX + 3], rb[ORC_VMAX + 4];
  /* poly value at the positive nodes: P[l][k] = h_l(z_k) or He_l(z_k)       */
  qf P[ORC_QMAX + 2][ORC_QMAX];
  double p[ORC_VMAX], wd[ORC_VMAX];  /* p_k and w_k over all V nodes (double) */
  double K[ORC_VMAX * ORC_VMAX];     /* force matrix, row-major K[k*V + k']   */
  double Kin[ORC_VMAX * ORC_VMAX];   /* half-range: within-half sum term only */
  double Kd[ORC_VMAX * ORC_VMAX];    /* half-range: the delta-term part only  */
  /* full range: He_l(p_k/p0) / l! at every node for the equilibrium orders
   * l <= min(Q-1, 20), computed once (the per-cell sums of Eq. (H_gk) read
   * them instead of re-running the recurrence) */
  qf heq[ORC_NEQ][ORC_VMAX];
  /* full range: the coefficients l!/(2^s s! (l-2s)!) of G_l, Eq. (H_gk) */
  qf gco[ORC_NEQ][ORC_NEQ];
} orc_tables;

/* Moments of the half-range weight omega(z) = exp(-z^2/2)/sqrt(2 pi) on
 * [0, inf): mu_0 = 1/2, mu_1 = 1/sqrt(2 pi), mu_s = (s-1) mu_{s-2}
 * (integration by parts).  Appendix B, Eq. (hh_omega). */
static void hh_moments(int smax, qf *mu) {
  mu[0] = 0.5Q;
  mu[1] = 1.0Q / sqrtq(2.0Q * M_PIq);
  for (int s = 2; s <= smax; ++s) mu[s] = (qf)(s - 1) * mu[s - 2];
}

static qf hh_inner(const qf *a, int da, const qf *b, int db, const qf *mu) {
  qf acc = 0;
  for (int i = 0; i <= da; ++i)
    for (int j = 0; j <= db; ++j) acc += a[i] * b[j] * mu[i + j];
  return acc;
}

/* Orthonormal half-range Hermite polynomials h_l (gamma_l = 1, Appendix B)
 * by Gram-Schmidt on the monomials in the inner product of Eq. (phi_ortho),
 * leading coefficient positive.  c[l][s] is the coefficient of z^s in h_l,
 * i.e. the paper's h_{l,s} of Eq. (phi_expl). */
static void hh_build_polys(orc_tables *t, int lmax) {
  qf mu[2 * ORC_CMAX + 2];
  hh_moments(2 * lmax + 2, mu);
  memset(t->c, 0, sizeof(t->c));
  for (int l = 0; l <= lmax; ++l) {
    qf v[ORC_CMAX];
    memset(v, 0, sizeof(v));
    v[l] = 1;
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < l; ++j) {
        qf pr = hh_inner(v, l, t->c[j], j, mu);
        for (int s = 0; s <= j; ++s) v[s] -= pr * t->c[j][s];
      }
    qf nr = sqrtq(hh_inner(v, l, v, l, mu));
    for (int s = 0; s <= l; ++s) t->c[l][s] = v[s] / nr;
  }
}

/* Member l of the half-range family held in t->c (Horner on its monomial
 * coefficients). */
static qf hh_eval(const orc_tables *t, int l, qf z) {
  qf acc = 0;
  for (int s = l; s >= 0; --s) acc = acc * z + t->c[l][s];
  return acc;
}

/* Probabilists' Hermite polynomials He_l (Sec. II, Eq. H_ortho up to the
 * normalisation of omega): He_0 = 1, He_1 = z, He_{l+1} = z He_l - l He_{l-1}. */
static qf he_eval(int l, qf z) {
  qf a = 1, b = z;
  if (l == 0) return a;
  for (int j = 1; j < l; ++j) {
    qf c = z * b - (qf)j * a;
    a = b;
    b = c;
  }
  return b;
}

typedef qf (*poly_fn)(const orc_tables *, int, qf);
static qf he_eval_t(const orc_tables *t, int l, qf z) { (void)t; return he_eval(l, z); }

/* Roots of the degree-n member of an orthogonal family by interlacing: the
 * roots of p_l separate those of p_{l+1}.  Plain bisection in __float128.
 * Every root of p_l lies below 4 + 3 sqrt(l) (Hermite families) or
 * 4l + 4 (Laguerre, whose largest root is below 4l + 2). */
static void family_roots(const orc_tables *t, poly_fn f, int n, qf lo_all, qf *roots) {
  qf prev[ORC_QMAX + 2];
  int nprev = 0;
  for (int l = 1; l <= n; ++l) {
    qf hi_all = t->quad == ORC_HALF_LAGUERRE ? 4.0Q * l + 4.0Q : 4.0Q + 3.0Q * sqrtq((qf)l);
    qf cur[ORC_QMAX + 2];
    for (int j = 0; j < l; ++j) {
      qf a = (j == 0) ? lo_all : prev[j - 1];
      qf b = (j == l - 1) ? hi_all : prev[j];
      qf fa = f(t, l, a);
      for (int it = 0; it < 400; ++it) {
        qf m = 0.5Q * (a + b);
        if (m <= a || m >= b) break;
        qf fm = f(t, l, m);
        if ((fm < 0) == (fa < 0)) { a = m; fa = fm; } else { b = m; }
      }
      cur[j] = 0.5Q * (a + b);
    }
    for (int j = 0; j < l; ++j) prev[j] = cur[j];
    nprev = l;
  }
  (void)nprev;
  for (int j = 0; j < n; ++j) roots[j] = prev[j];
}

/* ---- half-range Hermite beyond ORC_QMONO: the three-term recurrence ---- */

/* Test-only switch: half-range Hermite rules with Q above this use the
 * recurrence construction (default ORC_QMONO). */
static int g_qmono = ORC_QMONO;

/* Gauss-Legendre nodes and weights on [-1, 1] (Newton on the Legendre
 * recurrence), n points, in __float128. */
static void gl_nodes(int n, qf *x, qf *w) {
  for (int i = 0; i < n; ++i) {
    qf z = cosq(M_PIq * ((qf)i + 0.75Q) / ((qf)n + 0.5Q)), dp = 1;
    for (int it = 0; it < 100; ++it) {
      qf p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        qf p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      qf dz = p1 / dp;
      z -= dz;
      if (fabsq(dz) < 1e-33Q) break;
    }
    x[i] = z;
    w[i] = 2 / ((1 - z * z) * dp * dp);
  }
}

/* Recurrence coefficients of omega(z) = exp(-z^2/2)/sqrt(2 pi) on [0, inf)
 * by the discretised Stieltjes procedure (orthonormal form): the measure is
 * replaced by a composite 40-point Gauss-Legendre rule on 500 panels of
 * width 0.1 over [0, 50] (omega(50) = 1e-543, far below what the rules
 * resolve).  The panel width follows from the oscillation of h_l: a
 * half-range polynomial of degree l oscillates like a full-range one of
 * degree 2l, so near z = 0 the integrand h_l^2 has half-wavelength about
 * pi / (4 sqrt(l)), 0.05 at l = 256; 40 points on 0.1 integrate it to
 * float128 rounding for every l <= 258 (panels of 0.4 lost digits above
 * l = 150, reaching 1e-6 at l = 256).  Returns a_0..a_{n-1}, b_0..b_n
 * (b_0 = int omega). */
static int hh_stieltjes(int n, qf *a, qf *b) {
  enum { PAN = 500, PER = 40 };
  const qf width = 0.1Q;
  qf gx[PER], gw[PER];
  gl_nodes(PER, gx, gw);
  const int M = PAN * PER;
  qf *x = (qf *)malloc(sizeof(qf) * M), *wt = (qf *)malloc(sizeof(qf) * M);
  qf *pk = (qf *)malloc(sizeof(qf) * M), *pm = (qf *)calloc(M, sizeof(qf));
  if (!x || !wt || !pk || !pm) { free(x); free(wt); free(pk); free(pm); return -1; }
  const qf s2pi = sqrtq(2 * M_PIq);
  for (int q = 0; q < PAN; ++q)
    for (int i = 0; i < PER; ++i) {
      qf z = width * ((qf)q + (gx[i] + 1) / 2);
      x[q * PER + i] = z;
      wt[q * PER + i] = gw[i] * width / 2 * expq(-z * z / 2) / s2pi;
    }
  qf nrm = 0;
  for (int j = 0; j < M; ++j) nrm += wt[j];
  b[0] = nrm;
  for (int j = 0; j < M; ++j) pk[j] = 1 / sqrtq(nrm);
  for (int l = 0; l < n; ++l) {
    qf al = 0;
    for (int j = 0; j < M; ++j) al += wt[j] * x[j] * pk[j] * pk[j];
    a[l] = al;
    qf sb = l == 0 ? 0 : sqrtq(b[l]), nn = 0;
    for (int j = 0; j < M; ++j) {
      qf v = (x[j] - al) * pk[j] - sb * pm[j];
      pm[j] = pk[j];
      pk[j] = v;
      nn += wt[j] * v * v;
    }
    b[l + 1] = nn;
    qf inv = 1 / sqrtq(nn);
    for (int j = 0; j < M; ++j) pk[j] *= inv;
  }
  free(x); free(wt); free(pk); free(pm);
  return 0;
}

/* h_0(z) .. h_n(z) from the orthonormal recurrence. */
static void rec_values(const orc_tables *t, int n, qf z, qf *h) {
  h[0] = 1 / sqrtq(t->rb[0]);
  if (n >= 1) h[1] = (z - t->ra[0]) * h[0] / sqrtq(t->rb[1]);
  for (int l = 1; l < n; ++l) h[l + 1] = ((z - t->ra[l]) * h[l] - sqrtq(t->rb[l]) * h[l - 1]) / sqrtq(t->rb[l + 1]);
}

/* Roots of h_Q: the eigenvalues of the Q x Q Jacobi matrix (diagonal a_l,
 * off-diagonal sqrt(b_l)) by Sturm-sequence bisection. */
static void sturm_roots(const orc_tables *t, int Q, qf lo, qf hi, qf *roots) {
  for (int k = 0; k < Q; ++k) {
    qf a = lo, b = hi;
    for (int it = 0; it < 240; ++it) {
      qf m = (a + b) / 2;
      if (m <= a || m >= b) break;
      int cnt = 0;
      qf d = 1;
      for (int i = 0; i < Q; ++i) {
        qf dn = (t->ra[i] - m) - (i == 0 ? 0 : t->rb[i] / d);
        if (dn == 0) dn = -1e-4900Q;
        if (dn < 0) ++cnt;
        d = dn;
      }
      if (cnt > k) b = m; else a = m;
    }
    roots[k] = (a + b) / 2;
  }
}

/* Half-range Gauss-Hermite rule and force matrix from the recurrence: the
 * same Sec. IV.B.1 rule and Eq. (hh_Kk_hh) matrix as build_half, with
 * h_{l,0} = h_l(0) and h_{l,l}/h_{l+1,l+1} = sqrt(b_{l+1}) read off the
 * recurrence.  Weights by the general Eq. (wk_half_gen),
 * w_k = -a_Q gamma_Q / (h_{Q+1}(z_k) h_Q'(z_k)) with gamma_Q = 1 and h_Q'
 * from the differentiated recurrence: at Q = 200 the specialised
 * Eq. (wk_half) evaluated through the same recurrence loses 1e-12 (its
 * weights sum to 0.4999999999997), the general form keeps 1e-32.  The
 * equilibrium (N <= 20 here) keeps the monomial coefficients of h_0 .. h_21. */
static int build_half_rec(orc_tables *t, int Q, double p0) {
  t->quad = ORC_HALF; t->Q = Q; t->V = 2 * Q; t->H = Q; t->p0 = p0; t->rec = 1;
  if (hh_stieltjes(Q + 2, t->ra, t->rb)) return -1;
  hh_build_polys(t, 21);
  qf r[ORC_QMAX + 2];
  sturm_roots(t, Q, 0, 4.0Q + 3.0Q * sqrtq((qf)Q), r);
  const qf s2pi = sqrtq(2.0Q * M_PIq);
  qf h0[ORC_QMAX + 3], hv[ORC_QMAX + 3];
  rec_values(t, Q + 1, 0, h0);
  const qf aQ = 1 / sqrtq(t->rb[Q + 1]);
  for (int k = 0; k < Q; ++k) {
    const qf z = r[k];
    t->z[k] = z;
    rec_values(t, Q + 1, z, hv);
    /* h_l'(z): differentiate sqrt(b_{l+1}) h_{l+1} = (z - a_l) h_l - sqrt(b_l) h_{l-1} */
    qf dm = 0, dc = 1 / sqrtq(t->rb[1]) * hv[0];   /* h_0', h_1' */
    for (int l = 1; l < Q; ++l) {
      qf dn = ((z - t->ra[l]) * dc + hv[l] - sqrtq(t->rb[l]) * dm) / sqrtq(t->rb[l + 1]);
      dm = dc;
      dc = dn;
    }
    t->w[k] = -aQ / (hv[Q + 1] * dc);   /* dc = h_Q'(z_k) */
    for (int l = 0; l <= Q + 1; ++l) t->P[l][k] = hv[l];
  }
  const int V = 2 * Q;
  for (int k = 0; k < V; ++k) {
    int kk = k % Q;
    t->p[k] = (double)((k < Q ? 1 : -1) * (qf)p0 * t->z[kk]);
    t->wd[k] = (double)t->w[kk];
  }
  qf *Phi0 = (qf *)malloc(sizeof(qf) * Q), *tail = (qf *)malloc(sizeof(qf) * (size_t)Q * Q);
  qf *inner = (qf *)malloc(sizeof(qf) * (size_t)Q * Q);
  if (!Phi0 || !tail || !inner) { free(Phi0); free(tail); free(inner); return -1; }
  for (int k = 0; k < Q; ++k) {
    qf acc = 0;
    for (int s = 0; s < Q; ++s) acc += h0[s] * t->P[s][k];
    Phi0[k] = acc;
    /* tail[l][k] = sum_{s=l+1}^{Q-1} h_s(0) h_s(z_k) */
    qf tl = 0;
    for (int l = Q - 1; l >= 0; --l) {
      tail[(size_t)l * Q + k] = tl;
      tl += h0[l] * t->P[l][k];
    }
  }
  for (int k = 0; k < Q; ++k)
    for (int kq = 0; kq < Q; ++kq) {
      qf acc = 0;
      for (int l = 0; l <= Q - 2; ++l) {
        qf br = h0[l] / s2pi * tail[(size_t)l * Q + k] - sqrtq(t->rb[l + 1]) * t->P[l + 1][k];
        acc += t->P[l][kq] * br;
      }
      inner[(size_t)k * Q + kq] = acc;
    }
  for (int k = 0; k < V; ++k) {
    int kk = k % Q;
    qf sk = (k < Q) ? 1 : -1;
    for (int kp = 0; kp < V; ++kp) {
      int kq = kp % Q;
      qf skp = (kp < Q) ? 1 : -1;
      qf pref = t->w[kk] * sk / (qf)p0;
      qf within = pref * (1 + sk * skp) / 2 * inner[(size_t)kk * Q + kq];
      qf cross = -pref * Phi0[kk] * Phi0[kq] / (2 * s2pi);
      qf delta = pref * sk * skp * Phi0[kk] * Phi0[kq] / (2 * s2pi);
      t->Kin[(size_t)k * V + kp] = (double)within;
      t->Kd[(size_t)k * V + kp] = (double)delta;
      t->K[(size_t)k * V + kp] = (double)(within + cross);
    }
  }
  free(Phi0); free(tail); free(inner);
  return 0;
}

/* Half-range Gauss-Hermite rule and force matrix.
 * Nodes: the Q positive roots of h_Q (Sec. IV.B.1).
 * Weights: Eq. (wk_half), w_k = z_k a_Q^2 / (h_{Q+1}(z_k)^2 [z_k + h_{Q,0}^2/sqrt(2 pi)]),
 *          a_Q = h_{Q+1,Q+1}/h_{Q,Q} (Eq. a_def).
 * Force matrix: Eq. (hh_Kk_hh) with Phi^Q_0 of Eq. (Phi_def_hh). */
static int build_half(orc_tables *t, int Q, double p0) {
  if (Q > g_qmono) return build_half_rec(t, Q, p0);
  t->quad = ORC_HALF; t->Q = Q; t->V = 2 * Q; t->H = Q; t->p0 = p0;
  hh_build_polys(t, Q + 1);
  qf r[ORC_QMAX + 2];
  family_roots(t, hh_eval, Q, 0.0Q, r);
  qf aQ = t->c[Q + 1][Q + 1] / t->c[Q][Q];
  qf s2pi = sqrtq(2.0Q * M_PIq);
  for (int k = 0; k < Q; ++k) {
    t->z[k] = r[k];
    qf hq1 = hh_eval(t, Q + 1, r[k]);
    qf hq0 = t->c[Q][0];
    t->w[k] = r[k] * aQ * aQ / (hq1 * hq1 * (r[k] + hq0 * hq0 / s2pi));
  }
  for (int l = 0; l <= Q + 1; ++l)
    for (int k = 0; k < Q; ++k) t->P[l][k] = hh_eval(t, l, t->z[k]);
  int V = 2 * Q;
  for (int k = 0; k < V; ++k) {
    int kk = k % Q;
    t->p[k] = (double)((k < Q ? 1 : -1) * (qf)p0 * t->z[kk]);
    t->wd[k] = (double)t->w[kk];
  }
  /* Phi^Q_0(z_k) = sum_{s<Q} h_{s,0} h_s(z_k) */
  qf Phi0[ORC_QMAX];
  for (int k = 0; k < Q; ++k) {
    qf acc = 0;
    for (int s = 0; s < Q; ++s) acc += t->c[s][0] * t->P[s][k];
    Phi0[k] = acc;
  }
  /* within-half sum W(k, k') over |z_k|, |z_k'| */
  for (int k = 0; k < V; ++k) {
    int kk = k % Q;
    qf sk = (k < Q) ? 1 : -1;
    for (int kp = 0; kp < V; ++kp) {
      int kq = kp % Q;
      qf skp = (kp < Q) ? 1 : -1;
      qf inner = 0;
      for (int l = 0; l <= Q - 2; ++l) {
        qf tail = 0;
        for (int s = l + 1; s <= Q - 1; ++s) tail += t->c[s][0] * t->P[s][kk];
        qf br = t->c[l][0] / s2pi * tail - (t->c[l][l] / t->c[l + 1][l + 1]) * t->P[l + 1][kk];
        inner += t->P[l][kq] * br;
      }
      qf pref = t->w[kk] * sk / (qf)p0;
      qf within = pref * (1 + sk * skp) / 2 * inner;
      qf cross = -pref * Phi0[kk] * Phi0[kq] / (2 * s2pi);
      /* The cross term is the sum of the same-half boundary term of
       * Eq. (dfpm), -omega(0) Phi_0 Phi_0' theta(p p'), and the delta term of
       * Eq. (deltaf_full), +(omega(0)/2) sigma sigma' Phi_0 Phi_0'. */
      qf delta = pref * sk * skp * Phi0[kk] * Phi0[kq] / (2 * s2pi);
      t->Kin[k * V + kp] = (double)within;
      t->Kd[k * V + kp] = (double)delta;
      t->K[k * V + kp] = (double)(within + cross);
    }
  }
  return 0;
}

/* Laguerre polynomials L_l(z) = sum_s (-1)^s binom(l, s) z^s / s!, orthonormal
 * on [0, inf) with omega(z) = exp(-z) (gamma_l = 1, Sec. IV.B.4), L_l(0) = 1.
 * c[l][s] holds the coefficient of z^s, as for the half-range Hermite family. */
static void lag_build_polys(orc_tables *t, int lmax) {
  memset(t->c, 0, sizeof(t->c));
  for (int l = 0; l <= lmax; ++l) {
    qf binom = 1, fact = 1;   /* binom(l, s), s! */
    for (int s = 0; s <= l; ++s) {
      if (s > 0) { binom = binom * (qf)(l - s + 1) / (qf)s; fact *= (qf)s; }
      t->c[l][s] = ((s % 2) ? -binom : binom) / fact;
    }
  }
}

/* Half-range Gauss-Laguerre rule and force matrix.
 * Nodes: the Q roots of L_Q (Sec. IV.B.1 with phi_l = L_l).
 * Weights: Eq. (wk_half), w_k = z_k / ((Q + 1)^2 L_{Q+1}(z_k)^2).
 * Force matrix: Eq. (hh_Kk_L), with Phi^Q_0(z_k) = sum_{s<Q} L_s(z_k)
 * (omega(0) = 1, L_s(0) = 1). */
static int build_half_laguerre(orc_tables *t, int Q, double p0) {
  t->quad = ORC_HALF_LAGUERRE; t->Q = Q; t->V = 2 * Q; t->H = Q; t->p0 = p0;
  lag_build_polys(t, Q + 1);
  qf r[ORC_QMAX + 2];
  family_roots(t, hh_eval, Q, 0.0Q, r);
  for (int k = 0; k < Q; ++k) {
    t->z[k] = r[k];
    qf lq1 = hh_eval(t, Q + 1, r[k]);
    t->w[k] = r[k] / ((qf)(Q + 1) * (qf)(Q + 1) * lq1 * lq1);
  }
  for (int l = 0; l <= Q + 1; ++l)
    for (int k = 0; k < Q; ++k) t->P[l][k] = hh_eval(t, l, t->z[k]);
  int V = 2 * Q;
  for (int k = 0; k < V; ++k) {
    int kk = k % Q;
    t->p[k] = (double)((k < Q ? 1 : -1) * (qf)p0 * t->z[kk]);
    t->wd[k] = (double)t->w[kk];
  }
  qf Phi0[ORC_QMAX];
  for (int k = 0; k < Q; ++k) {
    qf acc = 0;
    for (int s = 0; s < Q; ++s) acc += t->P[s][k];
    Phi0[k] = acc;
  }
  for (int k = 0; k < V; ++k) {
    int kk = k % Q;
    qf sk = (k < Q) ? 1 : -1;
    for (int kp = 0; kp < V; ++kp) {
      int kq = kp % Q;
      qf skp = (kp < Q) ? 1 : -1;
      qf inner = 0;
      for (int l = 0; l <= Q - 2; ++l) {
        qf tail = 0;
        for (int s = l + 1; s <= Q - 1; ++s) tail += t->P[s][kk];
        inner += t->P[l][kq] * tail;
      }
      qf pref = t->w[kk] * sk / (qf)p0;
      qf within = pref * (1 + sk * skp) / 2 * inner;
      qf cross = -pref * Phi0[kk] * Phi0[kq] / 2;
      /* the part of the cross term due to the delta term of Eq. (deltaf_full),
       * +(omega(0)/2) sigma sigma' Phi_0 Phi_0' (as in build_half) */
      qf delta = pref * sk * skp * Phi0[kk] * Phi0[kq] / 2;
      t->Kin[k * V + kp] = (double)within;
      t->Kd[k * V + kp] = (double)delta;
      t->K[k * V + kp] = (double)(within + cross);
    }
  }
  return 0;
}

/* Full-range Gauss-Hermite rule (Sec. IV.A): nodes are the roots of He_Q,
 * weights Eq. (H_wk) w_k = Q!/He_{Q+1}(z_k)^2, force matrix Eq. (H_Kk).
 * Only even Q (no node at p = 0, Sec. IV.A.1). */
static int build_full(orc_tables *t, int Q, double p0) {
  if (Q % 2) return -1;
  t->quad = ORC_FULL; t->Q = Q; t->V = Q; t->H = Q / 2; t->p0 = p0;
  qf r[ORC_QMAX + 2];
  qf B = 4.0Q + 3.0Q * sqrtq((qf)Q);
  family_roots(t, he_eval_t, Q, -B, r);
  qf fact = 1;
  for (int j = 2; j <= Q; ++j) fact *= j;
  int H = Q / 2;
  /* roots ascending: r[0..Q/2-1] negative, r[Q/2..] positive */
  qf zall[ORC_VMAX], wall[ORC_VMAX];
  for (int k = 0; k < H; ++k) {
    qf z = r[H + k];
    qf he = he_eval(Q + 1, z);
    t->z[k] = z;
    t->w[k] = fact / (he * he);
  }
  for (int k = 0; k < Q; ++k) {
    zall[k] = (k < H) ? t->z[k] : -t->z[k - H];
    wall[k] = t->w[k % H];
    t->p[k] = (double)((qf)p0 * zall[k]);
    t->wd[k] = (double)wall[k];
  }
  for (int l = 0; l <= Q + 1; ++l)
    for (int k = 0; k < H; ++k) t->P[l][k] = he_eval(l, t->z[k]);
  for (int k = 0; k < Q; ++k)
    for (int kp = 0; kp < Q; ++kp) {
      qf acc = 0, lf = 1;  /* lf = l! */
      for (int l = 0; l <= Q - 2; ++l) {
        if (l > 0) lf *= l;
        acc += he_eval(l + 1, zall[k]) * he_eval(l, zall[kp]) / lf;
      }
      t->K[k * Q + kp] = (double)(-wall[k] / (qf)p0 * acc);
      t->Kin[k * Q + kp] = t->K[k * Q + kp];
      t->Kd[k * Q + kp] = 0;
    }
  return 0;
}

/* Full-range Gauss-Hermite rule of Sec. IV.A for large Q, through the
 * orthonormal Hermite functions h_l = He_l / sqrt(l!), which obey
 * sqrt(l+1) h_{l+1} = z h_l - sqrt(l) h_{l-1} (a_l = 0, b_l = l, b_0 = 1):
 *   nodes   the roots of He_Q, by Sturm bisection of that Jacobi matrix;
 *   weights Eq. (H_wk), Q!/He_{Q+1}(z_k)^2 = 1/((Q+1) h_{Q+1}(z_k)^2);
 *   K       Eq. (H_Kk), with He_{l+1}(z_k) He_l(z_k')/l!
 *           = sqrt(l+1) h_{l+1}(z_k) h_l(z_k').
 * The same formulas as build_full; the monomial evaluation there costs
 * O(Q^4) and its roots O(Q^3) bisections, which does not reach Q = 500.
 * P is not kept (the full-range equilibrium evaluates He_l directly). */
static int g_qfmono = ORC_QFMONO;

static int build_full_rec(orc_tables *t, int Q, double p0) {
  if (Q % 2 || Q > ORC_VMAX) return -1;
  const int V = Q, H = Q / 2;
  t->quad = ORC_FULL; t->Q = Q; t->V = V; t->H = H; t->p0 = p0; t->rec = 1;
  for (int l = 0; l <= Q + 2; ++l) t->ra[l] = 0;
  t->rb[0] = 1;
  for (int l = 1; l <= Q + 3; ++l) t->rb[l] = (qf)l;
  qf *r = (qf *)malloc(sizeof(qf) * Q);
  qf *hz = (qf *)malloc(sizeof(qf) * (size_t)V * (Q + 2));
  qf *sq = (qf *)malloc(sizeof(qf) * (Q + 2));
  if (!r || !hz || !sq) { free(r); free(hz); free(sq); return -1; }
  const qf B = 4.0Q + 3.0Q * sqrtq((qf)Q);
  sturm_roots(t, Q, -B, B, r);   /* ascending: r[H..Q-1] are the positive roots */
  for (int k = 0; k < V; ++k) {
    const qf z = k < H ? r[H + k] : -r[k];
    rec_values(t, Q + 1, z, hz + (size_t)k * (Q + 2));
  }
  for (int k = 0; k < H; ++k) {
    const qf hq = hz[(size_t)k * (Q + 2) + Q + 1];
    t->z[k] = r[H + k];
    t->w[k] = 1 / ((qf)(Q + 1) * hq * hq);
  }
  for (int k = 0; k < V; ++k) {
    t->p[k] = (double)((k < H ? 1 : -1) * (qf)p0 * t->z[k % H]);
    t->wd[k] = (double)t->w[k % H];
  }
  for (int l = 0; l <= Q; ++l) sq[l] = sqrtq((qf)(l + 1));
  for (int k = 0; k < V; ++k) {
    const qf *hk = hz + (size_t)k * (Q + 2);
    const qf pref = -t->w[k % H] / (qf)p0;
    for (int kp = 0; kp < V; ++kp) {
      const qf *hp = hz + (size_t)kp * (Q + 2);
      qf acc = 0;
      for (int l = 0; l <= Q - 2; ++l) acc += sq[l] * hk[l + 1] * hp[l];
      t->K[k * V + kp] = (double)(pref * acc);
      t->Kin[k * V + kp] = t->K[k * V + kp];
      t->Kd[k * V + kp] = 0;
    }
  }
  free(r); free(hz); free(sq);
  return 0;
}

static int build_tables(orc_tables *t, int quad, int Q, double p0) {
  memset(t, 0, sizeof(*t));
  if (Q < 1 || Q > (quad == ORC_FULL ? ORC_VMAX : ORC_QMAX) || !(p0 > 0)) return -1;
  /* monomial constructions (Laguerre, and Hermite up to the switch) hold
   * c[l][s] up to l = Q + 1; the full-range roots cost O(Q^3) */
  if (quad == ORC_HALF_LAGUERRE && Q > ORC_QLAG) return -1;
  if (quad == ORC_HALF) return build_half(t, Q, p0);
  if (quad == ORC_FULL) {
    int r = Q > g_qfmono ? build_full_rec(t, Q, p0) : build_full(t, Q, p0);
    if (r) return r;
    qf lf[ORC_NEQ + 1];
    lf[0] = 1;
    for (int l = 1; l <= ORC_NEQ; ++l) lf[l] = lf[l - 1] * l;
    for (int l = 0; l < ORC_NEQ && l < Q; ++l)
      for (int k = 0; k < t->V; ++k) t->heq[l][k] = he_eval(l, k < t->H ? t->z[k] : -t->z[k - t->H]) / lf[l];
    for (int l = 0; l < ORC_NEQ; ++l)
      for (int j = 0; 2 * j <= l; ++j) t->gco[l][j] = lf[l] / (powq(2, j) * lf[j] * lf[l - 2 * j]);
    return 0;
  }
  if (quad == ORC_HALF_LAGUERRE) return build_half_laguerre(t, Q, p0);
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium                                                               */
/* ------------------------------------------------------------------------ */

/* Half-range coefficients of the Maxwellian g(u, T; p) of Eq. (feq), by
 * their definition G^+_l = int_0^inf dp g h_l(p/p0) and
 * G^-_l = int_0^inf dp g(-p) h_l(p/p0) (Sec. IV.B.3; h_l is the rule's
 * orthonormal family, half-range Hermite or Laguerre), written through the
 * monomial moments  int_0^inf dp g (p/p0)^s = (2 m T/p0^2)^{s/2} I_s(zeta),
 * zeta = u sqrt(m/2T) (zeta -> -zeta for G^-), where
 *   I_s(zeta) = pi^{-1/2} int_0^inf y^s exp(-(y - zeta)^2) dy,
 *   I_0 = erfc(-zeta)/2, I_1 = zeta I_0 + exp(-zeta^2)/(2 sqrt(pi)),
 *   I_s = zeta I_{s-1} + (s-1)/2 I_{s-2}   (integration by parts).
 * Then g_k = w_k sum_{l<=N} G^sigma_l h_l(z_k).  Evaluated in __float128;
 * valid for |zeta| up to about 3 (subsonic flow). */
static void eq_half(const orc_tables *t, int N, qf u, qf T, double *gout) {
  const qf m = 1;
  int Q = t->Q;
  qf scale = sqrtq(2 * m * T) / (qf)t->p0;
  qf zeta = u * sqrtq(m / (2 * T));
  for (int half = 0; half < 2; ++half) {
    qf zt = half == 0 ? zeta : -zeta;
    qf I[ORC_QMAX + 2], M[ORC_QMAX + 2];
    I[0] = erfcq(-zt) / 2;
    if (N >= 1) I[1] = zt * I[0] + expq(-zt * zt) / (2 * sqrtq(M_PIq));
    for (int s = 2; s <= N; ++s) I[s] = zt * I[s - 1] + (qf)(s - 1) / 2 * I[s - 2];
    qf sc = 1;
    for (int s = 0; s <= N; ++s) { M[s] = sc * I[s]; sc *= scale; }
    qf G[ORC_QMAX + 2];
    for (int l = 0; l <= N; ++l) {
      qf acc = 0;
      for (int s = 0; s <= l; ++s) acc += t->c[l][s] * M[s];
      G[l] = acc;
    }
    for (int k = 0; k < Q; ++k) {
      qf acc = 0;
      for (int l = 0; l <= N; ++l) acc += G[l] * t->P[l][k];
      gout[half * Q + k] = (double)(t->w[k] * acc);
    }
  }
}

/* Full-range: Eq. (H_gk), g_k = w_k sum_{l<=N} G_l He_l(z_k)/l!, with
 * G_l = sum_s l!/(2^s s! (l-2s)!) (mT/p0^2 - 1)^s (mu/p0)^{l-2s}.  The paper
 * prints the power of (mT/p0^2 - 1) as 2; the definition
 * G_l = int dp g He_l(p/p0) gives s (G_0 = 1 only with s). */
static void eq_full(const orc_tables *t, int N, qf u, qf T, double *gout) {
  const qf m = 1;
  qf p0 = (qf)t->p0;
  qf a = m * T / (p0 * p0) - 1, b = m * u / p0;
  qf G[ORC_QMAX + 2], lf[ORC_QMAX + 2], ap[ORC_NEQ], bp[ORC_NEQ];
  lf[0] = 1;
  for (int l = 1; l <= N + 1; ++l) lf[l] = lf[l - 1] * l;
  ap[0] = bp[0] = 1;
  for (int s = 1; s <= N; ++s) { ap[s] = ap[s - 1] * a; bp[s] = bp[s - 1] * b; }
  for (int l = 0; l <= N; ++l) {
    qf acc = 0;
    for (int s = 0; 2 * s <= l; ++s) acc += t->gco[l][s] * ap[s] * bp[l - 2 * s];
    G[l] = acc;
  }
  int H = t->H;
  for (int k = 0; k < t->V; ++k) {
    qf acc = 0;
    for (int l = 0; l <= N; ++l) acc += G[l] * t->heq[l][k];
    gout[k] = (double)(t->w[k % H] * acc);
  }
}

static void equilibrium(const orc_tables *t, int N, double u, double T, double *g) {
  if (t->quad == ORC_FULL) eq_full(t, N, (qf)u, (qf)T, g);
  else eq_half(t, N, (qf)u, (qf)T, g);   /* half-range Hermite or Laguerre */
}

/* ------------------------------------------------------------------------ */
/* Advection: WENO-5 and third-order upwind face fluxes                     */
/* ------------------------------------------------------------------------ */

/* WENO-5 weights of Eqs. (weno5_omega) and (weno_sigma) for the upwind
 * stencil (a, b, c, d, e) = (f_{i-2}, ..., f_{i+2}), without the customary
 * epsilon.  r_q = delta_q / sigma_q^2 in IEEE arithmetic; when one or more
 * r_q are infinite (a vanishing or underflowing sigma) the weights are the
 * ideal weights restricted to those q and renormalised, which is the limit
 * listed in Table (weno). */
static void weno5_weights(double a, double b, double c, double d, double e, double *om) {
  const double dl[3] = {0.1, 0.6, 0.3};
  double t1 = a - 2 * b + c, t2 = a - 4 * b + 3 * c;
  double s1 = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;
  t1 = b - 2 * c + d; t2 = b - d;
  double s2 = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;
  t1 = c - 2 * d + e; t2 = 3 * c - 4 * d + e;
  double s3 = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;
  double sg[3] = {s1, s2, s3}, r[3];
  int ninf = 0;
  for (int q = 0; q < 3; ++q) {
    r[q] = dl[q] / (sg[q] * sg[q]);
    if (isinf(r[q])) ++ninf;
  }
  if (ninf) {
    double den = 0;
    for (int q = 0; q < 3; ++q) if (isinf(r[q])) den += dl[q];
    for (int q = 0; q < 3; ++q) om[q] = isinf(r[q]) ? dl[q] / den : 0.0;
    return;
  }
  double rmax = fmax(r[0], fmax(r[1], r[2]));
  double sum = 0;
  for (int q = 0; q < 3; ++q) { r[q] /= rmax; sum += r[q]; }
  for (int q = 0; q < 3; ++q) om[q] = r[q] / sum;
}

/* Reconstructed face value for the upwind stencil (Eq. weno5_flux divided
 * by the velocity): interpolants F^1, F^2, F^3 weighted by omega-bar. */
static double weno5_face(double a, double b, double c, double d, double e) {
  double om[3];
  weno5_weights(a, b, c, d, e, om);
  double F1 = a / 3.0 - 7.0 / 6.0 * b + 11.0 / 6.0 * c;
  double F2 = -b / 6.0 + 5.0 / 6.0 * c + d / 3.0;
  double F3 = c / 3.0 + 5.0 / 6.0 * d - e / 6.0;
  return om[0] * F1 + om[1] * F2 + om[2] * F3;
}

/* Third-order upwind-biased face value: the central WENO-5 candidate F^2
 * alone, (-f_{i-1} + 5 f_i + 2 f_{i+1})/6.  (Not in the paper; it is the
 * linear scheme the small channel configuration asks for.) */
static double upwind3_face(double b, double c, double d) {
  return -b / 6.0 + 5.0 / 6.0 * c + d / 3.0;
}

/* ------------------------------------------------------------------------ */
/* Grid: Eqs. (x_eta) and (etai)                                             */
/* ------------------------------------------------------------------------ */

/* xf[j] = position of face j+1/2 for j = 0..Nx (paper's i = j), dx[i-1] for
 * cells i = 1..Nx, xc[i-1] cell centres x(eta_i). */
/* Faces x(eta_{i+1/2}), widths dx_i = x(eta_{i+1/2}) - x(eta_{i-1/2}) and
 * centres x(eta_i) of Eqs. (x_eta), (etai), evaluated in __float128 and
 * rounded once: the width of a cell next to a wall is the difference of two
 * faces near +-L/2, which in double would keep only about 12 digits of it. */
static void grid(const orc_channel *ch, double *xf, double *dx, double *xc) {
  int Nx = ch->Nx;
  qf L = ch->L, A = ch->A;
  qf *f = (qf *)malloc(sizeof(qf) * (Nx + 1));
  if (A == 0) {
    for (int j = 0; j <= Nx; ++j) f[j] = -L / 2 + L * j / Nx;
    for (int i = 1; i <= Nx; ++i) if (xc) xc[i - 1] = (double)(-L / 2 + L * (i - 0.5Q) / Nx);
  } else {
    qf deta = 2 * atanhq(A) / Nx;
    for (int j = 0; j <= Nx; ++j) f[j] = L / (2 * A) * tanhq((j + 0.5Q - (Nx + 1) / 2.0Q) * deta);
    for (int i = 1; i <= Nx; ++i)
      if (xc) xc[i - 1] = (double)(L / (2 * A) * tanhq((i - (Nx + 1) / 2.0Q) * deta));
  }
  for (int j = 0; j <= Nx; ++j) xf[j] = (double)f[j];
  for (int i = 1; i <= Nx; ++i) dx[i - 1] = (double)(f[i] - f[i - 1]);
  free(f);
}

/* ------------------------------------------------------------------------ */
/* Right-hand side L[y] of Eq. (L_def) with the diffuse-reflection closure   */
/* ------------------------------------------------------------------------ */

typedef struct {
  orc_channel ch;
  orc_tables t;
  int V, H, N, Nx, Ne;   /* Ne = Nx + 6: cells -2..Nx+3 (paper numbering)    */
  double *xf, *dx;
  double gwL[ORC_VMAX], gwR[ORC_VMAX];   /* wall equilibria (n = 1)        */
  int drop_delta;                        /* test-only switch, see below    */
} orc_ctx;

/* extended index of paper cell i (i = -2 .. Nx+3) */
#define EX(i) ((i) + 2)

static double face_value(const orc_ctx *c, const double *y, int k, int i) {
  /* face i+1/2 of node k, y = extended row of node k */
  const double v = c->t.p[k];
  if (c->ch.adv == ORC_UPWIND3) {
    if (v > 0) return upwind3_face(y[EX(i - 1)], y[EX(i)], y[EX(i + 1)]);
    return upwind3_face(y[EX(i + 2)], y[EX(i + 1)], y[EX(i)]);
  }
  if (v > 0) return weno5_face(y[EX(i - 2)], y[EX(i - 1)], y[EX(i)], y[EX(i + 1)], y[EX(i + 2)]);
  return weno5_face(y[EX(i + 3)], y[EX(i + 2)], y[EX(i + 1)], y[EX(i)], y[EX(i - 1)]);
}

/* Evaluate L for the state ye (f rows then chi rows, each V rows of Ne
 * extended cells; the interior i = 1..Nx must be filled, the ghosts are
 * written here).  Output Lf, Lc: V x Nx.  nw[0], nw[1]: wall densities.
 *
 * Order (Sec. IV.C.3): incoming ghosts by quadratic extrapolation; incoming
 * wall-face fluxes with the same reconstruction; wall density from zero net
 * mass flux, Eq. (nplus_def) with the emergent velocities p_k/m in the
 * denominator (cf. the continuous form in Sec. V.A); emergent ghosts
 * n_w g^w_k in all three ghost cells, Eq. (weno_populate), whose face flux
 * is then exactly v_k n_w g^w_k (Eq. weno_flux_eq) and is imposed as such;
 * then all face fluxes, moments, equilibrium, force and collision. */
static void rhs(orc_ctx *c, double *ye, double *Lf, double *Lc, double *nw) {
  const int V = c->V, H = c->H, Nx = c->Nx, Ne = c->Ne;
  const orc_channel *ch = &c->ch;
  const double m = 1.0;
  const int nfun = ch->Dt > 0 ? 2 : 1;
  double *yf = ye, *yc = ye + (size_t)V * Ne;

  /* incoming ghosts: left wall p < 0 (k >= H), right wall p > 0 (k < H) */
  for (int fn = 0; fn < nfun; ++fn) {
    double *y = fn ? yc : yf;
    for (int k = 0; k < V; ++k) {
      double *r = y + (size_t)k * Ne;
      if (k >= H) {
        r[EX(0)] = 3 * r[EX(1)] - 3 * r[EX(2)] + r[EX(3)];
        r[EX(-1)] = 6 * r[EX(1)] - 8 * r[EX(2)] + 3 * r[EX(3)];
        r[EX(-2)] = 10 * r[EX(1)] - 15 * r[EX(2)] + 6 * r[EX(3)]; /* unused */
      } else {
        r[EX(Nx + 1)] = 3 * r[EX(Nx)] - 3 * r[EX(Nx - 1)] + r[EX(Nx - 2)];
        r[EX(Nx + 2)] = 6 * r[EX(Nx)] - 8 * r[EX(Nx - 1)] + 3 * r[EX(Nx - 2)];
        r[EX(Nx + 3)] = 10 * r[EX(Nx)] - 15 * r[EX(Nx - 1)] + 6 * r[EX(Nx - 2)]; /* unused */
      }
    }
  }
  /* wall densities from the incoming fluxes of f */
  double inL = 0, inR = 0, denL = 0, denR = 0;
  for (int k = 0; k < V; ++k) {
    double v = c->t.p[k] / m;
    const double *r = yf + (size_t)k * Ne;
    if (k >= H) { inL += v * face_value(c, r, k, 0); denR += v * c->gwR[k]; }
    else { inR += v * face_value(c, r, k, Nx); denL += v * c->gwL[k]; }
  }
  double nL = -inL / denL, nR = -inR / denR;
  nw[0] = nL; nw[1] = nR;
  /* emergent ghosts */
  for (int k = 0; k < V; ++k) {
    double *rf = yf + (size_t)k * Ne, *rc = yc + (size_t)k * Ne;
    if (k < H) {
      double fw = nL * c->gwL[k];
      for (int i = -2; i <= 0; ++i) rf[EX(i)] = fw;
      if (nfun > 1) for (int i = -2; i <= 0; ++i) rc[EX(i)] = 0.5 * ch->Dt * ch->T_left * fw;
    } else {
      double fw = nR * c->gwR[k];
      for (int i = Nx + 1; i <= Nx + 3; ++i) rf[EX(i)] = fw;
      if (nfun > 1) for (int i = Nx + 1; i <= Nx + 3; ++i) rc[EX(i)] = 0.5 * ch->Dt * ch->T_right * fw;
    }
  }
  /* advection: L = -(F_{i+1/2} - F_{i-1/2}) / dx_i */
  double *F = (double *)malloc(sizeof(double) * (Nx + 1));
  for (int fn = 0; fn < nfun; ++fn) {
    double *y = fn ? yc : yf;
    double *Lo = fn ? Lc : Lf;
    for (int k = 0; k < V; ++k) {
      const double *r = y + (size_t)k * Ne;
      double v = c->t.p[k] / m;
      for (int i = 0; i <= Nx; ++i) {
        if (v > 0 && i == 0) F[i] = v * r[EX(0)];
        else if (v < 0 && i == Nx) F[i] = v * r[EX(Nx + 1)];
        else F[i] = v * face_value(c, r, k, i);
      }
      for (int i = 1; i <= Nx; ++i) Lo[(size_t)k * Nx + i - 1] = -(F[i] - F[i - 1]) / c->dx[i - 1];
    }
  }
  free(F);
  /* per cell: moments (Eq. fmoms), tau = Kn/n (Eq. tau), equilibrium,
   * force -F (K y)_k and BGK collision -(y - y_eq)/tau */
  const double Fx = m * ch->g;
  double geq[ORC_VMAX], fcell[ORC_VMAX], ccell[ORC_VMAX];
  for (int i = 1; i <= Nx; ++i) {
    double n = 0, mom = 0, e2 = 0, ech = 0;
    for (int k = 0; k < V; ++k) {
      fcell[k] = yf[(size_t)k * Ne + EX(i)];
      ccell[k] = nfun > 1 ? yc[(size_t)k * Ne + EX(i)] : 0.0;
      n += fcell[k];
      mom += c->t.p[k] * fcell[k];
    }
    double u = mom / (m * n);
    for (int k = 0; k < V; ++k) {
      double dp = c->t.p[k] - m * u;
      e2 += dp * dp * fcell[k] / m;
      ech += ccell[k];
    }
    double T = (e2 + 2 * ech) / ((1 + ch->Dt) * n);
    double inv_tau = isinf(ch->Kn) ? 0.0 : n / ch->Kn;
    if (inv_tau != 0.0) equilibrium(&c->t, c->N, u, T, geq);
    for (int k = 0; k < V; ++k) {
      double kf = 0, kc = 0;
      for (int kp = 0; kp < V; ++kp) {
        double Kkk = c->t.K[k * V + kp];
        if (c->drop_delta) Kkk -= c->t.Kd[k * V + kp];
        kf += Kkk * fcell[kp];
        kc += Kkk * ccell[kp];
      }
      size_t o = (size_t)k * Nx + i - 1;
      Lf[o] += -Fx * kf;
      if (inv_tau != 0.0) Lf[o] += -(fcell[k] - n * geq[k]) * inv_tau;
      if (nfun > 1) {
        Lc[o] += -Fx * kc;
        if (inv_tau != 0.0) Lc[o] += -(ccell[k] - 0.5 * ch->Dt * T * n * geq[k]) * inv_tau;
      }
    }
  }
}

static int ctx_init(orc_ctx *c, const orc_channel *ch) {
  memset(c, 0, sizeof(*c));
  c->ch = *ch;
  if (ch->Nx < 8 || ch->Q < 1 || ch->N < 0 || ch->N >= ch->Q) return -1;
  if (!(ch->dt > 0) || !(ch->L > 0) || !(ch->A >= 0 && ch->A < 1)) return -1;
  if (!(ch->Kn > 0) || !(ch->T_left > 0) || !(ch->T_right > 0)) return -1;
  if (ch->Dt != 0 && ch->Dt != 2) return -1;
  if (ch->adv != ORC_WENO5 && ch->adv != ORC_UPWIND3) return -1;
  if (build_tables(&c->t, ch->quad, ch->Q, ch->p0)) return -1;
  if (c->t.rec && ch->N > 20) return -1;   /* recurrence rules keep h_0..h_21 in monomials */
  if (c->t.quad == ORC_FULL && ch->N >= ORC_NEQ) return -1;   /* He_l tabulated for l <= 20 */
  c->V = c->t.V; c->H = c->t.H; c->N = ch->N; c->Nx = ch->Nx; c->Ne = ch->Nx + 6;
  c->xf = (double *)malloc(sizeof(double) * (ch->Nx + 1));
  c->dx = (double *)malloc(sizeof(double) * ch->Nx);
  grid(ch, c->xf, c->dx, NULL);
  /* wall equilibria: the discrete equilibrium at u = 0, T = T_w, n = 1 */
  equilibrium(&c->t, c->N, 0.0, ch->T_left, c->gwL);
  equilibrium(&c->t, c->N, 0.0, ch->T_right, c->gwR);
  return 0;
}

static void ctx_free(orc_ctx *c) { free(c->xf); free(c->dx); }

/* ------------------------------------------------------------------------ */
/* Public C entry points (called through ctypes by the tests)                */
/* ------------------------------------------------------------------------ */

/* Nodes p_k (V), weights w_k (V, mirrored nodes repeat the weight) and the
 * force matrix K (V x V, row-major).  Kin: the within-half sum term of
 * Eq. (hh_Kk); Kd: the part contributed by the delta term of Eq. (deltaf_full)
 * (both for the half-range rule; Kin = K and Kd = 0 for HLB).
 * Returns V, or -1 on bad arguments. */
int orc_tables_get(int quad, int Q, double p0, double *p, double *w, double *K,
                   double *Kin, double *Kd) {
  orc_tables *t = (orc_tables *)malloc(sizeof(orc_tables));
  if (build_tables(t, quad, Q, p0)) { free(t); return -1; }
  int V = t->V;
  if (p) memcpy(p, t->p, sizeof(double) * V);
  if (w) memcpy(w, t->wd, sizeof(double) * V);
  if (K) memcpy(K, t->K, sizeof(double) * V * V);
  if (Kin) memcpy(Kin, t->Kin, sizeof(double) * V * V);
  if (Kd) memcpy(Kd, t->Kd, sizeof(double) * V * V);
  free(t);
  return V;
}

/* Monomial coefficients of the orthonormal half-range Hermite polynomials
 * h_0 .. h_lmax, row l holding h_{l,0..l} (out: (lmax+1)^2, row stride lmax+1). */
int orc_hh_coeffs(int lmax, double *out) {
  if (lmax < 0 || lmax > ORC_CMAX - 1) return -1;
  orc_tables *t = (orc_tables *)malloc(sizeof(orc_tables));
  memset(t, 0, sizeof(*t));
  hh_build_polys(t, lmax);
  for (int l = 0; l <= lmax; ++l)
    for (int s = 0; s <= lmax; ++s) out[l * (lmax + 1) + s] = s <= l ? (double)t->c[l][s] : 0.0;
  free(t);
  return 0;
}

/* Test-only: half-range Hermite rules with Q above qmono (clamped to
 * 0 .. ORC_QMONO) are built from the recurrence; returns the previous value.
 * Lets the tests compare both constructions where both apply. */
/* Test hook: full-range rules with Q > qfmono come from the recurrence
 * construction (0 .. ORC_QFMONO); returns the previous value. */
int orc_set_qfmono(int qfmono) {
  int old = g_qfmono;
  g_qfmono = qfmono < 0 ? 0 : (qfmono > ORC_QFMONO ? ORC_QFMONO : qfmono);
  return old;
}

int orc_set_qmono(int qmono) {
  int old = g_qmono;
  g_qmono = qmono < 0 ? 0 : (qmono > ORC_QMONO ? ORC_QMONO : qmono);
  return old;
}

/* Discrete equilibrium f^eq_k = n g_k(u, T) of order N (V values). */
int orc_equilibrium(int quad, int Q, int N, double p0, double n, double u, double T, double *feq) {
  if (N < 0 || N >= Q || !(T > 0)) return -1;
  orc_tables *t = (orc_tables *)malloc(sizeof(orc_tables));
  if (build_tables(t, quad, Q, p0) || (t->rec && N > 20) || (t->quad == ORC_FULL && N >= ORC_NEQ)) {
    free(t);
    return -1;
  }
  equilibrium(t, N, u, T, feq);
  for (int k = 0; k < t->V; ++k) feq[k] *= n;
  int V = t->V;
  free(t);
  return V;
}

/* WENO-5 weights and face value for one upwind stencil (a..e). */
void orc_weno5(double a, double b, double c, double d, double e, double *om, double *face) {
  weno5_weights(a, b, c, d, e, om);
  *face = weno5_face(a, b, c, d, e);
}

/* Grid of Eqs. (x_eta)/(etai): faces xf (Nx+1), widths dx (Nx), centres xc (Nx). */
int orc_grid(const orc_channel *ch, double *xf, double *dx, double *xc) {
  if (ch->Nx < 1 || !(ch->A >= 0 && ch->A < 1)) return -1;
  grid(ch, xf, dx, xc);
  return 0;
}

/* Right-hand side L[y] for one state: f, chi are V x Nx (chi may be NULL
 * when Dt = 0); Lf, Lc likewise.  nw[2] receives the wall densities. */
int orc_rhs(const orc_channel *ch, const double *f, const double *chi, double *Lf, double *Lc,
            double *nw) {
  orc_ctx *c = (orc_ctx *)malloc(sizeof(orc_ctx));   /* the tables are large: heap, not stack */
  if (!c) return -1;
  if (ctx_init(c, ch)) { ctx_free(c); free(c); return -1; }
  int V = c->V, Nx = c->Nx, Ne = c->Ne;
  double *ye = (double *)calloc((size_t)2 * V * Ne, sizeof(double));
  double *Lct = (double *)calloc((size_t)V * Nx, sizeof(double));
  for (int k = 0; k < V; ++k)
    for (int i = 1; i <= Nx; ++i) {
      ye[(size_t)k * Ne + EX(i)] = f[(size_t)k * Nx + i - 1];
      if (ch->Dt > 0) ye[(size_t)(V + k) * Ne + EX(i)] = chi[(size_t)k * Nx + i - 1];
    }
  rhs(c, ye, Lf, Lct, nw);
  if (ch->Dt > 0 && Lc) memcpy(Lc, Lct, sizeof(double) * V * Nx);
  free(ye); free(Lct);
  ctx_free(c);
  free(c);
  return 0;
}

/* Advance f (and chi when Dt > 0) by nsteps TVD RK-3 steps, Eq. (rk3):
 *   y1 = y + dt L[y];  y2 = 3/4 y + 1/4 y1 + 1/4 dt L[y1];
 *   y_new = 1/3 y + 2/3 y2 + 2/3 dt L[y2].
 * f, chi: V x Nx, in and out.  nw[2] (may be NULL) receives the wall
 * densities of the last stage.  drop_delta != 0 removes the delta-term part
 * of the force matrix: a planted mistake used only by the negative control
 * test of the mass-bias argument of Sec. I. */
int orc_run(const orc_channel *ch, long nsteps, double *f, double *chi, double *nw, int drop_delta) {
  orc_ctx *c = (orc_ctx *)malloc(sizeof(orc_ctx));   /* the tables are large: heap, not stack */
  if (!c) return -1;
  if (ctx_init(c, ch)) { ctx_free(c); free(c); return -1; }
  c->drop_delta = drop_delta;
  const int V = c->V, Nx = c->Nx, Ne = c->Ne;
  const int nfun = ch->Dt > 0 ? 2 : 1;
  const double dt = ch->dt;
  size_t ns = (size_t)V * Nx;
  double *y0 = (double *)calloc(2 * ns, sizeof(double));
  double *ys = (double *)calloc(2 * ns, sizeof(double));
  double *L = (double *)calloc(2 * ns, sizeof(double));
  double *ye = (double *)calloc((size_t)2 * V * Ne, sizeof(double));
  double nwl[2] = {0, 0};
  memcpy(y0, f, sizeof(double) * ns);
  if (nfun > 1) memcpy(y0 + ns, chi, sizeof(double) * ns);
  for (long step = 0; step < nsteps; ++step) {
    memcpy(ys, y0, sizeof(double) * 2 * ns);
    for (int stage = 0; stage < 3; ++stage) {
      for (int fn = 0; fn < nfun; ++fn)
        for (int k = 0; k < V; ++k)
          for (int i = 1; i <= Nx; ++i)
            ye[(size_t)(fn * V + k) * Ne + EX(i)] = ys[fn * ns + (size_t)k * Nx + i - 1];
      memset(L, 0, sizeof(double) * 2 * ns);
      rhs(c, ye, L, L + ns, nwl);
      for (size_t j = 0; j < (size_t)nfun * ns; ++j) {
        double y = y0[j], s = ys[j], l = L[j];
        if (stage == 0) ys[j] = y + dt * l;
        else if (stage == 1) ys[j] = 0.75 * y + 0.25 * s + 0.25 * dt * l;
        else ys[j] = 1.0 / 3.0 * y + 2.0 / 3.0 * s + 2.0 / 3.0 * dt * l;
      }
    }
    memcpy(y0, ys, sizeof(double) * 2 * ns);
  }
  memcpy(f, y0, sizeof(double) * ns);
  if (nfun > 1) memcpy(chi, y0 + ns, sizeof(double) * ns);
  if (nw) { nw[0] = nwl[0]; nw[1] = nwl[1]; }
  free(y0); free(ys); free(L); free(ye);
  ctx_free(c);
  free(c);
  return 0;
}

/* Macroscopic moments of a state (Eq. fmoms, with chi's transverse energy):
 * n, u, T per cell (Nx each), using the channel's velocity set. */
int orc_moments(const orc_channel *ch, const double *f, const double *chi, double *n, double *u,
                double *T) {
  orc_tables *t = (orc_tables *)malloc(sizeof(orc_tables));
  if (build_tables(t, ch->quad, ch->Q, ch->p0)) { free(t); return -1; }
  int V = t->V, Nx = ch->Nx;
  for (int i = 0; i < Nx; ++i) {
    double nn = 0, mom = 0, e2 = 0, ech = 0;
    for (int k = 0; k < V; ++k) { nn += f[(size_t)k * Nx + i]; mom += t->p[k] * f[(size_t)k * Nx + i]; }
    double uu = mom / nn;
    for (int k = 0; k < V; ++k) {
      double dp = t->p[k] - uu;
      e2 += dp * dp * f[(size_t)k * Nx + i];
      if (ch->Dt > 0) ech += chi[(size_t)k * Nx + i];
    }
    n[i] = nn; u[i] = uu; T[i] = (e2 + 2 * ech) / ((1 + ch->Dt) * nn);
  }
  free(t);
  return 0;
}
