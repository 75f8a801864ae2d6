/*
 * hhlb.h -- C ABI of the MI355X (gfx950) library for the time step of the
 * half-range Gauss-Hermite lattice Boltzmann model with a force term
 * (Ambrus, Sofonea, Fournier, Blanco, arXiv:1708.03249).
 *
 * The library advances force-driven 1-D channels between diffuse-reflecting
 * walls.  Per time step (Sec. IV.C, Eq. rk3, three stages) it takes the
 * moments n, u, T of the populations f and of the reduced transverse-energy
 * function chi, builds the truncated half-range equilibrium (Sec. IV.B.3),
 * applies BGK relaxation with tau = Kn/n (Eq. tau), the force term as the
 * discrete momentum-derivative matrix with the delta term at p = 0
 * (Eq. hh_Kk_hh), WENO-5 or third-order upwind advection on a tanh-stretched
 * grid (Eqs. x_eta, etai, weno5_flux), and the diffuse-reflection closure
 * with zero net wall mass flux (Eq. nplus_def).
 *
 * Conventions: m = 1; F = m g with g the acceleration along x (the paper's
 * F = -m g_p); walls at x = -L/2 (left, temperature T_left) and x = +L/2
 * (right, T_right).  Velocity index k < V/2: positive momenta p_k = p0 z_k in
 * ascending order; k >= V/2: the mirrored p_k = -p_{k-V/2}.
 * Half-range HHLB(N;Q): V = 2Q.  Full-range HLB(N;Q) (Sec. IV.A, Q even): V = Q.
 *
 * Memory: the caller owns every device buffer (allocate them with any
 * allocator, e.g. torch.empty(..., device="cuda")); the library allocates no
 * device memory.  The library owns its host-side tables and frees them in
 * hhlb_destroy.  All device work is enqueued on the HIP stream given to
 * hhlb_create; outputs are valid once the caller synchronises that stream.
 *
 * Errors: every call returns an hhlb_status; no C++ exception crosses the ABI.
 * Arguments are checked before any side effect (HHLB_E_ARG leaves all state
 * unchanged).  hhlb_last_error() describes the last failure on this thread.
 */
#ifndef HHLB_H
#define HHLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hhlb_status;
enum {
  HHLB_OK = 0,
  HHLB_E_ARG = -1,          /* invalid argument; nothing was changed          */
  HHLB_E_UNSUPPORTED = -2,  /* valid model, but no kernel for this shape      */
  HHLB_E_HIP = -3,          /* a HIP runtime call failed (see last_error)      */
  HHLB_E_NOMEM = -4,        /* host allocation failed                          */
  HHLB_E_NUMERIC = -5,      /* table construction lost accuracy                */
  HHLB_E_STATE = -6         /* call out of order (e.g. no workspace bound)     */
};

/* Quadrature kind.
 *  HHLB_HALF_HERMITE:  half-range Gauss-Hermite, omega(z) = exp(-z^2/2)/sqrt(2 pi)
 *                      on each half axis, V = 2Q (HHLB(N;Q), Sec. IV.B).
 *  HHLB_FULL_HERMITE:  full-range Gauss-Hermite, V = Q, Q even (HLB(N;Q), Sec. IV.A).
 *  HHLB_HALF_LAGUERRE: half-range Gauss-Laguerre, omega(z) = exp(-z) on each half
 *                      axis, V = 2Q: nodes the roots of L_Q, weights Eq. (wk_half),
 *                      force matrix Eq. (hh_Kk_L).  FP64 form only. */
enum { HHLB_HALF_HERMITE = 0, HHLB_FULL_HERMITE = 1, HHLB_HALF_LAGUERRE = 2 };
enum { HHLB_WENO5 = 0, HHLB_UPWIND3 = 1 };              /* advection scheme  */
/* Arithmetic form of a solver (hhlb_create).
 *  HHLB_FP64:       every step in FP64; state stored as f_k in FP64.
 *  HHLB_MIXED_F32:  state stored in FP32 as f_k / w_k (w_k the node weight);
 *                   advection, collision, force contraction and the RK-3
 *                   combination in FP32; moment sums, the wall-density flux
 *                   balance (Eq. nplus_def) and the equilibrium coefficients
 *                   in FP64.  Half-range Gauss-Hermite model only.
 *  HHLB_MIXED_BF16, HHLB_MIXED_F16: as HHLB_MIXED_F32 with the force block
 *                   K y contracted on the matrix cores from BF16 / FP16
 *                   operands with FP32 accumulation. */
enum { HHLB_FP64 = 0, HHLB_MIXED_F32 = 1, HHLB_MIXED_BF16 = 2, HHLB_MIXED_F16 = 3 };

/* One channel, following the paper's statement of the problem (Sec. IV.D,
 * Sec. V.A): quadrature kind and order Q, equilibrium order N, grid, Kn,
 * force, wall temperatures and time step. */
typedef struct {
  int32_t quad;            /* HHLB_HALF_HERMITE, HHLB_FULL_HERMITE or HHLB_HALF_LAGUERRE */
  int32_t Q;               /* quadrature order (nodes per half axis for HHLB)        */
  int32_t N;               /* equilibrium order, 0 <= N < Q; N < 0 selects min(20,Q-1) */
  int32_t Nx;              /* number of cells, >= 8                                  */
  int32_t adv;             /* HHLB_WENO5 or HHLB_UPWIND3                             */
  int32_t transverse_dof;  /* Dt: 0 (the paper's 1-D gas, chi absent) or 2          */
  double L;                /* channel width, > 0                                     */
  double stretch_A;        /* tanh stretching A in [0,1); 0 = uniform cells          */
  double Kn;               /* Knudsen number > 0; +INFINITY = collisionless          */
  double g;                /* acceleration along x (F = m g)                         */
  double T_left, T_right;  /* wall temperatures > 0                                  */
  double p0;               /* momentum scale > 0                                     */
  double dt;               /* > 0: time step; < 0: CFL number |dt|, see hhlb_time_steps */
} hhlb_channel;

typedef struct hhlb_solver hhlb_solver;   /* opaque */

/* ---- host-only tables (FP64, no GPU needed) ------------------------------ */

/* Velocity set of Sec. IV.A.1 / IV.B.1: p_out[V] momenta p_k and w_out[V]
 * quadrature weights (a mirrored node repeats its weight).  Host pointers,
 * caller-owned, V entries each (V = 2Q half-range, Q full-range). */
hhlb_status hhlb_nodes(int32_t quad, int32_t Q, double p0, double *p_out, double *w_out);

/* Discrete momentum-derivative matrix, Eq. (hh_Kk_hh) (half-range) or
 * Eq. (H_Kk) (full-range): K_out[k*V + k'] (row-major, V*V host doubles),
 * (d f/d p)_k = sum_k' K[k][k'] f_k'. */
hhlb_status hhlb_force_matrix(int32_t quad, int32_t Q, double p0, double *K_out);

/* Truncated discrete equilibrium f^eq_k = n g_k(u, T) of order N,
 * Eq. (hh_gk) / Eq. (H_gk): feq_out[V] host doubles. */
hhlb_status hhlb_equilibrium(int32_t quad, int32_t Q, int32_t N, double p0, double n, double u,
                             double T, double *feq_out);

/* ---- solver -------------------------------------------------------------- */

/* Validate n_ch channels and build their tables on the host (extended
 * precision, rounded to double).  precision is one of the HHLB_FP64 /
 * HHLB_MIXED_* forms (a mixed form with a full-range channel is
 * HHLB_E_UNSUPPORTED).  Q <= 16 runs every kind in every form; Q > 16 runs
 * a node-parallel FP64 stage with N <= 20 for the half-range Gauss-Hermite
 * model up to Q = 256 and the full-range one up to Q = 512 (the HHLB(20;200)
 * and HLB(20;500) models of Sec. V.E); other shapes are HHLB_E_UNSUPPORTED.
 * hip_stream is a hipStream_t (NULL = default stream).  *out receives the
 * solver. */
hhlb_status hhlb_create(const hhlb_channel *channels, int32_t n_ch, int32_t precision,
                        void *hip_stream, hhlb_solver **out);

/* Bytes of device workspace the solver needs (tables, grid, three RK
 * state copies -- 8 bytes per population in FP64, 4 in the mixed forms --
 * and diagnostics). */
hhlb_status hhlb_workspace_bytes(const hhlb_solver *s, size_t *bytes);

/* Bind caller-owned device memory of at least hhlb_workspace_bytes bytes,
 * 256-byte aligned, and upload the tables (synchronises the stream once).
 * The memory must stay valid until hhlb_destroy or the next bind. */
hhlb_status hhlb_bind_workspace(hhlb_solver *s, void *dev_ptr);

/* State layout at the boundary: per channel c, V*Nx doubles starting at
 * off[c] (off has n_ch+1 entries, off[n_ch] = total), node-major
 * (k = 0..V-1), cell index fastest (i = 0..Nx-1, left to right).  f and chi
 * use the same layout in separate arrays.  Host pointer. */
hhlb_status hhlb_state_offsets(const hhlb_solver *s, int64_t *off);

/* The time step of each channel after resolving CFL requests:
 * dt = min(|cfl| * min_i dx_i / max_k |p_k/m|, Kn/2) when dt < 0 was given
 * (the Kn/2 cap keeps the stiff BGK term inside RK-3's stability region).
 * The force term is not bounded by this rule: dt |g| rho(K), rho(K) the
 * spectral radius of the force matrix, must stay well inside the stability
 * region too.  rho(K) grows quickly with Q for the half-range sets, whose
 * nodes crowd towards p = 0 (about 1.2e2 at Q = 40, 1.4e3 at Q = 200, 2.0e3
 * at Q = 256); for large Q give dt explicitly (the paper's 1e-4 at Q = 200).
 * dt_out: n_ch host doubles. */
hhlb_status hhlb_time_steps(const hhlb_solver *s, double *dt_out);

/* Copy a state in (device pointers, boundary layout, FP64; the mixed forms
 * round f_k / w_k to FP32).  chi_dev may be NULL only if every channel has
 * Dt = 0.  Asynchronous on the stream. */
hhlb_status hhlb_set_state(hhlb_solver *s, const double *f_dev, const double *chi_dev);

/* Set f_k = n0 g_k(u0, T0) in every cell and chi_k = (Dt/2) T0 f_k. */
hhlb_status hhlb_init_equilibrium(hhlb_solver *s, double n0, double u0, double T0);

/* Advance every channel by n_steps TVD RK-3 steps (Eq. rk3).  Asynchronous:
 * ordered after the work already on the solver's stream and before work
 * enqueued there later.  By default every stage kernel is launched directly
 * on the solver's stream; hhlb_set_graph_steps switches to HIP graph replay.
 * Returns HHLB_E_NUMERIC without stepping when the last hhlb_diagnostics
 * found non-finite populations (it waits for that diagnostics to finish). */
hhlb_status hhlb_step(hhlb_solver *s, int64_t n_steps);

/* Launch configuration of hhlb_step (the arithmetic is the same in every
 * configuration; results are bit-identical).
 *  graph_steps:   0 = direct kernel launches on the solver's stream; K > 0 =
 *                 replay of HIP graphs of K steps (see hhlb_set_graph_steps).
 *  class_streams: 0 = the model classes (channels sharing quadrature, Q, N,
 *                 scheme and Dt) advance one after the other on the solver's
 *                 stream; 1 = with direct launches, each class runs its steps
 *                 on an internal stream of its own (default priority), forked
 *                 from and joined back into the solver's stream by events
 *                 (graph replay always records the one-stream order).
 *  xcd_map:       1 = consecutive windows of a channel go to the same XCD
 *                 (the hardware deals blocks round-robin over the 8 XCDs);
 *                 0 = block b handles window b.
 *  waves_per_window: 2 = one wave per momentum half holds both f and chi of
 *                 a 64-cell window; 4 = one wave per half and function (FP64
 *                 half-range channels with chi; other classes keep 2).
 *  step_fusion:   1 = the three stages of a step (Eq. rk3) in one launch per
 *                 class, y^n and the stage state kept in registers over
 *                 windows with 9-cell halos (FP64 half-range Gauss-Hermite
 *                 classes; others keep one launch per stage); 0 = one launch
 *                 per stage.  The stages' arithmetic is the same; results
 *                 agree to rounding (the equilibrium's correction count is
 *                 chosen per window of cells).
 *  merge_classes: 0 = one launch per stage for each model class; 1 = one
 *                 launch per stage for all FP64 half-range classes that share
 *                 the functions (f, or f and chi) and the scheme, each block
 *                 taking one window of any of them; 2 = the same launch with
 *                 as many blocks as the GPU holds at once, each taking
 *                 windows in turn (persistent).  Other classes keep their own
 *                 launches.  Needs class_streams 0, step_fusion 0 and
 *                 waves_per_window 2 (HHLB_E_ARG otherwise).
 *  ms_per_step:   filled in by hhlb_autotune (the measured time). */
typedef struct {
  int32_t graph_steps;
  int32_t class_streams;
  int32_t xcd_map;
  int32_t waves_per_window;
  int32_t step_fusion;
  int32_t merge_classes;
  float ms_per_step;
} hhlb_tuning;

/* Set / read the launch configuration (defaults: 0, 0, 1, 2, 0). */
hhlb_status hhlb_set_tuning(hhlb_solver *s, const hhlb_tuning *t);
hhlb_status hhlb_get_tuning(const hhlb_solver *s, hhlb_tuning *t);

/* Autotuner: times trial_steps steps of every candidate configuration
 * (step_fusion in {0, 1} when a class has the fused-step kernel;
 * waves_per_window in {2, 4} when a class has the four-wave kernel; direct
 * launches with class_streams in {0, 1} -- 1 only when there are several
 * classes -- and graphs of 16 steps; each with xcd_map in {1, 0}; and
 * merge_classes in {1, 2} when some classes can share a launch) on the
 * solver's own channels and keeps the fastest; *best_out (may be NULL)
 * receives it.  The trials advance the state like hhlb_step (candidates x
 * (trial_steps + 1) steps) and synchronise the stream; call it in place of
 * warm-up steps. */
hhlb_status hhlb_autotune(hhlb_solver *s, int32_t trial_steps, hhlb_tuning *best_out);

/* Steps captured per HIP graph (default 0 = direct launches on the solver's
 * stream).  With steps_per_graph > 0, hhlb_step replays graphs of that many
 * steps (and a 1-step graph for the remainder) on an internal stream of
 * default priority, ordered against the solver's stream by events; results
 * are bit-identical to direct launches.  Graphs are rebuilt on the next step.
 * steps_per_graph < 0 is HHLB_E_ARG. */
hhlb_status hhlb_set_graph_steps(hhlb_solver *s, int32_t steps_per_graph);

/* Copy the state out (device pointers, boundary layout, FP64).  chi_dev may
 * be NULL; the chi of a channel with Dt = 0 reads as zero.  Asynchronous on
 * the stream. */
hhlb_status hhlb_get_state(const hhlb_solver *s, double *f_dev, double *chi_dev);

/* Moments of Eq. (fmoms) per cell, with chi's transverse energy in T:
 * n, u, T as device arrays of sum(Nx) doubles, channels concatenated. */
hhlb_status hhlb_moments(const hhlb_solver *s, double *n_dev, double *u_dev, double *T_dev);

/* Diagnostics (device pointers, any may be NULL): n_wall_dev[2*c+{0,1}]
 * wall densities n_+ (left) and n_- (right) of the last evaluated stage,
 * Eq. (nplus_def); mass_dev[c] = sum_i dx_i n_i (Eq. Ndef);
 * residual_dev[c] = max over f (and chi) of ||y1 - y||_inf / (dt ||y||_inf)
 * with y1 = y + dt L[y] one forward-Euler stage from the current state
 * (the state itself is unchanged; this costs one extra stage launch);
 * nonfinite_dev[0] = number of non-finite populations in the state.  The
 * non-finite count is also kept by the solver: the next hhlb_step returns
 * HHLB_E_NUMERIC (and advances nothing) if it was non-zero.
 * Asynchronous on the stream. */
hhlb_status hhlb_diagnostics(hhlb_solver *s, double *n_wall_dev, double *mass_dev, double *residual_dev,
                             int32_t *nonfinite_dev);

/* Kernel launches one hhlb_step of one RK stage issues (for profiling). */
hhlb_status hhlb_launch_info(const hhlb_solver *s, int32_t *launches_per_stage,
                             int64_t *windows_total);

/* The correction ladder of the half-range equilibrium of channel `channel`
 * (Sec. IV.B.3 evaluated by a change of variables: an M-point half-range
 * Gauss rule plus a Gauss-Legendre correction over [y0, 0]): counts[8]
 * point counts and reach[8] the largest |y0| each count was calibrated to
 * cover (host arrays).  A wave uses the smallest count whose reach covers
 * its largest |y0|.  Full-range channels are HHLB_E_UNSUPPORTED. */
hhlb_status hhlb_equilibrium_ladder(const hhlb_solver *s, int32_t channel, int32_t *counts, double *reach);

/* Number of equilibrium evaluations (a wavefront's 64 cells of one momentum
 * half in one stage; one cell for Q > 16) since hhlb_bind_workspace whose
 * largest |y0| = |u| sqrt(m/T) lay beyond the range the correction ladder
 * of the half-range equilibrium (Sec. IV.B.3, evaluated by a change of
 * variables) was calibrated for on the host (|y0| <= 1 for the Hermite
 * sets).  Such evaluations split the correction integral into 2, 4, .., 64
 * equal panels of the calibrated width (|y0| up to 64 times that range; the
 * large-Q path uses the smallest panel count that covers it).  Synchronises
 * the solver's stream; *count is a host int64. */
hhlb_status hhlb_wide_equilibrium_count(const hhlb_solver *s, int64_t *count);

/* Wait for the solver's streams, then release its host tables, graphs,
 * streams and events (the caller's workspace is not freed). */
hhlb_status hhlb_destroy(hhlb_solver *s);

/* Text of the last error on this thread ("" if none); valid until the next
 * call on the same thread. */
const char *hhlb_last_error(void);

/* ---- mixed-quadrature velocity space (App. A), homogeneous gas ---------- */

/* One axis of a direct-product velocity set (App. A.1): quadrature kind
 * (HHLB_HALF_HERMITE, HHLB_FULL_HERMITE or HHLB_HALF_LAGUERRE) and order Q,
 * equilibrium order N (0 <= N < Q, N <= 20) and momentum scale p0 > 0.
 * The axis has V_a = 2Q velocities (half range) or Q (full range, Q even);
 * V_a <= 32, and the product V = prod V_a <= 512 (else HHLB_E_UNSUPPORTED). */
typedef struct {
  int32_t quad, Q, N;
  double p0;
} hhlb_axis;

/* App. A.1: the product velocity set of d = 2 or 3 axes, velocity
 * v = (i V_y + j) V_z + k (x index slowest).  p_out[a*V + v] (d*V host
 * doubles, caller-owned) and w_out[V] (the product of the axis weights). */
hhlb_status hhlb_multi_nodes(const hhlb_axis *axes, int32_t d, double *p_out, double *w_out);

/* Bytes of device workspace hhlb_multi_rhs / hhlb_multi_step need for npts
 * points: the tables (uploaded by each call) and two RK stage copies of f. */
hhlb_status hhlb_multi_workspace_bytes(const hhlb_axis *axes, int32_t d, int64_t npts, size_t *bytes);

/* Right-hand side of Eq. (boltz_multi_k) without advection (App. A), for
 * npts independent points:
 *   L_v = - sum_a F_a (K_a f)_v - (f_v - feq_v) n / Kn,
 * K_a the axis' matrix of Eq. (H_Kk) / (hh_Kk), feq = n g_x g_y [g_z] the
 * product of the axes' truncated equilibria (Eqs. H_gk / hh_gk) at the
 * point's n, u, T (App. A.2; d n T = sum |p - u|^2 f, m = 1).
 * f_dev, L_dev: device FP64, point-major [npts][V]; F: d host doubles (the
 * acceleration); Kn > 0 or +INFINITY (no collisions); work_dev: device
 * workspace of at least hhlb_multi_workspace_bytes(..., npts) bytes.
 * Asynchronous on hip_stream (a hipStream_t, NULL = default stream). */
hhlb_status hhlb_multi_rhs(const hhlb_axis *axes, int32_t d, const double *f_dev, int64_t npts,
                           const double *F, double Kn, double *L_dev, void *work_dev, size_t work_bytes,
                           void *hip_stream);

/* n_steps TVD RK-3 steps (Eq. rk3) of the same system with time step dt,
 * in place on f_dev.  Arguments as for hhlb_multi_rhs. */
hhlb_status hhlb_multi_step(const hhlb_axis *axes, int32_t d, double *f_dev, int64_t npts, const double *F,
                            double Kn, double dt, int32_t n_steps, void *work_dev, size_t work_bytes,
                            void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * n_steps TVD RK-3 steps as hhlb_multi_step, with the tables and the two
 * RK stage copies in a static device array of the library instead of a
 * workspace argument.  The array holds 32 MiB on each GPU the library runs
 * on and stays allocated until the process ends; npts is limited to what
 * fits: 256-byte-aligned tables plus 2 x align256(npts * V * 8) bytes
 * (about 16000 points at V = 128).  A larger npts is HHLB_E_ARG before any
 * side effect.  The call itself allocates no device memory and calls no
 * allocating HIP routine; the first call with a new set of axes builds and
 * caches that set's host tables (host memory), which hhlb_multi_nodes can
 * do beforehand.  Every call on one GPU shares that GPU's array and leaves
 * its contents behind: calls that overlap on one GPU (other streams or
 * threads) race and must be ordered by the caller.  f_dev, F, Kn, dt,
 * n_steps and hip_stream as for hhlb_multi_step. */
hhlb_status hhlb_multi_step_noalloc(const hhlb_axis *axes, int32_t d, double *f_dev, int64_t npts,
                                    const double *F, double Kn, double dt, int32_t n_steps, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* HHLB_H */
