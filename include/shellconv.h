/* libshellconv: Jacobian-vector product of the implicit-Coriolis IMEX step for Boussinesq
 * convection in a rotating spherical shell, on one AMD Instinct MI355X (gfx950).
 *
 * Method (Gonzalez Sembla, Rambert, Feudel, Tuckerman, Mathematics 13, 2113 (2025),
 * arXiv 2508.16635):
 *   - unknowns: toroidal and poloidal velocity potentials e, f and temperature T (Sec. 3.1),
 *     expanded in spherical harmonics Y_l^m (normalization N_l^m of Sec. 3.2) and sampled at
 *     the N Chebyshev-Gauss-Lobatto nodes in radius;
 *   - the IMEX Euler step B = (M - dt K)^{-1} (M + dt N) of Sec. 3.3 (eq:discrete) with the
 *     Coriolis force in K (Sec. 3.2, eq:impcor_e_final / eq:impcor_f_final), the drift term
 *     C i m M of a rotating wave (Sec. 3.4), boundary rows replaced (Sec. 3.1);
 *   - the Newton residual R = B_C(X) - X (Sec. 3.3, eq:finalrhs) and its Jacobian action
 *     (Sec. 3.3, eq:precond and the linearization rules; Sec. 3.4, the phase slot J that
 *     carries the drift-speed increment c).
 *
 * Packed state (real float64, Re/Im interleaved, the caller's layout everywhere):
 *     for field in (e, f, T); for k in 0..K (m = k*m0, K = min(M,L)/m0); for l in m..L;
 *     for j in 0..N-1 (x_j = cos(pi j/(N-1)), j = 0 at the outer sphere): (Re, Im)
 *   n_real = 6 * N * S,  S = sum_k (L - k*m0 + 1).
 *   The slots e, f at l = 0 and the Im parts at m = 0 carry no physical content: they are
 *   ignored on input and the step map sets them to 0 (so R = -X and jvp y = -v there).
 *
 * Ownership: every state/vector pointer is device memory owned by the caller, contiguous
 * in the packed layout (leading dimensions in elements).  The plan owns its tables, factors,
 * base-field caches and workspaces; they are allocated by sc_plan_create, never by sc_jvp.
 * Every call is asynchronous on the given stream (a hipStream_t; NULL = default stream),
 * except sc_layout and the host scalar of sc_newton_residual (documented synchronization).
 * A plan is not re-entrant across concurrent streams.
 *
 * Errors: every function returns 0 on success or one of SC_ERR_*; sc_last_error() gives a
 * thread-local message for the last nonzero return.  No C++ exception crosses the ABI.
 */
#ifndef SHELLCONV_H
#define SHELLCONV_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sc_plan sc_plan;

enum {
  SC_OK = 0,
  SC_ERR_ARG = 1,        /* bad size, leading dimension, phase slot or precision        */
  SC_ERR_STATE = 2,      /* jvp before factor/set_base, or a stale factor              */
  SC_ERR_NONFINITE = 3,  /* NaN/Inf in a residual norm                                  */
  SC_ERR_NOMEM = 4,      /* device allocation failed                                    */
  SC_ERR_HIP = 5,        /* HIP runtime error (message carries hipGetErrorString)       */
  SC_ERR_INTERNAL = 6
};

typedef enum { SC_FP64 = 0, SC_MIXED = 1 } sc_precision;

typedef struct {
  int L, M, m0, N;        /* truncations: l <= L, m in {0, m0, .., K m0}, N radial nodes (N >= 6) */
  double radius_ratio;    /* r_i / r_o (0.35 in Sec. 2.1); the gap r_o - r_i is 1            */
  double Ek, Ra, Pr, dt;  /* Ekman, Rayleigh (rotational), Prandtl (Sec. 2.1); step dt (Sec. 3.3) */
  int nr_phys, ntheta, nphi; /* 0 = dealiasing defaults: ceil(3N/2); smallest even >= (3L+1)/2;
                                smallest 2^a 3^b 5^c >= 3K+1 (Sec. 3.1)                      */
  int device;             /* HIP device ordinal                                              */
  int nvec_max;           /* largest batch passed to sc_jvp (0 = 16); sizes the workspaces   */
  int refine_fp64;        /* FP64 refinement passes after the FP64 solve (< 0: default 1)    */
  int refine_mixed;       /* SC_MIXED_SOLVE_FP32: FP64 refinement passes after the FP32 solve
                             (< 0: default 1); a pass is an FP64 residual and an FP64 correction
                             solve                                                             */
  int mixed_solve;        /* implicit solve of SC_MIXED: SC_MIXED_SOLVE_FP64 (0 = default) or
                             SC_MIXED_SOLVE_FP32                                               */
  int coriolis;           /* SC_CORIOLIS_IMPLICIT (0, default) or SC_CORIOLIS_EXPLICIT           */
  int graph_capture;      /* must be 0: capturing the Krylov chunks and batch calls into HIP
                             graphs is switched off in this build (a captured batch call crashed
                             the host process; cause not found); nonzero gives SC_ERR_ARG          */
} sc_params;

/* Treatment of the Coriolis force.  SC_CORIOLIS_IMPLICIT: in the implicit operator K, coupling
 * e_l with f_{l+-1} (Sec. 3.2, eq:impcor_e_final / eq:impcor_f_final): block-tridiagonal chains.
 * SC_CORIOLIS_EXPLICIT: the variant the paper compares against (Sec. 3.1, eq:expcor_e /
 * eq:expcor_f with the force of eq:defineFexp): -2 e_z x U is evaluated on the grid with the other
 * explicit forces, and K is block diagonal (the chain solves then run with zero couplings). */
enum { SC_CORIOLIS_IMPLICIT = 0, SC_CORIOLIS_EXPLICIT = 1 };

/* Implicit solve of the mixed path.  SC_MIXED_SOLVE_FP64: one solve with the FP64 factors (its
 * error, ~1e-11 relative, is far below that of the FP32 transforms).  SC_MIXED_SOLVE_FP32: a
 * solve with the FP32 factors, then refine_mixed FP64 refinement passes.  With factors resident
 * the solve streams them once per pass, so one FP64 pass costs less than an FP32 pass plus a
 * refinement pass. */
enum { SC_MIXED_SOLVE_FP64 = 1, SC_MIXED_SOLVE_FP32 = 2 };

typedef struct {
  long long n_real;       /* length of one packed state                                      */
  int L, M, m0, N, K, S;  /* truncations, number of m, number of (l, m) pairs                */
  int Np, ntheta, nphi;   /* physical grid: radial dealiasing nodes, Gauss-Legendre, sector  */
  int nvec_max;
} sc_layout_info;

/* Plan: grids, Legendre/radial tables and workspaces on params->device.  Sec. 3.1. */
int sc_plan_create(sc_plan** out, const sc_params* params);
int sc_plan_destroy(sc_plan* plan);
/* Sizes of the packed layout and of the physical grid (host only, no synchronization). */
int sc_layout(const sc_plan* plan, sc_layout_info* out);
/* Change Ra, Ek, dt.  A change of Ek or dt invalidates the factorization (SC_ERR_STATE from
 * step/jvp until sc_factor runs again); Ra enters only the explicit buoyancy (Sec. 3.2). */
int sc_set_params(sc_plan* plan, double Ra, double Ek, double dt);
/* Factor the implicit operator M - dt K (Sec. 3.2): per m, two block-tridiagonal chains in l
 * (odd-l e with even-l f, and the complement) with N x N complex blocks, plus one real block
 * per l for T.  Ruiz-equilibrated block LU in FP64 on the host, uploaded in FP64 and FP32.
 * Synchronizes the stream. */
int sc_factor(sc_plan* plan, void* stream);
/* One IMEX step x_next = B_C(x) with drift speed C (Sec. 3.3, eq:discrete; Sec. 3.4).
 * FP64 throughout, FP64 refinement of the implicit solve. */
int sc_step(sc_plan* plan, const double* x, double C, double* x_next, void* stream);
/* r = B_C(x) - x (Sec. 3.3, eq:finalrhs).  If rnorm_host is non-NULL the stream is
 * synchronized and ||r||_2 is stored there; SC_ERR_NONFINITE if it is not finite. */
int sc_newton_residual(sc_plan* plan, const double* x, double C, double* r, double* rnorm_host, void* stream);
/* For callers that cannot allocate or synchronize (code under HIP stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): r = B_C(x) - x as sc_newton_residual, and ||r||_2
 * written to the caller's device scalar *rnorm_dev on the stream (no host synchronization, no
 * finiteness check: a NaN or Inf is written as computed).  Calls no allocating routine.  The
 * norm's partial sums live in a fixed device array of the library (1024 doubles per GPU, held
 * until the process ends), so n_real is limited to 1024 * 8192 = 8388608 values (SC_ERR_ARG
 * beyond).  Every call on one GPU shares that array: calls that overlap on one GPU race.
 * x, r, rnorm_dev: device memory owned by the caller.  Errors as sc_newton_residual. */
int sc_newton_residual_noalloc(sc_plan* plan, const double* x, double C, double* r, double* rnorm_dev,
                               void* stream);
/* Base state of the Jacobian (Sec. 3.3, eq:precond: the linearized step B_U about U = x, with the
 * replacement rules of its linearization): caches the physical U, omega, grad T of x (FP64 and
 * FP32) and M x, the factor of the drift column c im M X.  J is the phase slot of Sec. 3.4 (the
 * index of the Im entry of one m > 0 coefficient, where the Krylov vectors carry the drift-speed
 * increment c) or -1 for no drift unknown. */
int sc_set_base(sc_plan* plan, const double* x, double C, long long J, void* stream);
/* Jacobian action y_i = (B_X - I)(u_i, c_i) on nvec vectors (Sec. 3.3 eq:precond, Sec. 3.4):
 * c_i = v_i[J], u_i = v_i with slot J zeroed; homogeneous boundary rows.
 * SC_FP64: every stage in FP64, refine_fp64 refinement passes.  SC_MIXED: Legendre transforms,
 * azimuthal transforms and products in FP32 with FP32 accumulation; FP64 radial operators and
 * right-hand side; the implicit solve as chosen by mixed_solve. */
int sc_jvp(sc_plan* plan, int nvec, const double* v, long long ldv, double* y, long long ldy,
           sc_precision prec, void* stream);
/* Newton-GMRES on R_C(X) = B_C(X) - X (+ forcing), Sec. 3.3 and 3.4: each Newton step solves
 * (B_X - I)(u, c) = R with restarted GMRES (Saad-Schultz) using sc_jvp in the chosen precision,
 * then X <- X - u, C <- C - c with c carried in slot J.  The Arnoldi steps run on the device:
 * classical Gram-Schmidt applied twice, the second pass of each basis vector delayed to the
 * next step and merged with that step's first pass (one pass over the basis for the dot
 * products and one for the update per step); the Hessenberg columns are finished there too.
 * The host reads them once per chunk of 8 steps, applies the Givens rotations and checks the
 * residual estimate, and solves the small triangular system once per cycle.
 * x: device state, updated in place; C: host drift speed, updated in place.  Synchronizes the
 * stream once per chunk of Krylov steps.  The Krylov basis is allocated by the first call (or a
 * call with a longer restart) and kept by the plan. */
typedef struct {
  double tol;             /* stop when ||R||_2 <= tol (absolute)                         */
  double gmres_tol;       /* relative tolerance of each GMRES solve                      */
  int restart;            /* GMRES restart length, 1..1024 (the basis holds restart + 1 vectors) */
  int max_newton;         /* Newton steps                                                */
  int max_matvec;         /* Jacobian actions per Newton step                            */
  int prec;               /* sc_precision of the Jacobian action                         */
  long long J;            /* phase slot (Im entry with m > 0), or -1: C stays fixed      */
  const double* forcing;  /* device vector added to the residual, or NULL                */
} sc_newton_opts;
typedef struct {
  int newton_steps, matvecs, converged;
  double rnorm[65];       /* ||R|| before each Newton step and at the end                 */
  int step_matvecs[64];   /* Jacobian actions per Newton step                            */
  double C;               /* final drift speed                                           */
} sc_newton_report;
int sc_newton(sc_plan* plan, double* x, double* C, const sc_newton_opts* opts, sc_newton_report* report,
              void* stream);

/* Stage profiler (tracing).  While enabled, every launch of the plan is bracketed by HIP
 * events on its stream; sc_profile_read synchronizes, returns per-stage total milliseconds
 * and launch counts (arrays of nstages entries indexed by SC_STAGE_*) and clears the record.
 * Events are created by the first enabling call, never inside step/jvp. */
enum {
  SC_STAGE_RADIAL_PREP = 0,     /* spectral profiles at the dealiasing nodes               */
  SC_STAGE_LEGENDRE_SYNTH = 1,  /* Legendre synthesis contractions                          */
  SC_STAGE_RING = 2,            /* azimuthal transforms and pointwise products             */
  SC_STAGE_LEGENDRE_ANAL = 3,   /* Legendre analysis contractions                          */
  SC_STAGE_PROJECT_RHS = 4,     /* curl projections and right-hand side                    */
  SC_STAGE_CHAIN_SOLVE = 5,     /* block-tridiagonal e/f solves                            */
  SC_STAGE_T_SOLVE = 6,         /* temperature solves                                      */
  SC_STAGE_RESIDUAL = 7,        /* FP64 residual of the implicit operator                  */
  SC_STAGE_AXPY = 8,            /* refinement update: folded into the correction solve, so no
                                   launch is recorded here; the index is kept stable     */
  SC_STAGE_FINALIZE = 9,        /* output assembly                                         */
  SC_NSTAGES = 10
};
int sc_profile(sc_plan* plan, int enable);
int sc_profile_read(sc_plan* plan, double* ms_total, long long* count, int nstages);
const char* sc_last_error(void);

/* Kernel choice by measurement (the transforms of Sec. 3.1 at this plan's L, M, m0, N).  Times
 * one transform pass (spectral prep, Legendre synthesis, azimuthal transforms and products,
 * Legendre analysis) of nvec zero vectors for every candidate, `reps` timed passes after one
 * untimed pass each, on `stream`, in three interleaved rounds over the ring candidates (each
 * kept at its fastest round), and keeps the fastest in the plan for later calls.  The pass
 * uses the Jacobian action's linearized products (the base fields of sc_set_base read at every
 * point) when a base state is set, else the nonlinear products of the step.  Candidates:
 *   ring kernel, per precision: the register-transform kernel (where N_phi = N1 N2 has one and
 *     N_phi >= 3K + 1) in each of its workgroup shapes (FP32: 32, 24 or 16 rings; FP64: 16 or 8;
 *     eight threads per ring) or the LDS kernel with 2^k rings per workgroup, k = 0 .. the LDS
 *     limit;
 *   analysis: the folded matrix-core kernel (where N_theta <= 256) or the plain batched GEMM,
 *     timed in FP32 and used by both precisions.
 * Results are unchanged in value (every candidate computes the same sums).  Allocates a
 * scratch vector block (nvec * n_real doubles) for the call.  nvec: 1 .. nvec_max; reps >= 1.
 * report (may be NULL): the choices (ring_fp32/ring_fp64: -1 - v register kernel of shape v,
 * k >= 0 LDS kernel with 2^k rings; anal_folded: 1 or 0), the best times in ms per pass and the number of
 * candidates timed.  Errors: SC_ERR_ARG (sizes), SC_ERR_STATE (the stage profiler is on).
 * Calls that overlap with other calls on the plan race. */
typedef struct {
  int ring_fp32, ring_fp64, anal_folded, ncand;
  double ms_fp32, ms_fp64;
  int linear_mode;        /* 1: timed with the Jacobian action's products (a base state was set) */
} sc_tune_report;
int sc_autotune(sc_plan* plan, int nvec, int reps, sc_tune_report* report, void* stream);

/* Kernel choices of a plan, set by hand (as sc_autotune sets them): ring_fp32 / ring_fp64 =
 * -1 - v for the register-transform ring kernel of shape v (where sc_autotune lists it as a
 * candidate; FP32: v = 0, 1, 2 for 32, 24, 16 rings per workgroup; FP64: v = 0, 1 for 16, 8),
 * k >= 0 for the LDS ring kernel with 2^k rings per workgroup up to the LDS limit;
 * anal_folded = 1 for the
 * folded analysis kernel (where N_theta <= 256), 0 for the batched GEMM.  Every choice computes
 * the same sums (Sec. 3.2, the transforms of the explicit forces); the choice only changes the
 * time.  Errors: SC_ERR_ARG (null plan, a choice this grid does not have; the plan is then
 * unchanged).  sc_get_kernels writes the choices in effect (any pointer may be NULL). */
int sc_set_kernels(sc_plan* plan, int ring_fp32, int ring_fp64, int anal_folded);
int sc_get_kernels(const sc_plan* plan, int* ring_fp32, int* ring_fp64, int* anal_folded);

/* Ragged batches of problems (plans of different L, M, m0, N, Ek, Ra, ...) on one device, e.g.
 * the points of a continuation in (Ra, Ek) (Sec. 4).  sc_batch_jvp applies the Jacobian of every
 * plan to its own vectors, each plan on a stream branch of its own forked from `stream` and
 * joined back into it, so that problems of uneven size share the device.
 *   plans: nplans >= 1 distinct plans on one device; the batch keeps the pointers, does not
 *          own the plans, and must be destroyed before them.
 *   nvec[i] (0..nvec_max of plan i), v[i], y[i]: vectors of plan i, leading dimension n_real.
 * Errors: SC_ERR_ARG (bad sizes, plans on different devices, a plan listed twice),
 * SC_ERR_STATE (a plan without factor or base, or with the stage profiler on).  Calls that
 * overlap on one batch, or that share a plan, race. */
typedef struct sc_batch sc_batch;
int sc_batch_create(sc_batch** out, sc_plan* const* plans, int nplans);
int sc_batch_destroy(sc_batch* batch);
int sc_batch_jvp(sc_batch* batch, const int* nvec, const double* const* v, double* const* y, sc_precision prec,
                 void* stream);

/* Newton-GMRES (as sc_newton, Sec. 3.3-3.4) on every plan of a batch at once, e.g. the points
 * of a continuation in (Ra, Ek): plan i runs on its own stream branch, forked from `stream`
 * and joined back into it, driven by a host thread of its own, so that the problems' Krylov
 * iterations share the device.  Arrays of nplans entries (the batch's plan order): x[i] (device,
 * n_real of plan i, updated in place), C[i] (host, in/out), opts[i], reports[i] (host, out).
 * Each plan needs sc_factor; sc_set_base is done by the solve itself.  Per-plan results are
 * those of sc_newton on that plan.  Errors: SC_ERR_ARG, SC_ERR_STATE as sc_newton (the first
 * failing plan's code and message; the other plans still finish), SC_ERR_STATE also for a plan
 * with the stage profiler on.  Calls that overlap on one batch, or that share a plan, race. */
int sc_batch_newton(sc_batch* batch, double* const* x, double* C, const sc_newton_opts* opts,
                    sc_newton_report* reports, void* stream);

/* Grid refinement (Sec. 4.2): y = x carried from the layout of `from` to that of `to` (same m0):
 * every (field, l, m) present in both is its interpolating Chebyshev polynomial evaluated at the
 * new Gauss-Lobatto nodes (the series padded with zeros); new degrees and orders are zero.
 * x: device, n_real of `from`; y: device, n_real of `to`.  Synchronizes the stream. */
int sc_interpolate(sc_plan* from, const double* x, sc_plan* to, double* y, void* stream);
/* Resolution check (Sec. 4.2): cheb_ratio = max |a_{N-1}| / max |a_n| over the Chebyshev
 * coefficients of every radial profile, sh_ratio = max |x at l = L| / max |x| (complex moduli).
 * A ratio above the threshold (1e-6 in the paper) means under-resolution.  Synchronizes. */
int sc_tail_ratios(sc_plan* plan, const double* x, double* cheb_ratio, double* sh_ratio, void* stream);

/* Continuation of a branch of rotating waves (Sec. 3.5, 3.6, 4.2), a session on one device:
 *   step size: p_new = p_i + alpha (p_i - p_{i-1}), alpha = (n_opt + 1)/(N_i + 1) with N_i the
 *     Newton steps of the last point (eq:new_Ra, eq:alpha_cont; a point that needed none counts
 *     as one); the first step from a single point is p_0 + dp_first from that point;
 *   prediction: the quadratic Lagrange weights of the last three parameter values at p_new,
 *     applied to the kept states and drift speeds (eq:lagrange);
 *   turning points (eq:tp_detection_Ra): with J the index of the largest |x| of the last point,
 *     if |dx_J/x_J| > gamma |dp/p| the component x_J is the independent variable instead
 *     (eq:quad_extra_Ra): p_new and the state come from the Lagrange weights in x_J;
 *   every point is a Newton-GMRES solve (sc_newton) at fixed p; if it fails, the step is taken
 *     again with alpha and gamma halved, up to max_retries times.
 * SC_CONT_RA: p = Ra.  SC_CONT_EK: p = log10 Ek with Ra = ra_coef Ek^(-1/3) (Sec. 4.2; 6.5 there);
 *   every new Ek re-factors the plan, and with refine_tol > 0 a converged point whose Chebyshev
 *   (or spherical-harmonic) tail ratio exceeds refine_tol grows N (or L and M) by refine_growth
 *   (N at most 64): a new plan is made, the kept points are carried over by sc_interpolate, the
 *   phase slot is chosen again (largest |Re| of an m = m0 entry of f or T) and the point is
 *   recomputed on the new grid.  The session owns the plans it makes; the caller's plan is not
 *   destroyed but its parameters change (Ra, Ek, factor) as the branch moves.
 * sc_cont_create: the plan must be factored; x0 (device) is converged first by Newton at the
 *   plan's parameters (SC_CONT_EK: at Ra = ra_coef Ek^(-1/3)); `first` (may be NULL) reports it.
 *   newton.J is the phase slot in the plan's layout; newton.forcing must be NULL.
 * sc_cont_step: one step; pt reports the point (converged = 0 if every retry failed; the branch
 *   is then unchanged).  sc_cont_layout / sc_cont_state: the layout of the current resolution
 *   and a copy of the newest state (device, n = its n_real) with its drift speed.
 * Errors: SC_ERR_ARG (options, sizes), SC_ERR_STATE (no factor, profiler on, no convergence at
 * the first point or after a refinement).  Every call synchronizes the stream. */
enum { SC_CONT_RA = 0, SC_CONT_EK = 1 };
typedef struct {
  int param;              /* SC_CONT_RA or SC_CONT_EK                                        */
  int n_opt;              /* target Newton steps per point (4..6 for Ra, 3 for Ek in the paper) */
  double gamma;           /* turning-point factor (10..100 for Ra, 400..500 for Ek)            */
  double ra_coef;         /* SC_CONT_EK: Ra = ra_coef Ek^(-1/3)                                */
  double refine_tol;      /* SC_CONT_EK: under-resolution threshold (<= 0: no refinement)      */
  double refine_growth;   /* resolution factor of a refinement (1.2 in the paper)              */
  int max_retries;        /* halvings of a failed step, 0..16                                  */
  sc_newton_opts newton;  /* Newton-GMRES of every point                                       */
} sc_cont_opts;
typedef struct {
  double param, Ra, Ek, C; /* the point: p, Rayleigh and Ekman numbers, drift speed            */
  double unorm;            /* ||x||_2                                                           */
  double cheb_ratio, sh_ratio; /* tail ratios (SC_CONT_EK with refinement)                     */
  int newton_steps, matvecs, converged, state_mode, refined, retries;
  int L, N;                /* resolution of the point                                           */
} sc_cont_point;
typedef struct sc_cont sc_cont;
int sc_cont_create(sc_cont** out, sc_plan* plan, const double* x0, double C0, const sc_cont_opts* opts,
                   sc_cont_point* first, void* stream);
int sc_cont_step(sc_cont* cont, double dp_first, sc_cont_point* pt, void* stream);
int sc_cont_layout(const sc_cont* cont, sc_layout_info* out);
int sc_cont_state(sc_cont* cont, double* x, long long n, double* C, void* stream);
int sc_cont_destroy(sc_cont* cont);

#ifdef __cplusplus
}
#endif
#endif
