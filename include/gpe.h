/*
 * gpe.h -- C ABI of the MI355X hot path of the manifold-optimisation
 * ground-state solver for spin-F Bose-Einstein condensates
 * (Tian, Cai, Wu, Wen: "Ground states and their characterization of spin-F
 * Bose-Einstein condensates").
 *
 * Plain C: pointers and sizes only.  Every entry point returns a gpe_status;
 * no exception, abort or longjmp crosses the ABI.  On any status other than
 * GPE_OK, gpe_last_error(handle) returns a message describing the failure.
 *
 * Field layout (all device buffers).  A "field" holds the sqrt(h)-scaled
 * unknown X = (sqrt(h) phi_jl) of Sec. 3: K = 2F+1 component blocks in the
 * order l = F, F-1, ..., -F; each block is the grid in C order
 * [n_z][n_y][n_x] (x fastest, trailing axes absent in 1D/2D) of interleaved
 * complex numbers (re, im).  Grid node j on axis a sits at
 * lo[a] + j (hi[a]-lo[a])/n[a], j = 0..n[a]-1, with periodic wrap (Sec. 3).
 * Under this scaling the mass constraint is sum |X|^2 = 1 and the
 * magnetization constraint is sum_l l ||X_l||^2 = M (Sec. 3, discrete
 * constraints).
 *
 * Element types.  "c128" is complex double (16 bytes), "c64" complex float
 * (8 bytes).  Master fields (X, G, Xout, X_inout) are always c128.  The HVP
 * direction and result (Z, HZ) use the handle's work precision: c128 for a
 * GPE_FP64 handle, c64 for a GPE_MIXED handle.
 *
 * Ownership.  The caller allocates and owns every field buffer (for example
 * through PyTorch); the library only reads/writes it during the call and
 * never frees it.  The handle owns its workspace (device), plans and
 * caches; gpe_destroy releases them.
 *
 * Streams.  All device work of a handle is ordered on the HIP stream given
 * at creation (NULL = the default stream).  Calls that return host scalars
 * (E, gnorm, stats) synchronise that stream before returning; gpe_hvp and
 * gpe_retract with no scalar outputs do not block the host.
 *
 * Thread safety.  A handle must not be used from two host threads at once.
 */
#ifndef GPE_H
#define GPE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GPE_OK = 0,
  GPE_EINVAL = 1,    /* invalid argument or problem description */
  GPE_EDOMAIN = 2,   /* retraction argument outside its domain (Omega or S, Sec. 6) */
  GPE_EDEGEN = 3,    /* degenerate projection: u^T Gamma^2 u - M^2 <= 0 (Lemma 4.1) */
  GPE_ENUMERIC = 4,  /* NaN or Inf met in a reduction */
  GPE_ENOTCONV = 5,  /* solver stopped before reaching the tolerance */
  GPE_ENOMEM = 6,    /* device allocation failed */
  GPE_EHIP = 7       /* a HIP runtime call failed */
} gpe_status;

typedef enum { GPE_FP64 = 0, GPE_MIXED = 1 } gpe_precision;

/* Retractions of Sec. 6: projective (6.1), orthogonal (6.2), closed form (6.3). */
typedef enum { GPE_R1_PROJECTIVE = 1, GPE_R2_ORTHOGONAL = 2, GPE_R3_CLOSED = 3 } gpe_retraction;

/* Problem statement (Sec. 2 energy with mass and magnetization constraints,
 * Sec. 3 discretisation).  F in {1,2,3}; dim in {1,2,3}; each used n[a] is
 * one of 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, i.e.
 * 2^k or 3*2^k (Sec. 3 asks for an even n; the line transforms take radix
 * 8/4/2 stages and at most one radix-3 stage); unused axes are ignored;
 * lo[a] < hi[a]; beta = (beta0, beta1, beta2, beta3) (beta2 used for F >= 2,
 * beta3 for F = 3); Zeeman shifts p, q give b_l = -p l + q l^2; |M| < F.
 * A negative M is handled by the symmetry M <-> -M, phi_l <-> phi_-l (Sec. 4),
 * which the caller applies by reversing the component order. */
typedef struct gpe_problem {
  int F;
  int dim;
  int n[3];
  double lo[3];
  double hi[3];
  double beta[4];
  double p;
  double q;
  double M;
} gpe_problem;

typedef struct gpe_handle gpe_handle;

/* Options of newton_solve (Algorithm 1 on one mesh).  gpe_solve_opts_default
 * fills the values of Sec. 7.1 and the readings documented with the library. */
typedef struct gpe_solve_opts {
  double tol;            /* stop when ||grad|| <= tol (Sec. 7.1: 1e-6) */
  int maxit;             /* ARNT outer iterations (10000) */
  int retraction;        /* gpe_retraction (1) */
  double rgbb_tol;       /* RGBB warm start stops at ||grad|| <= rgbb_tol (1e-2) */
  int rgbb_maxit;        /* ... or after rgbb_maxit iterations (2000) */
  double rgbb_rho, rgbb_delta, rgbb_varrho, rgbb_step0; /* 1e-4, 0.2, 0.85, 0.1 */
  double eta1, eta2, gamma0, gamma1, gamma2, sigma_hat0;  /* 0.01 0.9 0.2 1 10 1 */
  double rho, delta, alpha0;   /* Armijo on the model: 1e-4, 0.2, 1 */
  int ls_max;            /* backtracks per search (30) */
  int cg_maxit;          /* most truncated-CG iterations per subproblem (500) */
  double cg_T, cg_theta; /* CG stop ||r|| <= min(T, ||g||^theta) ||g|| (0.1, 1) */
  int max_reject_streak; /* consecutive ARNT rejections that end the run (30) */
  double sigma_hat_min;  /* lower bound of sigma_hat (1e-8) */
  int verbose;           /* 1: one line per outer iteration on stderr */
  double time_limit;     /* seconds of wall clock after which the run stops unconverged (0: none) */
  int mg_levels;         /* cascadic multigrid (Algorithm 1, outer loop): number of coarser meshes,
                            each halving every axis of the same box (0: one mesh) */
  double mg_coarse_tol;  /* ||grad|| tolerance on the coarse meshes (Sec. 7.1: 1e-5) */
  /* FP64 polish of a GPE_MIXED solve: its HVPs and CG switch to FP64 for the
   * rest of the run once ||grad|| <= polish_tol (0: never), or once
   * polish_window outer iterations in a row have not halved the best ||grad||
   * (0: never).  No effect on a GPE_FP64 handle.  Both are off by default: on
   * problems whose slowness is physical (soft modes) FP64 only costs time. */
  double polish_tol;     /* default 0 */
  int polish_window;     /* default 0 */
  /* Cap of subproblem k's truncated CG chosen from ||grad|| (Sec. 7.1 says it is
   * adaptive in ||grad|| and leaves the rule open): min(cg_maxit,
   * ceil(cg_per_digit * log10(1 / min(T, ||g||^theta)))), a number of iterations
   * per decimal digit the CG residual must gain (80; 0: the fixed cap cg_maxit). */
  double cg_per_digit;
  /* Optional trace of the run (NULL: none): host array of trace_cap rows of
   * GPE_TRACE_COLS doubles.  One row when the RGBB warm start ends, then one
   * per ARNT outer iteration after its acceptance test, on the finest mesh
   * only; gpe_solve_stats.trace_len says how many rows were written (rows
   * beyond trace_cap are dropped).  Columns: seconds since the solve began,
   * E and ||grad|| at the current point (after the step, if accepted),
   * cumulative Hessian-vector products, sigma of the subproblem, the ratio
   * rho_k (NaN on the RGBB row, -Inf if no trial point was formed), truncated
   * CG iterations, CG stop reason (0 none, 1 curvature, 2 residual, 3 cap;
   * -1 on the RGBB row), the accepted step length t, accepted (1) or
   * rejected (0).  Ignored by gpe_batch_newton_solve. */
  double* trace;
  int trace_cap;
} gpe_solve_opts;

#define GPE_TRACE_COLS 10

typedef struct gpe_solve_stats {
  double E;              /* final energy (FP64) */
  double gnorm;          /* final ||grad|| (FP64) */
  int converged;
  int rgbb_iters;
  int outer;
  int cg_total;
  int hvp_calls;         /* all HVPs (CG plus model evaluations) */
  int ls_trials;
  int rejected;
  double t_total;        /* seconds, host wall clock incl. synchronisation */
  double t_rgbb;
  double t_arnt;
  double mass_err;       /* |mass - 1| of the result */
  double mag_err;        /* |magnetization - M| of the result */
  int mg_levels;         /* coarse meshes actually used */
  double t_coarse;       /* seconds spent on the coarse meshes (included in t_total) */
  int polish_at;         /* outer iteration at which the FP64 polish began (-1: none) */
  int trace_len;         /* rows written to gpe_solve_opts.trace */
} gpe_solve_stats;

/* Fill *opts with the defaults listed in gpe_solve_opts.  Never fails. */
void gpe_solve_opts_default(gpe_solve_opts* opts);

/* Create a handle for one problem.  V: n_x*n_y*n_z doubles, the potential
 * V(x_j) on the grid (C order, x fastest), in host memory or in device memory
 * of the current device (told apart with hipPointerGetAttributes); it is
 * copied, so the caller keeps ownership and may free it after the call.
 * precision: gpe_precision.  stream: hipStream_t (NULL = default stream).
 * Allocates all device workspace; *out receives the handle.
 * Errors: GPE_EINVAL (bad problem: F, dim, an unsupported n, |M| >= F, M < 0,
 * an empty box; NULL pointers), GPE_ENOMEM, GPE_EHIP. */
gpe_status gpe_create(const gpe_problem* prob, const double* V, int precision,
                      void* stream, gpe_handle** out);

/* Release the handle and its device memory (synchronises its stream).  NULL is a no-op. */
gpe_status gpe_destroy(gpe_handle* h);

/* Discrete energy E_h(X) of Sec. 3 (eq. discrete:energy), FP64 throughout.
 * X: device c128 field.  *E: host. */
gpe_status gpe_energy(gpe_handle* h, const void* X, double* E);

/* Gradient of E_h at X (Sec. 3).  riemannian = 0: Euclidean gradient for the
 * convention E(X + D) = E(X) + Re<G, D> + ...;  riemannian != 0: its
 * projection onto the tangent space at X (Sec. 4, Riemannian gradient,
 * projection of Lemma 4.1 with the measured Gram system).
 * X, G: device c128 fields (distinct).  E, gnorm: host, may be NULL; gnorm is
 * the 2-norm of the returned G.  FP64 throughout. */
gpe_status gpe_grad(gpe_handle* h, const void* X, void* G, int riemannian, double* E,
                    double* gnorm);

/* Fix the point X for subsequent gpe_hvp calls: copies X into the handle,
 * computes grad E(X) in FP64 and the multipliers (alpha_g, beta_g) of its
 * projection (Lemma 4.2), and in a GPE_MIXED handle a c64 copy of X.
 * X: device c128 field; the caller may modify it afterwards. */
gpe_status gpe_set_point(gpe_handle* h, const void* X);

/* Hessian-vector product at the set point u (Sec. 3 HVP formula; Lemma 4.2).
 * riemannian = 0: HZ = nabla^2 E_h(u)[Z] (R-linear in Z).
 * riemannian != 0: HZ = P_u(nabla^2 E_h(u)[Z] - alpha_g Z - beta_g Gamma Z + sigma Z),
 *   i.e. Hess E(u)[Z] + sigma Z for tangent Z: the Hessian of the regularised
 *   model m_k of Sec. 5 (eq. prob-sub).
 * Z, HZ: device fields in the work precision (c128 / c64), distinct buffers.
 * Requires a prior gpe_set_point.  Does not synchronise. */
gpe_status gpe_hvp(gpe_handle* h, const void* Z, void* HZ, int riemannian, double sigma);

/* Like gpe_hvp with riemannian != 0, and also returns kappa = <Z, HZ>
 * (real inner product, FP64 accumulation) on the host; synchronises. */
gpe_status gpe_hvp_dot(gpe_handle* h, const void* Z, void* HZ, double sigma, double* kappa);

/* Retraction Xout = psi(X + t Xi) onto {mass 1, magnetization M} (Sec. 6).
 * kind: gpe_retraction.  X, Xi, Xout: device c128 fields; Xout may alias X.
 * Component norms are reduced in FP64 on the device; the scalar solve
 * (root of h1 for the projective, of h2 for the orthogonal retraction) runs
 * in FP64 on the host; synchronises.
 * Errors: GPE_EDOMAIN if X + t Xi is outside the retraction's domain. */
gpe_status gpe_retract(gpe_handle* h, const void* X, const void* Xi, double t, int kind,
                       void* Xout);

/* Retraction with no allocation, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc): gpe_retract
 * without a handle, for the problem *prob (validated as gpe_create does).
 * Xout = psi(X + t Xi) by retraction `kind` (Xi may be NULL: psi(X)); X, Xi,
 * Xout: device c128 fields of that problem on the current device; Xout may
 * alias X.  Work is ordered on `stream` (hipStream_t, NULL = default) and
 * the call synchronises it (the scalar solve runs on the host).  The same
 * kernels as gpe_retract run, so the results are identical.
 * Scratch: a static device array of the library (about 345 KB per GPU, kept
 * until the process ends) holds the FP64 partial sums; it fits every problem
 * gpe_problem admits (a larger partial count is rejected with GPE_EINVAL).
 * The array is shared by all calls on one GPU, so calls on one GPU must not
 * overlap (from several host threads or streams): overlapping calls race.
 * Errors: as gpe_retract, plus GPE_EINVAL for an invalid problem; message in
 * gpe_last_error(NULL). */
gpe_status gpe_retract_noalloc(const gpe_problem* prob, const void* X, const void* Xi, double t, int kind,
                               void* Xout, void* stream);

/* Orthogonal projection onto the tangent space at X (Lemma 4.1, solved with
 * the measured Gram matrix of u and Gamma u): out = W - alpha X - beta Gamma X.
 * X, W, out: device c128 fields; out may alias W.  Synchronises. */
gpe_status gpe_project(gpe_handle* h, const void* X, const void* W, void* out);

/* Prolongation for the cascadic multigrid (Algorithm 1): Xf = Fourier
 * interpolant of Xc on the mesh of `fine`, which must have twice the points
 * of `coarse` on every axis of the same box (coarse node j = fine node 2j);
 * the sqrt(h) scaling is carried over (Xf = 2^{-d/2} interp(Xc)).  Xc, Xf:
 * device c128 fields of the two handles.  Uses the fine handle's scratch, so
 * a prior gpe_set_point on `fine` must be repeated.  Synchronises. */
gpe_status gpe_prolong(const gpe_handle* coarse, const void* Xc, gpe_handle* fine, void* Xf);

/* Mass and magnetization of a c128 field (FP64 reductions); synchronises. */
gpe_status gpe_constraints(gpe_handle* h, const void* X, double* mass, double* mag);

/* Ground state from X_inout (Algorithm 1 on one mesh: X0 is first mapped onto
 * the manifold by the projective retraction, then RGBB warm start, then the
 * modified ARNT with truncated CG, Sec. 5).  X_inout: device c128 field,
 * overwritten with the result.  opts may be NULL (defaults).  stats may be NULL.
 * In a GPE_MIXED handle the CG Hessian products and model evaluations run in
 * c64 with FP64 reductions; energies, gradients, retractions and the
 * acceptance ratio stay FP64.
 * Returns GPE_ENOTCONV (with X_inout holding the last iterate) if the
 * tolerance was not reached. */
gpe_status gpe_newton_solve(gpe_handle* h, void* X_inout, const gpe_solve_opts* opts,
                            gpe_solve_stats* stats);

/* Launch schedule chosen at creation: the fused x-pass kernel of the HVP
 * comes in up to 3 variants (rows of the grid per workgroup: half, default,
 * double); gpe_create times each on the handle's grid and keeps the fastest.
 * Writes the chosen variant and up to nvariants measured times in
 * microseconds (0 where a variant was not timed). */
gpe_status gpe_schedule(const gpe_handle* h, int* xpass_variant, float* variant_us, int nvariants);

/* Force the fused x pass's schedule variant (0 .. count-1; count from
 * gpe_schedule_count, 3 for n_x in {64, 96, 128, 256}, else 1) instead of the
 * autotuned one, e.g. to compare every variant's results.  All variants
 * compute the same products (they differ in rows per workgroup only).
 * Errors: GPE_EINVAL for a variant out of range (the schedule is unchanged). */
gpe_status gpe_set_schedule(gpe_handle* h, int xpass_variant);
gpe_status gpe_schedule_count(const gpe_handle* h, int* nvariants);

/* Per-kernel timing with HIP events recorded on the handle's stream around
 * every kernel launched by the library.  gpe_timing_enable(h, 1) clears the
 * record and starts recording; gpe_timing_read synchronises and writes, for
 * up to max kernel kinds, the kind's name (names: array of max char* slots
 * receiving pointers to static strings), launch count and total milliseconds;
 * it returns the number of kinds in *nkinds.  Recording costs two events per
 * launch; it is off by default. */
gpe_status gpe_timing_enable(gpe_handle* h, int enable);
gpe_status gpe_timing_read(gpe_handle* h, int max, const char** names, int* counts, double* ms,
                           int* nkinds);

/* Message of the last failure on this handle ("" if none).  For a NULL
 * handle, the message of the last failed gpe_create in this process. */
const char* gpe_last_error(const gpe_handle* h);

/* Library version string. */
const char* gpe_version(void);

/* ---------------------------------------------------------------- batches
 * Many independent problems (one spin F and dimension; grids, boxes,
 * potentials, interaction strengths and magnetizations may all differ)
 * solved together.  The driver of Algorithm 1 (Sec. 5) runs for every
 * problem in lock step: at each of its steps the device work of all problems
 * that are at the same step is one launch per kernel stage (the fused HVP x
 * pass, the axis passes, the finalize, the CG updates, the energy and
 * gradient, the retraction), and the scalars of all problems come back in one
 * copy with one synchronisation.  Each problem runs the iteration
 * gpe_newton_solve runs (the same readings, tolerances and counters); the
 * batched kernels may sum partial results in another order, so iteration
 * counts and the last digits of a problem's iterates can differ from a lone
 * solve's, while its result meets the same tolerance.
 * Every grid length of a batch must be a power of two from 16 to 512.
 */
typedef struct gpe_batch gpe_batch;

/* Create a batch of count problems (count >= 1); V_host[i] is problem i's
 * potential (host, n_i reals).  Every problem gets its own handle (see
 * gpe_batch_handle), all on `stream`.  The schedule of the batched fused x
 * pass (rows per workgroup) is autotuned here on the batch's own grids.
 * Errors: GPE_EINVAL (mixed F or dim, unsupported n, anything gpe_create
 * rejects), GPE_ENOMEM, GPE_EHIP; message in gpe_batch_last_error(NULL). */
gpe_status gpe_batch_create(const gpe_problem* probs, const double* const* V_host, int count, int precision,
                            void* stream, gpe_batch** out);
gpe_status gpe_batch_destroy(gpe_batch* b);
gpe_status gpe_batch_size(const gpe_batch* b, int* count);

/* Handle of problem i (owned by the batch: never gpe_destroy it).  Every
 * single-problem call works on it (energy, grad, set_point, retract, ...). */
gpe_status gpe_batch_handle(gpe_batch* b, int i, gpe_handle** h);

/* HVPs of every problem at its set point (gpe_set_point on its handle
 * first) in one batched pass: HZ[i] = Hess(Z[i]) as gpe_hvp with sigma[i]
 * (NULL: 0); Z, HZ in the work precision.  kappa (count values, host)
 * receives <Z_i, HZ_i> and the call synchronises; with kappa NULL no kappa
 * is formed and the launches stay queued on the batch's stream (no
 * synchronisation, like gpe_hvp). */
gpe_status gpe_batch_hvp(gpe_batch* b, const void* const* Z, void* const* HZ, int riemannian, const double* sigma,
                         double* kappa);

/* gpe_newton_solve for every problem (X_inout[i] c128, stats: count records
 * or NULL) in lock step.  opts->mg_levels > 0: the cascadic hierarchy of
 * Algorithm 1 for the whole batch, level by level: each coarser level is a
 * batch of its own (created and destroyed inside the call), solved in lock
 * step to mg_coarse_tol, and every problem's solution is prolonged to the
 * next finer level.  Fewer levels are used where a coarse axis would fall
 * below 16 points; stats[i].mg_levels says how many.  Returns GPE_OK when
 * every problem converged, GPE_ENOTCONV when some did not (their stats say
 * which), else the first problem's error.  t_total, t_rgbb and t_arnt of a
 * problem are wall-clock times of the whole batch's run up to that
 * problem's end of the phase; t_coarse is the coarse levels' time. */
gpe_status gpe_batch_newton_solve(gpe_batch* b, void* const* X_inout, const gpe_solve_opts* opts,
                                  gpe_solve_stats* stats);

/* Chosen schedule variant of the batched x pass and the measured
 * microseconds per variant (0 if not timed; a batch of one is not timed). */
gpe_status gpe_batch_schedule(const gpe_batch* b, int* xpass_variant, float* variant_us, int nvariants);

/* Message of the last failure on the batch; for NULL, of the last failed
 * gpe_batch_create. */
const char* gpe_batch_last_error(const gpe_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* GPE_H */
