/*
 * condmpc -- condensed-space interior-point method for linear-quadratic MPC on MI355X.
 *
 * C ABI of the hot path of Cole, Shin, Pacaud, Zavala and Anitescu, "Exploiting GPU/SIMD
 * architectures for solving linear-quadratic MPC problems" (arXiv 2209.13049):
 *   - Section 2, eqns. (sparse), (x_def), (dense): the problem data and the elimination of
 *     the states, which leaves a dense QP  min 1/2 v'Hv + h'v + h0  s.t.  Jv <= d  in the
 *     n = nu*N controls;
 *   - Section 3, eqns. (aug_KKT), (cond_KKT) and Algorithm 1: each interior-point iteration
 *     forms K = H + J' Sigma_s J, factors it by dense Cholesky and recovers the step.
 *
 * Conventions (all functions):
 *   - Matrices are row-major float64.  A host pointer is read or written synchronously; a
 *     "device" pointer must address MI355X memory that stays valid until the call's work on
 *     the stream has finished.
 *   - The library copies every input it keeps.  A cmpc_problem owns all device memory it
 *     allocates and releases it in cmpc_problem_destroy.
 *   - Work is issued on the HIP stream given at creation (NULL = the default stream).
 *   - Return value: 0 on success, a positive solver outcome, or a negative error code
 *     (below).  cmpc_last_error() gives a message for the calling thread's last error.
 *   - The library has no global state besides per-thread error messages and the SYRK
 *     tuning table (cmpc_batch_tune).
 *
 * Readings of the paper that the library implements (Algorithm 1 leaves them open):
 *   objective with 1/2 on every quadratic term; Q_f = Q when NULL; state bounds for
 *   t = 1..N only (x_0 is data); feedback gain Kfb = 0 (v = u) unless one is given;
 *   general data folded into extra stage components (cmpc_lq_desc); right-hand side
 *   -r1 + J'r2 - J'Sigma r3; start mu = 0.1, v = 0, s = max(d - Jv, 1e-2),
 *   lambda = z = mu/s; monotone barrier rule (kappa_eps = 10, kappa_mu = 0.2,
 *   theta_mu = 1.5, mu_min = tol/10); fraction-to-boundary step lengths alpha (v, s,
 *   lambda) and alpha_z (z) with tau = max(0.99, 1 - mu); z safeguarded into
 *   [mu/(1e10 s), 1e10 mu/s]; stop when max(|r1|, |r3|, |lambda - z|, |s z|) <= tol.
 */
#ifndef CONDMPC_H
#define CONDMPC_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define CMPC_OK 0               /* converged to tol */
#define CMPC_MAX_ITER 1         /* iteration limit reached */
#define CMPC_SMALL_STEP 2       /* step length below 1e-14 */
#define CMPC_ERR_INVALID (-1)   /* bad argument or dimensions */
#define CMPC_ERR_NONFINITE (-2) /* NaN or Inf where a finite number is required */
#define CMPC_ERR_X0_BOUNDS (-3) /* x0 violates a state bound (the t = 0 rows) */
#define CMPC_ERR_CHOLESKY (-4)  /* K not numerically positive definite */
#define CMPC_ERR_HIP (-5)       /* HIP runtime error */
#define CMPC_ERR_NOMEM (-6)     /* device allocation failed */

/* ---- precision of the SYRK that forms K (Section 3 forms K in one precision; the
 *      mixed modes are this library's extension, with FP64 Cholesky and FP64 iterative
 *      refinement against the exact K).  A mixed solve starts at the given level and moves
 *      up (BF16 -> FP32 -> FP64) after two refinement steps that fail to shrink the
 *      residual 10x, after a Cholesky breakdown (the iteration is redone), and straight to
 *      FP64 once mu < mu_switch. ---- */
#define CMPC_FP64 0
#define CMPC_FP32_SYRK 1
#define CMPC_BF16_SYRK 2

typedef struct cmpc_problem cmpc_problem;

/* Problem data of eqn. (sparse).  A: ns x ns, B: ns x nu, Q, Qf: ns x ns (Qf may be NULL ->
 * Q), R: nu x nu symmetric positive definite.  xl, xu: length ns; ul, uu: length nu; an
 * infinite bound drops its rows (+INFINITY upper, -INFINITY lower).  N >= 1 is the horizon
 * (the paper's T).  The general data may be NULL / 0 (absent): the cross weight S (ns x nu,
 * stage cost 1/2 [x;u]'[[Q, S], [S', R]][x;u], which must be positive semidefinite), the nc
 * rows gl <= E x_t + F u_t <= gu for t = 0..N-1 (E nc x ns, F nc x nu, gl, gu length nc),
 * the disturbance w (N x ns, row t is w_t of eqn. (dyn)) and the stabilising feedback Kfb
 * (nu x ns) of eqn. (K_constraint), u_t = Kfb x_t + v_t: the decision variable becomes v,
 * the input bounds rows of J (Kfb Gamma + I), and Gamma is formed with A + B Kfb.  All
 * pointers are host memory, or device memory if data_on_device is nonzero (the library
 * reads them once during cmpc_problem_create). */
typedef struct {
  int ns, nu, N;
  const double *A, *B, *Q, *R, *Qf;
  const double *xl, *xu, *ul, *uu;
  int nc;
  const double *S, *E, *F, *gl, *gu, *w, *Kfb;
  int data_on_device;
} cmpc_lq_desc;

typedef struct {
  double tol;        /* KKT tolerance of the stopping test (default 1e-8) */
  int max_iter;      /* iteration limit (default 200) */
  int precision;     /* CMPC_FP64 (default), CMPC_FP32_SYRK or CMPC_BF16_SYRK (start level) */
  int max_refine;    /* mixed modes: refinement steps per solve (default 5) */
  double mu_switch;  /* mixed modes: use the FP64 SYRK once mu < mu_switch (default 1e-6) */
  int check_every;   /* iterations queued ahead of the convergence flag the host has seen
                        (default 2); after convergence the queued ones exit at once */
  int profile;       /* nonzero: time the formation and the Cholesky factorisation of K in
                        every iteration with HIP events on the problem's stream (fills
                        ms_syrk, ms_form, ms_potrf) */
  int equilibrate;   /* factor S K S with S = diag(K)^-1/2 instead of K: 1 on, 0 off,
                        -1 (default) on in the mixed modes only */
  double refine_contract; /* mixed modes: a refinement step whose FP64 residual exceeds
                             refine_contract x the previous step's counts as not contracting
                             (default 0.1; two such steps move the SYRK one level up) */
  void (*log)(const char* line, void* ctx); /* cmpc_solve only, if not NULL: called from the
                             calling thread once per iteration with a one-line summary (barrier
                             parameter, KKT error and residual norms at the top of the
                             iteration, step lengths, SYRK precision level) and once at the
                             end; the line is valid during the call only (default NULL) */
  void* log_ctx;     /* passed to log unchanged */
  double warm_mu;    /* cmpc_solve_warm: barrier parameter of the warm start (default 1e-3) */
} cmpc_options;

typedef struct {
  int status;          /* CMPC_OK, CMPC_MAX_ITER, CMPC_SMALL_STEP or a negative error */
  int iters;           /* interior-point iterations taken */
  int precision_switch_iter; /* mixed modes: first FP64-SYRK iteration (-1 if none) */
  int refine_steps;    /* mixed modes: refinement steps over the solve */
  double obj;          /* 1/2 v'Hv + h'v + h0 at the returned iterate */
  double primal_res;   /* |Jv - d + s|_inf */
  double dual_res;     /* |Hv + h + J'lambda|_inf */
  double compl_res;    /* |s z|_inf */
  double mu;           /* final barrier parameter */
  double gap;          /* s'z */
  double ms_total;     /* wall time of the solve on the stream, milliseconds */
  double ms_syrk;      /* profile: time in the split-K SYRK kernel over the iterations */
  double ms_form;      /* profile: time forming K (SYRK + adding H, diag and partials) */
  double ms_potrf;     /* profile: time in the Cholesky factorisation over the iterations */
} cmpc_result;

/* Sizes and per-iteration work of a problem. */
typedef struct {
  int n, mx, m;              /* as cmpc_problem_dims */
  long long gamma_nnz;       /* structural nonzeros of Gamma: ns nu N(N+1)/2 (only the N blocks
                              * G_m = A^m B, ns nu N entries, are stored) */
  double syrk_flops;         /* algorithmic FLOPs of one formation of K: 2 per multiply-add
                                over the structural nonzeros, lower triangle with diagonal,
                                sum_t ns (t nu)(t nu + 1) */
  double potrf_flops;        /* n^3 / 3 */
  int syrk_workgroups;       /* launch size of the SYRK */
  int syrk_partial_slots;    /* partial tiles written by one SYRK */
  double device_bytes;       /* device memory held by the problem */
} cmpc_info;

/* Default options (values above). */
void cmpc_default_options(cmpc_options* opts);

/* Build the reduced problem of Section 2: G_k = A^k B (k = 0..N-1) and
 * H = Gamma'Qbar Gamma + Rbar.  Gamma itself is block Toeplitz (block (t, j) = G_{t-1-j},
 * t = 1..N, j < t) and is never stored: every pass over it reads the blocks G_k (the paper's
 * Section 6 proposes keeping the Jacobian implicitly this way).  stream: a hipStream_t
 * (NULL = default).  On success *out owns device memory of about
 * 8 (2 ns nu N + 3 (nu N)^2 + 8 ns N) bytes.  Errors: CMPC_ERR_INVALID (dimensions,
 * NULL data, ns nu N 8 >= 4 GiB), CMPC_ERR_NONFINITE, CMPC_ERR_NOMEM, CMPC_ERR_HIP. */
int cmpc_problem_create(const cmpc_lq_desc* desc, void* stream, cmpc_problem** out);

/* Release all device memory of the problem (NULL is ignored).  Synchronises its stream. */
void cmpc_problem_destroy(cmpc_problem* p);

/* Fill *info (host). */
int cmpc_problem_info(const cmpc_problem* p, cmpc_info* info);

/* n = nu N (size of K), mx = ns N (rows of Gamma), m = 2 mx + 2 n (inequality rows of
 * eqn. (dense) before rows with infinite bounds are dropped).  Any output may be NULL.  With
 * general data the rows of the input bounds (under a feedback) and of E x + F u are carried
 * as extra rows of each stage of Gamma: mx = (ns + nz) N with nz = (Kfb ? nu : 0) + nc. */
int cmpc_problem_dims(const cmpc_problem* p, int* n, int* mx, int* m);

/* Set the initial state (length ns; host or device pointer by on_device) and form the
 * x0-dependent data of eqn. (dense): c = (A^t x0)_{t=1..N}, h = Gamma'Qbar c,
 * h0 = 1/2 x0'Q x0 + 1/2 c'Qbar c, d = [xu - c; c - xl; uu; -ul].
 * Errors: CMPC_ERR_NONFINITE, CMPC_ERR_X0_BOUNDS (x0 outside [xl, xu]). */
int cmpc_set_x0(cmpc_problem* p, const double* x0, int on_device);

/* Run Algorithm 1 from the start point above.  opts NULL = defaults.  res may be NULL.
 * Returns the solver status (also in res->status). */
int cmpc_solve(cmpc_problem* p, const cmpc_options* opts, cmpc_result* res);

/* Algorithm 1 from a warm start, for receding-horizon control (Section 1: the controller
 * solves the problem again from each new measured state and applies the first input).  The
 * start controls are v0 (length nu N, host or device by on_device) or, with v0 = NULL, this
 * problem's last solution shifted one stage earlier with its last stage repeated (call
 * cmpc_set_x0 with the new state first); then s = max(d - J v0, 1e-2), lambda = z =
 * warm_mu / s and the barrier parameter starts at opts->warm_mu.  Everything else is
 * cmpc_solve.  Errors: CMPC_ERR_INVALID (no x0, or v0 = NULL before any solve, warm_mu not
 * positive), CMPC_ERR_NONFINITE (host v0). */
int cmpc_solve_warm(cmpc_problem* p, const cmpc_options* opts, const double* v0, int on_device,
                    cmpc_result* res);

/* Copy out the last solve's inputs u_t = Kfb x_t + v_t (= v without a feedback; length
 * nu N) and, if x != NULL, the states x_1..x_N = c + Gamma v (length ns N, the problem's own
 * ns).  Host or device pointers by on_device. */
int cmpc_get_solution(const cmpc_problem* p, double* u, double* x, int on_device);

/* Copy out the current iterate: v (n), s, lambda, z (m each, rows in the order
 * [x <= xu | -x <= -xl | u <= uu | -u <= -ul]; rows with an infinite bound hold
 * s = 1, lambda = z = 0).  Any output may be NULL. */
int cmpc_get_iterate(const cmpc_problem* p, double* v, double* s, double* lam, double* z,
                     int on_device);

/* Copy the reduced problem to host memory for checking: H (n x n), h (n), h0 (1),
 * d (m; rows with an infinite bound hold +INFINITY), c (mx), Gamma (mx x n dense,
 * row-major, structural zeros written).  Any output may be NULL. */
int cmpc_export_dense(const cmpc_problem* p, double* H, double* h, double* h0, double* d,
                      double* c, double* Gamma);

/* Form the condensed matrix of eqn. (cond_KKT), K = H + J' diag(sigma) J (the lower
 * triangle; the strict upper triangle of K is left unchanged), for a given sigma >= 0
 * (length m, device; sigma of a dropped row is ignored).  K: n x n device, leading
 * dimension n.  precision selects the SYRK arithmetic (CMPC_FP64, CMPC_FP32_SYRK,
 * CMPC_BF16_SYRK); H is always added in FP64. */
int cmpc_form_condensed(cmpc_problem* p, const double* sigma, double* K, int precision);

/* One Newton direction of Section 3 from a given interior iterate (all device pointers):
 * v (n); s, lam, z (m, s > 0 and z > 0 on kept rows); barrier mu > 0; fraction tau.
 * Writes p_v (n), p_s, p_lambda, p_z (m) and, to host memory, alphas[0] = alpha,
 * alphas[1] = alpha_z (fraction-to-boundary lengths).  Uses the FP64 path.
 * Errors: CMPC_ERR_CHOLESKY. */
int cmpc_newton_step(cmpc_problem* p, const double* v, const double* s, const double* lam,
                     const double* z, double mu, double tau, double* pv, double* ps,
                     double* plam, double* pz, double* alphas);

/* Dense Cholesky K = L L' in place (lower triangle of K, row-major, leading dimension
 * ld >= n, device).  The strict upper triangle is not referenced.  *info (host, may be
 * NULL) receives 0 or the 1-based column where a pivot was not positive, in which case
 * CMPC_ERR_CHOLESKY is returned.  stream: hipStream_t (NULL = default).  Synchronises
 * the stream. */
int cmpc_potrf(double* K, int n, int ld, void* stream, int* info);

/* cmpc_potrf for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same factorisation, kernels and
 * results, but its scratch (the 64 x 64 tile inverses and the status flags) is a fixed
 * file-scope device array of the library, about 2 MiB per device, held until the process ends; the
 * call allocates nothing.  n <= CMPC_POTRF_NOALLOC_MAX_N, else CMPC_ERR_INVALID.  The
 * stream's device (the current device if stream is NULL) is the one used.  Every call on a
 * device shares that device's array: calls that overlap on one device (other streams or
 * threads) race and must be serialised by the caller.  Synchronises the stream, as
 * cmpc_potrf does. */
#define CMPC_POTRF_NOALLOC_MAX_N 4096
int cmpc_potrf_noalloc(double* K, int n, int ld, void* stream, int* info);

/* Solve L L' x = b in place (b: n, device) with the factor from cmpc_potrf. */
int cmpc_potrs(const double* L, int n, int ld, double* b, void* stream);

/* ---- ragged batches (library extension: many independent instances of eqn. (sparse),
 *      each reduced as in Section 2 and solved by Algorithm 1, advanced together) ---- */
typedef struct cmpc_batch cmpc_batch;

/* Result of cmpc_batch_tune. */
typedef struct {
  int quantum;        /* chosen SYRK work quantum: least work of one split-K workgroup, in
                         row x 16-block units (a piece holds at least quantum / 16 rows) */
  int persistent;     /* chosen grid policy: 1 = persistent workgroups loop over each work
                         list, 0 = one workgroup per work item */
  int candidates;     /* settings timed */
  double syrk_us;     /* time of one batched formation of K with the chosen setting */
  double default_us;  /* the same with the default setting (quantum 12000, persistent) */
} cmpc_tune_report;

/* Create `count` problems from descs[0..count) as cmpc_problem_create does, and set
 * instance i's initial state from the host array x0s[i] (length ns of that instance) when
 * x0s != NULL and x0s[i] != NULL.  Instances may differ in ns, nu and N.  stream is used
 * for the set-up work and for calls on the instance handles; solves run on a stream of
 * the batch's own.  Errors as cmpc_problem_create and cmpc_set_x0 (the message names the
 * instance); on error nothing is kept. */
int cmpc_batch_create(int count, const cmpc_lq_desc* descs, const double* const* x0s,
                      void* stream, cmpc_batch** out);

/* Release the batch and all of its instances (NULL is ignored). */
void cmpc_batch_destroy(cmpc_batch* b);

/* Number of instances (0 for NULL). */
int cmpc_batch_size(const cmpc_batch* b);

/* Borrowed handle of instance i (0 <= i < size), valid until cmpc_batch_destroy: use it with
 * cmpc_set_x0, cmpc_get_solution, cmpc_get_iterate, cmpc_problem_info and the other
 * per-problem calls.  cmpc_problem_destroy on it does nothing.  NULL if i is out of range. */
cmpc_problem* cmpc_batch_instance(cmpc_batch* b, int i);

/* Run Algorithm 1 on every instance at once: each stage of an iteration is one launch over
 * a work list of (instance, block) items, one iteration is a captured HIP graph, and
 * instances that have stopped are skipped until all have.  opts as cmpc_solve (NULL =
 * defaults; tol, max_iter, precision, max_refine, mu_switch, check_every; profile is
 * ignored).  results[i] (may be NULL) receives instance i's outcome; ms_total is the time of
 * the whole batch.  Every instance needs an x0.  In FP64 every instance's iterates equal
 * bit for bit those of cmpc_solve on that instance (same tuning-table entry).  Returns 0 if
 * all converged, else a negative error of some instance or its positive outcome. */
int cmpc_batch_solve(cmpc_batch* b, const cmpc_options* opts, cmpc_result* results);

/* cmpc_batch_solve from warm starts (cmpc_solve_warm for every instance): instance i starts
 * from the controls v0s[i] (nu_i N_i doubles, host or device by on_device) or, where v0s or
 * v0s[i] is NULL, from its last solution shifted one stage; the barrier parameter starts at
 * opts->warm_mu.  Errors: CMPC_ERR_INVALID (a shift without an earlier solve, warm_mu not
 * positive). */
int cmpc_batch_solve_warm(cmpc_batch* b, const cmpc_options* opts, const double* const* v0s,
                          int on_device, cmpc_result* results);

/* Autotuner: time the batched formation of K at the start point of the method for each
 * candidate SYRK work quantum (3000 ... 96000) and grid policy, keep the fastest for this
 * batch and record it in the process-wide tuning table under (n, mx, precision) of every
 * instance.  Later solves (batched or single) of a problem with such a key build their
 * SYRK plan from the table.  precision: CMPC_FP64, CMPC_FP32_SYRK or CMPC_BF16_SYRK.  rep
 * may be NULL.
 * Every instance needs an x0; their iterates are overwritten. */
int cmpc_batch_tune(cmpc_batch* b, int precision, cmpc_tune_report* rep);

/* Tuning-table entry for (n, mx, precision): returns 0 and fills the outputs (may be NULL)
 * if present, 1 if not. */
int cmpc_tune_lookup(int n, int mx, int precision, int* quantum, int* persistent);

/* Record a tuning-table entry for (n, mx, precision), e.g. one that cmpc_tune_lookup returned
 * in an earlier process: later solves of a problem with that key build their SYRK plan with
 * this work quantum (>= 256) and grid policy (persistent 0 or 1).  A batch whose instances'
 * plans change this way rebuilds its work lists and graph at its next solve. */
int cmpc_tune_store(int n, int mx, int precision, int quantum, int persistent);

/* Empty the tuning table (plans are rebuilt with the defaults at the next solve). */
void cmpc_tune_clear(void);

/* ---- surrogate policy (library extension): a multilayer perceptron x0 -> u trained on
 *      the solutions of Algorithm 1, whose answers Algorithm 1 judges and replaces ---- */
#define CMPC_MLP_BF16 0       /* bfloat16 weights and activations, float32 accumulation */
#define CMPC_MLP_FP32 1       /* float32 throughout (test mode) */
#define CMPC_JUDGE_VIOLATION 1e-4  /* largest accepted bound violation of the states */
#define CMPC_JUDGE_GAP 1e-3        /* largest accepted (f(u) - LB) / |LB| */

typedef struct cmpc_mlp cmpc_mlp;

typedef struct {
  int batch;           /* minibatch rows, 1..4096 (default 512) */
  int epochs;          /* passes over the data (default 20) */
  float lr, lr_final;  /* AdamW step size, cosine-decayed from lr to lr_final (1e-3, 1e-5) */
  float beta1, beta2, eps;  /* AdamW moments (0.9, 0.999, 1e-8) */
  float weight_decay;  /* decoupled decay of the weight matrices, not the biases (1e-4) */
} cmpc_train_opts;

typedef struct {
  int count, accepted;            /* queries, answers the judge certified */
  int fallback_solved;            /* rejected answers replaced by a converged solve */
  int fallback_failed;            /* rejected answers whose solve did not converge */
  double max_violation_accepted;  /* largest state-bound violation among accepted answers */
  double max_gap_accepted;        /* largest certified relative gap among accepted answers */
  double ms_infer, ms_judge;      /* device time of the network and of the judge */
  double ms_fallback, ms_total;   /* host wall time of the fallback solves and of the call */
} cmpc_surrogate_report;

void cmpc_default_train_opts(cmpc_train_opts* opts);

/* Network for problem p (it must outlive the network): widths ns -> hidden (depth times,
 * GELU) -> nu N, initial parameters `init` (host float32, packed W_1, b_1, ..., W_L+1,
 * b_L+1, each W_l row-major d_l x d_(l-1)).  hidden % 64 == 0, 1 <= depth <= 16.  The judge
 * needs diagonal Q and Q_f, nu <= 64 and ns <= 3500; creation also forms the unconstrained
 * cost-to-go P_0 of the Riccati recursion (FP64) for the judge's lower bound. */
int cmpc_mlp_create(cmpc_problem* p, int hidden, int depth, int precision, const float* init,
                    cmpc_mlp** out);
void cmpc_mlp_destroy(cmpc_mlp* m);
long long cmpc_mlp_param_count(const cmpc_mlp* m);
/* Packed float32 master parameters (layout as `init`), host. */
int cmpc_mlp_get_params(const cmpc_mlp* m, float* params);
/* Replace the parameters and reset the AdamW state. */
int cmpc_mlp_set_params(cmpc_mlp* m, const float* params);

/* One forward and backward pass without an update: gradients of the mean squared error
 * between the network output and ustars over `count` rows (x0s: count x ns, ustars:
 * count x nu N, device float64; count <= 4096).  grads (host, packed like the parameters),
 * loss (host) and y (host, count x nu N unclipped outputs) may be NULL. */
int cmpc_mlp_gradients(cmpc_mlp* m, const double* x0s, const double* ustars, int count,
                       float* grads, double* loss, float* y);

/* AdamW training: epoch e visits rows order[e count + i] (host; NULL = 0..count-1) in
 * minibatches of opts->batch.  epoch_loss (host, epochs entries, may be NULL) receives the
 * mean loss of each epoch.  x0s, ustars: device float64. */
int cmpc_mlp_train(cmpc_mlp* m, const double* x0s, const double* ustars, int count,
                   const cmpc_train_opts* opts, const int* order, double* epoch_loss);

/* u (device, count x nu N) = network output clipped to the control bounds. */
int cmpc_mlp_predict(cmpc_mlp* m, const double* x0s, int count, double* u);

/* FP64 judge of answers u for initial states x0s (device): simulate eqn. (dyn), take the
 * largest bound violation of x_1..x_N, the objective f(u) and LB = 1/2 x0'P_0 x0 (the
 * unconstrained minimum h0 - 1/2 h'H^-1 h); accept iff violation <= CMPC_JUDGE_VIOLATION
 * and (f - LB)/|LB| <= CMPC_JUDGE_GAP.  Host outputs, each may be NULL. */
int cmpc_judge(cmpc_mlp* m, const double* x0s, const double* u, int count, int* accepted,
               double* violation, double* f, double* lb);

/* Answer `count` queries: predict, judge, and replace every rejected answer by the FP64
 * solve of Algorithm 1 from that x0 (on the network's problem, whose x0 is overwritten).
 * u: device (count x nu N); accepted: host (may be NULL); rep may be NULL.  Returns 0, or
 * CMPC_MAX_ITER if a fallback solve did not converge. */
/* How cmpc_surrogate_solve replaces rejected answers.  batch NULL (the default): one FP64
 * solve after another on the network's problem.  Otherwise the rejected queries are solved
 * together, count(batch) at a time, by cmpc_batch_solve on that batch, whose instances must
 * all be copies of the network's problem (same ns, nu, N; their x0 are overwritten; the
 * batch must outlive its use here).  warm != 0: each fallback solve starts from the
 * network's clipped answer (cmpc_solve_warm) instead of the cold start.
 * Errors: CMPC_ERR_INVALID (dimensions differ). */
int cmpc_mlp_set_fallback(cmpc_mlp* m, cmpc_batch* batch, int warm);

int cmpc_surrogate_solve(cmpc_mlp* m, const double* x0s, int count, double* u, int* accepted,
                         cmpc_surrogate_report* rep);

/* Message of the calling thread's last error ("" if none). */
const char* cmpc_last_error(void);

/* Text for a status code. */
const char* cmpc_status_str(int status);

#ifdef __cplusplus
}
#endif
#endif /* CONDMPC_H */
