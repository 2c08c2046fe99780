/*
 * rs.h -- C ABI of the MI355X sketch-and-project ridge solver (librs.so).
 *
 * Method: sketch-and-project with momentum for ridge regression
 * (RidgeSketch, arXiv 2105.05565, Alg. 2). The library solves
 *
 *     A x = b,  A = Z Z^T + lambda I                              (eq:Axb)
 *
 * in the primal form (Z = X^T, b = X^T y, x = w; eq:linear) or the dual form
 * (Z = X, b = y, x = alpha, w = X^T alpha; eq:duallinear). Each iteration k
 * draws a sketch S_k (subsample, Def. 4.2; count, Sec. 4.2; SubCount,
 * Def. 4.3), forms AS_k = Z (Z^T S_k) + lambda S_k, solves the tau x tau
 * system (S_k^T A S_k) delta = S_k^T r^k (eq:sketched_system) and applies
 *
 *     x^{k+1} = (1 + beta_k) x^k - beta_k x^{k-1} - gamma_k S_k delta
 *     r^{k+1} = (1 + beta_k) r^k - beta_k r^{k-1} - gamma_k AS_k delta
 *
 * (eq:res_update_mom), with residual r = A x - b (Sec. 3) and
 * x^{-1} = x^0 = 0. All device work runs on the stream the caller passes.
 *
 * Conventions for every entry point:
 *  - Return value: RS_OK (0) on success, a negative rs_status on error, or
 *    the positive warning RS_NOT_CONVERGED. No exception crosses the ABI.
 *    After an error, rs_last_error(handle) describes it (thread-local text
 *    for rs_create failures, readable through rs_last_error(NULL)).
 *  - Pointers marked "host" are CPU memory, "device" are HIP device memory
 *    of the current device; rs_matrix.mem says which one X and y are.
 *  - The library copies X and y at rs_create; the caller keeps ownership of
 *    every buffer it passes and may free them once the call returns.
 *  - Handles are not thread-safe: one thread at a time per handle.
 */
#ifndef RS_H
#define RS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rs_status;

enum {
  RS_OK = 0,
  RS_NOT_CONVERGED = 1,   /* warning: max_iter reached before tol */
  RS_EINVAL = -1,         /* bad argument: shape, tau > m, lambda <= 0, NaN, ... */
  RS_ENOMEM = -2,         /* allocation failed (device memory, or host buffers of a copy-out) */
  RS_EDEVICE = -3,        /* a HIP call failed */
  RS_ESINGULAR = -4,      /* non-positive Cholesky pivot on a nonzero sketch column */
  RS_EUNSUPPORTED = -5    /* option combination not built */
};

/* Matrix X (n x d). Dense layouts are row-major (ld = d) or column-major
 * (ld = n); CSR uses row_ptr[n + 1] (int64) and col_idx[nnz] (int32, sorted
 * within each row, no duplicates). */
enum { RS_DENSE_ROWMAJOR = 0, RS_DENSE_COLMAJOR = 1, RS_CSR = 2 };
enum { RS_F64 = 0, RS_F32 = 1 };
enum { RS_HOST = 0, RS_DEVICE = 1 };

typedef struct rs_matrix {
  int64_t n, d;
  int32_t layout;           /* RS_DENSE_ROWMAJOR | RS_DENSE_COLMAJOR | RS_CSR */
  int32_t dtype;            /* RS_F64 | RS_F32 (values of X) */
  const void* vals;         /* n*d values (dense) or nnz values (CSR) */
  const int64_t* row_ptr;   /* CSR only */
  const int32_t* col_idx;   /* CSR only */
  int64_t nnz;              /* CSR only */
  int32_t mem;              /* RS_HOST | RS_DEVICE: where vals/row_ptr/col_idx/y live */
} rs_matrix;

/* Form of the linear system (Sec. 2.1): AUTO picks primal when d <= n. */
enum { RS_FORM_AUTO = 0, RS_FORM_PRIMAL = 1, RS_FORM_DUAL = 2 };
/* Sketch distribution D (Sec. 4). GAUSSIAN (Def. 4.1): S_ic ~ N(0, 1) from Box-Muller on
 * Philox uniforms. SRHT (Def. 4.4): S^T = I_C H D / sqrt(tau m') with m' = 2^ceil(log2 m) and
 * A padded with zero rows, i.e. S_ic = d_i (-1)^popcount(i & C_c) / sqrt(tau m') for i < m, C a
 * uniform tau-subset of [0, m'). Both are dense (m x tau per sketch; products on FP64 MFMA),
 * for dense X or kernel ridge, FP64, uniform sampling, momentum schedules (not the
 * accelerated method). A heavily padded SRHT (m well below m') can draw linearly dependent
 * columns; the factorisation then reports RS_ESINGULAR. */
enum { RS_SKETCH_SUBSAMPLE = 0, RS_SKETCH_COUNT = 1, RS_SKETCH_SUBCOUNT = 2, RS_SKETCH_GAUSSIAN = 3,
       RS_SKETCH_SRHT = 4 };
/* Momentum schedule (Sec. 6, Sec. 8.1):
 *  NONE      gamma = 1, beta = 0 (Alg. 1)
 *  CONSTANT  gamma = opts.gamma, beta = opts.beta (0.5 in the paper's comparison)
 *  HEURISTIC gamma = 1, beta_k = min(beta_max, 1 - (2 - eta) / ((k+1)(1 - eta) + 1))
 *            (eq:parametersheurististic)
 *  THEORY    increasing momentum of eq:parameterswitchtheory in the iterate-averaging
 *            parameters of Thm 6.2: eta_k = opts.eta before the switch and 1 from it on,
 *            zeta_k = (1 / eta_k) sum_{t<k} eta_t (1 - eta_t) (eq:zeta_kaptheo),
 *            gamma_k = eta_k / (zeta_{k+1} + 1), beta_k = zeta_k / (zeta_{k+1} + 1)
 *            (eq:etalambdatogammbetagen). The switch is the first k at which the
 *            constant-eta momentum of Cor 6.3, 1 - (2 - eta) / ((k+1)(1 - eta) + 1),
 *            reaches opts.beta_max (k = 201 for eta 0.995, beta_max 0.5); no switch when
 *            eta >= 1 or beta_max >= 1. Needs 0 < eta <= 1 (RS_EINVAL otherwise). */
enum { RS_MOMENTUM_NONE = 0, RS_MOMENTUM_CONSTANT = 1, RS_MOMENTUM_HEURISTIC = 2, RS_MOMENTUM_THEORY = 3 };
/* Arithmetic of the AS products: FP64 throughout, or BF16 products with FP32
 * accumulation and an FP64 Cholesky plus a periodic FP64 residual refresh. */
enum { RS_PREC_FP64 = 0, RS_PREC_MIXED_BF16 = 1 };

typedef struct rs_options {
  int32_t form;             /* RS_FORM_* */
  int32_t sketch;           /* RS_SKETCH_* */
  int32_t tau;              /* sketch size, 1 <= tau <= m */
  int32_t subcount_k;       /* SubCount sum size k; 0 = the paper's rule (k = 10 if 10 tau <= m,
                               else floor(m / tau)); s = k tau must be <= m */
  int32_t momentum;         /* RS_MOMENTUM_* */
  int32_t precision;        /* RS_PREC_* */
  double gamma, beta;       /* CONSTANT schedule */
  double eta, beta_max;     /* HEURISTIC and THEORY schedules (defaults 0.995, 0.5) */
  double tol;               /* stop when ||r^k|| / ||r^0|| <= tol (default 1e-6) */
  int64_t max_iter;         /* iteration cap (default 100000) */
  uint64_t seed;            /* Philox key word 0 */
  uint64_t problem_id;      /* Philox key word 1 */
  int32_t refresh_every;    /* mixed precision: FP64 recomputation of r every R iterations (default 20) */
  int32_t lookahead;        /* sketches drawn and factorised ahead per batch; 0 = library choice */
  int32_t profile;          /* 0: off; 1: batch-level HIP-event timing; 2: every launch (rs_get_profile);
                               3: the AS products of each batch only (the fewest events in the stream) */
  void* stream;             /* hipStream_t for all work; NULL = the default stream (a batch
                               then creates its own stream, since graph capture needs one) */
  int32_t graph_iters;      /* batch: iterations per captured HIP graph; 0 = 8, < 0 = no graph */
  int32_t autotune;         /* batch: 1 = time candidate launch shapes at rs_batch_create */
  int32_t sampler;          /* RS_SAMPLER_* coordinate proposal of the subsample sketch */
  int32_t trace_every;      /* > 0: record (features, credits) every that many iterations */
  int32_t trace_capacity;   /* records kept (0 = 1024); later ones are dropped */
  int32_t sparse_route;     /* CSR count / SubCount products: RS_ROUTE_* */
  int32_t pipeline;         /* 1 (default): prepare the next lookahead batch (sketches, AS,
                               G^{-1}) on a second stream of default priority while the current
                               batch iterates, in a second set of batch buffers (twice their
                               memory); 0: one stream. Off for the learned sampler, whose
                               proposal reads the iterate. */
  int32_t accelerated;      /* 1: the accelerated method (Alg. 3) with parameters accel_mu,
                               accel_nu instead of the momentum schedule; FP64, uniform
                               sampling. 0 (default): Alg. 2 with the momentum schedule. */
  double accel_mu, accel_nu; /* Alg. 3: 0 < mu <= 1 and 1 <= nu <= 1 / mu (defaults 1, 1: the
                               iterates of Alg. 1); beta = 1 - sqrt(mu / nu), gamma =
                               sqrt(1 / (mu nu)), alpha = 1 / (1 + sqrt(nu / mu)). The state
                               (rs_get_state) is w, v, r_w, r_v; the weights are w; the stop
                               test and the history use ||r_v^k|| / ||r_v^0||. */
  int32_t dense_route;      /* subsample sketch on dense data or kernel ridge: 0 (default) forms
                               each sketch's AS by the MFMA contraction Z Z[C,:]^T + lambda I_C;
                               1 forms A = Z Z^T + lambda I (kernel ridge: K K + lambda K) once at
                               creation with the same kernel (m x m, FP32 in mixed precision,
                               else FP64) and gathers each sketch's tau columns from it. Pays when
                               a solve takes more than about m / tau iterations and m^2 fits. */
  int32_t refresh_early;    /* mixed precision, single solves: 1 (default) also recomputes r in
                               FP64 at the end of a lookahead batch whose last tracked estimate
                               ||r^k|| / ||r^0|| has reached tol (at most once per 4 iterations),
                               so that the stop, which only a refreshed residual may trigger, is
                               not delayed to the next multiple of refresh_every; 0: refreshes only
                               every refresh_every iterations. Ignored by the batched solver. */
} rs_options;

/* How AS is formed for the count and SubCount sketches on CSR data (same result up to
 * rounding). SCATTER: per sketch, T = Z^T S (bucket, signed value) aligned with CSR(Z^T),
 * then each row j of AS is the signed scatter-add of Z_ji T[i, :] into tau buckets.
 * AROWS: A0 = Z Z^T is formed once (sparse, FP64); each row j of AS is the signed
 * scatter-add of row j of A0 into tau buckets, with several sketches sharing each pass
 * over A0, then G = S^T AS from the member rows. AUTO picks AROWS when the product
 * Z Z^T has fewer than 2^31 pairs and fits in a quarter of the device memory. */
enum { RS_ROUTE_AUTO = 0, RS_ROUTE_SCATTER = 1, RS_ROUTE_AROWS = 2 };

/* Coordinate proposals for the subsample sketch (dense X). UNIFORM: every tau-subset
 * equally likely (Def. 4.2). DIAG: q_j = A_jj / Tr A (the importance sampling of Sec. 7).
 * LEARNED: q = (1 - 0.1) softmax(s) + 0.1 / m with scores s from an MLP of per-coordinate
 * features (rs_set_sampler_params). A weighted sketch keeps the tau coordinates with the
 * smallest u_j / q_j (u_j uniform from the Philox stream tag 4). Every coordinate keeps a
 * positive probability, so the expected projection stays positive definite (Thm 5.1);
 * a non-finite q falls back to a uniform draw. The learned proposal is recomputed from
 * r^k, r^{k-1} at the start of every lookahead batch. */
enum { RS_SAMPLER_UNIFORM = 0, RS_SAMPLER_LEARNED = 1, RS_SAMPLER_DIAG = 2 };
/* MLP: features (6) -> 128 -> 128 -> 1, ReLU, FP32; parameters packed W1 [6][128], b1,
 * W2 [128][128], b2, w3 [128], b3. */
enum { RS_MLP_FEATURES = 6, RS_MLP_HIDDEN = 128, RS_MLP_PARAMS = 17537 };

typedef struct rs_report {
  int64_t iters;            /* iterations performed */
  double rel_res;           /* ||r^iters|| / ||r^0|| of the tracked residual */
  double seconds;           /* wall time of the solve on the stream */
  double rel_res_true;      /* ||A w - b|| / ||b|| recomputed in FP64 from the data (not the
                               recursion) for the returned iterate, after the timed solve */
} rs_report;

/* Per-kernel timing collected with HIP events on the solver's stream (indices
 * RS_PROF_*). rs_options.profile = 1 times each batch-level launch (sketch, AS,
 * Cholesky; RS_PROF_G: the separate G = S^T AS pass of the CSR route through the rows
 * of Z Z^T) and the whole per-iteration sequence of a batch (RS_PROF_ITERS);
 * profile = 2 also times every per-iteration launch (delta, update), which adds
 * event packets between them. `launches` counts timed launches (or sequences),
 * `slots` the sketches (iterations) they processed. */
enum { RS_PROF_SKETCH = 0, RS_PROF_AS = 1, RS_PROF_CHOL = 2, RS_PROF_DELTA = 3, RS_PROF_UPDATE = 4,
       RS_PROF_REFRESH = 5, RS_PROF_ITERS = 6, RS_PROF_G = 7, RS_PROF_COUNT = 8 };
typedef struct rs_profile {
  double ms[RS_PROF_COUNT];
  int64_t launches[RS_PROF_COUNT];
  int64_t slots[RS_PROF_COUNT];
} rs_profile;

typedef struct rs_handle rs_handle;

/* Fill *o with defaults: AUTO form, subsample, tau = 0 (must be set), heuristic
 * momentum, eta 0.995, beta_max 0.5, tol 1e-6, max_iter 100000, seed 1. */
rs_status rs_options_default(rs_options* o);

/* gamma_k and beta_k (host doubles) of iteration k >= 0 under the momentum settings of
 * *o (o->momentum, gamma, beta, eta, beta_max), exactly as the solvers use them (Sec. 6,
 * Sec. 8.1). Host-only, no device call. Errors: RS_EINVAL (unknown or unusable momentum
 * settings, k < 0, a NULL pointer). */
rs_status rs_momentum_schedule(const rs_options* o, int64_t k, double* gamma, double* beta);

/* Build a solver for X, y (y: n values, FP64, in the memory X.mem names) and
 * lambda > 0. Uploads X into library-owned device layouts, forms b, sets
 * x^0 = x^{-1} = 0, r^0 = r^{-1} = -b. Errors: RS_EINVAL (shapes, tau, lambda,
 * non-finite y), RS_ENOMEM, RS_EDEVICE, RS_EUNSUPPORTED. */
rs_status rs_create(const rs_matrix* X, const double* y, double lambda,
                    const rs_options* o, rs_handle** out);

/* Kernel ridge regression (Sec. 2.2, eq:kernelridge): solve K (K + lambda I) alpha = K y
 * for the Gaussian kernel K_ij = exp(-||p_i - p_j||^2 / (2 sigma^2)) (eq:Gausskernel) of
 * the n points P (an rs_matrix of n rows and d coordinates, dense, FP32 or FP64, host or
 * device; y: n values in the memory P.mem names). The library forms K (n x n, FP64) in
 * device memory (8 n^2 bytes), b = K y, and then runs the same iteration as rs_create's
 * dense path with m = n; the weights (rs_get_weights, rs_solve) are the n coefficients
 * alpha, and predictions at the points are K alpha. Options: every sketch (count and
 * SubCount take the dense-S products); RS_PREC_MIXED_BF16 with the subsample sketch runs the
 * products on a BF16 copy of K (another 2 n^2 bytes) and keeps K for the shift lambda K S and
 * the FP64 refresh; uniform sampling (RS_EUNSUPPORTED otherwise); the accelerated method with
 * the subsample sketch; o->form is ignored. Errors: RS_EINVAL (sigma or lambda not positive
 * and finite, CSR points, shapes, non-finite y), RS_ENOMEM, RS_EDEVICE, RS_EUNSUPPORTED. */
rs_status rs_create_kernel(const rs_matrix* P, const double* y, double sigma, double lambda,
                           const rs_options* o, rs_handle** out);

/* Advance up to `iters` iterations (fewer if ||r^k|| / ||r^0|| <= tol is met
 * first), then synchronise the stream. *rel_res_out (host, may be NULL)
 * receives ||r^k|| / ||r^0|| at the final k. */
rs_status rs_step(rs_handle* h, int64_t iters, double* rel_res_out);

/* Iterate until tol or max_iter. x_out (host, may be NULL) receives the
 * ridge weights w (d values; dual form maps alpha through X^T). rep (host,
 * may be NULL) gets the report. Returns RS_NOT_CONVERGED if max_iter hit. */
rs_status rs_solve(rs_handle* h, double* w_out, rs_report* rep);

/* Restart from x^0 = x^{-1} = 0, r^0 = r^{-1} = -b with a new sketch seed,
 * keeping the device layouts built by rs_create (k returns to 0). */
rs_status rs_reset(rs_handle* h, uint64_t seed);

/* Accumulated per-kernel timings since rs_create or the last call with
 * clear != 0 (which zeroes them after copying). Needs rs_options.profile. */
rs_status rs_get_profile(rs_handle* h, rs_profile* out, int32_t clear);

/* Current iteration count k. */
int64_t rs_iteration(const rs_handle* h);
/* m, the size of the system (d in primal form, n in dual form). */
int64_t rs_system_size(const rs_handle* h);

/* Copy the state to host buffers of m doubles each (any may be NULL):
 * x^k, x^{k-1}, r^k = A x^k - b (tracked), r^{k-1}. The accelerated method (Alg. 3)
 * returns w^k, v^k, r_w^k, r_v^k in the same four places. */
rs_status rs_get_state(const rs_handle* h, double* x, double* x_prev, double* r, double* r_prev);

/* Resume from a saved state (checkpoint): iteration k and x^k, x^{k-1}, r^k, r^{k-1}
 * (host buffers of m doubles, none NULL, all finite; copied before the call returns), as
 * rs_get_state returned them. Alg. 2's next iterate depends only on these and on S_k,
 * which is drawn from (seed, problem_id, k), so the iterations that follow equal those
 * of the uninterrupted solve (mixed precision recomputes r in FP64 when an rs_step or
 * rs_solve call ends, so there the solve whose call ended at k); only the stop test at
 * iteration k itself uses ||r^k||
 * summed here on the host (in index order) rather than the update's partial sums. Any
 * prepared lookahead batch is dropped; ||r^0|| stays the one of rs_create (= ||b||);
 * history entries before k keep what the handle held (undefined in a handle that never
 * iterated). Not to be called while another
 * call on the handle runs (handles are not thread-safe).
 * RS_EINVAL for a NULL or non-finite vector or k outside [0, max_iter];
 * RS_EUNSUPPORTED for the accelerated method and the learned sampler (their state holds
 * more than these four vectors). */
rs_status rs_set_state(rs_handle* h, int64_t k, const double* x, const double* x_prev, const double* r,
                       const double* r_prev);

/* Ridge weights from the current iterate (host, d doubles). */
rs_status rs_get_weights(rs_handle* h, double* w_out);

/* The sketch S_{k-1} used by the last iteration, as (rows, cols, signs)
 * triplets of its nonzeros (host buffers of capacity m). *nnz_out receives
 * the count. Bucket-major order: all nonzeros of column 0 first. RS_EUNSUPPORTED for the
 * Gaussian and SRHT sketches (dense S; rs_get_products gives A S). */
rs_status rs_get_last_sketch(const rs_handle* h, int32_t* rows, int32_t* cols, int8_t* signs,
                             int64_t* nnz_out);

/* Products of the last iteration's sketch S_{k-1} (host buffers, may be NULL):
 * as_out: m x tau row-major AS = Z (Z^T S) + lambda S as stored by the library (FP64,
 * or FP32 widened to FP64 in mixed precision); ginv_out: tau x tau row-major
 * (S^T A S)^{-1} as applied by the solve (identity rows/columns for empty buckets).
 * For parity tests and inspection. */
rs_status rs_get_products(const rs_handle* h, double* as_out, double* ginv_out);

/* Relative residual history ||r^k|| / ||r^0||, k = 0..count-1 (host). */
rs_status rs_get_history(const rs_handle* h, double* out, int64_t count);

rs_status rs_destroy(rs_handle* h);

/* tau of the handle's sketch. */
int32_t rs_sketch_size(const rs_handle* h);
/* Route the handle forms sparse products with (RS_ROUTE_SCATTER or RS_ROUTE_AROWS; 0 for
 * dense data) and, for RS_ROUTE_AROWS, the number of stored entries of Z Z^T (host). */
rs_status rs_get_route(const rs_handle* h, int32_t* route, int64_t* a_nnz);

/* ------------------------------------------------------------------------
 * Learned proposal: parameters, traces, training, and single-kernel entry points.
 *
 * Features of coordinate j at iteration k (r = r^k, rp = r^{k-1}, a = diag A, last_j the
 * latest earlier iteration whose sketch held j, or -1): f0 = standardised log a_j,
 * f1 = clip(log|r_j| - log(a_j)/2 - log||r|| + log(sum a)/2, -30, 30),
 * f2 = log(1 + k - last_j), f3 = clip(log|r_j - rp_j| - log||r|| + log(m)/2, -30, 30),
 * f4 = log(k + 1), f5 = [last_j == k - 1]. A trace record of iteration k holds the
 * features of the tau sketched coordinates and their credits c_b = delta_b rho_b, whose
 * sum delta^T G delta is the decrease of the squared A-norm error (eq:gradeqf).
 * Training minimises, per record, the cross-entropy between t = max(c, 0) / sum max(c, 0)
 * and softmax(s) over the record's coordinates, with Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) on mini-batches of records.
 * ------------------------------------------------------------------------ */
/* Parameters of the learned proposal (host, RS_MLP_PARAMS finite values). */
rs_status rs_set_sampler_params(rs_handle* h, const float* params);
/* Trace records held by the handle (rs_reset keeps them). */
rs_status rs_trace_count(const rs_handle* h, int64_t* count);
/* Records first .. first+count-1: F (count x tau x 6) and credits (count x tau), host. */
rs_status rs_get_trace(const rs_handle* h, float* F, float* credits, int64_t first, int64_t count);
/* The proposal q (m values, host) of the latest draw and its usable flag (may be NULL). */
rs_status rs_get_proposal(const rs_handle* h, float* q, int32_t* ok);

typedef struct rs_trainer rs_trainer;
/* Trainer for sketches of size tau; parameters initialised from Philox4x64-10 with key
 * (init_seed, 0), counter (index, 0, 5, 0): weights uniform on +-1/sqrt(fan_in), biases 0. */
rs_status rs_trainer_create(int32_t tau, uint64_t init_seed, rs_trainer** out);
/* Append a handle's trace records (same tau) or host records to the trainer's store. */
rs_status rs_trainer_add_traces(rs_trainer* t, const rs_handle* h);
rs_status rs_trainer_add_records(rs_trainer* t, const float* F, const float* credits, int64_t count);
rs_status rs_trainer_records(const rs_trainer* t, int64_t* count);
/* `epochs` passes over the records in an order shuffled per epoch from shuffle_seed;
 * mini-batches of `batch` records (a remainder is skipped); epoch_loss (host, may be
 * NULL) receives the mean loss of each epoch. */
rs_status rs_trainer_fit(rs_trainer* t, int32_t epochs, int32_t batch, double lr, uint64_t shuffle_seed,
                         double* epoch_loss);
/* Mean loss over all stored records with the current parameters (no update), and, when
 * floor_out is not NULL, the mean entropy of the records' targets t = max(c, 0) / sum: the
 * least value the cross-entropy can take (reached when softmax(s) = t on every record). */
rs_status rs_trainer_eval(rs_trainer* t, double* loss_out, double* floor_out);
rs_status rs_trainer_get_params(const rs_trainer* t, float* out);
rs_status rs_trainer_set_params(rs_trainer* t, const float* in);
const char* rs_trainer_last_error(const rs_trainer* t);
rs_status rs_trainer_destroy(rs_trainer* t);

/* Single kernels of the proposal on host arrays (for checking each piece). */
rs_status rs_mlp_init(uint64_t seed, float* params_out);
/* s_out[rows] = MLP(F[rows][6]). */
rs_status rs_mlp_forward(const float* params, const float* F, int64_t rows, float* s_out);
/* Mean loss over nrec records (F: nrec x tau x 6, credits: nrec x tau) and its gradient. */
rs_status rs_mlp_gradient(const float* params, const float* F, const float* credits, int32_t nrec,
                          int32_t tau, float* grad_out, double* loss_out);
/* One Adam step t >= 1 on host arrays of RS_MLP_PARAMS (updated in place). */
rs_status rs_adam_update(float* params, float* m1, float* m2, const float* grad, int64_t t, double lr,
                         double b1, double b2, double eps);
/* q = (1 - eps) softmax(s) + eps / m; *ok_out = 0 if q is not finite. */
rs_status rs_proposal(const float* s, int64_t m, double eps, float* q_out, int32_t* ok_out);
/* Features F_out (m x 6) of iteration k from a = diag A (> 0), r, rp and last. */
rs_status rs_features(const double* a, const double* r, const double* rp, const int32_t* last, int64_t m,
                      int64_t k, float* F_out);
/* The weighted sketch of iteration k: C_out (tau, ascending) = the tau smallest
 * (u_j / q_j, j), u_j = ((W0 >> 12) + 0.5) 2^-52 of Philox block (j, k, 4, 0) under key
 * (seed, problem_id); q > 0 and finite. */
rs_status rs_draw_weighted(const float* q, int64_t m, int32_t tau, uint64_t seed, uint64_t problem_id,
                           int64_t k, int32_t* C_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): rs_draw_weighted on device buffers,
 * enqueued on `stream` (hipStream_t; NULL = the default stream), allocating nothing.
 * q: device, m floats, every entry positive and finite; C_out: device, tau int32 (the tau
 * smallest (u_j / q_j, j), ascending, bit-identical to rs_draw_weighted); status_out:
 * device, one int32 that receives RS_OK, RS_EINVAL (an entry of q not positive and
 * finite: C_out is not written) or RS_EDEVICE (an internal selection limit) when the
 * stream reaches the end of this call's work. The selection's working memory is a fixed
 * array of about 16 MB in device memory that each device holds from the first call until
 * the process ends; every call on a device shares it and it keeps the last call's
 * contents, so calls whose work overlaps on one device (several streams or threads)
 * race and must be serialised by the caller. Returns RS_OK once the work is enqueued;
 * RS_EINVAL for NULL pointers, tau outside [1, m], k < 0 or m > 2^20 (nothing is
 * enqueued); RS_EDEVICE if a launch fails. */
rs_status rs_draw_weighted_noalloc(const float* q, int64_t m, int32_t tau, uint64_t seed,
                                   uint64_t problem_id, int64_t k, int32_t* C_out,
                                   int32_t* status_out, void* stream);

/* ------------------------------------------------------------------------
 * Batched solves: many ridge problems, each with a grid of regularisers and
 * several right-hand sides, in one lock-step iteration.
 *
 * Problem p has its own X_p (dense or CSR, any shape), nrhs_p right-hand sides and
 * nlambda_p regularisers; its J_p = nlambda_p * nrhs_p solves (slot j = l * nrhs_p + q
 * for lambda_l and right-hand side q) share one sketch sequence S_k drawn from the
 * Philox key (seed, problem_id + p) -- the sequence a single solve created with
 * rs_options.problem_id = problem_id + p draws -- so that B S_k = Z (Z^T S_k) is formed
 * once per problem and iteration and A(lambda) S_k = B S_k + lambda S_k (eq:Axb with
 * the lambda term split off; Alg. 2 otherwise unchanged). All problems advance in lock
 * step; a solve stops at the first iteration whose ||r^k|| / ||r^0|| <= tol and keeps
 * that iterate, a problem when all its solves stopped or at its iteration cap. Each
 * iteration is a fixed sequence of device-wide launches over ragged work tables, and the
 * sequence is captured once into a HIP graph (rs_options.graph_iters iterations per
 * graph) and replayed; with rs_options.autotune the launch shapes of the
 * iterate-independent kernels are timed on the batch's own tables and the fastest kept.
 * Batched solves use the subsample sketch for dense X and the count sketch for CSR X.
 * precision RS_PREC_FP64: FP64 throughout. RS_PREC_MIXED_BF16: the dense problems' products
 * B S come from a BF16 copy of Z with FP32 accumulation (stored FP64); after the update of
 * every iteration k with (k + 1) % refresh_every == 0 (default 20) their R^{k+1} and R^k are
 * recomputed in FP64 from the FP64 data (R = Z (Z^T X) + X diag(lambda) - B), and their slots
 * may stop only at such an iteration; the CSR problems keep FP64 products (their stop test is
 * unchanged). Options used: precision, refresh_every, momentum parameters, tol, max_iter
 * (upper bound of every cap), seed, problem_id, stream, graph_iters, autotune.
 * ------------------------------------------------------------------------ */
typedef struct rs_problem {
  rs_matrix X;              /* as for rs_create; X.mem also applies to y */
  const double* y;          /* n x nrhs, column-major, FP64 */
  int32_t nrhs;             /* 1 .. 8 */
  const double* lambdas;    /* host, nlambda values > 0 */
  int32_t nlambda;          /* nlambda * nrhs <= 64 */
  int32_t tau;              /* 0: a multiple of 64 nearest m^{2/3}, clamped to [64, 512] and to m */
  int32_t sketch;           /* -1: subsample for dense X, count for CSR X (the only pairs built) */
  int32_t form;             /* RS_FORM_* (AUTO: primal iff d <= n) */
  int64_t max_iter;         /* iteration cap of this problem; 0: rs_options.max_iter */
} rs_problem;

typedef struct rs_batch_report {
  int64_t iters;            /* lock-step iterations performed */
  int32_t solves;           /* sum of J_p */
  int32_t converged;        /* solves that met tol */
  double seconds;           /* wall time of the solve */
} rs_batch_report;

typedef struct rs_batch_problem_info_t {
  int64_t m, K;             /* system size and contraction length */
  int32_t form, sketch, tau, slots;
  int64_t max_iter;         /* the problem's cap */
  int64_t iters;            /* iterations performed when it stopped (0 while running) */
} rs_batch_problem_info_t;

typedef struct rs_tuning {
  int32_t tuned;            /* 1 when the shapes below were chosen by timing */
  int32_t dense_tk;         /* K-panel depth of the FP64 dense product tiles (128 x 128 tiles; 16) */
  int32_t dense_wg_per_cu, sparse_wg_per_cu, chol_wg_per_cu;  /* persistent grid sizes */
  int32_t graph_iters;      /* iterations per graph replay */
  int32_t compute_units;
  double dense_ms, sparse_ms, chol_ms;  /* best timed launch (ms), -1 if not timed (mixed precision:
                                          dense_ms times the BF16 product launch) */
} rs_tuning;

typedef struct rs_batch rs_batch;

/* Build a batch of `count` problems (host array). Copies every X and y into library
 * layouts, forms b, sets the initial states. Errors: RS_EINVAL (shapes, tau, lambdas,
 * nrhs, non-finite y, unknown precision), RS_EUNSUPPORTED (sketch/layout pair, dense_route),
 * RS_ENOMEM, RS_EDEVICE. rs_batch_last_error(NULL) describes a failure. */
rs_status rs_batch_create(int32_t count, const rs_problem* problems, const rs_options* o,
                          rs_batch** out);
/* Advance up to `iters` lock-step iterations (fewer once every problem stopped). */
rs_status rs_batch_step(rs_batch* b, int64_t iters);
/* Iterate until every problem stopped. RS_NOT_CONVERGED if some solve hit its cap. */
rs_status rs_batch_solve(rs_batch* b, rs_batch_report* rep);
/* Restart every solve from zero with a new sketch seed (layouts and tuning kept). */
rs_status rs_batch_reset(rs_batch* b, uint64_t seed);
int64_t rs_batch_iteration(const rs_batch* b);
rs_status rs_batch_problem_info(const rs_batch* b, int32_t p, rs_batch_problem_info_t* info);
/* Per slot of problem p (host arrays of J_p, either may be NULL): the iteration at which
 * the solve met tol (-1 if it has not) and its last ||r^k|| / ||r^0||. */
rs_status rs_batch_slot_report(const rs_batch* b, int32_t p, int64_t* stop_iter, double* rel_res);
/* State of one solve (host buffers of m_p doubles, any may be NULL), as rs_get_state. */
rs_status rs_batch_get_state(const rs_batch* b, int32_t p, int32_t slot, double* x, double* x_prev,
                             double* r, double* r_prev);
/* Ridge weights of problem p: d_p x J_p column-major (slot j in column j), host. */
rs_status rs_batch_get_weights(rs_batch* b, int32_t p, double* w_out);
rs_status rs_batch_get_tuning(const rs_batch* b, rs_tuning* out);
rs_status rs_batch_destroy(rs_batch* b);
const char* rs_batch_last_error(const rs_batch* b);

const char* rs_status_string(rs_status s);
/* Text of the last error on this handle (or of the last failed rs_create on
 * this thread when h is NULL). Valid until the next call on the handle. */
const char* rs_last_error(const rs_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* RS_H */
