/*
 * fisherbt.h -- C ABI of the MI355X (gfx950) library for exact Matern
 * maximum-likelihood estimation by Fisher scoring with backtracking
 * (Fisher-BT).
 *
 * Model (Section 2.1): a zero-mean Gaussian random field on R^2 observed at
 * locations s_1..s_n, with Matern covariance
 *     C(h; theta) = sigma2 2^(1-nu) / Gamma(nu) (h/alpha)^nu K_nu(h/alpha),
 * theta = (sigma2, alpha, nu), h the Euclidean distance.  (alpha is the range
 * parameter, sometimes written beta.)
 *
 * Conventions shared by every call:
 *   - theta is always double[3] = {sigma2, alpha, nu}; each must be finite and
 *     > 0, otherwise the call returns FBT_EINVAL and writes nothing.
 *   - Output pointers are host memory owned by the caller and are written only
 *     when the call returns FBT_OK.  Matrices are returned column-major.
 *   - Every call is synchronous with respect to the host; device work is
 *     ordered on the context's HIP stream, so other work on that stream (for
 *     example PyTorch's) is ordered with it.
 *   - One context per host thread; contexts share nothing.
 *   - Errors are negative.  FBT_ENOTPD is recoverable (Sigma(theta) is not
 *     numerically positive definite); FBT_EDEVICE and FBT_ENOMEM are not.
 *   - All arithmetic on the evaluation path is IEEE FP64 unless the context
 *     selects FBT_MIXED_FP32 (see fbt_precision).
 */
#ifndef FISHERBT_H
#define FISHERBT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fbt_ctx fbt_ctx; /* opaque; owns its device buffers */

typedef enum {
    FBT_OK = 0,
    FBT_EINVAL = -1,     /* bad argument (NULL, n < 1, non-finite input, theta <= 0, ...) */
    FBT_ENOTPD = -2,     /* Cholesky met a pivot <= 0 or NaN; see fbt_last_notpd_pivot */
    FBT_ENOMEM = -3,     /* device or pinned-host allocation failed */
    FBT_EDEVICE = -4,    /* HIP runtime error or no gfx950 device */
    FBT_ENONFINITE = -5, /* a result came out non-finite */
    FBT_EBUDGET = -6,    /* fit: call budget exhausted with the Nelder-Mead fallback off */
    FBT_ENODATA = -7     /* no data set on the context */
} fbt_status;

/* Arithmetic of the evaluation path.
 * FBT_FP64: everything in IEEE FP64 (the default).
 * FBT_MIXED_FP32: the O(n^3) updates of the W phase that forms
 *   W_i = L^{-1} Sigma_i L^{-T} (the trace terms of the score and Fisher
 *   information, about 6/7 of the flops of fbt_eval): the rank-2k and
 *   deferred-solve updates of the two-sided form, or the trailing updates of
 *   the block solves (fbt_set_wphase), multiply on FP32 MFMA with FP32 sums
 *   per 256-deep slice.  The Cholesky factorisation, log-determinant and
 *   quadratic form (so the log-likelihood and every line-search test), the
 *   Bessel terms, diagonal blocks, panels and all reductions stay FP64:
 *   fbt_loglik is unchanged and fbt_eval returns the FP64 log-likelihood.
 * FBT_MIXED_FP32_ALL: the Cholesky trailing updates in FP32 as well, so
 *   every term carries FP32 rounding of the factor amplified by the
 *   conditioning of Sigma, and the factorisation can fail for
 *   ill-conditioned Sigma.  The solve for w = Sigma^{-1} Z can be won back by
 *   iterative refinement (fbt_set_refinement), which makes the quadratic
 *   forms Z^T Sigma^{-1} Z and w^T Sigma_i w FP64-accurate; the
 *   log-determinant and the traces keep the factor's rounding.  fbt_fit
 *   refuses the form (its line-search tests take FP64 log-likelihoods).
 * FBT_MIXED_BF16: as FBT_MIXED_FP32, with the operands of those updates
 *   rounded to bfloat16 (8-bit significand) and the products summed in FP32
 *   (v_mfma_f32_16x16x16_bf16).  The log-likelihood is the FP64 one; score and
 *   Fisher carry bfloat16 rounding of the W phase's updates, amplified by the
 *   conditioning of Sigma (errors of order 1e-3 relative or worse).
 * FBT_MIXED_BF16_ALL: the Cholesky trailing updates with bfloat16 operands
 *   and FP32 sums as well (the W phase as FBT_MIXED_BF16): the factor carries
 *   bfloat16 rounding, so the form suits well-conditioned Sigma only (short
 *   range); the factorisation fails (FBT_ENOTPD) once that rounding exceeds
 *   Sigma's smallest eigenvalues.  Refinement of w (fbt_set_refinement) and
 *   the fit's refusal as under FBT_MIXED_FP32_ALL. */
typedef enum {
    FBT_FP64 = 0,
    FBT_MIXED_FP32 = 1,
    FBT_MIXED_FP32_ALL = 2,
    FBT_MIXED_BF16 = 3,
    FBT_MIXED_BF16_ALL = 4
} fbt_precision;

typedef struct {
    int32_t device;    /* HIP device ordinal */
    int32_t tile;      /* block size of the tiled factorisation; 0 = default (256); only 256 */
    int32_t precision; /* fbt_precision */
    void *hip_stream;  /* hipStream_t to order work on; NULL = the library creates its own */
} fbt_config;

/* Create a context on cfg->device.  On success *out owns a stream (unless one
 * was given) and no data.  Errors: FBT_EINVAL (NULL args, unsupported tile),
 * FBT_EDEVICE (no such device, or not gfx950). */
fbt_status fbt_create(const fbt_config *cfg, fbt_ctx **out);

/* Release every resource of ctx.  NULL is a no-op. */
void fbt_destroy(fbt_ctx *ctx);

/* Switch the arithmetic of later evaluations (fbt_precision).  Errors: FBT_EINVAL. */
fbt_status fbt_set_precision(fbt_ctx *ctx, int32_t precision);

/* Observations (Section 2.1): n locations as an n x 2 row-major array
 * (x_i, y_i) and the n observations Z.  Both host arrays are copied; the
 * caller keeps ownership.  Device buffers are (re)allocated for n: about
 * 3 n_pad^2 doubles with n_pad = 256 ceil((n + 1) / 256).
 * Errors: FBT_EINVAL (NULL, n < 1, non-finite input), FBT_ENOMEM. */
fbt_status fbt_set_data(fbt_ctx *ctx, int64_t n, const double *locs_xy, const double *z);

/* Same as fbt_set_data with device pointers (on ctx's device).  The arrays
 * are copied on the context's stream before the call returns, so the caller
 * may free them afterwards. */
fbt_status fbt_set_data_device(fbt_ctx *ctx, int64_t n, const double *d_locs_xy, const double *d_z);

/* Algorithm 2: exact log-likelihood, Eq. (1),
 *     l(theta) = -n/2 log(2 pi) - 1/2 log det Sigma - 1/2 Z^T Sigma^{-1} Z,
 * by a tiled Cholesky factorisation of Sigma(theta).  The factor is kept, so a
 * following fbt_eval at the same theta reuses it.
 * Errors: FBT_EINVAL, FBT_ENODATA, FBT_ENOTPD, FBT_EDEVICE. */
fbt_status fbt_loglik(fbt_ctx *ctx, const double theta[3], double *loglik);

/* Algorithm 3: log-likelihood, score (Eq. (2)) and expected Fisher information
 * (Eq. (3)) over theta = (sigma2, alpha, nu).  The traces are formed as
 * Frobenius products of W_i = L^{-1} Sigma_i L^{-T} (Eq. (5) is the same
 * identity); dSigma/dnu is the exact derivative of the Matern covariance.
 * score[3]; fisher[9] is the full symmetric 3 x 3 matrix, row-major.
 * Errors: as fbt_loglik. */
fbt_status fbt_eval(fbt_ctx *ctx, const double theta[3], double *loglik, double score[3],
                    double fisher[9]);

/* The intermediate scalars of Algorithm 3 at theta (for checking): terms[9] =
 * { log det Sigma, Z^T Sigma^{-1} Z, tr(Sigma^{-1} Sigma_alpha),
 *   tr(Sigma^{-1} Sigma_nu), w^T Sigma_alpha w, w^T Sigma_nu w,
 *   tr(Sigma^{-1} Sigma_a Sigma^{-1} Sigma_a), tr(.. a .. nu), tr(.. nu .. nu) }
 * with w = Sigma^{-1} Z.  Errors: as fbt_loglik. */
fbt_status fbt_eval_terms(fbt_ctx *ctx, const double theta[3], double terms[9]);

/* Adjoint gradient: the log-likelihood (Eq. (1)) and the score (Eq. (2))
 * without the Fisher information, at about a third of the cost of fbt_eval.
 * The score is evaluated as the Frobenius product
 *   dl/dtheta_i = < (w w^T - Sigma^{-1}) / 2, Sigma_i >_F,  w = Sigma^{-1} Z,
 * which is Eq. (2) with tr(A B) = <A, B^T>_F; Sigma^{-1} is formed from the
 * inverse of the Cholesky factor and Sigma_alpha, Sigma_nu are regenerated
 * entry by entry inside the contraction (never stored).  The sigma^2
 * component is (Z^T Sigma^{-1} Z - n) / (2 sigma^2) as in fbt_eval.
 * dloglik_dz: NULL, or host array of n doubles that receives dl/dZ = -w.
 * Reuses the factor of an immediately preceding fbt_loglik at the bitwise
 * same theta.  Errors: as fbt_loglik. */
fbt_status fbt_grad(fbt_ctx *ctx, const double theta[3], double *loglik, double score[3],
                    double *dloglik_dz);

/* Covariance generation (Section 2.1, and Section 2.2 for the derivatives):
 * writes the n x n matrix Sigma (which = 0), Sigma_alpha (1) or Sigma_nu (2)
 * at theta into out (host, column-major, leading dimension ld >= n).
 * Errors: FBT_EINVAL, FBT_ENODATA, FBT_EDEVICE. */
fbt_status fbt_covariance(fbt_ctx *ctx, const double theta[3], int32_t which, double *out,
                          int64_t ld);

/* The lower Cholesky factor L of Sigma(theta) (Algorithm 2, second step) into
 * out (host, column-major, ld >= n); the strict upper triangle is zeroed.
 * Errors: as fbt_loglik. */
fbt_status fbt_factor(fbt_ctx *ctx, const double theta[3], double *out, int64_t ld);

/* ---------------------------------------------------------------- fit ---- */

/* Called after every accepted Fisher-scoring iterate (iter 0 is the start). */
typedef void (*fbt_iter_cb)(void *user, int32_t iter, const double theta[3], double loglik,
                            const double score[3], const double fisher[9]);

/* Options of Algorithm 1; fbt_fit_options_default fills the paper's values. */
typedef struct {
    const double *theta0;     /* NULL: L9 start of Table 1 from [lo, hi] */
    double lo[3], hi[3];      /* (0.01, 0.01, 0.01), (5, 5, 2) */
    double armijo_c;          /* 1e-3   Eq. (4) */
    double armijo_relax;      /* 1e-3   relaxation of Eq. (4) */
    double backtrack_rho;     /* 0.5 */
    double grad_tol;          /* 1e-3   stop when ||grad l||_2 <= grad_tol */
    int32_t max_loglik_calls; /* 60     shift beyond this many l calls (L9 included) */
    int32_t max_grad_calls;   /* 20     shift beyond this many grad calls */
    int32_t max_iter;         /* 0 = no limit on accepted steps */
    int32_t nelder_mead;      /* 1: Nelder-Mead fallback on shift; 0: return FBT_EBUDGET */
    double nm_ftol;           /* 1e-9   Nelder-Mead stop: spread of l over the simplex */
    int32_t nm_max_evals;     /* 500 */
    fbt_iter_cb cb;           /* may be NULL */
    void *cb_user;
    /* 1e-4   fbt_fit on a context in a mixed precision: the score of the mixed
     * form carries FP32 rounding of the trace terms, so it cannot resolve the
     * stopping test at large n.  At the first derivative evaluation whose
     * score satisfies ||grad||_2 <= mixed_switch ||s||_2, with the per-term
     * scales s = ((q + n) / (2 sigma2), (|t_a| + |u_a|) / 2, (|t_nu| + |u_nu|) / 2)
     * (t_i = tr(Sigma^-1 Sigma_i), u_i = w^T Sigma_i w, q = Z^T Sigma^-1 Z), the
     * context switches to FP64 for the rest of the fit and that theta is
     * evaluated again in FP64 (on the same factor under FBT_MIXED_FP32); the
     * re-evaluation is not counted as a grad call.  0 never switches.  The
     * context's precision is restored when fbt_fit returns.  Ignored by
     * fbt_fit_evaluator and under FBT_FP64. */
    double mixed_switch;
} fbt_fit_options;

typedef struct {
    double theta[3], loglik, score[3], fisher[9];
    int32_t n_loglik_calls, n_grad_calls, n_iter, used_nelder_mead, converged, n_nm_evals;
    /* fbt_fit: the driver's derivative evaluations whose results are FP64
     * (all of them under FBT_FP64; under a mixed precision those from the
     * switch on, the one at the switch point included), and the 0-based index
     * of the derivative evaluation at which the switch happened (-1: none). */
    int32_t n_fp64_evals, precision_switch;
} fbt_fit_result;

void fbt_fit_options_default(fbt_fit_options *o);

/* Algorithm 1 (Fisher-BT): L9 start, Fisher scoring phi = I^{-1} grad with the
 * relaxed Armijo backtracking of Eq. (4), stop at ||grad|| <= grad_tol, shift
 * to Nelder-Mead when a call budget is exceeded, then one Fisher evaluation
 * at the result.  Every l and derivative evaluation runs on the GPU.
 * Errors: FBT_EINVAL (also for a context in FBT_MIXED_FP32_ALL or
 * FBT_MIXED_BF16_ALL: its log-likelihood is not the FP64 one that the
 * acceptance tests of Eq. (4) take), FBT_ENODATA, FBT_ENOTPD (every L9 candidate failed),
 * FBT_EBUDGET (budget exhausted with nelder_mead = 0; *out still holds the
 * last iterate), FBT_EDEVICE. */
fbt_status fbt_fit(fbt_ctx *ctx, const fbt_fit_options *opt, fbt_fit_result *out);

/* Algorithm 1 over any evaluator.  fbt_fit runs this with the GPU evaluator
 * of ctx; other evaluators (a CPU model, a test double) use the same driver.
 * loglik/eval return FBT_OK, FBT_ENOTPD (the trial counts as l = -inf) or
 * another error (the fit stops and returns it).  No device is touched here. */
typedef struct {
    void *user;
    fbt_status (*loglik)(void *user, const double theta[3], double *loglik);
    fbt_status (*eval)(void *user, const double theta[3], double *loglik, double score[3],
                       double fisher[9]);
} fbt_evaluator;

fbt_status fbt_fit_evaluator(const fbt_evaluator *ev, const fbt_fit_options *opt,
                             fbt_fit_result *out);

/* The nine L9 starting candidates of Table 1 for the cube [lo, hi], row-major 9 x 3. */
void fbt_l9_design(const double lo[3], const double hi[3], double out[27]);

/* ---------------------------------------------------------- diagnostics -- */

const char *fbt_status_string(fbt_status s);
/* Detail of the last error on ctx (static storage in ctx; valid until the next call). */
const char *fbt_last_error(const fbt_ctx *ctx);
/* 0-based index of the first failing pivot of the last FBT_ENOTPD, else -1. */
int64_t fbt_last_notpd_pivot(const fbt_ctx *ctx);

/* ---- Batched fields ----------------------------------------------------
 * Many independent fields evaluated together, e.g. one Fisher-BT iteration
 * (Algorithm 1) over a set of fields: a pool of `workers` contexts, each with
 * its own HIP streams and device buffers, driven by host threads that take
 * fields in order of decreasing n.  Each field's result is bitwise the one a
 * single context gives for it (the same kernels and reduction order).
 * cfg->hip_stream is ignored (workers own their streams); cfg->precision
 * applies to every worker.  Device memory: about 3 * 8 * npad^2 bytes per
 * worker for the largest field (npad = 256 ceil((n + 1) / 256)). */
typedef struct fbt_batch fbt_batch;
/* workers in [1, 64].  Every worker drives four HIP streams, and a process
 * has few hardware queues (4 by default), so workers beyond two mostly share
 * queues: on MI355X a 256-field round took 383, 348, 360 and 371 ms with 1,
 * 2, 4 and 8 workers.  Errors: FBT_EINVAL, FBT_EDEVICE, FBT_ENOMEM. */
fbt_status fbt_batch_create(const fbt_config *cfg, int32_t workers, fbt_batch **out);
void fbt_batch_destroy(fbt_batch *b); /* NULL-safe */
/* nf fields; field f: n[f] >= 1 observations, locs[f] (n[f] x 2, row-major,
 * host) and z[f] (n[f], host).  The data are copied.  Errors: FBT_EINVAL. */
fbt_status fbt_batch_set_fields(fbt_batch *b, int32_t nf, const int64_t *n,
                                const double *const *locs, const double *const *z);
/* thetas: nf x 3 (row-major); mode[f]: 0 skip, 1 log-likelihood (Algorithm 2),
 * 2 log-likelihood + score + Fisher (Algorithm 3), 3 log-likelihood + score
 * (adjoint form, see fbt_grad).  Outputs (host): loglik[nf] (modes >= 1),
 * score[3 nf] (modes 2, 3), fisher[9 nf] (mode 2); a buffer no field needs may
 * be NULL.  status[nf] receives each field's fbt_status (e.g. FBT_ENOTPD for a
 * theta whose covariance is not positive definite; that field's outputs are
 * then not written).  Returns FBT_OK unless a device error or allocation
 * failure stopped the batch (FBT_EDEVICE / FBT_ENOMEM, detail in
 * fbt_batch_last_error), or FBT_EINVAL for bad arguments. */
fbt_status fbt_batch_eval(fbt_batch *b, const double *thetas, const int32_t *mode,
                          double *loglik, double *score, double *fisher, int32_t *status);
const char *fbt_batch_last_error(const fbt_batch *b);
/* Algorithm 1 (Fisher-BT) for every field of the batch at once: each field's
 * fit is fbt_fit_evaluator's driver with options *opt (its theta0 is
 * ignored; theta0 here is nf x 3 row-major starts, or NULL for the L9 start
 * of Table 1 from [opt->lo, opt->hi]), and all the evaluations the running
 * fits ask for next (log-likelihood trials, derivative evaluations,
 * Nelder-Mead points) are made together in one fbt_batch_eval call per
 * round - one launch of the round kernel in the persistent execution.  A
 * field's fit is the one fbt_fit_evaluator gives over the batch's evaluation
 * of that field.  active (NULL: all) selects fields; res[nf] and status[nf]
 * receive each selected field's result and fbt_fit_evaluator's status
 * (FBT_EBUDGET with nelder_mead = 0 included); *rounds (may be NULL) the
 * number of evaluation rounds.  opt->cb runs on the fits' host threads
 * (cb_user is shared).  Returns FBT_OK unless a
 * round failed as a whole (FBT_EDEVICE, FBT_ENOMEM; the fits then stop with
 * that status), or FBT_EINVAL for bad arguments and for a batch in
 * FBT_MIXED_FP32_ALL or FBT_MIXED_BF16_ALL (as fbt_fit). */
fbt_status fbt_batch_fit(fbt_batch *b, const fbt_fit_options *opt, const double *theta0,
                         const int32_t *active, fbt_fit_result *res, int32_t *status,
                         int32_t *rounds);
/* Fits of fbt_batch_fit that run at once (one host thread each; 0: the
 * default, 512): the other fields' fits start as running ones end.  The
 * results of every fit do not depend on it.  threads in [0, 4096].
 * Errors: FBT_EINVAL. */
fbt_status fbt_batch_set_fit_threads(fbt_batch *b, int32_t threads);

/* Execution of fbt_batch_eval (batched evaluations of one Fisher-BT
 * iteration over many fields, the batching of Section 2's estimator across
 * replicates).
 *   FBT_BATCH_WORKERS (default): groups go to the worker contexts, driven by
 *     host threads.
 *   FBT_BATCH_GRAPH: every group of the call gets a context of its own
 *     (device memory for all groups at once) and the whole call - for every
 *     group the upload of its theta tables, generation, factorisation, W phase
 *     and the copies of the results - is captured in one HIP graph, rebuilt
 *     only when the fields, the modes, the group limits or the precision
 *     change; other calls replay it with their theta (one graph launch per
 *     call).  Adjoint-mode fields run after the graph, one by one.
 * Results are bitwise the same in both.  FBT_BATCH_GRAPH is switched off (its first capture and replay crashed the host process with a
 * segmentation fault; a host-only check of the capture sequence against a
 * recording stand-in of the runtime finds every stream joined, every waited
 * event captured, no allocation or host wait inside the capture and every
 * copy in bounds, so the cause is not identified): asking for it returns
 * FBT_EINVAL with the reason in fbt_batch_last_error.  Errors: FBT_EINVAL. */
/*   FBT_BATCH_PERSISTENT: every log-likelihood and derivative field of the
 *     call in ONE kernel launch (the batching of Algorithm 1's evaluations
 *     over replicate fields): the evaluations of all fields are split into
 *     tile tasks (generation of Sigma, Sigma_alpha, Sigma_nu tiles; left-looking
 *     Cholesky tiles with the diagonal factor and its inverse; forward
 *     substitution of [Sigma_alpha | Sigma_nu]; W_i = L^{-1} Sigma_i L^{-T}
 *     tiles with their shares of the traces of Eqs. (2), (3) and (5); a
 *     fixed-order reduction per field) that the launch's workgroups take in
 *     an order planned on the host (a list schedule of the task graph,
 *     checked before every launch so that no workgroup can wait on a task
 *     that no workgroup holds), each waiting on counters of the tiles it
 *     reads.  Tiles of 64 or 128 rows (fbt_batch_set_tile).  FP64 only
 *     (FBT_EINVAL for a batch of another precision).  Adjoint-mode fields
 *     run after the launch, one by one.  Results agree with the other
 *     executions to rounding (a different blocking and summation order), not
 *     bitwise.  A dependency wait that exceeds 5 s of wall-clock time ends the
 *     launch and the call returns FBT_EDEVICE. */
typedef enum {
    FBT_BATCH_WORKERS = 0,
    FBT_BATCH_GRAPH = 1,
    FBT_BATCH_PERSISTENT = 2
} fbt_batch_exec;
fbt_status fbt_batch_set_exec(fbt_batch *b, int32_t exec);
int32_t fbt_batch_get_exec(const fbt_batch *b); /* -1 for NULL */
/* Tile size of the persistent execution: 64, 128, or 0 for the default (128).
 * Errors: FBT_EINVAL. */
fbt_status fbt_batch_set_tile(fbt_batch *b, int32_t tile);
int32_t fbt_batch_get_tile(const fbt_batch *b); /* -1 for NULL */
/* Persistent execution of the last call: tasks of its plan, the planner's
 * makespan estimate (microseconds) and the kernel's time (ms; 0 before the
 * first call).  Errors: FBT_EINVAL for NULL b. */
fbt_status fbt_batch_round_stats(const fbt_batch *b, int64_t *ntasks, double *plan_us,
                                 double *kernel_ms);
/* HIP graph of the persistent execution's round (on by default): with on,
 * later calls without a trace replay one graph - the uploads of the theta
 * tables and field descriptors from pinned staging, a kernel that clears the
 * counters, the round kernel, and the result copies - captured on the first
 * such call for the current fields, modes and tile size.  Results are
 * bitwise those of the direct launch.  Errors: FBT_EINVAL, FBT_EDEVICE. */
fbt_status fbt_batch_set_round_graph(fbt_batch *b, int32_t on);
/* Per-task trace of the persistent execution (off by default): with on,
 * later calls record for every task the wall-clock ticks (the device's
 * constant-rate counter, hipDeviceAttributeWallClockRate kHz) at which a
 * workgroup took its ticket, finished its waits and finished the task.
 * fbt_batch_round_trace copies the last call's record, 5 int64 per task in
 * ticket order (the two task words as in fbt_round_plan, then the three
 * times), for at most cap tasks, and returns the task count (0: none).
 * Errors: FBT_EINVAL, FBT_EDEVICE. */
fbt_status fbt_batch_set_round_trace(fbt_batch *b, int32_t on);
int64_t fbt_batch_round_trace(const fbt_batch *b, int64_t *out, int64_t cap);
/* Task queues of the persistent execution: the fields are split over
 * `queues` queues (1, 2, 4 or 8; 0: the default, 8, one per XCD of MI355X),
 * each drained by the workgroups of one XCD.  Errors: FBT_EINVAL. */
fbt_status fbt_batch_set_queues(fbt_batch *b, int32_t queues);
int32_t fbt_batch_get_queues(const fbt_batch *b); /* -1 for NULL */
/* Host-only inspection of the persistent execution's plan (no device
 * needed): the ticket order of the tasks of nf fields with n[f]
 * observations and mode[f] (1, 2; other values: no tasks) for tiles of
 * `tile` rows, `slots` workgroups and `queues` queues (1..8).  *ntasks
 * receives the task count; tasks (NULL: not written) receives two int32 per
 * task, (field << 3 | type, i << 16 | j) with type 0 generation of tile
 * (i, j), 1 Cholesky tile (i, j), 2 forward-substitution tile (i, j) of
 * [Sigma_alpha | Sigma_nu] (j < 2T), 3 W tile (i, j), 4 the field's
 * reduction; qoff (NULL: not written) receives queues + 1 offsets, queue q
 * holding tasks [qoff[q], qoff[q + 1]); *est_us the planner's makespan
 * estimate.  Returns FBT_EINVAL for bad arguments or an order that fails
 * the check of the kernel's waits. */
fbt_status fbt_round_plan(int32_t nf, const int64_t *n, const int32_t *mode, int32_t tile,
                          int32_t slots, int32_t queues, int64_t *ntasks, int32_t *tasks,
                          int64_t *qoff, double *est_us);
/* The kernel's waits for task (ft, ij) of a field with T tiles and mode 1 or
 * 2: counters off[k] >= need[k], k < the return value (at most 4), and the
 * counters pub[k], k < *npub (at most 4), it advances by one when done. */
int32_t fbt_round_task_deps(int32_t T, int32_t mode, int32_t ft, int32_t ij, int32_t *off,
                            int32_t *need, int32_t *pub, int32_t *npub);

/* At most max_fields fields of padded order npad (a multiple of 256) per group
 * (0: only the 8 GB cap).  Errors: FBT_EINVAL. */
fbt_status fbt_batch_set_group_limit(fbt_batch *b, int64_t npad, int32_t max_fields);
int32_t fbt_batch_group_limit(const fbt_batch *b, int64_t npad); /* 0: none; -1 for NULL */
/* Autotuner: for every padded order among the fields of the workload (thetas,
 * mode as in fbt_batch_eval), time the calls of that order's fields alone with
 * group limits 1, 2, 4, 8, 16, 32 and none in the current execution (best of
 * two after one untimed call), keep the fastest limit, then time the whole
 * call in both executions and keep the faster (the workers only while the
 * graph execution is switched off).  The choices go to the JSON
 * file `path` (NULL: none) for fbt_batch_load_tuning.  The outputs of the
 * timed calls are discarded.  Errors: as fbt_batch_eval, FBT_EINVAL when the
 * file cannot be written. */
fbt_status fbt_batch_autotune(fbt_batch *b, const double *thetas, const int32_t *mode,
                              const char *path);
/* Group limits and execution from a file written by fbt_batch_autotune.
 * Errors: FBT_EINVAL (missing or malformed file). */
fbt_status fbt_batch_load_tuning(fbt_batch *b, const char *path);

/* How Sigma_nu = dSigma/dnu is computed (Section 2.2).
 *   FBT_SIGMA_NU_EXACT (default): the exact derivative of the Matern entry,
 *     by quadrature of the integral form of K_nu and its order derivative.
 *   FBT_SIGMA_NU_PAPER: the paper's own numerical scheme for d/dnu[x^nu K_nu]
 *     (Supplementary A): series for x < 8.5, uniform expansion for
 *     8.5 <= x < 30, Hankel expansion for x >= 30, and a central difference
 *     with lag 1e-9 where nu (x < 8.5) or nu + 1/2 (x >= 30) lies within 1e-6
 *     of an integer; the prefactor derivative is exact in both modes.  Its
 *     truncation and cancellation errors (up to ~1e-6 relative near x = 8.5,
 *     more as nu approaches an integer) move the score and the fit; this
 *     mode exists to measure that.
 * Affects fbt_eval, fbt_eval_terms, fbt_grad, fbt_fit and fbt_covariance(which = 2).
 * Errors: FBT_EINVAL (NULL context or unknown mode). */
typedef enum { FBT_SIGMA_NU_EXACT = 0, FBT_SIGMA_NU_PAPER = 1 } fbt_sigma_nu_mode;
fbt_status fbt_set_sigma_nu_mode(fbt_ctx *ctx, int32_t mode);

/* Iterative refinement under FBT_MIXED_FP32_ALL and FBT_MIXED_BF16_ALL (ignored otherwise and in
 * batched groups): after the factorisation, `iterations` steps (default 0)
 *   w <- w + (L L^T)^{-1} (Z - Sigma w),   w_0 = (L L^T)^{-1} Z,
 * with the residual in FP64 from a copy of Sigma taken before the
 * factorisation (8 npad^2 more bytes of device memory while the form is in
 * use), L the factor with FP32 or bfloat16 trailing updates; then Z^T Sigma^{-1} Z =
 * Z^T w, and in fbt_eval w^T Sigma_i w from the derivative matrices.  Each
 * step costs one product with Sigma and two triangular solves with the
 * factor.  The log-likelihood and score are not always closer to FP64 with
 * it: without refinement every term is that of the factor's own matrix
 * L L^T, and near the data's maximum-likelihood theta the first-order errors
 * of the log-determinant / traces and of the quadratic forms cancel (the
 * derivative of l in Sigma, (w w^T - Sigma^{-1}) / 2, averages to zero
 * there); refinement removes the second part only.  Far from it refinement
 * helps.  Hence the default 0.
 * Errors: FBT_EINVAL (NULL context, iterations outside [0, 16]); fbt_loglik
 * and the evaluations return FBT_ENOMEM if the copy cannot be allocated. */
fbt_status fbt_set_refinement(fbt_ctx *ctx, int32_t iterations);

/* Form of the W phase of fbt_eval / fbt_eval_terms / fbt_fit: the matrices
 * W_i = L^{-1} Sigma_i L^{-T}, i in {alpha, nu}, whose traces and Frobenius
 * products give the score and Fisher information (Eqs. (2), (3), (5)).
 *   FBT_WPHASE_TWO_SIDED (default): a blocked two-sided reduction.  Per block
 *     step k it forms W_kk = L_kk^{-1} S_kk L_kk^{-T}, Y = S_ik L_kk^{-T} - L_ik W_kk / 2
 *     and M = Y - L_ik W_kk / 2, updates the trailing lower blocks by
 *     S -= Y L^T + L Y^T, and solves L^{-1} M for the blocks below the
 *     diagonal: n^3 flops per matrix.
 *   FBT_WPHASE_SOLVES: the left block solve X_i = L^{-1} Sigma_i followed by
 *     the lower half of X_i L^{-T} (4 n^3 / 3 flops per matrix).
 * In the mixed precisions (fbt_precision) the O(n^3) updates of either form
 * are the low-precision ones.
 * Both forms give the same nine terms up to rounding.  If the two-sided
 * form's extra device memory (about 32 NB n_pad + 16 NB^2 (n_pad / NB) bytes,
 * NB = 256) cannot be allocated, the evaluation takes the block solves.
 * Errors: FBT_EINVAL (NULL context or unknown form). */
typedef enum { FBT_WPHASE_TWO_SIDED = 0, FBT_WPHASE_SOLVES = 1 } fbt_wphase;
fbt_status fbt_set_wphase(fbt_ctx *ctx, int32_t form);

/* ---- Allocation-free evaluation ------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * result as fbt_eval (log-likelihood, score, Fisher information; FP64, exact
 * Sigma_nu, two-sided W phase) for one field of 1 <= n <= FBT_NOALLOC_MAX_N
 * observations, with no context and no allocation: every device buffer lives
 * in one static array of the library (about 50 MB per GPU, held by each GPU
 * the library runs on from the library's load until the process ends; its
 * address on a device is looked up on the first call there).
 *   device      HIP device ordinal (< 16); made current for the call.
 *   hip_stream  hipStream_t the work is ordered on (NULL: the null stream);
 *               the call waits for it before returning.
 *   d_locs_xy   device, n x 2 row-major locations (x_i, y_i); read only.
 *   d_z         device, n observations; read only.
 *   theta, loglik, score[3], fisher[9] (row-major): host, as in fbt_eval.
 * The inputs stay owned by the caller.  Calls on one GPU share its array,
 * which keeps the last call's contents: calls that overlap on one GPU (from
 * several host threads, or on streams that run concurrently) race and must
 * be serialised by the caller.  Calls on different GPUs are independent.
 * Errors: FBT_EINVAL (NULL pointer, theta not finite and > 0, n out of range,
 * device >= 16, a non-finite location or observation), FBT_ENOTPD,
 * FBT_ENONFINITE, FBT_EDEVICE. */
#define FBT_NOALLOC_MAX_N 1023
fbt_status fbt_eval_noalloc(int32_t device, void *hip_stream, int64_t n, const double *d_locs_xy,
                            const double *d_z, const double theta[3], double *loglik,
                            double score[3], double fisher[9]);

/* Per-kernel-class timing with HIP events recorded on the context's stream.
 * enable != 0 starts recording (and clears the counters); 0 stops it. */
fbt_status fbt_set_timing(fbt_ctx *ctx, int32_t enable);
/* Kernel classes: 0 generation, 1 diagonal factor+inverse, 2 panel solve,
 * 3 trailing Cholesky update, 4 left-solve diagonal apply, 5 left-solve update,
 * 6 right-solve panel with trace reductions, 7 right-solve update, 8 reductions,
 * 9 inverse of the factor (adjoint), 10 X^T X product (adjoint),
 * 11 adjoint fill / extraction / contraction with the regenerated derivatives,
 * 12 two-sided W phase: diagonal blocks, 13 its panels (Y, M), 14 its symmetric
 * rank-2k trailing updates, 15 its deferred solve's diagonal apply, 16 the
 * deferred solve's updates, 17 its rank-2k updates of the next block columns.
 * Returns launches, summed milliseconds and summed algorithmic flops of the
 * class since timing was enabled (timing must have been enabled). */
fbt_status fbt_get_timing(fbt_ctx *ctx, int32_t kernel_class, int64_t *launches, double *ms,
                          double *flops);

#ifdef __cplusplus
}
#endif
#endif /* FISHERBT_H */
