/*
 * spmesl.h -- C ABI of the MI355X (gfx950) SPMESL library.
 *
 * SPMESL estimates a sparse precision matrix by p column-wise scaled-lasso
 * regressions (Lee, Kim & Yu, arXiv 2203.15031; Sun & Zhang's scaled lasso).
 * For data X (n x p) the library
 *   1. centres every column and scales it to x_k^T x_k = n (Section 2.2,
 *      the paragraph after Eq. (eq:spmesl));
 *   2. forms the sample covariance S = X^T X / n of the standardised data;
 *   3. for every column k solves the scaled lasso of Eq. (eq:spmesl),
 *        min_{beta: beta_kk = 0, sigma > 0}
 *            ||x_k - X beta||^2 / (2 n sigma) + sigma / 2 + lambda0 ||beta||_1,
 *      by the block coordinate descent of Section 2.1 / Algorithm 1:
 *      a lasso step at lambda = sigma * lambda0 solved by cyclic coordinate
 *      descent in ascending order (Section 3.1), then the noise update
 *      sigma = ||x_k - X beta||_2 / sqrt(n) (Eq. (eq:sigma)), repeated until
 *      |delta sigma| < tol;
 *   4. forms Omega_1 = -B D with D = diag(sigma^-2) (Eq. (eq:relation)) and
 *      applies the min-magnitude symmetrisation of Eq. (eq:symm);
 *   5. maps the result back to the scale of the data (Proposition 1) unless
 *      the standardised scale is asked for.
 *
 * Conventions
 *   - Every pointer in a problem or result struct is a DEVICE pointer owned
 *     by the caller unless the field says "host".  Matrices are row-major.
 *   - B is p x p with B[j*p + k] = beta_jk: column k holds the regression
 *     coefficients of response k, and the diagonal is 0 (the beta_kk = 0
 *     convention of Section 3.3).
 *   - Omega is p x p, symmetric bit for bit.
 *   - Calls are enqueued on the context's HIP stream.  spmesl_solve returns
 *     after the stream work it enqueued has finished and the status has
 *     been read back.
 *   - Functions return 0 (SPMESL_OK) or a negative SPMESL_E* code.  No C++
 *     exception crosses this interface.  After an error other than
 *     SPMESL_ENOCONV the outputs are undefined.  spmesl_last_error()
 *     returns a message for the last failing call on a context.
 *   - A context is not thread-safe; use one context per host thread/stream.
 */
#ifndef SPMESL_H
#define SPMESL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPMESL_VERSION_MAJOR 0
#define SPMESL_VERSION_MINOR 1

/* ---- status codes ----------------------------------------------------- */
#define SPMESL_OK 0
#define SPMESL_EINVAL (-1)      /* bad argument: NULL, n < 2, p < 2, ldx < p,
                                   lambda0 <= 0, tol <= 0, unknown enum */
#define SPMESL_ENONFINITE (-2)  /* NaN or Inf in X */
#define SPMESL_EZEROVAR (-3)    /* a column of X has zero variance, so the
                                   scale of Proposition 1 is undefined */
#define SPMESL_EDEGENERATE (-4) /* some sigma_k^2 fell to <= 1e-12 of the
                                   standardised variance (perfect fit) */
#define SPMESL_ENOCONV (-5)     /* an iteration cap was reached; outputs hold
                                   the last iterate and stats flag the columns */
#define SPMESL_EHIP (-6)        /* HIP runtime error */
#define SPMESL_ENOMEM (-7)      /* workspace allocation failed or the caller's
                                   workspace is too small */
#define SPMESL_EWORKSET (-8)    /* the dense tier ran out of room: the long
                                   supports of one solve together exceeded
                                   32p + 65536 entries, or (mixed form) the
                                   double stage of a group of wide columns
                                   needed more than 1024 variables */

/* Largest working set one LDS tier holds.  Columns whose working sets grow
 * beyond it are finished by the dense tier, which has no such bound (the
 * union of a group's working sets may reach p). */
#define SPMESL_MAX_WORKING_SET 128

/* ---- enums -------------------------------------------------------------- */
/* Arithmetic of the solve. */
#define SPMESL_FP64 0   /* S, coordinate descent and checks in double */
#define SPMESL_FP32 1   /* S and coordinate descent in float; tolerance
                           floored at SPMESL_FP32_TOL_FLOOR */
#define SPMESL_MIXED 2  /* S from a two-term bfloat16 split on the matrix
                           cores with float accumulation, float coordinate
                           descent, then a double-precision polish of every
                           column (its scaled-lasso fixed point and its KKT
                           conditions) so that results meet tol in double */

#define SPMESL_FP32_TOL_FLOOR 1e-6

/* Scale of the outputs. */
#define SPMESL_SCALE_ORIGINAL 0     /* Proposition 1: Omega^o = C Omega C with
                                       C = diag(s_jj^-1/2); b^o_jk = (c_j/c_k) b_jk;
                                       sigma^o_k = sigma_k / c_k */
#define SPMESL_SCALE_STANDARDIZED 1 /* results of the standardised problem */

/* ---- structs ----------------------------------------------------------- */
typedef struct spmesl_ctx spmesl_ctx;

typedef struct {
    const double *X; /* device, n x p row-major, row stride ldx (elements) */
    int64_t n;       /* samples, >= 2 */
    int64_t p;       /* variables, >= 2 */
    int64_t ldx;     /* >= p */
    /* Optional warm start of Algorithm 1 (NULL: the paper's start, beta = 0
     * and sigma = 1 for every column).  Device arrays in the scale of the
     * outputs (options.output_scale), so a result can be passed back in:
     * B0 is p x p row-major like the output B (column k = the coefficients
     * of response k; its diagonal is ignored, and at most
     * SPMESL_MAX_WORKING_SET nonzeros per column are used, the first in row
     * order), sigma0 has p entries (an entry that is not a positive finite
     * number starts that column at sigma = 1).  The minimiser is unique, so
     * a warm start changes the work, not the result: it resumes a solve that
     * stopped at an iteration cap (SPMESL_ENOCONV), or follows a path of
     * penalties.  Ignored by spmesl_covariance; spmesl_scaled_lasso refuses
     * it (SPMESL_EINVAL). */
    const double *B0;
    const double *sigma0;
} spmesl_problem;

typedef struct {
    double lambda0;      /* penalty level lambda0 > 0 of Eq. (eq:spmesl) */
    double tol;          /* delta of Algorithms 1-3: inner stop when the
                            largest coefficient change of a sweep is < tol,
                            outer stop when |delta sigma| < tol */
    int32_t max_outer;   /* cap on sigma updates per column (<= 0: 1000) */
    int32_t max_sweeps;  /* cap on sweeps of one lasso step (<= 0: 100000) */
    int32_t max_rounds;  /* cap on working-set growth rounds (<= 0: 64) */
    int32_t precision;   /* SPMESL_FP64 | SPMESL_FP32 | SPMESL_MIXED */
    int32_t output_scale;/* SPMESL_SCALE_ORIGINAL | SPMESL_SCALE_STANDARDIZED */
    int32_t flags;       /* SPMESL_FLAG_TIMING | SPMESL_FLAG_EAGER |
                            SPMESL_FLAG_FULL_KKT | SPMESL_FLAG_DATA_FORM */
} spmesl_options;

#define SPMESL_FLAG_TIMING 1
/* Enqueue the kernels one by one instead of replaying the context's cached
 * HIP graph of the call (the default for calls that repeat the pointers,
 * sizes and options of the previous call; timed calls are always eager). */
#define SPMESL_FLAG_EAGER 2
/* Mixed form: the double polish proves every column by a full pass over S
 * (every j with |g_j| within the float error bound of lambda joins the
 * double working set, which is then re-solved), instead of accepting a
 * column when the change of its gradient since the float solve is provably
 * smaller than the float near-threshold band.  Slower; the same minimiser. */
#define SPMESL_FLAG_FULL_KKT 4
/* The data form of Algorithm 3 (double precision only): no p x p S is
 * formed.  Every column is solved by the dense tier with the standardised
 * data as its source of S: groups of 16 columns, S restricted to the union V
 * of the group's working sets formed from the data, blocked sweeps on V, and
 * the full gradient X^T (x_k - X_V beta) / n for the KKT check.  Memory grows
 * with n p, not p^2, so it serves p beyond what an S fits (and n << p).  A
 * group whose V would exceed 1024 variables fails with SPMESL_EWORKSET. */
#define SPMESL_FLAG_DATA_FORM 8

typedef struct {
    /* host-side counters filled by a solve */
    int64_t columns;          /* p */
    int64_t total_outer;      /* sum over columns of sigma updates */
    int64_t max_outer;        /* largest per-column count of sigma updates */
    int64_t total_sweeps;     /* sum over columns of coordinate sweeps */
    int64_t total_updates;    /* nonzero coordinate changes */
    int64_t total_rounds;     /* working-set rounds summed over columns */
    int64_t max_working_set;  /* largest working set of any column */
    int64_t nnz_B;            /* nonzero off-diagonal coefficients */
    int64_t columns_noconv;   /* columns that hit a cap */
    int64_t polish_kkt_checks;/* double-precision KKT checks (mixed form) */
    int64_t polish_added;     /* variables the polish added (mixed form) */
    int64_t sum_working_set;  /* sum over columns of the final working-set
                                 sizes (in the mixed form, the polish's) */
    int64_t resolved_columns; /* columns the row-tiled KKT pass sent back for
                                 a re-solve */
    int64_t escalated_columns;/* columns handed to the 128-coordinate tier */
    /* phase times in milliseconds (only with SPMESL_FLAG_TIMING) */
    double ms_standardize, ms_covariance, ms_solve, ms_polish, ms_output, ms_total;
} spmesl_stats;

typedef struct {
    double *B;           /* device p x p or NULL (not written) */
    double *sigma;       /* device p or NULL */
    double *Omega;       /* device p x p or NULL */
    spmesl_stats *stats; /* HOST pointer or NULL */
} spmesl_result;

/* ---- lifetime ------------------------------------------------------------ */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The context owns a workspace that
 * grows on demand (hipMalloc) unless the caller supplies one. */
int spmesl_create(spmesl_ctx **ctx, int device, void *hip_stream);
void spmesl_destroy(spmesl_ctx *ctx);
int spmesl_set_stream(spmesl_ctx *ctx, void *hip_stream);
const char *spmesl_last_error(const spmesl_ctx *ctx);
const char *spmesl_version(void);

/* Workspace (device bytes) a solve of this shape and precision needs. */
int spmesl_workspace_size(const spmesl_problem *prob, const spmesl_options *opt,
                          size_t *bytes);
/* Hand the context a caller-owned device workspace (NULL releases it, and the
 * context goes back to allocating its own).  The memory must stay valid
 * until replaced or the context is destroyed. */
int spmesl_set_workspace(spmesl_ctx *ctx, void *device_ptr, size_t bytes);

/* ---- the solve ------------------------------------------------------------ */

/* Full SPMESL (steps 1-5 above) of one data matrix.  Output arrays that are
 * NULL are skipped.  Returns SPMESL_OK, SPMESL_ENOCONV (with the last
 * iterate), or an error code. */
int spmesl_solve(spmesl_ctx *ctx, const spmesl_problem *prob,
                 const spmesl_options *opt, spmesl_result *res);

/* As spmesl_solve, but returns once the work is enqueued on the context's
 * stream (host-side argument errors are still returned at once).  When the
 * solve completes on the stream, its status code (SPMESL_OK, SPMESL_ENOCONV
 * or an error code, as spmesl_solve would return) is written to the int at
 * `status_dev` (device memory, caller-owned).  No stats are reported.  The
 * outputs and *status_dev are valid once the stream has reached that point
 * (synchronise the stream or an event recorded after the call); the
 * context's workspace is reused by the next call on the same stream, which
 * stream order makes safe. */
int spmesl_solve_async(spmesl_ctx *ctx, const spmesl_problem *prob,
                       const spmesl_options *opt, spmesl_result *res, int *status_dev);

/* Size of the device array spmesl_solve_noalloc works in (64 MiB). */
#define SPMESL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * spmesl_solve_async, enqueued kernel by kernel, with every intermediate
 * buffer in one fixed device array of SPMESL_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU until the process ends.  The call allocates
 * nothing (no hipMalloc, no pinned host memory, no graph instantiation); the
 * caller passes X, the outputs and the device int `status_dev`, which
 * receives the status code when the solve completes on the stream, as for
 * spmesl_solve_async.  A problem whose workspace (spmesl_workspace_size) does
 * not fit the array is refused with SPMESL_ENOMEM before anything is
 * enqueued (64 MiB holds, for example, n = 1024, p = 2048 in every
 * precision).  Every call on one GPU, from any context, uses that GPU's one
 * array: calls whose stream work overlaps on the same GPU race and give
 * undefined results, so order them on one stream (or synchronise between
 * them).  SPMESL_FLAG_TIMING and SPMESL_FLAG_EAGER are ignored; no stats are
 * reported.  SPMESL_EHIP if the array's device address could not be found
 * when the context was created. */
int spmesl_solve_noalloc(spmesl_ctx *ctx, const spmesl_problem *prob,
                         const spmesl_options *opt, spmesl_result *res, int *status_dev);

/* The batched form (the paper's simulation study solves many independent
 * data sets per setting: Section 4.1, Tables 1-4).
 * Solve `count` independent problems (uneven n, p) with the same options,
 * except that problem i uses lambda0s[i] when lambda0s (HOST array of count
 * doubles) is not NULL.  status[i] (host) receives each problem's code; the
 * return value is the first non-OK code, or SPMESL_OK.
 * In the covariance forms (not SPMESL_FLAG_DATA_FORM; no warm starts; two or
 * more problems; every p within the row-tiled KKT pass's reach: p up to about
 * 20000 in float and mixed, 10000 in double) the problems run grouped: each step of the path is one launch over the work of
 * every problem (the covariance tiles, the first solves, the KKT pass, the
 * re-solves, the escalations and the polish), each problem with its own
 * workspace region; the results equal those of the problems' single solves
 * bit for bit.  Otherwise the problems run one after another.  Either way the
 * work goes on the context's stream, as one graph launch when the call
 * repeats the previous call's pointers, sizes and options. */
int spmesl_solve_batch(spmesl_ctx *ctx, int count, const spmesl_problem *probs,
                       const spmesl_options *opt, const double *lambda0s,
                       spmesl_result *res, int *status);
/* Workspace (device bytes) spmesl_solve_batch needs for these problems:
 * grouped, every problem's workspace, a control block per problem and the
 * launch tables; one after another, the largest problem's workspace and a
 * control block per problem. */
int spmesl_batch_workspace_size(const spmesl_ctx *ctx, int count, const spmesl_problem *probs,
                                const spmesl_options *opt, size_t *bytes);

/* ---- launch shapes and the autotuner ------------------------------------ */

/* Launch shapes a context applies to its solves.  None of them changes the
 * minimiser; they change how the work is laid out (and, for the screen and
 * the dense tier's block size, which path the iterates take).  0 in a field
 * selects the default. */
typedef struct {
    int32_t dense_block;      /* b, rows per block of the dense tier's delayed
                                 rank-b update (Proposition 2 blocked): 16, 32
                                 or 64 (default 32) */
    int32_t fill_blocks;      /* workgroups of the dense outputs' zero fill,
                                 which runs beside the covariance kernel
                                 (default 64) */
    int32_t kkt_rows;         /* rows of S per tile of the row-tiled KKT pass:
                                 1, 2 or 4 (default: the most that fit LDS) */
    int32_t screen_permille;  /* first working sets {j : |s_jk| > f lambda0 +
                                 tol}, f in thousandths (default 800) */
    int32_t fill_split;       /* where the zero fill of the dense outputs runs:
                                 0 both beside the covariance kernel (default),
                                 1 Omega's after the row-tiled KKT pass, 2 both
                                 after it */
} spmesl_tuning;

/* Set (NULL: reset to the defaults) or read the context's launch shapes. */
int spmesl_set_tuning(spmesl_ctx *ctx, const spmesl_tuning *t);
int spmesl_get_tuning(const spmesl_ctx *ctx, spmesl_tuning *t);

/* Autotuner: times solves of this problem (graph replays, the fastest of
 * three runs of `reps` per candidate, HIP events on the context's stream;
 * a candidate must be at least 1% faster to be kept) over the candidate values
 * of each field in turn (coordinate search from the current shapes: screen
 * 700/800/900/1000, KKT rows 4/2/1 as they fit, fill 32/64/128/256
 * workgroups, fill placement 0/1/2, dense block 16/32/64 when the problem
 * reaches the dense tier),
 * keeps the fastest, sets it on the context and writes it to *best (host,
 * may be NULL) with its time per solve in *ms_best (host, may be NULL).  The
 * outputs in `res` hold the last solve's result.  Allocates (workspace,
 * graphs, a status word).  Returns SPMESL_OK or the first error of a solve. */
int spmesl_autotune(spmesl_ctx *ctx, const spmesl_problem *prob, const spmesl_options *opt,
                    spmesl_result *res, int reps, spmesl_tuning *best, double *ms_best);

/* Kernel times of the last spmesl_solve run with SPMESL_FLAG_TIMING: one
 * entry per launch step in enqueue order, `names[i]` a static string naming
 * the kernel(s) and `ms[i]` its duration in milliseconds, from HIP events
 * recorded on the stream the step ran on (the zero fill of the dense outputs
 * runs on the context's second stream).  Fills at most `cap` entries (names
 * and ms may be NULL when cap is 0) and returns the number of steps
 * recorded, or SPMESL_EINVAL / SPMESL_EHIP. */
int spmesl_kernel_times(const spmesl_ctx *ctx, int cap, const char **names, double *ms);

/* ---- single steps (each is also a step of spmesl_solve) ---------------- */

/* Steps 1-2: standardise X and form S.  S is p x p row-major, double when
 * precision is SPMESL_FP64 and float (S_out must then point to floats)
 * otherwise; its diagonal is exactly 1.  mean and scale (c_k = s_kk^-1/2 of
 * the centred data), device arrays of p doubles, may be NULL. */
int spmesl_covariance(spmesl_ctx *ctx, const spmesl_problem *prob, int precision,
                      void *S_out, double *mean, double *scale);

/* The scaled lasso on its own (Section 3.1, Algorithm 1; objective Eq. (1)),
 * for m responses Y (device, n x m row-major, row stride ldy >= m) on the
 * design prob->X (n x p, p >= 1).  Each response is treated as SPMESL treats
 * one of its variables: the columns of X and of Y are centred and scaled to
 * unit variance, and response r is regressed on the p design columns only
 * (never on the other responses):
 *     (beta_r, sigma_r) = argmin_{beta, sigma > 0}
 *         ||y_r - X beta||^2 / (2 n sigma) + sigma / 2 + lambda0 ||beta||_1
 * by Algorithm 1 in covariance form from beta = 0, sigma = 1.  Outputs
 * (device, caller-owned): beta, p x m row-major (column r = beta_r, every
 * entry written), and sigma[m]; with SPMESL_SCALE_ORIGINAL these are on the
 * caller's scales (Proposition 1 with the response as column k:
 * beta_jr * c_j / c_r and sigma_r / c_r, i.e. the coefficients of the raw x_j
 * for the centred y_r, and the noise level in y_r's units), with
 * SPMESL_SCALE_STANDARDIZED those of the standardised problem.  outer
 * (device int[m], or NULL) receives each response's count of sigma updates.
 * opt: lambda0, tol, the caps and output_scale as for spmesl_solve;
 * precision must be SPMESL_FP64 (else SPMESL_EINVAL).  stats (host, or NULL)
 * counts over the m regressions.  Returns after the work is done: SPMESL_OK,
 * SPMESL_ENOCONV, or an error code as spmesl_solve (SPMESL_EZEROVAR also for
 * a constant response).  The workspace holds S of the p + m variables. */
int spmesl_scaled_lasso(spmesl_ctx *ctx, const spmesl_problem *prob, const double *Y,
                        int64_t m, int64_t ldy, const spmesl_options *opt, double *beta,
                        double *sigma, int *outer, spmesl_stats *stats);
/* Workspace (device bytes) spmesl_scaled_lasso needs for n samples, p design
 * columns and m responses. */
int spmesl_scaled_lasso_workspace_size(int64_t n, int64_t p, int64_t m, size_t *bytes);

/* Step 4's symmetrisation alone (Eq. (eq:symm)): Omega = symm(Omega1), p x p
 * row-major device arrays; for j < k both entries become the one of smaller
 * magnitude, and on a tie the upper entry Omega1[j*p+k]. */
int spmesl_symmetrize(spmesl_ctx *ctx, int64_t p, const double *Omega1,
                      double *Omega);

/* ---- penalty levels (host, pure; Section 2.2) --------------------------- */
/* lambda_univ = sqrt(2 log(p-1) / n). */
double spmesl_lambda_univ(double n, double p);
/* lambda_ub = sqrt(4 log p / n): the union bound over p scaled lassos. */
double spmesl_lambda_ub(double n, double p);
/* lambda_pb = sqrt(2) L_n(k/p), L_n(t) = n^-1/2 Phi^-1(1 - t), with k the
 * root in (0, p/2) of k = L_1^4(k/p) + 2 L_1^2(k/p).  Writes lambda_pb and
 * (if k_out != NULL) k.  Returns SPMESL_OK or SPMESL_EINVAL. */
int spmesl_lambda_pb(double n, double p, double *lambda_out, double *k_out);

#ifdef __cplusplus
}
#endif
#endif /* SPMESL_H */
