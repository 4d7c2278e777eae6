/*
 * spmesl_oracle.c -- plain FP64 CPU reference for SPMESL (scaled-lasso sparse
 * precision matrix estimation), Lee, Kim & Yu, "An efficient GPU-parallel
 * coordinate descent algorithm for sparse precision matrix estimation via
 * scaled lasso" (arXiv 2203.15031).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library.
 *
 * What it computes, and where the paper defines it:
 *   - standardisation: centre every column and scale it so that x_k^T x_k = n
 *     (Section 2.2, the paragraph after Eq. (eq:spmesl));
 *   - the scaled lasso of one response by Algorithm 1 (cyclic coordinate
 *     descent in ascending order with warm start; the update equations of
 *     Section 3.1, Eq. (eqn:lasso));
 *   - SPMESL by Algorithm 2: Algorithm 1 on every column k with design
 *     X_{-k}, then Omega_1 = -B D (Eq. (eq:relation)), then the
 *     min-magnitude symmetrisation (Eq. (eq:symm));
 *   - the map back to the original scale of the data (Proposition 1);
 *   - the three penalty levels of Section 2.2 (union bound, probabilistic
 *     bound, universal level).
 *
 * All arithmetic is IEEE double; the only parallelism is over the p
 * independent column problems of Algorithm 2 (OpenMP), which does not change
 * any column's arithmetic.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *   R1  In Algorithm 1 the residual e_j is the full residual with the
 *       current value of beta_j still in it, so a_j = x_j^T e / n + beta_j is
 *       the exact coordinate minimiser (this is the form Proposition 2 uses;
 *       the sum over l > j in Section 3.1 read literally would count beta_j
 *       twice).
 *   R2  Soft_lambda(a) at |a| = lambda is 0.
 *   R3  In Algorithm 2, omega_kk in omega_jk = -beta_jk * omega_kk is
 *       sigma_k^{-2}, so the diagonal is formed before the off-diagonal
 *       entries (the pseudo-code's loop order would read it before it is
 *       set).
 *   R4  Symmetrisation tie |omega_jk| == |omega_kj| (j < k) keeps the upper
 *       entry omega_jk (the else-branch of Algorithm 2, and Eq. (eq:symm)).
 *   R5  The covariance normalisation is 1/n after centring.
 *   R6  The penalty of Proposition 1's original-scale problem is
 *       lambda0 * sum_j sqrt(s_jj) |beta_jk|, so the original-scale outputs
 *       are b^o_jk = (c_j / c_k) b_jk, sigma^o_k = sigma_k / c_k and
 *       omega^o_jk = c_j c_k omega_jk with c_k = s_kk^{-1/2}.
 *   R7  The probabilistic-bound equation is k = L_1^4(k/p) + 2 L_1^2(k/p)
 *       (the form that the worked example k = 23.4748 at p = 1000
 *       satisfies); its root is taken in (0, p/2).
 *
 * Status codes returned by every entry point: 0 ok, -1 bad argument,
 * -2 zero-variance column, -3 iteration cap reached (outputs hold the last
 * iterate), -4 non-finite input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EZEROVAR (-2)
#define ORC_ENOCONV (-3)
#define ORC_ENONFINITE (-4)

/* Planted mistakes for the self-test of the pins (tests build this file with
 * -DORACLE_MUTANT=m and expect some pin to fail).  0 = the real oracle. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* Soft_lambda(a) = sign(a) (|a| - lambda)_+  (Section 3.1). */
static double soft(double a, double lambda)
{
#if ORACLE_MUTANT == 1
    /* mutant: wrong sign on the shrinkage */
    if (a > lambda) return a + lambda;
    if (a < -lambda) return a - lambda;
    return 0.0;
#else
    if (a > lambda) return a - lambda;
    if (a < -lambda) return a + lambda;
    return 0.0;
#endif
}

static double dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/*
 * Standardisation (Section 2.2): x_k <- (x_k - mean_k) * c_k with
 * c_k = (sum_i (x_ik - mean_k)^2 / n)^{-1/2}, so that x_k^T x_k = n.
 * X and Xs are column-major n x p (column k starts at k*n).  mean and c
 * receive the per-column mean and scale.  Xs may alias X.
 */
int oracle_standardize(int64_t n, int64_t p, const double *X, double *Xs,
                       double *mean, double *c)
{
    if (n < 2 || p < 1 || !X || !Xs || !mean || !c) return ORC_EINVAL;
    for (int64_t k = 0; k < p; ++k) {
        const double *x = X + k * n;
        double m = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!isfinite(x[i])) return ORC_ENONFINITE;
            m += x[i];
        }
        m /= (double)n;
#if ORACLE_MUTANT == 2
        m = 0.0; /* mutant: no centring */
#endif
        double ss = 0.0;
        for (int64_t i = 0; i < n; ++i) ss += (x[i] - m) * (x[i] - m);
        if (!(ss > 0.0)) return ORC_EZEROVAR;
#if ORACLE_MUTANT == 3
        double ck = 1.0 / sqrt(ss / (double)(n - 1)); /* mutant: 1/(n-1) */
#else
        double ck = 1.0 / sqrt(ss / (double)n);
#endif
        mean[k] = m;
        c[k] = ck;
        double *xs = Xs + k * n;
        for (int64_t i = 0; i < n; ++i) xs[i] = (x[i] - m) * ck;
    }
    return ORC_OK;
}

/*
 * Scaled lasso of y on the columns of X (Algorithm 1), with coordinate
 * `skip` held at beta_skip = 0 (Eq. (eq:sublasso); pass skip = -1 for no
 * such coordinate).  X is column-major n x p and is used as given: the
 * caller standardises when the problem calls for it (every column is assumed
 * to satisfy x_j^T x_j = n, which is what makes the coordinate minimiser a
 * plain soft-threshold).
 *
 * On entry beta[p] and *sigma hold the starting point (Algorithm 1 starts
 * from beta = 0, sigma = 1); on exit they hold beta^(r+1), sigma^(r+1) of the
 * last outer iteration.  e is scratch of length n.  The counts of outer
 * iterations and of inner sweeps (summed over outer iterations) are written
 * to *n_outer and *n_sweeps when those are not NULL.
 *
 * The inner loop stops when max_j |beta_j^[next] - beta_j^[cur]| < tol, the
 * outer loop when |sigma^(r+1) - sigma^(r)| < tol.  max_outer caps the outer
 * iterations and max_sweeps the sweeps of any one inner loop; hitting either
 * cap returns ORC_ENOCONV with the last iterate.
 */
int oracle_scaled_lasso(int64_t n, int64_t p, const double *X, const double *y,
                        int64_t skip, double lambda0, double tol, int max_outer,
                        int max_sweeps, double *beta, double *sigma, double *e,
                        int *n_outer, int *n_sweeps)
{
    if (n < 1 || p < 1 || !X || !y || !beta || !sigma || !e || !(tol > 0.0) ||
        max_outer < 1 || max_sweeps < 1)
        return ORC_EINVAL;
    int status = ORC_ENOCONV;
    int outer = 0, sweeps_total = 0;
    double sig = *sigma;
    if (skip >= 0 && skip < p) beta[skip] = 0.0;

    for (int r = 0; r < max_outer; ++r) {
        ++outer;
        /* lambda <- sigma^(r) lambda0 */
        double lambda = sig * lambda0;
        /* residual of the warm start: e = y - X beta^(r) */
        for (int64_t i = 0; i < n; ++i) e[i] = y[i];
        for (int64_t l = 0; l < p; ++l)
            if (beta[l] != 0.0) {
                const double *xl = X + l * n;
                for (int64_t i = 0; i < n; ++i) e[i] -= xl[i] * beta[l];
            }
        /* cyclic coordinate descent, ascending order, until the largest
         * change of one sweep is below tol */
        int inner_ok = 0;
        for (int m = 0; m < max_sweeps; ++m) {
            ++sweeps_total;
            double maxdiff = 0.0;
            for (int64_t j = 0; j < p; ++j) {
                if (j == skip) continue;
                const double *xj = X + j * n;
#if ORACLE_MUTANT == 4
                double a = dot(n, xj, e) / (double)n; /* mutant: drops +beta_j */
#else
                double a = dot(n, xj, e) / (double)n + beta[j];
#endif
                double bnew = soft(a, lambda);
                double d = bnew - beta[j];
                if (d != 0.0) {
                    /* keep e = y - X beta with beta_j now at bnew */
                    for (int64_t i = 0; i < n; ++i) e[i] -= xj[i] * d;
                    beta[j] = bnew;
                }
                if (fabs(d) > maxdiff) maxdiff = fabs(d);
            }
            if (maxdiff < tol) {
                inner_ok = 1;
                break;
            }
        }
        /* sigma^(r+1) = ||y - X beta^(r+1)||_2 / sqrt(n), from scratch */
        for (int64_t i = 0; i < n; ++i) e[i] = y[i];
        for (int64_t l = 0; l < p; ++l)
            if (beta[l] != 0.0) {
                const double *xl = X + l * n;
                for (int64_t i = 0; i < n; ++i) e[i] -= xl[i] * beta[l];
            }
#if ORACLE_MUTANT == 5
        double signew = dot(n, e, e) / (double)n; /* mutant: variance, not sd */
#else
        double signew = sqrt(dot(n, e, e) / (double)n);
#endif
        double dsig = fabs(signew - sig);
        sig = signew;
        if (!inner_ok) break; /* inner cap hit: report the last iterate */
        if (dsig < tol) {
            status = ORC_OK;
            break;
        }
    }
    *sigma = sig;
    if (n_outer) *n_outer = outer;
    if (n_sweeps) *n_sweeps = sweeps_total;
    return status;
}

/*
 * Min-magnitude symmetrisation of Algorithm 2 / Eq. (eq:symm), in place on a
 * column-major p x p matrix W (W[j + k*p] = omega_jk): for j < k, both
 * entries of the pair become the entry of smaller magnitude; on a tie the
 * upper entry omega_jk is kept (reading R4).
 */
void oracle_symmetrize(int64_t p, double *W)
{
    for (int64_t j = 0; j < p - 1; ++j)
        for (int64_t k = j + 1; k < p; ++k) {
            double *wjk = &W[j + k * p];
            double *wkj = &W[k + j * p];
#if ORACLE_MUTANT == 6
            if (fabs(*wjk) < fabs(*wkj)) /* mutant: keeps the larger one */
#else
            if (fabs(*wjk) > fabs(*wkj))
#endif
                *wjk = *wkj;
            else
                *wkj = *wjk;
        }
}

/*
 * SPMESL by Algorithm 2 on the n x p data matrix X (column-major).
 *
 *   lambda0, tol, max_outer, max_sweeps : as in oracle_scaled_lasso.
 *   original_scale : 0 -> outputs on the standardised scale;
 *                    1 -> outputs mapped back by Proposition 1 (reading R6).
 *   B      [p*p] out, column-major, column k = beta_{-k}, zero diagonal.
 *   sigma  [p]   out.
 *   Omega  [p*p] out, column-major, symmetric.
 *   Omega1 [p*p] out or NULL: -B D before symmetrisation (same scale).
 *   mean, c [p] out or NULL: per-column mean and scale of the data.
 *   n_outer, n_sweeps [p] out or NULL: per-column iteration counts.
 *   col_status [p] out or NULL: per-column status of Algorithm 1.
 *   nthreads : OpenMP threads over the columns (<= 0 -> runtime default).
 *
 * Returns ORC_OK, or the first non-zero column status (ORC_ENOCONV when a
 * cap was hit), or an argument / data error before any solving.
 */
int oracle_spmesl(int64_t n, int64_t p, const double *X, double lambda0,
                  double tol, int max_outer, int max_sweeps, int original_scale,
                  double *B, double *sigma, double *Omega, double *Omega1,
                  double *mean_out, double *c_out, int *n_outer, int *n_sweeps,
                  int *col_status, int nthreads)
{
    if (n < 2 || p < 2 || !X || !B || !sigma || !Omega || !(lambda0 > 0.0) ||
        !(tol > 0.0))
        return ORC_EINVAL;
    double *Xs = (double *)malloc(sizeof(double) * (size_t)(n * p));
    double *mean = (double *)malloc(sizeof(double) * (size_t)p);
    double *c = (double *)malloc(sizeof(double) * (size_t)p);
    int *cst = (int *)malloc(sizeof(int) * (size_t)p);
    if (!Xs || !mean || !c || !cst) {
        free(Xs); free(mean); free(c); free(cst);
        return ORC_EINVAL;
    }
    int st = oracle_standardize(n, p, X, Xs, mean, c);
    if (st != ORC_OK) {
        free(Xs); free(mean); free(c); free(cst);
        return st;
    }
    memset(B, 0, sizeof(double) * (size_t)(p * p));

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* Algorithm 2, first loop: Algorithm 1 on every column k with design
     * X_{-k}, from beta = 0, sigma = 1. */
#pragma omp parallel
    {
        double *e = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < p; ++k) {
            double *bk = B + k * p;
            double sg = 1.0;
            int no = 0, ns = 0;
            cst[k] = e ? oracle_scaled_lasso(n, p, Xs, Xs + k * n, k, lambda0, tol,
                                             max_outer, max_sweeps, bk, &sg, e,
                                             &no, &ns)
                       : ORC_EINVAL;
            bk[k] = 0.0;
            sigma[k] = sg;
            if (n_outer) n_outer[k] = no;
            if (n_sweeps) n_sweeps[k] = ns;
        }
        free(e);
    }

    /* Initial estimate Omega_1 = -B D with D = diag(sigma^{-2})
     * (Eq. (eq:relation)); the diagonal first (reading R3). */
    for (int64_t k = 0; k < p; ++k) {
#if ORACLE_MUTANT == 7
        double dk = 1.0 / sigma[k]; /* mutant: sigma^{-1} instead of sigma^{-2} */
#else
        double dk = 1.0 / (sigma[k] * sigma[k]);
#endif
        for (int64_t j = 0; j < p; ++j) {
#if ORACLE_MUTANT == 8
            /* mutant: scales row j by omega_jj instead of column k by omega_kk */
            double dj = 1.0 / (sigma[j] * sigma[j]);
            Omega[j + k * p] = (j == k) ? dk : -B[j + k * p] * dj;
#else
            Omega[j + k * p] = (j == k) ? dk : -B[j + k * p] * dk;
#endif
        }
    }
    if (Omega1) memcpy(Omega1, Omega, sizeof(double) * (size_t)(p * p));
    oracle_symmetrize(p, Omega);

    if (original_scale) {
        /* Proposition 1 (reading R6). */
        for (int64_t k = 0; k < p; ++k) {
            for (int64_t j = 0; j < p; ++j) {
#if ORACLE_MUTANT == 9
                B[j + k * p] *= c[k] / c[j]; /* mutant: ratio inverted */
#else
                B[j + k * p] *= c[j] / c[k];
#endif
                Omega[j + k * p] *= c[j] * c[k];
                if (Omega1) Omega1[j + k * p] *= c[j] * c[k];
            }
            sigma[k] /= c[k];
        }
    }
    if (mean_out) memcpy(mean_out, mean, sizeof(double) * (size_t)p);
    if (c_out) memcpy(c_out, c, sizeof(double) * (size_t)p);
    if (col_status) memcpy(col_status, cst, sizeof(int) * (size_t)p);
    int ret = ORC_OK;
    for (int64_t k = 0; k < p; ++k)
        if (cst[k] != ORC_OK) {
            ret = cst[k];
            break;
        }
    free(Xs); free(mean); free(c); free(cst);
    return ret;
}

/*
 * SPMESL on a subset of response columns: runs Algorithm 1 only for the
 * columns listed in cols[m] (the full-size parity checks sample columns this
 * way).  Outputs are on the standardised scale:
 *   Bcols [p*m] column i = beta_{-cols[i]}, sigma_cols [m].
 * mean and c (length p) receive the standardisation of all columns.
 */
int oracle_spmesl_columns(int64_t n, int64_t p, const double *X, double lambda0,
                          double tol, int max_outer, int max_sweeps, int64_t m,
                          const int64_t *cols, double *Bcols, double *sigma_cols,
                          double *mean_out, double *c_out, int *n_outer,
                          int *n_sweeps, int *col_status, int nthreads)
{
    if (n < 2 || p < 2 || !X || !cols || !Bcols || !sigma_cols || m < 0)
        return ORC_EINVAL;
    double *Xs = (double *)malloc(sizeof(double) * (size_t)(n * p));
    double *mean = (double *)malloc(sizeof(double) * (size_t)p);
    double *c = (double *)malloc(sizeof(double) * (size_t)p);
    int *cst = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    if (!Xs || !mean || !c || !cst) {
        free(Xs); free(mean); free(c); free(cst);
        return ORC_EINVAL;
    }
    int st = oracle_standardize(n, p, X, Xs, mean, c);
    if (st != ORC_OK) {
        free(Xs); free(mean); free(c); free(cst);
        return st;
    }
    for (int64_t i = 0; i < m; ++i)
        if (cols[i] < 0 || cols[i] >= p) {
            free(Xs); free(mean); free(c); free(cst);
            return ORC_EINVAL;
        }
    memset(Bcols, 0, sizeof(double) * (size_t)(p * m));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *e = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < m; ++i) {
            int64_t k = cols[i];
            double *bk = Bcols + i * p;
            double sg = 1.0;
            int no = 0, ns = 0;
            cst[i] = e ? oracle_scaled_lasso(n, p, Xs, Xs + k * n, k, lambda0, tol,
                                             max_outer, max_sweeps, bk, &sg, e,
                                             &no, &ns)
                       : ORC_EINVAL;
            bk[k] = 0.0;
            sigma_cols[i] = sg;
            if (n_outer) n_outer[i] = no;
            if (n_sweeps) n_sweeps[i] = ns;
        }
        free(e);
    }
    if (mean_out) memcpy(mean_out, mean, sizeof(double) * (size_t)p);
    if (c_out) memcpy(c_out, c, sizeof(double) * (size_t)p);
    if (col_status) memcpy(col_status, cst, sizeof(int) * (size_t)m);
    int ret = ORC_OK;
    for (int64_t i = 0; i < m; ++i)
        if (cst[i] != ORC_OK) {
            ret = cst[i];
            break;
        }
    free(Xs); free(mean); free(c); free(cst);
    return ret;
}

/*
 * Algorithm 2's estimate restricted to a set of response columns.  For
 * cols[m] (ascending, distinct) with their Algorithm 1 results Bcols [p*m]
 * (column i = beta_{-cols[i]}, standardised scale) and sigma_cols [m], writes
 * the m x m principal block of Omega (column-major, Om[a + b*m] = omega of
 * the pair (cols[a], cols[b])): the diagonal sigma^{-2} first (reading R3),
 * then omega_jk = -beta_jk sigma_k^{-2} (Eq. (eq:relation)), then the
 * min-magnitude symmetrisation of Eq. (eq:symm).  An entry of the symmetrised
 * estimate depends only on the two columns of its pair, so the block equals
 * that of the full estimate.  c (length p, or NULL) maps the block back to
 * the data's scale by Proposition 1 (omega^o_jk = c_j c_k omega_jk).
 */
void oracle_omega_subset(int64_t p, int64_t m, const int64_t *cols, const double *Bcols,
                         const double *sigma_cols, const double *c, double *Om)
{
    for (int64_t b = 0; b < m; ++b) {
        const double dk = 1.0 / (sigma_cols[b] * sigma_cols[b]);
        for (int64_t a = 0; a < m; ++a)
            Om[a + b * m] = (a == b) ? dk : -Bcols[cols[a] + b * p] * dk;
    }
    oracle_symmetrize(m, Om);
    if (c)
        for (int64_t b = 0; b < m; ++b)
            for (int64_t a = 0; a < m; ++a) Om[a + b * m] *= c[cols[a]] * c[cols[b]];
}

/* ---- penalty levels (Section 2.2) ------------------------------------- */

/* lambda_ub = sqrt(4 log p / n): the union bound over p scaled lassos. */
double oracle_lambda_ub(double n, double p) { return sqrt(4.0 * log(p) / n); }

/* lambda_univ = sqrt(2 log(p-1) / n): the universal level as the worked
 * example of Section 2.2 evaluates it (p-1 predictors per regression). */
double oracle_lambda_univ(double n, double p) { return sqrt(2.0 * log(p - 1.0) / n); }

/* Standard normal cdf from the complementary error function of libm. */
static double norm_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* Phi^{-1}(t) by bisection on norm_cdf (a deliberately plain method). */
static double norm_quantile(double t)
{
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (norm_cdf(mid) < t) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* L_n(t) = n^{-1/2} Phi^{-1}(1 - t). */
static double L_n(double n, double t) { return norm_quantile(1.0 - t) / sqrt(n); }

/*
 * lambda_pb = sqrt(2) L_n(k/p), with k the root in (0, p/2) of
 * k = L_1^4(k/p) + 2 L_1^2(k/p) (reading R7), found by bisection.
 * Writes k to *k_out when not NULL.  Returns lambda_pb.
 */
double oracle_lambda_pb(double n, double p, double *k_out)
{
    double lo = 1e-12 * p, hi = 0.5 * p;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        double L = L_n(1.0, mid / p);
        double f = mid - (L * L * L * L + 2.0 * L * L);
        if (f < 0.0) lo = mid;
        else hi = mid;
    }
    double k = 0.5 * (lo + hi);
    if (k_out) *k_out = k;
    return sqrt(2.0) * L_n(n, k / p);
}
