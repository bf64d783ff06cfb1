/*
 * dpt_oracle.c -- FP64 CPU oracle for dynamical perturbation theory (D-PT).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is loaded by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark, nothing else.  It
 * shares no code, header, table or helper with the HIP library and must never
 * be called from the product path.
 *
 * What it computes (Kenmoe, Smerlak, Zadorin, "Dynamical perturbation theory
 * for eigenvalue problems", arXiv:2002.12872):
 *
 *   M = D + lambda*Delta, D = diag(theta) with simple theta (Sec. II.B).
 *   For each requested eigenvector index n the candidate z_n (chart z_n[n] = 1)
 *   is iterated with the single-line map of eq. (single_line_dyn):
 *
 *     F_n(z)[m] = delta_nm + lambda * ((Delta z)[m] - (Delta z)[n] * z[m]) / (theta_n - theta_m),
 *
 *   with the gap factor taken as zero on the diagonal, starting from z = e_n,
 *   i.e. A^(0) = I (Sec. II.B, the iteration F^k(I) of eq. (dyn), whose n-th row
 *   evolves under F_n alone).  The eigenvalue attached to an iterate is
 *   E_n = theta_n + lambda * (Delta z_n)[n]  (Sec. II.B readout; the factor
 *   lambda is the one the main text omits and Supplement B makes explicit:
 *   the order-l eigenvalue coefficient is (a^(l-1) Delta')_nn).
 *
 * Stopping rule (the paper states none; reading recorded in the design notes):
 *   delta_k = max over requested rows and all m of |z^(k)[m] - z^(k-1)[m]|;
 *   stop with OK as soon as delta_k < tol; DIVERGED when an iterate is
 *   non-finite or max |z - e_n| exceeds `blowup`; NOT_CONVERGED at the cap.
 *   In fixed-step mode exactly max_iter applications are made (no tol stop).
 *   The returned iterate is the last one computed and E is read from it.
 *
 * Arithmetic: plain loops, FP64, products (Delta z)[m] summed over l in
 * ascending column order (dense) or in stored order (CSR), the gap applied by
 * division.  No blocking, no fusion, no reordering.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_DIVERGED 3
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

/* Problem description.  Exactly one of `dense` or (`indptr`,`indices`,`values`)
 * is set.  dense: n*n row-major, dense[m*n + l] = Delta[m][l].
 * CSR: row m holds entries indices[indptr[m] .. indptr[m+1]) with values. */
typedef struct {
    int64_t n;
    const double *theta;
    const double *dense;
    const int64_t *indptr;
    const int32_t *indices;
    const double *values;
    double lambda;
} or_problem;

/* (Delta z)[m] for one m. */
static double delta_row_dot(const or_problem *p, int64_t m, const double *z)
{
    double s = 0.0;
    if (p->dense) {
        const double *row = p->dense + m * p->n;
        for (int64_t l = 0; l < p->n; ++l) s += row[l] * z[l];
    } else {
        for (int64_t e = p->indptr[m]; e < p->indptr[m + 1]; ++e)
            s += p->values[e] * z[p->indices[e]];
    }
    return s;
}

/* One application of F_n (eq. single_line_dyn) with coupling lam to z, result
 * in znew.  c is scratch of length n holding Delta z. */
static void apply_single_line_map(const or_problem *p, int64_t nidx, double lam, const double *z,
                                  double *znew, double *c)
{
    const int64_t n = p->n;
    for (int64_t m = 0; m < n; ++m) c[m] = delta_row_dot(p, m, z);
    const double cn = c[nidx];
    for (int64_t m = 0; m < n; ++m) {
        if (m == nidx) {
            znew[m] = 1.0;
        } else {
            znew[m] = lam * (c[m] - cn * z[m]) / (p->theta[nidx] - p->theta[m]);
        }
    }
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Number of entries equal to x in the ascending array a[0..n). */
static int64_t count_equal(const double *a, int64_t n, double x)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) { /* first index with a[i] >= x */
        const int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    int64_t c = 0;
    while (lo + c < n && a[lo + c] == x) ++c;
    return c;
}

static int validate(const or_problem *p, int64_t nrows, const int64_t *rows)
{
    if (!p || p->n < 1 || !p->theta) return OR_EINVAL;
    if (!p->dense && !(p->indptr && p->indices && p->values)) return OR_EINVAL;
    if (!isfinite(p->lambda)) return OR_EINVAL;
    /* Each requested row n is iterated with its own single-line map, which
     * divides by theta_n - theta_m for every m != n (Sec. II.B, Sec. II.H):
     * theta_n must be simple.  Values of rows not requested may coincide.
     * Sort a copy and count the occurrences of each requested theta_n. */
    double *sorted = (double *)malloc(sizeof(double) * (size_t)p->n);
    if (!sorted) return OR_ENOMEM;
    for (int64_t i = 0; i < p->n; ++i) {
        if (!isfinite(p->theta[i])) {
            free(sorted);
            return OR_EINVAL;
        }
        sorted[i] = p->theta[i];
    }
    qsort(sorted, (size_t)p->n, sizeof(double), cmp_double);
    for (int64_t r = 0; r < nrows; ++r) {
        if (rows[r] < 0 || rows[r] >= p->n || count_equal(sorted, p->n, p->theta[rows[r]]) != 1) {
            free(sorted);
            return OR_EINVAL;
        }
    }
    free(sorted);
    if (!p->dense) {
        if (p->indptr[0] != 0) return OR_EINVAL;
        for (int64_t m = 0; m < p->n; ++m) {
            if (p->indptr[m + 1] < p->indptr[m]) return OR_EINVAL;
            for (int64_t e = p->indptr[m]; e < p->indptr[m + 1]; ++e)
                if (p->indices[e] < 0 || p->indices[e] >= p->n) return OR_EINVAL;
        }
    }
    return OR_OK;
}

/*
 * Iterate the rows `rows[0..nrows)` of A^(k) = F^k(A^(0)).
 *   z0        : nrows*n initial rows (row r is the start of eigenvector rows[r]),
 *               or NULL for e_n (A^(0) = I).  Entry rows[r] of each start row is
 *               forced to 1 (the chart z^n = 1).
 *   max_iter  : iteration cap (>= 0); in fixed mode the exact number of steps.
 *   tol       : stop when delta_k < tol (ignored in fixed mode).
 *   blowup    : DIVERGED threshold on max |z - e_n|.
 *   nthreads  : OpenMP threads (<= 0: library default).
 *   ramp_alpha: 0 for the autonomous map; in (0, 1) the non-autonomous scheme
 *               of Supplement E: the k-th application (k = 1, 2, ...) uses
 *               lambda_k = lambda (1 - a_k) with a_k = ramp_alpha^k formed by
 *               repeated multiplication, as long as a_k >= 2^-53, and lambda
 *               itself afterwards; the tol test is skipped while the ramp runs
 *               (the eigenvalue readout always uses lambda).
 *   per_row   : 0: the rows stop together (delta_k over all rows < tol).
 *               1: each row stops on its own (Sec. II.B: row n evolves under F_n
 *               alone): row r is frozen after the first step whose
 *               delta_k(r) = max_m |z^(k)[m] - z^(k-1)[m]| is below tol; the
 *               iteration ends when every row is frozen (OK) or at the cap.
 *               delta_hist records the maximum over the rows still running.
 *   row_iters : nrows entries (may be NULL): the step on which each row was
 *               frozen (per_row), 0 for a row still running at the end.
 * Outputs (all caller-owned):
 *   z         : nrows*n, final iterate rows
 *   e         : nrows, E_n = theta_n + lambda (Delta z_n)[n] of the final iterate
 *   delta_hist: max_iter entries (may be NULL); entries past *iters untouched
 *   iters     : number of applications of F made
 * Returns OR_OK / OR_NOT_CONVERGED / OR_DIVERGED, or OR_EINVAL / OR_ENOMEM.
 */
int or_iterate(const or_problem *p, int64_t nrows, const int64_t *rows, const double *z0,
               int max_iter, double tol, int fixed_steps, double blowup, int nthreads,
               double ramp_alpha, int per_row, double *z, double *e, double *delta_hist, int *iters,
               int *row_iters)
{
    if (nrows < 1 || !rows || !z || !e || !iters || max_iter < 0) return OR_EINVAL;
    if (per_row && fixed_steps) return OR_EINVAL;
    if (!(ramp_alpha >= 0.0 && ramp_alpha < 1.0)) return OR_EINVAL;
    int rc = validate(p, nrows, rows);
    if (rc != OR_OK) return rc;
    if (!fixed_steps && !(tol > 0.0)) return OR_EINVAL;
    const int64_t n = p->n;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= n) return OR_EINVAL;

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *znew = (double *)malloc(sizeof(double) * (size_t)(nrows * n));
    double *scratch = (double *)malloc(sizeof(double) * (size_t)n * (size_t)nth);
    int *frozen_at = (int *)calloc((size_t)nrows, sizeof(int)); /* 0: running */
    if (!znew || !scratch || !frozen_at) {
        free(znew);
        free(scratch);
        free(frozen_at);
        return OR_ENOMEM;
    }

    for (int64_t r = 0; r < nrows; ++r) {
        double *zr = z + r * n;
        if (z0) {
            memcpy(zr, z0 + r * n, sizeof(double) * (size_t)n);
        } else {
            for (int64_t m = 0; m < n; ++m) zr[m] = 0.0;
        }
        zr[rows[r]] = 1.0;
    }

    int status = fixed_steps ? OR_OK : OR_NOT_CONVERGED;
    int k = 0;
    double ak = 1.0; /* ramp_alpha^k */
    while (k < max_iter) {
        double lam = p->lambda;
        int ramping = 0;
        if (ramp_alpha > 0.0) {
            ak *= ramp_alpha;
            if (ak >= 0x1p-53) {
                lam = p->lambda * (1.0 - ak);
                ramping = 1;
            }
        }
        double dk = 0.0, wmax = 0.0;
        int nonfinite = 0, running = 0;
#pragma omp parallel for schedule(static) num_threads(nth) reduction(max : dk, wmax) reduction(| : nonfinite) \
    reduction(+ : running)
        for (int64_t r = 0; r < nrows; ++r) {
            if (frozen_at[r]) continue;
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            double *c = scratch + (size_t)t * (size_t)n;
            double *zr = z + r * n;
            double *zn = znew + r * n;
            apply_single_line_map(p, rows[r], lam, zr, zn, c);
            double dr = 0.0;
            for (int64_t m = 0; m < n; ++m) {
                if (!isfinite(zn[m])) nonfinite = 1;
                double ch = fabs(zn[m] - zr[m]);
                if (ch > dr) dr = ch;
                double off = fabs(zn[m] - (m == rows[r] ? 1.0 : 0.0));
                if (off > wmax) wmax = off;
            }
            if (dr > dk) dk = dr;
            memcpy(zr, zn, sizeof(double) * (size_t)n);
            if (per_row && !ramping && dr < tol) {
                frozen_at[r] = k + 1;
            } else {
                running += 1;
            }
        }
        if (delta_hist) delta_hist[k] = nonfinite ? NAN : dk;
        ++k;
        if (nonfinite || !(wmax <= blowup)) {
            status = OR_DIVERGED;
            break;
        }
        if (!fixed_steps && !ramping && (per_row ? running == 0 : dk < tol)) {
            status = OR_OK;
            break;
        }
    }
    if (row_iters)
        for (int64_t r = 0; r < nrows; ++r) row_iters[r] = frozen_at[r];
    free(frozen_at);
    free(scratch);
    free(znew);
    *iters = k;

    for (int64_t r = 0; r < nrows; ++r)
        e[r] = p->theta[rows[r]] + p->lambda * delta_row_dot(p, rows[r], z + r * n);
    return status;
}

/* Threads the OpenMP runtime would use (reported as the CPU-baseline core count). */
int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
