/*
 * oracle.c -- plain FP64 brute-force matrix profile.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path links, loads or calls
 * this file: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it. It shares no code, header or constant with the GPU
 * library.
 *
 * What it computes is the plain definition of the matrix profile, evaluated
 * pair by pair with the naive nested loop the paper mentions as the obvious
 * solution (Sec. 1): for every row window i and every admissible column
 * window j it sums the distance over the m samples directly, in natural order,
 * in double precision, and keeps the best and the runner-up. Nothing is
 * incremental, blocked or reordered.
 *
 *   windows       T_{i,m} = <t_i .. t_{i+m-1}>, 0 <= i < N = n-m+1 (Def. 2.2;
 *                 0-indexed here, the paper is 1-indexed)
 *   Euclidean     D_{i,j} = sqrt(sum_l (t_{i+l}-t_{j+l})^2)        (Def. 2.5, Eq. 1)
 *   p-norm        DP_{i,j} = (sum_l |t_{i+l}-t_{j+l}|^p)^(1/p)     (Def. 2.6, Eq. 2;
 *                 read with an absolute value, real p >= 1, as in Sec. 3.4)
 *   z-normalized  DZ_{i,j} = sqrt(sum_l ((t_{i+l}-mu_i)/s_i - (t_{j+l}-mu_j)/s_j)^2)
 *                 (Def. 2.7, Eq. 3), mu and s the window mean and population
 *                 standard deviation (App. A). A window whose samples are all
 *                 equal has s = 0; the paper states the z-normalized distance
 *                 is then infinite (Sec. 1), so such pairs never win.
 *   profile       p_i = min_j D_{i,j} (Def. 2.4) over admissible j, i.e.
 *                 |i - j| >= excl (excl >= 1 removes the self match; excl = 1
 *                 reproduces the paper's loops, which start at k = 1).
 *   index         I_i = the j attaining p_i; among exactly equal pre-root sums
 *                 the smallest j wins (strict '<' while j ascends).
 *   runner-up     Q_i = the best distance over admissible j != I_i.
 *
 * Rows with no finite candidate get P = +inf, I = -1, Q = +inf.
 *
 * Partial profiles (oracle_profile_diagonals): the same minimum taken only
 * over the pairs whose diagonal k = |i - j| is marked in a mask. Each outer
 * iteration k of the paper's algorithms (Sec. 3.2, Algs. 1-3) visits exactly
 * the pairs of diagonal k and nothing carries from one k to the next, which
 * is why the paper can call the algorithms anytime (Sec. 1, Sec. 7): stopping
 * after any set of iterations leaves the profile over those diagonals.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORACLE_EUCLID = 0, ORACLE_PNORM = 1, ORACLE_ZNORM = 2 };

/* |x|^p: integer p by repeated multiplication, otherwise pow(). */
static double abs_pow(double x, double p, int ip)
{
    double a = fabs(x);
    if (ip > 0) {
        double r = a;
        for (int q = 1; q < ip; ++q) r *= a;
        return r;
    }
    return pow(a, p);
}

static int integer_p(double p)
{
    if (p >= 1.0 && p <= 64.0 && p == floor(p)) return (int)p;
    return 0;
}

/* Window mean, population standard deviation (two passes, App. A) and the
 * exact all-samples-equal flag, for every window. The mean is evaluated as
 * t_i + (1/m) sum_l (t_{i+l} - t_i), the same quantity as (1/m) sum_l t_{i+l}
 * but with FP64 rounding at the scale of the window's deviations rather than
 * of the series' offset (which matters for near-constant windows far from
 * zero). */
int oracle_window_stats(const double *T, int64_t n, int32_t m,
                        double *mu, double *sigma, uint8_t *isconst)
{
    if (!T || n < 1 || m < 1 || m > n) return -1;
    int64_t N = n - m + 1;
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        int c = 1;
        for (int32_t l = 0; l < m; ++l) {
            s += T[i + l] - T[i];
            if (T[i + l] != T[i]) c = 0;
        }
        double mean = T[i] + s / (double)m;
        double v = 0.0;
        for (int32_t l = 0; l < m; ++l) {
            double d = T[i + l] - mean;
            v += d * d;
        }
        if (mu) mu[i] = mean;
        if (sigma) sigma[i] = sqrt(v / (double)m);
        if (isconst) isconst[i] = (uint8_t)c;
    }
    return 0;
}

/* The pre-root sum for one pair, straight from the definition. */
static double pair_sum(const double *T, int32_t m, int kind, double p, int ip,
                       int64_t i, int64_t j,
                       const double *mu, const double *sigma)
{
    double s = 0.0;
    if (kind == ORACLE_EUCLID) {
        for (int32_t l = 0; l < m; ++l) {
            double d = T[i + l] - T[j + l];
            s += d * d;
        }
    } else if (kind == ORACLE_PNORM) {
        for (int32_t l = 0; l < m; ++l)
            s += abs_pow(T[i + l] - T[j + l], p, ip);
    } else {
        for (int32_t l = 0; l < m; ++l) {
            double d = (T[i + l] - mu[i]) / sigma[i] - (T[j + l] - mu[j]) / sigma[j];
            s += d * d;
        }
    }
    return s;
}

static double root_of(double s, int kind, double p)
{
    if (isinf(s)) return s;
    if (kind == ORACLE_PNORM) {
        if (p == 1.0) return s;
        if (p == 2.0) return sqrt(s);
        return pow(s, 1.0 / p);
    }
    return sqrt(s);
}

/* Distance of one pair (after the root); +inf for a z-normalized pair that
 * involves a constant window. */
double oracle_distance(const double *T, int64_t n, int32_t m, int32_t kind,
                       double p, int64_t i, int64_t j)
{
    int64_t N = n - m + 1;
    if (!T || i < 0 || j < 0 || i >= N || j >= N) return NAN;
    int ip = integer_p(p);
    if (kind == ORACLE_ZNORM) {
        double mu2[2], sg2[2];
        uint8_t c2[2];
        oracle_window_stats(T + i, m, m, &mu2[0], &sg2[0], &c2[0]);
        oracle_window_stats(T + j, m, m, &mu2[1], &sg2[1], &c2[1]);
        if (c2[0] || c2[1]) return INFINITY;
        double s = 0.0;
        for (int32_t l = 0; l < m; ++l) {
            double d = (T[i + l] - mu2[0]) / sg2[0] - (T[j + l] - mu2[1]) / sg2[1];
            s += d * d;
        }
        return sqrt(s);
    }
    return root_of(pair_sum(T, m, kind, p, ip, i, j, NULL, NULL), kind, p);
}

/*
 * Matrix profile over the given rows (all rows when rows == NULL, then
 * nrows is ignored and outputs have N entries). Outputs are indexed by the
 * position in the row list. Q may be NULL. nthreads <= 0 uses the OpenMP
 * default. Returns 0, or -1 on invalid arguments.
 */
static int profile_impl(const double *T, int64_t n, int32_t m, int32_t kind,
                        double p, int32_t excl, const uint8_t *diag_ok,
                        const int64_t *rows, int64_t nrows,
                        double *P, int64_t *I, double *Q, int32_t nthreads);

int oracle_profile(const double *T, int64_t n, int32_t m, int32_t kind,
                   double p, int32_t excl, const int64_t *rows, int64_t nrows,
                   double *P, int64_t *I, double *Q, int32_t nthreads)
{
    return profile_impl(T, n, m, kind, p, excl, NULL, rows, nrows, P, I, Q, nthreads);
}

/* diag_ok: N entries; pair (i, j) is a candidate only if diag_ok[|i - j|] is
 * nonzero (and |i - j| >= excl as before). */
int oracle_profile_diagonals(const double *T, int64_t n, int32_t m, int32_t kind,
                             double p, int32_t excl, const uint8_t *diag_ok,
                             const int64_t *rows, int64_t nrows,
                             double *P, int64_t *I, double *Q, int32_t nthreads)
{
    if (!diag_ok) return -1;
    return profile_impl(T, n, m, kind, p, excl, diag_ok, rows, nrows, P, I, Q, nthreads);
}

static int profile_impl(const double *T, int64_t n, int32_t m, int32_t kind,
                        double p, int32_t excl, const uint8_t *diag_ok,
                        const int64_t *rows, int64_t nrows,
                        double *P, int64_t *I, double *Q, int32_t nthreads)
{
    if (!T || !P || !I || n < 1 || m < 1 || m > n || excl < 1) return -1;
    if (kind < ORACLE_EUCLID || kind > ORACLE_ZNORM) return -1;
    if (kind == ORACLE_PNORM && !(p >= 1.0 && isfinite(p))) return -1;
    int64_t N = n - m + 1;
    int64_t R = rows ? nrows : N;
    if (R < 0) return -1;
    for (int64_t r = 0; r < R; ++r)
        if (rows && (rows[r] < 0 || rows[r] >= N)) return -1;
    int ip = integer_p(p);

    double *mu = NULL, *sigma = NULL;
    uint8_t *isconst = NULL;
    if (kind == ORACLE_ZNORM) {
        mu = (double *)malloc(sizeof(double) * (size_t)N);
        sigma = (double *)malloc(sizeof(double) * (size_t)N);
        isconst = (uint8_t *)malloc((size_t)N);
        if (!mu || !sigma || !isconst) {
            free(mu); free(sigma); free(isconst);
            return -2;
        }
        oracle_window_stats(T, n, m, mu, sigma, isconst);
    }

#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
#endif
    for (int64_t r = 0; r < R; ++r) {
        int64_t i = rows ? rows[r] : r;
        double best = INFINITY, second = INFINITY;
        int64_t bi = -1;
        int row_ok = !(kind == ORACLE_ZNORM && isconst[i]);
        for (int64_t j = 0; row_ok && j < N; ++j) {
            int64_t gap = i > j ? i - j : j - i;
            if (gap < excl) continue;
            if (diag_ok && !diag_ok[gap]) continue;
            if (kind == ORACLE_ZNORM && isconst[j]) continue;
            double s = pair_sum(T, m, kind, p, ip, i, j, mu, sigma);
            if (s < best) {
                second = best;
                best = s;
                bi = j;
            } else if (s < second) {
                second = s;
            }
        }
        P[r] = root_of(best, kind, p);
        I[r] = bi;
        if (Q) Q[r] = root_of(second, kind, p);
    }
    free(mu);
    free(sigma);
    free(isconst);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
