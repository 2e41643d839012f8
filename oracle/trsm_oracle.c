/*
 * Reference oracle for left-side, lower-triangular, no-transpose TRSM.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU statement of what the GPU library computes.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the library
 * never links, includes or calls it, and it shares no code with the library.
 *
 * The operation (paper, Sec. 2.1 and the forward-substitution equation of
 * Sec. 4.2.1): solve L X = alpha B for X, where L is the m x m lower triangle
 * of A, and overwrite B with X.  Row i of the solution is
 *     x_ij = ( alpha b_ij - sum_{k<i} l_ik x_kj ) / l_ii ,
 * with l_ii taken as 1 when the diagonal is declared unit.
 *
 * Conventions the paper leaves open, fixed here (BLAS TRSM semantics):
 *   - storage is column-major with leading dimensions lda, ldb;
 *   - only the strict lower triangle of A is read, plus the diagonal when it
 *     is non-unit; the upper triangle is never read;
 *   - alpha == 0 sets B to zero and reads neither A nor B;
 *   - alpha is applied once per element before the substitution;
 *   - complex numbers are interleaved (re, im) pairs of doubles; complex
 *     multiply is (ac - bd, ad + bc) and complex divide is the textbook
 *     x * conj(d) / |d|^2.
 *
 * Two loop orders are provided.  The column (axpy) form, used by every caller,
 * walks k = 0..m-1: divide y_k by l_kk, then subtract l_ik y_k from every later
 * row i.  The row (dot-product) form follows the equation above literally and
 * exists only so the tests can check that the two orders agree.
 *
 * Columns of B are independent (Sec. 4.2.1), so the column form is spread over
 * OpenMP threads by columns; no column's arithmetic depends on the thread
 * count.  Build with -ffp-contract=off so no multiply-add is fused.
 *
 * The checkers (backward error, normwise relative error) use compensated
 * dot products (Ogita, Rump and Oishi, "Accurate sum and dot product",
 * SIAM J. Sci. Comput. 2005, algorithm Dot2), so the checker's own rounding
 * stays far below the tolerances it is used to enforce.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Real double                                                         */
/* ------------------------------------------------------------------ */

static void d_solve_column(int unit, int64_t m, double alpha,
                           const double *A, int64_t lda, double *y)
{
    for (int64_t i = 0; i < m; ++i) y[i] = alpha * y[i];
    for (int64_t k = 0; k < m; ++k) {
        if (!unit) y[k] = y[k] / A[k + k * lda];
        const double xk = y[k];
        const double *colk = A + k * lda;
        for (int64_t i = k + 1; i < m; ++i) y[i] = y[i] - colk[i] * xk;
    }
}

void oracle_trsm_d(int unit, int64_t m, int64_t n, double alpha,
                   const double *A, int64_t lda, double *B, int64_t ldb)
{
    if (m <= 0 || n <= 0) return;
    if (alpha == 0.0) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) B[i + j * ldb] = 0.0;
        return;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j)
        d_solve_column(unit, m, alpha, A, lda, B + j * ldb);
}

/* Row form: x_i = (alpha b_i - sum_{k<i} l_ik x_k) / l_ii, k ascending. */
void oracle_trsm_d_rowform(int unit, int64_t m, int64_t n, double alpha,
                           const double *A, int64_t lda, double *B, int64_t ldb)
{
    if (m <= 0 || n <= 0) return;
    for (int64_t j = 0; j < n; ++j) {
        double *x = B + j * ldb;
        for (int64_t i = 0; i < m; ++i) {
            if (alpha == 0.0) { x[i] = 0.0; continue; }
            double s = alpha * x[i];
            for (int64_t k = 0; k < i; ++k) s = s - A[i + k * lda] * x[k];
            x[i] = unit ? s : s / A[i + i * lda];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Complex double, interleaved (re, im)                                */
/* ------------------------------------------------------------------ */

static inline void z_mul(double ar, double ai, double br, double bi,
                         double *cr, double *ci)
{
    *cr = ar * br - ai * bi;
    *ci = ar * bi + ai * br;
}

static inline void z_div(double xr, double xi, double dr, double di,
                         double *qr, double *qi)
{
    const double den = dr * dr + di * di;
    const double nr = xr * dr + xi * di;  /* x * conj(d), real part */
    const double ni = xi * dr - xr * di;  /* x * conj(d), imag part */
    *qr = nr / den;
    *qi = ni / den;
}

static void z_solve_column(int unit, int64_t m, const double *alpha,
                           const double *A, int64_t lda, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double r, s;
        z_mul(alpha[0], alpha[1], y[2 * i], y[2 * i + 1], &r, &s);
        y[2 * i] = r;
        y[2 * i + 1] = s;
    }
    for (int64_t k = 0; k < m; ++k) {
        if (!unit) {
            const double *d = A + 2 * (k + k * lda);
            double r, s;
            z_div(y[2 * k], y[2 * k + 1], d[0], d[1], &r, &s);
            y[2 * k] = r;
            y[2 * k + 1] = s;
        }
        const double xr = y[2 * k], xi = y[2 * k + 1];
        const double *colk = A + 2 * k * lda;
        for (int64_t i = k + 1; i < m; ++i) {
            double pr, pi;
            z_mul(colk[2 * i], colk[2 * i + 1], xr, xi, &pr, &pi);
            y[2 * i] = y[2 * i] - pr;
            y[2 * i + 1] = y[2 * i + 1] - pi;
        }
    }
}

void oracle_trsm_z(int unit, int64_t m, int64_t n, const double *alpha,
                   const double *A, int64_t lda, double *B, int64_t ldb)
{
    if (m <= 0 || n <= 0) return;
    if (alpha[0] == 0.0 && alpha[1] == 0.0) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < 2 * m; ++i) B[i + 2 * j * ldb] = 0.0;
        return;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j)
        z_solve_column(unit, m, alpha, A, lda, B + 2 * j * ldb);
}

void oracle_trsm_z_rowform(int unit, int64_t m, int64_t n, const double *alpha,
                           const double *A, int64_t lda, double *B, int64_t ldb)
{
    if (m <= 0 || n <= 0) return;
    const int azero = (alpha[0] == 0.0 && alpha[1] == 0.0);
    for (int64_t j = 0; j < n; ++j) {
        double *x = B + 2 * j * ldb;
        for (int64_t i = 0; i < m; ++i) {
            if (azero) { x[2 * i] = 0.0; x[2 * i + 1] = 0.0; continue; }
            double sr, si;
            z_mul(alpha[0], alpha[1], x[2 * i], x[2 * i + 1], &sr, &si);
            for (int64_t k = 0; k < i; ++k) {
                double pr, pi;
                const double *a = A + 2 * (i + k * lda);
                z_mul(a[0], a[1], x[2 * k], x[2 * k + 1], &pr, &pi);
                sr = sr - pr;
                si = si - pi;
            }
            if (unit) { x[2 * i] = sr; x[2 * i + 1] = si; }
            else {
                const double *d = A + 2 * (i + i * lda);
                z_div(sr, si, d[0], d[1], &x[2 * i], &x[2 * i + 1]);
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Checkers                                                            */
/* ------------------------------------------------------------------ */

/* Error-free transformations (Ogita, Rump and Oishi 2005). */
static inline void two_sum(double a, double b, double *s, double *e)
{
    const double x = a + b;
    const double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e)
{
    const double x = a * b;
    *e = fma(a, b, -x);  /* exact low part; fma() is exact by definition */
    *p = x;
}

/* Compensated accumulator: Dot2 state (s, c). */
typedef struct { double s, c; } dot2_t;

static inline void dot2_add_prod(dot2_t *d, double a, double b)
{
    double p, pe, s, se;
    two_prod(a, b, &p, &pe);
    two_sum(d->s, p, &s, &se);
    d->s = s;
    d->c = d->c + (pe + se);
}

static inline double dot2_value(const dot2_t *d) { return d->s + d->c; }

/*
 * Residual R = L X - alpha B0 for real data, written to R (ldr), computed with
 * Dot2 per element.  Returns nothing; norms are taken by the caller.
 */
static void d_residual(int unit, int64_t m, int64_t n, double alpha,
                       const double *A, int64_t lda, const double *X,
                       int64_t ldx, const double *B0, int64_t ldb,
                       double *R, int64_t ldr)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        const double *x = X + j * ldx;
        for (int64_t i = 0; i < m; ++i) {
            dot2_t acc = {0.0, 0.0};
            for (int64_t k = 0; k < i; ++k) dot2_add_prod(&acc, A[i + k * lda], x[k]);
            dot2_add_prod(&acc, unit ? 1.0 : A[i + i * lda], x[i]);
            dot2_add_prod(&acc, -alpha, B0[i + j * ldb]);
            R[i + j * ldr] = dot2_value(&acc);
        }
    }
}

static double d_norm_inf_general(int64_t m, int64_t n, const double *M, int64_t ld)
{
    double best = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += fabs(M[i + j * ld]);
        if (s > best || isnan(s)) best = s;
    }
    return best;
}

static double d_norm_inf_lower(int unit, int64_t m, const double *A, int64_t lda)
{
    double best = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double s = unit ? 1.0 : fabs(A[i + i * lda]);
        for (int64_t k = 0; k < i; ++k) s += fabs(A[i + k * lda]);
        if (s > best || isnan(s)) best = s;
    }
    return best;
}

/*
 * Normwise backward error
 *   eta = ||L X - alpha B0||_inf / (||L||_inf ||X||_inf + |alpha| ||B0||_inf),
 * where ||.||_inf is the maximum absolute row sum.  R is caller scratch of
 * m x n doubles (leading dimension m).
 */
double oracle_backward_error_d(int unit, int64_t m, int64_t n, double alpha,
                               const double *A, int64_t lda, const double *X,
                               int64_t ldx, const double *B0, int64_t ldb,
                               double *R)
{
    if (m <= 0 || n <= 0) return 0.0;
    d_residual(unit, m, n, alpha, A, lda, X, ldx, B0, ldb, R, m);
    const double rn = d_norm_inf_general(m, n, R, m);
    const double den = d_norm_inf_lower(unit, m, A, lda) * d_norm_inf_general(m, n, X, ldx)
                     + fabs(alpha) * d_norm_inf_general(m, n, B0, ldb);
    return den > 0.0 ? rn / den : rn;
}

static void z_residual(int unit, int64_t m, int64_t n, const double *alpha,
                       const double *A, int64_t lda, const double *X,
                       int64_t ldx, const double *B0, int64_t ldb,
                       double *R, int64_t ldr)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        const double *x = X + 2 * j * ldx;
        const double *b = B0 + 2 * j * ldb;
        for (int64_t i = 0; i < m; ++i) {
            dot2_t re = {0.0, 0.0}, im = {0.0, 0.0};
            for (int64_t k = 0; k <= i; ++k) {
                double ar, ai;
                if (k == i && unit) { ar = 1.0; ai = 0.0; }
                else { ar = A[2 * (i + k * lda)]; ai = A[2 * (i + k * lda) + 1]; }
                const double xr = x[2 * k], xi = x[2 * k + 1];
                dot2_add_prod(&re, ar, xr);
                dot2_add_prod(&re, -ai, xi);
                dot2_add_prod(&im, ar, xi);
                dot2_add_prod(&im, ai, xr);
            }
            const double br = b[2 * i], bi = b[2 * i + 1];
            dot2_add_prod(&re, -alpha[0], br);
            dot2_add_prod(&re, alpha[1], bi);
            dot2_add_prod(&im, -alpha[0], bi);
            dot2_add_prod(&im, -alpha[1], br);
            R[2 * (i + j * ldr)] = dot2_value(&re);
            R[2 * (i + j * ldr) + 1] = dot2_value(&im);
        }
    }
}

static double z_norm_inf_general(int64_t m, int64_t n, const double *M, int64_t ld)
{
    double best = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            s += hypot(M[2 * (i + j * ld)], M[2 * (i + j * ld) + 1]);
        if (s > best || isnan(s)) best = s;
    }
    return best;
}

static double z_norm_inf_lower(int unit, int64_t m, const double *A, int64_t lda)
{
    double best = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double s = unit ? 1.0 : hypot(A[2 * (i + i * lda)], A[2 * (i + i * lda) + 1]);
        for (int64_t k = 0; k < i; ++k)
            s += hypot(A[2 * (i + k * lda)], A[2 * (i + k * lda) + 1]);
        if (s > best || isnan(s)) best = s;
    }
    return best;
}

double oracle_backward_error_z(int unit, int64_t m, int64_t n, const double *alpha,
                               const double *A, int64_t lda, const double *X,
                               int64_t ldx, const double *B0, int64_t ldb,
                               double *R)
{
    if (m <= 0 || n <= 0) return 0.0;
    z_residual(unit, m, n, alpha, A, lda, X, ldx, B0, ldb, R, m);
    const double rn = z_norm_inf_general(m, n, R, m);
    const double den = z_norm_inf_lower(unit, m, A, lda) * z_norm_inf_general(m, n, X, ldx)
                     + hypot(alpha[0], alpha[1]) * z_norm_inf_general(m, n, B0, ldb);
    return den > 0.0 ? rn / den : rn;
}

/* Threads the OpenMP loops above will use. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
