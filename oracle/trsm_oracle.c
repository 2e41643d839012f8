/*
 * Reference oracle for left-side, lower-triangular, no-transpose TRSM, and for
 * the general BLAS TRSM (either side, either triangle, op(A) = A, A^T or A^H;
 * see the section "The general BLAS TRSM" below).
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

/* ------------------------------------------------------------------ */
/* The general BLAS TRSM: op(A) X = alpha B or X op(A) = alpha B        */
/* ------------------------------------------------------------------ */
/*
 * The paper poses the problem as op(A) X = alpha B with A triangular (Sec.
 * 2.1); its kernels treat the left-side, lower, no-transpose case.  These
 * functions state every case directly from that definition, by substitution
 * on op(A) itself, with nothing reduced to the lower-left case (the library
 * reduces them by transposition and index reversal; the oracle must not share
 * that reasoning):
 *
 *   side  0 = left  (op(A) X = alpha B, A is m x m),
 *         1 = right (X op(A) = alpha B, A is n x n);
 *   uplo  0 = A's lower triangle is stored, 1 = its upper triangle;
 *   trans 0 = op(A) = A, 1 = A^T, 2 = A^H (conjugate transpose; for real
 *         data the same as 1);
 *   unit  1 = the diagonal of A is taken as 1 and never read.
 *
 * Only the stored triangle of A is read.  op(A) is upper triangular when the
 * upper triangle is stored and not transposed, or the lower one is stored and
 * transposed.  Left side, column j of X: op(A) x = alpha b, solved by the dot
 * form of substitution, top to bottom when op(A) is lower and bottom to top
 * when it is upper:
 *     x_i = (alpha b_i - sum_k op(A)_ik x_k) / op(A)_ii,
 * k over the already solved rows.  Right side, row i of X: sum_k x_ik
 * op(A)_kj = alpha b_ij for every j, solved left to right when op(A) is upper
 * (x_ij needs x_ik, k < j) and right to left when it is lower.
 */

/* op(A)_rc for real data: A_rc, or A_cr when transposed. */
static inline double d_op(int trans, const double *A, int64_t lda, int64_t r, int64_t c)
{
    return trans ? A[c + r * lda] : A[r + c * lda];
}

/* op(A)_rc for complex data, conjugated for trans == 2. */
static inline void z_op(int trans, const double *A, int64_t lda, int64_t r, int64_t c,
                        double *re, double *im)
{
    const double *a = trans ? A + 2 * (c + r * lda) : A + 2 * (r + c * lda);
    *re = a[0];
    *im = trans == 2 ? -a[1] : a[1];
}

static inline int op_is_upper(int uplo, int trans)
{
    return (uplo == 1) == (trans == 0);
}

void oracle_trsm_general_d(int side, int uplo, int trans, int unit, int64_t m, int64_t n,
                           double alpha, const double *A, int64_t lda, double *B, int64_t ldb)
{
    if (m <= 0 || n <= 0) return;
    if (alpha == 0.0) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) B[i + j * ldb] = 0.0;
        return;
    }
    const int upper = op_is_upper(uplo, trans);
    if (side == 0) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t j = 0; j < n; ++j) {
            double *x = B + j * ldb;
            for (int64_t t = 0; t < m; ++t) {
                const int64_t i = upper ? m - 1 - t : t;
                double s = alpha * x[i];
                if (upper)
                    for (int64_t k = i + 1; k < m; ++k) s = s - d_op(trans, A, lda, i, k) * x[k];
                else
                    for (int64_t k = 0; k < i; ++k) s = s - d_op(trans, A, lda, i, k) * x[k];
                x[i] = unit ? s : s / d_op(trans, A, lda, i, i);
            }
        }
    } else {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t t = 0; t < n; ++t) {
                const int64_t j = upper ? t : n - 1 - t;
                double s = alpha * B[i + j * ldb];
                if (upper)
                    for (int64_t k = 0; k < j; ++k) s = s - B[i + k * ldb] * d_op(trans, A, lda, k, j);
                else
                    for (int64_t k = j + 1; k < n; ++k) s = s - B[i + k * ldb] * d_op(trans, A, lda, k, j);
                B[i + j * ldb] = unit ? s : s / d_op(trans, A, lda, j, j);
            }
        }
    }
}

void oracle_trsm_general_z(int side, int uplo, int trans, int unit, int64_t m, int64_t n,
                           const double *alpha, const double *A, int64_t lda, double *B,
                           int64_t ldb)
{
    if (m <= 0 || n <= 0) return;
    if (alpha[0] == 0.0 && alpha[1] == 0.0) {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < 2 * m; ++i) B[i + 2 * j * ldb] = 0.0;
        return;
    }
    const int upper = op_is_upper(uplo, trans);
    if (side == 0) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t j = 0; j < n; ++j) {
            double *x = B + 2 * j * ldb;
            for (int64_t t = 0; t < m; ++t) {
                const int64_t i = upper ? m - 1 - t : t;
                double sr, si, ar, ai, pr, pi;
                z_mul(alpha[0], alpha[1], x[2 * i], x[2 * i + 1], &sr, &si);
                const int64_t k0 = upper ? i + 1 : 0, k1 = upper ? m : i;
                for (int64_t k = k0; k < k1; ++k) {
                    z_op(trans, A, lda, i, k, &ar, &ai);
                    z_mul(ar, ai, x[2 * k], x[2 * k + 1], &pr, &pi);
                    sr = sr - pr;
                    si = si - pi;
                }
                if (unit) {
                    x[2 * i] = sr;
                    x[2 * i + 1] = si;
                } else {
                    z_op(trans, A, lda, i, i, &ar, &ai);
                    z_div(sr, si, ar, ai, &x[2 * i], &x[2 * i + 1]);
                }
            }
        }
    } else {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t t = 0; t < n; ++t) {
                const int64_t j = upper ? t : n - 1 - t;
                double sr, si, ar, ai, pr, pi;
                double *b = B + 2 * (i + j * ldb);
                z_mul(alpha[0], alpha[1], b[0], b[1], &sr, &si);
                const int64_t k0 = upper ? 0 : j + 1, k1 = upper ? j : n;
                for (int64_t k = k0; k < k1; ++k) {
                    z_op(trans, A, lda, k, j, &ar, &ai);
                    const double *xk = B + 2 * (i + k * ldb);
                    z_mul(xk[0], xk[1], ar, ai, &pr, &pi);
                    sr = sr - pr;
                    si = si - pi;
                }
                if (unit) {
                    b[0] = sr;
                    b[1] = si;
                } else {
                    z_op(trans, A, lda, j, j, &ar, &ai);
                    z_div(sr, si, ar, ai, &b[0], &b[1]);
                }
            }
        }
    }
}

/*
 * Normwise backward error of the general problem,
 *   eta = ||R||_inf / (||op(A)||_inf ||X||_inf + |alpha| ||B0||_inf),
 *   R = op(A) X - alpha B0 (left) or X op(A) - alpha B0 (right),
 * with every element of R formed by Dot2 over the triangle of op(A) (the
 * diagonal taken as 1 when unit) and ||op(A)||_inf the largest row sum of
 * |op(A)|.  cx selects interleaved complex data (alpha then points to
 * {re, im}); R is caller scratch of m x n elements.
 */
double oracle_backward_error_general(int cx, int side, int uplo, int trans, int unit,
                                     int64_t m, int64_t n, const double *alpha,
                                     const double *A, int64_t lda, const double *X,
                                     int64_t ldx, const double *B0, int64_t ldb, double *R)
{
    if (m <= 0 || n <= 0) return 0.0;
    const int upper = op_is_upper(uplo, trans);
    const int64_t ka = side == 0 ? m : n;
    const int es = cx ? 2 : 1;
    /* op(A)_rc as (re, im); zero outside the triangle, 1 on a unit diagonal */
#define OPEL(r, c, re, im)                                                         \
    do {                                                                           \
        const int64_t r_ = (r), c_ = (c);                                          \
        if (upper ? (r_ > c_) : (r_ < c_)) { re = 0.0; im = 0.0; }                 \
        else if (r_ == c_ && unit) { re = 1.0; im = 0.0; }                         \
        else if (cx) z_op(trans, A, lda, r_, c_, &re, &im);                        \
        else { re = d_op(trans, A, lda, r_, c_); im = 0.0; }                       \
    } while (0)
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            dot2_t re = {0.0, 0.0}, im = {0.0, 0.0};
            for (int64_t k = 0; k < ka; ++k) {
                double ar, ai, xr, xi;
                if (side == 0) {
                    OPEL(i, k, ar, ai);
                    xr = X[es * (k + j * ldx)];
                    xi = cx ? X[es * (k + j * ldx) + 1] : 0.0;
                } else {
                    OPEL(k, j, ar, ai);
                    xr = X[es * (i + k * ldx)];
                    xi = cx ? X[es * (i + k * ldx) + 1] : 0.0;
                }
                if (ar == 0.0 && ai == 0.0) continue;
                dot2_add_prod(&re, ar, xr);
                if (cx) {
                    dot2_add_prod(&re, -ai, xi);
                    dot2_add_prod(&im, ar, xi);
                    dot2_add_prod(&im, ai, xr);
                }
            }
            const double br = B0[es * (i + j * ldb)], bi = cx ? B0[es * (i + j * ldb) + 1] : 0.0;
            dot2_add_prod(&re, -alpha[0], br);
            if (cx) {
                dot2_add_prod(&re, alpha[1], bi);
                dot2_add_prod(&im, -alpha[0], bi);
                dot2_add_prod(&im, -alpha[1], br);
            }
            R[es * (i + j * m)] = dot2_value(&re);
            if (cx) R[es * (i + j * m) + 1] = dot2_value(&im);
        }
    }
    double rn = 0.0, xn = 0.0, bn = 0.0, an = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double sr = 0.0, sx = 0.0, sb = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            sr += cx ? hypot(R[2 * (i + j * m)], R[2 * (i + j * m) + 1]) : fabs(R[i + j * m]);
            sx += cx ? hypot(X[2 * (i + j * ldx)], X[2 * (i + j * ldx) + 1]) : fabs(X[i + j * ldx]);
            sb += cx ? hypot(B0[2 * (i + j * ldb)], B0[2 * (i + j * ldb) + 1]) : fabs(B0[i + j * ldb]);
        }
        if (sr > rn || isnan(sr)) rn = sr;
        if (sx > xn || isnan(sx)) xn = sx;
        if (sb > bn || isnan(sb)) bn = sb;
    }
    for (int64_t r = 0; r < ka; ++r) {
        double s = 0.0;
        for (int64_t c = 0; c < ka; ++c) {
            double ar, ai;
            OPEL(r, c, ar, ai);
            s += cx ? hypot(ar, ai) : fabs(ar);
        }
        if (s > an || isnan(s)) an = s;
    }
#undef OPEL
    const double den = an * xn + (cx ? hypot(alpha[0], alpha[1]) : fabs(alpha[0])) * bn;
    return den > 0.0 ? rn / den : rn;
}

/* ------------------------------------------------------------------ */
/* Cholesky factorization, the TRSM's first consumer (Sec. 1)           */
/* ------------------------------------------------------------------ */
/*
 * A = L L^H for a real symmetric or complex Hermitian positive definite A
 * (n x n, lda): L overwrites the lower triangle; the strict upper triangle is
 * neither read nor written.  Column by column (left-looking):
 *     l_jj = sqrt(a_jj - sum_{k<j} |l_jk|^2),
 *     l_ij = (a_ij - sum_{k<j} l_ik conj(l_jk)) / l_jj   (i > j).
 * Only the real part of a complex diagonal is used (a Hermitian matrix has a
 * real diagonal).  Returns 0, or j + 1 when the pivot of column j is not
 * positive (the factorization stops there, as LAPACK's potrf does).
 */
int oracle_potrf_d(int64_t n, double *A, int64_t lda)
{
    for (int64_t j = 0; j < n; ++j) {
        double s = A[j + j * lda];
        for (int64_t k = 0; k < j; ++k) s = s - A[j + k * lda] * A[j + k * lda];
        if (!(s > 0.0)) return (int)(j + 1);
        const double d = sqrt(s);
        A[j + j * lda] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double t = A[i + j * lda];
            for (int64_t k = 0; k < j; ++k) t = t - A[i + k * lda] * A[j + k * lda];
            A[i + j * lda] = t / d;
        }
    }
    return 0;
}

int oracle_potrf_z(int64_t n, double *A, int64_t lda)
{
    for (int64_t j = 0; j < n; ++j) {
        double s = A[2 * (j + j * lda)];
        for (int64_t k = 0; k < j; ++k) {
            const double *l = A + 2 * (j + k * lda);
            s = s - (l[0] * l[0] + l[1] * l[1]);
        }
        if (!(s > 0.0)) return (int)(j + 1);
        const double d = sqrt(s);
        A[2 * (j + j * lda)] = d;
        A[2 * (j + j * lda) + 1] = 0.0;
        for (int64_t i = j + 1; i < n; ++i) {
            double tr = A[2 * (i + j * lda)], ti = A[2 * (i + j * lda) + 1];
            for (int64_t k = 0; k < j; ++k) {
                const double *a = A + 2 * (i + k * lda);   /* l_ik */
                const double *b = A + 2 * (j + k * lda);   /* l_jk, conjugated */
                double pr, pi;
                z_mul(a[0], a[1], b[0], -b[1], &pr, &pi);
                tr = tr - pr;
                ti = ti - pi;
            }
            A[2 * (i + j * lda)] = tr / d;
            A[2 * (i + j * lda) + 1] = ti / d;
        }
    }
    return 0;
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
