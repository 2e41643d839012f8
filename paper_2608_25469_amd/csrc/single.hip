// Single-precision small solves (STRSM/CTRSM with m <= 64) and the inversion
// of diagonal chunks (<= 64 rows) for the FP32 blocked path.
//
// Paper Sec. 4.2.1 and Alg. 1: the lower triangle of L is staged once in
// shared memory (LDS here) and each thread owns one column of B, walking the
// forward-substitution chain
//     x_k <- x_k / l_kk,   x_i <- x_i - l_ik x_k  (i > k)
// in registers.  One wavefront serves a panel of 64 columns; every lane reads
// the same l_ik at once, which LDS serves as a broadcast.  Rows beyond m are
// zero in LDS and in registers, so the unrolled chain over MAXM (the next of
// 16, 32, 64 at or above m) needs no per-row guards.
//
// The chunk inversion is the same chain against identity right-hand sides
// (lane j solves for column j of the inverse), the paper's E_j tiles
// (Sec. 4.3.1), written into the blocked path's workspace W.

#include "internal.h"

namespace hsma {
namespace {

template <bool CX>
struct F32;
template <>
struct F32<false> {
    struct V {
        float r;
    };
    static __device__ __forceinline__ V zero() { return V{0.f}; }
    static __device__ __forceinline__ V one() { return V{1.f}; }
    static __device__ __forceinline__ V ld(const float *p, int64_t i) { return V{p[i]}; }
    static __device__ __forceinline__ void st(float *p, int64_t i, V v) { p[i] = v.r; }
    static __device__ __forceinline__ V mul(V a, V b) { return V{a.r * b.r}; }
    static __device__ __forceinline__ V fnms(V acc, V a, V b) { return V{acc.r - a.r * b.r}; }
    static __device__ __forceinline__ V div(V a, V d) { return V{a.r / d.r}; }
};
template <>
struct F32<true> {
    struct V {
        float r, i;
    };
    static __device__ __forceinline__ V zero() { return V{0.f, 0.f}; }
    static __device__ __forceinline__ V one() { return V{1.f, 0.f}; }
    static __device__ __forceinline__ V ld(const float *p, int64_t i) { return V{p[2 * i], p[2 * i + 1]}; }
    static __device__ __forceinline__ void st(float *p, int64_t i, V v) {
        p[2 * i] = v.r;
        p[2 * i + 1] = v.i;
    }
    static __device__ __forceinline__ V mul(V a, V b) {
        return V{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
    }
    static __device__ __forceinline__ V fnms(V acc, V a, V b) {
        return V{acc.r - (a.r * b.r - a.i * b.i), acc.i - (a.r * b.i + a.i * b.r)};
    }
    static __device__ __forceinline__ V div(V a, V d) {  // a conj(d) / |d|^2
        const float den = d.r * d.r + d.i * d.i;
        return V{(a.r * d.r + a.i * d.i) / den, (a.i * d.r - a.r * d.i) / den};
    }
};

// Stage the m x m lower triangle of A (lda) into Ls (MAXM x MAXM, column
// major); everything else 0, the diagonal 1 for a unit diagonal (not read).
template <bool CX, int MAXM, bool UNIT>
__device__ __forceinline__ void stage_lower(const float *__restrict__ A, int64_t lda, int m,
                                            typename F32<CX>::V *Ls) {
    typedef F32<CX> O;
    for (int e = threadIdx.x; e < MAXM * MAXM; e += 64) {
        const int i = e % MAXM, k = e / MAXM;
        typename O::V v = O::zero();
        if (i < m && k < m) {
            if (k < i) v = O::ld(A, i + (int64_t)k * lda);
            else if (k == i) v = UNIT ? O::one() : O::ld(A, i + (int64_t)k * lda);
        } else if (i == k) {
            v = O::one();
        }
        Ls[e] = v;
    }
    __syncthreads();
}

// x <- inv(L) x in registers (L in LDS, rows beyond m inert).
template <bool CX, int MAXM, bool UNIT>
__device__ __forceinline__ void substitute(const typename F32<CX>::V *Ls, int m,
                                           typename F32<CX>::V (&x)[MAXM]) {
    typedef F32<CX> O;
#pragma unroll
    for (int k = 0; k < MAXM; ++k) {
        if (k < m) {
            if (!UNIT) x[k] = O::div(x[k], Ls[k + k * MAXM]);
            const typename O::V xk = x[k];
#pragma unroll
            for (int i = k + 1; i < MAXM; ++i) x[i] = O::fnms(x[i], Ls[i + k * MAXM], xk);
        }
    }
}

template <bool CX, int MAXM, bool UNIT>
__global__ __launch_bounds__(64) void hsma_small32(const float *__restrict__ A, int64_t lda,
                                                   float *__restrict__ B, int64_t ldb, int m,
                                                   int64_t n, float ar, float ai) {
    typedef F32<CX> O;
    typedef typename O::V V;
    __shared__ V Ls[MAXM * MAXM];
    stage_lower<CX, MAXM, UNIT>(A, lda, m, Ls);
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= n) return;
    float *col = B + (CX ? 2 : 1) * c * ldb;
    V alpha;
    if constexpr (CX) alpha = V{ar, ai};
    else alpha = V{ar};
    V x[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) x[i] = i < m ? O::mul(alpha, O::ld(col, i)) : O::zero();
    substitute<CX, MAXM, UNIT>(Ls, m, x);
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
        if (i < m) O::st(col, i, x[i]);
}

// Chunk c: rows [c*base, c*base + sz) of L; lane j < sz solves for column j
// of the chunk's inverse, written to W (blocks of ib x ib, ld ib).
template <bool CX, int MAXM, bool UNIT>
__global__ __launch_bounds__(64) void hsma_inv32(const float *__restrict__ A, int64_t lda, int m,
                                                 int base, int ib, float *__restrict__ W) {
    typedef F32<CX> O;
    typedef typename O::V V;
    __shared__ V Ls[MAXM * MAXM];
    const int64_t o = (int64_t)blockIdx.x * base;
    const int sz = (int)((m - o) < base ? (m - o) : base);
    const float *Ac = A + (CX ? 2 : 1) * (o + o * lda);
    stage_lower<CX, MAXM, UNIT>(Ac, lda, sz, Ls);
    const int j = threadIdx.x;
    if (j >= sz) return;
    V x[MAXM];
#pragma unroll
    for (int i = 0; i < MAXM; ++i) x[i] = i == j ? O::one() : O::zero();
    substitute<CX, MAXM, UNIT>(Ls, sz, x);
    const int64_t blk = o / ib, oo = o % ib;
    float *Wc = W + (CX ? 2 : 1) * (blk * (int64_t)ib * ib + oo + (oo + j) * ib);
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
        if (i < sz) O::st(Wc, i, x[i]);
}

// B <- 0 on rows 0..rows-1 (floats) of each column.
__global__ __launch_bounds__(256) void hsma_zero_fill32(float *__restrict__ B, int64_t rows,
                                                        int64_t n, int64_t ld) {
    const int64_t total = rows * n;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        const int64_t j = t / rows, i = t - j * rows;
        B[i + j * ld] = 0.f;
    }
}

template <bool CX, bool UNIT>
hsma_status small32_t(int m, int64_t n, cplx alpha, const float *A, int64_t lda, float *B,
                      int64_t ldb, hipStream_t s) {
    const int64_t panels = (n + 63) / 64;
    if (panels > 0x7fffffff) return HSMA_INVALID_SIZE;
    const dim3 g((unsigned)panels), b(64);
    const float ar = (float)alpha.re, ai = (float)alpha.im;
    if (m <= 16) hipLaunchKernelGGL((hsma_small32<CX, 16, UNIT>), g, b, 0, s, A, lda, B, ldb, m, n, ar, ai);
    else if (m <= 32) hipLaunchKernelGGL((hsma_small32<CX, 32, UNIT>), g, b, 0, s, A, lda, B, ldb, m, n, ar, ai);
    else hipLaunchKernelGGL((hsma_small32<CX, 64, UNIT>), g, b, 0, s, A, lda, B, ldb, m, n, ar, ai);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

template <bool CX, bool UNIT>
hsma_status inv32_t(int m, int base, int ib, const float *A, int64_t lda, float *W, hipStream_t s) {
    const int chunks = (m + base - 1) / base;
    const dim3 g((unsigned)chunks), b(64);
    if (base <= 16) hipLaunchKernelGGL((hsma_inv32<CX, 16, UNIT>), g, b, 0, s, A, lda, m, base, ib, W);
    else if (base <= 32) hipLaunchKernelGGL((hsma_inv32<CX, 32, UNIT>), g, b, 0, s, A, lda, m, base, ib, W);
    else hipLaunchKernelGGL((hsma_inv32<CX, 64, UNIT>), g, b, 0, s, A, lda, m, base, ib, W);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

}  // namespace

hsma_status launch_zero32(int64_t m, int64_t n, int es, float *B, int64_t ldb, hipStream_t s) {
    const int64_t rows = m * es, ld = ldb * es;
    int64_t blocks = (rows * n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) return HSMA_SUCCESS;
    ProfScope prof(HSMA_PHASE_OTHER, 0.0, s);
    hipLaunchKernelGGL(hsma_zero_fill32, dim3((unsigned)blocks), dim3(256), 0, s, B, rows, n, ld);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

hsma_status launch_small_solve(bool cplx_, bool unit, int m, int64_t n, cplx alpha, const float *A,
                               int64_t lda, float *B, int64_t ldb, hipStream_t s) {
    if (m < 1 || m > 64) return HSMA_INVALID_SIZE;
    ProfScope prof(HSMA_PHASE_SMALL, (cplx_ ? 8.0 : 2.0) * 0.5 * m * (m + 1.0) * (double)n, s);
    if (cplx_) return unit ? small32_t<true, true>(m, n, alpha, A, lda, B, ldb, s)
                           : small32_t<true, false>(m, n, alpha, A, lda, B, ldb, s);
    return unit ? small32_t<false, true>(m, n, alpha, A, lda, B, ldb, s)
                : small32_t<false, false>(m, n, alpha, A, lda, B, ldb, s);
}

hsma_status launch_diag_inv_base(bool cplx_, bool unit, int m, int base, int ib, const float *A,
                                 int64_t lda, float *W, hipStream_t s) {
    if (base < 8 || base > 64 || (base & 7) || ib % base) return HSMA_INVALID_SIZE;
    const int nblk = (m + ib - 1) / ib;
    const int es = cplx_ ? 2 : 1;
    // zero every block (ib * ib * es floats = half as many doubles; ib is even)
    HSMA_TRY(launch_zero((int64_t)ib * ib * es / 2, nblk, 1, reinterpret_cast<double *>(W),
                         (int64_t)ib * ib * es / 2, s));
    ProfScope prof(HSMA_PHASE_DIAG_INV, 0.0, s);
    if (cplx_) return unit ? inv32_t<true, true>(m, base, ib, A, lda, W, s)
                           : inv32_t<true, false>(m, base, ib, A, lda, W, s);
    return unit ? inv32_t<false, true>(m, base, ib, A, lda, W, s)
                : inv32_t<false, false>(m, base, ib, A, lda, W, s);
}

}  // namespace hsma
