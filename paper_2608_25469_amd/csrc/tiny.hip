// Fused solves of very small problems (m, n <= 16): four problems per
// wavefront.  The paper names kernel fusion for very small scales as future
// work (Sec. 6).
//
// The small-solve kernel gives each problem a whole 64-lane wavefront (lane =
// column) and stages L in 16-row blocks; a problem with n <= 16 then leaves
// at least 48 lanes idle and m <= 16 uses a single, mostly empty block.  Here
// each 16-lane quarter of the wavefront is one problem: its lower triangle
// (<= 16 x 16) sits in the quarter's own LDS region, lane j of the quarter
// holds column j in 16 registers, and the substitution chain
//     x_k <- x_k / l_kk,   x_i <- x_i - l_ik x_k  (i > k)
// runs over the problem's own m.  The lanes of a quarter read the same l_ik
// (an LDS broadcast); the four quarters' regions are offset so that their
// four addresses fall in different banks.  Rows beyond m are zero in LDS and
// in registers.  The per-problem arithmetic does not depend on which quarter
// or launch a problem lands in, so a problem gives the same bits alone and
// in a batch.

#include "small_kernels.h"

namespace hsma {
namespace {

// Same layout as the batched item of the small-solve kernel.
struct TinyItem {
    const double *A;
    double *B;
    int64_t lda, ldb;
    int32_t m, ncols;
    double ar, ai;
};

constexpr int kMax = 16;
// Quarter stride in elements: 16 x 17 plus padding that puts the four
// quarters' copies of one element in different LDS banks.
template <bool CX>
constexpr int quarter_stride() { return CX ? 276 : 280; }

// Element operations.  Every rounding is spelled out and in the same order
// as in the strip kernel's walk (strip.hip, dpp_fma.h): the update of a
// complex row is yr -= lr xr, yi -= lr xi, yr += li xi, yi -= li xr, each a
// fused multiply-add; the diagonal is applied as a product with its
// reciprocal; alpha scales only when it is not 1.  So a problem gives the
// same bits here as there.
template <bool CX>
struct D;
template <>
struct D<false> {
    typedef double V;
    static __device__ __forceinline__ V ld(const HSMA_GLOBAL double *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ void st(HSMA_GLOBAL double *p, int64_t i, V v) { p[i] = v; }
    static __device__ __forceinline__ V zero() { return 0.0; }
    static __device__ __forceinline__ V one() { return 1.0; }
    static __device__ __forceinline__ void fnms(V &acc, V l, V x) { acc = __fma_rn(-l, x, acc); }
    static __device__ __forceinline__ V scale(V x, V r) { return __dmul_rn(x, r); }
    static __device__ __forceinline__ V alpha(V x, double ar, double) { return __dmul_rn(x, ar); }
    static __device__ __forceinline__ V recip(V d) {
        double r, i;
        smallk::recip_rn(false, d, 0.0, r, i);
        return r;
    }
};
template <>
struct D<true> {
    typedef dbl2u V;
    static __device__ __forceinline__ V ld(const HSMA_GLOBAL double *p, int64_t i) {
        return *reinterpret_cast<const HSMA_GLOBAL dbl2u *>(p + 2 * i);
    }
    static __device__ __forceinline__ void st(HSMA_GLOBAL double *p, int64_t i, V v) {
        *reinterpret_cast<HSMA_GLOBAL dbl2u *>(p + 2 * i) = v;
    }
    static __device__ __forceinline__ V zero() { return V{0.0, 0.0}; }
    static __device__ __forceinline__ V one() { return V{1.0, 0.0}; }
    static __device__ __forceinline__ void fnms(V &acc, V l, V x) {
        double yr = acc.x, yi = acc.y;
        yr = __fma_rn(-l.x, x.x, yr);
        yi = __fma_rn(-l.x, x.y, yi);
        yr = __fma_rn(l.y, x.y, yr);
        yi = __fma_rn(-l.y, x.x, yi);
        acc = V{yr, yi};
    }
    static __device__ __forceinline__ V scale(V x, V r) {
        double a, b;
        smallk::cmul_rn(x.x, x.y, r.x, r.y, a, b);
        return V{a, b};
    }
    static __device__ __forceinline__ V alpha(V x, double ar, double ai) {
        double a, b;
        smallk::cmul_rn(ar, ai, x.x, x.y, a, b);
        return V{a, b};
    }
    static __device__ __forceinline__ V recip(V d) {
        double r, i;
        smallk::recip_rn(true, d.x, d.y, r, i);
        return V{r, i};
    }
};

// Workgroup b solves items 4b .. 4b + 3 (those below count); with items ==
// nullptr it solves `one` alone (a single call, no descriptor upload).
template <bool CX, bool UNIT>
__global__ __launch_bounds__(64) void hsma_tiny(TinyItem one, const TinyItem *__restrict__ items,
                                                int count) {
    typedef D<CX> O;
    typedef typename O::V V;
    constexpr int QS = quarter_stride<CX>();
    __shared__ V Ls[4 * QS];
    const int q = threadIdx.x >> 4, lane = threadIdx.x & 15;
    const int idx = blockIdx.x * 4 + q;
    const bool active = items ? idx < count : q == 0;
    TinyItem it = one;
    if (items && active) it = items[idx];
    V *L = Ls + q * QS;
    __shared__ V Rs[4 * kMax];  // reciprocals of each quarter's diagonal
    V *Rq = Rs + q * kMax;
    // alpha == 0: B <- 0, and neither A nor B is read (A may be null).
    const bool azero = it.ar == 0.0 && (!CX || it.ai == 0.0);
    const int m = (active && !azero) ? it.m : 0;
    const HSMA_GLOBAL double *A = (const HSMA_GLOBAL double *)it.A;
    // Stage the quarter's lower triangle (16 x 16, ld 17; zero elsewhere):
    // lane i of the quarter takes row i of every column, so each column is
    // one contiguous read, and the unrolled loop issues all 16 loads before
    // the first LDS store waits for one.
    const int i = lane;
    V lv[kMax];
#pragma unroll
    for (int k = 0; k < kMax; ++k) {
        const bool rd = i < m && k < m && (UNIT ? k < i : k <= i);
        lv[k] = rd ? O::ld(A, i + (int64_t)k * it.lda) : (i == k ? O::one() : O::zero());
    }
#pragma unroll
    for (int k = 0; k < kMax; ++k) L[i + k * (kMax + 1)] = lv[k];
    if (!UNIT) {
        V d = O::one();
#pragma unroll
        for (int k = 0; k < kMax; ++k)
            if (k == i) d = lv[k];
        Rq[i] = O::recip(d);
    }
    __syncthreads();
    if (!active || lane >= it.ncols) return;
    HSMA_GLOBAL double *col = (HSMA_GLOBAL double *)it.B + (CX ? 2 : 1) * (int64_t)lane * it.ldb;
    if (azero) {
        for (int r = 0; r < it.m; ++r) O::st(col, r, O::zero());
        return;
    }
    V x[kMax];
#pragma unroll
    for (int r = 0; r < kMax; ++r) x[r] = r < m ? O::ld(col, r) : O::zero();  // all loads in flight
    if (it.ar != 1.0 || it.ai != 0.0) {
#pragma unroll
        for (int r = 0; r < kMax; ++r) x[r] = O::alpha(x[r], it.ar, it.ai);
    }
#pragma unroll
    for (int k = 0; k < kMax; ++k) {
        if (k < m) {
            if (!UNIT) x[k] = O::scale(x[k], Rq[k]);
            const V xk = x[k];
#pragma unroll
            for (int r = k + 1; r < kMax; ++r) O::fnms(x[r], L[r + k * (kMax + 1)], xk);
        }
    }
#pragma unroll
    for (int r = 0; r < kMax; ++r)
        if (r < m) O::st(col, r, x[r]);
}

template <bool CX>
hsma_status tiny_t(bool unit, const TinyItem &one, const TinyItem *items, int count, hipStream_t s) {
    const unsigned wgs = items ? (unsigned)((count + 3) / 4) : 1u;
    if (unit) hipLaunchKernelGGL((hsma_tiny<CX, true>), dim3(wgs), dim3(64), 0, s, one, items, count);
    else hipLaunchKernelGGL((hsma_tiny<CX, false>), dim3(wgs), dim3(64), 0, s, one, items, count);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

}  // namespace

bool tiny_fits(int64_t m, int64_t n) { return m >= 1 && m <= HSMA_TINY_MAX && n >= 1 && n <= HSMA_TINY_MAX; }

size_t tiny_item_bytes() { return sizeof(TinyItem); }

// One problem with m, n <= 16 (a single call).
hsma_status launch_tiny_one(bool cx, bool unit, int m, int n, cplx alpha, const double *A,
                            int64_t lda, double *B, int64_t ldb, hipStream_t s) {
    if (!tiny_fits(m, n)) return HSMA_INVALID_SIZE;
    TinyItem one{A, B, lda, ldb, m, n, alpha.re, cx ? alpha.im : 0.0};
    return cx ? tiny_t<true>(unit, one, nullptr, 1, s) : tiny_t<false>(unit, one, nullptr, 1, s);
}

// `count` items (device table, the batched item layout), four per workgroup.
hsma_status launch_tiny_group(bool cx, bool unit, const void *items, int count, hipStream_t s) {
    if (count <= 0) return HSMA_SUCCESS;
    TinyItem none{};
    const TinyItem *t = static_cast<const TinyItem *>(items);
    return cx ? tiny_t<true>(unit, none, t, count, s) : tiny_t<false>(unit, none, t, count, s);
}

}  // namespace hsma
