// Fused solves of very small problems (m, n <= 16): four problems per
// wavefront.  The paper names kernel fusion for very small scales as future
// work (Sec. 6).
//
// Each 16-lane quarter of the wavefront (one DPP row) is one problem.  Lane i
// of the quarter holds row i of L in 16 registers and column i of B in 16
// more; the substitution chain
//     x_k <- x_k / l_kk,   x_i <- x_i - l_ik x_k  (i > k)
// runs in the registers: at step k every lane scales its row k by lane k's
// reciprocal of l_kk, and the coefficient l_ik reaches the lane through a
// row broadcast of lane i's register that is the source operand of the
// multiply-add (the diagonal walk of the strip kernel, on one 16-row block).
// B moves through a small LDS stage (one 16 x 16 block per quarter) so that
// global loads and stores walk down columns, 16 lanes on one segment; L's
// rows are read straight into registers.  The walk stops after the largest m
// among the wavefront's four problems.  Rows at or beyond a problem's m hold
// a unit diagonal and zero coefficients, so every value stays finite, and
// they only ever feed rows at or beyond m, which are never stored.  The arithmetic of a problem does not depend on its quarter or
// launch, and it is the strip kernel's, so a problem gives the same bits
// alone, in a batch and in a strip.

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

// Element operations (loads, stores, alpha, the reciprocal of a diagonal
// entry), rounded as in the strip kernel: alpha scales only when it is not
// 1, and complex products are spelled out (cmul_rn, recip_rn).
template <bool CX>
struct D;
template <>
struct D<false> {
    typedef double V;
    static __device__ __forceinline__ V ld(const HSMA_GLOBAL double *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ void st(HSMA_GLOBAL double *p, int64_t i, V v) { p[i] = v; }
    static __device__ __forceinline__ V zero() { return 0.0; }
    static __device__ __forceinline__ V one() { return 1.0; }
    static __device__ __forceinline__ V alpha(V x, double ar, double) { return __dmul_rn(x, ar); }
    static __device__ __forceinline__ V recip(V d) {
        double r, i;
        smallk::recip_rn(false, d, 0.0, r, i);
        return r;
    }
    static __device__ __forceinline__ void split(V v, double &r, double &i) {
        r = v;
        i = 0.0;
    }
    static __device__ __forceinline__ V join(double r, double) { return r; }
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
    static __device__ __forceinline__ void split(V v, double &r, double &i) {
        r = v.x;
        i = v.y;
    }
    static __device__ __forceinline__ V join(double r, double i) { return V{r, i}; }
};

// Step K of the walk: x_K is scaled by lane K's reciprocal of l_KK (one
// product with the reciprocal, as in the strip kernel), then rows K+1..15
// receive -l_iK x_K, with l_iK broadcast from lane i inside the multiply-add.
// Steps from the wavefront's largest m on are skipped (mmax is uniform).
template <bool CX, bool UNIT, int K>
__device__ __forceinline__ void reg_walk(double (&xr)[kMax], double (&xi)[kMax], const double (&lr)[kMax],
                                         const double (&li)[kMax], double rr, double ri, int mmax) {
    if constexpr (K < kMax) {
        if (K >= mmax) return;
        if (!UNIT) {
            const double dr = smallk::bcast16<K>(rr);
            if (CX) {
                const double di = smallk::bcast16<K>(ri);
                smallk::cmul_rn(xr[K], xi[K], dr, di, xr[K], xi[K]);
            } else {
                xr[K] = __dmul_rn(xr[K], dr);
            }
        }
        if constexpr (K + 1 < kMax) smallk::fnma_rows<CX, K + 1>(xr, xi, lr[K], li[K], xr[K], xi[K]);
        reg_walk<CX, UNIT, K + 1>(xr, xi, lr, li, rr, ri, mmax);
    }
}

// Workgroup b solves items 4b .. 4b + 3 (those below count); with items ==
// nullptr it solves `one` alone (a single call, no descriptor upload).
// Every lane stays active through the walk: lanes beyond a problem's n still
// hold rows of L that the others receive by broadcast.
template <bool CX, bool UNIT>
__global__ __launch_bounds__(64) void hsma_tiny(TinyItem one, const TinyItem *__restrict__ items,
                                                int count) {
    typedef D<CX> O;
    typedef typename O::V V;
    const int q = threadIdx.x >> 4, lane = threadIdx.x & 15;
    const int idx = blockIdx.x * 4 + q;
    const bool active = items ? idx < count : q == 0;
    TinyItem it = one;
    if (items && active) it = items[idx];
    if (!active) it.m = it.ncols = 0;
    // alpha == 0: B <- 0, and neither A nor B is read (A may be null).
    const bool azero = it.ar == 0.0 && (!CX || it.ai == 0.0);
    const int m = azero ? 0 : it.m;
    // the largest m of the wavefront's four problems
    int mmax = __builtin_amdgcn_readlane(m, 0);
    mmax = max(mmax, __builtin_amdgcn_readlane(m, 16));
    mmax = max(mmax, __builtin_amdgcn_readlane(m, 32));
    mmax = max(mmax, __builtin_amdgcn_readlane(m, 48));
    const HSMA_GLOBAL double *A = (const HSMA_GLOBAL double *)it.A;
    // Row i of L: this lane's coefficients (zero elsewhere, 1 on the diagonal
    // of rows >= m); all 16 loads are issued before the first use.
    const int i = lane;
    V lv[kMax];
#pragma unroll
    for (int k = 0; k < kMax; ++k) {
        const bool rd = i < m && k < m && (UNIT ? k < i : k <= i);
        lv[k] = rd ? O::ld(A, i + (int64_t)k * it.lda) : (i == k ? O::one() : O::zero());
    }
    // B passes through an LDS stage in whole column segments: lane r of the
    // quarter reads row r of every column (the quarter's 16 lanes on one
    // segment), and lane c then takes column c (zero beyond m and n).
    __shared__ V Bs[4 * kMax * (kMax + 1)];
    V *Bq = Bs + q * kMax * (kMax + 1);
    HSMA_GLOBAL double *Bb = (HSMA_GLOBAL double *)it.B;
    {
        V t[kMax];
#pragma unroll
        for (int c = 0; c < kMax; ++c)
            t[c] = (lane < m && c < it.ncols) ? O::ld(Bb, lane + (int64_t)c * it.ldb) : O::zero();
#pragma unroll
        for (int c = 0; c < kMax; ++c) Bq[c * (kMax + 1) + lane] = t[c];
    }
    __builtin_amdgcn_wave_barrier();
    V x[kMax];
#pragma unroll
    for (int r = 0; r < kMax; ++r) x[r] = Bq[lane * (kMax + 1) + r];
    // Reciprocal of this lane's diagonal entry (row i).
    V rcp = O::one();
    if (!UNIT) {
        V d = O::one();
#pragma unroll
        for (int k = 0; k < kMax; ++k)
            if (k == i) d = lv[k];
        rcp = O::recip(d);
    }
    if (it.ar != 1.0 || it.ai != 0.0) {
#pragma unroll
        for (int r = 0; r < kMax; ++r) x[r] = O::alpha(x[r], it.ar, it.ai);
    }
    double xr[kMax], xi[kMax], lr[kMax], li[kMax];
#pragma unroll
    for (int r = 0; r < kMax; ++r) {
        O::split(x[r], xr[r], xi[r]);
        O::split(lv[r], lr[r], li[r]);
    }
    double rr, ri;
    O::split(rcp, rr, ri);
    reg_walk<CX, UNIT, 0>(xr, xi, lr, li, rr, ri, mmax);
    // back through the stage: lane c writes column c, lane r stores row r
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < kMax; ++r) Bq[lane * (kMax + 1) + r] = azero ? O::zero() : O::join(xr[r], xi[r]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < kMax; ++c)
        if (lane < it.m && c < it.ncols) O::st(Bb, lane + (int64_t)c * it.ldb, Bq[c * (kMax + 1) + lane]);
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
