// Cholesky factorization and solve on the library's TRSM (the first consumer
// the paper names for TRSM, Sec. 1: the forward and backward substitutions of
// LU and Cholesky).
//
// A = L L^H (real symmetric or complex Hermitian positive definite, lower
// triangle) by recursion on halves:
//     L11 = chol(A11)
//     L21 = A21 inv(L11)^H            the right-side, conjugate-transpose TRSM
//     A22 <- A22 - L21 L21^H          lower triangle only, FP64 matrix cores
//     L22 = chol(A22)
// with diagonal blocks of at most 64 rows factored by one wavefront, a row
// per lane in registers.
// The split point is a multiple of 64, so every base block is whole except
// the last.  The solve L L^H X = B is two TRSMs: L Y = B, then L^H X = Y.
//
// No definiteness check is made: a non-positive pivot gives NaN (the square
// root of a negative number), which propagates, as the TRSM propagates a zero
// diagonal.  The strict upper triangle of A is neither read nor written.

#include <algorithm>

#include "internal.h"

namespace hsma {

hsma_status trsm_impl(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                      int64_t lda, void *B, int64_t ldb, hsma_dtype dtype, int ib_override,
                      int path, hipStream_t s, int *path_used, int *ib_used,
                      const hsma_trsm_options *opt, hsma_trsm_report *rep);

namespace {

constexpr int kBase = 64;

template <bool CX>
struct Z;
template <>
struct Z<false> {
    typedef double V;
    static __device__ __forceinline__ V ld(const double *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ void st(double *p, int64_t i, V v) { p[i] = v; }
    static __device__ __forceinline__ double re(V v) { return v; }
    static __device__ __forceinline__ V scale(V v, double s) { return v * s; }
    // a - b conj(c)
    static __device__ __forceinline__ V fnms_conj(V a, V b, V c) { return __fma_rn(-b, c, a); }
    static __device__ __forceinline__ V real(double d) { return d; }
};
template <>
struct Z<true> {
    typedef dbl2u V;
    static __device__ __forceinline__ V ld(const double *p, int64_t i) {
        return *reinterpret_cast<const dbl2u *>(p + 2 * i);
    }
    static __device__ __forceinline__ void st(double *p, int64_t i, V v) {
        *reinterpret_cast<dbl2u *>(p + 2 * i) = v;
    }
    static __device__ __forceinline__ double re(V v) { return v.x; }
    static __device__ __forceinline__ V scale(V v, double s) { return V{v.x * s, v.y * s}; }
    static __device__ __forceinline__ V fnms_conj(V a, V b, V c) {
        // b conj(c) = (br cr + bi ci, bi cr - br ci), as four fused steps
        const double x = __fma_rn(-b.y, c.y, __fma_rn(-b.x, c.x, a.x));
        const double y = __fma_rn(b.x, c.y, __fma_rn(-b.y, c.x, a.y));
        return V{x, y};
    }
    static __device__ __forceinline__ V real(double d) { return V{d, 0.0}; }
};

// Lane l's value of v, to every lane (a wavefront-uniform scalar).
__device__ __forceinline__ double from_lane(double v, int l) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// One n x n diagonal block (n <= 64), right-looking, on four wavefronts:
// lane i of every wavefront holds row i, and wavefront w the columns c with
// c % 4 == w (16 of them, c = 4u + w in slot u).  At step j the wavefront
// that owns column j takes lane j's a_jj (a lane read), forms d = sqrt(a_jj)
// and 1/d, scales its a_ij by 1/d in the lanes below j (lane j keeps d), and
// publishes the column in LDS; after one barrier every wavefront updates its
// own columns c > j, a_ic -= l_ij conj(l_cj), with l_ij and l_cj read from
// that LDS column (a broadcast for l_cj).  The column buffer alternates
// between two copies, so a step's writes never meet the previous step's
// reads and one barrier per step suffices.  Entries right of a lane's
// diagonal and rows at or beyond n take values that are never stored and
// never read as l_cj (only rows c > j are read at step j).  Rows are loaded
// and stored column by column, consecutive lanes on consecutive rows.
template <bool CX>
__global__ __launch_bounds__(256) void hsma_potrf_base(double *__restrict__ A, int64_t lda, int n) {
    typedef Z<CX> O;
    typedef typename O::V V;
    constexpr int NW = 4, NU = kBase / NW;
    __shared__ V col[2][kBase];
    const int i = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool row_ok = i < n;
    V r[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int c = NW * u + w;
        r[u] = (row_ok && c <= i && c < n) ? O::ld(A, i + (int64_t)c * lda) : O::real(0.0);
    }
#pragma unroll
    for (int j = 0; j < kBase; ++j) {
        if (j < n) {
            V *cj = col[j & 1];
            if (w == (j % NW)) {
                const int uj = j / NW;
                const double d = sqrt(from_lane(O::re(r[uj]), j));
                const double inv = 1.0 / d;
                const V rj = r[uj];
                r[uj] = i > j ? O::scale(rj, inv) : (i == j ? O::real(d) : rj);
                cj[i] = r[uj];
            }
            __syncthreads();
            const V lij = cj[i];
            // Slot u holds columns NW u .. NW u + NW - 1 across the
            // wavefronts: once the loops are unrolled, "all of them beyond
            // j" and "none of them" are constants, and only the one slot
            // that straddles j tests this wavefront's column.  Every live
            // slot's l_cj is read first and the multiply-adds follow, so the
            // LDS reads overlap instead of waiting one by one.
            V lc[NU];
#pragma unroll
            for (int u = 0; u < NU; ++u)
                if (NW * u + NW - 1 > j) lc[u] = cj[NW * u + w];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int c = NW * u + w;
                const bool all_after = NW * u > j;
                const bool straddles = !all_after && NW * u + NW - 1 > j;
                if (all_after || (straddles && c > j)) r[u] = O::fnms_conj(r[u], lij, lc[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int c = NW * u + w;
        if (row_ok && c <= i && c < n) O::st(A, i + (int64_t)c * lda, r[u]);
    }
}

hsma_status potrf_base(bool cx, int n, double *A, int64_t lda, hipStream_t s) {
    ProfScope prof(HSMA_PHASE_FACTOR, (cx ? 4.0 : 1.0) * n * (double)n * n / 3.0, s);
    if (cx) hipLaunchKernelGGL(hsma_potrf_base<true>, dim3(1), dim3(256), 0, s, A, lda, n);
    else hipLaunchKernelGGL(hsma_potrf_base<false>, dim3(1), dim3(256), 0, s, A, lda, n);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

// The split of an order-n step: n1 is n/2 rounded up to a multiple of 64.
int64_t split(int64_t n) { return ((n / 2 + kBase - 1) / kBase) * kBase; }

// Largest n1 * n2 over every step of the recursion (the first half can be
// larger than n/2, so a step inside it can need more than the top one).
int64_t max_split_product(int64_t n) {
    if (n <= kBase) return 0;
    const int64_t n1 = split(n), n2 = n - n1;
    return std::max(n1 * n2, std::max(max_split_product(n1), max_split_product(n2)));
}

// `work` holds at least es * n1 * n2 doubles for every split of the
// recursion (the copy of L21^H that the trailing update reads as its right
// operand).
hsma_status potrf_rec(bool cx, int64_t n, double *A, int64_t lda, double *work, hipStream_t s) {
    if (n <= kBase) return potrf_base(cx, (int)n, A, lda, s);
    const int es = cx ? 2 : 1;
    const int64_t n1 = split(n), n2 = n - n1;
    double *A11 = A, *A21 = A + es * n1, *A22 = A + es * (n1 + n1 * lda);
    HSMA_TRY(potrf_rec(cx, n1, A11, lda, work, s));
    // L21 = A21 inv(L11)^H: X L11^H = A21, the right-side conjugate-transpose
    // TRSM (transpose for real data), which also leaves L21^H (n1 x n2) in
    // work: the right operand of the update.
    HSMA_TRY(trsm_right_lower_keep(cx, n2, n1, A11, lda, A21, lda, work, s));
    // A22 <- A22 - L21 L21^H on the lower triangle: one product with the
    // lower-triangular store.
    GemmBatch one_b;
    HSMA_TRY(launch_gemm(cx, GemmRole::Herk, (int)(es * n2), (int)n2, (int)(es * n1), cplx{-1.0, 0.0},
                         A21, lda, work, es * n1, cplx{1.0, 0.0}, A22, es * lda, 0, one_b, s, 0, 1));
    return potrf_rec(cx, n2, A22, lda, work, s);
}

}  // namespace
}  // namespace hsma

extern "C" hsma_status hsma_potrf(int64_t n, void *A, int64_t lda, hsma_dtype dtype,
                                  hsma_stream_t stream) {
    using namespace hsma;
    if (dtype != HSMA_R64F && dtype != HSMA_C64F && !is_single(dtype)) return HSMA_INVALID_VALUE;
    if (is_single(dtype)) return HSMA_NOT_SUPPORTED;
    if (n < 0) return HSMA_INVALID_SIZE;
    if (lda < std::max<int64_t>(1, n)) return HSMA_INVALID_SIZE;
    if (n == 0) return HSMA_SUCCESS;
    if (!A) return HSMA_INVALID_POINTER;
    if (n > (int64_t)1 << 30) return HSMA_INVALID_SIZE;
    DeviceInfo dev;
    HSMA_TRY(device_info(&dev));
    if (!dev.arch_ok) return HSMA_NOT_SUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool cx = dtype == HSMA_C64F;
    const int es = cx ? 2 : 1;
    double *Ad = static_cast<double *>(A);
    if (n <= kBase) return potrf_base(cx, (int)n, Ad, lda, s);
    void *ws = nullptr;
    HSMA_TRY(ws_alloc(&ws, (size_t)es * max_split_product(n) * sizeof(double), s));
    hsma_status st = potrf_rec(cx, n, Ad, lda, static_cast<double *>(ws), s);
    hsma_status st2 = ws_free(ws, s);
    return st != HSMA_SUCCESS ? st : st2;
}

extern "C" hsma_status hsma_potrs(int64_t n, int64_t nrhs, const void *L, int64_t lda, void *B,
                                  int64_t ldb, hsma_dtype dtype, hsma_stream_t stream) {
    using namespace hsma;
    if (dtype != HSMA_R64F && dtype != HSMA_C64F && !is_single(dtype)) return HSMA_INVALID_VALUE;
    if (is_single(dtype)) return HSMA_NOT_SUPPORTED;
    if (n < 0 || nrhs < 0) return HSMA_INVALID_SIZE;
    if (lda < std::max<int64_t>(1, n) || ldb < std::max<int64_t>(1, n)) return HSMA_INVALID_SIZE;
    if (n == 0 || nrhs == 0) return HSMA_SUCCESS;
    if (!L || !B) return HSMA_INVALID_POINTER;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double one[2] = {1.0, 0.0};
    // L Y = B, then L^H X = Y
    HSMA_TRY(trsm_impl(HSMA_NON_UNIT, n, nrhs, one, L, lda, B, ldb, dtype, 0, 0, s, nullptr,
                       nullptr, nullptr, nullptr));
    return hsma_trsm_general(HSMA_LEFT, HSMA_LOWER, dtype == HSMA_C64F ? HSMA_OP_C : HSMA_OP_T,
                             HSMA_NON_UNIT, n, nrhs, one, L, lda, B, ldb, dtype, stream);
}
