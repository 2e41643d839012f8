// The general BLAS TRSM on the left-lower kernels.
//
// The paper poses op(A) X = alpha B with A triangular (Sec. 2.1) and builds
// its kernels for the left-side, lower, no-transpose case.  Every other case
// is the same computation on re-indexed data:
//   - the right side X op(A) = alpha B is, transposed, op(A)^T X^T = alpha B^T;
//   - an upper-triangular operator U becomes lower under the index reversal
//     p(i) = k - 1 - i: (J U J)(J X) = alpha J B, J the reversal permutation;
//   - A^T and A^H are read with their indices swapped (and conjugated).
// So the effective left operator T (op(A) on the left, op(A)^T on the right)
// is copied, reversed if it is upper, into a lower-triangular workspace A',
// the right-hand side is gathered into B' (rows reversed, transposed for the
// right side) unless it can be solved in place, the left-lower solve runs on
// (A', B') with the library's own small or blocked path, and B' is scattered
// back.  The copies are HBM-bound: O(k^2 + m n) elements against the solve's
// O(k^2 n) or O(k^2 m) flops.
//
// Copy kernel: one 32 x 32 destination tile per workgroup.  With an index
// swap the tile goes through LDS so both the source reads and the destination
// writes walk down columns (coalesced).

#include <algorithm>

#include "internal.h"

namespace hsma {

int lookup_block_size(bool cx, int64_t m, int64_t n);
size_t blocked_workspace_bytes(bool cx, int64_t m, int ib);
hsma_status trsm_impl(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                      int64_t lda, void *B, int64_t ldb, hsma_dtype dtype, int ib_override,
                      int path, hipStream_t s, int *path_used, int *ib_used,
                      const hsma_trsm_options *opt, hsma_trsm_report *rep);

namespace {

enum : int {
    kSwap = 1,        // dst(i, j) reads src(j', i') instead of src(i', j')
    kRevI = 2,        // i' = R - 1 - i
    kRevJ = 4,        // j' = C - 1 - j
    kConj = 8,        // complex conjugate
    kLower = 16,      // only j <= i is written
    kStrict = 32,     // only j < i is written (a unit diagonal is not read)
};

constexpr int kT = 32;

// One element of the data: TC is the component type (double or float);
// complex elements are (re, im) pairs moved as one access.
template <typename TC, bool CX>
struct Elem {
    typedef TC T;
    static __device__ __forceinline__ T ld(const TC *p, int64_t idx) { return p[idx]; }
    static __device__ __forceinline__ void st(TC *p, int64_t idx, T v, bool) { p[idx] = v; }
};
template <typename TC>
struct Elem<TC, true> {
    typedef TC T __attribute__((ext_vector_type(2), aligned(sizeof(TC))));
    static __device__ __forceinline__ T ld(const TC *p, int64_t idx) {
        return *reinterpret_cast<const T *>(p + 2 * idx);
    }
    static __device__ __forceinline__ void st(TC *p, int64_t idx, T v, bool conj) {
        if (conj) v.y = -v.y;
        *reinterpret_cast<T *>(p + 2 * idx) = v;
    }
};

// dst (R x C, ldd) from src (ldsrc) under `flags`; element (i, j) of dst is
// src(i', j') or, with kSwap, src(j', i'), where i' and j' are i and j
// reversed if asked.  Grid: one workgroup per 32 x 32 tile of dst, tiles
// numbered down the columns of tiles (tr tile rows).
template <typename TC, bool CX>
__global__ __launch_bounds__(256) void hsma_transform(const TC *__restrict__ src, int64_t ldsrc,
                                                      TC *__restrict__ dst, int64_t ldd,
                                                      int64_t R, int64_t C, int64_t tr, int flags) {
    typedef Elem<TC, CX> E;
    typedef typename E::T T;
    __shared__ T tile[kT][kT + 1];
    const int64_t b = blockIdx.x;
    const int64_t i0 = (b % tr) * kT, j0 = (b / tr) * kT;
    const bool tri = flags & (kLower | kStrict);
    if (tri && j0 > i0 + kT - 1) return;  // tile above the diagonal
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const bool conj = CX && (flags & kConj);
    auto keep = [&](int64_t i, int64_t j) {
        if (i >= R || j >= C) return false;
        if (flags & kStrict) return j < i;
        if (flags & kLower) return j <= i;
        return true;
    };
    auto ri = [&](int64_t i) { return (flags & kRevI) ? R - 1 - i : i; };
    auto rj = [&](int64_t j) { return (flags & kRevJ) ? C - 1 - j : j; };
    if (flags & kSwap) {
        // Read: lanes along j (consecutive source rows j'); write: lanes along i.
#pragma unroll
        for (int q = 0; q < kT / 8; ++q) {
            const int li = ty + 8 * q, lj = tx;
            const int64_t i = i0 + li, j = j0 + lj;
            if (keep(i, j)) tile[li][lj] = E::ld(src, rj(j) + ri(i) * ldsrc);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kT / 8; ++q) {
            const int lj = ty + 8 * q, li = tx;
            const int64_t i = i0 + li, j = j0 + lj;
            if (keep(i, j)) E::st(dst, i + j * ldd, tile[li][lj], conj);
        }
    } else {
#pragma unroll
        for (int q = 0; q < kT / 8; ++q) {
            const int li = tx, lj = ty + 8 * q;
            const int64_t i = i0 + li, j = j0 + lj;
            if (keep(i, j)) E::st(dst, i + j * ldd, E::ld(src, ri(i) + rj(j) * ldsrc), conj);
        }
    }
}

template <typename TC>
hsma_status launch_transform(bool cx, const TC *src, int64_t ldsrc, TC *dst, int64_t ldd,
                             int64_t R, int64_t C, int flags, hipStream_t s) {
    if (R <= 0 || C <= 0) return HSMA_SUCCESS;
    const int64_t tr = (R + kT - 1) / kT, tc = (C + kT - 1) / kT;
    if (tr * tc > 0x7fffffff) return HSMA_INVALID_SIZE;
    ProfScope prof(HSMA_PHASE_OTHER, 0.0, s);
    if (cx)
        hipLaunchKernelGGL((hsma_transform<TC, true>), dim3((unsigned)(tr * tc)), dim3(256), 0, s,
                           src, ldsrc, dst, ldd, R, C, tr, flags);
    else
        hipLaunchKernelGGL((hsma_transform<TC, false>), dim3((unsigned)(tr * tc)), dim3(256), 0, s,
                           src, ldsrc, dst, ldd, R, C, tr, flags);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

}  // namespace

// dst (R x C, ldd) = src^H, src being C x R (ldsrc); the transpose for real
// data.
hsma_status launch_conj_transpose(bool cx, const double *src, int64_t ldsrc, double *dst,
                                  int64_t ldd, int64_t R, int64_t C, hipStream_t s) {
    return launch_transform<double>(cx, src, ldsrc, dst, ldd, R, C, kSwap | kConj, s);
}

// How a general case maps onto the left-lower solve (host only).
struct GeneralPlan {
    int64_t k;        // order of the effective operator
    int64_t nrhs;     // right-hand sides of the left-lower solve
    bool rev;         // the effective operator is upper: reverse its indices
    bool swap_a;      // the effective operator reads A transposed
    bool conj_a;      // ... and conjugated
    bool in_place;    // B itself is the left-lower right-hand side
};

GeneralPlan plan_general(int side, int uplo, int trans, bool cx, int64_t m, int64_t n) {
    GeneralPlan g{};
    const bool left = side == HSMA_LEFT;
    const bool notrans = trans == HSMA_OP_N;
    g.k = left ? m : n;
    g.nrhs = left ? n : m;
    // left: T = op(A), lower iff (lower stored) == (not transposed);
    // right: T = op(A)^T, lower iff (upper stored) == (not transposed).
    const bool t_lower = left ? ((uplo == HSMA_LOWER) == notrans) : ((uplo == HSMA_UPPER) == notrans);
    g.rev = !t_lower;
    // left: T_rc = op(A)_rc (A_rc, or A_cr transposed); right: T_rc = op(A)_cr.
    g.swap_a = left ? !notrans : notrans;
    g.conj_a = cx && trans == HSMA_OP_C;
    g.in_place = left && !g.rev;
    return g;
}

// The re-indexed solve of one general case on components TC.  `keep`, when
// given for a case that gathers B (k x nrhs, leading dimension k), takes the
// place of the workspace copy of B and holds the solved copy afterwards.
template <typename TC>
hsma_status general_t(hsma_side side, hsma_uplo uplo, hsma_op trans, hsma_diag diag, int64_t m,
                      int64_t n, const void *alpha, const TC *A, int64_t lda, TC *B, int64_t ldb,
                      hsma_dtype dtype, hipStream_t s, TC *keep = nullptr) {
    const bool cx = is_complex(dtype);
    const int es = cx ? 2 : 1;
    const cplx al = read_alpha(dtype, alpha);
    if (al.re == 0.0 && al.im == 0.0) {
        if (is_single(dtype)) return launch_zero32(m, n, es, reinterpret_cast<float *>(B), ldb, s);
        return launch_zero(m, n, es, reinterpret_cast<double *>(B), ldb, s);
    }
    const GeneralPlan g = plan_general(side, uplo, trans, cx, m, n);
    const int64_t k = g.k, nr = g.nrhs;
    // Without a reversal or a swap the triangle is A's own lower triangle (the
    // right-side transposed solve, as in a Cholesky step), and the solve reads
    // A where it lies.  A conjugation then moves to B and alpha, which are
    // copied anyway: X A^H = alpha B is A X^H = conj(alpha) B^H.  Conjugation
    // is exact, so the result is the same either way.
    const bool direct_a = !g.rev && !g.swap_a;
    const bool conj_b = direct_a && g.conj_a;
    const TC alpha_c[2] = {(TC)al.re, (TC)-al.im};
    const void *alpha_s = conj_b ? static_cast<const void *>(alpha_c) : alpha;
    const bool use_keep = keep && !g.in_place;
    const size_t a_elems = direct_a ? 0 : (size_t)k * k, b_elems = g.in_place || use_keep ? 0 : (size_t)k * nr;
    void *ws = nullptr;
    if (a_elems + b_elems > 0) HSMA_TRY(ws_alloc(&ws, (a_elems + b_elems) * es * sizeof(TC), s));
    TC *Ap = static_cast<TC *>(ws);
    TC *Bp = g.in_place ? B : use_keep ? keep : Ap + es * a_elems;
    const int64_t ldbp = g.in_place ? ldb : k;
    const int rev = g.rev ? (kRevI | kRevJ) : 0;
    const int fa = (diag == HSMA_UNIT ? kStrict : kLower) | rev | (g.swap_a ? kSwap : 0) |
                   (g.conj_a ? kConj : 0);
    hsma_status st = direct_a ? HSMA_SUCCESS : launch_transform<TC>(cx, A, lda, Ap, k, k, k, fa, s);
    // B' = J B (left, reversed) or J B^T (right)
    const bool left = side == HSMA_LEFT;
    if (st == HSMA_SUCCESS && !g.in_place)
        st = launch_transform<TC>(cx, B, ldb, Bp, k, k, nr,
                                  (g.rev ? kRevI : 0) | (left ? 0 : kSwap) | (conj_b ? kConj : 0), s);
    if (st == HSMA_SUCCESS)
        st = trsm_impl(diag, k, nr, alpha_s, direct_a ? A : Ap, direct_a ? lda : k, Bp, ldbp, dtype, 0, 0, s,
                       nullptr, nullptr, nullptr, nullptr);
    // B = J B' (left) or B(r, c) = B'(p(c), r) (right)
    if (st == HSMA_SUCCESS && !g.in_place)
        st = launch_transform<TC>(cx, Bp, k, B, ldb, m, n,
                                  (left ? (g.rev ? kRevI : 0) : (kSwap | (g.rev ? kRevJ : 0))) |
                                      (conj_b ? kConj : 0),
                                  s);
    hsma_status st2 = ws ? ws_free(ws, s) : HSMA_SUCCESS;
    return st != HSMA_SUCCESS ? st : st2;
}

hsma_status trsm_right_lower_keep(bool cx, int64_t m, int64_t n, const double *A, int64_t lda, double *B,
                                  int64_t ldb, double *xh, hipStream_t s) {
    const double one[2] = {1.0, 0.0};
    return general_t<double>(HSMA_RIGHT, HSMA_LOWER, cx ? HSMA_OP_C : HSMA_OP_T, HSMA_NON_UNIT, m, n, one, A,
                             lda, B, ldb, cx ? HSMA_C64F : HSMA_R64F, s, xh);
}

}  // namespace hsma

extern "C" hsma_status hsma_trsm_general(hsma_side side, hsma_uplo uplo, hsma_op trans,
                                         hsma_diag diag, int64_t m, int64_t n, const void *alpha,
                                         const void *A, int64_t lda, void *B, int64_t ldb,
                                         hsma_dtype dtype, hsma_stream_t stream) {
    using namespace hsma;
    if ((side != HSMA_LEFT && side != HSMA_RIGHT) || (uplo != HSMA_LOWER && uplo != HSMA_UPPER) ||
        (trans != HSMA_OP_N && trans != HSMA_OP_T && trans != HSMA_OP_C) ||
        (diag != HSMA_NON_UNIT && diag != HSMA_UNIT) ||
        (dtype != HSMA_R64F && dtype != HSMA_C64F && dtype != HSMA_R32F && dtype != HSMA_C32F))
        return HSMA_INVALID_VALUE;
    if (m < 0 || n < 0) return HSMA_INVALID_SIZE;
    const int64_t ka = side == HSMA_LEFT ? m : n;
    if (lda < std::max<int64_t>(1, ka) || ldb < std::max<int64_t>(1, m)) return HSMA_INVALID_SIZE;
    if (m == 0 || n == 0) return HSMA_SUCCESS;
    if (!alpha) return HSMA_INVALID_POINTER;
    const cplx al = read_alpha(dtype, alpha);
    const bool azero = al.re == 0.0 && al.im == 0.0;
    if (!B || (!A && !azero)) return HSMA_INVALID_POINTER;
    if (m > (int64_t)1 << 30 || n > (int64_t)1 << 30) return HSMA_INVALID_SIZE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (side == HSMA_LEFT && uplo == HSMA_LOWER && trans == HSMA_OP_N)
        return trsm_impl(diag, m, n, alpha, A, lda, B, ldb, dtype, 0, 0, s, nullptr, nullptr,
                         nullptr, nullptr);
    DeviceInfo dev;
    HSMA_TRY(device_info(&dev));
    if (!dev.arch_ok) return HSMA_NOT_SUPPORTED;
    if (is_single(dtype))
        return general_t<float>(side, uplo, trans, diag, m, n, alpha, static_cast<const float *>(A),
                                lda, static_cast<float *>(B), ldb, dtype, s);
    return general_t<double>(side, uplo, trans, diag, m, n, alpha, static_cast<const double *>(A),
                             lda, static_cast<double *>(B), ldb, dtype, s);
}
