// Blocked path for m > 64 (paper Sec. 4.3).
//
// Phase 1 -- every diagonal block D_r (edge I_B, the last one ragged) is
// inverted independently: chunks of up to 64 rows by register substitution
// against identity right-hand sides (launch_diag_inv_base), then pairs of
// adjacent inverted blocks are merged level by level with the block formula
//      inv([[A, 0], [C, D]]) = [[inv(A), 0], [-inv(D) C inv(A), inv(D)]],
// two batched matrix-core products per level (T = C inv(A); W21 = -inv(D) T).
//
// Phase 2 -- the dependent part.  The paper walks the blocks left-looking
// (B_r -= A_{r,0:r} X_{0:r}, a product whose K grows with r).  Here the same
// algebra is walked recursively: solve the top half, apply one update
//      B_bot <- beta B_bot - L_{bot,top} X_top
// and solve the bottom half.  Half of all flops land in a single
// (m/2) x n x (m/2) product, so the matrix cores see large, square-ish
// products instead of I_B-tall slivers.  Leaves are X_r = alpha inv(D_r) B_r,
// written in place by a product whose single M-tile covers all I_B rows.
// alpha is folded into the first write of each row block (beta = alpha on
// the first update a block receives, or alpha in its leaf if none).

#include <algorithm>
#include <vector>

#include "internal.h"

namespace hsma {

namespace {

// T is double (DTRSM, ZTRSM) or float (STRSM, CTRSM); complex data is
// interleaved (re, im) of T, and every offset below counts components of T.
template <typename T>
struct Ctx {
    bool cx;
    bool unit;
    bool mixed = false;  // trailing updates on the FP32 matrix cores (double only)
    int64_t m, n;
    cplx alpha;
    const T *A;
    int64_t lda;
    T *B;
    int64_t ldb;
    int ib;
    T *W;  // nblk * ib * ib elements
    T *Tm; // combine scratch
    hipStream_t s;
    int es() const { return cx ? 2 : 1; }
};

// Merge inverted diagonal sub-blocks of edge `sz` into blocks of edge 2*sz.
// One batched launch pair per group of equally-sized pairs.
template <typename T>
hsma_status combine_group(const Ctx<T> &c, int sz, int64_t first_row, int npairs_outer,
                          int npairs_inner, int tsz) {
    // Pair (bo, bi): top-left at global row g = first_row + bo*ib + bi*2*sz,
    // top size sz, bottom size tsz (<= sz).
    if (npairs_outer <= 0 || npairs_inner <= 0 || tsz <= 0) return HSMA_SUCCESS;
    const int es = c.es();
    const int64_t ib = c.ib, lda = c.lda;
    const int64_t blk0 = first_row / ib, off0 = first_row % ib;
    // A operand (C block of L): rows g+sz.., cols g..
    const T *Lc = c.A + es * ((first_row + sz) + first_row * lda);
    // inv(A) and inv(D) and W21 inside W.
    const T *Wa = c.W + es * (blk0 * ib * ib + off0 + off0 * ib);
    const T *Wd = c.W + es * (blk0 * ib * ib + (off0 + sz) + (off0 + sz) * ib);
    T *W21 = c.W + es * (blk0 * ib * ib + (off0 + sz) + off0 * ib);
    GemmBatch b1, b2;
    b1.count = b2.count = npairs_outer * npairs_inner;
    b1.inner = b2.inner = npairs_inner;
    // Step 1: T = C * inv(A)   (tsz x sz) = (tsz x sz)(sz x sz)
    b1.a_outer = es * ib * (1 + lda);
    b1.a_inner = es * 2 * sz * (1 + lda);
    b1.b_outer = es * ib * ib;
    b1.b_inner = es * 2 * sz * (1 + ib);
    b1.c_outer = es * (int64_t)npairs_inner * sz * sz;
    b1.c_inner = es * (int64_t)sz * sz;
    HSMA_TRY(launch_gemm(c.cx, GemmRole::Inverse, es * tsz, sz, es * sz, cplx{1.0, 0.0}, Lc, lda,
                         Wa, es * ib, cplx{0.0, 0.0}, c.Tm, es * tsz, 0, b1, c.s));
    // Step 2: W21 = -inv(D) * T   (tsz x sz) = (tsz x tsz)(tsz x sz)
    b2.a_outer = es * ib * ib;
    b2.a_inner = es * 2 * sz * (1 + ib);
    b2.b_outer = b1.c_outer;
    b2.b_inner = b1.c_inner;
    b2.c_outer = es * ib * ib;
    b2.c_inner = es * 2 * sz * (1 + ib);
    HSMA_TRY(launch_gemm(c.cx, GemmRole::Inverse, es * tsz, sz, es * tsz, cplx{-1.0, 0.0}, Wd, ib,
                         c.Tm, es * tsz, cplx{0.0, 0.0}, W21, es * ib, 0, b2, c.s));
    return HSMA_SUCCESS;
}

template <typename T>
hsma_status invert_diagonal(const Ctx<T> &c, int base) {
    HSMA_TRY(launch_diag_inv_base(c.cx, c.unit, (int)c.m, base, c.ib, c.A, c.lda, c.W, c.s));
    const int64_t m = c.m, ib = c.ib;
    const int64_t nfull = m / ib;
    const int64_t rem = m - nfull * ib;
    for (int sz = base; sz < ib; sz *= 2) {
        // Full blocks: ib / (2 sz) uniform pairs each.
        HSMA_TRY(combine_group(c, sz, 0, (int)nfull, (int)(ib / (2 * sz)), sz));
        if (rem > 0) {
            const int64_t g = nfull * ib;
            const int64_t full_pairs = rem / (2 * sz);
            HSMA_TRY(combine_group(c, sz, g, 1, (int)full_pairs, sz));
            const int64_t a = full_pairs * 2 * sz;
            const int64_t t = rem - a - sz;
            if (t > 0) HSMA_TRY(combine_group(c, sz, g + a, 1, 1, (int)t));
        }
    }
    return HSMA_SUCCESS;
}

template <typename T>
hsma_status leaf(const Ctx<T> &c, int64_t blk, bool touched) {
    const int es = c.es();
    const int64_t r0 = blk * c.ib;
    const int mr = (int)std::min<int64_t>(c.ib, c.m - r0);
    const T *Wr = c.W + es * (blk * (int64_t)c.ib * c.ib);
    T *Br = c.B + es * r0;
    GemmBatch one;
    return launch_gemm(c.cx, GemmRole::Leaf, es * mr, (int)c.n, es * mr,
                       touched ? cplx{1.0, 0.0} : c.alpha, Wr, c.ib, Br, es * c.ldb,
                       cplx{0.0, 0.0}, Br, es * c.ldb, 0, one, c.s);
}

template <typename T>
hsma_status update(const Ctx<T> &c, int64_t r1, int64_t r2, int64_t k0, bool touched) {
    // B[r1:r2] = beta B[r1:r2] - L[r1:r2, k0:r1] B[k0:r1]
    const int es = c.es();
    GemmBatch one;
    const cplx beta = touched ? cplx{1.0, 0.0} : c.alpha;
    return launch_gemm(c.cx, c.mixed ? GemmRole::UpdateMixed : GemmRole::Update,
                       (int)(es * (r2 - r1)), (int)c.n, (int)(es * (r1 - k0)),
                       cplx{-1.0, 0.0}, c.A + es * (r1 + k0 * c.lda), c.lda, c.B + es * k0,
                       es * c.ldb, beta, c.B + es * r1, es * c.ldb, 0, one, c.s);
}

template <typename T>
hsma_status recurse(const Ctx<T> &c, int64_t b0, int64_t nb, bool touched) {
    if (nb == 1) return leaf(c, b0, touched);
    const int64_t h = nb / 2;
    HSMA_TRY(recurse(c, b0, h, touched));
    const int64_t r1 = (b0 + h) * c.ib;
    const int64_t r2 = std::min<int64_t>((b0 + nb) * c.ib, c.m);
    HSMA_TRY(update(c, r1, r2, b0 * c.ib, touched));
    return recurse(c, b0 + h, nb - h, true);
}

// Components of T the workspace needs: W (nblk blocks of ib x ib) and the
// combine scratch (at most m/2 rows by ib/2 columns at the top level).
size_t workspace_elems(bool cx, int64_t m, int ib) {
    const int64_t nblk = (m + ib - 1) / ib;
    const size_t es = cx ? 2 : 1;
    return (size_t)nblk * ib * ib * es + (size_t)((m + 1) / 2 + ib) * (size_t)ib * es;
}

template <typename T>
hsma_status blocked_t(bool cx, bool unit, int64_t m, int64_t n, cplx alpha, const T *A,
                      int64_t lda, T *B, int64_t ldb, int ib, void *ws, hipStream_t s, bool mixed) {
    Ctx<T> c;
    c.mixed = mixed;
    c.cx = cx;
    c.unit = unit;
    c.m = m;
    c.n = n;
    c.alpha = alpha;
    c.A = A;
    c.lda = lda;
    c.B = B;
    c.ldb = ldb;
    c.ib = ib;
    c.s = s;
    const int64_t nblk = (m + ib - 1) / ib;
    c.W = static_cast<T *>(ws);
    c.Tm = c.W + (cx ? 2 : 1) * nblk * (int64_t)ib * ib;
    const int base = std::min(ib, 64);
    HSMA_TRY(invert_diagonal(c, base));
    return recurse(c, 0, nblk, false);
}

}  // namespace

size_t blocked_workspace_bytes(bool cx, int64_t m, int ib) {
    return workspace_elems(cx, m, ib) * sizeof(double);
}

size_t blocked_workspace_bytes32(bool cx, int64_t m, int ib) {
    return workspace_elems(cx, m, ib) * sizeof(float);
}

// Enqueue the blocked solve.  `ws` must hold blocked_workspace_bytes().
hsma_status blocked_trsm(bool cx, bool unit, int64_t m, int64_t n, cplx alpha, const double *A,
                         int64_t lda, double *B, int64_t ldb, int ib, void *ws, hipStream_t s,
                         bool mixed) {
    return blocked_t<double>(cx, unit, m, n, alpha, A, lda, B, ldb, ib, ws, s, mixed);
}

// The FP32 solve (STRSM, CTRSM).  `ws` must hold blocked_workspace_bytes32().
hsma_status blocked_trsm32(bool cx, bool unit, int64_t m, int64_t n, cplx alpha, const float *A,
                           int64_t lda, float *B, int64_t ldb, int ib, void *ws, hipStream_t s) {
    return blocked_t<float>(cx, unit, m, n, alpha, A, lda, B, ldb, ib, ws, s, false);
}

// R <- R - tril(L) X, the residual of refinement and of the backward-error
// report (FP64 products).  One product over the whole triangle: each row
// tile accumulates its full row of L times X in one FP64 accumulator chain
// (K up to the tile's last row, the part above the diagonal masked to zero,
// a unit diagonal taken as 1) and subtracts it from R once.  This order has
// nothing in common with the solve's recursion, so the rounding of the solve's
// updates does not cancel out of the residual and the reported backward error
// measures the solve, not its leaves alone.
hsma_status triangular_residual(bool cx, bool unit, int64_t m, int64_t n, const double *A,
                                int64_t lda, const double *X, int64_t ldx, double *R, int64_t ldr,
                                hipStream_t s) {
    const int es = cx ? 2 : 1;
    GemmBatch one;
    return launch_gemm(cx, GemmRole::Residual, (int)(es * m), (int)n, (int)(es * m),
                       cplx{-1.0, 0.0}, A, lda, X, es * ldx, cplx{1.0, 0.0}, R, es * ldr,
                       unit ? 2 : 1, one, s, /*k_lower=*/1);
}

}  // namespace hsma
