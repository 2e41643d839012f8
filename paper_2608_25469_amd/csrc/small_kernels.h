// Register-resident forward substitution shared by the small-regime kernels.
//
// Paper, Sec. 4.2.1: columns of B are independent, so each column is a
// separate forward substitution; the triangular operand is shared.  Lane j
// of a 64-lane wavefront keeps column j in VGPRs, so the row-dependency chain
// runs inside a lane with no synchronisation at all.
//
// This header holds the DPP broadcast helpers (used here and by the strip
// kernel of general right-hand sides, strip.hip) and the right-looking Panel
// walk, which the blocked path uses with identity right-hand sides to invert
// its diagonal chunks (Sec. 4.3.1): the whole column stays live (y[0..m-1]).
// L's packed lower triangle is staged once in LDS with direct global-to-LDS
// loads (no VGPR round trip).  At step k, column k+1 is read from LDS into
// ceil(m/16) VGPRs laid out so that each 16-lane row of the wavefront holds
// 16 consecutive rows of the column, and each coefficient reaches all lanes
// through the 64-bit DPP row_newbcast broadcast with no further memory
// traffic.  The column for the next step is read before the current step's
// arithmetic, so LDS latency hides behind the dependency chain.  The loop
// nest is fully unrolled for a compile-time row bound MAXM (a multiple of 8)
// and guarded by the runtime m.  Reciprocals of the diagonal are computed one
// per lane and broadcast to the whole wave with v_readlane when row k is
// divided.

#pragma once

#include <type_traits>

#include "internal.h"
#include "dpp_fma.h"

namespace hsma {
namespace smallk {


__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Complex product and reciprocal with every rounding fixed (no contraction
// left to the compiler): the small-solve kernels share them, so the same
// problem gives the same bits in every kernel that solves it.
__device__ __forceinline__ void cmul_rn(double ar, double ai, double br, double bi, double &r,
                                        double &i) {
    r = __fma_rn(ar, br, -__dmul_rn(ai, bi));
    i = __fma_rn(ar, bi, __dmul_rn(ai, br));
}
// 1/d (real) or conj(d)/|d|^2 (complex).
__device__ __forceinline__ void recip_rn(bool cx, double dr, double di, double &rr, double &ri) {
    if (cx) {
        const double den = __fma_rn(dr, dr, __dmul_rn(di, di));
        rr = __ddiv_rn(dr, den);
        ri = -__ddiv_rn(di, den);
    } else {
        rr = __ddiv_rn(1.0, dr);
        ri = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Broadcast of L.  Every lane needs every coefficient l_ik (lane j works on
// column j).  Column k of L is loaded with vector loads into NQ = ceil(MAXM/16)
// VGPRs (two per complex value) such that each 16-lane row of the wavefront
// holds rows 16q..16q+15 of the column: lane l holds l_{16q + l%16, k}.  The
// 64-bit DPP control row_newbcast:r then hands lane r of each 16-lane row to
// all 16 lanes of that row, i.e. l_{16q+r, k} to the whole wave.  Row indices
// are clamped to m-1 (addresses never leave A); the values of rows >= m and
// of rows on or above the diagonal are never used by an update that matters.
// ---------------------------------------------------------------------------
// Every row and bank is enabled, so no lane keeps an old value: mov_dpp
// (old value undefined) needs no copy of the destination first, unlike
// update_dpp with a tied old operand.
template <int N>
__device__ __forceinline__ double bcast16(double v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xf, 0xf, false);  // row_newbcast:N
}

// Static dispatch of row_newbcast on a compile-time row number.
template <int I>
struct RowB {
    static __device__ __forceinline__ double get(double v) { return bcast16<(I & 15)>(v); }
};

// y -= l * x for real (li ignored) or complex values.
template <bool CX>
__device__ __forceinline__ void fms(double &yr, double &yi, double lr, double li, double xr,
                                    double xi) {
    if (CX) {
        yr = __fma_rn(-lr, xr, yr);
        yr = __fma_rn(li, xi, yr);
        yi = __fma_rn(-lr, xi, yi);
        yi = __fma_rn(-li, xr, yi);
    } else {
        yr = __fma_rn(-lr, xr, yr);
    }
}

// Applies column K (already final as xr/xi) to rows K+1..MAXM-1.
template <bool CX, int MAXM, int K, int I>
struct ApplyRows {
    static __device__ __forceinline__ void run(double (&yr)[MAXM], double (&yi)[MAXM],
                                               const double (&Lr)[(MAXM + 15) / 16],
                                               const double (&Li)[(MAXM + 15) / 16], double xr,
                                               double xi) {
        if constexpr (I < MAXM) {
            const double lr = RowB<I>::get(Lr[I / 16]);
            const double li = CX ? RowB<I>::get(Li[I / 16]) : 0.0;
            fms<CX>(yr[I], yi[I], lr, li, xr, xi);
            ApplyRows<CX, MAXM, K, I + 1>::run(yr, yi, Lr, Li, xr, xi);
        }
    }
};

// One 64-column panel: lane j solves column j (j < ncols) in registers.
// A: m x m, lda; B: m x ncols, ldb (element units; complex interleaved).
// m lies in (MAXM-8, MAXM].
template <bool CX, int MAXM, bool UNIT>
struct Panel {
    static constexpr int NQ = (MAXM + 15) / 16;
    static constexpr int ES = CX ? 2 : 1;
    // Packed lower triangle (rows k..MAXM-1 of column k), in doubles.
    static constexpr int TRI = MAXM * (MAXM + 1) / 2;
    static __host__ __device__ constexpr int col_off(int k) { return k * MAXM - k * (k - 1) / 2; }

    // Coefficients of column K for the 16-row groups holding rows below K:
    // lane l takes row 16q + l%16 (clamped into the column) from LDS.
    template <int K>
    static __device__ __forceinline__ void read_col(const double *Ls, int lane, double (&Lr)[NQ],
                                                    double (&Li)[NQ]) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            Lr[q] = Li[q] = 0.0;
            if (K < MAXM && 16 * q + 15 > K) {
                int row = 16 * q + (lane & 15);
                row = row < K ? K : (row > MAXM - 1 ? MAXM - 1 : row);
                const int e = col_off(K) + (row - K);
                if (CX) {
                    Lr[q] = Ls[2 * e];
                    Li[q] = Ls[2 * e + 1];
                } else {
                    Lr[q] = Ls[e];
                }
            }
        }
    }

    // Step K: x_K = y_K / l_KK, then rows below K receive -l_iK x_K.  The
    // coefficients of column K were read from LDS one step earlier (cur);
    // this step reads those of column K+1 (nxt) before its own arithmetic.
    template <int K>
    static __device__ __forceinline__ void step(const double *Ls, int m, int lane, double rr,
                                                double ri, double (&yr)[MAXM], double (&yi)[MAXM],
                                                double (&cr)[NQ], double (&ci)[NQ]) {
        if constexpr (K < MAXM) {
            double nr[NQ], ni[NQ];
            // Each column step is its own basic block (K < m is uniform): this
            // keeps the instruction selector from sinking the step's
            // multiply-adds to their final uses, which would keep every
            // broadcast coefficient of the unrolled body alive at once.  The
            // next step is nested inside this one's block, so the steps form a
            // chain with early exits and the row values never pass through a
            // join per step (which would cost a register copy of every row at
            // every step).
            if (K < m) {
                read_col<K + 1>(Ls, lane, nr, ni);
                if (!UNIT) {
                    const double dr = readlane_d(rr, K);
                    if (CX) {
                        const double di = readlane_d(ri, K);
                        cmul_rn(yr[K], yi[K], dr, di, yr[K], yi[K]);
                    } else {
                        yr[K] = __dmul_rn(yr[K], dr);
                    }
                }
                if constexpr (K + 1 < MAXM) ApplyRows<CX, MAXM, K, K + 1>::run(yr, yi, cr, ci, yr[K], yi[K]);
                step<K + 1>(Ls, m, lane, rr, ri, yr, yi, nr, ni);
            }
        }
    }

    // IDENT: the right-hand side is the identity (column j = e_j) and the
    // result goes to Bout; this produces inv(L) column by column (the
    // identity-tile right-hand side of the paper's Sec. 4.3.1).
    template <bool IDENT>
    static __device__ __forceinline__ void solve(const double *__restrict__ A, int64_t lda,
                                                 double *__restrict__ B, int64_t ldb, int m,
                                                 int ncols, cplx alpha) {
        // The lane id passes through an empty asm, so the compiler cannot
        // precompute the LDS and row indices that every unrolled step derives
        // from it and keep them all live at once (which costs registers).
        int lane = threadIdx.x & 63;
        asm volatile("" : "+v"(lane));
        const bool active = lane < ncols;
        HSMA_GLOBAL double *__restrict__ bc = (HSMA_GLOBAL double *)(B + ES * (int64_t)(active ? lane : 0) * ldb);

        // Reciprocal of the diagonal, one entry per lane: 1/d or conj(d)/|d|^2.
        double rr = 1.0, ri = 0.0;
        if (!UNIT && lane < m) {
            const HSMA_GLOBAL double *d = (const HSMA_GLOBAL double *)(A + ES * ((int64_t)lane + (int64_t)lane * lda));
            recip_rn(CX, d[0], CX ? d[1] : 0.0, rr, ri);
        }

        // Column j of the panel; rows >= m are read at row m-1 and then zeroed.
        double yr[MAXM], yi[MAXM];
#pragma unroll
        for (int i = 0; i < MAXM; ++i) {
            const int ic = i < m ? i : m - 1;
            if (IDENT) {
                yr[i] = (i == lane) ? 1.0 : 0.0;
                yi[i] = 0.0;
            } else if (CX) {
                const dbl2u v = reinterpret_cast<const HSMA_GLOBAL dbl2u *>(bc)[ic];
                yr[i] = v.x;
                yi[i] = v.y;
            } else {
                yr[i] = bc[ic];
                yi[i] = 0.0;
            }
            if (i >= m) yr[i] = yi[i] = 0.0;
        }
        if (alpha.re != 1.0 || alpha.im != 0.0) {
#pragma unroll
            for (int i = 0; i < MAXM; ++i) {
                if (CX) {
                    cmul_rn(alpha.re, alpha.im, yr[i], yi[i], yr[i], yi[i]);
                } else {
                    yr[i] = __dmul_rn(yr[i], alpha.re);
                }
            }
        }

        // Stage the packed lower triangle of L in LDS with direct
        // global-to-LDS loads (no VGPRs involved).  Each instruction writes a
        // whole wavefront's width (64 x 16 bytes for complex, 64 x 4 bytes for
        // real) contiguously from the start of column k's packed segment; the
        // part past the segment's end lands in the next column's segment,
        // which that column's own (later, in-order) loads overwrite, or in the
        // slack after the last column.  Source rows and columns are clamped
        // to m-1, so no load leaves A; the values of rows or columns >= m are
        // only ever combined into rows >= m, which are never stored.
        __shared__ double Ls[ES * TRI + (CX ? 128 : 32)];
        typedef __attribute__((address_space(3))) void lds_void;
        const int mc = m - 1;
#pragma unroll
        for (int k = 0; k < MAXM; ++k) {
            const int kc = k < mc ? k : mc;
            if (CX) {
                int row = k + lane;
                row = row < mc ? row : mc;
                const double *src = A + 2 * ((int64_t)kc * lda + row);
                __builtin_amdgcn_global_load_lds((const void *)src, (lds_void *)(Ls + 2 * col_off(k)),
                                                 16, 0, 0);
            } else {
#pragma unroll
                for (int h = 0; h * 32 < MAXM - k; ++h) {
                    int row = k + 32 * h + (lane >> 1);
                    row = row < mc ? row : mc;
                    const char *src = reinterpret_cast<const char *>(A + (int64_t)kc * lda + row) +
                                      4 * (lane & 1);
                    __builtin_amdgcn_global_load_lds((const void *)src,
                                                     (lds_void *)(Ls + col_off(k) + 32 * h), 4, 0, 0);
                }
            }
        }
        __syncthreads();
        double cr[NQ], ci[NQ];
        read_col<0>(Ls, lane, cr, ci);
        step<0>(Ls, m, lane, rr, ri, yr, yi, cr, ci);

        if (active) {
#pragma unroll
            for (int i = 0; i < MAXM; ++i) {
                if (i < m) {
                    if (CX)
                        reinterpret_cast<HSMA_GLOBAL dbl2u *>(bc)[i] = dbl2u{yr[i], yi[i]};
                    else
                        bc[i] = yr[i];
                }
            }
        }
    }
};

// Work item of the small-solve kernel (strip.hip): one strip of at most 16
// columns of one problem.
struct SmallItem {
    const double *A;
    double *B;        // first column of the strip
    int64_t lda, ldb; // element units
    int32_t m, ncols;
    double ar, ai;    // alpha
};

// Phase 1 of the blocked path (paper Sec. 4.3): the diagonal of L is cut
// into consecutive chunks of `base` rows (the last one ragged) and every chunk
// D is inverted independently, one wavefront per chunk: lane j solves
// D x = e_j in registers.  inv(D) lands in the ib x ib diagonal-block
// workspace W at its place inside its block (ld = ib).
template <bool CX, int NCH, bool UNIT>
__global__ __launch_bounds__(64) void hsma_diag_inv_base(const double *__restrict__ A, int64_t lda,
                                                         double *__restrict__ W, int m, int base,
                                                         int ib) {
    const int64_t o = (int64_t)blockIdx.x * base;
    const int mb = (int)((m - o) < base ? (m - o) : base);
    const int64_t blk = o / ib, oo = o % ib;
    constexpr int ES = CX ? 2 : 1;
    const double *Ad = A + ES * (o + o * lda);
    double *Wd = W + ES * (blk * (int64_t)ib * ib + oo + oo * ib);
    Panel<CX, 8 * NCH, UNIT>::template solve<true>(Ad, lda, Wd, ib, mb, mb, cplx{1.0, 0.0});
}

// The same for many matrices in one launch: workgroup b inverts the chunk
// described by items[b] (its diagonal chunk of L and where its inverse goes
// in that matrix's workspace, leading dimension ldw).
struct InvItem {
    const double *A;
    int64_t lda;
    double *W;
    int32_t ldw, mb;
};

template <bool CX, int NCH, bool UNIT>
__global__ __launch_bounds__(64) void hsma_diag_inv_group(const InvItem *__restrict__ items) {
    const InvItem d = items[blockIdx.x];
    Panel<CX, 8 * NCH, UNIT>::template solve<true>(d.A, d.lda, d.W, d.ldw, d.mb, d.mb,
                                                    cplx{1.0, 0.0});
}

}  // namespace smallk
}  // namespace hsma
