// Small-regime TRSM (m <= 64): register-resident forward substitution.
//
// Paper, Sec. 4.2.1: columns of B are independent, so each column is a
// separate forward substitution; the triangular operand is shared.  Here one
// 64-lane wavefront owns a panel of up to 64 columns: lane j keeps column j
// of the panel entirely in VGPRs (y[0..m-1]), so the row-dependency chain runs
// inside a lane with no synchronisation at all.
//
// L is the same for every lane.  Its packed lower triangle is staged once in
// LDS with direct global-to-LDS loads (no VGPR round trip).  At step k,
// column k+1 is read from LDS into ceil(m/16) VGPRs laid out so that each
// 16-lane row of the wavefront holds 16 consecutive rows of the column, and
// each coefficient reaches all lanes through the 64-bit DPP row_newbcast
// broadcast with no further memory traffic.  In the left-looking walk the
// broadcast is the DPP source operand of the multiply-add itself
// (v_fmac_f64_dpp, dpp_fma.h), so a real update costs one VALU instruction
// and a complex one four.  The column for the next step is read before the
// current step's arithmetic, so LDS latency hides behind the dependency
// chain.
//
// The loop nest is fully unrolled for a compile-time row bound MAXM (a
// multiple of 8) and guarded by the runtime m.  Two walks share this
// machinery: Panel (right-looking, the whole column live; used with identity
// right-hand sides to invert diagonal chunks) and PanelLL (left-looking over
// 16-row blocks, used for general right-hand sides: a lane holds one block
// at a time, so register use no longer grows with m and larger panels keep
// two or more wavefronts per SIMD).  Loads of a block are issued before its
// arithmetic and its rows are stored as soon as they are final, so global
// traffic overlaps the chain (the load/compute/store overlap of Sec. 4.2.1,
// Alg. 1, obtained by full unrolling and the hardware's in-order waits).
//
// Reciprocals of the diagonal are computed one per lane and broadcast to the
// whole wave with v_readlane when row k is divided: once per wavefront in the
// right-looking walk, per 16-row block from the staged panel in the
// left-looking one (so no separate load of the diagonal precedes the first
// block).

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
                        const double tr = yr[K] * dr - yi[K] * di;
                        const double ti = yr[K] * di + yi[K] * dr;
                        yr[K] = tr;
                        yi[K] = ti;
                    } else {
                        yr[K] *= dr;
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
            if (CX) {
                const double vx = d[0], vy = d[1];
                const double den = vx * vx + vy * vy;
                rr = vx / den;
                ri = -vy / den;
            } else {
                rr = 1.0 / d[0];
            }
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
                    const double tr = alpha.re * yr[i] - alpha.im * yi[i];
                    const double ti = alpha.re * yi[i] + alpha.im * yr[i];
                    yr[i] = tr;
                    yi[i] = ti;
                } else {
                    yr[i] *= alpha.re;
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

// ---------------------------------------------------------------------------
// The same solve walked left-looking over 16-row blocks (used for general
// right-hand sides; the identity right-hand sides of the diagonal-block
// inversion keep the right-looking Panel above).
//
// Holding a whole column in registers costs 2 m doubles per lane -- for
// complex m = 64 all 256 architectural VGPRs, so the compiler spills the
// working set to AGPRs and only one wavefront fits per SIMD.  Here a lane
// holds one 16-row block of its column (y) plus one finished block (x):
// block R is loaded, receives the updates of every finished block K < R
// (whose final values the same lane stored to B earlier and reloads), solves
// its own 16 x 16 triangle, and is stored.  Every element still receives its
// updates -l_ik x_k in ascending k, exactly as in the right-looking order, so
// the results are the same bit for bit.
// ---------------------------------------------------------------------------
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <bool CX, int MAXM, bool UNIT>
struct PanelLL {
    static constexpr int RB = 16;
    static constexpr int NB = (MAXM + RB - 1) / RB;
    static constexpr int ES = CX ? 2 : 1;
    // LDS: the 16-row panel of L that block R needs (rows R*16.., columns
    // 0..R*16+15), column-major with 16 rows per column.
    static constexpr int PANEL = RB * MAXM;

    // Coefficients l_{R*16 + l%16, k} of column k for the current panel.
    static __device__ __forceinline__ void coef(const double *Lp, int lane, int k, double &cr,
                                                double &ci) {
        const int e = k * RB + (lane & 15);
        if (CX) {
            cr = Lp[2 * e];
            ci = Lp[2 * e + 1];
        } else {
            cr = Lp[e];
            ci = 0.0;
        }
    }

    // Stage rows R*16..R*16+15 of columns 0..(R+1)*16-1 (at most MAXM) with
    // direct global-to-LDS loads.  Complex: one instruction moves 4 columns
    // (lane l: column 4c + l/16, row l%16, 16 bytes); real: 2 columns (lane
    // l: column 2c + l/32, row (l%32)/2, 4-byte half l%2).  Source rows are
    // clamped to [column, m-1] and columns to m-1, so only the lower triangle
    // of A is read and nothing outside it; rows and columns beyond m only feed
    // rows that are never stored, and rows on or above the diagonal are never
    // used.
    template <int R>
    static __device__ __forceinline__ void stage(const double *__restrict__ A, int64_t lda, int m,
                                                 int lane, double *Lp) {
        typedef __attribute__((address_space(3))) void lds_void;
        constexpr int NCOL = ((R + 1) * RB) < MAXM ? ((R + 1) * RB) : MAXM;
        const int mc = m - 1;
        if (CX) {
#pragma unroll
            for (int c = 0; c < NCOL / 4; ++c) {
                int col = 4 * c + (lane >> 4);
                col = col < mc ? col : mc;
                int row = R * RB + (lane & 15);
                row = row < col ? col : (row < mc ? row : mc);
                const double *src = A + 2 * ((int64_t)col * lda + row);
                __builtin_amdgcn_global_load_lds((const void *)src, (lds_void *)(Lp + 2 * (c * 64)), 16, 0,
                                                 0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < NCOL / 2; ++c) {
                int col = 2 * c + (lane >> 5);
                col = col < mc ? col : mc;
                int row = R * RB + ((lane & 31) >> 1);
                row = row < col ? col : (row < mc ? row : mc);
                const char *src = reinterpret_cast<const char *>(A + (int64_t)col * lda + row) + 4 * (lane & 1);
                __builtin_amdgcn_global_load_lds((const void *)src, (lds_void *)(Lp + c * 32), 4, 0, 0);
            }
        }
    }

    // A finished block goes back to B through LDS so that each store
    // instruction writes four whole 16-row column segments (four 256-byte
    // runs for complex, 128-byte runs for real) instead of one element of 64
    // different columns.  Chunk c of LDS holds columns 4c..4c+3, the element
    // (column 4c + r, row i) in slot 16 (r ^ f) + (i + r + 4 (c % 4)) % 16
    // with f = (c / 4) % 2: the lanes of a quarter (complex) or half (real)
    // wavefront then hit distinct LDS banks when they write their rows, and
    // every read of a chunk is contiguous.
    static constexpr bool COALESCED_STORE = (MAXM == 64);

    template <int R>
    static __device__ __forceinline__ void store_block(double *Lp, HSMA_GLOBAL double *__restrict__ Bp,
                                                       int64_t ldb, int ncols, int m, int lane,
                                                       const double (&yr)[RB], const double (&yi)[RB]) {
        __syncthreads();  // the panel's reads are complete
        {
            const int c = lane >> 2, r = lane & 3, q = c & 3, f = (c >> 2) & 1;
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                double *p = Lp + ES * (c * 64 + 16 * (r ^ f) + ((i + r + 4 * q) & 15));
                if (CX) {
                    p[0] = yr[i];
                    p[1] = yi[i];
                } else {
                    p[0] = yr[i];
                }
            }
        }
        __syncthreads();  // the block is in LDS
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int f = (c >> 2) & 1, q = c & 3;
            const int r = (lane >> 4) ^ f;
            const int i = ((lane & 15) - r - 4 * q) & 15;
            const int col = 4 * c + r;
            const double *p = Lp + ES * (c * 64 + lane);
            if (col < ncols && R * RB + i < m) {
                HSMA_GLOBAL double *dst = Bp + ES * ((int64_t)col * ldb + R * RB + i);
                if (CX)
                    *reinterpret_cast<HSMA_GLOBAL dbl2u *>(dst) = dbl2u{p[0], p[1]};
                else
                    dst[0] = p[0];
            }
        }
    }

    // Diagonal step KK of block R: x = y[KK] / l_KK, then rows KK+1.. of the
    // block receive -l_iK x.  c holds column K's coefficients (read one step
    // earlier); the next column's are read first.  Steps nest so that the
    // block's row values never pass through a join per step.
    template <int R, int BR, int KK>
    static __device__ __forceinline__ void diag_step(const double *Lp, int m, int lane, double rr,
                                                     double ri, double (&yr)[RB], double (&yi)[RB],
                                                     double cr, double ci) {
        if constexpr (KK < BR) {
            constexpr int K = R * RB + KK;
            if (K < m) {
                double nr = 0.0, ni = 0.0;
                if constexpr (KK + 1 < BR) coef(Lp, lane, K + 1, nr, ni);
                if (!UNIT) {
                    const double dr = readlane_d(rr, KK);
                    if (CX) {
                        const double di = readlane_d(ri, KK);
                        const double tr = yr[KK] * dr - yi[KK] * di;
                        const double ti = yr[KK] * di + yi[KK] * dr;
                        yr[KK] = tr;
                        yi[KK] = ti;
                    } else {
                        yr[KK] *= dr;
                    }
                }
                const double xr = yr[KK], xi = yi[KK];
                if constexpr (BR == RB) {
                    if constexpr (KK + 1 < RB) fnma_rows<CX, KK + 1>(yr, yi, cr, ci, xr, xi);
                } else {
                    static_for<KK + 1, BR>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        const double lr = bcast16<i & 15>(cr);
                        const double li = CX ? bcast16<i & 15>(ci) : 0.0;
                        fms<CX>(yr[i], yi[i], lr, li, xr, xi);
                    });
                }
                diag_step<R, BR, KK + 1>(Lp, m, lane, rr, ri, yr, yi, nr, ni);
            }
        }
    }

    // Block R: stage its panel of L, load, apply finished blocks, solve the
    // diagonal triangle, store.
    template <int R>
    static __device__ __forceinline__ void block(const double *__restrict__ A, int64_t lda,
                                                 double *Lp, HSMA_GLOBAL double *__restrict__ bc, bool active,
                                                 HSMA_GLOBAL double *__restrict__ Bp, int64_t ldb, int ncols,
                                                 int m, int lane, cplx alpha) {
        if constexpr (R < NB) {
            constexpr int BR = (MAXM - R * RB) < RB ? (MAXM - R * RB) : RB;  // rows of this block
            if (R * RB < m) {
                __syncthreads();  // the previous panel's reads are complete
                stage<R>(A, lda, m, lane, Lp);
                double yr[RB], yi[RB];
#pragma unroll
                for (int i = 0; i < BR; ++i) {
                    const int g = R * RB + i;
                    const int gc = g < m ? g : m - 1;
                    if (CX) {
                        const dbl2u v = reinterpret_cast<const HSMA_GLOBAL dbl2u *>(bc)[gc];
                        yr[i] = v.x;
                        yi[i] = v.y;
                    } else {
                        yr[i] = bc[gc];
                        yi[i] = 0.0;
                    }
                    if (g >= m) yr[i] = yi[i] = 0.0;
                }
                if (alpha.re != 1.0 || alpha.im != 0.0) {
#pragma unroll
                    for (int i = 0; i < BR; ++i) {
                        if (CX) {
                            const double tr = alpha.re * yr[i] - alpha.im * yi[i];
                            const double ti = alpha.re * yi[i] + alpha.im * yr[i];
                            yr[i] = tr;
                            yi[i] = ti;
                        } else {
                            yr[i] *= alpha.re;
                        }
                    }
                }
                __syncthreads();  // the panel has landed in LDS
                // Updates from the finished blocks, in ascending column order.
                static_for<0, R>([&](auto KB) {
                    constexpr int Kb = decltype(KB)::value;
                    double xr[RB], xi[RB];
#pragma unroll
                    for (int k = 0; k < RB; ++k) {
                        if (CX) {
                            const dbl2u v = reinterpret_cast<const HSMA_GLOBAL dbl2u *>(bc)[Kb * RB + k];
                            xr[k] = v.x;
                            xi[k] = v.y;
                        } else {
                            xr[k] = bc[Kb * RB + k];
                            xi[k] = 0.0;
                        }
                    }
                    double cr, ci;
                    coef(Lp, lane, Kb * RB, cr, ci);
                    static_for<0, RB>([&](auto KK) {
                        constexpr int kk = decltype(KK)::value;
                        double nr = 0.0, ni = 0.0;
                        if constexpr (kk + 1 < RB) coef(Lp, lane, Kb * RB + kk + 1, nr, ni);
                        if constexpr (BR == RB) {
                            fnma_rows<CX, 0>(yr, yi, cr, ci, xr[kk], xi[kk]);
                        } else {
                            static_for<0, BR>([&](auto I) {
                                constexpr int i = decltype(I)::value;
                                const double lr = bcast16<i & 15>(cr);
                                const double li = CX ? bcast16<i & 15>(ci) : 0.0;
                                fms<CX>(yr[i], yi[i], lr, li, xr[kk], xi[kk]);
                            });
                        }
                        cr = nr;
                        ci = ni;
                    });
                });
                // Reciprocals of this block's diagonal, from the staged panel:
                // lane l holds row R*16 + l%16 (1/d, or conj(d)/|d|^2).
                double rr = 1.0, ri = 0.0;
                if (!UNIT && (lane & 15) < BR) {
                    double vx, vy;
                    coef(Lp, lane, R * RB + (lane & 15), vx, vy);
                    if (CX) {
                        const double den = vx * vx + vy * vy;
                        rr = vx / den;
                        ri = -vy / den;
                    } else {
                        rr = 1.0 / vx;
                    }
                }
                double cr, ci;
                coef(Lp, lane, R * RB, cr, ci);
                diag_step<R, BR, 0>(Lp, m, lane, rr, ri, yr, yi, cr, ci);
                if constexpr (COALESCED_STORE && BR == RB) {
                    store_block<R>(Lp, Bp, ldb, ncols, m, lane, yr, yi);
                } else if (active) {
#pragma unroll
                    for (int i = 0; i < BR; ++i) {
                        if (R * RB + i < m) {
                            if (CX)
                                reinterpret_cast<HSMA_GLOBAL dbl2u *>(bc)[R * RB + i] = dbl2u{yr[i], yi[i]};
                            else
                                bc[R * RB + i] = yr[i];
                        }
                    }
                }
                block<R + 1>(A, lda, Lp, bc, active, Bp, ldb, ncols, m, lane, alpha);
            }
        }
    }

    static __device__ __forceinline__ void solve(const double *__restrict__ A, int64_t lda,
                                                 double *__restrict__ B, int64_t ldb, int m,
                                                 int ncols, cplx alpha) {
        // Laundered lane id: see Panel::solve.
        int lane = threadIdx.x & 63;
        asm volatile("" : "+v"(lane));
        const bool active = lane < ncols;
        HSMA_GLOBAL double *__restrict__ bc = (HSMA_GLOBAL double *)(B + ES * (int64_t)(active ? lane : 0) * ldb);
        __shared__ double Lp[ES * (COALESCED_STORE && PANEL < RB * 64 ? RB * 64 : PANEL)];
        block<0>(A, lda, Lp, bc, active, (HSMA_GLOBAL double *)B, ldb, ncols, m, lane, alpha);
    }
};

// Work item of the small-solve kernel: one 64-column panel of one problem.
struct SmallItem {
    const double *A;
    double *B;        // first column of the panel
    int64_t lda, ldb; // element units
    int32_t m, ncols;
    double ar, ai;    // alpha
};

// Device-side descriptor table of a grouped launch: the items of one
// (dtype, unit) group, one workgroup each.
struct SmallGroup {
    const SmallItem *items;
    int32_t count;
};

// Single problem (items == nullptr): workgroup b solves panel b of `one`.
// Grouped (items != nullptr): workgroup b solves item b.  Items are sorted by
// decreasing cost on the host and the hardware starts workgroups in order as
// slots free up, so the longest panels start first with no work counter.  (A
// persistent grid claiming items through an atomic counter was 22 % slower:
// the claim is one more dependent round trip per item.)
// Complex panels of 49..64 rows fit two wavefronts per SIMD (256 registers
// each) with the left-looking walk; without the hint the compiler spreads
// into the whole register file for one.
template <bool CX, int NCH>
constexpr int small_waves() { return (CX && NCH >= 7) ? 2 : 1; }

template <bool CX, int NCH, bool UNIT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(small_waves<CX, NCH>())))
void hsma_small_solve(SmallItem one, SmallGroup grp) {
    const int lane = threadIdx.x & 63;
    SmallItem d;
    if (grp.items == nullptr) {
        const int64_t col0 = (int64_t)blockIdx.x * 64;
        d = one;
        d.B = one.B + (CX ? 2 : 1) * col0 * one.ldb;
        const int64_t left = (int64_t)one.ncols - col0;  // ncols holds n here
        d.ncols = (int)(left < 64 ? left : 64);
    } else {
        if ((int)blockIdx.x >= grp.count) return;
        d = grp.items[blockIdx.x];
    }
    if (d.ar == 0.0 && d.ai == 0.0) {
        // alpha = 0: B := 0, neither A nor B is read.
        if (lane < d.ncols) {
            HSMA_GLOBAL double *bc = (HSMA_GLOBAL double *)(d.B + (CX ? 2 : 1) * (int64_t)lane * d.ldb);
            for (int i = 0; i < (CX ? 2 : 1) * d.m; ++i) bc[i] = 0.0;
        }
        return;
    }
    PanelLL<CX, 8 * NCH, UNIT>::solve(d.A, d.lda, d.B, d.ldb, d.m, d.ncols, cplx{d.ar, d.ai});
}

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
