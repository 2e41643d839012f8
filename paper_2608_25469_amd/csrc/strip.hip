// Small-regime TRSM (m <= 64) on 16-column strips.
//
// Paper, Sec. 4.2.1: the columns of B are independent forward substitutions
// that share the triangular operand, so each lane keeps one column in
// registers and the row-dependency chain runs inside the lane.  Here the unit
// of work is a strip of at most 16 columns, and each 16-lane row of a
// wavefront (one DPP row) solves its own strip: lane l works on column l%16
// of strip l/16.  A wavefront therefore solves four strips at once -- of one
// problem (a 64-column panel) or of up to four different problems that share
// m -- so a problem with n = 20 occupies two DPP rows rather than a whole
// wavefront, and the lanes that a one-problem-per-wavefront layout leaves idle
// (a third of them for n ~ U{8..64}) carry other problems' columns.
//
// The walk is left-looking over 16-row blocks.  In block R lane l holds rows
// 16R..16R+15 of its column (y), and l_{16R + l%16, k} for the columns k it
// is applying: the 64-bit DPP row_newbcast:i of that coefficient register
// hands row i's coefficient to the 16 lanes of the DPP row, inside the
// multiply-add itself (v_fmac_f64_dpp, dpp_fma.h).  Every DPP row broadcasts
// within itself, so the four strips of a wavefront never mix, and each reads
// its own problem's L.  Block R first receives the updates -l_ik x_k of the
// finished blocks (k < 16R; x_k read back from B, where this wavefront stored
// it), then solves its own 16 x 16 triangle, then is stored.  Every element
// receives its updates in ascending k, as in the column-oriented definition.
//
// B never moves one lane-column at a time: a load in which each lane reads
// its own column touches as many cache lines as there are lanes.  Instead B
// passes through an LDS stage of one 16-row block of the wavefront's 64
// columns (17 KB complex, 8.5 KB real): the global loads and stores move
// whole 16-row column segments (16 lanes per segment, four columns per
// instruction), and the transposition to one-column-per-lane happens in LDS,
// where an odd column stride keeps the column-wise accesses free of bank
// conflicts.  The first 16 rows of a block (y),
// the finished rows (x, staged while the previous stage is being applied)
// and the solved block (stored) all take this path.  L's coefficients are
// read straight into registers: a ring of D coefficient registers is filled
// D column steps ahead, so those loads are in flight while earlier steps
// compute.  Rows and columns are clamped into the problem (reads stay inside
// A and B); rows >= m of the last block hold values that only ever feed rows
// >= m, which are never stored.

#include <type_traits>

#include "small_kernels.h"

namespace hsma {
namespace strip {

using smallk::bcast16;
using smallk::fnma_rows;
using smallk::SmallItem;

constexpr int RB = 16;  // rows per block, lanes per DPP row

#ifndef HSMA_STRIP_LOOKAHEAD_CX
#define HSMA_STRIP_LOOKAHEAD_CX 4
#endif
#ifndef HSMA_STRIP_LOOKAHEAD_R
#define HSMA_STRIP_LOOKAHEAD_R 8
#endif

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <bool CX>
__device__ __forceinline__ void ld(const HSMA_GLOBAL double *p, double &r, double &i) {
    if (CX) {
        const dbl2u v = *reinterpret_cast<const HSMA_GLOBAL dbl2u *>(p);
        r = v.x;
        i = v.y;
    } else {
        r = *p;
        i = 0.0;
    }
}

// The four strips of a wavefront, as wavefront-uniform values (the strip of
// DPP row s: first column, leading dimension, columns owned).
struct Strips {
    const HSMA_GLOBAL double *B[4];
    int64_t ldb[4];
    int nc[4];
};

// NK: the last NK finished blocks also stay in LDS (a 16-row block of the
// 64 columns each, in a ring of NK slots), so the updates read them there
// instead of from B; older blocks are read back from B.  With NK = 3 no row
// is ever read back (m <= 64 has at most four blocks).  For one problem's
// call, where a few wavefronts cover the GPU and LDS capacity costs nothing,
// NK = 3 takes the reads of B off the critical path.  In a batch each kept
// block costs occupancy (LDS per wavefront) but saves re-reads that mostly
// miss L2 by the time they come: the launcher picks NK per data type.
template <bool CX, bool UNIT, int NK>
struct Strip {
    static constexpr int ES = CX ? 2 : 1;
    // Column steps between a coefficient load and its use: one complex step
    // is 64 multiply-adds, one real step 16.  (Compile-time tunables.)
    static constexpr int D = CX ? HSMA_STRIP_LOOKAHEAD_CX : HSMA_STRIP_LOOKAHEAD_R;
    // B moves through LDS one 16-row block at a time (256 bytes of a complex
    // column, 128 of a real one).  A lane moves one element, so LPS lanes
    // cover a column's segment and one staging instruction moves CPI
    // columns; NQ instructions move the wavefront's 64 columns.  (Two real
    // rows per lane halve the real instructions but measured slower: with
    // odd leading dimensions half of those 16-byte accesses straddle.)
    static constexpr int RPC = 1;  // rows per lane and instruction
    static constexpr int LPS = RB / RPC;
    static constexpr int CPI = 64 / LPS;
    static constexpr int NQ = 64 / CPI;
    static_assert(RB % D == 0, "the look-ahead must divide a block");
    typedef typename std::conditional<CX, dbl2u, double>::type E;  // one element of B

    // LDS slot of (column C of the wavefront, row k of the block): column C
    // owns RB consecutive slots and one of padding, so that lanes reading
    // one row of consecutive columns hit distinct banks (the column stride is
    // an odd number of elements), while a staging instruction writes nearly
    // contiguous runs.  Row k is an immediate offset from the column's base.
    static constexpr int CS = RB + 1;
    static __device__ __forceinline__ int slot(int C, int k) { return C * CS + k; }

    // The lane id passed through an empty asm: address arithmetic derived
    // from it is redone where it is used instead of being hoisted and kept
    // live in registers for the whole kernel.
    static __device__ __forceinline__ int fresh(int lane) {
        asm volatile("" : "+v"(lane));
        return lane;
    }

    // Element of staging instruction Q for rows r0..: this lane's column is
    // (Q * CPI) % 16 + lane / LPS of strip Q * CPI / 16 (the same strip for
    // the whole instruction), its first row r0 + RPC (lane % LPS).  Columns
    // the strip does not own read its column 0; rows are kept below m.
    template <int Q>
    static __device__ __forceinline__ E load_chunk(const Strips &S, int lane, int r0, int m) {
        constexpr int st = Q * CPI / 16;
        int c = (Q * CPI) % 16 + lane / LPS;
        c = c < S.nc[st] ? c : 0;
        const int row = r0 + RPC * (lane % LPS);
        const HSMA_GLOBAL double *col = S.B[st] + ES * (int64_t)c * S.ldb[st];
        return *reinterpret_cast<const HSMA_GLOBAL E *>(col + ES * (row < m ? row : m - 1));
    }
    // The same element back to B (owned columns, rows below m).
    template <int Q>
    static __device__ __forceinline__ void store_chunk(const Strips &S, int lane, int r0, int m, E v) {
        constexpr int st = Q * CPI / 16;
        const int c = (Q * CPI) % 16 + lane / LPS;
        const int row = r0 + RPC * (lane % LPS);
        if (c >= S.nc[st] || row >= m) return;
        HSMA_GLOBAL double *col = (HSMA_GLOBAL double *)S.B[st] + ES * (int64_t)c * S.ldb[st];
        *reinterpret_cast<HSMA_GLOBAL E *>(col + ES * row) = v;
    }
    // A block's NQ elements per lane (instruction order), rows r0..r0+RB-1.
    static __device__ __forceinline__ void load_block(const Strips &S, int lane, int r0, int m, E (&ch)[NQ]) {
        const int ln = fresh(lane);
        static_for<0, NQ>([&](auto Q) {
            constexpr int q = decltype(Q)::value;
            ch[q] = load_chunk<q>(S, ln, r0, m);
        });
    }
    // Instruction-ordered elements -> LDS; LDS -> this lane's own column.
    static __device__ __forceinline__ void put(E *lds, int lane, const E (&ch)[NQ]) {
        E *p = lds + slot(lane / LPS, RPC * (lane % LPS));
#pragma unroll
        for (int q = 0; q < NQ; ++q) p[q * CPI * CS] = ch[q];
    }
    static __device__ __forceinline__ E get(const E *lds, int lane, int k) { return lds[slot(lane, k)]; }

    static __device__ __forceinline__ void split(E v, double &r, double &i) {
        if constexpr (CX) {
            r = v.x;
            i = v.y;
        } else {
            r = v;
            i = 0.0;
        }
    }
    static __device__ __forceinline__ E join(double r, double i) {
        if constexpr (CX) return E{r, i};
        else return r;
    }

    // The last DP diagonal steps of a block take coefficients loaded at the
    // block's start: those steps are short (few rows left below K), so a
    // ring refilled D steps ahead would not cover the load latency there.
    // (All 16 for real data; the last 8 for complex, whose registers are
    // scarcer and whose steps are four times longer.)
    static constexpr int DP = CX ? 8 : 16;
    static constexpr int DR = RB - DP;  // diagonal steps served by the ring

    // Diagonal step KK of block R (K = K0 + KK): x_K = y_K / l_KK, then the
    // rows below K in the block receive -l_iK x_K.  Column K's coefficients
    // are in ring slot KK % D (refilled with column K + D's before the
    // arithmetic, while that column is still a ring step) or, for the last
    // DP steps, in the preloaded pr/pi.  Steps nest, so that the rows leave
    // through a single join once K reaches m.
    template <int KK>
    static __device__ __forceinline__ void diag(const HSMA_GLOBAL double *arow, int64_t ldaE, int K0,
                                                int m, double rr, double ri, double (&yr)[RB],
                                                double (&yi)[RB], double (&cr)[D], double (&ci)[D],
                                                const double (&pr)[DP], const double (&pi)[DP]) {
        if constexpr (KK < RB) {
            if (K0 + KK < m) {
                double lr, li;
                if constexpr (KK < DR) {
                    lr = cr[KK % D];
                    li = ci[KK % D];
                    if constexpr (KK + D < DR) {
                        const int kn = K0 + KK + D < m ? K0 + KK + D : m - 1;
                        ld<CX>(arow + kn * ldaE, cr[KK % D], ci[KK % D]);
                    }
                } else {
                    lr = pr[KK - DR];
                    li = pi[KK - DR];
                }
                if (!UNIT) {
                    const double dr = bcast16<KK>(rr);
                    if (CX) {
                        const double di = bcast16<KK>(ri);
                        smallk::cmul_rn(yr[KK], yi[KK], dr, di, yr[KK], yi[KK]);
                    } else {
                        yr[KK] = __dmul_rn(yr[KK], dr);
                    }
                }
                if constexpr (KK + 1 < RB) fnma_rows<CX, KK + 1>(yr, yi, lr, li, yr[KK], yi[KK]);
                diag<KK + 1>(arow, ldaE, K0, m, rr, ri, yr, yi, cr, ci, pr, pi);
            }
        }
    }

    // One strip per DPP row; m is the same for the whole wavefront.  `it` is
    // this lane's strip, S all four.
    static __device__ __forceinline__ void solve(const SmallItem &it, const Strips &S, int m, int lane) {
        __shared__ E lds[64 * CS];
        __shared__ E kept[NK > 0 ? NK * 64 * CS : 1];
        const int c = lane & 15;
        const HSMA_GLOBAL double *A = (const HSMA_GLOBAL double *)it.A;
        const int64_t ldaE = ES * it.lda;
        const bool scale = it.ar != 1.0 || it.ai != 0.0;
        const int nb = (m + RB - 1) / RB;
        for (int R = 0; R < nb; ++R) {
            const int K0 = R * RB;
            // This lane's row of L in the block, clamped into the matrix.
            const int row = K0 + c < m ? K0 + c : m - 1;
            const HSMA_GLOBAL double *arow = A + ES * row;

            // Loads in flight first: the block's rows of B, this lane's
            // diagonal entry, the first stage of finished rows, and the
            // first D coefficient columns (update steps, or diagonal steps
            // when no block is finished).
            E ych[NQ];
            load_block(S, lane, K0, m, ych);
            double dx = 1.0, dy = 0.0;
            if (!UNIT) ld<CX>(arow + row * ldaE, dx, dy);
            double pr[DP], pi[DP];
#pragma unroll
            for (int k = 0; k < DP; ++k) {
                const int kn = K0 + DR + k < m ? K0 + DR + k : m - 1;
                ld<CX>(arow + kn * ldaE, pr[k], pi[k]);
            }
            E xin[NQ];
            // finished blocks t < R - NK come back from B, t = 0 first
            // (none with NK >= 3: m <= 64 has at most four blocks)
            const int nread = (NK >= 3 || R <= NK) ? 0 : R - NK;
            if (nread > 0) load_block(S, lane, 0, m, xin);
            double cr[D], ci[D];
            const HSMA_GLOBAL double *cp = arow;  // coefficient column of the next update step
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int kn = j < m ? j : m - 1;
                ld<CX>(R > 0 ? cp : arow + kn * ldaE, cr[j], ci[j]);
                cp += ldaE;
            }

            // Transpose the block's rows into this lane's column.
            double yr[RB], yi[RB];
            put(lds, lane, ych);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < RB; ++k) split(get(lds, lane, k), yr[k], yi[k]);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                if (K0 + i >= m) yr[i] = yi[i] = 0.0;
                if (scale) {
                    if (CX) {
                        smallk::cmul_rn(it.ar, it.ai, yr[i], yi[i], yr[i], yi[i]);
                    } else {
                        yr[i] = __dmul_rn(yr[i], it.ar);
                    }
                }
            }

            // Updates from the finished blocks, k ascending: a finished block
            // goes through LDS, the next one's loads are issued, then its RB
            // column steps run.
            for (int t = 0; t < R; ++t) {
                const bool more = t + 1 < R;
                const E *xs = lds;
                if (t >= nread) {
                    xs = kept + (t % (NK > 0 ? NK : 1)) * 64 * CS;
                } else {
                    put(lds, lane, xin);
                    __builtin_amdgcn_wave_barrier();
                    if (t + 1 < nread) load_block(S, lane, (t + 1) * RB, m, xin);
                }
                E xq[2] = {get(xs, lane, 0), get(xs, lane, 1)};
                static_for<0, RB>([&](auto J) {
                    constexpr int j = decltype(J)::value;
                    constexpr int s = j % D;
                    const double lr = cr[s], li = ci[s];
                    double vr, vi;
                    split(xq[j % 2], vr, vi);
                    if constexpr (j + 2 < RB) xq[j % 2] = get(xs, lane, j + 2);
                    // refill the slot with step j + D (this block or the
                    // next), or with the first diagonal steps; the load is
                    // issued either way, from a selected address (a branch
                    // would make the compiler keep the ring in scratch)
                    if constexpr (j + D < RB) {
                        ld<CX>(cp, cr[s], ci[s]);
                    } else {
                        const int kn = K0 + j + D - RB < m ? K0 + j + D - RB : m - 1;
                        ld<CX>(more ? cp : arow + kn * ldaE, cr[s], ci[s]);
                    }
                    cp += ldaE;
                    fnma_rows<CX, 0>(yr, yi, lr, li, vr, vi);
                });
                __builtin_amdgcn_wave_barrier();
            }

            // Reciprocal of this lane's diagonal entry: 1/d or conj(d)/|d|^2.
            double rr = 1.0, ri = 0.0;
            if (!UNIT) smallk::recip_rn(CX, dx, dy, rr, ri);
            diag<0>(arow, ldaE, K0, m, rr, ri, yr, yi, cr, ci, pr, pi);

            // Back to B through LDS, whole column segments per instruction
            // (through the block's kept slot when a later block will read it).
            E *out = lds;
            if constexpr (NK > 0) out = R + 1 < nb ? kept + (R % NK) * 64 * CS : lds;
#pragma unroll
            for (int k = 0; k < RB; ++k) out[slot(lane, k)] = join(yr[k], yi[k]);
            __builtin_amdgcn_wave_barrier();
            {
                const int ln = fresh(lane);
                const E *p = out + slot(ln / LPS, RPC * (ln % LPS));
                static_for<0, NQ>([&](auto Q) {
                    constexpr int q = decltype(Q)::value;
                    store_chunk<q>(S, ln, K0, m, p[q * CPI * CS]);
                });
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
};

// Workgroup b (one wavefront) solves strips 4b .. 4b + 3.  With rows ==
// nullptr they are strips of `one` (ncols holds its n); otherwise rows[4b + r]
// describes DPP row r's strip: B at the strip's first column, ncols <= 16,
// the same m in all four, and unused rows padded with a copy of a used one
// whose ncols is 0.  A wavefront's strips either all have alpha = 0 (B <- 0,
// neither A nor B read) or none has; a single problem never has alpha = 0
// here (that call is a plain zero fill).
template <bool CX, bool UNIT, int NK>
__global__ __launch_bounds__(64) void hsma_strip_solve(SmallItem one, const SmallItem *__restrict__ rows) {
    // The lane id passes through an empty asm so that the compiler does not
    // derive every unrolled address from it up front.
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int r = lane >> 4;
    constexpr int ES = CX ? 2 : 1;
    SmallItem it;
    int m;
    if (rows) {
        it = rows[(int64_t)blockIdx.x * 4 + r];
        m = __builtin_amdgcn_readfirstlane(it.m);
        if (__builtin_amdgcn_readfirstlane(it.ar == 0.0 && it.ai == 0.0 ? 1 : 0)) {
            const int c = lane & 15;
            if (c < it.ncols) {
                HSMA_GLOBAL double *bc = (HSMA_GLOBAL double *)it.B + ES * (int64_t)c * it.ldb;
                for (int i = 0; i < ES * m; ++i) bc[i] = 0.0;
            }
            return;
        }
    } else {
        const int64_t nstrip = ((int64_t)one.ncols + RB - 1) / RB;
        const int64_t s = (int64_t)blockIdx.x * 4 + r;
        const int64_t sc = s < nstrip ? s : nstrip - 1;
        it = one;
        it.B = one.B + ES * RB * sc * one.ldb;
        const int64_t left = (int64_t)one.ncols - RB * s;
        it.ncols = s < nstrip ? (int)(left < RB ? left : RB) : 0;
        m = one.m;
    }
    Strips S;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t b = (uint64_t)it.B;
        const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 16 * q);
        const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 16 * q);
        S.B[q] = (const HSMA_GLOBAL double *)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        const int llo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)it.ldb, 16 * q);
        const int lhi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)it.ldb >> 32), 16 * q);
        S.ldb[q] = (int64_t)(((uint64_t)(uint32_t)lhi << 32) | (uint32_t)llo);
        S.nc[q] = __builtin_amdgcn_readlane(it.ncols, 16 * q);
    }
    Strip<CX, UNIT, NK>::solve(it, S, m, lane);
}

// Finished blocks a batch keeps in LDS per wavefront (compile-time
// tunables).  Real data keeps two (8.5 KB each beside the 8.5 KB stage: six
// wavefronts per CU); complex keeps none, as any kept block (17 KB) would
// halve the eight wavefronts per CU that its registers allow.
#ifndef HSMA_STRIP_BATCH_KEEP_CX
#define HSMA_STRIP_BATCH_KEEP_CX 0
#endif
#ifndef HSMA_STRIP_BATCH_KEEP_R
#define HSMA_STRIP_BATCH_KEEP_R 2
#endif

template <bool CX, bool UNIT>
void launch_t(unsigned waves, const SmallItem &one, const SmallItem *rows, hipStream_t s) {
    constexpr int NKB = CX ? HSMA_STRIP_BATCH_KEEP_CX : HSMA_STRIP_BATCH_KEEP_R;
    if (rows) hipLaunchKernelGGL((hsma_strip_solve<CX, UNIT, NKB>), dim3(waves), dim3(64), 0, s, one, rows);
    else hipLaunchKernelGGL((hsma_strip_solve<CX, UNIT, 3>), dim3(waves), dim3(64), 0, s, one, rows);
}

void launch(bool cx, bool unit, unsigned waves, const SmallItem &one, const SmallItem *rows,
            hipStream_t s) {
    if (cx) {
        if (unit) launch_t<true, true>(waves, one, rows, s);
        else launch_t<true, false>(waves, one, rows, s);
    } else {
        if (unit) launch_t<false, true>(waves, one, rows, s);
        else launch_t<false, false>(waves, one, rows, s);
    }
}

}  // namespace strip

// One problem, 1 <= m <= 64, alpha != 0: ceil(n / 16) strips, four per
// wavefront.
hsma_status launch_strip_one(bool cx, bool unit, int m, int64_t n, cplx alpha, const double *A,
                             int64_t lda, double *B, int64_t ldb, hipStream_t s) {
    if (m < 1 || m > 64 || n < 1 || n > 0x7fffffff) return HSMA_INVALID_SIZE;
    const int64_t waves = (n + 63) / 64;
    smallk::SmallItem one{A, B, lda, ldb, m, (int32_t)n, alpha.re, alpha.im};
    strip::launch(cx, unit, (unsigned)waves, one, nullptr, s);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

// Grouped launch: `rows` (device memory) holds 4 * waves strip descriptors.
hsma_status launch_strip_group(bool cx, bool unit, const void *rows, int waves, hipStream_t s) {
    if (waves < 1) return HSMA_INVALID_SIZE;
    smallk::SmallItem one{};
    strip::launch(cx, unit, (unsigned)waves, one, static_cast<const smallk::SmallItem *>(rows), s);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

size_t strip_item_bytes() { return sizeof(smallk::SmallItem); }

}  // namespace hsma
