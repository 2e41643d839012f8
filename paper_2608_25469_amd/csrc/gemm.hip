// FP64 matrix-core product for the blocked TRSM path.
//
// Paper, Sec. 4.3: after the diagonal blocks are inverted, the large solve is
// a sequence of matrix products: the trailing update B_r <- B_r - A_{r,:} X
// and the diagonal solve X_r = inv(D_r) B_r.  On gfx950 these run on the FP64
// matrix cores (v_mfma_f64_16x16x4_f64).
//
//   C = beta * C + alpha * A * B        (column-major, real-view units)
//
// Tiling: a 256-thread workgroup (4 wavefronts) owns a BM x BN tile of C,
// each wavefront a (BM/WM) x (BN/WN) sub-tile held as 16x16 accumulator
// blocks.  K advances 16 at a time through a two-stage LDS ring: global loads
// for stage k+1 are issued before the matrix-core work on stage k and written
// to the other LDS buffer afterwards, one barrier per stage.
//
// MFMA operand layout (16x16x4, f64, as measured on gfx950): lane l holds
// A[l%16][k0 + l/16] and B[k0 + l/16][l%16]; result element v of lane l is
// row 4v + l/16 of column l%16.  The A fragment is fed with its 16 rows in
// the transposed 4x4 order (slot s carries row 4(s%4) + s/4), which makes
// element v of lane l row 4(l/16) + v: each lane ends up with 4 consecutive
// rows of one column, so complex (re, im) row pairs stay inside one lane.
// A is staged k-major (column-major tile) and B n-major (column-major tile),
// so both operand reads touch 16 consecutive doubles per 16-lane group.
//
// Complex data: a complex M x K matrix A is the real 2M x 2K matrix whose
// 2x2 blocks are [[re, -im], [im, re]].  Viewed as real, complex B and C are
// simply 2K x N and 2M x N with interleaved rows.  So a complex product is
// this real kernel with A expanded while it is staged into LDS: real column
// 2k of the expansion is complex column k as stored (re, im interleaved) and
// real column 2k+1 is (-im, re).  The flop count equals four real products.
//
// Workgroup -> tile mapping is XCD-aware: consecutive workgroup ids land on
// different XCDs, so ids are remapped to give each XCD a contiguous run of
// tiles, walked in groups of 8 tile-rows so neighbouring workgroups share A
// and B panels in that XCD's L2.

#include <algorithm>

#include "internal.h"
#include "tile_choice.h"

namespace hsma {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct __attribute__((aligned(8))) d2 {
    double x, y;
};

// 16-byte load of two doubles through a generic or a global pointer.
__device__ __forceinline__ d2 ld_pair(const double *p) { return *reinterpret_cast<const d2 *>(p); }
__device__ __forceinline__ d2 ld_pair(const HSMA_GLOBAL double *p) {
    const dbl2u t = *reinterpret_cast<const HSMA_GLOBAL dbl2u *>(p);
    return d2{t.x, t.y};
}

constexpr int BK = 16;

// Workgroups per CU that the tile's LDS ring allows (160 KB per CU, at most
// 3); the launch bound then caps registers so that many stay resident.
static_assert(BK == kTileBK, "one slice depth for the kernels and the shape choice");
__host__ __device__ constexpr int lds_bytes(int bm, int bn) { return tile_lds_bytes(bm, bn); }
__host__ __device__ constexpr int occ_for(int bm, int bn) { return tile_occupancy(bm, bn); }

#ifndef HSMA_UPD_MIN_WG_PER_CU
#define HSMA_UPD_MIN_WG_PER_CU 4
#endif

#ifndef HSMA_UPD_BM
#define HSMA_UPD_BM 128
#define HSMA_UPD_BN 128
#define HSMA_UPD_WM 2
#define HSMA_UPD_WN 2
#endif

// One BM x BN tile (tm, tn) of C = beta C + alpha A B; Ag, Bg, Cg are the
// operand bases of this product (after any batch offset).
// GD is double (pointers the compiler already knows to be global: kernel
// arguments) or HSMA_GLOBAL double (pointers read from a descriptor table).
template <bool CX, int BM, int BN, int WM, int WN, typename GD>
__device__ __forceinline__ void gemm_tile(const GemmParams &p, const GD *__restrict__ Ag,
                                          const GD *__restrict__ Bg, GD *__restrict__ Cg, int tm,
                                          int tn) {
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int LDA_S = BM + 4;    // LDS stride of the A tile (per k)
    constexpr int LDB_S = BK + 1;    // LDS stride of the B tile (per column)
    static_assert(WM * WN == 4, "four wavefronts");
    static_assert(TM % 16 == 0 && TN % 16 == 0, "16x16 blocks");

    __shared__ double As[2][BK * LDA_S];
    __shared__ double Bs[2][BN * LDB_S];

    const int m0 = tm * BM, n0 = tn * BN;
    const int M = p.M, N = p.N;
    // Lower-triangular C (c_lower): a tile whose first column lies right of
    // its last row (in elements: real-view rows / 2 for complex) is empty.
    if (p.c_lower && n0 > (CX ? (m0 + BM - 1) / 2 : m0 + BM - 1)) return;
    // A lower-triangular A (k_lower) has nothing right of column m0 + BM - 1
    // in this tile's rows.
    const int K = (p.k_lower && m0 + BM < p.K) ? m0 + BM : p.K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WM) * TM, wn0 = (wave / WM) * TN;

    // ---- staging registers ----
    // A: real: BM*BK/2 pairs (2 rows each); complex: BM*BK/4 complex elements.
    constexpr int A_TOTAL = CX ? (BM * BK / 4) : (BM * BK / 2);
    constexpr int B_TOTAL = BN * BK / 2;
    constexpr int A_ITEMS = (A_TOTAL + 255) / 256;
    constexpr int B_ITEMS = (B_TOTAL + 255) / 256;
    d2 ra[A_ITEMS], rb[B_ITEMS];

    auto load_a = [&](int k0) {
#pragma unroll
        for (int it = 0; it < A_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (A_TOTAL % 256 && e >= A_TOTAL) break;
            if (!CX) {
                // pair e: column kk = e / (BM/2), rows 2*(e % (BM/2)) .. +1
                const int kk = e / (BM / 2), ii = 2 * (e % (BM / 2));
                const int gr = m0 + ii, gk = (K > 0) ? 0 : 0;
                const int gc = k0 + kk;
                (void)gk;
                d2 v = {0.0, 0.0};
                if (gc < K) {
                    const GD *src = Ag + (int64_t)gc * p.lda + gr;
                    if (gr + 1 < M) {
                        v = ld_pair(src);
                    } else if (gr < M) {
                        v.x = src[0];
                    }
                    if (p.tri_a) {
                        if (gr < gc) v.x = 0.0;
                        if (gr + 1 < gc) v.y = 0.0;
                        if (p.tri_a == 2) {
                            if (gr == gc) v.x = 1.0;
                            if (gr + 1 == gc) v.y = 1.0;
                        }
                    }
                }
                ra[it] = v;
            } else {
                // complex element e: complex column kc = e / (BM/2), complex row ic
                const int kc = e / (BM / 2), ic = e % (BM / 2);
                const int gr = m0 / 2 + ic, gc = k0 / 2 + kc;
                d2 v = {0.0, 0.0};
                if (gc < K / 2 && gr < M / 2) {
                    v = ld_pair(Ag + 2 * ((int64_t)gc * p.lda + gr));
                    if (p.tri_a) {
                        if (gr < gc) v.x = v.y = 0.0;
                        if (p.tri_a == 2 && gr == gc) {
                            v.x = 1.0;
                            v.y = 0.0;
                        }
                    }
                }
                ra[it] = v;
            }
        }
    };
    auto store_a = [&](int buf) {
#pragma unroll
        for (int it = 0; it < A_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (A_TOTAL % 256 && e >= A_TOTAL) break;
            if (!CX) {
                const int kk = e / (BM / 2), ii = 2 * (e % (BM / 2));
                double *dst = &As[buf][kk * LDA_S + ii];
                dst[0] = ra[it].x;
                dst[1] = ra[it].y;
            } else {
                const int kc = e / (BM / 2), ic = e % (BM / 2);
                double *d0 = &As[buf][(2 * kc) * LDA_S + 2 * ic];
                double *d1 = &As[buf][(2 * kc + 1) * LDA_S + 2 * ic];
                d0[0] = ra[it].x;
                d0[1] = ra[it].y;
                d1[0] = -ra[it].y;
                d1[1] = ra[it].x;
            }
        }
    };
    auto load_b = [&](int k0) {
#pragma unroll
        for (int it = 0; it < B_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (B_TOTAL % 256 && e >= B_TOTAL) break;
            const int jj = e / (BK / 2), kk = 2 * (e % (BK / 2));
            const int gn = n0 + jj, gk = k0 + kk;
            d2 v = {0.0, 0.0};
            if (gn < N) {
                const GD *src = Bg + (int64_t)gn * p.ldb + gk;
                if (gk + 1 < K) {
                    v = ld_pair(src);
                } else if (gk < K) {
                    v.x = src[0];
                }
            }
            rb[it] = v;
        }
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int it = 0; it < B_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (B_TOTAL % 256 && e >= B_TOTAL) break;
            const int jj = e / (BK / 2), kk = 2 * (e % (BK / 2));
            double *dst = &Bs[buf][jj * LDB_S + kk];
            dst[0] = rb[it].x;
            dst[1] = rb[it].y;
        }
    };

    dbl4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    const int nk = (K + BK - 1) / BK;
    if (nk > 0) {
        load_a(0);
        load_b(0);
        store_a(0);
        store_b(0);
        __syncthreads();
    }
    const int lr = lane & 15, lk = lane >> 4;
    const int lr_a = 4 * (lr & 3) + (lr >> 2);  // A-fragment row slot order
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) {
            load_a((kt + 1) * BK);
            load_b((kt + 1) * BK);
        }
        const double *as = As[buf];
        const double *bs = Bs[buf];
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            const int k = 4 * s + lk;
            double fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) fa[i] = as[k * LDA_S + wm0 + 16 * i + lr_a];
#pragma unroll
            for (int j = 0; j < FN; ++j) fb[j] = bs[(wn0 + 16 * j + lr) * LDB_S + k];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) {
            store_a(buf ^ 1);
            store_b(buf ^ 1);
        }
        __syncthreads();
    }

    // ---- epilogue: C = beta*C + alpha*acc ----
    const bool beta_zero = (p.beta_re == 0.0 && p.beta_im == 0.0);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn0 + 16 * j + lr;
            const int row = m0 + wm0 + 16 * i + 4 * lk;
            if (col >= N) continue;
            GD *dst = Cg + (int64_t)col * p.ldc + row;
            double v[4] = {acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]};
            if (CX) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double ar = v[2 * h], ai = v[2 * h + 1];
                    double r = p.alpha_re * ar - p.alpha_im * ai;
                    double q = p.alpha_re * ai + p.alpha_im * ar;
                    if (row + 2 * h < M && !(p.c_lower && col > (row + 2 * h) / 2)) {
                        if (!beta_zero) {
                            const double cr = dst[2 * h], ci = dst[2 * h + 1];
                            r += p.beta_re * cr - p.beta_im * ci;
                            q += p.beta_re * ci + p.beta_im * cr;
                        }
                        dst[2 * h] = r;
                        dst[2 * h + 1] = q;
                    }
                }
            } else {
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    if (row + h < M && !(p.c_lower && col > row + h)) {
                        double r = p.alpha_re * v[h];
                        if (!beta_zero) r = __fma_rn(p.beta_re, dst[h], r);
                        dst[h] = r;
                    }
                }
            }
        }
    }
}

template <bool CX, int BM, int BN, int WM, int WN, int ROLE>
__global__ __launch_bounds__(256, (occ_for(BM, BN))) void hsma_gemm(const GemmParams p) {
    // Tile selection, XCD-aware: consecutive workgroup ids land on different
    // XCDs, so ids are remapped to give each XCD a contiguous run of tiles,
    // walked in groups of 8 tile-rows.
    const int T = p.tiles_m * p.tiles_n;
    const int bid = blockIdx.x;
    int tm, tn;
    if (p.k_lower || p.c_lower) {
        // A triangular operand (K bounded by the tile row) or a triangular C
        // (tiles above the diagonal skipped): a tile row's work grows with
        // its index, so contiguous runs of rows per XCD would leave the XCD
        // holding the bottom rows with about twice the average.  Bottom rows
        // come first instead, and consecutive workgroups (which the hardware
        // deals out to the XCDs in turn) walk a row, so every XCD gets an
        // eighth of every row.
        if (bid >= T) return;
        tm = p.tiles_m - 1 - bid / p.tiles_n;
        tn = bid % p.tiles_n;
    } else {
        const int nb = gridDim.x;  // multiple of 8
        const int per = nb / 8;
        const int t = (bid % 8) * per + bid / 8;
        if (t >= T) return;
        constexpr int GROUP = 8;
        const int gsz_full = GROUP * p.tiles_n;
        const int g = t / gsz_full;
        const int first = g * GROUP;
        const int gsize = (p.tiles_m - first) < GROUP ? (p.tiles_m - first) : GROUP;
        tm = first + (t % gsz_full) % gsize;
        tn = (t % gsz_full) / gsize;
    }
    const int batch = blockIdx.y;
    const int bo = batch / p.inner, bi = batch % p.inner;
    gemm_tile<CX, BM, BN, WM, WN>(p, p.A + bo * p.a_outer + bi * p.a_inner,
                                  p.B + bo * p.b_outer + bi * p.b_inner,
                                  p.C + bo * p.c_outer + bi * p.c_inner, tm, tn);
}

// Grouped launch: descriptor d owns tiles [d.tile0, d.tile0 + tiles_m
// tiles_n) of the grid; each workgroup finds its descriptor by binary search
// over the ascending tile0 values and computes one tile of that product.
template <bool CX, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256, (occ_for(BM, BN))) void hsma_gemm_grouped(
    const GemmParams *__restrict__ descs, int nd) {
    const int t = blockIdx.x;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    const GemmParams p = descs[lo];
    const int local = t - p.tile0;
    if (local < 0 || local >= p.tiles_m * p.tiles_n) return;
    gemm_tile<CX, BM, BN, WM, WN>(p, (const HSMA_GLOBAL double *)p.A, (const HSMA_GLOBAL double *)p.B,
                                  (HSMA_GLOBAL double *)p.C, local % p.tiles_m, local / p.tiles_m);
}

template <bool CX, int BM, int BN, int WM, int WN, int ROLE>
hsma_status launch_t(GemmParams p, int count, hipStream_t s) {
    p.tiles_m = (p.M + BM - 1) / BM;
    p.tiles_n = (p.N + BN - 1) / BN;
    const int64_t T = (int64_t)p.tiles_m * p.tiles_n;
    const int64_t grid = (T + 7) / 8 * 8;
    if (grid > 0x7fffffff || count > 65535) return HSMA_INVALID_SIZE;
    const int phase = ROLE == (int)GemmRole::Update   ? HSMA_PHASE_UPDATE
                      : ROLE == (int)GemmRole::Leaf   ? HSMA_PHASE_LEAF
                      : ROLE == (int)GemmRole::Inverse ? HSMA_PHASE_DIAG_INV
                      : ROLE == (int)GemmRole::Herk   ? HSMA_PHASE_FACTOR
                                                      : HSMA_PHASE_OTHER;
    // A lower-triangular C (Herk) computes about half of the product.
    ProfScope prof(phase, (p.c_lower ? 1.0 : 2.0) * p.M * (double)p.N * p.K * count, s);
    hipLaunchKernelGGL((hsma_gemm<CX, BM, BN, WM, WN, ROLE>), dim3((unsigned)grid, count), dim3(256),
                       0, s, p);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

template <bool CX, int ROLE>
hsma_status launch_role(GemmParams p, int count, hipStream_t s) {
    if (ROLE == (int)GemmRole::Leaf) {
        // In place: one tile must cover every row so each workgroup reads all
        // K rows of its columns before it writes them.
        // Narrow column tiles keep >= 2 workgroups per CU busy for typical n.
        if (p.M <= 128) return launch_t<CX, 128, 32, 4, 1, ROLE>(p, count, s);
        if (p.M <= 256) return launch_t<CX, 256, 32, 4, 1, ROLE>(p, count, s);
        if (p.M <= 512) return launch_t<CX, 512, 16, 4, 1, ROLE>(p, count, s);
        return HSMA_NOT_SUPPORTED;
    }
    if (p.M <= 64 && p.N <= 64 && ROLE != (int)GemmRole::Update && ROLE != (int)GemmRole::Herk)
        return launch_t<CX, 64, 64, 2, 2, ROLE>(p, count, s);
    if (ROLE == (int)GemmRole::Herk) {
        // Lower-triangular C: the shape with the fewest rounds of non-empty
        // tiles (tile_choice.h).
        DeviceInfo dev;
        const int64_t cus = (device_info(&dev) == HSMA_SUCCESS && dev.num_cus > 0) ? dev.num_cus : 256;
        const int best = lower_tile_shape(p.M, p.N, CX, count, cus);
        if (best == 0) return launch_t<CX, 128, 128, 2, 2, ROLE>(p, count, s);
        if (best == 1) return launch_t<CX, 128, 64, 2, 2, ROLE>(p, count, s);
        if (best == 2) return launch_t<CX, 64, 64, 2, 2, ROLE>(p, count, s);
        if (best == 3) return launch_t<CX, 64, 32, 2, 2, ROLE>(p, count, s);
        return launch_t<CX, 32, 32, 2, 2, ROLE>(p, count, s);
    }
    if (ROLE == (int)GemmRole::Update) {
        // The trailing updates of the deepest recursion levels are thin
        // (M = K = one or two block sizes): below HSMA_UPD_MIN_WG_PER_CU
        // workgroups per CU, narrower tiles keep every CU busy.
        DeviceInfo dev;
        const int64_t cus = (device_info(&dev) == HSMA_SUCCESS && dev.num_cus > 0) ? dev.num_cus : 256;
        const int64_t want = HSMA_UPD_MIN_WG_PER_CU * cus;
        const int64_t rows128 = (p.M + 127) / 128;
        if (rows128 * ((p.N + HSMA_UPD_BN - 1) / HSMA_UPD_BN) * count >= want)
            return launch_t<CX, HSMA_UPD_BM, HSMA_UPD_BN, HSMA_UPD_WM, HSMA_UPD_WN, ROLE>(p, count, s);
        if (rows128 * ((p.N + 63) / 64) * count >= want) return launch_t<CX, 128, 64, 2, 2, ROLE>(p, count, s);
        // Fewer still (the thin updates of small solves, e.g. inside a
        // Cholesky factorization): smaller tiles spread the product over
        // more CUs.  Each element's K order is the same in every shape.
        const int64_t rows64 = (p.M + 63) / 64;
        if (rows64 * ((p.N + 63) / 64) * count >= want) return launch_t<CX, 64, 64, 2, 2, ROLE>(p, count, s);
        if (rows64 * ((p.N + 31) / 32) * count >= want) return launch_t<CX, 64, 32, 2, 2, ROLE>(p, count, s);
        return launch_t<CX, 32, 32, 2, 2, ROLE>(p, count, s);
    }
    return launch_t<CX, 128, 128, 2, 2, ROLE>(p, count, s);
}


// ---------------------------------------------------------------------------
// Mixed precision (real data only): the same product with operands rounded to
// FP32 (round to nearest even) and multiplied on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32, twice the FP64 rate on gfx950).  The FP32
// accumulators are flushed into FP64 accumulators every KCHUNK values of K,
// so rounding error grows with the chunk length, not with K.  The result and
// the epilogue are FP64.
//
// FP32 16x16x4 layout (measured on gfx950): lane l holds A[l%16][k0 + l/16],
// B[k0 + l/16][l%16]; result element v of lane l is row 4(l/16) + v -- already
// the consecutive-rows order, so no row permutation of the A fragment.
// ---------------------------------------------------------------------------
typedef float flt4 __attribute__((ext_vector_type(4)));

template <int BM, int BN, int WM, int WN, int KCHUNK>
__global__ __launch_bounds__(256, 2) void hsma_gemm_f32mfma(const GemmParams p) {
    // 32-deep K slices here (the FP64 kernel takes 16): a slice of FP32
    // products is half as long on the matrix cores, and a deeper one halves
    // the barriers and stores per product (51 KB of LDS per workgroup).
    constexpr int BK = 32;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int LDA_S = BM + 4;
    constexpr int LDB_S = BK + 1;
    static_assert(KCHUNK % BK == 0, "chunk of whole stages");
    __shared__ float As[2][BK * LDA_S];
    __shared__ float Bs[2][BN * LDB_S];

    const int T = p.tiles_m * p.tiles_n;
    const int bid = blockIdx.x;
    const int per = gridDim.x / 8;
    const int t = (bid % 8) * per + bid / 8;
    if (t >= T) return;
    constexpr int GROUP = 8;
    const int gsz_full = GROUP * p.tiles_n;
    const int g = t / gsz_full;
    const int first = g * GROUP;
    const int gsize = (p.tiles_m - first) < GROUP ? (p.tiles_m - first) : GROUP;
    const int tm = first + (t % gsz_full) % gsize;
    const int tn = (t % gsz_full) / gsize;
    const int batch = blockIdx.y;
    const int bo = batch / p.inner, bi = batch % p.inner;
    const double *__restrict__ Ag = p.A + bo * p.a_outer + bi * p.a_inner;
    const double *__restrict__ Bg = p.B + bo * p.b_outer + bi * p.b_inner;
    double *__restrict__ Cg = p.C + bo * p.c_outer + bi * p.c_inner;

    const int m0 = tm * BM, n0 = tn * BN;
    const int M = p.M, N = p.N, K = p.K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WM) * TM, wn0 = (wave / WM) * TN;

    constexpr int A_TOTAL = BM * BK / 2, B_TOTAL = BN * BK / 2;
    constexpr int A_ITEMS = (A_TOTAL + 255) / 256, B_ITEMS = (B_TOTAL + 255) / 256;
    d2 ra[A_ITEMS], rb[B_ITEMS];
    auto load_a = [&](int k0) {
#pragma unroll
        for (int it = 0; it < A_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (A_TOTAL % 256 && e >= A_TOTAL) break;
            const int kk = e / (BM / 2), ii = 2 * (e % (BM / 2));
            const int gr = m0 + ii, gc = k0 + kk;
            d2 v = {0.0, 0.0};
            if (gc < K) {
                const double *src = Ag + (int64_t)gc * p.lda + gr;
                if (gr + 1 < M) v = *reinterpret_cast<const d2 *>(src);
                else if (gr < M) v.x = src[0];
                if (p.tri_a) {
                    if (gr < gc) v.x = 0.0;
                    if (gr + 1 < gc) v.y = 0.0;
                    if (p.tri_a == 2) {
                        if (gr == gc) v.x = 1.0;
                        if (gr + 1 == gc) v.y = 1.0;
                    }
                }
            }
            ra[it] = v;
        }
    };
    auto store_a = [&](int buf) {
#pragma unroll
        for (int it = 0; it < A_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (A_TOTAL % 256 && e >= A_TOTAL) break;
            const int kk = e / (BM / 2), ii = 2 * (e % (BM / 2));
            float *dst = &As[buf][kk * LDA_S + ii];
            dst[0] = (float)ra[it].x;
            dst[1] = (float)ra[it].y;
        }
    };
    auto load_b = [&](int k0) {
#pragma unroll
        for (int it = 0; it < B_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (B_TOTAL % 256 && e >= B_TOTAL) break;
            const int jj = e / (BK / 2), kk = 2 * (e % (BK / 2));
            const int gn = n0 + jj, gk = k0 + kk;
            d2 v = {0.0, 0.0};
            if (gn < N) {
                const double *src = Bg + (int64_t)gn * p.ldb + gk;
                if (gk + 1 < K) v = *reinterpret_cast<const d2 *>(src);
                else if (gk < K) v.x = src[0];
            }
            rb[it] = v;
        }
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int it = 0; it < B_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (B_TOTAL % 256 && e >= B_TOTAL) break;
            const int jj = e / (BK / 2), kk = 2 * (e % (BK / 2));
            float *dst = &Bs[buf][jj * LDB_S + kk];
            dst[0] = (float)rb[it].x;
            dst[1] = (float)rb[it].y;
        }
    };

    dbl4 acc[FM][FN];
    flt4 acc32[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
            acc32[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
        }

    const int nk = (K + BK - 1) / BK;
    if (nk > 0) {
        load_a(0);
        load_b(0);
        store_a(0);
        store_b(0);
        __syncthreads();
    }
    const int lr = lane & 15, lk = lane >> 4;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) {
            load_a((kt + 1) * BK);
            load_b((kt + 1) * BK);
        }
        const float *as = As[buf];
        const float *bs = Bs[buf];
#pragma unroll
        for (int s = 0; s < BK / 4; ++s) {
            const int k = 4 * s + lk;
            float fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) fa[i] = as[k * LDA_S + wm0 + 16 * i + lr];
#pragma unroll
            for (int j = 0; j < FN; ++j) fb[j] = bs[(wn0 + 16 * j + lr) * LDB_S + k];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc32[i][j], 0, 0, 0);
        }
        if ((kt + 1) % (KCHUNK / BK) == 0 || kt + 1 == nk) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)acc32[i][j][v];
                    acc32[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
                }
        }
        if (kt + 1 < nk) {
            store_a(buf ^ 1);
            store_b(buf ^ 1);
        }
        __syncthreads();
    }

    const bool beta_zero = (p.beta_re == 0.0);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn0 + 16 * j + lr;
            const int row = m0 + wm0 + 16 * i + 4 * lk;
            if (col >= N) continue;
            double *dst = Cg + (int64_t)col * p.ldc + row;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                if (row + h < M) {
                    double r = p.alpha_re * acc[i][j][h];
                    if (!beta_zero) r = __fma_rn(p.beta_re, dst[h], r);
                    dst[h] = r;
                }
            }
        }
    }
}

hsma_status launch_mixed(GemmParams p, int count, hipStream_t s) {
    // 128 x 64 keeps both accumulator sets within 256 registers (two
    // workgroups per CU) without spilling.
    constexpr int BM = 128, BN = 64;
    p.tiles_m = (p.M + BM - 1) / BM;
    p.tiles_n = (p.N + BN - 1) / BN;
    const int64_t T = (int64_t)p.tiles_m * p.tiles_n;
    const int64_t grid = (T + 7) / 8 * 8;
    if (grid > 0x7fffffff || count > 65535) return HSMA_INVALID_SIZE;
    ProfScope prof(HSMA_PHASE_UPDATE, 2.0 * p.M * (double)p.N * p.K * count, s);
    hipLaunchKernelGGL((hsma_gemm_f32mfma<BM, BN, 2, 2, 256>), dim3((unsigned)grid, count), dim3(256), 0, s, p);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

template <bool CX, int BM, int BN, int WM, int WN>
hsma_status grouped_t(const GemmParams *descs, int nd, int64_t tiles, int phase, double flops,
                      hipStream_t s) {
    ProfScope prof(phase, flops, s);
    hipLaunchKernelGGL((hsma_gemm_grouped<CX, BM, BN, WM, WN>), dim3((unsigned)tiles), dim3(256), 0,
                       s, descs, nd);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

template <bool CX>
hsma_status grouped_shape(GemmRole role, int bm, int bn, const GemmParams *descs, int nd,
                          int64_t tiles, double flops, hipStream_t s) {
    const int phase = role == GemmRole::Update    ? HSMA_PHASE_UPDATE
                      : role == GemmRole::Leaf    ? HSMA_PHASE_LEAF
                      : role == GemmRole::Inverse ? HSMA_PHASE_DIAG_INV
                                                  : HSMA_PHASE_OTHER;
    if (bm == 128 && bn == 32) return grouped_t<CX, 128, 32, 4, 1>(descs, nd, tiles, phase, flops, s);
    if (bm == 256 && bn == 32) return grouped_t<CX, 256, 32, 4, 1>(descs, nd, tiles, phase, flops, s);
    if (bm == 512 && bn == 16) return grouped_t<CX, 512, 16, 4, 1>(descs, nd, tiles, phase, flops, s);
    if (bm == 64 && bn == 64) return grouped_t<CX, 64, 64, 2, 2>(descs, nd, tiles, phase, flops, s);
    if (bm == 128 && bn == 64) return grouped_t<CX, 128, 64, 2, 2>(descs, nd, tiles, phase, flops, s);
    if (bm == 128 && bn == 128) return grouped_t<CX, 128, 128, 2, 2>(descs, nd, tiles, phase, flops, s);
    return HSMA_NOT_SUPPORTED;
}

}  // namespace

int gemm_grouped_tile(GemmRole role, int max_m, int max_n, int *bm, int *bn) {
    if (role == GemmRole::Leaf) {
        if (max_m <= 128) { *bm = 128; *bn = 32; return 1; }
        if (max_m <= 256) { *bm = 256; *bn = 32; return 1; }
        if (max_m <= 512) { *bm = 512; *bn = 16; return 1; }
        return 0;
    }
    if (role == GemmRole::UpdateMixed) return 0;
    // Narrow right-hand sides: one column tile covers them, so each row
    // panel of A is read once.
    if (max_n <= 32) { *bm = max_m <= 128 ? 128 : 256; *bn = 32; return 1; }
    if (max_n <= 64) { *bm = max_m <= 64 ? 64 : 128; *bn = 64; return 1; }
    *bm = 128;
    *bn = 128;
    return 1;
}

hsma_status launch_gemm_grouped(bool cplx_, GemmRole role, int bm, int bn, const GemmParams *descs,
                                int nd, int64_t total_tiles, double flops, hipStream_t s) {
    if (nd <= 0 || total_tiles <= 0) return HSMA_SUCCESS;
    if (total_tiles > 0x7fffffff) return HSMA_INVALID_SIZE;
    return cplx_ ? grouped_shape<true>(role, bm, bn, descs, nd, total_tiles, flops, s)
                 : grouped_shape<false>(role, bm, bn, descs, nd, total_tiles, flops, s);
}

hsma_status launch_gemm(bool cplx_, GemmRole role, int M, int N, int K, cplx alpha,
                        const double *A, int64_t lda, const double *B, int64_t ldb, cplx beta,
                        double *C, int64_t ldc, int tri_a, const GemmBatch &batch,
                        hipStream_t s, int k_lower, int c_lower) {
    if (M <= 0 || N <= 0 || batch.count <= 0) return HSMA_SUCCESS;
    GemmParams p{};
    p.M = M;
    p.N = N;
    p.K = K;
    p.A = A;
    p.lda = lda;
    p.B = B;
    p.ldb = ldb;
    p.C = C;
    p.ldc = ldc;
    p.alpha_re = alpha.re;
    p.alpha_im = alpha.im;
    p.beta_re = beta.re;
    p.beta_im = beta.im;
    p.tri_a = tri_a;
    p.k_lower = (k_lower && tri_a) ? 1 : 0;
    p.c_lower = c_lower ? 1 : 0;
    p.inner = batch.inner > 0 ? batch.inner : 1;
    p.a_outer = batch.a_outer;
    p.a_inner = batch.a_inner;
    p.b_outer = batch.b_outer;
    p.b_inner = batch.b_inner;
    p.c_outer = batch.c_outer;
    p.c_inner = batch.c_inner;
    if (cplx_ && ((M | K) & 1)) return HSMA_INVALID_SIZE;
    if (role == GemmRole::UpdateMixed) {
        if (cplx_) return HSMA_NOT_SUPPORTED;
        return launch_mixed(p, batch.count, s);
    }
    switch (role) {
        case GemmRole::Update:
            return cplx_ ? launch_role<true, 0>(p, batch.count, s) : launch_role<false, 0>(p, batch.count, s);
        case GemmRole::Leaf:
            return cplx_ ? launch_role<true, 1>(p, batch.count, s) : launch_role<false, 1>(p, batch.count, s);
        case GemmRole::Inverse:
            return cplx_ ? launch_role<true, 2>(p, batch.count, s) : launch_role<false, 2>(p, batch.count, s);
        case GemmRole::Residual:
            return cplx_ ? launch_role<true, 3>(p, batch.count, s) : launch_role<false, 3>(p, batch.count, s);
        case GemmRole::Herk:
            return cplx_ ? launch_role<true, 5>(p, batch.count, s) : launch_role<false, 5>(p, batch.count, s);
        default:
            break;
    }
    return HSMA_INVALID_VALUE;
}

}  // namespace hsma
