// FP32 matrix-core product for the single-precision solves (STRSM, CTRSM).
//
// The same products as the FP64 blocked path (paper Sec. 4.3: trailing
// updates, diagonal solves, inverse merges), on FP32 data with FP32
// accumulation, on the FP32 matrix cores (v_mfma_f32_16x16x4_f32, twice the
// FP64 matrix rate on gfx950):
//
//   C = beta * C + alpha * A * B        (column-major, real-view units)
//
// Tiling: a 256-thread workgroup (4 wavefronts) owns a BM x BN tile of C;
// K advances 16 at a time through a two-stage LDS ring (loads for stage k+1
// issued before the matrix-core work on stage k, written to the other buffer
// after it, one barrier per stage).
//
// Operand layout of v_mfma_f32_16x16x4_f32: lane l holds A[l%16][k0 + l/16]
// and B[k0 + l/16][l%16]; result element v of lane l is row 4(l/16) + v of
// column l%16, so each lane holds 4 consecutive rows of one column and the
// (re, im) rows of a complex element stay in one lane.
//
// Complex data: a complex M x K matrix is the real 2M x 2K matrix of 2 x 2
// blocks [[re, -im], [im, re]], expanded while A is staged into LDS; complex
// B and C are real matrices of twice the rows (interleaved re, im).
//
// Workgroup -> tile mapping: consecutive workgroup ids go to different XCDs,
// so ids are remapped to give each XCD a contiguous run of tiles, walked in
// groups of 8 tile-rows that share A and B panels in that XCD's L2.

#include "internal.h"

namespace hsma {
namespace {

typedef float flt4 __attribute__((ext_vector_type(4)));
// Two floats moved as one 8-byte access; only 4-byte alignment assumed.
typedef float flt2u __attribute__((ext_vector_type(2), aligned(4)));

constexpr int BK = 16;

__host__ __device__ constexpr int lds_bytes32(int bm, int bn) {
    return 2 * (BK * (bm + 4) + bn * (BK + 1)) * 4;
}
__host__ __device__ constexpr int occ32(int bm, int bn) {
    return (160 * 1024 / lds_bytes32(bm, bn)) >= 3 ? 3 : ((160 * 1024 / lds_bytes32(bm, bn)) >= 2 ? 2 : 1);
}

template <bool CX, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256, (occ32(BM, BN))) void hsma_gemm32(const Gemm32Params p) {
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int LDA_S = BM + 4;
    constexpr int LDB_S = BK + 1;
    static_assert(WM * WN == 4, "four wavefronts");
    static_assert(TM % 16 == 0 && TN % 16 == 0, "16x16 blocks");
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
    const float *__restrict__ Ag = p.A + bo * p.a_outer + bi * p.a_inner;
    const float *__restrict__ Bg = p.B + bo * p.b_outer + bi * p.b_inner;
    float *__restrict__ Cg = p.C + bo * p.c_outer + bi * p.c_inner;

    const int m0 = tm * BM, n0 = tn * BN;
    const int M = p.M, N = p.N;
    const int K = (p.k_lower && m0 + BM < p.K) ? m0 + BM : p.K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WM) * TM, wn0 = (wave / WM) * TN;

    // A: real: BM*BK/2 row pairs; complex: BM*BK/4 complex elements.
    constexpr int A_TOTAL = CX ? (BM * BK / 4) : (BM * BK / 2);
    constexpr int B_TOTAL = BN * BK / 2;
    constexpr int A_ITEMS = (A_TOTAL + 255) / 256;
    constexpr int B_ITEMS = (B_TOTAL + 255) / 256;
    flt2u ra[A_ITEMS], rb[B_ITEMS];

    auto load_a = [&](int k0) {
#pragma unroll
        for (int it = 0; it < A_ITEMS; ++it) {
            const int e = tid + it * 256;
            if (A_TOTAL % 256 && e >= A_TOTAL) break;
            flt2u v = {0.f, 0.f};
            if (!CX) {
                const int kk = e / (BM / 2), ii = 2 * (e % (BM / 2));
                const int gr = m0 + ii, gc = k0 + kk;
                if (gc < K) {
                    const float *src = Ag + (int64_t)gc * p.lda + gr;
                    if (gr + 1 < M) v = *reinterpret_cast<const flt2u *>(src);
                    else if (gr < M) v.x = src[0];
                    if (p.tri_a) {
                        if (gr < gc) v.x = 0.f;
                        if (gr + 1 < gc) v.y = 0.f;
                        if (p.tri_a == 2) {
                            if (gr == gc) v.x = 1.f;
                            if (gr + 1 == gc) v.y = 1.f;
                        }
                    }
                }
            } else {
                const int kc = e / (BM / 2), ic = e % (BM / 2);
                const int gr = m0 / 2 + ic, gc = k0 / 2 + kc;
                if (gc < K / 2 && gr < M / 2) {
                    v = *reinterpret_cast<const flt2u *>(Ag + 2 * ((int64_t)gc * p.lda + gr));
                    if (p.tri_a) {
                        if (gr < gc) v.x = v.y = 0.f;
                        if (p.tri_a == 2 && gr == gc) {
                            v.x = 1.f;
                            v.y = 0.f;
                        }
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
            if (!CX) {
                const int kk = e / (BM / 2), ii = 2 * (e % (BM / 2));
                float *dst = &As[buf][kk * LDA_S + ii];
                dst[0] = ra[it].x;
                dst[1] = ra[it].y;
            } else {
                const int kc = e / (BM / 2), ic = e % (BM / 2);
                float *d0 = &As[buf][(2 * kc) * LDA_S + 2 * ic];
                float *d1 = &As[buf][(2 * kc + 1) * LDA_S + 2 * ic];
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
            flt2u v = {0.f, 0.f};
            if (gn < N) {
                const float *src = Bg + (int64_t)gn * p.ldb + gk;
                if (gk + 1 < K) v = *reinterpret_cast<const flt2u *>(src);
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
            dst[0] = rb[it].x;
            dst[1] = rb[it].y;
        }
    };

    flt4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

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
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) {
            store_a(buf ^ 1);
            store_b(buf ^ 1);
        }
        __syncthreads();
    }

    const bool beta_zero = (p.beta_re == 0.f && p.beta_im == 0.f);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn0 + 16 * j + lr;
            const int row = m0 + wm0 + 16 * i + 4 * lk;
            if (col >= N) continue;
            float *dst = Cg + (int64_t)col * p.ldc + row;
            const float v[4] = {acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]};
            if (CX) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (row + 2 * h < M) {
                        const float ar = v[2 * h], ai = v[2 * h + 1];
                        float r = p.alpha_re * ar - p.alpha_im * ai;
                        float q = p.alpha_re * ai + p.alpha_im * ar;
                        if (!beta_zero) {
                            const float cr = dst[2 * h], ci = dst[2 * h + 1];
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
                    if (row + h < M) {
                        float r = p.alpha_re * v[h];
                        if (!beta_zero) r = __fmaf_rn(p.beta_re, dst[h], r);
                        dst[h] = r;
                    }
                }
            }
        }
    }
}

template <bool CX, int BM, int BN, int WM, int WN>
hsma_status launch32_t(Gemm32Params p, int count, int phase, hipStream_t s) {
    p.tiles_m = (p.M + BM - 1) / BM;
    p.tiles_n = (p.N + BN - 1) / BN;
    const int64_t T = (int64_t)p.tiles_m * p.tiles_n;
    const int64_t grid = (T + 7) / 8 * 8;
    if (grid > 0x7fffffff || count > 65535) return HSMA_INVALID_SIZE;
    ProfScope prof(phase, 2.0 * p.M * (double)p.N * p.K * count, s);
    hipLaunchKernelGGL((hsma_gemm32<CX, BM, BN, WM, WN>), dim3((unsigned)grid, count), dim3(256), 0,
                       s, p);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

template <bool CX>
hsma_status launch32_role(GemmRole role, Gemm32Params p, int count, hipStream_t s) {
    const int phase = role == GemmRole::Update    ? HSMA_PHASE_UPDATE
                      : role == GemmRole::Leaf    ? HSMA_PHASE_LEAF
                      : role == GemmRole::Inverse ? HSMA_PHASE_DIAG_INV
                                                  : HSMA_PHASE_OTHER;
    if (role == GemmRole::Leaf) {
        // In place: one tile covers every row, so each workgroup reads all
        // of its columns before it writes them.
        if (p.M <= 128) return launch32_t<CX, 128, 32, 4, 1>(p, count, phase, s);
        if (p.M <= 256) return launch32_t<CX, 256, 32, 4, 1>(p, count, phase, s);
        if (p.M <= 512) return launch32_t<CX, 512, 16, 4, 1>(p, count, phase, s);
        return HSMA_NOT_SUPPORTED;
    }
    if (p.M <= 64 && p.N <= 64) return launch32_t<CX, 64, 64, 2, 2>(p, count, phase, s);
    if (role == GemmRole::Update) {
        // Thin updates of the deepest levels: narrower tiles when a 128 x 128
        // grid would leave CUs idle (fewer than 4 tiles per CU).
        DeviceInfo dev;
        const int64_t cus = (device_info(&dev) == HSMA_SUCCESS && dev.num_cus > 0) ? dev.num_cus : 256;
        const int64_t want = 4 * cus;
        const int64_t rows128 = (p.M + 127) / 128;
        if (rows128 * ((p.N + 127) / 128) * count >= want)
            return launch32_t<CX, 128, 128, 2, 2>(p, count, phase, s);
        if (rows128 * ((p.N + 63) / 64) * count >= want) return launch32_t<CX, 128, 64, 2, 2>(p, count, phase, s);
        return launch32_t<CX, 64, 64, 2, 2>(p, count, phase, s);
    }
    return launch32_t<CX, 128, 128, 2, 2>(p, count, phase, s);
}

}  // namespace

hsma_status launch_gemm(bool cplx_, GemmRole role, int M, int N, int K, cplx alpha,
                        const float *A, int64_t lda, const float *B, int64_t ldb, cplx beta,
                        float *C, int64_t ldc, int tri_a, const GemmBatch &batch, hipStream_t s,
                        int k_lower) {
    if (M <= 0 || N <= 0 || batch.count <= 0) return HSMA_SUCCESS;
    if (role == GemmRole::UpdateMixed) return HSMA_NOT_SUPPORTED;
    if (cplx_ && ((M | K) & 1)) return HSMA_INVALID_SIZE;
    Gemm32Params p{};
    p.M = M;
    p.N = N;
    p.K = K;
    p.A = A;
    p.lda = lda;
    p.B = B;
    p.ldb = ldb;
    p.C = C;
    p.ldc = ldc;
    p.alpha_re = (float)alpha.re;
    p.alpha_im = (float)alpha.im;
    p.beta_re = (float)beta.re;
    p.beta_im = (float)beta.im;
    p.tri_a = tri_a;
    p.k_lower = (k_lower && tri_a) ? 1 : 0;
    p.inner = batch.inner > 0 ? batch.inner : 1;
    p.a_outer = batch.a_outer;
    p.a_inner = batch.a_inner;
    p.b_outer = batch.b_outer;
    p.b_inner = batch.b_inner;
    p.c_outer = batch.c_outer;
    p.c_inner = batch.c_inner;
    return cplx_ ? launch32_role<true>(role, p, batch.count, s)
                 : launch32_role<false>(role, p, batch.count, s);
}

}  // namespace hsma
