// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "../../include/hsma.h"

// Problems with m, n <= HSMA_TINY_MAX take the fused four-per-wavefront
// kernel (tiny.hip), alone and in batches.
#ifndef HSMA_TINY_MAX
#define HSMA_TINY_MAX 16
#endif

// Size of the allocation-free entry point's per-device scratch array.
#define HSMA_NOALLOC_SCRATCH_BYTES (64ull << 20)

namespace hsma {

// Record a failing HIP call for hsma_last_hip_error() and turn it into a status.
hsma_status hip_fail(hipError_t e);

#define HSMA_HIP(call)                                   \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return ::hsma::hip_fail(e_); \
    } while (0)

#define HSMA_TRY(call)                                   \
    do {                                                 \
        hsma_status s_ = (call);                         \
        if (s_ != HSMA_SUCCESS) return s_;               \
    } while (0)

// Global-memory address space.  Pointers that kernels read out of descriptor
// tables are generic; loads and stores through a generic pointer become FLAT
// instructions, which count against the LDS wait counter as well, so every
// wait for an LDS read would also wait for the global loads in flight.
// Kernels convert such pointers with a cast to HSMA_GLOBAL before use.
#define HSMA_GLOBAL __attribute__((address_space(1)))

// Two doubles moved as one 16-byte access (a complex value, or two
// consecutive real entries); it assumes only 8-byte alignment.
typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));

// Complex scalar as two doubles (interleaved storage).
struct cplx {
    double re, im;
};

// Per-device facts read once.
struct DeviceInfo {
    int device = -1;
    int num_cus = 0;
    int arch_ok = 0;   // gfx950
};
hsma_status device_info(DeviceInfo *out);

// While profiling is enabled, records an event pair around the enclosed
// kernel launch on stream s (see hsma_profile_begin).
class ProfScope {
  public:
    ProfScope(int phase, double flops, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    hipStream_t s_;
    int idx_;
};

// Workspace from the library's per-device block cache (alloc.cpp): usable
// in stream order on s; ws_free hands the block back after the work already
// enqueued on s.
hsma_status ws_alloc(void **p, size_t bytes, hipStream_t s);
hsma_status ws_free(void *p, hipStream_t s);
// Return a block whose last use has completed on the device: reusable on any
// stream at once (no event).
hsma_status ws_free_idle(void *p);
size_t ws_cached_bytes();

// ---------------------------------------------------------------------------
// Kernel launchers (each enqueues on `s`; arguments already validated).
// ---------------------------------------------------------------------------

// B <- alpha * inv(tril(A)) * B for m <= 64; panels of 64 columns.
hsma_status launch_small_solve(bool cplx_, bool unit, int m, int64_t n, cplx alpha,
                               const double *A, int64_t lda, double *B, int64_t ldb,
                               hipStream_t s);

// Fused very small solves (m, n <= HSMA_TINY_MAX): one problem, or a device
// table of items in the batched layout, four per workgroup.
bool tiny_fits(int64_t m, int64_t n);
size_t tiny_item_bytes();
hsma_status launch_tiny_one(bool cx, bool unit, int m, int n, cplx alpha, const double *A,
                            int64_t lda, double *B, int64_t ldb, hipStream_t s);
hsma_status launch_tiny_group(bool cx, bool unit, const void *items, int count, hipStream_t s);

// The same on FP32 data (m <= 64).
hsma_status launch_small_solve(bool cplx_, bool unit, int m, int64_t n, cplx alpha,
                               const float *A, int64_t lda, float *B, int64_t ldb,
                               hipStream_t s);

// Argument checks of one problem (the documented order); FP32 data types
// pass only with allow32, else HSMA_NOT_SUPPORTED.
hsma_status validate(int diag, int dtype, int64_t m, int64_t n, const void *alpha, const void *A,
                     int64_t lda, const void *B, int64_t ldb, bool *quick, bool allow32 = false);
bool is_single(int dtype);
bool is_complex(int dtype);
cplx read_alpha(int dtype, const void *alpha);

// B <- 0 on FP32 data (m x n, leading dimension ldb, `es` floats per element).
hsma_status launch_zero32(int64_t m, int64_t n, int es, float *B, int64_t ldb, hipStream_t s);

// B <- 0 (m x n, leading dimension ldb, `es` doubles per element).
hsma_status launch_zero(int64_t m, int64_t n, int es, double *B, int64_t ldb, hipStream_t s);

// General matrix product used by the blocked path, in real-view units:
//   C = beta * C + alpha * op(A) * B,
// C is M x N (ldc), B is K x N (ldb).  Real: A is M x K (lda).  Complex: A is
// (M/2) x (K/2) complex (lda in complex elements) and is expanded on the fly
// to its M x K real representation; B and C are complex matrices viewed as
// real with twice the rows (ldb, ldc in doubles).  Batch b addresses
// (b / inner) * s_outer + (b % inner) * s_inner (in doubles) for each operand.
// tri_a: A is the m x m diagonal block of a lower-triangular matrix, read only
// on and below its diagonal (0: plain, 1: lower non-unit, 2: lower unit).
enum class GemmRole { Update = 0, Leaf = 1, Inverse = 2, Residual = 3, UpdateMixed = 4, Herk = 5 };

// Parameters of one product (also the descriptor of a grouped launch, read
// by the kernel from device memory).
struct GemmParams {
    int M, N, K;          // real-view sizes
    const double *A;
    int64_t lda;          // real: doubles; complex: complex elements
    const double *B;
    int64_t ldb;          // doubles
    double *C;
    int64_t ldc;          // doubles
    double alpha_re, alpha_im, beta_re, beta_im;
    int tri_a;            // 0 plain, 1 lower non-unit, 2 lower unit (diagonal block of L)
    int inner;            // batch decomposition
    int64_t a_outer, a_inner, b_outer, b_inner, c_outer, c_inner;
    int tiles_m, tiles_n;
    int tile0;            // grouped launch: first tile of this product in the grid
    int k_lower;          // 1: A is lower triangular as a whole (with tri_a), so a
                          // tile of rows [m0, m0 + BM) stops its K loop at m0 + BM
    int c_lower;          // 1: only the lower triangle of C (column <= row, in
                          // elements) is computed and stored
};

// Tile shape a grouped launch of `role` uses when its largest product has
// max_m real-view rows and max_n columns (leaves need one tile to span all
// rows); 0 if unsupported.
int gemm_grouped_tile(GemmRole role, int max_m, int max_n, int *bm, int *bn);
// Launch over nd descriptors already in device memory (tile0 / tiles_m /
// tiles_n filled for the shape gemm_grouped_tile returned); total_tiles is
// the grid size.  flops is for the phase profiler.
hsma_status launch_gemm_grouped(bool cplx_, GemmRole role, int bm, int bn, const GemmParams *descs,
                                int nd, int64_t total_tiles, double flops, hipStream_t s);

// Single-precision product (FP32 data, FP32 accumulation on the FP32 matrix
// cores): the same roles, sizes and conventions as GemmParams.
struct Gemm32Params {
    int M, N, K;
    const float *A;
    int64_t lda;
    const float *B;
    int64_t ldb;
    float *C;
    int64_t ldc;
    float alpha_re, alpha_im, beta_re, beta_im;
    int tri_a;
    int k_lower;
    int inner;
    int64_t a_outer, a_inner, b_outer, b_inner, c_outer, c_inner;
    int tiles_m, tiles_n;
};

struct GemmBatch {
    int count = 1, inner = 1;
    int64_t a_outer = 0, a_inner = 0, b_outer = 0, b_inner = 0, c_outer = 0, c_inner = 0;
};
// k_lower = 1: A (with tri_a != 0) is a whole lower-triangular matrix, so
// each row tile reads only the columns left of its last row.
// c_lower = 1: only C's lower triangle (element column <= element row) is
// written; tiles wholly above the diagonal do nothing.
hsma_status launch_gemm(bool cplx_, GemmRole role, int M, int N, int K,
                        cplx alpha, const double *A, int64_t lda, const double *B,
                        int64_t ldb, cplx beta, double *C, int64_t ldc, int tri_a,
                        const GemmBatch &batch, hipStream_t s, int k_lower = 0,
                        int c_lower = 0);
// The same product on FP32 data (FP32 matrix cores, FP32 accumulation).
hsma_status launch_gemm(bool cplx_, GemmRole role, int M, int N, int K, cplx alpha,
                        const float *A, int64_t lda, const float *B, int64_t ldb, cplx beta,
                        float *C, int64_t ldc, int tri_a, const GemmBatch &batch, hipStream_t s,
                        int k_lower = 0);

// Inverse of every diagonal sub-block of edge `base` (<= 64) along the
// diagonal of L (m rows, partitioned into consecutive chunks of `base`, last
// chunk ragged), written into W: chunk c starting at global row o goes to
// W + blk * ib*ib + oo + oo*ib (oo = o mod ib, blk = o / ib), in elements.
// Every element of W's ib x ib blocks not written by this call is zeroed.
hsma_status launch_diag_inv_base(bool cplx_, bool unit, int m, int base, int ib,
                                 const double *A, int64_t lda, double *W, hipStream_t s);
hsma_status launch_diag_inv_base(bool cplx_, bool unit, int m, int base, int ib,
                                 const float *A, int64_t lda, float *W, hipStream_t s);

// dst (R x C, ldd) = src^H for src C x R (ldsrc); the transpose for real data.
// X L^H = B for a lower, non-unit L (m x n X and B, n x n L; FP64 real or
// complex), the solve of a Cholesky step: X overwrites B, and xh (n x m,
// leading dimension n) receives X^H as well.
hsma_status trsm_right_lower_keep(bool cx, int64_t m, int64_t n, const double *A, int64_t lda, double *B,
                                  int64_t ldb, double *xh, hipStream_t s);
hsma_status launch_conj_transpose(bool cx, const double *src, int64_t ldsrc, double *dst,
                                  int64_t ldd, int64_t R, int64_t C, hipStream_t s);

// Synthetic serving inputs (Philox4x32-10, see hsma_generate_inputs).
struct GenRequest {
    double *L, *B;   // lda = ldb = m
    int64_t m, n;
    uint64_t key;
    bool cx;
};
hsma_status launch_gen_inputs(bool cx, int64_t m, int64_t n, uint64_t key, double *L, double *B,
                              hipStream_t s);
hsma_status gen_inputs_grouped(const GenRequest *reqs, int count, hipStream_t s);

}  // namespace hsma
