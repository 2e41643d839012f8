// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "../../include/hsma.h"

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

// Stream-ordered workspace from the device's default memory pool.
hsma_status ws_alloc(void **p, size_t bytes, hipStream_t s);
hsma_status ws_free(void *p, hipStream_t s);

// ---------------------------------------------------------------------------
// Kernel launchers (each enqueues on `s`; arguments already validated).
// ---------------------------------------------------------------------------

// B <- alpha * inv(tril(A)) * B for m <= 64; panels of 64 columns.
hsma_status launch_small_solve(bool cplx_, bool unit, int m, int64_t n, cplx alpha,
                               const double *A, int64_t lda, double *B, int64_t ldb,
                               hipStream_t s);

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
struct GemmBatch {
    int count = 1, inner = 1;
    int64_t a_outer = 0, a_inner = 0, b_outer = 0, b_inner = 0, c_outer = 0, c_inner = 0;
};
enum class GemmRole { Update = 0, Leaf = 1, Inverse = 2, Residual = 3, UpdateMixed = 4 };
hsma_status launch_gemm(bool cplx_, GemmRole role, int M, int N, int K,
                        cplx alpha, const double *A, int64_t lda, const double *B,
                        int64_t ldb, cplx beta, double *C, int64_t ldc, int tri_a,
                        const GemmBatch &batch, hipStream_t s);

// Inverse of every diagonal sub-block of edge `base` (<= 64) along the
// diagonal of L (m rows, partitioned into consecutive chunks of `base`, last
// chunk ragged), written into W: chunk c starting at global row o goes to
// W + blk * ib*ib + oo + oo*ib (oo = o mod ib, blk = o / ib), in elements.
// Every element of W's ib x ib blocks not written by this call is zeroed.
hsma_status launch_diag_inv_base(bool cplx_, bool unit, int m, int base, int ib,
                                 const double *A, int64_t lda, double *W, hipStream_t s);

}  // namespace hsma
