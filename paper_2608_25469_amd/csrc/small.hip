// Dispatch for the small-solve and diagonal-inversion kernels, and the
// zero fill used for alpha == 0 and for workspace initialisation (a kernel,
// not a memset, so the blocked schedule stays safe to capture in a graph).

#include "internal.h"

namespace hsma {

hsma_status launch_strip_one(bool cx, bool unit, int m, int64_t n, cplx alpha, const double *A,
                             int64_t lda, double *B, int64_t ldb, hipStream_t s);
hsma_status launch_inv_base(bool cx, bool unit, int m, int base, int ib, const double *A, int64_t lda,
                            double *W, hipStream_t s);


namespace {

// B <- 0 on rows 0..m-1 (es doubles per element).
__global__ __launch_bounds__(256) void hsma_zero_fill(double *__restrict__ B, int64_t rows,
                                                      int64_t n, int64_t ld) {
    const int64_t total = rows * n;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        const int64_t j = t / rows, i = t - j * rows;
        B[i + j * ld] = 0.0;
    }
}


}  // namespace

hsma_status launch_small_solve(bool cplx_, bool unit, int m, int64_t n, cplx alpha,
                               const double *A, int64_t lda, double *B, int64_t ldb,
                               hipStream_t s) {
    if (m < 1 || m > 64) return HSMA_INVALID_SIZE;
    const double flops = (cplx_ ? 8.0 : 2.0) * 0.5 * m * (m + 1.0) * (double)n;
    if (tiny_fits(m, n)) {
        ProfScope prof(HSMA_PHASE_TINY, flops, s);
        return launch_tiny_one(cplx_, unit, m, (int)n, alpha, A, lda, B, ldb, s);
    }
    ProfScope prof(HSMA_PHASE_SMALL, flops, s);
    return launch_strip_one(cplx_, unit, m, n, alpha, A, lda, B, ldb, s);
}

hsma_status launch_zero(int64_t m, int64_t n, int es, double *B, int64_t ldb, hipStream_t s) {
    const int64_t rows = m * es, ld = ldb * es;
    const int64_t total = rows * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) return HSMA_SUCCESS;
    ProfScope prof(HSMA_PHASE_OTHER, 0.0, s);
    hipLaunchKernelGGL(hsma_zero_fill, dim3((unsigned)blocks), dim3(256), 0, s, B, rows, n, ld);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

hsma_status launch_diag_inv_base(bool cplx_, bool unit, int m, int base, int ib, const double *A,
                                 int64_t lda, double *W, hipStream_t s) {
    if (base < 8 || base > 64 || (base & 7) || ib % base) return HSMA_INVALID_SIZE;
    const int nblk = (m + ib - 1) / ib;
    const int es = cplx_ ? 2 : 1;
    HSMA_TRY(launch_zero((int64_t)ib * ib, nblk, es, W, (int64_t)ib * ib, s));
    ProfScope prof(HSMA_PHASE_DIAG_INV, 0.0, s);
    return launch_inv_base(cplx_, unit, m, base, ib, A, lda, W, s);
}

}  // namespace hsma
