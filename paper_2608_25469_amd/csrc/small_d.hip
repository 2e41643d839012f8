// Small-solve and diagonal-inversion launchers, real double.
// (One translation unit per data type keeps compile times parallel.)

#include "small_kernels.h"

namespace hsma {

using namespace smallk;

namespace {

template <bool UNIT>
hsma_status small_t(int m, int64_t n, cplx alpha, const double *A, int64_t lda, double *B,
                    int64_t ldb, hipStream_t s) {
    const int64_t panels = (n + 63) / 64;
    if (panels > 0x7fffffff) return HSMA_INVALID_SIZE;
    dim3 grid((unsigned)panels), block(64);
    switch ((m + 7) / 8) {
#define HSMA_CASE(N)                                                                              \
    case N:                                                                                       \
        hipLaunchKernelGGL((hsma_small_solve<false, N, UNIT>), grid, block, 0, s, A, lda, B, ldb, m, \
                           n, alpha.re, alpha.im);                                                \
        break;
        HSMA_CASE(1) HSMA_CASE(2) HSMA_CASE(3) HSMA_CASE(4)
        HSMA_CASE(5) HSMA_CASE(6) HSMA_CASE(7) HSMA_CASE(8)
#undef HSMA_CASE
        default:
            return HSMA_INVALID_SIZE;
    }
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

template <bool UNIT>
hsma_status inv_t(int m, int base, int ib, const double *A, int64_t lda, double *W,
                  hipStream_t s) {
    dim3 grid((m + base - 1) / base), block(64);
    switch (base / 8) {
#define HSMA_CASE(N)                                                                              \
    case N:                                                                                       \
        hipLaunchKernelGGL((hsma_diag_inv_base<false, N, UNIT>), grid, block, 0, s, A, lda, W, m,  \
                           base, ib);                                                             \
        break;
        HSMA_CASE(1) HSMA_CASE(2) HSMA_CASE(4) HSMA_CASE(8)
#undef HSMA_CASE
        default:
            return HSMA_INVALID_SIZE;
    }
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

}  // namespace

hsma_status launch_small_d(bool unit, int m, int64_t n, cplx alpha, const double *A,
                              int64_t lda, double *B, int64_t ldb, hipStream_t s) {
    return unit ? small_t<true>(m, n, alpha, A, lda, B, ldb, s)
                : small_t<false>(m, n, alpha, A, lda, B, ldb, s);
}

hsma_status launch_inv_base_d(bool unit, int m, int base, int ib, const double *A,
                                 int64_t lda, double *W, hipStream_t s) {
    return unit ? inv_t<true>(m, base, ib, A, lda, W, s) : inv_t<false>(m, base, ib, A, lda, W, s);
}

}  // namespace hsma
