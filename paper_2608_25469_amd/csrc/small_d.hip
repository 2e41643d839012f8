// Small-solve and diagonal-inversion launchers, real double.
// (One translation unit per data type keeps compile times parallel.)

#include "small_kernels.h"

namespace hsma {

using namespace smallk;

namespace {

template <bool UNIT>
void small_launch(int nch, dim3 grid, const SmallItem &one, const SmallGroup &grp, hipStream_t s) {
    switch (nch) {
#define HSMA_CASE(N)                                                                               \
    case N:                                                                                        \
        hipLaunchKernelGGL((hsma_small_solve<false, N, UNIT>), grid, dim3(64), 0, s, one, grp);   \
        break;
        HSMA_CASE(1) HSMA_CASE(2) HSMA_CASE(3) HSMA_CASE(4)
        HSMA_CASE(5) HSMA_CASE(6) HSMA_CASE(7) HSMA_CASE(8)
#undef HSMA_CASE
        default:
            break;
    }
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

template <bool UNIT>
hsma_status inv_group_t(int base, const void *items, int count, hipStream_t s) {
    const InvItem *it = static_cast<const InvItem *>(items);
    switch (base / 8) {
#define HSMA_CASE(N)                                                                              \
    case N:                                                                                       \
        hipLaunchKernelGGL((hsma_diag_inv_group<false, N, UNIT>), dim3((unsigned)count), dim3(64), \
                           0, s, it);                                                             \
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

// Grouped diagonal-chunk inversion: `count` InvItems (device memory), all
// with chunk bound `base` (8, 16, 32 or 64).
hsma_status launch_inv_group_d(bool unit, int base, const void *items, int count, hipStream_t s) {
    if (count <= 0) return HSMA_SUCCESS;
    return unit ? inv_group_t<true>(base, items, count, s) : inv_group_t<false>(base, items, count, s);
}

size_t inv_item_bytes_d() { return sizeof(InvItem); }

hsma_status launch_small_d(bool unit, int m, int64_t n, cplx alpha, const double *A,
                              int64_t lda, double *B, int64_t ldb, hipStream_t s) {
    const int64_t panels = (n + 63) / 64;
    if (panels > 0x7fffffff || n > 0x7fffffff) return HSMA_INVALID_SIZE;
    SmallItem one{A, B, lda, ldb, m, (int32_t)n, alpha.re, alpha.im};
    SmallGroup none{nullptr, 0};
    const int nch = (m + 7) / 8;
    if (nch < 1 || nch > 8) return HSMA_INVALID_SIZE;
    if (unit) small_launch<true>(nch, dim3((unsigned)panels), one, none, s);
    else small_launch<false>(nch, dim3((unsigned)panels), one, none, s);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

// Grouped launch over `grp` (device table): one workgroup per item.
hsma_status launch_small_group_d(bool unit, int nch, const void *grp_items, int count,
                                    hipStream_t s) {
    SmallItem one{};
    SmallGroup grp{static_cast<const SmallItem *>(grp_items), count};
    if (nch < 1 || nch > 8 || count < 1) return HSMA_INVALID_SIZE;
    if (unit) small_launch<true>(nch, dim3((unsigned)count), one, grp, s);
    else small_launch<false>(nch, dim3((unsigned)count), one, grp, s);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

hsma_status launch_inv_base_d(bool unit, int m, int base, int ib, const double *A,
                                 int64_t lda, double *W, hipStream_t s) {
    return unit ? inv_t<true>(m, base, ib, A, lda, W, s) : inv_t<false>(m, base, ib, A, lda, W, s);
}

size_t small_item_bytes_d() { return sizeof(SmallItem); }

}  // namespace hsma
