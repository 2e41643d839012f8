// Diagonal-chunk inversion launchers (phase 1 of the blocked path), real and
// complex double: one wavefront per chunk of at most `base` rows, each lane
// solving D x = e_j in registers (the right-looking Panel walk).

#include "small_kernels.h"

namespace hsma {

using namespace smallk;

namespace {

template <bool CX, bool UNIT>
hsma_status inv_t(int m, int base, int ib, const double *A, int64_t lda, double *W, hipStream_t s) {
    dim3 grid((m + base - 1) / base), block(64);
    switch (base / 8) {
#define HSMA_CASE(N)                                                                             \
    case N:                                                                                      \
        hipLaunchKernelGGL((hsma_diag_inv_base<CX, N, UNIT>), grid, block, 0, s, A, lda, W, m,   \
                           base, ib);                                                            \
        break;
        HSMA_CASE(1) HSMA_CASE(2) HSMA_CASE(4) HSMA_CASE(8)
#undef HSMA_CASE
        default:
            return HSMA_INVALID_SIZE;
    }
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

template <bool CX, bool UNIT>
hsma_status inv_group_t(int base, const void *items, int count, hipStream_t s) {
    const InvItem *it = static_cast<const InvItem *>(items);
    switch (base / 8) {
#define HSMA_CASE(N)                                                                              \
    case N:                                                                                       \
        hipLaunchKernelGGL((hsma_diag_inv_group<CX, N, UNIT>), dim3((unsigned)count), dim3(64),   \
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

// Chunks of `base` rows (8, 16, 32 or 64) down the diagonal of one matrix.
hsma_status launch_inv_base(bool cx, bool unit, int m, int base, int ib, const double *A,
                            int64_t lda, double *W, hipStream_t s) {
    if (cx) return unit ? inv_t<true, true>(m, base, ib, A, lda, W, s) : inv_t<true, false>(m, base, ib, A, lda, W, s);
    return unit ? inv_t<false, true>(m, base, ib, A, lda, W, s) : inv_t<false, false>(m, base, ib, A, lda, W, s);
}

// Grouped diagonal-chunk inversion: `count` InvItems (device memory), all
// with chunk bound `base`.
hsma_status launch_inv_group(bool cx, bool unit, int base, const void *items, int count, hipStream_t s) {
    if (count <= 0) return HSMA_SUCCESS;
    if (cx) return unit ? inv_group_t<true, true>(base, items, count, s) : inv_group_t<true, false>(base, items, count, s);
    return unit ? inv_group_t<false, true>(base, items, count, s) : inv_group_t<false, false>(base, items, count, s);
}

size_t inv_item_bytes() { return sizeof(InvItem); }


}  // namespace hsma
