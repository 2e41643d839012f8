// Element-wise and reduction kernels used by iterative refinement and by the
// backward-error report (real or interleaved complex data):
//   R = alpha * B0           (scaled copy, the start of a residual)
//   X = X + D                (apply a correction; complex data is added as
//                             real data of twice the rows)
//   s_i = sum_j |M_ij|       (row sums of |.| -- the complex modulus for
//                             complex data -- for infinity norms; the
//                             triangular variant reads only the lower
//                             triangle and takes a unit diagonal as 1)

#include "internal.h"

namespace hsma {
namespace {

// One thread per (row, column-slab); rows are the fast index, so consecutive
// threads touch consecutive addresses of each column.
__global__ __launch_bounds__(256) void hsma_scale_copy(const double *__restrict__ S, int64_t lds,
                                                       double *__restrict__ D, int64_t ldd,
                                                       int64_t m, int64_t n, double alpha) {
    const int64_t total = m * n;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        const int64_t j = t / m, i = t - j * m;
        D[i + j * ldd] = alpha * S[i + j * lds];
    }
}

// Complex R = alpha * B0: (ar sr - ai si, ar si + ai sr) per element.
__global__ __launch_bounds__(256) void hsma_scale_copy_z(const double *__restrict__ S, int64_t lds,
                                                         double *__restrict__ D, int64_t ldd,
                                                         int64_t m, int64_t n, double ar, double ai) {
    const int64_t total = m * n;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        const int64_t j = t / m, i = t - j * m;
        const double sr = S[2 * (i + j * lds)], si = S[2 * (i + j * lds) + 1];
        D[2 * (i + j * ldd)] = ar * sr - ai * si;
        D[2 * (i + j * ldd) + 1] = ar * si + ai * sr;
    }
}

__global__ __launch_bounds__(256) void hsma_axpy_inplace(const double *__restrict__ S, int64_t lds,
                                                         double *__restrict__ D, int64_t ldd,
                                                         int64_t m, int64_t n) {
    const int64_t total = m * n;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        const int64_t j = t / m, i = t - j * m;
        D[i + j * ldd] += S[i + j * lds];
    }
}

// Row sums of |M| in two passes.  Pass 1: block (x, s) sums columns
// [s*cs, (s+1)*cs) of 256 consecutive rows into partial[s*m + i] (each column
// read coalesced across the block's threads).  Pass 2 adds the slabs of each
// row in slab order, so the result does not depend on scheduling.
// tri: 0 general m x n; 1 lower non-unit (n = m); 2 lower unit.
template <bool CX>
__device__ __forceinline__ double abs_at(const double *__restrict__ M, int64_t idx) {
    if (CX) return hypot(M[2 * idx], M[2 * idx + 1]);
    return fabs(M[idx]);
}

template <bool CX>
__global__ __launch_bounds__(256) void hsma_rowsum_abs_slab(const double *__restrict__ M,
                                                            int64_t ld, int64_t m, int64_t n,
                                                            int tri, int64_t cs,
                                                            double *__restrict__ partial) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t s = blockIdx.y;
    if (i >= m) return;
    const int64_t j0 = s * cs;
    int64_t j1 = j0 + cs < n ? j0 + cs : n;
    double acc = 0.0;
    if (tri) {
        const int64_t jl = i < j1 ? i : j1;  // strictly lower part in this slab
        for (int64_t j = j0; j < jl; ++j) acc += abs_at<CX>(M, i + j * ld);
        if (i >= j0 && i < j1) acc += (tri == 1) ? abs_at<CX>(M, i + i * ld) : 1.0;
    } else {
        for (int64_t j = j0; j < j1; ++j) acc += abs_at<CX>(M, i + j * ld);
    }
    partial[s * m + i] = acc;
}

__global__ __launch_bounds__(256) void hsma_rowsum_join(const double *__restrict__ partial,
                                                        int64_t m, int64_t slabs,
                                                        double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double acc = 0.0;
    for (int64_t s = 0; s < slabs; ++s) acc += partial[s * m + i];
    out[i] = acc;
}

unsigned grid_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hsma_status launch_scale_copy(bool cx, const double *S, int64_t lds, double *D, int64_t ldd,
                              int64_t m, int64_t n, cplx alpha, hipStream_t s) {
    if (m <= 0 || n <= 0) return HSMA_SUCCESS;
    ProfScope prof(HSMA_PHASE_OTHER, 0.0, s);
    if (cx)
        hipLaunchKernelGGL(hsma_scale_copy_z, dim3(grid_for(m * n)), dim3(256), 0, s, S, lds, D, ldd,
                           m, n, alpha.re, alpha.im);
    else
        hipLaunchKernelGGL(hsma_scale_copy, dim3(grid_for(m * n)), dim3(256), 0, s, S, lds, D, ldd,
                           m, n, alpha.re);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

hsma_status launch_axpy(bool cx, const double *S, int64_t lds, double *D, int64_t ldd, int64_t m,
                        int64_t n, hipStream_t s) {
    if (m <= 0 || n <= 0) return HSMA_SUCCESS;
    const int es = cx ? 2 : 1;
    ProfScope prof(HSMA_PHASE_OTHER, 0.0, s);
    hipLaunchKernelGGL(hsma_axpy_inplace, dim3(grid_for(es * m * n)), dim3(256), 0, s, S, es * lds,
                       D, es * ldd, es * m, n);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

// Slabs used by launch_rowsum_abs for an n-column matrix (partial needs
// rowsum_slabs(n) * m doubles).
int64_t rowsum_slabs(int64_t n) {
    const int64_t cs = 64;
    int64_t sl = (n + cs - 1) / cs;
    return sl > 64 ? 64 : (sl < 1 ? 1 : sl);
}

hsma_status launch_rowsum_abs(bool cx, const double *M, int64_t ld, int64_t m, int64_t n, int tri,
                              double *out, double *partial, hipStream_t s) {
    if (m <= 0) return HSMA_SUCCESS;
    const int64_t slabs = rowsum_slabs(n);
    const int64_t cs = (n + slabs - 1) / slabs;
    ProfScope prof(HSMA_PHASE_OTHER, 0.0, s);
    if (cx)
        hipLaunchKernelGGL(hsma_rowsum_abs_slab<true>, dim3((unsigned)((m + 255) / 256), (unsigned)slabs),
                           dim3(256), 0, s, M, ld, m, n, tri, cs > 0 ? cs : 1, partial);
    else
        hipLaunchKernelGGL(hsma_rowsum_abs_slab<false>, dim3((unsigned)((m + 255) / 256), (unsigned)slabs),
                           dim3(256), 0, s, M, ld, m, n, tri, cs > 0 ? cs : 1, partial);
    hipLaunchKernelGGL(hsma_rowsum_join, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, partial,
                       m, slabs, out);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

}  // namespace hsma
