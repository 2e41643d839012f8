// Synthetic request inputs generated on the device (serving load generator).
//
// A request of the synthetic kind carries a 64-bit key instead of data; its
// L and B are drawn here, in device memory the server allocated, so inputs
// never cross PCIe.  Numbers come from the counter-based generator
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): element e of matrix t (0 = L, 1 = B) uses
// counter (e mod 2^32, e div 2^32, t, 0) and key (key mod 2^32, key div 2^32);
// the four 32-bit outputs x0..x3 give two uniforms on [0, 1) with 53 bits,
//   u1 = ((x1 << 32 | x0) >> 11) 2^-53,  u2 = ((x3 << 32 | x2) >> 11) 2^-53.
// Distribution (the standard workload): strict lower L = (2 u1 - 1)/m (complex:
// imaginary part (2 u2 - 1)/m), diagonal 1 + u1 (complex: imaginary u2 - 1/2),
// upper triangle 0; B = sqrt(-2 ln(1 - u1)) cos(2 pi u2) (complex: imaginary
// part with sin).  Column-major, lda = ldb = m.

#include <vector>

#include "internal.h"

namespace hsma {
namespace {

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
        const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
        k0 += W0;
        k1 += W1;
    }
}

__device__ __forceinline__ void uniforms(uint64_t e, uint32_t tag, uint64_t key, double *u1,
                                         double *u2) {
    uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), tag, 0u};
    philox4x32_10(c, (uint32_t)key, (uint32_t)(key >> 32));
    const uint64_t a = ((uint64_t)c[1] << 32) | c[0];
    const uint64_t b = ((uint64_t)c[3] << 32) | c[2];
    *u1 = (double)(a >> 11) * 0x1.0p-53;
    *u2 = (double)(b >> 11) * 0x1.0p-53;
}

// L element (i, j), column-major index t = i + j m.
__device__ __forceinline__ void gen_l(int cx, int64_t m, uint64_t key, double *__restrict__ L,
                                      int64_t i, int64_t j) {
    const int64_t t = i + j * m;
    if (i < j) {  // upper triangle: zero, no draw needed
        if (cx) {
            L[2 * t] = 0.0;
            L[2 * t + 1] = 0.0;
        } else {
            L[t] = 0.0;
        }
        return;
    }
    double u1, u2;
    uniforms((uint64_t)t, 0u, key, &u1, &u2);
    double re, im;
    if (i > j) {
        re = (2.0 * u1 - 1.0) / (double)m;
        im = (2.0 * u2 - 1.0) / (double)m;
    } else if (i == j) {
        re = 1.0 + u1;
        im = u2 - 0.5;
    } else {
        re = im = 0.0;
    }
    if (cx) {
        L[2 * t] = re;
        L[2 * t + 1] = im;
    } else {
        L[t] = re;
    }
}

// B element with column-major index e.
__device__ __forceinline__ void gen_b(int cx, uint64_t key, double *__restrict__ B, int64_t e) {
    double u1, u2;
    uniforms((uint64_t)e, 1u, key, &u1, &u2);
    const double r = sqrt(-2.0 * log(1.0 - u1));
    const double th = 6.283185307179586 * u2;
    if (cx) {
        B[2 * e] = r * cos(th);
        B[2 * e + 1] = r * sin(th);
    } else {
        B[e] = r * cos(th);
    }
}

__global__ __launch_bounds__(256) void hsma_gen_inputs(int cx, int64_t m, int64_t n, uint64_t key,
                                                       double *__restrict__ L,
                                                       double *__restrict__ B) {
    const int64_t nl = m * m, total = nl + m * n;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        if (t < nl) {
            const int64_t j = t / m;
            gen_l(cx, m, key, L, t - j * m, j);
        } else {
            gen_b(cx, key, B, t - nl);
        }
    }
}

// Many requests in one launch: workgroup b fills columns [j0, j1) of L
// (which = 0) or of B (which = 1) of the request items[b] describes; the
// threads walk the rows of each column, so no index division is needed.
struct GenItem {
    double *L, *B;
    int64_t m;
    uint64_t key;
    int64_t j0, j1;
    int32_t cx, which;
};

__global__ __launch_bounds__(256) void hsma_gen_group(const GenItem *__restrict__ items) {
    const GenItem it = items[blockIdx.x];
    for (int64_t j = it.j0; j < it.j1; ++j) {
        if (it.which == 0) {
            for (int64_t i = threadIdx.x; i < it.m; i += 256) gen_l(it.cx, it.m, it.key, it.L, i, j);
        } else {
            for (int64_t i = threadIdx.x; i < it.m; i += 256) gen_b(it.cx, it.key, it.B, i + j * it.m);
        }
    }
}

constexpr int64_t kGenChunk = 256 * 32;  // elements per workgroup of a grouped launch

}  // namespace

hsma_status launch_gen_inputs(bool cx, int64_t m, int64_t n, uint64_t key, double *L, double *B,
                              hipStream_t s) {
    const int64_t total = m * m + m * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) return HSMA_SUCCESS;
    ProfScope prof(HSMA_PHASE_OTHER, 0.0, s);
    hipLaunchKernelGGL(hsma_gen_inputs, dim3((unsigned)blocks), dim3(256), 0, s, cx ? 1 : 0, m, n,
                       key, L, B);
    HSMA_HIP(hipGetLastError());
    return HSMA_SUCCESS;
}

hsma_status upload_async(const void *host, size_t bytes, void *dev, hipStream_t s);

// Fill the inputs of many synthetic requests with one launch on s.
hsma_status gen_inputs_grouped(const GenRequest *reqs, int count, hipStream_t s) {
    std::vector<GenItem> items;
    for (int i = 0; i < count; ++i) {
        const GenRequest &r = reqs[i];
        if (r.m <= 0) continue;
        const int64_t cols = kGenChunk / r.m > 1 ? kGenChunk / r.m : 1;
        for (int which = 0; which < 2; ++which) {
            const int64_t nc = which == 0 ? r.m : r.n;
            for (int64_t j0 = 0; j0 < nc; j0 += cols) {
                GenItem it;
                it.L = r.L;
                it.B = r.B;
                it.m = r.m;
                it.key = r.key;
                it.j0 = j0;
                it.j1 = j0 + cols < nc ? j0 + cols : nc;
                it.cx = r.cx ? 1 : 0;
                it.which = which;
                items.push_back(it);
            }
        }
    }
    if (items.empty()) return HSMA_SUCCESS;
    if (items.size() > 0x7fffffff) return HSMA_INVALID_SIZE;
    void *dev = nullptr;
    const size_t bytes = items.size() * sizeof(GenItem);
    HSMA_TRY(ws_alloc(&dev, bytes, s));
    hsma_status st = upload_async(items.data(), bytes, dev, s);
    if (st == HSMA_SUCCESS) {
        ProfScope prof(HSMA_PHASE_OTHER, 0.0, s);
        hipLaunchKernelGGL(hsma_gen_group, dim3((unsigned)items.size()), dim3(256), 0, s,
                           static_cast<const GenItem *>(dev));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = hip_fail(e);
    }
    const hsma_status st2 = ws_free(dev, s);
    return st != HSMA_SUCCESS ? st : st2;
}

}  // namespace hsma

// Standalone entry (tests, load generators): fill caller buffers the same way.
extern "C" hsma_status hsma_generate_inputs(hsma_dtype dtype, int64_t m, int64_t n, uint64_t key,
                                            void *L, void *B, hsma_stream_t stream) {
    if (dtype != HSMA_R64F && dtype != HSMA_C64F) return HSMA_INVALID_VALUE;
    if (m < 0 || n < 0) return HSMA_INVALID_SIZE;
    if (m == 0) return HSMA_SUCCESS;
    if (!L || (n > 0 && !B)) return HSMA_INVALID_POINTER;
    return hsma::launch_gen_inputs(dtype == HSMA_C64F, m, n, key, static_cast<double *>(L),
                                   static_cast<double *>(B), static_cast<hipStream_t>(stream));
}
