// Matrix-core peak probes: the FP64 (v_mfma_f64_16x16x4_f64) and FP32
// (v_mfma_f32_16x16x4_f32) rates this GPU sustains on register operands,
// measured next to the datasheet peaks that the benchmark's roofline
// fractions use.  Every wavefront runs independent accumulator chains (enough
// of them to cover the instruction latency) for a fixed number of
// iterations; the grid fills every CU several times over.  The accumulators
// are reduced into one store per lane so the work cannot be removed.  The
// first wavefront also reads the shader clock counter and the constant-rate
// wall clock around its loop, which gives the clock the CUs ran at.

#include <chrono>

#include "internal.h"

namespace hsma {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int kChains64 = 8;   // FP64 chains: enough to cover that instruction's latency
constexpr int kChains32 = 16;  // FP32 issues twice as fast, so twice the chains in flight
constexpr int kUnroll = 32;  // iterations per loop trip (iters is rounded down to a multiple); the
                             // compiler copies FP64 accumulators across the loop back-edge, so
                             // long trips keep those copies a few percent of the issue slots

// sink[0..1] <- shader cycles and wall-clock ticks of the first wavefront's
// loop; every thread then writes its reduction at 2 + its index.
__global__ __launch_bounds__(256) void hsma_peak_f64(int64_t iters, double *__restrict__ sink) {
    const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * blockIdx.x;
    dbl4 acc[kChains64];
#pragma unroll
    for (int c = 0; c < kChains64; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
    const uint64_t c0 = clock64(), w0 = wall_clock64();
    const int outer = (int)(iters / kUnroll);
    for (int it = 0; it < outer; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kChains64; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    const uint64_t c1 = clock64(), w1 = wall_clock64();
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains64; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sink[0] = (double)(c1 - c0);
        sink[1] = (double)(w1 - w0);
    }
    sink[2 + (int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void hsma_peak_f32(int64_t iters, double *__restrict__ sink) {
    const float a = 1.0f + 1e-6f * threadIdx.x, b = 1.0f - 1e-6f * blockIdx.x;
    flt4 acc[kChains32];
#pragma unroll
    for (int c = 0; c < kChains32; ++c) acc[c] = flt4{0.f, 0.f, 0.f, 0.f};
    const uint64_t c0 = clock64(), w0 = wall_clock64();
    const int outer = (int)(iters / kUnroll);
    for (int it = 0; it < outer; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kChains32; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    }
    const uint64_t c1 = clock64(), w1 = wall_clock64();
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains32; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sink[0] = (double)(c1 - c0);
        sink[1] = (double)(w1 - w0);
    }
    sink[2 + (int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace
}  // namespace hsma

extern "C" hsma_status hsma_mfma_peak(int32_t fp32, int64_t iters, double *tflops,
                                      double *shader_ghz) {
    using namespace hsma;
    if (!tflops) return HSMA_INVALID_POINTER;
    if (iters < kUnroll || iters > ((int64_t)1 << 24)) return HSMA_INVALID_SIZE;
    DeviceInfo dev;
    HSMA_TRY(device_info(&dev));
    int dev_id = 0, wall_khz = 0;
    HSMA_HIP(hipGetDevice(&dev_id));
    HSMA_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev_id));
    const int blocks = 8 * (dev.num_cus > 0 ? dev.num_cus : 256);  // 4 waves each, 32 per CU
    void *sink = nullptr;
    HSMA_TRY(ws_alloc(&sink, ((size_t)blocks * 256 + 2) * sizeof(double), nullptr));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hsma_status st = HSMA_SUCCESS;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he == hipSuccess) {
        // one warm launch, then the timed one
        for (int rep = 0; rep < 2 && he == hipSuccess; ++rep) {
            if (rep == 1) he = hipEventRecord(e0, nullptr);
            if (fp32) hipLaunchKernelGGL(hsma_peak_f32, dim3(blocks), dim3(256), 0, nullptr, iters,
                                         static_cast<double *>(sink));
            else hipLaunchKernelGGL(hsma_peak_f64, dim3(blocks), dim3(256), 0, nullptr, iters,
                                    static_cast<double *>(sink));
            if (he == hipSuccess) he = hipGetLastError();
        }
        if (he == hipSuccess) he = hipEventRecord(e1, nullptr);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        double clk[2] = {0.0, 0.0};
        if (he == hipSuccess) he = hipMemcpy(clk, sink, sizeof(clk), hipMemcpyDeviceToHost);
        if (he == hipSuccess) {
            // 16 x 16 x 4 multiply-adds = 2048 flops per instruction per wavefront
            const double flops = 2048.0 * (fp32 ? kChains32 : kChains64) * (double)(iters / kUnroll * kUnroll) * blocks * 4;
            *tflops = flops / (ms * 1e-3) / 1e12;
            if (shader_ghz)
                *shader_ghz = (clk[1] > 0 && wall_khz > 0) ? clk[0] / (clk[1] / (wall_khz * 1e3)) / 1e9 : 0.0;
        }
    }
    if (he != hipSuccess) st = hip_fail(he);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    hsma_status st2 = ws_free(sink, nullptr);
    return st != HSMA_SUCCESS ? st : st2;
}
