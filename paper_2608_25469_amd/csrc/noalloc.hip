// hsma_trsm_noalloc: the operation of hsma_trsm for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The only device memory hsma_trsm takes beyond its inputs and outputs is the
// blocked path's workspace: the inverted diagonal blocks W and the merge
// scratch T.  Here that workspace is a file-scope device array of fixed size,
// `scratch`, one copy per GPU that the library runs on, held until the
// process ends.  Its device address is looked up once per device with
// hipGetSymbolAddress (the array's name is a host-side stand-in in host code,
// never a device address) and passed to the same kernels hsma_trsm launches,
// in the same schedule, so the results are bit-for-bit those of hsma_trsm.
// The blocked path initialises all of the workspace it reads (W's blocks are
// zero-filled by a kernel before the inversion writes them; T is written
// before it is read), so nothing depends on what an earlier call left there.
// Calls that overlap in time on one GPU share the array and race.

#include <mutex>

#include "internal.h"

namespace hsma {

size_t blocked_workspace_bytes(bool cx, int64_t m, int ib);
hsma_status blocked_trsm(bool cx, bool unit, int64_t m, int64_t n, cplx alpha, const double *A,
                         int64_t lda, double *B, int64_t ldb, int ib, void *ws, hipStream_t s,
                         bool mixed);
int lookup_block_size(bool cx, int64_t m, int64_t n);

namespace {

constexpr size_t kScratchBytes = (size_t)HSMA_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[64] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call on each device, with that device current).
hsma_status scratch_address(void **out) {
    int dev = 0;
    HSMA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return HSMA_NOT_SUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!p) return HSMA_HIP_ERROR;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return HSMA_SUCCESS;
}

}  // namespace
}  // namespace hsma

extern "C" hsma_status hsma_trsm_noalloc(hsma_diag diag, int64_t m, int64_t n, const void *alpha,
                                         const void *A, int64_t lda, void *B, int64_t ldb,
                                         hsma_dtype dtype, hsma_stream_t stream) {
    using namespace hsma;
    bool quick = false;
    HSMA_TRY(validate(diag, dtype, m, n, alpha, A, lda, B, ldb, &quick));
    if (quick) return HSMA_SUCCESS;
    const bool cx = dtype == HSMA_C64F;
    const double *a = static_cast<const double *>(alpha);
    const cplx al{a[0], cx ? a[1] : 0.0};
    const bool azero = al.re == 0.0 && al.im == 0.0;
    const int ib = (m > 64 && !azero) ? lookup_block_size(cx, m, n) : 0;
    // Size check before any device call.
    if (ib && blocked_workspace_bytes(cx, m, ib) > kScratchBytes) return HSMA_WORKSPACE_TOO_SMALL;
    DeviceInfo dev;
    HSMA_TRY(device_info(&dev));
    if (!dev.arch_ok) return HSMA_NOT_SUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *Bd = static_cast<double *>(B);
    const double *Ad = static_cast<const double *>(A);
    if (azero) return launch_zero(m, n, cx ? 2 : 1, Bd, ldb, s);
    if (m <= 64) return launch_small_solve(cx, diag == HSMA_UNIT, (int)m, n, al, Ad, lda, Bd, ldb, s);
    void *ws = nullptr;
    HSMA_TRY(scratch_address(&ws));
    return blocked_trsm(cx, diag == HSMA_UNIT, m, n, al, Ad, lda, Bd, ldb, ib, ws, s, false);
}

extern "C" uint64_t hsma_noalloc_scratch_bytes(void) { return (uint64_t)hsma::kScratchBytes; }
