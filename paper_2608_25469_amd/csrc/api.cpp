// C ABI entry points: validation, path selection, workspace, errors.

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "internal.h"
#include "tuning_gfx950.h"

namespace hsma {

size_t blocked_workspace_bytes(bool cx, int64_t m, int ib);
hsma_status blocked_trsm(bool cx, bool unit, int64_t m, int64_t n, cplx alpha, const double *A,
                         int64_t lda, double *B, int64_t ldb, int ib, void *ws, hipStream_t s);

namespace {
thread_local int g_last_hip_error = 0;
std::mutex g_dev_mutex;
DeviceInfo g_dev[64];
}  // namespace

hsma_status hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    (void)hipGetLastError();  // clear the sticky-free error state for this thread
    return HSMA_HIP_ERROR;
}

hsma_status device_info(DeviceInfo *out) {
    int dev = 0;
    HSMA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return HSMA_NOT_SUPPORTED;
    std::lock_guard<std::mutex> lk(g_dev_mutex);
    DeviceInfo &d = g_dev[dev];
    if (d.device < 0) {
        hipDeviceProp_t prop;
        HSMA_HIP(hipGetDeviceProperties(&prop, dev));
        d.num_cus = prop.multiProcessorCount;
        d.arch_ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        // Keep freed workspace in the pool: stream-ordered allocations then
        // cost no driver round trip after the first call.
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        d.device = dev;
    }
    *out = d;
    return HSMA_SUCCESS;
}

hsma_status ws_alloc(void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) return HSMA_SUCCESS;
    hipError_t e = hipMallocAsync(p, bytes, s);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return HSMA_ALLOC_FAILED;
    }
    HSMA_HIP(e);
    return HSMA_SUCCESS;
}

hsma_status ws_free(void *p, hipStream_t s) {
    if (p) HSMA_HIP(hipFreeAsync(p, s));
    return HSMA_SUCCESS;
}

// Nearest tested scale in log2(m), then log2(n); ties go to the smaller scale.
int lookup_block_size(bool cx, int64_t m, int64_t n) {
    const int dt = cx ? 1 : 0;
    double best_dm = 1e300, best_dn = 1e300;
    int best_m = 0, best_n = 0, best = 128;
    const double lm = std::log2((double)std::max<int64_t>(m, 1));
    const double ln = std::log2((double)std::max<int64_t>(n, 1));
    for (const auto &e : tuning::kTable) {
        if (e.dtype != dt) continue;
        const double dm = std::fabs(std::log2((double)e.m) - lm);
        const double dn = std::fabs(std::log2((double)e.n) - ln);
        bool take = false;
        if (dm < best_dm - 1e-12) take = true;
        else if (std::fabs(dm - best_dm) <= 1e-12) {
            if (dn < best_dn - 1e-12) take = true;
            else if (std::fabs(dn - best_dn) <= 1e-12 &&
                     (e.m < best_m || (e.m == best_m && e.n < best_n)))
                take = true;
        }
        if (take) {
            best_dm = dm;
            best_dn = dn;
            best_m = e.m;
            best_n = e.n;
            best = e.ib;
        }
    }
    return best;
}

bool valid_block_size(bool cx, int ib) {
    (void)cx;
    return ib == 16 || ib == 32 || ib == 64 || ib == 128 || ib == 256;
}

// Argument checks in the documented order; nothing touches the device.
hsma_status validate(int diag, int dtype, int64_t m, int64_t n, const void *alpha, const void *A,
                     int64_t lda, const void *B, int64_t ldb, bool *quick) {
    *quick = false;
    if ((diag != HSMA_NON_UNIT && diag != HSMA_UNIT) || (dtype != HSMA_R64F && dtype != HSMA_C64F))
        return HSMA_INVALID_VALUE;
    if (m < 0 || n < 0) return HSMA_INVALID_SIZE;
    const int64_t lo = m > 1 ? m : 1;
    if (lda < lo || ldb < lo) return HSMA_INVALID_SIZE;
    if (m == 0 || n == 0) {
        *quick = true;
        return HSMA_SUCCESS;
    }
    if (!alpha) return HSMA_INVALID_POINTER;
    const double *a = static_cast<const double *>(alpha);
    const bool azero = (a[0] == 0.0) && (dtype == HSMA_R64F || a[1] == 0.0);
    if (!B || (!A && !azero)) return HSMA_INVALID_POINTER;
    // Largest index must fit the kernels' 64-bit arithmetic and int grids.
    if (m > (int64_t)1 << 30 || n > (int64_t)1 << 40) return HSMA_INVALID_SIZE;
    return HSMA_SUCCESS;
}

hsma_status trsm_impl(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                      int64_t lda, void *B, int64_t ldb, hsma_dtype dtype, int ib_override,
                      int path, hipStream_t s, int *path_used, int *ib_used) {
    bool quick = false;
    HSMA_TRY(validate(diag, dtype, m, n, alpha, A, lda, B, ldb, &quick));
    if (path_used) *path_used = 0;
    if (ib_used) *ib_used = 0;
    if (quick) return HSMA_SUCCESS;
    const bool cx = dtype == HSMA_C64F;
    const bool unit = diag == HSMA_UNIT;
    const double *a = static_cast<const double *>(alpha);
    const cplx al{a[0], cx ? a[1] : 0.0};
    DeviceInfo dev;
    HSMA_TRY(device_info(&dev));
    if (!dev.arch_ok) return HSMA_NOT_SUPPORTED;
    double *Bd = static_cast<double *>(B);
    const double *Ad = static_cast<const double *>(A);
    if (al.re == 0.0 && al.im == 0.0) return launch_zero(m, n, cx ? 2 : 1, Bd, ldb, s);

    const bool small_ok = m <= 64;
    const bool use_small = (path == 1) ? true : (path == 2 ? false : small_ok);
    if (use_small) {
        if (!small_ok) return HSMA_NOT_SUPPORTED;
        if (path_used) *path_used = 1;
        return launch_small_solve(cx, unit, (int)m, n, al, Ad, lda, Bd, ldb, s);
    }
    int ib = ib_override > 0 ? ib_override : lookup_block_size(cx, m, n);
    if (!valid_block_size(cx, ib)) return HSMA_INVALID_VALUE;
    if (path_used) *path_used = 2;
    if (ib_used) *ib_used = ib;
    void *ws = nullptr;
    HSMA_TRY(ws_alloc(&ws, blocked_workspace_bytes(cx, m, ib), s));
    hsma_status st = blocked_trsm(cx, unit, m, n, al, Ad, lda, Bd, ldb, ib, ws, s);
    hsma_status st2 = ws_free(ws, s);
    return st != HSMA_SUCCESS ? st : st2;
}

}  // namespace hsma

extern "C" {

const char *hsma_status_string(hsma_status s) {
    switch (s) {
        case HSMA_SUCCESS: return "success";
        case HSMA_INVALID_VALUE: return "invalid enumerator value";
        case HSMA_INVALID_SIZE: return "invalid size or leading dimension";
        case HSMA_INVALID_POINTER: return "invalid (null) pointer";
        case HSMA_ALLOC_FAILED: return "device allocation failed";
        case HSMA_HIP_ERROR: return "HIP runtime error";
        case HSMA_NOT_SUPPORTED: return "not supported on this device or path";
        case HSMA_TOO_LARGE: return "request larger than the memory budget";
        case HSMA_QUEUE_CLOSED: return "queue closed";
        case HSMA_PENDING: return "pending";
        case HSMA_TIMEOUT: return "timed out";
        case HSMA_NOT_FOUND: return "not found";
    }
    return "unknown status";
}

int hsma_last_hip_error(void) { return hsma::g_last_hip_error; }

const char *hsma_version(void) { return "0.1.0 gfx950"; }

hsma_status hsma_trsm(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                      int64_t lda, void *B, int64_t ldb, hsma_dtype dtype, hsma_stream_t stream) {
    return hsma::trsm_impl(diag, m, n, alpha, A, lda, B, ldb, dtype, 0, 0,
                           static_cast<hipStream_t>(stream), nullptr, nullptr);
}

hsma_status hsma_trsm_ex(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                         int64_t lda, void *B, int64_t ldb, hsma_dtype dtype,
                         const hsma_trsm_options *opts, hsma_trsm_report *report,
                         hsma_stream_t stream) {
    hsma_trsm_options o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (report) std::memset(report, 0, sizeof(*report));
    for (int i = 0; i < 6; ++i)
        if (o.reserved[i] != 0) return HSMA_INVALID_VALUE;
    if (o.path < 0 || o.path > 2) return HSMA_INVALID_VALUE;
    if (o.block_size != 0 && !hsma::valid_block_size(dtype == HSMA_C64F, o.block_size))
        return HSMA_INVALID_VALUE;
    int path_used = 0, ib_used = 0;
    hsma_status st = hsma::trsm_impl(diag, m, n, alpha, A, lda, B, ldb, dtype, o.block_size, o.path,
                                     static_cast<hipStream_t>(stream), &path_used, &ib_used);
    if (report) {
        report->path = path_used;
        report->block_size = ib_used;
    }
    return st;
}

int32_t hsma_lookup_block_size(hsma_dtype dtype, int64_t m, int64_t n) {
    return hsma::lookup_block_size(dtype == HSMA_C64F, m, n);
}

}  // extern "C"
