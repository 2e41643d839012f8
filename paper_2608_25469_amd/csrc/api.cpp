// C ABI entry points: validation, path selection, workspace, errors.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "internal.h"
#include "tuning_gfx950.h"

namespace hsma {

size_t blocked_workspace_bytes(bool cx, int64_t m, int ib);
size_t blocked_workspace_bytes32(bool cx, int64_t m, int ib);
hsma_status blocked_trsm32(bool cx, bool unit, int64_t m, int64_t n, cplx alpha, const float *A,
                           int64_t lda, float *B, int64_t ldb, int ib, void *ws, hipStream_t s);
hsma_status blocked_trsm(bool cx, bool unit, int64_t m, int64_t n, cplx alpha, const double *A,
                         int64_t lda, double *B, int64_t ldb, int ib, void *ws, hipStream_t s,
                         bool mixed);
hsma_status blocked_trsm_graph(bool cx, bool unit, int64_t m, int64_t n, cplx alpha,
                               const double *A, int64_t lda, double *B, int64_t ldb, int ib,
                               bool mixed, hipStream_t s);
hsma_status triangular_residual(bool cx, bool unit, int64_t m, int64_t n, const double *A,
                                int64_t lda, const double *X, int64_t ldx, double *R, int64_t ldr,
                                hipStream_t s);
hsma_status launch_scale_copy(bool cx, const double *S, int64_t lds, double *D, int64_t ldd,
                              int64_t m, int64_t n, cplx alpha, hipStream_t s);
hsma_status launch_axpy(bool cx, const double *S, int64_t lds, double *D, int64_t ldd, int64_t m,
                        int64_t n, hipStream_t s);
hsma_status launch_rowsum_abs(bool cx, const double *M, int64_t ld, int64_t m, int64_t n, int tri,
                              double *out, double *partial, hipStream_t s);
int64_t rowsum_slabs(int64_t n);

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

bool is_single(int dtype) { return dtype == HSMA_R32F || dtype == HSMA_C32F; }
bool is_complex(int dtype) { return dtype == HSMA_C64F || dtype == HSMA_C32F; }

// alpha as read from the caller's host scalar of the data type.
cplx read_alpha(int dtype, const void *alpha) {
    if (is_single(dtype)) {
        const float *a = static_cast<const float *>(alpha);
        return cplx{(double)a[0], dtype == HSMA_C32F ? (double)a[1] : 0.0};
    }
    const double *a = static_cast<const double *>(alpha);
    return cplx{a[0], dtype == HSMA_C64F ? a[1] : 0.0};
}

// Argument checks in the documented order; nothing touches the device.
// FP32 data types are accepted only where allow32 (else HSMA_NOT_SUPPORTED).
hsma_status validate(int diag, int dtype, int64_t m, int64_t n, const void *alpha, const void *A,
                     int64_t lda, const void *B, int64_t ldb, bool *quick, bool allow32) {
    *quick = false;
    if ((diag != HSMA_NON_UNIT && diag != HSMA_UNIT) ||
        (dtype != HSMA_R64F && dtype != HSMA_C64F && !is_single(dtype)))
        return HSMA_INVALID_VALUE;
    if (is_single(dtype) && !allow32) return HSMA_NOT_SUPPORTED;
    if (m < 0 || n < 0) return HSMA_INVALID_SIZE;
    const int64_t lo = m > 1 ? m : 1;
    if (lda < lo || ldb < lo) return HSMA_INVALID_SIZE;
    if (m == 0 || n == 0) {
        *quick = true;
        return HSMA_SUCCESS;
    }
    if (!alpha) return HSMA_INVALID_POINTER;
    const cplx a = read_alpha(dtype, alpha);
    const bool azero = a.re == 0.0 && a.im == 0.0;
    if (!B || (!A && !azero)) return HSMA_INVALID_POINTER;
    // Largest index must fit the kernels' 64-bit arithmetic and int grids.
    if (m > (int64_t)1 << 30 || n > (int64_t)1 << 40) return HSMA_INVALID_SIZE;
    return HSMA_SUCCESS;
}

// One solve in place (no refinement): small kernel or blocked path.
static hsma_status solve_once(bool cx, bool unit, int64_t m, int64_t n, cplx al, const double *Ad,
                              int64_t lda, double *Bd, int64_t ldb, int ib_override, int path,
                              bool mixed, hipStream_t s, int *path_used, int *ib_used,
                              bool use_graph = false) {
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
    if (use_graph) return blocked_trsm_graph(cx, unit, m, n, al, Ad, lda, Bd, ldb, ib, mixed, s);
    void *ws = nullptr;
    HSMA_TRY(ws_alloc(&ws, blocked_workspace_bytes(cx, m, ib), s));
    hsma_status st = blocked_trsm(cx, unit, m, n, al, Ad, lda, Bd, ldb, ib, ws, s, mixed);
    hsma_status st2 = ws_free(ws, s);
    return st != HSMA_SUCCESS ? st : st2;
}

// One FP32 solve in place (STRSM, CTRSM): small kernel or blocked path.
static hsma_status solve_once32(bool cx, bool unit, int64_t m, int64_t n, cplx al, const float *Ad,
                                int64_t lda, float *Bd, int64_t ldb, int ib_override, int path,
                                hipStream_t s, int *path_used, int *ib_used) {
    if (al.re == 0.0 && al.im == 0.0) return launch_zero32(m, n, cx ? 2 : 1, Bd, ldb, s);
    const bool small_ok = m <= 64;
    const bool use_small = (path == 1) ? true : (path == 2 ? false : small_ok);
    if (use_small) {
        if (!small_ok) return HSMA_NOT_SUPPORTED;
        if (path_used) *path_used = 1;
        return launch_small_solve(cx, unit, (int)m, n, al, Ad, lda, Bd, ldb, s);
    }
    // The I_B table is the FP64 one of the same kind (real or complex).
    int ib = ib_override > 0 ? ib_override : lookup_block_size(cx, m, n);
    if (!valid_block_size(cx, ib)) return HSMA_INVALID_VALUE;
    if (path_used) *path_used = 2;
    if (ib_used) *ib_used = ib;
    void *ws = nullptr;
    HSMA_TRY(ws_alloc(&ws, blocked_workspace_bytes32(cx, m, ib), s));
    hsma_status st = blocked_trsm32(cx, unit, m, n, al, Ad, lda, Bd, ldb, ib, ws, s);
    hsma_status st2 = ws_free(ws, s);
    return st != HSMA_SUCCESS ? st : st2;
}

// Normwise backward error from the residual R (on the device): max row sums
// of |R|, tril(L), X and B0 (complex modulus for complex data), combined on
// the host.
static hsma_status backward_error_host(bool cx, bool unit, int64_t m, int64_t n, cplx alpha,
                                       const double *Ad, int64_t lda, const double *X,
                                       int64_t ldx, const double *B0, int64_t ldb0,
                                       const double *R, int64_t ldr, double *sums, double *partial,
                                       double *lnorm, double *eta, hipStream_t s) {
    std::vector<double> h(3 * m);
    if (*lnorm < 0) {
        HSMA_TRY(launch_rowsum_abs(cx, Ad, lda, m, m, unit ? 2 : 1, sums, partial, s));
        std::vector<double> hl(m);
        HSMA_HIP(hipMemcpyAsync(hl.data(), sums, m * sizeof(double), hipMemcpyDeviceToHost, s));
        HSMA_HIP(hipStreamSynchronize(s));
        double mx = 0.0;
        for (double v : hl) mx = (v > mx || std::isnan(v)) ? v : mx;
        *lnorm = mx;
    }
    HSMA_TRY(launch_rowsum_abs(cx, R, ldr, m, n, 0, sums, partial, s));
    HSMA_TRY(launch_rowsum_abs(cx, X, ldx, m, n, 0, sums + m, partial, s));
    HSMA_TRY(launch_rowsum_abs(cx, B0, ldb0, m, n, 0, sums + 2 * m, partial, s));
    HSMA_HIP(hipMemcpyAsync(h.data(), sums, 3 * m * sizeof(double), hipMemcpyDeviceToHost, s));
    HSMA_HIP(hipStreamSynchronize(s));
    double r = 0, x = 0, b = 0;
    for (int64_t i = 0; i < m; ++i) {
        r = (h[i] > r || std::isnan(h[i])) ? h[i] : r;
        x = (h[m + i] > x || std::isnan(h[m + i])) ? h[m + i] : x;
        b = (h[2 * m + i] > b || std::isnan(h[2 * m + i])) ? h[2 * m + i] : b;
    }
    const double den = *lnorm * x + std::hypot(alpha.re, alpha.im) * b;
    *eta = den > 0 ? r / den : r;
    return HSMA_SUCCESS;
}

hsma_status trsm_impl(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                      int64_t lda, void *B, int64_t ldb, hsma_dtype dtype, int ib_override,
                      int path, hipStream_t s, int *path_used, int *ib_used,
                      const hsma_trsm_options *opt, hsma_trsm_report *rep) {
    bool quick = false;
    HSMA_TRY(validate(diag, dtype, m, n, alpha, A, lda, B, ldb, &quick, true));
    if (path_used) *path_used = 0;
    if (ib_used) *ib_used = 0;
    const bool cx = is_complex(dtype);
    const bool single = is_single(dtype);
    const bool mixed = opt && opt->precision == HSMA_PREC_MIXED;
    const int steps = opt ? opt->refine_steps : 0;
    const bool want_eta = opt && (opt->want_backward_error || opt->refine_steps < 0);
    if (mixed && cx) return HSMA_NOT_SUPPORTED;
    // FP32 data: plain solves only (no mixed mode, refinement, backward
    // error or graph replay).
    if (single && (mixed || steps != 0 || want_eta || (opt && opt->use_graph)))
        return HSMA_NOT_SUPPORTED;
    if (quick) {
        if (rep) rep->backward_error = want_eta ? 0.0 : -1.0;
        return HSMA_SUCCESS;
    }
    const bool unit = diag == HSMA_UNIT;
    const cplx al = read_alpha(dtype, alpha);
    DeviceInfo dev;
    HSMA_TRY(device_info(&dev));
    if (!dev.arch_ok) return HSMA_NOT_SUPPORTED;
    if (single)
        return solve_once32(cx, unit, m, n, al, static_cast<const float *>(A), lda,
                            static_cast<float *>(B), ldb, ib_override, path, s, path_used, ib_used);
    double *Bd = static_cast<double *>(B);
    const double *Ad = static_cast<const double *>(A);

    if (steps == 0 && !want_eta)
        return solve_once(cx, unit, m, n, al, Ad, lda, Bd, ldb, ib_override, path, mixed, s,
                          path_used, ib_used, opt && opt->use_graph == 1);

    // Refinement / backward error: keep B0, then iterate.
    const int es = cx ? 2 : 1;
    const double tol = (opt && opt->refine_tol > 0) ? opt->refine_tol : 1e-13;
    const int max_steps = steps < 0 ? 4 : steps;
    void *ws = nullptr;
    const size_t mn = (size_t)m * n * es;
    const size_t slabs = (size_t)std::max<int64_t>(rowsum_slabs(n), rowsum_slabs(m));
    HSMA_TRY(ws_alloc(&ws, (2 * mn + (3 + slabs) * (size_t)m) * sizeof(double), s));
    double *B0 = static_cast<double *>(ws);
    double *R = B0 + mn;
    double *sums = R + mn;
    double *partial = sums + 3 * m;
    hsma_status st = HSMA_SUCCESS;
    int used = 0;
    double eta = -1.0, lnorm = -1.0;
    const size_t col = (size_t)es * sizeof(double);
    if (hipMemcpy2DAsync(B0, m * col, Bd, ldb * col, m * col, n, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        st = hip_fail(hipGetLastError());
    if (st == HSMA_SUCCESS)
        st = solve_once(cx, unit, m, n, al, Ad, lda, Bd, ldb, ib_override, path, mixed, s,
                        path_used, ib_used);
    while (st == HSMA_SUCCESS) {
        const bool more = used < max_steps;
        if (!more && !want_eta) break;
        // R = alpha B0 - L X
        st = launch_scale_copy(cx, B0, m, R, m, m, n, al, s);
        if (st == HSMA_SUCCESS) st = triangular_residual(cx, unit, m, n, Ad, lda, Bd, ldb, R, m, s);
        if (st != HSMA_SUCCESS) break;
        if (want_eta) {
            st = backward_error_host(cx, unit, m, n, al, Ad, lda, Bd, ldb, B0, m, R, m, sums,
                                     partial, &lnorm, &eta, s);
            if (st != HSMA_SUCCESS) break;
            if (steps < 0 && eta <= tol) break;
        }
        if (!more) break;
        // L D = R, X += D
        st = solve_once(cx, unit, m, n, cplx{1.0, 0.0}, Ad, lda, R, m, ib_override, path, mixed, s,
                        nullptr, nullptr);
        if (st == HSMA_SUCCESS) st = launch_axpy(cx, R, m, Bd, ldb, m, n, s);
        if (st == HSMA_SUCCESS) ++used;
        if (!want_eta && used >= max_steps) break;
    }
    hsma_status st2 = ws_free(ws, s);
    if (rep) {
        rep->refine_steps = used;
        rep->backward_error = eta;
    }
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
        case HSMA_WORKSPACE_TOO_SMALL: return "problem needs more workspace than the fixed scratch array holds";
    }
    return "unknown status";
}

int hsma_last_hip_error(void) { return hsma::g_last_hip_error; }

const char *hsma_version(void) { return "0.1.0 gfx950"; }

hsma_status hsma_trsm(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                      int64_t lda, void *B, int64_t ldb, hsma_dtype dtype, hsma_stream_t stream) {
    return hsma::trsm_impl(diag, m, n, alpha, A, lda, B, ldb, dtype, 0, 0,
                           static_cast<hipStream_t>(stream), nullptr, nullptr, nullptr, nullptr);
}

hsma_status hsma_trsm_ex(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                         int64_t lda, void *B, int64_t ldb, hsma_dtype dtype,
                         const hsma_trsm_options *opts, hsma_trsm_report *report,
                         hsma_stream_t stream) {
    hsma_trsm_options o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (report) {
        std::memset(report, 0, sizeof(*report));
        report->backward_error = -1.0;
    }
    for (int i = 0; i < 2; ++i)
        if (o.reserved[i] != 0) return HSMA_INVALID_VALUE;
    if (o.use_graph != 0 && o.use_graph != 1) return HSMA_INVALID_VALUE;
    if (o.path < 0 || o.path > 2) return HSMA_INVALID_VALUE;
    if (o.block_size != 0 && !hsma::valid_block_size(hsma::is_complex(dtype), o.block_size))
        return HSMA_INVALID_VALUE;
    if (o.precision != HSMA_PREC_FP64 && o.precision != HSMA_PREC_MIXED) return HSMA_INVALID_VALUE;
    if (o.refine_steps < -1 || o.refine_steps > 4) return HSMA_INVALID_VALUE;
    if (o.want_backward_error != 0 && o.want_backward_error != 1) return HSMA_INVALID_VALUE;
    if (!(o.refine_tol >= 0.0)) return HSMA_INVALID_VALUE;
    int path_used = 0, ib_used = 0;
    hsma_status st = hsma::trsm_impl(diag, m, n, alpha, A, lda, B, ldb, dtype, o.block_size, o.path,
                                     static_cast<hipStream_t>(stream), &path_used, &ib_used, &o,
                                     report);
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
