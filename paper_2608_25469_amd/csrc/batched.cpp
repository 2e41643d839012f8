// Many independent solves per call (the paper lists batched TRSM as future
// work, Sec. 6).
//
// Problems with m <= 64 are cut into strips of at most 16 columns for the
// strip kernel (strip.hip), four strips per wavefront: the strips of a
// wavefront share m (and whether alpha is zero) but may come from different
// problems, so a problem occupies ceil(n / 16) quarter-wavefronts rather than
// a whole wavefront.  Strips are grouped by (data type, diagonal kind); inside
// a group the wavefronts are ordered by decreasing m (longest processing time
// first: the hardware starts workgroups in that order).  Problems with m, n
// <= 16 go to the fused very-small kernel when their group has no strips,
// and become one-strip items otherwise (the two kernels give the same bits).  The descriptor table is
// uploaded in one copy; the group launches are forked onto library-owned
// streams so they overlap on the device, and joined back into the caller's
// stream.  Problems with m > 64 take the grouped blocked path (grouped.cpp)
// on one more forked stream.

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"
#include "strip_pack.h"

namespace hsma {

// From api.cpp
hsma_status trsm_impl(hsma_diag diag, int64_t m, int64_t n, const void *alpha, const void *A,
                      int64_t lda, void *B, int64_t ldb, hsma_dtype dtype, int ib_override,
                      int path, hipStream_t s, int *path_used, int *ib_used,
                      const hsma_trsm_options *opt, hsma_trsm_report *rep);

// From grouped.cpp
hsma_status grouped_blocked(const hsma_problem *probs, int64_t count, hipStream_t s);

// From strip.hip
hsma_status launch_strip_group(bool cx, bool unit, const void *rows, int waves, hipStream_t s);
size_t strip_item_bytes();

namespace {

// Must match SmallItem in small_kernels.h (checked at run time by size).
struct Item {
    const double *A;
    double *B;
    int64_t lda, ldb;
    int32_t m, ncols;
    double ar, ai;
};

constexpr int kGroups = 2 * 2 * 2;  // complex x unit x (very small, strips)
constexpr int kForkStreams = 8;

// Problems with m, n <= HSMA_TINY_MAX form their own group (slot 0 of the
// pair), solved four per workgroup by the fused kernel; the others are cut
// into strips (slot 1).
int group_of(bool cx, bool unit, int m, int64_t n) {
    return ((cx ? 1 : 0) * 2 + (unit ? 1 : 0)) * 2 + (tiny_fits(m, n) ? 0 : 1);
}
bool group_is_tiny(int g) { return g % 2 == 0; }
bool group_cx(int g) { return g >= 4; }
bool group_unit(int g) { return (g / 2) % 2 == 1; }
constexpr int kStripCols = 16;

struct DevicePool {
    // Created on the first forking call only: a process that never forks
    // (the serving queue runs batches serially on its own streams) keeps
    // every stream it has on a hardware queue of its own.
    bool forks_made = false;
    hipStream_t fork[kForkStreams] = {};
    std::mutex mu;
    // Pinned staging buffers for descriptor uploads.  A buffer is reusable
    // once the copy out of it has finished (its event); the pool grows up to
    // kMaxStages rather than make the host wait for the device.
    struct Stage {
        void *host = nullptr;
        size_t bytes = 0;
        hipEvent_t done = nullptr;
        bool used = false;
    };
    std::vector<Stage> stages;
    size_t next = 0;  // wait-for-oldest victim once the pool is full
};
constexpr size_t kMaxStages = 64;
DevicePool g_pools[64];

hsma_status pool_for(DevicePool **out) {
    DeviceInfo di;
    HSMA_TRY(device_info(&di));
    *out = &g_pools[di.device];
    return HSMA_SUCCESS;
}

hsma_status fork_streams(DevicePool *p) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->forks_made) {
        for (int i = 0; i < kForkStreams; ++i)
            HSMA_HIP(hipStreamCreateWithFlags(&p->fork[i], hipStreamNonBlocking));
        p->forks_made = true;
    }
    return HSMA_SUCCESS;
}

}  // namespace

// The device-resident part of a batch: item table, group extents, and the
// problems that take the blocked path.
struct BatchTable {
    void *dev = nullptr;  // items, grouped and sorted
    size_t bytes = 0;
    // Per group: first item, and the launch size -- items of a very small
    // group, wavefronts (four items each) of a strip group.
    int start[kGroups] = {}, count[kGroups] = {};
    std::vector<hsma_problem> large;
};

static hsma_status check_all(const hsma_problem *probs, int64_t count, int64_t *first_bad) {
    if (first_bad) *first_bad = -1;
    if (count < 0) return HSMA_INVALID_SIZE;
    if (count > 0 && !probs) return HSMA_INVALID_POINTER;
    for (int64_t i = 0; i < count; ++i) {
        const hsma_problem &p = probs[i];
        double al[2] = {p.alpha_re, p.alpha_im};
        bool quick = false;
        hsma_status st = validate(p.diag, p.dtype, p.m, p.n, al, p.A, p.lda, p.B, p.ldb, &quick);
        if (st == HSMA_SUCCESS && p.dtype == HSMA_R64F && p.alpha_im != 0.0) st = HSMA_INVALID_VALUE;
        if (st != HSMA_SUCCESS) {
            if (first_bad) *first_bad = i;
            return st;
        }
    }
    return HSMA_SUCCESS;
}

// Host image of the table: items grouped and sorted.
static void build_image(const hsma_problem *probs, int64_t count, BatchTable *t,
                        std::vector<unsigned char> *img) {
    // Very small problems: one item each, by decreasing cost.
    std::vector<Item> tiny[kGroups];
    std::vector<double> tiny_cost[kGroups];
    // Strips, bucketed per group by (m, alpha == 0): bucket 2 m + azero, in
    // problem order, with each problem's span (first strip, strip count).
    std::vector<Item> strips[kGroups][2 * 65];
    std::vector<StripSpan> spans[kGroups][2 * 65];
    for (int64_t i = 0; i < count; ++i) {
        const hsma_problem &p = probs[i];
        if (p.m == 0 || p.n == 0) continue;
        if (p.m > 64) {
            t->large.push_back(p);
            continue;
        }
        const bool cx = p.dtype == HSMA_C64F, unit = p.diag == HSMA_UNIT;
        const int g = group_of(cx, unit, (int)p.m, p.n);
        const int es = cx ? 2 : 1;
        Item it;
        it.A = static_cast<const double *>(p.A);
        it.B = static_cast<double *>(p.B);
        it.lda = p.lda;
        it.ldb = p.ldb;
        it.m = (int32_t)p.m;
        it.ncols = (int32_t)p.n;
        it.ar = p.alpha_re;
        it.ai = cx ? p.alpha_im : 0.0;
        if (group_is_tiny(g)) {
            tiny[g].push_back(it);
            tiny_cost[g].push_back((double)p.m * p.m * p.n + 64.0 * p.m);
            continue;
        }
        const bool azero = it.ar == 0.0 && it.ai == 0.0;
        const int bk = 2 * (int)p.m + (azero ? 1 : 0);
        std::vector<Item> &b = strips[g][bk];
        const int first = (int)b.size();
        for (int64_t c0 = 0; c0 < p.n; c0 += kStripCols) {
            Item st = it;
            st.B = it.B + es * c0 * p.ldb;
            st.ncols = (int32_t)std::min<int64_t>(kStripCols, p.n - c0);
            b.push_back(st);
        }
        spans[g][bk].push_back(StripSpan{first, (int)b.size() - first});
    }
    // When a (data type, diagonal kind) also has strips, its very small
    // problems join them as one-strip items: one launch instead of two, and
    // the fused kernel gives the same bits as the strip kernel anyway.
    for (int g = 0; g < kGroups; g += 2) {
        bool strips_here = false;
        for (const std::vector<Item> &b : strips[g + 1]) strips_here = strips_here || !b.empty();
        if (!strips_here || tiny[g].empty()) continue;
        for (const Item &x : tiny[g]) {
            const bool azero = x.ar == 0.0 && x.ai == 0.0;
            const int bk = 2 * x.m + (azero ? 1 : 0);
            spans[g + 1][bk].push_back(StripSpan{(int)strips[g + 1][bk].size(), 1});
            strips[g + 1][bk].push_back(x);
        }
        tiny[g].clear();
        tiny_cost[g].clear();
    }
    std::vector<Item> out;
    for (int g = 0; g < kGroups; ++g) {
        t->start[g] = (int)out.size();
        if (group_is_tiny(g)) {
            std::vector<size_t> order(tiny[g].size());
            for (size_t i = 0; i < order.size(); ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(),
                             [&](size_t a, size_t b) { return tiny_cost[g][a] > tiny_cost[g][b]; });
            for (size_t i : order) out.push_back(tiny[g][i]);
            t->count[g] = (int)order.size();
            continue;
        }
        // Largest m first; within an m, alpha != 0 before alpha == 0 (a
        // zero fill is short).  Each bucket fills whole wavefronts; the last
        // one is padded with copies of its final strip that own no columns.
        //
        // Within a bucket, pack_bucket keeps each problem's strips in one
        // wavefront wherever strip counts fit (strip_pack.h).
        int waves = 0;
        for (int b = 2 * 64 + 1; b >= 0; --b) {
            const int bb = (b / 2) * 2 + (1 - b % 2);  // 2m before 2m + 1
            std::vector<Item> &v = strips[g][bb];
            if (v.empty()) continue;
            pack_bucket(v, spans[g][bb], out);
            Item pad = v.back();
            pad.ncols = 0;
            while ((out.size() - (size_t)t->start[g]) % 4) out.push_back(pad);
            waves += (int)((v.size() + 3) / 4);
        }
        t->count[g] = waves;
    }
    img->assign(out.size() * sizeof(Item), 0);
    if (!out.empty()) std::memcpy(img->data(), out.data(), img->size());
}

// The problems with m > 64: grouped blocked launches for alpha != 0, the
// single-problem path (a zero fill) for alpha == 0.
static hsma_status run_large(const std::vector<hsma_problem> &large, hipStream_t s) {
    std::vector<hsma_problem> grouped;
    for (const hsma_problem &p : large) {
        if (p.alpha_re == 0.0 && p.alpha_im == 0.0) {
            double al[2] = {0.0, 0.0};
            HSMA_TRY(trsm_impl((hsma_diag)p.diag, p.m, p.n, al, p.A, p.lda, p.B, p.ldb,
                               (hsma_dtype)p.dtype, 0, 0, s, nullptr, nullptr, nullptr, nullptr));
        } else {
            grouped.push_back(p);
        }
    }
    return grouped_blocked(grouped.data(), (int64_t)grouped.size(), s);
}

// Enqueue the grouped launches (and the large problems) on stream s; with
// fork, the launches are spread over library streams and joined back.
static hsma_status run_table(const BatchTable &t, hipStream_t s, bool fork = true) {
    DevicePool *pool;
    HSMA_TRY(pool_for(&pool));
    // Fused very small groups run on s itself, first: they are short, and a
    // fork and join would cost more than they take.  The other groups fork
    // when there are several.
    for (int g = 0; g < kGroups; ++g) {
        if (t.count[g] == 0 || !group_is_tiny(g)) continue;
        const bool cx = group_cx(g), unit = group_unit(g);
        const void *items = static_cast<const unsigned char *>(t.dev) + (size_t)t.start[g] * sizeof(Item);
        ProfScope prof(HSMA_PHASE_TINY, 0.0, s);
        HSMA_TRY(launch_tiny_group(cx, unit, items, t.count[g], s));
    }
    int ngroups = 0;
    for (int g = 0; g < kGroups; ++g) ngroups += t.count[g] > 0 && !group_is_tiny(g);
    if (!t.large.empty()) ngroups += 1;
    if (ngroups > 0) {
        // One launch (or no fork) stays on s: no events.
        const bool forking = fork && ngroups > 1;
        if (forking) HSMA_TRY(fork_streams(pool));
        hipEvent_t fork_ev = nullptr;
        if (forking) {
            HSMA_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
            HSMA_HIP(hipEventRecord(fork_ev, s));
        }
        std::vector<hipEvent_t> joins;
        int k = 0;
        hsma_status st = HSMA_SUCCESS;
        // Complex groups first: they hold the longest items.
        for (int g = kGroups - 1; g >= 0 && st == HSMA_SUCCESS; --g) {
            if (t.count[g] == 0 || group_is_tiny(g)) continue;
            hipStream_t fs = forking ? pool->fork[k++ % kForkStreams] : s;
            if (fs != s) HSMA_HIP(hipStreamWaitEvent(fs, fork_ev, 0));
            const bool cx = group_cx(g), unit = group_unit(g);
            const unsigned char *base = static_cast<const unsigned char *>(t.dev);
            const void *items = base + (size_t)t.start[g] * sizeof(Item);
            {
                ProfScope prof(HSMA_PHASE_SMALL, 0.0, fs);
                st = launch_strip_group(cx, unit, items, t.count[g], fs);
            }
            if (fs != s) {
                hipEvent_t j;
                HSMA_HIP(hipEventCreateWithFlags(&j, hipEventDisableTiming));
                HSMA_HIP(hipEventRecord(j, fs));
                joins.push_back(j);
            }
        }
        // The large problems run beside the small groups.
        if (st == HSMA_SUCCESS && !t.large.empty()) {
            hipStream_t fs = forking ? pool->fork[k++ % kForkStreams] : s;
            if (fs != s) HSMA_HIP(hipStreamWaitEvent(fs, fork_ev, 0));
            st = run_large(t.large, fs);
            if (fs != s) {
                hipEvent_t j;
                HSMA_HIP(hipEventCreateWithFlags(&j, hipEventDisableTiming));
                HSMA_HIP(hipEventRecord(j, fs));
                joins.push_back(j);
            }
        }
        for (hipEvent_t j : joins) {
            HSMA_HIP(hipStreamWaitEvent(s, j, 0));
            HSMA_HIP(hipEventDestroy(j));
        }
        if (fork_ev) HSMA_HIP(hipEventDestroy(fork_ev));
        HSMA_TRY(st);
    }
    return HSMA_SUCCESS;
}

// Copy `bytes` of host data to device memory `dev` through a pinned staging
// buffer, asynchronously on s (the host data may be reused on return).
hsma_status upload_async(const void *host, size_t bytes, void *dev, hipStream_t s) {
    if (bytes == 0) return HSMA_SUCCESS;
    DevicePool *pool;
    HSMA_TRY(pool_for(&pool));
    std::lock_guard<std::mutex> lk(pool->mu);
    auto idle = [](DevicePool::Stage &x) {
        if (!x.used) return true;
        const hipError_t e = hipEventQuery(x.done);
        if (e == hipSuccess) {
            x.used = false;
            return true;
        }
        if (e != hipErrorNotReady) (void)hipGetLastError();
        return false;
    };
    // Smallest idle buffer that is large enough.
    DevicePool::Stage *pick = nullptr;
    for (DevicePool::Stage &x : pool->stages)
        if (x.bytes >= bytes && idle(x) && (!pick || x.bytes < pick->bytes)) pick = &x;
    if (!pick && pool->stages.size() < kMaxStages) {
        pool->stages.emplace_back();
        pick = &pool->stages.back();
    }
    if (!pick) {
        // Pool full: wait for the oldest victim, then size it.
        pick = &pool->stages[pool->next];
        pool->next = (pool->next + 1) % pool->stages.size();
        if (pick->used) HSMA_HIP(hipEventSynchronize(pick->done));
        pick->used = false;
    }
    DevicePool::Stage &st = *pick;
    if (st.bytes < bytes) {
        if (st.host) HSMA_HIP(hipHostFree(st.host));
        st.host = nullptr;
        st.bytes = 0;
        size_t want = std::max<size_t>(bytes, 1 << 20);
        HSMA_HIP(hipHostMalloc(&st.host, want, hipHostMallocDefault));
        st.bytes = want;
    }
    if (!st.done) HSMA_HIP(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    std::memcpy(st.host, host, bytes);
    HSMA_HIP(hipMemcpyAsync(dev, st.host, bytes, hipMemcpyHostToDevice, s));
    HSMA_HIP(hipEventRecord(st.done, s));
    st.used = true;
    return HSMA_SUCCESS;
}

static hsma_status upload(const std::vector<unsigned char> &img, void *dev, hipStream_t s) {
    return upload_async(img.data(), img.size(), dev, s);
}

// hsma_trsm_batched with every launch on s itself (no fork onto library
// streams): for callers that run several batches side by side on their own
// streams, such as the serving queue.
hsma_status trsm_batched_serial(const hsma_problem *probs, int64_t count, hipStream_t s) {
    HSMA_TRY(check_all(probs, count, nullptr));
    if (count == 0) return HSMA_SUCCESS;
    if (strip_item_bytes() != sizeof(Item) || tiny_item_bytes() != sizeof(Item)) return HSMA_NOT_SUPPORTED;
    BatchTable t;
    std::vector<unsigned char> img;
    build_image(probs, count, &t, &img);
    if (!img.empty()) {
        HSMA_TRY(ws_alloc(&t.dev, img.size(), s));
        t.bytes = img.size();
        hsma_status st = upload(img, t.dev, s);
        if (st == HSMA_SUCCESS) st = run_table(t, s, false);
        hsma_status st2 = ws_free(t.dev, s);
        return st != HSMA_SUCCESS ? st : st2;
    }
    return run_table(t, s, false);
}

}  // namespace hsma

struct hsma_batch_plan {
    hsma::BatchTable table;
    int device = -1;
};

extern "C" {

hsma_status hsma_trsm_batched(const hsma_problem *probs, int64_t count, int64_t *first_bad,
                              hsma_stream_t stream) {
    using namespace hsma;
    HSMA_TRY(check_all(probs, count, first_bad));
    if (count == 0) return HSMA_SUCCESS;
    if (strip_item_bytes() != sizeof(Item) || tiny_item_bytes() != sizeof(Item)) return HSMA_NOT_SUPPORTED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchTable t;
    std::vector<unsigned char> img;
    build_image(probs, count, &t, &img);
    if (!img.empty()) {
        HSMA_TRY(ws_alloc(&t.dev, img.size(), s));
        t.bytes = img.size();
        hsma_status st = upload(img, t.dev, s);
        if (st == HSMA_SUCCESS) st = run_table(t, s);
        hsma_status st2 = ws_free(t.dev, s);
        return st != HSMA_SUCCESS ? st : st2;
    }
    return run_table(t, s);
}

hsma_status hsma_batch_plan_create(const hsma_problem *probs, int64_t count, int64_t *first_bad,
                                   hsma_batch_plan **plan) {
    using namespace hsma;
    if (!plan) return HSMA_INVALID_POINTER;
    *plan = nullptr;
    HSMA_TRY(check_all(probs, count, first_bad));
    if (strip_item_bytes() != sizeof(Item) || tiny_item_bytes() != sizeof(Item)) return HSMA_NOT_SUPPORTED;
    hsma_batch_plan *p = new hsma_batch_plan();
    std::vector<unsigned char> img;
    build_image(probs, count, &p->table, &img);
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess && !img.empty()) {
        e = hipMalloc(&p->table.dev, img.size());
        if (e == hipSuccess) e = hipMemcpy(p->table.dev, img.data(), img.size(), hipMemcpyHostToDevice);
        p->table.bytes = img.size();
    }
    if (e != hipSuccess) {
        if (p->table.dev) (void)hipFree(p->table.dev);
        delete p;
        return hip_fail(e);
    }
    *plan = p;
    return HSMA_SUCCESS;
}

hsma_status hsma_batch_plan_execute(hsma_batch_plan *plan, hsma_stream_t stream) {
    using namespace hsma;
    if (!plan) return HSMA_INVALID_POINTER;
    int dev = -1;
    HSMA_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return HSMA_INVALID_VALUE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run_table(plan->table, s);
}

hsma_status hsma_batch_plan_destroy(hsma_batch_plan *plan) {
    if (!plan) return HSMA_SUCCESS;
    hsma_status st = HSMA_SUCCESS;
    if (plan->table.dev) {
        hipError_t e = hipFree(plan->table.dev);
        if (e != hipSuccess) st = hsma::hip_fail(e);
    }
    delete plan;
    return st;
}

}  // extern "C"
