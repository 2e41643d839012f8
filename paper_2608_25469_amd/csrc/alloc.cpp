// Library workspace allocator: a per-device cache of device blocks with
// stream-ordered reuse.
//
// Workspaces (diagonal-block inverses, descriptor tables, residuals, served
// requests' inputs) are short-lived and of many sizes.  Freed blocks are kept,
// binned by rounded size, together with the stream they were freed on and an
// event recorded there.  An allocation takes a cached block of its bin: at
// once if it was freed on the same stream (stream order already separates
// the old and new uses), otherwise after making the new stream wait for the
// block's event.  A request takes the smallest idle block between its bin
// and twice that.  Only a miss calls hipMalloc.  Idle blocks are returned to
// the device when hipMalloc runs out of memory and by
// hsma_workspace_release().
//
// Bins: sizes up to 1 MiB round up to a power of two (at least 4 KiB);
// larger sizes round up to an eighth of their power of two, so a block is at
// most 12.5 % larger than asked for.

#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace hsma {

bool graph_capture_active();

namespace {

struct Idle {
    void *p;
    hipStream_t s;
    hipEvent_t ev;
};

struct Cache {
    std::mutex mu;
    std::multimap<size_t, Idle> idle;            // bin size -> blocks
    std::unordered_map<void *, size_t> live;     // block -> bin size
    size_t held = 0;                             // bytes obtained from hipMalloc
};

Cache g_cache[64];

size_t bin_size(size_t b) {
    if (b <= 4096) return 4096;
    size_t p2 = 4096;
    while (p2 < b) p2 <<= 1;
    if (p2 <= (1u << 20)) return p2;
    const size_t g = p2 / 8;
    return (b + g - 1) / g * g;
}

hsma_status current(Cache **c) {
    int dev = 0;
    HSMA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return HSMA_NOT_SUPPORTED;
    *c = &g_cache[dev];
    return HSMA_SUCCESS;
}

// Return every idle block to the device (waits for each block's last use).
// Lock held.
void trim(Cache &c) {
    for (auto &kv : c.idle) {
        if (kv.second.ev) {
            (void)hipEventSynchronize(kv.second.ev);
            (void)hipEventDestroy(kv.second.ev);
        }
        (void)hipFree(kv.second.p);
        c.held -= kv.first;
    }
    c.idle.clear();
}

}  // namespace

hsma_status ws_alloc(void **p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) return HSMA_SUCCESS;
    if (graph_capture_active()) {
        // Inside a capture, stay with stream-ordered allocation nodes.
        const hipError_t e = hipMallocAsync(p, bytes, s);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            return HSMA_ALLOC_FAILED;
        }
        HSMA_HIP(e);
        return HSMA_SUCCESS;
    }
    Cache *c;
    HSMA_TRY(current(&c));
    const size_t b = bin_size(bytes);
    std::lock_guard<std::mutex> lk(c->mu);
    // Best fit among idle blocks of at most twice the bin: the smallest
    // size present, preferring one usable at once (freed on this stream, or
    // known idle).
    auto pick = c->idle.end();
    int seen = 0;
    for (auto it = c->idle.lower_bound(b); it != c->idle.end() && it->first <= 2 * b && seen < 16;
         ++it, ++seen) {
        if (pick != c->idle.end() && it->first != pick->first) break;
        if (it->second.s == s || !it->second.ev) {  // usable at once
            pick = it;
            break;
        }
        if (pick == c->idle.end()) pick = it;
    }
    if (pick != c->idle.end()) {
        const size_t got = pick->first;
        Idle blk = pick->second;
        c->idle.erase(pick);
        if (blk.ev && blk.s != s) {
            const hipError_t e = hipStreamWaitEvent(s, blk.ev, 0);
            if (e != hipSuccess) {
                c->idle.emplace(got, blk);
                return hip_fail(e);
            }
        }
        if (blk.ev) (void)hipEventDestroy(blk.ev);
        c->live[blk.p] = got;
        *p = blk.p;
        return HSMA_SUCCESS;
    }
    hipError_t e = hipMalloc(p, b);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        trim(*c);
        e = hipMalloc(p, b);
    }
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        *p = nullptr;
        return HSMA_ALLOC_FAILED;
    }
    HSMA_HIP(e);
    c->live[*p] = b;
    c->held += b;
    return HSMA_SUCCESS;
}

hsma_status ws_free(void *p, hipStream_t s) {
    if (!p) return HSMA_SUCCESS;
    Cache *c;
    HSMA_TRY(current(&c));
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->live.find(p);
    if (it == c->live.end()) {
        // Not from the cache: a stream-ordered allocation made under capture.
        HSMA_HIP(hipFreeAsync(p, s));
        return HSMA_SUCCESS;
    }
    const size_t b = it->second;
    c->live.erase(it);
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, s);
    if (e != hipSuccess) {
        // Cannot track the last use: wait for it and give the block back.
        (void)hipStreamSynchronize(s);
        (void)hipFree(p);
        c->held -= b;
        return hip_fail(e);
    }
    c->idle.emplace(b, Idle{p, s, ev});
    return HSMA_SUCCESS;
}

// A block whose last use is known to have completed on the device (the
// caller has seen the completion of all work that touched it): it is
// reusable on any stream at once, with no event.  An event recorded now on
// the stream that used it would also cover everything enqueued there since,
// and make the next user wait for that unrelated work.
hsma_status ws_free_idle(void *p) {
    if (!p) return HSMA_SUCCESS;
    Cache *c;
    HSMA_TRY(current(&c));
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->live.find(p);
    if (it == c->live.end()) return HSMA_INVALID_POINTER;
    const size_t b = it->second;
    c->live.erase(it);
    c->idle.emplace(b, Idle{p, nullptr, nullptr});
    return HSMA_SUCCESS;
}

size_t ws_cached_bytes() {
    Cache *c;
    if (current(&c) != HSMA_SUCCESS) return 0;
    std::lock_guard<std::mutex> lk(c->mu);
    return c->held;
}

}  // namespace hsma

extern "C" hsma_status hsma_workspace_release(void) {
    hsma::Cache *c;
    HSMA_TRY(hsma::current(&c));
    std::lock_guard<std::mutex> lk(c->mu);
    hsma::trim(*c);
    return HSMA_SUCCESS;
}
