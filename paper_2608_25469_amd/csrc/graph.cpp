// HIP-graph capture and replay of the blocked schedule.
//
// A blocked solve is a fixed sequence of 2 log2(m/I_B) + ~10 dependent kernel
// launches for given (shape, pointers, alpha, I_B); for mid-size problems the
// host-side cost of issuing them dominates.  With use_graph the sequence is
// captured once on a library stream (with its own workspace, so nothing is
// allocated inside the capture and no memset node is recorded: workspace
// initialisation is a kernel) and replayed with one hipGraphLaunch per call.
// Entries are keyed by everything the captured kernels read from their
// arguments; a small LRU bounds the cache.

#include <cstring>
#include <list>
#include <mutex>

#include "internal.h"

namespace hsma {

size_t blocked_workspace_bytes(bool cx, int64_t m, int ib);
hsma_status blocked_trsm(bool cx, bool unit, int64_t m, int64_t n, cplx alpha, const double *A,
                         int64_t lda, double *B, int64_t ldb, int ib, void *ws, hipStream_t s,
                         bool mixed);

namespace {

struct Key {
    int device;
    int cx, unit, mixed, ib;
    int64_t m, n, lda, ldb;
    const void *A;
    void *B;
    double ar, ai;
    bool operator==(const Key &o) const { return std::memcmp(this, &o, sizeof(Key)) == 0; }
};

struct Entry {
    Key key;
    hipGraphExec_t exec = nullptr;
    void *ws = nullptr;
};

constexpr size_t kMaxEntries = 32;
std::mutex g_mu;
std::list<Entry> g_lru;        // front = most recently used
hipStream_t g_capture[64] = {};
// Per thread: captures use hipStreamCaptureModeThreadLocal, so only the
// capturing thread's own calls are recorded and must see the flag.
thread_local bool g_capturing = false;

void destroy(Entry &e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.ws) (void)hipFree(e.ws);  // hipFree waits for outstanding work on the buffer
    e.exec = nullptr;
    e.ws = nullptr;
}

}  // namespace

bool graph_capture_active() { return g_capturing; }

hsma_status blocked_trsm_graph(bool cx, bool unit, int64_t m, int64_t n, cplx alpha,
                               const double *A, int64_t lda, double *B, int64_t ldb, int ib,
                               bool mixed, hipStream_t s) {
    Key k;
    std::memset(&k, 0, sizeof(k));  // padding bytes take part in the comparison
    HSMA_HIP(hipGetDevice(&k.device));
    k.cx = cx;
    k.unit = unit;
    k.mixed = mixed;
    k.ib = ib;
    k.m = m;
    k.n = n;
    k.lda = lda;
    k.ldb = ldb;
    k.A = A;
    k.B = B;
    k.ar = alpha.re;
    k.ai = alpha.im;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_lru.begin(); it != g_lru.end(); ++it) {
        if (it->key == k) {
            g_lru.splice(g_lru.begin(), g_lru, it);
            HSMA_HIP(hipGraphLaunch(g_lru.front().exec, s));
            return HSMA_SUCCESS;
        }
    }
    if (k.device < 0 || k.device >= 64) return HSMA_NOT_SUPPORTED;
    if (!g_capture[k.device]) HSMA_HIP(hipStreamCreateWithFlags(&g_capture[k.device], hipStreamNonBlocking));
    hipStream_t cs = g_capture[k.device];
    Entry e;
    e.key = k;
    hipError_t he = hipMalloc(&e.ws, blocked_workspace_bytes(cx, m, ib));
    if (he == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return HSMA_ALLOC_FAILED;
    }
    HSMA_HIP(he);
    hipGraph_t graph = nullptr;
    he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) {
        destroy(e);
        return hip_fail(he);
    }
    g_capturing = true;
    hsma_status st = blocked_trsm(cx, unit, m, n, alpha, A, lda, B, ldb, ib, e.ws, cs, mixed);
    g_capturing = false;
    he = hipStreamEndCapture(cs, &graph);
    if (st == HSMA_SUCCESS && he != hipSuccess) st = hip_fail(he);
    if (st == HSMA_SUCCESS) {
        he = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
        if (he != hipSuccess) st = hip_fail(he);
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (st != HSMA_SUCCESS) {
        destroy(e);
        return st;
    }
    g_lru.push_front(e);
    if (g_lru.size() > kMaxEntries) {
        destroy(g_lru.back());
        g_lru.pop_back();
    }
    HSMA_HIP(hipGraphLaunch(g_lru.front().exec, s));
    return HSMA_SUCCESS;
}

}  // namespace hsma

extern "C" hsma_status hsma_graph_cache_clear(void) {
    std::lock_guard<std::mutex> lk(hsma::g_mu);
    for (auto &e : hsma::g_lru) hsma::destroy(e);
    hsma::g_lru.clear();
    return HSMA_SUCCESS;
}
