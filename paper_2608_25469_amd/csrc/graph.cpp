// HIP-graph replay of the blocked schedule, one graph per problem shape.
//
// A blocked solve is a fixed sequence of 2 log2(m/I_B) + ~10 dependent kernel
// launches whose shape -- the kernels, grids and dependencies -- depends only
// on (dtype, diag, m, n, lda, ldb, I_B, precision); the matrices and alpha
// only change kernel arguments.  So a graph is captured once per shape (on a
// library stream, with its own workspace, so nothing is allocated inside the
// capture and no memset node is recorded: workspace initialisation is a
// kernel) and instantiated once.  A later call with other pointers or
// another alpha records the same launch sequence again (recording only, no
// device submission) and moves the new arguments into the instantiated
// graph with hipGraphExecUpdate, then replays it with one hipGraphLaunch.
//
// Each shape keeps two instantiated graphs used in turn, sharing the shape's
// workspace: a graph is updated only after its previous replay (two calls
// back) has finished, and every replay waits on the device for the other
// graph's last replay, because both use the same workspace.  Replays of one
// shape therefore run one after another, on any stream.  A small LRU bounds
// the cache.

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
    bool operator==(const Key &o) const { return std::memcmp(this, &o, sizeof(Key)) == 0; }
};

// The arguments a graph was last recorded with.
struct Args {
    const void *A = nullptr;
    void *B = nullptr;
    double ar = 0, ai = 0;
    bool operator==(const Args &o) const {
        return A == o.A && B == o.B && ar == o.ar && ai == o.ai;
    }
};

struct Entry {
    Key key;
    void *ws = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    Args args[2];
    hipEvent_t done[2] = {nullptr, nullptr};
    bool launched[2] = {false, false};
    int turn = 0;
};

constexpr size_t kMaxEntries = 32;
std::mutex g_mu;
std::list<Entry> g_lru;        // front = most recently used
hipStream_t g_capture[64] = {};
// Per thread: captures use hipStreamCaptureModeThreadLocal, so only the
// capturing thread's own calls are recorded and must see the flag.
thread_local bool g_capturing = false;
// Replay counters (hsma_graph_stats).
int64_t g_captures = 0, g_updates = 0, g_replays = 0;

void destroy(Entry &e) {
    for (int i = 0; i < 2; ++i) {
        if (e.done[i]) (void)hipEventSynchronize(e.done[i]);
        if (e.exec[i]) (void)hipGraphExecDestroy(e.exec[i]);
        if (e.done[i]) (void)hipEventDestroy(e.done[i]);
        e.exec[i] = nullptr;
        e.done[i] = nullptr;
    }
    if (e.ws) (void)hipFree(e.ws);  // hipFree waits for outstanding work on the buffer
    e.ws = nullptr;
}

// Record the launch sequence for `a` on the capture stream into a new graph.
hsma_status record(const Key &k, const Args &a, void *ws, hipStream_t cs, hipGraph_t *out) {
    *out = nullptr;
    hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) return hip_fail(he);
    g_capturing = true;
    hsma_status st = blocked_trsm(k.cx, k.unit, k.m, k.n, cplx{a.ar, a.ai},
                                  static_cast<const double *>(a.A), k.lda, static_cast<double *>(a.B),
                                  k.ldb, k.ib, ws, cs, k.mixed);
    g_capturing = false;
    hipGraph_t graph = nullptr;
    he = hipStreamEndCapture(cs, &graph);
    if (st == HSMA_SUCCESS && he != hipSuccess) st = hip_fail(he);
    if (st != HSMA_SUCCESS) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    *out = graph;
    return HSMA_SUCCESS;
}

// Make exec[i] of `e` run the schedule for `a`: instantiate it on first use,
// else update it in place (re-instantiate if the update is refused).
hsma_status prepare(Entry &e, int i, const Args &a, hipStream_t cs) {
    if (e.exec[i] && e.args[i] == a) return HSMA_SUCCESS;
    if (e.launched[i]) HSMA_HIP(hipEventSynchronize(e.done[i]));  // its replay two calls back
    hipGraph_t g = nullptr;
    HSMA_TRY(record(e.key, a, e.ws, cs, &g));
    hsma_status st = HSMA_SUCCESS;
    if (e.exec[i]) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        const hipError_t he = hipGraphExecUpdate(e.exec[i], g, &bad, &res);
        if (he == hipSuccess && res == hipGraphExecUpdateSuccess) {
            ++g_updates;
        } else {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(e.exec[i]);
            e.exec[i] = nullptr;
        }
    }
    if (!e.exec[i]) {
        const hipError_t he = hipGraphInstantiate(&e.exec[i], g, nullptr, nullptr, 0);
        if (he != hipSuccess) {
            e.exec[i] = nullptr;
            st = hip_fail(he);
        } else {
            ++g_captures;
        }
    }
    (void)hipGraphDestroy(g);
    if (st == HSMA_SUCCESS) e.args[i] = a;
    return st;
}

}  // namespace

bool graph_capture_active() { return g_capturing; }

hsma_status blocked_trsm_graph(bool cx, bool unit, int64_t m, int64_t n, cplx alpha,
                               const double *A, int64_t lda, double *B, int64_t ldb, int ib,
                               bool mixed, hipStream_t s) {
    Key k;
    std::memset(&k, 0, sizeof(k));  // padding bytes take part in the comparison
    HSMA_HIP(hipGetDevice(&k.device));
    if (k.device < 0 || k.device >= 64) return HSMA_NOT_SUPPORTED;
    k.cx = cx;
    k.unit = unit;
    k.mixed = mixed;
    k.ib = ib;
    k.m = m;
    k.n = n;
    k.lda = lda;
    k.ldb = ldb;
    Args a;
    a.A = A;
    a.B = B;
    a.ar = alpha.re;
    a.ai = alpha.im;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_capture[k.device]) HSMA_HIP(hipStreamCreateWithFlags(&g_capture[k.device], hipStreamNonBlocking));
    const hipStream_t cs = g_capture[k.device];
    auto it = g_lru.begin();
    for (; it != g_lru.end(); ++it)
        if (it->key == k) break;
    if (it != g_lru.end()) {
        g_lru.splice(g_lru.begin(), g_lru, it);
    } else {
        Entry e;
        e.key = k;
        hipError_t he = hipMalloc(&e.ws, blocked_workspace_bytes(cx, m, ib));
        if (he == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            return HSMA_ALLOC_FAILED;
        }
        HSMA_HIP(he);
        for (int i = 0; i < 2 && he == hipSuccess; ++i) he = hipEventCreateWithFlags(&e.done[i], hipEventDisableTiming);
        if (he != hipSuccess) {
            destroy(e);
            return hip_fail(he);
        }
        g_lru.push_front(e);
        if (g_lru.size() > kMaxEntries) {
            destroy(g_lru.back());
            g_lru.pop_back();
        }
    }
    Entry &e = g_lru.front();
    const int i = e.turn;
    HSMA_TRY(prepare(e, i, a, cs));
    e.turn ^= 1;
    // The other graph's last replay uses the same workspace.
    if (e.launched[i ^ 1]) HSMA_HIP(hipStreamWaitEvent(s, e.done[i ^ 1], 0));
    HSMA_HIP(hipGraphLaunch(e.exec[i], s));
    HSMA_HIP(hipEventRecord(e.done[i], s));
    e.launched[i] = true;
    ++g_replays;
    return HSMA_SUCCESS;
}

}  // namespace hsma

extern "C" hsma_status hsma_graph_cache_clear(void) {
    std::lock_guard<std::mutex> lk(hsma::g_mu);
    for (auto &e : hsma::g_lru) hsma::destroy(e);
    hsma::g_lru.clear();
    return HSMA_SUCCESS;
}

extern "C" hsma_status hsma_graph_stats(int64_t *captures, int64_t *updates, int64_t *replays) {
    std::lock_guard<std::mutex> lk(hsma::g_mu);
    if (captures) *captures = hsma::g_captures;
    if (updates) *updates = hsma::g_updates;
    if (replays) *replays = hsma::g_replays;
    return HSMA_SUCCESS;
}
