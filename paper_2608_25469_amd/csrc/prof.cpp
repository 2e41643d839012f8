// Phase accounting: HIP events around every kernel launch while enabled.
//
// The paper breaks blocked-TRSM time into diagonal inversion, GEMM update,
// solve GEMM and copy/other (Sec. 5.3, Table 3).  When profiling is on, each
// launcher records an event pair on its own stream around its kernel, tagged
// with the phase and the launch's algorithmic flop count; hsma_profile_end()
// waits for the events and sums elapsed times per phase.

#include <mutex>
#include <vector>

#include "internal.h"

namespace hsma {

namespace {
struct Rec {
    int phase;
    double flops;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_free;

hipEvent_t take_event() {
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool graph_capture_active();

ProfScope::ProfScope(int phase, double flops, hipStream_t s) : s_(s), idx_(-1) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || graph_capture_active()) return;  // no event nodes inside a captured graph
    Rec r{phase, flops, take_event(), take_event()};
    if (!r.a || !r.b) return;
    if (hipEventRecord(r.a, s) != hipSuccess) return;
    idx_ = (int)g_recs.size();
    g_recs.push_back(r);
}

ProfScope::~ProfScope() {
    if (idx_ < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (idx_ < (int)g_recs.size()) (void)hipEventRecord(g_recs[idx_].b, s_);
}

}  // namespace hsma

extern "C" {

hsma_status hsma_profile_begin(void) {
    std::lock_guard<std::mutex> lk(hsma::g_mu);
    for (auto &r : hsma::g_recs) {
        hsma::g_free.push_back(r.a);
        hsma::g_free.push_back(r.b);
    }
    hsma::g_recs.clear();
    hsma::g_on = true;
    return HSMA_SUCCESS;
}

hsma_status hsma_profile_end(hsma_phase_stat *out, int count) {
    if (!out || count < HSMA_PHASE_COUNT) return HSMA_INVALID_POINTER;
    std::vector<hsma::Rec> recs;
    {
        std::lock_guard<std::mutex> lk(hsma::g_mu);
        hsma::g_on = false;
        recs.swap(hsma::g_recs);
    }
    for (int i = 0; i < HSMA_PHASE_COUNT; ++i) out[i] = hsma_phase_stat{0, 0.0, 0.0};
    hsma_status st = HSMA_SUCCESS;
    for (auto &r : recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) {
            st = hsma::hip_fail(e);
            continue;
        }
        if (r.phase >= 0 && r.phase < HSMA_PHASE_COUNT) {
            out[r.phase].launches += 1;
            out[r.phase].ms += ms;
            out[r.phase].flops += r.flops;
        }
    }
    std::lock_guard<std::mutex> lk(hsma::g_mu);
    for (auto &r : recs) {
        hsma::g_free.push_back(r.a);
        hsma::g_free.push_back(r.b);
    }
    return st;
}

}  // extern "C"
