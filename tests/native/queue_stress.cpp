// ThreadSanitizer stress of the serving queue: the simulation backend (no
// GPU) driven by four threads that submit, poll, wait and release at once.
#include <cstdio>
#include <thread>
#include <vector>
#include "hsma.h"

int main() {
    hsma_queue_config cfg{};
    cfg.backend = HSMA_BACKEND_SIMULATED;
    cfg.sim_flops_per_ns = 20000.0;
    cfg.hbm_budget_bytes = 256ull << 20;
    cfg.max_inflight = 64;
    hsma_queue *q = nullptr;
    if (hsma_queue_create(&cfg, &q) != HSMA_SUCCESS) return 1;
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t) {
        th.emplace_back([q, t] {
            for (int i = 0; i < 300; ++i) {
                hsma_request r{};
                r.prob.diag = HSMA_NON_UNIT;
                r.prob.dtype = (i % 3) ? HSMA_R64F : HSMA_C64F;
                r.prob.m = 8 + (i * 37 + t) % 700;
                r.prob.n = 1 + (i * 13) % 200;
                r.prob.alpha_re = 1.0;
                r.input = HSMA_INPUT_SYNTHETIC;
                r.release_on_completion = (i % 2 == 1) || (i % 5 != 0);  // kept results get released below
                r.key = (uint64_t)t << 32 | i;
                uint64_t tk = 0;
                if (hsma_queue_submit(q, &r, 1, &tk) != HSMA_SUCCESS) continue;
                hsma_request_info info;
                if (i % 2 == 0) {
                    hsma_queue_wait(q, tk, -1, &info);
                    hsma_queue_release(q, tk);
                } else {
                    hsma_queue_poll(q, tk, &info);
                }
                if (i % 50 == 0) {
                    hsma_queue_statistics st;
                    hsma_queue_stats(q, &st);
                }
            }
        });
    }
    for (auto &x : th) x.join();
    hsma_queue_statistics st;
    hsma_queue_stats(q, &st);
    std::printf("submitted %lld completed %lld failed %lld in_use %llu\n", (long long)st.submitted,
                (long long)st.completed, (long long)st.failed, (unsigned long long)st.bytes_in_use);
    hsma_queue_destroy(q);
    return 0;
}
