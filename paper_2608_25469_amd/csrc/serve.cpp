// Request queue with continuous batching (the paper's outlook on batched
// TRSM, Sec. 6, carried to a serving loop).
//
// Clients submit requests at any time; a scheduler thread
//   1. retires finished work (event polling), releasing its HBM budget and
//      recording its latency,
//   2. admits pending requests in arrival order while the HBM budget and the
//      in-flight limit allow (a request larger than the whole budget is
//      rejected at submit, so the head of the queue always fits once the
//      work ahead of it retires),
//   3. launches what it admitted by size class -- m <= 64, 64 < m <= 512,
//      m > 512, the last two split by data type -- each class as one batched
//      call (grouped small-solve launches, or grouped blocked launches that
//      advance all of the class's problems together) on its own stream, the
//      four blocked classes round-robin over the queue's streams,
// so requests arriving while others run reach the device as soon as slots
// and memory free up, and their work overlaps on the GPU.
//
// Requests either bring device pointers (the caller keeps them alive until
// completion) or ask the server to allocate and fill L and B from a Philox
// key (synthetic load).  A simulation backend runs the same policy with
// modelled completion times so the scheduler can be tested without a GPU.

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace hsma {

size_t blocked_workspace_bytes(bool cx, int64_t m, int ib);
int lookup_block_size(bool cx, int64_t m, int64_t n);
hsma_status trsm_batched_serial(const hsma_problem *probs, int64_t count, hipStream_t s);

namespace {

double clock_ns() {
    return (double)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum State { PENDING = 0, RUNNING = 1, DONE = 2, FAILED = 3 };

constexpr size_t kSmallShare = 4096;  // descriptor share of a small request
#ifndef HSMA_SMALL_CU_STRIDE
#define HSMA_SMALL_CU_STRIDE 16
#endif
constexpr int kSmallCuStride = HSMA_SMALL_CU_STRIDE;  // every k-th CU serves the small class

size_t data_bytes(const hsma_problem &p) {
    const size_t es = p.dtype == HSMA_C64F ? 16 : 8;
    return es * (size_t)(p.m * p.m + p.m * p.n);
}

size_t footprint(const hsma_request &r) {
    const hsma_problem &p = r.prob;
    const bool cx = p.dtype == HSMA_C64F;
    size_t f = r.input == HSMA_INPUT_SYNTHETIC ? data_bytes(p) : 0;
    f += p.m > 64 ? blocked_workspace_bytes(cx, p.m, lookup_block_size(cx, p.m, p.n)) : kSmallShare;
    return f;
}

// Device memory shared by the auto-released synthetic requests of one size
// class of one admission round (one allocation instead of one per request);
// freed when the last of them finishes.
struct Block {
    void *mem = nullptr;
    hipStream_t s = nullptr;
    int refs = 0;
};

struct Req {
    uint64_t ticket = 0;
    hsma_request r{};
    double t_arrival = 0, t_admit = 0, t_done = 0;
    size_t held = 0;          // budget this request holds now
    void *mem = nullptr;      // own server allocation (kept synthetic results)
    hipStream_t mem_stream = nullptr;
    Block *blk = nullptr;     // shared allocation (auto-released synthetic inputs)
    const double *A = nullptr;
    double *B = nullptr;
    int64_t lda = 0, ldb = 0;
    State state = PENDING;
    hsma_status status = HSMA_SUCCESS;
    int path = 0;
};

struct Inflight {
    hipEvent_t ev = nullptr;  // HIP backend
    double t_model_done = 0;  // simulation backend
    std::vector<Req *> reqs;
};

// Latency histogram: bin 0 holds samples below kLo; bin b >= 1 holds
// [kLo 2^((b-1)/kSub), kLo 2^(b/kSub)); the last bin also takes everything
// above its lower edge.  Fixed size, so recording and summarising cost the
// same however long the queue runs.
struct LatHist {
    static constexpr int kSub = 64;        // bins per doubling
    static constexpr double kLo = 1e3;     // 1 us
    static constexpr int kBins = 64 * 32;  // up to about 4.3e12 ns
    std::array<int64_t, kBins + 1> n{};
    int64_t count = 0;
    double sum = 0, min = 0, max = 0;

    void add(double x) {
        int b = 0;
        if (x >= kLo) {
            b = 1 + (int)std::floor(std::log2(x / kLo) * kSub);
            b = std::min(std::max(b, 1), kBins);
        }
        n[b]++;
        if (count == 0 || x < min) min = x;
        if (count == 0 || x > max) max = x;
        count++;
        sum += x;
    }
    // Sample of rank round(q (count - 1)) as its bin's geometric midpoint,
    // clamped to the observed range.
    double quantile(double q) const {
        if (count == 0) return 0.0;
        const int64_t rank = (int64_t)(q * (double)(count - 1) + 0.5);
        int64_t c = 0;
        int b = 0;
        for (; b <= kBins; ++b) {
            c += n[b];
            if (c > rank) break;
        }
        double v = b == 0 ? min : kLo * std::exp2(((double)b - 0.5) / kSub);
        return std::min(std::max(v, min), max);
    }
    void summary(hsma_latency_summary *o) const {
        o->count = count;
        o->p50_ns = quantile(0.50);
        o->p99_ns = quantile(0.99);
        o->max_ns = count ? max : 0.0;
        o->mean_ns = count ? sum / (double)count : 0.0;
    }
};

// Latency class of a request: m <= 64, 64 < m <= 512, m > 512.
int latency_class(int64_t m) { return m <= 64 ? 0 : (m <= 512 ? 1 : 2); }

}  // namespace
}  // namespace hsma

struct hsma_queue {
    hsma_queue_config cfg{};
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_retire;
    std::deque<hsma::Req *> pending;
    std::unordered_map<uint64_t, hsma::Req *> all;
    std::vector<hsma::Inflight> inflight;
    uint64_t next_ticket = 1;
    size_t budget_used = 0, budget_peak = 0;
    int64_t n_inflight = 0;
    bool closing = false, stopped = false, retire_stop = false;
    std::thread sched, retire;
    int device = 0;
    hipStream_t small_stream = nullptr;
    bool cu_reserved = false;  // small class on CUs of its own (CU-masked streams)
    std::vector<hipStream_t> streams;
    size_t rr = 0;
    std::vector<double> sim_free_at;  // simulation: per-stream busy-until (last = small)
    // Device frees decided under the lock, issued after it is released.
    std::vector<std::pair<void *, hipStream_t>> deferred;
    // statistics: [0] every class, [1 + c] latency class c
    hsma::LatHist lat[1 + HSMA_LATENCY_CLASSES];
    double stats_from_ns = -1e300;  // latency window: arrivals at or after this
    int64_t submitted = 0, rejected = 0, completed = 0, failed = 0, rounds = 0;
    double t_first_submit = 0, t_last_done = 0, launch_ns = 0;
};

namespace hsma {
namespace {

// Drop the request's hold on server memory (lock held); the actual frees
// are queued for free_deferred.
void release_mem(hsma_queue *q, Req *r) {
    if (r->mem) {
        q->deferred.emplace_back(r->mem, r->mem_stream);
        r->mem = nullptr;
    }
    if (r->blk) {
        if (--r->blk->refs == 0) {
            if (r->blk->mem) q->deferred.emplace_back(r->blk->mem, r->blk->s);
            delete r->blk;
        }
        r->blk = nullptr;
    }
}

// Issue the queued frees; takes and releases the lock itself.  Every
// queued block belongs to finished requests (their completion events have
// fired), so it goes back as idle: an event recorded now on its stream
// would also cover the later rounds enqueued there, and the next request to
// reuse the block would wait for them.
void free_deferred(hsma_queue *q, std::unique_lock<std::mutex> &lk) {
    if (q->deferred.empty()) return;
    std::vector<std::pair<void *, hipStream_t>> fr;
    fr.swap(q->deferred);
    lk.unlock();
    for (auto &f : fr) {
        if (q->cfg.backend == HSMA_BACKEND_HIP) (void)ws_free_idle(f.first);
        else (void)ws_free(f.first, f.second);
    }
    lk.lock();
}

// Called with the lock held.  A fire-and-forget request (release_on_completion
// = 2) is deleted here: the caller must not touch r afterwards.
void finish(hsma_queue *q, Req *r, double t, hsma_status st) {
    r->t_done = t;
    r->state = st == HSMA_SUCCESS ? DONE : FAILED;
    r->status = st;
    q->n_inflight--;
    if (st == HSMA_SUCCESS) {
        q->completed++;
        if (r->t_arrival >= q->stats_from_ns) {
            const double lat = t - r->t_arrival;
            q->lat[0].add(lat);
            q->lat[1 + latency_class(r->r.prob.m)].add(lat);
        }
    } else {
        q->failed++;
    }
    q->t_last_done = std::max(q->t_last_done, t);
    const bool keep = st == HSMA_SUCCESS && r->r.input == HSMA_INPUT_SYNTHETIC &&
                      r->r.release_on_completion == 0;
    const size_t keep_bytes = keep ? data_bytes(r->r.prob) : 0;
    if (!keep) release_mem(q, r);
    q->budget_used -= r->held - keep_bytes;
    r->held = keep_bytes;
    if (r->r.release_on_completion == 2) {
        q->all.erase(r->ticket);
        delete r;
    }
}

// Size classes of one admission round: m <= 64, then 64 < m <= 512 and
// m > 512, each of these two split by data type.  Each class is one batched
// call on its own stream with its own completion event, so a round's small
// solves do not wait for its largest blocked solve, and the real and complex
// blocked chains of a round (separate launches at every step) run side by
// side instead of interleaved on one stream.
int size_class(const hsma_problem &p) {
    if (p.m <= 64) return 0;
    return (p.m <= 512 ? 1 : 3) + (p.dtype == HSMA_C64F ? 1 : 0);
}
constexpr int kClasses = 5;

// Enqueue the admitted requests (HIP backend).  Called without the lock.
void launch_admitted(hsma_queue *q, std::vector<Req *> &adm) {
    std::vector<Req *> cls[kClasses];
    for (Req *r : adm) cls[size_class(r->r.prob)].push_back(r);
    for (int c = 0; c < kClasses; ++c) {
        if (cls[c].empty()) continue;
        hipStream_t s = c == 0 ? q->small_stream : q->streams[q->rr++ % q->streams.size()];
        // One allocation for the class's auto-released synthetic inputs.
        size_t shared_bytes = 0;
        for (Req *r : cls[c])
            if (r->r.input == HSMA_INPUT_SYNTHETIC && r->r.release_on_completion != 0)
                shared_bytes += (data_bytes(r->r.prob) + 255) / 256 * 256;
        Block *blk = nullptr;
        hsma_status blk_st = HSMA_SUCCESS;
        if (shared_bytes) {
            blk = new Block();
            blk->s = s;
            blk_st = ws_alloc(&blk->mem, shared_bytes, s);
        }
        size_t blk_off = 0;
        std::vector<Req *> run;
        std::vector<GenRequest> gen;
        for (Req *r : cls[c]) {
            const hsma_problem &p = r->r.prob;
            const bool cx = p.dtype == HSMA_C64F;
            r->path = p.m <= 64 ? 1 : 2;
            if (r->r.input == HSMA_INPUT_SYNTHETIC) {
                unsigned char *mem = nullptr;
                hsma_status st = HSMA_SUCCESS;
                if (r->r.release_on_completion != 0) {
                    st = blk_st;
                    if (st == HSMA_SUCCESS) {
                        mem = static_cast<unsigned char *>(blk->mem) + blk_off;
                        blk_off += (data_bytes(p) + 255) / 256 * 256;
                        r->blk = blk;
                        blk->refs++;
                    }
                } else {
                    st = ws_alloc(&r->mem, data_bytes(p), s);
                    if (st == HSMA_SUCCESS) {
                        r->mem_stream = s;
                        mem = static_cast<unsigned char *>(r->mem);
                    } else {
                        r->mem = nullptr;
                    }
                }
                if (st != HSMA_SUCCESS) {
                    std::lock_guard<std::mutex> lk(q->mu);
                    finish(q, r, clock_ns(), st);
                    continue;
                }
                r->A = reinterpret_cast<double *>(mem);
                r->B = reinterpret_cast<double *>(mem) + (cx ? 2 : 1) * p.m * p.m;
                r->lda = r->ldb = p.m;
                gen.push_back(GenRequest{const_cast<double *>(r->A), r->B, p.m, p.n, r->r.key, cx});
            } else {
                r->A = static_cast<const double *>(p.A);
                r->B = static_cast<double *>(p.B);
                r->lda = p.lda;
                r->ldb = p.ldb;
            }
            run.push_back(r);
        }
        if (blk && blk->refs == 0) {
            if (blk->mem) (void)ws_free(blk->mem, s);
            delete blk;
        }
        if (run.empty()) continue;
        std::vector<hsma_problem> probs;
        probs.reserve(run.size());
        for (Req *r : run) {
            hsma_problem sp = r->r.prob;
            sp.A = r->A;
            sp.B = r->B;
            sp.lda = r->lda;
            sp.ldb = r->ldb;
            probs.push_back(sp);
        }
        hsma_status st = gen_inputs_grouped(gen.data(), (int)gen.size(), s);
        if (st == HSMA_SUCCESS) st = trsm_batched_serial(probs.data(), (int64_t)probs.size(), s);
        Inflight f;
        f.reqs = run;
        if (st == HSMA_SUCCESS) {
            hipError_t e = hipEventCreateWithFlags(&f.ev, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(f.ev, s);
            if (e != hipSuccess) st = hip_fail(e);
        }
        if (st != HSMA_SUCCESS) (void)hipStreamSynchronize(s);  // work already enqueued may use r->mem
        std::lock_guard<std::mutex> lk(q->mu);
        if (st == HSMA_SUCCESS) {
            q->inflight.push_back(f);
        } else {
            if (f.ev) (void)hipEventDestroy(f.ev);
            for (Req *r : run) finish(q, r, clock_ns(), st);
        }
    }
}

// Simulation backend: the same size classes and stream assignment; streams
// run their launches one after another, and a class launch takes
// sim_fixed_ns + (its summed flops) / sim_flops_per_ns, flops = m^2 n (x4
// for complex).
void launch_simulated(hsma_queue *q, std::vector<Req *> &adm) {
    const double now = clock_ns();
    std::lock_guard<std::mutex> lk(q->mu);
    const size_t n_big = (size_t)q->cfg.n_streams;
    Inflight f[kClasses];
    double fl[kClasses] = {};
    for (Req *r : adm) {
        const hsma_problem &p = r->r.prob;
        const int c = size_class(p);
        fl[c] += (double)p.m * p.m * p.n * (p.dtype == HSMA_C64F ? 4.0 : 1.0);
        f[c].reqs.push_back(r);
        r->path = p.m <= 64 ? 1 : 2;
    }
    for (int c = 0; c < kClasses; ++c) {
        if (f[c].reqs.empty()) continue;
        double &free_at = c == 0 ? q->sim_free_at[n_big] : q->sim_free_at[q->rr++ % n_big];
        free_at = std::max(free_at, now) + q->cfg.sim_fixed_ns + fl[c] / q->cfg.sim_flops_per_ns;
        f[c].t_model_done = free_at;
        q->inflight.push_back(f[c]);
    }
}

// Retires finished work on a thread of its own, so that a completion is
// seen (and timed, and its budget returned) within a poll interval, not
// after the scheduler's current round of launches.
void retirer(hsma_queue *q) {
    const bool hip = q->cfg.backend == HSMA_BACKEND_HIP;
    if (hip) (void)hipSetDevice(q->device);
    std::unique_lock<std::mutex> lk(q->mu);
    while (!q->retire_stop) {
        const double t = clock_ns();
        bool retired = false;
        for (size_t i = 0; i < q->inflight.size();) {
            Inflight &f = q->inflight[i];
            bool done = false;
            hsma_status st = HSMA_SUCCESS;
            if (hip) {
                const hipError_t e = hipEventQuery(f.ev);
                if (e == hipSuccess) {
                    done = true;
                } else if (e != hipErrorNotReady) {
                    done = true;
                    st = hip_fail(e);
                }
            } else {
                done = t >= f.t_model_done;
            }
            if (done) {
                for (Req *r : f.reqs) finish(q, r, t, st);
                if (f.ev) (void)hipEventDestroy(f.ev);
                f = q->inflight.back();
                q->inflight.pop_back();
                retired = true;
            } else {
                ++i;
            }
        }
        if (retired) {
            q->cv_done.notify_all();
            q->cv_sched.notify_one();  // budget and in-flight slots were returned
            free_deferred(q, lk);
        }
        if (q->inflight.empty())
            q->cv_retire.wait_for(lk, std::chrono::milliseconds(5));
        else
            q->cv_retire.wait_for(lk, std::chrono::microseconds(q->cfg.poll_us));
    }
}

void scheduler(hsma_queue *q) {
    const bool hip = q->cfg.backend == HSMA_BACKEND_HIP;
    if (hip) (void)hipSetDevice(q->device);
    std::unique_lock<std::mutex> lk(q->mu);
    for (;;) {
        const double t = clock_ns();
        // 1. completions are the retirer's (above)
        free_deferred(q, lk);
        // 2. admission, strictly in arrival order
        std::vector<Req *> adm;
        while (!q->pending.empty() && q->n_inflight < q->cfg.max_inflight) {
            Req *r = q->pending.front();
            const size_t f = footprint(r->r);
            if (q->budget_used + f > q->cfg.hbm_budget_bytes) break;
            q->pending.pop_front();
            q->budget_used += f;
            r->held = f;
            q->budget_peak = std::max(q->budget_peak, q->budget_used);
            q->n_inflight++;
            r->state = RUNNING;
            r->t_admit = t;
            adm.push_back(r);
        }
        if (!adm.empty()) {
            lk.unlock();
            const double t0 = clock_ns();
            if (hip) launch_admitted(q, adm);
            else launch_simulated(q, adm);
            const double t1 = clock_ns();
            lk.lock();
            q->rounds++;
            q->launch_ns += t1 - t0;
            q->cv_retire.notify_one();
            continue;
        }
        if (q->closing && q->inflight.empty()) {
            // What is still pending can never be admitted: its budget is held
            // by kept results, and nobody will release them any more.
            while (!q->pending.empty()) {
                Req *r = q->pending.front();
                q->pending.pop_front();
                q->n_inflight++;  // finish() retires one in-flight request
                finish(q, r, t, HSMA_QUEUE_CLOSED);
            }
            break;
        }
        // 3. nothing to launch: wait for arrivals, releases or retirements
        q->cv_sched.wait_for(lk, std::chrono::milliseconds(q->inflight.empty() ? 5 : 1));
    }
    q->stopped = true;
    q->cv_done.notify_all();
}

void fill_info(const Req *r, hsma_request_info *info) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->status = r->state == DONE ? HSMA_SUCCESS : r->state == FAILED ? r->status : HSMA_PENDING;
    info->path = r->path;
    info->t_arrival_ns = r->t_arrival;
    info->t_admit_ns = r->t_admit;
    info->t_done_ns = r->t_done;
    info->A = r->A;
    info->B = r->B;
    info->lda = r->lda;
    info->ldb = r->ldb;
}

hsma_status state_status(const Req *r) {
    return r->state == DONE ? HSMA_SUCCESS : r->state == FAILED ? r->status : HSMA_PENDING;
}

}  // namespace
}  // namespace hsma

extern "C" {

double hsma_clock_ns(void) { return hsma::clock_ns(); }

hsma_status hsma_request_footprint(const hsma_request *req, uint64_t *bytes) {
    if (!req || !bytes) return HSMA_INVALID_POINTER;
    if (req->prob.dtype != HSMA_R64F && req->prob.dtype != HSMA_C64F) return HSMA_INVALID_VALUE;
    if (req->prob.m < 0 || req->prob.n < 0) return HSMA_INVALID_SIZE;
    *bytes = hsma::footprint(*req);
    return HSMA_SUCCESS;
}

hsma_status hsma_queue_create(const hsma_queue_config *cfg, hsma_queue **out) {
    using namespace hsma;
    if (!out) return HSMA_INVALID_POINTER;
    *out = nullptr;
    hsma_queue_config c{};
    if (cfg) c = *cfg;
    if (c.backend != HSMA_BACKEND_HIP && c.backend != HSMA_BACKEND_SIMULATED)
        return HSMA_INVALID_VALUE;
    if (c.max_inflight < 0 || c.n_streams < 0 || c.poll_us < 0 || c.sim_fixed_ns < 0)
        return HSMA_INVALID_VALUE;
    // 32 GiB by default; larger budgets (a third of the 288 GB, say) are for
    // offered loads well above 20 000 requests/s, where 32 GiB holds
    // admission back.
    if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = (uint64_t)32 << 30;
    if (c.max_inflight == 0) c.max_inflight = 8192;
    // Eight streams: an admission round has up to four blocked classes, and
    // rounds overlap (at 20 000 requests/s p50 fell from 27 to 23 ms going
    // from four to eight; more gained nothing).
    if (c.n_streams == 0) c.n_streams = 8;
    if (c.poll_us == 0) c.poll_us = 20;
    if (!(c.sim_flops_per_ns > 0)) c.sim_flops_per_ns = 40000.0;
    hsma_queue *q = new hsma_queue();
    q->cfg = c;
    if (c.backend == HSMA_BACKEND_HIP) {
        hipError_t e = hipGetDevice(&q->device);
        // The small class's stream gets one CU in sixteen to itself and the
        // blocked classes' streams the rest.  A blocked round's products fill
        // every CU with workgroups that run for hundreds of microseconds; a
        // small request's few wavefronts would otherwise wait for a free slot
        // behind them.
        int ncu = 0;
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, q->device);
        std::vector<uint32_t> small_mask, big_mask;
        if (e == hipSuccess && ncu >= 64 && kSmallCuStride > 1) {
            small_mask.assign((size_t)(ncu + 31) / 32, 0u);
            big_mask.assign(small_mask.size(), 0u);
            for (int cu = 0; cu < ncu; ++cu)
                ((cu % kSmallCuStride == 0) ? small_mask : big_mask)[cu / 32] |= 1u << (cu % 32);
        }
        // Each CU-masked stream takes a hardware queue of its own; where the
        // process has too few (GPU_MAX_HW_QUEUES), plain streams are used.
        auto make_all = [&](bool masked) {
            hipError_t r = masked ? hipExtStreamCreateWithCUMask(&q->small_stream, (uint32_t)small_mask.size(),
                                                                 small_mask.data())
                                  : hipStreamCreateWithFlags(&q->small_stream, hipStreamNonBlocking);
            for (int i = 0; r == hipSuccess && i < c.n_streams; ++i) {
                hipStream_t s;
                r = masked ? hipExtStreamCreateWithCUMask(&s, (uint32_t)big_mask.size(), big_mask.data())
                           : hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
                if (r == hipSuccess) q->streams.push_back(s);
            }
            if (r != hipSuccess) {
                for (auto s : q->streams) (void)hipStreamDestroy(s);
                q->streams.clear();
                if (q->small_stream) (void)hipStreamDestroy(q->small_stream);
                q->small_stream = nullptr;
                (void)hipGetLastError();
            }
            return r;
        };
        if (e == hipSuccess) {
            q->cu_reserved = !small_mask.empty() && make_all(true) == hipSuccess;
            if (!q->cu_reserved) e = make_all(false);
        }
        if (e != hipSuccess) {
            for (auto s : q->streams) (void)hipStreamDestroy(s);
            if (q->small_stream) (void)hipStreamDestroy(q->small_stream);
            delete q;
            return hip_fail(e);
        }
    } else {
        q->sim_free_at.assign((size_t)c.n_streams + 1, 0.0);
    }
    q->sched = std::thread(scheduler, q);
    q->retire = std::thread(retirer, q);
    *out = q;
    return HSMA_SUCCESS;
}

hsma_status hsma_queue_submit(hsma_queue *q, const hsma_request *reqs, int64_t count,
                              uint64_t *tickets) {
    using namespace hsma;
    if (!q) return HSMA_INVALID_POINTER;
    if (count < 0) return HSMA_INVALID_SIZE;
    if (count > 0 && (!reqs || !tickets)) return HSMA_INVALID_POINTER;
    for (int64_t i = 0; i < count; ++i) {
        const hsma_request &r = reqs[i];
        const hsma_problem &p = r.prob;
        if (r.input != HSMA_INPUT_DEVICE && r.input != HSMA_INPUT_SYNTHETIC)
            return HSMA_INVALID_VALUE;
        if (r.release_on_completion < 0 || r.release_on_completion > 2)
            return HSMA_INVALID_VALUE;
        const bool syn = r.input == HSMA_INPUT_SYNTHETIC;
        const double al[2] = {p.alpha_re, p.alpha_im};
        static const double dummy = 0.0;
        bool quick = false;
        const int64_t ld_syn = p.m > 1 ? p.m : 1;
        const hsma_status st =
            validate(p.diag, p.dtype, p.m, p.n, al, syn ? &dummy : p.A, syn ? ld_syn : p.lda,
                     syn ? &dummy : p.B, syn ? ld_syn : p.ldb, &quick);
        if (st != HSMA_SUCCESS) return st;
        if (quick) return HSMA_INVALID_SIZE;
        if (p.dtype == HSMA_R64F && p.alpha_im != 0.0) return HSMA_INVALID_VALUE;
        if (footprint(r) > q->cfg.hbm_budget_bytes) {
            std::lock_guard<std::mutex> lk(q->mu);
            q->rejected++;
            return HSMA_TOO_LARGE;
        }
    }
    {
        std::lock_guard<std::mutex> lk(q->mu);
        if (q->closing) return HSMA_QUEUE_CLOSED;
        const double t = clock_ns();
        for (int64_t i = 0; i < count; ++i) {
            Req *r = new Req();
            r->ticket = q->next_ticket++;
            r->r = reqs[i];
            r->t_arrival = reqs[i].t_arrival_ns > 0 ? reqs[i].t_arrival_ns : t;
            q->all[r->ticket] = r;
            q->pending.push_back(r);
            tickets[i] = r->ticket;
            if (q->submitted == 0) q->t_first_submit = std::min(t, r->t_arrival);
            q->submitted++;
        }
    }
    q->cv_sched.notify_one();
    return HSMA_SUCCESS;
}

hsma_status hsma_queue_poll(hsma_queue *q, uint64_t ticket, hsma_request_info *info) {
    if (!q) return HSMA_INVALID_POINTER;
    std::lock_guard<std::mutex> lk(q->mu);
    auto it = q->all.find(ticket);
    if (it == q->all.end()) return HSMA_NOT_FOUND;
    hsma::fill_info(it->second, info);
    return hsma::state_status(it->second);
}

hsma_status hsma_queue_wait(hsma_queue *q, uint64_t ticket, int64_t timeout_ns,
                            hsma_request_info *info) {
    if (!q) return HSMA_INVALID_POINTER;
    std::unique_lock<std::mutex> lk(q->mu);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::nanoseconds(timeout_ns < 0 ? (int64_t)1 << 62 : timeout_ns);
    for (;;) {
        auto it = q->all.find(ticket);
        if (it == q->all.end()) return HSMA_NOT_FOUND;
        const hsma::Req *r = it->second;
        if (r->state == hsma::DONE || r->state == hsma::FAILED) {
            hsma::fill_info(r, info);
            return hsma::state_status(r);
        }
        if (q->stopped) return HSMA_QUEUE_CLOSED;
        if (q->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            // Look the ticket up again: a fire-and-forget request may have
            // finished and been dropped while the lock was released.
            auto again = q->all.find(ticket);
            if (again == q->all.end()) return HSMA_NOT_FOUND;
            hsma::fill_info(again->second, info);
            return hsma::state_status(again->second) == HSMA_PENDING ? HSMA_TIMEOUT
                                                                     : hsma::state_status(again->second);
        }
    }
}

hsma_status hsma_queue_release(hsma_queue *q, uint64_t ticket) {
    if (!q) return HSMA_INVALID_POINTER;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        auto it = q->all.find(ticket);
        if (it == q->all.end()) return HSMA_NOT_FOUND;
        hsma::Req *r = it->second;
        if (r->state != hsma::DONE && r->state != hsma::FAILED) return HSMA_PENDING;
        hsma::release_mem(q, r);
        q->budget_used -= r->held;
        q->all.erase(it);
        delete r;
    }
    {
        std::unique_lock<std::mutex> lk(q->mu);
        hsma::free_deferred(q, lk);
    }
    q->cv_sched.notify_one();
    return HSMA_SUCCESS;
}

hsma_status hsma_queue_stats(hsma_queue *q, hsma_queue_statistics *st) {
    if (!q || !st) return HSMA_INVALID_POINTER;
    std::memset(st, 0, sizeof(*st));
    // Copy under the lock (a fixed-size histogram), summarise after it.
    std::vector<hsma::LatHist> lat(1 + HSMA_LATENCY_CLASSES);
    {
        std::lock_guard<std::mutex> lk(q->mu);
        st->submitted = q->submitted;
        st->rejected = q->rejected;
        st->completed = q->completed;
        st->failed = q->failed;
        st->pending = (int64_t)q->pending.size();
        st->inflight = q->n_inflight;
        st->bytes_in_use = q->budget_used;
        st->bytes_peak = q->budget_peak;
        st->rounds = q->rounds;
        st->launch_ms = q->launch_ns * 1e-6;
        st->t_first_submit_ns = q->t_first_submit;
        st->t_last_done_ns = q->t_last_done;
        for (int c = 0; c <= HSMA_LATENCY_CLASSES; ++c) lat[c] = q->lat[c];
    }
    lat[0].summary(&st->all);
    for (int c = 0; c < HSMA_LATENCY_CLASSES; ++c) lat[1 + c].summary(&st->by_class[c]);
    st->p50_ns = st->all.p50_ns;
    st->p99_ns = st->all.p99_ns;
    st->max_ns = st->all.max_ns;
    st->mean_ns = st->all.mean_ns;
    const double span = st->t_last_done_ns - st->t_first_submit_ns;
    st->solves_per_s = (st->completed > 0 && span > 0) ? (double)st->completed / (span * 1e-9) : 0.0;
    return HSMA_SUCCESS;
}

hsma_status hsma_queue_stats_reset(hsma_queue *q, double t_from_ns) {
    if (!q) return HSMA_INVALID_POINTER;
    std::lock_guard<std::mutex> lk(q->mu);
    for (auto &h : q->lat) h = hsma::LatHist();
    q->stats_from_ns = t_from_ns;
    return HSMA_SUCCESS;
}

hsma_status hsma_queue_destroy(hsma_queue *q) {
    if (!q) return HSMA_SUCCESS;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->closing = true;
    }
    q->cv_sched.notify_one();
    if (q->sched.joinable()) q->sched.join();
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->retire_stop = true;
    }
    q->cv_retire.notify_one();
    if (q->retire.joinable()) q->retire.join();
    {
        std::unique_lock<std::mutex> lk(q->mu);
        for (auto &kv : q->all) {
            hsma::release_mem(q, kv.second);
            delete kv.second;
        }
        hsma::free_deferred(q, lk);
    }
    for (auto s : q->streams) (void)hipStreamSynchronize(s);
    if (q->small_stream) (void)hipStreamSynchronize(q->small_stream);
    for (auto s : q->streams) (void)hipStreamDestroy(s);
    if (q->small_stream) (void)hipStreamDestroy(q->small_stream);
    delete q;
    return HSMA_SUCCESS;
}

}  // extern "C"
