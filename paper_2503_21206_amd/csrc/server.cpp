// Serving loop: continuous batching of single-query requests of uneven k and ef over an
// index.  The HBM budget covers the index's own tables and the slots' device arenas; a
// scheduler thread takes queued requests in arrival order into a free slot while the
// micro-batch's real device footprint (at its largest list size) fits the slot's arena,
// and enqueues projection, routing, entry selection and stage 1 for the micro-batch on
// that slot's stream (several slots overlap on the GPU).  A completion thread waits for
// each micro-batch in admission order, runs stages 2-3 for its requests on the host pool
// and publishes the results.  A request's result does not depend on the other requests:
// every step computes per query, the entry list of a query is its own prefix of length
// min(ef, n/r), and stage 1 takes a per-query list size.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "common.hpp"
#include "host.hpp"
#include "index.hpp"

namespace pa {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    std::vector<float> q;
    int k = 0, ef = 0;
    uint64_t tag = 0;
    double t_submit = 0, t_admit = 0;
};

struct Result {
    pa_result_info info{};
    std::vector<int64_t> ids;
    std::vector<float> d;
};

// One micro-batch slot: a stream and a device arena that is carved, per micro-batch, into
// the buffers of its m requests at the batch's largest list size ef_max.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    DevBuf arena;
    void *q = nullptr, *qr = nullptr, *cl = nullptr, *eid = nullptr, *ed = nullptr, *bid = nullptr, *bd = nullptr,
         *cnt = nullptr, *efq = nullptr, *scr = nullptr;
    PinBuf q_pin, beam_pin, efq_pin;
    std::vector<Request> reqs;
    int ef_max = 0;
    int64_t bytes = 0;
    bool busy = false;
};

}  // namespace
}  // namespace pa

struct pa_server {
    pa_index* idx = nullptr;
    pa_server_params p{};
    std::chrono::steady_clock::time_point t0;
    std::vector<std::unique_ptr<pa::Slot>> slots;
    std::deque<pa::Request> pending;
    std::deque<pa::Slot*> inflight;
    std::deque<pa::Result> done;
    int64_t submitted = 0, completed = 0;
    int64_t bytes_in_flight = 0;
    int64_t arena_bytes = 0;  // device bytes of each slot's arena
    int64_t max_batch_seen = 0, batches = 0;
    std::string error;
    pa_status error_code = PA_OK;
    bool stop = false;
    std::mutex mu;
    std::condition_variable cv_sched, cv_comp, cv_done;
    std::thread scheduler, completer;
    std::unique_ptr<pa::ThreadPool> pool;
    std::vector<pa::Visited> vis;
    std::vector<std::vector<pa::Cand>> lists;
};

namespace pa {
namespace {

double now_us(const pa_server* s) {
    return std::chrono::duration<double, std::micro>(Clock::now() - s->t0).count();
}

int entries_for(const pa_index* idx, int ef) { return std::min(ef, idx->n_b); }

constexpr int64_t kAlign = 256;
int64_t aligned(int64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Device bytes of a micro-batch of m requests whose largest list size is ef: the queries,
// reduced queries, clusters, entries (ids and distances), stage-1 lists (ids and
// distances) and counters at stride ef, the per-query list sizes and the entry-selection
// scratch, each buffer rounded up to 256 bytes.
int64_t batch_bytes(const pa_index* idx, int64_t m, int ef) {
    const int64_t D = idx->p.dim, d_r = idx->p.d_r, E = entries_for(idx, ef);
    return aligned(4 * m * D) + aligned(4 * m * d_r) + aligned(4 * m) + 2 * aligned(4 * m * E) +
           2 * aligned(4 * m * ef) + aligned(16 * m) + aligned(4 * m) +
           aligned(4 * static_cast<int64_t>(select_entries_scratch_ints(m, idx->p.r)));
}

// Points the slot's buffers into its arena for m requests at stride ef.
void carve(const pa_index* idx, Slot& sl, int64_t m, int ef) {
    const int64_t D = idx->p.dim, d_r = idx->p.d_r, E = entries_for(idx, ef);
    auto* base = static_cast<char*>(sl.arena.p);
    int64_t off = 0;
    auto take = [&](int64_t b) {
        void* p = base + off;
        off += aligned(b);
        return p;
    };
    sl.q = take(4 * m * D);
    sl.qr = take(4 * m * d_r);
    sl.cl = take(4 * m);
    sl.eid = take(4 * m * E);
    sl.ed = take(4 * m * E);
    sl.bid = take(4 * m * ef);
    sl.bd = take(4 * m * ef);
    sl.cnt = take(16 * m);
    sl.efq = take(4 * m);
    sl.scr = take(4 * static_cast<int64_t>(select_entries_scratch_ints(m, idx->p.r)));
    require(off <= static_cast<int64_t>(sl.arena.bytes), "micro-batch exceeds its slot", PA_EINTERNAL);
}

void fail_all(pa_server* s, pa_status code, const std::string& msg) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error_code == PA_OK) {
        s->error_code = code;
        s->error = msg;
    }
    s->stop = true;
    s->cv_sched.notify_all();
    s->cv_comp.notify_all();
    s->cv_done.notify_all();
}

void launch_slot(pa_server* s, Slot& sl) {
    pa_index* idx = s->idx;
    const int D = idx->p.dim, d_r = idx->p.d_r, r = idx->p.r;
    const int64_t m = static_cast<int64_t>(sl.reqs.size());
    const int ef = sl.ef_max;
    const int E = entries_for(idx, ef);
    auto* qp = static_cast<float*>(sl.q_pin.p);
    auto* ep = static_cast<int32_t*>(sl.efq_pin.p);
    for (int64_t i = 0; i < m; ++i) {
        std::memcpy(qp + i * D, sl.reqs[i].q.data(), sizeof(float) * D);
        ep[i] = sl.reqs[i].ef;
    }
    carve(idx, sl, m, ef);
    hipStream_t st = sl.stream;
    PA_HIP(hipMemcpyAsync(sl.q, qp, sizeof(float) * m * D, hipMemcpyHostToDevice, st));
    PA_HIP(hipMemcpyAsync(sl.efq, ep, sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
    launch_project(static_cast<const float*>(sl.q), m, D, static_cast<const float*>(idx->V_dev.p), d_r, sl.qr, PA_F32,
                   static_cast<const float*>(idx->cent_dev.p), r, static_cast<int32_t*>(sl.cl), st);
    index_select_entries(idx, static_cast<const float*>(sl.qr), static_cast<const int32_t*>(sl.cl), m, E,
                         static_cast<int32_t*>(sl.eid), static_cast<float*>(sl.ed), static_cast<int32_t*>(sl.scr), st);
    launch_beam(static_cast<const float*>(sl.qr), m, d_r, idx->Xr_dev.p, idx->p.xr_dtype, idx->xr_rows,
                static_cast<const int32_t*>(idx->adj_dev.p), idx->R_sub, static_cast<const int32_t*>(sl.eid), E, ef,
                idx->p.metric, 0, static_cast<int32_t*>(sl.bid), static_cast<float*>(sl.bd),
                static_cast<int32_t*>(sl.cnt), st, static_cast<const int32_t*>(sl.efq), PA_VISITED_EXACT,
                index_out_map(idx), false);  // the host stages read only the ids
    PA_HIP(hipMemcpyAsync(sl.beam_pin.p, sl.bid, sizeof(int32_t) * m * ef, hipMemcpyDeviceToHost, st));
    PA_HIP(hipEventRecord(sl.done, st));
}

void scheduler_loop(pa_server* s) {
    try {
        PA_HIP(hipSetDevice(s->idx->p.device));
        while (true) {
            Slot* sl = nullptr;
            {
                std::unique_lock<std::mutex> lk(s->mu);
                s->cv_sched.wait(lk, [&] {
                    if (s->stop) return true;
                    if (s->pending.empty()) return false;
                    for (auto& x : s->slots)
                        if (!x->busy) return true;
                    return false;
                });
                if (s->stop) return;
                for (auto& x : s->slots)
                    if (!x->busy) {
                        sl = x.get();
                        break;
                    }
                sl->reqs.clear();
                sl->ef_max = 0;
                sl->bytes = 0;
                const double t = now_us(s);
                // the head of the queue joins while the micro-batch, at its largest list
                // size, still fits the slot's arena (one request always fits: see create)
                while (!s->pending.empty() && static_cast<int>(sl->reqs.size()) < s->p.max_batch) {
                    const int ef = std::max(sl->ef_max, s->pending.front().ef);
                    const int64_t b = batch_bytes(s->idx, static_cast<int64_t>(sl->reqs.size()) + 1, ef);
                    if (b > s->arena_bytes) break;
                    Request rq = std::move(s->pending.front());
                    s->pending.pop_front();
                    rq.t_admit = t;
                    sl->bytes = b;
                    sl->ef_max = ef;
                    sl->reqs.push_back(std::move(rq));
                }
                s->bytes_in_flight += sl->bytes;
                sl->busy = true;
                s->batches += 1;
                s->max_batch_seen = std::max<int64_t>(s->max_batch_seen, static_cast<int64_t>(sl->reqs.size()));
            }
            launch_slot(s, *sl);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->inflight.push_back(sl);
            }
            s->cv_comp.notify_all();
        }
    } catch (const Error& e) {
        fail_all(s, e.code, e.what());
    } catch (const std::exception& e) {
        fail_all(s, PA_EINTERNAL, e.what());
    }
}

void completion_loop(pa_server* s) {
    try {
        PA_HIP(hipSetDevice(s->idx->p.device));
        pa_index* idx = s->idx;
        StageContext ctx{idx->X, idx->N, idx->p.dim, pick_distance(idx->p.metric),
                         HostGraph{idx->sub_adj.data(), idx->R_sub}, HostGraph{idx->full_adj.data(), idx->R_full}};
        while (true) {
            Slot* sl = nullptr;
            {
                std::unique_lock<std::mutex> lk(s->mu);
                s->cv_comp.wait(lk, [&] { return s->stop || !s->inflight.empty(); });
                if (s->inflight.empty()) return;  // stopping with nothing in flight
                sl = s->inflight.front();
            }
            PA_HIP(hipEventSynchronize(sl->done));
            const int64_t m = static_cast<int64_t>(sl->reqs.size());
            const int ef_max = sl->ef_max;
            std::vector<Result> out(static_cast<size_t>(m));
            const auto* beam = static_cast<const int32_t*>(sl->beam_pin.p);
            s->pool->parallel_for(m, [&](int64_t i, int w) {
                const Request& rq = sl->reqs[i];
                Result& r = out[i];
                r.ids.resize(rq.k);
                r.d.resize(rq.k);
                StageCounters c;
                host_stages_one(ctx, rq.q.data(), beam + i * ef_max, rq.ef, rq.ef, rq.k, idx->p.refine_steps,
                                s->vis[w], s->lists[w], r.ids.data(), r.d.data(), c);
                r.info.tag = rq.tag;
                r.info.k = rq.k;
                r.info.ef = rq.ef;
                r.info.t_submit_us = rq.t_submit;
                r.info.t_admit_us = rq.t_admit;
            });
            const double t = now_us(s);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                for (auto& r : out) {
                    r.info.t_done_us = t;
                    s->done.push_back(std::move(r));
                }
                s->completed += m;
                s->bytes_in_flight -= sl->bytes;
                sl->busy = false;
                s->inflight.pop_front();
            }
            s->cv_sched.notify_all();
            s->cv_done.notify_all();
        }
    } catch (const Error& e) {
        fail_all(s, e.code, e.what());
    } catch (const std::exception& e) {
        fail_all(s, PA_EINTERNAL, e.what());
    }
}

void alloc_slot(pa_server* s, Slot& sl) {
    pa_index* idx = s->idx;
    const int64_t B = s->p.max_batch, D = idx->p.dim, ef = PA_MAX_EF;
    int64_t& used = idx->hbm_used;
    PA_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    PA_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    sl.arena.ensure(static_cast<size_t>(s->arena_bytes), used, 0);
    sl.q_pin.ensure(sizeof(float) * B * D);
    sl.beam_pin.ensure(sizeof(int32_t) * B * ef);
    sl.efq_pin.ensure(sizeof(int32_t) * B);
}

void release_slots(pa_server* s) {
    for (auto& sl : s->slots) {
        if (sl->done) (void)hipEventDestroy(sl->done);
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
        sl->done = nullptr;
        sl->stream = nullptr;
    }
}

void shutdown(pa_server* s) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->cv_comp.notify_all();
    if (s->scheduler.joinable()) s->scheduler.join();
    if (s->completer.joinable()) s->completer.join();
    // anything the completion thread did not consume is still on the GPU: wait for it
    for (auto& sl : s->slots)
        if (sl->done) (void)hipEventSynchronize(sl->done);
    release_slots(s);
}

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" {

pa_status pa_server_create(pa_index* idx, const pa_server_params* params, pa_server** out) {
    return guarded([&] {
        require(idx && params && out, "null pointer");
        require(idx->has_data && idx->has_proj && idx->has_sub && idx->has_entries,
                "the index needs data, a projection, a subgraph and entries", PA_ESTATE);
        pa_server_params p = *params;
        if (p.max_batch <= 0) p.max_batch = 1024;
        if (p.streams <= 0) p.streams = 2;
        if (p.max_k <= 0) p.max_k = 128;
        require(p.hbm_budget > 0, "hbm_budget must be positive");
        require(p.max_batch <= (1 << 20) && p.streams <= 16 && p.max_k <= 4096, "server limits out of range");
        PA_HIP(hipSetDevice(idx->p.device));
        auto s = std::make_unique<pa_server>();
        s->idx = idx;
        s->p = p;
        s->t0 = Clock::now();
        // the budget holds the index first; the rest is split into the slots' arenas, each
        // no larger than a full micro-batch at the largest list size
        const int64_t index_bytes = idx->hbm_used;
        const int64_t per_slot = (p.hbm_budget - index_bytes) / p.streams / kAlign * kAlign;
        const int64_t one = batch_bytes(idx, 1, PA_MAX_EF);
        require(per_slot >= one, "hbm_budget (" + std::to_string(p.hbm_budget) + " bytes) cannot hold the index (" +
                                     std::to_string(index_bytes) + " bytes) and one request of list size " +
                                     std::to_string(PA_MAX_EF) + " per slot (" + std::to_string(one) + " bytes)",
                PA_EHBM);
        s->arena_bytes = std::min(per_slot, batch_bytes(idx, p.max_batch, PA_MAX_EF));
        for (int i = 0; i < p.streams; ++i) {
            s->slots.push_back(std::make_unique<Slot>());
            alloc_slot(s.get(), *s->slots.back());
        }
        int threads = p.threads > 0 ? p.threads : (idx->p.threads > 0 ? idx->p.threads : host_core_count());
        s->pool = std::make_unique<ThreadPool>(threads);
        s->vis.assign(static_cast<size_t>(threads), Visited());
        for (auto& v : s->vis) v.reset(idx->N);
        s->lists.assign(static_cast<size_t>(threads), {});
        pa_server* raw = s.get();
        s->scheduler = std::thread(scheduler_loop, raw);
        s->completer = std::thread(completion_loop, raw);
        *out = s.release();
    });
}

pa_status pa_server_submit(pa_server* s, const float* q_host, int32_t k, int32_t ef, uint64_t tag) {
    return guarded([&] {
        require(s && q_host, "null pointer");
        require(k >= 1 && k <= s->p.max_k, "k must be in [1, max_k]");
        require(ef >= 1 && ef <= PA_MAX_EF, "ef must be in [1, 512]");
        const int D = s->idx->p.dim;
        for (int i = 0; i < D; ++i)
            if (!std::isfinite(q_host[i])) fail(PA_ENONFINITE, "query holds a non-finite value");
        Request rq;
        rq.q.assign(q_host, q_host + D);
        rq.k = k;
        rq.ef = std::max(ef, k);
        rq.ef = std::min(rq.ef, static_cast<int>(PA_MAX_EF));
        rq.tag = tag;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->error_code != PA_OK) fail(s->error_code, "server failed: " + s->error);
            require(!s->stop, "server is stopped", PA_ESTATE);
            rq.t_submit = now_us(s);
            s->pending.push_back(std::move(rq));
            s->submitted += 1;
        }
        s->cv_sched.notify_all();
    });
}

pa_status pa_server_poll(pa_server* s, int32_t max_results, pa_result_info* info, int64_t* ids, float* dists,
                         int32_t* n_out) {
    return guarded([&] {
        require(s && n_out && (max_results == 0 || (info && ids && dists)), "null pointer");
        std::lock_guard<std::mutex> lk(s->mu);
        int n = 0;
        while (n < max_results && !s->done.empty()) {
            Result& r = s->done.front();
            info[n] = r.info;
            for (int j = 0; j < s->p.max_k; ++j) {
                ids[static_cast<int64_t>(n) * s->p.max_k + j] = j < r.info.k ? r.ids[j] : -1;
                dists[static_cast<int64_t>(n) * s->p.max_k + j] = j < r.info.k ? r.d[j] : __builtin_huge_valf();
            }
            s->done.pop_front();
            ++n;
        }
        *n_out = n;
        if (n == 0 && s->error_code != PA_OK) fail(s->error_code, "server failed: " + s->error);
    });
}

pa_status pa_server_drain(pa_server* s) {
    return guarded([&] {
        require(s, "null pointer");
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->completed == s->submitted || s->error_code != PA_OK; });
        if (s->error_code != PA_OK) fail(s->error_code, "server failed: " + s->error);
    });
}

pa_status pa_server_stats(const pa_server* s, int64_t* submitted, int64_t* completed, int64_t* batches,
                          int64_t* max_batch, int64_t* bytes_in_flight) {
    return guarded([&] {
        require(s, "null pointer");
        auto* m = const_cast<pa_server*>(s);
        std::lock_guard<std::mutex> lk(m->mu);
        if (submitted) *submitted = m->submitted;
        if (completed) *completed = m->completed;
        if (batches) *batches = m->batches;
        if (max_batch) *max_batch = m->max_batch_seen;
        if (bytes_in_flight) *bytes_in_flight = m->bytes_in_flight;
    });
}

pa_status pa_server_destroy(pa_server* s) {
    return guarded([&] {
        if (!s) return;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_done.wait(lk, [&] { return s->completed == s->submitted || s->error_code != PA_OK; });
        }
        shutdown(s);
        int64_t held = 0;
        for (auto& sl : s->slots) held += static_cast<int64_t>(sl->arena.bytes);
        for (auto& sl : s->slots) sl->arena.release();
        s->idx->hbm_used -= held;
        delete s;
    });
}

}  // extern "C"
