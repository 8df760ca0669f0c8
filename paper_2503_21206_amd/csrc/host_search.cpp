// Host stages of PilotANN (section 4.1): residual refinement (stage 2) and the final
// traversal (stage 3), both Algorithm 1 with exact fp32 distances on the full vectors in
// host RAM, plus the thread pool that runs them across queries.
#include <immintrin.h>
#include <sched.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "common.hpp"
#include "host.hpp"

namespace pa {

// ------------------------------------------------------------------ thread pool

ThreadPool::ThreadPool(int threads) {
    for (int i = 1; i < threads; ++i) workers_.emplace_back(&ThreadPool::worker_loop, this, i);
}

ThreadPool::~ThreadPool() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_start_.notify_all();
    for (auto& t : workers_) t.join();
}

void ThreadPool::worker_loop(int index) {
    uint64_t seen = 0;
    while (true) {
        const std::function<void(int64_t, int)>* job;
        int64_t n;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_start_.wait(lk, [&] { return stop_ || generation_ != seen; });
            if (stop_) return;
            seen = generation_;
            job = job_;
            n = job_n_;
        }
        for (int64_t i = next_.fetch_add(1); i < n; i = next_.fetch_add(1)) (*job)(i, index);
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (--active_ == 0) cv_done_.notify_all();
        }
    }
}

void ThreadPool::parallel_for(int64_t n, const std::function<void(int64_t, int)>& fn) {
    if (n <= 0) return;
    if (workers_.empty() || n == 1) {
        for (int64_t i = 0; i < n; ++i) fn(i, 0);
        return;
    }
    {
        std::lock_guard<std::mutex> lk(mu_);
        job_ = &fn;
        job_n_ = n;
        next_.store(0);
        active_ = static_cast<int>(workers_.size());
        ++generation_;
    }
    cv_start_.notify_all();
    for (int64_t i = next_.fetch_add(1); i < n; i = next_.fetch_add(1)) fn(i, 0);
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return active_ == 0; });
    job_ = nullptr;
}

int host_core_count() {
    for (const char* var : {"PA_THREADS", "OMP_NUM_THREADS"}) {
        const char* s = std::getenv(var);
        if (s != nullptr) {
            int v = std::atoi(s);
            if (v > 0) return v;
        }
    }
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) {
        int c = CPU_COUNT(&set);
        if (c > 0) return c;
    }
    unsigned h = std::thread::hardware_concurrency();
    return h > 0 ? static_cast<int>(h) : 1;
}

// ------------------------------------------------------------------ distances

namespace {

// Every distance is accumulated in fp64 (the difference of two floats and its square are
// exact there) and rounded once to fp32, so the single-precision value the search
// compares (section 6.1) is the exact distance correctly rounded, up to the fp64 sum's
// own ~D * 2^-53 relative error: the same value the device kernels produce, independent of
// the summation order.  The query is widened to fp64 once per search.

float l2_scalar(const double* q, const float* x, int D) {
    double s = 0.0;
    for (int i = 0; i < D; ++i) {
        const double d = q[i] - static_cast<double>(x[i]);
        s += d * d;
    }
    return static_cast<float>(s);
}
float ip_scalar(const double* q, const float* x, int D) {
    double s = 0.0;
    for (int i = 0; i < D; ++i) s += q[i] * static_cast<double>(x[i]);
    return static_cast<float>(-s);
}

__attribute__((target("avx2,fma"))) double hsum256d(__m256d v) {
    __m128d lo = _mm256_castpd256_pd128(v);
    __m128d hi = _mm256_extractf128_pd(v, 1);
    lo = _mm_add_pd(lo, hi);
    return _mm_cvtsd_f64(_mm_add_sd(lo, _mm_unpackhi_pd(lo, lo)));
}

__attribute__((target("avx2,fma"))) float l2_avx2(const double* q, const float* x, int D) {
    __m256d s0 = _mm256_setzero_pd(), s1 = _mm256_setzero_pd();
    int i = 0;
    for (; i + 8 <= D; i += 8) {
        __m256d d0 = _mm256_sub_pd(_mm256_loadu_pd(q + i), _mm256_cvtps_pd(_mm_loadu_ps(x + i)));
        __m256d d1 = _mm256_sub_pd(_mm256_loadu_pd(q + i + 4), _mm256_cvtps_pd(_mm_loadu_ps(x + i + 4)));
        s0 = _mm256_fmadd_pd(d0, d0, s0);
        s1 = _mm256_fmadd_pd(d1, d1, s1);
    }
    double s = hsum256d(_mm256_add_pd(s0, s1));
    for (; i < D; ++i) {
        const double d = q[i] - static_cast<double>(x[i]);
        s += d * d;
    }
    return static_cast<float>(s);
}

__attribute__((target("avx2,fma"))) float ip_avx2(const double* q, const float* x, int D) {
    __m256d s0 = _mm256_setzero_pd(), s1 = _mm256_setzero_pd();
    int i = 0;
    for (; i + 8 <= D; i += 8) {
        s0 = _mm256_fmadd_pd(_mm256_loadu_pd(q + i), _mm256_cvtps_pd(_mm_loadu_ps(x + i)), s0);
        s1 = _mm256_fmadd_pd(_mm256_loadu_pd(q + i + 4), _mm256_cvtps_pd(_mm_loadu_ps(x + i + 4)), s1);
    }
    double s = hsum256d(_mm256_add_pd(s0, s1));
    for (; i < D; ++i) s += q[i] * static_cast<double>(x[i]);
    return static_cast<float>(-s);
}

__attribute__((target("avx512f"))) float l2_avx512(const double* q, const float* x, int D) {
    __m512d s0 = _mm512_setzero_pd(), s1 = _mm512_setzero_pd();
    int i = 0;
    for (; i + 16 <= D; i += 16) {
        __m512d d0 = _mm512_sub_pd(_mm512_loadu_pd(q + i), _mm512_cvtps_pd(_mm256_loadu_ps(x + i)));
        __m512d d1 = _mm512_sub_pd(_mm512_loadu_pd(q + i + 8), _mm512_cvtps_pd(_mm256_loadu_ps(x + i + 8)));
        s0 = _mm512_fmadd_pd(d0, d0, s0);
        s1 = _mm512_fmadd_pd(d1, d1, s1);
    }
    for (; i + 8 <= D; i += 8) {
        __m512d d0 = _mm512_sub_pd(_mm512_loadu_pd(q + i), _mm512_cvtps_pd(_mm256_loadu_ps(x + i)));
        s0 = _mm512_fmadd_pd(d0, d0, s0);
    }
    double s = _mm512_reduce_add_pd(_mm512_add_pd(s0, s1));
    for (; i < D; ++i) {
        const double d = q[i] - static_cast<double>(x[i]);
        s += d * d;
    }
    return static_cast<float>(s);
}

__attribute__((target("avx512f"))) float ip_avx512(const double* q, const float* x, int D) {
    __m512d s0 = _mm512_setzero_pd(), s1 = _mm512_setzero_pd();
    int i = 0;
    for (; i + 16 <= D; i += 16) {
        s0 = _mm512_fmadd_pd(_mm512_loadu_pd(q + i), _mm512_cvtps_pd(_mm256_loadu_ps(x + i)), s0);
        s1 = _mm512_fmadd_pd(_mm512_loadu_pd(q + i + 8), _mm512_cvtps_pd(_mm256_loadu_ps(x + i + 8)), s1);
    }
    for (; i + 8 <= D; i += 8) s0 = _mm512_fmadd_pd(_mm512_loadu_pd(q + i), _mm512_cvtps_pd(_mm256_loadu_ps(x + i)), s0);
    double s = _mm512_reduce_add_pd(_mm512_add_pd(s0, s1));
    for (; i < D; ++i) s += q[i] * static_cast<double>(x[i]);
    return static_cast<float>(-s);
}

// The query widened to fp64, one buffer per thread.
const double* widen_query(const float* q, int D) {
    thread_local std::vector<double> buf;
    buf.assign(q, q + D);
    return buf.data();
}

inline void prefetch_row(const float* p, int D) {
    const char* c = reinterpret_cast<const char*>(p);
    const int bytes = D * 4;
    for (int off = 0; off < bytes; off += 64) _mm_prefetch(c + off, _MM_HINT_T0);
}

inline bool key_less(float da, int32_t ia, float db, int32_t ib) {
    return da < db || (da == db && ia < ib);
}

// Offer (d, v) to C (sorted, at most ef).  Returns the insert position or -1.
inline int offer(std::vector<Cand>& C, int ef, float d, int32_t v) {
    if (static_cast<int>(C.size()) == ef && !key_less(d, v, C.back().d, C.back().id)) return -1;
    auto it = std::lower_bound(C.begin(), C.end(), Cand{d, v, false}, [](const Cand& a, const Cand& b) {
        return key_less(a.d, a.id, b.d, b.id);
    });
    int pos = static_cast<int>(it - C.begin());
    C.insert(it, Cand{d, v, false});
    if (static_cast<int>(C.size()) > ef) C.pop_back();
    return pos;
}

// Algorithm 1 loop steps on graph g until no unchecked entry or max_steps (<0: no limit).
// Memory-level parallelism: the rows of all fresh neighbours are prefetched before any of
// them is scored, and the adjacency row of the next unchecked candidate is prefetched
// while the current one is processed (a guess: an insertion may still precede it).
int run_steps(const StageContext& ctx, const HostGraph& g, const double* q, int ef, int max_steps,
              Visited& vis, std::vector<Cand>& C, int32_t& n_dist) {
    int steps = 0;
    size_t lb = 0;
    int32_t fresh[1024];
    while (max_steps < 0 || steps < max_steps) {
        size_t pos = lb;
        while (pos < C.size() && C[pos].checked) ++pos;
        if (pos >= C.size()) break;
        C[pos].checked = true;
        lb = pos + 1;
        const int32_t u = C[pos].id;
        ++steps;
        size_t nxt = pos + 1;
        while (nxt < C.size() && C[nxt].checked) ++nxt;
        if (nxt < C.size()) __builtin_prefetch(g.adj + static_cast<int64_t>(C[nxt].id) * g.R);
        const int32_t* row = g.adj + static_cast<int64_t>(u) * g.R;
        int nf = 0;
        for (int j = 0; j < g.R; ++j) {
            const int32_t v = row[j];
            if (v < 0) break;
            if (!vis.test_and_set(v)) {
                fresh[nf++] = v;
                prefetch_row(ctx.X + static_cast<int64_t>(v) * ctx.D, ctx.D);
            }
        }
        for (int j = 0; j < nf; ++j) {
            const int32_t v = fresh[j];
            const float d = ctx.dist(q, ctx.X + static_cast<int64_t>(v) * ctx.D, ctx.D);
            ++n_dist;
            const int p = offer(C, ef, d, v);
            if (p >= 0 && static_cast<size_t>(p) < lb) lb = static_cast<size_t>(p);
        }
    }
    return steps;
}

void emit_topk(const std::vector<Cand>& C, int k, int64_t* out_ids, float* out_d) {
    for (int i = 0; i < k; ++i) {
        if (i < static_cast<int>(C.size())) {
            out_ids[i] = C[i].id;
            out_d[i] = C[i].d;
        } else {
            out_ids[i] = -1;
            out_d[i] = __builtin_huge_valf();
        }
    }
}

}  // namespace

DistFn pick_distance(int metric) {
    static const bool has512 = __builtin_cpu_supports("avx512f");
    static const bool has2 = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
    if (metric == PA_METRIC_L2) return has512 ? l2_avx512 : (has2 ? l2_avx2 : l2_scalar);
    return has512 ? ip_avx512 : (has2 ? ip_avx2 : ip_scalar);
}

void Visited::reset(int64_t n) {
    bits_.assign(static_cast<size_t>((n + 63) / 64), 0);
    touched_.clear();
    touched_.reserve(4096);
}

void Visited::next_epoch() {
    for (uint32_t w : touched_) bits_[w] = 0;
    touched_.clear();
}

void host_stages_one(const StageContext& ctx, const float* qf, const int32_t* beam, int n_beam, int ef_cpu,
                     int k, int refine_steps, Visited& vis, std::vector<Cand>& C, int64_t* out_ids,
                     float* out_d, StageCounters& cnt, bool final_stage) {
    vis.next_epoch();
    C.clear();
    const double* q = widen_query(qf, ctx.D);
    // stage 2: full distances of the handed-off candidates, re-rank, keep ef_cpu
    // all hand-off rows are requested before the first is scored
    constexpr int kAhead = 16;
    for (int i = 0; i < std::min(n_beam, kAhead); ++i)
        if (beam[i] >= 0 && beam[i] < ctx.N) prefetch_row(ctx.X + static_cast<int64_t>(beam[i]) * ctx.D, ctx.D);
    for (int i = 0; i < n_beam; ++i) {
        if (i + kAhead < n_beam && beam[i + kAhead] >= 0 && beam[i + kAhead] < ctx.N)
            prefetch_row(ctx.X + static_cast<int64_t>(beam[i + kAhead]) * ctx.D, ctx.D);
        const int32_t v = beam[i];
        if (v < 0 || v >= ctx.N) continue;
        if (vis.test_and_set(v)) continue;
        C.push_back(Cand{ctx.dist(q, ctx.X + static_cast<int64_t>(v) * ctx.D, ctx.D), v, false});
        ++cnt.dist2;
    }
    std::sort(C.begin(), C.end(), [](const Cand& a, const Cand& b) { return key_less(a.d, a.id, b.d, b.id); });
    if (static_cast<int>(C.size()) > ef_cpu) C.resize(static_cast<size_t>(ef_cpu));
    // stage 2: refinement steps on the subgraph
    if (refine_steps > 0) run_steps(ctx, ctx.sub, q, ef_cpu, refine_steps, vis, C, cnt.dist2);
    if (!final_stage) {
        emit_topk(C, k, out_ids, out_d);
        return;
    }
    // stage 3: Algorithm 1 on the full graph, candidates unchecked, visited kept
    for (auto& c : C) c.checked = false;
    const int ef = std::max(ef_cpu, k);
    int32_t d3 = 0;
    cnt.exp3 += run_steps(ctx, ctx.full, q, ef, -1, vis, C, d3);
    cnt.dist3 += d3;
    emit_topk(C, k, out_ids, out_d);
}

void host_search_one(const StageContext& ctx, const float* qf, const int32_t* entries, int E, int ef, int k,
                     Visited& vis, std::vector<Cand>& C, int64_t* out_ids, float* out_d, StageCounters& cnt) {
    vis.next_epoch();
    C.clear();
    const double* q = widen_query(qf, ctx.D);
    const int efe = std::max(ef, k);
    int32_t d3 = 0;
    for (int i = 0; i < E; ++i) {
        const int32_t v = entries[i];
        if (v < 0 || v >= ctx.N) continue;
        if (vis.test_and_set(v)) continue;
        ++d3;
        offer(C, efe, ctx.dist(q, ctx.X + static_cast<int64_t>(v) * ctx.D, ctx.D), v);
    }
    cnt.exp3 += run_steps(ctx, ctx.full, q, efe, -1, vis, C, d3);
    cnt.dist3 += d3;
    emit_topk(C, k, out_ids, out_d);
}

}  // namespace pa
