// Host-side building blocks: a persistent thread pool, SIMD distance functions and the
// stage-2/3 traversals.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace pa {

// Fixed-size pool; parallel_for runs fn(i) for i in [0, n) on all workers and the caller.
class ThreadPool {
public:
    explicit ThreadPool(int threads);
    ~ThreadPool();
    ThreadPool(const ThreadPool&) = delete;
    ThreadPool& operator=(const ThreadPool&) = delete;
    int size() const { return static_cast<int>(workers_.size()) + 1; }
    // fn(i, worker_index); worker_index in [0, size())
    void parallel_for(int64_t n, const std::function<void(int64_t, int)>& fn);

private:
    void worker_loop(int index);
    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_start_, cv_done_;
    const std::function<void(int64_t, int)>* job_ = nullptr;
    int64_t job_n_ = 0;
    std::atomic<int64_t> next_{0};
    uint64_t generation_ = 0;
    int active_ = 0;
    bool stop_ = false;
};

int host_core_count();

// distance from a query widened to fp64 to an fp32 vector of length D (squared L2 or
// -dot), accumulated in fp64 and rounded once to fp32
using DistFn = float (*)(const double*, const float*, int);
DistFn pick_distance(int metric);

// Per-thread visited table: one bit per node (N/8 bytes, small enough to stay in a core's
// L2 at N = 1M) and the list of words a query touched, which are cleared when the next
// query starts.
class Visited {
public:
    void reset(int64_t n);
    void next_epoch();
    bool test_and_set(int32_t v) {
        const size_t w = static_cast<uint32_t>(v) >> 6;
        const uint64_t bit = uint64_t{1} << (v & 63);
        const uint64_t b = bits_[w];
        if (b & bit) return true;
        if (b == 0) touched_.push_back(static_cast<uint32_t>(w));
        bits_[w] = b | bit;
        return false;
    }

private:
    std::vector<uint64_t> bits_;
    std::vector<uint32_t> touched_;
};

// One candidate of the host-side list C.
struct Cand {
    float d;
    int32_t id;
    bool checked;
};

struct HostGraph {
    const int32_t* adj;  // [N][R], -1 padded
    int R;
};

struct StageCounters {
    int32_t dist2 = 0, dist3 = 0, exp3 = 0;
};

struct StageContext {
    const float* X;
    int64_t N;
    int D;
    DistFn dist;
    HostGraph sub;
    HostGraph full;
};

// Stage 2 + stage 3 for one query.  beam: stage-1 ids (n_beam, -1 skipped).
// refine_steps < 0 skips the subgraph steps of stage 2 (candidates are still re-scored);
// final_stage false skips stage 3 (the output is the best k of the stage-2 list).
void host_stages_one(const StageContext& ctx, const float* q, const int32_t* beam, int n_beam,
                     int ef_cpu, int k, int refine_steps, Visited& vis, std::vector<Cand>& C,
                     int64_t* out_ids, float* out_d, StageCounters& cnt, bool final_stage = true);

// Plain Algorithm 1 on the full graph from entries (stage 3 alone).
void host_search_one(const StageContext& ctx, const float* q, const int32_t* entries, int E, int ef,
                     int k, Visited& vis, std::vector<Cand>& C, int64_t* out_ids, float* out_d,
                     StageCounters& cnt);

}  // namespace pa
