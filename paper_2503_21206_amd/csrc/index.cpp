// The index object and the pipelined search of section 4.1 / 4.2: stage 1 and entry
// selection on the GPU in sub-batches, stages 2-3 on host threads, batch b's host work
// overlapping the GPU work of the batches after it.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "host.hpp"
#include "index.hpp"

namespace pa {

void sample_nodes(int64_t N, const int64_t* rowptr, const int32_t* nbrs, const int64_t* order, int64_t n_target,
                  int mode, uint8_t* mask);
void check_subgraph(int64_t N, const int64_t* rowptr, const int32_t* nbrs, const uint8_t* mask, int R);
std::vector<int32_t> pad_rows(int64_t N, const int64_t* rowptr, const int32_t* nbrs, int R);
void build_entries(const float* P, int n_p, int d, int r, const int32_t* init, int iters, int32_t* buckets,
                   float* centroids_out);
void fit_projection_host(const float* X, int64_t N, int D, int d_r, int center, float* V_out, double* evals_out,
                         double* mean_out);

}  // namespace pa

namespace pa {
namespace {

void use_device(const pa_index* idx) { PA_HIP(hipSetDevice(idx->p.device)); }

void ensure_events(pa_index* idx, size_t n) {
    while (idx->events.size() < n) {
        hipEvent_t e;
        PA_HIP(hipEventCreate(&e));
        idx->events.push_back(e);
    }
}

void project_all(pa_index* idx) {
    const int D = idx->p.dim, d_r = idx->p.d_r;
    idx->V_dev.ensure(sizeof(float) * D * d_r, idx->hbm_used, idx->p.hbm_budget);
    PA_HIP(hipMemcpy(idx->V_dev.p, idx->V.data(), sizeof(float) * D * d_r, hipMemcpyHostToDevice));
    idx->has_proj = true;
    index_write_rows(idx);
}

void ensure_pool(pa_index* idx, int threads) {
    if (threads <= 0) threads = idx->p.threads > 0 ? idx->p.threads : host_core_count();
    if (!idx->pool || idx->pool->size() != threads) {
        idx->pool.reset();
        idx->pool = std::make_unique<ThreadPool>(threads);
        idx->vis.assign(static_cast<size_t>(threads), Visited());
        for (auto& v : idx->vis) v.reset(idx->N);
        idx->lists.assign(static_cast<size_t>(threads), {});
    }
}

}  // namespace

void index_select_entries(const pa_index* idx, const float* Qr, const int32_t* cluster, int64_t m, int E,
                          int32_t* ids, float* dists, int32_t* scratch, hipStream_t s) {
    const int r = idx->p.r, d_r = idx->p.d_r;
    if (idx->p.pivot_dtype == PA_FP8E4M3) {
        const int mult = idx->p.preselect > 0 ? idx->p.preselect : 4;
        // at most 1,024 pre-selected pivots per query: a 16-query tile's lists fill the LDS
        const int K = std::min(std::max(E, std::min(mult * E, 1024)), idx->n_b);
        launch_select_entries_chunked(Qr, cluster, m, d_r, static_cast<const float*>(idx->EV_dev.p),
                                      static_cast<const uint8_t*>(idx->EV8_dev.p),
                                      static_cast<const float*>(idx->EVs_dev.p),
                                      static_cast<const float*>(idx->EVn_dev.p),
                                      static_cast<const int32_t*>(idx->EVid_dev.p), r, idx->n_b, E, std::max(K, E),
                                      idx->p.metric, ids, dists, scratch, s);
    } else {
        launch_select_entries(Qr, cluster, m, d_r, static_cast<const float*>(idx->EV_dev.p),
                              static_cast<const float*>(idx->EVn_dev.p), static_cast<const int32_t*>(idx->EVid_dev.p),
                              r, idx->n_b, E, idx->p.metric, ids, dists, scratch, s);
    }
}

int32_t index_device_id(const pa_index* idx, int32_t node) {
    if (!index_compact(idx)) return node;
    const auto it = std::lower_bound(idx->cid.begin(), idx->cid.end(), node);
    return (it != idx->cid.end() && *it == node) ? static_cast<int32_t>(it - idx->cid.begin()) : -1;
}

void index_write_rows(pa_index* idx) {
    const int D = idx->p.dim, d_r = idx->p.d_r;
    const size_t es = dtype_size(idx->p.xr_dtype);
    const bool compact = index_compact(idx);
    idx->xr_rows = 0;
    if (!idx->has_proj || (compact && !idx->has_sub)) return;  // compact rows wait for the sample
    const int64_t n = compact ? static_cast<int64_t>(idx->cid.size()) : idx->N;
    idx->Xr_dev.ensure(std::max<size_t>(16, static_cast<size_t>(n) * d_r * es), idx->hbm_used, idx->p.hbm_budget);
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(std::max<int64_t>(n, 1), (int64_t{256} << 20) / (4 * D)));
    DevBuf stage;
    int64_t dummy = 0;
    stage.ensure(sizeof(float) * chunk * D, dummy, 0);
    std::vector<float> gathered(compact ? static_cast<size_t>(chunk) * D : 0);
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t rows = std::min(chunk, n - r0);
        const float* src = idx->X + r0 * D;
        if (compact) {  // the sampled rows, in device-id order
            for (int64_t i = 0; i < rows; ++i)
                std::memcpy(&gathered[static_cast<size_t>(i) * D], idx->X + static_cast<int64_t>(idx->cid[r0 + i]) * D,
                            sizeof(float) * D);
            src = gathered.data();
        }
        PA_HIP(hipMemcpyAsync(stage.p, src, sizeof(float) * rows * D, hipMemcpyHostToDevice, idx->stream));
        launch_project(static_cast<const float*>(stage.p), rows, D, static_cast<const float*>(idx->V_dev.p), d_r,
                       static_cast<char*>(idx->Xr_dev.p) + static_cast<size_t>(r0) * d_r * es, idx->p.xr_dtype,
                       nullptr, 0, nullptr, idx->stream);
        PA_HIP(hipStreamSynchronize(idx->stream));
    }
    idx->xr_rows = n;
}

void index_upload_subgraph(pa_index* idx) {
    const int R = idx->R_sub;
    if (!index_compact(idx)) {
        idx->adj_dev.ensure(sizeof(int32_t) * idx->sub_adj.size(), idx->hbm_used, idx->p.hbm_budget);
        PA_HIP(hipMemcpy(idx->adj_dev.p, idx->sub_adj.data(), sizeof(int32_t) * idx->sub_adj.size(),
                         hipMemcpyHostToDevice));
        return;
    }
    const int64_t n = static_cast<int64_t>(idx->cid.size());
    std::vector<int32_t> pos(static_cast<size_t>(idx->N), -1);
    for (int64_t i = 0; i < n; ++i) pos[idx->cid[i]] = static_cast<int32_t>(i);
    std::vector<int32_t> adj(static_cast<size_t>(std::max<int64_t>(n, 1)) * R, -1);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t* row = &idx->sub_adj[static_cast<size_t>(idx->cid[i]) * R];
        for (int j = 0; j < R; ++j) {
            if (row[j] < 0) continue;
            require(pos[row[j]] >= 0, "subgraph edge into a node outside the sample");
            adj[static_cast<size_t>(i) * R + j] = pos[row[j]];
        }
    }
    idx->adj_dev.ensure(sizeof(int32_t) * adj.size(), idx->hbm_used, idx->p.hbm_budget);
    PA_HIP(hipMemcpy(idx->adj_dev.p, adj.data(), sizeof(int32_t) * adj.size(), hipMemcpyHostToDevice));
    idx->cid_dev.ensure(sizeof(int32_t) * std::max<int64_t>(n, 1), idx->hbm_used, idx->p.hbm_budget);
    if (n > 0) PA_HIP(hipMemcpy(idx->cid_dev.p, idx->cid.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
}

// The model follows the ensure() calls of this file term by term: project_all (V),
// index_write_rows (X_r), index_upload_subgraph (adjacency, id map), build_entries (pivot
// table, centroids, FP8 codes) and search (its grow-only buffers).
int64_t index_hbm_model(const pa_memory_shape& s, double rho, int d_r) {
    const bool dtype_ok = s.xr_dtype == PA_F32 || s.xr_dtype == PA_F16 || s.xr_dtype == PA_BF16;
    if (s.N <= 0 || s.dim <= 0 || !dtype_ok || (s.pivot_dtype != PA_F32 && s.pivot_dtype != PA_FP8E4M3) ||
        s.R_sub < 1 || s.R_sub > 1024 || s.r < 1 || s.n_pivots < s.r || s.n_pivots % s.r != 0 || s.queries < 0 ||
        s.batch < 0 || s.ef_gpu < 1 || s.ef_gpu > PA_MAX_EF || s.E < 0 || s.E > PA_MAX_EF)
        return -1;
    if (!(rho > 0.0 && rho <= 1.0) || d_r < 16 || d_r > s.dim || d_r > PA_MAX_DR || d_r % 16 != 0) return -1;
    const int64_t D = s.dim, dr = d_r, np = s.n_pivots, r = s.r, R = s.R_sub;
    const int64_t es = static_cast<int64_t>(dtype_size(s.xr_dtype));
    const int64_t ns = std::llround(rho * static_cast<double>(s.N));
    const int64_t n = s.compact ? ns : s.N;
    int64_t b = 4 * D * dr;                                  // V
    b += std::max<int64_t>(16, n * dr * es);                 // X_r
    b += 4 * std::max<int64_t>(n, 1) * R;                    // device adjacency
    if (s.compact) b += 4 * std::max<int64_t>(ns, 1);        // device-to-node ids
    b += 4 * np * dr + 4 * np + 4 * np + 4 * r * dr;         // EV, EVnorm, EVid, centroids
    if (s.pivot_dtype == PA_FP8E4M3) b += np * dr + 4 * np;  // e4m3 codes, row scales
    if (s.queries > 0) {
        const int64_t m = s.queries;
        const int64_t E = s.E > 0 ? s.E : std::min<int64_t>(s.ef_gpu, np / r);
        const int64_t B = std::min<int64_t>(m, s.batch > 0 ? s.batch : 16384);
        if (!s.q_on_device) b += 4 * m * D;                  // queries
        b += 4 * m * dr + 4 * m;                             // reduced queries, buckets
        b += 8 * m * E + 8 * m * s.ef_gpu + 16 * m;          // entries, stage-1 lists, counters
        b += 4 * static_cast<int64_t>(select_entries_scratch_ints(B, s.r));
    }
    return b;
}

namespace {

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    PA_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
}

void search(pa_index* idx, const float* Q, int64_t m, int k, const pa_search_opts* o_in, int64_t* out_ids,
            float* out_d, int32_t* counters, pa_search_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    require(idx->has_data && idx->has_proj && idx->has_sub && idx->has_entries,
            "search needs set_data, a projection, build_subgraph and build_entries first", PA_ESTATE);
    pa_search_opts o{};
    if (o_in) o = *o_in;
    if (o.ef_gpu <= 0) o.ef_gpu = 64;
    if (o.ef_cpu <= 0) o.ef_cpu = o.ef_gpu;
    require(o.ef_gpu >= 1 && o.ef_gpu <= PA_MAX_EF, "ef_gpu must be in [1, 512]");
    require(k >= 1 && m >= 0, "need k >= 1 and m >= 0");
    const int E = o.E > 0 ? o.E : std::min(o.ef_gpu, idx->n_b);
    require(E >= 1 && E <= PA_MAX_EF, "E must be in [1, 512]");
    require(o.entries == PA_ENTRIES_FES || o.entries == PA_ENTRIES_FIXED, "entries must be FES (0) or fixed (1)");
    const bool fixed_entries = o.entries == PA_ENTRIES_FIXED;
    require(!fixed_entries || E <= idx->n_b * idx->p.r, "fixed entries: E must not exceed the pivot count");
    require(o.serial == 0 || o.serial == 1, "serial must be 0 or 1");
    require(o.visited == PA_VISITED_EXACT || o.visited == PA_VISITED_BLOOM, "visited must be exact (0) or bloom (1)");
    const int width = o.width <= 1 ? 1 : o.width;
    require(width == 1 || (width == 2 && idx->R_sub <= 32), "width must be 0, 1, or 2 with a subgraph degree <= 32");
    const int mask = o.stage_mask == 0 ? 3 : o.stage_mask;
    require(mask >= 1 && mask <= 7, "stage_mask must be in [0, 7]");
    const bool gpu_stage = (mask & 1) != 0;
    const int refine_steps = (mask & 2) ? idx->p.refine_steps : -1;
    const bool final_stage = (mask & 4) == 0;
    require(gpu_stage || final_stage, "without the GPU stage the final traversal must run");
    if (stats) *stats = pa_search_stats{};
    if (m == 0) return;
    require(Q && out_ids && out_d, "null pointer");
    for (int64_t i = 0; i < m * idx->p.dim; ++i)
        if (!std::isfinite(Q[i])) fail(PA_ENONFINITE, "queries hold a non-finite value");
    use_device(idx);
    ensure_pool(idx, o.threads);
    const int D = idx->p.dim, d_r = idx->p.d_r, r = idx->p.r, ef = o.ef_gpu;
    // Sub-batches; automatic: up to 16,384 queries per launch.  The traversal kernel runs
    // one wavefront per query and hides latency with many resident wavefronts: one launch
    // of 10,000 queries takes about the time of two launches of 4,096, while the host
    // stages, which start after the first sub-batch, take some 50 times longer.
    std::vector<int64_t> starts{0};
    const int64_t step = o.batch > 0 ? o.batch : 16384;
    for (int64_t b0 = step; b0 < m; b0 += step) starts.push_back(b0);
    starts.push_back(m);
    const int64_t nbatch = static_cast<int64_t>(starts.size()) - 1;
    int64_t B = 0;
    for (int64_t b = 0; b < nbatch; ++b) B = std::max(B, starts[b + 1] - starts[b]);

    int64_t& hb = idx->hbm_used;
    const int64_t bud = idx->p.hbm_budget;
    if (o.q_dev) {
        hipPointerAttribute_t pa{};
        const bool ok = hipPointerGetAttributes(&pa, o.q_dev) == hipSuccess && pa.type == hipMemoryTypeDevice &&
                        pa.device == idx->p.device;
        (void)hipGetLastError();  // a failed query leaves no error behind
        require(ok, "q_dev must be device memory on the index's device");
    }
    float* q_dev = o.q_dev ? nullptr : static_cast<float*>(idx->w_q.ensure(sizeof(float) * m * D, hb, bud));
    const float* q_src = o.q_dev ? o.q_dev : q_dev;
    auto* qr_dev = static_cast<float*>(idx->w_qr.ensure(sizeof(float) * m * d_r, hb, bud));
    auto* cl_dev = static_cast<int32_t*>(idx->w_cl.ensure(sizeof(int32_t) * m, hb, bud));
    auto* eid_dev = static_cast<int32_t*>(idx->w_eid.ensure(sizeof(int32_t) * m * E, hb, bud));
    auto* ed_dev = static_cast<float*>(idx->w_ed.ensure(sizeof(float) * m * E, hb, bud));
    auto* bid_dev = static_cast<int32_t*>(idx->w_bid.ensure(sizeof(int32_t) * m * ef, hb, bud));
    auto* bd_dev = static_cast<float*>(idx->w_bd.ensure(sizeof(float) * m * ef, hb, bud));
    auto* cnt_dev = static_cast<int32_t*>(idx->w_cnt.ensure(sizeof(int32_t) * m * 4, hb, bud));
    auto* scr_dev = static_cast<int32_t*>(idx->w_scr.ensure(sizeof(int32_t) * select_entries_scratch_ints(B, r), hb, bud));
    auto* q_pin = o.q_dev ? nullptr : static_cast<float*>(idx->p_q.ensure(sizeof(float) * m * D));
    auto* beam_pin = static_cast<int32_t*>(idx->p_beam.ensure(sizeof(int32_t) * m * ef));
    auto* cnt_pin = static_cast<int32_t*>(idx->p_cnt.ensure(sizeof(int32_t) * m * 4));
    auto* ent_pin = static_cast<int32_t*>(idx->p_ent.ensure(sizeof(int32_t) * m * E));
    ensure_events(idx, static_cast<size_t>(4 * nbatch));
    hipStream_t s = idx->stream;
    if (fixed_entries) {  // the same predefined pivots for every query, one per bucket in turn (device ids)
        const int r_ = idx->p.r, n_b = idx->n_b;
        std::vector<int32_t> fixed(static_cast<size_t>(E));
        for (int e = 0; e < E; ++e)
            fixed[e] = index_device_id(idx, idx->bucket_ids[static_cast<size_t>(e % r_) * n_b + e / r_]);
        for (int64_t i = 0; i < m; ++i) std::memcpy(ent_pin + i * E, fixed.data(), sizeof(int32_t) * E);
    }

    // enqueue every batch's GPU work; the host consumes them in order below
    for (int64_t b = 0; b < nbatch; ++b) {
        const int64_t b0 = starts[b], nb = starts[b + 1] - starts[b];
        hipEvent_t* ev = &idx->events[static_cast<size_t>(4 * b)];
        if (o.q_dev == nullptr) {
            std::memcpy(q_pin + b0 * D, Q + b0 * D, sizeof(float) * nb * D);
            PA_HIP(hipMemcpyAsync(q_dev + b0 * D, q_pin + b0 * D, sizeof(float) * nb * D, hipMemcpyHostToDevice, s));
        }
        PA_HIP(hipEventRecord(ev[0], s));
        launch_project(q_src + b0 * D, nb, D, static_cast<const float*>(idx->V_dev.p), d_r, qr_dev + b0 * d_r, PA_F32,
                       static_cast<const float*>(idx->cent_dev.p), r, cl_dev + b0, s);
        if (fixed_entries) {
            if (gpu_stage)
                PA_HIP(hipMemcpyAsync(eid_dev + b0 * E, ent_pin + b0 * E, sizeof(int32_t) * nb * E,
                                      hipMemcpyHostToDevice, s));
        } else {
            index_select_entries(idx, qr_dev + b0 * d_r, cl_dev + b0, nb, E, eid_dev + b0 * E, ed_dev + b0 * E, scr_dev,
                                 s);
        }
        PA_HIP(hipEventRecord(ev[1], s));
        if (gpu_stage) {
            launch_beam(qr_dev + b0 * d_r, nb, d_r, idx->Xr_dev.p, idx->p.xr_dtype, idx->xr_rows,
                        static_cast<const int32_t*>(idx->adj_dev.p), idx->R_sub, eid_dev + b0 * E, E, ef,
                        idx->p.metric, o.cache_log2, bid_dev + b0 * ef, bd_dev + b0 * ef, cnt_dev + b0 * 4, s,
                        nullptr, o.visited, index_out_map(idx), false, width);  // stage 2 reads only the ids
            PA_HIP(hipEventRecord(ev[2], s));
            PA_HIP(hipMemcpyAsync(beam_pin + b0 * ef, bid_dev + b0 * ef, sizeof(int32_t) * nb * ef,
                                  hipMemcpyDeviceToHost, s));
            PA_HIP(hipMemcpyAsync(cnt_pin + b0 * 4, cnt_dev + b0 * 4, sizeof(int32_t) * nb * 4, hipMemcpyDeviceToHost,
                                  s));
        } else {
            PA_HIP(hipEventRecord(ev[2], s));
            if (!fixed_entries)  // fixed entries are in ent_pin already
                PA_HIP(hipMemcpyAsync(ent_pin + b0 * E, eid_dev + b0 * E, sizeof(int32_t) * nb * E,
                                      hipMemcpyDeviceToHost, s));
        }
        PA_HIP(hipEventRecord(ev[3], s));
    }

    StageContext ctx{idx->X, idx->N, D, pick_distance(idx->p.metric), HostGraph{idx->sub_adj.data(), idx->R_sub},
                     HostGraph{idx->full_adj.data(), idx->R_full}};
    std::vector<StageCounters> sc(static_cast<size_t>(m));
    double wait_ms = 0.0;
    const int ef_cpu = o.ef_cpu;
    const int handoff = (o.handoff > 0 && o.handoff < ef) ? o.handoff : ef;
    for (int64_t b = 0; b < nbatch; ++b) {
        const int64_t b0 = starts[b], nb = starts[b + 1] - starts[b];
        const auto w0 = std::chrono::steady_clock::now();
        // pipelined: sub-batch b as soon as its GPU stage is done; serial: after the last one
        const int64_t wait_for = o.serial ? nbatch - 1 : b;
        PA_HIP(hipEventSynchronize(idx->events[static_cast<size_t>(4 * wait_for + 3)]));
        wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
        idx->pool->parallel_for(nb, [&](int64_t j, int w) {
            const int64_t i = b0 + j;
            if (gpu_stage) {
                host_stages_one(ctx, Q + i * D, beam_pin + i * ef, handoff, ef_cpu, k, refine_steps, idx->vis[w],
                                idx->lists[w], out_ids + i * k, out_d + i * k, sc[i], final_stage);
            } else {
                int32_t* ent = ent_pin + i * E;
                if (index_compact(idx))  // FES lists device ids
                    for (int e = 0; e < E; ++e) ent[e] = ent[e] >= 0 ? idx->cid[ent[e]] : -1;
                host_search_one(ctx, Q + i * D, ent, E, ef_cpu, k, idx->vis[w], idx->lists[w],
                                out_ids + i * k, out_d + i * k, sc[i]);
            }
        });
    }
    if (counters) {
        for (int64_t i = 0; i < m; ++i) {
            int32_t* c = counters + i * 8;
            c[0] = gpu_stage ? cnt_pin[i * 4 + 0] : 0;
            c[1] = gpu_stage ? cnt_pin[i * 4 + 1] : 0;
            c[2] = gpu_stage ? cnt_pin[i * 4 + 2] : 0;
            c[3] = sc[i].dist2;
            c[4] = sc[i].dist3;
            c[5] = sc[i].exp3;
            c[6] = 0;
            c[7] = 0;
        }
    }
    if (stats) {
        stats->host_wait_ms = wait_ms;
        for (int64_t b = 0; b < nbatch; ++b) {
            hipEvent_t* ev = &idx->events[static_cast<size_t>(4 * b)];
            stats->fes_ms += elapsed_ms(ev[0], ev[1]);
            if (gpu_stage) {
                stats->beam_ms += elapsed_ms(ev[1], ev[2]);
                stats->beam_launches += 1;
            }
        }
        for (int64_t i = 0; i < m; ++i) {
            if (gpu_stage) {
                stats->n_exp1 += cnt_pin[i * 4 + 0];
                stats->n_dist1 += cnt_pin[i * 4 + 1];
                stats->n_reset1 += cnt_pin[i * 4 + 2];
            }
            stats->n_dist2 += sc[i].dist2;
            stats->n_dist3 += sc[i].dist3;
            stats->n_exp3 += sc[i].exp3;
        }
        stats->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" {

pa_status pa_index_create(const pa_params* params, pa_index** out) {
    return guarded([&] {
        require(params && out, "null pointer");
        const pa_params& p = *params;
        require(p.dim > 0 && p.dim <= 4096, "dim must be in [1, 4096]");
        require(p.d_r > 0 && p.d_r % 16 == 0 && p.d_r <= PA_MAX_DR && p.d_r <= p.dim,
                "d_r must be a multiple of 16 in [16, min(256, dim)]");
        require(p.metric == PA_METRIC_L2 || p.metric == PA_METRIC_IP, "unknown metric");
        require((static_cast<size_t>(p.d_r) * dtype_size(p.xr_dtype)) % 16 == 0, "reduced rows must be 16-byte multiples");
        require(p.r >= 1 && p.r <= 64, "r must be in [1, 64]");
        require(p.refine_steps >= 0, "refine_steps must be >= 0");
        require(p.pivot_dtype == PA_F32 || p.pivot_dtype == PA_FP8E4M3, "pivot_dtype must be PA_F32 or PA_FP8E4M3");
        require(p.pivot_dtype != PA_FP8E4M3 || p.d_r % 32 == 0, "FP8 pivots need d_r % 32 == 0");
        require(p.preselect >= 0 && p.preselect <= 64, "preselect must be in [0, 64]");
        require(p.compact == 0 || p.compact == 1, "compact must be 0 or 1");
        auto idx = std::make_unique<pa_index>();
        idx->p = p;
        PA_HIP(hipSetDevice(p.device));
        PA_HIP(hipStreamCreateWithFlags(&idx->stream, hipStreamNonBlocking));
        *out = idx.release();
    });
}

pa_status pa_index_destroy(pa_index* idx) {
    return guarded([&] {
        if (!idx) return;
        (void)hipSetDevice(idx->p.device);
        delete idx;
    });
}

pa_status pa_index_set_data(pa_index* idx, const float* X_host, int64_t N, const int64_t* rowptr_host,
                            const int32_t* nbrs_host) {
    return guarded([&] {
        require(idx && X_host && rowptr_host && nbrs_host, "null pointer");
        require(N > 0 && N < (int64_t{1} << 31), "N must be in [1, 2^31)");
        int R = 1;
        for (int64_t u = 0; u < N; ++u) {
            const int64_t d = rowptr_host[u + 1] - rowptr_host[u];
            require(d >= 0, "rowptr must be non-decreasing");
            R = static_cast<int>(std::max<int64_t>(R, d));
        }
        require(R <= 1024, "full-graph degree above 1024");
        idx->full_adj = pad_rows(N, rowptr_host, nbrs_host, R);
        idx->full_rowptr.assign(rowptr_host, rowptr_host + N + 1);
        idx->full_nbrs.assign(nbrs_host, nbrs_host + rowptr_host[N]);
        idx->R_full = R;
        idx->X = X_host;
        idx->N = N;
        idx->has_data = true;
        idx->has_proj = idx->has_sub = idx->has_entries = false;
        idx->cid.clear();
        idx->xr_rows = 0;
        idx->pool.reset();
    });
}

pa_status pa_index_fit_projection(pa_index* idx, int32_t center) {
    return guarded([&] {
        require(idx, "null pointer");
        require(idx->has_data, "set_data first", PA_ESTATE);
        use_device(idx);
        const int c = center < 0 ? (idx->p.metric == PA_METRIC_L2 ? 1 : 0) : (center != 0);
        idx->V.assign(static_cast<size_t>(idx->p.dim) * idx->p.d_r, 0.0f);
        std::vector<double> ev(static_cast<size_t>(idx->p.dim)), mean(static_cast<size_t>(idx->p.dim));
        fit_projection_host(idx->X, idx->N, idx->p.dim, idx->p.d_r, c, idx->V.data(), ev.data(), mean.data());
        project_all(idx);
    });
}

pa_status pa_index_set_projection(pa_index* idx, const float* V_host) {
    return guarded([&] {
        require(idx && V_host, "null pointer");
        require(idx->has_data, "set_data first", PA_ESTATE);
        use_device(idx);
        idx->V.assign(V_host, V_host + static_cast<size_t>(idx->p.dim) * idx->p.d_r);
        for (float v : idx->V)
            if (!std::isfinite(v)) fail(PA_ENONFINITE, "V holds a non-finite value");
        project_all(idx);
    });
}

pa_status pa_index_sample_nodes(pa_index* idx, const int64_t* order_host, int64_t n_target, int32_t mode,
                                uint8_t* mask_host) {
    return guarded([&] {
        require(idx && order_host && mask_host, "null pointer");
        require(idx->has_data, "set_data first", PA_ESTATE);
        sample_nodes(idx->N, idx->full_rowptr.data(), idx->full_nbrs.data(), order_host, n_target, mode, mask_host);
    });
}

pa_status pa_index_build_subgraph(pa_index* idx, const uint8_t* mask_host, const int64_t* rowptr_host,
                                  const int32_t* nbrs_host) {
    return guarded([&] {
        require(idx && mask_host && rowptr_host, "null pointer");
        require(idx->has_data, "set_data first", PA_ESTATE);
        use_device(idx);
        int R = 1;
        for (int64_t u = 0; u < idx->N; ++u)
            R = static_cast<int>(std::max<int64_t>(R, rowptr_host[u + 1] - rowptr_host[u]));
        require(R <= PA_MAX_DEGREE, "subgraph degree above 64");
        check_subgraph(idx->N, rowptr_host, nbrs_host, mask_host, R);
        idx->sub_adj = pad_rows(idx->N, rowptr_host, nbrs_host, R);
        idx->R_sub = R;
        idx->cid.clear();
        if (index_compact(idx))
            for (int64_t u = 0; u < idx->N; ++u)
                if (mask_host[u]) idx->cid.push_back(static_cast<int32_t>(u));
        index_upload_subgraph(idx);
        idx->has_sub = true;
        idx->has_entries = false;
        if (index_compact(idx)) index_write_rows(idx);  // the sampled rows of X_r
    });
}

pa_status pa_index_build_entries(pa_index* idx, const int32_t* pivot_ids_host, int32_t n_p, const int32_t* init_host,
                                 int32_t iters) {
    return guarded([&] {
        require(idx && pivot_ids_host && init_host, "null pointer");
        require(idx->has_proj && idx->has_sub, "projection and subgraph first", PA_ESTATE);
        const int r = idx->p.r, D = idx->p.dim, d_r = idx->p.d_r;
        require(n_p >= r && n_p % r == 0, "n_p must be a positive multiple of r");
        use_device(idx);
        std::vector<char> seen(static_cast<size_t>(idx->N), 0);
        std::vector<float> xp(static_cast<size_t>(n_p) * D);
        for (int i = 0; i < n_p; ++i) {
            const int32_t v = pivot_ids_host[i];
            require(v >= 0 && v < idx->N, "pivot id out of range");
            require(!seen[v], "pivot ids must be distinct");
            seen[v] = 1;
            require(idx->sub_adj[static_cast<size_t>(v) * idx->R_sub] >= 0,
                    "pivot " + std::to_string(v) + " has no out-edge in the subgraph");
            std::memcpy(&xp[static_cast<size_t>(i) * D], idx->X + static_cast<int64_t>(v) * D, sizeof(float) * D);
        }
        // fp32 reduced vectors of the pivots, from the same projection kernel
        DevBuf xin, xout;
        int64_t dummy = 0;
        xin.ensure(sizeof(float) * xp.size(), dummy, 0);
        xout.ensure(sizeof(float) * static_cast<size_t>(n_p) * d_r, dummy, 0);
        PA_HIP(hipMemcpy(xin.p, xp.data(), sizeof(float) * xp.size(), hipMemcpyHostToDevice));
        launch_project(static_cast<const float*>(xin.p), n_p, D, static_cast<const float*>(idx->V_dev.p), d_r, xout.p,
                       PA_F32, nullptr, 0, nullptr, idx->stream);
        PA_HIP(hipStreamSynchronize(idx->stream));
        std::vector<float> P(static_cast<size_t>(n_p) * d_r);
        PA_HIP(hipMemcpy(P.data(), xout.p, sizeof(float) * P.size(), hipMemcpyDeviceToHost));
        const int n_b = n_p / r;
        std::vector<int32_t> buckets(static_cast<size_t>(n_p));
        idx->centroids.assign(static_cast<size_t>(r) * d_r, 0.0f);
        build_entries(P.data(), n_p, d_r, r, init_host, iters, buckets.data(), idx->centroids.data());
        std::vector<float> EV(static_cast<size_t>(n_p) * d_r), EVn(static_cast<size_t>(n_p));
        idx->bucket_ids.assign(static_cast<size_t>(n_p), -1);
        for (int i = 0; i < n_p; ++i) {
            const int pos = buckets[i];
            idx->bucket_ids[i] = pivot_ids_host[pos];
            double s = 0.0;
            for (int j = 0; j < d_r; ++j) {
                const float x = P[static_cast<size_t>(pos) * d_r + j];
                EV[static_cast<size_t>(i) * d_r + j] = x;
                s += static_cast<double>(x) * x;
            }
            EVn[i] = static_cast<float>(s);
        }
        idx->EV_dev.ensure(sizeof(float) * EV.size(), idx->hbm_used, idx->p.hbm_budget);
        idx->EVn_dev.ensure(sizeof(float) * EVn.size(), idx->hbm_used, idx->p.hbm_budget);
        idx->EVid_dev.ensure(sizeof(int32_t) * n_p, idx->hbm_used, idx->p.hbm_budget);
        idx->cent_dev.ensure(sizeof(float) * idx->centroids.size(), idx->hbm_used, idx->p.hbm_budget);
        PA_HIP(hipMemcpy(idx->EV_dev.p, EV.data(), sizeof(float) * EV.size(), hipMemcpyHostToDevice));
        PA_HIP(hipMemcpy(idx->EVn_dev.p, EVn.data(), sizeof(float) * EVn.size(), hipMemcpyHostToDevice));
        std::vector<int32_t> dev_ids(idx->bucket_ids);
        for (auto& v : dev_ids) v = index_device_id(idx, v);  // pivots are sampled nodes
        PA_HIP(hipMemcpy(idx->EVid_dev.p, dev_ids.data(), sizeof(int32_t) * n_p, hipMemcpyHostToDevice));
        PA_HIP(hipMemcpy(idx->cent_dev.p, idx->centroids.data(), sizeof(float) * idx->centroids.size(),
                         hipMemcpyHostToDevice));
        if (idx->p.pivot_dtype == PA_FP8E4M3) {
            std::vector<uint8_t> codes(EV.size());
            std::vector<float> scales(static_cast<size_t>(n_p));
            quantize_rows_e4m3(EV.data(), n_p, d_r, codes.data(), scales.data());
            idx->EV8_dev.ensure(codes.size(), idx->hbm_used, idx->p.hbm_budget);
            idx->EVs_dev.ensure(sizeof(float) * scales.size(), idx->hbm_used, idx->p.hbm_budget);
            PA_HIP(hipMemcpy(idx->EV8_dev.p, codes.data(), codes.size(), hipMemcpyHostToDevice));
            PA_HIP(hipMemcpy(idx->EVs_dev.p, scales.data(), sizeof(float) * scales.size(), hipMemcpyHostToDevice));
        }
        idx->n_b = n_b;
        idx->has_entries = true;
    });
}

pa_status pa_index_get_state(const pa_index* idx, float* V_host, int32_t* buckets_host, float* centroids_host) {
    return guarded([&] {
        require(idx, "null pointer");
        if (V_host) {
            require(idx->has_proj, "no projection yet", PA_ESTATE);
            std::copy(idx->V.begin(), idx->V.end(), V_host);
        }
        if (buckets_host || centroids_host) require(idx->has_entries, "no entries yet", PA_ESTATE);
        if (buckets_host) std::copy(idx->bucket_ids.begin(), idx->bucket_ids.end(), buckets_host);
        if (centroids_host) std::copy(idx->centroids.begin(), idx->centroids.end(), centroids_host);
    });
}

pa_status pa_index_device_tables(const pa_index* idx, const void** Xr_dev, const int32_t** adj_dev, const float** V_dev,
                                 const float** centroids_dev, const float** EV_dev, const float** EVnorm_dev,
                                 const int32_t** EVid_dev) {
    return guarded([&] {
        require(idx, "null pointer");
        if (Xr_dev) *Xr_dev = idx->Xr_dev.p;
        if (adj_dev) *adj_dev = static_cast<const int32_t*>(idx->adj_dev.p);
        if (V_dev) *V_dev = static_cast<const float*>(idx->V_dev.p);
        if (centroids_dev) *centroids_dev = static_cast<const float*>(idx->cent_dev.p);
        if (EV_dev) *EV_dev = static_cast<const float*>(idx->EV_dev.p);
        if (EVnorm_dev) *EVnorm_dev = static_cast<const float*>(idx->EVn_dev.p);
        if (EVid_dev) *EVid_dev = static_cast<const int32_t*>(idx->EVid_dev.p);
    });
}

int64_t pa_hbm_bytes(const pa_memory_shape* shape, double rho, int32_t d_r) {
    if (shape == nullptr) return -1;
    return index_hbm_model(*shape, rho, d_r);
}

pa_status pa_plan_memory(const pa_memory_shape* shape, int64_t hbm_budget, const double* rhos, int32_t n_rho,
                         const int32_t* d_rs, int32_t n_dr, double* rho_out, int32_t* d_r_out, int64_t* bytes_out) {
    return guarded([&] {
        require(shape && rhos && d_rs, "null pointer");
        require(n_rho >= 1 && n_dr >= 1, "need at least one candidate ratio and width");
        require(hbm_budget > 0, "hbm_budget must be positive");
        double best_rho = -1.0;
        int best_dr = -1;
        int64_t best_bytes = -1;
        for (int i = 0; i < n_rho; ++i)
            for (int j = 0; j < n_dr; ++j) {
                const int64_t b = index_hbm_model(*shape, rhos[i], d_rs[j]);
                require(b >= 0, "invalid shape, ratio " + std::to_string(rhos[i]) + " or width " +
                                    std::to_string(d_rs[j]));
                if (b > hbm_budget) continue;
                if (rhos[i] > best_rho || (rhos[i] == best_rho && d_rs[j] > best_dr)) {
                    best_rho = rhos[i];
                    best_dr = d_rs[j];
                    best_bytes = b;
                }
            }
        require(best_dr > 0, "no candidate fits " + std::to_string(hbm_budget) + " bytes of HBM", PA_EHBM);
        if (rho_out) *rho_out = best_rho;
        if (d_r_out) *d_r_out = best_dr;
        if (bytes_out) *bytes_out = best_bytes;
    });
}

pa_status pa_search(pa_index* idx, const float* Q_host, int64_t m, int32_t k, const pa_search_opts* opts,
                    int64_t* out_ids_host, float* out_d_host, int32_t* counters_host, pa_search_stats* stats) {
    return guarded([&] {
        require(idx, "null pointer");
        search(idx, Q_host, m, k, opts, out_ids_host, out_d_host, counters_host, stats);
    });
}

}  // extern "C"
