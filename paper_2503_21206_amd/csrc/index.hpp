// The index object shared by the search pipeline and the serving loop.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "host.hpp"

namespace pa {

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void* ensure(size_t need, int64_t& total, int64_t budget) {
        if (need <= bytes) return p;
        const int64_t after = total - static_cast<int64_t>(bytes) + static_cast<int64_t>(need);
        if (budget > 0 && after > budget) fail(PA_EHBM, "HBM budget exceeded (" + std::to_string(after) + " bytes)");
        release();
        total = after - static_cast<int64_t>(need);
        if (hipMalloc(&p, need) != hipSuccess) {
            p = nullptr;
            fail(PA_EHBM, "hipMalloc of " + std::to_string(need) + " bytes failed");
        }
        bytes = need;
        total += static_cast<int64_t>(need);
        return p;
    }
};

// Grow-only pinned host buffer.
struct PinBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~PinBuf() {
        if (p) (void)hipHostFree(p);
    }
    void* ensure(size_t need) {
        if (need <= bytes) return p;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        PA_HIP(hipHostMalloc(&p, need, hipHostMallocDefault));
        bytes = need;
        return p;
    }
};

}  // namespace pa

struct pa_index {
    pa_params p{};
    const float* X = nullptr;
    int64_t N = 0;
    std::vector<int64_t> full_rowptr;
    std::vector<int32_t> full_nbrs;
    std::vector<int32_t> full_adj;
    int R_full = 0;
    std::vector<int32_t> sub_adj;
    int R_sub = 0;
    std::vector<int32_t> cid;  // compact layout: device id -> node id (increasing)
    int64_t xr_rows = 0;       // rows of X_r and of the device adjacency
    std::vector<float> V;
    std::vector<int32_t> bucket_ids;
    std::vector<float> centroids;
    int n_b = 0;
    bool has_data = false, has_proj = false, has_sub = false, has_entries = false;

    int64_t hbm_used = 0;
    pa::DevBuf V_dev, Xr_dev, adj_dev, cent_dev, EV_dev, EVn_dev, EVid_dev, EV8_dev, EVs_dev, cid_dev;
    pa::DevBuf w_q, w_qr, w_cl, w_eid, w_ed, w_bid, w_bd, w_cnt, w_scr;
    pa::PinBuf p_q, p_beam, p_cnt, p_ent;
    hipStream_t stream = nullptr;
    std::vector<hipEvent_t> events;

    std::unique_ptr<pa::ThreadPool> pool;
    std::vector<pa::Visited> vis;
    std::vector<std::vector<pa::Cand>> lists;

    ~pa_index() {
        for (auto e : events) (void)hipEventDestroy(e);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace pa {
// Compact layout: device ids are positions in idx->cid; these map between the id spaces.
inline bool index_compact(const pa_index* idx) { return idx->p.compact != 0; }
inline const int32_t* index_out_map(const pa_index* idx) {
    return index_compact(idx) ? static_cast<const int32_t*>(idx->cid_dev.p) : nullptr;
}
int32_t index_device_id(const pa_index* idx, int32_t node);  // -1 if not held on the device
// (Re)writes X_r (all rows, or the sampled rows of the compact layout) from X and V.
void index_write_rows(pa_index* idx);
// Device bytes an index of shape s holds (pa_hbm_bytes); -1 if the shape is invalid.
int64_t index_hbm_model(const pa_memory_shape& s, double rho, int d_r);
// Uploads the device adjacency (and the id map of the compact layout) from sub_adj.
void index_upload_subgraph(pa_index* idx);
// Entry selection for m reduced queries with the index's tables (fp32 or FP8 form).
void index_select_entries(const pa_index* idx, const float* Qr, const int32_t* cluster, int64_t m, int E,
                          int32_t* ids, float* dists, int32_t* scratch, hipStream_t s);
}  // namespace pa
