// Checkpoint of a built index: header + checksummed sections (pa_index_save / pa_index_load),
// and the index's sizes (pa_index_get_info).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "index.hpp"

namespace pa {
namespace {

constexpr char kMagic[8] = {'P', 'A', 'N', 'N', 'I', 'D', 'X', '\0'};
constexpr uint32_t kFormat = 2;

enum Tag : uint32_t { kV = 1, kXr = 2, kSub = 3, kCent = 4, kBucketIds = 5, kEV = 6, kEVn = 7, kCid = 8 };

struct Header {
    char magic[8];
    uint32_t format;
    int32_t dim, d_r, metric, xr_dtype, r, pivot_dtype;
    int32_t R_sub, n_b;
    int64_t N;
    int64_t n_sections;
    int32_t compact, pad;
    int64_t xr_rows;  // rows of X_r as stored (N, or the sampled nodes when compact)
};

struct SectionHead {
    uint32_t tag;
    uint32_t pad;
    uint64_t bytes;
    uint64_t fnv;
};

// FNV-1a, 64 bit, continued from h.
uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
    const auto* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct File {
    std::FILE* f = nullptr;
    std::string path;
    File(const char* p, const char* mode) : path(p) {
        f = std::fopen(p, mode);
        if (!f) fail(PA_EIO, "cannot open " + path);
    }
    ~File() {
        if (f) std::fclose(f);
    }
    void write(const void* d, size_t n) {
        if (n && std::fwrite(d, 1, n, f) != n) fail(PA_EIO, "write to " + path + " failed");
    }
    void read(void* d, size_t n) {
        if (n && std::fread(d, 1, n, f) != n) fail(PA_EIO, path + " is truncated");
    }
    void close() {
        if (f && std::fclose(f) != 0) {
            f = nullptr;
            fail(PA_EIO, "closing " + path + " failed");
        }
        f = nullptr;
    }
};

void write_section(File& out, uint32_t tag, const void* data, size_t bytes) {
    SectionHead h{tag, 0, bytes, fnv1a(data, bytes)};
    out.write(&h, sizeof h);
    out.write(data, bytes);
}

// A device buffer written in 256 MB pieces through a host staging buffer.
void write_device_section(File& out, uint32_t tag, const void* dev, size_t bytes) {
    const long at = std::ftell(out.f);
    SectionHead h{tag, 0, bytes, 0};
    out.write(&h, sizeof h);
    const size_t piece = size_t{256} << 20;
    std::vector<unsigned char> buf(std::min(piece, bytes));
    uint64_t fnv = 1469598103934665603ull;
    for (size_t off = 0; off < bytes; off += piece) {
        const size_t n = std::min(piece, bytes - off);
        PA_HIP(hipMemcpy(buf.data(), static_cast<const unsigned char*>(dev) + off, n, hipMemcpyDeviceToHost));
        fnv = fnv1a(buf.data(), n, fnv);
        out.write(buf.data(), n);
    }
    const long end = std::ftell(out.f);
    h.fnv = fnv;
    if (std::fseek(out.f, at, SEEK_SET) != 0) fail(PA_EIO, "seek in " + out.path + " failed");
    out.write(&h, sizeof h);
    if (std::fseek(out.f, end, SEEK_SET) != 0) fail(PA_EIO, "seek in " + out.path + " failed");
}

std::vector<unsigned char> read_section(File& in, uint32_t tag, size_t expect) {
    SectionHead h{};
    in.read(&h, sizeof h);
    if (h.tag != tag) fail(PA_EIO, in.path + ": unexpected section " + std::to_string(h.tag));
    if (h.bytes != expect)
        fail(PA_EIO, in.path + ": section " + std::to_string(tag) + " holds " + std::to_string(h.bytes) +
                         " bytes, expected " + std::to_string(expect));
    std::vector<unsigned char> buf(expect);
    in.read(buf.data(), expect);
    if (fnv1a(buf.data(), expect) != h.fnv) fail(PA_EIO, in.path + ": checksum of section " + std::to_string(tag));
    return buf;
}

template <class T>
std::vector<T> as(const std::vector<unsigned char>& b) {
    std::vector<T> v(b.size() / sizeof(T));
    std::memcpy(v.data(), b.data(), v.size() * sizeof(T));
    return v;
}

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" {

pa_status pa_index_get_info(const pa_index* idx, pa_index_info* out) {
    return guarded([&] {
        require(idx && out, "null pointer");
        out->N = idx->N;
        out->R_full = idx->R_full;
        out->R_sub = idx->has_sub ? idx->R_sub : 0;
        out->n_pivots = idx->has_entries ? static_cast<int32_t>(idx->bucket_ids.size()) : 0;
        out->built = (idx->has_data ? 1 : 0) | (idx->has_proj ? 2 : 0) | (idx->has_sub ? 4 : 0) |
                     (idx->has_entries ? 8 : 0);
        out->hbm_bytes = idx->hbm_used;
        out->xr_rows = idx->xr_rows;
    });
}

pa_status pa_index_save(const pa_index* idx, const char* path) {
    return guarded([&] {
        require(idx && path, "null pointer");
        require(idx->has_proj && idx->has_sub && idx->has_entries, "save needs projection, subgraph and entries",
                PA_ESTATE);
        PA_HIP(hipSetDevice(idx->p.device));
        const int n_p = static_cast<int>(idx->bucket_ids.size());
        const size_t es = dtype_size(idx->p.xr_dtype);
        Header h{};
        std::memcpy(h.magic, kMagic, sizeof kMagic);
        h.format = kFormat;
        h.dim = idx->p.dim;
        h.d_r = idx->p.d_r;
        h.metric = idx->p.metric;
        h.xr_dtype = idx->p.xr_dtype;
        h.r = idx->p.r;
        h.pivot_dtype = idx->p.pivot_dtype;
        h.R_sub = idx->R_sub;
        h.n_b = idx->n_b;
        h.N = idx->N;
        h.compact = idx->p.compact;
        h.xr_rows = idx->xr_rows;
        h.n_sections = idx->p.compact ? 8 : 7;
        std::vector<float> EV(static_cast<size_t>(n_p) * idx->p.d_r), EVn(static_cast<size_t>(n_p));
        PA_HIP(hipMemcpy(EV.data(), idx->EV_dev.p, sizeof(float) * EV.size(), hipMemcpyDeviceToHost));
        PA_HIP(hipMemcpy(EVn.data(), idx->EVn_dev.p, sizeof(float) * EVn.size(), hipMemcpyDeviceToHost));
        File out(path, "wb");
        out.write(&h, sizeof h);
        const uint64_t hf = fnv1a(&h, sizeof h);
        out.write(&hf, sizeof hf);
        write_section(out, kV, idx->V.data(), sizeof(float) * idx->V.size());
        write_device_section(out, kXr, idx->Xr_dev.p, static_cast<size_t>(idx->xr_rows) * idx->p.d_r * es);
        write_section(out, kSub, idx->sub_adj.data(), sizeof(int32_t) * idx->sub_adj.size());
        write_section(out, kCent, idx->centroids.data(), sizeof(float) * idx->centroids.size());
        write_section(out, kBucketIds, idx->bucket_ids.data(), sizeof(int32_t) * idx->bucket_ids.size());
        write_section(out, kEV, EV.data(), sizeof(float) * EV.size());
        write_section(out, kEVn, EVn.data(), sizeof(float) * EVn.size());
        if (idx->p.compact) write_section(out, kCid, idx->cid.data(), sizeof(int32_t) * idx->cid.size());
        out.close();
    });
}

pa_status pa_index_load(pa_index* idx, const char* path) {
    return guarded([&] {
        require(idx && path, "null pointer");
        require(idx->has_data, "set_data first", PA_ESTATE);
        File in(path, "rb");
        Header h{};
        in.read(&h, sizeof h);
        if (std::memcmp(h.magic, kMagic, sizeof kMagic) != 0) fail(PA_EIO, in.path + " is not an index checkpoint");
        uint64_t hf = 0;
        in.read(&hf, sizeof hf);
        if (hf != fnv1a(&h, sizeof h)) fail(PA_EIO, in.path + ": header checksum");
        if (h.format != kFormat) fail(PA_EIO, in.path + ": unknown format " + std::to_string(h.format));
        const pa_params& p = idx->p;
        require(h.dim == p.dim && h.d_r == p.d_r && h.metric == p.metric && h.xr_dtype == p.xr_dtype && h.r == p.r &&
                    h.pivot_dtype == p.pivot_dtype && h.compact == p.compact,
                "checkpoint parameters differ from the index's (dim, d_r, metric, xr_dtype, r, pivot_dtype, compact)");
        require(h.N == idx->N, "checkpoint holds N=" + std::to_string(h.N) + ", the index's data has N=" +
                                   std::to_string(idx->N));
        if (h.R_sub < 1 || h.R_sub > PA_MAX_DEGREE || h.n_b < 1 || h.n_sections != (h.compact ? 8 : 7) ||
            h.xr_rows < 0 || h.xr_rows > h.N || (!h.compact && h.xr_rows != h.N))
            fail(PA_EIO, in.path + ": corrupt header");
        const size_t es = dtype_size(h.xr_dtype);
        const size_t n_p = static_cast<size_t>(h.r) * h.n_b;
        // read and verify everything before the index is touched
        auto V = as<float>(read_section(in, kV, sizeof(float) * p.dim * p.d_r));
        auto Xr = read_section(in, kXr, static_cast<size_t>(h.xr_rows) * p.d_r * es);
        auto sub = as<int32_t>(read_section(in, kSub, sizeof(int32_t) * static_cast<size_t>(h.N) * h.R_sub));
        auto cent = as<float>(read_section(in, kCent, sizeof(float) * p.r * p.d_r));
        auto bids = as<int32_t>(read_section(in, kBucketIds, sizeof(int32_t) * n_p));
        auto EV = as<float>(read_section(in, kEV, sizeof(float) * n_p * p.d_r));
        auto EVn = as<float>(read_section(in, kEVn, sizeof(float) * n_p));
        std::vector<int32_t> cid;
        if (h.compact) {
            cid = as<int32_t>(read_section(in, kCid, sizeof(int32_t) * static_cast<size_t>(h.xr_rows)));
            for (size_t i = 0; i < cid.size(); ++i)
                if (cid[i] < 0 || cid[i] >= h.N || (i > 0 && cid[i] <= cid[i - 1]))
                    fail(PA_EIO, in.path + ": the sampled-node list is not increasing within [0, N)");
        }
        for (int32_t v : sub)
            if (v < -1 || v >= h.N) fail(PA_EIO, in.path + ": subgraph id out of range");
        for (int32_t v : bids)
            if (v < 0 || v >= h.N) fail(PA_EIO, in.path + ": pivot id out of range");
        std::vector<int32_t> dev_ids(bids);  // the pivots' device ids
        if (h.compact)
            for (auto& v : dev_ids) {
                const auto it = std::lower_bound(cid.begin(), cid.end(), v);
                if (it == cid.end() || *it != v) fail(PA_EIO, in.path + ": a pivot is not a sampled node");
                v = static_cast<int32_t>(it - cid.begin());
            }

        PA_HIP(hipSetDevice(p.device));
        idx->has_proj = idx->has_sub = idx->has_entries = false;
        auto up = [&](DevBuf& b, const void* src, size_t bytes) {
            b.ensure(bytes, idx->hbm_used, p.hbm_budget);
            PA_HIP(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        };
        idx->cid = std::move(cid);
        idx->xr_rows = 0;
        idx->sub_adj = std::move(sub);
        idx->R_sub = h.R_sub;
        up(idx->V_dev, V.data(), sizeof(float) * V.size());
        if (!Xr.empty()) up(idx->Xr_dev, Xr.data(), Xr.size());
        index_upload_subgraph(idx);
        up(idx->cent_dev, cent.data(), sizeof(float) * cent.size());
        up(idx->EV_dev, EV.data(), sizeof(float) * EV.size());
        up(idx->EVn_dev, EVn.data(), sizeof(float) * EVn.size());
        up(idx->EVid_dev, dev_ids.data(), sizeof(int32_t) * dev_ids.size());
        if (p.pivot_dtype == PA_FP8E4M3) {
            std::vector<uint8_t> codes(EV.size());
            std::vector<float> scales(n_p);
            quantize_rows_e4m3(EV.data(), static_cast<int64_t>(n_p), p.d_r, codes.data(), scales.data());
            up(idx->EV8_dev, codes.data(), codes.size());
            up(idx->EVs_dev, scales.data(), sizeof(float) * scales.size());
        }
        idx->V = std::move(V);
        idx->xr_rows = h.xr_rows;
        idx->centroids = std::move(cent);
        idx->bucket_ids = std::move(bids);
        idx->n_b = h.n_b;
        idx->has_proj = idx->has_sub = idx->has_entries = true;
    });
}

}  // extern "C"
