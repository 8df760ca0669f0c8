// Stage 1 of PilotANN: batched greedy search (Algorithm 1) on the sampled subgraph with
// SVD-reduced vectors (section 4.1), one 64-lane wavefront per query.
//
// Per wavefront, in LDS:
//   keys[ef]   the candidate list C, sorted ascending by the 64-bit key
//              (orderable(distance) << 32) | (id << 1) | checked
//   stage      64-slot staging area for the current batch of neighbours
//   cache[H]   open-addressing visited cache of node ids (linear probing, LDS CAS)
//
// Exactness.  The paper keeps visited nodes in a lossy shared-memory Bloom filter
// (section 4.3) and lets the CPU stages repair its false positives.  This kernel instead
// reproduces Algorithm 1 with an exact visited set while holding only a bounded cache:
// the cache never reports an unvisited node as visited (it stores full ids), it may only
// forget nodes.  A forgotten node v that is met again is scored again; if v is still in
// C its key is bit-identical (fixed reduction order) and the duplicate is dropped during
// the merge, and if v had left C then C was full and its ef-th key has only decreased
// since, so v is rejected again.  Either way C evolves exactly as in Algorithm 1; only
// the count of distance evaluations can exceed |visited| (reported per query together
// with the number of cache resets).
//
// One loop step: find the first unchecked entry of C, mark it checked, fetch its
// adjacency row (one coalesced load of R ids), test-and-set the ids in the cache,
// gather the reduced vectors of the new ids (16 bytes per lane, GS lanes per vector,
// all loads in flight together), reduce distances across the GS lanes with a fixed
// butterfly, drop candidates not better than C[ef-1] or already in C, and merge the
// survivors into C by co-ranking (binary search of each survivor in C plus its rank among
// the survivors; existing entries shift by the number of survivors placed before them).
#include <hip/hip_runtime.h>

#include <climits>

#include "common.hpp"

namespace pa {
namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kRounds = 8;       // gather rounds kept in flight per batch
constexpr int kMaxChunks = PA_MAX_EF / 64;
constexpr int kProbes = 16;

__device__ __forceinline__ uint32_t ord_f32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u ^ 0x80000000u) : ~u);
}
__device__ __forceinline__ uint64_t make_key(float d, uint32_t id) {
    return (static_cast<uint64_t>(ord_f32(d)) << 32) | (static_cast<uint64_t>(id) << 1);
}
__device__ __forceinline__ int mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0));
}
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t hash_slot(uint32_t v, int hlog) {
    return (v * 0x9E3779B1u) >> (32 - hlog);
}

struct BeamArgs {
    const float* qr;
    int64_t m;
    int d_r;
    const unsigned char* xr;
    int64_t row_bytes;
    int64_t N;
    const int32_t* adj;
    int R;
    const int32_t* entries;
    int E;
    int ef;
    int ef_alloc;
    int hlog;
    int gs_log;  // log2 of lanes per gathered vector
    int cpr;     // 16-byte chunks per reduced row
    int wave_bytes;
    int32_t* out_ids;
    float* out_d;
    int32_t* counters;
};

template <int DT>
struct Chunk;
template <>
struct Chunk<PA_F32> {
    static constexpr int kElems = 4;
    __device__ static void widen(const uint4& raw, float* x) {
        x[0] = __uint_as_float(raw.x);
        x[1] = __uint_as_float(raw.y);
        x[2] = __uint_as_float(raw.z);
        x[3] = __uint_as_float(raw.w);
    }
};
template <>
struct Chunk<PA_F16> {
    static constexpr int kElems = 8;
    __device__ static void widen(const uint4& raw, float* x) {
        const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            _Float16 lo = __builtin_bit_cast(_Float16, static_cast<uint16_t>(w[i] & 0xFFFFu));
            _Float16 hi = __builtin_bit_cast(_Float16, static_cast<uint16_t>(w[i] >> 16));
            x[2 * i] = static_cast<float>(lo);
            x[2 * i + 1] = static_cast<float>(hi);
        }
    }
};
template <>
struct Chunk<PA_BF16> {
    static constexpr int kElems = 8;
    __device__ static void widen(const uint4& raw, float* x) {
        const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            x[2 * i] = __uint_as_float(w[i] << 16);
            x[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
        }
    }
};

template <int DT, int MET>
struct Wave {
    static constexpr int EPC = Chunk<DT>::kElems;

    const BeamArgs& a;
    int lane, sub, grp, gs, vpl, hmask;
    uint64_t* keys;
    uint64_t* st_key;
    uint32_t* st_id;
    int32_t* st_pos;
    uint32_t* cache;
    float qv[EPC];
    int size = 0;
    int n_dist = 0;
    int fill = 0;
    int forgot = 0;

    __device__ Wave(const BeamArgs& args, unsigned char* base, int64_t qi, int lane_)
        : a(args), lane(lane_) {
        gs = 1 << a.gs_log;
        vpl = 64 >> a.gs_log;
        sub = lane & (gs - 1);
        grp = lane >> a.gs_log;
        hmask = (1 << a.hlog) - 1;
        keys = reinterpret_cast<uint64_t*>(base);
        st_key = keys + a.ef_alloc;
        st_id = reinterpret_cast<uint32_t*>(st_key + 64);
        st_pos = reinterpret_cast<int32_t*>(st_id + 64);
        cache = reinterpret_cast<uint32_t*>(st_pos + 64);
        const float* q = a.qr + qi * a.d_r;
#pragma unroll
        for (int e = 0; e < EPC; ++e) qv[e] = (sub < a.cpr) ? q[sub * EPC + e] : 0.0f;
    }

    __device__ void clear_cache() {
        for (int i = lane; i <= hmask; i += 64) cache[i] = kEmpty;
        fill = 0;
        wave_sync();
    }

    // Test-and-set of v in the visited cache; true when v must be scored.
    __device__ bool test_and_set(int v, bool& stored) {
        stored = false;
        if (v < 0) return false;
        uint32_t h = hash_slot(static_cast<uint32_t>(v), a.hlog);
        for (int p = 0; p < kProbes; ++p) {
            uint32_t old = atomicCAS(&cache[h], kEmpty, static_cast<uint32_t>(v));
            if (old == kEmpty) {
                stored = true;
                return true;
            }
            if (old == static_cast<uint32_t>(v)) return false;
            h = (h + 1) & hmask;
        }
        return true;  // cache neighbourhood full: score it (never a false "visited")
    }

    // Re-populate the cache with the ids currently in C after a reset.
    __device__ void reseed_cache() {
        for (int t0 = 0; t0 < size; t0 += 64) {
            int t = t0 + lane;
            int v = (t < size) ? static_cast<int>(static_cast<uint32_t>(keys[t]) >> 1) : -1;
            bool stored;
            test_and_set(v, stored);
            fill += __popcll(__ballot(stored));
        }
        wave_sync();
    }

    __device__ float lane_partial(const uint4& raw) const {
        float x[EPC];
        Chunk<DT>::widen(raw, x);
        float s = 0.0f;
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
            if (MET == PA_METRIC_L2) {
                float d = qv[e] - x[e];
                s = __builtin_fmaf(d, d, s);
            } else {
                s = __builtin_fmaf(qv[e], x[e], s);
            }
        }
        return s;
    }

    // Offer one id per lane (-1 = none) to C.  Returns the smallest position at which an
    // entry was inserted (INT_MAX if none).
    __device__ int offer(int v) {
        bool stored;
        bool fresh = test_and_set(v, stored);
        fill += __popcll(__ballot(stored));
        forgot += __popcll(__ballot(fresh && !stored));  // scored but not remembered
        uint64_t newmask = __ballot(fresh);
        int n_new = __popcll(newmask);
        if (n_new == 0) return INT_MAX;
        if (fresh) st_id[mbcnt(newmask)] = static_cast<uint32_t>(v);
        wave_sync();
        n_dist += n_new;

        // gather and score, kRounds * vpl vectors per batch with all loads in flight
        for (int b0 = 0; b0 < n_new; b0 += kRounds * vpl) {
            uint4 raw[kRounds];
#pragma unroll
            for (int rr = 0; rr < kRounds; ++rr) {
                int c = b0 + rr * vpl + grp;
                raw[rr] = make_uint4(0, 0, 0, 0);
                if (c < n_new && sub < a.cpr) {
                    const uint32_t id = st_id[c];
                    const uint4* p = reinterpret_cast<const uint4*>(
                        a.xr + static_cast<int64_t>(id) * a.row_bytes + static_cast<int64_t>(sub) * 16);
                    raw[rr] = *p;
                }
            }
#pragma unroll
            for (int rr = 0; rr < kRounds; ++rr) {
                float s = (sub < a.cpr) ? lane_partial(raw[rr]) : 0.0f;
                for (int off = gs >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off);
                int c = b0 + rr * vpl + grp;
                if (sub == 0 && c < n_new) {
                    float d = (MET == PA_METRIC_L2) ? s : -s;
                    st_key[c] = make_key(d, st_id[c]);
                }
            }
        }
        wave_sync();

        // filter against the current ef-th key, de-duplicate against C, locate in C
        uint64_t key = (lane < n_new) ? st_key[lane] : ~0ull;
        bool cand = lane < n_new;
        if (size == a.ef) cand = cand && key < (keys[a.ef - 1] & ~1ull);
        int pos = 0;
        if (cand) {
            int lo = 0, hi = size;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if ((keys[mid] & ~1ull) < key) lo = mid + 1;
                else hi = mid;
            }
            pos = lo;
            if (pos < size && (keys[pos] & ~1ull) == key) cand = false;
        }
        uint64_t smask = __ballot(cand);
        int n_ins = __popcll(smask);
        if (n_ins == 0) return INT_MAX;
        wave_sync();
        if (cand) {
            int s = mbcnt(smask);
            st_key[s] = key;
            st_pos[s] = pos;
        }
        wave_sync();
        const bool mine = lane < n_ins;
        const uint64_t skey = mine ? st_key[lane] : ~0ull;
        const int spos = mine ? st_pos[lane] : INT_MAX;

        // rank among survivors and the shift of every existing entry at or after minpos
        int minpos = INT_MAX;
        for (int j = 0; j < n_ins; ++j) minpos = min(minpos, st_pos[j]);
        minpos = uniform(minpos);
        const int tail = size - minpos;
        const int nchunks = (tail + 63) >> 6;
        int rank = 0;
        int shift[kMaxChunks];
        int tpos[kMaxChunks];
#pragma unroll
        for (int c = 0; c < kMaxChunks; ++c) {
            shift[c] = 0;
            tpos[c] = minpos + c * 64 + lane;
        }
        for (int j = 0; j < n_ins; ++j) {
            const uint64_t kj = st_key[j];
            const int pj = st_pos[j];
            rank += (kj < skey) ? 1 : 0;
#pragma unroll
            for (int c = 0; c < kMaxChunks; ++c) shift[c] += (pj <= tpos[c]) ? 1 : 0;
        }
        uint64_t old[kMaxChunks];
#pragma unroll
        for (int c = 0; c < kMaxChunks; ++c) {
            old[c] = 0;
            if (c < nchunks && tpos[c] < size) old[c] = keys[tpos[c]];
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < kMaxChunks; ++c) {
            if (c < nchunks && tpos[c] < size) {
                int nt = tpos[c] + shift[c];
                if (nt < a.ef) keys[nt] = old[c];
            }
        }
        if (mine) {
            int fp = spos + rank;
            if (fp < a.ef) keys[fp] = skey;
        }
        wave_sync();
        size = min(size + n_ins, a.ef);
        return minpos;
    }
};

template <int DT, int MET>
__global__ __launch_bounds__(256) void beam_kernel(BeamArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int64_t qi = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wid;
    if (qi >= a.m) return;
    Wave<DT, MET> w(a, smem + static_cast<size_t>(wid) * a.wave_bytes, qi, lane);
    w.clear_cache();

    int n_exp = 0, n_reset = 0, aborted = 0;
    const int32_t* ent = a.entries + qi * a.E;
    for (int e0 = 0; e0 < a.E; e0 += 64) {
        int v = (e0 + lane < a.E) ? ent[e0 + lane] : -1;
        if (v < 0 || v >= a.N) v = -1;
        w.offer(v);
    }
    int lb = 0;  // every position below lb holds a checked entry
    const int half = 1 << (a.hlog - 1);
    while (true) {
        if (w.fill > half) {
            w.clear_cache();
            w.reseed_cache();
            ++n_reset;
        }
        int fu = -1;
        for (int b = lb; b < w.size; b += 64) {
            int t = b + lane;
            bool un = (t < w.size) && !(w.keys[t] & 1ull);
            uint64_t mk = __ballot(un);
            if (mk) {
                fu = b + __builtin_ctzll(mk);
                break;
            }
        }
        fu = uniform(fu);
        if (fu < 0) break;
        if (n_exp >= a.N) {  // unreachable for exact semantics (each node expands once)
            aborted = 1;
            break;
        }
        const uint64_t ku = w.keys[fu];
        wave_sync();
        if (lane == 0) w.keys[fu] = ku | 1ull;
        wave_sync();
        lb = fu + 1;
        const int u = uniform(static_cast<int>(static_cast<uint32_t>(ku) >> 1));
        ++n_exp;
        int v = -1;
        if (lane < a.R) {
            v = a.adj[static_cast<int64_t>(u) * a.R + lane];
            if (v >= a.N) v = -1;
        }
        int mp = w.offer(v);
        lb = min(lb, mp);
    }
    int32_t* oi = a.out_ids + qi * a.ef;
    float* od = a.out_d + qi * a.ef;
    for (int t = lane; t < a.ef; t += 64) {
        if (t < w.size) {
            uint64_t k = w.keys[t];
            oi[t] = static_cast<int32_t>(static_cast<uint32_t>(k) >> 1);
            od[t] = unord_f32(static_cast<uint32_t>(k >> 32));
        } else {
            oi[t] = -1;
            od[t] = __builtin_huge_valf();
        }
    }
    if (lane == 0) {
        int32_t* c = a.counters + qi * 4;
        c[0] = n_exp;
        c[1] = w.n_dist;
        c[2] = n_reset + w.forgot;
        c[3] = aborted;
    }
}

template <int DT, int MET>
void launch_typed(const BeamArgs& a, int waves_per_block, hipStream_t s) {
    const int blocks = static_cast<int>((a.m + waves_per_block - 1) / waves_per_block);
    const size_t lds = static_cast<size_t>(a.wave_bytes) * waves_per_block;
    hipLaunchKernelGGL((beam_kernel<DT, MET>), dim3(blocks), dim3(64 * waves_per_block), lds, s, a);
}

}  // namespace

int beam_auto_cache_log2(int ef, int R) {
    (void)R;
    int need = 32 * ef;
    int lg = 11;
    while ((1 << lg) < need && lg < 13) ++lg;
    return lg;
}

void launch_beam(const float* Qr, int64_t m, int d_r, const void* Xr, int xr_dtype, int64_t N,
                 const int32_t* adj, int R, const int32_t* entries, int E, int ef, int metric,
                 int cache_log2, int32_t* ids, float* dists, int32_t* counters, hipStream_t s) {
    if (m == 0) return;
    BeamArgs a{};
    a.qr = Qr;
    a.m = m;
    a.d_r = d_r;
    a.xr = static_cast<const unsigned char*>(Xr);
    a.row_bytes = static_cast<int64_t>(d_r) * static_cast<int64_t>(dtype_size(xr_dtype));
    a.N = N;
    a.adj = adj;
    a.R = R;
    a.entries = entries;
    a.E = E;
    a.ef = ef;
    a.ef_alloc = (ef + 63) / 64 * 64;
    a.hlog = cache_log2 > 0 ? cache_log2 : beam_auto_cache_log2(ef, R);
    a.cpr = static_cast<int>(a.row_bytes / 16);
    int gs_log = 0;
    while ((1 << gs_log) < a.cpr) ++gs_log;
    a.gs_log = gs_log;
    a.wave_bytes = a.ef_alloc * 8 + 64 * 8 + 64 * 4 + 64 * 4 + (4 << a.hlog);
    a.out_ids = ids;
    a.out_d = dists;
    a.counters = counters;
    require((1 << a.hlog) >= 4 * a.ef_alloc, "visited cache must hold at least 4*ef entries");
    require(a.cpr >= 1 && a.cpr <= 64, "reduced row must be 16..1024 bytes");
    const int wpb = a.wave_bytes * 2 <= 64 * 1024 ? 2 : 1;
    if (xr_dtype == PA_F32) {
        if (metric == PA_METRIC_L2) launch_typed<PA_F32, PA_METRIC_L2>(a, wpb, s);
        else launch_typed<PA_F32, PA_METRIC_IP>(a, wpb, s);
    } else if (xr_dtype == PA_F16) {
        if (metric == PA_METRIC_L2) launch_typed<PA_F16, PA_METRIC_L2>(a, wpb, s);
        else launch_typed<PA_F16, PA_METRIC_IP>(a, wpb, s);
    } else {
        if (metric == PA_METRIC_L2) launch_typed<PA_BF16, PA_METRIC_L2>(a, wpb, s);
        else launch_typed<PA_BF16, PA_METRIC_IP>(a, wpb, s);
    }
    PA_HIP(hipGetLastError());
}

}  // namespace pa
