// Fast entry selection (section 5, Algorithm 2, Table 2).
//
// Algorithm 2 assigns one block per cluster and skips, inside every block, the queries
// routed elsewhere.  Here the queries are first grouped by their routed cluster (a
// counting sort into a preallocated permutation - no allocation, as section 5 asks), and
// then every block works on one (cluster, 16-query tile) pair: a 16 x n_b x d product on
// MFMA against that cluster's bucket of pivots, the distance epilogue fused, a running
// pre-selection per query in LDS, and an exact re-score of the pre-selected pivots before
// the top-E is emitted.  The m x n distance matrix D of Algorithm 2 is never stored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "ffloat.hpp"

namespace pa {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTQ = 16;          // queries per tile (MFMA rows)
constexpr int kMaxClusters = 64;
constexpr int kRerankSlack = 16; // FP32 form pre-selects E + 16 pivots for the exact re-score
constexpr int kWaves = 16;       // one wavefront per query row of a tile: the per-row sorts and
                                 // re-scores are latency bound, so every row gets its own wave
constexpr int kThreads = 64 * kWaves;

__device__ __forceinline__ uint32_t ord_f32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u ^ 0x80000000u) : ~u);
}
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// scratch (int32): [0, r) counts | [r, 2r+1) offsets | [2r+1, 3r+2) tile prefix | perm[m]
__global__ __launch_bounds__(1024) void group_kernel(const int32_t* __restrict__ cluster, int64_t m, int r,
                                                     int32_t* __restrict__ scratch) {
    __shared__ int cnt[kMaxClusters];
    __shared__ int cur[kMaxClusters];
    __shared__ int off[kMaxClusters + 1];
    const int t = threadIdx.x;
    if (t < kMaxClusters) {
        cnt[t] = 0;
        cur[t] = 0;
    }
    __syncthreads();
    for (int64_t i = t; i < m; i += 1024) {
        const int c = cluster[i];
        if (c >= 0 && c < r) atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    if (t == 0) {
        int o = 0, tp = 0;
        for (int c = 0; c < r; ++c) {
            off[c] = o;
            scratch[c] = cnt[c];
            scratch[r + c] = o;
            scratch[2 * r + 1 + c] = tp;
            o += cnt[c];
            tp += (cnt[c] + kTQ - 1) / kTQ;
        }
        off[r] = o;
        scratch[2 * r] = o;
        scratch[3 * r + 1] = tp;
    }
    __syncthreads();
    int32_t* perm = scratch + 3 * r + 2;
    for (int64_t i = t; i < m; i += 1024) {
        const int c = cluster[i];
        if (c >= 0 && c < r) perm[off[c] + atomicAdd(&cur[c], 1)] = static_cast<int32_t>(i);
    }
}

// ---------------------------------------------------------------- pivot scoring
// Any bucket size.  Each query row keeps a running list of its best K2 = next_pow2(K)
// keys (ascending) in LDS.  The bucket is scanned in chunks of K2 pivots, scored on MFMA
// into an approximate distance in the expanded form |q|^2 + |p|^2 - 2 q.p (FP32 form:
// v_mfma_f32_16x16x4f32; FP8 form: queries encoded per row like the pivots, scale =
// max|q| / 448, e4m3 round to nearest even, then v_mfma_f32_16x16x32_fp8_fp8); the
// row's wavefront sorts the chunk descending, keeps the elementwise smaller of list and
// chunk (the lower half of a bitonic merge) and merges it back into ascending order.
// Pre-selection keys carry the pivot's index in its bucket.  The K pre-selected pivots
// are then re-scored in the direct form with float-float arithmetic, so the emitted
// distances are the correctly rounded fp32 ones, and the top E by (distance, node id) is
// emitted.  FP32 form: K = E + 16, so an exact top-E member is lost only if more than 16
// pivots fall within the expanded form's rounding error of it; FP8 form: K is a multiple
// of E that absorbs the e4m3 error.
typedef long fp8x8 __attribute__((ext_vector_type(1)));

__device__ __forceinline__ uint8_t dev_f32_to_e4m3(float x) {
    const uint32_t b = __float_as_uint(x);
    const uint8_t sign = static_cast<uint8_t>((b >> 24) & 0x80u);
    const uint32_t mag = b & 0x7FFFFFFFu;
    if (mag >= 0x43E80000u) return sign | 0x7Fu;
    const int e = static_cast<int>(mag >> 23) - 127;
    if (e < -6) {
        const float q = __builtin_rintf(__uint_as_float(mag) * 512.0f);
        return sign | static_cast<uint8_t>(q);
    }
    uint32_t m = mag & 0x7FFFFFu;
    uint32_t exp8 = static_cast<uint32_t>(e + 7);
    const uint32_t lsb = (m >> 20) & 1u;
    m += 0x7FFFFu + lsb;
    if (m & 0x800000u) {
        m = 0;
        exp8 += 1;
    }
    return sign | static_cast<uint8_t>((exp8 << 3) | ((m >> 20) & 7u));
}

struct FesArgs {
    const float* Qr;
    int d;
    const float* EV;
    const uint8_t* EV8;
    const float* EVscale;
    const float* EVnorm;
    const int32_t* EVid;
    int r, n_b, E, K, K2, CH, P, metric;  // K2 = next power of two >= K
    const int32_t* scratch;
    int32_t* out_ids;
    float* out_d;
};

// Bitonic sort of s[0, n) (n a power of two) by one wavefront, ascending or descending.
__device__ void bitonic_sort(uint64_t* s, int n, int lane, bool descending) {
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < n; i += 64) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t x = s[i], y = s[l];
                    const bool up = ((i & k) == 0) != descending;
                    if ((x > y) == up) {
                        s[i] = y;
                        s[l] = x;
                    }
                }
            }
            wave_sync();
        }
    }
}

// Ascending order of a bitonic sequence s[0, n) (n a power of two).
__device__ void bitonic_merge(uint64_t* s, int n, int lane) {
    for (int j = n >> 1; j > 0; j >>= 1) {
        for (int i = lane; i < n; i += 64) {
            const int l = i ^ j;
            if (l > i) {
                const uint64_t x = s[i], y = s[l];
                if (x > y) {
                    s[i] = y;
                    s[l] = x;
                }
            }
        }
        wave_sync();
    }
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

template <bool FP8>
__global__ __launch_bounds__(kThreads) void score_kernel(FesArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int d = a.d;
    float* Aq = reinterpret_cast<float*>(smem);          // [kTQ][d]
    float* qn = Aq + kTQ * d;                           // [kTQ]
    float* qs = qn + kTQ;                               // [kTQ]
    uint8_t* Aq8 = reinterpret_cast<uint8_t*>(qs + kTQ); // [kTQ][d]
    uint64_t* work = reinterpret_cast<uint64_t*>(Aq8 + ((kTQ * d + 15) / 16) * 16);  // [kTQ][P]
    __shared__ int qidx[kTQ];
    __shared__ int s_c, s_cnt;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r = a.r, n_b = a.n_b, K = a.K, K2 = a.K2, CH = a.CH, P = a.P;
    const int32_t* counts = a.scratch;
    const int32_t* offsets = a.scratch + r;
    const int32_t* tprefix = a.scratch + 2 * r + 1;
    const int32_t* perm = a.scratch + 3 * r + 2;
    const int b = blockIdx.x;
    if (t == 0) {
        int c = -1, cntq = 0;
        if (b < tprefix[r]) {
            c = 0;
            while (c + 1 < r && tprefix[c + 1] <= b) ++c;
            const int tile = b - tprefix[c];
            const int base = offsets[c] + tile * kTQ;
            cntq = min(kTQ, counts[c] - tile * kTQ);
            for (int i = 0; i < kTQ; ++i) qidx[i] = (i < cntq) ? perm[base + i] : -1;
        }
        s_c = c;
        s_cnt = cntq;
    }
    __syncthreads();
    const int c = s_c;
    if (c < 0) return;
    const int cntq = s_cnt;
    for (int idx = t; idx < kTQ * d; idx += kThreads) {
        const int i = idx / d, j = idx - (idx / d) * d;
        Aq[idx] = (i < cntq) ? a.Qr[static_cast<int64_t>(qidx[i]) * d + j] : 0.0f;
    }
    for (int idx = t; idx < kTQ * P; idx += kThreads) work[idx] = ~0ull;
    __syncthreads();
    if (t < kTQ) {
        float s2 = 0.0f, amax = 0.0f;
        for (int j = 0; j < d; ++j) {
            const float x = Aq[t * d + j];
            s2 = __builtin_fmaf(x, x, s2);
            amax = fmaxf(amax, fabsf(x));
        }
        qn[t] = s2;
        qs[t] = amax > 0.0f ? amax / 448.0f : 1.0f;
    }
    __syncthreads();
    if (FP8) {
        for (int idx = t; idx < kTQ * d; idx += kThreads) Aq8[idx] = dev_f32_to_e4m3(Aq[idx] / qs[idx / d]);
        __syncthreads();
    }

    const int64_t cb = static_cast<int64_t>(c) * n_b;
    const int nblk = CH / 16;
    for (int c0 = 0; c0 < n_b; c0 += CH) {
        for (int pb = w; pb < nblk; pb += kWaves) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const int p = c0 + pb * 16 + (lane & 15);
            const bool pv = p < n_b;
            if (FP8) {
                for (int k = 0; k < d; k += 32) {
                    const int kk = k + 8 * (lane >> 4);
                    long av, bv = 0;
                    __builtin_memcpy(&av, Aq8 + (lane & 15) * d + kk, 8);
                    if (pv) __builtin_memcpy(&bv, a.EV8 + (cb + p) * d + kk, 8);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
                }
            } else {
                // B operand of 16 k-steps loaded before the MFMA chain that consumes it
                for (int k0 = 0; k0 < d; k0 += 64) {
                    float bv[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int k = k0 + 4 * i;
                        bv[i] = (pv && k < d) ? a.EV[(cb + p) * d + k + (lane >> 4)] : 0.0f;
                    }
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int k = k0 + 4 * i;
                        if (k < d) {
                            const float av = Aq[(lane & 15) * d + k + (lane >> 4)];
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[i], acc, 0, 0, 0);
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 4 * (lane >> 4) + i;
                uint64_t key = ~0ull;
                if (pv) {
                    const float dot = FP8 ? acc[i] * (qs[row] * a.EVscale[cb + p]) : acc[i];
                    const float dist = (a.metric == PA_METRIC_L2) ? __builtin_fmaf(-2.0f, dot, qn[row] + a.EVnorm[cb + p])
                                                                  : -dot;
                    key = (static_cast<uint64_t>(ord_f32(dist)) << 32) | static_cast<uint32_t>(p);
                }
                work[row * P + CH + pb * 16 + (lane & 15)] = key;
            }
        }
        __syncthreads();
        // fold the chunk into the row's running list s[0, CH) (ascending): sort the chunk
        // descending, keep the smaller of s[i] and chunk[i] (the lower half of a bitonic
        // merge: the CH smallest of both, as a bitonic sequence), merge that ascending
        for (int row = w; row < cntq; row += kWaves) {
            uint64_t* srow = work + row * P;
            bitonic_sort(srow + CH, CH, lane, true);
            for (int i = lane; i < CH; i += 64) {
                const uint64_t x = srow[i], y = srow[CH + i];
                srow[i] = x < y ? x : y;
            }
            wave_sync();
            bitonic_merge(srow, CH, lane);
        }
        __syncthreads();
    }

    for (int row = w; row < cntq; row += kWaves) {
        uint64_t* s = work + row * P;
        // re-score the K pre-selected pivots in the direct form, keys by node id: four
        // lanes per pivot, each over a quarter of the dimensions in float-float, combined
        // symmetrically across the quad (so the value is the correctly rounded distance)
        const float* qv = Aq + row * d;
        const int per = d / 4;
        const int sub = lane & 3;
        for (int base = 0; base < K; base += 16) {
            const int j = base + (lane >> 2);
            const bool live = j < K && s[j] != ~0ull;
            const int p = live ? static_cast<int>(s[j] & 0xFFFFFFFFu) : 0;
            const int k0 = sub * per;  // d is a multiple of 16: per is a multiple of 4
            const float4* pv = reinterpret_cast<const float4*>(a.EV + (cb + p) * d + k0);
            ff32 acc{0.0f, 0.0f};
            // the lane's quarter of the row in pieces of up to 32 floats, every load of a
            // piece issued before its arithmetic
            for (int seg = 0; seg < per; seg += 32) {
                const int n4 = min(32, per - seg) / 4;
                float4 x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = (live && u < n4) ? pv[seg / 4 + u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (u < n4) {
                        const float* q4 = qv + k0 + seg + 4 * u;
                        const float xv[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            if (a.metric == PA_METRIC_L2) ff_add_sqdiff(acc, q4[c], xv[c]);
                            else ff_add_prod(acc, q4[c], xv[c]);
                        }
                    }
                }
            }
            acc = ff_add(acc, ff32{dpp<0xB1>(acc.hi), dpp<0xB1>(acc.lo)});  // lane ^ 1
            acc = ff_add(acc, ff32{dpp<0x4E>(acc.hi), dpp<0x4E>(acc.lo)});  // lane ^ 2
            if (sub == 0 && j < K) {
                uint64_t key = ~0ull;
                if (live) {
                    const float dist = (a.metric == PA_METRIC_L2) ? acc.hi : -acc.hi;
                    key = (static_cast<uint64_t>(ord_f32(dist)) << 32) | static_cast<uint32_t>(a.EVid[cb + p]);
                }
                s[j] = key;
            }
        }
        for (int j = K + lane; j < K2; j += 64) s[j] = ~0ull;
        wave_sync();
        bitonic_sort(s, K2, lane, false);
        const int64_t q = qidx[row];
        for (int e = lane; e < a.E; e += 64) {
            int32_t id = -1;
            float dist = __builtin_huge_valf();
            if (e < K && s[e] != ~0ull) {
                id = static_cast<int32_t>(s[e] & 0xFFFFFFFFu);
                dist = unord_f32(static_cast<uint32_t>(s[e] >> 32));
            }
            a.out_ids[q * a.E + e] = id;
            a.out_d[q * a.E + e] = dist;
        }
    }
}

}  // namespace

size_t select_entries_scratch_ints(int64_t m, int r) { return static_cast<size_t>(3 * r + 2 + m); }

// ---------------------------------------------------------------- static scratch
// For callers that cannot allocate device memory: entry selection's scratch (the
// grouping header and the query permutation) in a fixed device array, one copy per GPU,
// held until the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in symbol); it uses the device address looked up once per
// device with that device current.
constexpr int64_t kStaticFesQueries = 262144;
constexpr int64_t kStaticFesInts = 3 * kMaxClusters + 2 + kStaticFesQueries;
static __device__ __align__(256) int32_t scratch[kStaticFesInts];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int64_t static_scratch_max_queries() { return kStaticFesQueries; }

int32_t* static_scratch_for_device(int device) {
    require(device >= 0 && device < kMaxDevices, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device] == nullptr) {
        int cur = -1;
        PA_HIP(hipGetDevice(&cur));
        require(cur == device, "the static scratch must be looked up with its device current", PA_EINTERNAL);
        void* p = nullptr;
        PA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        require(p != nullptr, "no device address for the static scratch", PA_EHIP);
        g_scratch_ptr[device] = static_cast<int32_t*>(p);
    }
    return g_scratch_ptr[device];
}

void launch_select_entries_chunked(const float* Qr, const int32_t* cluster, int64_t m, int d, const float* EV,
                                   const uint8_t* EV8, const float* EVscale, const float* EVnorm,
                                   const int32_t* EVid, int r, int n_b, int E, int K, int metric, int32_t* ids,
                                   float* dists, int32_t* scratch_i32, hipStream_t s) {
    if (m == 0) return;
    require(r >= 1 && r <= kMaxClusters, "FES supports 1..64 clusters");
    const bool fp8 = EV8 != nullptr;
    if (fp8) require(d % 32 == 0, "FP8 entry selection needs d % 32 == 0", PA_EUNSUPPORTED);
    if (!fp8) K = E + kRerankSlack;
    K = std::max(K, E);
    int dev = 0, max_lds = 64 * 1024;
    PA_HIP(hipGetDevice(&dev));
    PA_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    auto lds_for = [&](int P) {
        return sizeof(float) * (kTQ * d + 2 * kTQ) + static_cast<size_t>((kTQ * d + 15) / 16) * 16 +
               sizeof(uint64_t) * static_cast<size_t>(kTQ) * P;
    };
    // running list of K2 = next_pow2(K) keys per query row, and chunks of the same size
    int K2 = 16;
    while (K2 < K) K2 <<= 1;
    const int CH = K2, P = 2 * K2;
    require(lds_for(P) <= static_cast<size_t>(max_lds), "FES pre-selection list does not fit in LDS", PA_EUNSUPPORTED);
    hipLaunchKernelGGL(group_kernel, dim3(1), dim3(1024), 0, s, cluster, m, r, scratch_i32);
    PA_HIP(hipGetLastError());
    FesArgs a{Qr, d, EV, EV8, EVscale, EVnorm, EVid, r, n_b, E, K, K2, CH, P, metric, scratch_i32, ids, dists};
    const int max_tiles = static_cast<int>((m + kTQ - 1) / kTQ) + r;
    if (fp8) hipLaunchKernelGGL(score_kernel<true>, dim3(max_tiles), dim3(kThreads), lds_for(P), s, a);
    else hipLaunchKernelGGL(score_kernel<false>, dim3(max_tiles), dim3(kThreads), lds_for(P), s, a);
    PA_HIP(hipGetLastError());
}

void launch_select_entries(const float* Qr, const int32_t* cluster, int64_t m, int d, const float* EV,
                           const float* EVnorm, const int32_t* EVid, int r, int n_b, int E, int metric,
                           int32_t* ids, float* dists, int32_t* scratch_i32, hipStream_t s) {
    launch_select_entries_chunked(Qr, cluster, m, d, EV, nullptr, nullptr, EVnorm, EVid, r, n_b, E, E, metric, ids,
                                  dists, scratch_i32, s);
}

}  // namespace pa
