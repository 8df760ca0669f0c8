// Fast entry selection (section 5, Algorithm 2, Table 2).
//
// Algorithm 2 assigns one block per cluster and skips, inside every block, the queries
// routed elsewhere.  Here the queries are first grouped by their routed cluster (a
// counting sort into a preallocated permutation - no allocation, as section 5 asks), and
// then every block works on one (cluster, 16-query tile) pair: a 16 x n_b x d product on
// MFMA against that cluster's bucket of pivots, the distance epilogue fused, a running
// candidate list per query in LDS, and an exact re-score of the candidates before the
// top-E is emitted.  The m x n distance matrix D of Algorithm 2 is never stored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "common.hpp"

namespace pa {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTQ = 16;          // queries per tile (MFMA rows)
constexpr int kMaxClusters = 64;
constexpr int kWaves = 16;       // one wavefront per query row of a tile: the per-row selection
                                 // and re-scores are latency bound, so every row gets its own wave
constexpr int kThreads = 64 * kWaves;

__device__ __forceinline__ uint32_t ord_f32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u ^ 0x80000000u) : ~u);
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

// scratch (int32): [0, r) counts | [r, 2r+1) offsets | [2r+1, 3r+2) tile prefix | perm[m]
// One block of 16 wavefronts.  Each wavefront counts its queries in a private histogram
// (no contention between wavefronts); the counts give every (wavefront, cluster) pair its
// own run of the permutation, which the second pass fills.
constexpr int kGroupWaves = 16;
__global__ __launch_bounds__(64 * kGroupWaves) void group_kernel(const int32_t* __restrict__ cluster, int64_t m,
                                                                   int r, int32_t* __restrict__ scratch) {
    __shared__ int hist[kGroupWaves][kMaxClusters];
    __shared__ int base[kGroupWaves][kMaxClusters];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int i = t; i < kGroupWaves * kMaxClusters; i += 64 * kGroupWaves) (&hist[0][0])[i] = 0;
    __syncthreads();
    // wavefront w takes queries [w, w + 16, ...) in runs of 64
    for (int64_t i0 = static_cast<int64_t>(w) * 64; i0 < m; i0 += 64 * kGroupWaves) {
        const int64_t i = i0 + lane;
        const int c = i < m ? cluster[i] : -1;
        if (c >= 0 && c < r) atomicAdd(&hist[w][c], 1);
    }
    __syncthreads();
    if (w == 0) {  // lane c: cluster c's count, then exclusive prefix sums over the clusters
        int cnt = 0;
        if (lane < r)
            for (int v = 0; v < kGroupWaves; ++v) cnt += hist[v][lane];
        const int tiles = (cnt + kTQ - 1) / kTQ;
        int o = cnt, tp = tiles;  // inclusive scans
        for (int d = 1; d < 64; d <<= 1) {
            const int a = __shfl_up(o, d), b = __shfl_up(tp, d);
            if (lane >= d) {
                o += a;
                tp += b;
            }
        }
        o -= cnt;
        tp -= tiles;
        if (lane < r) {
            scratch[lane] = cnt;
            scratch[r + lane] = o;
            scratch[2 * r + 1 + lane] = tp;
            int run = o;
            for (int v = 0; v < kGroupWaves; ++v) {
                base[v][lane] = run;
                run += hist[v][lane];
            }
        }
        if (lane == r - 1) {
            scratch[2 * r] = o + cnt;
            scratch[3 * r + 1] = tp + tiles;
        }
    }
    __syncthreads();
    int32_t* perm = scratch + 3 * r + 2;
    for (int64_t i0 = static_cast<int64_t>(w) * 64; i0 < m; i0 += 64 * kGroupWaves) {
        const int64_t i = i0 + lane;
        const int c = i < m ? cluster[i] : -1;
        if (c >= 0 && c < r) perm[atomicAdd(&base[w][c], 1)] = static_cast<int32_t>(i);
    }
}

// ---------------------------------------------------------------- pivot scoring
// One block per (cluster, 16-query tile); one wavefront per query row of the tile.
//
// The bucket is scanned in chunks of CH pivots (128, or 256 with the scores in registers).
// Per chunk the block scores the 16 x CH tile on MFMA in the expanded form
// ||q||^2 + ||p||^2 - 2 q.p (L2) or -q.p (IP): FP32
// form v_mfma_f32_16x16x4f32; FP8 form v_mfma_f32_16x16x32_fp8_fp8 on per-row e4m3 codes
// (queries encoded on the fly like the pivots: scale = max|q| / 448, round to nearest
// even).  Each row's wavefront then offers the chunk's pivots to the row's candidate
// buffer in LDS and shrinks the buffer when it fills:
//
// * FP32 form (exact).  Each score comes with a rigorous bound eps on its error (the
//   expanded form in fp32: products, their sum, the norms and the final fma each add at
//   most a few units of 2^-24 of (||q||^2 + ||p||^2 + |score|) per term, and eps takes
//   4 (d + 4) of them).  T is the E-th smallest upper end score + eps among the pivots
//   seen so far; a pivot whose lower end score - eps exceeds T has at least E pivots
//   certainly closer and can never be in the top E.  Every other pivot stays.  At the end
//   the survivors (typically E and a few near the boundary) are re-scored exactly (the
//   direct form in fp64, rounded once to fp32: below) and the top E by (distance, node id)
//   are emitted in order.  The result is the exact top E, whatever the rounding of the
//   MFMA pass.
// * FP8 form (approximate, the paper's reduced-precision selection).  The buffer keeps the
//   K best pivots by (FP8 score, position); these are re-scored exactly and the top E by
//   (distance, node id) are emitted.
//
// The E-th / K-th smallest value of a buffer is found by a bitwise search over the ordered
// encoding (one ballot per buffer slot and bit), so no sort runs before the final E.
//
// Exact distances.  Each term of the direct form is formed in fp64 (the difference of two
// fp32 values, or the product of two fp32 values, which is exact) and accumulated by fp64
// fmas; four lanes share a pivot and their partial sums are added pairwise, the same way on
// every lane.  The fp64 sum is within (d + 4) 2^-53 of sum |term| of the exact value and is
// rounded once to fp32: the correctly rounded distance unless the exact one lies within
// that distance of a rounding boundary of fp32 (at d = 128 about 2^23 times closer than
// fp32's own spacing).
// One fp64 fma per term replaces a float-float update of about 15 fp32 instructions, at
// the same issue rate on CDNA.
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

constexpr int kCH = 128;  // pivots per chunk: 8 MFMA column blocks

struct FesArgs {
    const float* Qr;
    int d;
    const float* EV;
    const uint8_t* EV8;
    const float* EVscale;
    const float* EVnorm;
    const int32_t* EVid;
    int r, n_b, E, K, cap, metric;  // K: FP8 pre-selection size; cap: buffer entries per row
    int xcd;                        // 1: tiles grouped by XCD (pivot tables larger than an L2)
    const int32_t* scratch;
    int32_t* out_ids;
    float* out_d;
};

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(u & 0xFFFFFFFFu), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}
__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// A threshold v with exactly the k smallest valid values <= v when the k-th and (k+1)-th
// differ, else the smallest v with #{valid x_i <= v} >= k (k >= 1, at least k valid
// entries), over S values per lane.  Bitwise from the highest bit in which the valid
// values differ (the bits above it are common to all of them), one ballot per slot and
// bit; it stops at the first probe that has exactly k values at or below it.  Either
// result selects the same set {x <= v}.
template <typename T>
__device__ __forceinline__ T wave_min_t(T v) {
    for (int o = 32; o > 0; o >>= 1) {
        const T w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max_t(T v) {
    for (int o = 32; o > 0; o >>= 1) {
        const T w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}
template <typename T, int BITS, int S>
__device__ T kth_smallest(const T (&x)[S], const bool (&ok)[S], int slots, int k) {
    T lo = ~T(0), hi = 0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        if (i < slots && ok[i]) {
            lo = x[i] < lo ? x[i] : lo;
            hi = x[i] > hi ? x[i] : hi;
        }
    }
    lo = wave_min_t(lo);
    hi = wave_max_t(hi);
    if (lo == hi) return lo;
    const int top = (BITS == 64) ? 63 - __clzll(static_cast<unsigned long long>(lo ^ hi))
                                 : 31 - __clz(static_cast<unsigned int>(lo ^ hi));
    // the bits above `top`, common to every valid value (none when top is the highest bit)
    const T v0 = top == BITS - 1 ? T(0) : (lo & ~((T(2) << top) - 1));
    T v = v0;
    for (int bit = top; bit >= 0; --bit) {
        const T probe = v | ((T(1) << bit) - 1);
        int c = 0;
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (i < slots) c += __popcll(__ballot(ok[i] && x[i] <= probe));
        if (c == k) return probe;
        if (c < k) v |= T(1) << bit;
    }
    return v;
}

// Narrows the search for the k-th smallest valid x (1 <= k < valid) while more values than
// `room` share its leading bits.  Returns b >= 0 when the values in [v, v | (2^b - 1)]
// (those sharing v's bits above b) number at most `room`, with `below` values under v; or
// -1 with v a threshold: exactly k values are <= v (`exact`), or v is the k-th smallest
// value itself and some of the values equal to it are taken.  Bitwise from the highest
// bit in which the values differ, one ballot per slot and bit.
template <int S>
__device__ int narrow_kth(const uint32_t (&x)[S], const bool (&ok)[S], int slots, int k, int valid, int room,
                          uint32_t& v, int& below, bool& exact) {
    uint32_t lo = ~0u, hi = 0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        if (i < slots && ok[i]) {
            lo = x[i] < lo ? x[i] : lo;
            hi = x[i] > hi ? x[i] : hi;
        }
    }
    lo = wave_min_t(lo);
    hi = wave_max_t(hi);
    below = 0;
    exact = false;
    if (lo == hi) {
        v = lo;
        return -1;
    }
    const int top = 31 - __clz(lo ^ hi);
    v = top == 31 ? 0u : (lo & ~((2u << top) - 1));
    int upper = valid;  // values <= v | (2^(bit+1) - 1)
    for (int bit = top; bit >= 0; --bit) {
        const uint32_t probe = v | ((1u << bit) - 1);
        int c = 0;
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (i < slots) c += __popcll(__ballot(ok[i] && x[i] <= probe));
        if (c == k) {
            v = probe;
            exact = true;
            return -1;
        }
        if (c < k) {
            below = c;
            v |= 1u << bit;
        } else {
            upper = c;
        }
        if (upper - below <= room) return bit;
    }
    return -1;
}

// The state of one row: its candidate buffer in LDS and the running threshold.  An entry
// is (ordered value << 32) | position in the bucket, plus (FP32 form) the bound of the
// value's error, 0 once the value is exact.  S slots per lane hold up to 64 S entries.
template <bool FP8, int S>
struct Row {
    const FesArgs& a;
    int64_t cb;
    int lane, cnt = 0;
    uint64_t* key;  // [cap]
    float* eps;     // [cap] (FP32 form)
    uint32_t T32 = 0xFFFFFFFFu;  // FP32 form: ordered upper-bound threshold
    uint64_t T64 = ~0ull;        // FP8 form: ordered (score, position) threshold

    __device__ Row(const FesArgs& args, int64_t cb_, uint64_t* k, float* e, int l)
        : a(args), cb(cb_), lane(l), key(k), eps(e) {}

    __device__ static bool finite(float v) { return fabsf(v) <= 3.0e38f; }
    __device__ static uint32_t lo_ord(float v, float e) { return ord_f32(v - e); }
    __device__ static uint32_t hi_ord(float v, float e) { return ord_f32(v + e); }

    // Offer one pivot per lane (ok: the lane holds one).
    __device__ void offer(bool ok, float v, float e, int pos) {
        const uint64_t k = (static_cast<uint64_t>(ord_f32(v)) << 32) | static_cast<uint32_t>(pos);
        bool admit;
        if (FP8) admit = ok && k <= T64;
        else admit = ok && (!finite(v) || lo_ord(v, e) <= T32);
        const uint64_t m = __ballot(admit);
        if (admit) {
            const int at = cnt + mbcnt(m);
            key[at] = k;
            if (!FP8) eps[at] = e;
        }
        cnt += __popcll(m);
        wave_sync();
    }

    __device__ void load(uint64_t (&kk)[S], float (&ee)[S], bool (&ok)[S], int slots) const {
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const int t = i * 64 + lane;
            ok[i] = i < slots && t < cnt;
            kk[i] = ok[i] ? key[t] : ~0ull;
            ee[i] = (!FP8 && ok[i]) ? eps[t] : 0.0f;
        }
    }

    __device__ void store_kept(const uint64_t (&kk)[S], const float (&ee)[S], const bool (&keep)[S], int slots) {
        wave_sync();
        int n = 0;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            if (i < slots) {
                const uint64_t m = __ballot(keep[i]);
                if (keep[i]) {
                    const int at = n + mbcnt(m);
                    key[at] = kk[i];
                    if (!FP8) eps[at] = ee[i];
                }
                n += __popcll(m);
            }
        }
        cnt = n;
        wave_sync();
    }

    // Drops the entries that can no longer be among the best `want`.
    __device__ void shrink(int want) {
        if (cnt <= want) return;
        const int slots = (cnt + 63) / 64;
        uint64_t kk[S];
        float ee[S];
        bool ok[S], keep[S];
        load(kk, ee, ok, slots);
        if (FP8) {
            T64 = kth_smallest<uint64_t, 64, S>(kk, ok, slots, want);
#pragma unroll
            for (int i = 0; i < S; ++i) keep[i] = ok[i] && kk[i] <= T64;
        } else {
            uint32_t ub[S];
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const float v = unord_f32(static_cast<uint32_t>(kk[i] >> 32));
                // a value outside the finite range never bounds T and is never dropped
                ub[i] = (ok[i] && finite(v)) ? hi_ord(v, ee[i]) : 0xFFFFFFFFu;
            }
            const uint32_t t = kth_smallest<uint32_t, 32, S>(ub, ok, slots, want);
            T32 = t < T32 ? t : T32;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                const float v = unord_f32(static_cast<uint32_t>(kk[i] >> 32));
                keep[i] = ok[i] && (!finite(v) || lo_ord(v, ee[i]) <= T32);
            }
        }
        store_kept(kk, ee, keep, slots);
    }

    // Re-scores every entry exactly (fp64 direct form, rounded once): four lanes per pivot,
    // lane s of the four taking the row's 16-byte pieces s, s + 4, s + 8, ... (a quad reads
    // 64 contiguous bytes of the pivot per step, and the query's matching 64 bytes of LDS,
    // without bank conflicts); up to 4 pieces per lane and the node id are loaded before
    // the arithmetic.  Sixteen pivots per pass.  qv: the query row (fp32, in LDS).
    __device__ void rescore(const float* qv, bool node_ids = false, int from = 0) {
        const int d = a.d, nq = d / 16, sub = lane & 3;  // pieces per lane (d % 16 == 0)
        constexpr int PW = 4;  // pieces loaded together
        for (int base = from; base < cnt; base += 16) {
            const int t = base + (lane >> 2);
            const bool live = t < cnt;
            const int pos = live ? static_cast<int>(key[t] & 0xFFFFFFFFu) : 0;
            const float4* pv = reinterpret_cast<const float4*>(a.EV + (cb + pos) * d);
            const uint32_t low = (node_ids && live && sub == 0) ? static_cast<uint32_t>(a.EVid[cb + pos])
                                                               : static_cast<uint32_t>(pos);
            double acc = 0.0;
            for (int s0 = 0; s0 < nq; s0 += PW) {
                float4 x[PW];
#pragma unroll
                for (int u = 0; u < PW; ++u)
                    x[u] = (s0 + u < nq && live) ? pv[4 * (s0 + u) + sub] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int u = 0; u < PW; ++u) {
                    if (s0 + u < nq) {
                        const float4 qa = reinterpret_cast<const float4*>(qv)[4 * (s0 + u) + sub];
                        const double qd[4] = {qa.x, qa.y, qa.z, qa.w};
                        const float xv[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            if (a.metric == PA_METRIC_L2) {
                                const double df = qd[c] - static_cast<double>(xv[c]);
                                acc = __builtin_fma(df, df, acc);
                            } else {
                                acc = __builtin_fma(qd[c], static_cast<double>(xv[c]), acc);
                            }
                        }
                    }
                }
            }
            acc += dpp64<0xB1>(acc);  // lane ^ 1
            acc += dpp64<0x4E>(acc);  // lane ^ 2
            const float v = (a.metric == PA_METRIC_L2) ? static_cast<float>(acc) : -static_cast<float>(acc);
            if (live && sub == 0) {
                key[t] = (static_cast<uint64_t>(ord_f32(v)) << 32) | low;
                if (!FP8) eps[t] = 0.0f;
            }
        }
        wave_sync();
    }

    // Exact values: keeps the best `want` by (distance, node id) (distinct: the node ids of
    // a bucket are distinct).  Returns the largest kept distance's ordered encoding.
    // With node_ids the keys already carry node ids in their low bits.
    __device__ uint32_t keep_best(int want, bool node_ids = false) {
        const int slots = (cnt + 63) / 64;
        uint64_t kk[S], nk[S];
        float ee[S];
        bool ok[S], keep[S];
        load(kk, ee, ok, slots);
#pragma unroll
        for (int i = 0; i < S; ++i)
            nk[i] = !ok[i] ? ~0ull
                           : node_ids ? kk[i]
                                      : ((kk[i] & 0xFFFFFFFF00000000ull) |
                                         static_cast<uint32_t>(a.EVid[cb + static_cast<int64_t>(kk[i] & 0xFFFFFFFFu)]));
        const uint64_t t = cnt > want ? kth_smallest<uint64_t, 64, S>(nk, ok, slots, want) : ~0ull;
#pragma unroll
        for (int i = 0; i < S; ++i) keep[i] = ok[i] && nk[i] <= t;
        store_kept(kk, ee, keep, slots);
        return static_cast<uint32_t>(t >> 32);
    }

};

// SL > 0: the row's n_b <= 64 SL scores stay in registers (SL per lane) and one selection
// runs after the last chunk; SL == 0: the candidate list in LDS is shrunk as chunks arrive
// (any bucket size).
template <bool FP8, int S, int SL, bool WIDE>
__global__ __launch_bounds__(kThreads) void score_kernel(FesArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    // pivots per chunk: the register path takes 256 where LDS allows (one 16 x 16 block per
    // wavefront, half as many block barriers), else 128 like the list path (whose list
    // keeps room for one chunk)
    constexpr int CH = (SL > 0 && WIDE) ? 2 * kCH : kCH;
    const int d = a.d;
    float* Aq = reinterpret_cast<float*>(smem);                      // [kTQ][d]
    float* sc = Aq + kTQ * d;                                        // [kTQ][CH] chunk scores
    uint64_t* bkey = reinterpret_cast<uint64_t*>(sc + kTQ * CH);    // [kTQ][cap]
    float* beps = reinterpret_cast<float*>(bkey + kTQ * a.cap);      // [kTQ][cap] (FP32 form)
    uint8_t* Aq8 = reinterpret_cast<uint8_t*>(beps + (FP8 ? 0 : kTQ * a.cap));  // [kTQ][d] (FP8)
    __shared__ int qidx[kTQ];
    __shared__ float qn[kTQ], qs[kTQ];
    __shared__ int s_c, s_cnt;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int r = a.r, n_b = a.n_b;
    const int32_t* counts = a.scratch;
    const int32_t* offsets = a.scratch + r;
    const int32_t* tprefix = a.scratch + 2 * r + 1;
    const int32_t* perm = a.scratch + 3 * r + 2;
    // workgroups go to the 8 XCDs round robin (workgroup i to XCD i mod 8).  With xcd set,
    // tile b of the cluster-ordered tiles is given to workgroup 8 (b mod T) + b / T
    // (T = gridDim.x / 8): every XCD takes a contiguous run of tiles (a few whole clusters),
    // so the pivots it reads stay in its L2
    const int b = a.xcd ? static_cast<int>(blockIdx.x % 8) * static_cast<int>(gridDim.x / 8) + static_cast<int>(blockIdx.x / 8)
                        : static_cast<int>(blockIdx.x);
    if (w == 0) {
        // this block's cluster: the number of clusters whose tiles all come before tile b
        // (the tile prefix is non-decreasing)
        const bool before = lane < r && tprefix[lane + 1] <= b;
        const int c = __popcll(__ballot(before));
        int cntq = 0, base = 0;
        if (c < r) {
            const int tile = b - tprefix[c];
            base = offsets[c] + tile * kTQ;
            cntq = min(kTQ, counts[c] - tile * kTQ);
        }
        if (lane < kTQ) qidx[lane] = (c < r && lane < cntq) ? perm[base + lane] : -1;
        if (lane == 0) {
            s_c = c < r ? c : -1;
            s_cnt = cntq;
        }
    }
    __syncthreads();
    const int c = s_c;
    if (c < 0) return;
    const int cntq = s_cnt;
    const int d4 = d / 4;
    for (int idx = t; idx < kTQ * d4; idx += kThreads) {
        const int i = idx / d4, j = idx - i * d4;
        const float4 v = (i < cntq) ? reinterpret_cast<const float4*>(a.Qr + static_cast<int64_t>(qidx[i]) * d)[j]
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
        reinterpret_cast<float4*>(Aq)[idx] = v;
    }
    __syncthreads();
    {  // the row's squared norm and FP8 scale (one wavefront per row)
        float s2 = 0.0f, amax = 0.0f;
        for (int j = lane; j < d; j += 64) {
            const float x = Aq[w * d + j];
            s2 = __builtin_fmaf(x, x, s2);
            amax = fmaxf(amax, fabsf(x));
        }
        s2 = wave_sum(s2);
        amax = wave_max(amax);
        if (lane == 0) {
            qn[w] = s2;
            qs[w] = amax > 0.0f ? amax / 448.0f : 1.0f;
        }
    }
    __syncthreads();
    if (FP8) {
        for (int idx = t; idx < kTQ * d; idx += kThreads) Aq8[idx] = dev_f32_to_e4m3(Aq[idx] / qs[idx / d]);
        __syncthreads();
    }

    const int64_t cb = static_cast<int64_t>(c) * n_b;
    const int want = FP8 ? a.K : a.E;
    Row<FP8, S> row(a, cb, bkey + static_cast<size_t>(w) * a.cap, beps + static_cast<size_t>(w) * a.cap, lane);
    // error bound of a score: 4 (d + 4) units of 2^-24 of ||q||^2 + ||p||^2 + |score|
    const float eps_c = 4.0f * static_cast<float>(d + 4) * 5.9604645e-8f;
    const int g = lane >> 4, col = lane & 15;
    float sv[SL > 0 ? SL : 1], se[SL > 0 ? SL : 1];  // register path: the row's scores and bounds
#pragma unroll
    for (int ci = 0; ci < (SL > 0 ? SL / (CH / 64) : 1 << 30); ++ci) {
        const int c0 = ci * CH;
        if (c0 >= n_b) break;
        if (w < CH / 16) {  // one 16 x 16 block of the tile per wavefront
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const int p = c0 + w * 16 + col;
            const bool pv = p < n_b;
            if (FP8) {
                for (int k0 = 0; k0 < d; k0 += 256) {  // the pivot's loads of 8 k-steps in flight together
                    long bv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        bv[u] = 0;
                        const int k = k0 + 32 * u;
                        if (pv && k < d) __builtin_memcpy(&bv[u], a.EV8 + (cb + p) * d + k + 8 * g, 8);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int k = k0 + 32 * u;
                        if (k < d) {
                            long av;
                            __builtin_memcpy(&av, Aq8 + col * d + k + 8 * g, 8);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv[u], acc, 0, 0, 0);
                        }
                    }
                }
            } else {
                // product step s = 4 i + e takes element 16 i + 4 g + e in lane group g, so
                // each lane reads 16 contiguous bytes of its row per four steps
                const float4* prow = reinterpret_cast<const float4*>(a.EV + (cb + (pv ? p : 0)) * d);
                const float4* qrow = reinterpret_cast<const float4*>(Aq + col * d);
                const int n16 = d / 16;
                for (int i0 = 0; i0 < n16; i0 += 4) {
                    float4 bv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        bv[u] = (pv && i0 + u < n16) ? prow[4 * (i0 + u) + g] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (i0 + u < n16) {
                            const float4 av = qrow[4 * (i0 + u) + g];
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv[u].x, acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv[u].y, acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv[u].z, acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv[u].w, acc, 0, 0, 0);
                        }
                    }
                }
            }
            const float pn = pv ? a.EVnorm[cb + p] : 0.0f;
            const float ps = (FP8 && pv) ? a.EVscale[cb + p] : 1.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {  // output element i of the lane: row 4 g + i, column col
                const int rw = 4 * g + i;
                const float dot = FP8 ? acc[i] * (qs[rw] * ps) : acc[i];
                sc[rw * CH + w * 16 + col] =
                    (a.metric == PA_METRIC_L2) ? __builtin_fmaf(-2.0f, dot, qn[rw] + pn) : -dot;
            }
        }
        __syncthreads();
        if constexpr (SL > 0) {
            if (w < cntq) {
#pragma unroll
                for (int h = 0; h < CH / 64; ++h) {
                    const int p = c0 + 64 * h + lane;
                    sv[(CH / 64) * ci + h] = sc[w * CH + 64 * h + lane];
                    se[(CH / 64) * ci + h] = (!FP8 && p < n_b) ? a.EVnorm[cb + p] : 0.0f;  // the norm, for now
                }
            }
        } else if (w < cntq) {
            const float qnw = qn[w];
            float pn[CH / 64];
#pragma unroll
            for (int h = 0; h < CH / 64; ++h) {  // all norm loads in flight before the offers
                const int p = c0 + 64 * h + lane;
                pn[h] = (!FP8 && p < n_b) ? a.EVnorm[cb + p] : 0.0f;
            }
#pragma unroll
            for (int h = 0; h < CH / 64; ++h) {
                const int p = c0 + 64 * h + lane;
                const bool ok = p < n_b;
                const float v = sc[w * CH + 64 * h + lane];
                const float e = (!FP8 && ok) ? eps_c * (qnw + pn[h] + fabsf(v)) : 0.0f;
                row.offer(ok, v, e, p);
            }
            if (row.cnt > a.cap - CH) {
                row.shrink(want);
                if (!FP8 && row.cnt > a.cap - CH) {
                    // (the FP8 list keeps exactly K) more near ties around the
                    // threshold than the slack holds; decide them on exact distances now
                    row.rescore(Aq + w * d);
                    const uint32_t worst = row.keep_best(a.E);
                    row.T32 = worst < row.T32 ? worst : row.T32;
                }
            }
        }
        __syncthreads();
    }
    if (w >= cntq) return;
    if constexpr (SL > 0) {
        // one selection over the row's scores (position of slot i, lane l: 64 i + l)
        const int used = (n_b + 63) / 64;
        uint32_t key[SL];
        bool ok[SL];
        int valid = 0;
#pragma unroll
        for (int i = 0; i < SL; ++i) {
            ok[i] = i < used && 64 * i + lane < n_b;
            valid += __popcll(__ballot(ok[i]));
        }
        if (FP8) {
            // the K best by (score, position): every score below the K-th smallest, and of
            // the scores equal to it the ones at the lowest positions
            const int k = min(a.K, valid);
#pragma unroll
            for (int i = 0; i < SL; ++i) key[i] = ok[i] ? ord_f32(sv[i]) : 0xFFFFFFFFu;
            uint32_t T = 0xFFFFFFFFu;
            int below = 0;
            bool exact = false;
            // the search is narrowed over all of the row's scores until the candidates for
            // the K-th fit the row's list; they are finished there by (score, position)
            const int nbit = k == valid ? -1 : narrow_kth<SL>(key, ok, used, k, valid, a.cap, T, below, exact);
            if (nbit >= 0) {
                const uint32_t top_r = T | ((1u << nbit) - 1);
#pragma unroll
                for (int i = 0; i < SL; ++i) {
                    if (i < used) {
                        const bool in = ok[i] && key[i] >= T && key[i] <= top_r;
                        const uint64_t m = __ballot(in);
                        if (in) row.key[row.cnt + mbcnt(m)] = (static_cast<uint64_t>(key[i]) << 32) | (64 * i + lane);
                        row.cnt += __popcll(m);
                    }
                }
                wave_sync();
                row.shrink(k - below);
#pragma unroll
                for (int i = 0; i < SL; ++i) {  // and every score under the range
                    if (i < used) {
                        const bool in = ok[i] && key[i] < T;
                        const uint64_t m = __ballot(in);
                        if (in) row.key[row.cnt + mbcnt(m)] = (static_cast<uint64_t>(key[i]) << 32) | (64 * i + lane);
                        row.cnt += __popcll(m);
                    }
                }
            } else {
                if (k < valid) {
                    below = 0;
#pragma unroll
                    for (int i = 0; i < SL; ++i)
                        if (i < used) below += __popcll(__ballot(ok[i] && key[i] < T));
                }
                int ties = 0;
#pragma unroll
                for (int i = 0; i < SL; ++i) {
                    if (i < used) {
                        const bool tie = ok[i] && key[i] == T;
                        const uint64_t tm = __ballot(tie);
                        const bool in = ok[i] && (key[i] < T || (tie && ties + mbcnt(tm) < k - below));
                        ties += __popcll(tm);
                        const uint64_t m = __ballot(in);
                        if (in) row.key[row.cnt + mbcnt(m)] = (static_cast<uint64_t>(key[i]) << 32) | (64 * i + lane);
                        row.cnt += __popcll(m);
                    }
                }
            }
            wave_sync();
            row.rescore(Aq + w * d, true);
        } else {
            // drop the scores whose lower end exceeds the E-th smallest upper end
            const float qnw = qn[w];
#pragma unroll
            for (int i = 0; i < SL; ++i) {
                se[i] = eps_c * (qnw + se[i] + fabsf(sv[i]));
                key[i] = !ok[i] ? 0xFFFFFFFFu : (Row<FP8, S>::finite(sv[i]) ? Row<FP8, S>::hi_ord(sv[i], se[i]) : 0xFFFFFFFFu);
            }
            const uint32_t T = valid > a.E ? kth_smallest<uint32_t, 32, SL>(key, ok, used, a.E) : 0xFFFFFFFFu;
            int exact = 0;  // entries [0, exact) of the list are already exact
#pragma unroll
            for (int i = 0; i < SL; ++i) {
                if (i < used) {
                    const bool in = ok[i] && (!Row<FP8, S>::finite(sv[i]) || Row<FP8, S>::lo_ord(sv[i], se[i]) <= T);
                    const uint64_t m = __ballot(in);
                    if (row.cnt + __popcll(m) > a.cap) {  // near ties beyond the slack: decide a batch
                        row.rescore(Aq + w * d, true, exact);
                        row.keep_best(a.E, true);
                        exact = row.cnt;
                    }
                    if (in) row.key[row.cnt + mbcnt(m)] = (static_cast<uint64_t>(ord_f32(sv[i])) << 32) | (64 * i + lane);
                    row.cnt += __popcll(m);
                }
            }
            wave_sync();
            row.rescore(Aq + w * d, true, exact);
        }
    } else {
        row.shrink(want);
        row.rescore(Aq + w * d, true);
    }
    // a long list is cut to the best E first; a short one (at most 128 exact, distinct keys)
    // is ranked as it is
    if (row.cnt > 128 && row.cnt > a.E) row.keep_best(a.E, true);
    // emit in (distance, node id) order: the rank of each key among the list's keys; ranks
    // from E on are not emitted
    const int n = row.cnt;
    const int64_t q = qidx[w];
    for (int e = min(n, a.E) + lane; e < a.E; e += 64) {
        a.out_ids[q * a.E + e] = -1;
        a.out_d[q * a.E + e] = __builtin_huge_valf();
    }
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        const uint64_t mine = i < n ? row.key[i] : ~0ull;
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += row.key[j] < mine ? 1 : 0;
        if (i < n && rank < a.E) {
            a.out_ids[q * a.E + rank] = static_cast<int32_t>(mine & 0xFFFFFFFFu);
            a.out_d[q * a.E + rank] = unord_f32(static_cast<uint32_t>(mine >> 32));
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
    require(d % 16 == 0, "entry selection needs d % 16 == 0", PA_EUNSUPPORTED);
    const bool fp8 = EV8 != nullptr;
    if (fp8) require(d % 32 == 0, "FP8 entry selection needs d % 32 == 0", PA_EUNSUPPORTED);
    K = std::max(K, E);
    // registers for the scores of buckets that span several chunks, up to 2,048 pivots
    // (FP8) or 1,024 (FP32: scores and their bounds); a bucket of one chunk gains nothing
    // from them (its list is shrunk once either way) and keeps the smaller register
    // footprint of the list path, which leaves room for two blocks per CU
    const int need = (n_b + 63) / 64;
    int sl = 0;
    if (fp8) sl = need <= 2 ? 0 : (need <= 8 ? 8 : (need <= 32 ? 32 : 0));
    else sl = need <= 2 ? 0 : (need <= 8 ? 8 : (need <= 16 ? 16 : 0));
    // per-row list: the kept entries (FP32 form: E plus a slack of 64 for candidates whose
    // error interval reaches the threshold), and with the scores not in registers room for
    // one more chunk
    const int keep = fp8 ? K : E + 64;
    const int cap = (keep + (sl > 0 ? 0 : kCH) + 63) / 64 * 64;
    int dev = 0, max_lds = 64 * 1024;
    PA_HIP(hipGetDevice(&dev));
    PA_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // the kernel's LDS for a chunk width: query rows, chunk scores, lists, FP8 query codes
    auto lds_for = [&](int ch) {
        return sizeof(float) * static_cast<size_t>(kTQ) * (d + ch) +
               static_cast<size_t>(kTQ) * cap * (sizeof(uint64_t) + (fp8 ? 0 : sizeof(float))) +
               (fp8 ? static_cast<size_t>(kTQ) * d : 0);
    };
    // the register path takes 256-pivot chunks where they fit
    const bool wide = sl > 0 && lds_for(2 * kCH) <= static_cast<size_t>(max_lds);
    const size_t lds = lds_for(wide ? 2 * kCH : kCH);
    require(cap <= 16 * 64 && lds <= static_cast<size_t>(max_lds),
            "FES candidate list of a 16-query tile does not fit in LDS", PA_EUNSUPPORTED);
    hipLaunchKernelGGL(group_kernel, dim3(1), dim3(64 * kGroupWaves), 0, s, cluster, m, r, scratch_i32);
    PA_HIP(hipGetLastError());
    // pivot rows (fp32, and FP8 codes) of all buckets beyond 4 MiB, the L2 of one XCD: group
    // the tiles by XCD (the grid is then a multiple of 8; the extra blocks find no tile)
    const int64_t table = static_cast<int64_t>(r) * n_b * d * (4 + (fp8 ? 1 : 0));
    const int xcd = table > (int64_t(4) << 20) ? 1 : 0;
    FesArgs a{Qr, d, EV, EV8, EVscale, EVnorm, EVid, r, n_b, E, K, cap, metric, xcd, scratch_i32, ids, dists};
    int blocks = static_cast<int>((m + kTQ - 1) / kTQ) + r;
    if (xcd) blocks = (blocks + 7) / 8 * 8;
    const int slots = cap / 64;
    auto go = [&](auto fp8_tag, auto s_tag, auto sl_tag) {
        constexpr bool F = decltype(fp8_tag)::value;
        constexpr int S_ = decltype(s_tag)::value;
        constexpr int SL_ = decltype(sl_tag)::value;
        if constexpr (SL_ > 0) {
            if (wide) hipLaunchKernelGGL((score_kernel<F, S_, SL_, true>), dim3(blocks), dim3(kThreads), lds, s, a);
            else hipLaunchKernelGGL((score_kernel<F, S_, SL_, false>), dim3(blocks), dim3(kThreads), lds, s, a);
        } else {
            hipLaunchKernelGGL((score_kernel<F, S_, SL_, false>), dim3(blocks), dim3(kThreads), lds, s, a);
        }
    };
    auto by_sl = [&](auto fp8_tag, auto s_tag) {
        using I = std::integral_constant<int, 0>;
        if constexpr (decltype(fp8_tag)::value) {
            if (sl == 8) go(fp8_tag, s_tag, std::integral_constant<int, 8>{});
            else if (sl == 32) go(fp8_tag, s_tag, std::integral_constant<int, 32>{});
            else go(fp8_tag, s_tag, I{});
        } else {
            if (sl == 8) go(fp8_tag, s_tag, std::integral_constant<int, 8>{});
            else if (sl == 16) go(fp8_tag, s_tag, std::integral_constant<int, 16>{});
            else go(fp8_tag, s_tag, I{});
        }
    };
    auto by_s = [&](auto fp8_tag) {
        if (slots <= 4) by_sl(fp8_tag, std::integral_constant<int, 4>{});
        else if (slots <= 8) by_sl(fp8_tag, std::integral_constant<int, 8>{});
        else by_sl(fp8_tag, std::integral_constant<int, 16>{});
    };
    if (fp8) by_s(std::true_type{});
    else by_s(std::false_type{});
    PA_HIP(hipGetLastError());
}

void launch_select_entries(const float* Qr, const int32_t* cluster, int64_t m, int d, const float* EV,
                           const float* EVnorm, const int32_t* EVid, int r, int n_b, int E, int metric,
                           int32_t* ids, float* dists, int32_t* scratch_i32, hipStream_t s) {
    launch_select_entries_chunked(Qr, cluster, m, d, EV, nullptr, nullptr, EVnorm, EVid, r, n_b, E, E, metric, ids,
                                  dists, scratch_i32, s);
}

}  // namespace pa
