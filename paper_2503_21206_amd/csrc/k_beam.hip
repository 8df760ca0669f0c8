// Stage 1 of PilotANN: batched greedy search (Algorithm 1) on the sampled subgraph with
// SVD-reduced vectors (section 4.1), one 64-lane wavefront per query.
//
// Per wavefront:
//   c[CH] (VGPRs)  the candidate list C, sorted ascending by the 64-bit key
//                  (orderable(distance) << 32) | (id << 2) | inexact << 1 | checked; entry t
//                  lives in lane t % 64 of register t / 64; slots at or beyond |C| hold +inf
//   LDS            a scatter area for merges, a 64-slot staging area for the current batch
//                  of neighbours, and an open-addressing visited cache of node ids
//
// Exactness.  The paper keeps visited nodes in a lossy shared-memory Bloom filter
// (section 4.3) and lets the CPU stages repair its false positives.  This kernel instead
// reproduces Algorithm 1 with an exact visited set while holding only a bounded cache:
// the cache never reports an unvisited node as visited (it stores full ids), it may only
// forget nodes.  A forgotten node v that is met again is scored again; if v is still in
// C the duplicate is recognised by its id and dropped, and if v had left C then C was
// full and its ef-th key has only decreased since, so v is rejected again.  Either way C
// evolves exactly as in Algorithm 1; only the count of distance evaluations can exceed
// |visited| (reported per query together with the number of forget events).
//
// Expansion width 2 (an option; not in the paper): each step expands the first two
// unchecked entries of C together, their adjacency rows filling the two halves of the
// wavefront, which halves the number of steps and their fixed costs.
//
// The paper's own visited set is available as an option: a Bloom filter of 32 << hlog
// bits in the same LDS words, two multiplicative hashes per id.  A node whose two bits
// are set counts as visited, also when other nodes set them (a false positive: the node
// is never scored, as in the paper; the host stages can still reach it).  All ids of a
// batch are tested against the filter as it was before the batch, then their bits are
// set, so the outcome does not depend on the order of the lanes' atomics.
//
// Distances (L2).  Every decision must follow the exact distance rounded once to fp32.
// A plain fp32 sum of 16 fused squares per lane plus the lane reduction lies within a
// few dozen units of the orderable encoding of the correctly rounded exact distance, so
// each new candidate is first scored that way (its key flagged inexact).  Two keys whose
// encodings are farther apart than twice that radius are ordered as their exact values,
// which decides nearly every comparison (the ef-th-key filter, the position in C, the
// order among the new candidates).  When some comparison involves closer keys, the
// batch's candidates and the inexact entries of C are re-scored exactly (float-float:
// the correctly rounded value, which any summation order also rounds to) and that step
// is decided on exact keys.  A re-scored key stays within the radius of its plain value,
// so C stays sorted and every decision equals the exact one; the list's order is exact at
// the end, and its remaining plain values are re-scored exactly when the caller reads the
// distances (the search pipeline reads only the ids).  Inner products have no
// relative bound of this kind and are scored exactly at once.
//
// One loop step: find the first unchecked entry of C (one ballot per register), mark it
// checked, take its adjacency row (one coalesced load of R ids, issued one step early for
// the entry that was next in line when it still is), test-and-set the ids in the cache,
// gather the reduced vectors of the new ids (GS lanes per vector, 16 elements per lane,
// all loads of a round in flight together), reduce each distance across its GS lanes
// with DPP butterflies, drop candidates not better than C[ef-1] or already in C, rank
// the survivors against C and against each other with ballots, and apply the merge as
// one scatter to LDS and one gather back into the registers.
#include <hip/hip_runtime.h>

#include <climits>

#include "common.hpp"
#include "ffloat.hpp"

namespace pa {
namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint64_t kInf = ~0ull;
constexpr int kLaneElems = 16;  // vector elements each lane scores per gathered vector
constexpr int kProbes = 16;
constexpr uint32_t kBloomA = 0x9E3779B1u;  // multipliers of the Bloom filter's two hashes
constexpr uint32_t kBloomB = 0x85EBCA77u;

__device__ __forceinline__ uint32_t ord_f32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u ^ 0x80000000u) : ~u);
}
constexpr uint64_t kChecked = 1;
constexpr uint64_t kInexact = 2;
constexpr uint64_t kFlags = 3;
__device__ __forceinline__ uint64_t make_key(float d, uint32_t id) {
    return (static_cast<uint64_t>(ord_f32(d)) << 32) | (static_cast<uint64_t>(id) << 2);
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return static_cast<uint32_t>(k) >> 2; }

// A plain fp32 squared distance s (16 fused squares per lane, then the lane reduction) is
// within 2^-19.4 (relative) of the exact one: each term, all of them non-negative, meets
// at most 24 roundings of 2^-24.  In the orderable encoding that is at most 49 units
// between s and the correctly rounded exact value (24.3 ulps of s's binade, twice as many
// units in the binade below, plus the final rounding); kNear adds a margin.  Keys whose
// encodings differ by more than 2 kNear are therefore ordered as their exact values.
constexpr uint32_t kNear = 80;
// Plain values outside [2^-60, 2^60] (where the relative bound may fail) and non-finite
// ones are never used for a decision: orderable encodings of 2^-60 and 2^60.
constexpr uint32_t kOrdLo = 0x80000000u | (67u << 23);
constexpr uint32_t kOrdHi = 0x80000000u | (187u << 23);
__device__ __forceinline__ bool near(uint32_t a, uint32_t b) { return a - b + 2 * kNear <= 4 * kNear; }
__device__ __forceinline__ uint32_t hi32(uint64_t k) { return static_cast<uint32_t>(k >> 32); }
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
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), l);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), l);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ ff32 dpp(ff32 v) {
    return ff32{dpp<CTRL>(v.hi), dpp<CTRL>(v.lo)};
}
__device__ __forceinline__ ff32 shfl_xor(ff32 v, int m) { return ff32{__shfl_xor(v.hi, m), __shfl_xor(v.lo, m)}; }
// Float-float sum over aligned groups of gs lanes, returned rounded to fp32.  Every step
// pairs two lanes with a symmetric addition, so every lane of a group ends with the same
// bits, and a vector's distance does not depend on which group scored it.
__device__ __forceinline__ float group_sum(ff32 s, int gs) {
    if (gs >= 2) s = ff_add(s, dpp<0xB1>(s));   // quad_perm [1,0,3,2]: lane ^ 1
    if (gs >= 4) s = ff_add(s, dpp<0x4E>(s));   // quad_perm [2,3,0,1]: lane ^ 2
    if (gs >= 8) s = ff_add(s, dpp<0x141>(s));  // row_half_mirror: the other quad of the 8
    if (gs >= 16) s = ff_add(s, dpp<0x140>(s)); // row_mirror: the other half of the 16
    if (gs >= 32) s = ff_add(s, shfl_xor(s, 16));
    if (gs >= 64) s = ff_add(s, shfl_xor(s, 32));
    if (gs == 1) s = ff_norm(s);
    return s.hi;
}
// Plain fp32 sum over aligned groups of gs lanes (same pairing; every lane of a group ends
// with the same bits).
__device__ __forceinline__ float group_sum_plain(float s, int gs) {
    if (gs >= 2) s += dpp<0xB1>(s);
    if (gs >= 4) s += dpp<0x4E>(s);
    if (gs >= 8) s += dpp<0x141>(s);
    if (gs >= 16) s += dpp<0x140>(s);
    if (gs >= 32) s += __shfl_xor(s, 16);
    if (gs >= 64) s += __shfl_xor(s, 32);
    return s;
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
    int ef;             // list size, and the output row stride
    const int32_t* efq; // optional per-query list size (<= ef); entries used = min(E, efq[i])
    int hlog;
    int gs_log;  // log2 of lanes per gathered vector (each lane holds kLaneElems elements)
    int cpr;     // 16-byte chunks per reduced row
    int wave_bytes;
    int bloom;  // 1: the visited set is the Bloom filter described above
    const int32_t* out_map;  // optional: the id written out for row id v is out_map[v]
    int exact_out;           // 0: the caller reads only the ids (and their order) of the output
    int width;               // entries expanded per step: 1, or 2 (R <= 32)
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

template <int CH>
constexpr int wave_lds_bytes(int hlog) {
    return CH * 64 * 8 + 64 * 8 + 64 * 4 + (4 << hlog);
}

// GSL: log2 of the lanes per vector when fixed at compile time (the group reductions and
// load offsets then fold to constants), or -1 to take it from the arguments.
template <int DT, int MET, int CH, int GSL>
struct Wave {
    static constexpr int EPC = Chunk<DT>::kElems;
    static constexpr int KC = kLaneElems / EPC;  // 16-byte chunks per lane per vector

    const BeamArgs& a;
    int lane, sub, grp, gs, vpl, hmask;
    bool ragged;  // gs * KC chunks exceed the row: some lanes hold chunks past its end
    uint64_t c[CH];
    uint64_t* tmp;
    uint64_t* st_key;
    uint32_t* st_id;
    uint32_t* cache;
    float qv[KC][EPC];  // the query elements of this lane's chunks sub, sub + gs, ...
    int ef;
    int size = 0;
    int n_dist = 0;
    int fill = 0;
    int forgot = 0;
    int n_exact = 0;  // steps decided on exact keys after an undecided interval comparison

    __device__ Wave(const BeamArgs& args, unsigned char* base, int64_t qi, int lane_, int ef_) : a(args), lane(lane_) {
        ef = ef_;
        const int gsl = GSL >= 0 ? GSL : a.gs_log;
        gs = 1 << gsl;
        vpl = 64 >> gsl;
        sub = lane & (gs - 1);
        grp = lane >> gsl;
        hmask = (1 << a.hlog) - 1;
        ragged = gs * KC > a.cpr;
        tmp = reinterpret_cast<uint64_t*>(base);
        st_key = tmp + CH * 64;
        st_id = reinterpret_cast<uint32_t*>(st_key + 64);
        cache = st_id + 64;
#pragma unroll
        for (int w = 0; w < CH; ++w) c[w] = kInf;
        const float* q = a.qr + qi * a.d_r;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int ch = sub + j * gs;
#pragma unroll
            for (int e = 0; e < EPC; ++e) qv[j][e] = (ch < a.cpr) ? q[ch * EPC + e] : 0.0f;
        }
    }

    __device__ uint64_t key_at(int t) const {  // t uniform, t < CH * 64
        uint64_t k = kInf;
#pragma unroll
        for (int w = 0; w < CH; ++w)
            if (w == (t >> 6)) k = readlane64(c[w], t & 63);
        return k;
    }

    __device__ void mark_checked(int t) {  // t uniform, t < size
#pragma unroll
        for (int w = 0; w < CH; ++w)
            if (w == (t >> 6) && lane == (t & 63)) c[w] |= kChecked;
    }

    __device__ void clear_cache() {
        const uint32_t empty = a.bloom ? 0u : kEmpty;
        for (int i = lane; i <= hmask; i += 64) cache[i] = empty;
        fill = 0;
        wave_sync();
    }

    // Bloom filter: bit (v * A mod 2^32) >> (32 - log2 bits) for the two multipliers.
    __device__ uint32_t bloom_bit(int v, uint32_t mul) const {
        return (static_cast<uint32_t>(v) * mul) >> (32 - (a.hlog + 5));
    }
    __device__ bool bloom_seen(int v) const {
        const uint32_t b1 = bloom_bit(v, kBloomA), b2 = bloom_bit(v, kBloomB);
        return ((cache[b1 >> 5] >> (b1 & 31)) & (cache[b2 >> 5] >> (b2 & 31)) & 1u) != 0;
    }
    __device__ void bloom_add(int v) {
        const uint32_t b1 = bloom_bit(v, kBloomA), b2 = bloom_bit(v, kBloomB);
        atomicOr(&cache[b1 >> 5], 1u << (b1 & 31));
        atomicOr(&cache[b2 >> 5], 1u << (b2 & 31));
    }

    // Test-and-set of v in the visited cache; true when v must be scored.  The 2^hlog slots
    // form buckets of 4: one 16-byte LDS read tests a bucket; v is visited if the bucket
    // holds it; otherwise a free slot ends the search (v is stored there with a CAS, and a
    // slot taken by another lane meanwhile means reading the bucket again), and a full
    // bucket sends v on to the next one.  Slots are only ever cleared all at once, so the
    // first bucket with a free slot is the last one that can hold v.
    __device__ bool test_and_set(int v, bool& stored) {
        stored = false;
        if (v < 0) return false;
        const uint32_t u = static_cast<uint32_t>(v);
        const uint32_t bmask = static_cast<uint32_t>(hmask) >> 2;
        uint32_t b = hash_slot(u, a.hlog - 2);
#pragma nounroll
        for (int p = 0; p < kProbes; ++p) {
            const uint4 s = reinterpret_cast<const uint4*>(cache)[b];
            if (s.x == u || s.y == u || s.z == u || s.w == u) return false;
            const int e = s.x == kEmpty ? 0 : (s.y == kEmpty ? 1 : (s.z == kEmpty ? 2 : (s.w == kEmpty ? 3 : 4)));
            if (e == 4) {
                b = (b + 1) & bmask;
                continue;
            }
            const uint32_t old = atomicCAS(&cache[b * 4 + e], kEmpty, u);
            if (old == kEmpty) {
                stored = true;
                return true;
            }
            if (old == u) return false;
        }
        return true;  // no free slot nearby: score it (never a false "visited")
    }

    // Re-populate the cache with the ids currently in C after a reset.
    __device__ void reseed_cache() {
#pragma unroll
        for (int w = 0; w < CH; ++w) {
            const int t = w * 64 + lane;
            const int v = (t < size) ? static_cast<int>(key_id(c[w])) : -1;
            bool stored;
            test_and_set(v, stored);
            fill += __popcll(__ballot(stored));
        }
        wave_sync();
    }

    // Float-float partial over this lane's chunks; chunks past the row are zero on both
    // sides and add exactly nothing.
    __device__ ff32 lane_partial(const uint4 (&raw)[KC]) const {
        ff32 s{0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            float x[EPC];
            Chunk<DT>::widen(raw[j], x);
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                if (MET == PA_METRIC_L2) ff_add_sqdiff(s, qv[j][e], x[e]);
                else ff_add_prod(s, qv[j][e], x[e]);
            }
        }
        return s;
    }

    // Plain fp32 partial of the squared distance over this lane's chunks (16 fused squares).
    __device__ float lane_plain(const uint4 (&raw)[KC]) const {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            float x[EPC];
            Chunk<DT>::widen(raw[j], x);
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                const float d = qv[j][e] - x[e];
                s = __builtin_fmaf(d, d, s);
            }
        }
        return s;
    }

    // The key of row id scored by this lane's group (live: the group holds a vector), exact
    // or plain (then flagged inexact).  Every lane of the group returns the same key.
    template <bool EXACT>
    __device__ uint64_t score_row(uint32_t id, bool live) const {
        // idle groups load row 0 (their keys are discarded)
        const unsigned char* row = a.xr + static_cast<int64_t>(live ? id : 0u) * a.row_bytes + sub * 16;
        uint4 raw[KC];
        if (!ragged) {
#pragma unroll
            for (int j = 0; j < KC; ++j) raw[j] = *reinterpret_cast<const uint4*>(row + j * gs * 16);
        } else {  // chunks past the row stay zero
#pragma unroll
            for (int j = 0; j < KC; ++j) {
                raw[j] = make_uint4(0, 0, 0, 0);
                if (sub + j * gs < a.cpr) raw[j] = *reinterpret_cast<const uint4*>(row + j * gs * 16);
            }
        }
        if (EXACT) {
            const float s = group_sum(lane_partial(raw), gs);
            return make_key((MET == PA_METRIC_L2) ? s : -s, id);
        }
        return make_key(group_sum_plain(lane_plain(raw), gs), id) | kInexact;
    }

    // Scores the n staged ids into st_key: vpl vectors per round, gs lanes per vector, KC
    // 16-byte loads per lane (lane sub takes chunks sub, sub + gs, ...: every load
    // instruction reads gs * 16 contiguous bytes of each of vpl rows), all loads of a round
    // in flight.
    template <bool EXACT>
    __device__ void score_staged(int n) {
        for (int b0 = 0; b0 < n; b0 += vpl) {
            const int ci = b0 + grp;
            const bool live = ci < n;
            const uint32_t id = live ? st_id[ci] : 0u;
            const uint64_t k = score_row<EXACT>(id, live);
            if (sub == 0 && live) st_key[ci] = k;
        }
        wave_sync();
    }

    // Re-scores the inexact entries of C exactly (keys keep their checked flag).
    __device__ void exactify_list() {
#pragma unroll
        for (int w = 0; w < CH; ++w) {
            const int t = w * 64 + lane;
            if (t < size) tmp[t] = c[w];
        }
        wave_sync();
        for (int b0 = 0; b0 < size; b0 += vpl) {
            const int t = b0 + grp;
            const uint64_t k = (t < size) ? tmp[t] : 0ull;
            const bool live = t < size && (k & kInexact);
            if (__ballot(live) == 0) continue;
            const uint64_t e = score_row<true>(key_id(k), live);
            if (sub == 0 && live) tmp[t] = e | (k & kChecked);
        }
        wave_sync();
#pragma unroll
        for (int w = 0; w < CH; ++w) {
            const int t = w * 64 + lane;
            if (t < size) c[w] = tmp[t];
        }
        wave_sync();
    }

    // Offer one id per lane (-1 = none) to C.  Returns the smallest position at which an
    // entry was inserted (INT_MAX if none).
    __device__ int offer(int v) {
        bool fresh;
        if (a.bloom) {
            fresh = v >= 0 && !bloom_seen(v);
            wave_sync();  // every test of the batch has read the filter before any bit is set
            if (fresh) bloom_add(v);
        } else {
            bool stored;
            fresh = test_and_set(v, stored);
            fill += __popcll(__ballot(stored));
            forgot += __popcll(__ballot(fresh && !stored));  // scored but not remembered
        }
        const uint64_t newmask = __ballot(fresh);
        const int n_new = __popcll(newmask);
        if (n_new == 0) return INT_MAX;
        if (fresh) st_id[mbcnt(newmask)] = static_cast<uint32_t>(v);
        wave_sync();
        n_dist += n_new;
        constexpr bool kLazy = MET == PA_METRIC_L2;
        score_staged<!kLazy>(n_new);
        for (int pass = 0;; ++pass) {
            const int r = place(n_new, !kLazy || pass > 0);
            if (r != kUndecided) return r;
            // some comparison was not decided by the intervals: decide the step exactly
            score_staged<true>(n_new);
            exactify_list();
            ++n_exact;
        }
    }

    static constexpr int kUndecided = INT_MIN;

    // Merges the scored candidates in st_key[0, n_new) into C.  Returns the smallest
    // position at which an entry was inserted (INT_MAX if none), or kUndecided, with C
    // unchanged, when an inexact key takes part in a comparison that its error could
    // flip (never when all_exact: exact keys are equal only for equal ids).
    __device__ int place(int n_new, bool all_exact) {
        const bool lazy = !all_exact;
        const uint64_t key = (lane < n_new) ? st_key[lane] : kInf;  // stored with its flags
        const uint64_t kc = key & ~kFlags;                           // compared without
        const uint32_t ko = hi32(key);
        uint64_t cw[CH];
#pragma unroll
        for (int w = 0; w < CH; ++w) cw[w] = c[w] & ~kFlags;
        if (lazy && __ballot(lane < n_new && (ko < kOrdLo || ko > kOrdHi)) != 0) return kUndecided;

        // candidates in lanes [0, n_new); drop those not better than the ef-th key (equal
        // keys: the same node)
        uint64_t cand = __ballot(lane < n_new);
        if (size == ef) {
            const uint64_t kth = key_at(ef - 1) & ~kFlags;
            cand = __ballot(lane < n_new && kc < kth);
            if (lazy && __ballot(lane < n_new && kc != kth && near(ko, hi32(kth))) != 0) return kUndecided;
        }
        if (cand == 0) return INT_MAX;

        // position of every candidate in C: a binary search over tmp, which mirrors C
        // (checked flags aside); a candidate equal to an entry is a duplicate, and one
        // close to a neighbouring entry is undecided (entries farther away are farther
        // in the encoding too)
        const bool is_cand = (cand >> lane) & 1ull;
        int pos = 0;
        bool dup = false, open = false;
        if (is_cand && size > 0) {
            int step = 1;
            while (step * 2 <= size) step *= 2;
            for (; step > 0; step >>= 1) {
                const int probe = pos + step - 1;
                if (probe < size && (tmp[probe] & ~kFlags) < kc) pos += step;
            }
            if (pos < size) {
                const uint64_t nx = tmp[pos] & ~kFlags;
                dup = nx == kc;
                open = !dup && near(hi32(nx), ko);
            }
            if (pos > 0) open = open || near(hi32(tmp[pos - 1]), ko);
        }
        uint64_t surv = cand & ~__ballot(dup);
        if (lazy && __ballot(is_cand && !dup && open) != 0) return kUndecided;
        if (surv == 0) return INT_MAX;

        // rank of every survivor among the survivors; shift of every entry of C.  The same
        // id can arrive twice in one batch (when the cache could not store it); the later
        // copy is dropped.
        int rank = 0;
        int shift[CH];
        int minpos = INT_MAX;
        // Common case: the survivors take distinct positions in C.  Positions then order the
        // survivors among themselves (two survivors whose keys are close enough to need a
        // comparison share a position, or an entry of C between them is close to both and
        // was caught above), so ranks and shifts are population counts of the occupied
        // positions, flagged in tmp (the merge below rewrites it).
        bool distinct = false;
        {
            uint32_t* flag = reinterpret_cast<uint32_t*>(tmp);
            const bool mine = (surv >> lane) & 1ull;
#pragma unroll
            for (int w = 0; w < CH; ++w) flag[w * 64 + lane] = 0u;
            wave_sync();
            uint32_t before = 0;
            if (mine) before = atomicAdd(&flag[pos], 1u);
            wave_sync();
            if (__ballot(mine && before != 0) == 0) {
                distinct = true;
                int below = 0;  // survivors placed before register w
#pragma unroll
                for (int w = 0; w < CH; ++w) {
                    const uint64_t occ = __ballot(flag[w * 64 + lane] != 0);
                    shift[w] = below + mbcnt(occ) + static_cast<int>((occ >> lane) & 1ull);
                    if (mine && (pos >> 6) == w) rank = below + __popcll(occ & ((1ull << (pos & 63)) - 1));
                    if (minpos == INT_MAX && occ != 0) minpos = w * 64 + __builtin_ctzll(occ);
                    below += __popcll(occ);
                }
            }
        }
        while (!distinct) {
            const bool mine = (surv >> lane) & 1ull;
            rank = 0;
            minpos = INT_MAX;
#pragma unroll
            for (int w = 0; w < CH; ++w) shift[w] = 0;
            uint64_t close = 0;
            for (uint64_t mm = surv; mm; mm &= mm - 1) {
                const int k = __builtin_ctzll(mm);
                const uint64_t kk = readlane64(kc, k);
                minpos = min(minpos, __builtin_amdgcn_readlane(pos, k));
                rank += (kk < kc) ? 1 : 0;
#pragma unroll
                for (int w = 0; w < CH; ++w) shift[w] += (kk < cw[w]) ? 1 : 0;
                close |= __ballot(mine && k != lane && near(hi32(kk), ko));
            }
            if (close == 0) break;
            // rare: survivors close to each other; equal keys are the same node twice
            bool drop = false, opn = false;
            for (uint64_t mm = surv; mm; mm &= mm - 1) {
                const int k = __builtin_ctzll(mm);
                const uint64_t kk = readlane64(kc, k);
                if (mine && k != lane && near(hi32(kk), ko)) {
                    if (kk == kc) drop = drop || k < lane;
                    else opn = true;
                }
            }
            if (lazy && __ballot(opn) != 0) return kUndecided;
            const uint64_t dropped = __ballot(drop);
            if (dropped == 0) break;
            surv &= ~dropped;
        }
        const int n_ins = __popcll(surv);
        const bool mine = (surv >> lane) & 1ull;

        // merge: scatter old entries and survivors to their final positions, read back
        wave_sync();  // the searches above have read tmp
#pragma unroll
        for (int w = 0; w < CH; ++w) {
            const int t = w * 64 + lane;
            if (t < size) {
                const int nt = t + shift[w];
                if (nt < ef) tmp[nt] = c[w];
            }
        }
        if (mine) {
            const int fp = pos + rank;
            if (fp < ef) tmp[fp] = key;
        }
        wave_sync();
        size = min(size + n_ins, ef);
#pragma unroll
        for (int w = 0; w < CH; ++w) {
            const int t = w * 64 + lane;
            c[w] = (t < size) ? tmp[t] : kInf;
        }
        wave_sync();
        return uniform(minpos);
    }
};

// One-register lists fit in 72 VGPRs, which allows 7 waves per SIMD (LDS allows about as
// many), two-register lists in 80 (6 waves); only the variants with a run-time lane count
// spill a few values.  Larger lists keep the compiler's choice.
template <int DT, int MET, int CH, int GSL, int WIDTH>
__global__ __launch_bounds__(256, (CH == 1 ? 7 : (CH == 2 ? 6 : 1))) void beam_kernel(BeamArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int64_t qi = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + wid;
    if (qi >= a.m) return;
    int ef = a.ef, E = a.E;
    if (a.efq != nullptr) {
        ef = min(max(a.efq[qi], 1), a.ef);
        E = min(E, ef);
    }
    ef = uniform(ef);
    E = uniform(E);
    Wave<DT, MET, CH, GSL> w(a, smem + static_cast<size_t>(wid) * a.wave_bytes, qi, lane, ef);
    w.clear_cache();

    int n_exp = 0, n_reset = 0, aborted = 0;
    const int32_t* ent = a.entries + qi * a.E;
    for (int e0 = 0; e0 < E; e0 += 64) {
        int v = (e0 + lane < E) ? ent[e0 + lane] : -1;
        if (v < 0 || v >= a.N) v = -1;
        w.offer(v);
    }
    int lb = 0;  // every position below lb holds a checked entry
    const int half = 1 << (a.hlog - 1);
    // One step expands the first unchecked entry (width 1: Algorithm 1), or the first two
    // (width 2, R <= 32: lanes 0-31 take the first one's adjacency row, lanes 32-63 the
    // second's).  Speculation: the rows of the entries next in line are loaded while the
    // current step gathers and merges; the next step uses them when the same entries come
    // up, and loads the right rows otherwise.
    auto load_rows = [&](int x, int y) {
        int v = -1;
        if (WIDTH == 2) {
            const int owner = lane < 32 ? x : y;
            const int j = lane & 31;
            if (owner >= 0 && j < a.R) v = a.adj[static_cast<int64_t>(owner) * a.R + j];
        } else if (x >= 0 && lane < a.R) {
            v = a.adj[static_cast<int64_t>(x) * a.R + lane];
        }
        return v;
    };
    int spec_x = -1, spec_y = -1;
    int spec_v = -1;
    while (true) {
        if (w.fill > half) {
            w.clear_cache();
            w.reseed_cache();
            ++n_reset;
        }
        // the first unchecked entries at or after lb: two for width 1 (the one expanded and
        // the next in line), four for width 2 (scalars: an indexed array would live in
        // scratch memory)
        int f0 = -1, f1 = -1, f2 = -1, f3 = -1;
        if (WIDTH == 1) {
#pragma unroll
            for (int wi = 0; wi < CH; ++wi) {
                if (f1 < 0 && (wi + 1) * 64 > lb && wi * 64 < w.size) {
                    const int t = wi * 64 + lane;
                    uint64_t mk = __ballot(t >= lb && t < w.size && !(w.c[wi] & kChecked));
                    if (f0 < 0 && mk) {
                        f0 = wi * 64 + __builtin_ctzll(mk);
                        mk &= mk - 1;
                    }
                    if (f0 >= 0 && mk) f1 = wi * 64 + __builtin_ctzll(mk);
                }
            }
        } else {
            int nf = 0;
#pragma unroll
            for (int wi = 0; wi < CH; ++wi) {
                if (nf < 4 && (wi + 1) * 64 > lb && wi * 64 < w.size) {
                    const int t = wi * 64 + lane;
                    uint64_t mk = __ballot(t >= lb && t < w.size && !(w.c[wi] & kChecked));
                    while (mk && nf < 4) {
                        const int pos = wi * 64 + __builtin_ctzll(mk);
                        if (nf == 0) f0 = pos;
                        else if (nf == 1) f1 = pos;
                        else if (nf == 2) f2 = pos;
                        else f3 = pos;
                        ++nf;
                        mk &= mk - 1;
                    }
                }
            }
        }
        f0 = uniform(f0);
        f1 = uniform(f1);
        if (f0 < 0) break;
        if (n_exp >= a.N) {  // unreachable for exact semantics (each node expands once)
            aborted = 1;
            break;
        }
        const int nw = (WIDTH == 2 && f1 >= 0) ? 2 : 1;  // entries expanded now
        auto id_at = [&](int t) { return t >= 0 ? uniform(static_cast<int>(key_id(w.key_at(t)))) : -1; };
        const int x = id_at(f0);
        int y = -1, nx, ny = -1;
        if (nw == 2) {
            y = id_at(f1);
            nx = id_at(f2);
            ny = id_at(f3);
        } else {
            nx = id_at(f1);
        }
        w.mark_checked(f0);
        if (nw == 2) w.mark_checked(f1);
        lb = (nw == 2 ? f1 : f0) + 1;
        n_exp += nw;
        int v = spec_v;
        if (x != spec_x || y != spec_y) v = load_rows(x, y);
        if (v >= a.N) v = -1;
        spec_x = nx;
        spec_y = ny;
        spec_v = nx >= 0 ? load_rows(nx, ny) : -1;
        const int mp = w.offer(v);
        lb = min(lb, mp);
    }
    // the list's order is already exact; its remaining plain values are re-scored only when
    // the caller reads the distances
    if (MET == PA_METRIC_L2 && a.exact_out) w.exactify_list();
    int32_t* oi = a.out_ids + qi * a.ef;
    float* od = a.out_d + qi * a.ef;
#pragma unroll
    for (int wi = 0; wi < CH; ++wi) {
        const int t = wi * 64 + lane;
        if (t < a.ef) {
            if (t < w.size) {
                const uint32_t v = key_id(w.c[wi]);
                oi[t] = a.out_map ? a.out_map[v] : static_cast<int32_t>(v);
                od[t] = unord_f32(static_cast<uint32_t>(w.c[wi] >> 32));
            } else {
                oi[t] = -1;
                od[t] = __builtin_huge_valf();
            }
        }
    }
    if (lane == 0) {
        int32_t* cnt = a.counters + qi * 4;
        cnt[0] = n_exp;
        cnt[1] = w.n_dist;
        cnt[2] = n_reset + w.forgot;
        cnt[3] = aborted;
    }
}

template <int DT, int MET, int CH, int GSL, int WIDTH>
void launch_wide(BeamArgs a, hipStream_t s) {
    a.wave_bytes = wave_lds_bytes<CH>(a.hlog);
    const int wpb = a.wave_bytes * 2 <= 64 * 1024 ? 2 : 1;
    const int blocks = static_cast<int>((a.m + wpb - 1) / wpb);
    const size_t lds = static_cast<size_t>(a.wave_bytes) * wpb;
    hipLaunchKernelGGL((beam_kernel<DT, MET, CH, GSL, WIDTH>), dim3(blocks), dim3(64 * wpb), lds, s, a);
}

// width 1 (Algorithm 1) and width 2 get separate code, so that width 1 pays nothing for 2
template <int DT, int MET, int CH, int GSL>
void launch_typed(const BeamArgs& a, hipStream_t s) {
    if (a.width == 2) launch_wide<DT, MET, CH, GSL, 2>(a, s);
    else launch_wide<DT, MET, CH, GSL, 1>(a, s);
}

// 4 and 8 lanes per vector (reduced rows of 64 to 128 fp32 or 128 to 256 16-bit elements)
// get their own code; other widths take the lane count at run time.
template <int DT, int MET, int CH>
void launch_gs(const BeamArgs& a, hipStream_t s) {
    if (a.gs_log == 2) launch_typed<DT, MET, CH, 2>(a, s);
    else if (a.gs_log == 3) launch_typed<DT, MET, CH, 3>(a, s);
    else launch_typed<DT, MET, CH, -1>(a, s);
}

template <int DT, int MET>
void launch_ch(const BeamArgs& a, hipStream_t s) {
    const int ch = (a.ef + 63) / 64;
    if (ch <= 1) launch_gs<DT, MET, 1>(a, s);
    else if (ch <= 2) launch_gs<DT, MET, 2>(a, s);
    else if (ch <= 4) launch_gs<DT, MET, 4>(a, s);
    else launch_gs<DT, MET, 8>(a, s);
}

}  // namespace

int beam_auto_cache_log2(int ef, int R) {
    // about 2.5 distance evaluations per expansion and ~ef expansions per query: size the
    // cache so that it stays below half full (its reset threshold) for typical queries.
    // Lists of more than 256 entries take the smallest cache the kernel accepts instead:
    // there the cache's LDS decides how many wavefronts share a CU, and more of them
    // outweigh the re-scores after forgets (at ef 512 on 768-d rows: 2,048 slots 7.9 ms per
    // 10,000 queries, 4,096 slots 12.3 ms, the same lists)
    (void)R;
    const int ef_alloc = (ef + 63) / 64 * 64;
    int need = ef > 256 ? 0 : 6 * ef;
    if (need < 4 * ef_alloc) need = 4 * ef_alloc;
    int lg = 10;
    while ((1 << lg) < need && lg < 13) ++lg;
    return lg;
}

void launch_beam(const float* Qr, int64_t m, int d_r, const void* Xr, int xr_dtype, int64_t N,
                 const int32_t* adj, int R, const int32_t* entries, int E, int ef, int metric,
                 int cache_log2, int32_t* ids, float* dists, int32_t* counters, hipStream_t s,
                 const int32_t* efq, int visited, const int32_t* out_map, bool exact_dists, int width) {
    if (m == 0) return;
    require(width == 1 || (width == 2 && R <= 32), "expansion width must be 1, or 2 with R <= 32");
    BeamArgs a{};
    a.width = width;
    a.efq = efq;
    a.out_map = out_map;
    a.exact_out = exact_dists ? 1 : 0;
    a.bloom = visited == PA_VISITED_BLOOM ? 1 : 0;
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
    a.hlog = cache_log2 > 0 ? cache_log2 : beam_auto_cache_log2(ef, R);
    a.cpr = static_cast<int>(a.row_bytes / 16);
    // lanes per vector: enough lanes of kLaneElems elements (16 / element-size chunks) each
    const int kc = kLaneElems / (16 / static_cast<int>(dtype_size(xr_dtype)));
    int gs_log = 0;
    while ((1 << gs_log) * kc < a.cpr) ++gs_log;
    a.gs_log = gs_log;
    a.out_ids = ids;
    a.out_d = dists;
    a.counters = counters;
    require((1 << a.hlog) >= 4 * ((ef + 63) / 64 * 64), "visited cache must hold at least 4*ef entries");
    require(N <= (int64_t{1} << 30), "the traversal supports at most 2^30 nodes (ids take 30 bits of a key)");
    require(a.row_bytes % 16 == 0, "reduced row must be a multiple of 16 bytes");
    require(a.cpr >= 1 && a.cpr <= 64, "reduced row must be 16..1024 bytes");
    if (xr_dtype == PA_F32) {
        if (metric == PA_METRIC_L2) launch_ch<PA_F32, PA_METRIC_L2>(a, s);
        else launch_ch<PA_F32, PA_METRIC_IP>(a, s);
    } else if (xr_dtype == PA_F16) {
        if (metric == PA_METRIC_L2) launch_ch<PA_F16, PA_METRIC_L2>(a, s);
        else launch_ch<PA_F16, PA_METRIC_IP>(a, s);
    } else {
        if (metric == PA_METRIC_L2) launch_ch<PA_BF16, PA_METRIC_L2>(a, s);
        else launch_ch<PA_BF16, PA_METRIC_IP>(a, s);
    }
    PA_HIP(hipGetLastError());
}

}  // namespace pa
