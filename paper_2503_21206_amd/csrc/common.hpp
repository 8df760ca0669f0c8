// Internal helpers shared by the host translation units and the kernel launchers.
#pragma once

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "pilotann.h"

namespace pa {

// Error carrying a pa_status; converted to a status code at the C boundary.
struct Error : std::runtime_error {
    pa_status code;
    Error(pa_status c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

void set_last_error(const std::string& msg);
void clear_last_error();

[[noreturn]] inline void fail(pa_status code, const std::string& msg) { throw Error(code, msg); }

inline void require(bool ok, const std::string& msg, pa_status code = PA_EINVAL) {
    if (!ok) fail(code, msg);
}

inline void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        fail(PA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

#define PA_HIP(call) ::pa::hip_check((call), #call)

// Runs `body` and maps exceptions to status codes (the only way out of the ABI).
template <class F>
pa_status guarded(F&& body) {
    try {
        clear_last_error();
        body();
        return PA_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return PA_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return PA_EINTERNAL;
    } catch (...) {
        set_last_error("unknown internal error");
        return PA_EINTERNAL;
    }
}

inline size_t dtype_size(int dt) {
    switch (dt) {
        case PA_F32: return 4;
        case PA_F16: return 2;
        case PA_BF16: return 2;
        default: fail(PA_EUNSUPPORTED, "unknown dtype " + std::to_string(dt));
    }
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// float -> OCP FP8 e4m3 (finite range +-448, no infinities), round to nearest even.  Values
// at or beyond 464 in magnitude have no e4m3 neighbour and map to NaN (0x7F | sign); callers
// scale rows so that |x| <= 448.  The same bit-level rounding is used on the device.
inline uint8_t f32_to_e4m3(float x) {
    uint32_t b;
    __builtin_memcpy(&b, &x, 4);
    const uint8_t sign = static_cast<uint8_t>((b >> 24) & 0x80u);
    const uint32_t mag = b & 0x7FFFFFFFu;
    if (mag >= 0x43E80000u) return sign | 0x7Fu;  // >= 464 (or NaN / Inf)
    const int e = static_cast<int>(mag >> 23) - 127;
    if (e < -6) {  // subnormal e4m3: multiples of 2^-9
        float a;
        __builtin_memcpy(&a, &mag, 4);
        const float q = __builtin_nearbyintf(a * 512.0f);  // exact scaling, RNE
        return sign | static_cast<uint8_t>(q);           // q == 8 is the smallest normal
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

// Per-row FP8 encoding of X [n][d]: scale_i = max|x_ij| / 448 (1 for an all-zero row),
// code_ij = e4m3(x_ij / scale_i).
inline void quantize_rows_e4m3(const float* X, int64_t n, int d, uint8_t* codes, float* scales) {
    for (int64_t i = 0; i < n; ++i) {
        float amax = 0.0f;
        for (int j = 0; j < d; ++j) amax = std::max(amax, std::fabs(X[i * d + j]));
        const float s = amax > 0.0f ? amax / 448.0f : 1.0f;
        scales[i] = s;
        for (int j = 0; j < d; ++j) codes[i * d + j] = f32_to_e4m3(X[i * d + j] / s);
    }
}

// ---- kernel launchers (defined in the .hip translation units) ----

void launch_gram_f64(const float* X, int64_t n, int D, double* G, double* colsum, bool accumulate,
                     hipStream_t s);
void launch_project(const float* X, int64_t n, int D, const float* V, int d_r, void* Y, int y_dtype,
                    const float* centroids, int r, int32_t* cluster, hipStream_t s);
void launch_select_entries(const float* Qr, const int32_t* cluster, int64_t m, int d,
                           const float* EV, const float* EVnorm, const int32_t* EVid, int r, int n_b,
                           int E, int metric, int32_t* ids, float* dists, int32_t* scratch_i32,
                           hipStream_t s);
size_t select_entries_scratch_ints(int64_t m, int r);
// Entry selection's static scratch on `device` (which must be current), for the
// allocation-free entry point; it holds the scratch of this many queries.
int32_t* static_scratch_for_device(int device);
int64_t static_scratch_max_queries();
void launch_select_entries_chunked(const float* Qr, const int32_t* cluster, int64_t m, int d, const float* EV,
                                   const uint8_t* EV8, const float* EVscale, const float* EVnorm,
                                   const int32_t* EVid, int r, int n_b, int E, int K, int metric, int32_t* ids,
                                   float* dists, int32_t* scratch_i32, hipStream_t s);
void launch_beam(const float* Qr, int64_t m, int d_r, const void* Xr, int xr_dtype, int64_t N,
                 const int32_t* adj, int R, const int32_t* entries, int E, int ef, int metric,
                 int cache_log2, int32_t* ids, float* dists, int32_t* counters, hipStream_t s,
                 const int32_t* efq = nullptr, int visited = PA_VISITED_EXACT,
                 const int32_t* out_map = nullptr, bool exact_dists = true, int width = 1);
int beam_auto_cache_log2(int ef, int R);

}  // namespace pa
