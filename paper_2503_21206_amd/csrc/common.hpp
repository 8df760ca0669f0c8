// Internal helpers shared by the host translation units and the kernel launchers.
#pragma once

#include <hip/hip_runtime_api.h>

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
void launch_beam(const float* Qr, int64_t m, int d_r, const void* Xr, int xr_dtype, int64_t N,
                 const int32_t* adj, int R, const int32_t* entries, int E, int ef, int metric,
                 int cache_log2, int32_t* ids, float* dists, int32_t* counters, hipStream_t s,
                 const int32_t* efq = nullptr);
int beam_auto_cache_log2(int ef, int R);

}  // namespace pa
