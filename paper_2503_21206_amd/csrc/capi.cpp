// C ABI entry points that operate on caller buffers (no index object): setup steps of
// sections 4.1 / 4.3 / 5 on the host and the stage-isolated GPU calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "common.hpp"
#include "host.hpp"

namespace pa {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }

// ---------------------------------------------------------------- setup helpers

void sample_nodes(int64_t N, const int64_t* rowptr, const int32_t* nbrs, const int64_t* order, int64_t n_target,
                  int mode, uint8_t* mask) {
    require(N >= 0 && n_target >= 0 && n_target <= N, "n_target must be in [0, N]");
    require(mode == PA_SAMPLE_UNIFORM || mode == PA_SAMPLE_SEED_EXPAND, "unknown sampling mode");
    std::memset(mask, 0, static_cast<size_t>(N));
    int64_t count = 0;
    for (int64_t i = 0; i < N && count < n_target; ++i) {
        const int64_t s = order[i];
        require(s >= 0 && s < N, "order entry out of range");
        if (mask[s]) continue;
        mask[s] = 1;
        ++count;
        if (mode == PA_SAMPLE_UNIFORM) continue;
        for (int64_t e = rowptr[s]; e < rowptr[s + 1] && count < n_target; ++e) {
            const int32_t v = nbrs[e];
            require(v >= 0 && v < N, "neighbour id out of range");
            if (!mask[v]) {
                mask[v] = 1;
                ++count;
            }
        }
    }
    require(count == n_target, "order is not a permutation covering n_target nodes");
}

void check_subgraph(int64_t N, const int64_t* rowptr, const int32_t* nbrs, const uint8_t* mask, int R) {
    require(rowptr[0] == 0, "rowptr[0] must be 0");
    std::vector<int64_t> seen(static_cast<size_t>(N), -1);
    for (int64_t u = 0; u < N; ++u) {
        const int64_t b = rowptr[u], e = rowptr[u + 1];
        require(e >= b, "rowptr must be non-decreasing (row " + std::to_string(u) + ")");
        require(e - b <= R, "node " + std::to_string(u) + " has degree " + std::to_string(e - b) + " > " +
                                std::to_string(R));
        if (!mask[u]) require(e == b, "unsampled node " + std::to_string(u) + " has out-edges");
        for (int64_t i = b; i < e; ++i) {
            const int32_t v = nbrs[i];
            require(v >= 0 && v < N, "edge " + std::to_string(u) + "->" + std::to_string(v) + " out of range");
            require(v != u, "self loop at node " + std::to_string(u));
            require(mask[v], "edge " + std::to_string(u) + "->" + std::to_string(v) + " enters an unsampled node");
            require(seen[v] != u, "node " + std::to_string(u) + " has a duplicate neighbour " + std::to_string(v));
            seen[v] = u;
        }
    }
}

std::vector<int32_t> pad_rows(int64_t N, const int64_t* rowptr, const int32_t* nbrs, int R) {
    std::vector<int32_t> out(static_cast<size_t>(N) * R, -1);
    for (int64_t u = 0; u < N; ++u) {
        const int64_t b = rowptr[u], e = rowptr[u + 1];
        require(e >= b && e - b <= R, "row " + std::to_string(u) + " exceeds the padded width");
        for (int64_t i = b; i < e; ++i) {
            require(nbrs[i] >= 0 && nbrs[i] < N, "neighbour id out of range in row " + std::to_string(u));
            out[static_cast<size_t>(u) * R + (i - b)] = nbrs[i];
        }
    }
    return out;
}

void build_entries(const float* P, int n_p, int d, int r, const int32_t* init, int iters, int32_t* buckets,
                   float* centroids_out) {
    require(n_p > 0 && d > 0 && r > 0 && n_p % r == 0, "n_p must be a positive multiple of r");
    const int cap = n_p / r;
    std::vector<double> X(static_cast<size_t>(n_p) * d), C(static_cast<size_t>(r) * d);
    for (size_t i = 0; i < X.size(); ++i) X[i] = P[i];
    std::vector<char> used(static_cast<size_t>(n_p), 0);
    for (int c = 0; c < r; ++c) {
        require(init[c] >= 0 && init[c] < n_p && !used[init[c]], "k-means seeds must be distinct positions");
        used[init[c]] = 1;
        std::copy_n(&X[static_cast<size_t>(init[c]) * d], d, &C[static_cast<size_t>(c) * d]);
    }
    auto sqd = [&](int p, int c) {
        double s = 0.0;
        const double* x = &X[static_cast<size_t>(p) * d];
        const double* y = &C[static_cast<size_t>(c) * d];
        for (int j = 0; j < d; ++j) {
            const double t = x[j] - y[j];
            s += t * t;
        }
        return s;
    };
    std::vector<int> assign(static_cast<size_t>(n_p));
    for (int it = 0; it < iters; ++it) {
        for (int p = 0; p < n_p; ++p) {
            int best = 0;
            double bd = sqd(p, 0);
            for (int c = 1; c < r; ++c) {
                const double dd = sqd(p, c);
                if (dd < bd) {
                    bd = dd;
                    best = c;
                }
            }
            assign[p] = best;
        }
        std::vector<double> sum(static_cast<size_t>(r) * d, 0.0);
        std::vector<int> cnt(static_cast<size_t>(r), 0);
        for (int p = 0; p < n_p; ++p) {
            ++cnt[assign[p]];
            for (int j = 0; j < d; ++j) sum[static_cast<size_t>(assign[p]) * d + j] += X[static_cast<size_t>(p) * d + j];
        }
        for (int c = 0; c < r; ++c)
            if (cnt[c] > 0)
                for (int j = 0; j < d; ++j) C[static_cast<size_t>(c) * d + j] = sum[static_cast<size_t>(c) * d + j] / cnt[c];
    }
    // balanced assignment in (distance, pivot position, cluster) order
    struct Pair {
        double d;
        int p, c;
    };
    std::vector<Pair> pairs;
    pairs.reserve(static_cast<size_t>(n_p) * r);
    for (int p = 0; p < n_p; ++p)
        for (int c = 0; c < r; ++c) pairs.push_back(Pair{sqd(p, c), p, c});
    std::sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {
        if (a.d != b.d) return a.d < b.d;
        if (a.p != b.p) return a.p < b.p;
        return a.c < b.c;
    });
    std::vector<int> owner(static_cast<size_t>(n_p), -1), size(static_cast<size_t>(r), 0);
    for (const Pair& pr : pairs) {
        if (owner[pr.p] < 0 && size[pr.c] < cap) {
            owner[pr.p] = pr.c;
            ++size[pr.c];
        }
    }
    std::vector<int> fill(static_cast<size_t>(r), 0);
    for (int p = 0; p < n_p; ++p) {
        const int c = owner[p];
        require(c >= 0, "balanced assignment left a pivot unassigned", PA_EINTERNAL);
        buckets[static_cast<size_t>(c) * cap + fill[c]++] = p;
    }
    for (int c = 0; c < r; ++c) {
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int i = 0; i < cap; ++i) s += X[static_cast<size_t>(buckets[static_cast<size_t>(c) * cap + i]) * d + j];
            centroids_out[static_cast<size_t>(c) * d + j] = static_cast<float>(s / cap);
        }
    }
}

// Cyclic Jacobi eigensolver for a symmetric matrix (fp64).  Sweeps until every
// off-diagonal entry is negligible relative to the diagonal scale.
void eigh_jacobi(const double* A_in, int D, double* evals, double* evecs) {
    std::vector<double> A(A_in, A_in + static_cast<size_t>(D) * D);
    std::vector<double> V(static_cast<size_t>(D) * D, 0.0);
    for (int i = 0; i < D; ++i) V[static_cast<size_t>(i) * D + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[static_cast<size_t>(i) * D + j]; };
    auto v = [&](int i, int j) -> double& { return V[static_cast<size_t>(i) * D + j]; };
    for (int i = 0; i < D; ++i)
        for (int j = i + 1; j < D; ++j) {
            const double s = 0.5 * (a(i, j) + a(j, i));
            a(i, j) = s;
            a(j, i) = s;
        }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < D; ++i) {
            diag += a(i, i) * a(i, i);
            for (int j = i + 1; j < D; ++j) off += a(i, j) * a(i, j);
        }
        if (off <= 1e-30 * diag || off == 0.0) break;
        for (int p = 0; p < D - 1; ++p) {
            for (int q = p + 1; q < D; ++q) {
                const double apq = a(p, q);
                if (std::fabs(apq) <= 1e-300) continue;
                const double app = a(p, p), aqq = a(q, q);
                if (std::fabs(apq) <= 1e-18 * std::sqrt(std::fabs(app * aqq))) {
                    a(p, q) = a(q, p) = 0.0;
                    continue;
                }
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0);
                const double s = t * c;
                for (int k = 0; k < D; ++k) {
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < D; ++k) {
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < D; ++k) {
                    const double vkp = v(k, p), vkq = v(k, q);
                    v(k, p) = c * vkp - s * vkq;
                    v(k, q) = s * vkp + c * vkq;
                }
            }
        }
    }
    std::vector<int> order(static_cast<size_t>(D));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return a(x, x) > a(y, y); });
    for (int j = 0; j < D; ++j) {
        const int src = order[j];
        evals[j] = a(src, src);
        double mx = 0.0;
        for (int i = 0; i < D; ++i) mx = std::max(mx, std::fabs(v(i, src)));
        int lead = 0;
        for (int i = 0; i < D; ++i)
            if (std::fabs(v(i, src)) >= mx * (1.0 - 1e-12)) {
                lead = i;
                break;
            }
        const double sign = v(lead, src) < 0 ? -1.0 : 1.0;
        for (int i = 0; i < D; ++i) evecs[static_cast<size_t>(i) * D + j] = sign * v(i, src);
    }
}

void fit_projection_host(const float* X, int64_t N, int D, int d_r, int center, float* V_out, double* evals_out,
                         double* mean_out) {
    require(N > 0 && D > 0 && D <= 1024 && d_r > 0 && d_r <= D, "fit_projection: need N > 0, 0 < d_r <= D <= 1024");
    hipStream_t s;
    PA_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } sg{s};
    const int64_t chunk_rows = std::max<int64_t>(1, std::min<int64_t>(N, (int64_t{256} << 20) / (4 * D)));
    float* xdev = nullptr;
    double *G = nullptr, *cs = nullptr;
    PA_HIP(hipMalloc(reinterpret_cast<void**>(&xdev), sizeof(float) * chunk_rows * D));
    std::unique_ptr<void, void (*)(void*)> gx(xdev, [](void* p) { (void)hipFree(p); });
    PA_HIP(hipMalloc(reinterpret_cast<void**>(&G), sizeof(double) * D * D));
    std::unique_ptr<void, void (*)(void*)> gg(G, [](void* p) { (void)hipFree(p); });
    PA_HIP(hipMalloc(reinterpret_cast<void**>(&cs), sizeof(double) * D));
    std::unique_ptr<void, void (*)(void*)> gc(cs, [](void* p) { (void)hipFree(p); });
    for (int64_t r0 = 0; r0 < N; r0 += chunk_rows) {
        const int64_t rows = std::min(chunk_rows, N - r0);
        const float* src = X + r0 * D;
        for (int64_t i = 0; i < rows * D; ++i)
            if (!std::isfinite(src[i])) fail(PA_ENONFINITE, "X holds a non-finite value");
        PA_HIP(hipMemcpyAsync(xdev, src, sizeof(float) * rows * D, hipMemcpyHostToDevice, s));
        launch_gram_f64(xdev, rows, D, G, cs, r0 > 0, s);
        PA_HIP(hipStreamSynchronize(s));
    }
    std::vector<double> Gh(static_cast<size_t>(D) * D), csh(static_cast<size_t>(D));
    PA_HIP(hipMemcpy(Gh.data(), G, sizeof(double) * D * D, hipMemcpyDeviceToHost));
    PA_HIP(hipMemcpy(csh.data(), cs, sizeof(double) * D, hipMemcpyDeviceToHost));
    std::vector<double> M(static_cast<size_t>(D) * D);
    for (int i = 0; i < D; ++i) mean_out[i] = csh[i] / static_cast<double>(N);
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            double m = Gh[static_cast<size_t>(i) * D + j] / static_cast<double>(N);
            if (center) m -= mean_out[i] * mean_out[j];
            M[static_cast<size_t>(i) * D + j] = m;
        }
    std::vector<double> evecs(static_cast<size_t>(D) * D);
    eigh_jacobi(M.data(), D, evals_out, evecs.data());
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < d_r; ++j) V_out[static_cast<size_t>(i) * d_r + j] = static_cast<float>(evecs[static_cast<size_t>(i) * D + j]);
}

std::mutex g_pool_mu;
std::unique_ptr<ThreadPool> g_pool;
std::vector<Visited> g_vis;
int64_t g_vis_n = -1;

}  // namespace pa

using namespace pa;

extern "C" {

const char* pa_last_error(void) { return g_last_error.c_str(); }

int32_t pa_abi_version(void) { return 12; }

pa_status pa_device_init(int32_t device) {
    return guarded([&] {
        int count = 0;
        PA_HIP(hipGetDeviceCount(&count));
        require(device >= 0 && device < count, "no HIP device " + std::to_string(device), PA_EHIP);
        PA_HIP(hipSetDevice(device));
        hipDeviceProp_t prop;
        PA_HIP(hipGetDeviceProperties(&prop, device));
        std::string arch = prop.gcnArchName;
        require(arch.rfind("gfx950", 0) == 0, "device " + std::to_string(device) + " is " + arch + ", not gfx950",
                PA_EUNSUPPORTED);
        static_scratch_for_device(device);  // device address of the allocation-free entry point's scratch
    });
}

pa_status pa_gram_f64(const float* X_dev, int64_t n, int32_t D, double* G_dev, double* colsum_dev,
                      int32_t accumulate, void* stream) {
    return guarded([&] {
        require(X_dev != nullptr || n == 0, "X_dev is null");
        require(G_dev != nullptr && colsum_dev != nullptr, "outputs are null");
        require(n >= 0 && D > 0 && D <= 1024, "need n >= 0 and 0 < D <= 1024");
        if (n == 0) {
            require(accumulate != 0, "n == 0 without accumulate leaves the outputs undefined");
            return;
        }
        launch_gram_f64(X_dev, n, D, G_dev, colsum_dev, accumulate != 0, as_stream(stream));
    });
}

pa_status pa_eigh_f64(const double* A_host, int32_t D, double* evals_host, double* evecs_host) {
    return guarded([&] {
        require(A_host && evals_host && evecs_host, "null pointer");
        require(D > 0 && D <= 1024, "need 0 < D <= 1024");
        for (int64_t i = 0; i < static_cast<int64_t>(D) * D; ++i)
            if (!std::isfinite(A_host[i])) fail(PA_ENONFINITE, "A holds a non-finite value");
        eigh_jacobi(A_host, D, evals_host, evecs_host);
    });
}

pa_status pa_fit_projection(const float* X_host, int64_t N, int32_t D, int32_t d_r, int32_t center, float* V_host,
                            double* evals_host, double* mean_host) {
    return guarded([&] {
        require(X_host && V_host && evals_host && mean_host, "null pointer");
        fit_projection_host(X_host, N, D, d_r, center, V_host, evals_host, mean_host);
    });
}

pa_status pa_project(const float* X_dev, int64_t n, int32_t D, const float* V_dev, int32_t d_r, void* Y_dev,
                     int32_t y_dtype, void* stream) {
    return guarded([&] {
        require(n >= 0 && D > 0 && D <= 4096, "need n >= 0 and 0 < D <= 4096");
        require(d_r > 0 && d_r % 16 == 0 && d_r <= PA_MAX_DR, "d_r must be a multiple of 16 in [16, 256]");
        (void)dtype_size(y_dtype);
        if (n == 0) return;
        require(X_dev && V_dev && Y_dev, "null pointer");
        launch_project(X_dev, n, D, V_dev, d_r, Y_dev, y_dtype, nullptr, 0, nullptr, as_stream(stream));
    });
}

pa_status pa_project_route(const float* Q_dev, int64_t m, int32_t D, const float* V_dev, int32_t d_r,
                           const float* centroids_dev, int32_t r, float* Qr_dev, int32_t* cluster_dev,
                           void* stream) {
    return guarded([&] {
        require(m >= 0 && D > 0 && D <= 4096, "need m >= 0 and 0 < D <= 4096");
        require(d_r > 0 && d_r % 16 == 0 && d_r <= PA_MAX_DR, "d_r must be a multiple of 16 in [16, 256]");
        require(r >= 1 && r <= 64, "r must be in [1, 64]");
        if (m == 0) return;
        require(Q_dev && V_dev && centroids_dev && Qr_dev && cluster_dev, "null pointer");
        launch_project(Q_dev, m, D, V_dev, d_r, Qr_dev, PA_F32, centroids_dev, r, cluster_dev, as_stream(stream));
    });
}

pa_status pa_sample_nodes(int64_t N, const int64_t* rowptr_host, const int32_t* nbrs_host, const int64_t* order_host,
                          int64_t n_target, int32_t mode, uint8_t* mask_host) {
    return guarded([&] {
        require(rowptr_host && order_host && mask_host && (nbrs_host || N == 0), "null pointer");
        sample_nodes(N, rowptr_host, nbrs_host, order_host, n_target, mode, mask_host);
    });
}

pa_status pa_check_subgraph(int64_t N, const int64_t* rowptr_host, const int32_t* nbrs_host, const uint8_t* mask_host,
                            int32_t R) {
    return guarded([&] {
        require(rowptr_host && mask_host, "null pointer");
        require(N >= 0 && N < (int64_t{1} << 31), "N must be below 2^31");
        check_subgraph(N, rowptr_host, nbrs_host, mask_host, R);
    });
}

pa_status pa_pack_adjacency(int64_t N, const int64_t* rowptr_host, const int32_t* nbrs_host, int32_t R,
                            int32_t* adj_dev, void* stream) {
    return guarded([&] {
        require(rowptr_host && adj_dev, "null pointer");
        require(N >= 0 && N < (int64_t{1} << 31), "N must be below 2^31");
        require(R >= 1 && R <= 1024, "R must be in [1, 1024]");
        std::vector<int32_t> padded = pad_rows(N, rowptr_host, nbrs_host, R);
        PA_HIP(hipMemcpyAsync(adj_dev, padded.data(), sizeof(int32_t) * padded.size(), hipMemcpyHostToDevice,
                              as_stream(stream)));
        PA_HIP(hipStreamSynchronize(as_stream(stream)));
    });
}

pa_status pa_build_entries(const float* P_host, int32_t n_p, int32_t d, int32_t r, const int32_t* init_host,
                           int32_t iters, int32_t* buckets_host, float* centroids_host) {
    return guarded([&] {
        require(P_host && init_host && buckets_host && centroids_host, "null pointer");
        require(iters >= 0, "iters must be >= 0");
        for (int64_t i = 0; i < static_cast<int64_t>(n_p) * d; ++i)
            if (!std::isfinite(P_host[i])) fail(PA_ENONFINITE, "pivot vectors hold a non-finite value");
        build_entries(P_host, n_p, d, r, init_host, iters, buckets_host, centroids_host);
    });
}

pa_status pa_quantize_fp8_rows(const float* X_host, int64_t n, int32_t d, uint8_t* codes_host, float* scales_host) {
    return guarded([&] {
        require(n >= 0 && d > 0, "need n >= 0 and d > 0");
        if (n == 0) return;
        require(X_host && codes_host && scales_host, "null pointer");
        for (int64_t i = 0; i < n * d; ++i)
            if (!std::isfinite(X_host[i])) fail(PA_ENONFINITE, "rows hold a non-finite value");
        quantize_rows_e4m3(X_host, n, d, codes_host, scales_host);
    });
}

pa_status pa_select_entries(const float* Qr_dev, const int32_t* cluster_dev, int64_t m, int32_t d,
                            const float* EV_dev, const float* EVnorm_dev, const int32_t* EVid_dev, int32_t r,
                            int32_t n_b, int32_t E, int32_t metric, int32_t* ids_dev, float* d_dev, void* stream) {
    return guarded([&] {
        require(m >= 0, "m must be >= 0");
        require(d > 0 && d % 16 == 0 && d <= PA_MAX_DR, "d must be a multiple of 16 in [16, 256]");
        require(r >= 1 && r <= 64 && n_b >= 1 && E >= 1 && E <= PA_MAX_EF, "need 1<=r<=64, n_b>=1, 1<=E<=512");
        require(metric == PA_METRIC_L2 || metric == PA_METRIC_IP, "unknown metric");
        if (m == 0) return;
        require(Qr_dev && cluster_dev && EV_dev && EVnorm_dev && EVid_dev && ids_dev && d_dev, "null pointer");
        hipStream_t s = as_stream(stream);
        int32_t* scratch = nullptr;
        PA_HIP(hipMallocAsync(reinterpret_cast<void**>(&scratch), sizeof(int32_t) * select_entries_scratch_ints(m, r), s));
        launch_select_entries(Qr_dev, cluster_dev, m, d, EV_dev, EVnorm_dev, EVid_dev, r, n_b, E, metric, ids_dev,
                              d_dev, scratch, s);
        PA_HIP(hipFreeAsync(scratch, s));
    });
}

pa_status pa_select_entries_noalloc(const float* Qr_dev, const int32_t* cluster_dev, int64_t m, int32_t d,
                                    const float* EV_dev, const float* EVnorm_dev, const int32_t* EVid_dev, int32_t r,
                                    int32_t n_b, int32_t E, int32_t metric, int32_t* ids_dev, float* d_dev,
                                    void* stream) {
    return guarded([&] {
        require(m >= 0, "m must be >= 0");
        require(m <= static_scratch_max_queries(),
                "pa_select_entries_noalloc takes at most " + std::to_string(static_scratch_max_queries()) +
                    " queries per call (its static scratch holds that many)");
        require(d > 0 && d % 16 == 0 && d <= PA_MAX_DR, "d must be a multiple of 16 in [16, 256]");
        require(r >= 1 && r <= 64 && n_b >= 1 && E >= 1 && E <= PA_MAX_EF, "need 1<=r<=64, n_b>=1, 1<=E<=512");
        require(metric == PA_METRIC_L2 || metric == PA_METRIC_IP, "unknown metric");
        if (m == 0) return;
        require(Qr_dev && cluster_dev && EV_dev && EVnorm_dev && EVid_dev && ids_dev && d_dev, "null pointer");
        int dev = 0;
        PA_HIP(hipGetDevice(&dev));
        int32_t* scratch = static_scratch_for_device(dev);  // written in full before it is read
        launch_select_entries(Qr_dev, cluster_dev, m, d, EV_dev, EVnorm_dev, EVid_dev, r, n_b, E, metric, ids_dev,
                              d_dev, scratch, as_stream(stream));
    });
}

pa_status pa_select_entries_fp8(const float* Qr_dev, const int32_t* cluster_dev, int64_t m, int32_t d,
                                const float* EV_dev, const uint8_t* EV8_dev, const float* EVscale_dev,
                                const float* EVnorm_dev, const int32_t* EVid_dev, int32_t r, int32_t n_b, int32_t E,
                                int32_t K, int32_t metric, int32_t* ids_dev, float* d_dev, void* stream) {
    return guarded([&] {
        require(m >= 0, "m must be >= 0");
        require(d > 0 && d % 32 == 0 && d <= PA_MAX_DR, "d must be a multiple of 32 in [32, 256]");
        require(r >= 1 && r <= 64 && n_b >= 1 && E >= 1 && E <= PA_MAX_EF && K >= E && K <= 4096,
                "need 1<=r<=64, n_b>=1, 1<=E<=512, E<=K<=4096");
        require(metric == PA_METRIC_L2 || metric == PA_METRIC_IP, "unknown metric");
        if (m == 0) return;
        require(Qr_dev && cluster_dev && EV_dev && EV8_dev && EVscale_dev && EVnorm_dev && EVid_dev && ids_dev && d_dev,
                "null pointer");
        hipStream_t s = as_stream(stream);
        int32_t* scratch = nullptr;
        PA_HIP(hipMallocAsync(reinterpret_cast<void**>(&scratch), sizeof(int32_t) * select_entries_scratch_ints(m, r), s));
        launch_select_entries_chunked(Qr_dev, cluster_dev, m, d, EV_dev, EV8_dev, EVscale_dev, EVnorm_dev, EVid_dev, r,
                                      n_b, E, std::min(K, n_b), metric, ids_dev, d_dev, scratch, s);
        PA_HIP(hipFreeAsync(scratch, s));
    });
}

pa_status pa_gpu_traverse(const float* Qr_dev, int64_t m, int32_t d_r, const void* Xr_dev, int32_t xr_dtype, int64_t N,
                          const int32_t* adj_dev, int32_t R, const int32_t* entries_dev, int32_t E, int32_t ef,
                          int32_t metric, const pa_traverse_opts* opts, int32_t* ids_dev, float* d_dev,
                          int32_t* counters_dev, void* stream) {
    return guarded([&] {
        const pa_traverse_opts o = opts ? *opts : pa_traverse_opts{PA_VISITED_EXACT, 0, 1, nullptr};
        require(m >= 0 && N >= 0 && N < (int64_t{1} << 31), "need m >= 0 and 0 <= N < 2^31");
        require(ef >= 1 && ef <= PA_MAX_EF, "ef must be in [1, 512]");
        require(R >= 1 && R <= PA_MAX_DEGREE, "R must be in [1, 64]");
        require(E >= 0, "E must be >= 0");
        require(d_r > 0 && d_r <= PA_MAX_DR, "d_r must be in [1, 256]");
        require(metric == PA_METRIC_L2 || metric == PA_METRIC_IP, "unknown metric");
        require(o.visited == PA_VISITED_EXACT || o.visited == PA_VISITED_BLOOM, "visited must be exact or bloom");
        require(o.width == 0 || o.width == 1 || (o.width == 2 && R <= 32), "width must be 1, or 2 with R <= 32");
        const size_t row = static_cast<size_t>(d_r) * dtype_size(xr_dtype);
        require(row % 16 == 0 && row <= 1024, "reduced rows must be a multiple of 16 bytes (at most 1024)");
        require(o.cache_log2 == 0 || (o.cache_log2 >= 8 && o.cache_log2 <= 13), "cache_log2 must be 0 or 8..13");
        if (o.cache_log2 != 0)
            require((1 << o.cache_log2) >= 4 * ((ef + 63) / 64 * 64),
                    o.visited == PA_VISITED_BLOOM ? "the Bloom filter must have at least 128*ef bits"
                                                  : "the visited cache must hold 4*ef ids");
        if (m == 0) return;
        require(Qr_dev && Xr_dev && adj_dev && ids_dev && d_dev && counters_dev && (entries_dev || E == 0),
                "null pointer");
        launch_beam(Qr_dev, m, d_r, Xr_dev, xr_dtype, N, adj_dev, R, entries_dev, E, ef, metric, o.cache_log2, ids_dev,
                    d_dev, counters_dev, as_stream(stream), o.ef_dev, o.visited, nullptr, true, o.width <= 1 ? 1 : 2);
    });
}

namespace {
ThreadPool& shared_pool(int threads, int64_t N) {
    if (threads <= 0) threads = host_core_count();
    if (!g_pool || g_pool->size() != threads) {
        g_pool.reset();
        g_pool = std::make_unique<ThreadPool>(threads);
        g_vis.clear();
        g_vis_n = -1;
    }
    if (g_vis_n != N) {
        g_vis.assign(static_cast<size_t>(g_pool->size()), Visited());
        for (auto& v : g_vis) v.reset(N);
        g_vis_n = N;
    }
    return *g_pool;
}
}  // namespace

pa_status pa_cpu_stages(const float* X_host, int64_t N, int32_t D, const int32_t* sub_adj_host, int32_t R_sub,
                        const int32_t* full_adj_host, int32_t R_full, const float* Q_host, int64_t m,
                        const int32_t* beam_host, int32_t n_beam, int32_t ef_cpu, int32_t k, int32_t refine_steps,
                        int32_t metric, int32_t threads, int64_t* out_ids_host, float* out_d_host,
                        int32_t* counters_host) {
    return guarded([&] {
        require(N > 0 && N < (int64_t{1} << 31) && D > 0 && m >= 0, "bad sizes");
        require(R_sub >= 1 && R_sub <= 1024 && R_full >= 1 && R_full <= 1024, "degrees must be in [1, 1024]");
        require(ef_cpu >= 1 && k >= 1 && n_beam >= 0, "need ef_cpu >= 1, k >= 1, n_beam >= 0");
        require(metric == PA_METRIC_L2 || metric == PA_METRIC_IP, "unknown metric");
        if (m == 0) return;
        require(X_host && sub_adj_host && full_adj_host && Q_host && (beam_host || n_beam == 0) && out_ids_host &&
                    out_d_host,
                "null pointer");
        std::lock_guard<std::mutex> lk(g_pool_mu);
        ThreadPool& pool = shared_pool(threads, N);
        StageContext ctx{X_host, N, D, pick_distance(metric), HostGraph{sub_adj_host, R_sub},
                         HostGraph{full_adj_host, R_full}};
        std::vector<std::vector<Cand>> lists(static_cast<size_t>(pool.size()));
        pool.parallel_for(m, [&](int64_t i, int w) {
            StageCounters c;
            host_stages_one(ctx, Q_host + i * D, beam_host + i * n_beam, n_beam, ef_cpu, k, refine_steps, g_vis[w],
                            lists[w], out_ids_host + i * k, out_d_host + i * k, c);
            if (counters_host) {
                int32_t* o = counters_host + i * 4;
                o[0] = c.dist2;
                o[1] = c.dist3;
                o[2] = c.exp3;
                o[3] = 0;
            }
        });
    });
}

pa_status pa_cpu_search(const float* X_host, int64_t N, int32_t D, const int32_t* full_adj_host, int32_t R_full,
                        const float* Q_host, int64_t m, const int32_t* entries_host, int32_t E, int32_t ef, int32_t k,
                        int32_t metric, int32_t threads, int64_t* out_ids_host, float* out_d_host,
                        int32_t* counters_host) {
    return guarded([&] {
        require(N > 0 && N < (int64_t{1} << 31) && D > 0 && m >= 0 && E >= 0, "bad sizes");
        require(R_full >= 1 && R_full <= 1024, "degree must be in [1, 1024]");
        require(ef >= 1 && k >= 1, "need ef >= 1 and k >= 1");
        require(metric == PA_METRIC_L2 || metric == PA_METRIC_IP, "unknown metric");
        if (m == 0) return;
        require(X_host && full_adj_host && Q_host && (entries_host || E == 0) && out_ids_host && out_d_host,
                "null pointer");
        std::lock_guard<std::mutex> lk(g_pool_mu);
        ThreadPool& pool = shared_pool(threads, N);
        StageContext ctx{X_host, N, D, pick_distance(metric), HostGraph{full_adj_host, R_full},
                         HostGraph{full_adj_host, R_full}};
        std::vector<std::vector<Cand>> lists(static_cast<size_t>(pool.size()));
        pool.parallel_for(m, [&](int64_t i, int w) {
            StageCounters c;
            host_search_one(ctx, Q_host + i * D, entries_host + i * E, E, ef, k, g_vis[w], lists[w],
                            out_ids_host + i * k, out_d_host + i * k, c);
            if (counters_host) {
                int32_t* o = counters_host + i * 4;
                o[0] = 0;
                o[1] = c.dist3;
                o[2] = c.exp3;
                o[3] = 0;
            }
        });
    });
}

}  // extern "C"
