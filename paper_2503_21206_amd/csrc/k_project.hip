// Projection to the SVD subspace (section 4.1: x_primary = x^T V_d), correctly rounded, the FES
// routing of a reduced query to its nearest coarse centroid (section 5), and the FP64
// second-moment accumulation that fixes V (the only FP64 work on the GPU).
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace pa {
namespace {

// ---------------------------------------------------------------- projection
// y = x^T V_d for a block of 64 rows x 64 columns (256 threads, 4 x 4 outputs each).  The
// method compares single-precision distances (section 6.1), and every later stage sees
// only the reduced vectors, so the projection's fp32 output is defined as the exact
// product rounded once: each product x_k v_k of two fp32 values is exact in fp64, the
// products are accumulated by fp64 fmas in order of k, and the sum is rounded to fp32 at
// the end; fp16 / bf16 outputs are that fp32 value rounded to nearest even.  The sum is
// within D 2^-53 of sum |x_k v_k| of the exact value, so the result is the correctly
// rounded value except when the exact sum lies that close to a rounding boundary of fp32,
// and it does not depend on the batch around a row.  A plain fp32 MFMA product would
// differ from it in the last bits of most outputs, and those bits move near-tied
// decisions of every stage after it.  The product is a small part of a search (2 m D d_r
// flops against the traversal's gathers), so it runs on the vector ALUs (fp64 fma issues
// at the fp32 rate on CDNA); the FES distance products stay on MFMA (their fp32 results
// only pre-select candidates that are re-scored exactly).
constexpr int kPM = 64;  // rows per block
constexpr int kPN = 64;  // columns per block
constexpr int kPK = 16;  // K slice staged in LDS

__device__ __forceinline__ uint16_t f32_to_f16_bits(float v) {
    _Float16 h = static_cast<_Float16>(v);  // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7F800000u) == 0x7F800000u) {  // Inf / NaN: keep class, quiet NaN
        return static_cast<uint16_t>((u >> 16) | ((u & 0x007FFFFFu) ? 0x40u : 0u));
    }
    uint32_t rounding = 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>((u + rounding) >> 16);
}

__global__ __launch_bounds__(256) void project_kernel(const float* __restrict__ X, int64_t n, int D,
                                                      const float* __restrict__ V, int d_r, void* Y,
                                                      int y_dtype) {
    __shared__ float Xs[kPK][kPM + 4];  // X slice, transposed: Xs[k][row]
    __shared__ float Vs[kPK][kPN + 4];  // V slice: Vs[k][column]
    const int t = threadIdx.x;
    const int tr = t >> 4;  // rows 4*tr .. 4*tr+3 of the block
    const int tc = t & 15;  // columns tc, tc+16, tc+32, tc+48 of the block
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kPM;
    const int col0 = blockIdx.y * kPN;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

    for (int k0 = 0; k0 < D; k0 += kPK) {
        {  // X: 64 rows x 16 k, four per thread
            const int r = t >> 2;
            const int c = (t & 3) * 4;
            const int64_t gr = row0 + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + c + e;
                Xs[c + e][r] = (gr < n && k < D) ? X[gr * D + k] : 0.0f;
            }
        }
        {  // V: 16 k x 64 columns, four per thread
            const int kk = t >> 4;
            const int j = (t & 15) * 4;
            const int k = k0 + kk;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int col = col0 + j + e;
                Vs[kk][j + e] = (k < D && col < d_r) ? V[static_cast<int64_t>(k) * d_r + col] : 0.0f;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < kPK; ++kk) {
            const float4 xv = *reinterpret_cast<const float4*>(&Xs[kk][4 * tr]);
            const double xs[4] = {xv.x, xv.y, xv.z, xv.w};
            double vs[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) vs[j] = Vs[kk][tc + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fma(xs[i], vs[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + 4 * tr + i;
        if (row >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = col0 + tc + 16 * j;
            if (col >= d_r) continue;
            const float v = static_cast<float>(acc[i][j]);  // rounded once, to nearest even
            const int64_t off = row * d_r + col;
            if (y_dtype == PA_F32) static_cast<float*>(Y)[off] = v;
            else if (y_dtype == PA_F16) static_cast<uint16_t*>(Y)[off] = f32_to_f16_bits(v);
            else static_cast<uint16_t*>(Y)[off] = f32_to_bf16_bits(v);
        }
    }
}

// ---------------------------------------------------------------- routing
// One wave per query.  Centroid c is scored by lanes c and c + 32 (r <= 32: each over one
// half of the dimensions) or by lane c alone (r > 32): squared differences formed in fp64
// and accumulated by fp64 fmas, the halves added (the same sum on both lanes), and the
// result rounded once to fp32, which is the correctly rounded distance except within
// (d_r + 2) 2^-53 (relative) of a rounding boundary of fp32.  The wave takes the minimum
// (ties to the lowest c).
__global__ __launch_bounds__(256) void route_kernel(const float* __restrict__ Qr, int64_t m, int d_r,
                                                    const float* __restrict__ C, int r,
                                                    int32_t* __restrict__ cluster) {
    const int lane = threadIdx.x & 63;
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (q >= m) return;
    const bool halves = r <= 32;
    const int c = halves ? (lane & 31) : lane;
    const int len = halves ? d_r / 2 : d_r;  // d_r is a multiple of 16: both halves are float4 rows
    const int off = (halves && lane >= 32) ? d_r / 2 : 0;
    double s = 0.0;
    if (c < r) {
        const float4* cv = reinterpret_cast<const float4*>(C + static_cast<int64_t>(c) * d_r + off);
        const float4* q4 = reinterpret_cast<const float4*>(Qr + q * d_r + off);
        for (int seg = 0; seg < len / 4; seg += 4) {  // every load of a piece before its arithmetic
            float4 cc[4], x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool in = seg + u < len / 4;
                cc[u] = in ? cv[seg + u] : make_float4(0.f, 0.f, 0.f, 0.f);
                x[u] = in ? q4[seg + u] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float xa[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
                const float ca[4] = {cc[u].x, cc[u].y, cc[u].z, cc[u].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double df = static_cast<double>(xa[e]) - static_cast<double>(ca[e]);
                    s = __builtin_fma(df, df, s);
                }
            }
        }
    }
    if (halves) s += __shfl_xor(s, 32);
    const float best = static_cast<float>(s);
    // (distance, index) minimum across the wave, lowest index on ties
    uint64_t key = (static_cast<uint64_t>(__float_as_uint(best)) << 32) | static_cast<uint32_t>(c);
    if (c >= r) key = ~0ull;
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t v = __shfl_xor(key, o);
        key = v < key ? v : key;
    }
    if (lane == 0) cluster[q] = static_cast<int32_t>(key & 0xFFFFFFFFu);
}

// ---------------------------------------------------------------- FP64 second moment
// partial[chunk][i][j] = sum over the chunk's rows of x_i x_j (32x32 tile per block,
// rows consumed in order of increasing index); colsum partials likewise; a second pass sums
// the chunk partials in chunk order, so the result does not depend on scheduling.
constexpr int kGT = 32;

__global__ __launch_bounds__(256) void gram_partial_kernel(const float* __restrict__ X, int64_t n, int D,
                                                           int64_t rows_per_chunk,
                                                           double* __restrict__ partial) {
    __shared__ double A[kGT][kGT + 1];
    __shared__ double B[kGT][kGT + 1];
    const int ti = blockIdx.x, tj = blockIdx.y, chunk = blockIdx.z;
    const int t = threadIdx.x;
    const int a = t >> 3;         // row of the G tile
    const int b = (t & 7) * 4;    // first of 4 columns
    const int64_t r_begin = static_cast<int64_t>(chunk) * rows_per_chunk;
    const int64_t r_end = r_begin + rows_per_chunk < n ? r_begin + rows_per_chunk : n;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kGT) {
        for (int idx = t; idx < kGT * kGT; idx += 256) {
            const int rr = idx / kGT, cc = idx % kGT;
            const int64_t row = r0 + rr;
            const int ca = ti * kGT + cc, cb = tj * kGT + cc;
            const bool ok = row < r_end;
            A[rr][cc] = (ok && ca < D) ? static_cast<double>(X[row * D + ca]) : 0.0;
            B[rr][cc] = (ok && cb < D) ? static_cast<double>(X[row * D + cb]) : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < kGT; ++rr) {
            const double va = A[rr][a];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = __builtin_fma(va, B[rr][b + e], acc[e]);
        }
        __syncthreads();
    }
    const int gi = ti * kGT + a;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int gj = tj * kGT + b + e;
        if (gi < D && gj < D) partial[(static_cast<int64_t>(chunk) * D + gi) * D + gj] = acc[e];
    }
}

__global__ __launch_bounds__(256) void colsum_partial_kernel(const float* __restrict__ X, int64_t n, int D,
                                                             int64_t rows_per_chunk,
                                                             double* __restrict__ partial) {
    const int chunk = blockIdx.y;
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= D) return;
    const int64_t r_begin = static_cast<int64_t>(chunk) * rows_per_chunk;
    const int64_t r_end = r_begin + rows_per_chunk < n ? r_begin + rows_per_chunk : n;
    double s = 0.0;
    for (int64_t r = r_begin; r < r_end; ++r) s += static_cast<double>(X[r * D + col]);
    partial[static_cast<int64_t>(chunk) * D + col] = s;
}

__global__ __launch_bounds__(256) void sum_chunks_kernel(const double* __restrict__ partial, int chunks,
                                                         int64_t len, double* __restrict__ out,
                                                         int accumulate) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += partial[static_cast<int64_t>(c) * len + i];
    out[i] = accumulate ? out[i] + s : s;
}

}  // namespace

void launch_project(const float* X, int64_t n, int D, const float* V, int d_r, void* Y, int y_dtype,
                    const float* centroids, int r, int32_t* cluster, hipStream_t s) {
    if (n == 0) return;
    const int blocks = static_cast<int>((n + kPM - 1) / kPM);
    const int col_blocks = (d_r + kPN - 1) / kPN;
    hipLaunchKernelGGL(project_kernel, dim3(blocks, col_blocks), dim3(256), 0, s, X, n, D, V, d_r, Y, y_dtype);
    PA_HIP(hipGetLastError());
    if (centroids != nullptr) {
        const int rb = static_cast<int>((n + 3) / 4);
        hipLaunchKernelGGL(route_kernel, dim3(rb), dim3(256), 0, s, static_cast<const float*>(Y), n, d_r,
                           centroids, r, cluster);
        PA_HIP(hipGetLastError());
    }
}

void launch_gram_f64(const float* X, int64_t n, int D, double* G, double* colsum, bool accumulate,
                     hipStream_t s) {
    int chunks = static_cast<int>((n + 4095) / 4096);
    if (chunks > 64) chunks = 64;
    if (chunks < 1) chunks = 1;
    const int64_t rows_per_chunk = (n + chunks - 1) / chunks;
    const int64_t dd = static_cast<int64_t>(D) * D;
    double* part = nullptr;
    PA_HIP(hipMallocAsync(reinterpret_cast<void**>(&part),
                          sizeof(double) * (static_cast<size_t>(chunks) * dd + static_cast<size_t>(chunks) * D), s));
    double* part_cs = part + static_cast<int64_t>(chunks) * dd;
    const int tiles = (D + kGT - 1) / kGT;
    hipLaunchKernelGGL(gram_partial_kernel, dim3(tiles, tiles, chunks), dim3(256), 0, s, X, n, D,
                       rows_per_chunk, part);
    PA_HIP(hipGetLastError());
    hipLaunchKernelGGL(colsum_partial_kernel, dim3((D + 255) / 256, chunks), dim3(256), 0, s, X, n, D,
                       rows_per_chunk, part_cs);
    PA_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(static_cast<int>((dd + 255) / 256)), dim3(256), 0, s, part,
                       chunks, dd, G, accumulate ? 1 : 0);
    PA_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_chunks_kernel, dim3((D + 255) / 256), dim3(256), 0, s, part_cs, chunks,
                       static_cast<int64_t>(D), colsum, accumulate ? 1 : 0);
    PA_HIP(hipGetLastError());
    PA_HIP(hipFreeAsync(part, s));
}

}  // namespace pa
