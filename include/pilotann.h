/*
 * pilotann.h - C ABI of the PilotANN GPU-stage library for AMD Instinct MI355X (gfx950).
 *
 * PilotANN (multi-stage graph ANNS) splits a top-k query into
 *   stage 1  GPU piloting: greedy search (Algorithm 1) on a sampled subgraph with
 *            SVD-reduced vectors, started from fast-entry-selection (FES) entries;
 *   stage 2  residual refinement on the host: full distances of the GPU candidates,
 *            re-rank, two traversal steps on the subgraph, a visited table;
 *   stage 3  final traversal on the host: Algorithm 1 on the full graph with full
 *            vectors from the stage-2 candidates and visited table.
 * Section numbers below refer to the paper (4.1 multi-stage processing, 4.3
 * methodology details, 5 fast entry selection, Algorithm 1, Algorithm 2, Table 2).
 *
 * Conventions shared by every call
 *   - Every call returns a pa_status: PA_OK (0) or a negative code.  On failure
 *     pa_last_error() returns a message for the calling thread; no C++ exception
 *     crosses this boundary and outputs are left unspecified.
 *   - "_dev" pointers are device (HBM) pointers on the current HIP device;
 *     "_host" pointers are host pointers.  The library never guesses the memory
 *     space of a pointer.
 *   - stream arguments are hipStream_t passed as void*; NULL is the null stream.
 *     Device calls are asynchronous on that stream unless stated otherwise;
 *     arguments are validated on the host before anything is enqueued.
 *   - Matrices are row-major and dense: element (i, j) of an [n][d] matrix is at
 *     i*d + j.  Node ids are int32 in [0, N), N < 2^31; -1 marks an empty slot.
 *   - Distances: squared Euclidean for PA_METRIC_L2, -<q, x> for PA_METRIC_IP;
 *     smaller is better and ranks order by the key (distance, id).
 *   - Buffers passed in are borrowed for the duration of the call (or of the
 *     stream work the call enqueues); outputs are caller-owned unless stated.
 */
#ifndef PILOTANN_H
#define PILOTANN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pa_status;

#define PA_OK 0
#define PA_EINVAL (-1)       /* bad argument (shape, range, null pointer, layout) */
#define PA_ESTATE (-2)       /* call out of order (e.g. search before build)      */
#define PA_ENOMEM (-3)       /* host allocation failed                            */
#define PA_EHBM (-4)         /* device allocation failed or over the HBM budget   */
#define PA_EHIP (-5)         /* HIP runtime error (message has hipGetErrorString) */
#define PA_ENONFINITE (-6)   /* NaN or Inf in an input that must be finite        */
#define PA_EUNSUPPORTED (-7) /* valid request the build does not support          */
#define PA_EINTERNAL (-8)    /* internal invariant violated                       */
#define PA_EIO (-9)          /* file cannot be read or written, or is corrupt     */

#define PA_METRIC_L2 0
#define PA_METRIC_IP 1

#define PA_F32 0  /* float32 */
#define PA_F16 1  /* IEEE binary16, round-to-nearest-even from float32 */
#define PA_BF16 2 /* bfloat16, round-to-nearest-even from float32 */
#define PA_FP8E4M3 3 /* OCP FP8 e4m3 with a float32 scale per row (entry pivots only) */

#define PA_SAMPLE_UNIFORM 0
#define PA_SAMPLE_SEED_EXPAND 1

#define PA_VISITED_EXACT 0 /* stage-1 visited set: exact (bounded LDS cache that only forgets) */
#define PA_VISITED_BLOOM 1 /* stage-1 visited set: the paper's lossy Bloom filter in LDS       */
#define PA_ENTRIES_FES 0   /* entry points: fast entry selection (section 5)                 */
#define PA_ENTRIES_FIXED 1 /* entry points: predefined nodes, the same for every query      */

#define PA_MAX_EF 512    /* largest candidate-list size of the GPU traversal */
#define PA_MAX_DEGREE 64 /* largest subgraph out-degree                       */
#define PA_MAX_DR 256    /* largest reduced dimension                         */

/* ------------------------------------------------------------------ misc */

/* Message of the last failed call on this thread ("" if none).  Owned by the library. */
const char* pa_last_error(void);

/* ABI version; bumped whenever a declaration below changes. */
int32_t pa_abi_version(void);

/* Make `device` current for the calling thread and initialise the library on it.
 * PA_EHIP if the device does not exist or is not gfx950 (PA_EUNSUPPORTED). */
pa_status pa_device_init(int32_t device);

/* ------------------------------------------------- projection (section 4.1) */

/* FP64 second-moment accumulation for the SVD projection (section 4.1: X = U S V^T,
 * V^T V = I).  G_dev [D][D] (fp64) += X^T X and colsum_dev [D] (fp64) += sum of rows,
 * over the n rows of X_dev [n][D] (fp32).  With accumulate = 0 both outputs are
 * overwritten instead, so a large X can be streamed in chunks.  The summation order is
 * fixed (deterministic).  D <= 1024. */
pa_status pa_gram_f64(const float* X_dev, int64_t n, int32_t D, double* G_dev,
                      double* colsum_dev, int32_t accumulate, void* stream);

/* Symmetric eigendecomposition in FP64 on the host (cyclic Jacobi).  A_host [D][D]
 * symmetric (only read); evals_host [D] descending; evecs_host [D][D] with column j the
 * eigenvector of evals[j], each column signed so that its entry of largest magnitude is
 * positive (ties up to rounding: the lowest row).  Blocking.  D <= 1024. */
pa_status pa_eigh_f64(const double* A_host, int32_t D, double* evals_host, double* evecs_host);

/* Fit the projection (section 4.1): streams X_host [N][D] (fp32, pageable or pinned)
 * through the GPU in chunks, accumulates the FP64 second moment, centres it when
 * center != 0 (covariance about the mean; used for L2) and keeps the d_r leading
 * eigenvectors.  Outputs (host, caller-owned): V_host [D][d_r] fp32 (x_r = x^T V),
 * evals_host [D] fp64 descending (of the possibly centred moment divided by N),
 * mean_host [D] fp64.  Blocking.  PA_ENONFINITE if X holds NaN/Inf. */
pa_status pa_fit_projection(const float* X_host, int64_t N, int32_t D, int32_t d_r,
                            int32_t center, float* V_host, double* evals_host,
                            double* mean_host);

/* Y_dev [n][d_r] = X_dev [n][D] * V_dev [D][d_r]: the reduced vectors x_primary of section
 * 4.1.  Each fp32 output is the exact product rounded once to fp32 (the exact fp32
 * products accumulated in fp64; it can differ by one ulp only where the exact value lies
 * within D 2^-53 of sum |x_k v_k| of a rounding midpoint), independent of n and of the other rows;
 * PA_F16 / PA_BF16 outputs are that fp32 value rounded to nearest even.
 * d_r % 16 == 0, d_r <= PA_MAX_DR, D <= 4096. */
pa_status pa_project(const float* X_dev, int64_t n, int32_t D, const float* V_dev,
                     int32_t d_r, void* Y_dev, int32_t y_dtype, void* stream);

/* Query projection fused with FES routing (section 5: a query is routed to the cluster
 * whose centroid is nearest).  Qr_dev [m][d_r] fp32 = Q_dev [m][D] * V_dev, rounded as in
 * pa_project; cluster_dev
 * [m] int32 = argmin_c ||q_r - centroid_c||^2 over centroids_dev [r][d_r] (fp32), ties
 * to the lowest c.  1 <= r <= 64. */
pa_status pa_project_route(const float* Q_dev, int64_t m, int32_t D, const float* V_dev,
                           int32_t d_r, const float* centroids_dev, int32_t r, float* Qr_dev,
                           int32_t* cluster_dev, void* stream);

/* ---------------------------------------- sampling and subgraph (sections 4.1, 4.3) */

/* Node sampling (section 4.1): seeds taken in the given order (order_host: a permutation
 * of [0, N), int64); PA_SAMPLE_SEED_EXPAND adds each new seed and then its
 * out-neighbours in stored order, PA_SAMPLE_UNIFORM takes the first n_target seeds.
 * Stops exactly at n_target nodes.  Full graph as CSR (rowptr_host [N+1] int64,
 * nbrs_host int32).  mask_host [N] uint8 receives 1 for sampled nodes.  Host only. */
pa_status pa_sample_nodes(int64_t N, const int64_t* rowptr_host, const int32_t* nbrs_host,
                          const int64_t* order_host, int64_t n_target, int32_t mode,
                          uint8_t* mask_host);

/* Validate a reconnected subgraph (section 4.3 layout): CSR over all N rows; rows of
 * unsampled nodes (mask_host[v] == 0) are empty, no edge enters an unsampled node, no
 * self loops, no duplicate neighbours, out-degree <= R, ids in range.  PA_OK if valid,
 * PA_EINVAL naming the first violation otherwise.  Host only. */
pa_status pa_check_subgraph(int64_t N, const int64_t* rowptr_host, const int32_t* nbrs_host,
                            const uint8_t* mask_host, int32_t R);

/* Pack a CSR graph into the device traversal layout: adj_dev [N][R] int32, row v holds
 * v's out-neighbours in stored order followed by -1 padding.  Node ids are unchanged
 * (zero-degree rows stay, section 4.3).  PA_EINVAL if a row exceeds R or an id is out of
 * range.  Blocking (the host staging copy is released on return). */
pa_status pa_pack_adjacency(int64_t N, const int64_t* rowptr_host, const int32_t* nbrs_host,
                            int32_t R, int32_t* adj_dev, void* stream);

/* -------------------------------------------- fast entry selection (section 5) */

/* Coarse clustering of the entry vectors (section 5: r equal buckets, the layout
 * EV[r][n/r][d] of Algorithm 2), FP64 on the host: Lloyd iterations in squared L2 from
 * the seeds init_host [r] (distinct positions in [0, n_p)), then a balanced assignment
 * in the order of (distance, pivot position, cluster) that fills every bucket with exactly
 * n_p / r pivots, then centroids = bucket means.  P_host [n_p][d] fp32 (pivot reduced
 * vectors).  Outputs: buckets_host [r][n_p/r] int32 pivot positions (ascending within a
 * bucket), centroids_host [r][d] fp32.  n_p % r == 0.  Blocking, deterministic. */
pa_status pa_build_entries(const float* P_host, int32_t n_p, int32_t d, int32_t r,
                           const int32_t* init_host, int32_t iters, int32_t* buckets_host,
                           float* centroids_host);

/* FES scoring and top-E (Algorithm 2 with a fused top-E): every query i is scored only
 * against the n_b pivots of its cluster cluster_dev[i] (from pa_project_route), on MFMA in
 * the expanded form ||q||^2 + ||p||^2 - 2 q.p (L2) or -q.p (IP), fp32, together with a
 * rigorous bound on each score's rounding error.  Only pivots whose error interval can
 * still reach the E-th smallest upper bound are kept, and those are re-scored exactly, so
 * the result is the exact top E: ids_dev [m][E] int32 and d_dev [m][E] fp32, the
 * correctly rounded distance (squared L2 or -IP, direct form), ordered by (distance,
 * id), padded with (-1, +inf) when E > n_b.  EV_dev [r][n_b][d] fp32 bucket-major pivot
 * vectors, EVnorm_dev [r][n_b] fp32 squared norms, EVid_dev [r][n_b] int32 node ids.
 * d % 16 == 0.  Buckets are scanned in chunks of 128 pivots per 16-query tile.
 * PA_EUNSUPPORTED if a 16-query tile's candidate list (E + 192 entries) does not fit the
 * device's LDS.  Results of a query do not depend on the other queries of the batch. */
pa_status pa_select_entries(const float* Qr_dev, const int32_t* cluster_dev, int64_t m,
                            int32_t d, const float* EV_dev, const float* EVnorm_dev,
                            const int32_t* EVid_dev, int32_t r, int32_t n_b, int32_t E,
                            int32_t metric, int32_t* ids_dev, float* d_dev, void* stream);

/* Allocation-free variant of pa_select_entries, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, layouts and results as pa_select_entries (the same kernels
 * run); the scratch that pa_select_entries allocates per call (3 r + 2 + m int32: the
 * grouping header and the query permutation) lives instead in a static device array of
 * 3 * 64 + 2 + 262,144 int32 (about 1 MiB) per GPU, held until the process ends; the
 * kernels write every scratch word they read before reading it, so nothing needs
 * clearing.  m > 262,144 -> PA_EINVAL.  The call makes no device allocation and frees
 * nothing.  Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (different streams or host threads without ordering) race and must be serialised by
 * the caller.  pa_device_init looks the array's device address up; otherwise the first
 * call on a device does, with that device current. */
pa_status pa_select_entries_noalloc(const float* Qr_dev, const int32_t* cluster_dev, int64_t m,
                                    int32_t d, const float* EV_dev, const float* EVnorm_dev,
                                    const int32_t* EVid_dev, int32_t r, int32_t n_b, int32_t E,
                                    int32_t metric, int32_t* ids_dev, float* d_dev, void* stream);

/* FP8 encoding of the entry pivots (the precision form of fast entry selection): for every
 * row of X_host [n][d] fp32, scales_host[i] = max_j |x_ij| / 448 (1 for an all-zero row) and
 * codes_host[i][j] = e4m3(x_ij / scales_host[i]) with round-to-nearest-even (OCP e4m3,
 * bit-equal to torch.float8_e4m3fn on this range).  Host only. */
pa_status pa_quantize_fp8_rows(const float* X_host, int64_t n, int32_t d, uint8_t* codes_host,
                               float* scales_host);

/* FES in the precision form: as pa_select_entries, but each tile is scored with FP8 MFMA
 * (v_mfma_f32_16x16x32_fp8_fp8, fp32 accumulation) on the pivots' e4m3 codes EV8_dev
 * [r][n_b][d] uint8 with row scales EVscale_dev [r][n_b] fp32 (pa_quantize_fp8_rows) and the
 * queries encoded the same way on the fly; the K best pivots of that approximate score
 * (ties by position in the bucket; E <= K) are re-scored exactly from EV_dev (direct form:
 * ||q - p||^2 or -q.p, correctly rounded fp32) and the best E by (distance, id) are
 * returned.  d % 32 == 0.  PA_EUNSUPPORTED if the K-list of a 16-query tile (K + 128
 * entries) does not fit the device's LDS. */
pa_status pa_select_entries_fp8(const float* Qr_dev, const int32_t* cluster_dev, int64_t m, int32_t d,
                                const float* EV_dev, const uint8_t* EV8_dev, const float* EVscale_dev,
                                const float* EVnorm_dev, const int32_t* EVid_dev, int32_t r, int32_t n_b,
                                int32_t E, int32_t K, int32_t metric, int32_t* ids_dev, float* d_dev,
                                void* stream);

/* ----------------------------------------------- stage 1: GPU piloting (4.1, Alg. 1) */

/* Options of pa_gpu_traverse (NULL: all zero = Algorithm 1 with the exact visited set, an
 * automatic cache size, one list size for every query). */
typedef struct {
    int32_t visited;       /* PA_VISITED_EXACT (Algorithm 1) or PA_VISITED_BLOOM: the
                              paper's visited filter (section 4.3), see below            */
    int32_t cache_log2;    /* exact: 2^cache_log2 LDS cache slots per query (8..13);
                              Bloom: a filter of 32 << cache_log2 bits; 0: automatic
                              (from ef: the ef_max of a per-query run)                   */
    int32_t width;         /* entries of C expanded per step: 0 or 1 (Algorithm 1), or 2
                              (the first two unchecked entries together; needs R <= 32).
                              Width 2 is not the paper's algorithm: it may expand a node
                              that Algorithm 1 would have dropped from C first           */
    const int32_t* ef_dev; /* nullable: per-query list sizes [m] int32 in [1, ef], so
                              that requests of uneven ef share one launch (the serving
                              loop): query i keeps ef_dev[i] entries and uses the first
                              min(E, ef_dev[i]) of its entries; rows keep the stride ef,
                              padded with (-1, +inf) after ef_dev[i]; with the same
                              cache_log2 a row equals a run of that query alone with
                              ef = ef_dev[i]                                               */
} pa_traverse_opts;

/* Stage 1: batched Algorithm 1 on the subgraph with reduced vectors, one 64-lane
 * wavefront per query.  Qr_dev [m][d_r] fp32 reduced queries; Xr_dev [N][d_r] reduced base
 * vectors of xr_dtype (rows 16-byte aligned: d_r*sizeof % 16 == 0, at most 1024 bytes);
 * adj_dev [N][R] (pa_pack_adjacency); entries_dev [m][E] int32 (-1 skipped; ids outside
 * [0, N) are skipped).  Outputs: ids_dev/d_dev [m][ef] - the final candidate list C in
 * (delta, id) order with the correctly rounded fp32 distances, padded with (-1, +inf);
 * counters_dev [m][4] int32 = (expansions, distance evaluations, visited-cache forget
 * events, termination-guard flag).  1 <= ef <= PA_MAX_EF, 1 <= R <= PA_MAX_DEGREE,
 * N <= 2^30.  All device pointers; asynchronous on the stream.
 *
 * Exact visited set (default): the per-query LDS cache stores full ids, so it may forget
 * a visited node (a cache reset, or an id that found no free slot: a forget event) but
 * never claims an unvisited one; a forgotten node met again is re-scored and dropped, so
 * the result equals Algorithm 1 with an exact visited set, and the distance-evaluation
 * count equals |visited| when no forget event happened (it exceeds it by the re-scores
 * otherwise).  The guard flag is 1 only if a query stopped at the N-expansion guard
 * (never expected).
 *
 * Bloom visited filter (visited = PA_VISITED_BLOOM): each query tracks visited nodes in
 * a Bloom filter in LDS with two hashes, bit_i(v) = ((uint32)v * A_i mod 2^32) >>
 * (32 - log2 bits), A_1 = 0x9E3779B1, A_2 = 0x85EBCA77.  A node whose two bits are set
 * counts as visited, also when other nodes set them (a false positive: it is never scored
 * here).  The ids of one adjacency row (and each group of 64 entries) are all tested
 * against the filter as it was before the group, then their bits are set; an id that
 * appears twice in a group is scored twice and listed once.  Counters as above with
 * counters[i][2] = 0. */
pa_status pa_gpu_traverse(const float* Qr_dev, int64_t m, int32_t d_r, const void* Xr_dev,
                          int32_t xr_dtype, int64_t N, const int32_t* adj_dev, int32_t R,
                          const int32_t* entries_dev, int32_t E, int32_t ef, int32_t metric,
                          const pa_traverse_opts* opts, int32_t* ids_dev, float* d_dev,
                          int32_t* counters_dev, void* stream);

/* ------------------------------------------- stages 2 and 3 on the host (4.1) */

/* Residual refinement (stage 2) and final traversal (stage 3) for m queries, on host
 * threads.  X_host [N][D] fp32 full vectors; sub_adj_host [N][R_sub] and full_adj_host
 * [N][R_full] int32 padded rows (-1); Q_host [m][D] fp32; beam_host [m][n_beam] int32
 * stage-1 candidate ids (-1 skipped).  Stage 2 scores the beam with full distances, keeps
 * the best ef_cpu, runs refine_steps Algorithm-1 steps on the subgraph and passes its
 * candidates (all unchecked) and visited set to stage 3, which runs Algorithm 1 on the
 * full graph with list size max(ef_cpu, k).  With refine_steps < 0 stage 2 is skipped
 * (the beam is re-scored and handed on directly).  Outputs out_ids_host [m][k] int64,
 * out_d_host [m][k] fp32 padded with (-1, +inf); counters_host [m][4] int32 (nullable)
 * = (stage-2 distances, stage-3 distances, stage-3 expansions, 0).  threads <= 0 uses
 * every host core.  Blocking. */
pa_status pa_cpu_stages(const float* X_host, int64_t N, int32_t D, const int32_t* sub_adj_host,
                        int32_t R_sub, const int32_t* full_adj_host, int32_t R_full,
                        const float* Q_host, int64_t m, const int32_t* beam_host,
                        int32_t n_beam, int32_t ef_cpu, int32_t k, int32_t refine_steps,
                        int32_t metric, int32_t threads, int64_t* out_ids_host,
                        float* out_d_host, int32_t* counters_host);

/* Plain Algorithm 1 on the full graph from given entries (the graceful-degradation mode
 * of section 4.1: stage 3 alone).  entries_host [m][E] int32.  Outputs as
 * pa_cpu_stages; counters = (0, distances, expansions, 0).  Blocking. */
pa_status pa_cpu_search(const float* X_host, int64_t N, int32_t D, const int32_t* full_adj_host,
                        int32_t R_full, const float* Q_host, int64_t m,
                        const int32_t* entries_host, int32_t E, int32_t ef, int32_t k,
                        int32_t metric, int32_t threads, int64_t* out_ids_host,
                        float* out_d_host, int32_t* counters_host);

/* ------------------------------------------------------ index and pipeline */

typedef struct pa_index pa_index;

typedef struct {
    int32_t dim;          /* D: full dimension                                   */
    int32_t d_r;          /* reduced dimension (multiple of 16)                  */
    int32_t metric;       /* PA_METRIC_L2 / PA_METRIC_IP                         */
    int32_t xr_dtype;     /* storage type of the reduced base vectors            */
    int32_t r;            /* FES clusters (the paper uses 32)                    */
    int32_t refine_steps; /* stage-2 traversal steps (the paper uses 2)          */
    int32_t threads;      /* host threads for stages 2-3 (<= 0: all cores)       */
    int32_t device;       /* HIP device ordinal                                  */
    int64_t hbm_budget;   /* bytes of HBM the index and search buffers may use (0 = no limit) */
    int32_t pivot_dtype;  /* PA_F32 or PA_FP8E4M3 (precision form of entry selection)   */
    int32_t preselect;    /* FP8 form: pivots re-scored in fp32 per query = preselect*E
                             (0: 4), capped by the bucket size and by 1,024 (at least E) */
    int32_t compact;      /* 1: HBM holds X_r and the subgraph for the sampled nodes
                             only (memory-bounded layout, section 4.3 drops the
                             unsampled nodes' vectors; see pa_index_build_subgraph);
                             0: X_r for all N rows                                     */
} pa_params;

/* Create an empty index.  params is copied.  *out receives the handle (library-owned;
 * release with pa_index_destroy). */
pa_status pa_index_create(const pa_params* params, pa_index** out);
pa_status pa_index_destroy(pa_index* idx);

/* Attach the full data (section 3: the full index stays in host RAM).  X_host [N][D] fp32
 * is BORROWED until destroy (stages 2-3 read it); the full graph CSR is copied into a
 * padded host table [N][max degree] (max degree <= 1024). */
pa_status pa_index_set_data(pa_index* idx, const float* X_host, int64_t N,
                            const int64_t* rowptr_host, const int32_t* nbrs_host);

/* Fit the projection on the attached X (pa_fit_projection) and write the reduced base
 * vectors of all N rows to HBM in xr_dtype (compact layout: of the sampled rows, once
 * the subgraph is built).  center: 1 centred, 0 uncentred, -1 the metric's default
 * (centred for L2, uncentred for IP). */
pa_status pa_index_fit_projection(pa_index* idx, int32_t center);

/* Use a caller-supplied projection V_host [D][d_r] fp32 instead of fitting one. */
pa_status pa_index_set_projection(pa_index* idx, const float* V_host);

/* Sampling on the attached full graph (pa_sample_nodes). */
pa_status pa_index_sample_nodes(pa_index* idx, const int64_t* order_host, int64_t n_target,
                                int32_t mode, uint8_t* mask_host);

/* build_subgraph: validate (pa_check_subgraph against mask_host) and upload the
 * reconnected subgraph; a host copy is kept for stage 2.  Compact layout: the n_s
 * sampled nodes get device ids 0..n_s-1 in increasing node-id order (so ties between
 * equal distances break the same way), X_r and the adjacency are stored for them only
 * (n_s rows instead of N, ids rewritten), and stage 1 maps its output back to node
 * ids; results equal the full layout's (with the Bloom filter the hashes see the
 * device ids, so its false positives differ).  The reduced rows are (re)written here. */
pa_status pa_index_build_subgraph(pa_index* idx, const uint8_t* mask_host,
                                  const int64_t* rowptr_host, const int32_t* nbrs_host);

/* build_entries: cluster the pivots pivot_ids_host [n_p] (node ids, each with out-edges in
 * the subgraph) on their reduced vectors as stored in HBM (pa_build_entries), and upload
 * the bucket-major entry table.  init_host [r] seeds, iters Lloyd iterations. */
pa_status pa_index_build_entries(pa_index* idx, const int32_t* pivot_ids_host, int32_t n_p,
                                 const int32_t* init_host, int32_t iters);

/* Copy out index state for inspection: V_host [D][d_r]; buckets_host [r][n_p/r] node ids;
 * centroids_host [r][d_r]; any pointer may be NULL. */
pa_status pa_index_get_state(const pa_index* idx, float* V_host, int32_t* buckets_host,
                             float* centroids_host);

/* Checkpoint of the built index (the state sections 4.1 and 5 build offline: the
 * projection V, the reduced vectors X_r as stored, the packed subgraph, and the entry
 * table with its centroids and bucket ids).  The caller-owned inputs (X and the full
 * graph) are not written: they are the data, not the index.
 *
 * pa_index_save writes `path` (created or truncated): a fixed header (magic, format
 * version, dim, d_r, metric, X_r dtype, r, pivot dtype, N, subgraph degree, pivots per
 * bucket) and its FNV-1a 64-bit checksum, then sections, each with its byte length and
 * checksum.  Host byte order.
 * PA_ESTATE unless projection, subgraph and entries are built; PA_EIO on a write error.
 *
 * pa_index_load reads such a file into an index created with the same parameters (dim,
 * d_r, metric, xr_dtype, r, pivot_dtype) after pa_index_set_data with the same N; it
 * replaces any projection, subgraph and entries the index held and leaves it ready to
 * search.  PA_EIO if the file cannot be read, is truncated or fails a checksum (or
 * holds an id out of range); PA_EINVAL if its header disagrees with the index;
 * PA_ESTATE before set_data.  The file is read and verified completely before the index
 * is touched, so these failures leave the index unchanged; a device allocation or copy
 * failure after that (PA_EHBM, PA_EHIP) leaves it with no projection, subgraph or
 * entries. */
pa_status pa_index_save(const pa_index* idx, const char* path);
pa_status pa_index_load(pa_index* idx, const char* path);

/* Sizes and build state of an index. */
typedef struct {
    int64_t N;           /* nodes (0 before set_data)                           */
    int32_t R_full;      /* padded full-graph degree                            */
    int32_t R_sub;       /* padded subgraph degree (0 before the subgraph)      */
    int32_t n_pivots;    /* entry pivots, r buckets of n_pivots / r (0 before)  */
    int32_t built;       /* bit 0 data, bit 1 projection, bit 2 subgraph, bit 3 entries */
    int64_t hbm_bytes;   /* device bytes the index holds, work buffers included */
    int64_t xr_rows;     /* rows of X_r and of the device subgraph (N, or n_s when
                            compact; 0 before they are written)                  */
} pa_index_info;

pa_status pa_index_get_info(const pa_index* idx, pa_index_info* out);

/* ----------------------------------------------------- memory-bounded mode */

/* The HBM an index and its searches hold, as a function of the sampling ratio and the
 * reduced width: the paper fits the subgraph and the reduced vectors to the GPU's memory
 * (section 6.2, minimum GPU memory study; the sampling and SVD ratios of Table 3). */
typedef struct {
    int64_t N;            /* base vectors                                               */
    int32_t dim;          /* D                                                          */
    int32_t xr_dtype;     /* PA_F32 / PA_F16 / PA_BF16                                  */
    int32_t pivot_dtype;  /* PA_F32 / PA_FP8E4M3                                        */
    int32_t compact;      /* layout, as pa_params.compact                               */
    int32_t R_sub;        /* padded subgraph degree (1..1024)                           */
    int32_t n_pivots;     /* FES pivots, a multiple of r                                */
    int32_t r;            /* FES buckets                                                */
    int64_t queries;      /* queries of the largest pa_search call (0: none yet)        */
    int32_t batch;        /* pa_search_opts.batch (0: 16,384)                           */
    int32_t ef_gpu;       /* pa_search_opts.ef_gpu (1..PA_MAX_EF)                       */
    int32_t E;            /* pa_search_opts.E (0: min(ef_gpu, n_pivots / r))            */
    int32_t q_on_device;  /* 1: the searches pass their queries as q_dev                */
} pa_memory_shape;

/* Device bytes that an index of this shape holds once built with n_s = round(rho * N)
 * sampled nodes and reduced width d_r and after searches of up to `queries` queries: the
 * value pa_index_get_info then reports as hbm_bytes.  With s = 4, 2, 2 bytes per element
 * for F32, F16, BF16, n = n_s in the compact layout and N otherwise, m = queries and B =
 * min(m, batch) (the largest sub-batch), it is the sum of
 *   4*D*d_r                                       projection
 *   max(16, n*d_r*s) + 4*max(n, 1)*R_sub           X_r and the device subgraph
 *   4*max(n_s, 1)                                 device-to-node ids (compact layout)
 *   4*n_p*(d_r + 2) + 4*r*d_r                     pivot rows, norms and ids; centroids
 *   n_p*(d_r + 4)                                 FP8 pivot codes and scales (FP8 form)
 *   m*(4*D + 4*d_r + 4 + 8*E + 8*ef_gpu + 16) + 4*(3*r + 2 + B)   search buffers (m > 0;
 *                                                 the 4*D term only without q_on_device)
 * Returns -1 for an invalid shape, rho outside (0, 1], or d_r outside 16..min(D,
 * PA_MAX_DR) or not a multiple of 16. */
int64_t pa_hbm_bytes(const pa_memory_shape* shape, double rho, int32_t d_r);

/* Memory-bounded mode: from the candidate ratios rhos[n_rho] and widths d_rs[n_dr],
 * choose the pair whose pa_hbm_bytes fits hbm_budget with the largest rho (a larger
 * sample holds more of each query's answers for stage 1), and at that rho the largest
 * d_r.  Writes the pair and its bytes (any output may be NULL).  PA_EHBM when no pair
 * fits; PA_EINVAL for an invalid shape or candidate, or an empty candidate list.  An
 * index built with the chosen pair (and hbm_budget as pa_params.hbm_budget) and searched
 * as the shape describes holds exactly the predicted bytes. */
pa_status pa_plan_memory(const pa_memory_shape* shape, int64_t hbm_budget, const double* rhos, int32_t n_rho,
                         const int32_t* d_rs, int32_t n_dr, double* rho_out, int32_t* d_r_out,
                         int64_t* bytes_out);

/* Device pointers of the index's tables (for stage-isolated calls); any may be NULL.
 * In the compact layout X_r, the adjacency and EVid hold device ids (see
 * pa_index_build_subgraph). */
pa_status pa_index_device_tables(const pa_index* idx, const void** Xr_dev,
                                 const int32_t** adj_dev, const float** V_dev,
                                 const float** centroids_dev, const float** EV_dev,
                                 const float** EVnorm_dev, const int32_t** EVid_dev);

typedef struct {
    int32_t ef_gpu;       /* stage-1 list size (1..PA_MAX_EF)                     */
    int32_t ef_cpu;       /* stage-2/3 list size                                   */
    int32_t E;            /* entries per query (0: min(ef_gpu, n_p / r))           */
    int32_t batch;        /* queries per pipelined sub-batch (0: 16,384)           */
    int32_t stage_mask;   /* bit 0 GPU stage, bit 1 refinement (0: both); bit 2 set
                             skips the final traversal (needs the GPU stage): the
                             output is the best k of the stage-2 list, so with a
                             subgraph of every node and d_r = D the GPU alone finds
                             the candidates (the paper's GPU-only special case)    */
    int32_t cache_log2;   /* GPU visited-cache size (0: automatic)                 */
    int32_t threads;      /* host threads (0: index default)                       */
    int32_t handoff;      /* stage-1 candidates handed to stage 2 per query, the
                             best by reduced distance (0: all ef_gpu)               */
    const float* q_dev;   /* nullable: device copy of Q_host [m][D] fp32, already
                             resident in HBM and complete (its writes finished);
                             the GPU stage then reads the queries from it and skips
                             their upload.  Q_host is still read by stages 2-3.  */
    int32_t visited;      /* stage-1 visited set: PA_VISITED_EXACT (0) or
                             PA_VISITED_BLOOM (cache_log2 then sizes the filter:
                             32 << cache_log2 bits)                                 */
    int32_t width;        /* stage-1 expansion width (0 or 1: Algorithm 1; 2: see
                             pa_traverse_opts)                                       */
    int32_t entries;      /* PA_ENTRIES_FES (0), or PA_ENTRIES_FIXED: no entry
                             selection; every query starts from the same E pivots,
                             taken one per bucket in turn (pivot j of bucket c for
                             entry e = j * r + c), the "predefined nodes" start of
                             section 5 (the ablation of Table 5)                      */
    int32_t serial;       /* 0: the host stages of sub-batch b overlap the GPU stage
                             of the later ones (pipelining, section 4.1); 1: the host
                             stages start after the GPU stage of every sub-batch
                             (the ablation of Table 5)                               */
} pa_search_opts;

typedef struct {
    double wall_ms;          /* whole call                                          */
    double beam_ms;          /* sum of stage-1 kernel durations (HIP events)        */
    double fes_ms;           /* projection + routing + FES kernels (HIP events)     */
    int64_t beam_launches;   /* stage-1 kernel launches                             */
    int64_t n_exp1;          /* stage-1 expansions, summed over queries             */
    int64_t n_dist1;         /* stage-1 distance evaluations                        */
    int64_t n_dist2;         /* stage-2 distance evaluations                        */
    int64_t n_dist3;         /* stage-3 distance evaluations                        */
    int64_t n_exp3;          /* stage-3 expansions                                  */
    int64_t n_reset1;        /* stage-1 visited-cache resets                        */
    double host_wait_ms;     /* host time spent waiting for GPU batches             */
} pa_search_stats;

/* Full search (section 4.1 stages 1-3 with FES): Q_host [m][D] fp32 (pageable or
 * pinned) -> out_ids_host [m][k] int64, out_d_host [m][k] fp32 (full squared L2 or
 * -IP), padded with (-1, +inf).  Queries are split into sub-batches; stage 1 of batch b+1
 * runs on the GPU while the host threads run stages 2-3 of batch b (section 4.2
 * pipelining).  Blocking.  counters_host [m][8] int32 (nullable) = (n_exp1, n_dist1,
 * reset1, n_dist2, n_dist3, n_exp3, 0, 0).  stats nullable.  PA_ESTATE before the
 * projection, subgraph and entries are built. */
pa_status pa_search(pa_index* idx, const float* Q_host, int64_t m, int32_t k,
                    const pa_search_opts* opts, int64_t* out_ids_host, float* out_d_host,
                    int32_t* counters_host, pa_search_stats* stats);

/* ------------------------------------------------------------ serving loop */

/* Continuous batching over an index (the serving form of the search; the paper batches
 * and pipelines queries, section 4.2).  hbm_budget bounds the device memory of the index
 * and the server together: the index's own tables (pa_index_get_info hbm_bytes at create)
 * come first, and what remains is split into `streams` micro-batch slots, each with one
 * device arena of min((hbm_budget - index bytes) / streams, the bytes of a full micro-batch
 * at list size 512) allocated at create.  Requests of uneven k and ef are queued in arrival
 * order; when a slot is free the scheduler takes the head of the queue into its
 * micro-batch while the batch's real footprint fits the arena: for m requests whose
 * largest list size is f, with e = min(f, n_p / r), the sum of
 *   4 m dim, 4 m d_r, 4 m, 4 m e (twice), 4 m f (twice), 16 m, 4 m, 4 (3 r + 2 + m)
 * bytes, each rounded up to 256 (queries, reduced queries, clusters, entries, stage-1
 * lists, counters, list sizes, entry-selection scratch).  Projection, routing, entry
 * selection and stage 1 of a micro-batch run on its slot's stream, so several
 * micro-batches overlap on the GPU, and stage-1 lists stay in HBM until the hand-off.
 * Stages 2-3 run on host threads with ef_cpu = ef.  Each request's result is the same
 * whatever else is in flight.  The index must outlive the server and must not be rebuilt
 * while it runs; pa_search on the same index may run concurrently (its buffers are not
 * covered by the server's budget). */
typedef struct pa_server pa_server;

typedef struct {
    int64_t hbm_budget;  /* device bytes of the index plus the server's slots (> 0)     */
    int32_t max_batch;   /* requests per micro-batch (0: 1024)                          */
    int32_t streams;     /* micro-batch slots / GPU streams (0: 2)                      */
    int32_t threads;     /* host threads for stages 2-3 (0: index default)             */
    int32_t max_k;       /* largest k a request may ask; result rows have this width (0: 128) */
} pa_server_params;

typedef struct {
    uint64_t tag;        /* the caller's tag                                            */
    int32_t k, ef;       /* as submitted (ef raised to k if smaller)                     */
    double t_submit_us;  /* monotonic microseconds since pa_server_create                */
    double t_admit_us;   /* when its micro-batch was formed                              */
    double t_done_us;    /* when its result was published                                */
} pa_result_info;

/* Start the scheduler and completion threads; allocates the slots' device arenas and
 * pinned host buffers for max_batch requests up front (none later).  PA_EHBM if the budget
 * cannot hold the index and one request of list size 512 per slot. */
pa_status pa_server_create(pa_index* idx, const pa_server_params* params, pa_server** out);

/* Queue one query q_host [dim] fp32 (copied) with its k and ef.  Never blocks and never
 * rejects for lack of budget: the request waits in the queue (every request fits a slot
 * alone, as create checked).  PA_EINVAL for k or ef out of range, PA_ENONFINITE for a
 * non-finite query, PA_ESTATE after a failure. */
pa_status pa_server_submit(pa_server* s, const float* q_host, int32_t k, int32_t ef, uint64_t tag);

/* Non-blocking: move up to max_results finished requests out.  info [max_results];
 * ids [max_results][max_k] int64 and dists [max_results][max_k] fp32, each row padded with
 * (-1, +inf) after its k results.  *n_out receives the count.  Reports a failure of the
 * server's threads once no result is left. */
pa_status pa_server_poll(pa_server* s, int32_t max_results, pa_result_info* info, int64_t* ids,
                         float* dists, int32_t* n_out);

/* Block until every submitted request has finished (results stay available to poll). */
pa_status pa_server_drain(pa_server* s);

/* Counters (any pointer may be NULL): requests submitted and finished, micro-batches
 * formed, the largest micro-batch, device bytes currently in flight. */
pa_status pa_server_stats(const pa_server* s, int64_t* submitted, int64_t* completed, int64_t* batches,
                          int64_t* max_batch, int64_t* bytes_in_flight);

/* Drain, stop the threads and release the slots. */
pa_status pa_server_destroy(pa_server* s);

#ifdef __cplusplus
}
#endif

#endif /* PILOTANN_H */
