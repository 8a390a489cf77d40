/*
 * deg.h -- C ABI of the MI355X (gfx950) search library for the Dynamic
 * Exploration Graph (DEG) of Hezel, Barthel, Schall and Jung (PVLDB 17).
 *
 * The library searches a DEG: an undirected, even-regular graph (every vertex
 * has exactly `degree` neighbours, Sec. 5.1) over N base vectors, with the
 * range search of Algorithm 1. It also computes exact kNN ground truth
 * (Eq. knn) with matrix cores, builds reduced-precision vector stores, and
 * trains and runs a small MLP that stops a search early.
 *
 * Conventions for every call:
 *   - Pointers to arrays are DEVICE pointers owned by the caller unless the
 *     comment says "host". The library never allocates device memory on the
 *     search path; scratch memory is a caller-provided workspace sized by the
 *     matching *_workspace_bytes call.
 *   - Calls only enqueue work on `stream` (a hipStream_t; NULL = the null
 *     stream) and return. Outputs are valid after the stream is synchronised.
 *   - Host-side argument errors return a status at once and enqueue nothing.
 *     Errors the device detects (an id outside [0, N)) set a bit in the
 *     query's flags and its result row is padded.
 *   - Distances: L2 is the SQUARED Euclidean distance; IP is 1 - <x, q>.
 *   - Every ordering is by (distance, vertex id) ascending. Result rows are
 *     padded with id -1 and distance +inf when fewer than k vertices are found.
 *   - FP32 distances are reduced in one fixed order ("C32x4"): 32 partial
 *     sums, chunk c of 4 consecutive dims goes to partial c mod 32 with fused
 *     multiply-adds in increasing dim order, then a halving tree
 *     p[i] += p[i + w] for w = 16, 8, 4, 2, 1.
 */
#ifndef DEG_H
#define DEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DEG_OK = 0,
    DEG_ERR_INVALID_ARG = 1,
    DEG_ERR_UNSUPPORTED = 2,
    DEG_ERR_WORKSPACE = 3,
    DEG_ERR_HIP = 4
} deg_status;

typedef enum { DEG_METRIC_L2 = 0, DEG_METRIC_IP = 1 } deg_metric;

typedef enum { DEG_F32 = 0, DEG_BF16 = 1, DEG_FP8_E4M3 = 2 } deg_dtype;

/* Per-query flag bits written to out_stats[q*4 + 2]. */
#define DEG_FLAG_QUEUE_OVERFLOW 1 /* a live candidate was dropped because S was full */
#define DEG_FLAG_HASH_SPILL 2     /* the visited set moved from LDS to the workspace */
#define DEG_FLAG_HASH_FULL 4      /* never set: the workspace visited tables grow until they hold
                                     all n vertices below 3/4 load (kept for the bit layout) */
#define DEG_FLAG_BAD_ID 8         /* a seed, query vertex or adjacency id was outside [0, N) */
#define DEG_FLAG_LEARNED_STOP 16  /* the stop predictor ended the search */

/*
 * Base vectors. `data` holds n rows of `row_stride` elements of `dtype`
 * (row_stride >= dim). BF16 rows are the upper halves of FP32 values (round
 * to nearest even). FP8 rows are OCP E4M3 codes with one FP32 scale per row
 * (value = scale[i] * e4m3(code)). `f32_data` holds the FP32 rows
 * (f32_stride elements each); it is read for the exact rerank and for the
 * query vector of an exploratory search, and may equal `data` for DEG_F32.
 */
typedef struct {
    const void *data;
    int64_t n;
    int32_t dim;
    int32_t row_stride;
    int32_t dtype;
    int32_t metric;
    const float *scale;
    const float *f32_data;
    int32_t f32_stride;
    int32_t reserved;
} deg_vectors;

/*
 * The graph: n rows of `row_stride` int32 neighbour ids, the first `degree`
 * of which are the vertex's neighbours (Sec. 5.4: search reads ids only, no
 * edge weights). degree must be even and >= 4 (Sec. 5.1) and <= 128 (a row of
 * more than 64 neighbours is expanded in two parts of up to 64; such graphs take
 * pools of up to 256, up to 512 dims and no learned stop or trace rows, else
 * DEG_ERR_UNSUPPORTED).
 */
typedef struct {
    const int32_t *adj;
    int64_t n;
    int32_t degree;
    int32_t row_stride;
} deg_graph;

/*
 * Learned early stop: a 16-64-64-1 MLP (ReLU, sigmoid) in BF16 as written by
 * deg_mlp_export_bf16 (5313 values: W1[64][16], b1[64], W2[64][64], b2[64],
 * w3[64], b3). Inference is one fixed FP32 computation: x = bf16(features);
 * h1_j = bf16(relu(b1_j + W1_j0 x_0 + ... + W1_j15 x_15)) and h2_j = relu(b2_j +
 * W2_j0 h1_0 + ... + W2_j63 h1_63), each a chain of fused multiply-adds in
 * increasing index; logit = (halving tree over w3_j * h2_j, w = 32..1) + b3.
 * At the hops h = interval, 2 interval, ... (after the pop passed the test of
 * Algorithm 1, before the row is expanded) the search forms 16 features from
 * its state, with kq = min(k, |R|) and d1, dk the distances of R's first and
 * kq-th entries (FP32, correctly rounded division and square root; a ratio
 * with a zero or non-finite divisor is 1):
 *   0 sqrt(h)  1 sqrt(evaluations)  2 d1/dk  3 d1/(smallest seed distance)
 *   4 r/(r at the previous checkpoint)  5 sqrt(hops since the first min(pool, 10)
 *   results changed)  6 sqrt(hops since the first result changed)  7 (new
 *   candidates of the last expanded row within the end-of-row range)/degree
 *   8 (new candidates of the last row in R after it)/degree  9 min(64, entries
 *   of S before the kq-th result)/64  10 min(4, popped distance/dk)
 *   11 min(eps, 4)  12 sqrt(k)  13 1 if exploratory  14 sqrt(hops since r
 *   changed)  15 1.
 * Features are standardised as (f - mean) * inv_std in FP32; if the logit is
 * >= log(tau / (1 - tau)) the search stops (from hop `long_hops` on, when
 * long_hops > 0, with tau_long instead: long queries set the makespan of a
 * batch). The plain rule of Algorithm 1 still applies.
 */
typedef struct {
    const uint16_t *weights_bf16; /* device */
    const float *feat_mean;       /* device, 16: features are standardised */
    const float *feat_inv_std;    /* device, 16 */
    float tau;
    int32_t interval;
    float tau_long;               /* threshold from hop long_hops on */
    int32_t long_hops;            /* 0 = tau throughout */
} deg_stop_model;

/* Search options. Zero-initialised means: defaults. */
typedef struct {
    int32_t queue_cap;  /* capacity L of the candidate set S (Algorithm 1's S is unbounded):
                           the same as evicting the (distance, id)-largest entry at every
                           push into a full S. DEG_FLAG_QUEUE_OVERFLOW marks a query that
                           lost an entry within r(1+eps) (without it the result is Algorithm
                           1's exactly); 0 = default 16384, at most 2^24 (the workspace
                           holds L + 256 keys per resident wave) */
    int32_t hash_slots; /* LDS visited-table slots (power of 2, 256..16384); 0 = the tuned
                           value if one is registered, else 512. At 3/4 load the set moves
                           to a workspace table, and from there to one four times larger
                           at each 3/8 load (the last, shared, holds all n vertices
                           below 3/4 load). */
    int32_t k_pool;     /* traversal result size (>= k); the pool is reranked in FP32
                           from f32_data when k_pool > k or dtype != DEG_F32; 0 = k */
    int32_t rerank;     /* 1 = always rerank the pool in FP32, 0 = only when needed */
    const deg_stop_model *stop; /* host pointer to the model descriptor, NULL = plain rule */
    float *trace;       /* device; non-NULL = write stop-predictor training rows */
    int64_t trace_rows_per_query; /* rows per query in `trace` (each 20 floats) */
    int32_t trace_interval;       /* hops between two trace rows */
    int32_t waves_per_cu;         /* resident waves per CU of the persistent grid; 0 = tuned */
    int32_t queue_lds;  /* keys of S held in LDS beyond the 64 in registers (multiple of 64,
                           256..8192; 0 = 512); the farthest keys live in the workspace */
    /* Exclusion lists (Sec. 4: the exploratory task keeps vertices out of the result):
     * query i (row, vertex or descriptor i) never returns the ids
     * exclude_ids[exclude_offsets[i] .. exclude_offsets[i+1]); they are still checked,
     * enter S and are expanded. Both device pointers or both NULL; ids outside [0, n)
     * set DEG_FLAG_BAD_ID. An exploratory query also excludes its own vertex. */
    const int64_t *exclude_offsets;
    const int32_t *exclude_ids;
} deg_search_opts;

/*
 * Workspace bytes needed by deg_search / deg_search_indexed / deg_search_batch
 * for `nq` queries with results of size up to `k` and these options: a work
 * counter, one region of visited tables per resident wave (16384 slots, then
 * four times larger up to 262144), S's far part (L + 256 keys per resident
 * wave) and, when n needs larger tables, up to 64
 * shared tables of the smallest power of two >= 4n/3 int32 slots (a query
 * that needs one while all are held waits for one). Concurrent calls must not
 * share a workspace.
 */
size_t deg_search_workspace_bytes(const deg_vectors *v, const deg_graph *g, int64_t nq,
                                  int32_t k, const deg_search_opts *o);

/*
 * Waves per compute unit a search launch with these options keeps resident
 * (the persistent grid's size per CU when waves_per_cu is 0; a larger request
 * is capped at it). Launch tuning helper; 0 when the arguments are invalid.
 * Host-side only (reads the device's occupancy and CU count).
 */
int32_t deg_search_resident_waves(const deg_vectors *v, const deg_graph *g, int32_t k,
                                  const deg_search_opts *o);

/*
 * RangeSearch (Algorithm 1) of nq query vectors, one wavefront per query.
 *   queries   nq rows of q_stride FP32 (dim used)
 *   seed_ids  nq x n_seeds distinct seed vertices (Sec. 5.4: the search starts
 *             from the graph's median vertex, see deg_medoid)
 *   k         results per query (1..1024; up to 512 with a stop model or trace
 *             rows), eps >= 0 the range factor
 *   out_ids   nq x k int32, out_dists nq x k FP32 (the traversal distance, or
 *             the FP32 distance after a rerank)
 *   out_stats nullable; nq x 4 int32 {hops, distance evaluations, flags, 0}
 * With DEG_F32 data, no rerank and no stop model, the result equals the
 * oracle's Algorithm 1 exactly: same ids, distances, hops and evaluations.
 */
deg_status deg_search(const deg_vectors *v, const deg_graph *g, const float *queries,
                      int64_t nq, int64_t q_stride, const int32_t *seed_ids, int32_t n_seeds,
                      int32_t k, float eps, const deg_search_opts *o, int32_t *out_ids,
                      float *out_dists, int32_t *out_stats, void *workspace, size_t ws_bytes,
                      void *stream);

/*
 * deg_search without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, serving loops, harnesses that forbid
 * hipMalloc). Same arguments and results as deg_search. Its scratch is one
 * 128 MiB device array per GPU inside the library (held while the library is
 * loaded; every call on that GPU shares it and finds it as the last call left
 * it: the work counter and table owners are cleared by a kernel at each call).
 * To fit it the launch keeps one 8192-slot visited table per wave, at most 4
 * shared tables of the smallest power of two >= 4n/3 slots, and fewer resident
 * waves when needed (results are the same). Returns DEG_ERR_WORKSPACE when n is
 * too large for one wave's table and one shared table to fit (n above
 * 12,582,912). Calls that overlap on one GPU (other streams, other threads) race
 * on the array: serialise them. Allocates nothing (no hipMalloc / hipFree).
 */
deg_status deg_search_noalloc(const deg_vectors *v, const deg_graph *g, const float *queries,
                              int64_t nq, int64_t q_stride, const int32_t *seed_ids,
                              int32_t n_seeds, int32_t k, float eps, const deg_search_opts *o,
                              int32_t *out_ids, float *out_dists, int32_t *out_stats,
                              void *stream);

/*
 * Exploratory search (Sec. 4 and 6.7): each query is a base vertex; the
 * search starts at that vertex, uses its FP32 row as the query, and never
 * returns it (other vertices at distance 0 are returned).
 *   query_ids  nq vertex ids
 */
deg_status deg_search_indexed(const deg_vectors *v, const deg_graph *g, const int32_t *query_ids,
                              int64_t nq, int32_t k, float eps, const deg_search_opts *o,
                              int32_t *out_ids, float *out_dists, int32_t *out_stats,
                              void *workspace, size_t ws_bytes, void *stream);

/*
 * A mixed stream of queries in one persistent launch fed by a device work
 * queue. Each descriptor names its kind (0 = vector query, 1 = exploratory),
 * its seed (kind 0) or vertex (kind 1), its query row (kind 0, a row of
 * `queries`, which holds n_query_rows rows; may be NULL if every descriptor
 * is exploratory), its own k (1..k_max) and eps, and where its k results
 * start in out_ids / out_dists (the caller sizes those arrays). A descriptor
 * outside these bounds is skipped and flagged DEG_FLAG_BAD_ID.
 */
typedef struct {
    int32_t kind;
    int32_t seed_or_vertex;
    int64_t query_row;
    int32_t k;
    float eps;
    int64_t out_offset;
} deg_query_desc;

deg_status deg_search_batch(const deg_vectors *v, const deg_graph *g, const float *queries,
                            int64_t n_query_rows, int64_t q_stride, const deg_query_desc *descs,
                            int64_t nq,
                            int32_t k_max, const deg_search_opts *o, int32_t *out_ids,
                            float *out_dists, int32_t *out_stats, void *workspace,
                            size_t ws_bytes, void *stream);

/*
 * Exact k nearest neighbours (Eq. knn) by brute force on matrix cores, k <= 1024.
 * Candidates come from matrix products of the norm expansion: BF16 inputs with
 * FP32 accumulation (v_mfma_f32_32x32x16_bf16) when every base and query value
 * is an integer of magnitude <= 255 and dim <= 128 (a device-side check; every
 * product, sum and candidate distance is then an exact integer, so the result
 * equals the FP64 definition), FP32 inputs (v_mfma_f32_32x32x2f32) otherwise.
 * The best k + 32 per query and base slice are then recomputed as direct FP32
 * differences in the C32x4 order and sorted by (distance, id). exclude_ids:
 * nullable, one id per query kept out of its result (exploratory ground
 * truth). base rows are read as float4: b_stride must be a multiple of 4.
 */
size_t deg_knn_workspace_bytes(int64_t n, int32_t dim, int64_t nq, int32_t k);
deg_status deg_knn_bruteforce(const float *base, int64_t n, int32_t dim, int64_t b_stride,
                              const float *queries, int64_t nq, int64_t q_stride, int32_t k,
                              int32_t metric, const int32_t *exclude_ids, int32_t *out_ids,
                              float *out_dists, void *workspace, size_t ws_bytes, void *stream);

/* The median (seed) vertex of Sec. 5.4: the vertex nearest to the coordinate
 * mean (L2), or with the largest inner product with it (IP); ties -> smallest
 * id. out_id: one int32 on the device. */
size_t deg_medoid_workspace_bytes(int64_t n, int32_t dim);
deg_status deg_medoid(const float *vec, int64_t n, int32_t dim, int64_t stride, int32_t metric,
                      int32_t *out_id, void *workspace, size_t ws_bytes, void *stream);

/*
 * Graph construction (Sec. 5.2 with Algorithm 3's scheme C: the complete graph
 * on vertices 0..d, then every further vertex in id order: a search for its
 * k_ext nearest vertices from vertex 0, a pass over the result that takes each
 * vertex b passing the MRNG check (Algorithm 2) against the tentative
 * neighbours, cuts b's longest edge to a vertex outside them (equal weights:
 * the smaller id) and gives the new vertex both ends, and a second pass
 * without the check while fewer than d were found). optimizeEdge (Algorithm
 * 4) is not applied.
 * Batched schedule: the searches of a block of vertices all run on the graph
 * as it stands when the block starts, in one deg_search launch (FP32 traversal,
 * default options); the block's edits then follow in id order on the host,
 * each on the live graph, and the changed rows are copied to `adjacency`
 * before the next block. A block holds at most `batch` vertices and at most
 * nv / 8 of the nv vertices already in the graph (at least 1); batch = 1 is
 * the one-at-a-time build. With lag = 1 the size limit counts only the
 * vertices already in the graph, and the block's searches overlap the host
 * edits of the previous block.
 *   v              the n vectors (device, DEG_F32, L2 or IP): the searched store,
 *                  whose rows are also the new vertices' queries
 *   host_vectors   the same vectors on the host (row stride host_stride floats),
 *                  for the distances of the edges the edits create (FP32, the
 *                  library's fixed reduction order, equal to the search's)
 *   adjacency      device, n x degree int32, overwritten: the built graph,
 *                  every row holding exactly `degree` neighbours
 *   weights        nullable host n x degree FP32: the edge weights, row-aligned
 *   counters       nullable host int64[6]: {blocks, searches, vertices that
 *                  needed the pass without MRNG check, searches that lost a
 *                  candidate to the capacity of S (0 means every search was
 *                  Algorithm 1's exactly), microseconds from each block's row
 *                  upload to its results on the host, microseconds of the
 *                  host edits}
 * degree even in [4, 128], n >= degree + 1, k_ext in [1, 1024], eps_ext >= 0,
 * batch >= 1, lag 0 or 1. The call allocates its own device and pinned host buffers
 * (the host graph takes n x round_up(2 + 2 degree, 16) x 4 bytes of pinned memory),
 * frees them before it returns, and returns when the graph is complete on
 * `stream` (it synchronises the stream once per block). DEG_ERR_UNSUPPORTED
 * when a search result cannot supply degree neighbours (k_ext too small);
 * DEG_ERR_HIP when an allocation (device or host) or a HIP call fails.
 */
typedef struct {
    int32_t degree;  /* d */
    int32_t k_ext;   /* result size of a new vertex's search */
    float eps_ext;   /* range factor of that search */
    int32_t lag;     /* 0: a block searches the graph with every earlier block in it;
                        1: a block searches before the previous block's edits are applied
                        (its edits then run on the host while this block searches) */
    int64_t batch;   /* the most vertices in one block */
} deg_build_params;

deg_status deg_build_graph(const deg_vectors *v, const float *host_vectors, int64_t host_stride,
                           const deg_build_params *p, int32_t *adjacency, float *weights,
                           int64_t *counters, void *stream);

/*
 * MRNG conformity of every edge (Algorithm 2) and every vertex's longest edge:
 * the selection step of the dynamic edge optimisation (Algorithm 5 optimises a
 * vertex's edges that fail the check, then its longest edge). Edge (v1, v2)
 * fails when a common neighbour u of v1 and v2 has
 * max(w(v1, u), w(v2, u)) < w(v1, v2); only stored weights are compared.
 *   g          device adjacency (degree <= 128; id -1 marks an empty slot)
 *   weights    device, n rows of w_stride FP32: weights[v][j] is the weight of
 *              the edge to adj[v][j] (as deg_build_graph returns them)
 *   out_ok     device, n x degree bytes: 1 the edge passes, 0 it fails, 255 the
 *              slot is empty (or holds an id outside [0, n))
 *   out_fail_count nullable device int64: the number of failing entries (each
 *              undirected edge is counted from both ends)
 *   out_longest nullable device int32[n]: the slot of the vertex's longest edge
 *              (equal weights: the smaller neighbour id; -1 for an empty row)
 * Asynchronous on `stream`; allocates nothing.
 */
deg_status deg_graph_check_mrng(const deg_graph *g, const float *weights, int64_t w_stride,
                                uint8_t *out_ok, int64_t *out_fail_count, int32_t *out_longest,
                                void *stream);

/* Reduced-precision stores. BF16: round to nearest even. FP8: per row
 * scale = max|x| / 448 (1 if the row is zero), code = E4M3 round to nearest
 * even of x / scale, saturating at 448. Rows beyond dim are zero-filled up to
 * out_stride. */
deg_status deg_encode_bf16(const float *x, int64_t n, int32_t dim, int64_t x_stride,
                           uint16_t *out, int64_t out_stride, void *stream);
deg_status deg_encode_fp8(const float *x, int64_t n, int32_t dim, int64_t x_stride,
                          uint8_t *out, int64_t out_stride, float *scale, void *stream);

/*
 * Stop-predictor training (FP32): one fused forward + backward pass of the
 * 16-64-64-1 MLP with mean binary cross-entropy over B rows, then one Adam
 * step. params/m/v: 5313 FP32 each (layout as deg_stop_model). X: B x 16,
 * y: B labels in {0,1}. grad (nullable, 5313) receives the gradient and
 * loss (nullable, 1) the mean loss. step >= 1; lr = 0 skips the update.
 */
size_t deg_mlp_workspace_bytes(int64_t B);
deg_status deg_mlp_train_step(float *params, float *m, float *v, const float *X, const float *y,
                              int64_t B, int64_t step, float lr, float *grad, float *loss,
                              void *workspace, size_t ws_bytes, void *stream);
/* Logits of B rows with FP32 params (out: B floats). */
deg_status deg_mlp_forward(const float *params, const float *X, int64_t B, float *out,
                           void *stream);
/* Logits of B rows with the BF16 weights the search uses (out: B floats). */
deg_status deg_mlp_forward_bf16(const uint16_t *w, const float *X, int64_t B, float *out,
                                void *stream);
/* FP32 params -> BF16 weights for deg_stop_model. */
deg_status deg_mlp_export_bf16(const float *params, uint16_t *out, void *stream);
/* Standardisation of the stop predictor's inputs: per column of B x 16 rows X
 * the mean and 1 / (unbiased standard deviation) (0 when it is <= 1e-6), summed
 * in FP64 in a fixed order; and out = (X - mean) * inv_std in FP32 (out may
 * equal X). mean, inv_std: 16 floats each (device). */
deg_status deg_mlp_feature_stats(const float *X, int64_t B, float *mean, float *inv_std,
                                 void *stream);
deg_status deg_mlp_standardise(const float *X, int64_t B, const float *mean,
                               const float *inv_std, float *out, void *stream);

/*
 * Autotuner table (written by the package's tuner, read at launch): for
 * searches over `dtype` rows of `dim` dims on a graph of `degree`, with a pool
 * size in the bucket kp_bucket (16, 64, 128, 256 or 512), use `hash_slots`
 * LDS visited slots and at most `waves_per_cu` resident waves per CU
 * (0 = as many as fit). Explicit deg_search_opts fields take precedence.
 */
deg_status deg_tune_register(int32_t dtype, int32_t dim, int32_t degree, int32_t kp_bucket,
                             int32_t hash_slots, int32_t waves_per_cu);
void deg_tune_clear(void);

/* Number of compute units of the current device (for workspace sizing). */
int32_t deg_device_cu_count(void);

const char *deg_status_string(deg_status s);

#ifdef __cplusplus
}
#endif

#endif /* DEG_H */
