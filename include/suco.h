/*
 * suco.h -- C ABI of the MI355X (gfx950) SuCo query library.
 *
 * SuCo answers k-approximate-nearest-neighbour queries with the Subspace
 * Collision framework (arXiv 2411.14754).  The problem (Sec. 1): given a
 * dataset D of n points in R^d, a query q and k, return k points of D close
 * to q; quality is recall |R intersect R*|/k against the exact k-NN R*.
 *
 * Conventions for every call:
 *  - Return value: SUCO_OK (0) or a negative SUCO_E_* code.  On error nothing
 *    is enqueued and no output is written; suco_last_error() (thread-local)
 *    describes the failure.  No C++ exception crosses this boundary.
 *  - Arguments are validated synchronously, before any GPU work is enqueued.
 *  - "device" pointers are HIP device memory on the index's device (for
 *    example torch.cuda tensors' data_ptr()); "host" pointers are ordinary
 *    CPU memory.  The caller owns every pointer it passes; the library never
 *    frees or keeps a caller pointer after the call returns (the dataset is
 *    copied into the index).
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Query
 *    calls are asynchronous on that stream: outputs are valid once the stream
 *    has been synchronised.  Build calls synchronise before returning.
 *  - An index is read-only after it is built and may be queried from several
 *    host threads, but queries on one index share its workspace: the library
 *    serialises them (a query on a new stream waits for the previous query's
 *    stream), so concurrent queries on one index do not overlap on the GPU.
 *  - Results are deterministic: identical inputs give bitwise identical
 *    outputs, on any stream and any batching.
 *  - Row-major layouts everywhere: D [n][d], Q [nq][d], ids/dists [nq][k].
 */
#ifndef SUCO_H
#define SUCO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define SUCO_API __attribute__((visibility("default")))
#else
#define SUCO_API
#endif

#define SUCO_OK 0
#define SUCO_E_INVAL -1        /* an argument is out of range or NULL          */
#define SUCO_E_NOMEM -2        /* device or host allocation failed             */
#define SUCO_E_HIP -3          /* a HIP runtime call or kernel launch failed    */
#define SUCO_E_STATE -4        /* wrong device, freed or unusable handle       */
#define SUCO_E_UNSUPPORTED -5  /* valid but outside what the GPU path handles  */

typedef struct suco_index suco_index;

/* Optional build parameters (pass NULL for the defaults). */
typedef struct suco_build_params {
    int32_t iters;      /* k-means iterations t (Table 1, Alg. 2); <= 0 means 25      */
    uint64_t seed;      /* k-means initialisation seed; 0 means 1                      */
    int32_t tile_max;   /* most point ids per collision tile, a multiple of 256 in
                           [256, 65536]; 0 means 65536.  Each query's SC-scores are
                           counted tile by tile in on-chip memory.                    */
    int32_t query_chunk;/* queries processed per internal pass; 0 means automatic:
                           as many as 16 GiB of per-query workspace (2 bytes per
                           point, 2 bytes per cell and subspace) allow, at most
                           16384; a query call's nq is split into equal passes
                           of at most this many.
                           The workspace is allocated by the index on first use
                           and kept until suco_index_free.                         */
    int32_t flags;      /* SUCO_BUILD_* bits                                          */
} suco_build_params;

/* When every coordinate of D is an integer in 0..255 the index also keeps a
 * byte copy of D, from which the re-rank reads its rows (they convert to FP32
 * exactly, so results are unchanged).  This flag keeps FP32 rows only. */
#define SUCO_BUILD_NO_BYTE_ROWS 1
/* Also keep what suco_query_bf16 reads: a BF16 copy of D (2*n*d bytes), a
 * per-row bound of its rounding error (4*n bytes) and BF16 centres.  Needs d
 * to be a multiple of 8. */
#define SUCO_BUILD_BF16 2
/* Leave out the sparse collision step and its cell-major copy of the IMI
 * (4*n*n_s bytes): every query counts SC-scores tile by tile over the whole
 * id range.  The results are the same either way. */
#define SUCO_BUILD_NO_SPARSE 4
/* SuCo-L1 (Sec. 5.3, Table 5): the Manhattan distance instead of the
 * Euclidean one throughout.  suco_build clusters each half with k-medians
 * (nearest centre by L1 in FP64, ties to the lower centre id; each centre
 * coordinate the lower median, the ceil(m/2)-th smallest of its m members'
 * values; an empty cluster keeps its centre; the same initial centres and
 * final assignment pass as the k-means).  Queries rank centres and cells by
 * L1 distance (a cell's key is the L1 distance to its product centre), count
 * and select as usual, re-rank by L1 (FP32, dimension order) and return L1
 * distances.  Not with SUCO_BUILD_BF16 (SUCO_E_UNSUPPORTED); the Multi-
 * sequence rule, SC-Linear and the batched and no-alloc forms follow the
 * index's metric. */
#define SUCO_BUILD_L1 8

SUCO_API int suco_version(void);
SUCO_API const char *suco_last_error(void);

/* Number of points activated per subspace, A = max(1, ceil(alpha*n)) capped at n
 * (Alg. 3 stops once alpha*n points are retrieved), and the number of
 * candidates re-ranked, B = max(k, floor(beta*n)) capped at n (Alg. 4 re-ranks
 * beta*n points; raised to k so that a top-k exists).  Both are evaluated in
 * FP64 with a 1e-9 guard against representation error. */
SUCO_API int64_t suco_count_A(double alpha, int64_t n);
SUCO_API int64_t suco_count_B(double beta, int64_t n, int32_t k);

/* ---------------------------------------------------------------- build --
 * Create Index (Alg. 2).  The d dimensions are divided into n_s contiguous
 * subspaces (Sec. 3.2; the last takes the remainder, Def. 3), each split into
 * two halves (first floor(s/2) dims, then the rest).  Each half is clustered
 * by Lloyd's k-means into sqrt_k centres with FP64 sums (t iterations from a
 * SplitMix64-drawn set of distinct rows, then a final assignment); the
 * inverted multi-index of subspace i maps cell a1*sqrt_k + a2 to its point
 * ids in ascending order.  Centres are stored in FP32 (rounded once).
 *
 *  D      device [n][d] float32, copied into the index.
 *  limits 1 <= n < 2^31; 2 <= d; 1 <= n_s <= d/2; 1 <= sqrt_k <= n
 *         (SUCO_E_INVAL otherwise).  The kernels take n_s <= 127 and
 *         sqrt_k <= 128 (SUCO_E_UNSUPPORTED beyond).
 *  out    receives the new handle (unchanged on error).
 */
SUCO_API int suco_build(const float *D, int64_t n, int32_t d, int32_t n_s, int32_t sqrt_k,
               const suco_build_params *p, void *stream, suco_index **out);

/* Create an index from given centres and assignments instead of running
 * k-means (for example an index saved earlier, or one computed elsewhere).
 *  centroids  host float32, the 2*n_s halves one after another: half g
 *             (g = 2*i + h) is sqrt_k rows of its width, starting at element
 *             sqrt_k * (first dimension of the half).  Total sqrt_k*d values.
 *  assign     host int32 [2*n_s][n], values in [0, sqrt_k).
 */
SUCO_API int suco_build_from_index(const float *D, int64_t n, int32_t d, int32_t n_s, int32_t sqrt_k,
                          const float *centroids, const int32_t *assign,
                          const suco_build_params *p, void *stream, suco_index **out);

/* Copy the canonical index out: FP32 centres (layout as above) and the
 * assignments, both host memory; either may be NULL. */
SUCO_API int suco_index_export(const suco_index *ix, float *centroids, int32_t *assign);

/* Shape of an index; any output may be NULL. */
SUCO_API int suco_index_info(const suco_index *ix, int64_t *n, int32_t *d, int32_t *n_s, int32_t *sqrt_k);

/* What the index keeps besides the FP32 data: bit SUCO_INDEX_BYTE_ROWS when the
 * re-rank reads a byte copy of D (every coordinate an integer in 0..255, the
 * default unless SUCO_BUILD_NO_BYTE_ROWS), bit SUCO_INDEX_BF16 when it was built
 * with SUCO_BUILD_BF16.  flags: host int32. */
#define SUCO_INDEX_BYTE_ROWS 1
#define SUCO_INDEX_BF16 2
#define SUCO_INDEX_L1 4       /* built with SUCO_BUILD_L1: the Manhattan distance throughout */
#define SUCO_INDEX_SPARSE 8   /* queries may take the sparse collision step (N_s <= 31, n <= 2^24, not
                                 SUCO_BUILD_NO_SPARSE, and the device's LDS holds its tables) */
SUCO_API int suco_index_flags(const suco_index *ix, int32_t *flags);

/* Activation rule of step 2 for the queries that follow on this index (each
 * query call reads it when it starts; a batcher reads it when it builds a
 * bucket's graph, so set it before creating one).
 *  SUCO_ACT_DYNAMIC   Dynamic Activation (Alg. 3), the default.
 *  SUCO_ACT_MULTISEQ  Multi-sequence, the inverted multi-index traversal that
 *                     Sec. 4.2 compares it with: a priority queue of cells by
 *                     ascending key, seeded with the cell of both nearest
 *                     centres, where taking a cell queues its two neighbours
 *                     in the rank grid.  It activates the same cells (ties in
 *                     the key by the first rank, then the second); it exists
 *                     to measure the two rules against each other (Sec. 5.2).
 *                     Cells are exported in retrieval order, where Dynamic
 *                     Activation exports them row by row.
 *  errors  SUCO_E_INVAL for another value; SUCO_E_UNSUPPORTED for
 *          SUCO_ACT_MULTISEQ on an index with sqrt_k > 64. */
#define SUCO_ACT_DYNAMIC 0
#define SUCO_ACT_MULTISEQ 1
SUCO_API int suco_index_set_activation(suco_index *ix, int32_t form);

/* Release an index (NULL is accepted).  Waits for its pending queries. */
SUCO_API int suco_index_free(suco_index *ix);

/* Save an index to a file and load it back (the output of Create Index,
 * Alg. 2, with the data it indexes), so that a query process need not run
 * k-means again.  The file holds a 64-byte header (magic "SUCOIDX1", version
 * 1, n, d, n_s, sqrt_k, the SUCO_BUILD_* flags, tile_max and query_chunk the
 * index was built with, and a 64-bit checksum of the rest), then the FP32
 * centres (layout of suco_build_from_index), the assignments as bytes
 * [2*n_s][n] and D [n][d] FP32, each section zero-padded to a multiple of 8
 * bytes; little-endian.  Save writes `path`.tmp and renames it; it
 * synchronises the index's device.  Load checks the header and the file size
 * before any device work, rebuilds the index from the stored centres and
 * assignments (as suco_build_from_index), and fails with SUCO_E_INVAL if the
 * checksum does not match.  p overrides the stored build parameters (NULL:
 * those recorded in the file) except SUCO_BUILD_L1, which is always the
 * file's (the centres belong to that metric).  A loaded index answers every query bitwise
 * as the saved one did.
 *  path  host NUL-terminated file name. */
SUCO_API int suco_index_save(const suco_index *ix, const char *path);
SUCO_API int suco_index_load(const char *path, const suco_build_params *p, void *stream, suco_index **out);

/* ---------------------------------------------------------------- query --
 * k-ANN Query (Alg. 4 with Dynamic Activation, Alg. 3), one batch:
 *  1. per subspace, squared distances from each query half to the sqrt_k
 *     centres of that half, sorted ascending (ties by centre id);
 *  2. Dynamic Activation: cells are taken in ascending order of
 *     dist1 + dist2 (ties by the two ranks) until at least A points are
 *     retrieved -- the shortest such prefix, whole cells;
 *  3. every point in an activated cell gets +1 SC-score (Def. 4);
 *  4. the B points with the highest SC-scores (ties: lowest ids) are kept;
 *  5. they are re-ranked by exact squared L2 in FP32 and the k nearest are
 *     returned by (distance, id).
 *
 *  Q      device [nq][d] float32 queries.
 *  ids    device [nq][k] int32 result point ids, nearest first.
 *  dists  device [nq][k] float32 Euclidean (not squared) distances.
 *  limits nq >= 0 (0 is a no-op), 1 <= k <= n, 0 < alpha <= 1,
 *         0 < beta <= 1 (SUCO_E_INVAL otherwise); the kernels take k <= 64
 *         (SUCO_E_UNSUPPORTED beyond).
 */
SUCO_API int suco_query(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha,
               double beta, int32_t *ids, float *dists, void *stream);

/* suco_query for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid it): the same
 * kernels and the same results, bitwise, with the workspace taken from a
 * fixed 64 MiB device array inside the library (each device the library runs
 * on holds its own copy until the process ends) instead of an allocation.
 * The call allocates nothing and records no events.  The batch is split into
 * passes whose workspace fits the array (about 2 bytes per point and query,
 * 4 bytes per candidate); SUCO_E_UNSUPPORTED when even one query does not
 * fit (n above about 30 million at beta = 0.005).  Every call on a device
 * shares that device's array and needs no state from an earlier call: calls
 * that overlap on one device (several streams, several host threads) race,
 * so the caller must order them.  Arguments as in suco_query. */
SUCO_API int suco_query_noalloc(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha,
                                double beta, int32_t *ids, float *dists, void *stream);

/* As suco_query with one collision ratio per query: alpha_q device [nq]
 * float32, each meant to lie in (0, 1]; query j activates
 * A_j = max(1, ceil(alpha_q[j]*n)) points per subspace (the value is widened
 * to FP64 before the product).  Device values are not checked on the host:
 * a value above 1, +inf or NaN activates every cell (A_j = n) and a value
 * <= 0 activates A_j = 1 point. */
SUCO_API int suco_query_alpha(const suco_index *ix, const float *Q, int64_t nq, int32_t k,
                     const float *alpha_q, double beta, int32_t *ids, float *dists, void *stream);

/* As suco_query_alpha (alpha_q may be NULL, then `alpha` is used for every
 * query), also exporting the intermediate results of every step; each extra
 * output is device memory and may be NULL:
 *  scores  uint8 [nq][n]      SC-scores after step 3
 *  cand    int32 [nq][B]      step-4 candidates (the set is defined; its order
 *                             within a row is not, compare rows as sets)
 *  ncells  int32 [nq][n_s]    number of cells activated per subspace
 *  aprime  int32 [nq][n_s]    points in those cells (>= A)
 *  cells   uint16 [nq][n_s][sqrt_k^2]  activated cell ids (a1*sqrt_k + a2),
 *                             the first ncells entries of each row are valid
 *  feat    float32 [nq][2*n_s] distance from each query half to its nearest
 *                             centre (sqrt of the smallest step-1 value; on a
 *                             SUCO_BUILD_L1 index the smallest L1 distance)
 */
SUCO_API int suco_query_debug(const suco_index *ix, const float *Q, int64_t nq, int32_t k,
                     const float *alpha_q, double alpha, double beta, int32_t *ids, float *dists,
                     uint8_t *scores, int32_t *cand, int32_t *ncells, int32_t *aprime,
                     uint16_t *cells, float *feat, void *stream);

/* ------------------------------------------------- BF16 split precision --
 * The query of suco_query with BF16 arithmetic where it cannot change the
 * answer, on an index built with SUCO_BUILD_BF16.
 *  - flags & SUCO_BF16_S1: step 1 runs on the matrix cores, the centre
 *    distances being |q^|^2 + |c^|^2 - 2 q^.c^ from BF16-rounded query halves
 *    q^ and centres c^ with FP32 accumulation.  The keys of step 2 then carry
 *    the BF16 rounding, so cells whose keys nearly tie may be activated
 *    differently from suco_query.  Without the flag step 1 is that of
 *    suco_query (FP32) and the activated cells are identical.
 *  - Step 5 in two passes: a first pass over all B candidates reads the BF16
 *    copy of D (half the bytes) and brackets each candidate's FP32 squared
 *    distance between certified lower and upper bounds (from a per-row bound
 *    of the BF16 rounding error and the FP32 rounding of both sums); the
 *    survivors are the candidates whose lower bound does not exceed the k-th
 *    smallest upper bound, a set that provably contains the FP32 top-k.  The
 *    survivors are re-ranked exactly as suco_query re-ranks, so for the same
 *    candidates ids and dists are bitwise those of suco_query.
 *
 *  Q, ids, dists, k, alpha, beta   as in suco_query.
 *  nsurv   device int32 [nq] survivor count per query, or NULL.
 *  relerr  device double [nq][k] |dists - t| / t per result, t the FP64
 *          Euclidean distance of the returned point, or NULL.
 *  cdist   device float32 [nq][2*n_s][sqrt_k] the BF16 centre distances
 *          (only with SUCO_BF16_S1), or NULL.
 *  errors  SUCO_E_STATE if the index was built without SUCO_BUILD_BF16.
 */
#define SUCO_BF16_S1 1
SUCO_API int suco_query_bf16(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha,
                             double beta, int32_t flags, int32_t *ids, float *dists, int32_t *nsurv,
                             double *relerr, float *cdist, void *stream);
/* As suco_query_bf16, also exporting the intermediate results of steps 2-4
 * (scores, cand, ncells, aprime, cells: layouts and meaning as in
 * suco_query_debug; each may be NULL). */
SUCO_API int suco_query_bf16_debug(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha,
                                   double beta, int32_t flags, int32_t *ids, float *dists, int32_t *nsurv,
                                   double *relerr, float *cdist, uint8_t *scores, int32_t *cand,
                                   int32_t *ncells, int32_t *aprime, uint16_t *cells, void *stream);

/* ------------------------------------------------------------ SC-Linear --
 * The subspace collision framework without an index (Alg. 1): for each query
 * and subspace i (the division of the index, Sec. 3.2), the A = max(1,
 * ceil(alpha*n)) points nearest to the query in that subspace collide (Def. 2,
 * squared distances in FP32 summed in dimension order, ties by lower id); a
 * point's SC-score is the number of subspaces where it collides (Def. 4); the
 * B = max(k, floor(beta*n)) points of highest score (ties by lower id) are
 * re-ranked as in suco_query.  Reads all of D per pass of queries; the index
 * supplies D, the subspace division and the re-rank's rows only.
 *  Q, ids, dists, k, alpha, beta   as in suco_query.
 *  scores  device uint8 [nq][n] SC-scores, or NULL.
 *  limits  subspaces of at most 64 dimensions (SUCO_E_UNSUPPORTED beyond). */
SUCO_API int suco_query_sclinear(const suco_index *ix, const float *Q, int64_t nq, int32_t k, double alpha,
                                 double beta, int32_t *ids, float *dists, uint8_t *scores, void *stream);

/* ------------------------------------------------------- single steps --
 * The steps of the query path on their own, fed by the caller; they let each
 * step be checked in isolation and let other activation rules reuse the rest.
 *
 * Collision counting and selection (steps 3-4) from given activated cells:
 *  cells   device uint16 [nq][n_s][sqrt_k^2], ncells device int32 [nq][n_s]
 *  scores  device uint8 [nq][n] (may be NULL), cand device int32 [nq][B]
 *          with B = suco_count_B(beta, n, k).
 */
SUCO_API int suco_collide_select(const suco_index *ix, int64_t nq, const uint16_t *cells,
                        const int32_t *ncells, int32_t k, double beta, uint8_t *scores,
                        int32_t *cand, void *stream);

/* Re-rank (step 5) given candidate lists: cand device int32 [nq][B] of ids
 * in [0, n) (repeats not allowed); returns the k nearest by (distance, id). */
SUCO_API int suco_rerank(const suco_index *ix, const float *Q, int64_t nq, const int32_t *cand,
                int64_t B, int32_t k, int32_t *ids, float *dists, void *stream);

/* ------------------------------------------------------------ batcher --
 * Batched form of suco_query for streams of batches of uneven size.  A batcher
 * holds staging buffers and a workspace sized for max_batch queries and, per
 * power-of-two batch-size bucket, one HIP graph of the whole query path whose
 * kernels stride over their work and read the batch size on the device.  A call
 * writes the caller's pointers and nq into a device mailbox (one small kernel)
 * and launches the bucket's graph.  On a bucket's first use its launch shapes
 * (re-rank rows per work-group, grid caps) are tuned by timing candidate
 * graphs on that batch; the choice is appended to `tune_file` when one is given
 * and read back by later batchers.  Results are bitwise those of
 * suco_query/suco_query_alpha with the same arguments.
 *
 *  ix         the index (must outlive the batcher); not modified.
 *  max_batch  largest nq, 1..65536 (rounded up to a power of two).
 *  k, beta    as in suco_query, fixed for the batcher.
 *  tune_file  host path of the tuning record, or NULL.
 * suco_batcher_query: Q device [nq][d]; alpha_q device [nq] float32 or NULL
 *  (then `alpha`); ids/dists device [nq][k]; asynchronous on `stream`; calls on
 *  one batcher are serialised.  The caller's buffers must stay valid until the
 *  stream reaches the call.  The first call of a bucket synchronises `stream`
 *  while it tunes. */
typedef struct suco_batcher suco_batcher;
SUCO_API int suco_batcher_create(const suco_index *ix, int32_t max_batch, int32_t k, double beta,
                                 const char *tune_file, suco_batcher **out);
SUCO_API int suco_batcher_query(suco_batcher *b, const float *Q, int64_t nq, const float *alpha_q,
                                double alpha, int32_t *ids, float *dists, void *stream);
/* Several batches of uneven size in one launch: nb (1..16) batches, batch j
 * with nq[j] >= 0 queries at Q[j] (device [nq[j]][d]), results to ids[j] and
 * dists[j] (device [nq[j]][k]); alpha_q NULL (then `alpha` for all) or
 * alpha_q[j] device [nq[j]] float32 for every non-empty batch.  Q, nq, alpha_q,
 * ids and dists are host arrays of nb entries, read during the call.  The
 * batches are placed back to back in the staging buffers and the graph of the
 * bucket of their total (at most max_batch, else SUCO_E_INVAL) runs once; each
 * batch's results are bitwise those of suco_batcher_query on it alone.  Same
 * stream, ordering and lifetime rules as suco_batcher_query. */
SUCO_API int suco_batcher_query_multi(suco_batcher *b, int32_t nb, const float *const *Q, const int64_t *nq,
                                      const float *const *alpha_q, double alpha, int32_t *const *ids,
                                      float *const *dists, void *stream);
/* Tuned launch shape of a built bucket: params[3] = {re-rank rows per
 * work-group, collision grid cap, re-rank grid cap} (0 = one block per item),
 * ms = the tuned graph's time on its first batch. */
SUCO_API int suco_batcher_tuning(const suco_batcher *b, int32_t bucket, int32_t *params, double *ms);
SUCO_API int suco_batcher_free(suco_batcher *b);

/* ---------------------------------------------------- learned budget --
 * The paper fixes one collision ratio alpha for all queries (Alg. 4) and names
 * combining the method with learned models as future work (Sec. 6).  A small
 * network predicts a per-query alpha instead:
 *   features f (2*n_s + 1 per query): for each subspace half, the Euclidean
 *     distance from the query half to its nearest centre, then the query norm;
 *   x = (f - mu) / sigma; h1 = GELU(W1 x + b1); h2 = GELU(W2 h1 + b2);
 *   y = W3 h2 + b3 (y predicts log alpha); GELU(x) = x * Phi(x);
 *   alpha = clamp(scale * exp(y), alpha_min, alpha_max) (NaN gives alpha_max).
 * Parameters are one FP32 array in the order W1 [H][n_in], b1 [H], W2 [H][H],
 * b2 [H], W3 [H], b3 [1]; H = 128.  Training runs in FP32 on the GPU (mean
 * squared error, Adam with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias
 * correction); inference rounds weights and layer inputs to BF16 and
 * accumulates in FP32.  All device arrays below are row-major FP32. */
typedef struct suco_mlp suco_mlp;
/* Parameter count, or -1 if (n_in, hidden) is not supported. */
SUCO_API int64_t suco_mlp_num_params(int32_t n_in, int32_t hidden);
/* params: host array (NULL: uniform +-sqrt(3/fan_in) from SplitMix64 draws of
 * `seed`, biases 0).  mu = 0 and sigma = 1 until suco_mlp_set_norm. */
SUCO_API int suco_mlp_create(int32_t n_in, int32_t hidden, const float *params, uint64_t seed, suco_mlp **out);
SUCO_API int suco_mlp_set_norm(suco_mlp *m, const float *mu, const float *sigma);         /* host [n_in] */
SUCO_API int suco_mlp_get_params(const suco_mlp *m, float *params);                       /* host, synchronises */
SUCO_API int suco_mlp_set_params(suco_mlp *m, const float *params);                       /* host */
/* Loss and its gradient for rows F [m][n_in], targets t [m] (device); grads
 * device [num_params], loss device [1] or NULL.  Asynchronous on `stream`. */
SUCO_API int suco_mlp_forward_backward(suco_mlp *m, const float *F, const float *t, int64_t rows, float *loss,
                                       float *grads, void *stream);
/* One epoch of mini-batch Adam over F [m][n_in], t [m] (device): batches of
 * `batch` consecutive positions of `order` (device int32 [m], a permutation of
 * the rows; NULL = row order).  mean_loss (host, may be NULL) receives the
 * mean batch loss, which synchronises the stream after every batch. */
SUCO_API int suco_mlp_train_epoch(suco_mlp *m, const float *F, const float *t, int64_t rows, int32_t batch,
                                  float lr, const int32_t *order, float *mean_loss, void *stream);
/* BF16 inference: y [m] (log alpha) and alpha [m], device, either may be NULL. */
SUCO_API int suco_mlp_predict(suco_mlp *m, const float *F, int64_t rows, float scale, float alpha_min,
                              float alpha_max, float *y, float *alpha, void *stream);
SUCO_API int suco_mlp_free(suco_mlp *m);
/* Query features F device [nq][2*n_s + 1].  The learned budget (features,
 * suco_query_learned, suco_batcher_set_model) is Euclidean: on a
 * SUCO_BUILD_L1 index these calls return SUCO_E_UNSUPPORTED. */
SUCO_API int suco_query_features(const suco_index *ix, const float *Q, int64_t nq, float *F, void *stream);
/* k-ANN query with the network's per-query alpha: features, BF16 inference,
 * then exactly suco_query_alpha with those alphas; alpha_used (device [nq],
 * may be NULL) receives them.  The alphas equal, bit for bit, those of
 * suco_query_features followed by suco_mlp_predict with the same arguments. */
SUCO_API int suco_query_learned(const suco_index *ix, suco_mlp *m, const float *Q, int64_t nq, int32_t k,
                                double beta, float scale, float alpha_min, float alpha_max, int32_t *ids,
                                float *dists, float *alpha_used, void *stream);
/* Attach a model to a batcher (NULL detaches): its graphs then compute the
 * features and the alphas on the device before the query path, and each
 * batch's results equal suco_query_learned's.  The model must outlive the
 * batcher or be detached first. */
SUCO_API int suco_batcher_set_model(suco_batcher *b, suco_mlp *m, float scale, float alpha_min, float alpha_max);

/* ----------------------------------------------------------- timing --
 * Per-step timing for measurement: while enabled, every launch of a query
 * call is bracketed by a pair of HIP events on the query stream (a few
 * microseconds per launch).  suco_profile_read waits for the recorded work
 * and returns, per step, the summed milliseconds and launch counts since the
 * last read, then resets.  Steps, in order: 0 activate (centre distances and
 * Dynamic Activation), 1 collide (SC-score counting over id tiles), 2 select
 * (top-B by score), 3 rerank (candidate distances, partial top-k), 4 merge
 * (final top-k), 5 BF16 centre distances, 6 BF16 first re-rank pass,
 * 7 survivors, 8 ordering of a pass's queries by activated points (heaviest
 * first), 9 sparse collide (SC-scores and top-B of the queries whose
 * activated points are few next to n, per bucket of 4096 ids).
 *  ms        host double [10]
 *  launches  host int64 [10] */
SUCO_API int suco_profile(suco_index *ix, int enable);
SUCO_API int suco_profile_read(suco_index *ix, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* SUCO_H */
