// Internal declarations shared by the SuCo runtime and its gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace suco {

constexpr int kWave = 64;
constexpr int kMaxSqrtK = 128;   // LDS tables of the activation step are sized for this
constexpr int kMaxNs = 127;      // SC-scores are bytes counted with 7-bit SWAR compares
constexpr int kMaxK = 64;        // one result per lane of a wave in the top-k lists
constexpr int kMaxU = 8;         // float4 slices of a row per lane in the re-rank
constexpr int kRowChunk = 1024;  // candidate ids staged in LDS at a time by the re-rank kernels

struct HalfDims {
    int dim0;  // first dimension of the half
    int w;     // width of the half
};

// Read-only index data resident in HBM.
struct IndexView {
    const float *X;          // [n][d] points
    const float *cent;       // [sqrt_k * d] FP32 centres, half g at sqrt_k*dim0[g]
    const HalfDims *halves;  // [2*ns]
    const uint32_t *toffs;   // [ns][P][K+1] start of cell c's ids inside tile p
    const uint16_t *ids16;   // [ns][P*TILE] tile-local ids, tile-major, cell-major, ascending
    const uint32_t *csize;   // [ns][K] points per cell
    const uint32_t *coffs;   // [ns][K+1] start of cell c in ids32, or null (no sparse collision step)
    const uint32_t *ids32;   // [ns][n] point ids, cell-major, ascending within a cell
    const uint16_t *cbh;     // [ns*K][sp_nb_padded(NB)] ids of each cell per bucket of kSpBucket ids
    int64_t n;
    int d, ns, sk, K, P, TILE;
    int NB;                  // buckets of kSpBucket consecutive ids (sparse collision step)
    int act_form;            // activation rule: 0 Dynamic Activation, 1 Multi-sequence (sqrt_k <= 64)
    int metric;              // 0: squared Euclidean keys and re-rank, Euclidean result; 1: Manhattan (SuCo-L1)
};

// Sparse collision step (query_kernels.hip): ids are grouped in buckets of
// 4096 consecutive ids, one 2 KB window of 4-bit scores per wave, one
// work-group of 1024 threads per CU with all of its LDS.
constexpr int kSpShift = 12;
constexpr int kSpBucket = 1 << kSpShift;
constexpr int kSpThreads = 1024;
constexpr int kSpWaves = kSpThreads / kWave;
constexpr int kSpMaxNs = 15;        // 4-bit scores, 8 ids a window word
constexpr int kSpMaxNs5 = 31;       // 5-bit scores, 6 ids a window word (N_s of 16 to 31)
__host__ __device__ constexpr int sp_score_bits(int ns) { return ns <= kSpMaxNs ? 4 : 5; }
// words of one wave's score window: 4096 ids at 8 a word, or at 6 a word (683, padded to 16 bytes)
__host__ __device__ constexpr int sp_win_words(int sb) { return sb == 4 ? kSpBucket / 8 : 688; }
constexpr int kSpMaxBuckets = 4096; // n <= 2^24
constexpr int kSpMaxRuns = 1024;    // activated cells of a query, all subspaces
constexpr int kSpMaxChunks = 128;   // 1024-position chunks of a query's activated ids (the slots hold fewer)
// Dynamic LDS of the sparse step for NB buckets and `cap` slots: the run
// table and the runs' cells, three per-bucket arrays padded to 16 bytes, the
// waves' score windows and the slots (a query's activated ids, then its list
// of points of score >= 2).
__host__ __device__ inline int sp_nb_padded(int NB) { return (NB + 4) & ~3; }
__host__ __device__ inline size_t sp_lds_bytes(int NB, int cap, int sb) {
    return 12 * (size_t)kSpMaxRuns + 12 * (size_t)sp_nb_padded(NB) + 4 * (size_t)kSpWaves * sp_win_words(sb) +
           2 * (size_t)((cap + 7) & ~7);
}

// One pass of the query path over a chunk of queries.
struct QueryPass {
    IndexView ix;
    const float *Q;           // [nq][d]
    int nq;
    const float *alpha_q;     // [nq] or null
    const double *alpha_qd;   // [nq] or null (takes precedence over alpha_q)
    double alpha;             // used when both are null
    int64_t B;
    int k;
    int runs_per_sub;         // collision step: runs of each subspace per batch (power of two)
    int tgroups;              // collision step: tile groups per query (1..P), one block each
    const int *nq_dev;        // if set: the batch size is read here and this pass takes
    int q_base;               //   queries [q_base, q_base + nq) of it (nq is the capacity)
    // workspace
    uint16_t *cells;          // [nq][ns][K]
    int32_t *ncells;          // [nq][ns]
    int32_t *aprime;          // [nq][ns]
    float *feat;              // [nq][2ns] or null
    uint32_t *hist;           // [nq][P][ns+2] tile counts of score >= t
    uint16_t *lvl;            // [nq][P][TILE] non-zero-score tile-local ids by level (the levels the
                              //   selection can no longer take are left out)
    uint8_t *scores;          // [nq][P*TILE] dense scores, or null
    uint32_t *cand;           // [nq][B]
    const float *Dext;        // [nq][2ns][sqrt_k] centre distances computed elsewhere, or null
    const int32_t *order;     // [nq] order in which the collision step takes the queries, or null
    int32_t *order_out;       // [nq] written by the ordering kernel
    int32_t *route;           // [nq] 0: scored and selected by the sparse step; 1: by the tiled
                              //   steps; null: no sparse step (every query takes the tiled steps)
    int32_t *tlist;           // [nq] with route: the queries the sparse step leaves to the tiled
    int32_t *ntl;             //   steps, and their count (zeroed by the kernel before the sparse step)
    int sp_cap;               // sparse step: ids per round (LDS)
};

struct RerankPass {
    const float *X;
    const uint8_t *X8;        // byte copy of X, or null
    const float *Q;
    const uint32_t *cand;     // [nq][B]
    int64_t B;
    int64_t n;                // points in X
    int d, k, nq;
    int parts;                // work-groups per query
    const int *nq_dev;        // as in QueryPass
    int q_base;
    int64_t rows_per_part;
    const int32_t *rows_dev;  // [nq] candidates per query (<= B), or null for B
    int G;                    // lanes per row (power of two)
    int U;                    // float4 slices per lane
    int metric;               // 0: squared Euclidean, Euclidean result; 1: Manhattan
    uint64_t *part_keys;      // [nq][parts][k] (squared distance bits << 32 | id)
    int32_t *ids;             // [nq][k]
    float *dists;             // [nq][k]
};

// Launchers (query_kernels.hip)
int collide_static_lds();   // bytes of LDS the collision kernel declares statically
int sparse_static_lds();    // the same for the sparse collision kernel

// A kernel with its launch shape: the same plan serves a direct launch and a graph node.
struct Launch {
    const void *func = nullptr;
    dim3 grid, block;
    size_t lds = 0;
};
// The activation step runs as a persistent grid of at most this many blocks
// (one block per (query, subspace) item otherwise spends its time in dispatch).
constexpr int kActivateGrid = 8192;
Launch plan_activate(const QueryPass &p, int cap);
Launch plan_collide(const QueryPass &p, int cap);
Launch plan_collide_sparse(const QueryPass &p, int cap);
// Points in the given activated cells per (query, subspace), for the sparse
// step when the cells come from the caller.
struct SizesPass {
    IndexView ix;
    const uint16_t *cells;    // [nq][ns][K]
    const int32_t *ncells;    // [nq][ns]
    int nq;
    int32_t *aprime;          // [nq][ns]
    int32_t *ntl;             // count of the tiled list, zeroed here, or null
};
Launch plan_cell_points(const SizesPass &p);
constexpr int kOrderMax = 1024;   // largest pass the ordering kernel sorts
constexpr int kOrderWide = 16384; // largest pass the bucketed ordering kernel takes
Launch plan_order(const QueryPass &p);
Launch plan_select(const QueryPass &p, int cap);
Launch plan_rerank(const RerankPass &r, int cap);
Launch plan_merge(const RerankPass &r, int cap);
hipError_t launch(const Launch &L, void *arg, hipStream_t s);
hipError_t launch_activate(const QueryPass &p, hipStream_t s);
hipError_t launch_collide(const QueryPass &p, hipStream_t s);
hipError_t launch_select(const QueryPass &p, hipStream_t s);
hipError_t launch_rerank(const RerankPass &r, hipStream_t s);
hipError_t launch_merge(const RerankPass &r, hipStream_t s);
hipError_t launch_check_bytes(const float *X, int64_t m, int *bad, hipStream_t s);
hipError_t launch_to_bytes(const float *X, int64_t m, uint8_t *X8, hipStream_t s);

// The learned-budget network (mlp.hip): parameter views and per-pass arguments.
struct MlpView {
    int n_in, H;
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    const float *mu, *sigma;
};
struct FeatPass {
    IndexView ix;
    const float *Q;
    int nq;
    const int *nq_dev;        // if set, the number of queries is read here
    float *F;                 // [nq][2ns+1]
};
struct InferPass {
    MlpView w;                // BF16-rounded weights
    const float *F;
    int m;
    const int *m_dev;         // if set, the number of rows is read here
    float scale, amin, amax;
    float *y;                 // [m] log-alpha predictions or null
    float *alpha;             // [m] or null
    double *alpha64;          // [m] or null
};
Launch plan_features(const IndexView &ix, int nq_cap);
Launch plan_mlp_infer(int m_cap);
Launch plan_learned_alpha(const IndexView &ix, int wmax, int nq_cap);   // features and inference fused (args: FeatPass,
                                                                        // InferPass); wmax: widest half

// BF16 split precision (bf16.hip).
struct CentreBf16Pass {
    const float *Q;           // [nq][d]
    int nq, d, sk, nh;        // nh = 2 n_s halves
    const HalfDims *halves;   // [nh]
    const uint16_t *centb;    // BF16 centres, layout of IndexView::cent
    const float *cnorm2;      // [nh][sk] squared norms of the BF16 centres
    float *D;                 // [nq][nh][sk]
};
struct Bf16RerankPass {
    const uint16_t *Xb;       // [n][d] BF16 copy of X
    const float *xerr;        // [n] upper bound of |bf16(x) - x| per row
    const float *Q;
    const uint32_t *cand;     // [nq][B]
    int64_t B, n;
    int d, k, nq, parts;
    int64_t rows_per_part;
    int G, U;                 // lanes per row, 16-byte slices (8 values) per lane
    uint64_t *part_keys;      // [nq][parts][k] upper-bound keys
    float *lo;                // [nq][B] lower bounds
    uint32_t *surv;           // [nq][B] survivors, first nsurv[q] valid
    int32_t *nsurv;           // [nq]
};
struct RelErrPass {
    const float *X, *Q;
    const int32_t *ids;
    const float *dists;
    int64_t n;
    int nq, d, k;
    double *relerr;           // [nq][k]
};
constexpr int kMaxU16 = 4;    // BF16 slices of 8 values per lane in the first pass
Launch plan_centre_dists_bf16(const CentreBf16Pass &p);
Launch plan_rerank_bf16(const Bf16RerankPass &r, int cap);
Launch plan_survivors(const Bf16RerankPass &r);
Launch plan_relerr(const RelErrPass &r);
hipError_t launch_bf16_rows(const float *X, int64_t n, int d, uint16_t *Xb, float *xerr, hipStream_t s);
hipError_t launch_bf16_centres(const float *cent, const HalfDims *halves, int nh, int sk, int d, uint16_t *centb,
                               float *cnorm2, hipStream_t s);

// Launchers (build_kernels.hip)
struct KmeansPass {
    const float *X;
    int64_t n;
    int d, ns, sk, nb;        // nb = blocks of 256 points
    int wmax;                 // widest half
    const HalfDims *halves;   // [2ns]
    double *cent64;           // [sk*d] half g at sk*dim0[g]
    uint8_t *assign;          // [2ns][n]
    uint32_t *bh;             // [2ns][nb][sk]  block histograms, then block offsets
    uint32_t *cbase;          // [2ns][sk+1]    cluster starts
    uint32_t *order;          // [2ns][n]       point ids grouped by cluster, ascending
    int metric;               // 0: k-means (squared L2, means); 1: k-medians (L1, lower medians)
    int16_t hsel[2 * kMaxNs]; // assignment launches: the halves of one width, grid.y indexes them
};
hipError_t launch_gather_rows(const float *X, int d, const int64_t *ids, int m, int dim0, int w,
                              float *out, hipStream_t s);
hipError_t launch_km_assign(const KmeansPass &k, const HalfDims *halves_h, bool with_hist, hipStream_t s);
hipError_t launch_km_scan(const KmeansPass &k, hipStream_t s);
hipError_t launch_km_scatter(const KmeansPass &k, hipStream_t s);
hipError_t launch_km_update(const KmeansPass &k, hipStream_t s);
hipError_t launch_km_median(const KmeansPass &k, hipStream_t s);
hipError_t launch_cent_to_f32(const double *c64, float *c32, int64_t m, hipStream_t s);
hipError_t launch_imi_build(const uint8_t *assign, int64_t n, int ns, int sk, int P, int TILE,
                            uint32_t *toffs, uint16_t *ids16, uint32_t *csize, hipStream_t s);
hipError_t launch_cell_major(const uint32_t *toffs, const uint16_t *ids16, const uint32_t *csize, int64_t n,
                             int ns, int K, int P, int TILE, uint32_t *coffs, uint32_t *ids32, hipStream_t s);
hipError_t launch_cell_buckets(const uint32_t *coffs, const uint32_t *ids32, int64_t n, int ns, int K, int NB,
                               uint16_t *cbh, hipStream_t s);

}  // namespace suco
