/*
 * SuCo FP64 oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of the SuCo method
 * (Subspace Collision, arXiv 2411.14754).  It is the parity judge for the
 * GPU library and the timed CPU baseline; no product code may load it.
 * It shares no code, header or table with the GPU path.
 *
 * All arithmetic is FP64: FP32 inputs are promoted exactly.  Every function
 * names the passage of the paper it follows.  Readings where the paper is
 * silent or ambiguous (see the list in the design notes) are marked READING.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -shared -fPIC
 * (-ffp-contract=off keeps every a*b+c as two rounded operations, so the
 *  arithmetic is exactly what the source says.)
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Counts A and B.  Alg. 3 stops once the retrieved points reach alpha*n;    */
/* Alg. 1 and Alg. 4 take the first beta*n points of the score order.        */
/* READING: A = ceil(alpha*n), B = floor(beta*n), both in FP64 with a 1e-9   */
/* guard against representation error (0.03*1e6 is 30000.000000000004),     */
/* A >= 1, and B raised to k so that a top-k of the candidates exists.       */
/* ------------------------------------------------------------------------ */
#define SO_SUM_GROUP 256   /* members per group of the k-means update's sums */

EXPORT int64_t so_count_A(double alpha, int64_t n) {
    int64_t a = (int64_t)ceil(alpha * (double)n - 1e-9);
    if (a < 1) a = 1;
    if (a > n) a = n;
    return a;
}

EXPORT int64_t so_count_B(double beta, int64_t n, int k) {
    int64_t b = (int64_t)floor(beta * (double)n + 1e-9);
    if (b < k) b = k;
    if (b > n) b = n;
    return b;
}

/* ------------------------------------------------------------------------ */
/* Subspace division (Sec. 3.2 contiguous division, a special case of        */
/* Def. 3; the last subspace takes the remaining dimensions) and the split   */
/* of each subspace into the two halves Alg. 2 clusters separately.         */
/* READING: half 1 = first floor(s_i/2) dims, half 2 = the rest.            */
/* Output: for half g = 2*i + h, its first dim and its width.               */
/* ------------------------------------------------------------------------ */
EXPORT void so_layout(int d, int ns, int *dim0, int *width) {
    int s = d / ns;
    for (int i = 0; i < ns; ++i) {
        int start = i * s;
        int si = (i == ns - 1) ? d - (ns - 1) * s : s;
        int h1 = si / 2;
        dim0[2 * i] = start;
        width[2 * i] = h1;
        dim0[2 * i + 1] = start + h1;
        width[2 * i + 1] = si - h1;
    }
}

/* ------------------------------------------------------------------------ */
/* k-means initial centres.  The paper calls Kmeans(D, sqrtK, t) without     */
/* saying how it starts.  READING: SplitMix64 (Steele, Lea, Flood, OOPSLA    */
/* 2014) in counter form draws row ids; the first sqrtK rows whose half-     */
/* vectors are pairwise distinct become the initial centres.  After          */
/* 16*sqrtK + 1024 draws, remaining slots accept any drawn row.              */
/* ------------------------------------------------------------------------ */
static uint64_t splitmix64_at(uint64_t base, uint64_t m) {
    uint64_t z = base + (m + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

EXPORT void so_init_ids(const float *X, int64_t n, int d, int dim0, int w, int sk,
                        uint64_t seed, int g, int64_t *ids) {
    uint64_t base = seed ^ (0x632BE59BD9B4E019ULL * (uint64_t)(g + 1));
    int got = 0;
    int64_t limit = 16LL * sk + 1024;
    for (int64_t m = 0; got < sk; ++m) {
        int64_t id = (int64_t)(splitmix64_at(base, (uint64_t)m) % (uint64_t)n);
        int ok = 1;
        if (m < limit) {
            for (int c = 0; c < got && ok; ++c) {
                int same = 1;
                for (int j = 0; j < w; ++j)
                    if (X[ids[c] * d + dim0 + j] != X[id * d + dim0 + j]) { same = 0; break; }
                if (same) ok = 0;
            }
        }
        if (ok) ids[got++] = id;
    }
}

/* Distance of row p's half (dims dim0..dim0+w) to centre c, summed in
 * dimension order: the squared Euclidean distance (metric 0) or the
 * Manhattan distance (metric 1, SuCo-L1 of Sec. 5.3). */
static double half_dist(const float *X, int d, int64_t p, int dim0, int w, const double *c, int metric) {
    double s = 0.0;
    for (int j = 0; j < w; ++j) {
        double t = (double)X[p * d + dim0 + j] - c[j];
        s += metric ? fabs(t) : t * t;
    }
    return s;
}

static int nearest_centre(const float *X, int d, int64_t p, int dim0, int w,
                          const double *cent, int sk, int metric, double *best_out) {
    int best = 0;
    double bd = half_dist(X, d, p, dim0, w, cent, metric);
    for (int c = 1; c < sk; ++c) {
        double t = half_dist(X, d, p, dim0, w, cent + (int64_t)c * w, metric);
        if (t < bd) { bd = t; best = c; }   /* ties keep the lowest centre id */
    }
    *best_out = bd;
    return best;
}

/* ------------------------------------------------------------------------ */
/* Lloyd's k-means on one half (Alg. 2, the two Kmeans calls).              */
/* READING: t fixed iterations of {assign to nearest centre (ties -> lowest  */
/* id), recompute each centre as the FP64 mean of its members; an empty      */
/* cluster keeps its centre}, then one final assignment against the final   */
/* centres.  obj[it] = sum of squared distances at the it-th assignment      */
/* (it = 0..iters, the last one being the final pass).  READING (summation   */
/* order, which Alg. 2 leaves open): a cluster's members in ascending id     */
/* are taken in groups of SO_SUM_GROUP; each group is summed in order from   */
/* zero, and the group sums are added in order.                              */
/* ------------------------------------------------------------------------ */
EXPORT int so_kmeans(const float *X, int64_t n, int d, int dim0, int w, int sk, int iters,
                     const int64_t *init_ids, double *cent, int32_t *assign, double *obj,
                     int nthreads) {
    for (int c = 0; c < sk; ++c)
        for (int j = 0; j < w; ++j)
            cent[(int64_t)c * w + j] = (double)X[init_ids[c] * d + dim0 + j];
    double *sum = (double *)malloc(sizeof(double) * (size_t)sk * w);
    double *gsum = (double *)malloc(sizeof(double) * (size_t)sk * w);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)sk);
    double *md = (double *)malloc(sizeof(double) * (size_t)n);
    if (!sum || !gsum || !cnt || !md) { free(sum); free(gsum); free(cnt); free(md); return -2; }
    if (nthreads < 1) nthreads = 1;
    for (int it = 0; it <= iters; ++it) {
        /* assignment step: each point independently (order-free) */
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int64_t p = 0; p < n; ++p) assign[p] = nearest_centre(X, d, p, dim0, w, cent, sk, 0, &md[p]);
        double o = 0.0;
        for (int64_t p = 0; p < n; ++p) o += md[p];
        if (obj) obj[it] = o;
        if (it == iters) break;
        /* update step: members in id order, summed group by group */
        memset(sum, 0, sizeof(double) * (size_t)sk * w);
        memset(gsum, 0, sizeof(double) * (size_t)sk * w);
        memset(cnt, 0, sizeof(int64_t) * (size_t)sk);
        for (int64_t p = 0; p < n; ++p) {
            int a = assign[p];
            for (int j = 0; j < w; ++j) gsum[(int64_t)a * w + j] += (double)X[p * d + dim0 + j];
            cnt[a] += 1;
            if (cnt[a] % SO_SUM_GROUP == 0)                    /* a group is complete */
                for (int j = 0; j < w; ++j) {
                    sum[(int64_t)a * w + j] += gsum[(int64_t)a * w + j];
                    gsum[(int64_t)a * w + j] = 0.0;
                }
        }
        for (int c = 0; c < sk; ++c)
            if (cnt[c] > 0)
                for (int j = 0; j < w; ++j) {
                    if (cnt[c] % SO_SUM_GROUP) sum[(int64_t)c * w + j] += gsum[(int64_t)c * w + j];
                    cent[(int64_t)c * w + j] = sum[(int64_t)c * w + j] / (double)cnt[c];
                }
    }
    free(sum); free(gsum); free(cnt); free(md);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The clustering of SuCo-L1 (Sec. 5.3 only says the distance measure        */
/* changes).  READING: k-medians, Lloyd's iteration under the Manhattan      */
/* distance: the same initial centres and t iterations of {assign to the    */
/* nearest centre by L1 (ties -> lowest id), replace each coordinate of a    */
/* centre by the lower median of its members' values (the ceil(m/2)-th       */
/* smallest of m, which minimises the sum of absolute deviations); an empty  */
/* cluster keeps its centre}, then one final assignment.  obj[it] = the sum  */
/* of L1 distances at the it-th assignment (non-increasing).                 */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

EXPORT int so_kmedians(const float *X, int64_t n, int d, int dim0, int w, int sk, int iters,
                       const int64_t *init_ids, double *cent, int32_t *assign, double *obj, int nthreads) {
    for (int c = 0; c < sk; ++c)
        for (int j = 0; j < w; ++j)
            cent[(int64_t)c * w + j] = (double)X[init_ids[c] * d + dim0 + j];
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(sk + 1));
    int64_t *mem = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *md = (double *)malloc(sizeof(double) * (size_t)n);
    double *vals = (double *)malloc(sizeof(double) * (size_t)n);
    if (!cnt || !mem || !md || !vals) { free(cnt); free(mem); free(md); free(vals); return -2; }
    if (nthreads < 1) nthreads = 1;
    for (int it = 0; it <= iters; ++it) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int64_t p = 0; p < n; ++p) assign[p] = nearest_centre(X, d, p, dim0, w, cent, sk, 1, &md[p]);
        double o = 0.0;
        for (int64_t p = 0; p < n; ++p) o += md[p];
        if (obj) obj[it] = o;
        if (it == iters) break;
        /* members of every cluster, grouped by cluster */
        memset(cnt, 0, sizeof(int64_t) * (size_t)(sk + 1));
        for (int64_t p = 0; p < n; ++p) cnt[assign[p] + 1] += 1;
        for (int c = 0; c < sk; ++c) cnt[c + 1] += cnt[c];
        {
            int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)sk);
            memcpy(fill, cnt, sizeof(int64_t) * (size_t)sk);
            for (int64_t p = 0; p < n; ++p) mem[fill[assign[p]]++] = p;
            free(fill);
        }
        for (int c = 0; c < sk; ++c) {
            int64_t m = cnt[c + 1] - cnt[c];
            if (m == 0) continue;
            for (int j = 0; j < w; ++j) {
                for (int64_t t = 0; t < m; ++t) vals[t] = (double)X[mem[cnt[c] + t] * d + dim0 + j];
                qsort(vals, (size_t)m, sizeof(double), cmp_double);
                cent[(int64_t)c * w + j] = vals[(m - 1) / 2];
            }
        }
    }
    free(cnt); free(mem); free(md); free(vals);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Create Index (Alg. 2): for every subspace, k-means on both halves.        */
/* Outputs the FP64 centres, their single rounding to FP32 (the canonical    */
/* index the queries read) and the assignments [2*ns][n].                    */
/* Centres are packed half after half: half g occupies sk*width[g] values    */
/* starting at sk*dim0[g].                                                   */
/* ------------------------------------------------------------------------ */
EXPORT int so_build_metric(const float *X, int64_t n, int d, int ns, int sk, int iters, uint64_t seed,
                           int metric, double *cent64, float *cent32, int32_t *assign,
                           double *obj /*[2ns][iters+1]*/, int nthreads) {
    int *dim0 = (int *)malloc(sizeof(int) * 2 * ns), *wd = (int *)malloc(sizeof(int) * 2 * ns);
    int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * sk);
    if (!dim0 || !wd || !ids) return -2;
    so_layout(d, ns, dim0, wd);
    int rc = 0;
    for (int g = 0; g < 2 * ns && rc == 0; ++g) {
        so_init_ids(X, n, d, dim0[g], wd[g], sk, seed, g, ids);
        double *cg = cent64 + (int64_t)sk * dim0[g];
        if (metric)
            rc = so_kmedians(X, n, d, dim0[g], wd[g], sk, iters, ids, cg, assign + (int64_t)g * n,
                             obj ? obj + (int64_t)g * (iters + 1) : NULL, nthreads);
        else
            rc = so_kmeans(X, n, d, dim0[g], wd[g], sk, iters, ids, cg, assign + (int64_t)g * n,
                           obj ? obj + (int64_t)g * (iters + 1) : NULL, nthreads);
        for (int64_t t = 0; t < (int64_t)sk * wd[g]; ++t) cent32[(int64_t)sk * dim0[g] + t] = (float)cg[t];
    }
    free(dim0); free(wd); free(ids);
    return rc;
}

EXPORT int so_build(const float *X, int64_t n, int d, int ns, int sk, int iters, uint64_t seed,
                    double *cent64, float *cent32, int32_t *assign, double *obj, int nthreads) {
    return so_build_metric(X, n, d, ns, sk, iters, seed, 0, cent64, cent32, assign, obj, nthreads);
}

/* ------------------------------------------------------------------------ */
/* The oracle's index object: the data, the FP32 centres, the assignments   */
/* and one IMI per subspace (Alg. 2, the loop appending j to                */
/* IMI_i[a1(j), a2(j)]): cell = a1*sqrtK + a2, member ids in ascending order.*/
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* BF16 model (not in the paper; the split-precision form).  BF16 keeps 8    */
/* significant bits (1 implicit + 7 stored) and the FP32 exponent range.     */
/* Rounding to nearest, ties to even, done arithmetically: scale the value   */
/* so that its 8 significant bits form the integer part, round that with     */
/* nearbyint (ties to even in the default rounding mode), scale back.  Below */
/* 2^-126 the grid is that of BF16 subnormals, spacing 2^-133.  Results past */
/* the largest BF16 value round to infinity; inf and nan pass through.       */
/* ------------------------------------------------------------------------ */
EXPORT double so_bf16(float x) {
    double v = (double)x;
    if (isnan(v) || isinf(v) || v == 0.0) return v;
    int e;
    (void)frexp(v, &e);                 /* v = m * 2^e, 0.5 <= |m| < 1 */
    if (e - 1 < -126) e = -125;         /* subnormal grid: spacing 2^-133 */
    double step = ldexp(1.0, e - 8);    /* 8 significant bits above it */
    double r = nearbyint(v / step) * step;
    return (double)(float)r;            /* exact, or +-inf past the BF16 range */
}

EXPORT void so_bf16_round(const float *x, int64_t m, float *out) {
    for (int64_t t = 0; t < m; ++t) out[t] = (float)so_bf16(x[t]);
}

typedef struct {
    const float *X;
    int64_t n;
    int d, ns, sk, K;
    int *dim0, *wd;
    float *cent;       /* [sk*d] packed per half */
    int64_t *offs;     /* [ns][K+1] */
    int32_t *ids;      /* [ns][n]   */
    int s1_bf16;       /* centre distances from BF16-rounded values (model) */
    int metric;        /* 0: squared Euclidean keys, Euclidean result; 1: Manhattan (SuCo-L1) */
} so_index;

EXPORT so_index *so_index_create(const float *X, int64_t n, int d, int ns, int sk,
                                 const float *cent32, const int32_t *assign) {
    so_index *ix = (so_index *)calloc(1, sizeof(so_index));
    if (!ix) return NULL;
    ix->X = X; ix->n = n; ix->d = d; ix->ns = ns; ix->sk = sk; ix->K = sk * sk;
    ix->dim0 = (int *)malloc(sizeof(int) * 2 * ns);
    ix->wd = (int *)malloc(sizeof(int) * 2 * ns);
    ix->cent = (float *)malloc(sizeof(float) * (size_t)sk * d);
    ix->offs = (int64_t *)calloc((size_t)ns * (ix->K + 1), sizeof(int64_t));
    ix->ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)ns * n);
    if (!ix->dim0 || !ix->wd || !ix->cent || !ix->offs || !ix->ids) return NULL;
    so_layout(d, ns, ix->dim0, ix->wd);
    memcpy(ix->cent, cent32, sizeof(float) * (size_t)sk * d);
    for (int i = 0; i < ns; ++i) {
        const int32_t *a1 = assign + (int64_t)(2 * i) * n, *a2 = assign + (int64_t)(2 * i + 1) * n;
        int64_t *off = ix->offs + (int64_t)i * (ix->K + 1);
        for (int64_t j = 0; j < n; ++j) off[a1[j] * sk + a2[j] + 1] += 1;
        for (int c = 0; c < ix->K; ++c) off[c + 1] += off[c];
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ix->K);
        memcpy(fill, off, sizeof(int64_t) * ix->K);
        int32_t *ids = ix->ids + (int64_t)i * n;
        for (int64_t j = 0; j < n; ++j) ids[fill[a1[j] * sk + a2[j]]++] = (int32_t)j;
        free(fill);
    }
    return ix;
}

EXPORT void so_index_free(so_index *ix) {
    if (!ix) return;
    free(ix->dim0); free(ix->wd); free(ix->cent); free(ix->offs); free(ix->ids); free(ix);
}

EXPORT const int64_t *so_index_offs(const so_index *ix) { return ix->offs; }
EXPORT const int32_t *so_index_ids(const so_index *ix) { return ix->ids; }

/* ------------------------------------------------------------------------ */
/* Alg. 4, first loop: squared distances from the query's half g to the     */
/* sqrtK FP32 centres of that half.                                          */
/* READING: squared L2, so that dists1 + dists2 is the squared distance to   */
/* the cell's product centre.                                                */
/* ------------------------------------------------------------------------ */
EXPORT void so_centroid_dists(const so_index *ix, const float *q, int g, double *dist) {
    int w = ix->wd[g], d0 = ix->dim0[g];
    const float *cg = ix->cent + (int64_t)ix->sk * d0;
    for (int c = 0; c < ix->sk; ++c) {
        double s = 0.0;
        for (int j = 0; j < w; ++j) {
            double a = (double)q[d0 + j], b = (double)cg[(int64_t)c * w + j];
            if (ix->s1_bf16) { a = so_bf16(q[d0 + j]); b = so_bf16(cg[(int64_t)c * w + j]); }
            double t = a - b;
            s += ix->metric ? fabs(t) : t * t;
        }
        dist[c] = s;
    }
}

/* SuCo-L1 (Sec. 5.3): centre distances, keys and the re-rank by the
 * Manhattan distance.  With it, dists1 + dists2 is the L1 distance to the
 * cell's product centre (L1 is a sum over dimensions, like squared L2). */
EXPORT void so_index_set_metric(so_index *ix, int metric) { ix->metric = metric != 0; }

/* Model of the split-precision step 1 (not in the paper): the same squared
 * distances, from the query half and centres first rounded to BF16. */
EXPORT void so_index_set_s1_bf16(so_index *ix, int on) { ix->s1_bf16 = on != 0; }

/* Alg. 4, first loop: the centres of a half ordered by ascending distance.
 * READING: ties by centre id. */
static int cmp_by_dist_then_id(const void *a, const void *b, void *ctx) {
    const double *dd = (const double *)ctx;
    int x = *(const int *)a, y = *(const int *)b;
    if (dd[x] < dd[y]) return -1;
    if (dd[x] > dd[y]) return 1;
    return (x > y) - (x < y);
}
EXPORT void so_argsort(const double *dist, int sk, int *idx) {
    for (int c = 0; c < sk; ++c) idx[c] = c;
    qsort_r(idx, (size_t)sk, sizeof(int), cmp_by_dist_then_id, (void *)dist);
}

/* ------------------------------------------------------------------------ */
/* Dynamic Activation (Alg. 3) in three independent forms.                   */
/* All three visit cells in the order of the key dists1[idx1[r1]] +          */
/* dists2[idx2[r2]] and stop once the retrieved points reach A.              */
/* Output: activated cells (cell id = c1*sqrtK + c2) in retrieval order,     */
/* their count, and the number of points retrieved A' (whole cells, >= A).   */
/* ------------------------------------------------------------------------ */

/* Form 0: the retrieval order by its definition, walked row by row.  Alg. 3
 * takes cells in ascending key order (Sec. 4.2: a smaller distance sum is
 * retrieved earlier), and with the READINGS on what it leaves open (ties of
 * the argmin to the first row, an exhausted row never taken again) that order
 * is ascending (key, r1, r2).  Inside one row r1 the keys are non-decreasing
 * in r2 because the second half's distances are sorted, so each row's
 * untaken cells begin at a column pointer; the next cell of the whole order is
 * the smallest (key, r1) among the rows' pointer cells.  The walk takes it,
 * advances that row's pointer and stops once the retrieved points reach A.
 * active_trace[t], if given, is the number of first-half rows Alg. 3 has
 * activated after round t: row r + 1 joins when cell (r, 0) is retrieved, so
 * it is 1 + the rows whose column 0 is taken, at most sqrtK. */
static int64_t da_frontier(const so_index *ix, int i, const double *d1, const int *idx1,
                           const double *d2, const int *idx2, int64_t A, int32_t *cells, int64_t *ncells,
                           int32_t *active_trace) {
    int sk = ix->sk;
    const int64_t *off = ix->offs + (int64_t)i * (ix->K + 1);
    int *col = (int *)calloc((size_t)sk, sizeof(int));   /* next untaken column of each row */
    int64_t retrieved = 0, nc = 0;
    int started = 0;                                     /* rows whose column 0 is taken */
    for (;;) {
        int best = -1;
        double bkey = 0.0;
        for (int r = 0; r < sk; ++r) {
            if (col[r] == sk) continue;                  /* row exhausted */
            double key = d1[idx1[r]] + d2[idx2[col[r]]];
            if (best < 0 || key < bkey) { best = r; bkey = key; }   /* equal keys: smaller r1 */
        }
        if (best < 0) break;                             /* every cell taken */
        int cell = idx1[best] * sk + idx2[col[best]];
        if (col[best] == 0) started += 1;
        col[best] += 1;
        cells[nc++] = cell;
        retrieved += off[cell + 1] - off[cell];
        if (active_trace) active_trace[nc - 1] = started + 1 < sk ? started + 1 : sk;
        if (retrieved >= A) break;
    }
    free(col);
    *ncells = nc;
    return retrieved;
}

/* Form 1: sort all K cells by (key, r1, r2) and take the shortest prefix
 * whose total size reaches A (the paper: smaller distance sums are retrieved
 * earlier). */
typedef struct { double key; int r1, r2; } cellkey;
static int cmp_cellkey(const void *a, const void *b) {
    const cellkey *x = (const cellkey *)a, *y = (const cellkey *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    if (x->r1 != y->r1) return x->r1 < y->r1 ? -1 : 1;
    return (x->r2 > y->r2) - (x->r2 < y->r2);
}
static int64_t da_sortall(const so_index *ix, int i, const double *d1, const int *idx1,
                          const double *d2, const int *idx2, int64_t A, int32_t *cells, int64_t *ncells) {
    int sk = ix->sk, K = ix->K;
    const int64_t *off = ix->offs + (int64_t)i * (K + 1);
    cellkey *ck = (cellkey *)malloc(sizeof(cellkey) * K);
    for (int r1 = 0; r1 < sk; ++r1)
        for (int r2 = 0; r2 < sk; ++r2) {
            cellkey *e = &ck[r1 * sk + r2];
            e->key = d1[idx1[r1]] + d2[idx2[r2]];
            e->r1 = r1; e->r2 = r2;
        }
    qsort(ck, (size_t)K, sizeof(cellkey), cmp_cellkey);
    int64_t retrieved = 0, nc = 0;
    for (int t = 0; t < K; ++t) {
        int cell = idx1[ck[t].r1] * sk + idx2[ck[t].r2];
        cells[nc++] = cell;
        retrieved += off[cell + 1] - off[cell];
        if (retrieved >= A) break;
    }
    free(ck);
    *ncells = nc;
    return retrieved;
}

/* Form 2: Multi-sequence (the IMI traversal the paper compares against):
 * a priority queue over (key, r1, r2) seeded with (0,0); popping (r1,r2)
 * pushes its right and lower neighbours once each. */
typedef struct { cellkey *h; int size; } heap;
static void heap_push(heap *q, cellkey e) {
    int i = q->size++;
    q->h[i] = e;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (cmp_cellkey(&q->h[i], &q->h[p]) >= 0) break;
        cellkey t = q->h[i]; q->h[i] = q->h[p]; q->h[p] = t;
        i = p;
    }
}
static cellkey heap_pop(heap *q) {
    cellkey top = q->h[0];
    q->h[0] = q->h[--q->size];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < q->size && cmp_cellkey(&q->h[l], &q->h[m]) < 0) m = l;
        if (r < q->size && cmp_cellkey(&q->h[r], &q->h[m]) < 0) m = r;
        if (m == i) break;
        cellkey t = q->h[i]; q->h[i] = q->h[m]; q->h[m] = t;
        i = m;
    }
    return top;
}
static int64_t da_multiseq(const so_index *ix, int i, const double *d1, const int *idx1,
                           const double *d2, const int *idx2, int64_t A, int32_t *cells, int64_t *ncells) {
    int sk = ix->sk, K = ix->K;
    const int64_t *off = ix->offs + (int64_t)i * (K + 1);
    heap q;
    q.h = (cellkey *)malloc(sizeof(cellkey) * (K + 1));
    q.size = 0;
    unsigned char *pushed = (unsigned char *)calloc((size_t)K, 1);
    cellkey e0 = {d1[idx1[0]] + d2[idx2[0]], 0, 0};
    heap_push(&q, e0);
    pushed[0] = 1;
    int64_t retrieved = 0, nc = 0;
    while (q.size > 0) {
        cellkey e = heap_pop(&q);
        int cell = idx1[e.r1] * sk + idx2[e.r2];
        cells[nc++] = cell;
        retrieved += off[cell + 1] - off[cell];
        if (retrieved >= A) break;
        if (e.r1 + 1 < sk && !pushed[(e.r1 + 1) * sk + e.r2]) {
            cellkey f = {d1[idx1[e.r1 + 1]] + d2[idx2[e.r2]], e.r1 + 1, e.r2};
            heap_push(&q, f);
            pushed[(e.r1 + 1) * sk + e.r2] = 1;
        }
        if (e.r2 + 1 < sk && !pushed[e.r1 * sk + e.r2 + 1]) {
            cellkey f = {d1[idx1[e.r1]] + d2[idx2[e.r2 + 1]], e.r1, e.r2 + 1};
            heap_push(&q, f);
            pushed[e.r1 * sk + e.r2 + 1] = 1;
        }
    }
    free(q.h); free(pushed);
    *ncells = nc;
    return retrieved;
}

EXPORT int64_t so_da(const so_index *ix, int i, const double *d1, const int *idx1, const double *d2,
                     const int *idx2, int64_t A, int form, int32_t *cells, int64_t *ncells) {
    if (form == 0) return da_frontier(ix, i, d1, idx1, d2, idx2, A, cells, ncells, NULL);
    if (form == 1) return da_sortall(ix, i, d1, idx1, d2, idx2, A, cells, ncells);
    return da_multiseq(ix, i, d1, idx1, d2, idx2, A, cells, ncells);
}

/* ------------------------------------------------------------------------ */
/* Selection (Alg. 4): the points ordered by descending SC-score, the first  */
/* beta*n kept.  READING: order by (score descending, id ascending) and     */
/* keep exactly B.  Output in that order.                                    */
/* ------------------------------------------------------------------------ */
static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}
EXPORT void so_select(const uint8_t *scores, int64_t n, int64_t B, int32_t *cand) {
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) key[j] = ((uint64_t)(255 - scores[j]) << 32) | (uint64_t)j;
    qsort(key, (size_t)n, sizeof(uint64_t), cmp_u64);
    for (int64_t t = 0; t < B; ++t) cand[t] = (int32_t)(key[t] & 0xffffffffu);
    free(key);
}

/* ------------------------------------------------------------------------ */
/* Re-rank (Alg. 4 last lines): exact squared L2 of each candidate to q in   */
/* FP64, top-k by (distance, id); returns the Euclidean distance.           */
/* ------------------------------------------------------------------------ */
typedef struct { double d2; int32_t id; } distid;
static int cmp_distid(const void *a, const void *b) {
    const distid *x = (const distid *)a, *y = (const distid *)b;
    if (x->d2 < y->d2) return -1;
    if (x->d2 > y->d2) return 1;
    return (x->id > y->id) - (x->id < y->id);
}
/* Squared Euclidean (metric 0) or Manhattan (metric 1) distance of row p to
 * q; the returned distance is the Euclidean one (square root) or the
 * Manhattan one. */
static double full_dist(const float *X, int d, int64_t p, const float *q, int metric) {
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
        double t = (double)X[p * d + j] - (double)q[j];
        s += metric ? fabs(t) : t * t;
    }
    return s;
}
static double returned_dist(double v, int metric) { return metric ? v : sqrt(v); }

EXPORT void so_rerank_metric(const float *X, int d, const float *q, const int32_t *cand, int64_t B, int k,
                             int metric, int32_t *ids, double *dists) {
    distid *e = (distid *)malloc(sizeof(distid) * (size_t)B);
    for (int64_t t = 0; t < B; ++t) { e[t].id = cand[t]; e[t].d2 = full_dist(X, d, cand[t], q, metric); }
    qsort(e, (size_t)B, sizeof(distid), cmp_distid);
    for (int t = 0; t < k; ++t) { ids[t] = e[t].id; dists[t] = returned_dist(e[t].d2, metric); }
    free(e);
}
EXPORT void so_rerank(const float *X, int d, const float *q, const int32_t *cand, int64_t B, int k,
                      int32_t *ids, double *dists) {
    so_rerank_metric(X, d, q, cand, B, k, 0, ids, dists);
}

/* ------------------------------------------------------------------------ */
/* k-ANN query (Alg. 4).  alpha is per query (a constant array for the       */
/* plain method).  Optional outputs: the SC-scores [nq][n], the candidates   */
/* [nq][B] (in selection order), activated-cell counts and A' [nq][ns].      */
/* ------------------------------------------------------------------------ */
EXPORT int so_query(const so_index *ix, const float *Q, int64_t nq, int k, const double *alpha,
                    double beta, int da_form, int32_t *ids, double *dists, uint8_t *scores_out,
                    int32_t *cand_out, int64_t *ncells_out, int64_t *aprime_out, int nthreads) {
    int64_t n = ix->n;
    int ns = ix->ns, sk = ix->sk, K = ix->K, d = ix->d;
    int64_t B = so_count_B(beta, n, k);
    if (nthreads < 1) nthreads = 1;
    int rc = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; ++qi) {
        const float *q = Q + qi * d;
        int64_t A = so_count_A(alpha[qi], n);
        uint8_t *sc = (uint8_t *)calloc((size_t)n, 1);
        double *d1 = (double *)malloc(sizeof(double) * sk), *d2 = (double *)malloc(sizeof(double) * sk);
        int *i1 = (int *)malloc(sizeof(int) * sk), *i2 = (int *)malloc(sizeof(int) * sk);
        int32_t *cells = (int32_t *)malloc(sizeof(int32_t) * K);
        int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)B);
        if (!sc || !d1 || !d2 || !i1 || !i2 || !cells || !cand) { rc = -2; continue; }
        for (int i = 0; i < ns; ++i) {
            so_centroid_dists(ix, q, 2 * i, d1);
            so_centroid_dists(ix, q, 2 * i + 1, d2);
            so_argsort(d1, sk, i1);
            so_argsort(d2, sk, i2);
            int64_t nc = 0;
            int64_t ap = so_da(ix, i, d1, i1, d2, i2, A, da_form, cells, &nc);
            const int64_t *off = ix->offs + (int64_t)i * (K + 1);
            const int32_t *mem = ix->ids + (int64_t)i * n;
            for (int64_t t = 0; t < nc; ++t)                           /* counting */
                for (int64_t m = off[cells[t]]; m < off[cells[t] + 1]; ++m) sc[mem[m]] += 1;
            if (ncells_out) ncells_out[qi * ns + i] = nc;
            if (aprime_out) aprime_out[qi * ns + i] = ap;
        }
        so_select(sc, n, B, cand);
        so_rerank_metric(ix->X, d, q, cand, B, k, ix->metric, ids + qi * k, dists + qi * k);
        if (scores_out) memcpy(scores_out + qi * n, sc, (size_t)n);
        if (cand_out) memcpy(cand_out + qi * B, cand, sizeof(int32_t) * (size_t)B);
        free(sc); free(d1); free(d2); free(i1); free(i2); free(cells); free(cand);
    }
    return rc;
}

/* Form 0, also reporting after each retrieval round how many rows of the
 * first half Alg. 3 has activated (the running example of Fig. 5). */
EXPORT int64_t so_da_trace(const so_index *ix, int i, const double *d1, const int *idx1,
                                   const double *d2, const int *idx2, int64_t A, int32_t *cells,
                                   int64_t *ncells, int32_t *active_trace) {
    return da_frontier(ix, i, d1, idx1, d2, idx2, A, cells, ncells, active_trace);
}

/* Activated cells of one query in one subspace, exposed for stage tests. */
EXPORT int64_t so_query_cells(const so_index *ix, const float *q, int i, double alpha, int da_form,
                              int32_t *cells, int64_t *ncells, double *d1, double *d2, int *i1, int *i2) {
    int sk = ix->sk;
    so_centroid_dists(ix, q, 2 * i, d1);
    so_centroid_dists(ix, q, 2 * i + 1, d2);
    so_argsort(d1, sk, i1);
    so_argsort(d2, sk, i2);
    return so_da(ix, i, d1, i1, d2, i2, so_count_A(alpha, ix->n), da_form, cells, ncells);
}

/* ------------------------------------------------------------------------ */
/* SC-Linear (Alg. 1): per subspace, exact subspace distances to all n      */
/* points, the A nearest collide (READING: order by (distance, id)); then   */
/* the same selection and re-rank.                                           */
/* ------------------------------------------------------------------------ */
EXPORT int so_sclinear_metric(const float *X, int64_t n, int d, int ns, const float *Q, int64_t nq, int k,
                              double alpha, double beta, int metric, int32_t *ids, double *dists,
                              uint8_t *scores_out, int nthreads) {
    int *dim0 = (int *)malloc(sizeof(int) * 2 * ns), *wd = (int *)malloc(sizeof(int) * 2 * ns);
    so_layout(d, ns, dim0, wd);
    int64_t A = so_count_A(alpha, n), B = so_count_B(beta, n, k);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; ++qi) {
        const float *q = Q + qi * d;
        uint8_t *sc = (uint8_t *)calloc((size_t)n, 1);
        distid *e = (distid *)malloc(sizeof(distid) * (size_t)n);
        int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)B);
        for (int i = 0; i < ns; ++i) {
            int s0 = dim0[2 * i], sw = wd[2 * i] + wd[2 * i + 1];
            for (int64_t p = 0; p < n; ++p) {
                double s = 0.0;
                for (int j = 0; j < sw; ++j) {
                    double t = (double)X[p * d + s0 + j] - (double)q[s0 + j];
                    s += metric ? fabs(t) : t * t;
                }
                e[p].d2 = s; e[p].id = (int32_t)p;
            }
            qsort(e, (size_t)n, sizeof(distid), cmp_distid);
            for (int64_t z = 0; z < A; ++z) sc[e[z].id] += 1;
        }
        so_select(sc, n, B, cand);
        so_rerank_metric(X, d, q, cand, B, k, metric, ids + qi * k, dists + qi * k);
        if (scores_out) memcpy(scores_out + qi * n, sc, (size_t)n);
        free(sc); free(e); free(cand);
    }
    free(dim0); free(wd);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact k-NN by (squared distance, id) -- the problem statement (Sec. 1).   */
/* ------------------------------------------------------------------------ */
EXPORT int so_bruteforce_metric(const float *X, int64_t n, int d, const float *Q, int64_t nq, int k,
                                int metric, int32_t *ids, double *dists, int nthreads) {
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; ++qi) {
        distid *e = (distid *)malloc(sizeof(distid) * (size_t)n);
        for (int64_t p = 0; p < n; ++p) { e[p].id = (int32_t)p; e[p].d2 = full_dist(X, d, p, Q + qi * d, metric); }
        qsort(e, (size_t)n, sizeof(distid), cmp_distid);
        for (int t = 0; t < k; ++t) { ids[qi * k + t] = e[t].id; dists[qi * k + t] = returned_dist(e[t].d2, metric); }
        free(e);
    }
    return 0;
}
EXPORT int so_bruteforce(const float *X, int64_t n, int d, const float *Q, int64_t nq, int k,
                         int32_t *ids, double *dists, int nthreads) {
    return so_bruteforce_metric(X, n, d, Q, nq, k, 0, ids, dists, nthreads);
}
