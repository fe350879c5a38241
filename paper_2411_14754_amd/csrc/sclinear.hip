// SC-Linear on the GPU (Alg. 1): the subspace collision framework without an
// index.  For a query and each subspace i, the A = ceil(alpha*n) points
// nearest to the query in that subspace collide (Def. 2; ties by id); a
// point's SC-score is the number of subspaces in which it collides (Def. 4);
// the B points of highest score (ties by lowest id) are re-ranked by exact
// distance.  A pass of up to C queries runs as four launches, then the
// re-rank of the index path:
//   dist    subspace distances of every (query, subspace, point), FP32, in
//           dimension order, into a [C][n_s][n] array (squared Euclidean,
//           or Manhattan on a SuCo-L1 index)
//   thresh  per (query, subspace): the key of the A-th nearest point (keys are
//           the distances' bit patterns, monotone for non-negative floats) by
//           a radix select of four 8-bit digits, and the id of the last point
//           with that key that still collides, by counting ties in id order
//   score   per (query, point): the subspaces where it collides, and the
//           query's score histogram
//   pick    per query: threshold T and the candidates in ascending id (all of
//           score > T, the lowest ids of score T)
#include "runtime_impl.h"
#include "wave.h"

namespace suco {

constexpr int kScMaxSub = 64;        // widest subspace (dimensions) the distance kernel holds in registers
constexpr int kScThreads = 1024;     // threshold and pick kernels

struct ScPass {
    const float *X, *Q;
    const HalfDims *halves;    // subspace i = halves 2i and 2i+1, contiguous
    int64_t n;
    int d, ns, C;              // C: queries in this pass
    int metric;                // 0: squared Euclidean, 1: Manhattan
    uint32_t A;                // points colliding per subspace
    int64_t B;
    float *D;                  // [C][ns][n]
    uint32_t *thr;             // [C][ns][2]: key, last colliding id among that key
    uint32_t *hist;            // [C][ns+1] points per score
    uint8_t *sc;               // [C][n] scores
    uint32_t *cand;            // [C][B]
};

// Block of 256 points and one subspace; the pass's query subspaces sit in LDS.
template <int SW>
__global__ __launch_bounds__(256) void k_sc_dist(ScPass a) {
    extern __shared__ float qs[];     // [C][sw]
    const int i = blockIdx.y;
    const int s0 = a.halves[2 * i].dim0, sw = a.halves[2 * i].w + a.halves[2 * i + 1].w;
    for (int t = threadIdx.x; t < a.C * sw; t += blockDim.x) {
        const int c = t / sw, j = t - c * sw;
        qs[t] = a.Q[(int64_t)c * a.d + s0 + j];
    }
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    float x[SW];
    const float *row = a.X + p * a.d + s0;
#pragma unroll
    for (int j = 0; j < SW; ++j) x[j] = j < sw ? row[j] : 0.f;
    for (int c = 0; c < a.C; ++c) {
        const float *q = qs + c * sw;
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < SW; ++j) {
            if (j < sw) s = dist_acc(s, x[j] - q[j], a.metric);
        }
        a.D[((int64_t)c * a.ns + i) * a.n + p] = s;
    }
}

// Block per (query, subspace).
__global__ __launch_bounds__(kScThreads) void k_sc_thresh(ScPass a) {
    __shared__ uint32_t h[kScThreads / kWave][256];
    __shared__ uint32_t red[kScThreads / kWave + 1];
    __shared__ uint32_t sel[2];
    const int item = blockIdx.x, c = item / a.ns, i = item - c * a.ns;
    const int tid = threadIdx.x, w = tid / kWave;
    const uint32_t *key = reinterpret_cast<const uint32_t *>(a.D + ((int64_t)c * a.ns + i) * a.n);
    const int64_t n = a.n;
    if (i == 0)
        for (int t = tid; t <= a.ns; t += kScThreads) a.hist[(int64_t)c * (a.ns + 1) + t] = 0u;
    uint32_t prefix = 0u, mask = 0u, kth = a.A;        // kth: 1-based rank among the keys matching prefix
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int t = tid; t < (kScThreads / kWave) * 256; t += kScThreads) (&h[0][0])[t] = 0u;
        __syncthreads();
        for (int64_t p = tid; p < n; p += kScThreads) {
            const uint32_t kv = key[p];
            if ((kv & mask) == prefix) atomicAdd(&h[w][(kv >> shift) & 255u], 1u);
        }
        __syncthreads();
        uint32_t tot = 0;
        if (tid < 256)
            for (int ww = 0; ww < kScThreads / kWave; ++ww) tot += h[ww][tid];
        uint32_t all;
        const uint32_t ex = block_excl_scan<kScThreads>(tot, red, &all);
        if (tid < 256 && ex < kth && kth <= ex + tot) {
            sel[0] = prefix | ((uint32_t)tid << shift);
            sel[1] = kth - ex;
        }
        __syncthreads();
        prefix = sel[0];
        kth = sel[1];
        mask |= 255u << shift;
        __syncthreads();
    }
    // the kth point (in id order) among those with key == prefix
    const int64_t per = (n + kScThreads - 1) / kScThreads;
    const int64_t p0 = (int64_t)tid * per < n ? (int64_t)tid * per : n, p1 = p0 + per < n ? p0 + per : n;
    uint32_t eq = 0;
    for (int64_t p = p0; p < p1; ++p) eq += key[p] == prefix;
    uint32_t all;
    const uint32_t ex = block_excl_scan<kScThreads>(eq, red, &all);
    if (ex < kth && kth <= ex + eq) {
        uint32_t r = kth - ex;
        for (int64_t p = p0; p < p1; ++p)
            if (key[p] == prefix && --r == 0u) {
                uint32_t *o = a.thr + ((int64_t)c * a.ns + i) * 2;
                o[0] = prefix;
                o[1] = (uint32_t)p;
                break;
            }
    }
}

// Block of 256 points of one query.
__global__ __launch_bounds__(256) void k_sc_score(ScPass a, uint8_t *dense) {
    __shared__ uint32_t th[2 * 128];
    __shared__ uint32_t hs[128 + 1];
    const int c = blockIdx.y, ns = a.ns;
    for (int t = threadIdx.x; t < 2 * ns; t += blockDim.x) th[t] = a.thr[(int64_t)c * ns * 2 + t];
    for (int t = threadIdx.x; t <= ns; t += blockDim.x) hs[t] = 0u;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < a.n) {
        uint32_t s = 0;
        for (int i = 0; i < ns; ++i) {
            const uint32_t kv = reinterpret_cast<const uint32_t *>(a.D)[((int64_t)c * ns + i) * a.n + p];
            s += (kv < th[2 * i] || (kv == th[2 * i] && (uint32_t)p <= th[2 * i + 1])) ? 1u : 0u;
        }
        a.sc[(int64_t)c * a.n + p] = (uint8_t)s;
        if (dense) dense[(int64_t)c * a.n + p] = (uint8_t)s;
        atomicAdd(&hs[s], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= ns; t += blockDim.x)
        if (hs[t]) atomicAdd(&a.hist[(int64_t)c * (ns + 1) + t], hs[t]);
}

// Block per query: T = max{t : #{score >= t} >= B}, then the candidates in
// ascending id, each thread a contiguous range of ids.
__global__ __launch_bounds__(kScThreads) void k_sc_pick(ScPass a) {
    __shared__ uint32_t red[kScThreads / kWave + 1];
    const int c = blockIdx.x, ns = a.ns, tid = threadIdx.x;
    const uint32_t *hq = a.hist + (int64_t)c * (ns + 1);
    const uint32_t B = (uint32_t)a.B;
    int T = 0;
    uint32_t g = 0;                       // #{score > T} once T is found
    for (int t = ns; t >= 0; --t) {
        if (g + hq[t] >= B) { T = t; break; }
        g += hq[t];
    }
    const uint32_t R = B - g;
    const uint8_t *sq = a.sc + (int64_t)c * a.n;
    const int64_t n = a.n, per = (n + kScThreads - 1) / kScThreads;
    const int64_t p0 = (int64_t)tid * per < n ? (int64_t)tid * per : n, p1 = p0 + per < n ? p0 + per : n;
    uint32_t gt = 0, eq = 0;
    for (int64_t p = p0; p < p1; ++p) {
        gt += sq[p] > T;
        eq += sq[p] == T;
    }
    uint32_t all;
    const uint32_t eb = block_excl_scan<kScThreads>(eq, red, &all);
    const uint32_t take = eb >= R ? 0u : (R - eb < eq ? R - eb : eq);
    uint32_t pos = block_excl_scan<kScThreads>(gt + take, red, &all);
    uint32_t *cq = a.cand + (int64_t)c * a.B;
    uint32_t taken = 0;
    for (int64_t p = p0; p < p1; ++p) {
        const uint32_t s = sq[p];
        if (s > (uint32_t)T || (s == (uint32_t)T && taken++ < take))
            if (pos < B) cq[pos++] = (uint32_t)p;
    }
}


namespace {

// The pass workspace: distances, thresholds, histograms, scores, candidates
// and the re-rank's partial lists.
struct ScWork {
    float *D; uint32_t *thr, *hist, *cand; uint8_t *sc; uint64_t *part_keys;
};

ScWork sc_carve(char *base, size_t C, int64_t n, int ns, int64_t B, int parts, int k, size_t *bytes) {
    Carve cv{base};
    ScWork w;
    w.D = cv.take<float>(C * ns * (size_t)n);
    w.thr = cv.take<uint32_t>(C * ns * 2);
    w.hist = cv.take<uint32_t>(C * (ns + 1));
    w.sc = cv.take<uint8_t>(C * (size_t)n);
    w.cand = cv.take<uint32_t>(C * (size_t)B);
    w.part_keys = cv.take<uint64_t>(C * (size_t)parts * k);
    if (bytes) *bytes = cv.off;
    return w;
}

}  // namespace
}  // namespace suco

using namespace suco;

extern "C" int suco_query_sclinear(const suco_index *cix, const float *Q, int64_t nq, int32_t k, double alpha,
                                   double beta, int32_t *ids, float *dists, uint8_t *scores, void *stream) {
    if (!index_ok(cix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (nq < 0) return fail(SUCO_E_INVAL, "nq must be >= 0");
    if (k < 1 || k > cix->n) return fail(SUCO_E_INVAL, "k must be in [1, n]");
    if (k > kMaxK) return fail(SUCO_E_UNSUPPORTED, "the kernels take k <= 64");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(SUCO_E_INVAL, "alpha must be in (0, 1]");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SUCO_E_INVAL, "beta must be in (0, 1]");
    if (nq > 0 && (!Q || !ids || !dists)) return fail(SUCO_E_INVAL, "Q, ids and dists must not be NULL");
    suco_index *ix = const_cast<suco_index *>(cix);
    int swmax = 0;
    for (int i = 0; i < ix->ns; ++i) swmax = std::max(swmax, ix->halves_h[2 * i].w + ix->halves_h[2 * i + 1].w);
    if (swmax > kScMaxSub) return fail(SUCO_E_UNSUPPORTED, "SC-Linear takes subspaces of at most 64 dimensions");
    if (nq == 0) return SUCO_OK;
    const int64_t n = ix->n, B = count_B_host(beta, n, k);
    RerankCfg rc32;
    int rc = rerank_cfg(ix->d, B, &rc32);
    if (rc) return rc;
    // queries per pass: the distances of a pass take at most 8 GiB, and the
    // pass's query subspaces fit the distance kernel's LDS
    const int64_t per_q = (int64_t)ix->ns * n * 4;
    const int64_t cmax = std::clamp<int64_t>((int64_t(8) << 30) / per_q, 1, std::min<int64_t>(256, 16384 / swmax));
    const int64_t C = pass_size(nq, (int)cmax);
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(ix->mu);
    DeviceGuard dg(ix->device);
    size_t bytes = 0;
    sc_carve(nullptr, (size_t)C, n, ix->ns, B, rc32.parts, k, &bytes);
    if ((rc = ensure_arena(ix, bytes))) return rc;
    if (ix->pending) HIPCHECK(hipStreamWaitEvent(st, ix->done, 0));
    ScWork w = sc_carve(ix->arena, (size_t)C, n, ix->ns, B, rc32.parts, k, nullptr);
    for (int64_t c0 = 0; c0 < nq; c0 += C) {
        const int cn = (int)std::min<int64_t>(C, nq - c0);
        ScPass a{};
        a.X = ix->X; a.Q = Q + c0 * ix->d; a.halves = ix->halves; a.n = n; a.d = ix->d; a.ns = ix->ns; a.C = cn;
        a.A = (uint32_t)count_A_host(alpha, n); a.B = B; a.metric = ix->metric;
        a.D = w.D; a.thr = w.thr; a.hist = w.hist; a.sc = w.sc; a.cand = w.cand;
        const dim3 gd((unsigned)((n + 255) / 256), (unsigned)ix->ns);
        const size_t qlds = sizeof(float) * cn * swmax;
        if (swmax <= 16) hipLaunchKernelGGL(k_sc_dist<16>, gd, dim3(256), qlds, st, a);
        else hipLaunchKernelGGL(k_sc_dist<kScMaxSub>, gd, dim3(256), qlds, st, a);
        HIPCHECK(hipGetLastError());
        hipLaunchKernelGGL(k_sc_thresh, dim3((unsigned)(cn * ix->ns)), dim3(kScThreads), 0, st, a);
        HIPCHECK(hipGetLastError());
        uint8_t *dense = scores ? scores + c0 * n : nullptr;
        hipLaunchKernelGGL(k_sc_score, dim3((unsigned)((n + 255) / 256), (unsigned)cn), dim3(256), 0, st, a, dense);
        HIPCHECK(hipGetLastError());
        hipLaunchKernelGGL(k_sc_pick, dim3((unsigned)cn), dim3(kScThreads), 0, st, a);
        HIPCHECK(hipGetLastError());
        RerankPass rp{};
        rp.X = ix->X; rp.X8 = ix->X8; rp.Q = a.Q; rp.cand = w.cand; rp.B = B; rp.n = n; rp.d = ix->d; rp.k = k;
        rp.metric = ix->metric;
        rp.nq = cn; rp.parts = rc32.parts; rp.rows_per_part = rc32.rpp; rp.G = rc32.G; rp.U = rc32.U;
        rp.part_keys = w.part_keys; rp.ids = ids + c0 * k; rp.dists = dists + c0 * k;
        HIPCHECK(launch_rerank(rp, st));
        HIPCHECK(launch_merge(rp, st));
    }
    HIPCHECK(hipEventRecord(ix->done, st));
    ix->pending = true;
    return SUCO_OK;
}
