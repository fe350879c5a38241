// gfx950 kernels of the SuCo query path (k-ANN Query, Alg. 4, with Dynamic
// Activation, Alg. 3).  One pass over a chunk of queries is four launches:
//
//   activate  one wave-group per (query, subspace): centre distances of both
//             halves, their ranks, and the activated cell set (Alg. 4 first
//             loop body and Alg. 3)
//   collide   one work-group per (query, id tile): SC-scores of the tile's
//             points counted in LDS (Alg. 4 counting loops), per-tile
//             histogram of scores
//   select    one work-group per (query, id tile): global score threshold
//             from the tile histograms, stable compaction of the candidates
//             (Alg. 4 "sort SC_scores", first beta*n)
//   rerank    gathered FP32 distances of the candidates with per-wave top-k
//             lists, then a per-query merge (Alg. 4 last lines)
#include <hip/hip_runtime.h>

#include "suco_impl.h"

namespace suco {

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    uint32_t lo = __shfl((uint32_t)v, src, kWave);
    uint32_t hi = __shfl((uint32_t)(v >> 32), src, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d) {
    uint32_t lo = __shfl_up((uint32_t)v, d, kWave);
    uint32_t hi = __shfl_up((uint32_t)(v >> 32), d, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// Sum over the block; every thread gets the total.
template <int NT>
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *red) {
    v = wave_sum(v);
    if constexpr (NT == kWave) {
        return v;
    } else {
        __syncthreads();
        if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
        __syncthreads();
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < NT / kWave; ++j) s += red[j];
        return s;
    }
}

// Exclusive prefix over threads in index order; *total gets the block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *red, uint32_t *total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == kWave - 1) red[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int j = 0; j < NT / kWave; ++j) {
        uint32_t r = red[j];
        base += (j < w) ? r : 0u;
        tot += r;
    }
    *total = tot;
    return base + x - v;
}

// A = max(1, ceil(alpha*n - 1e-9)), capped at n, in FP64 without contraction.
__device__ __forceinline__ uint32_t count_A_dev(double alpha, int64_t n) {
#pragma clang fp contract(off)
    double prod = alpha * (double)n;
    double v = ceil(prod - 1e-9);
    int64_t a = (int64_t)v;
    if (a < 1) a = 1;
    if (a > n) a = n;
    return (uint32_t)a;
}

// ============================================================== activate ==
// Block of NT threads (NT >= sqrt_k) per (query, subspace).
//
// The cells of subspace i form a sqrt_k x sqrt_k grid indexed by the ranks
// (r1, r2) of their two centres.  Alg. 3 retrieves them in ascending order of
// key = D1s[r1] + D2s[r2] (ties by r1, then r2) and stops at the first cell
// that brings the retrieved count to A.  Because D1s and D2s are sorted and
// rounded addition is monotone, the cells with key <= v form a staircase: in
// row r1 they are the first cnt(r1, v) columns.  With per-row prefix sums of
// cell sizes, W(v) = sum_r1 P[r1][cnt(r1, v)] is the number of points in
// cells of key <= v.  A bisection over the bit pattern of v (monotone for
// non-negative floats) finds the smallest key value v* with W(v*) >= A; all
// cells with key < v* are taken, and among the cells with key == v* the
// first ones in (r1, r2) order until A is reached.  The result is exactly the
// prefix Alg. 3 retrieves, computed without a serial walk.
template <int NT>
__global__ __launch_bounds__(NT) void k_activate(QueryPass a) {
    extern __shared__ uint32_t Ptab[];          // [sk][sk+1] row prefix sums of sizes
    __shared__ float Dr[2][kMaxSqrtK];
    __shared__ float Ds[2][kMaxSqrtK];
    __shared__ int Ix[2][kMaxSqrtK];
    __shared__ uint32_t red[NT / kWave + 1];

    const int sk = a.ix.sk, K = a.ix.K, ns = a.ix.ns;
    const int ql = blockIdx.x / ns, i = blockIdx.x - ql * ns;
    const int tid = threadIdx.x;
    const float *q = a.Q + (int64_t)ql * a.ix.d;

    // centre distances of both halves (squared L2, FP32, dimension order)
    for (int t = tid; t < 2 * sk; t += NT) {
        const int h = t >= sk, c = t - h * sk;
        const HalfDims hd = a.ix.halves[2 * i + h];
        const float *cp = a.ix.cent + (int64_t)sk * hd.dim0 + (int64_t)c * hd.w;
        const float *qp = q + hd.dim0;
        float s = 0.f;
        for (int j = 0; j < hd.w; ++j) {
            const float t2 = qp[j] - cp[j];
            s = fmaf(t2, t2, s);
        }
        Dr[h][c] = s;
    }
    __syncthreads();
    // ranks: ascending distance, ties by centre id
    for (int t = tid; t < 2 * sk; t += NT) {
        const int h = t >= sk, c = t - h * sk;
        const float v = Dr[h][c];
        int r = 0;
        for (int c2 = 0; c2 < sk; ++c2) {
            const float v2 = Dr[h][c2];
            r += (v2 < v) || (v2 == v && c2 < c);
        }
        Ds[h][r] = v;
        Ix[h][r] = c;
    }
    __syncthreads();
    // cell sizes in rank order, then per-row prefix sums
    const int stride = sk + 1;
    const uint32_t *cs = a.ix.csize + (int64_t)i * K;
    for (int t = tid; t < sk * sk; t += NT) {
        const int r1 = t / sk, r2 = t - r1 * sk;
        Ptab[r1 * stride + r2 + 1] = cs[Ix[0][r1] * sk + Ix[1][r2]];
    }
    __syncthreads();
    if (tid < sk) {
        uint32_t *row = Ptab + tid * stride;
        uint32_t run = 0;
        row[0] = 0;
        for (int r2 = 1; r2 <= sk; ++r2) {
            run += row[r2];
            row[r2] = run;
        }
    }
    __syncthreads();
    if (a.feat != nullptr && tid < 2) a.feat[(int64_t)ql * 2 * ns + 2 * i + tid] = __fsqrt_rn(Ds[tid][0]);

    const uint32_t A = count_A_dev(a.alpha_q ? (double)a.alpha_q[ql] : a.alpha, a.ix.n);
    const bool row = tid < sk;
    const float d1 = row ? Ds[0][tid] : 0.f;
    const uint32_t *prow = Ptab + (row ? tid : 0) * stride;
    auto cnt = [&](float v) -> int {   // #{r2 : d1 + D2s[r2] <= v}
        int lo2 = 0, hi2 = sk;
        while (lo2 < hi2) {
            const int m = (lo2 + hi2) >> 1;
            if (d1 + Ds[1][m] <= v) lo2 = m + 1; else hi2 = m;
        }
        return lo2;
    };
    // W(lo) < A <= W(hi) throughout
    const float kmin = Ds[0][0] + Ds[1][0];
    const float kmax = Ds[0][sk - 1] + Ds[1][sk - 1];
    int64_t lo = (int64_t)__float_as_uint(kmin) - 1;
    int64_t hi = (int64_t)__float_as_uint(kmax);
    uint32_t Wlo = 0;
    while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const float v = __uint_as_float((uint32_t)mid);
        uint32_t w = row ? prow[cnt(v)] : 0u;
        w = block_sum<NT>(w, red);
        if (w >= A) hi = mid; else { lo = mid; Wlo = w; }
    }
    // cells with key < v* (= hi) and the tie cells with key == v*
    int cl = 0, ch = 0;
    if (row) {
        cl = lo < 0 ? 0 : cnt(__uint_as_float((uint32_t)lo));
        ch = cnt(__uint_as_float((uint32_t)hi));
    }
    const uint32_t tw = row ? prow[ch] - prow[cl] : 0u;
    const uint32_t R = A - Wlo;
    uint32_t tot;
    const uint32_t S = block_excl_scan<NT>(tw, red, &tot);
    int len = cl;
    if (row && S < R) {
        if (S + tw < R) {
            len = ch;
        } else {
            int m = cl + 1;
            while (S + prow[m] - prow[cl] < R) ++m;
            len = m;
        }
    }
    const uint32_t myw = row ? prow[len] : 0u;
    uint32_t ntot;
    const uint32_t off = block_excl_scan<NT>((uint32_t)len, red, &ntot);
    const uint32_t ap = block_sum<NT>(myw, red);
    uint16_t *out = a.cells + ((int64_t)ql * ns + i) * K;
    if (row) {
        const int c1 = Ix[0][tid] * sk;
        for (int r2 = 0; r2 < len; ++r2) out[off + r2] = (uint16_t)(c1 + Ix[1][r2]);
    }
    if (tid == 0) {
        a.ncells[ql * ns + i] = (int32_t)ntot;
        a.aprime[ql * ns + i] = (int32_t)ap;
    }
}

// =============================================================== collide ==
// Block per (query, tile).  The tile's TILE scores live in LDS as bytes packed
// in 32-bit words; each point id occurs once per subspace, so a 32-bit LDS
// atomic add of 1 << 8*(id & 3) increments exactly one byte without carry
// (scores never exceed ns <= 127).  One wave walks one activated cell's run
// of ids inside the tile (ids are stored tile-major, so the run is contiguous).
// Afterwards the block counts G[t] = #{score >= t} with 7-bit SWAR compares and
// writes the scores and the counts out.
template <int NT>
__global__ __launch_bounds__(NT) void k_collide(QueryPass a) {
    extern __shared__ uint32_t sc[];   // TILE/4 words
    __shared__ uint32_t G[kMaxNs + 2];
    const int P = a.ix.P, ns = a.ix.ns, K = a.ix.K, TILE = a.ix.TILE;
    const int p = blockIdx.x % P, ql = blockIdx.x / P;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int words = TILE >> 2;
    for (int w = tid; w < words; w += NT) sc[w] = 0u;
    for (int t = tid; t < ns + 2; t += NT) G[t] = 0u;
    __syncthreads();
    for (int i = 0; i < ns; ++i) {
        const int nc = a.ncells[ql * ns + i];
        const uint16_t *cl = a.cells + ((int64_t)ql * ns + i) * K;
        const uint32_t *to = a.ix.toffs + ((int64_t)i * P + p) * (K + 1);
        const uint16_t *idl = a.ix.ids16 + (int64_t)i * P * TILE;
        for (int j = wv; j < nc; j += NT / kWave) {
            const int c = cl[j];
            const uint32_t s = to[c], e = to[c + 1];
            for (uint32_t m = s + lane; m < e; m += kWave) {
                const uint32_t lid = idl[m];
                atomicAdd(&sc[lid >> 2], 1u << ((lid & 3u) << 3));
            }
        }
    }
    __syncthreads();
    for (int t0 = 1; t0 <= ns; t0 += 8) {
        uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = tid; w < words; w += NT) {
            const uint32_t x = sc[w];
            if (x == 0u) continue;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                c[u] += __popc((x + (0x80u - (uint32_t)(t0 + u)) * 0x01010101u) & 0x80808080u);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (t0 + u <= ns) {
                const uint32_t s = wave_sum(c[u]);
                if (lane == 0) atomicAdd(&G[t0 + u], s);
            }
        }
    }
    const int64_t t0 = (int64_t)p * TILE;
    const int64_t valid = a.ix.n - t0 < TILE ? a.ix.n - t0 : TILE;
    uint4 *dst = reinterpret_cast<uint4 *>(a.scores + ((int64_t)ql * P + p) * TILE);
    const uint4 *src = reinterpret_cast<const uint4 *>(sc);
    for (int w = tid; w < (words >> 2); w += NT) dst[w] = src[w];
    __syncthreads();
    uint32_t *h = a.hist + ((int64_t)ql * P + p) * (ns + 2);
    for (int t = tid; t < ns + 2; t += NT) h[t] = t == 0 ? (uint32_t)valid : (t == ns + 1 ? 0u : G[t]);
}

// ================================================================ select ==
// Block per (query, tile).  From all tiles' counts G_p[t] it derives the
// threshold T = max{t : sum_p G_p[t] >= B}; every point with score > T is a
// candidate, and of those with score == T the R = B - #{score > T} lowest ids
// (taken tile by tile in id order).  The block then compacts its tile in id
// order with a block-wide scan, so the candidates come out in ascending id.
template <int NT>
__global__ __launch_bounds__(NT) void k_select(QueryPass a) {
    __shared__ uint32_t Gt[kMaxNs + 2];
    __shared__ uint32_t s_T, s_taken, s_base, s_any;
    __shared__ uint32_t red_g[NT / kWave], red_e[NT / kWave];
    const int P = a.ix.P, ns = a.ix.ns, TILE = a.ix.TILE, H = ns + 2;
    const int p = blockIdx.x % P, ql = blockIdx.x / P;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const uint32_t B = (uint32_t)a.B;
    const uint32_t *hq = a.hist + (int64_t)ql * P * H;
    for (int t = tid; t < H; t += NT) {
        uint32_t s = 0;
        for (int pp = 0; pp < P; ++pp) s += hq[pp * H + t];
        Gt[t] = s;
    }
    __syncthreads();
    if (tid == 0) {
        int T = 0;
        for (int t = ns; t >= 0; --t)
            if (Gt[t] >= B) { T = t; break; }
        const uint32_t R = B - Gt[T + 1];
        uint32_t eq_before = 0, base = 0;
        for (int pp = 0; pp < p; ++pp) {
            const uint32_t E = hq[pp * H + T] - hq[pp * H + T + 1];
            const uint32_t left = R > eq_before ? R - eq_before : 0u;
            base += hq[pp * H + T + 1] + (E < left ? E : left);
            eq_before += E;
        }
        const uint32_t E = hq[p * H + T] - hq[p * H + T + 1];
        const uint32_t left = R > eq_before ? R - eq_before : 0u;
        s_taken = E < left ? E : left;
        s_T = (uint32_t)T;
        s_base = base;
        s_any = (hq[p * H + T + 1] + s_taken) > 0u;
    }
    __syncthreads();
    if (!s_any) return;
    const uint32_t T = s_T, taken = s_taken;
    const int64_t t0 = (int64_t)p * TILE;
    const int valid = (int)(a.ix.n - t0 < TILE ? a.ix.n - t0 : TILE);
    const uint8_t *src = a.scores + ((int64_t)ql * P + p) * TILE;
    uint32_t *out = a.cand + (int64_t)ql * a.B + s_base;
    uint32_t gt_carry = 0, eq_carry = 0;
    for (int r0 = 0; r0 < valid; r0 += NT * 16) {
        const int j0 = r0 + tid * 16;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (j0 < valid) v = *reinterpret_cast<const uint4 *>(src + j0);
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
        uint32_t gt = 0, eq = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint32_t b = (wd[u >> 2] >> ((u & 3) * 8)) & 0xffu;
            const bool in = j0 + u < valid;
            gt += (in && b > T);
            eq += (in && b == T);
        }
        // block exclusive scans of gt and eq
        uint32_t xg = gt, xe = eq;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t yg = __shfl_up(xg, o, kWave), ye = __shfl_up(xe, o, kWave);
            if (lane >= o) { xg += yg; xe += ye; }
        }
        __syncthreads();
        if (lane == kWave - 1) { red_g[wv] = xg; red_e[wv] = xe; }
        __syncthreads();
        uint32_t bg = 0, be = 0, tg = 0, te = 0;
#pragma unroll
        for (int j = 0; j < NT / kWave; ++j) {
            bg += j < wv ? red_g[j] : 0u;
            be += j < wv ? red_e[j] : 0u;
            tg += red_g[j];
            te += red_e[j];
        }
        uint32_t er = eq_carry + be + xe - eq;              // eq-rank of this thread's first tie
        uint32_t pos = gt_carry + bg + xg - gt + (er < taken ? er : taken);
        if (gt + eq > 0) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const uint32_t b = (wd[u >> 2] >> ((u & 3) * 8)) & 0xffu;
                if (j0 + u >= valid) continue;
                if (b > T) {
                    out[pos++] = (uint32_t)(t0 + j0 + u);
                } else if (b == T) {
                    if (er < taken) out[pos++] = (uint32_t)(t0 + j0 + u);
                    ++er;
                }
            }
        }
        gt_carry += tg;
        eq_carry += te;
    }
}

// ================================================================ rerank ==
// Block of NT threads per (query, part of the candidate list).  G lanes share
// a row: lane li of the group reads float4 slices li, li+G, ... of the row,
// accumulates (x - q)^2 with FMA in slice order, and the group reduces with
// a xor butterfly (every lane of the group ends with the same sum).  Each wave
// keeps its k best (squared distance bits << 32 | id) sorted across lanes
// 0..k-1; the waves' lists are merged at the end.  Keys order exactly by
// (distance, id) because the distances are non-negative.
__device__ __forceinline__ void topk_insert(uint64_t &best, uint64_t kk, int k, int lane) {
    const uint64_t kth = shfl64(best, k - 1);
    if (kk < kth) {
        const int pos = __popcll(__ballot(lane < k && best < kk));
        const uint64_t up = shfl_up64(best, 1);
        if (lane < k) {
            if (lane == pos) best = kk;
            else if (lane > pos) best = up;
        }
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_rerank(RerankPass r) {
    __shared__ uint64_t wl[NT / kWave][kMaxK];
    const int ql = blockIdx.x / r.parts, part = blockIdx.x - ql * r.parts;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int G = r.G, R = kWave / G, li = lane & (G - 1), slot = lane / G;
    const int d4 = r.d >> 2, k = r.k;
    float4 qr[kMaxU];
    const float4 *q4 = reinterpret_cast<const float4 *>(r.Q + (int64_t)ql * r.d);
#pragma unroll
    for (int u = 0; u < kMaxU; ++u) {
        const int j = li + G * u;
        qr[u] = (u < r.U && j < d4) ? q4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    uint64_t best = ~0ull;
    const int64_t rb = (int64_t)part * r.rows_per_part;
    const int64_t re = rb + r.rows_per_part < r.B ? rb + r.rows_per_part : r.B;
    const uint32_t *cq = r.cand + (int64_t)ql * r.B;
    for (int64_t base = rb + (int64_t)wv * R; base < re; base += (int64_t)(NT / kWave) * R) {
        const int64_t rw = base + slot;
        uint32_t id = rw < re ? cq[rw] : 0u;
        const bool valid = rw < re && id < r.n;   // ids outside [0, n) are ignored
        id = valid ? id : 0u;
        const float4 *xr = reinterpret_cast<const float4 *>(r.X + (int64_t)id * r.d);
        float acc = 0.f;
#pragma unroll
        for (int u = 0; u < kMaxU; ++u) {
            const int j = li + G * u;
            if (u < r.U && j < d4) {
                const float4 x = xr[j];
                float t;
                t = x.x - qr[u].x; acc = fmaf(t, t, acc);
                t = x.y - qr[u].y; acc = fmaf(t, t, acc);
                t = x.z - qr[u].z; acc = fmaf(t, t, acc);
                t = x.w - qr[u].w; acc = fmaf(t, t, acc);
            }
        }
        for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
        const uint64_t key = valid ? (((uint64_t)__float_as_uint(acc) << 32) | id) : ~0ull;
        for (int s = 0; s < R; ++s) topk_insert(best, shfl64(key, s * G), k, lane);
    }
    if (lane < k) wl[wv][lane] = best;
    __syncthreads();
    if (wv == 0) {
        for (int w2 = 1; w2 < NT / kWave; ++w2) {
            for (int j = 0; j < k; ++j) {
                const uint64_t kk = wl[w2][j];
                if (kk >= shfl64(best, k - 1)) break;
                topk_insert(best, kk, k, lane);
            }
        }
        if (lane < k) r.part_keys[((int64_t)ql * r.parts + part) * k + lane] = best;
    }
}

// One wave per query: merge the parts' lists, write ids and Euclidean distances.
__global__ __launch_bounds__(kWave) void k_merge(RerankPass r) {
    const int ql = blockIdx.x, lane = threadIdx.x, k = r.k;
    const uint64_t *pk = r.part_keys + (int64_t)ql * r.parts * k;
    uint64_t best = lane < k ? pk[lane] : ~0ull;
    for (int p = 1; p < r.parts; ++p) {
        const uint64_t mine = lane < k ? pk[(int64_t)p * k + lane] : ~0ull;
        for (int j = 0; j < k; ++j) {
            const uint64_t kk = shfl64(mine, j);
            if (kk >= shfl64(best, k - 1)) break;
            topk_insert(best, kk, k, lane);
        }
    }
    if (lane < k) {
        r.ids[(int64_t)ql * k + lane] = (int32_t)(uint32_t)(best & 0xffffffffu);
        // Euclidean distance: FP64 square root of the FP32 squared distance, rounded once
        r.dists[(int64_t)ql * k + lane] = (float)sqrt((double)__uint_as_float((uint32_t)(best >> 32)));
    }
}

// ============================================================= launchers ==
hipError_t launch_activate(const QueryPass &p, hipStream_t s) {
    const size_t lds = sizeof(uint32_t) * (size_t)p.ix.sk * (p.ix.sk + 1);
    const dim3 grid((unsigned)(p.nq * p.ix.ns));
    if (p.ix.sk <= 64)
        hipLaunchKernelGGL(k_activate<64>, grid, dim3(64), lds, s, p);
    else
        hipLaunchKernelGGL(k_activate<128>, grid, dim3(128), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_collide(const QueryPass &p, hipStream_t s) {
    const size_t lds = (size_t)p.ix.TILE;
    hipLaunchKernelGGL(k_collide<512>, dim3((unsigned)(p.nq * p.ix.P)), dim3(512), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_select(const QueryPass &p, hipStream_t s) {
    hipLaunchKernelGGL(k_select<256>, dim3((unsigned)(p.nq * p.ix.P)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_rerank(const RerankPass &r, hipStream_t s) {
    hipLaunchKernelGGL(k_rerank<256>, dim3((unsigned)(r.nq * r.parts)), dim3(256), 0, s, r);
    return hipGetLastError();
}

hipError_t launch_merge(const RerankPass &r, hipStream_t s) {
    hipLaunchKernelGGL(k_merge, dim3((unsigned)r.nq), dim3(kWave), 0, s, r);
    return hipGetLastError();
}

}  // namespace suco
