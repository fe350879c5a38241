// gfx950 kernels of the SuCo query path (k-ANN Query, Alg. 4, with Dynamic
// Activation, Alg. 3).  One pass over a chunk of queries is these launches:
//
//   activate  one wave per (query, subspace): centre distances of both halves
//             and the activated cell set (Alg. 4 first loop body and Alg. 3),
//             by Alg. 3's walk for small budgets or a bisection over the key
//   order     one block: the pass's queries, heaviest first
//   collide   one work-group per (query, group of id tiles): SC-scores of a
//             tile's points counted in LDS (Alg. 4 counting loops), per-tile
//             histogram of scores, non-zero ids listed by score level
//   select    one work-group per query, one wave per tile: global score
//             threshold from the tile histograms, candidates in ascending id
//             (Alg. 4 selection: the first beta*n of the score order)
//   rerank    gathered distances of the candidates with per-wave top-k lists,
//   merge     then a per-query merge (Alg. 4 last lines)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "suco_impl.h"
#include "wave.h"

namespace suco {

// A = max(1, ceil(alpha*n - 1e-9)), capped at n, in FP64 without contraction.
// A per-query alpha is not validated on the host: above 1, +inf and NaN
// activate every point, and alpha <= 0 activates one.
__device__ __forceinline__ uint32_t count_A_dev(double alpha, int64_t n) {
#pragma clang fp contract(off)
    if (!(alpha <= 1.0)) return (uint32_t)n;
    if (!(alpha > 0.0)) return 1u;
    double prod = alpha * (double)n;
    double v = ceil(prod - 1e-9);
    int64_t a = (int64_t)v;
    if (a < 1) a = 1;
    if (a > n) a = n;
    return (uint32_t)a;
}

// A half's smallest centre distance as exported: Euclidean (the square root of
// the squared distance) or Manhattan.
__device__ __forceinline__ float feat_of(float v, int metric) { return metric ? v : __fsqrt_rn(v); }

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
// Small budgets (one wave, sqrt_k <= 64): Alg. 3's walk itself.  Lane c holds
// the row of first-half centre c; the second half's centres are sorted only
// as far as kWalkCols (ascending distance, ties by id), with the sizes of the
// row's cells in those columns gathered ahead.  Each step takes the smallest
// frontier key (d1 + d2 of a row's next column; equal keys go to the row of
// smaller d1, then smaller centre id, which is the rank order), so the cells
// come in exactly the order the bisection's prefix is defined by, and the walk
// stops at the cell that brings the count to A.  A row that would need a
// column past kWalkCols, or a walk longer than kWalkSteps, returns false and
// the caller takes the general path.
constexpr int kWalkCols = 12;
constexpr int kWalkSteps = 64;
constexpr int kWalkRatio = 16;   // walk when A*K <= kWalkRatio*n (about that many cells of average size)

__device__ __forceinline__ bool activate_walk(const QueryPass &a, const int ql, const int i, const float v0,
                                              const float v1, const bool live, const uint32_t A) {
    const int sk = a.ix.sk, K = a.ix.K, ns = a.ix.ns, lane = threadIdx.x;
    const uint32_t kNone = 0xffffffffu;          // above every finite non-negative float's bits
    const int ncol = sk < kWalkCols ? sk : kWalkCols;
    // the second half's first ncol centres in rank order (uniform values)
    uint32_t b1 = live ? __float_as_uint(v1) : kNone;
    float D2[kWalkCols];
    int I2[kWalkCols];
#pragma unroll
    for (int j = 0; j < kWalkCols; ++j) {
        D2[j] = 0.f;
        I2[j] = 0;
        if (j < ncol) {
            const uint32_t m = wave_min(b1);
            const int r = __ffsll((unsigned long long)__ballot(b1 == m)) - 1;
            D2[j] = __uint_as_float(m);
            I2[j] = r;
            if (lane == r) b1 = kNone;
        }
    }
    // sizes of this row's cells in those columns
    const uint32_t *cs = a.ix.csize + (int64_t)i * K;
    uint32_t sz[kWalkCols];
#pragma unroll
    for (int j = 0; j < kWalkCols; ++j) sz[j] = cs[(live ? lane * sk : 0) + I2[j]];
    const uint32_t v0b = live ? __float_as_uint(v0) : kNone;
    int ptr = 0;
    uint32_t kb = live ? __float_as_uint(v0 + D2[0]) : kNone;
    uint32_t cur = live ? sz[0] : 0u;
    uint32_t W = 0;
    for (int step = 0;; ++step) {
        if (step == kWalkSteps) return false;
        const uint32_t m = wave_min(kb);
        uint64_t cand = __ballot(kb == m);
        if (__popcll(cand) > 1) {
            const uint32_t mv = wave_min(kb == m ? v0b : kNone);
            cand = __ballot(kb == m && v0b == mv);
        }
        const int r = __ffsll((unsigned long long)cand) - 1;
        W += (uint32_t)__builtin_amdgcn_readlane((int)cur, r);
        const int np = __builtin_amdgcn_readlane(ptr, r) + 1;
        if (lane == r) ptr = np;                      // the cell is taken
        if (W >= A) break;
        if (np == ncol && ncol < sk) return false;    // its row's next column is not sorted here
        if (lane == r) {
            float d2 = D2[0];
            uint32_t c = sz[0];
#pragma unroll
            for (int j = 1; j < kWalkCols; ++j)
                if (np == j) { d2 = D2[j]; c = sz[j]; }
            kb = np < ncol ? __float_as_uint(v0 + d2) : kNone;
            cur = c;
        }
    }
    const uint32_t incl = wave_incl_scan((uint32_t)ptr);
    const uint32_t off = incl - (uint32_t)ptr;
    const uint32_t ntot = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    const uint32_t d1min = wave_min(v0b);
    uint16_t *out = a.cells + ((int64_t)ql * ns + i) * K;
#pragma unroll
    for (int j = 0; j < kWalkCols; ++j)
        if (j < ptr) out[off + j] = (uint16_t)(lane * sk + I2[j]);
    if (a.feat != nullptr && lane < 2)
        a.feat[(int64_t)ql * 2 * ns + 2 * i + lane] = feat_of(lane == 0 ? __uint_as_float(d1min) : D2[0], a.ix.metric);
    if (lane == 0) {
        a.ncells[ql * ns + i] = (int32_t)ntot;
        a.aprime[ql * ns + i] = (int32_t)W;
    }
    return true;
}

// Multi-sequence (the inverted multi-index traversal Sec. 4.2 compares
// Dynamic Activation with), for sqrt_k <= 64: a priority queue of cells
// ordered by (key, r1, r2), seeded with (0, 0); taking a cell pushes its
// neighbours (r1 + 1, r2) and (r1, r2 + 1) unless they were pushed before (a
// bitmap over the rank grid), and the traversal stops once the points taken
// reach A.  The queue is a pool of 64 x kMsSlots entries held in the wave's
// registers, (key bits << 32 | r1 << 16 | r2) with the cell's size beside
// it; taking the smallest is a wave minimum.  The queue holds at most one
// entry more than the cells taken so far, so it cannot overflow before
// 64 * kMsSlots - 1 cells are taken; a longer traversal returns false and
// the caller takes the general path, which activates the same cells.  The
// cells come out in retrieval order (Dynamic Activation's paths write them
// row by row; the sets are equal).
constexpr int kMsSlots = 8;

__device__ __forceinline__ bool activate_ms(const QueryPass &a, const int ql, const int i, const float *Ds0,
                                            const float *Ds1, const int *Ix0, const int *Ix1, const uint32_t A,
                                            uint32_t *pushed) {
    const int sk = a.ix.sk, K = a.ix.K, ns = a.ix.ns, lane = threadIdx.x;
    const uint64_t kEmpty = ~0ull;
    const uint32_t *cs = a.ix.csize + (int64_t)i * K;
    for (int w = lane; w < (K + 31) / 32; w += kWave) pushed[w] = 0u;
    __syncthreads();
    uint64_t key[kMsSlots];
    uint32_t csz[kMsSlots];
#pragma unroll
    for (int j = 0; j < kMsSlots; ++j) { key[j] = kEmpty; csz[j] = 0u; }
    auto entry = [&](int r1, int r2) -> uint64_t {
        return ((uint64_t)__float_as_uint(Ds0[r1] + Ds1[r2]) << 32) | ((uint32_t)r1 << 16) | (uint32_t)r2;
    };
    if (lane == 0) {
        key[0] = entry(0, 0);
        csz[0] = cs[Ix0[0] * sk + Ix1[0]];
        pushed[0] = 1u;
    }
    __syncthreads();
    uint16_t *out = a.cells + ((int64_t)ql * ns + i) * K;
    uint32_t W = 0;
    int nc = 0;
    for (;;) {
        uint64_t lm = key[0];
#pragma unroll
        for (int j = 1; j < kMsSlots; ++j) lm = key[j] < lm ? key[j] : lm;
        const uint32_t mh = wave_min((uint32_t)(lm >> 32));
        if (mh == 0xffffffffu) break;                            // every cell taken
        const uint32_t ml = wave_min((uint32_t)(lm >> 32) == mh ? (uint32_t)lm : 0xffffffffu);
        const uint64_t m = ((uint64_t)mh << 32) | ml;
        uint32_t sz = 0u;
        bool own = false;
#pragma unroll
        for (int j = 0; j < kMsSlots; ++j)
            if (key[j] == m) { key[j] = kEmpty; sz = csz[j]; own = true; }
        const int ol = __ffsll((unsigned long long)__ballot(own)) - 1;
        sz = (uint32_t)__builtin_amdgcn_readlane((int)sz, ol);
        const int r1 = (int)(ml >> 16), r2 = (int)(ml & 0xffffu);
        if (lane == 0) out[nc] = (uint16_t)(Ix0[r1] * sk + Ix1[r2]);
        ++nc;
        W += sz;
        if (W >= A) break;
        if (nc == kWave * kMsSlots - 1) return false;            // the pool could overflow
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int n1 = r1 + e, n2 = r2 + 1 - e;
            if (n1 >= sk || n2 >= sk) continue;
            const int c = n1 * sk + n2;
            const uint32_t word = pushed[c >> 5];
            if (word & (1u << (c & 31))) continue;
            if (lane == 0) pushed[c >> 5] = word | (1u << (c & 31));
            bool fr = false;
#pragma unroll
            for (int j = 0; j < kMsSlots; ++j) fr |= key[j] == kEmpty;
            const int fl = __ffsll((unsigned long long)__ballot(fr)) - 1;
            if (lane == fl) {
                bool placed = false;
#pragma unroll
                for (int j = 0; j < kMsSlots; ++j)
                    if (!placed && key[j] == kEmpty) {
                        key[j] = entry(n1, n2);
                        csz[j] = cs[Ix0[n1] * sk + Ix1[n2]];
                        placed = true;
                    }
            }
        }
    }
    if (a.feat != nullptr && lane < 2)
        a.feat[(int64_t)ql * 2 * ns + 2 * i + lane] = feat_of(lane == 0 ? Ds0[0] : Ds1[0], a.ix.metric);
    if (lane == 0) {
        a.ncells[ql * ns + i] = (int32_t)nc;
        a.aprime[ql * ns + i] = (int32_t)W;
    }
    return true;
}

template <int NT>
__device__ __forceinline__ void activate_item(const QueryPass &a, const int item) {
    extern __shared__ uint32_t Ptab[];          // [sk][sk+1] row prefix sums of sizes
    __shared__ float Dr[2][kMaxSqrtK];
    __shared__ float Ds[2][kMaxSqrtK];
    __shared__ int Ix[2][kMaxSqrtK];
    __shared__ uint32_t red[NT / kWave + 1];

    const int sk = a.ix.sk, K = a.ix.K, ns = a.ix.ns;
    const int ql = item / ns, i = item - ql * ns;
    const int tid = threadIdx.x;
    const float *q = a.Q + (int64_t)ql * a.ix.d;

    // centre distances of both halves (squared L2, FP32, dimension order), or
    // the ones given by an earlier kernel.  Query and centre values are loaded
    // eight dimensions at a time before their FMAs (same order), so a half
    // costs a few memory round trips rather than one per dimension.
    const HalfDims hd2[2] = {a.ix.halves[2 * i], a.ix.halves[2 * i + 1]};
    auto centre_dist = [&](const int h, const int c) -> float {
        if (a.Dext) return a.Dext[((int64_t)ql * 2 * ns + 2 * i + h) * sk + c];
        const HalfDims hd = hd2[h];
        const float *cp = a.ix.cent + (int64_t)sk * hd.dim0 + (int64_t)c * hd.w;
        const float *qp = q + hd.dim0;
        float s = 0.f;
        for (int j0 = 0; j0 < hd.w; j0 += 8) {
            float qv[8], cv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int jj = j0 + u < hd.w ? j0 + u : hd.w - 1;   // unconditional loads
                qv[u] = qp[jj];
                cv[u] = cp[jj];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (j0 + u < hd.w) {
                    const float t2 = qv[u] - cv[u];
                    s = dist_acc(s, t2, a.ix.metric);
                }
            }
        }
        return s;
    };
    if constexpr (NT == kWave) {
        // one wave, sk <= 64: lane c holds centre c of each half in a register.
        // A small budget is taken by the walk; otherwise a centre's rank
        // (ascending distance, ties by centre id) counts the lanes before it,
        // read one at a time with readlane
        const bool live = tid < sk;
        float v[2] = {0.f, 0.f};
        if (live && a.Dext) {
            v[0] = centre_dist(0, tid);
            v[1] = centre_dist(1, tid);
        } else if (live) {
            // both halves' loads issued together, each half summed in its own
            // dimension order
            const float *cp[2], *qp[2];
            int w[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                w[h] = hd2[h].w;
                cp[h] = a.ix.cent + (int64_t)sk * hd2[h].dim0 + (int64_t)tid * hd2[h].w;
                qp[h] = q + hd2[h].dim0;
            }
            const int wmax = w[0] > w[1] ? w[0] : w[1];
            for (int j0 = 0; j0 < wmax; j0 += 8) {
                float qv[2][8], cv[2][8];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        // unconditional loads: indices past the half repeat its last dimension
                        const int jj = j0 + u < w[h] ? j0 + u : w[h] - 1;
                        qv[h][u] = qp[h][jj];
                        cv[h][u] = cp[h][jj];
                    }
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        if (j0 + u < w[h]) {
                            const float t2 = qv[h][u] - cv[h][u];
                            v[h] = dist_acc(v[h], t2, a.ix.metric);
                        }
                    }
            }
        }
        const double alpha0 = a.alpha_qd ? a.alpha_qd[ql] : (a.alpha_q ? (double)a.alpha_q[ql] : a.alpha);
        const uint32_t A0 = count_A_dev(alpha0, a.ix.n);
        if (a.ix.act_form == 0 && (uint64_t)A0 * (uint64_t)K <= (uint64_t)kWalkRatio * (uint64_t)a.ix.n &&
            activate_walk(a, ql, i, v[0], v[1], live, A0))
            return;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int r = 0;
            for (int c2 = 0; c2 < sk; ++c2) {
                const float v2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[h]), c2));
                r += (v2 < v[h]) || (v2 == v[h] && c2 < tid);
            }
            if (live) {
                Ds[h][r] = v[h];
                Ix[h][r] = tid;
            }
        }
        if (a.ix.act_form == 1) {
            __shared__ uint32_t pushed[kWave * kWave / 32];
            __syncthreads();
            if (activate_ms(a, ql, i, Ds[0], Ds[1], Ix[0], Ix[1], A0, pushed)) return;
        }
    } else {
        for (int t = tid; t < 2 * sk; t += NT) {
            const int h = t >= sk, c = t - h * sk;
            Dr[h][c] = centre_dist(h, c);
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
    }
    __syncthreads();
    // cell sizes in rank order, eight gathers in flight per thread (a missing
    // slot reads cell 0 and is not stored), then per-row prefix sums
    const int stride = sk + 1;
    const uint32_t *cs = a.ix.csize + (int64_t)i * K;
    {
        const int rq = NT / sk, rr = NT - rq * sk;      // NT = rq rows + rr columns
        int r1 = tid / sk, r2 = tid - r1 * sk;
        for (int t0 = 0; t0 < sk * sk; t0 += 8 * NT) {
            uint32_t val[8];
            int at[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool in = r1 < sk;
                at[u] = in ? r1 * stride + r2 + 1 : -1;
                val[u] = cs[in ? Ix[0][r1] * sk + Ix[1][r2] : 0];
                r1 += rq;
                r2 += rr;
                if (r2 >= sk) { r2 -= sk; ++r1; }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (at[u] >= 0) Ptab[at[u]] = val[u];
        }
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
    if (a.feat != nullptr && tid < 2) a.feat[(int64_t)ql * 2 * ns + 2 * i + tid] = feat_of(Ds[tid][0], a.ix.metric);

    const double alpha = a.alpha_qd ? a.alpha_qd[ql] : (a.alpha_q ? (double)a.alpha_q[ql] : a.alpha);
    const uint32_t A = count_A_dev(alpha, a.ix.n);
    const bool row = tid < sk;
    const float d1 = row ? Ds[0][tid] : 0.f;
    const uint32_t *prow = Ptab + (row ? tid : 0) * stride;
    // #{r2 : d1 + D2s[r2] <= v}, known to lie in [l2, h2]
    auto cnt = [&](float v, int l2, int h2) -> int {
        while (l2 < h2) {
            const int m = (l2 + h2) >> 1;
            if (d1 + Ds[1][m] <= v) l2 = m + 1; else h2 = m;
        }
        return l2;
    };
    auto total = [&](uint32_t w) -> uint32_t {
        if constexpr (NT == kWave) return wave_sum(w);
        else return block_sum<NT>(w, red);
    };
    // W(lo) < A <= W(hi) throughout; every row keeps its counts at lo and hi
    // (the keys are monotone in both ranks, so each row's count at a value
    // between them lies between its counts there).  At lo = kmin - 1 ulp no
    // key is counted; at hi = kmax every key is.
    const float kmin = Ds[0][0] + Ds[1][0];
    const float kmax = Ds[0][sk - 1] + Ds[1][sk - 1];
    int64_t lo = (int64_t)__float_as_uint(kmin) - 1;
    int64_t hi = (int64_t)__float_as_uint(kmax);
    uint32_t Wlo = 0;
    int cl = 0, ch = row ? sk : 0;
    while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        const float v = __uint_as_float((uint32_t)mid);
        const int c = row ? cnt(v, cl, ch) : 0;
        const uint32_t w = total(row ? prow[c] : 0u);
        if (w >= A) { hi = mid; ch = c; } else { lo = mid; cl = c; Wlo = w; }
    }
    // cells with key < v* (= hi): the first cl of each row; the tie cells with
    // key == v*: columns [cl, ch)
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
    const uint32_t ap = total(myw);
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

// Queries in this pass: the pass's own count, or, for a batch whose size is
// read on the device (captured graphs), what is left of it after q_base,
// capped at the pass capacity.
__device__ __forceinline__ int pass_nq(const int *nq_dev, int q_base, int nq) {
    if (nq_dev == nullptr) return nq;
    const int left = *nq_dev - q_base;
    return left <= 0 ? 0 : (left < nq ? left : nq);
}

// Every kernel walks its work items with a grid stride, so a launch may use
// fewer blocks than items (a persistent grid) and one launch shape serves any
// batch up to the pass capacity.
template <int NT>
__global__ __launch_bounds__(NT) void k_activate(QueryPass a) {
    const int items = pass_nq(a.nq_dev, a.q_base, a.nq) * a.ix.ns;
    if (a.ntl != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.ntl = 0;   // read after this kernel
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        activate_item<NT>(a, item);
        __syncthreads();
    }
}

// =============================================================== collide ==
// Block per (query, group of tiles): the block takes the tiles p = g, g + S,
// g + 2S, ... of its query (S = tile groups per query) one after another.  A
// tile's TILE scores live in LDS as bytes packed in 32-bit words; each point
// id occurs once per subspace, so a 32-bit LDS atomic add of 1 << 8*(id & 3)
// increments exactly one byte without carry (scores never exceed ns <= 127).
// The LDS scores are zeroed once per block and cleared after every tile (only
// the touched words when they were listed), so later tiles start from zero.
// The activated cells of all subspaces are runs of contiguous ids inside the
// tile (ids are stored tile-major).  The block loads up to NT run descriptors
// at once into LDS (one thread per run), scans their lengths, and then the
// threads take the flattened ids of all those runs, kCollideUnroll at a time
// with their loads issued together, each finding its run through a table of
// every 32nd position (or a binary search past it).  A query's first batches
// of cells are read once and kept in registers for all its tiles.
// The block then has G[t] = #{score >= t} (from the counting atomics' old
// values, or by 7-bit SWAR compares over the words) and lists every point of
// non-zero score, as its tile-local id, grouped by score level in descending
// order: level s occupies [G[s+1], G[s]) of the tile's list.  Points of score
// 0 are not written, nor the levels the selection can no longer take (see
// kPruneLevels); the dense scores are written only when asked for.
// Words of the tile touched by the counting are listed as they are first
// incremented (a wave appends its first touches with one atomic), so the
// passes after the counting visit only those words; when more than kTouchCap
// words are touched the passes scan the whole tile instead.
constexpr int kCollideUnroll = 4;
constexpr int kTouchCap = 4096;
constexpr int kBucketShift = 5;     // run lookup table: one entry per 32 consecutive id positions
constexpr int kBuckets = 1024;      // positions beyond kBuckets << kBucketShift use a binary search
// Levels 1..kPruneLevels-1 may be left out of a tile's lists: a tile need not
// list its ids of score s when the block's earlier tiles of the query (lower
// ids) already hold at least B ids of score >= s.  Then either the threshold
// T exceeds s, or T == s and those earlier tiles hold at least
// B - (their own #{score > s}) >= B - #{score > T} = R ids of level s; the
// selection takes the R lowest level-T ids, all of which lie there, and none
// of this tile's.  The tile's histogram still counts every point.
constexpr int kPruneLevels = 32;
// With N_s <= kIncLevels the tile histogram is gathered while counting: the
// atomic add returns the byte's old value o, and that increment is exactly
// one of the #{score >= o+1} points, so G[t] = #{increments with o = t-1}.  A
// thread keeps 8-bit counts per level in two 64-bit registers; they cannot
// overflow while a tile gives a thread at most 255 increments (a batch of
// runs with m ids gives a thread at most ceil(m / NT)); tiles with more are
// tallied from their words instead.
constexpr int kIncLevels = 16;
constexpr uint32_t kIncMax = 255;

template <int NT>
struct CollideLds {
    // per-tile counters, two sets used by alternate tiles: a tile resets the
    // next tile's set while it builds its own lists, so no barrier is needed
    // between the end of one tile and the counting of the next
    uint32_t G[2][kMaxNs + 2];
    uint32_t cur[2][kMaxNs + 2];
    int64_t rstart[NT];          // start in ids16 of each non-empty run of the batch (compacted)
    uint32_t rpre[NT];           // ids before each of those runs in the batch
    uint32_t red[2 * (NT / kWave) + 2];
    uint16_t first[kBuckets];    // run holding position b << kBucketShift
    uint16_t touched[kTouchCap];
    uint32_t n_touched[2];
    uint32_t Gc[kPruneLevels];   // #{score >= s} over the block's earlier tiles of its query
};

struct RunBatch {
    uint32_t tot;                // ids in the batch
    int nr;                      // non-empty runs
};

// Scan one run per thread (length len at ids16 offset st) into the block's run
// table: the non-empty runs are compacted in slot order, and a table gives for
// every 32nd position the run that holds it.  Ends with a barrier.
template <int NT>
__device__ __forceinline__ RunBatch collide_runs(CollideLds<NT> &L, uint32_t len, int64_t st) {
    uint32_t ex, idx, tot, nr;
    block_excl_scan2<NT>(len, len != 0u ? 1u : 0u, L.red, &ex, &idx, &tot, &nr);
    if (len != 0u) {
        L.rstart[idx] = st;
        L.rpre[idx] = ex;
        // table entries of the positions b << kBucketShift inside this run
        const uint32_t bfirst = (ex + (1u << kBucketShift) - 1u) >> kBucketShift;
        const uint32_t blast = (ex + len - 1u) >> kBucketShift;
        for (uint32_t b = bfirst; b <= blast && b < (uint32_t)kBuckets; ++b) L.first[b] = (uint16_t)idx;
    }
    __syncthreads();
    return RunBatch{tot, (int)nr};
}

// Issue the loads of ids e0 + u*NT + tid (u < kCollideUnroll) of the run table;
// bit u of the result says whether slot u holds an id.  An id's run is the
// table's run for its 32-position bucket or one of the next few (runs are at
// least one id long); past the table a binary search finds it.  The loads are
// unconditional (an empty slot reads entry 0) so that no later instruction has
// to wait for them before they are used.
template <int NT>
__device__ __forceinline__ uint32_t collide_fetch(const QueryPass &a, const CollideLds<NT> &L, uint32_t e0,
                                                  RunBatch rb, uint32_t (&lid)[kCollideUnroll]) {
    uint32_t vm = 0u;
#pragma unroll
    for (int u = 0; u < kCollideUnroll; ++u) {
        const uint32_t e = e0 + (uint32_t)(u * NT + threadIdx.x);
        int64_t at = 0;
        if (e < rb.tot) {
            int m;
            if ((e >> kBucketShift) < (uint32_t)kBuckets) {
                m = L.first[e >> kBucketShift];
                while (m + 1 < rb.nr && L.rpre[m + 1] <= e) ++m;
            } else {
                int lo = 0, hi = rb.nr - 1;           // largest m with rpre[m] <= e
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.rpre[mid] <= e) lo = mid; else hi = mid - 1;
                }
                m = lo;
            }
            at = L.rstart[m] + (e - L.rpre[m]);
            vm |= 1u << u;
        }
        lid[u] = a.ix.ids16[at];
    }
    return vm;
}

// +1 on the scores of the fetched ids; words touched for the first time are
// listed.  All slots' atomics are issued before any result is used, and the
// first touches of all slots are appended with one atomic per wave.  With
// `inc`, each increment is also counted at its level in hc (see kIncLevels).
template <int NT>
__device__ __forceinline__ void collide_count(CollideLds<NT> &L, uint32_t *sc, const uint32_t (&lid)[kCollideUnroll],
                                              const uint32_t vm, const int b, const bool inc, uint64_t (&hc)[2]) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below_mask = (1ull << lane) - 1ull;
    uint32_t old[kCollideUnroll];
#pragma unroll
    for (int u = 0; u < kCollideUnroll; ++u) {
        old[u] = 1u;
        if ((vm >> u) & 1u) old[u] = atomicAdd(&sc[lid[u] >> 2], 1u << ((lid[u] & 3u) << 3));
    }
    if (inc) {
#pragma unroll
        for (int u = 0; u < kCollideUnroll; ++u) {
            if (((vm >> u) & 1u) == 0u) continue;
            const uint32_t o = (old[u] >> ((lid[u] & 3u) << 3)) & 0xffu;   // < N_s <= kIncLevels
            const uint64_t one = 1ull << ((o & 7u) << 3);
            if (o < 8u) hc[0] += one; else hc[1] += one;
        }
    }
    uint64_t m[kCollideUnroll];
    uint32_t nfirst = 0u;
#pragma unroll
    for (int u = 0; u < kCollideUnroll; ++u) {
        m[u] = __ballot(old[u] == 0u);
        nfirst += (uint32_t)__popcll(m[u]);
    }
    if (nfirst != 0u) {
        uint32_t base = 0u;
        if (lane == 0) base = atomicAdd(&L.n_touched[b], nfirst);
        base = (uint32_t)__builtin_amdgcn_readlane((int)base, 0);
#pragma unroll
        for (int u = 0; u < kCollideUnroll; ++u) {
            if (old[u] == 0u) {
                const uint32_t pos = base + (uint32_t)__popcll(m[u] & below_mask);
                if (pos < (uint32_t)kTouchCap) L.touched[pos] = (uint16_t)(lid[u] >> 2);
            }
            base += (uint32_t)__popcll(m[u]);
        }
    }
}

// After the counting of tile p (counters of set b): tile histogram, level
// lists, optional dense scores; the scores are left zero for the next tile and
// the other counter set is reset for it.  Starts with a barrier.  When the
// tile's words were listed and no dense scores are written, each listed word
// is read once into a register and zeroed at once, and the function ends
// without a barrier (the next tile's counting touches nothing this tile still
// reads); otherwise it ends with one after clearing the scores.
template <int NT>
__device__ __forceinline__ void collide_finish(const QueryPass &a, CollideLds<NT> &L, uint32_t *sc, const int ql,
                                               const int p, const int b, const bool inc, uint64_t (&hc)[2]) {
    const int P = a.ix.P, ns = a.ix.ns, TILE = a.ix.TILE;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int words = TILE >> 2;
    // the caller's last barrier follows the counting
    const uint32_t nt = L.n_touched[b];
    const bool sparse = nt <= (uint32_t)kTouchCap;
    const bool early = sparse && a.scores == nullptr;
    const int nw = sparse ? (int)nt : words;
    // levels 1..s0 are not listed (see kPruneLevels); Gc was last written by
    // the previous tile's finish, before the barrier that ended this counting
    uint32_t s0 = 0;
    for (int sl = (ns < kPruneLevels - 1 ? ns : kPruneLevels - 1); sl >= 1; --sl)
        if (L.Gc[sl] >= (uint32_t)a.B) { s0 = (uint32_t)sl; break; }
    // Counts of bytes >= t, two thresholds per 32-bit counter (16-bit halves:
    // a thread sees at most 4 * 32 bytes, a wave at most 64 times that).  In
    // the listed-words case a thread has at most kTouchCap / NT words; they are
    // kept in registers for the level pass.
    constexpr int kKeep = kTouchCap / NT;
    int wk[kKeep];
    uint32_t xk[kKeep];
#pragma unroll
    for (int q = 0; q < kKeep; ++q) {
        const int j = tid + q * NT;
        wk[q] = 0;
        xk[q] = 0u;
        if (sparse && j < nw) {
            wk[q] = L.touched[j];
            xk[q] = sc[wk[q]];
            if (early) sc[wk[q]] = 0u;
        }
    }
    // the other set was last used by the tile before this one, which every
    // wave finished before the barrier that ended this tile's counting
    for (int t = tid; t < ns + 2; t += NT) {
        L.G[b ^ 1][t] = 0u;
        L.cur[b ^ 1][t] = 0u;
    }
    if (tid == 0) L.n_touched[b ^ 1] = 0u;
    if (inc) {
        // two levels per wave sum, in 16-bit halves (a wave counts at most
        // 64 * 255 increments per level)
#pragma unroll
        for (int t0 = 1; t0 <= kIncLevels; t0 += 2) {
            if (t0 > ns) break;
            const uint32_t fa = (uint32_t)(hc[(t0 - 1) >> 3] >> (((t0 - 1) & 7) * 8)) & 0xffu;
            const uint32_t fb = (uint32_t)(hc[t0 >> 3] >> ((t0 & 7) * 8)) & 0xffu;
            const uint32_t sum = wave_sum(fa | (t0 + 1 <= ns ? fb << 16 : 0u));
            if (lane == 0) {
                atomicAdd(&L.G[b][t0], sum & 0xffffu);
                if (t0 + 1 <= ns) atomicAdd(&L.G[b][t0 + 1], sum >> 16);
            }
        }
    }
    for (int t0 = 1; !inc && t0 <= ns; t0 += 8) {
        uint32_t c[4] = {0, 0, 0, 0};
        auto tally = [&](uint32_t x) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t ta = (uint32_t)(t0 + 2 * v), tb = ta + 1u;
                c[v] += __popc((x + (0x80u - ta) * 0x01010101u) & 0x80808080u) +
                        (__popc((x + (0x80u - tb) * 0x01010101u) & 0x80808080u) << 16);
            }
        };
        if (sparse) {
#pragma unroll
            for (int q = 0; q < kKeep; ++q)
                if (xk[q] != 0u) tally(xk[q]);
        } else {
            for (int j = tid; j < nw; j += NT) {
                const uint32_t x = sc[j];
                if (x != 0u) tally(x);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if (t0 + 2 * v <= ns) {
                const uint32_t sum = wave_sum(c[v]);
                if (lane == 0) {
                    atomicAdd(&L.G[b][t0 + 2 * v], sum & 0xffffu);
                    if (t0 + 2 * v + 1 <= ns) atomicAdd(&L.G[b][t0 + 2 * v + 1], sum >> 16);
                }
            }
        }
    }
    __syncthreads();
    // level s starts at G[s+1]; cur[s] counts the ids placed in it so far
    uint16_t *seg = a.lvl + ((int64_t)ql * P + p) * TILE;
    auto place = [&](int w, uint32_t x) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t sv = (x >> (8 * u)) & 0xffu;
            if (sv > s0) seg[L.G[b][sv + 1] + atomicAdd(&L.cur[b][sv], 1u)] = (uint16_t)(4 * w + u);
        }
    };
    // a word is skipped at once when none of its bytes exceeds s0: bytes are
    // at most N_s <= 127, so b + (127 - s0) sets bit 7 exactly when b > s0,
    // without a carry into the next byte
    const uint32_t above = (0x7fu - s0) * 0x01010101u;
    auto listed = [&](uint32_t x) { return ((x + above) & 0x80808080u) != 0u; };
    if (sparse) {
#pragma unroll
        for (int q = 0; q < kKeep; ++q)
            if (listed(xk[q])) place(wk[q], xk[q]);
    } else {
        const uint4 *sc4 = reinterpret_cast<const uint4 *>(sc);
        for (int j4 = tid; j4 < (nw >> 2); j4 += NT) {
            const uint4 x = sc4[j4];
            if (listed(x.x)) place(4 * j4, x.x);
            if (listed(x.y)) place(4 * j4 + 1, x.y);
            if (listed(x.z)) place(4 * j4 + 2, x.z);
            if (listed(x.w)) place(4 * j4 + 3, x.w);
        }
    }
    if (a.scores != nullptr) {
        uint4 *dst = reinterpret_cast<uint4 *>(a.scores + ((int64_t)ql * P + p) * TILE);
        const uint4 *src = reinterpret_cast<const uint4 *>(sc);
        for (int w = tid; w < (words >> 2); w += NT) dst[w] = src[w];
    }
    const int64_t t0 = (int64_t)p * TILE;
    const int64_t valid = a.ix.n - t0 < TILE ? a.ix.n - t0 : TILE;
    uint32_t *h = a.hist + ((int64_t)ql * P + p) * (ns + 2);
    for (int t = tid; t < ns + 2; t += NT) h[t] = t == 0 ? (uint32_t)valid : L.G[b][t];
    // every wave read Gc above, before the barrier after the histogram
    for (int t = 1 + tid; t < kPruneLevels && t <= ns; t += NT) L.Gc[t] += L.G[b][t];
    if (early) return;
    __syncthreads();
    if (sparse) {
#pragma unroll
        for (int q = 0; q < kKeep; ++q)
            if (tid + q * NT < nw) sc[wk[q]] = 0u;
    } else {
        uint4 *z = reinterpret_cast<uint4 *>(sc);
        for (int w = tid; w < (words >> 2); w += NT) z[w] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
}

// One tile with any number of run batches (a subspace with more activated
// cells than one batch holds): runs are reloaded batch by batch.
template <int NT>
__device__ __forceinline__ void collide_tile(const QueryPass &a, CollideLds<NT> &L, uint32_t *sc, const int ql,
                                             const int p, const int my_nc, const int c_first, const int c_second,
                                             int &b) {
    const int P = a.ix.P, ns = a.ix.ns, K = a.ix.K, TILE = a.ix.TILE;
    const int RJ = a.runs_per_sub;
    const int i = threadIdx.x / RJ, jj = threadIdx.x - i * RJ;
    const bool has_i = i < ns;
    const uint16_t *my_cells = a.cells + ((int64_t)ql * ns + (has_i ? i : 0)) * K;
    const uint32_t *to = a.ix.toffs + ((int64_t)(has_i ? i : 0) * P + p) * (K + 1);
    const bool levels = ns <= kIncLevels;
    uint64_t hc[2] = {0ull, 0ull};
    uint32_t per_thread = 0;                                // ids per thread in this tile, at most (capped)
    for (int jb = 0; __syncthreads_or(jb < my_nc); jb += RJ) {
        const int j = jb + jj;
        uint32_t len = 0;
        int64_t st = 0;
        if (has_i && j < my_nc) {
            const int c = jb == 0 ? c_first : (jb == RJ ? c_second : (int)my_cells[j]);
            const uint32_t s = to[c];
            len = to[c + 1] - s;
            st = (int64_t)i * P * TILE + s;
        }
        const RunBatch rb = collide_runs<NT>(L, len, st);
        const uint32_t per = (rb.tot + NT - 1) / NT;       // this batch's ids per thread, at most
        per_thread = per <= kIncMax - per_thread ? per_thread + per : kIncMax + 1;
        for (uint32_t e0 = 0; e0 < rb.tot; e0 += NT * kCollideUnroll) {
            uint32_t lid[kCollideUnroll];
            const uint32_t vm = collide_fetch<NT>(a, L, e0, rb, lid);
            collide_count<NT>(L, sc, lid, vm, b, levels, hc);
        }
        __syncthreads();
    }
    collide_finish<NT>(a, L, sc, ql, p, b, levels && per_thread <= kIncMax, hc);
    b ^= 1;
}

// The tiles of one (query, tile group) when every subspace's activated cells
// fit one batch, as a two-stage pipeline: while tile p's histogram and level
// lists are built, the ids of the group's next tile and the run offsets of the
// one after it are already being loaded.  Those loads are unconditional (from
// a valid tile when there is no next one) so the compiler has no reason to wait
// for them before they are needed.
template <int NT>
__device__ __forceinline__ void collide_tiles_pipelined(const QueryPass &a, CollideLds<NT> &L, uint32_t *sc,
                                                        const int ql, const int g, const int my_nc, const int c_first,
                                                        int &b) {
    const int P = a.ix.P, K = a.ix.K, TILE = a.ix.TILE, S = a.tgroups;
    const int RJ = a.runs_per_sub, ns = a.ix.ns;
    const int i = threadIdx.x / RJ, jj = threadIdx.x - i * RJ;
    const bool has_run = i < ns && jj < my_nc;
    const int ic = i < ns ? i : 0;
    // run offsets of cell c_first (cell 0 of subspace 0 for threads without a run) in tile p
    const uint32_t *tob = a.ix.toffs + (int64_t)ic * P * (K + 1) + c_first;
    const int64_t rbase = (int64_t)ic * P * TILE;
    uint32_t rs = tob[(int64_t)g * (K + 1)], re = tob[(int64_t)g * (K + 1) + 1];
    uint32_t lid[kCollideUnroll];
    RunBatch rb = collide_runs<NT>(L, has_run ? re - rs : 0u, rbase + rs);
    uint32_t vm = collide_fetch<NT>(a, L, 0, rb, lid);
    {
        const int pn = g + S < P ? g + S : g;
        rs = tob[(int64_t)pn * (K + 1)];
        re = tob[(int64_t)pn * (K + 1) + 1];
    }
    const bool levels = ns <= kIncLevels;
    for (int p = g; p < P; p += S) {
        uint64_t hc[2] = {0ull, 0ull};
        const bool inc = levels && (rb.tot + NT - 1) / NT <= kIncMax;
        collide_count<NT>(L, sc, lid, vm, b, inc, hc);
        for (uint32_t e0 = NT * kCollideUnroll; e0 < rb.tot; e0 += NT * kCollideUnroll) {
            uint32_t lid2[kCollideUnroll];
            const uint32_t vm2 = collide_fetch<NT>(a, L, e0, rb, lid2);
            collide_count<NT>(L, sc, lid2, vm2, b, inc, hc);
        }
        __syncthreads();
        // stage the next tile of the group (an empty one after the last) and
        // prefetch the run offsets of the one after it; every load here is
        // unconditional, so nothing waits for them before the next iteration
        const bool more = p + S < P;
        rb = collide_runs<NT>(L, (has_run && more) ? re - rs : 0u, rbase + rs);
        vm = collide_fetch<NT>(a, L, 0, rb, lid);
        const int pn = p + 2 * S < P ? p + 2 * S : p;
        rs = tob[(int64_t)pn * (K + 1)];
        re = tob[(int64_t)pn * (K + 1) + 1];
        collide_finish<NT>(a, L, sc, ql, p, b, inc, hc);
        b ^= 1;
    }
}

// Items are (query, tile group); a grid smaller than the items strides over
// them.
template <int NT>
__global__ __launch_bounds__(NT) void k_collide(QueryPass a) {
    extern __shared__ uint32_t sc[];   // TILE/4 words
    __shared__ CollideLds<NT> L;
    // with the sparse step: only the queries it left, from its list; they are
    // few, so each is spread over more tile groups (about 2,048 blocks' worth
    // of items in all, as the host's choice for a full pass)
    const int nt = a.tlist != nullptr ? *a.ntl : pass_nq(a.nq_dev, a.q_base, a.nq);
    if (a.tlist != nullptr) a.tgroups = nt > 0 ? min(a.ix.P, max(1, (2048 + nt - 1) / nt)) : 1;
    const int S = a.tgroups;
    const int items = nt * S;
    if ((int)blockIdx.x >= items) return;
    {
        uint4 *z = reinterpret_cast<uint4 *>(sc);
        for (int w = threadIdx.x; w < (a.ix.TILE >> 4); w += NT) z[w] = make_uint4(0u, 0u, 0u, 0u);
        for (int t = threadIdx.x; t < a.ix.ns + 2; t += NT) {
            L.G[0][t] = 0u;
            L.cur[0][t] = 0u;
        }
        if (threadIdx.x == 0) L.n_touched[0] = 0u;
    }
    int b = 0;                         // counter set of the block's next tile
    const int RJ = a.runs_per_sub, ns = a.ix.ns;
    const int i = threadIdx.x / RJ, jj = threadIdx.x - i * RJ;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int rq = item / S, g = item - rq * S;
        const int ql = a.tlist ? a.tlist[rq] : (a.order ? a.order[rq] : rq);   // heaviest queries first
        // this thread's subspace: activated cell count and its cell of the first batch
        const int my_nc = i < ns ? a.ncells[ql * ns + i] : 0;
        const int c_first = jj < my_nc ? (int)a.cells[((int64_t)ql * ns + i) * a.ix.K + jj] : 0;
        const bool batched = __syncthreads_or(my_nc > RJ);
        // a new query: no earlier tiles (read after the next barrier, the one
        // that ends the counting of its first tile)
        for (int t = threadIdx.x; t < kPruneLevels; t += NT) L.Gc[t] = 0u;
        if (batched) {
            // the second batch's cell is kept too (it is the same for every tile)
            const int c_second = jj + RJ < my_nc ? (int)a.cells[((int64_t)ql * ns + i) * a.ix.K + jj + RJ] : 0;
            for (int p = g; p < a.ix.P; p += S) collide_tile<NT>(a, L, sc, ql, p, my_nc, c_first, c_second, b);
        } else {
            collide_tiles_pipelined<NT>(a, L, sc, ql, g, my_nc, c_first, b);
        }
    }
}

// ======================================================== collide (sparse) ==
// One work-group per query whose activated points are few next to n: its
// SC-scores are counted per bucket of kSpBucket consecutive ids that holds
// some of them, so the work follows the activated points (counting is
// O(alpha*n*N_s) per query, Sec. 4.3) instead of visiting every tile of the
// id range, and everything after the id reads stays in LDS:
//  1. the query's activated cells become runs of the cell-major id copy (one
//     run per cell); one walk over all their ids as a single sequence (every
//     thread an equal share) places the low 12 bits of each into its bucket's
//     slots (buckets sized exactly beforehand from the index's count of each
//     cell's ids per bucket);
//  2. a wave takes a bucket: its scores are counted in the wave's window, 4
//     bits an id (8 ids a word, 2 KB, for N_s <= 15) or 5 bits (6 a word,
//     2.7 KB, for N_s <= 31), with 32-bit LDS atomic adds of 1 at the id's
//     field (an id occurs once per subspace, so no field carries), then
//     every id claims its field with an atomic AND that clears it: the first claimant of a
//     point gets its score, later ones get 0, and the window ends clear.  The
//     bucket's points of score 1 replace its slots' front (the slots already
//     read), those of score s >= 2 go to one list of the work-group as
//     (id << 4 | s), held in the slots past the query's own, and add one to
//     H[s] (the histogram G[t] = #{score >= t});
//  3. T = max{t : G[t] >= B} and R = B - G[T+1]: every listed point above T is
//     a candidate, and of the points at T the R lowest ids.  Per bucket, its
//     points at T (the front count when T = 1, else counted over the list); a
//     block scan in bucket order gives each bucket's share of the R; buckets
//     with all or none of theirs copy them, and the one bucket cut inside
//     finds its cut id by marking its level-T ids in a 4096-bit map and
//     counting.  Candidates are appended in no particular order.
// A query is left to the tiled steps (route 1) when N_s > 31, it has
// kSpMaxRuns activated cells or more, more activated ids than the slots, more
// points of score 2 or more than the slots past its ids hold, or T = 0 (fewer
// than B points collide: the score-0 points are the tiled selection's case);
// otherwise route 0, and the tiled collision and selection kernels skip the
// query.
struct SparseLds {
    uint32_t H[kSpMaxNs5 + 2];       // H[s]: points of score s >= 2
    uint32_t sink[kWave];            // targets of the atomics of empty slots, one word per lane
    uint32_t red[2 * kSpWaves + 2];
    uint32_t zfree[kSpWaves];        // unmarked ids below B per bucket (fewer than B points collide)
    uint32_t cpre[kSpMaxNs5 + 1];    // activated cells of the subspaces before i
    uint32_t nh;                     // points in the list of scores >= 2 (may pass its capacity)
    uint32_t out;                    // candidates written
    int nruns, flag, cutb;
    uint32_t cut;
    uint32_t crun[kSpMaxChunks];     // run holding position 1024*q of the walk's sequence
};

// Every id of the query's activated cells, as one sequence: runs[r] =
// (start of run r in ids32, its first position in the sequence),
// runs[nruns].y = the total, and crun[q] = the run holding position 1024*q.
// Thread t takes positions t, t + kSpThreads, ..., 2*kSpU of them per step:
// position p lies in chunk p / 1024, the same for every thread of the step, so
// its run is found from that chunk's first run in a step or two, independently
// of the step's other positions; then the loads are issued together.
// Consecutive threads read consecutive ids of a run.  The loads are
// unconditional (a position past the end reads the first slot of run 0), so
// none waits for another; f gets the ids, a bit mask of the valid ones and a
// mask of the slots valid in some thread of the block.
constexpr int kSpU = 8;
static_assert(kSpThreads == 1024, "a step's positions are one per 1024-position chunk");
template <class F>
__device__ __forceinline__ void sp_walk(const QueryPass &a, const uint2 *runs, const uint32_t *crun,
                                        uint32_t total, F &&f) {
    constexpr int U = 2 * kSpU;
    const uint32_t tid = threadIdx.x;
    for (uint32_t base = 0; base < total; base += (uint32_t)(U * kSpThreads)) {
        uint32_t at[U], vm = 0u, um = 0u;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t p = base + tid + (uint32_t)(u * kSpThreads);
            const bool v = p < total;
            int r = 0;
            if (v) {
                r = (int)crun[(base >> 10) + (uint32_t)u];
                while (runs[r + 1].y <= p) ++r;
            }
            const uint2 rr = runs[r];
            at[u] = v ? rr.x + (p - rr.y) : rr.x;
            vm |= (v ? 1u : 0u) << u;
            um |= (base + (uint32_t)(u * kSpThreads) < total ? 1u : 0u) << u;
        }
        uint32_t id[U];
#pragma unroll
        for (int u = 0; u < U; ++u) id[u] = a.ix.ids32[at[u]];
        f(id, vm, um);
    }
}

// A wave's score window for SB-bit scores: the word of low id lo and the
// position of its field (8 ids a word at 4 bits, 6 at 5 bits; a field never
// carries: an id occurs once per subspace and N_s < 2^SB).
template <int SB>
__device__ __forceinline__ uint32_t sp_word(uint32_t lo) { return SB == 4 ? lo >> 3 : lo / 6u; }
template <int SB>
__device__ __forceinline__ uint32_t sp_shift(uint32_t lo) { return SB == 4 ? (lo & 7u) << 2 : (lo - 6u * (lo / 6u)) * 5u; }

// One bucket by one wave (step 2).  seg holds its len low ids and receives
// its points of score 1 at the front; those of higher score go to the list
// hl (capacity hcap, count *hn); sink takes the atomics of empty slots.
// Returns the number of points of score 1.
template <int SB>
__device__ __forceinline__ uint32_t sp_bucket(const QueryPass &a, const int ql, const int b, uint16_t *seg,
                                              const uint32_t len, uint32_t *win, uint32_t *hl, const uint32_t hcap,
                                              uint32_t *hn, uint32_t *H, uint32_t *sink) {
    constexpr uint32_t SM = (1u << SB) - 1u;
    const int lane = threadIdx.x & (kWave - 1);
    constexpr int UQ = 4;
    // a bucket of at most UQ*64 ids (the common case) is read once: the claims
    // reuse the counting pass's registers
    uint32_t u0[UQ];
    for (uint32_t j0 = 0; j0 < len; j0 += (uint32_t)(UQ * kWave)) {
        uint32_t u[UQ];
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const uint32_t j = j0 + (uint32_t)(q * kWave + lane);
            u[q] = seg[j < len ? j : 0u];
            u0[q] = u[q];
        }
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            if (j0 + (uint32_t)(q * kWave) >= len) break;             // the same in every lane
            const bool v = j0 + (uint32_t)(q * kWave + lane) < len;
            atomicAdd(v ? &win[sp_word<SB>(u[q])] : &sink[lane], v ? 1u << sp_shift<SB>(u[q]) : 0u);
        }
    }
    const bool one = len <= (uint32_t)(UQ * kWave);
    if (a.scores != nullptr) {
        // dense scores on request (parity tests): lane l writes ids 64l .. 64l + 63 below n
        uint8_t *row = a.scores + (int64_t)ql * a.ix.P * a.ix.TILE;
        const int64_t id0 = (int64_t)b * kSpBucket;
        for (int k = 0; k < 64; ++k) {
            const uint32_t lo = 64u * (uint32_t)lane + (uint32_t)k;
            if (id0 + lo < a.ix.n) row[id0 + lo] = (uint8_t)((win[sp_word<SB>(lo)] >> sp_shift<SB>(lo)) & SM);
        }
    }
    // claims; the front entries written in a step lie below the step's end,
    // whose slots were all read at the start of the step
    uint32_t n1 = 0;
    const uint32_t id0 = (uint32_t)b << kSpShift;
    for (uint32_t j0 = 0; j0 < len; j0 += (uint32_t)(UQ * kWave)) {
        uint32_t u[UQ], sv[UQ];
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const uint32_t j = j0 + (uint32_t)(q * kWave + lane);
            u[q] = one ? u0[q] : seg[j < len ? j : 0u];
        }
        // all UQ claims are issued before any result is used (the slots past the
        // bucket's end claim a lane's sink word with a mask that changes nothing)
        uint32_t old[UQ];
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const bool v = j0 + (uint32_t)(q * kWave + lane) < len;
            const uint32_t sh = sp_shift<SB>(u[q]);
            old[q] = atomicAnd(v ? &win[sp_word<SB>(u[q])] : &sink[lane], v ? ~(SM << sh) : ~0u);
        }
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const bool v = j0 + (uint32_t)(q * kWave + lane) < len;
            sv[q] = v ? (old[q] >> sp_shift<SB>(u[q])) & SM : 0u;
        }
        uint64_t mh[UQ];
        uint32_t nh = 0;
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const uint64_t m1 = __ballot(sv[q] == 1u);
            mh[q] = __ballot(sv[q] >= 2u);
            nh += (uint32_t)__popcll(mh[q]);
            if (sv[q] == 1u) seg[n1 + lanes_below(m1)] = (uint16_t)u[q];
            n1 += (uint32_t)__popcll(m1);
        }
        if (nh) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(hn, nh);
            base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
#pragma unroll
            for (int q = 0; q < UQ; ++q) {
                if (sv[q] >= 2u) {
                    const uint32_t at = base + lanes_below(mh[q]);
                    if (at < hcap) hl[at] = ((id0 | u[q]) << SB) | sv[q];
                    atomicAdd(&H[sv[q]], 1u);
                }
                base += (uint32_t)__popcll(mh[q]);
            }
        }
    }
    return n1;
}

// Two buckets by one wave, each of at most 4*64 ids, in windows win0 and
// win1: the same steps as sp_bucket, with the loads, the counting atomics and
// the claims of both buckets issued together, so that the wave has two
// buckets' round trips in flight.  n1[k] receives bucket k's points of score 1.
template <int SB>
__device__ __forceinline__ void sp_bucket_pair(const QueryPass &a, const int ql, const int b0, const int b1,
                                               uint16_t *seg0, const uint32_t len0, uint16_t *seg1,
                                               const uint32_t len1, uint32_t *win0, uint32_t *win1, uint32_t *hl,
                                               const uint32_t hcap, uint32_t *hn, uint32_t *H, uint32_t *sink,
                                               uint32_t (&n1)[2]) {
    constexpr uint32_t SM = (1u << SB) - 1u;
    constexpr int UQ = 4;
    const int lane = threadIdx.x & (kWave - 1);
    uint16_t *seg[2] = {seg0, seg1};
    const uint32_t len[2] = {len0, len1};
    uint32_t *win[2] = {win0, win1};
    const int bb[2] = {b0, b1};
    uint32_t u[2][UQ];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const uint32_t j = (uint32_t)(q * kWave + lane);
            u[k][q] = seg[k][j < len[k] ? j : 0u];
        }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            if ((uint32_t)(q * kWave) >= len[k]) continue;              // the same in every lane
            const bool v = (uint32_t)(q * kWave + lane) < len[k];
            atomicAdd(v ? &win[k][sp_word<SB>(u[k][q])] : &sink[lane], v ? 1u << sp_shift<SB>(u[k][q]) : 0u);
        }
    if (a.scores != nullptr) {
        // dense scores on request (parity tests): lane l writes ids 64l .. 64l + 63 below n
        uint8_t *row = a.scores + (int64_t)ql * a.ix.P * a.ix.TILE;
        for (int k = 0; k < 2; ++k) {
            const int64_t id0 = (int64_t)bb[k] * kSpBucket;
            for (int e = 0; e < 64; ++e) {
                const uint32_t lo = 64u * (uint32_t)lane + (uint32_t)e;
                if (id0 + lo < a.ix.n) row[id0 + lo] = (uint8_t)((win[k][sp_word<SB>(lo)] >> sp_shift<SB>(lo)) & SM);
            }
        }
    }
    uint32_t old[2][UQ];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            old[k][q] = 0u;
            if ((uint32_t)(q * kWave) >= len[k]) continue;
            const bool v = (uint32_t)(q * kWave + lane) < len[k];
            const uint32_t sh = sp_shift<SB>(u[k][q]);
            old[k][q] = atomicAnd(v ? &win[k][sp_word<SB>(u[k][q])] : &sink[lane], v ? ~(SM << sh) : ~0u);
        }
    uint32_t sv[2][UQ];
    uint64_t mh[2][UQ];
    uint32_t nh = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        n1[k] = 0u;
#pragma unroll
        for (int q = 0; q < UQ; ++q) {
            const bool v = (uint32_t)(q * kWave + lane) < len[k];
            sv[k][q] = v ? (old[k][q] >> sp_shift<SB>(u[k][q])) & SM : 0u;
            const uint64_t m1 = __ballot(sv[k][q] == 1u);
            mh[k][q] = __ballot(sv[k][q] >= 2u);
            nh += (uint32_t)__popcll(mh[k][q]);
            // the front entries lie below the bucket's end, whose slots were all read above
            if (sv[k][q] == 1u) seg[k][n1[k] + lanes_below(m1)] = (uint16_t)u[k][q];
            n1[k] += (uint32_t)__popcll(m1);
        }
    }
    if (nh) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(hn, nh);
        base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const uint32_t id0 = (uint32_t)bb[k] << kSpShift;
#pragma unroll
            for (int q = 0; q < UQ; ++q) {
                if (sv[k][q] >= 2u) {
                    const uint32_t at = base + lanes_below(mh[k][q]);
                    if (at < hcap) hl[at] = ((id0 | u[k][q]) << SB) | sv[k][q];
                    atomicAdd(&H[sv[k][q]], 1u);
                }
                base += (uint32_t)__popcll(mh[k][q]);
            }
        }
    }
}

// The id below which a set's `take` lowest ids lie (its take-th lowest + 1),
// for ids inside one bucket: one wave marks their low bits in a 4096-bit map
// (its clear window), counts set bits in id order and clears the map.
// mark(j) returns the low id of element j, or kSpBucket to skip it.
template <class M>
__device__ __forceinline__ uint32_t sp_cut(uint32_t cnt, uint32_t take, uint32_t *bm, M &&mark) {
    const int lane = threadIdx.x & (kWave - 1);
    for (uint32_t j = (uint32_t)lane; j < cnt; j += kWave) {
        const uint32_t lo = mark(j);
        if (lo < (uint32_t)kSpBucket) atomicOr(&bm[lo >> 5], 1u << (lo & 31u));
    }
    const uint32_t w0 = bm[2 * lane], w1 = bm[2 * lane + 1];        // ids 64l .. 64l + 63
    const uint32_t c = (uint32_t)(__popc(w0) + __popc(w1));
    const uint32_t incl = wave_incl_scan(c);
    const uint32_t k = take - 1u;                                  // 0-based rank of the last taken
    const uint64_t hit = __ballot(incl > k && incl - c <= k);
    const int src = __builtin_ctzll(hit);
    uint32_t cut = 0;
    if (lane == src) {
        uint64_t m = ((uint64_t)w1 << 32) | w0;
        for (uint32_t r = k - (incl - c); r > 0; --r) m &= m - 1ull;
        cut = (uint32_t)(64 * lane) + (uint32_t)__builtin_ctzll(m) + 1u;
    }
    bm[2 * lane] = 0u;
    bm[2 * lane + 1] = 0u;
    return (uint32_t)__builtin_amdgcn_readlane((int)cut, src);
}

// Append the selected ones of a wave's 64 candidates (one per lane) to the
// query's list: one atomic per wave for the positions.
__device__ __forceinline__ void sp_emit(bool t, uint32_t id, uint32_t *cq, uint32_t B, uint32_t *out) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t m = __ballot(t);
    if (m == 0ull) return;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(out, (uint32_t)__popcll(m));
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
    const uint32_t at = base + lanes_below(m);
    if (t && at < B) cq[at] = id;
}

// A query the sparse step leaves: route 1 and appended to the tiled steps' list.
__device__ __forceinline__ void leave_to_tiled(const QueryPass &a, const int ql) {
    a.route[ql] = 1;
    a.tlist[atomicAdd(a.ntl, 1)] = ql;
}

constexpr int kSpPairSlots = kSpWaves * (kSpBucket / 8) * 2;   // 16-bit slots of the second 4-bit windows
constexpr int kSpPairMinList = 4096;                             // list entries a query keeps when paired

template <int SB>
__global__ __launch_bounds__(kSpThreads) void k_collide_sparse(QueryPass a) {
    constexpr uint32_t SM = (1u << SB) - 1u;
    constexpr int WW = sp_win_words(SB);
    constexpr int kMaxNsSB = SB == 4 ? kSpMaxNs : kSpMaxNs5;
    extern __shared__ uint4 sp_dyn[];
    __shared__ SparseLds S;
    const int NB = a.ix.NB, ns = a.ix.ns, K = a.ix.K;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int NBp = sp_nb_padded(NB);
    uint2 *runs = reinterpret_cast<uint2 *>(sp_dyn);                      // [kSpMaxRuns] (start, first position)
    uint32_t *rcell = reinterpret_cast<uint32_t *>(runs + kSpMaxRuns);     // [kSpMaxRuns] the run's cell (i*K + c)
    uint32_t *bfill = rcell + kSpMaxRuns;                                  // [NB] the walk's cursor in each bucket
    uint32_t *boff = bfill + NBp;                                          // [NB] first slot of each bucket
    uint32_t *bx = boff + NBp;                                             // [NB] points of score 1, then level-T points
    uint32_t *win_all = bx + NBp;                                          // [kSpWaves][WW], 16-byte aligned
    uint16_t *raw = reinterpret_cast<uint16_t *>(win_all + kSpWaves * WW); // slots: each bucket's low ids, then its score-1 points
    uint32_t *win = win_all + w * WW;
    const int nq = pass_nq(a.nq_dev, a.q_base, a.nq);
    const int per = (NB + kSpThreads - 1) / kSpThreads;
    const int b0t = tid * per < NB ? tid * per : NB, b1t = b0t + per < NB ? b0t + per : NB;
    for (int j = tid; j < kSpWaves * WW; j += kSpThreads) win_all[j] = 0u;
    for (int j = tid; j < kWave; j += kSpThreads) S.sink[j] = 0u;
    for (int rq = blockIdx.x; rq < nq; rq += gridDim.x) {
        const int ql = a.order ? a.order[rq] : rq;
        // ---- the query's size: activated cells (wave 0, a lane per subspace)
        if (w == 0) {
            const bool on = lane < ns && ns <= kMaxNsSB;
            const uint32_t c = on ? (uint32_t)a.ncells[ql * ns + lane] : 0u;
            const uint32_t ci = wave_incl_scan(c);
            if (lane <= kMaxNsSB) S.cpre[lane] = ci - c;
            const uint32_t nr = (uint32_t)__builtin_amdgcn_readlane((int)ci, kWave - 1);
            if (lane == 0) {
                S.nruns = (int)nr;
                S.flag = (ns > kMaxNsSB || nr >= (uint32_t)kSpMaxRuns || a.sp_cap == 0) ? 1 : 0;
                S.nh = 0u;
                S.out = 0u;
            }
        }
        for (int t = tid; t < kMaxNsSB + 2; t += kSpThreads) S.H[t] = 0u;
        __syncthreads();
        if (S.flag) {
            if (tid == 0) leave_to_tiled(a, ql);
            __syncthreads();
            continue;
        }
        // ---- runs of the activated cells (a thread per run, nruns < kSpThreads)
        // and their first positions in the sequence of all activated ids
        const int nruns = S.nruns;
        uint32_t rstart = 0u, rlen = 0u;
        if (tid < nruns) {
            int i = 0;
            while (i + 1 < ns && S.cpre[i + 1] <= (uint32_t)tid) ++i;
            const int j = tid - (int)S.cpre[i];
            const int c = a.cells[((int64_t)ql * ns + i) * K + j];
            const uint32_t *co = a.ix.coffs + (int64_t)i * (K + 1);
            rstart = co[c];
            rlen = co[c + 1] - rstart;
            rstart = rlen ? (uint32_t)((int64_t)i * a.ix.n) + rstart : 0u;   // an empty run points at id 0's slot
            rcell[tid] = (uint32_t)(i * K + c);
        }
        uint32_t total;
        const uint32_t rpos = block_excl_scan<kSpThreads>(rlen, S.red, &total);
        if (total > (uint32_t)a.sp_cap) {            // more activated ids than the slots hold
            if (tid == 0) leave_to_tiled(a, ql);
            __syncthreads();
            continue;
        }
        // the list of points of score >= 2 takes the slots past the query's own;
        // when enough are left, the last kSpPairSlots of them hold a second
        // window per wave and the buckets go two at a time
        const uint32_t tot2 = (total + 1u) & ~1u;
        uint32_t *hl = reinterpret_cast<uint32_t *>(raw + tot2);                // (id << SB | score), score >= 2
        const uint32_t hcap1 = tot2 < (uint32_t)a.sp_cap ? ((uint32_t)a.sp_cap - tot2) / 2u : 0u;
        const bool paired = SB == 4 && hcap1 >= (uint32_t)(kSpPairSlots / 2 + kSpPairMinList);
        const uint32_t hcap = paired ? hcap1 - (uint32_t)(kSpPairSlots / 2) : hcap1;
        if (tid <= nruns) runs[tid] = make_uint2(tid < nruns ? rstart : 0u, tid < nruns ? rpos : total);
        for (uint32_t q = (rpos + 1023u) >> 10; rlen && (q << 10) < rpos + rlen; ++q) S.crun[q] = (uint32_t)tid;
        __syncthreads();
        // ---- exact bucket sizes, from the index's count of each cell's ids per
        // bucket summed over the query's runs: a wave takes four buckets at a
        // time, a lane per run reads their four counts (one 8-byte load, two
        // 16-bit counts a word: a bucket's total stays below 2^16, so the packed
        // halves add without carry) and two wave sums finish them; then the
        // buckets' offsets in the slots
        {
            // a wave's four groups of four buckets j0, j0 + 16, ... at once: their
            // loads are issued together (a group past the end reloads group j0)
            const int nb4 = (NB + 3) >> 2;
            for (int j0 = w; j0 < nb4; j0 += 4 * kSpWaves) {
                uint32_t lo[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u};
                for (int r = lane; r < nruns; r += kWave) {
                    const uint16_t *row = a.ix.cbh + (size_t)rcell[r] * NBp;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int j = j0 + u * kSpWaves < nb4 ? j0 + u * kSpWaves : j0;
                        const uint2 v = *reinterpret_cast<const uint2 *>(row + 4 * j);
                        lo[u] += v.x;
                        hi[u] += v.y;
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + u * kSpWaves;
                    const uint32_t l = wave_sum(lo[u]), h = wave_sum(hi[u]);
                    if (lane == 0 && j < nb4) {
                        bx[4 * j] = l & 0xffffu;
                        bx[4 * j + 1] = l >> 16;
                        bx[4 * j + 2] = h & 0xffffu;
                        bx[4 * j + 3] = h >> 16;
                    }
                }
            }
        }
        __syncthreads();
        {
            uint32_t mine = 0;
            for (int b = b0t; b < b1t; ++b) mine += bx[b];
            uint32_t all;
            uint32_t off = block_excl_scan<kSpThreads>(mine, S.red, &all);
            for (int b = b0t; b < b1t; ++b) {
                const uint32_t f = bx[b];
                boff[b] = off;
                bfill[b] = off;
                off += f;
            }
        }
        __syncthreads();
        // ---- 1. one walk into the buckets' slots (the cursor of a bucket starts
        // at its first slot); all sixteen atomics of a step are issued before
        // the stores they place
        sp_walk(a, runs, S.crun, total, [&](const uint32_t (&id)[2 * kSpU], uint32_t vm, uint32_t um) {
            uint32_t pos[2 * kSpU];
#pragma unroll
            for (int u = 0; u < 2 * kSpU; ++u) {
                const bool v = (vm >> u) & 1u;
                pos[u] = 0u;
                if ((um >> u) & 1u) pos[u] = atomicAdd(v ? &bfill[id[u] >> kSpShift] : &S.sink[lane], v ? 1u : 0u);
            }
#pragma unroll
            for (int u = 0; u < 2 * kSpU; ++u)    // (the sizes are exact, so pos < total <= sp_cap; kept as a guard)
                if (((vm >> u) & 1u) && pos[u] < (uint32_t)a.sp_cap) raw[pos[u]] = (uint16_t)(id[u] & (kSpBucket - 1));
        });
        __syncthreads();
        // ---- 2. every bucket
        if (paired) {
            uint32_t *win2all = reinterpret_cast<uint32_t *>(raw + a.sp_cap - kSpPairSlots);
            uint4 *z = reinterpret_cast<uint4 *>(win2all);          // slots of earlier queries: cleared
            for (int j = tid; j < kSpPairSlots / 8; j += kSpThreads) z[j] = make_uint4(0u, 0u, 0u, 0u);
            __syncthreads();
            uint32_t *win2 = win2all + w * WW;
            for (int b = w; b < NB; b += 2 * kSpWaves) {
                const int b1 = b + kSpWaves;
                const uint32_t l0 = bfill[b] - boff[b], l1 = b1 < NB ? bfill[b1] - boff[b1] : 0u;
                uint32_t n1[2] = {0u, 0u};
                if (b1 < NB && l0 <= 4u * kWave && l1 <= 4u * kWave) {
                    sp_bucket_pair<SB>(a, ql, b, b1, raw + boff[b], l0, raw + boff[b1], l1, win, win2, hl, hcap, &S.nh,
                                       S.H, S.sink, n1);
                } else {
                    n1[0] = sp_bucket<SB>(a, ql, b, raw + boff[b], l0, win, hl, hcap, &S.nh, S.H, S.sink);
                    if (b1 < NB) n1[1] = sp_bucket<SB>(a, ql, b1, raw + boff[b1], l1, win2, hl, hcap, &S.nh, S.H, S.sink);
                }
                if (lane == 0) {
                    bx[b] = n1[0];
                    if (b1 < NB) bx[b1] = n1[1];
                }
            }
        } else {
            for (int b = w; b < NB; b += kSpWaves) {
                const uint32_t n1 = sp_bucket<SB>(a, ql, b, raw + boff[b], bfill[b] - boff[b], win, hl, hcap, &S.nh, S.H, S.sink);
                if (lane == 0) bx[b] = n1;
            }
        }
        __syncthreads();
        // ---- 3. threshold: G[t] = sum of H[s] for s >= t >= 2; G[1] adds the score-1 points
        const uint32_t B = (uint32_t)a.B;
        int T = 0;
        uint32_t GT1 = 0;                    // G[T + 1]
        uint32_t R0 = 0;                     // points of score 0 to take (fewer than B collide)
        {
            uint32_t g = 0;
            for (int t = ns; t >= 2; --t) {
                if (g + S.H[t] >= B) { T = t; GT1 = g; break; }
                g += S.H[t];
            }
            if (T == 0) {
                uint32_t e = 0;
                for (int b = b0t; b < b1t; ++b) e += bx[b];
                e = block_sum<kSpThreads>(e, S.red);
                if (g + e >= B) { T = 1; GT1 = g; }
                else { T = 1; GT1 = g; R0 = B - g - e; }    // every colliding point, then R0 of score 0
            }
        }
        const uint32_t nhl = S.nh;
        const uint32_t nb0 = (B + (uint32_t)kSpBucket - 1u) >> kSpShift;   // buckets below B
        if (nhl > hcap || (R0 > 0u && nb0 > (uint32_t)kSpWaves)) {
            if (tid == 0) leave_to_tiled(a, ql);
            __syncthreads();
            continue;
        }
        const uint32_t R = B - GT1 - R0;
        // level-T points per bucket: the score-1 counts, or counted over the list
        if (T > 1) {
            for (int b = b0t; b < b1t; ++b) bx[b] = 0u;
            __syncthreads();
            for (uint32_t j = (uint32_t)tid; j < nhl; j += kSpThreads)
                if ((hl[j] & SM) == (uint32_t)T) atomicAdd(&bx[hl[j] >> (SB + kSpShift)], 1u);
            __syncthreads();
        }
        // each bucket's share of the R lowest level-T ids (bfill: take), and the cut bucket
        {
            uint32_t eql = 0;
            for (int b = b0t; b < b1t; ++b) eql += bx[b];
            uint32_t tot;
            uint32_t eb = block_excl_scan<kSpThreads>(eql, S.red, &tot);
            for (int b = b0t; b < b1t; ++b) {
                const uint32_t eq = bx[b];
                const uint32_t take = eb >= R ? 0u : (R - eb < eq ? R - eb : eq);
                eb += eq;
                bfill[b] = take;
            }
            if (tid == 0) S.cutb = -1;
        }
        __syncthreads();
        // the cut bucket: the one (at most) that takes some but not all of its level-T points
        for (int b = b0t; b < b1t; ++b)
            if (bfill[b] != 0u && bfill[b] != bx[b]) S.cutb = b;
        __syncthreads();
        const int cutb = S.cutb;
        if (w == 0) {
            uint32_t cut = 0;
            if (cutb >= 0) {
                const uint32_t take = bfill[cutb];
                if (T == 1) {
                    const uint16_t *f = raw + boff[cutb];
                    cut = sp_cut(bx[cutb], take, win, [&](uint32_t j) { return (uint32_t)f[j]; });
                } else {
                    cut = sp_cut(nhl, take, win, [&](uint32_t j) {
                        const uint32_t e = hl[j];
                        return ((e & SM) == (uint32_t)T && (int)(e >> (SB + kSpShift)) == cutb)
                                   ? (e >> SB) & (kSpBucket - 1) : (uint32_t)kSpBucket;
                    });
                }
            }
            if (lane == 0) S.cut = cut;
        }
        __syncthreads();
        const uint32_t cut = S.cut;
        // ---- candidates: the listed points above T, and the level-T points of
        // buckets before the cut bucket and below the cut inside it
        uint32_t *cq = a.cand + (int64_t)ql * a.B;
        auto take_t = [&](uint32_t id) {
            const int b = (int)(id >> kSpShift);
            return bfill[b] == bx[b] ? bfill[b] != 0u : (b == cutb && (id & (kSpBucket - 1)) < cut);
        };
        for (uint32_t j0 = (uint32_t)(w * kWave); j0 < nhl; j0 += (uint32_t)kSpThreads) {
            const uint32_t j = j0 + (uint32_t)lane;
            const uint32_t e = hl[j < nhl ? j : 0u];
            const uint32_t sv = e & SM, id = e >> SB;
            const bool t = j < nhl && (sv > (uint32_t)T || (sv == (uint32_t)T && take_t(id)));
            sp_emit(t, id, cq, B, &S.out);
        }
        if (T == 1) {
            for (int b = w; b < NB; b += kSpWaves) {
                const uint32_t take = bfill[b], n1 = bx[b];
                if (take == 0u) continue;
                const uint16_t *f = raw + boff[b];
                const uint32_t id0 = (uint32_t)b << kSpShift;
                const uint32_t lim = take == n1 ? (uint32_t)kSpBucket : cut;
                for (uint32_t j0 = 0; j0 < n1; j0 += kWave) {
                    const uint32_t j = j0 + (uint32_t)lane;
                    const uint32_t lo = f[j < n1 ? j : 0u];
                    sp_emit(j < n1 && lo < lim, id0 | lo, cq, B, &S.out);
                }
            }
        }
        if (R0 > 0u) {
            // ---- fewer than B points collide: the R0 lowest ids of score 0 as well.
            // They lie below B; the colliding ids below B are marked in bitmaps, bucket
            // b's in wave b's window (clear), and wave b takes its bucket's share of
            // the unmarked ids in id order
            for (uint32_t j = (uint32_t)tid; j < nhl; j += kSpThreads) {
                const uint32_t id = hl[j] >> SB;
                if (id < B) atomicOr(&win_all[(id >> kSpShift) * WW + ((id & (kSpBucket - 1)) >> 5)], 1u << (id & 31u));
            }
            if ((uint32_t)w < nb0) {
                const uint16_t *f = raw + boff[w];
                const uint32_t n1 = bx[w], id0 = (uint32_t)w << kSpShift;
                for (uint32_t j = (uint32_t)lane; j < n1; j += kWave) {
                    const uint32_t lo = f[j];
                    if (id0 + lo < B) atomicOr(&win[lo >> 5], 1u << (lo & 31u));
                }
            }
            __syncthreads();
            uint64_t fr = 0;                 // this lane's unmarked ids below B: 64 * lane .. + 63 of the bucket
            const uint32_t idl = ((uint32_t)w << kSpShift) + 64u * (uint32_t)lane;
            if ((uint32_t)w < nb0) {
                const uint64_t mk = ((uint64_t)win[2 * lane + 1] << 32) | win[2 * lane];
                const uint32_t nv = B > idl ? (B - idl < 64u ? B - idl : 64u) : 0u;
                fr = ~mk & (nv == 64u ? ~0ull : ((1ull << nv) - 1ull));
                win[2 * lane] = 0u;
                win[2 * lane + 1] = 0u;
                const uint32_t z = wave_sum((uint32_t)__popcll(fr));
                if (lane == 0) S.zfree[w] = z;
            }
            __syncthreads();
            if ((uint32_t)w < nb0) {
                uint32_t pre = 0;
                for (int v = 0; v < w; ++v) pre += S.zfree[v];
                const uint32_t take = pre >= R0 ? 0u : (R0 - pre < S.zfree[w] ? R0 - pre : S.zfree[w]);
                if (take > 0u) {
                    const uint32_t c = (uint32_t)__popcll(fr);
                    uint32_t r = wave_incl_scan(c) - c;   // rank of this lane's first unmarked id
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(&S.out, take);
                    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
                    for (; fr != 0ull && r < take; ++r, fr &= fr - 1ull)
                        if (base + r < B) cq[base + r] = idl + (uint32_t)__builtin_ctzll(fr);
                }
            }
        }
        if (tid == 0) a.route[ql] = 0;
        __syncthreads();
    }
}

// Points in the activated cells of every (query, subspace): one wave each.
__global__ __launch_bounds__(kWave) void k_cell_points(SizesPass a) {
    const int item = blockIdx.x, q = item / a.ix.ns, i = item - q * a.ix.ns;
    if (a.ntl != nullptr && item == 0 && threadIdx.x == 0) *a.ntl = 0;
    if (q >= a.nq) return;
    const int nc = a.ncells[item];
    const uint16_t *cl = a.cells + (int64_t)item * a.ix.K;
    uint32_t s = 0;
    for (int j = threadIdx.x; j < nc; j += kWave) s += a.ix.csize[(int64_t)i * a.ix.K + cl[j]];
    s = wave_sum(s);
    if (threadIdx.x == 0) a.aprime[item] = (int32_t)s;
}

// ================================================================= order ==
// One block of kOrderMax threads: the pass's queries sorted by their number of
// activated points (descending, ties by query), so that the collision step's
// blocks take the heaviest queries first and a pass does not end waiting for a
// few large ones (queries with their own collision ratio differ a lot).
__global__ __launch_bounds__(kOrderMax) void k_order(QueryPass a) {
    __shared__ uint64_t key[kOrderMax];
    const int nq = pass_nq(a.nq_dev, a.q_base, a.nq), ns = a.ix.ns;
    const int t = threadIdx.x;
    uint64_t w = 0;
    if (t < nq)
        for (int i = 0; i < ns; ++i) w += (uint32_t)a.aprime[t * ns + i];
    // ascending keys: heavier first, then lower query index; empty slots last
    key[t] = t < nq ? (((~w) & 0xffffffffffull) << 20) | (uint64_t)t : ~0ull;
    __syncthreads();
    for (int size = 2; size <= kOrderMax; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int j = t ^ stride;
            if (j > t) {
                const uint64_t x = key[t], y = key[j];
                const bool up = (t & size) == 0;
                if ((x > y) == up) { key[t] = y; key[j] = x; }
            }
            __syncthreads();
        }
    }
    if (t < nq) a.order_out[t] = (int32_t)(key[t] & 0xfffffull);
}

// Wider passes (up to kOrderWide queries): the queries bucketed by
// floor(log2(activated points)), heaviest bucket first; inside a bucket the
// order is whatever the atomics give, which only decides which block takes
// which query first (every query's results are its own).
__global__ __launch_bounds__(1024) void k_order_wide(QueryPass a) {
    __shared__ uint32_t cnt[32];
    __shared__ uint8_t key[kOrderWide];
    const int nq = pass_nq(a.nq_dev, a.q_base, a.nq), ns = a.ix.ns;
    if (threadIdx.x < 32) cnt[threadIdx.x] = 0u;
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += 1024) {
        uint32_t w = 0;
        for (int i = 0; i < ns; ++i) w += (uint32_t)a.aprime[q * ns + i];
        const uint32_t kq = (uint32_t)__clz(w | 1u);      // 31 - floor(log2 w): heavier first
        key[q] = (uint8_t)kq;
        atomicAdd(&cnt[kq], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int j = 0; j < 32; ++j) {
            const uint32_t c = cnt[j];
            cnt[j] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += 1024) a.order_out[atomicAdd(&cnt[key[q]], 1u)] = q;
}

// ================================================================ select ==
// One block per query.  The threshold is T = max{t : sum_p G_p[t] >= B};
// every point with score > T is a candidate and, of those with score == T,
// the R = B - #{score > T} lowest ids.  Tiles contribute in id order: each
// takes gt (its ids above T) plus take (its share of the level-T ids) at an
// offset known from the histograms, so the tiles are independent and each
// wave of the block takes its own tiles with its own LDS bitmap (no block
// barrier inside a tile).  A tile's chosen ids are marked in the bitmap (score
// > T from the front of the tile's list, level-T ids up to a cut) with a
// summary bitmap of non-zero words, and the wave walks the summaries in id
// order: the work per tile follows the number of candidates, not the tile
// size, and the bitmap is cleared through its summary.  When only some of the
// tile's level-T ids are taken, they are first marked alone to find the cut
// (the id of the take-th lowest).  When T == 0 the points of score 0 are the
// ones missing from the tile's list; such a tile is handled densely.
struct SelectTile {
    int p;
    uint32_t gt, E, take, base;
};

// One wave: the candidates of tile t.p in id order at out + t.base.  bm
// (TILE bits) and sm (64 words) are the wave's own and are left zero.
__device__ __forceinline__ void select_tile(const QueryPass &a, const int ql, const int T, const SelectTile t,
                                            uint32_t *bm, uint32_t *sm, uint32_t *out) {
    const int P = a.ix.P, TILE = a.ix.TILE;
    const int lane = threadIdx.x & (kWave - 1);
    const int bwords = TILE >> 5, swords = (bwords + 31) >> 5;   // swords <= 64
    const uint16_t *seg = a.lvl + ((int64_t)ql * P + t.p) * TILE;
    const uint32_t id0 = (uint32_t)t.p * TILE;
    const int64_t vv = a.ix.n - (int64_t)id0;
    const int valid = (int)(vv < TILE ? vv : TILE);
    const bool partial = t.take > 0u && (t.take < t.E || T == 0);
    auto mark = [&](uint32_t lid) {
        atomicOr(&bm[lid >> 5], 1u << (lid & 31u));
        atomicOr(&sm[lid >> 10], 1u << ((lid >> 5) & 31u));
    };
    if (T == 0 && partial) {
        // fewer than B points collide: the tile's score-0 ids are taken too,
        // lowest first; dense bitmap, a range of words per lane
        const int per = (bwords + kWave - 1) / kWave;
        const int w0 = lane * per < bwords ? lane * per : bwords;
        const int w1 = w0 + per < bwords ? w0 + per : bwords;
        for (uint32_t j = lane; j < t.gt; j += kWave) {
            const uint32_t lid = seg[j];
            atomicOr(&bm[lid >> 5], 1u << (lid & 31u));
        }
        __builtin_amdgcn_wave_barrier();
        auto zeros = [&](int w) {   // this word's score-0 ids inside the tile
            const uint32_t m = (w + 1) * 32 <= valid ? ~0u : (w * 32 >= valid ? 0u : (1u << (valid - w * 32)) - 1u);
            return ~bm[w] & m;
        };
        uint32_t cnt = 0;
        for (int w = w0; w < w1; ++w) cnt += __popc(zeros(w));
        uint32_t r = wave_incl_scan(cnt) - cnt;
        for (int w = w0; w < w1; ++w) {
            uint32_t x = zeros(w), keep = 0u;
            while (x != 0u && r < t.take) {
                const uint32_t bit = x & (0u - x);
                keep |= bit;
                x ^= bit;
                ++r;
            }
            bm[w] |= keep;
        }
        cnt = 0;
        for (int w = w0; w < w1; ++w) cnt += __popc(bm[w]);
        uint32_t pos = t.base + wave_incl_scan(cnt) - cnt;
        for (int w = w0; w < w1; ++w) {
            uint32_t x = bm[w];
            while (x != 0u) {
                const int bq = __ffs(x) - 1;
                out[pos++] = id0 + (uint32_t)(w * 32 + bq);
                x &= x - 1u;
            }
            bm[w] = 0u;
        }
        __builtin_amdgcn_wave_barrier();
        return;
    }
    // sparse tile.  Some of the level-T ids: mark them all, find the id of
    // the take-th lowest (cut) by walking the summaries in id order, clear.
    uint32_t cut = 0xffffffffu;
    if (partial) {
        for (uint32_t j = t.gt + lane; j < t.gt + t.E; j += kWave) mark(seg[j]);
        __builtin_amdgcn_wave_barrier();
        // lane l owns summary word l
        const uint32_t sl = lane < swords ? sm[lane] : 0u;
        uint32_t c = 0;
        for (uint32_t x = sl; x != 0u; x &= x - 1u) c += __popc(bm[lane * 32 + __ffs(x) - 1]);
        uint32_t r = wave_incl_scan(c) - c;               // level-T ids before this lane's words
        uint32_t mine = 0u;                               // cut + 1 in the lane that holds it
        for (uint32_t x = sl; x != 0u; x &= x - 1u) {
            const int w = lane * 32 + __ffs(x) - 1;
            const uint32_t y = bm[w];
            bm[w] = 0u;
            const uint32_t cy = (uint32_t)__popc(y);
            if (r < t.take && r + cy >= t.take) {
                // the cut lies in this word: its (take - r)-th set bit
                uint32_t z = y;
                for (uint32_t k2 = t.take - r; k2 > 1u; --k2) z &= z - 1u;
                mine = 1u + (uint32_t)(w * 32 + __ffs(z) - 1);
            }
            r += cy;
        }
        if (lane < swords) sm[lane] = 0u;
        // exactly one lane found it (0 < take < E, and the tile lists its E
        // level-T ids whenever it takes some of them)
        const uint64_t who = __ballot(mine != 0u);
        if (who != 0ull) cut = (uint32_t)__builtin_amdgcn_readlane((int)mine, __ffsll((unsigned long long)who) - 1) - 1u;
        __builtin_amdgcn_wave_barrier();
    }
    // mark the candidates: ids above T, and the level-T ids up to the cut
    const uint32_t hiA = partial ? t.gt : t.gt + t.take;
    for (uint32_t j = lane; j < hiA; j += kWave) mark(seg[j]);
    if (partial)
        for (uint32_t j = t.gt + lane; j < t.gt + t.E; j += kWave) {
            const uint32_t lid = seg[j];
            if (lid <= cut) mark(lid);
        }
    __builtin_amdgcn_wave_barrier();
    // candidates in id order: lane l writes the ids of its summary word
    const uint32_t sl = lane < swords ? sm[lane] : 0u;
    uint32_t c = 0;
    for (uint32_t x = sl; x != 0u; x &= x - 1u) c += __popc(bm[lane * 32 + __ffs(x) - 1]);
    uint32_t pos = t.base + wave_incl_scan(c) - c;
    for (uint32_t x = sl; x != 0u; x &= x - 1u) {
        const int w = lane * 32 + __ffs(x) - 1;
        uint32_t y = bm[w];
        bm[w] = 0u;
        while (y != 0u) {
            const int bq = __ffs(y) - 1;
            out[pos++] = id0 + (uint32_t)(w * 32 + bq);
            y &= y - 1u;
        }
    }
    if (lane < swords) sm[lane] = 0u;
    __builtin_amdgcn_wave_barrier();
}

template <int NT>
__device__ __forceinline__ void select_item(const QueryPass &a, const int ql, const int g, const int S, uint32_t *bm,
                                            uint32_t *sum) {
    __shared__ uint32_t Gt[kMaxNs + 2];
    __shared__ uint32_t red[NT / kWave + 1];
    const int P = a.ix.P, ns = a.ix.ns, TILE = a.ix.TILE, H = ns + 2;
    const int tid = threadIdx.x, wv = tid / kWave;
    const int bwords = TILE >> 5;
    uint32_t *bmw = bm + (int64_t)wv * bwords, *smw = sum + wv * 64;
    const uint32_t B = (uint32_t)a.B;
    const uint32_t *hq = a.hist + (int64_t)ql * P * H;
    // Gt[t] = sum over the tiles of G_p[t]: the P*H histogram words are read
    // by all threads at once (contiguous) and added up in LDS
    for (int t = tid; t < H; t += NT) Gt[t] = 0u;
    __syncthreads();
    for (int j = tid; j < P * H; j += NT) atomicAdd(&Gt[j % H], hq[j]);
    __syncthreads();
    int T = 0;
    for (int t = ns; t >= 0; --t)
        if (Gt[t] >= B) { T = t; break; }
    const uint32_t R = B - Gt[T + 1];
    uint32_t *out = a.cand + (int64_t)ql * a.B;
    // Per-tile plan for NT tiles at a time, from the histograms in parallel:
    // ids above T (gt), at T (E), level-T ids taken (the lowest R overall, so a
    // tile takes what the tiles before it left) and the tile's output offset.
    __shared__ uint32_t pl_gt[NT], pl_E[NT], pl_take[NT], pl_base[NT];
    uint32_t base_carry = 0, eq_carry = 0;
    for (int p0 = 0; p0 < P; p0 += NT) {
        const int np = P - p0 < NT ? P - p0 : NT;
        {
            uint32_t gt_t = 0, E_t = 0;
            if (tid < np) {
                const uint32_t *h = hq + (int64_t)(p0 + tid) * H;
                gt_t = h[T + 1];
                E_t = h[T] - gt_t;
            }
            uint32_t totE, totS;
            const uint32_t eqb = eq_carry + block_excl_scan<NT>(E_t, red, &totE);
            const uint32_t left = R > eqb ? R - eqb : 0u;
            const uint32_t take_t = E_t < left ? E_t : left;
            const uint32_t exS = block_excl_scan<NT>(gt_t + take_t, red, &totS);
            if (tid < np) {
                pl_gt[tid] = gt_t;
                pl_E[tid] = E_t;
                pl_take[tid] = take_t;
                pl_base[tid] = base_carry + exS;
            }
            base_carry += totS;
            eq_carry += totE;
            __syncthreads();
        }
        // this block's tiles: p = g, g + S, ... (S tile groups per query)
        const int first = ((g - p0) % S + S) % S;
        for (int pi = first + wv * S; pi < np; pi += S * (NT / kWave)) {
            const SelectTile t{p0 + pi, pl_gt[pi], pl_E[pi], pl_take[pi], pl_base[pi]};
            if (t.gt + t.take == 0u) continue;
            select_tile(a, ql, T, t, bmw, smw, out);
        }
        __syncthreads();
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_select(QueryPass a) {
    extern __shared__ uint32_t bm[];       // per wave: a bitmap of TILE bits
    __shared__ uint32_t sum[(NT / kWave) * 64];    // per wave: its summary (bit w of word s = bitmap word 32s + w non-zero)
    // the queries the sparse step left are few: each is spread over S groups
    // of its tiles (one tile per wave at the most), each block planning all
    // tiles from the histograms and selecting in its own
    const int nt = a.tlist != nullptr ? *a.ntl : pass_nq(a.nq_dev, a.q_base, a.nq);
    const int smax = (a.ix.P + NT / kWave - 1) / (NT / kWave);
    const int S = a.tlist != nullptr && nt > 0 ? min(smax, max(1, (4096 + nt - 1) / nt)) : 1;
    const int items = nt * S;
    if ((int)blockIdx.x >= items) return;
    for (int w = threadIdx.x; w < (NT / kWave) * (a.ix.TILE >> 5); w += NT) bm[w] = 0u;
    for (int w = threadIdx.x; w < (NT / kWave) * 64; w += NT) sum[w] = 0u;
    __syncthreads();
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int rq = item / S, g = item - rq * S;
        select_item<NT>(a, a.tlist != nullptr ? a.tlist[rq] : rq, g, S, bm, sum);
        __syncthreads();
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
// ROWS8: the rows are read from the index's byte copy of X (kept when every
// coordinate is an integer in 0..255); each byte converts to FP32 exactly, so
// the arithmetic, its order and the result are those of the FP32 rows, with a
// quarter of the bytes moved.
// UM: most slices per lane (U <= UM); NRG = kMaxU / UM row groups are taken
// per wave iteration, and the loads of all of them are issued before any
// arithmetic so that more bytes are in flight per wave.
// Insertion: a key can enter the wave's list only if it is below the current
// k-th key, so one ballot per iteration finds the few rows that need the
// (cross-lane) insertion; the others cost nothing more.  The list is the set
// of the k smallest keys seen, whatever the insertion order (keys are unique).
//
// Byte rows and a query whose values are all integers in 0..255, with d a
// multiple of 16 and at most 256: every squared difference and every partial
// sum of the FP32 computation is an integer below 2^24, so that computation
// is exact and equals the integer sum of (x - q)^2 = x.x - 2 x.q + q.q, which
// is taken here with 4-byte dot products (v_dot4_u32_u8) on 16-byte slices:
// the same keys as the FP32 arithmetic, with a fraction of the instructions.
constexpr int kIntSlices = 2;                // 16-byte slices per lane
constexpr int kIntGroups = kMaxU / kIntSlices;   // row groups per wave iteration

__device__ __forceinline__ uint32_t dot16(const uint4 a, const uint4 b, uint32_t c) {
    c = __builtin_amdgcn_udot4(a.x, b.x, c, false);
    c = __builtin_amdgcn_udot4(a.y, b.y, c, false);
    c = __builtin_amdgcn_udot4(a.z, b.z, c, false);
    return __builtin_amdgcn_udot4(a.w, b.w, c, false);
}

// Lanes per row of the integer path: the smallest power of two with at most
// kIntSlices slices per lane (d/16 <= 16, so at most 8).
__device__ __forceinline__ int int_group(int d16) {
    int G = 1;
    while (G * kIntSlices < d16) G *= 2;
    return G;
}

template <int NT>
__device__ __forceinline__ void rerank_rows_int(const RerankPass &r, const uint32_t *cid, const int cn,
                                                const uint4 (&qb)[kIntSlices], const uint32_t qq, const int G,
                                                uint64_t &best) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int R = kWave / G, li = lane & (G - 1), slot = lane / G;
    const int d16 = r.d >> 4, k = r.k;
    const bool full = d16 == G * kIntSlices;   // every lane's slices lie in the row
    for (int base = wv * R * kIntGroups; base < cn; base += (NT / kWave) * R * kIntGroups) {
        uint32_t id[kIntGroups];
        bool valid[kIntGroups];
        uint4 x[kIntGroups][kIntSlices];
        // the LDS reads and the row loads are all issued before any is waited
        // for: a slot past the chunk reads an id it does not use, a slice past
        // the row reads the row's first one and is not counted
#pragma unroll
        for (int g = 0; g < kIntGroups; ++g) {
            const int rw = base + g * R + slot;
            id[g] = cid[rw < kRowChunk ? rw : kRowChunk - 1];
            valid[g] = rw < cn && id[g] < r.n;   // ids outside [0, n) are ignored
        }
#pragma unroll
        for (int g = 0; g < kIntGroups; ++g) {
            id[g] = valid[g] ? id[g] : 0u;
#pragma unroll
            for (int u = 0; u < kIntSlices; ++u) {
                const int j = li + G * u;
                x[g][u] = reinterpret_cast<const uint4 *>(r.X8 + (int64_t)id[g] * r.d)[j < d16 ? j : 0];
            }
        }
        uint64_t key[kIntGroups];
#pragma unroll
        for (int g = 0; g < kIntGroups; ++g) {
            uint32_t s = qq;
#pragma unroll
            for (int u = 0; u < kIntSlices; ++u) {
                const uint32_t t = dot16(x[g][u], x[g][u], 0u) - 2u * dot16(x[g][u], qb[u], 0u);
                s += (full || li + G * u < d16) ? t : 0u;
            }
            s = group_sum(s, G);
            key[g] = valid[g] ? (((uint64_t)__float_as_uint((float)s) << 32) | id[g]) : ~0ull;
        }
#pragma unroll
        for (int g = 0; g < kIntGroups; ++g) {
            const uint64_t kth = shfl64(best, k - 1);
            uint64_t m = __ballot(li == 0 && key[g] < kth);
            while (m != 0ull) {
                const int src = __ffsll((unsigned long long)m) - 1;
                m &= m - 1ull;
                topk_insert(best, shfl64(key[g], src), k, lane);
            }
        }
    }
}

template <int NT, bool ROWS8, int UM>
__device__ __forceinline__ void rerank_item(const RerankPass &r, const int item) {
    constexpr int NRG = kMaxU / UM;
    __shared__ uint64_t wl[NT / kWave][kMaxK];
    // candidate ids are staged in LDS a chunk at a time (one coalesced read),
    // so each row's load depends on an LDS read rather than a global one
    __shared__ uint32_t cid[kRowChunk];
    const int ql = item / r.parts, part = item - ql * r.parts;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int k = r.k;
    uint64_t best = ~0ull;
    const int64_t rb = (int64_t)part * r.rows_per_part;
    const int64_t rows = r.rows_dev ? (r.rows_dev[ql] < r.B ? (int64_t)r.rows_dev[ql] : r.B) : r.B;
    const int64_t re = rb + r.rows_per_part < rows ? rb + r.rows_per_part : rows;
    const uint32_t *cq = r.cand + (int64_t)ql * r.B;
    auto stage = [&](int64_t cb) -> int {
        const int cn = (int)(re - cb < kRowChunk ? re - cb : kRowChunk);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += NT) cid[t] = cq[cb + t];
        __syncthreads();
        return cn;
    };
    bool int_path = false;
    if constexpr (ROWS8) {
        if (r.metric == 0 && (r.d & 15) == 0 && r.d <= 256) {
            const float *qf = r.Q + (int64_t)ql * r.d;
            bool ok = true;
            for (int t = threadIdx.x; t < r.d; t += NT) {
                const float v = qf[t];
                ok = ok && v >= 0.f && v <= 255.f && v == rintf(v);
            }
            int_path = __syncthreads_and(ok);
        }
    }
    if (ROWS8 && int_path) {
        // the query's slices as bytes and their squared norm
        const int d16 = r.d >> 4;
        const int Gi = int_group(d16), lii = lane & (Gi - 1);
        uint4 qb[kIntSlices];
        uint32_t qq = 0u;
#pragma unroll
        for (int u = 0; u < kIntSlices; ++u) {
            const int j = lii + Gi * u;
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            if (j < d16) {
                const float4 *q4s = reinterpret_cast<const float4 *>(r.Q + (int64_t)ql * r.d + 16 * j);
#pragma unroll
                for (int v4 = 0; v4 < 4; ++v4) {
                    const float4 f = q4s[v4];
                    w[v4] = (uint32_t)f.x | ((uint32_t)f.y << 8) | ((uint32_t)f.z << 16) | ((uint32_t)f.w << 24);
                }
            }
            qb[u] = make_uint4(w[0], w[1], w[2], w[3]);
            qq = dot16(qb[u], qb[u], qq);
        }
        for (int64_t cb = rb; cb < re; cb += kRowChunk) {
            const int cn = stage(cb);
            rerank_rows_int<NT>(r, cid, cn, qb, qq, Gi, best);
        }
    } else {
        const int G = r.G, R = kWave / G, li = lane & (G - 1), slot = lane / G;
        const int d4 = r.d >> 2;
        float4 qr[UM];
        const float4 *q4 = reinterpret_cast<const float4 *>(r.Q + (int64_t)ql * r.d);
#pragma unroll
        for (int u = 0; u < UM; ++u) {
            const int j = li + G * u;
            qr[u] = (u < r.U && j < d4) ? q4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        for (int64_t cb = rb; cb < re; cb += kRowChunk) {
            const int cn = stage(cb);
            for (int base = wv * R * NRG; base < cn; base += (NT / kWave) * R * NRG) {
                uint32_t id[NRG];
                bool valid[NRG];
                float4 x[NRG][UM];
                uint32_t x8[NRG][UM];
#pragma unroll
                for (int g = 0; g < NRG; ++g) {
                    const int rw = base + g * R + slot;
                    id[g] = rw < cn ? cid[rw] : 0u;
                    valid[g] = rw < cn && id[g] < r.n;   // ids outside [0, n) are ignored
                    id[g] = valid[g] ? id[g] : 0u;
                }
#pragma unroll
                for (int g = 0; g < NRG; ++g) {
#pragma unroll
                    for (int u = 0; u < UM; ++u) {
                        const int j = li + G * u;
                        const bool in = u < r.U && j < d4;
                        if constexpr (ROWS8) {
                            x8[g][u] = in ? reinterpret_cast<const uint32_t *>(r.X8 + (int64_t)id[g] * r.d)[j] : 0u;
                        } else {
                            x[g][u] = in ? reinterpret_cast<const float4 *>(r.X + (int64_t)id[g] * r.d)[j]
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
                        }
                    }
                }
                uint64_t key[NRG];
#pragma unroll
                for (int g = 0; g < NRG; ++g) {
                    float acc = 0.f;
#pragma unroll
                    for (int u = 0; u < UM; ++u) {
                        const int j = li + G * u;
                        if (u < r.U && j < d4) {
                            float4 xv;
                            if constexpr (ROWS8) {
                                const uint32_t b = x8[g][u];
                                xv = make_float4((float)(b & 0xffu), (float)((b >> 8) & 0xffu), (float)((b >> 16) & 0xffu),
                                                 (float)(b >> 24));
                            } else {
                                xv = x[g][u];
                            }
                            acc = dist_acc(acc, xv.x - qr[u].x, r.metric);
                            acc = dist_acc(acc, xv.y - qr[u].y, r.metric);
                            acc = dist_acc(acc, xv.z - qr[u].z, r.metric);
                            acc = dist_acc(acc, xv.w - qr[u].w, r.metric);
                        }
                    }
                    for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
                    key[g] = valid[g] ? (((uint64_t)__float_as_uint(acc) << 32) | id[g]) : ~0ull;
                }
#pragma unroll
                for (int g = 0; g < NRG; ++g) {
                    const uint64_t kth = shfl64(best, k - 1);   // every lane takes part in the shuffle
                    uint64_t m = __ballot(li == 0 && key[g] < kth);
                    while (m != 0ull) {
                        const int src = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1ull;
                        topk_insert(best, shfl64(key[g], src), k, lane);
                    }
                }
            }
        }
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

template <int NT, bool ROWS8, int UM>
__global__ __launch_bounds__(NT) void k_rerank(RerankPass r) {
    const int items = pass_nq(r.nq_dev, r.q_base, r.nq) * r.parts;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        rerank_item<NT, ROWS8, UM>(r, item);
        __syncthreads();
    }
}

// One wave per query: merge the parts' lists, write ids and distances.
__device__ __forceinline__ void merge_item(const RerankPass &r, const int ql) {
    const int lane = threadIdx.x, k = r.k;
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
        // Euclidean distance: FP64 square root of the FP32 squared distance, rounded
        // once; Manhattan distance (SuCo-L1): the FP32 sum itself
        const float v = __uint_as_float((uint32_t)(best >> 32));
        r.dists[(int64_t)ql * k + lane] = r.metric ? v : (float)sqrt((double)v);
    }
}

__global__ __launch_bounds__(kWave) void k_merge(RerankPass r) {
    const int items = pass_nq(r.nq_dev, r.q_base, r.nq);
    for (int item = blockIdx.x; item < items; item += gridDim.x) merge_item(r, item);
}

// ======================================================== byte rows ==
// Flags (as 1) any coordinate that is not an integer in 0..255.
__global__ __launch_bounds__(256) void k_check_bytes(const float *X, int64_t m, int *bad) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int mine = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const float x = X[t];
        mine |= !(x >= 0.f && x <= 255.f && x == rintf(x));
    }
    if (mine) any = 1;
    __syncthreads();
    if (threadIdx.x == 0 && any) atomicOr(bad, 1);
}

__global__ __launch_bounds__(256) void k_to_bytes(const float *X, int64_t m, uint8_t *X8) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
        X8[t] = (uint8_t)X[t];
}

hipError_t launch_check_bytes(const float *X, int64_t m, int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_check_bytes, dim3(2048), dim3(256), 0, s, X, m, bad);
    return hipGetLastError();
}

hipError_t launch_to_bytes(const float *X, int64_t m, uint8_t *X8, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bytes, dim3(2048), dim3(256), 0, s, X, m, X8);
    return hipGetLastError();
}

// ============================================================= launchers ==
// A plan names the kernel, its launch shape and dynamic LDS.  `cap` > 0 limits
// the grid (the kernels stride over their items); 0 launches one block per item
// of a full pass.
namespace {
unsigned grid_for(int64_t items, int cap) {
    if (items < 1) items = 1;
    return (unsigned)(cap > 0 && cap < items ? cap : items);
}
}  // namespace

Launch plan_activate(const QueryPass &p, int cap) {
    Launch L;
    L.lds = sizeof(uint32_t) * (size_t)p.ix.sk * (p.ix.sk + 1);
    L.grid = dim3(grid_for((int64_t)p.nq * p.ix.ns, cap));
    if (p.ix.sk <= 64) { L.func = reinterpret_cast<const void *>(&k_activate<64>); L.block = dim3(64); }
    else { L.func = reinterpret_cast<const void *>(&k_activate<128>); L.block = dim3(128); }
    return L;
}

// With the sparse step on, the tiled steps take only the queries it leaves,
// counted on the device: their grids are capped at this many blocks, which
// stride over the listed queries (few or none in the common case, where a
// grid sized for every query's tile groups would spend its time dispatching
// idle blocks; all of them when every query has too many activated points).
constexpr int kTiledGrid = 8192;

Launch plan_collide(const QueryPass &p, int cap) {
    Launch L;
    L.lds = (size_t)p.ix.TILE;
    if (p.tlist != nullptr && cap == 0) cap = kTiledGrid;
    const int64_t items = (int64_t)p.nq * p.tgroups;
    L.grid = dim3(grid_for(items, cap));
    L.block = dim3(512);
    L.func = reinterpret_cast<const void *>(&k_collide<512>);
    return L;
}

Launch plan_collide_sparse(const QueryPass &p, int cap) {
    Launch L;
    const int sb = sp_score_bits(p.ix.ns);
    L.lds = sp_lds_bytes(p.ix.NB, p.sp_cap, sb);
    L.grid = dim3(grid_for(p.nq, cap));
    L.block = dim3(kSpThreads);
    L.func = sb == 4 ? reinterpret_cast<const void *>(&k_collide_sparse<4>)
                     : reinterpret_cast<const void *>(&k_collide_sparse<5>);
    return L;
}

Launch plan_cell_points(const SizesPass &p) {
    Launch L;
    L.grid = dim3((unsigned)std::max(1, p.nq * p.ix.ns));
    L.block = dim3(kWave);
    L.func = reinterpret_cast<const void *>(&k_cell_points);
    return L;
}

Launch plan_order(const QueryPass &p) {
    Launch L;
    L.func = p.nq <= kOrderMax ? reinterpret_cast<const void *>(&k_order)
                               : reinterpret_cast<const void *>(&k_order_wide);
    L.grid = dim3(1);
    L.block = dim3(1024);
    return L;
}

// Two waves per selection block: more blocks fit a CU than with four (each
// wave brings TILE/8 bytes of bitmap), and that measured faster.
constexpr int kSelectThreads = 128;

Launch plan_select(const QueryPass &p, int cap) {
    Launch L;
    if (p.tlist != nullptr && cap == 0) cap = kTiledGrid;
    L.lds = (size_t)(kSelectThreads / kWave) * (p.ix.TILE / 8);
    L.grid = dim3(grid_for(p.nq, cap));
    L.block = dim3(kSelectThreads);
    L.func = reinterpret_cast<const void *>(&k_select<kSelectThreads>);
    return L;
}

Launch plan_rerank(const RerankPass &r, int cap) {
    Launch L;
    L.lds = 0;
    L.grid = dim3(grid_for((int64_t)r.nq * r.parts, cap));
    L.block = dim3(256);
    // the smallest slice bound that holds U (U <= kMaxU = 8)
    const int um = r.U <= 2 ? 2 : (r.U <= 4 ? 4 : 8);
    if (r.X8) L.func = um == 2 ? reinterpret_cast<const void *>(&k_rerank<256, true, 2>)
                     : um == 4 ? reinterpret_cast<const void *>(&k_rerank<256, true, 4>)
                               : reinterpret_cast<const void *>(&k_rerank<256, true, 8>);
    else L.func = um == 2 ? reinterpret_cast<const void *>(&k_rerank<256, false, 2>)
                : um == 4 ? reinterpret_cast<const void *>(&k_rerank<256, false, 4>)
                          : reinterpret_cast<const void *>(&k_rerank<256, false, 8>);
    return L;
}

Launch plan_merge(const RerankPass &r, int cap) {
    Launch L;
    L.lds = 0;
    L.grid = dim3(grid_for(r.nq, cap));
    L.block = dim3(kWave);
    L.func = reinterpret_cast<const void *>(&k_merge);
    return L;
}

hipError_t launch(const Launch &L, void *arg, hipStream_t s) {
    void *args[] = {arg};
    return hipLaunchKernel(L.func, L.grid, L.block, args, L.lds, s);
}

int sparse_static_lds() {
    hipFuncAttributes at{};
    hipFuncAttributes at5{};
    if (hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_collide_sparse<4>)) != hipSuccess ||
        hipFuncGetAttributes(&at5, reinterpret_cast<const void *>(&k_collide_sparse<5>)) != hipSuccess)
        return -1;
    return (int)std::max(at.sharedSizeBytes, at5.sharedSizeBytes);
}

int collide_static_lds() {
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_collide<512>)) != hipSuccess) return -1;
    return (int)at.sharedSizeBytes;
}

hipError_t launch_activate(const QueryPass &p, hipStream_t s) {
    QueryPass c = p;
    return launch(plan_activate(p, kActivateGrid), &c, s);
}

hipError_t launch_collide(const QueryPass &p, hipStream_t s) {
    QueryPass c = p;
    return launch(plan_collide(p, 0), &c, s);
}

hipError_t launch_select(const QueryPass &p, hipStream_t s) {
    QueryPass c = p;
    return launch(plan_select(p, 0), &c, s);
}

hipError_t launch_rerank(const RerankPass &r, hipStream_t s) {
    RerankPass c = r;
    return launch(plan_rerank(r, 0), &c, s);
}

hipError_t launch_merge(const RerankPass &r, hipStream_t s) {
    RerankPass c = r;
    return launch(plan_merge(r, 0), &c, s);
}

}  // namespace suco
