// gfx950 kernels that build the SuCo index (Create Index, Alg. 2):
// Lloyd's k-means on every subspace half with FP64 arithmetic, and the
// inverted multi-index stored tile-major for the collision step.
//
// k-means iteration, all 2*ns halves in one launch each (grid.y = half):
//   assign   nearest centre per point in FP64 (ties -> lowest centre id) and
//            a per-block histogram of the labels
//   scan     per label, exclusive prefix of the block histograms over blocks;
//            label starts over labels
//   scatter  stable placement of every point id into its label's range, so
//            each label's members are listed in ascending id
//   update   one thread per (centre, dimension) sums its members' values in
//            ascending id order in FP64 and divides by the count; an empty
//            label keeps its centre
// Summing each centre's members one after another in id order, with no
// contraction into FMA, is the same arithmetic as a sequential CPU loop.
#include <hip/hip_runtime.h>

#include "suco_impl.h"

namespace suco {

__global__ void k_gather_rows(const float *X, int d, const int64_t *ids, int m, int dim0, int w,
                              float *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * w) return;
    const int r = t / w, j = t - r * w;
    out[t] = X[ids[r] * d + dim0 + j];
}

// One point per thread.  WMAX > 0: the point's half is held in registers.
template <int WMAX>
__global__ __launch_bounds__(256) void k_km_assign(KmeansPass k, int with_hist) {
#pragma clang fp contract(off)
    extern __shared__ double cs[];            // [sk][w] centres of this half (WMAX > 0)
    __shared__ uint32_t hcnt[kMaxSqrtK];
    const int g = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const HalfDims hd = k.halves[g];
    const int w = hd.w, sk = k.sk;
    const double *cg = k.cent64 + (int64_t)sk * hd.dim0;
    if constexpr (WMAX > 0)
        for (int e = t; e < sk * w; e += 256) cs[e] = cg[e];
    if (with_hist)
        for (int c = t; c < sk; c += 256) hcnt[c] = 0u;
    __syncthreads();
    const int64_t p = (int64_t)b * 256 + t;
    if (p < k.n) {
        const float *xp = k.X + p * k.d + hd.dim0;
        int best = 0;
        double bd = 0.0;
        if constexpr (WMAX > 0) {
            double x[WMAX];
#pragma unroll
            for (int j = 0; j < WMAX; ++j) x[j] = j < w ? (double)xp[j] : 0.0;
            for (int c = 0; c < sk; ++c) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < WMAX; ++j) {
                    if (j < w) {
                        const double dd = x[j] - cs[c * w + j];
                        s = s + dd * dd;
                    }
                }
                if (c == 0 || s < bd) { bd = s; best = c; }
            }
        } else {
            for (int c = 0; c < sk; ++c) {
                double s = 0.0;
                for (int j = 0; j < w; ++j) {
                    const double dd = (double)xp[j] - cg[c * w + j];
                    s = s + dd * dd;
                }
                if (c == 0 || s < bd) { bd = s; best = c; }
            }
        }
        k.assign[(int64_t)g * k.n + p] = (uint8_t)best;
        if (with_hist) atomicAdd(&hcnt[best], 1u);
    }
    if (with_hist) {
        __syncthreads();
        uint32_t *bh = k.bh + ((int64_t)g * k.nb + b) * sk;
        for (int c = t; c < sk; c += 256) bh[c] = hcnt[c];
    }
}

// grid = 2*ns, block = 128 (>= sk)
__global__ __launch_bounds__(128) void k_km_scan(KmeansPass k) {
    __shared__ uint32_t tot[kMaxSqrtK];
    const int g = blockIdx.x, c = threadIdx.x, sk = k.sk;
    if (c < sk) {
        uint32_t run = 0;
        uint32_t *bh = k.bh + (int64_t)g * k.nb * sk + c;
        for (int b = 0; b < k.nb; ++b) {
            const uint32_t v = bh[(int64_t)b * sk];
            bh[(int64_t)b * sk] = run;
            run += v;
        }
        tot[c] = run;
    }
    __syncthreads();
    if (c == 0) {
        uint32_t *cb = k.cbase + (int64_t)g * (sk + 1);
        uint32_t run = 0;
        for (int j = 0; j < sk; ++j) {
            cb[j] = run;
            run += tot[j];
        }
        cb[sk] = run;
    }
}

__global__ __launch_bounds__(256) void k_km_scatter(KmeansPass k) {
    __shared__ uint32_t wc[4][kMaxSqrtK];
    const int g = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const int lane = t & (kWave - 1), wv = t / kWave, sk = k.sk;
    for (int e = t; e < 4 * kMaxSqrtK; e += 256) (&wc[0][0])[e] = 0u;
    __syncthreads();
    const int64_t p = (int64_t)b * 256 + t;
    const bool valid = p < k.n;
    const uint32_t key = valid ? k.assign[(int64_t)g * k.n + p] : 0u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const bool on = (key >> bit) & 1u;
        const uint64_t bal = __ballot(on);
        m &= on ? bal : ~bal;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t rank = (uint32_t)__popcll(m & lt), cnt = (uint32_t)__popcll(m);
    if (valid && rank == cnt - 1) wc[wv][key] = cnt;
    __syncthreads();
    if (valid) {
        uint32_t before = 0;
        for (int w2 = 0; w2 < wv; ++w2) before += wc[w2][key];
        const uint32_t pos = k.cbase[(int64_t)g * (sk + 1) + key] +
                             k.bh[((int64_t)g * k.nb + b) * sk + key] + before + rank;
        k.order[(int64_t)g * k.n + pos] = (uint32_t)p;
    }
}

__global__ __launch_bounds__(256) void k_km_update(KmeansPass k) {
#pragma clang fp contract(off)
    const int g = blockIdx.y;
    const HalfDims hd = k.halves[g];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= k.sk * hd.w) return;
    const int c = t / hd.w, j = t - c * hd.w;
    const uint32_t *cb = k.cbase + (int64_t)g * (k.sk + 1);
    const uint32_t s0 = cb[c], s1 = cb[c + 1];
    if (s1 == s0) return;
    const uint32_t *ord = k.order + (int64_t)g * k.n;
    const float *xc = k.X + hd.dim0 + j;
    double s = 0.0;
#pragma unroll 8
    for (uint32_t m = s0; m < s1; ++m) s = s + (double)xc[(int64_t)ord[m] * k.d];
    k.cent64[(int64_t)k.sk * hd.dim0 + t] = s / (double)(s1 - s0);
}

__global__ void k_cent_to_f32(const double *c64, float *c32, int64_t m) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) c32[t] = (float)c64[t];
}

// One wave per (tile, subspace): counting sort of the tile's ids by cell,
// stable (ids ascending inside each cell), written tile-major.
__global__ __launch_bounds__(64) void k_imi_build(const uint8_t *assign, int64_t n, int sk, int P, int TILE,
                                                   uint32_t *toffs, uint16_t *ids16, uint32_t *csize) {
    extern __shared__ uint32_t cur[];          // [K]
    const int p = blockIdx.x, i = blockIdx.y, lane = threadIdx.x, K = sk * sk;
    const int64_t t0 = (int64_t)p * TILE;
    const int valid = (int)(n - t0 < TILE ? n - t0 : TILE);
    const uint8_t *a1 = assign + (int64_t)(2 * i) * n + t0;
    const uint8_t *a2 = assign + (int64_t)(2 * i + 1) * n + t0;
    for (int c = lane; c < K; c += kWave) cur[c] = 0u;
    __syncthreads();
    for (int m = lane; m < valid; m += kWave) atomicAdd(&cur[a1[m] * sk + a2[m]], 1u);
    __syncthreads();
    for (int c = lane; c < K; c += kWave)
        if (cur[c]) atomicAdd(&csize[(int64_t)i * K + c], cur[c]);
    // exclusive scan of the counts: lane owns a contiguous block of cells
    const int per = (K + kWave - 1) / kWave;
    const int c0 = lane * per < K ? lane * per : K, c1 = c0 + per < K ? c0 + per : K;
    uint32_t local = 0;
    for (int c = c0; c < c1; ++c) local += cur[c];
    uint32_t x = local;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    uint32_t off = x - local;
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
        const uint32_t v = cur[c];
        cur[c] = off;
        off += v;
    }
    __syncthreads();
    uint32_t *to = toffs + ((int64_t)i * P + p) * (K + 1);
    for (int c = lane; c < K; c += kWave) to[c] = (uint32_t)t0 + cur[c];
    if (lane == 0) to[K] = (uint32_t)(t0 + valid);
    int nbits = 0;
    while ((1 << nbits) < K) ++nbits;
    uint16_t *dst = ids16 + (int64_t)i * P * TILE + t0;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    __syncthreads();
    for (int m0 = 0; m0 < valid; m0 += kWave) {
        const int m = m0 + lane;
        const bool v = m < valid;
        const uint32_t key = v ? (uint32_t)(a1[m] * sk + a2[m]) : 0u;
        uint64_t mk = __ballot(v);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (key >> bit) & 1u;
            const uint64_t bal = __ballot(on);
            mk &= on ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(mk & lt), cnt = (uint32_t)__popcll(mk);
        uint32_t base = v ? cur[key] : 0u;
        if (v) dst[base + rank] = (uint16_t)m;
        __syncthreads();
        if (v && rank == cnt - 1) cur[key] = base + cnt;
        __syncthreads();
    }
}

// Cell-major copy of the IMI for the sparse collision step: the ids of cell c
// of subspace i, ascending, at ids32[i*n + coffs[i*(K+1) + c] ...].  The
// tile-major runs of a cell are concatenated in tile order (tiles hold
// consecutive id ranges, each run ascending), one wave per (cell, subspace).
__global__ __launch_bounds__(64) void k_cell_major(const uint32_t *toffs, const uint16_t *ids16,
                                                    const uint32_t *csize, int64_t n, int K, int P, int TILE,
                                                    uint32_t *coffs, uint32_t *ids32) {
    const int c = blockIdx.x, i = blockIdx.y, lane = threadIdx.x;
    // start of cell c: the sizes of the cells before it (lanes sum strided parts)
    uint32_t part = 0;
    for (int c2 = lane; c2 < c; c2 += kWave) part += csize[(int64_t)i * K + c2];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
    uint32_t at = part;
    if (lane == 0) {
        coffs[(int64_t)i * (K + 1) + c] = at;
        if (c == K - 1) coffs[(int64_t)i * (K + 1) + K] = at + csize[(int64_t)i * K + c];
    }
    uint32_t *dst = ids32 + (int64_t)i * n;
    for (int p = 0; p < P; ++p) {
        const uint32_t *to = toffs + ((int64_t)i * P + p) * (K + 1);
        const uint32_t s = to[c], e = to[c + 1];
        const uint16_t *src = ids16 + (int64_t)i * P * TILE;
        const uint32_t t0 = (uint32_t)p * (uint32_t)TILE;
        for (uint32_t m = s + lane; m < e; m += kWave) dst[at + (m - s)] = t0 + src[m];
        at += e - s;
    }
}

// ============================================================= launchers ==
hipError_t launch_gather_rows(const float *X, int d, const int64_t *ids, int m, int dim0, int w,
                              float *out, hipStream_t s) {
    const int tot = m * w;
    hipLaunchKernelGGL(k_gather_rows, dim3((tot + 255) / 256), dim3(256), 0, s, X, d, ids, m, dim0, w, out);
    return hipGetLastError();
}

hipError_t launch_km_assign(const KmeansPass &k, bool with_hist, hipStream_t s) {
    const dim3 grid((unsigned)k.nb, (unsigned)(2 * k.ns));
    if (k.wmax <= 8)
        hipLaunchKernelGGL(k_km_assign<8>, grid, dim3(256), sizeof(double) * k.sk * 8, s, k, (int)with_hist);
    else if (k.wmax <= 32)
        hipLaunchKernelGGL(k_km_assign<32>, grid, dim3(256), sizeof(double) * k.sk * 32, s, k, (int)with_hist);
    else
        hipLaunchKernelGGL(k_km_assign<0>, grid, dim3(256), 0, s, k, (int)with_hist);
    return hipGetLastError();
}

hipError_t launch_km_scan(const KmeansPass &k, hipStream_t s) {
    hipLaunchKernelGGL(k_km_scan, dim3((unsigned)(2 * k.ns)), dim3(128), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_km_scatter(const KmeansPass &k, hipStream_t s) {
    hipLaunchKernelGGL(k_km_scatter, dim3((unsigned)k.nb, (unsigned)(2 * k.ns)), dim3(256), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_km_update(const KmeansPass &k, hipStream_t s) {
    const unsigned bx = (unsigned)((k.sk * k.wmax + 255) / 256);
    hipLaunchKernelGGL(k_km_update, dim3(bx, (unsigned)(2 * k.ns)), dim3(256), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_cent_to_f32(const double *c64, float *c32, int64_t m, hipStream_t s) {
    hipLaunchKernelGGL(k_cent_to_f32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, c64, c32, m);
    return hipGetLastError();
}

hipError_t launch_cell_major(const uint32_t *toffs, const uint16_t *ids16, const uint32_t *csize, int64_t n,
                             int ns, int K, int P, int TILE, uint32_t *coffs, uint32_t *ids32, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_major, dim3((unsigned)K, (unsigned)ns), dim3(kWave), 0, s, toffs, ids16, csize, n, K, P,
                       TILE, coffs, ids32);
    return hipGetLastError();
}

hipError_t launch_imi_build(const uint8_t *assign, int64_t n, int ns, int sk, int P, int TILE,
                            uint32_t *toffs, uint16_t *ids16, uint32_t *csize, hipStream_t s) {
    const size_t lds = sizeof(uint32_t) * (size_t)sk * sk;
    hipLaunchKernelGGL(k_imi_build, dim3((unsigned)P, (unsigned)ns), dim3(kWave), lds, s, assign, n, sk, P, TILE,
                       toffs, ids16, csize);
    return hipGetLastError();
}

}  // namespace suco
