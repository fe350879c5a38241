// gfx950 kernels that build the SuCo index (Create Index, Alg. 2):
// Lloyd's k-means on every subspace half with FP64 arithmetic, and the
// inverted multi-index stored tile-major for the collision step.
//
// k-means iteration, all 2*ns halves in one launch each (grid.y = half):
//   assign   nearest centre per point in FP64 (ties -> lowest centre id) and
//            a per-block histogram of the labels
//   scan     per (label, half) block, exclusive prefix of the block
//            histograms over blocks; then label starts over labels
//   scatter  stable placement of every point id into its label's range, so
//            each label's members are listed in ascending id
//   update   one block per (centre, half) sums its members' values in FP64,
//            ascending id in groups of 256 (each group in order, then the
//            group sums in order), and divides by the count; an empty label
//            keeps its centre
//   median   (k-medians, SuCo-L1) one block per (centre, half) replaces each
//            coordinate by the lower median of its members' values
// With SuCo-L1 the assignment takes the nearest centre by L1 instead.
// Summing each group of a centre's members one after another in id order,
// with no contraction into FMA, then the group sums in order, is the same
// arithmetic as the sequential CPU loop that keeps a running group sum.
#include <hip/hip_runtime.h>

#include <vector>

#include "suco_impl.h"
#include "wave.h"

namespace suco {

__global__ void k_gather_rows(const float *X, int d, const int64_t *ids, int m, int dim0, int w,
                              float *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * w) return;
    const int r = t / w, j = t - r * w;
    out[t] = X[ids[r] * d + dim0 + j];
}

// One point per thread, the halves listed in k.hsel (grid.y), all of width W
// (W = 0: any width, read from the half).  With a fixed width the point's half
// is loaded at once into registers and the centres, the same for the whole
// block, are read through the scalar cache (uniform loads the compiler keeps in
// SGPRs, operands of the FP64 arithmetic as they are): three FP64 operations
// per dimension and centre (squared L2) or two (L1), no branches, no LDS.
template <int W, int METRIC>
__device__ __forceinline__ double half_dist64(const double *x, const double *__restrict__ c) {
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const double dd = x[j] - c[j];
        s = s + (METRIC ? fabs(dd) : dd * dd);
    }
    return s;
}

template <int W, int METRIC>
__global__ __launch_bounds__(256) void k_km_assign(KmeansPass k, int with_hist) {
#pragma clang fp contract(off)
    __shared__ uint32_t hcnt[kMaxSqrtK];
    const int g = k.hsel[blockIdx.y], b = blockIdx.x, t = threadIdx.x;
    const HalfDims hd = k.halves[g];
    const int w = hd.w, sk = k.sk;
    const double *__restrict__ cg = k.cent64 + (int64_t)sk * hd.dim0;
    if (with_hist)
        for (int c = t; c < sk; c += 256) hcnt[c] = 0u;
    __syncthreads();
    const int64_t p = (int64_t)b * 256 + t;
    if (p < k.n) {
        const float *xp = k.X + p * k.d + hd.dim0;
        int best = 0;
        double bd = 0.0;
        if constexpr (W > 0) {
            double x[W];
#pragma unroll
            for (int j = 0; j < W; ++j) x[j] = (double)xp[j];
            bd = half_dist64<W, METRIC>(x, cg);
            for (int c = 1; c < sk; ++c) {
                const double s = half_dist64<W, METRIC>(x, cg + c * W);
                if (s < bd) { bd = s; best = c; }        // ties keep the lower centre id
            }
        } else {
            for (int c = 0; c < sk; ++c) {
                double s = 0.0;
                for (int j = 0; j < w; ++j) {
                    const double dd = (double)xp[j] - cg[c * w + j];
                    s = s + (METRIC ? fabs(dd) : dd * dd);
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

// One block per (label, half): the label's block counts become exclusive
// offsets over the blocks (a block-wide scan per 256 blocks), and the
// label's total goes to cbase[label + 1].
__global__ __launch_bounds__(256) void k_km_scan(KmeansPass k) {
    __shared__ uint32_t red[256 / kWave + 1];
    const int c = blockIdx.x, g = blockIdx.y, t = threadIdx.x, sk = k.sk;
    uint32_t *bh = k.bh + (int64_t)g * k.nb * sk + c;
    uint32_t run = 0;
    for (int b0 = 0; b0 < k.nb; b0 += 256) {
        const int b = b0 + t;
        const uint32_t v = b < k.nb ? bh[(int64_t)b * sk] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<256>(v, red, &tot);
        if (b < k.nb) bh[(int64_t)b * sk] = run + ex;
        run += tot;
    }
    if (t == 0) k.cbase[(int64_t)g * (sk + 1) + c + 1] = run;
}

// One thread per half: label totals into label starts.
__global__ void k_km_bases(KmeansPass k) {
    const int g = blockIdx.x;
    uint32_t *cb = k.cbase + (int64_t)g * (k.sk + 1);
    uint32_t run = 0;
    cb[0] = 0u;
    for (int j = 0; j < k.sk; ++j) {
        run += cb[j + 1];
        cb[j + 1] = run;
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

// One block per (centre, half): the centre becomes the FP64 mean of its
// members (ascending id), summed group by group: thread t sums the groups t,
// t + 256, ... of kSumGroup consecutive members, each in order from zero, for
// up to 8 dimensions at a time, and the group sums are then added in group
// order; an empty label keeps its centre.
constexpr int kSumGroup = 256;
__global__ __launch_bounds__(256) void k_km_update(KmeansPass k) {
#pragma clang fp contract(off)
    __shared__ double part[256][8];
    const int c = blockIdx.x, g = blockIdx.y, t = threadIdx.x;
    const HalfDims hd = k.halves[g];
    const uint32_t *cb = k.cbase + (int64_t)g * (k.sk + 1);
    const uint32_t s0 = cb[c], s1 = cb[c + 1];
    if (s1 == s0) return;
    const uint32_t m = s1 - s0, ngroups = (m + kSumGroup - 1) / kSumGroup;
    const uint32_t *ord = k.order + (int64_t)g * k.n + s0;
    double *cent = k.cent64 + (int64_t)k.sk * hd.dim0 + (int64_t)c * hd.w;
    for (int j0 = 0; j0 < hd.w; j0 += 8) {
        const int nj = hd.w - j0 < 8 ? hd.w - j0 : 8;
        double tot = 0.0;                                   // dimension j0 + t, threads t < nj
        for (uint32_t g0 = 0; g0 < ngroups; g0 += 256) {
            const uint32_t gi = g0 + (uint32_t)t;
            double acc[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = 0.0;
            if (gi < ngroups) {
                const uint32_t r0 = gi * kSumGroup, r1 = r0 + kSumGroup < m ? r0 + kSumGroup : m;
#pragma unroll 4
                for (uint32_t r = r0; r < r1; ++r) {
                    const float *xr = k.X + (int64_t)ord[r] * k.d + hd.dim0 + j0;
                    // eight loads issued together (indices past the half repeat its last
                    // dimension, so no load is conditional), then the additions
                    float v[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) v[j] = xr[j < nj ? j : nj - 1];
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (j < nj) acc[j] = acc[j] + (double)v[j];
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) part[t][j] = acc[j];
            __syncthreads();
            if (t < nj) {
                const uint32_t ng = ngroups - g0 < 256u ? ngroups - g0 : 256u;
                for (uint32_t u = 0; u < ng; ++u) tot = tot + part[u][t];
            }
            __syncthreads();
        }
        if (t < nj) cent[j0 + t] = tot / (double)m;
    }
}

__global__ void k_cent_to_f32(const double *c64, float *c32, int64_t m) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) c32[t] = (float)c64[t];
}

// Order-preserving bit patterns of floats: unsigned comparison of the keys
// is the comparison of the values (-0 below +0).
__device__ __forceinline__ uint32_t float_key(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// One block per (centre, half).  Each coordinate of the centre becomes the
// lower median of its m members' values, the ceil(m/2)-th smallest, found by
// a radix select over the values' keys, 8 bits a pass from the top, for up to
// kMedDims coordinates at a time (a histogram of the next digit among the
// members whose key matches the prefix found so far); an empty cluster keeps
// its centre.  The members are read in the label order the scatter produced.
constexpr int kMedDims = 16;
__global__ __launch_bounds__(256) void k_km_median(KmeansPass k) {
    __shared__ uint32_t hist[kMedDims][256];
    __shared__ uint32_t pre[kMedDims], rank[kMedDims];
    const int c = blockIdx.x, g = blockIdx.y, t = threadIdx.x;
    const HalfDims hd = k.halves[g];
    const uint32_t *cb = k.cbase + (int64_t)g * (k.sk + 1);
    const uint32_t s0 = cb[c], s1 = cb[c + 1];
    if (s1 == s0) return;
    const uint32_t m = s1 - s0;
    const uint32_t *ord = k.order + (int64_t)g * k.n + s0;
    for (int j0 = 0; j0 < hd.w; j0 += kMedDims) {
        const int nj = hd.w - j0 < kMedDims ? hd.w - j0 : kMedDims;
        if (t < kMedDims) { pre[t] = 0u; rank[t] = (m + 1) / 2; }      // 1-based rank of the lower median
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (int e = t; e < kMedDims * 256; e += 256) (&hist[0][0])[e] = 0u;
            __syncthreads();
            const uint32_t hmask = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
            for (uint32_t r = t; r < m; r += 256) {
                const float *xr = k.X + (int64_t)ord[r] * k.d + hd.dim0 + j0;
                float v[kMedDims];
#pragma unroll
                for (int j = 0; j < kMedDims; ++j) v[j] = xr[j < nj ? j : nj - 1];    // unconditional loads
#pragma unroll
                for (int j = 0; j < kMedDims; ++j) {
                    const uint32_t key = float_key(v[j]);
                    if (j < nj && (key & hmask) == (pre[j] & hmask)) atomicAdd(&hist[j][(key >> shift) & 255u], 1u);
                }
            }
            __syncthreads();
            if (t < nj) {
                uint32_t run = 0;
                const uint32_t rk = rank[t];
                int b = 0;
                for (; b < 255; ++b) {
                    const uint32_t h = hist[t][b];
                    if (run + h >= rk) break;
                    run += h;
                }
                pre[t] |= (uint32_t)b << shift;
                rank[t] = rk - run;
            }
            __syncthreads();
        }
        if (t < nj) k.cent64[(int64_t)k.sk * hd.dim0 + (int64_t)c * hd.w + j0 + t] = (double)key_float(pre[t]);
        __syncthreads();
    }
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

template <int METRIC>
hipError_t launch_assign_width(const KmeansPass &k, int w, int nsel, bool with_hist, hipStream_t s) {
    const dim3 grid((unsigned)k.nb, (unsigned)nsel);
    const int h = (int)with_hist;
    switch (w) {
    case 4: hipLaunchKernelGGL((k_km_assign<4, METRIC>), grid, dim3(256), 0, s, k, h); break;
    case 6: hipLaunchKernelGGL((k_km_assign<6, METRIC>), grid, dim3(256), 0, s, k, h); break;
    case 8: hipLaunchKernelGGL((k_km_assign<8, METRIC>), grid, dim3(256), 0, s, k, h); break;
    case 12: hipLaunchKernelGGL((k_km_assign<12, METRIC>), grid, dim3(256), 0, s, k, h); break;
    case 16: hipLaunchKernelGGL((k_km_assign<16, METRIC>), grid, dim3(256), 0, s, k, h); break;
    case 24: hipLaunchKernelGGL((k_km_assign<24, METRIC>), grid, dim3(256), 0, s, k, h); break;
    case 32: hipLaunchKernelGGL((k_km_assign<32, METRIC>), grid, dim3(256), 0, s, k, h); break;
    default: hipLaunchKernelGGL((k_km_assign<0, METRIC>), grid, dim3(256), 0, s, k, h); break;
    }
    return hipGetLastError();
}

// One launch per distinct half width (the halves of that width in hsel).
hipError_t launch_km_assign(const KmeansPass &k0, const HalfDims *halves_h, bool with_hist, hipStream_t s) {
    const int nh = 2 * k0.ns;
    std::vector<bool> done(nh, false);
    for (int g0 = 0; g0 < nh; ++g0) {
        if (done[g0]) continue;
        KmeansPass k = k0;
        const int w = halves_h[g0].w;
        int nsel = 0;
        for (int g = g0; g < nh; ++g)
            if (!done[g] && halves_h[g].w == w) { k.hsel[nsel++] = (int16_t)g; done[g] = true; }
        const hipError_t e = k.metric ? launch_assign_width<1>(k, w, nsel, with_hist, s)
                                      : launch_assign_width<0>(k, w, nsel, with_hist, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_km_scan(const KmeansPass &k, hipStream_t s) {
    hipLaunchKernelGGL(k_km_scan, dim3((unsigned)k.sk, (unsigned)(2 * k.ns)), dim3(256), 0, s, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_km_bases, dim3((unsigned)(2 * k.ns)), dim3(1), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_km_scatter(const KmeansPass &k, hipStream_t s) {
    hipLaunchKernelGGL(k_km_scatter, dim3((unsigned)k.nb, (unsigned)(2 * k.ns)), dim3(256), 0, s, k);
    return hipGetLastError();
}

hipError_t launch_km_update(const KmeansPass &k, hipStream_t s) {
    hipLaunchKernelGGL(k_km_update, dim3((unsigned)k.sk, (unsigned)(2 * k.ns)), dim3(256), 0, s, k);
    return hipGetLastError();
}

// One block per (cell, subspace): how many of the cell's ids fall in each
// bucket of kSpBucket consecutive ids (LDS counters, then u16 counts; a
// bucket holds at most 4,096 ids), for the sparse collision step's exact
// bucket sizes.
__global__ __launch_bounds__(256) void k_cell_buckets(const uint32_t *coffs, const uint32_t *ids32, int64_t n,
                                                      int K, int NB, uint16_t *cbh) {
    extern __shared__ uint32_t cnt[];          // [NBp]
    const int c = blockIdx.x, i = blockIdx.y, NBp = sp_nb_padded(NB);
    for (int b = threadIdx.x; b < NBp; b += 256) cnt[b] = 0u;
    __syncthreads();
    const uint32_t *co = coffs + (int64_t)i * (K + 1);
    const uint32_t *ids = ids32 + (int64_t)i * n;
    for (uint32_t m = co[c] + threadIdx.x; m < co[c + 1]; m += 256) atomicAdd(&cnt[ids[m] >> kSpShift], 1u);
    __syncthreads();
    uint16_t *out = cbh + ((int64_t)i * K + c) * NBp;
    for (int b = threadIdx.x; b < NBp; b += 256) out[b] = (uint16_t)cnt[b];
}

hipError_t launch_cell_buckets(const uint32_t *coffs, const uint32_t *ids32, int64_t n, int ns, int K, int NB,
                               uint16_t *cbh, hipStream_t s) {
    const size_t lds = sizeof(uint32_t) * (size_t)sp_nb_padded(NB);
    hipLaunchKernelGGL(k_cell_buckets, dim3((unsigned)K, (unsigned)ns), dim3(256), lds, s, coffs, ids32, n, K, NB, cbh);
    return hipGetLastError();
}

hipError_t launch_km_median(const KmeansPass &k, hipStream_t s) {
    hipLaunchKernelGGL(k_km_median, dim3((unsigned)k.sk, (unsigned)(2 * k.ns)), dim3(256), 0, s, k);
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
