// BF16 split precision: the query path with BF16 arithmetic where it is safe.
//
// Centre distances (step 1) on the matrix cores.  For 16 queries and 16 centres
// of one subspace half, q.c comes from the 16x16x32 BF16 MFMA with FP32
// accumulation over the half's dimensions (zero-padded to a multiple of 16),
// and D = |q^|^2 + |c^|^2 - 2 q^.c^ (clamped at 0), where ^ is rounding to BF16.
//
// Re-rank (step 5) in two passes with a certified filter between them.
//  - First pass: every candidate row is read from a BF16 copy of X (half the
//    bytes of FP32) and d~ = sum_j (x^_j - q_j)^2 is accumulated in FP32 with
//    the query kept in FP32.  With eps(o) >= |x^ - x| stored per row at build,
//    the exact squared distances satisfy
//        |d~exact - dexact| <= 2 sqrt(d~exact) eps + eps^2,
//    and the FP32 sums of this pass and of the plain FP32 re-rank are each
//    within (d + 2) 2^-24 (relative) of their exact values.  Folding these
//    together gives e(o) such that every candidate's plain FP32 squared distance
//    D32(o) lies in [d~(o) - e(o), d~(o) + e(o)], d~ the computed first pass:
//        e0 = 2 (sqrt(d~) + eps) eps + eps^2,   e = e0 + (4d + 64) 2^-24 (d~ + e0)
//    (the 64 ulps absorb the rounding of computing e itself).
//  - Survivors: with U the k-th smallest d~ + e over the query's candidates, at
//    least k candidates have D32 <= U, so every member of the FP32 top-k has
//    D32 <= U and hence d~ - e <= U.  The survivors {d~ - e <= U} therefore hold
//    the plain path's top-k.
//  - Second pass: the plain FP32 re-rank on the survivors only; it returns the
//    plain path's top-k of the same candidates, bit for bit.
#include "runtime_impl.h"
#include "wave.h"

namespace suco {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Round to nearest even, FP32 -> BF16 bits (finite inputs; inf and nan kept).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_val(uint32_t b) { return __uint_as_float(b << 16); }

// Smallest float >= v (v >= 0).
__device__ __forceinline__ float float_up(double v) {
    float f = (float)v;
    if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

// ------------------------------------------------------------ build time --
// One wave per row: the BF16 copy of the row and an upper bound of the norm
// of its rounding error (FP64 sum of the exact per-coordinate errors).
__global__ __launch_bounds__(256) void k_bf16_rows(const float *X, int64_t n, int d, uint16_t *Xb, float *xerr) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; r < n; r += waves) {
        double s = 0.0;
        for (int j = lane; j < d; j += kWave) {
            const float x = X[r * d + j];
            const uint16_t b = bf16_bits(x);
            Xb[r * d + j] = b;
            const double t = (double)(bf16_val(b) - x);   // exact: both within a factor 2
            s += t * t;
        }
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
        if (lane == 0) xerr[r] = float_up(sqrt(s * (1.0 + 0x1p-40)));
    }
}

// BF16 centres (same layout as the FP32 ones) and their squared norms per half.
__global__ __launch_bounds__(256) void k_bf16_centres(const float *cent, const HalfDims *halves, int nh, int sk,
                                                     int d, uint16_t *centb, float *cnorm2) {
    const int64_t m = (int64_t)sk * d;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
        centb[t] = bf16_bits(cent[t]);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)nh * sk;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(t / sk), c = (int)(t - (int64_t)g * sk);
        const HalfDims hd = halves[g];
        const float *cp = cent + (int64_t)sk * hd.dim0 + (int64_t)c * hd.w;
        double s = 0.0;
        for (int j = 0; j < hd.w; ++j) {
            const double v = (double)bf16_val(bf16_bits(cp[j]));
            s += v * v;
        }
        cnorm2[t] = (float)s;
    }
}

// --------------------------------------------------- centre distances --
// Block (16 queries, one half); wave w takes centres 16w .. 16w+15, with
// gfx950's 16x16x32 BF16 MFMA: lane l supplies row l % 16 of A and column
// l % 16 of B, eight K positions each (the same eight for A and B: 8(l/16) ..
// 8(l/16)+7 of the step's 32), and receives D[4(l/16) .. +3][l % 16].
__global__ __launch_bounds__(512) void k_centre_dists_bf16(CentreBf16Pass p) {
    const int g = blockIdx.y, q0 = blockIdx.x * 16;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const HalfDims hd = p.halves[g];
    const int sk = p.sk, c0 = 16 * w;
    if (c0 >= sk || q0 >= p.nq) return;
    const int r = lane & 15, kq = 8 * (lane >> 4);
    const int qa = q0 + r, cb = c0 + r;
    const bool qok = qa < p.nq, cok = cb < sk;
    const float *qrow = p.Q + (int64_t)(qok ? qa : 0) * p.d + hd.dim0;
    const uint16_t *crow = p.centb + (int64_t)sk * hd.dim0 + (int64_t)(cok ? cb : 0) * hd.w;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    float qn = 0.f;   // this lane's part of |q^|^2 for query qa
    for (int k0 = 0; k0 < hd.w; k0 += 32) {
        bf16x8_t a, b;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int kk = k0 + kq + t;
            const bool in = kk < hd.w;
            const uint16_t qb = (in && qok) ? bf16_bits(qrow[kk]) : (uint16_t)0;
            const uint16_t cbits = (in && cok) ? crow[kk] : (uint16_t)0;
            a[t] = __builtin_bit_cast(__bf16, qb);
            b[t] = __builtin_bit_cast(__bf16, cbits);
            const float qv = bf16_val(qb);
            qn = fmaf(qv, qv, qn);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    // lanes r, r+16, r+32, r+48 hold the four k-slices of query q0 + r
    qn += __shfl_xor(qn, 16, kWave);
    qn += __shfl_xor(qn, 32, kWave);
    const int cj = c0 + (lane & 15);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int row = 4 * (lane >> 4) + t;
        const float qni = __shfl(qn, row, kWave);
        const int qi = q0 + row;
        if (qi < p.nq && cj < sk) {
            const float v = qni + p.cnorm2[(int64_t)g * sk + cj] - 2.0f * acc[t];
            p.D[((int64_t)qi * p.nh + g) * sk + cj] = v > 0.f ? v : 0.f;
        }
    }
}

// --------------------------------------------------- BF16 first pass --
// Block of 256 threads per (query, part of the candidate list), G lanes per
// row, each lane U slices of 8 BF16 values (16 bytes); keys are the upper
// bounds d~ + e (bits << 32 | id), kept per wave as in the FP32 re-rank.
__global__ __launch_bounds__(256) void k_rerank_bf16(Bf16RerankPass r) {
    __shared__ uint64_t wl[4][kMaxK];
    __shared__ uint32_t cid[kRowChunk];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int G = r.G, R = kWave / G, li = lane & (G - 1), slot = lane / G;
    const int d8 = r.d >> 3, k = r.k;
    const float gam = (float)(4 * r.d + 64) * 0x1p-24f;
    for (int item = blockIdx.x; item < r.nq * r.parts; item += gridDim.x) {
        const int ql = item / r.parts, part = item - ql * r.parts;
        const float4 *q4 = reinterpret_cast<const float4 *>(r.Q + (int64_t)ql * r.d);
        float4 qa[kMaxU16], qb[kMaxU16];
#pragma unroll
        for (int u = 0; u < kMaxU16; ++u) {
            const int s = li + G * u;
            const bool in = u < r.U && s < d8;
            qa[u] = in ? q4[2 * s] : make_float4(0.f, 0.f, 0.f, 0.f);
            qb[u] = in ? q4[2 * s + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        uint64_t best = ~0ull;
        const int64_t rb = (int64_t)part * r.rows_per_part;
        const int64_t re = rb + r.rows_per_part < r.B ? rb + r.rows_per_part : r.B;
        const uint32_t *cq = r.cand + (int64_t)ql * r.B;
        // candidate ids staged in LDS a chunk at a time (see the FP32 re-rank)
        for (int64_t cb = rb; cb < re; cb += kRowChunk) {
        const int cn = (int)(re - cb < kRowChunk ? re - cb : kRowChunk);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += 256) cid[t] = cq[cb + t];
        __syncthreads();
        for (int base = wv * R; base < cn; base += 4 * R) {
            const int lr = base + slot;
            const int64_t rw = cb + lr;
            uint32_t id = lr < cn ? cid[lr] : 0u;
            const bool valid = lr < cn && id < r.n;
            id = valid ? id : 0u;
            const uint4 *xr = reinterpret_cast<const uint4 *>(r.Xb + (int64_t)id * r.d);
            uint4 xs[kMaxU16];
#pragma unroll
            for (int u = 0; u < kMaxU16; ++u) {
                const int s = li + G * u;
                xs[u] = (u < r.U && s < d8) ? xr[s] : make_uint4(0u, 0u, 0u, 0u);
            }
            float acc = 0.f;
#pragma unroll
            for (int u = 0; u < kMaxU16; ++u) {
                const int s = li + G * u;
                if (u < r.U && s < d8) {
                    const float qv[8] = {qa[u].x, qa[u].y, qa[u].z, qa[u].w, qb[u].x, qb[u].y, qb[u].z, qb[u].w};
                    const uint32_t wd[4] = {xs[u].x, xs[u].y, xs[u].z, xs[u].w};
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const uint32_t h = (t & 1) ? (wd[t >> 1] >> 16) : (wd[t >> 1] & 0xffffu);
                        const float df = bf16_val(h) - qv[t];
                        acc = fmaf(df, df, acc);
                    }
                }
            }
            for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
            const float E = r.xerr[id];
            const float e0 = 2.0f * (sqrtf(acc) + E) * E + E * E;
            const float e = e0 + gam * (acc + e0) + 1e-30f;
            if (valid && li == 0) r.lo[(int64_t)ql * r.B + rw] = acc - e;
            const uint64_t key = valid ? (((uint64_t)__float_as_uint(acc + e) << 32) | id) : ~0ull;
            // only keys below the current k-th can enter the list
            const uint64_t kth = shfl64(best, k - 1);   // every lane takes part in the shuffle
            uint64_t m = __ballot(li == 0 && key < kth);
            while (m != 0ull) {
                const int src = __ffsll((unsigned long long)m) - 1;
                m &= m - 1ull;
                topk_insert(best, shfl64(key, src), k, lane);
            }
        }
        }
        if (lane < k) wl[wv][lane] = best;
        __syncthreads();
        if (wv == 0) {
            for (int w2 = 1; w2 < 4; ++w2)
                for (int j = 0; j < k; ++j) {
                    const uint64_t kk = wl[w2][j];
                    if (kk >= shfl64(best, k - 1)) break;
                    topk_insert(best, kk, k, lane);
                }
            if (lane < k) r.part_keys[((int64_t)ql * r.parts + part) * k + lane] = best;
        }
        __syncthreads();
    }
}

// One block per query: U = k-th smallest upper bound over the parts' lists,
// then the survivors {lower bound <= U} (in no particular order).
__global__ __launch_bounds__(256) void k_survivors(Bf16RerankPass r) {
    __shared__ float Ush;
    __shared__ uint32_t cnt;
    const int lane = threadIdx.x & (kWave - 1), k = r.k;
    for (int ql = blockIdx.x; ql < r.nq; ql += gridDim.x) {
        if (threadIdx.x < kWave) {
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
            const uint64_t kth = shfl64(best, k - 1);
            if (lane == 0) {
                // fewer than k valid candidates: keep them all
                Ush = kth == ~0ull ? __uint_as_float(0x7f800000u) : __uint_as_float((uint32_t)(kth >> 32));
                cnt = 0u;
            }
        }
        __syncthreads();
        const float U = Ush;
        const float *lo = r.lo + (int64_t)ql * r.B;
        const uint32_t *cq = r.cand + (int64_t)ql * r.B;
        uint32_t *out = r.surv + (int64_t)ql * r.B;
        for (int64_t c = threadIdx.x; c < r.B; c += blockDim.x) {
            const uint32_t id = cq[c];
            if (id < r.n && lo[c] <= U) out[atomicAdd(&cnt, 1u)] = id;
        }
        __syncthreads();
        if (threadIdx.x == 0) r.nsurv[ql] = (int32_t)cnt;
        __syncthreads();
    }
}

// One wave per query: relative error of each returned distance against the
// FP64 distance of the same point.
__global__ __launch_bounds__(kWave) void k_relerr(RelErrPass p) {
    const int lane = threadIdx.x;
    for (int ql = blockIdx.x; ql < p.nq; ql += gridDim.x) {
        const float *q = p.Q + (int64_t)ql * p.d;
        for (int j = 0; j < p.k; ++j) {
            const int32_t id = p.ids[(int64_t)ql * p.k + j];
            if (id < 0 || id >= p.n) {   // no result in this slot
                if (lane == 0) p.relerr[(int64_t)ql * p.k + j] = __builtin_nan("");
                continue;
            }
            const float *x = p.X + (int64_t)id * p.d;
            double s = 0.0;
            for (int t = lane; t < p.d; t += kWave) {
                const double v = (double)x[t] - (double)q[t];
                s += v * v;
            }
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
            if (lane == 0) {
                const double t64 = sqrt(s), g = (double)p.dists[(int64_t)ql * p.k + j];
                p.relerr[(int64_t)ql * p.k + j] = t64 > 0.0 ? fabs(g - t64) / t64 : fabs(g);
            }
        }
    }
}

// ------------------------------------------------------------- plans --
Launch plan_centre_dists_bf16(const CentreBf16Pass &p) {
    Launch L;
    L.func = reinterpret_cast<const void *>(&k_centre_dists_bf16);
    L.grid = dim3((unsigned)std::max(1, (p.nq + 15) / 16), (unsigned)p.nh);
    L.block = dim3((unsigned)(kWave * ((p.sk + 15) / 16)));
    return L;
}

Launch plan_rerank_bf16(const Bf16RerankPass &r, int cap) {
    Launch L;
    int64_t items = (int64_t)r.nq * r.parts;
    if (items < 1) items = 1;
    L.func = reinterpret_cast<const void *>(&k_rerank_bf16);
    L.grid = dim3((unsigned)(cap > 0 && cap < items ? cap : items));
    L.block = dim3(256);
    return L;
}

Launch plan_survivors(const Bf16RerankPass &r) {
    Launch L;
    L.func = reinterpret_cast<const void *>(&k_survivors);
    L.grid = dim3((unsigned)std::max(1, r.nq));
    L.block = dim3(256);
    return L;
}

Launch plan_relerr(const RelErrPass &p) {
    Launch L;
    L.func = reinterpret_cast<const void *>(&k_relerr);
    L.grid = dim3((unsigned)std::max(1, p.nq));
    L.block = dim3(kWave);
    return L;
}

hipError_t launch_bf16_rows(const float *X, int64_t n, int d, uint16_t *Xb, float *xerr, hipStream_t s) {
    hipLaunchKernelGGL(k_bf16_rows, dim3(2048), dim3(256), 0, s, X, n, d, Xb, xerr);
    return hipGetLastError();
}

hipError_t launch_bf16_centres(const float *cent, const HalfDims *halves, int nh, int sk, int d, uint16_t *centb,
                               float *cnorm2, hipStream_t s) {
    hipLaunchKernelGGL(k_bf16_centres, dim3(64), dim3(256), 0, s, cent, halves, nh, sk, d, centb, cnorm2);
    return hipGetLastError();
}

}  // namespace suco
