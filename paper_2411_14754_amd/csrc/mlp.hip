// Learned activation budget: a small MLP that predicts a per-query collision
// ratio alpha from cheap query features.
//
// Features (2*ns + 1 per query): for every subspace half, the Euclidean
// distance from the query half to its nearest centre (the square root of the
// smallest step-1 distance, computed with the activation step's arithmetic),
// and the query norm.
//
// Network: x = (f - mu) / sigma; h1 = GELU(W1 x + b1); h2 = GELU(W2 h1 + b2);
// y = W3 h2 + b3, y predicting log alpha; GELU(x) = x * Phi(x) (Hendrycks and
// Gimpel 2016), Phi from erff.  Parameters in one flat FP32 array in the order
// W1 [H][n_in], b1 [H], W2 [H][H], b2 [H], W3 [H], b3 [1].
//
// Training (FP32): per row, a block computes the forward pass and the row's
// back-propagated pre-activation gradients; a second kernel forms the
// parameter gradients as sums over the rows in row order (deterministic); a
// third applies Adam (Kingma and Ba 2015, with bias correction).  Loss is the
// mean squared error over the batch.
//
// Inference (BF16): weights and layer inputs are rounded to BF16 (nearest,
// ties to even) and products are accumulated in FP32 in index order; the
// collision ratio is alpha = clamp(scale * exp(y), alpha_min, alpha_max).  The
// rounded copy the inference kernels read holds W1 and W2 transposed (W1 as
// [n_in][H], W2 as [H][H] by column), so that hidden unit j's weights are read
// by thread j with the loads of a wave falling on consecutive words.
#include "runtime_impl.h"

namespace suco {

constexpr int kH = 128;        // hidden width supported by the kernels
constexpr int kMaxIn = 255;    // 2*ns + 1 for ns <= 127

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Round to the nearest BF16 value (ties to even), returned as FP32.
__device__ __forceinline__ float bf16r(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;   // inf / nan unchanged
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// ------------------------------------------------------------- features --
// A block's copies for the feature computation, in dynamic LDS: the half
// table, the centre table when it has at most kFeatCentMax values, and the
// current query row when d <= kFeatQMax (otherwise those are read from HBM;
// the values and the arithmetic are the same either way).
constexpr int kFeatCentMax = 16384;   // values of the centre table (64 KB)
constexpr int kFeatQMax = 4096;
constexpr int kFeatHalfBytes = 256;    // 2*kMaxNs HalfDims, padded

__host__ __device__ inline bool feat_cent_staged(int sk, int d) { return (int64_t)sk * d <= kFeatCentMax; }
__host__ __device__ inline bool feat_q_staged(int d) { return d <= kFeatQMax; }
inline size_t feat_lds_bytes(int sk, int d) {
    return kFeatHalfBytes + (feat_cent_staged(sk, d) ? 4 * (size_t)sk * d : 0) + (feat_q_staged(d) ? 4 * (size_t)d : 0);
}

struct FeatSrc {
    const HalfDims *hs;   // [2ns] in LDS
    const float *cent;    // centre table (LDS or HBM): half g's centre c at sk*dim0 + c*w
    float *qs;            // query row copy in LDS, or null
};

// Fill a block's copies (ends with a barrier), sixteen loads in flight per thread.
__device__ __forceinline__ FeatSrc feat_stage(const IndexView &ix, uint4 *dyn) {
    const int tid = threadIdx.x, sk = ix.sk;
    HalfDims *hs = reinterpret_cast<HalfDims *>(dyn);
    float *cs = reinterpret_cast<float *>(reinterpret_cast<char *>(dyn) + kFeatHalfBytes);
    const bool cst = feat_cent_staged(sk, ix.d);
    for (int g = tid; g < 2 * ix.ns; g += blockDim.x) hs[g] = ix.halves[g];
    const int nc = cst ? sk * ix.d : 0;
    for (int i0 = tid; i0 < nc; i0 += 16 * blockDim.x) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            v[u] = ix.cent[i < nc ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < nc) cs[i] = v[u];
        }
    }
    __syncthreads();
    FeatSrc F;
    F.hs = hs;
    F.cent = cst ? cs : ix.cent;
    F.qs = feat_q_staged(ix.d) ? cs + nc : nullptr;
    return F;
}

// The 2*n_s + 1 features of one query into out[] (global or LDS), by the
// whole block of 128 threads: each half has a group of tph lanes (a power of
// two, 128 / tph >= 2*n_s) that take its centres c = r, r + tph, ... with the
// activation step's arithmetic (FMA over the half's dimensions in order,
// values loaded eight at a time) and keep a running minimum; the group's
// minimum comes from lane shuffles (a minimum is exact in any order); then
// the query norm (lane-strided partial sums, a fixed reduction order).  Ends
// with a barrier.
__device__ __forceinline__ void query_features(const IndexView &ix, const FeatSrc &src, const float *qv, float *out,
                                               uint32_t *mins, float *part) {
    const int sk = ix.sk, nh = 2 * ix.ns;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    if (src.qs)
        for (int j = tid; j < ix.d; j += blockDim.x) src.qs[j] = qv[j];
    __syncthreads();
    const float *q = src.qs ? src.qs : qv;
    int tph = 64;
    while (tph * nh > (int)blockDim.x) tph >>= 1;
    const int g = tid / tph, r = tid - g * tph;
    float m = __int_as_float(0x7f800000);
    if (g < nh) {
        const HalfDims hd = src.hs[g];
        const float *qp = q + hd.dim0;
        for (int c = r; c < sk; c += tph) {
            const float *cp = src.cent + (int64_t)sk * hd.dim0 + (int64_t)c * hd.w;
            float s = 0.f;
            for (int j0 = 0; j0 < hd.w; j0 += 8) {
                // sixteen loads issued together (indices past the half repeat its last
                // dimension, so none is conditional), then the FMAs in dimension order
                float a8[8], c8[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int jj = j0 + u < hd.w ? j0 + u : hd.w - 1;
                    a8[u] = qp[jj];
                    c8[u] = cp[jj];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (j0 + u < hd.w) {
                        const float t2 = a8[u] - c8[u];
                        s = fmaf(t2, t2, s);
                    }
                }
            }
            m = fminf(m, s);
        }
    }
    for (int o = 1; o < tph; o <<= 1) m = fminf(m, __shfl_xor(m, o, kWave));
    if (g < nh && r == 0) mins[g] = __float_as_uint(m);
    float nsq = 0.f;
    for (int j = tid; j < ix.d; j += blockDim.x) nsq = fmaf(q[j], q[j], nsq);
    for (int o = 32; o > 0; o >>= 1) nsq += __shfl_xor(nsq, o, kWave);
    if (lane == 0) part[tid / kWave] = nsq;
    __syncthreads();
    for (int g = tid; g < nh; g += blockDim.x) out[g] = __fsqrt_rn(__uint_as_float(mins[g]));
    if (tid == 0) out[nh] = __fsqrt_rn(part[0] + part[1]);
    __syncthreads();
}

__global__ __launch_bounds__(128) void k_features(FeatPass fp) {
    extern __shared__ uint4 feat_dyn[];
    __shared__ uint32_t mins[2 * kMaxNs];   // bits of each half's smallest distance (non-negative floats)
    __shared__ float part[128 / kWave];
    const int nq = fp.nq_dev ? *fp.nq_dev : fp.nq;
    if ((int)blockIdx.x >= nq) return;
    const int nf = 2 * fp.ix.ns + 1;
    const FeatSrc src = feat_stage(fp.ix, feat_dyn);
    for (int q = blockIdx.x; q < nq; q += gridDim.x)
        query_features(fp.ix, src, fp.Q + (int64_t)q * fp.ix.d, fp.F + (int64_t)q * nf, mins, part);
}

// ---------------------------------------------------------- inference --
// Blocks of H threads, persistent over rows; weights are pre-rounded BF16
// values in FP32.  Thread j keeps row j of the second layer's weights in
// registers for all its rows (read once per block), so the per-row work reads
// only the previous layer's outputs, broadcast from LDS.
struct InferRegs {
    float w2[kH];
    float b1, b2, w3;
};

__device__ __forceinline__ void infer_regs(const MlpView &w, InferRegs &R) {
    const int j = threadIdx.x;
#pragma unroll
    for (int i = 0; i < kH; ++i) R.w2[i] = w.W2[i * kH + j];   // transposed copy: W2[j][i]
    R.b1 = w.b1[j];
    R.b2 = w.b2[j];
    R.w3 = w.W3[j];
}

// Row r of the network from its raw features fr[] (any memory): standardised
// and rounded into x, two hidden layers, the output and its alpha.  Ends with
// a barrier.
__device__ __forceinline__ void infer_row(const InferPass &ip, const InferRegs &R, const float *fr, const int r,
                                          float *x, float *h, float *red) {
    const MlpView &w = ip.w;
    const int j = threadIdx.x;
    for (int i = j; i < w.n_in; i += kH) x[i] = bf16r((fr[i] - w.mu[i]) / w.sigma[i]);
    __syncthreads();
    float z = R.b1;
    for (int i = 0; i < w.n_in; ++i) z = fmaf(w.W1[i * kH + j], x[i], z);   // transposed copy: W1[j][i]
    h[j] = bf16r(gelu_f(z));
    __syncthreads();
    float z2 = R.b2;
#pragma unroll
    for (int i = 0; i < kH; ++i) z2 = fmaf(R.w2[i], h[i], z2);
    const float h2 = bf16r(gelu_f(z2));
    float part = R.w3 * h2;
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
    if ((j & (kWave - 1)) == 0) red[j / kWave] = part;
    __syncthreads();
    if (j == 0) {
        const float yv = w.b3[0] + red[0] + red[1];
        if (ip.y) ip.y[r] = yv;
        float a = ip.scale * expf(yv);
        // a NaN prediction takes the largest budget, like +inf
        a = a <= ip.amax ? (a >= ip.amin ? a : ip.amin) : ip.amax;
        if (ip.alpha) ip.alpha[r] = a;
        if (ip.alpha64) ip.alpha64[r] = (double)a;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kH) void k_mlp_infer(InferPass ip) {
    __shared__ float x[kMaxIn + 1];
    __shared__ float h[kH];
    __shared__ float red[kH / kWave];
    const int m = ip.m_dev ? *ip.m_dev : ip.m;
    if ((int)blockIdx.x >= m) return;
    InferRegs R;
    infer_regs(ip.w, R);
    for (int r = blockIdx.x; r < m; r += gridDim.x) infer_row(ip, R, ip.F + (int64_t)r * ip.w.n_in, r, x, h, red);
}

// The query path's alphas in one kernel: each query's features go straight
// from the feature computation (LDS) into the network, the same values and
// arithmetic as k_features followed by k_mlp_infer.
__global__ __launch_bounds__(kH) void k_learned_alpha(FeatPass fp, InferPass ip) {
    static_assert(kH == 128, "the feature computation is written for blocks of 128 threads");
    extern __shared__ uint4 feat_dyn[];
    __shared__ uint32_t mins[2 * kMaxNs];
    __shared__ float part[kH / kWave];
    __shared__ float fq[2 * kMaxNs + 1];
    __shared__ float x[kMaxIn + 1];
    __shared__ float h[kH];
    __shared__ float red[kH / kWave];
    const int nq = fp.nq_dev ? *fp.nq_dev : fp.nq;
    if ((int)blockIdx.x >= nq) return;
    InferRegs R;
    infer_regs(ip.w, R);
    const FeatSrc src = feat_stage(fp.ix, feat_dyn);
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {
        query_features(fp.ix, src, fp.Q + (int64_t)q * fp.ix.d, fq, mins, part);
        infer_row(ip, R, fq, q, x, h, red);
    }
}

// The same computation sixteen query rows at a time (the query path's form
// when the centre table is staged, the widest half has at most 16 dimensions
// and the tile's rows fit in LDS): blocks of 256 threads; a thread takes one
// (row, half) pair for the features, keeping the half of the query in
// registers, and hidden unit j = t mod 128 of eight rows for the network.
// Every value is computed with the arithmetic and in the order of
// k_features and k_mlp_infer (FMA chains in index order, the norm's and the
// output's partial sums over the same lanes and reduced with the same
// shuffles), so the alphas equal theirs bit for bit; the latencies of a row
// (loads, barriers, the reductions) are paid once per sixteen rows.
constexpr int kRT = 16;            // rows per tile
constexpr int kRTHalfW = 16;       // widest half kept in registers
constexpr int kRTQMax = 16384;     // floats of a tile's staged rows (padded to d + 1)

constexpr size_t kRTLdsMax = 128 * 1024;   // dynamic LDS of the tile kernel (its static arrays take ~13 KB more)

__host__ __device__ inline size_t learned_tile_lds(int sk, int d) {
    return kFeatHalfBytes + 4 * (size_t)sk * d + 4 * (size_t)kRT * (d + 1) + 2 * (size_t)kH * kH;
}
__host__ __device__ inline bool learned_tiles_ok(int sk, int d, int ns, int wmax) {
    return feat_cent_staged(sk, d) && kRT * (d + 1) <= kRTQMax && wmax <= kRTHalfW && 2 * ns + 1 <= 32 &&
           learned_tile_lds(sk, d) <= kRTLdsMax;
}

// The smallest squared distance from a query half qp (w <= HW values) to the
// half's sk centres (centre c at cb + c*w), the activation step's arithmetic.
template <int HW>
__device__ __forceinline__ float nearest_centre(const float *qp, const float *cb, const int sk, const int w) {
    float qr[HW];
#pragma unroll
    for (int u = 0; u < HW; ++u) qr[u] = qp[u < w ? u : w - 1];
    float m = __int_as_float(0x7f800000);
#pragma unroll 2
    for (int c = 0; c < sk; ++c) {
        const float *cp = cb + c * w;
        float cv[HW];
#pragma unroll
        for (int u = 0; u < HW; ++u) cv[u] = cp[u < w ? u : w - 1];
        float s = 0.f;
#pragma unroll
        for (int u = 0; u < HW; ++u) {
            if (u < w) {
                const float t2 = qr[u] - cv[u];
                s = fmaf(t2, t2, s);
            }
        }
        m = fminf(m, s);
    }
    return m;
}

__global__ __launch_bounds__(256) void k_learned_alpha_tiles(FeatPass fp, InferPass ip) {
    static_assert(kH == 128 && kRT == 16, "the tile kernel is written for 128 hidden units and 16 rows");
    extern __shared__ uint4 feat_dyn[];
    __shared__ float fq[kRT][33];      // raw features
    __shared__ float xs[kRT][33];      // standardised, rounded
    __shared__ __align__(16) float h1[kRT][kH];
    __shared__ float red[4][kRT];
    __shared__ float mus[32], sgs[32];
    const IndexView &ix = fp.ix;
    const MlpView &W = ip.w;
    const int nq = fp.nq_dev ? *fp.nq_dev : fp.nq;
    const int ntiles = (nq + kRT - 1) / kRT;
    if ((int)blockIdx.x >= ntiles) return;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int j = tid & (kH - 1), rg = tid / kH;
    const int d = ix.d, sk = ix.sk, nh = 2 * ix.ns, nin = W.n_in, ds = d + 1;
    const float b1 = W.b1[j], b2 = W.b2[j], w3 = W.W3[j];
    // unit j's first-layer weights (n_in <= 32), all loads in flight at once
    float w1r[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) w1r[i] = W.W1[(i < nin ? i : nin - 1) * kH + j];   // transposed copy: W1[j][i]
    for (int i = tid; i < nin; i += blockDim.x) { mus[i] = W.mu[i]; sgs[i] = W.sigma[i]; }
    float *qt = reinterpret_cast<float *>(reinterpret_cast<char *>(feat_dyn) + kFeatHalfBytes) + (size_t)sk * d;
    // the second layer in LDS as BF16 bits, unit j's weight of input i at i*kH + j
    // (the rounded copy's values have zero low halves, so this is exact)
    uint16_t *w2s = reinterpret_cast<uint16_t *>(qt + kRT * ds);
    for (int e0 = tid; e0 < kH * kH; e0 += 16 * blockDim.x) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = W.W2[e0 + u * (int)blockDim.x];       // kH*kH is a multiple of 16*256
#pragma unroll
        for (int u = 0; u < 16; ++u) w2s[e0 + u * (int)blockDim.x] = (uint16_t)(__float_as_uint(v[u]) >> 16);
    }
    const FeatSrc src = feat_stage(ix, feat_dyn);          // staged centres (checked on the host); ends with a barrier
    int wmax = 0;
    for (int g = 0; g < nh; ++g) wmax = src.hs[g].w > wmax ? src.hs[g].w : wmax;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int r0 = tile * kRT, nr = nq - r0 < kRT ? nq - r0 : kRT;
        // the tile's rows (rows past the last query repeat it), sixteen loads in flight
        for (int e0 = tid; e0 < kRT * d; e0 += 16 * blockDim.x) {
            float v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = e0 + u * (int)blockDim.x, ee = e < kRT * d ? e : 0;
                const int r = ee / d, c = ee - r * d;
                v[u] = fp.Q[(int64_t)(r0 + (r < nr ? r : nr - 1)) * d + c];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = e0 + u * (int)blockDim.x;
                if (e < kRT * d) {
                    const int r = e / d, c = e - r * d;
                    qt[r * ds + c] = v[u];
                }
            }
        }
        __syncthreads();
        // each half's nearest centre: pair p = (row p mod 16, half p / 16)
        for (int p = tid; p < kRT * nh; p += blockDim.x) {
            const int r = p & (kRT - 1), g = p / kRT;
            const HalfDims hd = src.hs[g];
            const float *qp = qt + r * ds + hd.dim0;
            const float *cb = src.cent + (int64_t)sk * hd.dim0;
            fq[r][g] = __fsqrt_rn(wmax <= 8 ? nearest_centre<8>(qp, cb, sk, hd.w) : nearest_centre<kRTHalfW>(qp, cb, sk, hd.w));
        }
        // the norm of row r by wave r mod 4: the partial sums of threads t and
        // 64 + t of a 128-thread block, each reduced over its wave, then added
        for (int r = wv; r < kRT; r += 4) {
            const float *q = qt + r * ds;
            float plo = 0.f, phi = 0.f;
            for (int jj = lane; jj < d; jj += 128) plo = fmaf(q[jj], q[jj], plo);
            for (int jj = 64 + lane; jj < d; jj += 128) phi = fmaf(q[jj], q[jj], phi);
            for (int o = 32; o > 0; o >>= 1) {
                plo += __shfl_xor(plo, o, kWave);
                phi += __shfl_xor(phi, o, kWave);
            }
            if (lane == 0) fq[r][nh] = __fsqrt_rn(plo + phi);
        }
        __syncthreads();
        for (int e = tid; e < kRT * nin; e += blockDim.x) {
            const int r = e / nin, i = e - r * nin;
            xs[r][i] = bf16r((fq[r][i] - mus[i]) / sgs[i]);
        }
        __syncthreads();
        // first layer: unit j of rows 8rg .. 8rg + 7
        float z[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) z[u] = b1;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            if (i < nin) {
#pragma unroll
                for (int u = 0; u < 8; ++u) z[u] = fmaf(w1r[i], xs[8 * rg + u][i], z[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) h1[8 * rg + u][j] = bf16r(gelu_f(z[u]));
        __syncthreads();
        // second layer and the output's partial sums (waves 2rg, 2rg + 1 hold units 0..63, 64..127)
        float z2[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) z2[u] = b2;
#pragma unroll 2
        for (int i = 0; i < kH; i += 4) {
            float wi[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) wi[v] = __uint_as_float((uint32_t)w2s[(i + v) * kH + j] << 16);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float4 hv = *reinterpret_cast<const float4 *>(&h1[8 * rg + u][i]);
                z2[u] = fmaf(wi[0], hv.x, z2[u]);
                z2[u] = fmaf(wi[1], hv.y, z2[u]);
                z2[u] = fmaf(wi[2], hv.z, z2[u]);
                z2[u] = fmaf(wi[3], hv.w, z2[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            float part = w3 * bf16r(gelu_f(z2[u]));
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
            if (lane == 0) red[wv][8 * rg + u] = part;
        }
        __syncthreads();
        float yv = 0.f;
        if (tid < nr) yv = W.b3[0] + red[2 * (tid / 8)][tid] + red[2 * (tid / 8) + 1][tid];
        // the tile's LDS is free once red[] is read; the stores go out after the
        // barrier, so that it does not wait for them
        __syncthreads();
        if (tid < nr) {
            if (ip.y) ip.y[r0 + tid] = yv;
            float a = ip.scale * expf(yv);
            // a NaN prediction takes the largest budget, like +inf
            a = a <= ip.amax ? (a >= ip.amin ? a : ip.amin) : ip.amax;
            if (ip.alpha) ip.alpha[r0 + tid] = a;
            if (ip.alpha64) ip.alpha64[r0 + tid] = (double)a;
        }
    }
}

// ------------------------------------------------------------ training --
struct TrainRows {
    MlpView w;
    const float *F, *t;
    const int32_t *order;   // row permutation or null
    int m;                  // rows in this batch
    int64_t row0;           // first position in `order` (or in F) of this batch
    float *xs, *z1, *h1, *z2, *h2, *dz1, *dz2, *dy, *sq;   // per-row workspaces
};

// One block of H threads per row: forward pass, squared error, and the row's
// gradients with respect to the pre-activations of both hidden layers.
__global__ __launch_bounds__(kH) void k_mlp_rows(TrainRows a) {
    __shared__ float x[kMaxIn + 1];
    __shared__ float h[kH];
    __shared__ float d2[kH];
    __shared__ float red[kH / kWave];
    const int j = threadIdx.x, r = blockIdx.x, n_in = a.w.n_in;
    const int64_t pos = a.row0 + r;
    const int64_t src = a.order ? a.order[pos] : pos;
    for (int i = j; i < n_in; i += kH) {
        const float v = (a.F[src * n_in + i] - a.w.mu[i]) / a.w.sigma[i];
        x[i] = v;
        a.xs[(int64_t)r * n_in + i] = v;
    }
    __syncthreads();
    float z = a.w.b1[j];
    for (int i = 0; i < n_in; ++i) z = fmaf(a.w.W1[j * n_in + i], x[i], z);
    const float g1 = gelu_f(z);
    a.z1[(int64_t)r * kH + j] = z;
    a.h1[(int64_t)r * kH + j] = g1;
    h[j] = g1;
    __syncthreads();
    float z2 = a.w.b2[j];
    for (int i = 0; i < kH; ++i) z2 = fmaf(a.w.W2[j * kH + i], h[i], z2);
    const float g2 = gelu_f(z2);
    a.z2[(int64_t)r * kH + j] = z2;
    a.h2[(int64_t)r * kH + j] = g2;
    float part = a.w.W3[j] * g2;
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
    if ((j & (kWave - 1)) == 0) red[j / kWave] = part;
    __syncthreads();
    const float y = a.w.b3[0] + red[0] + red[1];
    const float e = y - a.t[src];
    const float dy = 2.0f * e / (float)a.m;
    if (j == 0) {
        a.dy[r] = dy;
        a.sq[r] = e * e;
    }
    const float dz2 = dy * a.w.W3[j] * gelu_grad_f(z2);
    a.dz2[(int64_t)r * kH + j] = dz2;
    d2[j] = dz2;
    __syncthreads();
    float dh1 = 0.f;
    for (int o = 0; o < kH; ++o) dh1 = fmaf(a.w.W2[o * kH + j], d2[o], dh1);
    a.dz1[(int64_t)r * kH + j] = dh1 * gelu_grad_f(z);
}

// Parameter gradients: one thread per parameter, summing over the rows in order.
__global__ __launch_bounds__(256) void k_mlp_grads(TrainRows a, float *g, float *loss) {
    const int n_in = a.w.n_in;
    const int64_t nW1 = (int64_t)kH * n_in, nW2 = (int64_t)kH * kH;
    const int64_t total = nW1 + kH + nW2 + kH + kH + 1;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == total && loss) {
        float s = 0.f;
        for (int r = 0; r < a.m; ++r) s += a.sq[r];
        *loss = s / (float)a.m;
    }
    if (p >= total) return;
    float s = 0.f;
    if (p < nW1) {                                   // dW1[j][i] = sum_r dz1[r][j] x[r][i]
        const int jj = (int)(p / n_in), i = (int)(p % n_in);
        for (int r = 0; r < a.m; ++r) s = fmaf(a.dz1[(int64_t)r * kH + jj], a.xs[(int64_t)r * n_in + i], s);
    } else if (p < nW1 + kH) {                       // db1
        const int jj = (int)(p - nW1);
        for (int r = 0; r < a.m; ++r) s += a.dz1[(int64_t)r * kH + jj];
    } else if (p < nW1 + kH + nW2) {                 // dW2[j][i] = sum_r dz2[r][j] h1[r][i]
        const int64_t q = p - nW1 - kH;
        const int jj = (int)(q / kH), i = (int)(q % kH);
        for (int r = 0; r < a.m; ++r) s = fmaf(a.dz2[(int64_t)r * kH + jj], a.h1[(int64_t)r * kH + i], s);
    } else if (p < nW1 + kH + nW2 + kH) {            // db2
        const int jj = (int)(p - nW1 - kH - nW2);
        for (int r = 0; r < a.m; ++r) s += a.dz2[(int64_t)r * kH + jj];
    } else if (p < total - 1) {                      // dW3[j] = sum_r dy[r] h2[r][j]
        const int jj = (int)(p - nW1 - kH - nW2 - kH);
        for (int r = 0; r < a.m; ++r) s = fmaf(a.dy[r], a.h2[(int64_t)r * kH + jj], s);
    } else {                                         // db3
        for (int r = 0; r < a.m; ++r) s += a.dy[r];
    }
    g[p] = s;
}

__global__ __launch_bounds__(256) void k_adam(float *w, const float *g, float *m1, float *m2, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float gp = g[p];
    const float a = b1 * m1[p] + (1.0f - b1) * gp;
    const float v = b2 * m2[p] + (1.0f - b2) * gp * gp;
    m1[p] = a;
    m2[p] = v;
    w[p] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// The inference copy: every parameter rounded to BF16, W1 and W2 transposed.
__global__ void k_round_bf16(const float *src, float *dst, int64_t n, int n_in) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t nW1 = (int64_t)kH * n_in, o2 = nW1 + kH;
    int64_t at = p;
    if (p < nW1) {
        at = (p % n_in) * kH + p / n_in;                     // W1[j][i] -> [i][j]
    } else if (p >= o2 && p < o2 + (int64_t)kH * kH) {
        const int64_t e = p - o2;
        at = o2 + (e % kH) * kH + e / kH;                    // W2[j][i] -> [i][j]
    }
    dst[at] = bf16r(src[p]);
}

}  // namespace suco

using namespace suco;

struct suco_mlp {
    uint64_t magic = 0x5375436f4d4c5031ULL;
    int device = 0, n_in = 0, H = kH;
    int64_t np = 0;
    float *w = nullptr, *wb = nullptr;       // FP32 parameters; BF16-rounded copy for inference (W1, W2 transposed)
    float *m1 = nullptr, *m2 = nullptr, *g = nullptr;
    float *mu = nullptr, *sigma = nullptr;
    float *loss = nullptr;
    int64_t steps = 0;
    bool wb_valid = false;
    // training workspace (rows)
    int rows_cap = 0;
    float *ws = nullptr;
    std::mutex mu_lock;

    MlpView view(const float *params) const {
        MlpView v;
        v.n_in = n_in; v.H = H;
        v.W1 = params;
        v.b1 = v.W1 + (int64_t)H * n_in;
        v.W2 = v.b1 + H;
        v.b2 = v.W2 + (int64_t)H * H;
        v.W3 = v.b2 + H;
        v.b3 = v.W3 + H;
        v.mu = mu; v.sigma = sigma;
        return v;
    }
    void release() {
        for (void *p : {(void *)w, (void *)wb, (void *)m1, (void *)m2, (void *)g, (void *)mu, (void *)sigma,
                        (void *)loss, (void *)ws})
            if (p) (void)hipFree(p);
        w = wb = m1 = m2 = g = mu = sigma = loss = ws = nullptr;
        magic = 0;
    }
};

namespace {

bool mlp_ok(const suco_mlp *p) { return p != nullptr && p->magic == 0x5375436f4d4c5031ULL; }

int64_t nparams(int n_in, int H) { return (int64_t)H * n_in + H + (int64_t)H * H + H + H + 1; }

int ensure_rows(suco_mlp *p, int rows) {
    if (rows <= p->rows_cap) return SUCO_OK;
    if (p->ws) (void)hipFree(p->ws);
    p->ws = nullptr;
    p->rows_cap = 0;
    const size_t per = (size_t)p->n_in + 6 * kH + 2;
    int rc = dev_alloc(&p->ws, per * rows);
    if (rc) return rc;
    p->rows_cap = rows;
    return SUCO_OK;
}

TrainRows rows_args(suco_mlp *p, const float *F, const float *t, const int32_t *order, int m, int64_t row0) {
    TrainRows a{};
    a.w = p->view(p->w);
    a.F = F; a.t = t; a.order = order; a.m = m; a.row0 = row0;
    float *q = p->ws;
    const int cap = p->rows_cap;
    a.xs = q; q += (size_t)cap * p->n_in;
    a.z1 = q; q += (size_t)cap * kH;
    a.h1 = q; q += (size_t)cap * kH;
    a.z2 = q; q += (size_t)cap * kH;
    a.h2 = q; q += (size_t)cap * kH;
    a.dz1 = q; q += (size_t)cap * kH;
    a.dz2 = q; q += (size_t)cap * kH;
    a.dy = q; q += cap;
    a.sq = q;
    return a;
}

hipError_t grads_pass(suco_mlp *p, const TrainRows &a, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_rows, dim3((unsigned)a.m), dim3(kH), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tot = p->np + 1;
    hipLaunchKernelGGL(k_mlp_grads, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a, p->g, p->loss);
    return hipGetLastError();
}

int refresh_bf16(suco_mlp *p, hipStream_t st) {
    if (p->wb_valid) return SUCO_OK;
    hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)((p->np + 255) / 256)), dim3(256), 0, st, p->w, p->wb, p->np,
                       p->n_in);
    HIPCHECK(hipGetLastError());
    p->wb_valid = true;
    return SUCO_OK;
}

}  // namespace

namespace suco {
Launch plan_features(const IndexView &ix, int nq_cap) {
    Launch L;
    L.func = reinterpret_cast<const void *>(&k_features);
    L.grid = dim3((unsigned)std::max(1, std::min(nq_cap, 2048)));
    L.block = dim3(128);
    L.lds = feat_lds_bytes(ix.sk, ix.d);
    return L;
}

Launch plan_learned_alpha(const IndexView &ix, int wmax, int nq_cap) {
    Launch L;
    if (learned_tiles_ok(ix.sk, ix.d, ix.ns, wmax)) {
        L.func = reinterpret_cast<const void *>(&k_learned_alpha_tiles);
        L.grid = dim3((unsigned)std::max(1, std::min((nq_cap + kRT - 1) / kRT, 2048)));
        L.block = dim3(256);
        L.lds = learned_tile_lds(ix.sk, ix.d);
        return L;
    }
    L.func = reinterpret_cast<const void *>(&k_learned_alpha);
    L.grid = dim3((unsigned)std::max(1, std::min(nq_cap, 2048)));
    L.block = dim3(kH);
    L.lds = feat_lds_bytes(ix.sk, ix.d);
    return L;
}

Launch plan_mlp_infer(int m_cap) {
    Launch L;
    L.func = reinterpret_cast<const void *>(&k_mlp_infer);
    L.grid = dim3((unsigned)std::max(1, std::min(m_cap, 2048)));
    L.block = dim3(kH);
    return L;
}

MlpView mlp_infer_view(suco_mlp *p) { return p->view(p->wb); }
int mlp_n_in(const suco_mlp *p) { return p->n_in; }
int mlp_prepare(suco_mlp *p, hipStream_t st) { return refresh_bf16(p, st); }
bool mlp_valid(const suco_mlp *p) { return mlp_ok(p); }
}  // namespace suco

extern "C" {

int64_t suco_mlp_num_params(int32_t n_in, int32_t hidden) {
    return (n_in < 1 || hidden != kH) ? -1 : nparams(n_in, hidden);
}

int suco_mlp_create(int32_t n_in, int32_t hidden, const float *params, uint64_t seed, suco_mlp **out) {
    if (!out) return fail(SUCO_E_INVAL, "out must not be NULL");
    if (n_in < 1 || n_in > kMaxIn) return fail(SUCO_E_INVAL, "n_in must be in [1, 255]");
    if (hidden != kH) return fail(SUCO_E_UNSUPPORTED, "the kernels support hidden = 128");
    suco_mlp *p = new (std::nothrow) suco_mlp();
    if (!p) return fail(SUCO_E_NOMEM, "host allocation failed");
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return fail(SUCO_E_HIP, "no device"); }
    p->n_in = n_in;
    p->np = nparams(n_in, kH);
    int rc;
    if ((rc = dev_alloc(&p->w, p->np)) || (rc = dev_alloc(&p->wb, p->np)) || (rc = dev_alloc(&p->m1, p->np)) ||
        (rc = dev_alloc(&p->m2, p->np)) || (rc = dev_alloc(&p->g, p->np)) || (rc = dev_alloc(&p->mu, n_in)) ||
        (rc = dev_alloc(&p->sigma, n_in)) || (rc = dev_alloc(&p->loss, 1))) {
        p->release();
        delete p;
        return rc;
    }
    std::vector<float> h((size_t)p->np, 0.f);
    if (params) {
        std::memcpy(h.data(), params, sizeof(float) * p->np);
    } else {
        // uniform in +-sqrt(3 / fan_in) from SplitMix64 draws; biases zero
        const int64_t segs[3][2] = {{0, (int64_t)kH * n_in}, {(int64_t)kH * n_in + kH, (int64_t)kH * kH},
                                    {(int64_t)kH * n_in + kH + (int64_t)kH * kH + kH, kH}};
        const int fan[3] = {n_in, kH, kH};
        uint64_t m = 0;
        for (int s = 0; s < 3; ++s) {
            const double bound = std::sqrt(3.0 / fan[s]);
            for (int64_t t = 0; t < segs[s][1]; ++t) {
                const double u = (double)(splitmix64_at(seed, m++) >> 11) * (1.0 / 9007199254740992.0);
                h[segs[s][0] + t] = (float)((2.0 * u - 1.0) * bound);
            }
        }
    }
    std::vector<float> zeros((size_t)p->np, 0.f), ones((size_t)n_in, 1.f), zin((size_t)n_in, 0.f);
    hipError_t e = hipMemcpy(p->w, h.data(), sizeof(float) * p->np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->m1, zeros.data(), sizeof(float) * p->np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->m2, zeros.data(), sizeof(float) * p->np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->mu, zin.data(), sizeof(float) * n_in, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->sigma, ones.data(), sizeof(float) * n_in, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        p->release();
        delete p;
        return fail(SUCO_E_HIP, std::string("mlp upload: ") + hipGetErrorString(e));
    }
    *out = p;
    return SUCO_OK;
}

int suco_mlp_set_norm(suco_mlp *p, const float *mu, const float *sigma) {
    if (!mlp_ok(p)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    if (!mu || !sigma) return fail(SUCO_E_INVAL, "mu and sigma must not be NULL");
    for (int i = 0; i < p->n_in; ++i)
        if (!(sigma[i] > 0.f)) return fail(SUCO_E_INVAL, "sigma must be positive");
    std::lock_guard<std::mutex> lock(p->mu_lock);
    DeviceGuard dg(p->device);
    HIPCHECK(hipMemcpy(p->mu, mu, sizeof(float) * p->n_in, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(p->sigma, sigma, sizeof(float) * p->n_in, hipMemcpyHostToDevice));
    return SUCO_OK;
}

int suco_mlp_get_params(const suco_mlp *p, float *params) {
    if (!mlp_ok(p)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    if (!params) return fail(SUCO_E_INVAL, "params must not be NULL");
    DeviceGuard dg(p->device);
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(params, p->w, sizeof(float) * p->np, hipMemcpyDeviceToHost));
    return SUCO_OK;
}

int suco_mlp_set_params(suco_mlp *p, const float *params) {
    if (!mlp_ok(p)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    if (!params) return fail(SUCO_E_INVAL, "params must not be NULL");
    std::lock_guard<std::mutex> lock(p->mu_lock);
    DeviceGuard dg(p->device);
    HIPCHECK(hipMemcpy(p->w, params, sizeof(float) * p->np, hipMemcpyHostToDevice));
    p->wb_valid = false;
    return SUCO_OK;
}

int suco_mlp_forward_backward(suco_mlp *p, const float *F, const float *t, int64_t m, float *loss, float *grads,
                              void *stream) {
    if (!mlp_ok(p)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    if (m < 1 || m > (1 << 20)) return fail(SUCO_E_INVAL, "m must be in [1, 2^20]");
    if (!F || !t || !grads) return fail(SUCO_E_INVAL, "F, t and grads must not be NULL");
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(p->mu_lock);
    DeviceGuard dg(p->device);
    int rc = ensure_rows(p, (int)m);
    if (rc) return rc;
    const TrainRows a = rows_args(p, F, t, nullptr, (int)m, 0);
    HIPCHECK(grads_pass(p, a, st));
    HIPCHECK(hipMemcpyAsync(grads, p->g, sizeof(float) * p->np, hipMemcpyDeviceToDevice, st));
    if (loss) HIPCHECK(hipMemcpyAsync(loss, p->loss, sizeof(float), hipMemcpyDeviceToDevice, st));
    return SUCO_OK;
}

int suco_mlp_train_epoch(suco_mlp *p, const float *F, const float *t, int64_t m, int32_t batch, float lr,
                         const int32_t *order, float *mean_loss, void *stream) {
    if (!mlp_ok(p)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    if (m < 1 || batch < 1 || batch > 65536) return fail(SUCO_E_INVAL, "m >= 1 and batch in [1, 65536]");
    if (!(lr > 0.f)) return fail(SUCO_E_INVAL, "lr must be positive");
    if (!F || !t) return fail(SUCO_E_INVAL, "F and t must not be NULL");
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(p->mu_lock);
    DeviceGuard dg(p->device);
    int rc = ensure_rows(p, batch);
    if (rc) return rc;
    double lsum = 0.0;
    for (int64_t r0 = 0; r0 < m; r0 += batch) {
        const int mb = (int)std::min<int64_t>(batch, m - r0);
        const TrainRows a = rows_args(p, F, t, order, mb, r0);
        HIPCHECK(grads_pass(p, a, st));
        ++p->steps;
        const float c1 = 1.0f - std::pow(0.9f, (float)p->steps), c2 = 1.0f - std::pow(0.999f, (float)p->steps);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((p->np + 255) / 256)), dim3(256), 0, st, p->w, p->g, p->m1,
                           p->m2, p->np, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
        HIPCHECK(hipGetLastError());
        if (mean_loss) {
            float l = 0.f;
            HIPCHECK(hipMemcpyAsync(&l, p->loss, sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
            lsum += (double)l * mb;
        }
    }
    p->wb_valid = false;
    if (mean_loss) *mean_loss = (float)(lsum / (double)m);
    return SUCO_OK;
}

int suco_mlp_predict(suco_mlp *p, const float *F, int64_t m, float scale, float alpha_min, float alpha_max,
                     float *y, float *alpha, void *stream) {
    if (!mlp_ok(p)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    if (m < 0 || (m > 0 && !F)) return fail(SUCO_E_INVAL, "F must not be NULL");
    if (!(alpha_min > 0.f && alpha_min <= alpha_max && alpha_max <= 1.f))
        return fail(SUCO_E_INVAL, "need 0 < alpha_min <= alpha_max <= 1");
    if (m == 0) return SUCO_OK;
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(p->mu_lock);
    DeviceGuard dg(p->device);
    int rc = refresh_bf16(p, st);
    if (rc) return rc;
    InferPass ip{};
    ip.w = p->view(p->wb);
    ip.F = F; ip.m = (int)m; ip.scale = scale; ip.amin = alpha_min; ip.amax = alpha_max; ip.y = y; ip.alpha = alpha;
    HIPCHECK(launch(plan_mlp_infer((int)m), &ip, st));
    return SUCO_OK;
}

int suco_query_features(const suco_index *ix, const float *Q, int64_t nq, float *F, void *stream) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (ix->metric) return fail(SUCO_E_UNSUPPORTED, "the learned budget's features are Euclidean (not SUCO_BUILD_L1)");
    if (nq < 0 || (nq > 0 && (!Q || !F))) return fail(SUCO_E_INVAL, "Q and F must not be NULL");
    if (nq == 0) return SUCO_OK;
    DeviceGuard dg(ix->device);
    for (int64_t q0 = 0; q0 < nq; q0 += 65536) {
        const int cn = (int)std::min<int64_t>(65536, nq - q0);
        FeatPass fp{};
        fp.ix = ix->view(); fp.Q = Q + q0 * ix->d; fp.nq = cn; fp.F = F + q0 * (2 * ix->ns + 1);
        HIPCHECK(launch(plan_features(fp.ix, cn), &fp, (hipStream_t)stream));
    }
    return SUCO_OK;
}

int suco_mlp_free(suco_mlp *p) {
    if (!p) return SUCO_OK;
    if (!mlp_ok(p)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    {
        DeviceGuard dg(p->device);
        (void)hipDeviceSynchronize();
        std::lock_guard<std::mutex> lock(p->mu_lock);
        p->release();
    }
    delete p;
    return SUCO_OK;
}

}  // extern "C"

// ------------------------------------------------------ learned query --
extern "C" int suco_query_learned(const suco_index *ix, suco_mlp *p, const float *Q, int64_t nq, int32_t k,
                                  double beta, float scale, float alpha_min, float alpha_max, int32_t *ids,
                                  float *dists, float *alpha_used, void *stream) {
    if (!index_ok(ix)) return fail(SUCO_E_STATE, "invalid or freed index handle");
    if (!mlp_ok(p)) return fail(SUCO_E_STATE, "invalid or freed model handle");
    if (ix->metric) return fail(SUCO_E_UNSUPPORTED, "the learned budget's features are Euclidean (not SUCO_BUILD_L1)");
    if (p->n_in != 2 * ix->ns + 1) return fail(SUCO_E_INVAL, "the model's n_in must be 2*n_s + 1");
    if (!(scale > 0.f)) return fail(SUCO_E_INVAL, "scale must be positive");
    if (!(alpha_min > 0.f && alpha_min <= alpha_max && alpha_max <= 1.f))
        return fail(SUCO_E_INVAL, "need 0 < alpha_min <= alpha_max <= 1");
    if (nq < 0 || (nq > 0 && (!Q || !ids || !dists))) return fail(SUCO_E_INVAL, "Q, ids and dists must not be NULL");
    if (k < 1 || k > ix->n) return fail(SUCO_E_INVAL, "k must be in [1, n]");
    if (k > kMaxK) return fail(SUCO_E_UNSUPPORTED, "the kernels take k <= 64");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SUCO_E_INVAL, "beta must be in (0, 1]");
    if (nq == 0) return SUCO_OK;
    hipStream_t st = (hipStream_t)stream;
    // features and alphas are staged in buffers owned by the index (on its device),
    // serialised by the index's staging mutex
    suco_index *mix = const_cast<suco_index *>(ix);
    suco_index::LearnedStage &S = mix->lstage;
    std::lock_guard<std::mutex> lock(S.mu);
    DeviceGuard dg(ix->device);
    if (!S.done) HIPCHECK(hipEventCreateWithFlags(&S.done, hipEventDisableTiming));
    if (nq * p->n_in > S.cap_f || nq > S.cap_a) {
        if (S.pending) HIPCHECK(hipEventSynchronize(S.done));
        if (S.F) (void)hipFree(S.F);
        if (S.alpha) (void)hipFree(S.alpha);
        S.F = nullptr; S.alpha = nullptr; S.cap_f = 0; S.cap_a = 0;
        int rc;
        if ((rc = dev_alloc(&S.F, (size_t)nq * p->n_in)) || (rc = dev_alloc(&S.alpha, (size_t)nq))) {
            if (S.F) (void)hipFree(S.F);
            S.F = nullptr;
            return rc;
        }
        S.cap_f = nq * p->n_in;
        S.cap_a = nq;
    }
    if (S.pending) HIPCHECK(hipStreamWaitEvent(st, S.done, 0));
    {
        std::lock_guard<std::mutex> mlock(p->mu_lock);
        int rc = refresh_bf16(p, st);
        if (rc) return rc;
        // features and inference in one kernel per 65,536 queries
        for (int64_t q0 = 0; q0 < nq; q0 += 65536) {
            const int cn = (int)std::min<int64_t>(65536, nq - q0);
            FeatPass fp{};
            fp.ix = ix->view(); fp.Q = Q + q0 * ix->d; fp.nq = cn;
            InferPass ip{};
            ip.w = p->view(p->wb); ip.m = cn; ip.scale = scale; ip.amin = alpha_min; ip.amax = alpha_max;
            ip.alpha = S.alpha + q0;
            const Launch L = plan_learned_alpha(fp.ix, half_wmax(ix), cn);
            void *args[] = {&fp, &ip};
            HIPCHECK(hipLaunchKernel(L.func, L.grid, L.block, args, L.lds, st));
        }
    }
    int rc = suco_query_alpha(ix, Q, nq, k, S.alpha, beta, ids, dists, stream);
    if (rc) return rc;
    if (alpha_used) HIPCHECK(hipMemcpyAsync(alpha_used, S.alpha, sizeof(float) * nq, hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipEventRecord(S.done, st));
    S.pending = true;
    return SUCO_OK;
}
