// Wave-level helpers shared by the gfx950 kernels (64-lane wavefronts).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "suco_impl.h"

namespace suco {

// One term of a distance sum in FP32: t*t (squared Euclidean, one FMA) or |t|
// (Manhattan, SuCo-L1).
__device__ __forceinline__ float dist_acc(float s, float t, int metric) {
    return metric ? s + fabsf(t) : fmaf(t, t, s);
}

// Inclusive prefix sum over the 64 lanes with DPP moves (row shifts within
// 16-lane rows, then the row broadcasts of lanes 15 and 31); lanes a move
// does not reach add zero.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Minimum over the 64 lanes, the same in every lane (all lanes active): the
// same DPP steps as the scan, lanes a move does not reach keep their value.
__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x111, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x112, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x114, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x118, 0xf, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x142, 0xa, 0xf, false));
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x143, 0xc, 0xf, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
}

// Set bits of a 64-bit wave mask in the lanes below this one (v_mbcnt).
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Sum over the 64 lanes, the same in every lane (all lanes active).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), kWave - 1);
}

// Sum over aligned groups of G lanes (G in {1, 2, 4, 8, 16}) with DPP moves
// (quad permutations, then the half-row and row mirrors); every lane of a
// group ends with the group's sum.
__device__ __forceinline__ uint32_t group_sum(uint32_t v, int G) {
    if (G >= 2) v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xb1, 0xf, 0xf, false);    // quad_perm 1,0,3,2
    if (G >= 4) v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4e, 0xf, 0xf, false);    // quad_perm 2,3,0,1
    if (G >= 8) v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xf, 0xf, false);   // row_half_mirror
    if (G >= 16) v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xf, 0xf, false);  // row_mirror
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

// A wave keeps its k best keys sorted ascending in lanes 0..k-1 (lanes >= k
// hold ~0); insert one key, given to every lane, keeping the k smallest.
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

// Sum over the block; every thread gets the total.  Like the scans below, it
// is called by every thread of the block.
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
    const uint32_t x = wave_incl_scan(v);
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

// Two exclusive prefixes at once (one pass of barriers); *ta, *tb get the sums.
template <int NT>
__device__ __forceinline__ void block_excl_scan2(uint32_t va, uint32_t vb, uint32_t *red2, uint32_t *ea,
                                                 uint32_t *eb, uint32_t *ta, uint32_t *tb) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t xa = wave_incl_scan(va), xb = wave_incl_scan(vb);
    __syncthreads();
    if (lane == kWave - 1) { red2[2 * w] = xa; red2[2 * w + 1] = xb; }
    __syncthreads();
    uint32_t ba = 0, bb = 0, sa = 0, sb = 0;
#pragma unroll
    for (int j = 0; j < NT / kWave; ++j) {
        const uint32_t ra = red2[2 * j], rb = red2[2 * j + 1];
        ba += (j < w) ? ra : 0u;
        bb += (j < w) ? rb : 0u;
        sa += ra;
        sb += rb;
    }
    *ea = ba + xa - va;
    *eb = bb + xb - vb;
    *ta = sa;
    *tb = sb;
}

}  // namespace suco
