// Plain FP32 direct sum on the vector ALUs (the comparison path).
//
//     W[i][k] = sum_{m=-M_i}^{M_i} t_i[m] * x~[k*hop + m]     (Eq. (1), Sec. II-A/II-B)
//
// Work-group tile: 64 consecutive frames (one per lane) x 64 sorted scales (four
// waves, sixteen scales each: sixteen FMAs per signal value read from LDS and
// per scalar load of a tap row).  The taps of a wave's scales are wave-uniform
// and come through the scalar cache; the signal is staged in LDS in chunks of
// kDirectChunk taps as X[c][f] = x~[(k0+f)*hop + m_c + c] (row stride 65 floats,
// so both the staging writes and the per-lane reads are bank-conflict free for
// every hop).  Each coefficient is one FP32 FMA chain in ascending tap order.
#include "cwt_internal.h"

namespace cwth {

constexpr int kRowStride = kDirectFrames + 1;

__device__ __forceinline__ int xcd_remap_d(int id, int n) {
    int q = n >> 3, r = n & 7;
    int xcd = id & 7, slot = id >> 3;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// One tile: 64 frames of clip c starting at frame tile `tile`, scale super-group sg.
__device__ __forceinline__ void direct_tile(const DirectArgs& a, const ClipArg& c, int tile, int sg,
                                            float* X) {
    const int gpw = kDirectWaves;                                   // groups per work-group
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t k0 = (int64_t)tile * kDirectFrames;
    const int gi = sg * gpw + w;
    const bool active = gi < a.ngroups;

    int P = 0;
    int64_t off = 0;
    if (active) {
        P = a.groups[gi].P;
        off = a.groups[gi].off;
    }
    int Pwg = 0;                                                     // widest group in the work-group
    for (int j = 0; j < gpw; ++j) {
        int gj = sg * gpw + j;
        if (gj < a.ngroups) Pwg = max(Pwg, a.groups[gj].P);
    }
    const float* __restrict__ taps = a.taps + off;

    float acc[kDirectRows];
#pragma unroll
    for (int r = 0; r < kDirectRows; ++r) acc[r] = 0.0f;

    for (int mc = -Pwg; mc <= Pwg; mc += kDirectChunk) {
        __syncthreads();
        for (int q = threadIdx.x; q < kDirectFrames * kDirectChunk; q += 256) {
            int f = q / kDirectChunk, cc = q - f * kDirectChunk;
            int64_t j = (k0 + f) * c.hop + mc + cc;
            X[cc * kRowStride + f] = (j >= 0 && j < c.len) ? c.x[j] : 0.0f;
        }
        __syncthreads();
        if (!active) continue;
        const int m_lo = max(mc, -P), m_hi = min(mc + kDirectChunk - 1, P);
#pragma unroll 4
        for (int m = m_lo; m <= m_hi; ++m) {
            const float xv = X[(m - mc) * kRowStride + lane];
            const float* tp = taps + (int64_t)(m + P) * kDirectRows;
#pragma unroll
            for (int r = 0; r < kDirectRows; ++r) acc[r] = fmaf(tp[r], xv, acc[r]);
        }
    }
    if (!active) return;
    const int64_t k = k0 + lane;
    if (k >= c.K) return;
#pragma unroll
    for (int r = 0; r < kDirectRows; ++r) {
        const int row = a.groups[gi].rows[r];
        if (row < 0) continue;
        float v = a.signed_out ? acc[r] : fabsf(acc[r]);
        __builtin_nontemporal_store(v, c.out + (int64_t)row * c.K + k);
    }
}


__global__ __launch_bounds__(256) void k_direct(DirectArgs a) {
    __shared__ float X[kDirectChunk * kRowStride];
    const int nsg = (a.ngroups + kDirectWaves - 1) / kDirectWaves;
    int id = blockIdx.x;
    if (a.xcd_remap) id = xcd_remap_d(id, gridDim.x);
    const int tile = id / nsg, sg = id - tile * nsg;
    direct_tile(a, a.clip, tile, sg, X);
}

// Batch: a flat grid over the tiles of every clip; clip c owns tiles
// [prefix[c], prefix[c+1]).
__global__ __launch_bounds__(256) void k_direct_batch(DirectArgs a, const ClipArg* __restrict__ clips,
                                                      const int32_t* __restrict__ prefix, int nclips) {
    __shared__ float X[kDirectChunk * kRowStride];
    const int nsg = (a.ngroups + kDirectWaves - 1) / kDirectWaves;
    const int t = blockIdx.x;
    int lo = 0, hi = nclips - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int local = t - prefix[lo];
    const int tile = local / nsg, sg = local - tile * nsg;
    const ClipArg c = clips[lo];
    direct_tile(a, c, tile, sg, X);
}

hipError_t launch_direct(const DirectArgs& a, hipStream_t s) {
    const int nsg = (a.ngroups + kDirectWaves - 1) / kDirectWaves;
    const int64_t ntile = a.clip.ntile;
    const int64_t grid = ntile * nsg;
    if (grid <= 0) return hipSuccess;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_direct, dim3((unsigned)grid), dim3(256), 0, s, a);
    return hipGetLastError();
}


hipError_t launch_direct_batch(const DirectArgs& a, const ClipArg* d_clips, const int32_t* d_prefix,
                               int nclips, int total_tiles, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_direct_batch, dim3((unsigned)total_tiles), dim3(256), 0, s, a, d_clips,
                       d_prefix, nclips);
    return hipGetLastError();
}

}  // namespace cwth
