// Plain FP32 direct sum on the vector ALUs (the comparison path).
//
//     W[i][k] = sum_{m=-M_i}^{M_i} t_i[m] * x~[k*hop + m]     (Eq. (1), Sec. II-A/II-B)
//
// Work-group tile: 256 consecutive frames (one per thread, 64 per wave) x one
// group of 16 sorted scales, which every wave runs: sixteen FMAs per signal
// value read from LDS and per scalar load of a tap row, and all four waves
// walk the same tap range, so none idles through a wider group's chunks (a
// work-group of four groups, one per wave, kept the narrow-scale waves
// waiting at every chunk of its widest group).  The taps of the group are
// wave-uniform and come through the scalar cache; the signal is staged in LDS
// in chunks of kDirectChunk taps as X[c][f] = x~[(k0+f)*hop + m_c + c] (row
// stride 257 floats, so the per-lane reads are bank-conflict free for every
// hop).  Each coefficient is one FP32 FMA chain in ascending tap order.
#include "cwt_internal.h"

namespace cwth {

constexpr int kRowStride = kDirectFrames + 1;

// One tile: kDirectFrames frames of clip c starting at frame tile `tile`, scale group g.
__device__ __forceinline__ void direct_tile(const DirectArgs& a, const ClipArg& c, int tile, int g, float* X) {
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)tile * kDirectFrames;
    const int P = a.groups[g].P;
    const float* __restrict__ taps = a.taps + a.groups[g].off;

    float acc[kDirectRows];
#pragma unroll
    for (int r = 0; r < kDirectRows; ++r) acc[r] = 0.0f;

    // thread t stages frame t: taps c = 0 .. kDirectChunk-1 of the chunk are
    // kDirectChunk consecutive samples from (k0 + t) * hop + mc
    const int64_t j0 = (k0 + t) * c.hop;
    for (int mc = -P; mc <= P; mc += kDirectChunk) {
        __syncthreads();
        const int64_t jb = j0 + mc;
#pragma unroll 8
        for (int cc = 0; cc < kDirectChunk; ++cc) {
            const int64_t j = jb + cc;
            X[cc * kRowStride + t] = (j >= 0 && j < c.len) ? c.x[j] : 0.0f;
        }
        __syncthreads();
        const int m_hi = min(mc + kDirectChunk - 1, P);
#pragma unroll 4
        for (int m = mc; m <= m_hi; ++m) {
            const float xv = X[(m - mc) * kRowStride + t];
            const float* tp = taps + (int64_t)(m + P) * kDirectRows;
#pragma unroll
            for (int r = 0; r < kDirectRows; ++r) acc[r] = fmaf(tp[r], xv, acc[r]);
        }
    }
    const int64_t k = k0 + t;
    if (k >= c.K) return;
#pragma unroll
    for (int r = 0; r < kDirectRows; ++r) {
        const int row = a.groups[g].rows[r];
        if (row < 0) continue;
        float v = a.signed_out ? acc[r] : fabsf(acc[r]);
        __builtin_nontemporal_store(v, c.out + (int64_t)row * c.K + k);
    }
}

// Work-groups: frame tiles x scale groups, the widest group's tiles first
// (groups are stored narrowest first), so the grid drains evenly; dealt to
// the XCDs round-robin, every XCD gets its share of wide and narrow groups.
__global__ __launch_bounds__(256) void k_direct(DirectArgs a) {
    __shared__ float X[kDirectChunk * kRowStride];
    const int id = blockIdx.x;
    const int ntile = a.clip.ntile;
    const int g = a.ngroups - 1 - id / ntile, tile = id - (a.ngroups - 1 - g) * ntile;
    direct_tile(a, a.clip, tile, g, X);
}

// Batch: a flat grid over the tiles of every clip; clip c owns tiles
// [prefix[c], prefix[c+1]).
__global__ __launch_bounds__(256) void k_direct_batch(DirectArgs a, const ClipArg* __restrict__ clips,
                                                      const int32_t* __restrict__ prefix, int nclips) {
    __shared__ float X[kDirectChunk * kRowStride];
    const int t = blockIdx.x;
    int lo = 0, hi = nclips - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int local = t - prefix[lo];
    const ClipArg c = clips[lo];
    const int g = a.ngroups - 1 - local / c.ntile, tile = local - (a.ngroups - 1 - g) * c.ntile;
    direct_tile(a, c, tile, g, X);
}

hipError_t launch_direct(const DirectArgs& a, hipStream_t s) {
    const int64_t grid = (int64_t)a.clip.ntile * a.ngroups;
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
