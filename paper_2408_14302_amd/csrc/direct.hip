// Plain FP32 direct sum on the vector ALUs (the comparison path).
//
//     W[i][k] = sum_{m=-M_i}^{M_i} t_i[m] * x~[k*hop + m]     (Eq. (1), Sec. II-A/II-B)
//
// Each coefficient is one FP32 FMA chain in ascending tap order, whatever the
// work-group layout, so both layouts give the same bits.  The taps of a
// wave's group are wave-uniform and come through the scalar cache: sixteen
// FMAs per signal value read from LDS and per scalar load of a tap row.  The
// signal is staged in LDS chunk by chunk as X[c][f] = x~[(k0+f)*hop + m_c + c]
// with a row stride of frames + 1 floats, so the per-lane reads and the
// staging writes are bank-conflict free for every hop; a chunk's loads are
// spread so that consecutive threads read consecutive samples of one frame.
//
// Layout 1 (hops below 256): 256 consecutive frames (one per thread, 64 per
// wave) x one group of 16 sorted scales that every wave runs, chunks of 32
// taps.
// All four waves walk the same tap range, so none idles through a wider
// group's chunks, and neighbouring frames share most of their samples, so
// staging is cheap.
//
// Layout 4 (hops from 256 on): 64 consecutive frames (one per lane) x four
// groups, one per wave, chunks of 128 taps.  Frames far apart share few samples;
// each staged value now feeds 64 scales instead of 16, which cuts the L2
// traffic of the staging four-fold where it, not the FMAs, is the cost (a
// 256-clip batch at hop 512: 1.7 against 3.4 ms; equal at hop 128, and
// layout 1 up to 2.3x faster below).
#include "cwt_internal.h"

namespace cwth {

constexpr int kRowStride = kDirectFrames + 1;
constexpr int kWideStride = kDirectWideFrames + 1;
constexpr int kXFloats = kDirectChunk * kRowStride > kDirectWideChunk * kWideStride ? kDirectChunk * kRowStride
                                                                                    : kDirectWideChunk * kWideStride;

// Chunk [mc, mc + CH) of frames k0 .. k0 + F - 1 into X (row stride F + 1):
// CH consecutive threads stage one frame's CH consecutive samples.
template <int F, int CH>
__device__ __forceinline__ void stage_chunk(const ClipArg& c, int64_t k0, int mc, float* X) {
    static_assert((F * CH) % 256 == 0 && 256 % CH == 0, "chunk must tile the work-group");
    constexpr int FPP = 256 / CH;   // frames per pass
    const int cc = threadIdx.x % CH, f0 = threadIdx.x / CH;
    const int64_t j0 = (k0 + f0) * c.hop + mc + cc;
    const int64_t js = (int64_t)FPP * c.hop;
#pragma unroll 8
    for (int i = 0; i < F / FPP; ++i) {
        const int64_t j = j0 + i * js;
        X[cc * (F + 1) + f0 + FPP * i] = (j >= 0 && j < c.len) ? c.x[j] : 0.0f;
    }
}

// The same chunk at hop 1 (layout 1), thread t staging frame t: the
// consecutive frames' samples then arrive as consecutive addresses across
// the wave with no index arithmetic per sample (10% faster there; at larger
// hops the lanes' addresses spread and stage_chunk wins from hop 4 on).
__device__ __forceinline__ void stage_frames_hop1(const ClipArg& c, int64_t k0, int mc, float* X) {
    const int64_t jb = k0 + threadIdx.x + mc;
#pragma unroll 8
    for (int cc = 0; cc < kDirectChunk; ++cc) {
        const int64_t j = jb + cc;
        X[cc * kRowStride + threadIdx.x] = (j >= 0 && j < c.len) ? c.x[j] : 0.0f;
    }
}

__device__ __forceinline__ void store_group(const DirectArgs& a, const ClipArg& c, int g, int64_t k,
                                            const float (&acc)[kDirectRows]) {
    if (k >= c.K) return;
#pragma unroll
    for (int r = 0; r < kDirectRows; ++r) {
        const int row = a.groups[g].rows[r];
        if (row < 0) continue;
        float v = a.signed_out ? acc[r] : fabsf(acc[r]);
        __builtin_nontemporal_store(v, c.out + (int64_t)row * c.K + k);
    }
}

// Layout 1: frames k0 .. k0+255 of clip c (tile `tile`), scale group g.
__device__ __forceinline__ void direct_tile(const DirectArgs& a, const ClipArg& c, int tile, int g, float* X) {
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)tile * kDirectFrames;
    const int P = a.groups[g].P;
    const float* __restrict__ taps = a.taps + a.groups[g].off;
    float acc[kDirectRows];
#pragma unroll
    for (int r = 0; r < kDirectRows; ++r) acc[r] = 0.0f;
    for (int mc = -P; mc <= P; mc += kDirectChunk) {
        __syncthreads();
        if (c.hop == 1)
            stage_frames_hop1(c, k0, mc, X);
        else
            stage_chunk<kDirectFrames, kDirectChunk>(c, k0, mc, X);
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
    store_group(a, c, g, k0 + t, acc);
}

// Layout 4: frames k0 .. k0+63 of clip c (tile `tile`), groups 4 sg .. 4 sg+3
// (wave w runs group 4 sg + w; the chunks span the widest of them).
__device__ __forceinline__ void direct_tile_wide(const DirectArgs& a, const ClipArg& c, int tile, int sg,
                                                 float* X) {
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t k0 = (int64_t)tile * kDirectWideFrames;
    const int g = sg * kDirectGroups + w;
    const bool active = g < a.ngroups;
    const int P = active ? a.groups[g].P : 0;
    int Pwg = 0;
    for (int j = 0; j < kDirectGroups; ++j)
        if (sg * kDirectGroups + j < a.ngroups) Pwg = max(Pwg, a.groups[sg * kDirectGroups + j].P);
    const float* __restrict__ taps = a.taps + (active ? a.groups[g].off : 0);
    float acc[kDirectRows];
#pragma unroll
    for (int r = 0; r < kDirectRows; ++r) acc[r] = 0.0f;
    for (int mc = -Pwg; mc <= Pwg; mc += kDirectWideChunk) {
        __syncthreads();
        stage_chunk<kDirectWideFrames, kDirectWideChunk>(c, k0, mc, X);
        __syncthreads();
        if (!active) continue;
        const int m_lo = max(mc, -P), m_hi = min(mc + kDirectWideChunk - 1, P);
#pragma unroll 4
        for (int m = m_lo; m <= m_hi; ++m) {
            const float xv = X[(m - mc) * kWideStride + lane];
            const float* tp = taps + (int64_t)(m + P) * kDirectRows;
#pragma unroll
            for (int r = 0; r < kDirectRows; ++r) acc[r] = fmaf(tp[r], xv, acc[r]);
        }
    }
    if (active) store_group(a, c, g, k0 + lane, acc);
}

// Work-group `local` of clip c: frame tiles x groups (layout 1) or x groups of
// four (layout 4), the widest first (groups are stored narrowest first).
__device__ __forceinline__ void direct_unit(const DirectArgs& a, const ClipArg& c, int local, float* X) {
    if (c.ws == kDirectGroups) {
        const int nsg = (a.ngroups + kDirectGroups - 1) / kDirectGroups;
        const int sg = nsg - 1 - local / c.ntile, tile = local - (nsg - 1 - sg) * c.ntile;
        direct_tile_wide(a, c, tile, sg, X);
    } else {
        const int g = a.ngroups - 1 - local / c.ntile, tile = local - (a.ngroups - 1 - g) * c.ntile;
        direct_tile(a, c, tile, g, X);
    }
}

__global__ __launch_bounds__(256) void k_direct(DirectArgs a) {
    __shared__ float X[kXFloats];
    direct_unit(a, a.clip, blockIdx.x, X);
}

// Batch: a flat grid over the work-groups of every clip; clip c owns
// work-groups [prefix[c], prefix[c+1]).
__global__ __launch_bounds__(256) void k_direct_batch(DirectArgs a, const ClipArg* __restrict__ clips,
                                                      const int32_t* __restrict__ prefix, int nclips) {
    __shared__ float X[kXFloats];
    const int t = blockIdx.x;
    int lo = 0, hi = nclips - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    direct_unit(a, clips[lo], t - prefix[lo], X);
}

hipError_t launch_direct(const DirectArgs& a, hipStream_t s) {
    const int64_t units = a.clip.ws == kDirectGroups ? (a.ngroups + kDirectGroups - 1) / kDirectGroups : a.ngroups;
    const int64_t grid = (int64_t)a.clip.ntile * units;
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
