// Decimation for the decimate-then-transform reading of the paper's workflow
// (Sec. III-B: the signal is re-sampled, then transformed):
//
//     y[n] = sum_{j=0}^{L-1} h[j] * x~[n*factor + j - (L-1)/2],   n = 0 .. ceil(len/factor) - 1
//
// x~ = x inside [0, len), 0 outside; L odd (h[0] = 1, L = 1 is plain
// decimation).  Short filters: one output per lane, an FP32 FMA chain in
// ascending j, the filter wave-uniform (scalar loads), the input through the
// caches (each sample is used by about L / factor outputs).  Long filters
// (L >= 64, the anti-alias filters of large factors, where outputs are few):
// one output per wave, lane l summing taps j = l, l + 64, .. in ascending
// order (coalesced input reads), then a fixed butterfly across the lanes.
#include "cwt_internal.h"

namespace cwth {

__global__ __launch_bounds__(256) void k_decimate(const float* __restrict__ x, int64_t len, int factor,
                                                  const float* __restrict__ h, int L, float* __restrict__ y,
                                                  int64_t ny) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= ny) return;
    const int64_t lo = n * factor - (L - 1) / 2;      // input index of h[0]
    const int j0 = lo < 0 ? (int)(-lo) : 0;
    const int64_t rem = len - lo;
    const int j1 = rem < L ? (int)rem : L;
    float acc = 0.0f;
    for (int j = j0; j < j1; ++j) acc = fmaf(h[j], x[lo + j], acc);
    y[n] = acc;
}

__global__ __launch_bounds__(256) void k_decimate_wave(const float* __restrict__ x, int64_t len, int factor,
                                                       const float* __restrict__ h, int L, float* __restrict__ y,
                                                       int64_t ny) {
    const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (n >= ny) return;                                  // wave-uniform
    const int64_t lo = n * factor - (L - 1) / 2;
    float acc = 0.0f;
    for (int j = lane; j < L; j += 64) {
        const int64_t i = lo + j;
        if (i >= 0 && i < len) acc = fmaf(h[j], x[i], acc);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) y[n] = acc;
}

hipError_t launch_decimate(const float* x, int64_t len, int factor, const float* h, int L, float* y, int64_t ny,
                           hipStream_t s) {
    if (ny <= 0) return hipSuccess;
    if (L >= 64) {
        const int64_t grid = (ny + 3) / 4;
        if (grid > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_decimate_wave, dim3((unsigned)grid), dim3(256), 0, s, x, len, factor, h, L, y, ny);
    } else {
        const int64_t grid = (ny + 255) / 256;
        if (grid > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_decimate, dim3((unsigned)grid), dim3(256), 0, s, x, len, factor, h, L, y, ny);
    }
    return hipGetLastError();
}

}  // namespace cwth
