// Scalogram to image: the step after the transform, where the scalogram
// becomes a CNN input image (Sec. II-A with Fig. 1, Sec. III-B).
//
//     D[i][k]   = 20 log10(max(|W[i][k]|, amin))
//     image[r][c] = (B(r, c) - min D) / (max D - min D)     (0 if max D == min D)
//
// B is D resampled bilinearly to height x width with half-pixel centres (source
// row (r + 0.5) * n_scales / height - 0.5, clamped below at 0; likewise for
// columns); min and max are taken over the full-resolution D.  log10 is
// monotonic, so they are the dB of the extreme magnitudes.
//
// Pass 1 (k_minmax): each work-group reduces a grid-strided share of |W| to
// (min, max) and writes it to the workspace; min and max are exact, so the
// result does not depend on the split.  Pass 2 (k_image): every work-group
// folds the partials, then each thread makes one pixel from four samples.
#include "cwt_internal.h"

namespace cwth {

__device__ __forceinline__ float wave_min_f(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// (min, max) of two per-wave values across the 4 waves of the work-group.
__device__ __forceinline__ void block_minmax(float& mn, float& mx, float* red) {
    mn = wave_min_f(mn);
    mx = wave_max_f(mx);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w] = mn;
        red[4 + w] = mx;
    }
    __syncthreads();
    mn = fminf(fminf(red[0], red[1]), fminf(red[2], red[3]));
    mx = fmaxf(fmaxf(red[4], red[5]), fmaxf(red[6], red[7]));
}

__global__ __launch_bounds__(256) void k_minmax(const float* __restrict__ w, int64_t total, float2* __restrict__ part) {
    __shared__ float red[8];
    float mn = INFINITY, mx = 0.0f;
    const int64_t stride = (int64_t)gridDim.x * 256 * 4;
    const bool al16 = ((uintptr_t)w & 15) == 0;
    for (int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4; i < total; i += stride) {
        if (al16 && i + 4 <= total) {
            const float4 v = *(const float4*)(w + i);
            mn = fminf(mn, fminf(fminf(fabsf(v.x), fabsf(v.y)), fminf(fabsf(v.z), fabsf(v.w))));
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        } else {
            for (int64_t j = i; j < i + 4 && j < total; ++j) {
                mn = fminf(mn, fabsf(w[j]));
                mx = fmaxf(mx, fabsf(w[j]));
            }
        }
    }
    block_minmax(mn, mx, red);
    if (threadIdx.x == 0) part[blockIdx.x] = make_float2(mn, mx);
}

__device__ __forceinline__ float to_db(float v, float amin) { return 20.0f * log10f(fmaxf(fabsf(v), amin)); }

// One axis of the resampling: source indices i0, i1 and the weight of i1,
// formed in double (frame counts exceed 2^24).
__device__ __forceinline__ void axis(int64_t dst, int64_t n_in, int64_t n_out, int64_t& i0, int64_t& i1,
                                     float& lam) {
    double src = ((double)dst + 0.5) * ((double)n_in / (double)n_out) - 0.5;
    src = src < 0.0 ? 0.0 : src;
    i0 = (int64_t)floor(src);
    if (i0 > n_in - 1) i0 = n_in - 1;
    i1 = i0 < n_in - 1 ? i0 + 1 : i0;
    lam = (float)(src - (double)i0);
}

__global__ __launch_bounds__(256) void k_image(const float* __restrict__ w, int n_scales, int64_t n_frames,
                                               float amin, const float2* __restrict__ part, int nparts,
                                               float* __restrict__ image, int height, int width) {
    __shared__ float red[8];
    float mn = INFINITY, mx = 0.0f;
    for (int i = threadIdx.x; i < nparts; i += 256) {
        const float2 p = part[i];
        mn = fminf(mn, p.x);
        mx = fmaxf(mx, p.y);
    }
    block_minmax(mn, mx, red);
    const float dlo = to_db(mn, amin), dhi = to_db(mx, amin);
    const float inv = dhi > dlo ? 1.0f / (dhi - dlo) : 0.0f;

    const int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= (int64_t)height * width) return;
    const int64_t r = pix / width, c = pix - r * width;
    int64_t r0, r1, c0, c1;
    float wr, wc;
    axis(r, n_scales, height, r0, r1, wr);
    axis(c, n_frames, width, c0, c1, wc);
    const float* row0 = w + r0 * n_frames;
    const float* row1 = w + r1 * n_frames;
    const float top = to_db(row0[c0], amin) * (1.0f - wc) + to_db(row0[c1], amin) * wc;
    const float bot = to_db(row1[c0], amin) * (1.0f - wc) + to_db(row1[c1], amin) * wc;
    image[pix] = (top * (1.0f - wr) + bot * wr - dlo) * inv;
}

constexpr int kMinmaxParts = 1024;

int64_t image_workspace_bytes() { return (int64_t)kMinmaxParts * sizeof(float2); }

hipError_t launch_image(const float* w, int n_scales, int64_t n_frames, float amin, float* image, int height,
                        int width, void* workspace, hipStream_t s) {
    const int64_t total = (int64_t)n_scales * n_frames;
    int64_t nb = (total + 256 * 16 - 1) / (256 * 16);      // at least 16 elements per thread
    nb = nb < 1 ? 1 : (nb > kMinmaxParts ? kMinmaxParts : nb);
    float2* part = (float2*)workspace;
    hipLaunchKernelGGL(k_minmax, dim3((unsigned)nb), dim3(256), 0, s, w, total, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t pixels = (int64_t)height * width;
    const int64_t grid = (pixels + 255) / 256;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_image, dim3((unsigned)grid), dim3(256), 0, s, w, n_scales, n_frames, amin, part, (int)nb,
                       image, height, width);
    return hipGetLastError();
}

}  // namespace cwth
