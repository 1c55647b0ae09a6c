// DWT scalogram (Sec. II-A, Fig. 1c): the dyadic transform by a two-channel
// filter bank with down-sampling by two, level after level, its detail
// coefficients spread back over the time axis to form a scale-by-time matrix.
//
//   a_j[n] = sum_k h[k] a_{j-1}[c(2n + k)],  d_j[n] = sum_k g[k] a_{j-1}[c(2n + k)]
//   c(i) = min(i mod P, len_{j-1} - 1),  P = len_{j-1} rounded up to even
//   S[j-1][t] = |d_j[t >> j]|,  t < len,  j = 1 .. J
//
// a_0 = x, len_j = ceil(len_{j-1} / 2).  The index map c is periodic
// extension, with an odd level first made even by repeating its last sample.
//
// Three kernels.  Levels whose input is longer than the LDS tail: one output
// pair per lane, input through the caches (consecutive lanes read
// overlapping windows).  The remaining short levels: one workgroup per clip
// keeps the level in LDS and runs every remaining level behind workgroup
// barriers (one launch instead of one per level).  Finally the expansion
// writes the J x len matrix, a float4 per lane per level: this is the part
// that moves most bytes (J floats out per input sample), so it is the one
// that is HBM bound.  Every output pair is the same FP32 FMA chain in
// ascending k, wherever it is computed, so results do not depend on which
// kernel produced a level.
#include "cwt_internal.h"

namespace cwth {

namespace {

constexpr int kTailIn = 8192;      // longest level input the LDS tail takes
constexpr int kTailThreads = 1024;
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t level_len(int64_t len, int j) { return ((len - 1) >> j) + 1; }

// One (a, d) pair from level input `a` (len_in samples) at output n.  LT > 0
// is the filter length fixed at compile time (the loops unroll and the taps
// stay in scalar registers); LT == 0 takes f.L.
template <int LT, typename Ptr>
__device__ __forceinline__ void dwt_pair(Ptr a, int64_t len_in, int64_t n, const DwtFilter& f, float& sa,
                                         float& sd) {
    const int L = LT > 0 ? LT : f.L;
    const int64_t i0 = 2 * n;
    float pa = 0.0f, pd = 0.0f;
    if (i0 + L <= len_in) {
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const float v = a[i0 + k];
            pa = fmaf(f.h[k], v, pa);
            pd = fmaf(f.g[k], v, pd);
        }
    } else {
        const int64_t P = len_in + (len_in & 1);
#pragma unroll
        for (int k = 0; k < L; ++k) {
            int64_t i = (i0 + k) % P;
            if (i > len_in - 1) i = len_in - 1;
            const float v = a[i];
            pa = fmaf(f.h[k], v, pa);
            pd = fmaf(f.g[k], v, pd);
        }
    }
    sa = pa;
    sd = pd;
}

// Two neighbouring pairs (outputs n, n + 1, n even) from an 8-byte aligned
// level: the shared window x[2n .. 2n + L + 1] is read as float2s once.
// Same FMA chains as dwt_pair.
template <int LT>
__device__ __forceinline__ void dwt_pair2(const float* __restrict__ a, int64_t n, const DwtFilter& f, float* sa,
                                          float* sd) {
    constexpr int L = LT;
    float w[L + 2];
    const float2* a2 = reinterpret_cast<const float2*>(a + 2 * n);
#pragma unroll
    for (int k = 0; k < L / 2 + 1; ++k) {
        const float2 v = a2[k];
        w[2 * k] = v.x;
        w[2 * k + 1] = v.y;
    }
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        float pa = 0.0f, pd = 0.0f;
#pragma unroll
        for (int k = 0; k < L; ++k) {
            pa = fmaf(f.h[k], w[2 * o + k], pa);
            pd = fmaf(f.g[k], w[2 * o + k], pd);
        }
        sa[o] = pa;
        sd[o] = pd;
    }
}

// One level for the whole batch: lane -> outputs 2i, 2i + 1 (the paired path
// needs a compile-time length and an 8-byte aligned level; otherwise one
// pair at a time).
template <int LT, bool VEC>
__global__ __launch_bounds__(256) void k_dwt_level(const float* __restrict__ src, int64_t src_stride, int64_t len_in,
                                                   float* __restrict__ pyr, int64_t pyr_stride, int64_t off,
                                                   int64_t len_out, DwtFilter f) {
    const int64_t n = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
    if (n >= len_out) return;
    const int L = LT > 0 ? LT : f.L;
    const int64_t c = blockIdx.y;
    const float* a = src + c * src_stride;
    float* p = pyr + c * pyr_stride + off;
    float sa[2], sd[2];
    const bool two = n + 1 < len_out;
    if constexpr (VEC && LT > 0) {
        if (two && 2 * n + 2 + L <= len_in) {
            dwt_pair2<LT>(a, n, f, sa, sd);
            *reinterpret_cast<float2*>(p + n) = make_float2(sa[0], sa[1]);     // off and n are even
            p[len_out + n] = sd[0];
            p[len_out + n + 1] = sd[1];
            return;
        }
    }
    dwt_pair<LT>(a, len_in, n, f, sa[0], sd[0]);
    p[n] = sa[0];
    p[len_out + n] = sd[0];
    if (two) {
        dwt_pair<LT>(a, len_in, n + 1, f, sa[1], sd[1]);
        p[n + 1] = sa[1];
        p[len_out + n + 1] = sd[1];
    }
}

// Levels j0 .. J of one clip; `src` holds a_{j0-1} (len_in <= kTailIn).
template <int LT>
__global__ __launch_bounds__(kTailThreads) void k_dwt_tail(const float* __restrict__ src, int64_t src_stride,
                                                           int64_t len_in, int j0, int J, float* __restrict__ pyr,
                                                           int64_t pyr_stride, int64_t off, DwtFilter f) {
    __shared__ float buf_a[kTailIn];
    __shared__ float buf_b[kTailIn / 2];
    const int64_t c = blockIdx.x;
    const float* s = src + c * src_stride;
    for (int i = threadIdx.x; i < len_in; i += kTailThreads) buf_a[i] = s[i];
    __syncthreads();
    float* p = pyr + c * pyr_stride;
    int64_t lin = len_in;
    for (int j = j0; j <= J; ++j) {
        const bool even = ((j - j0) & 1) == 0;
        const float* in = even ? buf_a : buf_b;
        float* out = even ? buf_b : buf_a;
        const int64_t lout = (lin + 1) >> 1;
        for (int n = threadIdx.x; n < lout; n += kTailThreads) {
            float sa, sd;
            dwt_pair<LT>(in, lin, n, f, sa, sd);
            out[n] = sa;
            p[off + n] = sa;
            p[off + lout + n] = sd;
        }
        __syncthreads();
        off += 2 * lout;
        lin = lout;
    }
}

// S[c][j-1][t] = |d_j[t >> j]| for four consecutive t per lane.
__global__ __launch_bounds__(256) void k_dwt_expand(const float* __restrict__ pyr, int64_t pyr_stride, int64_t len,
                                                    int J, float* __restrict__ out, bool vec) {
    const int64_t t0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (t0 >= len) return;
    const int64_t c = blockIdx.y;
    const float* p = pyr + c * pyr_stride;
    float* o = out + c * (int64_t)J * len;
    int64_t off = 0;
    for (int j = 1; j <= J; ++j) {
        const int64_t lj = level_len(len, j);
        const float* d = p + off + lj;
        float v[4];
        if (j >= 2) {
            const float a = fabsf(d[t0 >> j]);  // t0 is a multiple of 4: one coefficient covers all four
            v[0] = v[1] = v[2] = v[3] = a;
        } else {
            const int64_t i = t0 >> 1;
            const int64_t i1 = (i + 1 < lj) ? i + 1 : lj - 1;
            v[0] = v[1] = fabsf(d[i]);
            v[2] = v[3] = fabsf(d[i1]);
        }
        float* row = o + (int64_t)(j - 1) * len + t0;
        if (vec) {
            const f4 w = {v[0], v[1], v[2], v[3]};
            __builtin_nontemporal_store(w, reinterpret_cast<f4*>(row));
        } else {
            const int m = (len - t0) < 4 ? (int)(len - t0) : 4;
            for (int q = 0; q < m; ++q) row[q] = v[q];
        }
        off += 2 * lj;
    }
}

}  // namespace

int64_t dwt_pyramid_length(int64_t len, int J) {
    int64_t total = 0;
    for (int j = 1; j <= J; ++j) total += 2 * (((len - 1) >> j) + 1);
    return total;
}

template <int LT>
static void launch_levels(const float* x, int64_t len, int clips, const DwtFilter& f, int J, float* pyr,
                          float* out, hipStream_t s) {
    const int64_t pstride = dwt_pyramid_length(len, J);
    const float* src = x;
    int64_t sstride = len, lin = len, off = 0;
    int j = 1;
    for (; j <= J && lin > kTailIn; ++j) {
        const int64_t lout = (lin + 1) >> 1;
        const int64_t grid = (lout + 511) / 512;
        const bool vec = (sstride % 2 == 0) && (reinterpret_cast<uintptr_t>(src) % 8 == 0) &&
                         (reinterpret_cast<uintptr_t>(pyr) % 8 == 0);
        if (vec)
            hipLaunchKernelGGL((k_dwt_level<LT, true>), dim3((unsigned)grid, (unsigned)clips), dim3(256), 0, s, src,
                               sstride, lin, pyr, pstride, off, lout, f);
        else
            hipLaunchKernelGGL((k_dwt_level<LT, false>), dim3((unsigned)grid, (unsigned)clips), dim3(256), 0, s, src,
                               sstride, lin, pyr, pstride, off, lout, f);
        src = pyr + off;
        sstride = pstride;
        off += 2 * lout;
        lin = lout;
    }
    if (j <= J)
        hipLaunchKernelGGL((k_dwt_tail<LT>), dim3((unsigned)clips), dim3(kTailThreads), 0, s, src, sstride, lin, j, J,
                           pyr, pstride, off, f);
    if (out) {
        const int64_t grid = (len + 1023) / 1024;
        // float4 rows when every row starts 16-byte aligned (then t0 + 3 < len too)
        const bool vec = (len % 4 == 0) && (reinterpret_cast<uintptr_t>(out) % 16 == 0);
        hipLaunchKernelGGL(k_dwt_expand, dim3((unsigned)grid, (unsigned)clips), dim3(256), 0, s, pyr, pstride, len,
                           J, out, vec);
    }
}

hipError_t launch_dwt(const float* x, int64_t len, int clips, const DwtFilter& f, int J, float* pyr,
                      float* out, hipStream_t s) {
    if (len <= 0 || clips <= 0 || J <= 0) return hipSuccess;
    switch (f.L) {      // the Daubechies lengths db1 .. db10 unrolled; any other even length generic
        case 2: launch_levels<2>(x, len, clips, f, J, pyr, out, s); break;
        case 4: launch_levels<4>(x, len, clips, f, J, pyr, out, s); break;
        case 6: launch_levels<6>(x, len, clips, f, J, pyr, out, s); break;
        case 8: launch_levels<8>(x, len, clips, f, J, pyr, out, s); break;
        case 10: launch_levels<10>(x, len, clips, f, J, pyr, out, s); break;
        case 12: launch_levels<12>(x, len, clips, f, J, pyr, out, s); break;
        case 14: launch_levels<14>(x, len, clips, f, J, pyr, out, s); break;
        case 16: launch_levels<16>(x, len, clips, f, J, pyr, out, s); break;
        case 18: launch_levels<18>(x, len, clips, f, J, pyr, out, s); break;
        case 20: launch_levels<20>(x, len, clips, f, J, pyr, out, s); break;
        default: launch_levels<0>(x, len, clips, f, J, pyr, out, s); break;
    }
    return hipGetLastError();
}

}  // namespace cwth
