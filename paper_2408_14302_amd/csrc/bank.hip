// Wavelet-bank generation on the device.
//
// Each tap is the dilated, 1/sqrt(a)-normalised Morlet of Eq. (1) (Sec. II-A):
//     t_s[m] = psi(|m| / s) / sqrt(s),  psi(u) = exp(-u^2/2) cos(5u),  |m| <= floor(8 s),
// evaluated in FP64 with the device's exp/cos/sqrt and rounded ONCE to the
// operand type (round to nearest, ties to even), so no double rounding occurs
// on the way to BF16, FP16 or FP8.
#include "cwt_internal.h"

namespace cwth {

__device__ __forceinline__ double morlet_tap(double s, int m) {
    double u = (double)(m < 0 ? -m : m) / s;
    return exp(-0.5 * u * u) * cos(5.0 * u) / sqrt(s);
}

// Round |a| (finite, >= 0) to the nearest value of a binary format with
// `mbits` stored mantissa bits and minimum normal exponent `emin`
// (subnormals below it), ties to even, saturating at `maxfinite`.
// The scaling by a power of two and rint() are exact in FP64.
__device__ __forceinline__ double round_format(double a, int mbits, int emin, double maxfinite) {
    if (a == 0.0) return 0.0;
    int e = ilogb(a);
    if (e < emin) e = emin;
    double q = ldexp(1.0, e - mbits);
    double r = rint(a / q) * q;
    return r > maxfinite ? maxfinite : r;
}

__device__ __forceinline__ uint16_t to_bf16_bits(double v) {
    double r = round_format(fabs(v), 7, -126, 3.3895313892515355e38);
    float f = (float)r;  // exact: r has at most 8 significant bits
    uint32_t u = __float_as_uint(f) >> 16;
    if (v < 0.0) u |= 0x8000u;
    return (uint16_t)u;
}

__device__ __forceinline__ uint16_t to_f16_bits(double v) {
    double r = round_format(fabs(v), 10, -14, 65504.0);
    _Float16 h = (_Float16)(float)r;  // exact: r is representable in FP16
    uint16_t u = __builtin_bit_cast(uint16_t, h);
    if (v < 0.0) u |= 0x8000u;
    return u;
}

// OCP FP8 E4M3: bias 7, 3 mantissa bits, max finite 448, subnormal step 2^-9.
__device__ __forceinline__ uint8_t to_e4m3_bits(double v) {
    double r = round_format(fabs(v), 3, -6, 448.0);
    uint32_t code = 0;
    if (r != 0.0) {
        int e = ilogb(r);
        if (e < -6) {                           // subnormal: r = mant * 2^-9
            code = (uint32_t)(r * 512.0);
        } else {
            uint32_t mant = (uint32_t)((r / ldexp(1.0, e) - 1.0) * 8.0);
            code = ((uint32_t)(e + 7) << 3) | mant;
        }
    }
    if (v < 0.0) code |= 0x80u;
    return (uint8_t)code;
}

__device__ __forceinline__ double from_bf16_bits(uint16_t b) {
    return (double)__uint_as_float(((uint32_t)b) << 16);
}
__device__ __forceinline__ double from_f16_bits(uint16_t b) {
    return (double)(float)__builtin_bit_cast(_Float16, b);
}
__device__ __forceinline__ double from_e4m3_bits(uint8_t b) {
    int sgn = b >> 7, e = (b >> 3) & 15, m = b & 7;
    double v = e == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7);
    return sgn ? -v : v;
}

// ---------------------------------------------------------------------------
// FP32 direct bank: one thread per (group, m).
__global__ void k_gen_direct(const double* __restrict__ scales, int nscales,
                             const DirectGroup* __restrict__ groups, int ngroups,
                             float* __restrict__ taps) {
    int g = blockIdx.y;
    if (g >= ngroups) return;
    const DirectGroup G = groups[g];
    int span = 2 * G.P + 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < span; i += gridDim.x * blockDim.x) {
        int m = i - G.P;
        for (int r = 0; r < kDirectRows; ++r) {
            int pos = g * kDirectRows + r;   // sorted position
            float v = 0.0f;
            if (pos < nscales) {
                double s = scales[pos];
                int M = (int)floor(8.0 * s);
                if (m >= -M && m <= M) v = (float)morlet_tap(s, m);
            }
            taps[G.off + (int64_t)i * kDirectRows + r] = v;
        }
    }
}

// MFMA bank: one thread per (block, step, lane).  The lane holds row r = lane % 32
// and the `per` consecutive K positions starting at (lane / 32) * per.
template <int DT>
__global__ void k_gen_mfma(const double* __restrict__ scales, int nscales,
                           const MfmaBlock* __restrict__ blocks, int nblocks,
                           uint8_t* __restrict__ frags, const double* __restrict__ alpha) {
    constexpr int KS = kstep_of(DT);
    constexpr int PER = KS / 2;                       // K values per lane
    constexpr int FRAG = DT == DT_FP8 ? 32 : 16;      // bytes per lane fragment
    constexpr int STEP = (DT == DT_BF16X3 ? 2 : 1) * 64 * FRAG;
    int b = blockIdx.y;
    if (b >= nblocks) return;
    const MfmaBlock B = blocks[b];
    int nsteps = B.hi - B.lo + 1;
    int total = nsteps * 64;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        int step = i / 64, lane = i % 64;
        int ks = B.lo + step;
        int r = lane % 32, g = lane / 32;
        int pos = b * kBlockRows + r;
        bool valid = pos < nscales;
        double s = valid ? scales[pos] : 1.0;
        int M = valid ? (int)floor(8.0 * s) : -1;
        double al = (DT == DT_FP8 && valid) ? alpha[pos] : 1.0;
        uint8_t* dst = frags + B.frag_off + (int64_t)step * STEP + (int64_t)lane * FRAG;
        for (int j = 0; j < PER; ++j) {
            int m = ks * KS + g * PER + j;
            double t = (m >= -M && m <= M) ? morlet_tap(s, m) : 0.0;
            if constexpr (DT == DT_BF16) {
                ((uint16_t*)dst)[j] = to_bf16_bits(t);
            } else if constexpr (DT == DT_FP16) {
                ((uint16_t*)dst)[j] = to_f16_bits(t);
            } else if constexpr (DT == DT_BF16X3) {
                uint16_t hi = to_bf16_bits(t);
                double lo = t - from_bf16_bits(hi);   // exact in FP64
                ((uint16_t*)dst)[j] = hi;
                ((uint16_t*)(dst + 64 * FRAG))[j] = to_bf16_bits(lo);
            } else {
                dst[j] = to_e4m3_bits(t * al);
            }
        }
    }
}

// Toeplitz bank: one thread per (group, scale, unit k, copy r); element i of
// the unit is t[8 k + i + jb - 24 - r].
template <int DT>
__global__ void k_gen_toep(const double* __restrict__ scales, int nscales, const ToepGroup* __restrict__ groups,
                           int ngroups, uint8_t* __restrict__ frags) {
    const int g = blockIdx.y;
    if (g >= ngroups) return;
    const ToepGroup G = groups[g];
    const int CL = toep_copy_units(G.D);
    const int total = kToepScales * CL * 8;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int r = i % 8, k = (i / 8) % CL, sc = i / (8 * CL);
        const int pos = g * kToepScales + sc;
        const bool valid = pos < nscales;
        const double s = valid ? scales[pos] : 1.0;
        const int M = valid ? (int)floor(8.0 * s) : -1;
        uint16_t* dst = (uint16_t*)(frags + G.frag_off + (int64_t)i * 16);
        const int m0 = 8 * k + G.jb - 24 - r;
        for (int e = 0; e < 8; ++e) {
            const int m = m0 + e;
            const double t = (m >= -M && m <= M) ? morlet_tap(s, m) : 0.0;
            dst[e] = DT == DT_BF16 ? to_bf16_bits(t) : to_f16_bits(t);
        }
    }
}

hipError_t gen_toep_bank(int dt, const double* d_scales_sorted, int nscales, const ToepGroup* d_groups,
                         int ngroups, uint8_t* d_frags, hipStream_t st) {
    dim3 grid(64, ngroups), block(256);
    if (dt == DT_BF16)
        hipLaunchKernelGGL((k_gen_toep<DT_BF16>), grid, block, 0, st, d_scales_sorted, nscales, d_groups, ngroups, d_frags);
    else if (dt == DT_FP16)
        hipLaunchKernelGGL((k_gen_toep<DT_FP16>), grid, block, 0, st, d_scales_sorted, nscales, d_groups, ngroups, d_frags);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t gen_direct_bank(const double* d_scales_sorted, int nscales, const DirectGroup* d_groups,
                           int ngroups, float* d_taps, int64_t, hipStream_t st) {
    dim3 grid(16, ngroups), block(256);
    hipLaunchKernelGGL(k_gen_direct, grid, block, 0, st, d_scales_sorted, nscales, d_groups,
                       ngroups, d_taps);
    return hipGetLastError();
}

hipError_t gen_mfma_bank(int dt, const double* d_scales_sorted, int nscales,
                         const MfmaBlock* d_blocks, int nblocks, uint8_t* d_frags, int64_t,
                         const double* d_alpha, hipStream_t st) {
    dim3 grid(64, nblocks), block(256);
    switch (dt) {
        case DT_BF16: hipLaunchKernelGGL((k_gen_mfma<DT_BF16>), grid, block, 0, st, d_scales_sorted, nscales, d_blocks, nblocks, d_frags, d_alpha); break;
        case DT_FP16: hipLaunchKernelGGL((k_gen_mfma<DT_FP16>), grid, block, 0, st, d_scales_sorted, nscales, d_blocks, nblocks, d_frags, d_alpha); break;
        case DT_BF16X3: hipLaunchKernelGGL((k_gen_mfma<DT_BF16X3>), grid, block, 0, st, d_scales_sorted, nscales, d_blocks, nblocks, d_frags, d_alpha); break;
        case DT_FP8: hipLaunchKernelGGL((k_gen_mfma<DT_FP8>), grid, block, 0, st, d_scales_sorted, nscales, d_blocks, nblocks, d_frags, d_alpha); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Read back one sorted scale's stored taps, decoded to double.
__global__ void k_decode(int dt, const uint8_t* __restrict__ frags, const MfmaBlock* __restrict__ blocks,
                         const float* __restrict__ direct, const DirectGroup* __restrict__ dgroups,
                         int pos, int M, double* __restrict__ out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= 2 * M; i += gridDim.x * blockDim.x) {
        int m = i - M;
        double v;
        if (dt == DT_FP32) {
            const DirectGroup G = dgroups[pos / kDirectRows];
            v = (double)direct[G.off + (int64_t)(m + G.P) * kDirectRows + pos % kDirectRows];
        } else {
            const MfmaBlock& B = blocks[pos / kBlockRows];
            int r = pos % kBlockRows;
            int KS = kstep_of(dt), per = KS / 2, frag = dt == DT_FP8 ? 32 : 16;
            int step_bytes = (dt == DT_BF16X3 ? 2 : 1) * 64 * frag;
            int ks = (m >= 0) ? m / KS : -((-m + KS - 1) / KS);
            int k = m - ks * KS;
            int lane = r + 32 * (k / per), j = k % per;
            const uint8_t* p = frags + B.frag_off + (int64_t)(ks - B.lo) * step_bytes + lane * frag;
            if (dt == DT_BF16) v = from_bf16_bits(((const uint16_t*)p)[j]);
            else if (dt == DT_FP16) v = from_f16_bits(((const uint16_t*)p)[j]);
            else if (dt == DT_BF16X3) v = from_bf16_bits(((const uint16_t*)p)[j]) +
                                          from_bf16_bits(((const uint16_t*)(p + 64 * frag))[j]);
            else v = from_e4m3_bits(p[j]) * (double)B.inv_alpha[r];
        }
        out[i] = v;
    }
}

hipError_t decode_bank_taps(int dt, const uint8_t* d_frags, const MfmaBlock* d_blocks,
                            const float* d_direct, const DirectGroup* d_dgroups, int sorted_pos,
                            int M, double* d_out, hipStream_t st) {
    hipLaunchKernelGGL(k_decode, dim3(32), dim3(256), 0, st, dt, d_frags, d_blocks, d_direct,
                       d_dgroups, sorted_pos, M, d_out);
    return hipGetLastError();
}

}  // namespace cwth
