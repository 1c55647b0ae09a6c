// Strided-frame contraction on the matrix cores (gfx950 MFMA).
//
// For one work-group tile (consecutive frames k0 .. k0+F-1 of one clip and one
// or more 32-scale blocks) it computes
//     W[i][k] = sum_m t_i[m] * x~[k*hop + m]          (Eq. (1), Sec. II-A/II-B)
// as C[32 scales x 32 frames] += T[32 x KS] * X[KS x 32] per MFMA, where
//     T[r][kk] = t_r[KS*ks + kk]                (bank fragment, L2 resident)
//     X[kk][n] = x~[(k0+n)*hop + KS*ks + kk]    (Hankel view of the signal, LDS)
// with KS = 16 (BF16/FP16: v_mfma_f32_32x32x16_*) or 64 (FP8:
// v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales).  Accumulation is FP32.
//
// Signal staging (samples outside [0, len) are zero):
//   WIN     the tile's whole window x~[k0*hop + KS*glo + p] over the K range of
//           its scale blocks, converted once from global memory and shared by
//           up to four blocks (one per wave); kept in `copies` copies shifted
//           by multiples of gcd(hop, U) so every lane's 16-byte read is aligned
//           (U = elements per 16 bytes); with one copy and an even frame
//           stride an XOR swizzle of the 16-byte unit index spreads the
//           frame-strided reads over the LDS banks.  The default whenever the
//           window fits.
//   LINEAR  the same layout, walked in chunks of `chunk_steps` K-steps through
//           two LDS buffers fed from a raw FP32 window (very wide scales at
//           small hops).
//   ROWS    one padded row per frame holding x~[(k0+f)*hop + KS*ks_c + c],
//           chunked (frames so far apart that no window fits).
// Summation order per coefficient: K-steps ascending, fixed per block, so the
// result does not depend on the tile, the launch shape or the batch.
#include "cwt_internal.h"

namespace cwth {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Clip signals and outputs are device (global) memory, reached through
// pointers the compiler cannot place: accessed through these, they compile to
// global rather than flat instructions (a flat access also counts on the LDS
// counter, so a later wait for LDS reads would wait for it as well).
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) f32x4 gf32x4;

template <int DT>
struct Tr {
    static constexpr int ES = DT == DT_FP8 ? 1 : 2;   // bytes per operand element
    static constexpr int KS = kstep_of(DT);           // K per MFMA
    static constexpr int U = 16 / ES;                 // elements per 16-byte unit
    static constexpr int PER = KS / 2;                // K values held by one lane
    static constexpr int LU = PER / U;                // 16-byte units per lane fragment
    static constexpr int PLANES = DT == DT_BF16X3 ? 2 : 1;
    static constexpr int FRAG = 16 * LU;              // bytes per lane fragment
    static constexpr int STEP = PLANES * 64 * FRAG;   // bank bytes per K-step
};

template <int DT>
struct Frag {
    i32x4 u[Tr<DT>::PLANES][Tr<DT>::LU];
};

template <int DT>
__device__ __forceinline__ f32x16 mma(const i32x4* a, const i32x4* b, f32x16 c) {
    if constexpr (DT == DT_BF16 || DT == DT_BF16X3) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[0]),
                                                       __builtin_bit_cast(bf16x8, b[0]), c, 0, 0, 0);
    } else if constexpr (DT == DT_FP16) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a[0]),
                                                      __builtin_bit_cast(f16x8, b[0]), c, 0, 0, 0);
    } else {
        i32x8 av = {a[0][0], a[0][1], a[0][2], a[0][3], a[1][0], a[1][1], a[1][2], a[1][3]};
        i32x8 bv = {b[0][0], b[0][1], b[0][2], b[0][3], b[1][0], b[1][1], b[1][2], b[1][3]};
        // cbsz = blgp = 0: both operands FP8 E4M3; scale exponents 127 = 2^0.
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
    }
}

// Product of T-fragment and X-fragment into acc, including the split terms.
template <int DT>
__device__ __forceinline__ f32x16 mma_all(const Frag<DT>& t, const Frag<DT>& x, f32x16 acc) {
    if constexpr (DT == DT_BF16X3) {
        acc = mma<DT>(t.u[1], x.u[0], acc);   // lo(t) * hi(x)
        acc = mma<DT>(t.u[0], x.u[1], acc);   // hi(t) * lo(x)
        acc = mma<DT>(t.u[0], x.u[0], acc);   // hi(t) * hi(x)
        return acc;
    } else {
        return mma<DT>(t.u[0], x.u[0], acc);
    }
}

// Per-tile staging geometry (uniform across the work-group).
struct Geo {
    int mode, copies, gh, cs, swz, rs;  // see host: cs/rs in 16-byte units
    int len_u;                          // linear: logical units per copy
    int plane_bytes;
};

template <int DT>
__device__ __forceinline__ Geo make_geo(const ClipArg& c, int F, int chunk) {
    using T = Tr<DT>;
    Geo g;
    g.mode = c.mode;
    g.copies = c.copies;
    g.gh = T::U / c.copies;
    g.swz = c.swz;
    if (g.mode != STAGE_ROWS) {
        int pmax = (F - 1) * c.hop + T::KS * chunk - 1;
        g.len_u = ((pmax / T::U + 1) + 15) & ~15;
        g.cs = g.len_u + (g.copies > 1 ? c.cso : 0);
        g.rs = 0;
        g.plane_bytes = g.copies * g.cs * 16;
    } else {
        g.len_u = 0;
        g.cs = 0;
        g.rs = T::KS * chunk / T::U + 1;
        g.plane_bytes = F * g.rs * 16;
    }
    return g;
}

__device__ __forceinline__ int swizzle(int unit, int swz) {
    return swz >= 0 ? (unit ^ ((unit >> swz) & 15)) : unit;
}

// ---------------------------------------------------------------------------
// Staging.  One chunk of signal is brought in with aligned float4 loads into
// registers before the MFMAs of the previous chunk are issued, and converted
// and written to LDS after them, so the global-load latency overlaps the
// matrix work.  A LINEAR unit is a span of 2U floats that supplies one 16-byte
// unit to every shifted copy; a ROWS unit is U floats of one frame's row.

// CNT samples x~[j .. j+CNT) into v[OFF ..]: float4 loads when the span is
// inside [0, len) and 16-byte aligned, otherwise clamped scalar loads with the
// out-of-range samples replaced by zero (no divergent branches).
template <int CNT, int OFF, int N>
__device__ __forceinline__ void load_span(const float* __restrict__ x, int64_t len, int64_t j,
                                          bool al16, float (&v)[N]) {
    static_assert(OFF + CNT <= N, "span outside the register array");
    if (j >= 0 && j + CNT <= len && al16 && (j & 3) == 0) {
#pragma unroll
        for (int e = 0; e < CNT; e += 4) {
            const f32x4 f4 = *(const gf32x4*)((const gfloat*)x + j + e);
            v[OFF + e] = f4[0]; v[OFF + e + 1] = f4[1]; v[OFF + e + 2] = f4[2]; v[OFF + e + 3] = f4[3];
        }
    } else {
#pragma unroll
        for (int e = 0; e < CNT; ++e) {
            const int64_t jj = j + e;
            const int64_t jc = jj < 0 ? 0 : (jj >= len ? len - 1 : jj);
            const float t = ((const gfloat*)x)[jc];
            v[OFF + e] = (jj >= 0 && jj < len) ? t : 0.0f;
        }
    }
}

// ---------------------------------------------------------------------------
// Packing.  A span of CNT samples is converted once into packed operand
// dwords (per plane); a 16-byte LDS unit that starts SH elements into the span
// is then four funnel shifts (v_alignbyte) of those dwords.
template <int DT, int CNT>
struct Packed {
    static constexpr int ND = CNT * Tr<DT>::ES / 4;   // dwords per plane
    uint32_t d[Tr<DT>::PLANES][ND];
};

template <int DT, int CNT, int OFF, int N>
__device__ __forceinline__ void pack_span(const float (&v)[N], float beta, Packed<DT, CNT>& pk) {
    if constexpr (DT == DT_BF16 || DT == DT_BF16X3) {
#pragma unroll
        for (int i = 0; i < CNT / 2; ++i) {
            const float a0 = v[OFF + 2 * i], a1 = v[OFF + 2 * i + 1];
            const __bf16 h0 = (__bf16)a0, h1 = (__bf16)a1;
            pk.d[0][i] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
            if constexpr (DT == DT_BF16X3) {
                const __bf16 l0 = (__bf16)(a0 - (float)h0), l1 = (__bf16)(a1 - (float)h1);   // exact residuals
                pk.d[1][i] = (uint32_t)__builtin_bit_cast(uint16_t, l0) | ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16);
            }
        }
    } else if constexpr (DT == DT_FP16) {
#pragma unroll
        for (int i = 0; i < CNT / 2; ++i) {
            const _Float16 h0 = (_Float16)v[OFF + 2 * i], h1 = (_Float16)v[OFF + 2 * i + 1];
            pk.d[0][i] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < CNT / 4; ++i) {
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[OFF + 4 * i] * beta, v[OFF + 4 * i + 1] * beta, 0, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(v[OFF + 4 * i + 2] * beta, v[OFF + 4 * i + 3] * beta, w, true);
            pk.d[0][i] = (uint32_t)w;
        }
    }
}

// 16 bytes of plane p starting SH elements into the packed span.
template <int DT, int CNT, int SH>
__device__ __forceinline__ i32x4 window(const Packed<DT, CNT>& pk, int p) {
    constexpr int B = SH * Tr<DT>::ES, q = B / 4, r = B % 4;
    static_assert(q + 4 + (r ? 1 : 0) <= Packed<DT, CNT>::ND, "window outside the span");
    i32x4 o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if constexpr (r == 0)
            o[i] = (int)pk.d[p][q + i];
        else
            o[i] = (int)__builtin_amdgcn_alignbyte(pk.d[p][q + i + 1], pk.d[p][q + i], r);
    }
    return o;
}

template <int DT>
__device__ __forceinline__ void put_unit(uint8_t* lds, int off, int plane_bytes, const i32x4* pk) {
#pragma unroll
    for (int p = 0; p < Tr<DT>::PLANES; ++p) *(i32x4*)(lds + off + p * plane_bytes) = pk[p];
}

// Write the copies of one multi-copy unit: copy cp is the window at SH = cp*gh.
template <int DT, int CNT, int SH = 0>
__device__ __forceinline__ void put_copies(const Packed<DT, CNT>& pk, const Geo& g, int su, uint8_t* lds, int buf) {
    if constexpr (SH < Tr<DT>::U) {
        if (SH % g.gh == 0) {
            i32x4 u[Tr<DT>::PLANES];
#pragma unroll
            for (int p = 0; p < Tr<DT>::PLANES; ++p) u[p] = window<DT, CNT, SH>(pk, p);
            put_unit<DT>(lds, buf + ((SH / g.gh) * g.cs + su) * 16, g.plane_bytes, u);
        }
        put_copies<DT, CNT, SH + 1>(pk, g, su, lds, buf);
    }
}

// Units of staging work.  A unit is one span of samples that one thread loads
// and turns into 16-byte LDS units:
//   LINEAR with copies > 1: 2U samples, one 16-byte unit for every copy;
//   LINEAR with one copy, and ROWS: U samples, one 16-byte unit.
// Per-thread register budget of one prefetched chunk (floats).
template <int DT>
__device__ constexpr int stage_floats() { return 32; }

template <int DT>
__device__ __forceinline__ bool multi_copy(const Geo& g) { return g.mode != STAGE_ROWS && g.copies > 1; }

template <int DT>
__device__ __forceinline__ int stage_units(const Geo& g, int F, int chunk) {
    using T = Tr<DT>;
    return g.mode != STAGE_ROWS ? g.len_u : F * (T::KS * chunk / T::U);
}

// Source sample of single-span unit q and its 16-byte LDS unit.
template <int DT>
__device__ __forceinline__ void unit_geo(const ClipArg& c, const Geo& g, int chunk, int64_t k0, int ks_c, int q,
                                         int64_t& j, int& dst) {
    using T = Tr<DT>;
    if (g.mode != STAGE_ROWS) {
        j = k0 * c.hop + (int64_t)T::KS * ks_c + (int64_t)q * T::U;
        dst = swizzle(q, g.swz);
    } else {
        const int per_row = T::KS * chunk / T::U;
        const int f = q / per_row, cu = q - f * per_row;
        j = (k0 + f) * c.hop + (int64_t)T::KS * ks_c + cu * T::U;
        dst = f * g.rs + cu;
    }
}

template <int DT, int I = 0>
__device__ __forceinline__ void load_single(const ClipArg& c, const Geo& g, int chunk, int64_t k0, int ks_c,
                                            int total, bool al16, float (&r)[stage_floats<DT>()]) {
    constexpr int U = Tr<DT>::U;
    if constexpr ((I + 1) * U <= stage_floats<DT>()) {
        const int q = threadIdx.x + I * 256;
        if (q < total) {
            int64_t j;
            int dst;
            unit_geo<DT>(c, g, chunk, k0, ks_c, q, j, dst);
            load_span<U, I * U>(c.x, c.len, j, al16, r);
        }
        load_single<DT, I + 1>(c, g, chunk, k0, ks_c, total, al16, r);
    }
}

template <int DT, int I = 0>
__device__ __forceinline__ void store_single(const ClipArg& c, const Geo& g, int chunk, int64_t k0, int ks_c,
                                             int total, float beta, const float (&r)[stage_floats<DT>()],
                                             uint8_t* lds, int buf) {
    constexpr int U = Tr<DT>::U;
    if constexpr ((I + 1) * U <= stage_floats<DT>()) {
        const int q = threadIdx.x + I * 256;
        if (q < total) {
            int64_t j;
            int dst;
            unit_geo<DT>(c, g, chunk, k0, ks_c, q, j, dst);
            Packed<DT, U> pk;
            pack_span<DT, U, I * U>(r, beta, pk);
            i32x4 u[Tr<DT>::PLANES];
#pragma unroll
            for (int p = 0; p < Tr<DT>::PLANES; ++p) u[p] = window<DT, U, 0>(pk, p);
            put_unit<DT>(lds, buf + dst * 16, g.plane_bytes, u);
        }
        store_single<DT, I + 1>(c, g, chunk, k0, ks_c, total, beta, r, lds, buf);
    }
}

template <int DT, int I = 0>
__device__ __forceinline__ void load_multi(const ClipArg& c, const Geo& g, int64_t jb, bool al16,
                                           float (&r)[stage_floats<DT>()]) {
    constexpr int SP = 2 * Tr<DT>::U;
    if constexpr ((I + 1) * SP <= stage_floats<DT>()) {
        const int uu = threadIdx.x + I * 256;
        if (uu < g.len_u) load_span<SP, I * SP>(c.x, c.len, jb + (int64_t)uu * Tr<DT>::U, al16, r);
        load_multi<DT, I + 1>(c, g, jb, al16, r);
    }
}

template <int DT, int I = 0>
__device__ __forceinline__ void store_multi(const Geo& g, float beta, const float (&r)[stage_floats<DT>()],
                                            uint8_t* lds, int buf) {
    constexpr int SP = 2 * Tr<DT>::U;
    if constexpr ((I + 1) * SP <= stage_floats<DT>()) {
        const int uu = threadIdx.x + I * 256;
        if (uu < g.len_u) {
            Packed<DT, SP> pk;
            pack_span<DT, SP, I * SP>(r, beta, pk);
            put_copies<DT, SP>(pk, g, swizzle(uu, g.swz), lds, buf);
        }
        store_multi<DT, I + 1>(g, beta, r, lds, buf);
    }
}

// ---------------------------------------------------------------------------
// LINEAR staging through a raw FP32 window in LDS.  raw[p] = x~[jb + p] for
// p < raw_floats(): whole float4s that lie inside [0, len) arrive by direct
// global-to-LDS loads (no registers held across the MFMAs); the conversion
// pass then builds the operand copies from LDS, reading the few float4s that
// straddle the clip edges from global memory with clamped loads.
template <int DT>
__device__ __forceinline__ int raw_floats(const Geo& g) {
    return ((g.len_u + 1) * Tr<DT>::U + 255) & ~255;
}

__device__ __forceinline__ bool float4_direct(int64_t j, int64_t len, bool al16) {
    return al16 && j >= 0 && j + 4 <= len;
}

template <int DT>
__device__ __forceinline__ void raw_issue(const ClipArg& c, const Geo& g, int64_t jb, bool al16, uint8_t* raw) {
    const int nv = raw_floats<DT>(g) / 4;            // float4s, a multiple of 64
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int v0 = w * 64; v0 < nv; v0 += 256) {     // one wave instruction covers 64 float4s
        const int64_t j = jb + 4 * (int64_t)(v0 + lane);
        if (float4_direct(j, c.len, al16))
            __builtin_amdgcn_global_load_lds((const void*)(c.x + j),
                                             (__attribute__((address_space(3))) void*)(raw + v0 * 16), 16, 0, 0);
    }
}

// CNT raw samples starting at p (a multiple of 4) into v[OFF ..].
template <int CNT, int OFF, int N>
__device__ __forceinline__ void raw_span(const ClipArg& c, int64_t jb, bool al16, const uint8_t* raw, int p,
                                         float (&v)[N]) {
#pragma unroll
    for (int e = 0; e < CNT; e += 4) {
        const int64_t j = jb + p + e;
        if (float4_direct(j, c.len, al16)) {
            const float4 f4 = *(const float4*)(raw + (p + e) * 4);
            v[OFF + e] = f4.x; v[OFF + e + 1] = f4.y; v[OFF + e + 2] = f4.z; v[OFF + e + 3] = f4.w;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t jj = j + i;
                const int64_t jc = jj < 0 ? 0 : (jj >= c.len ? c.len - 1 : jj);
                const float t = c.x[jc];
                v[OFF + e + i] = (jj >= 0 && jj < c.len) ? t : 0.0f;
            }
        }
    }
}

// Raw window -> operand copies in LDS buffer `buf`.
template <int DT>
__device__ __forceinline__ void raw_convert(const ClipArg& c, const Geo& g, int64_t jb, bool al16, float beta,
                                            const uint8_t* raw, uint8_t* lds, int buf) {
    constexpr int U = Tr<DT>::U;
    if (g.copies > 1) {
        constexpr int SP = 2 * U;
        for (int uu = threadIdx.x; uu < g.len_u; uu += 256) {
            float v[SP];
            raw_span<SP, 0>(c, jb, al16, raw, uu * U, v);
            Packed<DT, SP> pk;
            pack_span<DT, SP, 0>(v, beta, pk);
            put_copies<DT, SP>(pk, g, swizzle(uu, g.swz), lds, buf);
        }
    } else {
        for (int uu = threadIdx.x; uu < g.len_u; uu += 256) {
            float v[U];
            raw_span<U, 0>(c, jb, al16, raw, uu * U, v);
            Packed<DT, U> pk;
            pack_span<DT, U, 0>(v, beta, pk);
            i32x4 u[Tr<DT>::PLANES];
#pragma unroll
            for (int p = 0; p < Tr<DT>::PLANES; ++p) u[p] = window<DT, U, 0>(pk, p);
            put_unit<DT>(lds, buf + swizzle(uu, g.swz) * 16, g.plane_bytes, u);
        }
    }
}

// Issue the loads of a chunk's first units (as many as the register budget holds).
template <int DT>
__device__ __forceinline__ void stage_load(const ClipArg& c, const Geo& g, int F, int chunk, int64_t k0,
                                           int ks_c, bool al16, float (&r)[stage_floats<DT>()]) {
    using T = Tr<DT>;
    if (multi_copy<DT>(g))
        load_multi<DT>(c, g, k0 * c.hop + (int64_t)T::KS * ks_c, al16, r);
    else
        load_single<DT>(c, g, chunk, k0, ks_c, stage_units<DT>(g, F, chunk), al16, r);
}

// Convert and write the prefetched units, then stage any remaining units directly.
template <int DT>
__device__ __forceinline__ void stage_store(const ClipArg& c, const Geo& g, int F, int chunk, int64_t k0,
                                            int ks_c, bool al16, float beta, const float (&r)[stage_floats<DT>()],
                                            uint8_t* lds, int buf) {
    using T = Tr<DT>;
    constexpr int U = T::U;
    if (multi_copy<DT>(g)) {
        constexpr int SP = 2 * U, UP = stage_floats<DT>() / SP;
        store_multi<DT>(g, beta, r, lds, buf);
        const int64_t jb = k0 * c.hop + (int64_t)T::KS * ks_c;
        for (int uu = threadIdx.x + UP * 256; uu < g.len_u; uu += 256) {
            float v[SP];
            load_span<SP, 0>(c.x, c.len, jb + (int64_t)uu * U, al16, v);
            Packed<DT, SP> pk;
            pack_span<DT, SP, 0>(v, beta, pk);
            put_copies<DT, SP>(pk, g, swizzle(uu, g.swz), lds, buf);
        }
    } else {
        constexpr int UP = stage_floats<DT>() / U;
        const int total = stage_units<DT>(g, F, chunk);
        store_single<DT>(c, g, chunk, k0, ks_c, total, beta, r, lds, buf);
        for (int q = threadIdx.x + UP * 256; q < total; q += 256) {
            int64_t j;
            int dst;
            unit_geo<DT>(c, g, chunk, k0, ks_c, q, j, dst);
            float v[U];
            load_span<U, 0>(c.x, c.len, j, al16, v);
            Packed<DT, U> pk;
            pack_span<DT, U, 0>(v, beta, pk);
            i32x4 u[T::PLANES];
#pragma unroll
            for (int p = 0; p < T::PLANES; ++p) u[p] = window<DT, U, 0>(pk, p);
            put_unit<DT>(lds, buf + dst * 16, g.plane_bytes, u);
        }
    }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Power-of-two signal scale beta = 2^floor(log2(448 / max|x~|)), the maximum
// taken over the samples that frames k0 .. k0+F-1 touch in the K range
// [glo, ghi] (the union of the windows [(k0+f)*hop + KS*glo,
// (k0+f)*hop + KS*(ghi+1)) ).
template <int DT>
__device__ float tile_beta(const ClipArg& c, int F, int64_t k0, int glo, int ghi, float* red) {
    using T = Tr<DT>;
    float m = 0.0f;
    const int nt = kMfmaWaves * kWaveSize;
    const int64_t w = (int64_t)T::KS * (ghi - glo + 1);   // one frame's window
    if (c.hop <= w) {                                     // windows overlap: one range
        int64_t a = k0 * c.hop + (int64_t)T::KS * glo;
        int64_t b = (k0 + F - 1) * c.hop + (int64_t)T::KS * (ghi + 1);
        if (a < 0) a = 0;
        if (b > c.len) b = c.len;
        for (int64_t j = a + threadIdx.x; j < b; j += nt) m = fmaxf(m, fabsf(c.x[j]));
    } else {
        for (int f = 0; f < F; ++f) {
            int64_t a = (k0 + f) * c.hop + (int64_t)T::KS * glo, b = a + w;
            if (a < 0) a = 0;
            if (b > c.len) b = c.len;
            for (int64_t j = a + threadIdx.x; j < b; j += nt) m = fmaxf(m, fabsf(c.x[j]));
        }
    }
    m = wave_max(m);
    int wv = threadIdx.x / kWaveSize;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wv] = m;
    __syncthreads();
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    if (m == 0.0f) return 1.0f;
    int e;
    frexp(448.0 / (double)m, &e);     // 448/m = f * 2^e, f in [0.5, 1)
    // at most 2^126, a normal float whose reciprocal is normal too: a segment
    // whose largest sample lies below ~5e-36 would otherwise get beta = inf
    // (and 0 * inf = NaN for its zero samples); with the clamp its samples
    // still scale to at most 448
    return (float)ldexp(1.0, min(e - 1, 126));
}

// The FP8 tile scale.  Up to hop kFp8SegmentMaxHop: beta of the
// kFp8Segment-frame segment that holds the tile, over the K range of the
// bank's widest block (the last: blocks are sorted by scale); every FP8 tile
// there has 32, 64 or 128 frames and starts at a multiple of its size, so it
// lies in one segment, and beta, hence every FP8 result, is the same for
// every tile configuration and batch.  Beyond, where a segment's samples
// outnumber a 32-frame tile's several times over, beta of the tile's own
// frames and K range (glo, ghi), FP8 then having one configuration.
template <int DT>
__device__ float fp8_beta(const MfmaArgs& a, const ClipArg& c, int F, int64_t k0, int glo, int ghi, float* red) {
    if (c.hop > kFp8SegmentMaxHop) return tile_beta<DT>(c, F, k0, glo, ghi, red);
    const MfmaBlock* __restrict__ W = a.blocks + a.ngroups - 1;
    return tile_beta<DT>(c, kFp8Segment, k0 / kFp8Segment * kFp8Segment, W->lo, W->hi, red);
}

template <int DT>
__device__ __forceinline__ void load_tap(const uint8_t* __restrict__ tp, int lane, Frag<DT>& t) {
    using T = Tr<DT>;
    const uint8_t* p0 = tp + lane * T::FRAG;
#pragma unroll
    for (int p = 0; p < T::PLANES; ++p)
#pragma unroll
        for (int u = 0; u < T::LU; ++u) t.u[p][u] = *((const i32x4*)(p0 + p * 64 * T::FRAG) + u);
}

// Staging layouts as seen by the K loop: linear window without swizzle (every
// read is a per-lane base plus an immediate offset), linear window with the
// XOR swizzle (power-of-two hops), or one row per frame.
enum LoopMode : int { LM_LINEAR = 0, LM_LINEAR_SWZ = 1, LM_ROWS = 2 };

// Signal fragments of step d (relative to the chunk's first step) for the
// lane's A frame blocks.  `vb[fa]` is the lane's byte offset of step 0.
template <int DT, int LM>
__device__ __forceinline__ void load_x1(const uint8_t* lds, int plane_bytes, int swz, int vb, int unit0, int d,
                                        Frag<DT>& x) {
    using T = Tr<DT>;
#pragma unroll
    for (int u = 0; u < T::LU; ++u) {
        int off;
        if constexpr (LM == LM_LINEAR_SWZ) {
            const int unit = unit0 + d * (T::KS / T::U) + u;
            off = vb + ((unit ^ ((unit >> swz) & 15)) << 4);
        } else {
            off = vb + ((d * (T::KS / T::U) + u) << 4);
        }
#pragma unroll
        for (int p = 0; p < T::PLANES; ++p) x.u[p][u] = *(const i32x4*)(lds + p * plane_bytes + off);
    }
}

template <int DT, int A, int LM>
__device__ __forceinline__ void load_x(const uint8_t* lds, int plane_bytes, int swz, const int (&vb)[A],
                                       const int (&unit0)[A], int d, Frag<DT> (&x)[A]) {
#pragma unroll
    for (int fa = 0; fa < A; ++fa) load_x1<DT, LM>(lds, plane_bytes, swz, vb[fa], unit0[fa], d, x[fa]);
}

// Per-lane LDS byte offset of step 0 of a chunk (within one buffer) and, for
// the swizzled layout, the logical 16-byte unit of step 0.
// fb0 is the wave's first 32-frame block within the tile.
template <int DT, int A, int LM>
__device__ __forceinline__ void lane_bases(const ClipArg& c, const Geo& g, int fb0, int (&base)[A], int (&unit0)[A]) {
    using T = Tr<DT>;
    const int lane = threadIdx.x & 63;
    const int n = lane & 31, hg = lane >> 5;
#pragma unroll
    for (int fa = 0; fa < A; ++fa) {
        const int f = 32 * (fb0 + fa) + n;
        if constexpr (LM == LM_ROWS) {
            base[fa] = (f * g.rs + hg * T::LU) * 16;
            unit0[fa] = 0;
        } else {
            const int p = f * c.hop + hg * T::PER;
            const int cbase = ((p % T::U) / g.gh) * g.cs * 16;
            unit0[fa] = p / T::U;
            base[fa] = LM == LM_LINEAR ? cbase + unit0[fa] * 16 : cbase;
        }
    }
}

// Instruction order of one K-step, fixed for the scheduler: for each frame
// block, its MFMA(s) and then the read of its next signal fragment into the
// registers the MFMA has just consumed; last the tap load eight steps ahead.
// Each signal read then has the other A - 1 frame blocks' MFMAs to land.
// Without the order the reads sink next to the MFMAs that consume them.
template <int DT, int A, bool NEXT>
__device__ __forceinline__ void sched_step() {
    using T = Tr<DT>;
    constexpr int NX = T::LU * T::PLANES;            // ds_read_b128 per frame block
    constexpr int NM = DT == DT_BF16X3 ? 3 : 1;      // MFMAs per frame block
    constexpr int NT = T::LU * T::PLANES;            // tap loads per step
#pragma unroll
    for (int fa = 0; fa < A; ++fa) {
        __builtin_amdgcn_sched_group_barrier(0x008, NM, 0);                        // MFMA
        if constexpr (NEXT) __builtin_amdgcn_sched_group_barrier(0x100, NX, 0);   // DS read
    }
    __builtin_amdgcn_sched_group_barrier(0x020, NT, 0);                            // VMEM read
}

// Signal fragments in flight per frame block: with few frame blocks per wave
// a fragment read right after its MFMA would be needed again only A MFMAs
// later, too soon for LDS, so small A reads two steps ahead.
template <int A>
constexpr int x_depth() { return A >= 4 ? 1 : 2; }

// Eight K-steps starting q steps into the range.  Tap fragments (from L2) are
// loaded eight steps ahead into two banks of four register sets; each frame
// block's signal fragment (from LDS) for step j + XD is read into the
// registers that step j's MFMA has just consumed.  Every register slot is a
// compile-time constant.  LAST: the final group (no reads past its end).
// FRONT: a range that starts halfway into this group: steps 0-3 do nothing
// (their slots already hold the taps of steps 8-11).
template <int DT, int A, int LM, int XD, bool LAST, bool FRONT = false>
__device__ __forceinline__ void step_group(const uint8_t* cur, const Geo& g, int swz, const int (&base)[A],
                                           const int (&unit0)[A], int dq, int s8, int hi, int lo,
                                           const uint8_t* __restrict__ tbase, Frag<DT> (&ta)[4], Frag<DT> (&tb)[4],
                                           Frag<DT> (&x)[XD][A], f32x16 (&acc)[A]) {
    using T = Tr<DT>;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        Frag<DT>& tcur = j < 4 ? ta[j & 3] : tb[j & 3];
        const bool next = !(LAST && j + XD > 7);
        if (FRONT && j < 4) continue;
#pragma unroll
        for (int fa = 0; fa < A; ++fa) {
            acc[fa] = mma_all<DT>(tcur, x[j % XD][fa], acc[fa]);
            if (next) load_x1<DT, LM>(cur, g.plane_bytes, swz, base[fa], unit0[fa], dq + j + XD, x[j % XD][fa]);
        }
        load_tap<DT>(tbase + (int64_t)(min(s8 + 8 + j, hi) - lo) * T::STEP, lane, tcur);
        if (next)
            sched_step<DT, A, true>();
        else
            sched_step<DT, A, false>();
    }
}

// The MFMAs of steps ks_c+d0 .. ks_c+d0+ns-1 of the chunk starting at ks_c,
// from LDS buffer `cur`.  ns is a multiple of 8, or with WHOLE of 4 (a
// block's whole range, rounded up): then an odd half group comes first, as
// the second half of a group that starts four steps early.  On entry ta/tb
// hold the taps of the first eight steps (with an odd half first, tb holds
// its four and ta the four after them); chunked tiles leave in them the taps
// of the eight steps after the range.
template <int DT, int A, int LM, bool WHOLE = false>
__device__ __forceinline__ void compute_chunk(const uint8_t* cur, const Geo& g, int swz, const int (&base)[A],
                                              const int (&unit0)[A], int ks_c, int d0, int ns, int hi, int lo,
                                              const uint8_t* __restrict__ tbase, Frag<DT> (&ta)[4],
                                              Frag<DT> (&tb)[4], f32x16 (&acc)[A]) {
    constexpr int XD = x_depth<A>();
    Frag<DT> x[XD][A];
#pragma unroll
    for (int d = 0; d < XD; ++d) load_x<DT, A, LM>(cur, g.plane_bytes, swz, base, unit0, d0 + d, x[d]);
    int q = 0;
    if (WHOLE && (ns & 4)) {
        step_group<DT, A, LM, XD, false, true>(cur, g, swz, base, unit0, d0 - 4, ks_c + d0 - 4, hi, lo, tbase, ta, tb,
                                               x, acc);
        q = 4;
        if (ns == 4) return;
    }
    for (; q + 8 < ns; q += 8)
        step_group<DT, A, LM, XD, false>(cur, g, swz, base, unit0, d0 + q, ks_c + d0 + q, hi, lo, tbase, ta, tb, x,
                                         acc);
    step_group<DT, A, LM, XD, true>(cur, g, swz, base, unit0, d0 + q, ks_c + d0 + q, hi, lo, tbase, ta, tb, x, acc);
}

// LINEAR layouts: raw window by direct loads, converted between chunks.
//   chunk c computes from copies[c & 1] while raw(c+1) is in flight; then the
//   work-group waits for it, converts it into copies[(c+1) & 1] and issues raw(c+2).
template <int DT, int A, int LM>
__device__ __forceinline__ void tile_loop_linear(const MfmaArgs& a, const ClipArg& c, const Geo& g, int64_t k0,
                                                 int lo, int hi, const uint8_t* __restrict__ tbase, bool al16,
                                                 float beta, uint8_t* lds, f32x16 (&acc)[A]) {
    using T = Tr<DT>;
    const int chunk = a.chunk_steps;   // multiple of 8
    const int lane = threadIdx.x & 63;
    const int swz = g.swz < 0 ? 31 : g.swz;
    uint8_t* raw = lds + 2 * a.buf_bytes;
    int base[A], unit0[A];
    lane_bases<DT, A, LM>(c, g, A * (threadIdx.x >> 6), base, unit0);
    auto jb_of = [&](int ks_c) { return k0 * c.hop + (int64_t)T::KS * ks_c; };
    auto tap = [&](int ks) { return tbase + (int64_t)(min(ks, hi) - lo) * T::STEP; };

    const int nchunks = (hi - lo + chunk) / chunk;
    raw_issue<DT>(c, g, jb_of(lo), al16, raw);
    Frag<DT> ta[4], tb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        load_tap<DT>(tap(lo + j), lane, ta[j]);
        load_tap<DT>(tap(lo + 4 + j), lane, tb[j]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    raw_convert<DT>(c, g, jb_of(lo), al16, beta, raw, lds, 0);
    __syncthreads();
    if (nchunks > 1) raw_issue<DT>(c, g, jb_of(lo + chunk), al16, raw);

    for (int ci = 0; ci < nchunks; ++ci) {
        const int ks_c = lo + ci * chunk;
        const int ns = min(chunk, hi - ks_c + 1);   // multiple of 8
        compute_chunk<DT, A, LM>(lds + (ci & 1) * a.buf_bytes, g, swz, base, unit0, ks_c, 0, ns, hi, lo, tbase,
                                 ta, tb, acc);
        if (ci + 1 < nchunks) {
            __builtin_amdgcn_s_waitcnt(0);             // raw(ci+1) has landed in LDS
            __syncthreads();
            raw_convert<DT>(c, g, jb_of(ks_c + chunk), al16, beta, raw, lds, ((ci + 1) & 1) * a.buf_bytes);
            __syncthreads();
            if (ci + 2 < nchunks) raw_issue<DT>(c, g, jb_of(ks_c + 2 * chunk), al16, raw);
        }
    }
}

// SPLIT tile (row layout): F = 32*WF consecutive frames against up to WB =
// 4/WF consecutive 32-scale blocks; wave w takes frame block w / WB and block
// slot (w + tile) % WB (rotated so that the widest block of a group does not
// always land on the same SIMD).  All waves share the staged rows; each wave
// runs only the K-steps of its own block.
// The lane's 16 output rows of a block (and the FP8 descale factors), loaded
// together so that the epilogue's stores wait on at most one memory round
// trip.  Loaded one per store instead, each load was waited for with every
// earlier store still in flight (loads and stores complete in order), which
// serialised the epilogue: it took about as long as the block's K loop.
template <int DT>
struct RowMap {
    int row[16];
    float scale[DT == DT_FP8 ? 16 : 1];
};

template <int DT>
__device__ __forceinline__ void load_rows(const MfmaBlock* __restrict__ B, int hg, RowMap<DT>& m) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int rr = 8 * (v >> 2) + 4 * hg + (v & 3);
        m.row[v] = B->rows[rr];
        if constexpr (DT == DT_FP8) m.scale[v] = B->inv_alpha[rr];
    }
}

// The same from the copy of a group's rows that WIN tiles keep in LDS beside
// their window (slot: the block's place in its group).  LDS reads wait on
// their own counter, not behind the wave's outstanding stores.
template <int DT>
__device__ __forceinline__ void lds_rows(const int* srow, const float* sscale, int slot, int hg, RowMap<DT>& m) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int rr = kBlockRows * slot + 8 * (v >> 2) + 4 * hg + (v & 3);
        m.row[v] = srow[rr];
        if constexpr (DT == DT_FP8) m.scale[v] = sscale[rr];
    }
}

// Epilogue of one 32x32 accumulator: FP8 descale, |.| unless signed output,
// non-temporal stores of the lane's column k.
template <int DT>
__device__ __forceinline__ void store_rows(const RowMap<DT>& m, const f32x16& acc, float inv_beta, int signed_out,
                                           float* out, int64_t K, int64_t k) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        if (m.row[v] < 0) continue;
        float val = acc[v];
        // both factors are powers of two: exact whenever the result is normal,
        // also for a clip so faint that inv_beta sits at 2^-126
        if constexpr (DT == DT_FP8) val = val * m.scale[v] * inv_beta;
        if (!signed_out) val = fabsf(val);
        __builtin_nontemporal_store(val, (gfloat*)out + (int64_t)m.row[v] * K + k);
    }
}

template <int DT>
__device__ __forceinline__ void process_tile_split(const MfmaArgs& a, const ClipArg& c, int tile, int grp,
                                                   uint8_t* lds, float* red) {
    using T = Tr<DT>;
    const int WB = a.split_wb, WF = kMfmaWaves / WB, F = 32 * WF;
    const int chunk = a.split_chunk;   // multiple of 8
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 31, hg = lane >> 5;
    const int wf = w / WB, wb = w - wf * WB;
    const int64_t k0 = (int64_t)tile * F;
    const int b0 = grp * WB, nb = min(WB, a.ngroups - b0);
    int glo = a.blocks[b0].lo, ghi = a.blocks[b0].hi;
    for (int i = 1; i < nb; ++i) {
        glo = min(glo, a.blocks[b0 + i].lo);
        ghi = max(ghi, a.blocks[b0 + i].hi);
    }
    const int slot = (wb + tile) % WB;
    const bool has = slot < nb;
    const MfmaBlock* __restrict__ B = a.blocks + b0 + (has ? slot : 0);
    const int lo = B->lo, hi = B->hi;
    const uint8_t* __restrict__ tbase = a.frags + B->frag_off;
    const Geo g = make_geo<DT>(c, F, chunk);
    const bool al16 = (((uintptr_t)c.x) & 15) == 0;
    float beta = 1.0f;
    if constexpr (DT == DT_FP8) beta = fp8_beta<DT>(a, c, F, k0, glo, ghi, red);

    f32x16 acc[1];
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[0][v] = 0.0f;
    const int base[1] = {((32 * wf + n) * g.rs + hg * T::LU) * 16};
    const int unit0[1] = {0};
    auto tap = [&](int ks) { return tbase + (int64_t)(min(ks, hi) - lo) * T::STEP; };

    const int nchunks = (ghi - glo + chunk) / chunk;
    float r[stage_floats<DT>()];
    stage_load<DT>(c, g, F, chunk, k0, glo, al16, r);
    stage_store<DT>(c, g, F, chunk, k0, glo, al16, beta, r, lds, 0);
    Frag<DT> ta[4], tb[4];
    if (has) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            load_tap<DT>(tap(lo + j), lane, ta[j]);
            load_tap<DT>(tap(lo + 4 + j), lane, tb[j]);
        }
    }
    __syncthreads();
    for (int ci = 0; ci < nchunks; ++ci) {
        const int ks_c = glo + ci * chunk;
        const int ks_e = min(ks_c + chunk - 1, ghi);
        const bool more = ci + 1 < nchunks;
        if (more) stage_load<DT>(c, g, F, chunk, k0, ks_c + chunk, al16, r);
        const int s0 = max(ks_c, lo), s1 = min(ks_e, hi);   // block ranges are 8-aligned
        if (has && s0 <= s1)
            compute_chunk<DT, 1, LM_ROWS>(lds + (ci & 1) * a.buf_bytes, g, 31, base, unit0, ks_c, s0 - ks_c,
                                          s1 - s0 + 1, hi, lo, tbase, ta, tb, acc);
        if (more) stage_store<DT>(c, g, F, chunk, k0, ks_c + chunk, al16, beta, r, lds, ((ci + 1) & 1) * a.buf_bytes);
        __syncthreads();
    }
    if (!has) return;
    const float inv_beta = 1.0f / beta;
    const int64_t k = k0 + 32 * wf + n;
    if (k >= c.K) return;
    RowMap<DT> rm;
    load_rows<DT>(B, hg, rm);
    store_rows<DT>(rm, acc[0], inv_beta, a.signed_out, c.out, c.K, k);
}

// LINEAR work-group tile: F = 128*A consecutive frames of one clip against one
// 32-scale block.  Each wave owns A 32-frame blocks; every K-step is A MFMAs
// sharing one tap fragment.
template <int DT, int A>
__device__ __forceinline__ void process_tile(const MfmaArgs& a, const ClipArg& c, int tile, int blk,
                                             uint8_t* lds, float* red) {
    const int F = 32 * A * kMfmaWaves;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int n = lane & 31, hg = lane >> 5;
    const int64_t k0 = (int64_t)tile * F;

    const MfmaBlock* __restrict__ B = a.blocks + blk;
    const int lo = B->lo, hi = B->hi;
    const uint8_t* __restrict__ tbase = a.frags + B->frag_off;
    const Geo g = make_geo<DT>(c, F, a.chunk_steps);
    const bool al16 = (((uintptr_t)c.x) & 15) == 0;
    float beta = 1.0f;
    if constexpr (DT == DT_FP8) beta = fp8_beta<DT>(a, c, F, k0, lo, hi, red);

    f32x16 acc[A];
#pragma unroll
    for (int fa = 0; fa < A; ++fa)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[fa][v] = 0.0f;

    if (g.swz >= 0)
        tile_loop_linear<DT, A, LM_LINEAR_SWZ>(a, c, g, k0, lo, hi, tbase, al16, beta, lds, acc);
    else
        tile_loop_linear<DT, A, LM_LINEAR>(a, c, g, k0, lo, hi, tbase, al16, beta, lds, acc);

    // Epilogue: optional descale (FP8), |.| unless signed output, coalesced store.
    const float inv_beta = 1.0f / beta;
    RowMap<DT> rm;
    load_rows<DT>(B, hg, rm);
#pragma unroll
    for (int fa = 0; fa < A; ++fa) {
        const int64_t k = k0 + 32 * (A * w + fa) + n;
        if (k >= c.K) continue;
        store_rows<DT>(rm, acc[fa], inv_beta, a.signed_out, c.out, c.K, k);
    }
}

// Register budget of the WIN kernels: W waves per SIMD (512 / W registers per
// lane), enough to overlap one work-group's staging with another's MFMAs, and
// SF staging floats in flight per thread.  Two-plane (BF16x3) and FP8 tap
// fragments are twice as wide.
template <int DT, int A>
struct WinOcc {
    static constexpr bool wide = DT == DT_BF16X3 || DT == DT_FP8;
    static constexpr int W = wide ? (A >= 4 ? 1 : 2) : (A >= 8 ? 2 : (A >= 2 ? 3 : 4));
    static constexpr int SF = 32;
};

// ---------------------------------------------------------------------------
// WIN staging: the whole window, straight from global memory.  Each pass
// issues the loads of R units per thread (SF floats in flight) before it
// converts and writes any of them.
template <int DT, int SF>
__device__ __forceinline__ void win_stage(const ClipArg& c, const Geo& g, int64_t jb, bool al16, float beta,
                                          uint8_t* lds) {
    constexpr int U = Tr<DT>::U;
    if (g.copies > 1) {
        constexpr int SP = 2 * U, R = SF / SP > 0 ? SF / SP : 1;
        for (int u0 = threadIdx.x; u0 < g.len_u; u0 += 256 * R) {
            float v[R][SP];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int uu = u0 + 256 * i;
                if (uu < g.len_u) load_span<SP, 0>(c.x, c.len, jb + (int64_t)uu * U, al16, v[i]);
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int uu = u0 + 256 * i;
                if (uu < g.len_u) {
                    Packed<DT, SP> pk;
                    pack_span<DT, SP, 0>(v[i], beta, pk);
                    put_copies<DT, SP>(pk, g, swizzle(uu, g.swz), lds, 0);
                }
            }
        }
    } else {
        constexpr int R = SF / U > 0 ? SF / U : 1;
        for (int u0 = threadIdx.x; u0 < g.len_u; u0 += 256 * R) {
            float v[R][U];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int uu = u0 + 256 * i;
                if (uu < g.len_u) load_span<U, 0>(c.x, c.len, jb + (int64_t)uu * U, al16, v[i]);
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int uu = u0 + 256 * i;
                if (uu < g.len_u) {
                    Packed<DT, U> pk;
                    pack_span<DT, U, 0>(v[i], beta, pk);
                    i32x4 u[Tr<DT>::PLANES];
#pragma unroll
                    for (int p = 0; p < Tr<DT>::PLANES; ++p) u[p] = window<DT, U, 0>(pk, p);
                    put_unit<DT>(lds, swizzle(uu, g.swz) * 16, g.plane_bytes, u);
                }
            }
        }
    }
}

// Work-group barrier for LDS hand-offs: waits for this wave's LDS accesses
// only, so global loads in flight and stores not yet acknowledged stay so.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block i (0, 1, ..) of the wave's list within its group: waves with the same
// frames split the group's WB blocks WS ways in snake order (WS = 2, WB = 4:
// {0, 3} and {1, 2}), which evens out the K ranges when they grow with the
// block index.  With one block per wave (WS = WB) the assignment rotates with
// the tile so that the widest block does not always land on the same SIMD.
__device__ __forceinline__ int wave_block(int i, int ws, int WS, int WB, int tile) {
    if (WS == WB) return i == 0 ? (ws + tile) % WB : WB;
    const int r = i >> 1;
    return (i & 1) ? 2 * WS * r + 2 * WS - 1 - ws : 2 * WS * r + ws;
}

// K-steps, MFMAs and epilogue of one block (slot `slot` of its group) for
// the wave's A frame blocks (fb0 ..); ta/tb hold the block's first eight tap
// fragments on entry.
template <int DT, int A>
__device__ __forceinline__ void win_block(const MfmaArgs& a, const ClipArg& c, const Geo& g, const uint8_t* lds,
                                          const int* srow, const float* sscale, const MfmaBlock* __restrict__ B,
                                          int slot, int glo, int64_t k0, int fb0, float inv_beta,
                                          Frag<DT> (&ta)[4], Frag<DT> (&tb)[4]) {
    const int lane = threadIdx.x & 63;
    const int n = lane & 31, hg = lane >> 5;
    const int lo = B->lo, elo = B->elo, ns = (B->ehi - elo + 4) & ~3;   // steps, rounded up to four
    const uint8_t* __restrict__ tbase = a.frags + B->frag_off;
    f32x16 acc[A];
#pragma unroll
    for (int fa = 0; fa < A; ++fa)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[fa][v] = 0.0f;
    int base[A], unit0[A];
    if (g.swz >= 0) {
        lane_bases<DT, A, LM_LINEAR_SWZ>(c, g, fb0, base, unit0);
        compute_chunk<DT, A, LM_LINEAR_SWZ, true>(lds, g, g.swz, base, unit0, glo, elo - glo, ns, elo + ns - 1, lo,
                                                  tbase, ta, tb, acc);
    } else {
        lane_bases<DT, A, LM_LINEAR>(c, g, fb0, base, unit0);
        compute_chunk<DT, A, LM_LINEAR, true>(lds, g, 31, base, unit0, glo, elo - glo, ns, elo + ns - 1, lo, tbase,
                                              ta, tb, acc);
    }
    RowMap<DT> rm;
    lds_rows<DT>(srow, sscale, slot, hg, rm);
#pragma unroll
    for (int fa = 0; fa < A; ++fa) {
        const int64_t k = k0 + 32 * (fb0 + fa) + n;
        if (k >= c.K) continue;
        store_rows<DT>(rm, acc[fa], inv_beta, a.signed_out, c.out, c.K, k);
    }
}

// WIN tile: F = 32*A*(4/WS) consecutive frames against the WB consecutive
// 32-scale blocks of group grp, over one shared window.  Wave w takes frame
// group w / WS (A frame blocks) and runs its share of the group's blocks
// (wave_block) one after the other: the stores of one block drain while the
// next one's MFMAs run.
template <int DT, int A>
__device__ __forceinline__ void process_tile_win(const MfmaArgs& a, const ClipArg& c, int tile, int grp,
                                                 uint8_t* lds, float* red) {
    using T = Tr<DT>;
    const int WB = c.wb, WS = c.ws, WF = kMfmaWaves / WS, F = 32 * A * WF;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wf = w / WS, ws = w - wf * WS;
    const int64_t k0 = (int64_t)tile * F;
    const int b0 = grp * WB, nb = min(WB, a.ngroups - b0);
    int glo = a.blocks[b0].lo, ghi = a.blocks[b0].hi;
    for (int i = 1; i < nb; ++i) {
        glo = min(glo, a.blocks[b0 + i].lo);
        ghi = max(ghi, a.blocks[b0 + i].hi);
    }
    const Geo g = make_geo<DT>(c, F, ghi - glo + 1);
    const bool al16 = (((uintptr_t)c.x) & 15) == 0;
    float beta = 1.0f;
    if constexpr (DT == DT_FP8) beta = fp8_beta<DT>(a, c, F, k0, glo, ghi, red);
    const float inv_beta = 1.0f / beta;

    // taps of the first steps of the wave's first block (compute_chunk with
    // WHOLE): elo <= 0 and hi >= 7, so steps elo .. elo+7 lie in the block's
    // stored range (those past ehi hold zeros)
    int j = wave_block(0, ws, WS, WB, tile);
    Frag<DT> ta[4], tb[4];
    auto prefetch = [&](const MfmaBlock* __restrict__ B) {
        const uint8_t* __restrict__ tbase = a.frags + B->frag_off + (int64_t)(B->elo - B->lo) * T::STEP;
        const int front = ((B->ehi - B->elo + 4) & 4) ? 4 : 0;   // an odd half group comes first
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            load_tap<DT>(tbase + (int64_t)(front + s) * T::STEP, lane, ta[s]);
            load_tap<DT>(tbase + (int64_t)(4 - front + s) * T::STEP, lane, tb[s]);
        }
    };
    if (j < nb) prefetch(a.blocks + b0 + j);
    win_stage<DT, WinOcc<DT, A>::SF>(c, g, k0 * c.hop + (int64_t)T::KS * glo, al16, beta, lds);
    // the group's output rows (and FP8 descale factors) beside the window,
    // in the room the host reserves after it (kWinRowBytes)
    int* srow = (int*)(lds + T::PLANES * g.plane_bytes);
    float* sscale = (float*)(srow + 4 * kBlockRows);
    for (int i = threadIdx.x; i < nb * kBlockRows; i += kMfmaWaves * kWaveSize) {
        const MfmaBlock* __restrict__ Bi = a.blocks + b0 + i / kBlockRows;
        srow[i] = Bi->rows[i % kBlockRows];
        if constexpr (DT == DT_FP8) sscale[i] = Bi->inv_alpha[i % kBlockRows];
    }
    lds_barrier();
    for (int i = 0; j < nb; j = wave_block(++i, ws, WS, WB, tile)) {
        if (i > 0) prefetch(a.blocks + b0 + j);
        win_block<DT, A>(a, c, g, lds, srow, sscale, a.blocks + b0 + j, j, glo, k0, A * wf, inv_beta, ta, tb);
    }
}

// ---------------------------------------------------------------------------
// Toeplitz tiles (hop 1, BF16/FP16).  For one scale (taps t[m], |m| <= M) and
// the 1024 frames k = k1 + 32 i + j (i, j < 32) of a block:
//     W[k] = sum_p t[p - j] * x~[k1 + 32 i + p],   p = jb + 16 d + u  (u < 16),
// so every K-step d is one MFMA  C[i][j] += X_d[i][u] * T_d[u][j]  with
//     X_d[i][u] = x~[k1 + 32 i + jb + 16 d + u]   (strided rows of the staged
//                 window: a lane reads 8 consecutive samples, 16-byte aligned)
//     T_d[u][j] = t[jb + 16 d + u - j]             (a Toeplitz block of the taps:
//                 one aligned 16-byte unit of a shifted copy per lane).
// The signal fragment of a step serves every scale of the wave and the tap
// fragment every block, so a wave holding kToepScales scales x NB blocks
// issues kToepScales * NB MFMAs per kToepScales + NB LDS fragment reads (the
// 32-scale blocks of the other tiles share one tap fragment between at most
// A frame blocks and pad every scale to its block's widest range).  The K
// range of a scale group starts at jb (<= -M, a multiple of 8) and spans D
// steps (jb + 16 D >= M + 32, D a multiple of 4); every coefficient adds its
// steps in ascending d in one accumulator, so the result depends neither on
// NB nor on the launch.  A work-group (4 waves) owns 4 * 1024 * NB
// consecutive frames of one clip and one scale group.
//
// The taps reach the K loop through LDS: the work-group copies the units of
// the next kToepChunk steps (the group's shifted copies, 17 KiB for 32 steps
// and two scales, against 64 KiB of fragments per wave when every wave loaded
// its own from L2) into the free one of two buffers while it runs the
// current chunk, with one barrier per chunk.  LDS holds the two tap buffers
// (kToepTapBytes) and then the signal window.

// 16-byte unit u of a Toeplitz window sits at LDS unit u ^ ((u >> 4) & 3):
// the eight lanes of a 128-bit read pass, 4 units apart, then fall on eight
// different 16-byte slots of a 256-byte bank row instead of four.
__device__ __forceinline__ int toep_swz(int u) { return u ^ ((u >> 4) & 3); }

// x~[j0 + 8 u .. j0 + 8 u + 8) converted to the operand type, for u < nunits;
// R units per thread in flight.
template <int DT, int R = 4>
__device__ __forceinline__ void toep_stage(const ClipArg& c, int64_t j0, int nunits, bool al16, uint8_t* lds) {
    for (int u0 = threadIdx.x; u0 < nunits; u0 += R * kMfmaWaves * kWaveSize) {
        float v[R][8];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int u = u0 + i * kMfmaWaves * kWaveSize;
            if (u < nunits) load_span<8, 0>(c.x, c.len, j0 + 8 * (int64_t)u, al16, v[i]);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int u = u0 + i * kMfmaWaves * kWaveSize;
            if (u < nunits) {
                Packed<DT, 8> pk;
                pack_span<DT, 8, 0>(v[i], 1.0f, pk);
                *(i32x4*)(lds + toep_swz(u) * 16) = window<DT, 8, 0>(pk, 0);
            }
        }
    }
}

// Tap chunks.  Chunk c of group G is units k = 2 c kToepChunk + kk,
// kk < kToepChunkK, of every copy of both scales, in LDS as
// [scale][kk][copy]; the eight lanes of a read pass (fixed l / 8) then read
// eight different copies of one unit: eight different 16-byte slots.
constexpr int kToepFetch = (kToepChunkUnits + kMfmaWaves * kWaveSize - 1) / (kMfmaWaves * kWaveSize);

__device__ __forceinline__ void toep_fetch(const MfmaArgs& a, const ToepGroup* __restrict__ G, int c,
                                           i32x4 (&pre)[kToepFetch]) {
    const int CL = toep_copy_units(G->D), k0 = 2 * kToepChunk * c;
    const uint8_t* __restrict__ base = a.tfrags + G->frag_off;
#pragma unroll
    for (int i = 0; i < kToepFetch; ++i) {
        const int x = threadIdx.x + i * kMfmaWaves * kWaveSize;
        const int sc = x >= kToepChunkK * 8 ? 1 : 0, xs = x - sc * kToepChunkK * 8;
        if (x < kToepChunkUnits && k0 + xs / 8 < CL)
            pre[i] = *(const i32x4*)(base + ((int64_t)(sc * CL + k0) * 8 + xs) * 16);
        else
            pre[i] = i32x4{0, 0, 0, 0};
    }
}

__device__ __forceinline__ void toep_put(uint8_t* buf, const i32x4 (&pre)[kToepFetch]) {
#pragma unroll
    for (int i = 0; i < kToepFetch; ++i) {
        const int x = threadIdx.x + i * kMfmaWaves * kWaveSize;
        if (x < kToepChunkUnits) *(i32x4*)(buf + x * 16) = pre[i];
    }
}

// The K loop of one scale group over the wave's frames, into acc, from the
// staged window `win` (16-byte unit ubase is row i = lane % 32, K half
// lane / 32, of step 0, block 0) and the tap buffers `taps`, whose buffer 0
// holds the group's chunk 0 (visible to every wave) on entry.  Every wave of
// the work-group runs the chunks and their barriers; a wave whose frames lie
// past the clip (`active` false) skips the MFMAs.
template <int DT, int NB>
__device__ __forceinline__ void toep_loop(const MfmaArgs& a, const ToepGroup* __restrict__ G, int ubase, bool active,
                                          const uint8_t* win, uint8_t* taps, f32x16 (&acc)[kToepScales][NB]) {
    constexpr int TS = kToepScales;
    constexpr int CB = kToepChunkUnits * 16;   // bytes per tap buffer
    const int lane = threadIdx.x & 63;
    const int D = G->D;
    const int nch = (D + kToepChunk - 1) / kToepChunk;
    // lane's unit at local step 0: copy (j mod 8) of unit 2 d + h - j / 8 + 3 (j = l % 32, h = l / 32)
    const int tu = ((lane >> 5) - ((lane & 31) >> 3) + 3) * 8 + (lane & 7);
    i32x4 sg[2][NB], tp[2][TS];
#pragma unroll
    for (int s = 0; s < TS; ++s)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[s][b][v] = 0.0f;
#pragma unroll
    for (int b = 0; b < NB; ++b) sg[0][b] = *(const i32x4*)(win + toep_swz(ubase + 128 * b) * 16);
#pragma unroll
    for (int s = 0; s < TS; ++s) tp[0][s] = *(const i32x4*)(taps + (s * kToepChunkK * 8 + tu) * 16);
    for (int ch = 0; ch < nch; ++ch) {
        const int d0 = ch * kToepChunk, steps = min(kToepChunk, D - d0);   // a multiple of 4
        const bool more = ch + 1 < nch;
        i32x4 pre[kToepFetch];
        if (more) toep_fetch(a, G, ch + 1, pre);
        const uint8_t* cur = taps + (ch & 1) * CB;
        if (active) {
            // one K-step d = d0 + q + jo from register buffers jo & 1 (q is a
            // multiple of 4, jo a constant)
            auto step = [&](const int q, const int jo) __attribute__((always_inline)) {
                const int jj = q + jo, d = d0 + jj;
                // the next step's signal rows (step D, read last, lies inside
                // the window) and taps (the chunk's last step re-reads its own),
                // issued first so that they land during this step's MFMAs
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    sg[(jo + 1) & 1][b] = *(const i32x4*)(win + toep_swz(ubase + 128 * b + 2 * (d + 1)) * 16);
                const int jn = min(jj + 1, steps - 1);
#pragma unroll
                for (int s = 0; s < TS; ++s)
                    tp[(jo + 1) & 1][s] = *(const i32x4*)(cur + (s * kToepChunkK * 8 + tu + 16 * jn) * 16);
#pragma unroll
                for (int s = 0; s < TS; ++s)
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[s][b] = mma<DT>(&sg[jo & 1][b], &tp[jo & 1][s], acc[s][b]);
                // pin that order (left alone, the scheduler sinks every read
                // next to its first use and waits for it there)
                __builtin_amdgcn_sched_group_barrier(0x100, NB + TS, 0);   // DS read
                __builtin_amdgcn_sched_group_barrier(0x008, TS * NB, 0);   // MFMA
            };
            for (int q = 0; q < steps; q += 4) {
                step(q, 0);
                step(q, 1);
                step(q, 2);
                step(q, 3);
            }
        }
        if (more) {
            uint8_t* nxt = taps + ((ch + 1) & 1) * CB;
            toep_put(nxt, pre);
            lds_barrier();
#pragma unroll
            for (int s = 0; s < TS; ++s) tp[0][s] = *(const i32x4*)(nxt + (s * kToepChunkK * 8 + tu) * 16);
        }
    }
}

// Epilogue through LDS: half a 1024-frame block at a time, the wave writes its
// accumulators into its 2.5 KiB slice of `scr` and reads them back four
// consecutive frames per lane, so that one 16-byte store per lane covers
// 1 KiB of a row: 32 stores per wave for two scales and four blocks, against
// 128 of 4 bytes (a wave keeps at most 63 memory instructions in flight, so
// the 4-byte form waits for half of its own stores).  Frame f of the half
// block sits at float f + 16 (f / 64): a 16-lane read pass takes one 64-frame
// run (64 banks), and the two half-waves' writes (frames 128 apart) fall on
// opposite halves of the banks.
constexpr int kToepTrFloats = 512 + 16 * 8;
constexpr int kToepTrBytes = kMfmaWaves * kToepTrFloats * 4;
static_assert(kToepTrBytes <= kToepChunkUnits * 16, "the transposes fit one tap buffer");

template <int NB>
__device__ __forceinline__ void toep_store_tr(const MfmaArgs& a, const ClipArg& c, const ToepGroup* __restrict__ G,
                                              int64_t kw, const f32x16 (&acc)[kToepScales][NB], float* scr) {
    constexpr int TS = kToepScales;
    const int lane = threadIdx.x & 63;
    const int j = lane & 31, hg = lane >> 5;
    float* my = scr + (threadIdx.x >> 6) * kToepTrFloats;
    const float* rd = my + 4 * lane + 16 * (lane >> 4);
#pragma unroll
    for (int s = 0; s < TS; ++s) {
        const int row = G->rows[s];
        if (row < 0) continue;
        gfloat* __restrict__ orow = (gfloat*)c.out + (int64_t)row * c.K;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
                for (int vv = 0; vv < 8; ++vv) {
                    const int v = 8 * hh + vv;
                    const int f = 32 * (8 * (v >> 2) + 4 * hg + (v & 3) - 16 * hh) + j;
                    const float val = acc[s][b][v];
                    my[f + 16 * (f >> 6)] = a.signed_out ? val : fabsf(val);
                }
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const f32x4 o = *(const f32x4*)(rd + 320 * g);
                    const int64_t k = kw + 1024 * b + 512 * hh + 256 * g + 4 * lane;
                    gfloat* dst = orow + k;
                    if (k + 3 < c.K && (((uintptr_t)dst) & 15) == 0) {
                        __builtin_nontemporal_store(o, (gf32x4*)dst);
                    } else {
                        if (k < c.K) __builtin_nontemporal_store(o[0], dst);
                        if (k + 1 < c.K) __builtin_nontemporal_store(o[1], dst + 1);
                        if (k + 2 < c.K) __builtin_nontemporal_store(o[2], dst + 2);
                        if (k + 3 < c.K) __builtin_nontemporal_store(o[3], dst + 3);
                    }
                }
            }
        }
    }
}

// One scale group over the wave's frames: the K loop, then (once every wave
// is done with the tap buffers) the epilogue through tap buffer 1.
template <int DT, int NB>
__device__ __forceinline__ void toep_group(const MfmaArgs& a, const ClipArg& c, const ToepGroup* __restrict__ G,
                                           int64_t kw, int ubase, bool active, const uint8_t* win, uint8_t* taps) {
    f32x16 acc[kToepScales][NB];
    toep_loop<DT, NB>(a, G, ubase, active, win, taps, acc);
    lds_barrier();
    if (active) toep_store_tr<NB>(a, c, G, kw, acc, (float*)(taps + kToepChunkUnits * 16));
}

// Stage a tile starting at frame k0 for group G0 (and a narrower G1 run
// after it over the same window): the window of its signal and chunk 0 of
// G0's taps, into LDS (no barrier).  R: window units per thread in flight.
template <int DT, int NB, int R = 4>
__device__ __forceinline__ void toep_tile_stage(const MfmaArgs& a, const ClipArg& c, int64_t k0,
                                                const ToepGroup* __restrict__ G0, const ToepGroup* __restrict__ G1,
                                                uint8_t* lds) {
    const bool al16 = (((uintptr_t)c.x) & 15) == 0;
    i32x4 pre[kToepFetch];
    toep_fetch(a, G0, 0, pre);
    // the window starts at g0's jb; g1 (narrower: jb1 >= jb0) reads it from
    // an offset of (jb1 - jb0) / 8 units, its steps reaching up to 3 units
    // past g0's (toep_window_units)
    toep_stage<DT, R>(c, k0 + G0->jb, toep_window_units(NB, G0->jb, G0->D, G1 ? G1->jb : G0->jb, G1 ? G1->D : 0),
                      al16, lds + kToepTapBytes);
    toep_put(lds, pre);
}

// One Toeplitz work-group tile: frames tile * 4096 NB .. of one clip against
// one scale group, or two (g1 >= 0) run one after the other over one staged
// window (sized for the wider, g0).  Every wave of the work-group runs to the
// end (the tap chunks take all four to load and to pass their barriers).
template <int DT, int NB>
__device__ __forceinline__ void process_tile_toep(const MfmaArgs& a, const ClipArg& c, int tile, int g0, int g1,
                                                  uint8_t* lds) {
    static_assert(DT == DT_BF16 || DT == DT_FP16, "Toeplitz tiles hold 16-bit operands");
    constexpr int FW = 1024 * NB;   // frames per wave
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const ToepGroup* __restrict__ G0 = a.tgroups + g0;
    const ToepGroup* __restrict__ G1 = g1 >= 0 ? a.tgroups + g1 : nullptr;
    const int64_t k0 = (int64_t)tile * (kMfmaWaves * FW);
    uint8_t* taps = lds;
    uint8_t* win = lds + kToepTapBytes;
    toep_tile_stage<DT, NB>(a, c, k0, G0, G1, lds);
    lds_barrier();
    const int64_t kw = k0 + (int64_t)w * FW;
    const bool active = kw < c.K;   // the clip ends before this wave's frames
    const int ubase = (w * FW) / 8 + 4 * (lane & 31) + (lane >> 5);
    toep_group<DT, NB>(a, c, G0, kw, ubase, active, win, taps);
    if (G1) {
        lds_barrier();   // every wave is done with g0's tap buffers
        i32x4 pre[kToepFetch];
        toep_fetch(a, G1, 0, pre);
        toep_put(taps, pre);
        lds_barrier();
        toep_group<DT, NB>(a, c, G1, kw, ubase + (G1->jb - G0->jb) / 8, active, win, taps);
    }
}

// Work-group id -> (frame tile, scale groups).  With bundles (bg = 2) a
// work-group runs group ng-1-u and group u (u < ng/2) over one window: the
// widest with the narrowest, so every work-group carries about the same K
// steps.  Work-groups are dealt to the 8 XCDs round-robin; when the unit count
// (groups, or bundles) is a multiple of 8, XCD x takes every eighth unit
// (snake order over the groups, so the XCDs' K ranges balance), each over all
// its frame tiles: a group's tap fragments then stay in one XCD's L2.  Groups
// are stored narrowest first; single groups run widest first.
__device__ __forceinline__ void toep_unit(int id, int ntg, int bg, int ntile, int* g0, int* g1, int* tile) {
    const int nu = bg == 2 ? (ntg + 1) / 2 : ntg;   // units
    int u;
    if ((nu & 7) == 0) {
        const int x = id & 7, slot = id >> 3;
        const int oct = nu / 8 - 1 - slot / ntile;   // last octet first
        *tile = slot % ntile;
        u = 8 * oct + ((oct & 1) ? 7 - x : x);
    } else {
        u = nu - 1 - id / ntile;
        *tile = id % ntile;
    }
    if (bg == 2) {
        *g0 = ntg - 1 - u;
        *g1 = u < ntg - 1 - u ? u : -1;
    } else {
        *g0 = u;
        *g1 = -1;
    }
}

__device__ __forceinline__ int xcd_remap(int id, int n) {
    // Work-groups are dealt to the 8 XCDs round-robin; give each XCD a
    // contiguous range of tiles so neighbouring tiles share its L2.
    int q = n >> 3, r = n & 7;
    int xcd = id & 7, slot = id >> 3;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

template <int DT, int A>
__global__ __launch_bounds__(256) void k_mfma_grid(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ float red[kMfmaWaves];
    int id = blockIdx.x;
    if (a.xcd_remap) id = xcd_remap(id, gridDim.x);
    const int tile = id / a.ngroups, blk = id - tile * a.ngroups;
    process_tile<DT, A>(a, a.clip, tile, blk, lds, red);
}

template <int DT>
__global__ __launch_bounds__(256) void k_mfma_split(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ float red[kMfmaWaves];
    int id = blockIdx.x;
    if (a.xcd_remap) id = xcd_remap(id, gridDim.x);
    const int ng = (a.ngroups + a.split_wb - 1) / a.split_wb;
    const int tile = id / ng, grp = id - tile * ng;
    process_tile_split<DT>(a, a.clip, tile, grp, lds, red);
}

template <int DT, int A>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WinOcc<DT, A>::W)))
void k_mfma_win(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ float red[kMfmaWaves];
    int id = blockIdx.x;
    if (a.xcd_remap) id = xcd_remap(id, gridDim.x);
    const int ng = (a.ngroups + a.clip.wb - 1) / a.clip.wb;
    const int tile = id / ng, grp = id - tile * ng;
    process_tile_win<DT, A>(a, a.clip, tile, grp, lds, red);
}

// Toeplitz tiles of one clip: grid = scale groups x frame tiles.
template <int DT, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_toep(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    int g0, g1, tile;
    toep_unit(blockIdx.x, a.ntgroups, a.toep_bg, a.clip.ntile, &g0, &g1, &tile);
    process_tile_toep<DT, NB>(a, a.clip, tile, g0, g1, lds);
}

// Toeplitz tiles of a batch of hop-1 clips in one grid.  The frame tiles of
// all clips form one sequence (clip c's start at tile_prefix[c] / ntgroups)
// and work-group ids map to (group, tile) as for one clip over that
// sequence: the widest groups first across all clips, each XCD one group in
// eight.  One launch then pays one tail for all its clips, where separate
// launches each wait for their own widest groups' last work items.
template <int DT, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_toep_batch(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int ntg = a.ntgroups;
    int g0, g1, t;
    toep_unit(blockIdx.x, ntg, 1, a.total_tiles / ntg, &g0, &g1, &t);
    int lo = 0, hi = a.nclips - 1;   // last clip c with tile_prefix[c] / ntg <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.tile_prefix[mid] / ntg <= t) lo = mid; else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const ClipArg c = a.clips[lo];
    process_tile_toep<DT, NB>(a, c, t - a.tile_prefix[lo] / ntg, g0, -1, lds);
}

// Persistent batch kernel: work-group g takes tiles g, g + G, g + 2G, ...
// (G = gridDim.x, every work-group resident) with no atomics; the host picks G
// coprime with the number of block groups so that a work-group's tiles rotate
// through the groups (whose K ranges differ).  The clip of tile t is the last
// c with tile_prefix[c] <= t, searched in an LDS copy of the prefix table when
// it fits.  ANY = 0 is the variant for batches whose clips all use WIN tiles
// (compiled for the WIN register budget); ANY = 1 handles every layout.
constexpr int kPrefixLds = 1024;

template <int DT, int A, int ANY>
__device__ __forceinline__ void persistent_body(const MfmaArgs& a, uint8_t* lds, float* red, int* spre) {
    const bool in_lds = a.nclips + 1 <= kPrefixLds;
    if (in_lds) {
        for (int i = threadIdx.x; i <= a.nclips; i += 256) spre[i] = a.tile_prefix[i];
        __syncthreads();
    }
    for (int t = blockIdx.x; t < a.total_tiles; t += gridDim.x) {
        int lo = 0, hi = a.nclips - 1;         // last clip c with tile_prefix[c] <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            const int pm = in_lds ? spre[mid] : a.tile_prefix[mid];
            if (pm <= t) lo = mid; else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);   // uniform: the descriptor stays scalar
        const int local = t - (in_lds ? spre[lo] : a.tile_prefix[lo]);
        const ClipArg c = a.clips[lo];
        if constexpr (ANY) {
            if constexpr (DT == DT_BF16 || DT == DT_FP16) {
                if (c.mode == STAGE_TOEP) {
                    int g0, g1, tile;
                    toep_unit(local, a.ntgroups, a.toep_bg, c.ntile, &g0, &g1, &tile);
                    process_tile_toep<DT, kToepBatchNB>(a, c, tile, g0, g1, lds);
                    lds_barrier();
                    continue;
                }
            }
            if (c.mode == STAGE_LINEAR) {
                const int tile = local / a.ngroups, blk = local - tile * a.ngroups;
                process_tile<DT, A>(a, c, tile, blk, lds, red);
                lds_barrier();
                continue;
            }
            if (c.mode == STAGE_ROWS) {
                const int ng = (a.ngroups + a.split_wb - 1) / a.split_wb;
                const int tile = local / ng, grp = local - tile * ng;
                process_tile_split<DT>(a, c, tile, grp, lds, red);
                lds_barrier();
                continue;
            }
        }
        {
            const int ng = (a.ngroups + c.wb - 1) / c.wb;
            const int tile = local / ng, grp = local - tile * ng;
            process_tile_win<DT, A>(a, c, tile, grp, lds, red);
        }
        lds_barrier();                          // LDS free for the next tile
    }
}

// The every-layout kernel holds the chunked and row tiles' state beside the
// WIN tile's: two waves per SIMD for BF16/FP16 up to A = 2 (it serves mixed
// batches such as a hop-1 request among larger hops), one otherwise.
template <int DT, int A>
struct AnyOcc {
    static constexpr int W = (DT == DT_BF16 || DT == DT_FP16) && A <= 2 ? 2 : 1;
};

template <int DT, int A>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AnyOcc<DT, A>::W)))
void k_mfma_persistent(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ float red[kMfmaWaves];
    __shared__ int spre[kPrefixLds];
    persistent_body<DT, A, 1>(a, lds, red, spre);
}

template <int DT, int A>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WinOcc<DT, A>::W)))
void k_mfma_persistent_win(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ float red[kMfmaWaves];
    __shared__ int spre[kPrefixLds];
    persistent_body<DT, A, 0>(a, lds, red, spre);
}

// Dynamic LDS limit: a CU's 160 KiB less room for the static arrays (prefix
// table, reductions).
static int dyn_lds_max() { return mfma_max_lds_bytes() - 8192; }

// A = 8 (256 frames per wave) exists for the WIN kernels of the 2-byte types only.
template <int DT, int A>
constexpr bool kWinOnly = A == 8;
template <int DT, int A>
constexpr bool kHasA = A != 8 || DT == DT_BF16 || DT == DT_FP16;

template <int DT, int A>
static hipError_t launch2(const MfmaArgs& a, int persistent, int grid, hipStream_t s) {
    const size_t shm = (size_t)a.shm_bytes;
    if (shm > (size_t)dyn_lds_max()) return hipErrorInvalidValue;
    if constexpr (!kHasA<DT, A>) {
        return hipErrorInvalidValue;
    } else {
        const bool win = persistent == 2 || (!persistent && a.clip.mode == STAGE_WIN);
        if (kWinOnly<DT, A> && !win) return hipErrorInvalidValue;
        (void)hipGetLastError();   // report only this launch's error
        if (persistent == 2) {
            hipLaunchKernelGGL((k_mfma_persistent_win<DT, A>), dim3(grid), dim3(256), shm, s, a);
        } else if (win) {
            hipLaunchKernelGGL((k_mfma_win<DT, A>), dim3(grid), dim3(256), shm, s, a);
        } else if constexpr (!kWinOnly<DT, A>) {
            if (persistent)
                hipLaunchKernelGGL((k_mfma_persistent<DT, A>), dim3(grid), dim3(256), shm, s, a);
            else if (a.clip.mode == STAGE_ROWS)
                hipLaunchKernelGGL((k_mfma_split<DT>), dim3(grid), dim3(256), shm, s, a);
            else
                hipLaunchKernelGGL((k_mfma_grid<DT, A>), dim3(grid), dim3(256), shm, s, a);
        }
        return hipGetLastError();
    }
}

template <int DT, int A>
static hipError_t attrs2() {
    const int lds = dyn_lds_max();
    if constexpr (!kHasA<DT, A>) {
        return hipSuccess;
    } else if constexpr (kWinOnly<DT, A>) {
        const void* fns[2] = {(const void*)k_mfma_win<DT, A>, (const void*)k_mfma_persistent_win<DT, A>};
        for (const void* fn : fns) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    } else {
        const void* fns[5] = {(const void*)k_mfma_persistent<DT, A>, (const void*)k_mfma_grid<DT, A>,
                              (const void*)k_mfma_split<DT>, (const void*)k_mfma_win<DT, A>,
                              (const void*)k_mfma_persistent_win<DT, A>};
        for (const void* fn : fns) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
}

template <int DT>
static hipError_t attrs1() {
    hipError_t e = attrs2<DT, 1>();
    if (e == hipSuccess) e = attrs2<DT, 2>();
    if (e == hipSuccess) e = attrs2<DT, 4>();
    if (e == hipSuccess) e = attrs2<DT, 8>();
    return e;
}

template <int DT, int NB>
static hipError_t toep_attr() {
    return hipFuncSetAttribute((const void*)k_toep<DT, NB>, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_lds_max());
}

hipError_t mfma_init_attributes() {
    hipError_t e = hipSuccess;
    for (const void* fn : {(const void*)k_toep_batch<DT_BF16, 1>, (const void*)k_toep_batch<DT_BF16, 2>,
                           (const void*)k_toep_batch<DT_BF16, 4>, (const void*)k_toep_batch<DT_FP16, 1>,
                           (const void*)k_toep_batch<DT_FP16, 2>, (const void*)k_toep_batch<DT_FP16, 4>})
        if (e == hipSuccess) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_lds_max());
    if (e == hipSuccess) e = toep_attr<DT_BF16, 1>();
    if (e == hipSuccess) e = toep_attr<DT_BF16, 2>();
    if (e == hipSuccess) e = toep_attr<DT_BF16, 4>();
    if (e == hipSuccess) e = toep_attr<DT_FP16, 1>();
    if (e == hipSuccess) e = toep_attr<DT_FP16, 2>();
    if (e == hipSuccess) e = toep_attr<DT_FP16, 4>();
    if (e == hipSuccess) e = attrs1<DT_BF16>();
    if (e == hipSuccess) e = attrs1<DT_FP16>();
    if (e == hipSuccess) e = attrs1<DT_BF16X3>();
    if (e == hipSuccess) e = attrs1<DT_FP8>();
    return e;
}

template <int DT>
static hipError_t launch1(int A, const MfmaArgs& a, int persistent, int grid, hipStream_t s) {
    switch (A) {
        case 1: return launch2<DT, 1>(a, persistent, grid, s);
        case 2: return launch2<DT, 2>(a, persistent, grid, s);
        case 4: return launch2<DT, 4>(a, persistent, grid, s);
        case 8: return launch2<DT, 8>(a, persistent, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mfma(int dt, int A, int, const MfmaArgs& a, int persistent, int grid, hipStream_t s) {
    switch (dt) {
        case DT_BF16: return launch1<DT_BF16>(A, a, persistent, grid, s);
        case DT_FP16: return launch1<DT_FP16>(A, a, persistent, grid, s);
        case DT_BF16X3: return launch1<DT_BF16X3>(A, a, persistent, grid, s);
        case DT_FP8: return launch1<DT_FP8>(A, a, persistent, grid, s);
        default: return hipErrorInvalidValue;
    }
}

int mfma_max_lds_bytes() { return 160 * 1024; }

template <int DT, int NB>
static hipError_t launch_toep2(const MfmaArgs& a, int grid, hipStream_t s) {
    if ((size_t)a.shm_bytes > (size_t)dyn_lds_max()) return hipErrorInvalidValue;
    (void)hipGetLastError();
    hipLaunchKernelGGL((k_toep<DT, NB>), dim3(grid), dim3(256), (size_t)a.shm_bytes, s, a);
    return hipGetLastError();
}

template <int DT>
static hipError_t launch_toep1(int NB, const MfmaArgs& a, int grid, hipStream_t s) {
    switch (NB) {
        case 1: return launch_toep2<DT, 1>(a, grid, s);
        case 2: return launch_toep2<DT, 2>(a, grid, s);
        case 4: return launch_toep2<DT, 4>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <int DT>
static void launch_toep_batch1(int NB, const MfmaArgs& a, int grid, hipStream_t s) {
    const size_t shm = (size_t)a.shm_bytes;
    if (NB == 4)
        hipLaunchKernelGGL((k_toep_batch<DT, 4>), dim3(grid), dim3(256), shm, s, a);
    else if (NB == 2)
        hipLaunchKernelGGL((k_toep_batch<DT, 2>), dim3(grid), dim3(256), shm, s, a);
    else
        hipLaunchKernelGGL((k_toep_batch<DT, 1>), dim3(grid), dim3(256), shm, s, a);
}

hipError_t launch_toep_batch(int dt, int NB, const MfmaArgs& a, int grid, hipStream_t s) {
    if ((size_t)a.shm_bytes > (size_t)dyn_lds_max() || grid <= 0 || a.ntgroups <= 0) return hipErrorInvalidValue;
    if (NB != 1 && NB != 2 && NB != 4) return hipErrorInvalidValue;
    (void)hipGetLastError();
    if (dt == DT_BF16)
        launch_toep_batch1<DT_BF16>(NB, a, grid, s);
    else if (dt == DT_FP16)
        launch_toep_batch1<DT_FP16>(NB, a, grid, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_toep(int dt, int NB, const MfmaArgs& a, int grid, hipStream_t s) {
    switch (dt) {
        case DT_BF16: return launch_toep1<DT_BF16>(NB, a, grid, s);
        case DT_FP16: return launch_toep1<DT_FP16>(NB, a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <int DT, int NB>
static int toep_occ2(size_t shm) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)k_toep<DT, NB>, 256, shm) != hipSuccess) return 1;
    return n;
}

int toep_occupancy(int dt, int NB, size_t shm) {
    if (dt != DT_BF16 && dt != DT_FP16) return 1;
    const bool h = dt == DT_FP16;
    switch (NB) {
        case 1: return h ? toep_occ2<DT_FP16, 1>(shm) : toep_occ2<DT_BF16, 1>(shm);
        case 2: return h ? toep_occ2<DT_FP16, 2>(shm) : toep_occ2<DT_BF16, 2>(shm);
        default: return h ? toep_occ2<DT_FP16, 4>(shm) : toep_occ2<DT_BF16, 4>(shm);
    }
}

template <int DT, int A>
static int occ2(int persistent, size_t shm) {
    if constexpr (!kHasA<DT, A>) {
        return 1;
    } else {
        int n = 0;
        const void* fn = persistent == 2 ? (const void*)k_mfma_persistent_win<DT, A> : (const void*)k_mfma_win<DT, A>;
        if constexpr (!kWinOnly<DT, A>)
            if (persistent == 1) fn = (const void*)k_mfma_persistent<DT, A>;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 256, shm) != hipSuccess) return 1;
        return n;
    }
}
template <int DT>
static int occ1(int A, int persistent, size_t shm) {
    switch (A) {
        case 1: return occ2<DT, 1>(persistent, shm);
        case 2: return occ2<DT, 2>(persistent, shm);
        case 4: return occ2<DT, 4>(persistent, shm);
        default: return occ2<DT, 8>(persistent, shm);
    }
}
int mfma_occupancy(int dt, int A, int, int persistent, size_t shm) {
    switch (dt) {
        case DT_BF16: return occ1<DT_BF16>(A, persistent, shm);
        case DT_FP16: return occ1<DT_FP16>(A, persistent, shm);
        case DT_BF16X3: return occ1<DT_BF16X3>(A, persistent, shm);
        case DT_FP8: return occ1<DT_FP8>(A, persistent, shm);
        default: return 1;
    }
}

}  // namespace cwth
