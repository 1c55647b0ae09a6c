// Strided-frame contraction on the matrix cores (gfx950 MFMA).
//
// For one work-group tile (F consecutive frames k0 .. k0+F-1 of one clip, and
// one group of up to four 32-scale blocks) it computes
//     W[i][k] = sum_m t_i[m] * x~[k*hop + m]          (Eq. (1), Sec. II-A/II-B)
// as C[32 scales x 32 frames] += T[32 x KS] * X[KS x 32] per MFMA, where
//     T[r][kk] = t_r[KS*ks + kk]                (bank fragment, L2 resident)
//     X[kk][n] = x~[(k0+n)*hop + KS*ks + kk]    (Hankel view of the signal, LDS)
// with KS = 16 (BF16/FP16: v_mfma_f32_32x32x16_*) or 64 (FP8:
// v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales).  Accumulation is FP32.
//
// Signal staging.  The taps are walked in chunks of `chunk_steps` K-steps.  For
// each chunk the work-group converts the needed samples (zero outside
// [0, len)) to the operand type and writes them to one of two LDS buffers
// while the other buffer feeds the MFMAs.  Two layouts:
//   LINEAR  the window x~[k0*hop + KS*ks_c + p], p = 0 .. (F-1)*hop + KS*chunk,
//           kept in `copies` copies shifted by multiples of gcd(hop, U) so every
//           lane's 16-byte read is aligned (U = elements per 16 bytes); for
//           power-of-two hops an XOR swizzle of the 16-byte unit index spreads
//           the frame-strided reads over the LDS banks.
//   ROWS    one padded row per frame holding x~[(k0+f)*hop + KS*ks_c + c]; used
//           when the frames are so far apart that the linear window would be
//           larger.
// Summation order per coefficient: K-steps ascending, fixed per block, so the
// result does not depend on the tile, the launch shape or the batch.
#include "cwt_internal.h"

namespace cwth {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

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

// Convert U consecutive float samples into one 16-byte unit per plane.
template <int DT>
__device__ __forceinline__ void pack_unit(const float* v, float beta, i32x4* out) {
    if constexpr (DT == DT_BF16 || DT == DT_BF16X3) {
        bf16x8 h;
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = (__bf16)v[e];
        out[0] = __builtin_bit_cast(i32x4, h);
        if constexpr (DT == DT_BF16X3) {
            bf16x8 l;
#pragma unroll
            for (int e = 0; e < 8; ++e) l[e] = (__bf16)(v[e] - (float)h[e]);  // exact residual
            out[1] = __builtin_bit_cast(i32x4, l);
        }
    } else if constexpr (DT == DT_FP16) {
        f16x8 h;
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = (_Float16)v[e];
        out[0] = __builtin_bit_cast(i32x4, h);
    } else {
        i32x4 r;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            int word = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * w] * beta, v[4 * w + 1] * beta, 0, false);
            word = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * w + 2] * beta, v[4 * w + 3] * beta, word, true);
            r[w] = word;
        }
        out[0] = r;
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
    if (g.mode == STAGE_LINEAR) {
        int pmax = (F - 1) * c.hop + T::KS * chunk - 1;
        g.len_u = ((pmax / T::U + 1) + 15) & ~15;
        g.cs = g.len_u + (g.copies > 1 ? 16 / g.copies : 0);
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

// Stage chunk (first K-step ks_c) into LDS buffer `buf`.
template <int DT>
__device__ __forceinline__ void stage_chunk(const ClipArg& c, const Geo& g, int F, int chunk,
                                            int64_t k0, int ks_c, float beta, bool aligned16,
                                            uint8_t* buf) {
    using T = Tr<DT>;
    const float* __restrict__ x = c.x;
    const int64_t len = c.len;
    const int tid = threadIdx.x;
    int total;
    int per_row = T::KS * chunk / T::U;   // rows mode: units per row
    if (g.mode == STAGE_LINEAR) total = g.copies * g.len_u;
    else total = F * per_row;
    for (int q = tid; q < total; q += kMfmaWaves * kWaveSize) {
        int64_t j;
        int dst_unit;
        if (g.mode == STAGE_LINEAR) {
            int cp = q / g.len_u, uu = q - cp * g.len_u;
            j = k0 * c.hop + (int64_t)T::KS * ks_c + cp * g.gh + uu * T::U;
            dst_unit = cp * g.cs + swizzle(uu, g.swz);
        } else {
            int f = q / per_row, cu = q - f * per_row;
            j = (k0 + f) * c.hop + (int64_t)T::KS * ks_c + cu * T::U;
            dst_unit = f * g.rs + cu;
        }
        float v[T::U];
        if (j >= 0 && j + T::U <= len && aligned16 && (j & 3) == 0) {
#pragma unroll
            for (int e = 0; e < T::U; e += 4) {
                float4 f4 = *(const float4*)(x + j + e);
                v[e] = f4.x; v[e + 1] = f4.y; v[e + 2] = f4.z; v[e + 3] = f4.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < T::U; ++e) {
                int64_t jj = j + e;
                v[e] = (jj >= 0 && jj < len) ? x[jj] : 0.0f;
            }
        }
        i32x4 pk[T::PLANES];
        pack_unit<DT>(v, beta, pk);
#pragma unroll
        for (int p = 0; p < T::PLANES; ++p)
            *(i32x4*)(buf + p * g.plane_bytes + dst_unit * 16) = pk[p];
    }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Power-of-two signal scale beta = 2^floor(log2(448 / max|x~|)), the maximum
// taken over exactly the samples the tile's frames touch (the union of the
// windows [(k0+f)*hop + KS*glo, (k0+f)*hop + KS*(ghi+1)) ), so beta depends only
// on the tile's frame range and the scale group, never on the staging layout.
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
    return (float)ldexp(1.0, e - 1);
}

template <int DT, int A, int NB>
__device__ __forceinline__ void process_tile(const MfmaArgs& a, const ClipArg& c, int tile, int grp,
                                             uint8_t* lds, float* red) {
    using T = Tr<DT>;
    const int F = 32 * A * kMfmaWaves;
    const int chunk = a.chunk_steps;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int n = lane & 31, hg = lane >> 5;
    const int64_t k0 = (int64_t)tile * F;

    const MfmaGroup G = a.groups[grp];
    int lo[NB], hi[NB];
    int64_t foff[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b < G.nblk) {
            const MfmaBlock& B = a.blocks[G.blk[b]];
            lo[b] = B.lo; hi[b] = B.hi; foff[b] = B.frag_off;
        } else {
            lo[b] = 1; hi[b] = 0; foff[b] = 0;   // empty range: never active
        }
    }
    const Geo g = make_geo<DT>(c, F, chunk);
    const bool aligned16 = (((uintptr_t)c.x) & 15) == 0;
    float beta = 1.0f;
    if constexpr (DT == DT_FP8) beta = tile_beta<DT>(c, F, k0, G.lo, G.hi, red);

    f32x16 acc[A][NB];
#pragma unroll
    for (int fa = 0; fa < A; ++fa)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[fa][b][v] = 0.0f;

    const int nchunks = (G.hi - G.lo + chunk) / chunk;
    uint8_t* bufs[2] = {lds, lds + a.buf_bytes};
    stage_chunk<DT>(c, g, F, chunk, k0, G.lo, beta, aligned16, bufs[0]);
    __syncthreads();
    for (int ci = 0; ci < nchunks; ++ci) {
        const int ks_c = G.lo + ci * chunk;
        uint8_t* cur = bufs[ci & 1];
        if (ci + 1 < nchunks)
            stage_chunk<DT>(c, g, F, chunk, k0, ks_c + chunk, beta, aligned16, bufs[(ci + 1) & 1]);
        const int ks_end = min(ks_c + chunk - 1, G.hi);
        // Per-lane LDS byte offset (copy or row) and first 16-byte unit at ks = ks_c.
        int base[A], unit0[A];
#pragma unroll
        for (int fa = 0; fa < A; ++fa) {
            const int f = 32 * (A * w + fa) + n;
            if (g.mode == STAGE_LINEAR) {
                const int p = f * c.hop + hg * T::PER;
                base[fa] = ((p % T::U) / g.gh) * g.cs * 16;
                unit0[fa] = p / T::U;
            } else {
                base[fa] = (f * g.rs + hg * T::LU) * 16;
                unit0[fa] = 0;
            }
        }
        for (int ks = ks_c; ks <= ks_end; ++ks) {
            const int d = ks - ks_c;
            Frag<DT> xf[A];
#pragma unroll
            for (int fa = 0; fa < A; ++fa) {
#pragma unroll
                for (int t = 0; t < T::LU; ++t) {
                    int off;
                    if (g.mode == STAGE_LINEAR) {
                        int unit = unit0[fa] + d * (T::KS / T::U) + t;
                        off = base[fa] + swizzle(unit, g.swz) * 16;
                    } else {
                        off = base[fa] + (d * (T::KS / T::U) + t) * 16;
                    }
#pragma unroll
                    for (int p = 0; p < T::PLANES; ++p)
                        xf[fa].u[p][t] = *(const i32x4*)(cur + p * g.plane_bytes + off);
                }
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (ks >= lo[b] && ks <= hi[b]) {
                    const uint8_t* tp = a.frags + foff[b] + (int64_t)(ks - lo[b]) * T::STEP + lane * T::FRAG;
                    Frag<DT> tf;
#pragma unroll
                    for (int p = 0; p < T::PLANES; ++p)
#pragma unroll
                        for (int t = 0; t < T::LU; ++t)
                            tf.u[p][t] = *((const i32x4*)(tp + p * 64 * T::FRAG) + t);
#pragma unroll
                    for (int fa = 0; fa < A; ++fa) acc[fa][b] = mma_all<DT>(tf, xf[fa], acc[fa][b]);
                }
            }
        }
        __syncthreads();
    }

    // Epilogue: optional descale (FP8), |.| unless signed output, coalesced store.
    const float inv_beta = 1.0f / beta;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= G.nblk) continue;
        const MfmaBlock& B = a.blocks[G.blk[b]];
#pragma unroll
        for (int fa = 0; fa < A; ++fa) {
            const int64_t k = k0 + 32 * (A * w + fa) + n;
            if (k >= c.K) continue;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                int r = 8 * (v >> 2) + 4 * hg + (v & 3);
                int row = B.rows[r];
                if (row < 0) continue;
                float val = acc[fa][b][v];
                if constexpr (DT == DT_FP8) val = val * (B.inv_alpha[r] * inv_beta);
                if (!a.signed_out) val = fabsf(val);
                __builtin_nontemporal_store(val, c.out + (int64_t)row * c.K + k);
            }
        }
    }
}

__device__ __forceinline__ int xcd_remap(int id, int n) {
    // Work-groups are dealt to the 8 XCDs round-robin; give each XCD a
    // contiguous range of tiles so neighbouring tiles share its L2.
    int q = n >> 3, r = n & 7;
    int xcd = id & 7, slot = id >> 3;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

template <int DT, int A, int NB>
__global__ __launch_bounds__(256) void k_mfma_grid(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ float red[kMfmaWaves];
    int id = blockIdx.x;
    if (a.xcd_remap) id = xcd_remap(id, gridDim.x);
    int tile = id / a.ngroups, grp = id - tile * a.ngroups;
    process_tile<DT, A, NB>(a, a.clip, tile, grp, lds, red);
}

template <int DT, int A, int NB>
__global__ __launch_bounds__(256) void k_mfma_persistent(MfmaArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ float red[kMfmaWaves];
    __shared__ int s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&a.counter[0], 1);
        __syncthreads();
        const int t = s_tile;
        __syncthreads();
        if (t >= a.total_tiles) break;
        int lo = 0, hi = a.nclips - 1;         // last clip c with tile_prefix[c] <= t
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (a.tile_prefix[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const int local = t - a.tile_prefix[lo];
        const int tile = local / a.ngroups, grp = local - tile * a.ngroups;
        const ClipArg c = a.clips[lo];
        process_tile<DT, A, NB>(a, c, tile, grp, lds, red);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        int done = atomicAdd(&a.counter[1], 1);
        if (done == (int)gridDim.x - 1) {      // last work-group out re-arms the counters
            atomicExch(&a.counter[0], 0);
            atomicExch(&a.counter[1], 0);
        }
    }
}

template <int DT, int A, int NB>
static hipError_t launch3(const MfmaArgs& a, int persistent, int grid, hipStream_t s) {
    const size_t shm = 2 * (size_t)a.buf_bytes;
    static bool attr_set[2] = {false, false};
    if (shm > 64 * 1024 && !attr_set[persistent]) {
        const void* fn = persistent ? (const void*)k_mfma_persistent<DT, A, NB>
                                    : (const void*)k_mfma_grid<DT, A, NB>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           mfma_max_lds_bytes() - 1024);
        if (e != hipSuccess) return e;
        attr_set[persistent] = true;
    }
    if (persistent)
        hipLaunchKernelGGL((k_mfma_persistent<DT, A, NB>), dim3(grid), dim3(256), shm, s, a);
    else
        hipLaunchKernelGGL((k_mfma_grid<DT, A, NB>), dim3(grid), dim3(256), shm, s, a);
    return hipGetLastError();
}

template <int DT, int A>
static hipError_t launch2(int nb, const MfmaArgs& a, int persistent, int grid, hipStream_t s) {
    if (nb <= 1) return launch3<DT, A, 1>(a, persistent, grid, s);
    if (nb <= 2) return launch3<DT, A, 2>(a, persistent, grid, s);
    return launch3<DT, A, 4>(a, persistent, grid, s);
}

template <int DT>
static hipError_t launch1(int A, int nb, const MfmaArgs& a, int persistent, int grid, hipStream_t s) {
    if (A == 1) return launch2<DT, 1>(nb, a, persistent, grid, s);
    if (A == 2) return launch2<DT, 2>(nb, a, persistent, grid, s);
    return launch2<DT, 4>(nb, a, persistent, grid, s);
}

hipError_t launch_mfma(int dt, int A, int nb, const MfmaArgs& a, int persistent, int grid,
                       hipStream_t s) {
    switch (dt) {
        case DT_BF16: return launch1<DT_BF16>(A, nb, a, persistent, grid, s);
        case DT_FP16: return launch1<DT_FP16>(A, nb, a, persistent, grid, s);
        case DT_BF16X3: return launch1<DT_BF16X3>(A, nb, a, persistent, grid, s);
        case DT_FP8: return launch1<DT_FP8>(A, nb, a, persistent, grid, s);
        default: return hipErrorInvalidValue;
    }
}

int mfma_max_lds_bytes() { return 160 * 1024; }

template <int DT, int A, int NB>
static int occ3(int persistent, size_t shm) {
    int n = 0;
    const void* fn = persistent ? (const void*)k_mfma_persistent<DT, A, NB>
                                : (const void*)k_mfma_grid<DT, A, NB>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 256, shm) != hipSuccess) return 1;
    return n;
}
template <int DT, int A>
static int occ2(int nb, int persistent, size_t shm) {
    if (nb <= 1) return occ3<DT, A, 1>(persistent, shm);
    if (nb <= 2) return occ3<DT, A, 2>(persistent, shm);
    return occ3<DT, A, 4>(persistent, shm);
}
template <int DT>
static int occ1(int A, int nb, int persistent, size_t shm) {
    if (A == 1) return occ2<DT, 1>(nb, persistent, shm);
    if (A == 2) return occ2<DT, 2>(nb, persistent, shm);
    return occ2<DT, 4>(nb, persistent, shm);
}
int mfma_occupancy(int dt, int A, int nb, int persistent, size_t shm) {
    switch (dt) {
        case DT_BF16: return occ1<DT_BF16>(A, nb, persistent, shm);
        case DT_FP16: return occ1<DT_FP16>(A, nb, persistent, shm);
        case DT_BF16X3: return occ1<DT_BF16X3>(A, nb, persistent, shm);
        case DT_FP8: return occ1<DT_FP8>(A, nb, persistent, shm);
        default: return 1;
    }
}

}  // namespace cwth
