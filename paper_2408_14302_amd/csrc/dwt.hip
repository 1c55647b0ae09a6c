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
// Long levels (input > kTailIn samples) run in groups of up to kMaxFused
// levels per launch (k_dwt_fused): a work-group owns T outputs of the
// group's deepest level, loads the input window they depend on
// (2^F T + (2^F - 1)(L - 2) samples) into LDS once and computes every level
// of the group there, writing its own coefficients and its own stretch of
// the group's matrix rows.  Work-groups whose window would run past the end
// of the level (where the periodic extension wraps to the start) are left
// out; one work-group per clip finishes those outputs (k_dwt_edge_tail),
// taking the wrapped values, which the fused launch has written, from the
// level record.  The same work-group then runs every remaining short level
// of the clip in LDS behind work-group barriers.  Level record stores are
// never read back by the launch that writes them, so barriers order LDS
// only.  A last kernel writes the
// matrix rows of the levels not written yet (k_dwt_expand).  Every
// coefficient is the same FP32 FMA chain in ascending k wherever it is
// computed, so the result depends neither on the grouping nor on alignment.
#include "cwt_internal.h"

namespace cwth {

namespace {

constexpr int kTailIn = 8192;      // longest level input the LDS tail takes
constexpr int kTailThreads = 1024;
constexpr int kMaxFused = 5;       // levels per fused launch
constexpr int kEdgeIn = 4096;      // longest edge window of a fused group's input level
constexpr int kEdgeExtra = 64;     // room for the wrapped extension of an edge window
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t level_len(int64_t len, int j) { return ((len - 1) >> j) + 1; }

// Work-group barrier that orders LDS only: the level record written between
// barriers is not read back by the launch that writes it, so its stores need
// not drain here.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// i mod P for 0 <= i < P + L: a subtraction or two (a few more only for
// levels shorter than the filter), where a 64-bit modulo would hold up the
// whole wave.
__device__ __forceinline__ int64_t wrap(int64_t i, int64_t P) {
    while (i >= P) i -= P;
    return i;
}

// The chain over a window w[0 .. L-1] that needs no index mapping.
template <int LT, typename Ptr>
__device__ __forceinline__ void chain(Ptr w, const DwtFilter& f, float& sa, float& sd) {
    const int L = LT > 0 ? LT : f.L;
    float pa = 0.0f, pd = 0.0f;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const float v = w[k];
        pa = fmaf(f.h[k], v, pa);
        pd = fmaf(f.g[k], v, pd);
    }
    sa = pa;
    sd = pd;
}

// The same chain from an 8-byte aligned LDS window, read as float2.
template <int LT>
__device__ __forceinline__ void chain2(const float* w, const DwtFilter& f, float& sa, float& sd) {
    const int L = LT > 0 ? LT : f.L;
    const float2* w2 = reinterpret_cast<const float2*>(w);
    float pa = 0.0f, pd = 0.0f;
#pragma unroll
    for (int k = 0; k < L / 2; ++k) {
        const float2 v = w2[k];
        pa = fmaf(f.h[2 * k], v.x, pa);
        pd = fmaf(f.g[2 * k], v.x, pd);
        pa = fmaf(f.h[2 * k + 1], v.y, pa);
        pd = fmaf(f.g[2 * k + 1], v.y, pd);
    }
    sa = pa;
    sd = pd;
}

// One (a, d) pair from level input `a` (len_in samples) at output n, with
// the index map where the window runs past the end.
template <int LT, typename Ptr>
__device__ __forceinline__ void dwt_pair(Ptr a, int64_t len_in, int64_t n, const DwtFilter& f, float& sa,
                                         float& sd) {
    const int L = LT > 0 ? LT : f.L;
    const int64_t i0 = 2 * n;
    if (i0 + L <= len_in) {
        chain<LT>(a + i0, f, sa, sd);
        return;
    }
    const int64_t P = len_in + (len_in & 1);
    float pa = 0.0f, pd = 0.0f;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        int64_t i = wrap(i0 + k, P);
        if (i > len_in - 1) i = len_in - 1;
        const float v = a[i];
        pa = fmaf(f.h[k], v, pa);
        pd = fmaf(f.g[k], v, pd);
    }
    sa = pa;
    sd = pd;
}

// Matrix row entries t .. t+3 (t a multiple of 4): va for t, t+1 and vb for
// t+2, t+3, clipped at len.
__device__ __forceinline__ void put4(float* row, int64_t t, int64_t len, float va, float vb, bool vec) {
    if (vec && t + 3 < len) {
        const f4 w = {va, va, vb, vb};
        __builtin_nontemporal_store(w, reinterpret_cast<f4*>(row + t));
    } else {
        const float v[4] = {va, va, vb, vb};
        for (int q = 0; q < 4 && t + q < len; ++q) row[t + q] = v[q];
    }
}

// One level for the whole batch, two outputs per lane: a long level that no
// fused group can take.
template <int LT>
__global__ __launch_bounds__(256) void k_dwt_level(const float* __restrict__ src, int64_t src_stride, int64_t len_in,
                                                   float* __restrict__ pyr, int64_t pyr_stride, int64_t off,
                                                   int64_t len_out, DwtFilter f) {
    const int64_t n = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
    if (n >= len_out) return;
    const int64_t c = blockIdx.y;
    const float* a = src + c * src_stride;
    float* p = pyr + c * pyr_stride + off;
    float sa, sd;
    dwt_pair<LT>(a, len_in, n, f, sa, sd);
    p[n] = sa;
    p[len_out + n] = sd;
    if (n + 1 < len_out) {
        dwt_pair<LT>(a, len_in, n + 1, f, sa, sd);
        p[n + 1] = sa;
        p[len_out + n + 1] = sd;
    }
}

struct FusedArgs {
    const float* src;    // level j0 - 1 of clip 0
    int64_t sstride;     // floats between clips in src
    int64_t len_in;      // len_{j0-1}
    float* pyr;
    int64_t pstride;
    int64_t off;         // offset of level j0 in the level record
    int64_t len;         // signal length (matrix row length)
    float* out;          // matrix or null
    int J;               // matrix rows
    int j0, F, T;        // first level, levels, deepest-level outputs per work-group
    bool vec_in, vec_out;
};

// Window of a tile r levels above the group's deepest level.
__host__ __device__ __forceinline__ int64_t win_len(int r, int T, int L) {
    return ((int64_t)T << r) + (((int64_t)1 << r) - 1) * (L - 2);
}

// Levels j0 .. j0+F-1 of one tile; grid (interior tiles, clips).
template <int LT>
__global__ __launch_bounds__(256) void k_dwt_fused(FusedArgs A, DwtFilter f) {
    extern __shared__ float lds[];
    const int L = LT > 0 ? LT : f.L;
    const int F = A.F, T = A.T;
    const int64_t RF = win_len(F, T, L);
    float* b0 = lds;                                   // windows are even lengths: float2 alignment holds
    float* b1 = lds + RF;
    float* ds = b1 + win_len(F - 1, T, L);             // |d| of the tile's own outputs, level by level
    const int64_t m0 = (int64_t)blockIdx.x * T;
    const int64_t c = blockIdx.y;
    const int tid = threadIdx.x;

    const float* a = A.src + c * A.sstride + (m0 << F);        // interior tile: the window lies inside the level
    if (A.vec_in) {
        const int64_t n4 = RF >> 2;
        for (int64_t i = tid; i < n4; i += 256) {
            const float4 v = reinterpret_cast<const float4*>(a)[i];
            b0[4 * i] = v.x;
            b0[4 * i + 1] = v.y;
            b0[4 * i + 2] = v.z;
            b0[4 * i + 3] = v.w;
        }
        for (int64_t i = 4 * n4 + tid; i < RF; i += 256) b0[i] = a[i];
    } else {
        for (int64_t i = tid; i < RF; i += 256) b0[i] = a[i];
    }
    lds_barrier();

    float* p = A.pyr + c * A.pstride;
    float* in = b0;
    float* nxt = b1;
    int64_t lin = A.len_in, off = A.off, dsoff = 0;
    for (int i = 0; i < F; ++i) {
        const int r = F - 1 - i;
        const int64_t R = win_len(r, T, L), own = (int64_t)T << r, s = m0 << r;
        const int64_t lout = (lin + 1) >> 1;
        for (int64_t q = tid; q < R; q += 256) {
            float sa, sd;
            chain2<LT>(in + 2 * q, f, sa, sd);
            nxt[q] = sa;
            if (q < own) {
                p[off + s + q] = sa;
                p[off + lout + s + q] = sd;
                ds[dsoff + q] = fabsf(sd);
            }
        }
        lds_barrier();
        float* t = in;
        in = nxt;
        nxt = t;
        dsoff += own;
        off += 2 * lout;
        lin = lout;
    }

    if (!A.out) return;
    const int j1 = A.j0 + F - 1;
    const int64_t t0 = m0 << j1, span = (int64_t)T << j1;
    dsoff = 0;
    for (int i = 0; i < F; ++i) {
        const int j = A.j0 + i, r = F - 1 - i;
        const int64_t s = m0 << r;
        float* row = A.out + (c * A.J + j - 1) * A.len;
        for (int64_t q = 4 * tid; q < span; q += 4 * 256) {
            const int64_t t = t0 + q;
            if (t >= A.len) break;
            put4(row, t, A.len, ds[dsoff + (t >> j) - s], ds[dsoff + ((t + 2) >> j) - s], A.vec_out);
        }
        dsoff += (int64_t)T << r;
    }
}

struct EdgeTailArgs {
    const float* src;    // level j0 - 1 of clip 0 (x or the level record)
    int64_t sstride;
    int64_t len_in;      // len_{j0-1}
    float* pyr;
    int64_t pstride;
    int64_t off;         // offset of level j0 in the level record
    int64_t len;
    float* out;          // matrix or null (edge stretches of the group's rows only)
    int J;               // last level of the transform
    int j0, j1;          // fused group whose edge is finished here (j1 < j0: none)
    int64_t e_in;        // first input sample of the edge ((interior tiles * T) << F)
    bool tail;           // then run levels j1 + 1 .. J in LDS
};

// One work-group per clip.  Everything it needs from memory is loaded in one
// round at the start (the edge window, the wrapped values of each edge
// level, the interior part of the tail's first input); after that the levels
// run from LDS, so no load ever waits behind the level record's stores.
template <int LT>
__global__ __launch_bounds__(kTailThreads) void k_dwt_edge_tail(EdgeTailArgs A, DwtFilter f) {
    __shared__ float tin[kTailIn];                        // the tail's first input level
    __shared__ float u[kEdgeIn + kEdgeIn / 2 + 3 * kEdgeExtra];   // edge windows, later the tail's second buffer
    __shared__ float extv[kMaxFused][kEdgeExtra];         // wrapped values of the edge levels
    float* e1 = u;
    float* e2 = u + kEdgeIn + kEdgeExtra;
    float* tb = u;
    const int L = LT > 0 ? LT : f.L;
    const int64_t c = blockIdx.x;
    const int tid = threadIdx.x;
    float* p = A.pyr + c * A.pstride;
    const float* s = A.src + c * A.sstride;
    int64_t lin = A.len_in, off = A.off;
    int j = A.j0;

    if (A.j1 >= A.j0) {
        {   // edge window of the group's input level
            const int64_t win = 2 * ((lin + 1) >> 1) + L - 2 - A.e_in;
            const int64_t P = lin + (lin & 1);
            for (int64_t i = tid; i < win; i += kTailThreads) {
                int64_t q = wrap(A.e_in + i, P);
                if (q > lin - 1) q = lin - 1;
                e1[i] = s[q];
            }
        }
        {   // per edge level: values past its end that wrap below its edge
            int64_t l = lin, o = off, e = A.e_in >> 1;
            for (int jj = A.j0; jj <= A.j1; ++jj) {
                const int64_t lo = (l + 1) >> 1;
                if (jj < A.j1) {
                    const int64_t ext = 2 * ((lo + 1) >> 1) + L - 2 - lo;
                    const int64_t P = lo + (lo & 1);
                    for (int64_t q = tid; q < ext; q += kTailThreads) {
                        int64_t m = wrap(lo + q, P);
                        if (m > lo - 1) m = lo - 1;
                        if (m < e) extv[jj - A.j0][q] = p[o + m];      // written by the fused launch
                    }
                } else if (A.tail) {
                    for (int64_t i = tid; i < e; i += kTailThreads) tin[i] = p[o + i];
                }
                o += 2 * lo;
                l = lo;
                e >>= 1;
            }
        }
        lds_barrier();
        int64_t e = A.e_in >> 1;
        float* in = e1;
        float* nxt = e2;
        for (; j <= A.j1; ++j) {
            const int64_t lout = (lin + 1) >> 1;
            const int64_t cnt = lout - e;
            const int64_t ext = (j < A.j1) ? 2 * ((lout + 1) >> 1) + L - 2 - lout : 0;
            const int64_t P = lout + (lout & 1);
            const bool last = j == A.j1 && A.tail;
            for (int64_t q = tid; q < cnt + ext; q += kTailThreads) {
                if (q < cnt) {
                    const int64_t n = e + q;
                    float sa, sd;
                    chain2<LT>(in + 2 * q, f, sa, sd);
                    nxt[q] = sa;
                    if (last) tin[n] = sa;
                    p[off + n] = sa;
                    p[off + lout + n] = sd;
                    if (A.out) {
                        float* row = A.out + (c * A.J + j - 1) * A.len;
                        const int64_t t_lo = n << j;
                        const int64_t t_hi = ((n + 1) << j) < A.len ? ((n + 1) << j) : A.len;
                        const float v = fabsf(sd);
                        for (int64_t t = t_lo; t < t_hi; ++t) row[t] = v;
                    }
                } else {
                    int64_t m = wrap(lout + (q - cnt), P);         // index this position maps to
                    if (m > lout - 1) m = lout - 1;
                    float v, unused;
                    if (m >= e)
                        chain2<LT>(in + 2 * (m - e), f, v, unused);  // the chain of output m
                    else
                        v = extv[j - A.j0][q - cnt];
                    nxt[q] = v;
                }
            }
            lds_barrier();
            float* t = in;
            in = nxt;
            nxt = t;
            off += 2 * lout;
            lin = lout;
            e >>= 1;
        }
    } else {
        if (!A.tail) return;
        for (int64_t i = tid; i < lin; i += kTailThreads) tin[i] = s[i];
        lds_barrier();
    }

    if (!A.tail || j > A.J) return;
    const int jt = j;
    for (; j <= A.J; ++j) {
        const bool even = ((j - jt) & 1) == 0;
        const float* in = even ? tin : tb;
        float* out = even ? tb : tin;
        const int64_t lout = (lin + 1) >> 1;
        for (int64_t n = tid; n < lout; n += kTailThreads) {
            float sa, sd;
            dwt_pair<LT>(in, lin, n, f, sa, sd);
            out[n] = sa;
            p[off + n] = sa;
            p[off + lout + n] = sd;
        }
        lds_barrier();
        off += 2 * lout;
        lin = lout;
    }
}

// S[c][j-1][t] = |d_j[t >> j]| for the rows in `mask` (bit j-1), four
// consecutive t per lane.
__global__ __launch_bounds__(256) void k_dwt_expand(const float* __restrict__ pyr, int64_t pyr_stride, int64_t len,
                                                    int J, uint32_t mask, float* __restrict__ out, bool vec) {
    const int64_t t0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (t0 >= len) return;
    const int64_t c = blockIdx.y;
    const float* p = pyr + c * pyr_stride;
    float* o = out + c * (int64_t)J * len;
    int64_t off = 0;
    for (int j = 1; j <= J; ++j) {
        const int64_t lj = level_len(len, j);
        if ((mask >> (j - 1)) & 1u) {
            const float* d = p + off + lj;
            const int64_t i1 = ((t0 + 2) >> j) < lj ? ((t0 + 2) >> j) : lj - 1;
            put4(o + (int64_t)(j - 1) * len, t0, len, fabsf(d[t0 >> j]), fabsf(d[i1]), vec);
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
static hipError_t launch_levels(const float* x, int64_t len, int clips, const DwtFilter& f, int J, float* pyr,
                                float* out, hipStream_t s) {
    const int L = f.L;
    const int64_t pstride = dwt_pyramid_length(len, J);
    const bool vec_out = out && (len % 4 == 0) && (reinterpret_cast<uintptr_t>(out) % 16 == 0);
    const float* src = x;
    int64_t sstride = len, lin = len, off = 0;
    int j = 1;
    uint32_t expand_mask = J >= 32 ? 0xffffffffu : ((1u << J) - 1u);
    bool tail_done = false;
    while (j <= J && lin > kTailIn) {
        int F = 0;
        for (int64_t l = lin; F < kMaxFused && j + F <= J && l > kTailIn; l = (l + 1) >> 1) ++F;
        // tile size: the smallest T (more work-groups, less LDS each, measured
        // fastest) whose recomputed halo, (2^F - 1)(L - 2) samples per
        // 2^F T, stays under about a quarter; larger ones next, then smaller,
        // taking the first whose edge fits the edge work-group
        const int64_t lout0 = (lin + 1) >> 1;
        static const int kOrder[3][3] = {{32, 64, 128}, {64, 128, 32}, {128, 64, 32}};
        const int pref = 4 * (L - 2) <= 32 ? 0 : (4 * (L - 2) <= 64 ? 1 : 2);
        int T = 0;
        int64_t W = 0, e_in = 0;
        for (int k = 0; k < 3 && T == 0; ++k) {
            const int cand = kOrder[pref][k];
            const int64_t RF = win_len(F, cand, L);
            if (lin < RF) continue;
            const int64_t w = (lin - RF) / ((int64_t)cand << F) + 1;
            const int64_t e = (w * cand) << F;
            if (2 * lout0 + L - 2 - e > kEdgeIn || w > 0x7fffffff) continue;
            T = cand;
            W = w;
            e_in = e;
        }
        if (T == 0) {
            const int64_t grid = (lout0 + 511) / 512;
            hipLaunchKernelGGL((k_dwt_level<LT>), dim3((unsigned)grid, (unsigned)clips), dim3(256), 0, s, src,
                               sstride, lin, pyr, pstride, off, lout0, f);
            src = pyr + off;
            sstride = pstride;
            off += 2 * lout0;
            lin = lout0;
            ++j;
            continue;
        }
        const FusedArgs fa{src, sstride, lin, pyr, pstride, off, len, out, J, j, F, T,
                           (sstride % 4 == 0) && (reinterpret_cast<uintptr_t>(src) % 16 == 0), vec_out};
        const size_t shm = sizeof(float) * (win_len(F, T, L) + win_len(F - 1, T, L) + (((int64_t)1 << F) - 1) * T);
        hipLaunchKernelGGL((k_dwt_fused<LT>), dim3((unsigned)W, (unsigned)clips), dim3(256), shm, s, fa, f);
        int64_t l = lin, o = off;               // o: offset of the group's deepest level
        for (int i = 0; i < F; ++i) {
            const int64_t lo = (l + 1) >> 1;
            if (i < F - 1) o += 2 * lo;
            l = lo;
        }
        const int j1 = j + F - 1;
        const bool tail = l <= kTailIn && j1 < J;
        const EdgeTailArgs ea{src, sstride, lin, pyr, pstride, off, len, out, J, j, j1, e_in, tail};
        hipLaunchKernelGGL((k_dwt_edge_tail<LT>), dim3((unsigned)clips), dim3(kTailThreads), 0, s, ea, f);
        for (int jj = j; jj <= j1; ++jj) expand_mask &= ~(1u << (jj - 1));
        tail_done = tail;
        src = pyr + o;
        sstride = pstride;
        off = o + 2 * l;
        lin = l;
        j = j1 + 1;
        if (tail) break;
    }
    if (j <= J && !tail_done) {
        const EdgeTailArgs ea{src, sstride, lin, pyr, pstride, off, len, out, J, j, j - 1, 0, true};
        hipLaunchKernelGGL((k_dwt_edge_tail<LT>), dim3((unsigned)clips), dim3(kTailThreads), 0, s, ea, f);
    }
    if (out && expand_mask) {
        const int64_t grid = (len + 1023) / 1024;
        hipLaunchKernelGGL(k_dwt_expand, dim3((unsigned)grid, (unsigned)clips), dim3(256), 0, s, pyr, pstride, len,
                           J, expand_mask, out, vec_out);
    }
    return hipGetLastError();
}

hipError_t launch_dwt(const float* x, int64_t len, int clips, const DwtFilter& f, int J, float* pyr,
                      float* out, hipStream_t s) {
    if (len <= 0 || clips <= 0 || J <= 0) return hipSuccess;
    switch (f.L) {      // the Daubechies lengths db1 .. db10 unrolled; any other even length generic
        case 2: return launch_levels<2>(x, len, clips, f, J, pyr, out, s);
        case 4: return launch_levels<4>(x, len, clips, f, J, pyr, out, s);
        case 6: return launch_levels<6>(x, len, clips, f, J, pyr, out, s);
        case 8: return launch_levels<8>(x, len, clips, f, J, pyr, out, s);
        case 10: return launch_levels<10>(x, len, clips, f, J, pyr, out, s);
        case 12: return launch_levels<12>(x, len, clips, f, J, pyr, out, s);
        case 14: return launch_levels<14>(x, len, clips, f, J, pyr, out, s);
        case 16: return launch_levels<16>(x, len, clips, f, J, pyr, out, s);
        case 18: return launch_levels<18>(x, len, clips, f, J, pyr, out, s);
        case 20: return launch_levels<20>(x, len, clips, f, J, pyr, out, s);
        default: return launch_levels<0>(x, len, clips, f, J, pyr, out, s);
    }
}

}  // namespace cwth
