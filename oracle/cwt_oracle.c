/*
 * FP64 reference implementation of the hop-strided Morlet continuous wavelet
 * transform (CWTH).  TEST INFRASTRUCTURE ONLY: it is loaded by the test suite,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by
 * the library.  It shares no code, header or table with the HIP path.
 *
 * What it computes (paper, Sec. II-A Eq. (1), its discrete form, and Sec. II-B):
 *   X(b, a) = a^{-1/2} * sum_n x[n] * psi((n - b) / a)
 * evaluated at translations b = k * hop (k = 0 .. ceil(N / hop) - 1) and at every
 * requested scale a = s_i (in samples).  hop = 1 is the full CWT; CWTH keeps
 * every hop-th column of it.
 *
 * Readings taken where the paper is silent (each one is listed in the design
 * notes):
 *   - psi(t) = exp(-t^2 / 2) * cos(5 t), the real Morlet wavelet; psi is even
 *     and real, so psi* = psi and correlation equals convolution.
 *   - support truncated to |t| <= 8 (inclusive): M = floor(8 s), L = 2 M + 1 taps.
 *   - no sampling-interval factor; samples outside [0, N) are zero ('same').
 *   - frame k is centred on sample k * hop.
 *
 * Summation order: every coefficient sums its taps in ascending tap offset
 * m = -M .. M.  The frame loop is innermost only so that the compiler can use
 * independent accumulators; no coefficient's own order is changed.  Build with
 * -O3 -ffp-contract=off and without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CWTO_OK 0
#define CWTO_EINVAL -1
#define CWTO_ENOMEM -2

/* Morlet mother wavelet (real part), evaluated at u >= 0. */
static double morlet(double u) { return exp(-0.5 * u * u) * cos(5.0 * u); }

/* Half-width M = floor(8 s) of the truncated support at scale s. */
int64_t cwto_half_width(double s) { return (int64_t)floor(8.0 * s); }

/* Number of frames for a signal of n samples at the given hop: ceil(n / hop). */
int64_t cwto_num_frames(int64_t n, int32_t hop) {
    if (n < 0 || hop < 1) return -1;
    return (n + hop - 1) / hop;
}

static int scale_ok(double s) { return isfinite(s) && s > 0.0 && 8.0 * s < 1e9; }

/* Taps t[m + M] = psi(|m| / s) / sqrt(s) for m = -M .. M (Eq. (1): the dilated
 * wavelet with the 1/sqrt(a) energy normalisation).  Returns L or a negative
 * error.  Using |m| makes t symmetric bit for bit. */
int64_t cwto_taps(double s, double* t, int64_t cap) {
    if (!scale_ok(s) || t == NULL) return CWTO_EINVAL;
    int64_t M = cwto_half_width(s), L = 2 * M + 1;
    if (cap < L) return CWTO_EINVAL;
    double rs = sqrt(s);
    for (int64_t m = -M; m <= M; ++m) {
        double u = (double)llabs(m) / s;
        t[m + M] = morlet(u) / rs;
    }
    return L;
}

/* Signed coefficients for one scale: W[k] for k = 0 .. K-1. */
static int one_scale(const double* x, int64_t n, double s, int32_t hop, double* W) {
    int64_t M = cwto_half_width(s), L = 2 * M + 1;
    int64_t K = cwto_num_frames(n, hop);
    double* t = (double*)malloc(sizeof(double) * (size_t)L);
    /* x~ : x padded with M zeros on either side, so x~[p + M] = x[p] for
     * 0 <= p < n and 0 elsewhere in [-M, n + M). */
    int64_t span = (K - 1) * (int64_t)hop + 2 * M + 1;
    if (span < n + 2 * M) span = n + 2 * M;
    double* xp = (double*)calloc((size_t)span, sizeof(double));
    if (!t || !xp) { free(t); free(xp); return CWTO_ENOMEM; }
    cwto_taps(s, t, L);
    memcpy(xp + M, x, sizeof(double) * (size_t)n);
    enum { FB = 64 };
    for (int64_t k0 = 0; k0 < K; k0 += FB) {
        int64_t nb = K - k0 < FB ? K - k0 : FB;
        double acc[FB];
        for (int64_t j = 0; j < nb; ++j) acc[j] = 0.0;
        for (int64_t m = 0; m < L; ++m) {          /* tap offset m - M, ascending */
            const double tm = t[m];
            for (int64_t j = 0; j < nb; ++j)
                acc[j] += tm * xp[(k0 + j) * (int64_t)hop + m];
        }
        for (int64_t j = 0; j < nb; ++j) W[k0 + j] = acc[j];
    }
    free(t);
    free(xp);
    return CWTO_OK;
}

/* Full signed CWTH: W is row-major [n_scales][ceil(n / hop)]. */
int cwto_cwt(const double* x, int64_t n, const double* scales, int32_t n_scales,
             int32_t hop, double* W) {
    if (n < 0 || hop < 1 || n_scales < 1 || scales == NULL) return CWTO_EINVAL;
    if (n > 0 && (x == NULL || W == NULL)) return CWTO_EINVAL;
    for (int32_t i = 0; i < n_scales; ++i)
        if (!scale_ok(scales[i])) return CWTO_EINVAL;
    int64_t K = cwto_num_frames(n, hop);
    if (K == 0) return CWTO_OK;
    int err = CWTO_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t i = 0; i < n_scales; ++i) {
        int e = one_scale(x, n, scales[i], hop, W + (int64_t)i * K);
        if (e != CWTO_OK) {
#pragma omp critical
            err = e;
        }
    }
    return err;
}

/* Selected signed coefficients W[scale_idx[p], frame_idx[p]], p = 0 .. np-1,
 * each summed on its own in the same ascending order as cwto_cwt. */
int cwto_points(const double* x, int64_t n, const double* scales, int32_t n_scales,
                int32_t hop, const int32_t* scale_idx, const int64_t* frame_idx,
                int64_t np, double* out) {
    if (n < 0 || hop < 1 || n_scales < 1 || scales == NULL || np < 0) return CWTO_EINVAL;
    if (np > 0 && (scale_idx == NULL || frame_idx == NULL || out == NULL)) return CWTO_EINVAL;
    int64_t K = cwto_num_frames(n, hop);
    for (int64_t p = 0; p < np; ++p)
        if (scale_idx[p] < 0 || scale_idx[p] >= n_scales || frame_idx[p] < 0 || frame_idx[p] >= K)
            return CWTO_EINVAL;
    for (int32_t i = 0; i < n_scales; ++i)
        if (!scale_ok(scales[i])) return CWTO_EINVAL;
    int err = CWTO_OK;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; ++p) {
        double s = scales[scale_idx[p]];
        int64_t M = cwto_half_width(s), L = 2 * M + 1;
        double* t = (double*)malloc(sizeof(double) * (size_t)L);
        if (!t) {
#pragma omp critical
            err = CWTO_ENOMEM;
            continue;
        }
        cwto_taps(s, t, L);
        int64_t c = frame_idx[p] * (int64_t)hop;
        double acc = 0.0;
        for (int64_t m = -M; m <= M; ++m) {
            int64_t q = c + m;
            double xv = (q >= 0 && q < n) ? x[q] : 0.0;
            acc += t[m + M] * xv;
        }
        out[p] = acc;
        free(t);
    }
    return err;
}

/* Threads the parallel regions will use (for reporting). */
int cwto_max_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void cwto_set_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
