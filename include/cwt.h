/*
 * cwt.h -- C ABI of libcwth, a hop-strided continuous wavelet transform
 * (CWTH) for AMD Instinct MI355X (gfx950).
 *
 * The operation (paper: Sec. II-A, Eq. (1) and its discrete form; Sec. II-B
 * for the hop size H):
 *
 *     W[i][k] = sum_{m=-M_i}^{M_i} t_i[m] * x~[k*hop + m],
 *     t_i[m]  = psi(m / s_i) / sqrt(s_i),   psi(u) = exp(-u^2/2) * cos(5u),
 *     M_i     = floor(8 * s_i),  x~[j] = x[j] for 0 <= j < len, else 0,
 *     k       = 0 .. K-1,  K = ceil(len / hop).
 *
 * hop = 1 is the full CWT; any hop gives exactly every hop-th column of it.
 * The scalogram is S = |W| (the default output), stored row-major
 * [n_scales][K] in the caller's scale order.  Scales are in samples; fs only
 * maps scale to frequency, f_i = (5 / (2*pi)) * fs / s_i.
 *
 * Conventions for every function below:
 *   - Every call returns a cwt_status; nothing aborts or throws across the ABI.
 *     cwt_last_error() returns a thread-local message for the last failure.
 *   - Pointers named x, out, xs[], outs[] are DEVICE pointers owned by the
 *     caller; they must stay valid until the work queued on `stream`
 *     completes.  All other pointers are HOST pointers; their contents are
 *     copied before the call returns.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   - Arguments are validated before anything is launched.
 */
#ifndef CWT_H
#define CWT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cwt_plan_s* cwt_plan_t;   /* opaque, owned by the library */
typedef struct cwt_batch_s* cwt_batch_t; /* opaque, owned by the library */

typedef enum {
    CWT_OK = 0,
    CWT_ERR_INVALID_ARG = 1,   /* a bad argument; nothing was launched          */
    CWT_ERR_UNSUPPORTED = 2,   /* unknown wavelet/dtype, or a batch mixing plans */
    CWT_ERR_OUT_OF_MEMORY = 3, /* a device or pinned allocation failed           */
    CWT_ERR_DEVICE = 4,        /* no usable gfx950 device, or a launch failed    */
    CWT_ERR_INTERNAL = 5
} cwt_status;

typedef enum { CWT_WAVELET_MORLET = 0 } cwt_wavelet; /* psi(t)=exp(-t^2/2)cos(5t), |t|<=8 */

typedef enum {
    CWT_DTYPE_FP32 = 0,    /* plain FP32 direct sum on the vector ALUs                */
    CWT_DTYPE_BF16 = 1,    /* BF16 operands on MFMA, FP32 accumulation                */
    CWT_DTYPE_FP16 = 2,    /* FP16 operands on MFMA, FP32 accumulation                */
    CWT_DTYPE_BF16X3 = 3,  /* hi+lo BF16 split, three MFMA products, FP32 accumulation */
    CWT_DTYPE_FP8_E4M3 = 4 /* OCP e4m3 operands on MFMA; power-of-two scale per scale
                              (taps) and per 128-frame segment up to hop 128, per
                              tile beyond (signal), removed in the epilogue; results
                              independent of configuration and batch                   */
} cwt_dtype;

typedef enum { CWT_OUT_MAGNITUDE = 0, CWT_OUT_SIGNED = 1 } cwt_output;

/*
 * Create a plan: validates the scales, builds the device-resident wavelet bank
 * (taps evaluated in FP64 on the device, Eq. (1), then rounded once to the
 * operand type) and picks a kernel configuration.  Banks are shared between
 * plans with the same (fs, wavelet, scales, dtype) and reference counted.
 *   fs        sampling rate in Hz, > 0 and finite (used only for frequencies)
 *   scales    n_scales host doubles, each finite and > 0, at most 2^20 / 8
 *             (M_i = floor(8 s_i) <= 131072); duplicates allowed
 *   hop       translation stride H >= 1 (Sec. II-B)
 *   plan_out  receives the plan on CWT_OK; untouched otherwise
 * Errors: CWT_ERR_INVALID_ARG (fs, scales, n_scales < 1 or > 4096, hop < 1,
 * NULL pointers), CWT_ERR_UNSUPPORTED (wavelet, dtype), CWT_ERR_DEVICE (no
 * gfx950 device), CWT_ERR_OUT_OF_MEMORY.
 */
cwt_status cwt_plan_create(double fs, cwt_wavelet wavelet, const double* scales,
                           int32_t n_scales, int32_t hop, cwt_dtype dtype,
                           cwt_plan_t* plan_out);

/* Output mode: magnitude |W| (default) or signed W.  Plans are otherwise
 * immutable; change the mode only while no work using the plan is queued. */
cwt_status cwt_plan_set_output(cwt_plan_t plan, cwt_output mode);

/* Release a plan.  Synchronises the device first, so queued work that uses
 * the plan's bank completes before the bank can be freed. NULL is a no-op. */
cwt_status cwt_plan_destroy(cwt_plan_t plan);

/* K = ceil(len / hop) for this plan; -1 on a NULL plan or len < 0. */
int64_t cwt_num_frames(cwt_plan_t plan, int64_t len);

/* Plan properties (host scalars). */
int32_t cwt_plan_num_scales(cwt_plan_t plan); /* -1 on NULL */
int32_t cwt_plan_hop(cwt_plan_t plan);        /* -1 on NULL */

/* hz_out[i] = (5 / (2*pi)) * fs / s_i, i in caller order (host array). */
cwt_status cwt_scale_frequencies(cwt_plan_t plan, double* hz_out);

/*
 * Queue the transform of one clip on `stream` (asynchronous, no allocation, no
 * host synchronisation).
 *   x    device float32[len]
 *   out  device float32[n_scales * cwt_num_frames(plan, len)], written fully
 * len == 0 is a no-op returning CWT_OK.  Errors: CWT_ERR_INVALID_ARG (NULL
 * plan, len < 0, NULL x/out when len > 0, S*K overflowing int64),
 * CWT_ERR_DEVICE (launch failure; asynchronous faults surface at the caller's
 * next synchronisation).
 */
cwt_status cwt_execute(cwt_plan_t plan, const float* x, int64_t len, float* out,
                       void* stream);

/*
 * Queue n clips as ONE launch (the persistent batch kernel; a batch of hop-1
 * Toeplitz clips only runs their tiles in one grid): clip c is transformed
 * with plans[c] (its own hop) from xs[c] (device float32[lens[c]]) into
 * outs[c] (device float32[n_scales * cwt_num_frames(plans[c], lens[c])]).  All
 * plans must share dtype, output mode and scale set (CWT_ERR_UNSUPPORTED
 * otherwise); hops may differ.  Each clip's result is bit-identical to
 * cwt_execute of that clip.
 * Uses a library-owned batch context for the calling thread and device and
 * launches directly (no graph); see cwt_batch_create for the explicit form,
 * which can also replay the launch as a captured HIP graph.
 */
cwt_status cwt_execute_batch(const cwt_plan_t* plans, const float* const* xs,
                             const int64_t* lens, float* const* outs, int32_t n,
                             void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * contract and results as cwt_execute_batch, bit for bit, but the call
 * allocates nothing.  The batch descriptors go to a fixed device array of
 * 36 KiB per GPU, held until the process ends, written by small kernels on
 * `stream` that carry them in their arguments; no hipMalloc, hipFree, host
 * staging buffer or copy.  At most 512 clips per call (CWT_ERR_INVALID_ARG
 * beyond).  Every call on one GPU shares that array: calls whose work
 * overlaps on the device (on different streams, or from several threads)
 * race and must be ordered by the caller; calls queued on one stream are
 * ordered by it.  The plans' device must be the current device.
 */
cwt_status cwt_execute_batch_noalloc(const cwt_plan_t* plans, const float* const* xs,
                                     const int64_t* lens, float* const* outs, int32_t n,
                                     void* stream);

/*
 * Explicit batch context: owns two pinned and two device descriptor buffers
 * sized for up to max_clips clips and captured HIP graphs (descriptor upload +
 * the persistent launch, or the launch alone) that cwt_batch_execute replays.
 * A batch whose descriptors equal those already held by one of the device
 * buffers (the same plans, buffers and lengths run again) is launched without
 * an upload, and without any host preparation while no plan's configuration
 * and no tuned class has changed since.  Calls on one context are serialised by a mutex; a call may wait
 * on the host until the pinned buffer it reuses has been consumed (two calls
 * back), and a device buffer is overwritten only after the launches that read
 * it have completed, also when they were queued on another stream.
 */
cwt_status cwt_batch_create(int32_t max_clips, cwt_batch_t* batch_out);
cwt_status cwt_batch_destroy(cwt_batch_t batch);
/* Same contract as cwt_execute_batch; use_graph = 0 launches without a graph. */
cwt_status cwt_batch_execute(cwt_batch_t batch, const cwt_plan_t* plans,
                             const float* const* xs, const int64_t* lens,
                             float* const* outs, int32_t n, int32_t use_graph,
                             void* stream);

/*
 * Autotuner.  Times, on the launch described, the per-launch automatic
 * choice and every kernel configuration that fits every clip's hop
 * (synchronous; allocates its own input, output and descriptor buffers, fills
 * the input with a seeded noise signal; the cost does not depend on the
 * values).  Where a configuration beats the automatic choice by more than 3%,
 * it is recorded for the launch's class: (device arch and CU count, dtype,
 * scale count, widest half-width, log2 buckets of the smallest and largest
 * hop, of the clip count and of the mean length).  Later launches of that
 * class by plans left at their default configuration run it (cwt_execute,
 * cwt_execute_batch, cwt_batch_execute, cwt_plan_launch_config); a
 * configuration set with cwt_plan_set_config is never overridden.  Where the
 * automatic choice wins, a record of the class is removed.  Records live for
 * the process and, with $CWTH_AUTOTUNE_CACHE naming a file, in that file
 * (read on first use, rewritten after every tuning).  BF16, FP16 and BF16x3
 * results do not depend on the configuration; FP8's do not either, under the
 * configurations it accepts.
 *   plans, lens  host arrays of n >= 1 plans (one bank and output mode, hops
 *                may differ, as in cwt_execute_batch) and lengths >= 1
 *   chosen_out   host, may be NULL: the configuration such launches now run
 * Errors: CWT_ERR_INVALID_ARG, CWT_ERR_UNSUPPORTED (plans that cannot share a
 * launch), CWT_ERR_OUT_OF_MEMORY, CWT_ERR_DEVICE.  FP32 plans have one
 * configuration; the call then only reports it.
 */
cwt_status cwt_autotune_batch(const cwt_plan_t* plans, const int64_t* lens, int32_t n, int32_t* chosen_out);

/* cwt_autotune_batch of one clip of len samples (the cwt_execute launch). */
cwt_status cwt_autotune(cwt_plan_t plan, int64_t len, int32_t* chosen_out);

/* Kernel configuration of the plan (index into the candidate list) and the
 * number of candidates; a forced choice via cwt_plan_set_config.  A plan left
 * at its default configuration may run a launch under another candidate: a
 * smaller-tile one when the launch has few frames or a larger tile's signal
 * window does not fit LDS, or the one tuned for the launch's class
 * (cwt_autotune_batch); BF16, FP16 and BF16x3 results do not depend on the
 * configuration.  A set configuration is used for every launch. */
int32_t cwt_plan_config(cwt_plan_t plan);

/* The configuration that a launch of n_clips clips of len samples each under
 * this plan runs (cwt_execute for one clip, a batch of the plan for more):
 * cwt_plan_config for a set plan, else the tuned configuration of the
 * launch's class, else the per-launch choice.  Host only, no device work.
 * Returns -1 for a NULL plan, len < 1 or n_clips < 1. */
int32_t cwt_plan_launch_config(cwt_plan_t plan, int64_t len, int32_t n_clips);
int32_t cwt_plan_num_configs(cwt_plan_t plan);

/* The kind of configuration `index` for this plan: 0 = tiles of 32-scale
 * blocks (every hop), 1 = Toeplitz tiles (hop 1, BF16/FP16: each scale runs
 * its own K range; the default there), -1 = no such configuration.  BF16,
 * FP16 and BF16x3 results are bit-identical across the configurations of one
 * kind (and between a clip alone and in a batch); the two kinds sum each
 * coefficient's products in different groups of 16 and agree within the
 * dtype's tolerance.  A batch runs a Toeplitz plan's clips as Toeplitz tiles:
 * in one grid when every clip of the batch is one (configuration 13's, 14's
 * or 15's, the first that gives four work-groups per CU), else configuration
 * 14's in the persistent kernel. */
int32_t cwt_plan_config_kind(cwt_plan_t plan, int32_t index);
cwt_status cwt_plan_set_config(cwt_plan_t plan, int32_t index);

/*
 * Read back the operand values the bank holds for caller scale `scale_index`,
 * decoded to double: taps_out[m + M] for m = -M .. M (host array of 2M+1).
 * For CWT_DTYPE_BF16X3 the value is hi + lo; for FP8 it is the stored code
 * times 1/alpha.  For checking the bank against the FP64 definition.
 */
cwt_status cwt_plan_bank_taps(cwt_plan_t plan, int32_t scale_index, double* taps_out,
                              int64_t cap);

/* ------------------------------------------------------------------------
 * Decimate-then-transform (the paper's workflow description, Sec. III-B: the
 * signal is re-sampled and the re-sampled signal is transformed).  The
 * transform of the decimated signal is a hop-1 plan at scales s / factor.
 */

/* ceil(len / factor); -1 if len < 0 or factor < 1. */
int64_t cwt_decimated_length(int64_t len, int32_t factor);

/*
 * Anti-alias filter for decimation by `factor` (host, FP64): n_taps (odd,
 * >= 1) windowed-sinc taps with cutoff fs/(2 factor) and a Hamming window,
 * h[j] = w[j] sinc((j - c)/factor)/factor, c = (n_taps-1)/2,
 * w[j] = 0.54 - 0.46 cos(2 pi j/(n_taps-1)), scaled to unit DC gain.
 * h_out: host double[n_taps].  Errors: CWT_ERR_INVALID_ARG (factor < 1,
 * n_taps even or < 1, NULL h_out).
 */
cwt_status cwt_lowpass_fir(int32_t factor, int32_t n_taps, double* h_out);

/*
 * y[n] = sum_{j=0}^{h_len-1} h[j] * x~[n*factor + j - (h_len-1)/2] for
 * n = 0 .. cwt_decimated_length(len, factor) - 1, x~ zero outside [0, len):
 * output sample n sits on input sample n*factor, like frame n of a hop-factor
 * transform.  x: device float32[len]; h: device float32[h_len] (h_len odd;
 * h = {1} is plain decimation); y: device float32[cwt_decimated_length].
 * FP32 accumulation: in ascending j for h_len < 64, else 64 interleaved
 * partial sums (lane l takes j = l, l + 64, ..) combined by a fixed butterfly;
 * deterministic either way.  Asynchronous on `stream`.  Errors:
 * CWT_ERR_INVALID_ARG (len < 0, factor < 1, h_len even or < 1, NULL pointers
 * when len > 0), CWT_ERR_DEVICE (launch failure).  len == 0 is a no-op.
 */
cwt_status cwt_decimate(const float* x, int64_t len, int32_t factor, const float* h, int32_t h_len,
                        float* y, void* stream);

/* ------------------------------------------------------------------------
 * Scalogram to image: the step after the transform, where scalograms become
 * the CNN's input images (Sec. II-A with Fig. 1, Sec. III-B).
 *
 *   D[i][k]     = 20 log10(max(|W[i][k]|, amin))
 *   image[r][c] = (B(r, c) - min D) / (max D - min D),  0 if max D == min D
 *
 * B is D resampled bilinearly to height x width with half-pixel centres (the
 * source row of output row r is (r + 0.5) * n_scales / height - 0.5, clamped
 * below at 0, interpolating rows floor(.) and floor(.) + 1 or the last row;
 * likewise columns over frames; no anti-aliasing); min and max over the full
 * n_scales x n_frames D.
 */

/* Bytes of device workspace cwt_scalogram_image needs (partial extrema). */
int64_t cwt_image_workspace_bytes(void);

/*
 * scalogram: device float32[n_scales][n_frames] (|W| or signed W; the
 * magnitude is taken); image: device float32[height][width]; workspace:
 * device buffer of cwt_image_workspace_bytes() bytes, owned by the caller, not
 * shared by calls in flight at the same time.  FP32 arithmetic (log10f; source
 * coordinates in double).  Asynchronous on `stream`.  Errors:
 * CWT_ERR_INVALID_ARG (n_scales, n_frames, height or width < 1, amin not
 * finite and > 0, NULL pointers), CWT_ERR_DEVICE (launch failure).
 */
cwt_status cwt_scalogram_image(const float* scalogram, int32_t n_scales, int64_t n_frames, float amin,
                               float* image, int32_t height, int32_t width, void* workspace,
                               void* stream);

/* ------------------------------------------------------------------------
 * DWT scalogram (Sec. II-A, Fig. 1c): the dyadic transform, scale 2^j and
 * translation n 2^j at level j, computed by a two-channel filter bank with
 * down-sampling by two, its detail coefficients spread back over the time
 * axis to form a matrix.  With a_0 = x, len_0 = len, len_j = ceil(len_{j-1}/2):
 *
 *   a_j[n] = sum_k h[k] a_{j-1}[c(2n + k)],   d_j[n] = sum_k g[k] a_{j-1}[c(2n + k)]
 *   g[k]   = (-1)^k h[h_len - 1 - k]
 *   c(i)   = min(i mod P, len_{j-1} - 1),   P = len_{j-1} rounded up to even
 *   S[j-1][t] = |d_j[t >> j]|,  t = 0 .. len - 1,  j = 1 .. levels
 *
 * (periodic extension; a level of odd length first repeats its last sample).
 */

/* Lowpass Daubechies filter with `order` vanishing moments (host, FP64):
 * 2*order taps, sum sqrt(2), orthonormal under shifts by two, minimum phase;
 * h_out[0] is the tap of the smallest delay.  h_out: host double[2*order].
 * Errors: CWT_ERR_INVALID_ARG (order outside 1 .. 10, NULL h_out). */
cwt_status cwt_daubechies(int32_t order, double* h_out);

/* Floats per clip of the level record: 2 * sum_{j=1}^{levels} ceil(len / 2^j).
 * -1 if len < 1 or levels outside 1 .. 30. */
int64_t cwt_dwt_pyramid_length(int64_t len, int32_t levels);

/*
 * x: device float32[clips][len]; h: host double[h_len] (h_len even, 2 .. 64,
 * any filter; rounded to FP32, g derived as above); pyramid: device
 * float32[clips][cwt_dwt_pyramid_length(len, levels)], per level j = 1 ..
 * levels a_j then d_j (ceil(len/2^j) each), written (it is also the
 * intermediate between levels); out: device float32[clips][levels][len], the
 * matrix S, or NULL to skip it.  All buffers owned by the caller.  FP32:
 * every coefficient is an FMA chain over k in ascending order.  Asynchronous
 * on `stream`.  Errors: CWT_ERR_INVALID_ARG (len outside 1 .. 2^31 - 1, clips
 * outside 1 .. 65535, levels outside 1 .. 30, bad h_len, non-finite taps,
 * NULL x, h or pyramid), CWT_ERR_DEVICE (launch failure).
 */
cwt_status cwt_dwt_scalogram(const float* x, int64_t len, int32_t clips, const double* h, int32_t h_len,
                             int32_t levels, float* pyramid, float* out, void* stream);

const char* cwt_status_string(cwt_status s);
const char* cwt_last_error(void);

/* Library version string, e.g. "1.0.0 gfx950". */
const char* cwt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CWT_H */
