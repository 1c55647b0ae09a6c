// Internal declarations shared by the host side of libcwth and its kernels.
// Nothing here is part of the public ABI (include/cwt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cwth {

// ---------------------------------------------------------------------------
// Operand types of the contraction.  Values match cwt_dtype.
enum Dtype : int { DT_FP32 = 0, DT_BF16 = 1, DT_FP16 = 2, DT_BF16X3 = 3, DT_FP8 = 4 };

// Rows of a 32-scale MFMA block, and the tile geometry of the direct kernel.
constexpr int kBlockRows = 32;     // scales per MFMA block (the M side of 32x32xK)
constexpr int kWaveSize = 64;
constexpr int kMfmaWaves = 4;      // waves per MFMA work-group (split along frames)
constexpr int kFp8Segment = 128;        // frames per FP8 signal-scale segment (the largest FP8 tile)
constexpr int kFp8SegmentMaxHop = 128;  // FP8 scales per segment up to this hop, per tile beyond
// Direct (FP32) work-groups of kDirectWaves waves, in one of two layouts
// (ClipArg::ws of an FP32 clip): 1 = kDirectFrames frames (one per thread)
// x one group of kDirectRows scales that every wave runs, staged
// kDirectChunk taps at a time; kDirectGroups = kDirectWideFrames frames (one
// per lane) x kDirectGroups groups, one per wave, staged kDirectWideChunk
// taps at a time (each staged value then feeds 64 scales: the layout for
// large hops, whose frames share few samples).
constexpr int kDirectWaves = 4;
constexpr int kDirectFrames = 64 * kDirectWaves;
constexpr int kDirectRows = 16;
constexpr int kDirectChunk = 32;
constexpr int kDirectGroups = kDirectWaves;
constexpr int kDirectWideFrames = 64;
constexpr int kDirectWideChunk = 128;
constexpr int kDirectWideHop = 256;   // layout kDirectGroups from this hop on

// K (taps) consumed by one MFMA for the operand type.
__host__ __device__ constexpr int kstep_of(int dt) { return dt == DT_FP8 ? 64 : 16; }

// ---------------------------------------------------------------------------
// Wavelet bank layouts (built on the device by bank.hip, read by the kernels).
//
// Scales are sorted by half-width M (ascending); `rows` map sorted positions
// back to the caller's row index (-1 for padding rows).
//
// Direct (FP32) bank: groups of kDirectRows consecutive sorted scales.  Group
// g stores taps for m = -P_g .. P_g (P_g = max M in the group) as
// taps[off_g + (m + P_g) * kDirectRows + r], zero outside each scale's own
// support.
struct DirectGroup {
    int32_t P;         // padded half-width of the group
    int32_t rows[kDirectRows];
    int64_t off;       // float offset into the bank
};

// MFMA bank: blocks of kBlockRows sorted scales.  Block b covers K-steps
// ks = lo .. hi (taps m in [kstep*ks, kstep*(ks+1)) ); for every step it stores
// one A-operand fragment in exact lane order (64 lanes x fragment bytes), so a
// wave loads it with one coalesced access per lane.  BF16X3 stores the hi
// fragment followed by the lo fragment.
struct MfmaBlock {
    int32_t lo, hi;        // K-step range in whole groups of 8 (zero-tap padding), hi >= ehi + 3
    int32_t elo, ehi;      // the steps that hold the block's taps: [elo, ehi] within [lo, hi]
    int64_t frag_off;      // byte offset of step `lo` in the fragment buffer
    int32_t rows[kBlockRows];
    float inv_alpha[kBlockRows]; // FP8 only: 1/alpha_r; 1 otherwise
};

// Toeplitz bank (BF16/FP16, hop 1): groups of kToepScales consecutive sorted
// scales.  Group g runs K-steps d = 0 .. D-1 over p = jb + 16 d + u (u < 16).
// The B-operand fragment of step d and one scale gives lane l the eight taps
// t[jb + 16 d + 8 (l / 32) - l % 32 + e], e = 0 .. 7: a Toeplitz block, fixed
// by 47 consecutive taps, and lane l's run always starts at an index
// congruent to -(l % 32) mod 8.  The bank therefore holds, per scale, eight
// shifted copies of the taps: copy r has t[8 k + i + jb - 24 - r] (zero
// outside the scale's support) at element i < 8 of its 16-byte unit k, so that
// lane l reads one aligned unit of copy (l % 32) mod 8, unit 2 d + l / 32 -
// (l % 32) / 8 + 3.  Units k = 0 .. 2 D + 2, stored [scale][k][copy]: the eight
// copies of a unit are 128 consecutive bytes.
constexpr int kToepScales = 2;
constexpr int kToepBatchNB = 2;    // 1024-frame blocks per wave in batch tiles
// The K loop takes the taps from LDS, kToepChunk steps at a time: units
// 2 d0 .. 2 d0 + kToepChunkK - 1 of every copy of both scales, two buffers.
constexpr int kToepChunk = 32;
constexpr int kToepChunkK = 2 * kToepChunk + 3;
constexpr int kToepChunkUnits = kToepScales * kToepChunkK * 8;
constexpr int kToepTapBytes = 2 * kToepChunkUnits * 16;
__host__ __device__ constexpr int toep_copy_units(int D) { return 2 * D + 3; }
__host__ __device__ constexpr int64_t toep_group_bytes(int D) { return (int64_t)kToepScales * toep_copy_units(D) * 8 * 16; }
// First p and K-steps of a group whose widest scale has half-width M, and the
// LDS (2-byte operands, plus the tap buffers) of a tile of 4 * 1024 * NB
// frames over D steps.
__host__ __device__ constexpr int toep_jb(int M) { return -8 * ((M + 7) / 8); }
__host__ __device__ constexpr int toep_steps(int M) { return (((M + 32 - toep_jb(M) + 15) / 16) + 3) & ~3; }
__host__ __device__ constexpr int toep_window_bytes(int NB, int D) { return (kMfmaWaves * 1024 * NB + 16 * D) * 2 + kToepTapBytes; }
// 16-byte units of the window of a work-group running group (jb0, D0) and,
// if D1 > 0, a narrower group (jb1 >= jb0, D1) after it: every step of both,
// plus the signal rows read one step past the last, rounded up to whole
// groups of four units (the XOR swizzle permutes within them).
__host__ __device__ constexpr int toep_window_units(int NB, int jb0, int D0, int jb1, int D1) {
    return (512 * NB + (2 * D0 > 2 * D1 + (jb1 - jb0) / 8 ? 2 * D0 : 2 * D1 + (jb1 - jb0) / 8) + 3) & ~3;
}
struct ToepGroup {
    int32_t jb;            // first p of step 0: a multiple of 8, <= -M of every scale
    int32_t D;             // K-steps (a multiple of 4); jb + 16 D >= M + 32
    int32_t rows[kToepScales];   // caller rows (-1: none)
    int64_t frag_off;      // byte offset of the group's shifted tap copies in the bank
};

// ---------------------------------------------------------------------------
// Per-launch arguments.

// One clip as seen by a kernel.
struct ClipArg {
    const float* x;
    float* out;
    int64_t len;     // samples
    int64_t K;       // frames = ceil(len / hop)
    int32_t hop;
    int32_t ntile;   // frame tiles of this clip
    int32_t mode;    // staging mode for the MFMA kernel (see StageMode)
    int32_t copies;  // shifted copies (linear mode)
    int32_t swz;     // XOR-swizzle shift (linear and window modes), -1 for none
    int32_t wb;      // window mode: 32-scale blocks per work-group (1, 2 or 4)
    int32_t cso;     // linear and window modes with copies > 1: copy stride = units + cso (16-byte units)
    int32_t ws;      // window mode: waves sharing one frame group (their blocks split WS ways);
                     // FP32 clips: scale groups per work-group (1 or kDirectGroups)
};

// LINEAR: chunked linear window, one block per tile; ROWS: chunked per-frame
// rows (SPLIT tiles); WIN: the whole linear window of a tile staged once.
// TOEP: hop-1 Toeplitz tiles (one scale group over 4 * 1024 * NB frames).
enum StageMode : int { STAGE_LINEAR = 0, STAGE_ROWS = 1, STAGE_WIN = 2, STAGE_TOEP = 3 };

struct MfmaArgs {
    const uint8_t* frags;
    const MfmaBlock* blocks;
    int32_t ngroups;       // number of 32-scale blocks (one per work-group tile)
    int32_t signed_out;
    int32_t chunk_steps;   // K-steps staged per LDS chunk (a multiple of 8)
    int32_t frames;        // frames per tile (= 32 * A * kMfmaWaves)
    int32_t buf_bytes;     // bytes of one LDS staging buffer (two are used)
    int32_t raw_bytes;     // bytes of the raw FP32 window buffer (linear staging)
    int32_t xcd_remap;     // 1: map consecutive tiles to the same XCD
    int32_t split_wb;      // row-layout tiles: scale blocks per work-group (1, 2 or 4)
    int32_t split_chunk;   // row-layout tiles: K-steps per chunk (a multiple of 8)
    int32_t shm_bytes;     // dynamic LDS of the launch (the largest need over its clips)
    // Toeplitz tiles (STAGE_TOEP clips)
    const uint8_t* tfrags;
    const ToepGroup* tgroups;
    int32_t ntgroups;
    int32_t toep_bg;       // scale groups per Toeplitz work-group: 1, or 2 (group ng-1-u with group u)
    // single clip (grid launch)
    ClipArg clip;
    // batch (persistent launch)
    const ClipArg* clips;  // device array, longest-first order
    const int32_t* tile_prefix; // device: tile_prefix[c] = first tile of clip c (n+1 entries)
    int32_t nclips;
    int32_t total_tiles;   // tiles over all clips and groups
};

struct DirectArgs {
    const float* taps;
    const DirectGroup* groups;
    int32_t ngroups;
    int32_t signed_out;
    ClipArg clip;
    int32_t xcd_remap;
};

// Host-side launchers (defined in the .hip files).
hipError_t launch_direct(const DirectArgs& a, hipStream_t s);
hipError_t launch_direct_batch(const DirectArgs& a, const ClipArg* d_clips, const int32_t* d_prefix,
                               int nclips, int total_tiles, hipStream_t s);
// A = 32-frame blocks per wave (1, 2, 4; 8 for WIN tiles of BF16/FP16); the
// third argument is unused.
// persistent: 0 = one grid tile per work-group (single clip), 1 = persistent
// batch kernel for any layout, 2 = persistent batch kernel for WIN tiles only.
hipError_t launch_mfma(int dt, int cfgA, int nb, const MfmaArgs& a, int persistent,
                       int grid, hipStream_t s);
int mfma_max_lds_bytes();
// Toeplitz tiles of one clip (a.clip, mode STAGE_TOEP): NB = 1, 2 or 4
// 1024-frame blocks per wave, grid = a.ntgroups * a.clip.ntile.
hipError_t launch_toep(int dt, int NB, const MfmaArgs& a, int grid, hipStream_t s);
// Toeplitz tiles (NB = 1, 2 or 4) of a batch of hop-1 clips in one grid:
// a.clips, a.tile_prefix (tiles x groups per clip), a.nclips, grid =
// a.total_tiles.
hipError_t launch_toep_batch(int dt, int NB, const MfmaArgs& a, int grid, hipStream_t s);
int toep_occupancy(int dt, int NB, size_t shm);
// Allow every MFMA kernel the full dynamic LDS; call once, outside graph capture.
hipError_t mfma_init_attributes();
// Resident work-groups per CU for a kernel instance with `shm` bytes of dynamic LDS.
int mfma_occupancy(int dt, int A, int nb, int persistent, size_t shm);

// Decimation (decim.hip): y[n] = sum_j h[j] x~[n*factor + j - (L-1)/2].
hipError_t launch_decimate(const float* x, int64_t len, int factor, const float* h, int L, float* y, int64_t ny,
                           hipStream_t s);

// Scalogram image (image.hip): dB, bilinear resize, min-max over the full scalogram.
int64_t image_workspace_bytes();
hipError_t launch_image(const float* w, int n_scales, int64_t n_frames, float amin, float* image, int height,
                        int width, void* workspace, hipStream_t s);

// DWT scalogram (dwt.hip): filter bank levels, then the scale-by-time matrix.
constexpr int kDwtMaxTaps = 64;
struct DwtFilter {      // analysis pair, FP32, passed by value as a kernel argument
    float h[kDwtMaxTaps];
    float g[kDwtMaxTaps];
    int L;
};
// Floats per clip of the level record: per level j, a_j then d_j, ceil(len/2^j) each.
int64_t dwt_pyramid_length(int64_t len, int J);
hipError_t launch_dwt(const float* x, int64_t len, int clips, const DwtFilter& f, int J, float* pyramid,
                      float* out, hipStream_t s);

// Bank generation (bank.hip).
struct BankScale {      // one sorted scale as the generator sees it
    double s;
    int32_t M;
};
hipError_t gen_direct_bank(const double* d_scales_sorted, int nscales, const DirectGroup* d_groups,
                           int ngroups, float* d_taps, int64_t total_floats, hipStream_t st);
hipError_t gen_mfma_bank(int dt, const double* d_scales_sorted, int nscales,
                         const MfmaBlock* d_blocks, int nblocks, uint8_t* d_frags,
                         int64_t total_bytes, const double* d_alpha, hipStream_t st);
hipError_t gen_toep_bank(int dt, const double* d_scales_sorted, int nscales, const ToepGroup* d_groups,
                         int ngroups, uint8_t* d_frags, hipStream_t st);
hipError_t decode_bank_taps(int dt, const uint8_t* d_frags, const MfmaBlock* d_blocks,
                            const float* d_direct, const DirectGroup* d_dgroups,
                            int sorted_pos, int M, double* d_out, hipStream_t st);

// Allocation-free batches (noalloc.hip): descriptors of up to
// kNoallocMaxClips clips in a file-scope device array of kNoallocScratchBytes
// per GPU, written by kernels that carry them in their arguments
// (kDescPieceWords 16-byte words, under 4 KiB of arguments, per launch).
constexpr int kNoallocMaxClips = 512;
constexpr int kNoallocScratchBytes = 36 * 1024;   // >= 16 + 512 * 64 + 4 * 513 + 16
constexpr int kDescPieceWords = 240;
// The device address of that GPU's array (looked up once, `device` current).
hipError_t scratch_address(int device, void** out);
// Write `bytes` of host descriptors to device memory dst, in order on stream s.
hipError_t put_desc(const uint8_t* host, size_t bytes, uint8_t* dst, hipStream_t s);

}  // namespace cwth
