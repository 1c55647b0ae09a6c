// Host side of libcwth: argument checks, plans, the shared wavelet-bank cache,
// launch geometry, batch contexts (descriptor upload + persistent launch,
// optionally replayed from a captured HIP graph), the autotuner and the
// exported C ABI declared in include/cwt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cwt.h"
#include "cwt_internal.h"

using namespace cwth;

// ---------------------------------------------------------------------------
// Status and thread-local error text.
static thread_local std::string g_last_error;

static cwt_status fail(cwt_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr, what)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            cwt_status st_ = (e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation) \
                                 ? CWT_ERR_OUT_OF_MEMORY                                 \
                                 : CWT_ERR_DEVICE;                                       \
            return fail(st_, std::string(what) + ": " + hipGetErrorString(e_));          \
        }                                                                                \
    } while (0)

// ---------------------------------------------------------------------------
// Device facts, looked up once per device.
struct DeviceInfo {
    bool ok = false;
    int cus = 0;
    std::string arch;
    std::string why;
};

static std::mutex g_dev_mu;
static std::map<int, DeviceInfo> g_dev;

static cwt_status current_device(int* dev, DeviceInfo* info) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1)
        return fail(CWT_ERR_DEVICE, "no HIP device available");
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return fail(CWT_ERR_DEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev.find(d);
    if (it == g_dev.end()) {
        DeviceInfo di;
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, d) != hipSuccess) {
            di.why = "hipGetDeviceProperties failed";
        } else {
            di.arch = p.gcnArchName;
            di.cus = p.multiProcessorCount;
            di.ok = di.arch.rfind("gfx950", 0) == 0;
            if (!di.ok) di.why = "device " + std::to_string(d) + " is " + di.arch + ", library is built for gfx950";
        }
        it = g_dev.emplace(d, di).first;
    }
    if (!it->second.ok) return fail(CWT_ERR_DEVICE, it->second.why);
    *dev = d;
    if (info) *info = it->second;
    return CWT_OK;
}

// ---------------------------------------------------------------------------
// Kernel configurations.  MFMA: A = 32-frame blocks per wave; wb = preferred
// 32-scale blocks per work-group and ws = waves that share one frame group
// (each running wb/ws of the blocks in turn) for WIN tiles of 32*A*(4/ws)
// frames; chunk = upper bound of the K-steps per LDS buffer of chunked LINEAR
// tiles (a multiple of 8; pick_chunk() shrinks it to what the LDS budget holds).
struct MfmaCfg {
    int A;       // Toeplitz configurations: 1024-frame blocks per wave (NB)
    int wb;
    int ws;
    int chunk;
    int toep;    // 1: hop-1 Toeplitz tiles (BF16/FP16), 4 * 1024 * A frames per work-group
};
static const MfmaCfg kMfmaCfgs[] = {
    {4, 4, 1, 32},   // 0: 512 frames, every wave runs all 4 blocks
    {4, 4, 2, 32},   // 1: 256 frames, blocks {0,3} / {1,2} per wave
    {2, 4, 1, 64},   // 2: 256 frames, every wave runs all 4 blocks
    {4, 4, 4, 32},   // 3: 128 frames, one block per wave
    {2, 4, 4, 64},   // 4:  64 frames, one block per wave
    {1, 4, 4, 64},   // 5:  32 frames, one block per wave
    {2, 4, 2, 64},   // 6: 128 frames, blocks {0,3} / {1,2} per wave
    {1, 4, 2, 64},   // 7:  64 frames, blocks {0,3} / {1,2} per wave
    {1, 4, 1, 64},   // 8: 128 frames, every wave runs all 4 blocks
    {4, 1, 1, 32},   // 9: 512 frames x 1 block
    {8, 4, 4, 32},   // 10: 256 frames, one block per wave (WIN only, BF16/FP16)
    {8, 4, 2, 32},   // 11: 512 frames, blocks {0,3} / {1,2} per wave (WIN only, BF16/FP16)
    {8, 4, 1, 32},   // 12: 1024 frames, every wave runs all 4 blocks (WIN only, BF16/FP16)
    // Toeplitz tiles (hop 1, BF16/FP16): A = 1024-frame blocks per wave, wb =
    // scale groups (of two scales) per work-group, the widest with the narrowest
    {4, 1, 0, 0, 1}, // 13: Toeplitz, 16384 frames x one scale group per work-group
    {2, 1, 0, 0, 1}, // 14: Toeplitz, 8192 frames
    {1, 1, 0, 0, 1}, // 15: Toeplitz, 4096 frames
    {4, 2, 0, 0, 1}, // 16: Toeplitz, 16384 frames x two groups over one window
    {2, 2, 0, 0, 1}, // 17: Toeplitz, 8192 frames x two groups
    {1, 2, 0, 0, 1}, // 18: Toeplitz, 4096 frames x two groups
};
static const int kToepCfg0 = 13;   // the Toeplitz configurations are 13 .. 15
static const int kNumMfmaCfgs = sizeof(kMfmaCfgs) / sizeof(kMfmaCfgs[0]);
static const int kFp8Cfg = 5;   // FP8's fallback configuration (see cfg_fits)

static int elem_bytes(int dt) { return dt == DT_FP8 ? 1 : 2; }
static int planes_of(int dt) { return dt == DT_BF16X3 ? 2 : 1; }

static int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Staging geometry of one clip for the MFMA kernel; mirrors make_geo() in mfma.hip.
struct Staging {
    int mode, copies, swz, cso;
    int64_t bytes;      // one LDS operand buffer (all planes); two are used
    int64_t raw_bytes;  // LINEAR: the raw FP32 window buffer
};

static const int64_t kLdsBudget = 52 * 1024;   // chunked tiles: three work-groups per CU
static const int64_t kWinBudget = 80 * 1024;   // WIN tiles: at least two work-groups per CU

// LDS after a WIN tile's window: its group's output rows (up to four blocks of
// kBlockRows int32) and, for FP8, their descale factors (float).
static int64_t win_row_bytes(int dt) { return (dt == DT_FP8 ? 2 : 1) * 4 * kBlockRows * 4; }

// Extra 16-byte units between the shifted copies of a linear window, by hop
// mod 128 (copies > 1 only).  The X-fragment reads of a wave hit lane
// addresses (p % U / gh) * stride + p / U, p = frame * hop + 8 * half; this
// offset maximises their measured LDS b128 read rate on MI355X (2-byte
// operands; e.g. hop 1: 168 B/clk/CU at offset 4 against 110 at offset 2).
// FP8 windows (16 elements per unit) keep 16 / copies.
static const int8_t kCopyStrideOffset[128] = {
     0,  4,  4,  6,  8,  1,  2,  0,  0,  3,  3,  3,  7,  1,  1,  0,
     0,  2,  2,  0,  6,  4,  0,  1,  0,  1,  1,  0,  5,  0,  0,  0,
     0,  0,  0,  2,  4, 10,  0,  1,  0,  7,  7,  7,  3,  6,  2,  0,
     0,  6,  6,  4,  2,  0,  0,  1,  0,  5,  5,  1,  1,  3,  0,  1,
     0,  4,  4,  1,  0,  6,  1,  3,  0,  3,  3,  0, 15,  2,  2,  1,
     0,  2,  2,  7, 14, 12,  3,  5,  0,  1,  1, 20, 13,  0,  0,  0,
     0,  0,  0,  2, 12, 11,  1,  1,  0,  7,  7,  2, 11, 22,  2,  0,
     0,  6,  6,  1, 10,  8,  5,  6,  0,  5,  5,  1,  9,  4, 14, 15,
};

// The LINEAR layout for F frames and `chunk` K-steps.
static Staging linear_staging(int dt, int hop, int F, int chunk) {
    const int U = 16 / elem_bytes(dt), KS = kstep_of(dt), P = planes_of(dt);
    Staging s;
    s.mode = STAGE_LINEAR;
    const int gh = (int)gcd64(hop, U);
    s.copies = U / gh;
    s.cso = s.copies == 1 ? 0 : dt == DT_FP8 ? 16 / s.copies : kCopyStrideOffset[hop % 128];
    const int64_t pmax = (int64_t)(F - 1) * hop + (int64_t)KS * chunk - 1;
    const int64_t len_u = ((pmax / U + 1) + 15) & ~int64_t(15);
    const int64_t cs = len_u + s.cso;
    s.bytes = (int64_t)s.copies * cs * 16 * P;
    s.raw_bytes = (((len_u + 1) * U + 255) & ~int64_t(255)) * 4;   // raw_floats() in mfma.hip
    // One copy and an even frame stride q (16-byte units): lane n of a read
    // hits unit n*q + c, so the 8 lanes of a b128 pass share only 16 / 2^v of
    // the 16 unit slots of 256 bytes (2^v the largest power of two dividing
    // q): 4-way conflicts from v = 3 on, 8-way from v = 4.  XOR of the unit's
    // low four bits with the four bits above bit v spreads them over distinct
    // slots for every even q (a bijection within each aligned block of 16
    // units; checked for all offsets c and q up to 256 in a model of the
    // reads).  Applied from v = 3 on and for powers of two; where the
    // conflicts are at most 2-way (hops 48 and 96) its address arithmetic cost
    // more than it saved (single 10 s clips 9.2 -> 11.1 and 10.2 -> 12.0 us),
    // while at hops 192-768 256-clip batches ran 1.35-2x faster with it.
    s.swz = -1;
    const int64_t q = hop / U;
    if (s.copies == 1 && hop % U == 0 && q % 2 == 0) {
        int v = 0;
        while (((q >> v) & 1) == 0) ++v;
        if (v >= 3 || (q & (q - 1)) == 0) s.swz = v;
    }
    return s;
}

// The row layout of SPLIT tiles (F frames, `chunk` K-steps).
static Staging split_staging(int dt, int F, int chunk) {
    const int U = 16 / elem_bytes(dt), KS = kstep_of(dt), P = planes_of(dt);
    Staging s;
    s.mode = STAGE_ROWS;
    s.copies = 1;
    s.swz = -1;
    s.cso = 0;
    s.bytes = (int64_t)F * (KS * chunk / U + 1) * 16 * P;
    s.raw_bytes = 0;
    return s;
}

// Chunked tiles: a clip uses the LINEAR layout (128*A-frame tiles, one scale
// block each) when that layout fits kLdsBudget at the smallest chunk;
// otherwise SPLIT tiles.
static bool use_linear(int dt, int hop, int F) {
    Staging s = linear_staging(dt, hop, F, 8);
    return 2 * s.bytes + s.raw_bytes <= kLdsBudget;
}

// Largest LINEAR chunk (multiple of 8, <= chunk_max) within kLdsBudget.
static int pick_chunk(int dt, int hop, int F, int chunk_max) {
    for (int chunk = chunk_max; chunk >= 8; chunk -= 8) {
        Staging s = linear_staging(dt, hop, F, chunk);
        if (2 * s.bytes + s.raw_bytes <= kLdsBudget) return chunk;
    }
    return 8;
}

// SPLIT geometry of a bank with `nblocks` 32-scale blocks: blocks per
// work-group (1, 2 or 4), frames per tile, and the largest chunk (<= 32) whose
// two row buffers take at most 40 KiB.
struct SplitGeo {
    int wb, F, chunk, groups;
};
static int wb_cap(int nblocks) { return nblocks >= 3 ? 4 : (nblocks == 2 ? 2 : 1); }
static SplitGeo split_geo(int dt, int nblocks) {
    SplitGeo g;
    g.wb = wb_cap(nblocks);
    g.F = 32 * (4 / g.wb);
    g.groups = (nblocks + g.wb - 1) / g.wb;
    g.chunk = 8;
    for (int ch = 32; ch >= 8; ch -= 8)
        if (2 * split_staging(dt, g.F, ch).bytes <= 40 * 1024) {
            g.chunk = ch;
            break;
        }
    return g;
}

static int log2_small(int v) { return v >= 4 ? 2 : (v >= 2 ? 1 : 0); }

// ---------------------------------------------------------------------------
// Wavelet bank: device-resident, shared by plans with the same key.
struct Bank {
    int dt = 0;
    int device = 0;
    std::vector<double> scales;        // caller order
    std::vector<int> sorted_to_caller; // sorted position -> caller row
    std::vector<int> caller_to_sorted;
    std::vector<int> M_sorted;
    // direct
    std::vector<DirectGroup> dgroups;
    float* d_dtaps = nullptr;
    DirectGroup* d_dgroups = nullptr;
    // mfma
    std::vector<MfmaBlock> blocks;
    uint8_t* d_frags = nullptr;
    MfmaBlock* d_blocks = nullptr;
    int64_t frag_bytes = 0;
    int Mmax = 0;
    int win_steps[3] = {0, 0, 0};      // widest union K range of a group of 1, 2, 4 blocks
    // Toeplitz fragments (BF16/FP16; built by the first hop-1 plan, ensure_toep)
    std::mutex toep_mu;
    bool toep_built = false;
    std::vector<ToepGroup> tgroups;
    ToepGroup* d_tgroups = nullptr;
    uint8_t* d_tfrags = nullptr;
    int toep_Dmax = 0;
    int toep_w1 = 0, toep_w2 = 0;   // window units beyond the frames: one group, a bundle of two

    ~Bank() {
        if (d_tgroups) (void)hipFree(d_tgroups);
        if (d_tfrags) (void)hipFree(d_tfrags);
        if (d_dtaps) (void)hipFree(d_dtaps);
        if (d_dgroups) (void)hipFree(d_dgroups);
        if (d_frags) (void)hipFree(d_frags);
        if (d_blocks) (void)hipFree(d_blocks);
    }
};

typedef std::tuple<int, int, std::vector<double>> BankKey;
static std::mutex g_bank_mu;
static std::map<BankKey, std::weak_ptr<Bank>> g_banks;

static cwt_status build_bank(int dt, int device, const std::vector<double>& scales,
                             std::shared_ptr<Bank>* out) {
    auto bk = std::make_shared<Bank>();
    bk->dt = dt;
    bk->device = device;
    bk->scales = scales;
    const int S = (int)scales.size();
    std::vector<int> order(S);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        int Ma = (int)std::floor(8.0 * scales[a]), Mb = (int)std::floor(8.0 * scales[b]);
        if (Ma != Mb) return Ma < Mb;
        return scales[a] < scales[b];
    });
    bk->sorted_to_caller = order;
    bk->caller_to_sorted.assign(S, 0);
    std::vector<double> sorted(S);
    for (int p = 0; p < S; ++p) {
        bk->caller_to_sorted[order[p]] = p;
        sorted[p] = scales[order[p]];
        bk->M_sorted.push_back((int)std::floor(8.0 * sorted[p]));
    }
    bk->Mmax = bk->M_sorted.back();

    double* d_sorted = nullptr;
    double* d_alpha = nullptr;
    HIP_TRY(hipMalloc(&d_sorted, sizeof(double) * S), "bank scales");
    std::unique_ptr<double, void (*)(double*)> g1(d_sorted, [](double* p) { (void)hipFree(p); });
    HIP_TRY(hipMemcpy(d_sorted, sorted.data(), sizeof(double) * S, hipMemcpyHostToDevice), "bank scales copy");

    if (dt == DT_FP32) {
        const int ng = (S + kDirectRows - 1) / kDirectRows;
        int64_t off = 0;
        for (int g = 0; g < ng; ++g) {
            DirectGroup G;
            G.P = 0;
            for (int r = 0; r < kDirectRows; ++r) {
                int p = g * kDirectRows + r;
                G.rows[r] = p < S ? order[p] : -1;
                if (p < S) G.P = std::max(G.P, bk->M_sorted[p]);
            }
            G.off = off;
            off += (int64_t)(2 * G.P + 1) * kDirectRows;
            bk->dgroups.push_back(G);
        }
        HIP_TRY(hipMalloc(&bk->d_dtaps, sizeof(float) * off), "direct bank");
        HIP_TRY(hipMalloc(&bk->d_dgroups, sizeof(DirectGroup) * ng), "direct groups");
        HIP_TRY(hipMemcpy(bk->d_dgroups, bk->dgroups.data(), sizeof(DirectGroup) * ng, hipMemcpyHostToDevice), "direct groups copy");
        HIP_TRY(gen_direct_bank(d_sorted, S, bk->d_dgroups, ng, bk->d_dtaps, off, 0), "direct bank generation");
    } else {
        const int KS = kstep_of(dt);
        const int step_bytes = planes_of(dt) * 64 * (dt == DT_FP8 ? 32 : 16);
        const int nbk = (S + kBlockRows - 1) / kBlockRows;
        std::vector<double> alpha(S, 1.0);
        if (dt == DT_FP8) {
            // alpha = 2^floor(log2(448 / max|t|)); max|t| = psi(0)/sqrt(s) = 1/sqrt(s).
            for (int p = 0; p < S; ++p) {
                int e;
                std::frexp(448.0 * std::sqrt(sorted[p]), &e);
                alpha[p] = std::ldexp(1.0, e - 1);
            }
        }
        int64_t off = 0;
        for (int b = 0; b < nbk; ++b) {
            MfmaBlock B;
            int Mb = 0;
            for (int r = 0; r < kBlockRows; ++r) {
                int p = b * kBlockRows + r;
                B.rows[r] = p < S ? order[p] : -1;
                B.inv_alpha[r] = p < S ? (float)(1.0 / alpha[p]) : 1.0f;
                if (p < S) Mb = std::max(Mb, bk->M_sorted[p]);
            }
            // steps ks with [KS*ks, KS*ks + KS) meeting [-Mb, Mb]: [elo, ehi].
            // Stored widened to whole groups of eight steps aligned to
            // multiples of 8 and reaching at least three steps past ehi (the
            // extra steps hold zero taps): chunked tiles run the widened range,
            // so any 8-aligned chunk meets every block on group boundaries; WIN
            // tiles run [elo, ehi] rounded up to a multiple of four steps.
            const int lo0 = (int)std::floor(-(double)Mb / KS), hi0 = Mb / KS;
            B.elo = lo0;
            B.ehi = hi0;
            B.lo = (int)std::floor(lo0 / 8.0) * 8;
            B.hi = (int)std::ceil((hi0 + 4) / 8.0) * 8 - 1;
            B.frag_off = off;
            off += (int64_t)(B.hi - B.lo + 1) * step_bytes;
            bk->blocks.push_back(B);
        }
        bk->frag_bytes = off;
        for (int l = 0; l < 3; ++l) {
            const int wb = 1 << l;
            for (int b0 = 0; b0 < nbk; b0 += wb) {
                int glo = bk->blocks[b0].lo, ghi = bk->blocks[b0].hi;
                for (int b = b0 + 1; b < std::min(nbk, b0 + wb); ++b) {
                    glo = std::min(glo, bk->blocks[b].lo);
                    ghi = std::max(ghi, bk->blocks[b].hi);
                }
                bk->win_steps[l] = std::max(bk->win_steps[l], ghi - glo + 1);
            }
        }
        HIP_TRY(hipMalloc(&d_alpha, sizeof(double) * S), "alpha");
        std::unique_ptr<double, void (*)(double*)> g2(d_alpha, [](double* p) { (void)hipFree(p); });
        HIP_TRY(hipMemcpy(d_alpha, alpha.data(), sizeof(double) * S, hipMemcpyHostToDevice), "alpha copy");
        HIP_TRY(hipMalloc(&bk->d_frags, off), "mfma bank");
        HIP_TRY(hipMalloc(&bk->d_blocks, sizeof(MfmaBlock) * nbk), "mfma blocks");
        HIP_TRY(hipMemcpy(bk->d_blocks, bk->blocks.data(), sizeof(MfmaBlock) * nbk, hipMemcpyHostToDevice), "blocks copy");
        HIP_TRY(gen_mfma_bank(dt, d_sorted, S, bk->d_blocks, nbk, bk->d_frags, off, d_alpha, 0), "mfma bank generation");
        HIP_TRY(hipDeviceSynchronize(), "bank generation");
    }
    HIP_TRY(hipDeviceSynchronize(), "bank generation");
    *out = bk;
    return CWT_OK;
}

static cwt_status acquire_bank(int dt, int device, const std::vector<double>& scales,
                               std::shared_ptr<Bank>* out) {
    std::lock_guard<std::mutex> lk(g_bank_mu);
    BankKey key(dt, device, scales);
    auto it = g_banks.find(key);
    if (it != g_banks.end()) {
        if (auto sp = it->second.lock()) {
            *out = sp;
            return CWT_OK;
        }
    }
    std::shared_ptr<Bank> bk;
    cwt_status st = build_bank(dt, device, scales, &bk);
    if (st != CWT_OK) return st;
    g_banks[key] = bk;
    *out = bk;
    return CWT_OK;
}

// Toeplitz windows must fit the WIN budget at one block per wave.
// LDS bytes of a Toeplitz work-group of the bank (its widest group, or its
// widest bundle of two), and whether it fits the WIN budget.
static int64_t toep_bytes(const Bank& bk, int NB, int bg) {
    return kToepTapBytes + 16 * (int64_t)((512 * NB + (bg == 2 ? bk.toep_w2 : bk.toep_w1) + 3) & ~3);
}
static bool toep_fits(const Bank& bk, int NB) { return toep_window_bytes(NB, toep_steps(bk.Mmax)) + 64 <= kWinBudget; }

// Build the bank's Toeplitz fragments once (BF16/FP16 banks whose widest
// window fits): groups of kToepScales consecutive sorted scales, jb = -M of
// the group rounded down to a multiple of 8, D = ceil((M + 32 - jb) / 16)
// rounded up to a multiple of 4.
static cwt_status ensure_toep(Bank& bk) {
    std::lock_guard<std::mutex> lk(bk.toep_mu);
    if (bk.toep_built) return CWT_OK;
    if (bk.dt != DT_BF16 && bk.dt != DT_FP16) return fail(CWT_ERR_UNSUPPORTED, "Toeplitz tiles hold BF16/FP16 only");
    const int S = (int)bk.scales.size();
    const int ng = (S + kToepScales - 1) / kToepScales;
    std::vector<ToepGroup> gs(ng);
    int64_t off = 0;
    int dmax = 0;
    for (int g = 0; g < ng; ++g) {
        ToepGroup& G = gs[g];
        int Mg = 0;
        for (int r = 0; r < kToepScales; ++r) {
            const int p = g * kToepScales + r;
            G.rows[r] = p < S ? bk.sorted_to_caller[p] : -1;
            if (p < S) Mg = std::max(Mg, bk.M_sorted[p]);
        }
        G.jb = toep_jb(Mg);
        G.D = toep_steps(Mg);
        G.frag_off = off;
        off += toep_group_bytes(G.D);
        dmax = std::max(dmax, G.D);
    }
    std::vector<double> sorted(S);
    for (int p = 0; p < S; ++p) sorted[p] = bk.scales[bk.sorted_to_caller[p]];
    double* d_sorted = nullptr;
    HIP_TRY(hipMalloc(&d_sorted, sizeof(double) * S), "bank scales");
    std::unique_ptr<double, void (*)(double*)> g1(d_sorted, [](double* q) { (void)hipFree(q); });
    HIP_TRY(hipMemcpy(d_sorted, sorted.data(), sizeof(double) * S, hipMemcpyHostToDevice), "bank scales copy");
    HIP_TRY(hipMalloc(&bk.d_tfrags, off), "Toeplitz bank");
    HIP_TRY(hipMalloc(&bk.d_tgroups, sizeof(ToepGroup) * ng), "Toeplitz groups");
    HIP_TRY(hipMemcpy(bk.d_tgroups, gs.data(), sizeof(ToepGroup) * ng, hipMemcpyHostToDevice), "Toeplitz groups copy");
    HIP_TRY(gen_toep_bank(bk.dt, d_sorted, S, bk.d_tgroups, ng, bk.d_tfrags, 0), "Toeplitz bank generation");
    HIP_TRY(hipDeviceSynchronize(), "Toeplitz bank generation");
    int w1 = 0, w2 = 0;
    for (int u = 0; u < ng; ++u) {
        w1 = std::max(w1, 2 * gs[u].D);
        const int v = ng - 1 - u;   // a bundle runs group v (the wider) and u
        if (u <= v) {
            int w = 2 * gs[v].D;
            if (u < v) w = std::max(w, 2 * gs[u].D + (gs[u].jb - gs[v].jb) / 8);
            w2 = std::max(w2, w);
        }
    }
    bk.tgroups = std::move(gs);
    bk.toep_Dmax = dmax;
    bk.toep_w1 = w1;
    bk.toep_w2 = w2;
    bk.toep_built = true;
    return CWT_OK;
}

// ---------------------------------------------------------------------------
// Plans.
// One clip's tile layout (see clip_layout()).
struct ClipLayout {
    Staging s;
    int wb = 1;          // scale blocks per work-group
    int ws = 1;          // WIN: waves sharing a frame group
    int F = 0;           // frames per tile
    int64_t groups = 0;  // work-group tiles per frame tile
};

// Configuration epoch: advanced whenever a plan's configuration or the tuned
// classes change, so that a batch context's prepared launches (prepared under
// an older epoch) are prepared again.  Plans carry a process-unique id.
static std::atomic<uint64_t> g_cfg_epoch{1};
static std::atomic<uint64_t> g_plan_uid{1};

struct cwt_plan_s {
    uint64_t uid = g_plan_uid.fetch_add(1);
    double fs;
    int hop;
    int dt;
    int signed_out = 0;
    int cfg = 0;
    int device = 0;
    int cus = 0;
    std::string arch;
    uint64_t arch_hash = 0;   // fnv1a(arch): the device part of a tuned launch class
    std::shared_ptr<Bank> bank;
    ClipLayout lay;      // MFMA layout under cfg ...
    int lay_chunk = 8;   // ... for chunked LINEAR tiles of this chunk
    bool cfg_user = false;    // configuration set by cwt_plan_set_config: no tuned override
    bool cfg_auto = false;    // default configuration: each launch picks one of auto_set (auto_cfg)
    int auto_set[3] = {6, 4, 5};   // scale-block tiles 6, 4, 5, or Toeplitz tiles 13, 14, 15
    ClipLayout auto_lay[3];   // layouts under those configurations
};

// ---------------------------------------------------------------------------
// Tuned launch classes.  cwt_autotune_batch times the configurations on the
// launch it is given and, where one beats the automatic per-launch choice by
// more than kTuneMargin, records it for the launch's class: (arch, CUs, dtype,
// scale count, widest half-width bucket, hop buckets of the batch, clip-count
// bucket, mean-length bucket).  Launches of a plan left at its default
// configuration look their class up (cwt_execute, batches, launch_config); a
// configuration set with cwt_plan_set_config is never overridden.  The
// classes are kept per process and, with $CWTH_AUTOTUNE_CACHE set, in that
// file ("class": index lines of a JSON object), read on first use.
static const double kTuneMargin = 0.03;

static int log2_bucket(int64_t v) {
    int b = 0;
    while (b < 62 && (int64_t(1) << (b + 1)) <= v) ++b;
    return b;
}

// A launch class.  Held as integers, so a launch looks its class up without
// allocating; written to and read from the cache file as text.
struct TuneKey {
    uint64_t arch;   // FNV-1a hash of the device's arch name
    int cus, dt, S, Mb, hlo, hhi, C, N;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, cus, dt, S, Mb, hlo, hhi, C, N) <
               std::tie(o.arch, o.cus, o.dt, o.S, o.Mb, o.hlo, o.hhi, o.C, o.N);
    }
};

static uint64_t fnv1a(const std::string& v) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char ch : v) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    return h;
}

static TuneKey launch_class(const cwt_plan_s* p0, int hop_lo, int hop_hi, int64_t n_clips, int64_t mean_len) {
    TuneKey k;
    k.arch = p0->arch_hash;
    k.cus = p0->cus;
    k.dt = p0->dt;
    k.S = (int)p0->bank->scales.size();
    k.Mb = log2_bucket(std::max(1, p0->bank->Mmax));
    k.hlo = log2_bucket(hop_lo);
    k.hhi = log2_bucket(hop_hi);
    k.C = log2_bucket(std::max<int64_t>(1, n_clips));
    k.N = log2_bucket(std::max<int64_t>(1, mean_len));
    return k;
}

static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tuned;   // launch class -> configuration
static bool g_tuned_loaded = false;
static std::atomic<int> g_tuned_count{0};   // entries of g_tuned (a lock-free "none" test)

// Cache file lines: "<arch hash hex>/<cus>/dt<d>/S<s>/M<m>/h<lo>-<hi>/C<c>/N<n>": <configuration>
static void load_tuned_locked() {
    if (g_tuned_loaded) return;
    g_tuned_loaded = true;
    const char* path = std::getenv("CWTH_AUTOTUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    if (!f) return;
    std::string line;
    while (std::getline(f, line)) {
        unsigned long long arch = 0;
        TuneKey k;
        int v = -1;
        if (std::sscanf(line.c_str(), " \"%llx/%d/dt%d/S%d/M%d/h%d-%d/C%d/N%d\": %d", &arch, &k.cus, &k.dt, &k.S,
                        &k.Mb, &k.hlo, &k.hhi, &k.C, &k.N, &v) != 10)
            continue;
        k.arch = arch;
        if (v >= 0 && v < kNumMfmaCfgs) g_tuned[k] = v;
        g_cfg_epoch.fetch_add(1);
    }
    g_tuned_count = (int)g_tuned.size();
}

static void save_tuned_locked() {
    const char* path = std::getenv("CWTH_AUTOTUNE_CACHE");
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (auto& kv : g_tuned) {
        const TuneKey& k = kv.first;
        char buf[160];
        std::snprintf(buf, sizeof(buf), "  \"%llx/%d/dt%d/S%d/M%d/h%d-%d/C%d/N%d\": %d", (unsigned long long)k.arch,
                      k.cus, k.dt, k.S, k.Mb, k.hlo, k.hhi, k.C, k.N, kv.second);
        f << buf << (++i < g_tuned.size() ? ",\n" : "\n");
    }
    f << "}\n";
    f.close();
    std::rename(tmp.c_str(), path);
}

static void ensure_tuned_loaded() {
    static std::once_flag once;
    std::call_once(once, [] {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tuned_locked();
    });
}

// The tuned configuration of a launch class, or -1.
static int tuned_lookup(const TuneKey& cls) {
    ensure_tuned_loaded();
    if (g_tuned_count.load(std::memory_order_relaxed) == 0) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(cls);
    return it == g_tuned.end() ? -1 : it->second;
}

// Default configuration by hop (measured on MI355X, 128 linear scales, 10 s
// clips): small hops share a 128-frame window between two pairs of waves,
// each running a balanced pair of blocks ({0,3}, {1,2}); larger hops take
// narrower frame tiles with one block per wave.  FP8 has one configuration.

static ClipLayout clip_layout(int dt, const Bank& bk, int hop, const MfmaCfg& c, int chunk);

// Default tile configuration, from configuration sweeps on MI355X (batches of
// 10 s clips with 128 linear scales, 8 x 60 s at 48 kHz with 256 geometric
// scales up to 1024, 10 s clips with 64 geometric scales up to 256, hops 1 to
// 1024).  6 selects the per-launch choice (set_auto/auto_cfg below): 128-frame
// tiles with two 32-frame blocks per wave where their window fits and the
// launch has the work-groups, then 64-frame tiles (4), then 32-frame tiles
// (5).  Up to hop 128 that is the default whenever configuration 6 stages its
// whole window in LDS (else 5).  Beyond hop 128 it is the default whenever any
// of the three does: 256-clip batches ran 11-27% faster at hops 192, 256 and
// 512 than with 32-frame tiles throughout (tap fragments shared by two frame
// blocks), equal at 1024 and 4% slower at 384; single clips there have too
// few frames for the wider tiles and keep 5.  With no whole window, 5.
static bool cfg_fits(const cwt_plan_s* p, int cfg, int hop);

static int default_cfg(const cwt_plan_s* p, int hop) {
    if (p->dt == DT_FP32) return 0;
    // hop 1 at 16-bit operands: Toeplitz tiles (each scale runs its own K
    // range, ~1.03x the algorithmic work against ~1.30x for 32-scale blocks)
    if (cfg_fits(p, kToepCfg0, hop)) return kToepCfg0;
    auto win = [&](int cfg) {
        const MfmaCfg& c = kMfmaCfgs[cfg];
        return clip_layout(p->dt, *p->bank, hop, c, c.chunk).s.mode == STAGE_WIN;
    };
    // FP8 takes the per-launch choice only where its last resort, 5, stages
    // the whole window too: no FP8 launch may fall back to a chunked tile of
    // 256 frames (see cfg_fits)
    if (p->dt == DT_FP8) return hop <= kFp8SegmentMaxHop && win(5) && (win(6) || win(4)) ? 6 : kFp8Cfg;
    if (hop > 128) return (win(6) || win(4) || win(5)) ? 6 : 5;
    if (!win(6) && win(5)) return 5;
    return 6;
}

static bool cfg_fits(const cwt_plan_s* p, int cfg, int hop) {
    if (p->dt == DT_FP32) return cfg == 0;
    if (cfg < 0 || cfg >= kNumMfmaCfgs) return false;
    const MfmaCfg& c = kMfmaCfgs[cfg];
    // Toeplitz tiles: hop 1, 16-bit operands, a built Toeplitz bank whose
    // widest window fits at this tile size
    if (c.toep)
        return hop == 1 && (p->dt == DT_BF16 || p->dt == DT_FP16) && p->bank->toep_built &&
               toep_bytes(*p->bank, c.A, c.wb) <= kWinBudget;
    // FP8 scales the signal per 128-frame segment up to hop 128 (fp8_beta):
    // every tile must lie in one segment, i.e. have at most 128 frames.
    // Configuration 5 (32-frame WIN, 128-frame chunked and 32-128-frame row
    // tiles) always does; 4 and 6 (two frame blocks per wave) only with WIN
    // tiles of 64 and 128 frames, their chunked tiles having 256.  Beyond hop
    // 128 the scale is per tile and 5 is the only configuration.
    if (p->dt == DT_FP8)
        return cfg == kFp8Cfg ||
               (hop <= kFp8SegmentMaxHop && (cfg == 4 || cfg == 6) &&
                clip_layout(p->dt, *p->bank, hop, c, c.chunk).s.mode == STAGE_WIN);
    if (c.A == 8)   // WIN tiles of the 2-byte types only
        return (p->dt == DT_BF16 || p->dt == DT_FP16) &&
               clip_layout(p->dt, *p->bank, hop, c, c.chunk).s.mode == STAGE_WIN;
    return true;   // a layout always exists: WIN, chunked LINEAR or SPLIT tiles
}

// Per-clip layout under a configuration: WIN tiles with the first wb >= cfg.wb
// (up to the bank's block count) whose whole window fits kWinBudget; else
// chunked LINEAR tiles if they fit kLdsBudget; else SPLIT tiles.  The choice
// depends only on (dtype, bank, hop, configuration), never on the batch.
static ClipLayout clip_layout(int dt, const Bank& bk, int hop, const MfmaCfg& c, int chunk) {
    ClipLayout L;
    if (c.toep) {
        // Toeplitz tiles for hop-1 clips of a built bank; any other clip of a
        // launch under a Toeplitz configuration takes configuration 6's tiles
        if (hop == 1 && bk.toep_built && toep_bytes(bk, c.A, c.wb) <= kWinBudget) {
            L.s.mode = STAGE_TOEP;
            L.s.copies = 1;
            L.s.swz = -1;
            L.s.cso = 0;
            L.s.bytes = toep_bytes(bk, c.A, c.wb);
            L.s.raw_bytes = 0;
            L.F = kMfmaWaves * 1024 * c.A;
            L.wb = c.wb;
            L.groups = c.wb == 2 ? ((int64_t)bk.tgroups.size() + 1) / 2 : (int64_t)bk.tgroups.size();
            return L;
        }
        const MfmaCfg& h = kMfmaCfgs[6];
        return clip_layout(dt, bk, hop, h, h.chunk);
    }
    const int nblk = (int)bk.blocks.size(), cap = wb_cap(nblk);
    for (int wb = std::min(c.wb, cap); wb <= cap; wb *= 2) {
        const int ws = std::min(c.ws, wb);
        const int F = 32 * c.A * (4 / ws);
        Staging s = linear_staging(dt, hop, F, bk.win_steps[log2_small(wb)]);
        s.bytes += win_row_bytes(dt);
        if (s.bytes <= kWinBudget) {
            s.mode = STAGE_WIN;
            s.raw_bytes = 0;
            L.s = s;
            L.wb = wb;
            L.ws = ws;
            L.F = F;
            L.groups = (nblk + wb - 1) / wb;
            return L;
        }
    }
    if (use_linear(dt, hop, 128 * c.A)) {
        L.s = linear_staging(dt, hop, 128 * c.A, chunk);
        L.wb = 1;
        L.F = 128 * c.A;
        L.groups = nblk;
        return L;
    }
    const SplitGeo sg = split_geo(dt, nblk);
    L.s = split_staging(dt, sg.F, sg.chunk);
    L.wb = sg.wb;
    L.F = sg.F;
    L.groups = sg.groups;
    return L;
}

// Dynamic LDS a layout needs: one window (WIN), two buffers plus the raw
// window (LINEAR), two row buffers (ROWS).
static int64_t layout_lds(const ClipLayout& L) {
    if (L.s.mode == STAGE_WIN || L.s.mode == STAGE_TOEP) return L.s.bytes;
    return 2 * L.s.bytes + L.s.raw_bytes;
}

// Set the plan's configuration and cache its layout.
static void set_cfg(cwt_plan_s* p, int cfg) {
    g_cfg_epoch.fetch_add(1);
    p->cfg = cfg;
    p->cfg_auto = false;
    if (p->dt == DT_FP32) return;
    const MfmaCfg& c = kMfmaCfgs[cfg];
    p->lay_chunk = c.toep ? 8 : pick_chunk(p->dt, p->hop, 128 * c.A, c.chunk);
    p->lay = clip_layout(p->dt, *p->bank, p->hop, c, p->lay_chunk);
}

// Toeplitz formulation (configurations 13 .. 15) of a plan; batches run its
// clips as tiles of kToepBatchNB blocks per wave (configuration kToepBatchCfg).
static bool plan_toep(const cwt_plan_s* p) { return p->dt != DT_FP32 && kMfmaCfgs[p->cfg].toep != 0; }
static const int kToepBatchCfg = 14;   // kMfmaCfgs[14].A == kToepBatchNB

// The default configuration (6) is chosen for throughput when work is
// plentiful; a launch with few frames fills the chip better with smaller
// tiles.  Per launch, an automatic plan takes the first of configurations 6
// (two 32-frame blocks per wave, 128-frame tiles), 4 (two blocks per wave,
// 64-frame tiles, one scale block per wave) and 5 (one block per wave,
// 32-frame tiles) that stages its whole window in LDS and gives the launch at
// least two work-groups per CU, else 5.  Measured on single clips and
// batches (10 s with 128 linear scales, 60 s at 48 kHz with 256 geometric
// scales, hops 1-256): the best configuration or within a few percent of it
// in every case, where a fixed one is up to 2x slower.  BF16/FP16/BF16x3
// results do not depend on the configuration.
// For a hop-1 clip of a Toeplitz plan the set is 13, 14, 15 (Toeplitz tiles
// of 16384, 8192 and 4096 frames) and the bar four work-groups per CU: one
// 10 s clip with 128 linear scales ran in 48.4 / 46.7 / 47.0 us under
// 13 / 14 / 15, a 5 s clip in 33.5 / 28.3 / 25.6 and a 30 s clip in 121.7 /
// 125.0 / 131.7 (with taps through LDS, whose per-work-group barriers favour
// more and shorter items where a launch has under two rounds of them).
static const int kAutoCfgs[3] = {6, 4, 5};
static const int kAutoToep[3] = {13, 14, 15};
static const int kAutoPerCu = 2, kAutoToepPerCu = 4;

// The tiles of a batch of Toeplitz clips only (one grid of them): the first
// of 13, 14, 15 that gives the launch kAutoToepPerCu work-groups per CU,
// else 15 (frames(j): frames of clip j of n).
template <class FR>
static int toep_batch_cfg(const Bank& bk, int cus, int n, FR&& frames) {
    for (int i = 0; i < 3; ++i) {
        const int64_t F = (int64_t)kMfmaWaves * 1024 * kMfmaCfgs[kAutoToep[i]].A;
        int64_t t = 0;
        for (int j = 0; j < n; ++j) t += (frames(j) + F - 1) / F * (int64_t)bk.tgroups.size();
        if (t >= (int64_t)kAutoToepPerCu * std::max(1, cus)) return kAutoToep[i];
    }
    return kAutoToep[2];
}

static void set_auto(cwt_plan_s* p) {
    g_cfg_epoch.fetch_add(1);
    p->cfg_auto = true;
    const int* set = kMfmaCfgs[p->cfg].toep ? kAutoToep : kAutoCfgs;
    for (int i = 0; i < 3; ++i) {
        p->auto_set[i] = set[i];
        const MfmaCfg& c = kMfmaCfgs[set[i]];
        p->auto_lay[i] = clip_layout(p->dt, *p->bank, p->hop, c, c.chunk);
    }
}

// wgs(L): work-groups the launch would have under layout L.
template <class WG>
static int auto_cfg(const cwt_plan_s* p, WG&& wgs) {
    if (!p->cfg_auto) return p->cfg;
    const int per_cu = kMfmaCfgs[p->auto_set[0]].toep ? kAutoToepPerCu : kAutoPerCu;
    const int64_t need = per_cu * (int64_t)std::max(1, p->cus);
    for (int i = 0; i < 3; ++i) {
        const ClipLayout& L = p->auto_lay[i];
        if (L.s.mode != STAGE_WIN && L.s.mode != STAGE_TOEP) continue;
        if (i == 2 || wgs(L) >= need) return p->auto_set[i];
    }
    return p->cfg;
}

// The per-launch choice for a launch of n clips (one clip: cwt_execute's).
static int batch_auto_cfg(const cwt_plan_t* plans, const int64_t* lens, int n) {
    return auto_cfg(plans[0], [&](const ClipLayout& L) {
        int64_t t = 0;
        for (int i = 0; i < n; ++i) {
            const int64_t K = (lens[i] + plans[i]->hop - 1) / plans[i]->hop;
            t += (K + L.F - 1) / L.F * L.groups;
        }
        return t;
    });
}

// A tuned configuration for this launch (see launch_class), or `cfg` when
// none is recorded, the plan's configuration was set by the caller, or the
// tuned one does not fit one of the launch's hops.
static int with_tuned(const cwt_plan_t* plans, const int64_t* lens, int n, int cfg) {
    const cwt_plan_s* p0 = plans[0];
    if (p0->cfg_user || p0->dt == DT_FP32) return cfg;
    ensure_tuned_loaded();
    if (g_tuned_count.load(std::memory_order_relaxed) == 0) return cfg;
    int hlo = p0->hop, hhi = p0->hop, cnt = 0;
    int64_t sum = 0;
    for (int i = 0; i < n; ++i) {
        if (lens[i] <= 0) continue;
        hlo = std::min(hlo, plans[i]->hop);
        hhi = std::max(hhi, plans[i]->hop);
        sum += lens[i];
        ++cnt;
    }
    if (cnt == 0) return cfg;
    const int t = tuned_lookup(launch_class(p0, hlo, hhi, cnt, sum / cnt));
    if (t < 0 || kMfmaCfgs[t].toep != kMfmaCfgs[cfg].toep) return cfg;   // never across formulations
    for (int i = 0; i < n; ++i)
        if (lens[i] > 0 && !cfg_fits(plans[i], t, plans[i]->hop)) return cfg;
    return t;
}

// ---------------------------------------------------------------------------
// Launch of one clip.
// One clip's kernel record and, for the MFMA path, its layout (*lay) and its
// work-group tiles (*tiles_out: frame tiles x block groups).
static ClipArg make_clip(const cwt_plan_s* p, const float* x, int64_t len, float* out, const MfmaCfg& mc,
                         bool cached_ok, int chunk, ClipLayout* lay, int64_t* tiles_out) {
    ClipArg c;
    std::memset(&c, 0, sizeof(c));
    c.x = x;
    c.out = out;
    c.len = len;
    c.hop = p->hop;
    c.K = (len + p->hop - 1) / p->hop;
    c.wb = 1;
    c.ws = 1;
    if (p->dt == DT_FP32) {
        // four scale groups per work-group from hop kDirectWideHop on (see direct.hip)
        const bool wide = p->hop >= kDirectWideHop;
        const int64_t ng = (int64_t)p->bank->dgroups.size();
        c.ws = wide ? kDirectGroups : 1;
        const int F = wide ? kDirectWideFrames : kDirectFrames;
        c.ntile = (int32_t)((c.K + F - 1) / F);
        if (tiles_out) *tiles_out = (int64_t)c.ntile * (wide ? (ng + kDirectGroups - 1) / kDirectGroups : ng);
        return c;
    }
    const bool cached = cached_ok && (p->lay.s.mode != STAGE_LINEAR || chunk == p->lay_chunk);
    const ClipLayout L = cached ? p->lay : clip_layout(p->dt, *p->bank, p->hop, mc, chunk);
    c.ntile = (int32_t)((c.K + L.F - 1) / L.F);
    c.mode = L.s.mode;
    c.copies = L.s.copies;
    c.swz = L.s.swz;
    c.cso = L.s.cso;
    c.wb = L.wb;
    c.ws = L.ws;
    if (lay) *lay = L;
    if (tiles_out) *tiles_out = (int64_t)c.ntile * L.groups;
    return c;
}

static cwt_status launch_one(const cwt_plan_s* p, int cfg, const float* x, int64_t len, float* out,
                             hipStream_t stream) {
    const Bank& bk = *p->bank;
    int64_t tiles = 0;
    if (p->dt == DT_FP32) {
        DirectArgs a;
        std::memset(&a, 0, sizeof(a));
        a.taps = bk.d_dtaps;
        a.groups = bk.d_dgroups;
        a.ngroups = (int)bk.dgroups.size();
        a.signed_out = p->signed_out;
        a.clip = make_clip(p, x, len, out, kMfmaCfgs[0], false, 8, nullptr, &tiles);
        a.xcd_remap = 1;
        HIP_TRY(launch_direct(a, stream), "direct launch");
        return CWT_OK;
    }
    const MfmaCfg& c = kMfmaCfgs[cfg];
    if (c.toep) {
        MfmaArgs a;
        std::memset(&a, 0, sizeof(a));
        a.signed_out = p->signed_out;
        a.tfrags = bk.d_tfrags;
        a.tgroups = bk.d_tgroups;
        a.ntgroups = (int)bk.tgroups.size();
        a.toep_bg = c.wb;
        ClipLayout L;
        a.clip = make_clip(p, x, len, out, c, cfg == p->cfg, 8, &L, &tiles);
        if (L.s.mode != STAGE_TOEP) return fail(CWT_ERR_INTERNAL, "Toeplitz configuration without Toeplitz tiles");
        a.shm_bytes = (int32_t)layout_lds(L);
        if (tiles > 0x7fffffff) return fail(CWT_ERR_INVALID_ARG, "signal too long for one launch");
        HIP_TRY(launch_toep(p->dt, c.A, a, (int)tiles, stream), "Toeplitz launch");
        return CWT_OK;
    }
    const int chunk = pick_chunk(p->dt, p->hop, 128 * c.A, c.chunk);
    const SplitGeo sg = split_geo(p->dt, (int)bk.blocks.size());
    MfmaArgs a;
    std::memset(&a, 0, sizeof(a));
    a.frags = bk.d_frags;
    a.blocks = bk.d_blocks;
    a.ngroups = (int)bk.blocks.size();
    a.signed_out = p->signed_out;
    a.chunk_steps = chunk;
    a.frames = 128 * c.A;
    a.split_wb = sg.wb;
    a.split_chunk = sg.chunk;
    ClipLayout L;
    a.clip = make_clip(p, x, len, out, c, cfg == p->cfg, chunk, &L, &tiles);
    a.buf_bytes = L.s.mode == STAGE_WIN ? 0 : (int32_t)L.s.bytes;
    a.raw_bytes = (int32_t)L.s.raw_bytes;
    a.shm_bytes = (int32_t)layout_lds(L);
    a.xcd_remap = 1;
    if (tiles > 0x7fffffff) return fail(CWT_ERR_INVALID_ARG, "signal too long for one launch");
    HIP_TRY(launch_mfma(p->dt, c.A, 1, a, 0, (int)tiles, stream), "mfma launch");
    return CWT_OK;
}

// ---------------------------------------------------------------------------
// Batch contexts.
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy_node = nullptr;
    hipGraphNode_t kernel_node = nullptr;
    MfmaArgs args;            // kernel arguments of the last replay
    size_t copy_bytes = 0;    // descriptor bytes of the last replay
};

// Everything a persistent batch launch needs, computed on the host from the
// batch alone (batch_prepare); the descriptors themselves go to a caller's
// host buffer, laid out as [int32 nclips, int32 total_tiles, pad to 16]
// [ClipArg x nc] [int32 prefix x (nc+1)], nc = clips with len > 0.
struct BatchLaunch {
    bool fp32 = false;
    int nc = 0;              // clips in the launch (len > 0), longest first
    int64_t total = 0;       // tiles over all clips
    size_t used_bytes = 0;   // descriptor bytes
    int dt = 0, A = 1, pkind = 0, grid = 0;
    MfmaArgs a;              // clips / tile_prefix filled in by batch_launch
    DirectArgs d;
};

struct cwt_batch_s {
    int device = 0;
    int max_clips = 0;
    int cus = 0;
    size_t desc_cap = 0;
    uint8_t* pinned[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    int flip = 0;
    // Two device descriptor buffers; shadow[i] is what d_desc[i] holds (or will
    // hold once its upload has run), ddone[i] completes after the last launch
    // that read it.
    uint8_t* d_desc[2] = {nullptr, nullptr};
    std::vector<uint8_t> shadow[2];
    hipEvent_t ddone[2] = {nullptr, nullptr};
    hipStream_t dstream[2] = {nullptr, nullptr};
    bool dused[2] = {false, false};
    // launches reading d_desc[i] queued on dstream[i] since ddone[i] was last
    // recorded: the event is recorded only when something has to wait for
    // them (an upload into the buffer, a launch from another stream), since
    // an event marker between two launches holds the second one back
    bool dpending[2] = {false, false};
    int dnext = 0;
    hipStream_t cap_stream = nullptr;
    std::map<std::tuple<int, int, int, int, int, int>, GraphEntry> graphs;
    std::mutex mu;
    // Prepared launches: pkey[i] describes the call (epoch, forced
    // configuration, and per clip plan id, input, length, output) whose
    // descriptors d_desc[i] holds and whose launch record is pbl[i]; a call
    // with the same key reuses both without preparing anything on the host.
    std::vector<uint64_t> pkey[2];
    BatchLaunch pbl[2];
    std::vector<uint64_t> kbuf;

    ~cwt_batch_s() {
        for (int i = 0; i < 2; ++i) {
            if (done[i]) {
                (void)hipEventSynchronize(done[i]);
                (void)hipEventDestroy(done[i]);
            }
            if (pinned[i]) (void)hipHostFree(pinned[i]);
        }
        for (auto& kv : graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        }
        // launches still reading the descriptors (their stream may be gone)
        if (dpending[0] || dpending[1]) (void)hipDeviceSynchronize();
        for (int i = 0; i < 2; ++i) {
            if (ddone[i]) {
                (void)hipEventSynchronize(ddone[i]);
                (void)hipEventDestroy(ddone[i]);
            }
            if (d_desc[i]) (void)hipFree(d_desc[i]);
        }
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

// Descriptor buffer: [int32 nclips, int32 total_tiles, pad to 16] [ClipArg x n] [int32 prefix x (n+1)]
static size_t desc_bytes(int n) {
    return 16 + sizeof(ClipArg) * (size_t)n + sizeof(int32_t) * (size_t)(n + 1) + 16;
}

static cwt_status batch_init(cwt_batch_s* b, int max_clips) {
    DeviceInfo di;
    cwt_status st = current_device(&b->device, &di);
    if (st != CWT_OK) return st;
    b->cus = di.cus;
    b->max_clips = max_clips;
    b->desc_cap = desc_bytes(max_clips);
    b->kbuf.reserve(4 + 4 * (size_t)max_clips);
    for (int i = 0; i < 2; ++i) b->pkey[i].reserve(4 + 4 * (size_t)max_clips);
    for (int i = 0; i < 2; ++i) {
        HIP_TRY(hipHostMalloc((void**)&b->pinned[i], b->desc_cap, hipHostMallocDefault), "pinned descriptors");
        HIP_TRY(hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming), "batch event");
    }
    for (int i = 0; i < 2; ++i) {
        HIP_TRY(hipMalloc(&b->d_desc[i], b->desc_cap), "device descriptors");
        HIP_TRY(hipEventCreateWithFlags(&b->ddone[i], hipEventDisableTiming), "descriptor event");
    }
    HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "capture stream");
    HIP_TRY(hipDeviceSynchronize(), "batch init");
    return CWT_OK;
}

// Persistent grid: every work-group resident (CUs x occupancy), reduced to
// the nearest size coprime with `groups` (the lcm of the clips' block-group
// counts) so that the static tile stride rotates each work-group through
// the groups.
static int persistent_grid(int cus, int dt, int A, int kind, int64_t lds_bytes, int64_t groups) {
    const int per_cu = mfma_occupancy(dt, A, 0, kind, (size_t)lds_bytes);
    int g = cus * std::max(1, per_cu);
    while (g > 1 && gcd64(g, std::max<int64_t>(1, groups)) != 1) --g;
    return g;
}


// Host scratch batch_prepare needs for n clips: order[n], clips[n], ctiles[n].
struct BatchScratch {
    int* order;
    ClipArg* clips;
    int64_t* ctiles;
};

static cwt_status batch_validate(const cwt_plan_t* plans, const float* const* xs, const int64_t* lens,
                                 float* const* outs, int32_t n) {
    if (!plans || !xs || !lens || !outs) return fail(CWT_ERR_INVALID_ARG, "NULL batch array");
    const cwt_plan_s* p0 = plans[0];
    if (!p0) return fail(CWT_ERR_INVALID_ARG, "NULL plan");
    for (int i = 0; i < n; ++i) {
        const cwt_plan_s* p = plans[i];
        if (!p) return fail(CWT_ERR_INVALID_ARG, "NULL plan in batch");
        if (p->bank != p0->bank || p->signed_out != p0->signed_out)
            return fail(CWT_ERR_UNSUPPORTED, "batch plans differ in dtype, scales or output mode");
        if (lens[i] < 0) return fail(CWT_ERR_INVALID_ARG, "negative length in batch");
        if (lens[i] > 0 && (!xs[i] || !outs[i])) return fail(CWT_ERR_INVALID_ARG, "NULL buffer in batch");
        int64_t K = (lens[i] + p->hop - 1) / p->hop;
        if (K > 0 && (int64_t)p->bank->scales.size() > INT64_MAX / K)
            return fail(CWT_ERR_INVALID_ARG, "output size overflows int64");
    }
    return CWT_OK;
}

// Configuration, chunk, per-clip records (longest first) and launch geometry
// of a validated batch; descriptors written to `host` (host_cap bytes).  No
// device work and no heap allocation beyond what the caller passes in.
static cwt_status batch_prepare(const cwt_plan_t* plans, const float* const* xs, const int64_t* lens,
                                float* const* outs, int32_t n, int cus, int force_cfg, const BatchScratch& sc,
                                uint8_t* host, size_t host_cap, BatchLaunch* bl) {
    const cwt_plan_s* p0 = plans[0];
    const Bank& bk = *p0->bank;

    // One configuration for the whole launch (the first plan's) and one chunk
    // for its chunked LINEAR clips: the largest for which the worst such clip's
    // LDS (operand buffers plus raw window) fits the budget.  WIN and SPLIT
    // clips have a fixed geometry per (bank, hop, configuration).
    const bool fp32 = p0->dt == DT_FP32;
    int cfg = force_cfg >= 0 ? force_cfg : with_tuned(plans, lens, n, batch_auto_cfg(plans, lens, n));
    // Clips of Toeplitz plans run Toeplitz tiles of kToepBatchNB blocks per
    // wave whatever the launch's configuration; the configuration then
    // describes the batch's other clips (6 when it names Toeplitz tiles).
    if (!fp32 && kMfmaCfgs[cfg].toep) cfg = 6;
    MfmaCfg c = kMfmaCfgs[fp32 ? 0 : cfg];
    bool cached_ok = true;   // plans[i]->lay is valid for this launch when plans[i]->cfg == cfg
    int chunk = 8;
    bool any_linear = false, all_win = true;
    auto scan = [&]() {
        any_linear = false;
        all_win = true;
        for (int i = 0; i < n && !fp32; ++i)
            if (lens[i] > 0) {
                if (plan_toep(plans[i])) {
                    all_win = false;   // the every-layout kernel runs Toeplitz tiles
                    continue;
                }
                const ClipLayout& L = plans[i]->cfg == cfg ? plans[i]->lay
                                      : clip_layout(p0->dt, bk, plans[i]->hop, c, c.chunk);
                any_linear = any_linear || L.s.mode == STAGE_LINEAR;
                all_win = all_win && L.s.mode == STAGE_WIN;
            }
    };
    scan();
    bool fp8_large_hop = false;
    for (int i = 0; i < n; ++i) fp8_large_hop = fp8_large_hop || plans[i]->hop > kFp8SegmentMaxHop;
    if (p0->dt == DT_FP8 && cfg != kFp8Cfg && (!all_win || fp8_large_hop)) {
        // every FP8 tile must lie in one 128-frame segment, and clips beyond
        // hop 128 (a scale per tile) have only configuration 5: a clip that
        // this configuration gives chunked (256-frame) tiles, or one beyond
        // hop 128, sends the batch to 5
        cfg = kFp8Cfg;
        c = kMfmaCfgs[cfg];
        scan();
    }
    if (c.A == 8 && !all_win) {
        // 256-frame waves exist for WIN tiles only: run this batch with A = 4
        c.A = 4;
        cached_ok = false;
        any_linear = false;
        for (int i = 0; i < n; ++i)
            if (lens[i] > 0 && !plan_toep(plans[i]))
                any_linear = any_linear || clip_layout(p0->dt, bk, plans[i]->hop, c, c.chunk).s.mode == STAGE_LINEAR;
    }
    if (any_linear) {
        for (int ch = c.chunk; ch >= 8; ch -= 8) {
            int64_t mb = 0, mr = 0;
            for (int i = 0; i < n; ++i) {
                if (lens[i] == 0 || plan_toep(plans[i])) continue;
                const ClipLayout L = clip_layout(p0->dt, bk, plans[i]->hop, c, ch);
                if (L.s.mode != STAGE_LINEAR) continue;
                mb = std::max(mb, L.s.bytes);
                mr = std::max(mr, L.s.raw_bytes);
            }
            if (2 * mb + mr <= kLdsBudget) {
                chunk = ch;
                break;
            }
        }
    }
    const SplitGeo sg = fp32 ? SplitGeo{1, 32, 8, 1} : split_geo(p0->dt, (int)bk.blocks.size());

    int nc = 0;
    for (int i = 0; i < n; ++i)
        if (lens[i] > 0) sc.order[nc++] = i;
    bl->fp32 = fp32;
    bl->nc = nc;
    if (nc == 0) return CWT_OK;
    // A batch of Toeplitz clips only runs them in one grid of their
    // single-clip tiles (k_toep_batch); Toeplitz clips among others run in
    // the every-layout persistent kernel with kToepBatchNB blocks per wave.
    bool toep_only = !fp32;
    for (int j = 0; j < nc; ++j) toep_only = toep_only && plan_toep(plans[sc.order[j]]);
    const int tcfg = toep_only ? toep_batch_cfg(bk, cus, nc, [&](int j) { return lens[sc.order[j]]; }) : kToepBatchCfg;
    const MfmaCfg& ct = kMfmaCfgs[tcfg];
    // Longest first (most tiles first) so the persistent grid drains evenly.
    int64_t maxbuf = 16, maxraw = 0, maxwin = 0;
    for (int j = 0; j < nc; ++j) {
        const int i = sc.order[j];
        ClipLayout L;
        const bool tp = plan_toep(plans[i]);
        sc.clips[i] = make_clip(plans[i], xs[i], lens[i], outs[i], tp ? ct : c,
                                !tp && cached_ok && plans[i]->cfg == cfg, chunk, &L, &sc.ctiles[i]);
        if (fp32) continue;
        if (L.s.mode == STAGE_WIN || L.s.mode == STAGE_TOEP) {
            maxwin = std::max(maxwin, L.s.bytes);
        } else {
            maxbuf = std::max(maxbuf, L.s.bytes);
            maxraw = std::max(maxraw, L.s.raw_bytes);
        }
    }
    // (most tiles first, then input order: what a stable sort gives, without
    // its temporary buffer)
    std::sort(sc.order, sc.order + nc, [&](int a, int bq) {
        return sc.ctiles[a] != sc.ctiles[bq] ? sc.ctiles[a] > sc.ctiles[bq] : a < bq;
    });
    const size_t used_bytes = 16 + sizeof(ClipArg) * nc + sizeof(int32_t) * (nc + 1);
    if (used_bytes > host_cap) return fail(CWT_ERR_INTERNAL, "descriptor buffer too small");
    ClipArg* hc = (ClipArg*)(host + 16);
    int32_t* hp = (int32_t*)(host + 16 + sizeof(ClipArg) * nc);
    int64_t total = 0;
    for (int j = 0; j < nc; ++j) {
        hc[j] = sc.clips[sc.order[j]];
        hp[j] = (int32_t)total;
        total += sc.ctiles[sc.order[j]];
        if (total > 0x7fffffff) return fail(CWT_ERR_INVALID_ARG, "batch has too many tiles");
    }
    hp[nc] = (int32_t)total;
    std::memset(host, 0, 16);
    ((int32_t*)host)[0] = nc;
    ((int32_t*)host)[1] = (int32_t)total;
    bl->total = total;
    bl->used_bytes = used_bytes;
    bl->dt = p0->dt;
    bl->A = c.A;

    if (fp32) {
        std::memset(&bl->d, 0, sizeof(bl->d));
        bl->d.taps = bk.d_dtaps;
        bl->d.groups = bk.d_dgroups;
        bl->d.ngroups = (int)bk.dgroups.size();
        bl->d.signed_out = p0->signed_out;
        return CWT_OK;
    }
    MfmaArgs& a = bl->a;
    std::memset(&a, 0, sizeof(a));
    a.frags = bk.d_frags;
    a.blocks = bk.d_blocks;
    a.ngroups = (int)bk.blocks.size();
    a.signed_out = p0->signed_out;
    a.chunk_steps = chunk;
    a.frames = 128 * c.A;
    a.split_wb = sg.wb;
    a.split_chunk = sg.chunk;
    a.buf_bytes = (int32_t)maxbuf;
    a.raw_bytes = (int32_t)maxraw;
    a.shm_bytes = (int32_t)std::max(2 * maxbuf + maxraw, maxwin);
    a.xcd_remap = 0;
    a.nclips = nc;
    a.total_tiles = (int32_t)total;
    bool any_toep = false;
    for (int j = 0; j < nc; ++j) any_toep = any_toep || hc[j].mode == STAGE_TOEP;
    if (any_toep) {   // the bank's Toeplitz part is built (a Toeplitz plan exists)
        a.tfrags = bk.d_tfrags;
        a.tgroups = bk.d_tgroups;
        a.ntgroups = (int)bk.tgroups.size();
        a.toep_bg = kMfmaCfgs[kToepBatchCfg].wb;
    }
    if (toep_only) {   // one grid of the clips' tiles, ct.A 1024-frame blocks per wave
        bl->pkind = 4;
        bl->A = ct.A;
        bl->grid = (int)total;
        return CWT_OK;
    }
    // WIN-only batches run the kernel compiled for the WIN register budget.
    bool win_only = true;
    for (int j = 0; j < nc; ++j) win_only = win_only && hc[j].mode == STAGE_WIN;
    bl->pkind = win_only ? 2 : 1;
    int64_t groups_lcm = 1;
    for (int j = 0; j < nc; ++j) {
        const int64_t ng = hc[j].mode == STAGE_WIN ? (a.ngroups + hc[j].wb - 1) / hc[j].wb
                           : hc[j].mode == STAGE_TOEP ? (a.toep_bg == 2 ? (a.ntgroups + 1) / 2 : a.ntgroups)
                           : hc[j].mode == STAGE_LINEAR ? a.ngroups : sg.groups;
        groups_lcm = groups_lcm / gcd64(groups_lcm, ng) * ng;
        if (groups_lcm > 4096) groups_lcm = 4096;   // bounded: a heuristic, not a requirement
    }
    bl->grid = (int)std::min<int64_t>(persistent_grid(cus, p0->dt, c.A, bl->pkind, a.shm_bytes, groups_lcm), total);
    return CWT_OK;
}

// Point a prepared launch at descriptors resident at device address dd.
static void batch_bind(BatchLaunch* bl, const uint8_t* dd) {
    bl->a.clips = (const ClipArg*)(dd + 16);
    bl->a.tile_prefix = (const int32_t*)(dd + 16 + sizeof(ClipArg) * bl->nc);
}

// The persistent launch (or the plain path's flat launch) of a prepared and
// bound batch whose descriptors are in device memory at dd.
static hipError_t batch_launch(const BatchLaunch& bl, const uint8_t* dd, hipStream_t stream) {
    if (bl.fp32)
        return launch_direct_batch(bl.d, (const ClipArg*)(dd + 16), (const int32_t*)(dd + 16 + sizeof(ClipArg) * bl.nc),
                                   bl.nc, (int)bl.total, stream);
    if (bl.pkind == 4) return launch_toep_batch(bl.dt, bl.A, bl.a, bl.grid, stream);
    return launch_mfma(bl.dt, bl.A, 1, bl.a, bl.pkind, bl.grid, stream);
}

// Make `stream` wait for the launches that read descriptor buffer ds
// (recording their event first if it is pending).
static hipError_t wait_desc(cwt_batch_s* b, int ds, hipStream_t stream) {
    if (!b->dused[ds]) return hipSuccess;
    if (b->dpending[ds]) {
        hipError_t e = hipEventRecord(b->ddone[ds], b->dstream[ds]);
        if (e != hipSuccess) return e;
        b->dpending[ds] = false;
    }
    return hipStreamWaitEvent(stream, b->ddone[ds], 0);
}

static cwt_status batch_run(cwt_batch_s* b, const cwt_plan_t* plans, const float* const* xs,
                            const int64_t* lens, float* const* outs, int32_t n, int use_graph,
                            hipStream_t stream, int force_cfg = -1) {
    if (n < 0) return fail(CWT_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return CWT_OK;
    if (n > b->max_clips) return fail(CWT_ERR_INVALID_ARG, "batch larger than the context's max_clips");
    cwt_status st = batch_validate(plans, xs, lens, outs, n);
    if (st != CWT_OK) return st;
    const cwt_plan_s* p0 = plans[0];
    if (p0->device != b->device) return fail(CWT_ERR_INVALID_ARG, "plan and batch context on different devices");

    // The call's key: a prepared launch with the same key (the same plans,
    // buffers and lengths under the same configuration epoch) is run again
    // as it is, its descriptors already resident.  kbuf's capacity is
    // reserved at creation: no allocation here.
    std::vector<uint64_t>& ckey = b->kbuf;
    ckey.clear();
    ckey.push_back((uint64_t)n);
    ckey.push_back((uint64_t)(int64_t)force_cfg);
    ckey.push_back(g_cfg_epoch.load());
    for (int i = 0; i < n; ++i) {
        ckey.push_back(plans[i]->uid);
        ckey.push_back((uint64_t)(uintptr_t)xs[i]);
        ckey.push_back((uint64_t)lens[i]);
        ckey.push_back((uint64_t)(uintptr_t)outs[i]);
    }
    int ds = -1;
    for (int i = 0; i < 2; ++i)
        if (b->pkey[i].size() == ckey.size() && std::memcmp(b->pkey[i].data(), ckey.data(), ckey.size() * 8) == 0) ds = i;
    BatchLaunch bl;
    bool upload = false;
    const int slot = b->flip;
    uint8_t* host = b->pinned[slot];
    size_t used_bytes = 0;
    if (ds >= 0) {
        bl = b->pbl[ds];
        used_bytes = bl.used_bytes;
        if (b->dused[ds] && b->dstream[ds] != stream) HIP_TRY(wait_desc(b, ds, stream), "descriptor upload wait");
    } else {
        // Wait until the pinned buffer we are about to overwrite has been consumed.
        b->flip ^= 1;
        if (b->used[slot]) HIP_TRY(hipEventSynchronize(b->done[slot]), "batch reuse wait");
        std::vector<int> order(n);
        std::vector<ClipArg> clips(n);
        std::vector<int64_t> ctiles(n, 0);
        st = batch_prepare(plans, xs, lens, outs, n, b->cus, force_cfg,
                           BatchScratch{order.data(), clips.data(), ctiles.data()}, host, b->desc_cap, &bl);
        if (st != CWT_OK || bl.nc == 0) return st;
        used_bytes = bl.used_bytes;

        // Device descriptors: reuse the buffer that already holds exactly these
        // (no upload); otherwise overwrite the other one once the launches that
        // read it have completed.
        for (int i = 0; i < 2; ++i)
            if (b->shadow[i].size() == used_bytes && std::memcmp(b->shadow[i].data(), host, used_bytes) == 0) ds = i;
        upload = ds < 0;
        if (upload) {
            ds = b->dnext;
            b->dnext ^= 1;
            HIP_TRY(wait_desc(b, ds, stream), "descriptor reuse wait");
            b->shadow[ds].assign(host, host + used_bytes);
        } else if (b->dused[ds] && b->dstream[ds] != stream) {
            HIP_TRY(wait_desc(b, ds, stream), "descriptor upload wait");
        }
        batch_bind(&bl, b->d_desc[ds]);
        b->pkey[ds].assign(ckey.begin(), ckey.end());
        b->pbl[ds] = bl;
    }
    uint8_t* const dd = b->d_desc[ds];
    batch_bind(&bl, dd);
    auto finish = [&]() -> cwt_status {
        if (upload) {   // the copy reads the pinned buffer: its next writer waits for this
            HIP_TRY(hipEventRecord(b->done[slot], stream), "batch event");
            b->used[slot] = true;
        }
        b->dused[ds] = true;
        b->dstream[ds] = stream;
        b->dpending[ds] = true;
        return CWT_OK;
    };

    if (bl.fp32 || !use_graph) {
        // descriptor upload (unless resident) and one launch
        if (upload) HIP_TRY(hipMemcpyAsync(dd, host, used_bytes, hipMemcpyHostToDevice, stream), "descriptor upload");
        HIP_TRY(batch_launch(bl, dd, stream), bl.fp32 ? "direct batch launch" : "persistent launch");
        return finish();
    }
    const MfmaArgs& a = bl.a;
    // One graph per (shape, pinned buffer, device buffer, with or without
    // the upload): the copy's source and destination are then fixed, and
    // its size and the kernel arguments (counts, chunk) are refreshed only
    // when they differ from the previous replay.
    auto key = std::make_tuple(bl.dt, bl.A, (int)a.shm_bytes, bl.grid, bl.pkind, 4 * slot + 2 * ds + (upload ? 1 : 0));
    GraphEntry& ge = b->graphs[key];
    if (!ge.exec) {
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        hipError_t e1 = upload ? hipMemcpyAsync(dd, host, used_bytes, hipMemcpyHostToDevice, b->cap_stream)
                               : hipSuccess;
        hipError_t e2 = batch_launch(bl, dd, b->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e3 = hipStreamEndCapture(b->cap_stream, &g);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            b->graphs.erase(key);
            return fail(CWT_ERR_DEVICE, "graph capture failed");
        }
        ge.graph = g;
        size_t nn = 0;
        HIP_TRY(hipGraphGetNodes(g, nullptr, &nn), "graph nodes");
        std::vector<hipGraphNode_t> nodes(nn);
        HIP_TRY(hipGraphGetNodes(g, nodes.data(), &nn), "graph nodes");
        for (auto nd : nodes) {
            hipGraphNodeType t;
            HIP_TRY(hipGraphNodeGetType(nd, &t), "graph node type");
            if (t == hipGraphNodeTypeMemcpy) ge.copy_node = nd;
            if (t == hipGraphNodeTypeKernel) ge.kernel_node = nd;
        }
        if ((upload && !ge.copy_node) || !ge.kernel_node) return fail(CWT_ERR_INTERNAL, "unexpected graph shape");
        HIP_TRY(hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0), "graph instantiate");
        std::memcpy(&ge.args, &a, sizeof(a));   // padding included, for the memcmp below
        ge.copy_bytes = used_bytes;
    } else {
        if (upload && ge.copy_bytes != used_bytes) {
            HIP_TRY(hipGraphExecMemcpyNodeSetParams1D(ge.exec, ge.copy_node, dd, host, used_bytes,
                                                      hipMemcpyHostToDevice), "graph copy update");
            ge.copy_bytes = used_bytes;
        }
        if (std::memcmp(&ge.args, &a, sizeof(a)) != 0) {
            hipKernelNodeParams kp;
            HIP_TRY(hipGraphKernelNodeGetParams(ge.kernel_node, &kp), "kernel node params");
            MfmaArgs ak = a;
            void* args[1] = {&ak};
            kp.kernelParams = args;
            kp.extra = nullptr;
            HIP_TRY(hipGraphExecKernelNodeSetParams(ge.exec, ge.kernel_node, &kp), "kernel node update");
            std::memcpy(&ge.args, &a, sizeof(a));
        }
    }
    HIP_TRY(hipGraphLaunch(ge.exec, stream), "graph launch");
    return finish();
}

// Implicit batch contexts, one per (thread, device, stream).
// They live until the process ends (never torn down after the HIP runtime).
static thread_local std::map<std::pair<int, void*>, cwt_batch_s*> t_batches;

// ---------------------------------------------------------------------------
// Exported ABI.
extern "C" {

const char* cwt_status_string(cwt_status s) {
    switch (s) {
        case CWT_OK: return "CWT_OK";
        case CWT_ERR_INVALID_ARG: return "CWT_ERR_INVALID_ARG";
        case CWT_ERR_UNSUPPORTED: return "CWT_ERR_UNSUPPORTED";
        case CWT_ERR_OUT_OF_MEMORY: return "CWT_ERR_OUT_OF_MEMORY";
        case CWT_ERR_DEVICE: return "CWT_ERR_DEVICE";
        case CWT_ERR_INTERNAL: return "CWT_ERR_INTERNAL";
    }
    return "CWT_ERR_UNKNOWN";
}

const char* cwt_last_error(void) { return g_last_error.c_str(); }

const char* cwt_version(void) { return "1.0.0 gfx950"; }

cwt_status cwt_plan_create(double fs, cwt_wavelet wavelet, const double* scales, int32_t n_scales,
                           int32_t hop, cwt_dtype dtype, cwt_plan_t* plan_out) {
    try {
        if (!plan_out) return fail(CWT_ERR_INVALID_ARG, "plan_out is NULL");
        if (!(fs > 0.0) || !std::isfinite(fs)) return fail(CWT_ERR_INVALID_ARG, "fs must be finite and > 0");
        if (n_scales < 1 || n_scales > 4096) return fail(CWT_ERR_INVALID_ARG, "n_scales must be in [1, 4096]");
        if (!scales) return fail(CWT_ERR_INVALID_ARG, "scales is NULL");
        if (hop < 1) return fail(CWT_ERR_INVALID_ARG, "hop must be >= 1");
        for (int i = 0; i < n_scales; ++i) {
            double s = scales[i];
            if (!std::isfinite(s) || !(s > 0.0) || std::floor(8.0 * s) > 131072.0)
                return fail(CWT_ERR_INVALID_ARG, "scale " + std::to_string(i) + " must be finite, > 0 and <= 16384");
        }
        if (wavelet != CWT_WAVELET_MORLET) return fail(CWT_ERR_UNSUPPORTED, "unknown wavelet");
        if ((int)dtype < 0 || (int)dtype > 4) return fail(CWT_ERR_UNSUPPORTED, "unknown dtype");
        DeviceInfo di;
        int dev = 0;
        cwt_status st = current_device(&dev, &di);
        if (st != CWT_OK) return st;
        std::vector<double> sc(scales, scales + n_scales);
        auto p = std::make_unique<cwt_plan_s>();
        p->fs = fs;
        p->hop = hop;
        p->dt = (int)dtype;
        p->device = dev;
        p->cus = di.cus;
        p->arch = di.arch;
        p->arch_hash = fnv1a(di.arch);
        st = acquire_bank(p->dt, dev, sc, &p->bank);
        if (st != CWT_OK) return st;
        {
            static std::once_flag attr_once;   // kernel attributes, never during a graph capture
            hipError_t ae = hipSuccess;
            std::call_once(attr_once, [&] { ae = mfma_init_attributes(); });
            if (ae != hipSuccess) return fail(CWT_ERR_DEVICE, std::string("kernel attributes: ") + hipGetErrorString(ae));
        }
        if (hop == 1 && (p->dt == DT_BF16 || p->dt == DT_FP16) && toep_fits(*p->bank, 1)) {
            st = ensure_toep(*p->bank);
            if (st != CWT_OK) return st;
        }
        set_cfg(p.get(), default_cfg(p.get(), hop));
        if (p->cfg == 6 || p->cfg == kToepCfg0) set_auto(p.get());
        ensure_tuned_loaded();   // here, so that no launch reads the cache file
        // an automatic plan's 6 stands for the per-launch choice (auto_cfg)
        if (!p->cfg_auto && !cfg_fits(p.get(), p->cfg, hop)) {
            bool found = false;
            for (int c = 0; c < (p->dt == DT_FP32 ? 1 : kNumMfmaCfgs); ++c)
                if (cfg_fits(p.get(), c, hop)) {
                    set_cfg(p.get(), c);
                    found = true;
                    break;
                }
            if (!found) return fail(CWT_ERR_UNSUPPORTED, "no kernel configuration fits this hop");
        }
        *plan_out = p.release();
        return CWT_OK;
    } catch (const std::bad_alloc&) {
        return fail(CWT_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

cwt_status cwt_plan_set_output(cwt_plan_t plan, cwt_output mode) {
    if (!plan) return fail(CWT_ERR_INVALID_ARG, "NULL plan");
    if (mode != CWT_OUT_MAGNITUDE && mode != CWT_OUT_SIGNED) return fail(CWT_ERR_INVALID_ARG, "bad output mode");
    plan->signed_out = mode == CWT_OUT_SIGNED;
    return CWT_OK;
}

cwt_status cwt_plan_destroy(cwt_plan_t plan) {
    if (!plan) return CWT_OK;
    (void)hipDeviceSynchronize();
    delete plan;
    return CWT_OK;
}

int64_t cwt_num_frames(cwt_plan_t plan, int64_t len) {
    if (!plan || len < 0) return -1;
    return (len + plan->hop - 1) / plan->hop;
}

int32_t cwt_plan_num_scales(cwt_plan_t plan) { return plan ? (int32_t)plan->bank->scales.size() : -1; }
int32_t cwt_plan_hop(cwt_plan_t plan) { return plan ? plan->hop : -1; }

cwt_status cwt_scale_frequencies(cwt_plan_t plan, double* hz_out) {
    if (!plan || !hz_out) return fail(CWT_ERR_INVALID_ARG, "NULL argument");
    const double fc = 5.0 / (2.0 * M_PI);
    for (size_t i = 0; i < plan->bank->scales.size(); ++i) hz_out[i] = fc * plan->fs / plan->bank->scales[i];
    return CWT_OK;
}

cwt_status cwt_execute(cwt_plan_t plan, const float* x, int64_t len, float* out, void* stream) {
    try {
        if (!plan) return fail(CWT_ERR_INVALID_ARG, "NULL plan");
        if (len < 0) return fail(CWT_ERR_INVALID_ARG, "len < 0");
        if (len == 0) return CWT_OK;
        if (!x || !out) return fail(CWT_ERR_INVALID_ARG, "NULL x or out");
        int64_t K = (len + plan->hop - 1) / plan->hop;
        if ((int64_t)plan->bank->scales.size() > INT64_MAX / K)
            return fail(CWT_ERR_INVALID_ARG, "output size overflows int64");
        int cfg = auto_cfg(plan, [&](const ClipLayout& L) { return (K + L.F - 1) / L.F * L.groups; });
        cfg = with_tuned(&plan, &len, 1, cfg);
        return launch_one(plan, cfg, x, len, out, (hipStream_t)stream);
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

cwt_status cwt_batch_create(int32_t max_clips, cwt_batch_t* batch_out) {
    try {
        if (!batch_out) return fail(CWT_ERR_INVALID_ARG, "batch_out is NULL");
        if (max_clips < 1 || max_clips > (1 << 20)) return fail(CWT_ERR_INVALID_ARG, "max_clips must be in [1, 2^20]");
        auto b = std::make_unique<cwt_batch_s>();
        cwt_status st = batch_init(b.get(), max_clips);
        if (st != CWT_OK) return st;
        *batch_out = b.release();
        return CWT_OK;
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

cwt_status cwt_batch_destroy(cwt_batch_t batch) {
    if (!batch) return CWT_OK;
    delete batch;
    return CWT_OK;
}

cwt_status cwt_batch_execute(cwt_batch_t batch, const cwt_plan_t* plans, const float* const* xs,
                             const int64_t* lens, float* const* outs, int32_t n, int32_t use_graph,
                             void* stream) {
    try {
        if (!batch) return fail(CWT_ERR_INVALID_ARG, "NULL batch");
        std::lock_guard<std::mutex> lk(batch->mu);
        return batch_run(batch, plans, xs, lens, outs, n, use_graph, (hipStream_t)stream);
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

cwt_status cwt_execute_batch(const cwt_plan_t* plans, const float* const* xs, const int64_t* lens,
                             float* const* outs, int32_t n, void* stream) {
    try {
        if (n < 0) return fail(CWT_ERR_INVALID_ARG, "n < 0");
        if (n == 0) return CWT_OK;
        if (!plans || !plans[0]) return fail(CWT_ERR_INVALID_ARG, "NULL plans");
        int dev = 0;
        cwt_status st = current_device(&dev, nullptr);
        if (st != CWT_OK) return st;
        auto key = std::make_pair(dev, stream);
        cwt_batch_s*& slot = t_batches[key];
        if (!slot || slot->max_clips < n) {
            int cap = 64;
            while (cap < n) cap *= 2;
            auto b = std::make_unique<cwt_batch_s>();
            st = batch_init(b.get(), cap);
            if (st != CWT_OK) return st;
            delete slot;   // its last replay has completed once a new context is needed
            slot = b.release();
        }
        std::lock_guard<std::mutex> lk(slot->mu);
        // a direct launch: a graph replay adds ~8 us of device-side launch
        // processing per call (the explicit context offers it)
        return batch_run(slot, plans, xs, lens, outs, n, 0, (hipStream_t)stream);
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

cwt_status cwt_execute_batch_noalloc(const cwt_plan_t* plans, const float* const* xs, const int64_t* lens,
                                     float* const* outs, int32_t n, void* stream) {
    static_assert(16 + sizeof(ClipArg) * kNoallocMaxClips + sizeof(int32_t) * (kNoallocMaxClips + 1) <=
                      (size_t)kNoallocScratchBytes, "scratch too small for the clip maximum");
    try {
        if (n < 0) return fail(CWT_ERR_INVALID_ARG, "n < 0");
        if (n == 0) return CWT_OK;
        if (n > kNoallocMaxClips)
            return fail(CWT_ERR_INVALID_ARG, "cwt_execute_batch_noalloc takes at most 512 clips per call");
        cwt_status st = batch_validate(plans, xs, lens, outs, n);
        if (st != CWT_OK) return st;
        const cwt_plan_s* p0 = plans[0];
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess) return fail(CWT_ERR_DEVICE, "hipGetDevice failed");
        if (p0->device != dev) return fail(CWT_ERR_INVALID_ARG, "plans belong to another device than the current one");
        void* sp = nullptr;
        HIP_TRY(scratch_address(dev, &sp), "descriptor scratch address");
        // host working storage on the stack: nothing is allocated
        int order[kNoallocMaxClips];
        ClipArg clips[kNoallocMaxClips];
        int64_t ctiles[kNoallocMaxClips];
        alignas(16) uint8_t host[kNoallocScratchBytes];
        BatchLaunch bl;
        st = batch_prepare(plans, xs, lens, outs, n, p0->cus, -1, BatchScratch{order, clips, ctiles}, host,
                           sizeof(host), &bl);
        if (st != CWT_OK || bl.nc == 0) return st;
        uint8_t* dd = (uint8_t*)sp;
        HIP_TRY(put_desc(host, bl.used_bytes, dd, (hipStream_t)stream), "descriptor write");
        batch_bind(&bl, dd);
        HIP_TRY(batch_launch(bl, dd, (hipStream_t)stream), bl.fp32 ? "direct batch launch" : "persistent launch");
        return CWT_OK;
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

int32_t cwt_plan_config(cwt_plan_t plan) { return plan ? plan->cfg : -1; }

int32_t cwt_plan_launch_config(cwt_plan_t plan, int64_t len, int32_t n_clips) {
    if (!plan || len < 1 || n_clips < 1) return -1;
    if (plan->dt == DT_FP32) return plan->cfg;
    const int64_t K = (len + plan->hop - 1) / plan->hop;
    if (n_clips > 1 && plan_toep(plan))   // batches of Toeplitz clips: one grid of these tiles
        return toep_batch_cfg(*plan->bank, plan->cus, n_clips, [&](int) { return K; });
    const int cfg = auto_cfg(plan, [&](const ClipLayout& L) { return (K + L.F - 1) / L.F * L.groups * n_clips; });
    std::vector<cwt_plan_t> pl(n_clips, plan);
    std::vector<int64_t> ln(n_clips, len);
    return with_tuned(pl.data(), ln.data(), n_clips, cfg);
}

int32_t cwt_plan_config_kind(cwt_plan_t plan, int32_t index) {
    if (!plan) return -1;
    if (plan->dt == DT_FP32) return index == 0 ? 0 : -1;
    if (index < 0 || index >= kNumMfmaCfgs) return -1;
    return kMfmaCfgs[index].toep ? 1 : 0;
}
int32_t cwt_plan_num_configs(cwt_plan_t plan) {
    if (!plan) return -1;
    return plan->dt == DT_FP32 ? 1 : kNumMfmaCfgs;
}

cwt_status cwt_plan_set_config(cwt_plan_t plan, int32_t index) {
    if (!plan) return fail(CWT_ERR_INVALID_ARG, "NULL plan");
    if (!cfg_fits(plan, index, plan->hop)) return fail(CWT_ERR_INVALID_ARG, "configuration does not fit this plan");
    set_cfg(plan, index);
    plan->cfg_user = true;
    return CWT_OK;
}

cwt_status cwt_autotune_batch(const cwt_plan_t* plans, const int64_t* lens, int32_t n, int32_t* chosen_out) {
    try {
        if (n < 1 || !plans || !lens) return fail(CWT_ERR_INVALID_ARG, "need n >= 1 plans and lengths");
        const cwt_plan_s* p0 = plans[0];
        if (!p0) return fail(CWT_ERR_INVALID_ARG, "NULL plan");
        int64_t total_x = 0, total_out = 0, sum = 0;
        int hlo = p0->hop, hhi = p0->hop;
        for (int i = 0; i < n; ++i) {
            if (!plans[i]) return fail(CWT_ERR_INVALID_ARG, "NULL plan");
            if (plans[i]->bank != p0->bank || plans[i]->signed_out != p0->signed_out)
                return fail(CWT_ERR_UNSUPPORTED, "batch plans differ in dtype, scales or output mode");
            if (lens[i] < 1) return fail(CWT_ERR_INVALID_ARG, "lengths must be >= 1");
            const int64_t K = (lens[i] + plans[i]->hop - 1) / plans[i]->hop;
            total_x += lens[i];
            total_out += (int64_t)p0->bank->scales.size() * K;
            sum += lens[i];
            hlo = std::min(hlo, plans[i]->hop);
            hhi = std::max(hhi, plans[i]->hop);
        }
        int dev = 0;
        cwt_status st = current_device(&dev, nullptr);
        if (st != CWT_OK) return st;
        if (p0->device != dev) return fail(CWT_ERR_INVALID_ARG, "plans belong to another device");
        if (p0->dt == DT_FP32) {   // one configuration: nothing to tune
            if (chosen_out) *chosen_out = p0->cfg;
            return CWT_OK;
        }
        // a seeded noise signal (the kernels' cost does not depend on the values)
        std::vector<float> hx((size_t)std::min<int64_t>(total_x, 1 << 20));
        uint32_t r = 1430200u;
        for (auto& v : hx) {
            r = r * 1664525u + 1013904223u;
            v = (float)((int32_t)r) * (1.0f / 2147483648.0f);
        }
        float *x = nullptr, *out = nullptr;
        HIP_TRY(hipMalloc(&x, sizeof(float) * total_x), "autotune input");
        std::unique_ptr<float, void (*)(float*)> gx(x, [](float* q) { (void)hipFree(q); });
        HIP_TRY(hipMalloc(&out, sizeof(float) * total_out), "autotune output");
        std::unique_ptr<float, void (*)(float*)> go(out, [](float* q) { (void)hipFree(q); });
        for (int64_t o = 0; o < total_x; o += (int64_t)hx.size())
            HIP_TRY(hipMemcpy(x + o, hx.data(), sizeof(float) * std::min<int64_t>(hx.size(), total_x - o),
                              hipMemcpyHostToDevice), "autotune input upload");
        std::vector<const float*> xs(n);
        std::vector<float*> outs(n);
        {
            int64_t ox = 0, oo = 0;
            for (int i = 0; i < n; ++i) {
                xs[i] = x + ox;
                outs[i] = out + oo;
                ox += lens[i];
                oo += (int64_t)p0->bank->scales.size() * ((lens[i] + plans[i]->hop - 1) / plans[i]->hop);
            }
        }
        std::unique_ptr<cwt_batch_s> bctx;
        if (n > 1) {
            bctx = std::make_unique<cwt_batch_s>();
            st = batch_init(bctx.get(), n);
            if (st != CWT_OK) return st;
        }
        hipStream_t sm = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&sm, hipStreamNonBlocking), "autotune stream");
        std::unique_ptr<void, void (*)(void*)> gs(sm, [](void* q) { (void)hipStreamDestroy((hipStream_t)q); });
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0), "event");
        HIP_TRY(hipEventCreate(&e1), "event");
        std::unique_ptr<void, void (*)(void*)> ge0(e0, [](void* q) { (void)hipEventDestroy((hipEvent_t)q); });
        std::unique_ptr<void, void (*)(void*)> ge1(e1, [](void* q) { (void)hipEventDestroy((hipEvent_t)q); });
        // the automatic choice for this launch (what runs without tuning)
        const int auto_choice = batch_auto_cfg(plans, lens, n);
        auto run = [&](int cfg) -> cwt_status {
            if (n == 1) return launch_one(p0, cfg, xs[0], lens[0], outs[0], sm);
            return batch_run(bctx.get(), plans, xs.data(), lens, outs.data(), n, 0, sm, cfg);
        };
        // mean of timed launches after two untimed ones, >= 5 launches and
        // >= 20 ms of device time
        auto time_cfg = [&](int cfg, float* ms_out) -> cwt_status {
            for (int w = 0; w < 2; ++w) {
                cwt_status s2 = run(cfg);
                if (s2 != CWT_OK) return s2;
            }
            int reps = 5;
            for (;;) {
                HIP_TRY(hipEventRecord(e0, sm), "event");
                for (int q = 0; q < reps; ++q) {
                    cwt_status s2 = run(cfg);
                    if (s2 != CWT_OK) return s2;
                }
                HIP_TRY(hipEventRecord(e1, sm), "event");
                HIP_TRY(hipEventSynchronize(e1), "event");
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "event");
                if (ms >= 20.0f || reps >= 4096) {
                    *ms_out = ms / reps;
                    return CWT_OK;
                }
                reps *= 4;
            }
        };
        // candidates: the automatic choice, then every configuration of its
        // formulation (scale-block or Toeplitz tiles, whose results differ by
        // rounding) that fits every clip's hop; a batch's Toeplitz clips run
        // one tile size, so only its other clips have a choice
        float auto_ms = 0;
        st = time_cfg(auto_choice, &auto_ms);
        if (st != CWT_OK) return st;
        int best = -1;
        float best_ms = auto_ms;
        const int kind = kMfmaCfgs[auto_choice].toep;
        for (int c = 0; c < kNumMfmaCfgs; ++c) {
            if (kMfmaCfgs[c].toep != kind || (kind && n > 1)) continue;
            bool ok = true;
            for (int i = 0; i < n && ok; ++i) ok = cfg_fits(plans[i], c, plans[i]->hop);
            if (!ok) continue;
            float ms = 0;
            st = time_cfg(c, &ms);
            if (st != CWT_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        HIP_TRY(hipStreamSynchronize(sm), "autotune sync");
        const TuneKey cls = launch_class(p0, hlo, hhi, n, sum / n);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            load_tuned_locked();
            if (best >= 0 && best_ms < (1.0 - kTuneMargin) * auto_ms)
                g_tuned[cls] = best;
            else
                g_tuned.erase(cls);
            g_cfg_epoch.fetch_add(1);
            g_tuned_count = (int)g_tuned.size();
            save_tuned_locked();
        }
        if (chosen_out) *chosen_out = with_tuned(plans, lens, n, auto_choice);
        return CWT_OK;
    } catch (const std::bad_alloc&) {
        return fail(CWT_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

cwt_status cwt_autotune(cwt_plan_t plan, int64_t len, int32_t* chosen_out) {
    if (!plan) return fail(CWT_ERR_INVALID_ARG, "NULL plan");
    return cwt_autotune_batch(&plan, &len, 1, chosen_out);
}

int64_t cwt_image_workspace_bytes(void) { return image_workspace_bytes(); }

cwt_status cwt_scalogram_image(const float* scalogram, int32_t n_scales, int64_t n_frames, float amin, float* image,
                               int32_t height, int32_t width, void* workspace, void* stream) {
    try {
        if (n_scales < 1 || n_frames < 1 || height < 1 || width < 1)
            return fail(CWT_ERR_INVALID_ARG, "n_scales, n_frames, height and width must be >= 1");
        if (!(amin > 0.0f) || !std::isfinite(amin)) return fail(CWT_ERR_INVALID_ARG, "amin must be finite and > 0");
        if (!scalogram || !image || !workspace) return fail(CWT_ERR_INVALID_ARG, "NULL scalogram, image or workspace");
        if ((int64_t)n_scales > INT64_MAX / n_frames) return fail(CWT_ERR_INVALID_ARG, "scalogram size overflows");
        int dev = 0;
        cwt_status st = current_device(&dev, nullptr);
        if (st != CWT_OK) return st;
        HIP_TRY(launch_image(scalogram, n_scales, n_frames, amin, image, height, width, workspace,
                             (hipStream_t)stream), "image launch");
        return CWT_OK;
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

int64_t cwt_decimated_length(int64_t len, int32_t factor) {
    if (len < 0 || factor < 1) return -1;
    return (len + factor - 1) / factor;
}

cwt_status cwt_lowpass_fir(int32_t factor, int32_t n_taps, double* h_out) {
    if (factor < 1) return fail(CWT_ERR_INVALID_ARG, "factor must be >= 1");
    if (n_taps < 1 || n_taps % 2 == 0) return fail(CWT_ERR_INVALID_ARG, "n_taps must be odd and >= 1");
    if (!h_out) return fail(CWT_ERR_INVALID_ARG, "h_out is NULL");
    if (n_taps == 1) {
        h_out[0] = 1.0;
        return CWT_OK;
    }
    const double c = 0.5 * (n_taps - 1);
    double sum = 0.0;
    for (int j = 0; j < n_taps; ++j) {
        const double t = (j - c) / factor;
        const double sinc = t == 0.0 ? 1.0 : std::sin(M_PI * t) / (M_PI * t);
        const double w = 0.54 - 0.46 * std::cos(2.0 * M_PI * j / (n_taps - 1));
        h_out[j] = w * sinc / factor;
        sum += h_out[j];
    }
    for (int j = 0; j < n_taps; ++j) h_out[j] /= sum;
    return CWT_OK;
}

cwt_status cwt_decimate(const float* x, int64_t len, int32_t factor, const float* h, int32_t h_len, float* y,
                        void* stream) {
    try {
        if (len < 0) return fail(CWT_ERR_INVALID_ARG, "len < 0");
        if (factor < 1) return fail(CWT_ERR_INVALID_ARG, "factor must be >= 1");
        if (h_len < 1 || h_len % 2 == 0) return fail(CWT_ERR_INVALID_ARG, "h_len must be odd and >= 1");
        if (len == 0) return CWT_OK;
        if (!x || !h || !y) return fail(CWT_ERR_INVALID_ARG, "NULL x, h or y");
        int dev = 0;
        cwt_status st = current_device(&dev, nullptr);
        if (st != CWT_OK) return st;
        HIP_TRY(launch_decimate(x, len, factor, h, h_len, y, (len + factor - 1) / factor, (hipStream_t)stream),
                "decimate launch");
        return CWT_OK;
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

// Daubechies lowpass filter of `order` vanishing moments by spectral
// factorisation.  |H|^2 = cos^{2N}(w/2) P(sin^2(w/2)) with
// P(y) = sum_{k<N} C(N-1+k, k) y^k; each root y of P gives the pair z, 1/z
// with z + 1/z = 2 - 4y, and the minimum-phase factor keeps |z| < 1:
// H(w) = sqrt(2) ((1 + w)/2)^N prod_i (w - z_i)/(1 - z_i), w = e^{-i omega}.
// The roots of P come from Durand-Kerner iteration, polished by Newton steps.
static void daubechies_taps(int N, double* h_out) {
    using cd = std::complex<double>;
    const int deg = N - 1;
    std::vector<double> p(N);                     // ascending powers of y
    for (int k = 0; k < N; ++k) {
        double c = 1.0;                           // C(N-1+k, k)
        for (int i = 1; i <= k; ++i) c = c * (N - 1 + i) / i;
        p[k] = c;
    }
    auto peval = [&](cd y, cd* dp) {
        cd v = 0.0, d = 0.0;
        for (int k = deg; k >= 0; --k) {
            d = d * y + v;
            v = v * y + p[k];
        }
        if (dp) *dp = d;
        return v;
    };
    std::vector<cd> y(deg);
    for (int i = 0; i < deg; ++i) y[i] = std::pow(cd(0.4, 0.9), i);
    for (int it = 0; it < 2000; ++it) {
        double step = 0.0;
        for (int i = 0; i < deg; ++i) {
            cd den = p[deg];
            for (int k = 0; k < deg; ++k)
                if (k != i) den *= (y[i] - y[k]);
            const cd dy = peval(y[i], nullptr) / den;
            y[i] -= dy;
            step = std::max(step, std::abs(dy) / std::max(1.0, std::abs(y[i])));
        }
        if (step < 1e-15) break;
    }
    for (int i = 0; i < deg; ++i)
        for (int it = 0; it < 3; ++it) {
            cd d;
            const cd v = peval(y[i], &d);
            if (std::abs(d) > 0.0) y[i] -= v / d;
        }
    std::vector<cd> q(1, cd(1.0));                // prod (w - z_i) / (1 - z_i), ascending in w
    for (int i = 0; i < deg; ++i) {
        const cd b = 2.0 - 4.0 * y[i];
        const cd disc = std::sqrt(b * b - 4.0);
        cd z = 0.5 * (b + disc);
        if (std::abs(z) >= 1.0) z = 0.5 * (b - disc);
        std::vector<cd> nq(q.size() + 1, cd(0.0));
        for (size_t k = 0; k < q.size(); ++k) {
            nq[k] -= z * q[k];
            nq[k + 1] += q[k];
        }
        const cd scale = 1.0 / (1.0 - z);
        for (auto& c : nq) c *= scale;
        q.swap(nq);
    }
    std::vector<double> hb(N + 1);                // ((1 + w)/2)^N
    for (int k = 0; k <= N; ++k) {
        double c = 1.0;
        for (int i = 1; i <= k; ++i) c = c * (N - k + i) / i;
        hb[k] = std::ldexp(c, -N);
    }
    for (int k = 0; k < 2 * N; ++k) {
        double acc = 0.0;
        for (int i = 0; i <= N; ++i) {
            const int m = k - i;
            if (m >= 0 && m < (int)q.size()) acc += hb[i] * q[m].real();
        }
        h_out[k] = std::sqrt(2.0) * acc;
    }
}

cwt_status cwt_daubechies(int32_t order, double* h_out) {
    if (order < 1 || order > 10) return fail(CWT_ERR_INVALID_ARG, "order must be in 1 .. 10");
    if (!h_out) return fail(CWT_ERR_INVALID_ARG, "h_out is NULL");
    daubechies_taps(order, h_out);
    return CWT_OK;
}

int64_t cwt_dwt_pyramid_length(int64_t len, int32_t levels) {
    if (len < 1 || levels < 1 || levels > 30) return -1;
    return dwt_pyramid_length(len, levels);
}

cwt_status cwt_dwt_scalogram(const float* x, int64_t len, int32_t clips, const double* h, int32_t h_len,
                             int32_t levels, float* pyramid, float* out, void* stream) {
    try {
        if (len < 1 || len > 0x7fffffffLL) return fail(CWT_ERR_INVALID_ARG, "len must be in 1 .. 2^31 - 1");
        if (clips < 1 || clips > 65535) return fail(CWT_ERR_INVALID_ARG, "clips must be in 1 .. 65535");
        if (levels < 1 || levels > 30) return fail(CWT_ERR_INVALID_ARG, "levels must be in 1 .. 30");
        if (h_len < 2 || h_len > kDwtMaxTaps || h_len % 2) return fail(CWT_ERR_INVALID_ARG, "h_len must be even, 2 .. 64");
        if (!x || !h || !pyramid) return fail(CWT_ERR_INVALID_ARG, "NULL x, h or pyramid");
        DwtFilter f{};
        f.L = h_len;
        for (int k = 0; k < h_len; ++k) {
            if (!std::isfinite(h[k])) return fail(CWT_ERR_INVALID_ARG, "non-finite filter tap");
            f.h[k] = (float)h[k];
            f.g[k] = (float)((k & 1) ? -h[h_len - 1 - k] : h[h_len - 1 - k]);
        }
        int dev = 0;
        cwt_status st = current_device(&dev, nullptr);
        if (st != CWT_OK) return st;
        HIP_TRY(launch_dwt(x, len, clips, f, levels, pyramid, out, (hipStream_t)stream), "dwt launch");
        return CWT_OK;
    } catch (...) {
        return fail(CWT_ERR_INTERNAL, "unexpected exception");
    }
}

cwt_status cwt_plan_bank_taps(cwt_plan_t plan, int32_t scale_index, double* taps_out, int64_t cap) {
    if (!plan || !taps_out) return fail(CWT_ERR_INVALID_ARG, "NULL argument");
    const Bank& bk = *plan->bank;
    if (scale_index < 0 || scale_index >= (int)bk.scales.size()) return fail(CWT_ERR_INVALID_ARG, "scale_index out of range");
    const int pos = bk.caller_to_sorted[scale_index];
    const int M = bk.M_sorted[pos];
    if (cap < 2 * (int64_t)M + 1) return fail(CWT_ERR_INVALID_ARG, "taps_out too small");
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(double) * (2 * M + 1)), "readback buffer");
    std::unique_ptr<double, void (*)(double*)> gd(d, [](double* p) { (void)hipFree(p); });
    HIP_TRY(decode_bank_taps(plan->dt, bk.d_frags, bk.d_blocks, bk.d_dtaps, bk.d_dgroups, pos, M, d, 0), "bank decode");
    HIP_TRY(hipMemcpy(taps_out, d, sizeof(double) * (2 * M + 1), hipMemcpyDeviceToHost), "bank readback");
    return CWT_OK;
}

}  // extern "C"
