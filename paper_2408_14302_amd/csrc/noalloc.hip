// Device memory of the allocation-free batch entry point
// (cwt_execute_batch_noalloc): the batch descriptors live in a file-scope
// device array instead of memory the library allocates, and reach it through
// kernel arguments (no copy from host memory, no staging buffer).
//
// Each GPU holds its own copy of `scratch` for the life of the process.  Host
// code never names the array as a device address: scratch_address() looks
// its address up once per device (hipGetSymbolAddress, with that device
// current) and every kernel argument uses that address.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "cwt_internal.h"

namespace cwth {

static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return hipSuccess;
}

// One piece of the descriptor block, carried in the kernel's arguments.
struct DescPiece {
    uint32_t off;     // byte offset in the destination (a multiple of 16)
    uint32_t words;   // 16-byte words in w[]
    uint4 w[kDescPieceWords];
};

__global__ __launch_bounds__(256) void k_put_desc(DescPiece piece, uint8_t* dst) {
    uint4* d = (uint4*)(dst + piece.off);
    for (uint32_t i = threadIdx.x; i < piece.words; i += blockDim.x) d[i] = piece.w[i];
}

hipError_t put_desc(const uint8_t* host, size_t bytes, uint8_t* dst, hipStream_t s) {
    if (bytes > (size_t)kNoallocScratchBytes) return hipErrorInvalidValue;
    const size_t words = (bytes + 15) / 16;
    for (size_t w0 = 0; w0 < words; w0 += kDescPieceWords) {
        DescPiece pc;
        pc.off = (uint32_t)(16 * w0);
        pc.words = (uint32_t)std::min<size_t>(kDescPieceWords, words - w0);
        const size_t nb = std::min<size_t>(16 * (size_t)pc.words, bytes - 16 * w0);
        std::memcpy(pc.w, host + 16 * w0, nb);
        if (nb < 16 * (size_t)pc.words) std::memset((uint8_t*)pc.w + nb, 0, 16 * (size_t)pc.words - nb);
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(256), 0, s, pc, dst);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace cwth
