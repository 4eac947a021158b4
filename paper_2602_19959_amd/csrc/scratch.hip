// The library's fixed per-device working area, for pvf_execute_scratch
// (callers that cannot allocate device memory).
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy, at its own address, until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host that name is a
// stand-in, not a device address); it resolves the device address once per
// device with hipGetSymbolAddress, while that device is current, at engine
// initialisation, and uses that pointer everywhere.
//
// Per-batch regions in the scratch are laid out afresh for every call's batch
// size, so the previous call's data can sit where this call expects zeros:
// the guard rows around each sequence of every activation tensor (the
// convolutions' zero padding) are cleared by zero_guard_rows before the path
// runs.  Everything else a call reads is written by the call first (the
// histogram rows, the activations' interior rows, and the track queue's
// counters, which the ordering kernel resets).
#include <mutex>

#include "pvf_internal.h"

namespace pvf {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_lock;
bool g_resolved[kMaxDevices] = {};
char* g_ptr[kMaxDevices] = {};

// Zero the first and last kGuard rows of every sequence of region blockIdx.y;
// 4-byte stores (row sizes are multiples of 4 bytes).
__global__ __launch_bounds__(256) void zero_guard_rows(GuardZeroArgs a)
{
    const GuardRegion g = a.r[blockIdx.y];
    const int words = g.row_bytes / 4 * kGuard;          // per end of a sequence
    const int64_t total = a.n_seq * 2 * words;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t seq = i / (2 * words);
        const int r = (int)(i - seq * 2 * words);
        const int end = r / words, w = r - end * words;
        const int64_t row = seq * g.rows_per_seq + (end ? g.rows_per_seq - kGuard : 0);
        reinterpret_cast<uint32_t*>(g.base + row * g.row_bytes)[w] = 0u;
    }
}

}  // namespace

char* scratch_base(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_lock);
    if (!g_resolved[device]) {
        void* p = nullptr;
        const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess) {
            (void)hipGetLastError();   // leave no sticky error for the caller's next call
            return nullptr;            // not cached: a later init on this device retries
        }
        g_ptr[device] = static_cast<char*>(p);
        g_resolved[device] = true;
    }
    return g_ptr[device];
}

hipError_t launch_zero_guard_rows(const GuardZeroArgs& a, hipStream_t s)
{
    if (a.n < 1 || a.n > kMaxGuardRegions || a.n_seq < 1) return hipErrorInvalidValue;
    int64_t most = 0;
    for (int i = 0; i < a.n; ++i) {
        if (a.r[i].row_bytes % 4 != 0 || a.r[i].rows_per_seq < 2 * kGuard) return hipErrorInvalidValue;
        const int64_t t = a.n_seq * 2 * (a.r[i].row_bytes / 4 * kGuard);
        most = t > most ? t : most;
    }
    const int64_t blocks = (most + 255) / 256;
    const unsigned gx = (unsigned)(blocks < 1024 ? blocks : 1024);
    hipLaunchKernelGGL(zero_guard_rows, dim3(gx, (unsigned)a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace pvf
