// Allocation-free scan-based active-set query: the mask-domain scratch of the
// scan-based construction (box header, occupancy, flags, Phi, scan partials)
// lives in one fixed static device array instead of a context allocation, for
// callers that cannot allocate device memory.
//
// The array holds a mask domain of at most SB_STATIC_MAX_M blocks (16 MiB in
// all) and stays resident on every device the library runs on until the
// process ends.  Every call on a device uses that device's one copy: the
// header and the occupancy are cleared by each call's own kernels, and calls
// that overlap on one device (two streams, two host threads) race.
#include <mutex>

#include "internal.h"

namespace mpmx {

constexpr long long SB_STATIC_MAX_M = 1ll << 20;  // blocks of the mask domain
constexpr size_t SB_STATIC_BYTES = sb_scratch_size(SB_STATIC_MAX_M);

// Host code must not pass this name to a kernel (it is a host-side stand-in);
// the device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[SB_STATIC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up on the
// first call per device.
hipError_t static_scratch(void** out) {
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

long long scan_active_static_max_blocks() { return SB_STATIC_MAX_M; }

hipError_t launch_scan_active_static(const DevParams& P, const float* x, int n, uint64_t* keys_out,
                                     uint64_t* masks_out, int cap, SbBox* box_host, hipStream_t s) {
    if (sb_scratch_bytes(SB_STATIC_MAX_M) > SB_STATIC_BYTES) return hipErrorInvalidValue;
    void* base = nullptr;
    hipError_t e = static_scratch(&base);
    if (e != hipSuccess) return e;
    const SbScratch S = sb_carve(base, SB_STATIC_MAX_M, nullptr, nullptr);
    e = launch_scan_active(P, x, n, S, keys_out, masks_out, cap, s);
    if (e == hipSuccess) e = hipMemcpyAsync(box_host, S.box, sizeof(SbBox), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

}  // namespace mpmx
