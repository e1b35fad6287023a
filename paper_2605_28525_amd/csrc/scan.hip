// Device-wide exclusive prefix sum (reduce-then-scan over tiles of 2048 values).
//
// Used by the radix sort (digit offsets), and to turn per-block chunk counts
// into work-item offsets.  The compaction of occupied hash slots uses the same
// tile pattern with its own fused write-out (build.hip).
#include "internal.h"

namespace mpmx {

__global__ __launch_bounds__(WG) void k_scan_reduce(const unsigned* __restrict__ in, int n, const int* n_dev,
                                                    unsigned* __restrict__ partials) {
    __shared__ unsigned lds[WG / 64];
    const int nn = n_dev ? min(n, *n_dev) : n;
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    unsigned s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int idx = base + j;
        if (idx < nn) s += in[idx];
    }
    unsigned tot;
    wg_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(WG) void k_scan_partials(unsigned* __restrict__ partials, int n_tiles,
                                                      unsigned* total_out) {
    __shared__ unsigned lds[WG / 64];
    unsigned carry = 0;
    for (int base = 0; base < n_tiles; base += WG) {
        int idx = base + threadIdx.x;
        unsigned v = idx < n_tiles ? partials[idx] : 0u;
        unsigned tot;
        unsigned ex = wg_excl_scan(v, lds, &tot);
        if (idx < n_tiles) partials[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(WG) void k_scan_down(const unsigned* __restrict__ in, unsigned* __restrict__ out, int n,
                                                  const int* n_dev, const unsigned* __restrict__ partials) {
    __shared__ unsigned lds[WG / 64];
    const int nn = n_dev ? min(n, *n_dev) : n;
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    unsigned v[SCAN_ITEMS];
    unsigned s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int idx = base + j;
        v[j] = idx < nn ? in[idx] : 0u;
        s += v[j];
    }
    unsigned tot;
    unsigned run = wg_excl_scan(s, lds, &tot) + partials[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int idx = base + j;
        if (idx < n) out[idx] = run;
        run += v[j];
    }
}

hipError_t scan_partials(unsigned* partials, int tiles, unsigned* total_out, hipStream_t s) {
    k_scan_partials<<<1, WG, 0, s>>>(partials, tiles, total_out);
    return hipGetLastError();
}

int scan_partials_size(int n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

// out[i] = sum_{j<i} in[j] for i < n (entries at or beyond the device count
// *n_dev, if given, read as zero); *total_out (device) receives the sum.
hipError_t scan_exclusive(const unsigned* in, unsigned* out, int n, const int* n_dev, unsigned* partials,
                          unsigned* total_out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    k_scan_reduce<<<tiles, WG, 0, s>>>(in, n, n_dev, partials);
    k_scan_partials<<<1, WG, 0, s>>>(partials, tiles, total_out);
    k_scan_down<<<tiles, WG, 0, s>>>(in, out, n, n_dev, partials);
    return hipGetLastError();
}

}  // namespace mpmx
