// Device-wide exclusive prefix sum (reduce-then-scan over tiles of 2048 values,
// two launches: tile sums, then each tile scanned from the sum of the tiles
// before it, which every workgroup reads for itself).
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
    // tiles past the device count hold no values (k_scan_down reads only the
    // partials of the tiles below it)
    if (blockIdx.x > 0 && blockIdx.x * SCAN_TILE >= nn) return;
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    // every load issued before the first is consumed: the index is clamped
    // into range and the value masked, rather than the load guarded
    unsigned v[SCAN_ITEMS];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) v[j] = in[max(min(base + j, nn - 1), 0)];
    unsigned s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) s += base + j < nn ? v[j] : 0u;
    unsigned tot;
    wg_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(WG) void k_scan_down(const unsigned* __restrict__ in, unsigned* __restrict__ out, int n,
                                                  const int* n_dev, const unsigned* __restrict__ partials, int tiles,
                                                  unsigned* total_out) {
    __shared__ unsigned lds[WG / 64];
    const int nn = n_dev ? min(n, *n_dev) : n;
    // with a device count, only the tiles that hold values are scanned (the
    // launch is sized for the host bound n); outputs at or past nn are not
    // written then
    const int live = n_dev ? max(1, min(tiles, (nn + SCAN_TILE - 1) / SCAN_TILE)) : tiles;
    if (blockIdx.x >= live) return;
    // the tile's values are loaded before the tile sums are read and scanned
    // (the barriers of that scan would otherwise hold them back)
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    unsigned v[SCAN_ITEMS];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int idx = base + j;
        v[j] = idx < nn ? in[idx] : 0u;
    }
    unsigned before, total;
    tile_offset(partials, blockIdx.x, live, lds, &before, &total);
    if (blockIdx.x == 0 && threadIdx.x == 0 && total_out) *total_out = total;
    unsigned s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) s += v[j];
    unsigned tot;
    unsigned run = wg_excl_scan(s, lds, &tot) + before;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int idx = base + j;
        if (idx < n) out[idx] = run;
        run += v[j];
    }
}

int scan_partials_size(int n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

// out[i] = sum_{j<i} in[j] for i < n; with a device count *n_dev, for
// i < min(n, *n_dev) (entries at or beyond it read as zero and outputs past the
// last tile that holds values are left unwritten); *total_out (device)
// receives the sum.
hipError_t scan_exclusive(const unsigned* in, unsigned* out, int n, const int* n_dev, unsigned* partials,
                          unsigned* total_out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    k_scan_reduce<<<tiles, WG, 0, s>>>(in, n, n_dev, partials);
    k_scan_down<<<tiles, WG, 0, s>>>(in, out, n, n_dev, partials, tiles, total_out);
    return hipGetLastError();
}

}  // namespace mpmx
