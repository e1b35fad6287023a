// Stable LSD radix sort of (u32 key, u32 value) pairs, 8-bit digits.
//
// Each pass is reduce-then-scan: a per-tile digit histogram, a device scan of
// the (digit-major, tile-minor) histogram matrix, then a stable scatter.  A tile
// is 4096 keys; each wave64 owns a contiguous quarter of it.
//
// Histogram: the keys arrive nearly sorted (the previous step's order), so a
// wave counts runs of equal digits among its 64 lanes (a neighbour compare and
// a ballot) and adds each run's length to its digit with one LDS atomic.
// Scatter: each wave ranks its keys round by round with a wave-wide digit match
// (8 ballots) against per-wave running digit counts in LDS, which keeps the
// sort stable without intra-tile barriers until the wave offsets are combined;
// the tile is then reordered by digit in LDS so that the global stores of each
// digit's run are contiguous.
#include "internal.h"

namespace mpmx {

__device__ __forceinline__ unsigned long long digit_match(unsigned dg, bool valid) {
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (dg >> b) & 1u;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__global__ __launch_bounds__(WG) void k_radix_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                   unsigned* __restrict__ hist, int n_tiles) {
    __shared__ unsigned cnt[WG / 64][256];
    for (int t = threadIdx.x; t < (WG / 64) * 256; t += WG) (&cnt[0][0])[t] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const int base = blockIdx.x * SORT_TILE + w * (SORT_TILE / (WG / 64));
    // all loads of the wave's keys first (one round trip), then the counting
    uint32_t k[SORT_ITEMS];
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int pos = base + r * 64 + lane;
        k[r] = pos < n ? keys[pos] : 0u;
    }
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const bool valid = base + r * 64 + lane < n;  // the valid lanes are a prefix of the wave
        const unsigned dg = (k[r] >> shift) & 255u;
        const unsigned prev = __shfl_up(dg, 1);
        const bool start = valid && (lane == 0 || dg != prev);
        const unsigned long long starts = __ballot(start);
        const int n_valid = __popcll(__ballot(valid));
        if (start) {
            const unsigned long long later = starts & ~((2ull << lane) - 1ull);
            const int end = later ? __ffsll((long long)later) - 1 : n_valid;
            atomicAdd(&cnt[w][dg], (unsigned)(end - lane));
        }
    }
    __syncthreads();
    const int t = threadIdx.x;  // one digit per thread (WG == 256)
    hist[(size_t)t * n_tiles + blockIdx.x] = cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
}

__global__ __launch_bounds__(WG) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                      const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                      uint32_t* __restrict__ vout, int n, int shift,
                                                      const unsigned* __restrict__ hist, int n_tiles) {
    __shared__ unsigned run[WG / 64][256];   // per-wave digit counts, then local offsets
    __shared__ int delta[256];               // global minus local position, per digit
    __shared__ unsigned lds_scan[WG / 64];
    __shared__ uint32_t sk[SORT_TILE], sv[SORT_TILE];  // the tile ordered by digit
    for (int t = threadIdx.x; t < (WG / 64) * 256; t += WG) (&run[0][0])[t] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int tile0 = blockIdx.x * SORT_TILE;
    const int base = tile0 + w * (SORT_TILE / (WG / 64));
    uint32_t k[SORT_ITEMS], v[SORT_ITEMS];
    unsigned rk[SORT_ITEMS];
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int pos = base + r * 64 + lane;
        const bool valid = pos < n;
        k[r] = valid ? kin[pos] : 0u;
        v[r] = valid ? (vin ? vin[pos] : (uint32_t)pos) : 0u;
    }
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int pos = base + r * 64 + lane;
        const bool valid = pos < n;
        const unsigned dg = (k[r] >> shift) & 255u;
        const unsigned long long m = digit_match(dg, valid);
        const unsigned cur = run[w][dg];
        rk[r] = cur + (unsigned)__popcll(m & lt);
        if (valid && (__ffsll((long long)m) - 1) == lane) run[w][dg] = cur + (unsigned)__popcll(m);
    }
    __syncthreads();
    {
        // digit t: its first slot in the tile (exclusive scan over digits), the
        // per-wave starts inside it, and the shift to its global position
        const int t = threadIdx.x;
        unsigned cnt = 0;
#pragma unroll
        for (int ww = 0; ww < WG / 64; ++ww) cnt += run[ww][t];
        unsigned tot;
        const unsigned start = wg_excl_scan(cnt, lds_scan, &tot);
        delta[t] = (int)(hist[(size_t)t * n_tiles + blockIdx.x] - start);
        unsigned o = start;
#pragma unroll
        for (int ww = 0; ww < WG / 64; ++ww) {
            const unsigned c = run[ww][t];
            run[ww][t] = o;
            o += c;
        }
    }
    __syncthreads();
    // stable placement inside the tile, ordered by digit
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int pos = base + r * 64 + lane;
        if (pos < n) {
            const unsigned dg = (k[r] >> shift) & 255u;
            const unsigned lp = run[w][dg] + rk[r];
            sk[lp] = k[r];
            sv[lp] = v[r];
        }
    }
    __syncthreads();
    // each digit's keys are contiguous in the tile and in the output: the
    // stores of consecutive threads land on consecutive addresses
    const int tile_n = min(SORT_TILE, n - tile0);
    for (int j = threadIdx.x; j < tile_n; j += WG) {
        const uint32_t kk = sk[j];
        const unsigned dst = (unsigned)((int)j + delta[(kk >> shift) & 255u]);
        if (dst < (unsigned)n) {
            kout[dst] = kk;
            vout[dst] = sv[j];
        }
    }
}

int radix_hist_size(int n) { return 256 * ((n + SORT_TILE - 1) / SORT_TILE); }

// Sorts n keys read from keys_in (which must be neither k0 nor ... k0 is the
// first destination).  Values start as the identity 0..n-1.  Pass p writes
// (k0, v0) when p is even and (k1, v1) when odd; *keys_out / *vals_out point
// at the final pair.
hipError_t radix_sort(const uint32_t* keys_in, uint32_t* k0, uint32_t* k1, uint32_t* v0, uint32_t* v1, int n,
                      int key_bits, unsigned* hist, unsigned* partials, uint32_t** keys_out, uint32_t** vals_out,
                      hipStream_t s) {
    const int n_tiles = (n + SORT_TILE - 1) / SORT_TILE;
    const int passes = key_bits <= 8 ? 1 : (key_bits + 7) / 8;
    const uint32_t* kin = keys_in;
    const uint32_t* vin = nullptr;
    for (int p = 0; p < passes; ++p) {
        uint32_t* ko = (p & 1) ? k1 : k0;
        uint32_t* vo = (p & 1) ? v1 : v0;
        k_radix_hist<<<n_tiles, WG, 0, s>>>(kin, n, 8 * p, hist, n_tiles);
        hipError_t e = scan_exclusive(hist, hist, 256 * n_tiles, nullptr, partials, nullptr, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<n_tiles, WG, 0, s>>>(kin, vin, ko, vo, n, 8 * p, hist, n_tiles);
        kin = ko;
        vin = vo;
    }
    *keys_out = const_cast<uint32_t*>(kin);
    *vals_out = const_cast<uint32_t*>(vin);
    return hipGetLastError();
}

}  // namespace mpmx
