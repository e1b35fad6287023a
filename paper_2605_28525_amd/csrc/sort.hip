// Stable LSD radix sort of (u32 key, u32 value) pairs, 8-bit digits, one
// scatter kernel per digit ("onesweep": decoupled look-back instead of a
// per-pass histogram and device-wide scan).
//
//   k_radix_counts   one read of the keys: every tile's digit counts of every
//                    pass, written digit-major (pass, digit, tile);
//   k_radix_totals   per (pass, digit) the sum over tiles; then k_radix_bases
//                    turns the totals into each digit's first output slot;
//   k_onesweep       per pass: a workgroup takes the next tile number from a
//                    counter (so every smaller tile is already running), ranks
//                    its keys (each wave64 owns a quarter of the tile and matches
//                    digits with 8 ballots), publishes its digit counts, walks
//                    back over earlier tiles' published counts until it meets an
//                    inclusive prefix, publishes its own inclusive prefix, and
//                    scatters stably.
//
// The look-back wait is bounded: a tile that sees no status from a predecessor
// after LB_SPIN_LIMIT polls raises MPM_FLAG_WAIT and stops waiting (its
// destinations are then wrong but stay inside [0, n), and the kernels that
// dereference the permutation skip the step when the flag is set).  With
// tiles numbered in start order every predecessor is resident or done, so the
// bound is never reached by a correct run.
#include "internal.h"

namespace mpmx {

constexpr unsigned LB_AGG = 1u << 30;        // status holds the tile's own count
constexpr unsigned LB_PRE = 2u << 30;        // status holds the inclusive prefix
constexpr unsigned LB_VAL = (1u << 30) - 1u;
constexpr int LB_SPIN_LIMIT = 1 << 22;
constexpr int MAX_PASSES = 4;

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

__global__ __launch_bounds__(WG) void k_radix_counts(const uint32_t* __restrict__ keys, int n, int passes,
                                                     unsigned* __restrict__ tilecnt, int n_tiles) {
    __shared__ unsigned cnt[WG / 64][MAX_PASSES][256];
    for (int t = threadIdx.x; t < (WG / 64) * MAX_PASSES * 256; t += WG) (&cnt[0][0][0])[t] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const int base = blockIdx.x * SORT_TILE + w * (SORT_TILE / (WG / 64));
    uint32_t k[SORT_ITEMS];
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int pos = base + r * 64 + lane;
        k[r] = pos < n ? keys[pos] : 0u;
    }
    for (int p = 0; p < passes; ++p) {
#pragma unroll
        for (int r = 0; r < SORT_ITEMS; ++r) {
            const bool valid = base + r * 64 + lane < n;
            const unsigned dg = (k[r] >> (8 * p)) & 255u;
            const unsigned long long m = digit_match(dg, valid);
            if (valid && (__ffsll((long long)m) - 1) == lane) cnt[w][p][dg] += (unsigned)__popcll(m);
        }
    }
    __syncthreads();
    const int t = threadIdx.x;  // one digit per thread (WG == 256)
    for (int p = 0; p < passes; ++p)
        tilecnt[((size_t)p * 256 + t) * n_tiles + blockIdx.x] = cnt[0][p][t] + cnt[1][p][t] + cnt[2][p][t] + cnt[3][p][t];
}

// One workgroup per (pass, digit): the digit's total over all tiles.
__global__ __launch_bounds__(WG) void k_radix_totals(const unsigned* __restrict__ tilecnt, int n_tiles,
                                                     unsigned* __restrict__ totals) {
    __shared__ unsigned lds[WG / 64];
    const unsigned* row = tilecnt + (size_t)blockIdx.x * n_tiles;
    unsigned s = 0;
    for (int i = threadIdx.x; i < n_tiles; i += WG) s += row[i];
    unsigned tot;
    wg_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// Exclusive scan over the 256 digits of each pass: first output slot per digit.
__global__ __launch_bounds__(WG) void k_radix_bases(const unsigned* __restrict__ totals, int passes,
                                                    unsigned* __restrict__ bases) {
    __shared__ unsigned lds[WG / 64];
    for (int p = 0; p < passes; ++p) {
        unsigned tot;
        const unsigned ex = wg_excl_scan(totals[p * 256 + threadIdx.x], lds, &tot);
        bases[p * 256 + threadIdx.x] = ex;
    }
}

__global__ __launch_bounds__(WG) void k_radix_clear(unsigned* __restrict__ a, size_t count) {
    for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < count; i += (size_t)gridDim.x * WG) a[i] = 0u;
}

__global__ __launch_bounds__(WG) void k_onesweep(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                 uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int n,
                                                 int shift, const unsigned* __restrict__ bases,
                                                 unsigned* __restrict__ stat, unsigned* __restrict__ tile_ctr,
                                                 DevCounters* ctr) {
    __shared__ unsigned run[WG / 64][256];
    __shared__ unsigned off[WG / 64][256];
    __shared__ int tile_sh;
    for (int t = threadIdx.x; t < (WG / 64) * 256; t += WG) (&run[0][0])[t] = 0;
    if (threadIdx.x == 0) tile_sh = (int)atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const int tile = tile_sh;
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int base = tile * SORT_TILE + w * (SORT_TILE / (WG / 64));
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
        const bool valid = base + r * 64 + lane < n;
        const unsigned dg = (k[r] >> shift) & 255u;
        const unsigned long long m = digit_match(dg, valid);
        const unsigned cur = run[w][dg];
        rk[r] = cur + (unsigned)__popcll(m & lt);
        if (valid && (__ffsll((long long)m) - 1) == lane) run[w][dg] = cur + (unsigned)__popcll(m);
    }
    __syncthreads();
    {
        const int t = threadIdx.x;  // one digit per thread
        unsigned local = 0;
#pragma unroll
        for (int ww = 0; ww < WG / 64; ++ww) {
            off[ww][t] = local;
            local += run[ww][t];
        }
        unsigned* my = stat + (size_t)tile * 256 + t;
        unsigned excl = 0;
        if (tile == 0) {
            __hip_atomic_store(my, LB_PRE | local, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(my, LB_AGG | local, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int j = tile - 1, spins = 0;
            while (j >= 0) {
                const unsigned sv =
                    __hip_atomic_load(stat + (size_t)j * 256 + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((sv & ~LB_VAL) == 0u) {
                    if (++spins > LB_SPIN_LIMIT) {
                        raise_flag(ctr, MPM_FLAG_WAIT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += sv & LB_VAL;
                if (sv & LB_PRE) break;
                --j;
            }
            __hip_atomic_store(my, LB_PRE | ((excl + local) & LB_VAL), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const unsigned b0 = bases[t] + excl;
#pragma unroll
        for (int ww = 0; ww < WG / 64; ++ww) off[ww][t] += b0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int pos = base + r * 64 + lane;
        if (pos < n) {
            const unsigned dg = (k[r] >> shift) & 255u;
            const unsigned dst = off[w][dg] + rk[r];
            if (dst < (unsigned)n) {
                kout[dst] = k[r];
                vout[dst] = v[r];
            }
        }
    }
}

static int passes_for(int key_bits) { return key_bits <= 8 ? 1 : (key_bits + 7) / 8; }

// tile counts (passes x 256 x tiles), look-back status (passes x tiles x 256),
// totals and bases (passes x 256 each), tile counters (passes)
int radix_hist_size(int n) {
    const int n_tiles = (n + SORT_TILE - 1) / SORT_TILE;
    return 2 * MAX_PASSES * 256 * n_tiles + 2 * MAX_PASSES * 256 + 64;
}

// Sorts n keys read from keys_in.  Values start as the identity 0..n-1.  Pass
// p writes (k0, v0) when p is even and (k1, v1) when odd; *keys_out /
// *vals_out point at the final pair.  keys_in may alias k1 (it is read by the
// first pass only, which writes k0).
hipError_t radix_sort(const uint32_t* keys_in, uint32_t* k0, uint32_t* k1, uint32_t* v0, uint32_t* v1, int n,
                      int key_bits, unsigned* hist, DevCounters* ctr, uint32_t** keys_out, uint32_t** vals_out,
                      hipStream_t s) {
    const int n_tiles = (n + SORT_TILE - 1) / SORT_TILE;
    const int passes = passes_for(key_bits);
    if (passes > MAX_PASSES) return hipErrorInvalidValue;
    unsigned* tilecnt = hist;
    unsigned* stat = tilecnt + (size_t)MAX_PASSES * 256 * n_tiles;
    unsigned* totals = stat + (size_t)MAX_PASSES * 256 * n_tiles;
    unsigned* bases = totals + MAX_PASSES * 256;
    unsigned* tile_ctr = bases + MAX_PASSES * 256;
    // zero the look-back status and the tile counters (a kernel, so the sort
    // can be captured in a graph)
    const size_t clear_n = (size_t)passes * 256 * n_tiles;
    k_radix_clear<<<(int)std::min<size_t>((clear_n + WG - 1) / WG, 4096), WG, 0, s>>>(stat, clear_n);
    k_radix_clear<<<1, WG, 0, s>>>(tile_ctr, MAX_PASSES);
    k_radix_counts<<<n_tiles, WG, 0, s>>>(keys_in, n, passes, tilecnt, n_tiles);
    k_radix_totals<<<passes * 256, WG, 0, s>>>(tilecnt, n_tiles, totals);
    k_radix_bases<<<1, WG, 0, s>>>(totals, passes, bases);
    const uint32_t* kin = keys_in;
    const uint32_t* vin = nullptr;
    for (int p = 0; p < passes; ++p) {
        uint32_t* ko = (p & 1) ? k1 : k0;
        uint32_t* vo = (p & 1) ? v1 : v0;
        k_onesweep<<<n_tiles, WG, 0, s>>>(kin, vin, ko, vo, n, 8 * p, bases + p * 256,
                                          stat + (size_t)p * 256 * n_tiles, tile_ctr + p, ctr);
        kin = ko;
        vin = vo;
    }
    *keys_out = const_cast<uint32_t*>(kin);
    *vals_out = const_cast<uint32_t*>(vin);
    return hipGetLastError();
}

}  // namespace mpmx
