// Internal declarations of the sparse-grid MPM library (gfx950, wave64).
//
// Device data layout (all in HBM, owned by the context):
//   sort      key/value ping-pong buffers, u32 x max_particles each; per-tile
//             digit histograms;
//   hash      H slots: packed block key (u64, EMPTY = ~0), node mask (u64),
//             compact index (i32), first/one-past-last sorted particle of the
//             block's owner segment (i32);
//   blocks    block_capacity entries in compact order Phi: key, node mask,
//             2^d neighbour compact indices (upper neighbours), owner segment
//             start and length, P2G/G2P chunk count and offset;
//   work      (block, first, last) particle ranges of at most CHUNK particles;
//   grid      block_capacity * 4^d nodes, one float4 per node (p_x, p_y, p_z, m),
//             then (v_x, v_y, v_z, m) after the grid update.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpm.h"

namespace mpmx {

constexpr int WG = 256;            // workgroup size of every kernel (4 wave64s)
constexpr int BLK = 4;             // block edge B (Methods 3.2)
constexpr int KEY_M = 21;          // bits per packed coordinate (Eq. 22)
constexpr int64_t KEY_BIAS = 1 << 20;
constexpr uint64_t EMPTY_KEY = ~0ull;

constexpr int SORT_ITEMS = 16;                 // keys per thread per radix tile
constexpr int SORT_TILE = WG * SORT_ITEMS;     // 4096 keys per tile
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = WG * SCAN_ITEMS;     // 2048 values per scan tile
constexpr int MIN_CHUNK = 64;                  // smallest particles-per-work-item setting
constexpr int MAX_CHUNK = 768;                 // largest (G2P stages a work item in LDS)
// Particles a G2P workgroup of gs threads stages per work item: three per
// thread at 256 threads (a full 4^3 block of 8-per-cell material, slightly
// compressed, stays one item), two per thread below.
constexpr int g2p_max_items(int gs) { return (gs == 256 ? 3 : 2) * gs; }

struct DevCounters {
    int nb;          // active blocks (compact count, <= capacity)
    int n_touched;   // occupied hash slots (may exceed capacity on overflow)
    int n_work;      // P2G/G2P work items
    unsigned flags;  // sticky MPM_FLAG_* bits
    int rs_n_new;    // incremental re-sort: blocks without a previous slot
    int rs_n_ent;    //   entries (previous blocks, then new blocks)
    int rs_n_mov;    //   particles that changed owner block (0 between builds)
    int pad;
};

// Per-instance material and step constants (one entry for a single simulation).
struct InstMat {
    float mu, lam, alpha, dp_coef;
    float dt, p_mass, p_vol0, E;
    float dalpha_dphi, pad[3];
};

constexpr int MAX_INSTANCES = 64;
constexpr int ENS_KEY_M = 19;                 // ensemble block keys: bits per coordinate
constexpr int64_t ENS_KEY_BIAS = 1 << 18;
constexpr int ENS_INST_SHIFT = 57;            // instance id in bits 57..62

struct DevParams {
    int dim;
    int cells[3];
    int nblk[3];          // blocks per axis over the node range [0, cells]
    int dense;
    double dx, inv_dx;
    float dxf, inv_dxf, dt;
    float g[3];
    float mu, lam, alpha, dp_coef;   // Lame, DP cone alpha, (d lambda + 2 mu)/(2 mu)
    int model;
    float p_mass, p_vol0;
    int bound;
    int bc[3][2];
    const float* heightmap;
    float mu_terrain;
    int has_terrain;
    // hash table
    uint64_t* h_keys;
    uint64_t* h_mask;
    int* h_vals;
    int* h_start;
    int* h_end;
    unsigned h_mask_bits;   // H - 1
    int n_probe;
    // compact blocks
    uint64_t* b_keys;
    uint64_t* b_mask;
    int* b_nbr;
    int* b_start;
    int* b_count;
    unsigned* b_chunks;
    unsigned* b_chunk_off;
    int block_cap;
    // work items
    int* w_block;
    int* w_start;
    int* w_end;
    int work_cap;
    int chunk;
    // grid
    float4* grid;
    float4* tiles;        // sparse P2G: each block's (4+2)^d node tile, block-major
    int* b_lo;            // sparse P2G: 2^d lower neighbours (d = 0: the block) owning particles, else -1
    DevCounters* ctr;
    // reverse mode (allocated with MPM_FLAG_ADJOINT)
    float4* grid_u;      // pre-boundary nodal velocity u = p/m + dt g, and m
    float4* grid_bar;    // adjoint of the nodal velocity, then (p_bar, m_bar)
    float* adj_scratch;  // per sorted particle: v'_bar (d), B_bar (d*d), W_bar (d*d); plane stride n
    float* param_bar;    // accumulated dL/dE, dL/dphi (per degree)
    float E;
    float dalpha_dphi;   // d alpha / d phi, per degree
    // incremental re-sort (resort.hip): per entry (previous block, then new
    // block) and base cell, NC = 4^d columns
    uint32_t* rs_stay;    // stayers per previous block and cell
    uint32_t* rs_in;      // movers per entry and cell (counted down to zero as they are placed)
    uint32_t* rs_off;     // first sorted position per entry and cell
    unsigned* rs_cnt;     // particles per entry (stayers from G2P or the count pass, plus movers)
    unsigned* rs_start;   // first sorted position per entry
    uint32_t* rs_oldblk;  // owner-block part of the sort key of each entry (~0: empty previous block)
    uint64_t* nh_keys;    // second hash table (same size as the block table): blocks
    uint32_t* nh_cnt;     //   with no previous slot, their movers per cell,
    int* nh_idx;          //   their entry index
    uint32_t* nh_owner;   //   and the owner-block part of their sort key
    uint32_t* rs_new;     // second-table slots in the order of their claims (block_cap entries)
    int* h_entry;         // re-sort entry of each hash slot's owner block (-1: none)
    int* b_entry;         // re-sort entry of each compact block (-1: none): its cell
                          // ranges are the entry's row of rs_off
    // ensembles
    int n_inst;          // 1 = single simulation
    int blk_bits;        // bits of the linear block id inside the sort key
    const InstMat* inst; // device table, n_inst entries
};

// ---------------------------------------------------------------------------
// device helpers
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 output function (Steele, Lea, Flood 2014), a 64-bit mixer of
    // the kind cited for Eq. 23.
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int DIM>
__device__ __forceinline__ uint64_t pack_key(int bx, int by, int bz) {
    // Eq. 22: ((i + b) << 2m) | ((j + b) << m) | (k + b); 2D packs (i, j) low.
    if (DIM == 3)
        return ((uint64_t)(bx + KEY_BIAS) << (2 * KEY_M)) | ((uint64_t)(by + KEY_BIAS) << KEY_M) |
               (uint64_t)(bz + KEY_BIAS);
    return ((uint64_t)(bx + KEY_BIAS) << KEY_M) | (uint64_t)(by + KEY_BIAS);
}

template <int DIM>
__device__ __forceinline__ void unpack_key(uint64_t k, int* b) {
    const uint64_t m = (1ull << KEY_M) - 1;
    if (DIM == 3) {
        b[0] = (int)((k >> (2 * KEY_M)) & m) - (int)KEY_BIAS;
        b[1] = (int)((k >> KEY_M) & m) - (int)KEY_BIAS;
        b[2] = (int)(k & m) - (int)KEY_BIAS;
    } else {
        b[0] = (int)((k >> KEY_M) & m) - (int)KEY_BIAS;
        b[1] = (int)(k & m) - (int)KEY_BIAS;
        b[2] = 0;
    }
}

// Block key with the instance folded in.  A single simulation uses Eq. 22
// as printed (m = 21, bias 2^20); an ensemble uses m = 19 (bias 2^18) and puts
// the instance id in bits 57-62, which keeps 3m + 6 <= 63.
template <int DIM>
__device__ __forceinline__ uint64_t block_key(const DevParams& P, int bx, int by, int bz, int inst) {
    if (P.n_inst <= 1) return pack_key<DIM>(bx, by, bz);
    const uint64_t ib = (uint64_t)inst << ENS_INST_SHIFT;
    if (DIM == 3)
        return ib | ((uint64_t)(bx + ENS_KEY_BIAS) << (2 * ENS_KEY_M)) | ((uint64_t)(by + ENS_KEY_BIAS) << ENS_KEY_M) |
               (uint64_t)(bz + ENS_KEY_BIAS);
    return ib | ((uint64_t)(bx + ENS_KEY_BIAS) << ENS_KEY_M) | (uint64_t)(by + ENS_KEY_BIAS);
}

template <int DIM>
__device__ __forceinline__ void unblock_key(const DevParams& P, uint64_t k, int* b, int* inst) {
    if (P.n_inst <= 1) {
        unpack_key<DIM>(k, b);
        *inst = 0;
        return;
    }
    const uint64_t m = (1ull << ENS_KEY_M) - 1;
    *inst = (int)((k >> ENS_INST_SHIFT) & 63u);
    if (DIM == 3) {
        b[0] = (int)((k >> (2 * ENS_KEY_M)) & m) - (int)ENS_KEY_BIAS;
        b[1] = (int)((k >> ENS_KEY_M) & m) - (int)ENS_KEY_BIAS;
        b[2] = (int)(k & m) - (int)ENS_KEY_BIAS;
    } else {
        b[0] = (int)((k >> ENS_KEY_M) & m) - (int)ENS_KEY_BIAS;
        b[1] = (int)(k & m) - (int)ENS_KEY_BIAS;
        b[2] = 0;
    }
}

// Base node floor(x * (1/dx) - 1/2) in float64, multiply and subtract rounded
// separately (no contraction), and the fractional offset s - floor(s).
__device__ __forceinline__ double index_arg(float x, double inv_dx) {
#pragma clang fp contract(off)
    double s = (double)x * inv_dx;
    return s - 0.5;
}

// Sort key of one particle (binning, a1): base node floor(x/dx - 1/2) per axis
// in float64, clamped into the grid with MPM_FLAG_DOMAIN (MPM_FLAG_NAN for a
// non-finite coordinate) ORed into *bad; key = instance << (block bits + 2d)
// | linear owner block << 2d | local cell of the base node.
template <int DIM>
__device__ __forceinline__ uint32_t bin_key(const DevParams& P, const float* xv, uint32_t inst, unsigned* bad) {
    int b[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double f = floor(index_arg(xv[a], P.inv_dx));
        if (!(f == f)) {
            *bad |= MPM_FLAG_NAN;
            f = 0.0;
        } else if (f < 0.0 || f + 2.0 > (double)P.cells[a]) {
            *bad |= MPM_FLAG_DOMAIN;
            f = fmin(fmax(f, 0.0), (double)(P.cells[a] - 2));
        }
        b[a] = (int)f;
    }
    uint32_t bl, cell;
    if (DIM == 3) {
        bl = ((uint32_t)(b[2] >> 2) * (uint32_t)P.nblk[1] + (uint32_t)(b[1] >> 2)) * (uint32_t)P.nblk[0] +
             (uint32_t)(b[0] >> 2);
        cell = (b[0] & 3) | ((b[1] & 3) << 2) | ((b[2] & 3) << 4);
    } else {
        bl = (uint32_t)(b[1] >> 2) * (uint32_t)P.nblk[0] + (uint32_t)(b[0] >> 2);
        cell = (b[0] & 3) | ((b[1] & 3) << 2);
    }
    return (inst << (P.blk_bits + 2 * DIM)) | (bl << (2 * DIM)) | cell;
}

template <int DIM>
__device__ __forceinline__ void linear_to_block(const DevParams& P, uint32_t bl, int* bc) {
    bc[0] = (int)(bl % (uint32_t)P.nblk[0]);
    uint32_t r = bl / (uint32_t)P.nblk[0];
    if (DIM == 3) {
        bc[1] = (int)(r % (uint32_t)P.nblk[1]);
        bc[2] = (int)(r / (uint32_t)P.nblk[1]);
    } else {
        bc[1] = (int)r;
        bc[2] = 0;
    }
}

// Block coordinates (and instance) of compact block b (sparse: from its packed
// key; dense: b is the linear block index).
template <int DIM>
__device__ __forceinline__ void block_coords(const DevParams& P, int b, int* bc, int* inst = nullptr) {
    int i = 0;
    if (P.dense)
        linear_to_block<DIM>(P, (uint32_t)b, bc);
    else
        unblock_key<DIM>(P, P.b_keys[b], bc, &i);
    if (inst) *inst = i;
}

// Material of an instance (a single simulation reads the scalar fields).
__device__ __forceinline__ InstMat material(const DevParams& P, int inst) {
    if (P.n_inst > 1) return P.inst[inst];
    InstMat m;
    m.mu = P.mu;
    m.lam = P.lam;
    m.alpha = P.alpha;
    m.dp_coef = P.dp_coef;
    m.dt = P.dt;
    m.p_mass = P.p_mass;
    m.p_vol0 = P.p_vol0;
    m.E = P.E;
    m.dalpha_dphi = P.dalpha_dphi;
    return m;
}

// Compact index of block key K in the block hash table (Eqs. 23-25), -1 if
// the key has no slot or its block did not fit the capacity.
// The slot's value is loaded beside its key, so a hit costs one round trip.
__device__ __forceinline__ int hash_lookup(const DevParams& P, uint64_t K) {
    unsigned s = (unsigned)mix64(K) & P.h_mask_bits;
    for (int r = 0; r < P.n_probe; ++r) {
        const uint64_t cur = P.h_keys[s];
        int val = P.h_vals[s];
        asm volatile("" : "+v"(val));  // keeps the load beside the key's, not behind the compare
        if (cur == K) return val;
        if (cur == EMPTY_KEY) return -1;
        s = (s + 1) & P.h_mask_bits;
    }
    return -1;
}

__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
    unsigned lo = __builtin_amdgcn_readlane((unsigned)v, lane);
    unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int readlane32(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

__device__ __forceinline__ void raise_flag(DevCounters* c, unsigned f) { atomicOr(&c->flags, f); }

// Inclusive scan across a wave64.
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan across a 256-thread workgroup; lds needs 4 entries.
__device__ __forceinline__ unsigned wg_excl_scan(unsigned v, unsigned* lds, unsigned* total) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    unsigned inc = wave_incl_scan(v);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    unsigned off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) {
        unsigned s = lds[i];
        off += (i < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// For a pass over tiles whose sums are partials[0 .. tiles): the sum of the
// tiles before `tile` (its exclusive offset) and the sum of all of them, both
// computed by the whole 256-thread workgroup (each workgroup reads the few
// tile sums itself instead of waiting for a separate scan of them).
__device__ __forceinline__ void tile_offset(const unsigned* __restrict__ partials, int tile, int tiles,
                                            unsigned* lds, unsigned* before, unsigned* total) {
    unsigned b = 0, t = 0;
    for (int i = threadIdx.x; i < tiles; i += WG) {
        const unsigned v = partials[i];
        t += v;
        b += i < tile ? v : 0u;
    }
    wg_excl_scan(b, lds, before);
    wg_excl_scan(t, lds, total);
}

// Scan-based construction (scanbuild.hip): the mask domain (bounding box of the
// owner blocks grown by one block on each upper side), written on the device.
struct SbBox {
    int lo[3], hi[3];  // owner-block bounds (lo = INT_MAX, hi = -1 while empty)
    int ext[3];        // extents of the mask domain
    int m;             // its volume in blocks (0: no particle, or above max_m)
    int too_big;       // the volume exceeded max_m
    unsigned total;    // active blocks (sum of the flags)
    int pad[2];
};

// Scratch of the scan-based construction, carved from one allocation: box
// header, the bounding-box partials of the SB_BBOX_WGS workgroups of its pass,
// occupancy (u64), flags and Phi (u32) for up to max_m blocks of the domain,
// scan partials; owner segment bounds (step build only, may be null).
constexpr int SB_BBOX_WGS = 1024;
constexpr size_t sb_scratch_size(long long max_m) {
    return 256 + (size_t)SB_BBOX_WGS * 8 * sizeof(int) + (size_t)max_m * (8 + 4 + 4) +
           (size_t)((max_m + SCAN_TILE - 1) / SCAN_TILE + 1) * sizeof(unsigned) + 256;
}
struct SbScratch {
    SbBox* box;
    int* bbp;  // per workgroup of the bounding-box pass: lo[3], hi[3]
    uint64_t* occ;
    unsigned* flag;
    unsigned* phi;
    unsigned* partials;
    int* seg_lo;
    int* seg_hi;
    long long max_m;
};

// ---------------------------------------------------------------------------
// host-side launchers (each returns hipError_t of the launch)
hipError_t scan_exclusive(const unsigned* in, unsigned* out, int n, const int* n_dev, unsigned* partials,
                          unsigned* total_out, hipStream_t s);
int scan_partials_size(int n);
size_t sb_scratch_bytes(long long max_m);
SbScratch sb_carve(void* base, long long max_m, int* seg_lo, int* seg_hi);
hipError_t launch_scan_active(const DevParams& P, const float* x, int n, const SbScratch& S, uint64_t* keys_out,
                              uint64_t* masks_out, int cap, hipStream_t s);
hipError_t launch_build_scan(const DevParams& P, const uint32_t* skeys, int n, const SbScratch& S,
                             unsigned* partials, hipStream_t s);
hipError_t launch_work_items(const DevParams& P, unsigned* partials, hipStream_t s);
long long scan_active_static_max_blocks();
hipError_t launch_scan_active_static(const DevParams& P, const float* x, int n, uint64_t* keys_out,
                                     uint64_t* masks_out, int cap, SbBox* box_host, hipStream_t s);

hipError_t radix_sort(const uint32_t* keys_in, uint32_t* k0, uint32_t* k1, uint32_t* v0, uint32_t* v1, int n,
                      int key_bits, unsigned* hist, unsigned* partials, uint32_t** keys_out, uint32_t** vals_out,
                      hipStream_t s);
int radix_hist_size(int n);

hipError_t launch_bin(const DevParams& P, const float* x, const uint32_t* inst, int n, uint32_t* keys, hipStream_t s);
// keys_out may be null: the sorted keys are then not written (after an
// incremental re-sort nothing reads them; P2G takes the cell ranges from the
// re-sort's per-entry table).  movers and tgt: n entries each (the mover list
// and each mover's target, which the route records for the placement).
hipError_t launch_resort(const DevParams& P, const uint32_t* keys_new, uint32_t* keys_out, uint32_t* vals_out,
                         uint32_t* movers, uint32_t* tgt, int n, unsigned H, unsigned* partials, hipStream_t s,
                         bool counted = false);
hipError_t launch_resort_init(const DevParams& P, unsigned H, hipStream_t s);
// Buffers of the ascending-key Phi order (MPM_FLAG_DETERMINISTIC_ORDER): block
// tables in slot order, the slot of each, and a radix sort of block_cap
// entries (keys, values, histograms).
struct DetTables {
    uint64_t* keys;
    uint64_t* mask;
    int* start;
    int* count;
    int* slot;
    uint32_t* k[2];
    uint32_t* v[2];
    unsigned* hist;
};
hipError_t launch_build_sparse(const DevParams& P, const uint32_t* skeys, int n, unsigned H, unsigned* partials,
                               hipStream_t s, bool from_resort = false, const DetTables* det = nullptr);
hipError_t launch_build_dense(const DevParams& P, const uint32_t* skeys, int n, int n_blocks, unsigned* partials,
                              hipStream_t s);
// update: the grid update (Eqs. 8-12) is applied in P2G's second pass (sparse
// grids), which then leaves velocities instead of momenta in the grid.
hipError_t launch_p2g(const DevParams& P, const float* x, const float* v, const float* C, const float* tau, int n,
                      const uint32_t* order, const uint32_t* skeys, uint32_t* osrc, int grid_blocks, hipStream_t s,
                      bool update = false);
hipError_t launch_grid_update(const DevParams& P, long long n_nodes_host, int grid_blocks, hipStream_t s);
hipError_t launch_g2p(const DevParams& P, const float* x_in, const float* F_in, const uint32_t* id_in,
                      const uint32_t* inst_in, float* x_out, float* v_out, float* C_out, float* F_out, float* tau_out,
                      uint32_t* id_out, uint32_t* inst_out, int n, const uint32_t* osrc, int block_size,
                      int grid_blocks, hipStream_t s, uint32_t* keys_out = nullptr,
                      uint32_t* movers_out = nullptr);
hipError_t launch_clear_flags(DevCounters* c, hipStream_t s);
hipError_t launch_g2p_adj(const DevParams& P, const float* x, const float* F, const float* const* out_bar, float* x_bar,
                          float* F_bar, int n, const uint32_t* order, const uint32_t* skeys, int grid_blocks,
                          hipStream_t s);
hipError_t launch_scatter_adj(const DevParams& P, const float* x, int n, const uint32_t* order, const uint32_t* skeys,
                              int grid_blocks, hipStream_t s);
hipError_t launch_grid_adj(const DevParams& P, long long n_nodes_host, int grid_blocks, hipStream_t s);
hipError_t launch_p2g_adj(const DevParams& P, const float* const* in, float* const* in_bar, int n,
                          const uint32_t* order, int grid_blocks, hipStream_t s);
hipError_t launch_copy_active(const DevParams& P, uint64_t* keys, uint64_t* masks, int cap, hipStream_t s);

}  // namespace mpmx
