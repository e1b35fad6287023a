// Active-node indexing on the GPU (Methods 3.3, Algorithms 5-6; Eqs. 22-25).
//
//   k_bin           base node per particle (float64 index arithmetic), owner
//                   block and a u32 sort key = linear block id << 2d | local
//                   cell of the base node;
//   sort            groups particles by owner block: the radix sort of
//                   sort.hip, or after a build of as many particles the
//                   incremental re-sort of resort.hip;
//   k_hash_clear    keys <- EMPTY, masks <- 0 (Algorithm 5, initialisation);
//   k_hash_insert   per sorted particle: the stencil touches its owner block and
//                   only the upper neighbours it spills into (base local index
//                   >= 2 on an axis), so at most 2^d blocks.  Lanes of a wave64
//                   that share an owner block are merged (ballot/readlane loop)
//                   and their node masks OR-reduced, then one lane per touched
//                   block claims or finds the slot: packed key (Eq. 22), mixer
//                   (Eq. 23), slot h & (H - 1) (Eq. 24), linear probing (Eq. 25)
//                   with a compare-and-swap on EMPTY (Algorithm 6), and ORs the
//                   node mask into the slot.  The owner run boundaries of the
//                   sorted order are recorded per slot.
//   (after an incremental re-sort the insertion runs per re-sort entry
//   instead, k_hash_insert_entries, from the entry's per-cell table)
//   compaction      prefix scan over occupied slots -> Phi in slot order; block
//                   keys, masks and owner segments in Phi order; overflow when
//                   more than block_capacity slots are occupied (the counter
//                   check of Algorithm 6); the same scan numbers the work
//                   items (owner segments in chunks) in Phi order and writes
//                   them, except for the key-ordered Phi, whose items follow
//                   from a scan of per-block counts after the reordering.
//   block setup     upper- and lower-neighbour compact indices (so P2G/G2P
//                   never probe) and the per-block state the next incremental
//                   re-sort's counting in G2P needs (the dense baseline also
//                   clears its grid; the sparse P2G writes every node of every
//                   active block).
#include "internal.h"
#include "../../include/mpm.h"

namespace mpmx {

constexpr int BIN_PER_THREAD = 2;  // particles per thread of k_bin (loads issued together)

template <int DIM>
__global__ __launch_bounds__(WG) void k_bin(DevParams P, const float* __restrict__ x,
                                            const uint32_t* __restrict__ inst, int n, uint32_t* __restrict__ keys) {
    const int i0 = blockIdx.x * WG * BIN_PER_THREAD + threadIdx.x;
    float xv[BIN_PER_THREAD][3];
    uint32_t iv[BIN_PER_THREAD];
#pragma unroll
    for (int k = 0; k < BIN_PER_THREAD; ++k) {
        const int i = i0 + k * WG;
        iv[k] = 0u;
#pragma unroll
        for (int a = 0; a < 3; ++a) xv[k][a] = 0.f;
        if (i < n) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) xv[k][a] = x[(size_t)a * n + i];
            if (P.n_inst > 1 && inst) iv[k] = inst[i];
        }
    }
    unsigned bad = 0;
#pragma unroll
    for (int k = 0; k < BIN_PER_THREAD; ++k) {
        const int i = i0 + k * WG;
        if (i >= n) break;
        uint32_t in = iv[k];
        if (in >= (uint32_t)max(P.n_inst, 1)) {
            bad |= MPM_FLAG_DOMAIN;
            in = (uint32_t)max(P.n_inst, 1) - 1;
        }
        keys[i] = bin_key<DIM>(P, xv[k], in, &bad);
    }
    if (bad) raise_flag(P.ctr, bad);
}

// Claims or finds the slot of key K (Eqs. 23-25): a probed slot is read
// first and compare-and-swapped from EMPTY only when it is empty (most inserts
// find their block already claimed by another wave: each block is the owner
// or an upper neighbour of up to 2^d inserting waves).
__device__ int hash_insert(const DevParams& P, uint64_t K) {
    unsigned s = (unsigned)mix64(K) & P.h_mask_bits;
    for (int r = 0; r < P.n_probe; ++r) {
        const uint64_t cur = __hip_atomic_load(&P.h_keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == K) return (int)s;
        if (cur == EMPTY_KEY) {
            const uint64_t old = atomicCAS((unsigned long long*)&P.h_keys[s], (unsigned long long)EMPTY_KEY,
                                           (unsigned long long)K);
            if (old == EMPTY_KEY || old == K) return (int)s;
        }
        s = (s + 1) & P.h_mask_bits;
    }
    raise_flag(P.ctr, MPM_FLAG_OVERFLOW);
    return -1;
}

__global__ __launch_bounds__(WG) void k_hash_clear(DevParams P, unsigned H) {
    for (unsigned s = blockIdx.x * WG + threadIdx.x; s < H; s += gridDim.x * WG) {
        P.h_keys[s] = EMPTY_KEY;
        P.h_mask[s] = 0ull;
        P.h_start[s] = -1;
        P.h_end[s] = -1;
        if (P.h_entry) P.h_entry[s] = -1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.ctr->nb = 0;
        P.ctr->n_touched = 0;
        P.ctr->n_work = 0;
    }
}

// Node masks from the occupied base cells of a block.  With bit i + 4 j + 16 k
// for cell / node (i, j, k), the stencil of a base cell covers nodes +0..+2 on
// each axis; along one axis that is a dilation inside the block ("own") and a
// spill of cells 2 and 3 into nodes 0 and 1 of the upper neighbour ("spill").
// The node mask of neighbour d = (dx, dy, dz) is the composition of the per-axis
// own/spill maps selected by the bits of d.
__device__ __forceinline__ uint64_t own_x(uint64_t o) {
    return o | ((o << 1) & 0xEEEEEEEEEEEEEEEEull) | ((o << 2) & 0xCCCCCCCCCCCCCCCCull);
}
__device__ __forceinline__ uint64_t spill_x(uint64_t o) {
    return ((o >> 2) & 0x1111111111111111ull) | ((o >> 3) & 0x1111111111111111ull) |
           ((o >> 2) & 0x2222222222222222ull);
}
template <int DIM>
__device__ __forceinline__ uint64_t own_y(uint64_t o) {
    if (DIM == 2) return (o | (o << 4) | (o << 8)) & 0xFFFFull;
    return o | ((o << 4) & ~0x000F000F000F000Full) | ((o << 8) & ~0x00FF00FF00FF00FFull);
}
template <int DIM>
__device__ __forceinline__ uint64_t spill_y(uint64_t o) {
    if (DIM == 2) return ((o >> 8) & 0xFull) | ((o >> 12) & 0xFull) | ((o >> 8) & 0xF0ull);
    return ((o >> 8) & 0x000F000F000F000Full) | ((o >> 12) & 0x000F000F000F000Full) |
           ((o >> 8) & 0x00F000F000F000F0ull);
}
__device__ __forceinline__ uint64_t own_z(uint64_t o) { return o | (o << 16) | (o << 32); }
__device__ __forceinline__ uint64_t spill_z(uint64_t o) {
    return ((o >> 32) & 0xFFFFull) | ((o >> 48) & 0xFFFFull) | ((o >> 32) & 0xFFFF0000ull);
}

template <int DIM>
__device__ __forceinline__ uint64_t neighbour_mask(uint64_t occ, int d) {
    uint64_t o = (d & 1) ? spill_x(occ) : own_x(occ);
    if (DIM == 2) o &= 0xFFFFull;
    o = (d & 2) ? spill_y<DIM>(o) : own_y<DIM>(o);
    if (DIM == 3) o = (d & 4) ? spill_z(o) : own_z(o);
    return o;
}

constexpr int HI_ROUNDS = 4;  // sorted particles per lane of k_hash_insert (a wave covers 256)

// Sorted particles in runs of 256 per wave.  A run of equal owner blocks is one
// group; a group that continues from the previous round of the same wave is
// merged, so each wave inserts each of its owner blocks once.  Per group: the
// OR of its base-cell bits, the node masks of the owner and its 2^d - 1 upper
// neighbours by bit dilation, one insert per touched block (lane d takes
// neighbour d), and the owner segment's first / one-past-last sorted position
// where the segment starts / ends inside this wave.
template <int DIM>
__global__ __launch_bounds__(WG) void k_hash_insert(DevParams P, const uint32_t* __restrict__ skeys, int n) {
    constexpr int NB = 1 << DIM;
    constexpr int CB = 2 * DIM;
    const int lane = __lane_id();
    const int base = ((blockIdx.x * WG + (int)threadIdx.x) >> 6) * 64 * HI_ROUNDS;
    if (base >= n) return;  // whole wave
    const int stop = min(base + 64 * HI_ROUNDS, n);
    // owner segments (instance and block) just before and after this wave's range
    const uint32_t seg_before = base > 0 ? (skeys[base - 1] >> CB) : ~0u;
    const uint32_t seg_after = stop < n ? (skeys[stop] >> CB) : ~0u;
    uint32_t key[HI_ROUNDS];
#pragma unroll
    for (int r = 0; r < HI_ROUNDS; ++r) {
        const int i = base + r * 64 + lane;
        key[r] = i < n ? skeys[i] : 0u;
    }
    bool have = false;
    uint32_t p_seg = 0;
    uint64_t p_occ = 0;
    int p_first = 0, p_end = 0;
    auto flush = [&]() {
        const uint32_t bl = p_seg & ((1u << P.blk_bits) - 1u);
        const int inst = (int)(p_seg >> P.blk_bits);
        int bc[3];
        linear_to_block<DIM>(P, bl, bc);
        int slot = -1;
        if (lane < NB) {
            const uint64_t mymask = neighbour_mask<DIM>(p_occ, lane);
            if (mymask != 0ull) {
                const uint64_t Kd =
                    block_key<DIM>(P, bc[0] + (lane & 1), bc[1] + ((lane >> 1) & 1), bc[2] + ((lane >> 2) & 1), inst);
                slot = hash_insert(P, Kd);
                if (slot >= 0) atomicOr((unsigned long long*)&P.h_mask[slot], (unsigned long long)mymask);
            }
        }
        if (lane == 0 && slot >= 0) {  // lane 0 holds the owner block
            if (p_first > base || seg_before != p_seg) P.h_start[slot] = p_first;
            if (p_end < stop || seg_after != p_seg) P.h_end[slot] = p_end;
        }
    };
#pragma unroll
    for (int r = 0; r < HI_ROUNDS; ++r) {
        const int i = base + r * 64 + lane;
        const bool valid = i < n;
        const uint32_t seg = key[r] >> CB;
        const uint32_t cell = key[r] & ((1u << CB) - 1u);
        unsigned long long todo = __ballot(valid);
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const uint32_t g = (uint32_t)readlane32((int)seg, leader);
            const bool mine = valid && seg == g;
            const unsigned long long grp = __ballot(mine);
            const uint64_t occ = readlane64(wave_or64(mine ? (1ull << cell) : 0ull), leader);
            const int first = base + r * 64 + leader;
            const int last = base + r * 64 + (63 - __clzll((long long)grp));
            if (have && g == p_seg) {
                p_occ |= occ;
                p_end = last + 1;
            } else {
                if (have) flush();
                have = true;
                p_seg = g;
                p_occ = occ;
                p_first = first;
                p_end = last + 1;
            }
            todo &= ~grp;
        }
    }
    if (have) flush();
}

// Insertion after an incremental re-sort: one wave per entry (a previous block
// or a new one) of the re-sort, whose per-cell first positions and particle
// count are known, so the base-cell occupancy of the owner block is a ballot
// over its cells; node masks, inserts and owner segment as in k_hash_insert.
template <int DIM>
__global__ __launch_bounds__(WG) void k_hash_insert_entries(DevParams P) {
    constexpr int NB = 1 << DIM;
    constexpr int NC = 1 << (2 * DIM);
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int ne = P.ctr->rs_n_ent;
    for (int e = blockIdx.x * (WG / 64) + w; e < ne; e += gridDim.x * (WG / 64)) {
        // every load of the entry issued at once (none waits for the count)
        const unsigned tot = P.rs_cnt[e];
        const unsigned first = P.rs_start[e];
        const unsigned off_raw = lane < NC ? P.rs_off[(size_t)e * NC + lane] : 0u;
        const uint32_t owner = P.rs_oldblk[e];
        if (tot == 0u) continue;
        const unsigned end = first + tot;
        const unsigned off = lane < NC ? off_raw : end;
        const unsigned next = __shfl_down(off, 1);
        const bool occupied = lane < NC && (lane == NC - 1 ? end : next) > off;
        const uint64_t occ = (uint64_t)__ballot(occupied);
        const uint32_t bl = owner & ((1u << P.blk_bits) - 1u);
        const int inst = (int)(owner >> P.blk_bits);
        int bc[3];
        linear_to_block<DIM>(P, bl, bc);
        int slot = -1;
        if (lane < NB) {
            const uint64_t mymask = neighbour_mask<DIM>(occ, lane);
            if (mymask != 0ull) {
                const uint64_t Kd =
                    block_key<DIM>(P, bc[0] + (lane & 1), bc[1] + ((lane >> 1) & 1), bc[2] + ((lane >> 2) & 1), inst);
                slot = hash_insert(P, Kd);
                if (slot >= 0) atomicOr((unsigned long long*)&P.h_mask[slot], (unsigned long long)mymask);
            }
        }
        if (lane == 0 && slot >= 0) {  // lane 0 holds the owner block
            P.h_start[slot] = (int)first;
            P.h_end[slot] = (int)end;
            if (P.h_entry) P.h_entry[slot] = e;
        }
    }
}

// Work items of a block holding cnt particles (none for a block that only
// holds stencil nodes).
__device__ __forceinline__ unsigned block_chunks(const DevParams& P, int cnt) {
    return cnt > 0 ? (unsigned)((cnt + P.chunk - 1) / P.chunk) : 0u;
}

// Compaction, first pass: occupied slots per tile of the hash table
// (partials[tile]) and, with `items`, the work items of their blocks
// (partials[tiles + tile]).
__global__ __launch_bounds__(WG) void k_compact_count(DevParams P, int H, unsigned* __restrict__ partials, int tiles,
                                                      bool items) {
    __shared__ unsigned lds[WG / 64];
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    // all loads in flight at once: clamped index, masked result
    uint64_t key[SCAN_ITEMS];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) key[j] = P.h_keys[min(base + j, H - 1)];
    unsigned s = 0, w = 0;
    int st[SCAN_ITEMS], en[SCAN_ITEMS];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const bool occ = base + j < H && key[j] != EMPTY_KEY;
        s += occ ? 1u : 0u;
        st[j] = -1;
        en[j] = -1;
        if (items && occ) {
            st[j] = P.h_start[base + j];
            en[j] = P.h_end[base + j];
        }
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) w += st[j] >= 0 ? block_chunks(P, en[j] - st[j]) : 0u;
    unsigned tot;
    wg_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    if (items) {
        wg_excl_scan(w, lds, &tot);
        if (threadIdx.x == 0) partials[tiles + blockIdx.x] = tot;
    }
}

// Compaction, second pass: Phi in slot order and the block tables; with
// `items` also the work items of each block, at the exclusive prefix of the
// item counts in slot order (which is Phi order), so no separate scan of the
// per-block counts is needed.
__global__ __launch_bounds__(WG) void k_compact_write(DevParams P, int H, const unsigned* __restrict__ partials,
                                                      int tiles, int* __restrict__ slot_of, bool items) {
    __shared__ unsigned lds[WG / 64];
    // Loads first: the keys, then the fields of the occupied slots, all in
    // flight while the tile sums are read and scanned (the barriers of those
    // scans would otherwise hold them back).
    const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint64_t key[SCAN_ITEMS], mask[SCAN_ITEMS];
    int st[SCAN_ITEMS], en[SCAN_ITEMS], ent[SCAN_ITEMS];
    bool occ[SCAN_ITEMS];
    unsigned s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int idx = base + j;
        key[j] = idx < H ? P.h_keys[idx] : EMPTY_KEY;
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int idx = base + j;
        occ[j] = key[j] != EMPTY_KEY;
        s += occ[j];
        st[j] = -1;
        en[j] = -1;
        if (occ[j]) {
            mask[j] = P.h_mask[idx];
            st[j] = P.h_start[idx];
            en[j] = P.h_end[idx];
            ent[j] = P.b_entry ? P.h_entry[idx] : -1;
        }
    }
    unsigned wsum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) wsum += st[j] >= 0 ? block_chunks(P, en[j] - st[j]) : 0u;
    unsigned before, total, wbefore = 0, wtotal = 0;
    tile_offset(partials, blockIdx.x, tiles, lds, &before, &total);
    if (items) tile_offset(partials + tiles, blockIdx.x, tiles, lds, &wbefore, &wtotal);
    unsigned tot;
    unsigned phi = wg_excl_scan(s, lds, &tot) + before;
    unsigned w = items ? wg_excl_scan(wsum, lds, &tot) + wbefore : 0u;
    bool over = false;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        if (!occ[j]) continue;
        const int idx = base + j;
        const int cnt = st[j] >= 0 ? en[j] - st[j] : 0;
        const unsigned chunks = block_chunks(P, cnt);
        if ((int)phi < P.block_cap) {
            P.b_keys[phi] = key[j];
            P.b_mask[phi] = mask[j];
            P.b_start[phi] = st[j];
            P.b_count[phi] = cnt;
            P.h_vals[idx] = (int)phi;
            if (slot_of) slot_of[phi] = idx;
            if (P.b_entry) P.b_entry[phi] = ent[j];
            if (items) {
                P.b_chunks[phi] = chunks;
                for (unsigned k = 0; k < chunks; ++k) {
                    if (w + k >= (unsigned)P.work_cap) {
                        over = true;
                        break;
                    }
                    P.w_block[w + k] = (int)phi;
                    P.w_start[w + k] = st[j] + (int)k * P.chunk;
                    P.w_end[w + k] = min(st[j] + ((int)k + 1) * P.chunk, en[j]);
                }
            }
        } else {
            P.h_vals[idx] = -1;
            over = true;
        }
        w += chunks;
        ++phi;
    }
    if (over) raise_flag(P.ctr, MPM_FLAG_OVERFLOW);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.ctr->n_touched = total;
        P.ctr->nb = min((int)total, P.block_cap);
        // items of blocks past the capacity were not written: no work then
        if (items) P.ctr->n_work = total <= (unsigned)P.block_cap ? (int)wtotal : 0;
    }
}

// Ascending-key order of Phi (MPM_FLAG_DETERMINISTIC_ORDER).  The compaction
// wrote the block tables in slot order into the alternate arrays; the blocks
// are sorted by their coordinates (instance, i, j, k), which is the order of
// the Eq. 22 keys, and gathered into the block tables in that order.
template <int DIM>
__global__ __launch_bounds__(WG) void k_det_keys(DevParams P, const uint64_t* __restrict__ alt_keys,
                                                 uint32_t* __restrict__ rank_keys, uint32_t sentinel) {
    const int nb = P.ctr->nb;
    for (int b = blockIdx.x * WG + threadIdx.x; b < P.block_cap; b += gridDim.x * WG) {
        uint32_t r = sentinel;
        if (b < nb) {
            int bc[3], inst;
            unblock_key<DIM>(P, alt_keys[b], bc, &inst);
            const uint32_t lin = DIM == 3 ? ((uint32_t)bc[0] * (uint32_t)P.nblk[1] + (uint32_t)bc[1]) *
                                                    (uint32_t)P.nblk[2] + (uint32_t)bc[2]
                                          : (uint32_t)bc[0] * (uint32_t)P.nblk[1] + (uint32_t)bc[1];
            r = ((uint32_t)inst << P.blk_bits) | lin;
        }
        rank_keys[b] = r;
    }
}

__global__ __launch_bounds__(WG) void k_det_apply(DevParams P, DetTables T, const uint32_t* __restrict__ sorted) {
    const int nb = P.ctr->nb;
    for (int r = blockIdx.x * WG + threadIdx.x; r < nb; r += gridDim.x * WG) {
        const int b = (int)sorted[r];
        P.b_keys[r] = T.keys[b];
        P.b_mask[r] = T.mask[b];
        P.b_start[r] = T.start[b];
        P.b_count[r] = T.count[b];
        P.h_vals[T.slot[b]] = r;
    }
}

// Neighbour tables and chunking of the compact blocks, 2^(d+1) lanes per block:
// lane j < 2^d looks up upper neighbour j, lane 2^d + j lower neighbour j (so
// the probe chains of a block run side by side, not one after another).
template <int DIM>
__global__ __launch_bounds__(WG) void k_block_setup(DevParams P) {
    constexpr int NB = 1 << DIM;
    constexpr int LPB = 2 * NB;
    constexpr int NC = 1 << (2 * DIM);
    const int nb = P.ctr->nb;
    const long long total = (long long)nb * LPB;
    for (long long t = (long long)blockIdx.x * WG + threadIdx.x; t < total; t += (long long)gridDim.x * WG) {
        const int b = (int)(t / LPB), j = (int)(t % LPB);
        const int d = j % NB;
        // the block's count is loaded beside its key, not after the lookups
        const uint64_t bkey = P.b_keys[b];
        int bcount = P.b_count[b];
        asm volatile("" : "+v"(bcount));
        int bc[3], inst;
        unblock_key<DIM>(P, bkey, bc, &inst);
        if (j < NB) {
            P.b_nbr[b * NB + d] =
                d == 0 ? b
                       : hash_lookup(P, block_key<DIM>(P, bc[0] + (d & 1), bc[1] + ((d >> 1) & 1),
                                                       bc[2] + ((d >> 2) & 1), inst));
        } else if (P.b_lo) {
            // lower neighbours that own particles (the blocks whose P2G tiles
            // reach this block), -1 for the others
            const int lo = d == 0 ? b
                                  : hash_lookup(P, block_key<DIM>(P, bc[0] - (d & 1), bc[1] - ((d >> 1) & 1),
                                                                  bc[2] - ((d >> 2) & 1), inst));
            P.b_lo[b * NB + d] = (lo >= 0 && P.b_count[lo] > 0) ? lo : -1;
        }
        const unsigned chunks = (unsigned)((bcount + P.chunk - 1) / P.chunk);
        if (j == 0) P.b_chunks[b] = chunks;
        if (P.rs_stay) {
            // for the next incremental re-sort, when a G2P bins its output:
            // the owner part of the block's sort key, and cleared per-cell
            // stayer counts and entry total where G2P will not store them
            // whole (no particle, or several work items adding theirs)
            if (j == 0) {
                bool in_range = inst < max(P.n_inst, 1);
#pragma unroll
                for (int a = 0; a < DIM; ++a) in_range = in_range && bc[a] >= 0 && bc[a] < P.nblk[a];
                uint32_t owner = ~0u;
                if (in_range) {
                    const uint32_t bl = DIM == 3 ? ((uint32_t)bc[2] * (uint32_t)P.nblk[1] + (uint32_t)bc[1]) *
                                                           (uint32_t)P.nblk[0] + (uint32_t)bc[0]
                                                 : (uint32_t)bc[1] * (uint32_t)P.nblk[0] + (uint32_t)bc[0];
                    owner = ((uint32_t)inst << P.blk_bits) | bl;
                }
                P.rs_oldblk[b] = owner;
            }
            if (chunks != 1u) {
                for (int c = j; c < NC; c += LPB) P.rs_stay[(size_t)b * NC + c] = 0u;
                if (j == 0) P.rs_cnt[b] = 0u;
            }
        }
    }
    if (P.rs_stay && blockIdx.x == 0 && threadIdx.x == 0) {
        P.ctr->rs_n_mov = 0;  // the movers the next G2P lists
        P.ctr->rs_n_new = 0;  // the new blocks the next re-sort's route claims
    }
}

__global__ __launch_bounds__(WG) void k_work_write(DevParams P) {
    const int nb = P.ctr->nb;
    bool over = false;
    for (int b = blockIdx.x * WG + threadIdx.x; b < nb; b += gridDim.x * WG) {
        const int c = (int)P.b_chunks[b];
        const int off = (int)P.b_chunk_off[b];
        const int st = P.b_start[b], cnt = P.b_count[b];
        for (int j = 0; j < c; ++j) {
            const int w = off + j;
            if (w >= P.work_cap) {
                over = true;
                break;
            }
            P.w_block[w] = b;
            P.w_start[w] = st + j * P.chunk;
            P.w_end[w] = min(st + (j + 1) * P.chunk, st + cnt);
        }
    }
    if (over) raise_flag(P.ctr, MPM_FLAG_OVERFLOW);
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_grid_clear(DevParams P, long long n_nodes) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (long long s = (long long)blockIdx.x * WG + threadIdx.x; s < n_nodes; s += (long long)gridDim.x * WG)
        P.grid[s] = z;
}

// ---- dense baseline: Phi(b) = linear block index over the whole domain ----
__global__ __launch_bounds__(WG) void k_dense_clear_seg(DevParams P, int n_blocks) {
    for (int b = blockIdx.x * WG + threadIdx.x; b < n_blocks; b += gridDim.x * WG) {
        P.b_start[b] = -1;
        P.b_count[b] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.ctr->nb = n_blocks;
        P.ctr->n_touched = n_blocks;
        P.ctr->n_work = 0;
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_dense_segments(DevParams P, const uint32_t* __restrict__ skeys, int n) {
    constexpr int CB = 2 * DIM;
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= n) return;
    const uint32_t bl = skeys[i] >> CB;
    if (i == 0 || (skeys[i - 1] >> CB) != bl) P.b_start[bl] = i;
    if (i == n - 1 || (skeys[i + 1] >> CB) != bl) P.b_count[bl] = i + 1;  // end, converted below
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_dense_setup(DevParams P, int n_blocks) {
    constexpr int NB = 1 << DIM;
    for (int b = blockIdx.x * WG + threadIdx.x; b < n_blocks; b += gridDim.x * WG) {
        const int st = P.b_start[b];
        const int cnt = st >= 0 ? P.b_count[b] - st : 0;
        P.b_count[b] = cnt;
        P.b_chunks[b] = (unsigned)((cnt + P.chunk - 1) / P.chunk);
        int bc[3];
        linear_to_block<DIM>(P, (uint32_t)b, bc);
#pragma unroll
        for (int d = 0; d < NB; ++d) {
            const int x = bc[0] + (d & 1), y = bc[1] + ((d >> 1) & 1), z = bc[2] + ((d >> 2) & 1);
            const bool in = x < P.nblk[0] && y < P.nblk[1] && (DIM == 2 || z < P.nblk[2]);
            P.b_nbr[b * NB + d] = in ? (DIM == 3 ? (z * P.nblk[1] + y) * P.nblk[0] + x : y * P.nblk[0] + x) : -1;
        }
    }
}

__global__ __launch_bounds__(WG) void k_copy_active(DevParams P, uint64_t* keys, uint64_t* masks, int cap) {
    const int nb = min(P.ctr->nb, cap);
    for (int b = blockIdx.x * WG + threadIdx.x; b < nb; b += gridDim.x * WG) {
        keys[b] = P.b_keys[b];
        masks[b] = P.b_mask[b];
    }
}

static int grid_for(long long items, int cap_wgs = 8192) {
    long long g = (items + WG - 1) / WG;
    if (g < 1) g = 1;
    if (g > cap_wgs) g = cap_wgs;
    return (int)g;
}

hipError_t launch_bin(const DevParams& P, const float* x, const uint32_t* inst, int n, uint32_t* keys, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int g = (n + WG * BIN_PER_THREAD - 1) / (WG * BIN_PER_THREAD);
    if (P.dim == 3)
        k_bin<3><<<g, WG, 0, s>>>(P, x, inst, n, keys);
    else
        k_bin<2><<<g, WG, 0, s>>>(P, x, inst, n, keys);
    return hipGetLastError();
}

hipError_t launch_build_sparse(const DevParams& P, const uint32_t* skeys, int n, unsigned H, unsigned* partials,
                               hipStream_t s, bool from_resort, const DetTables* det) {
    if (!from_resort) k_hash_clear<<<grid_for(H), WG, 0, s>>>(P, H);  // the re-sort's last pass clears it
    if (n > 0 && from_resort) {
        const int ge = grid_for(2ll * P.block_cap * 64, 16384);  // one wave per entry
        if (P.dim == 3)
            k_hash_insert_entries<3><<<ge, WG, 0, s>>>(P);
        else
            k_hash_insert_entries<2><<<ge, WG, 0, s>>>(P);
    } else if (n > 0) {
        const int per_wg = WG * HI_ROUNDS;
        if (P.dim == 3)
            k_hash_insert<3><<<(n + per_wg - 1) / per_wg, WG, 0, s>>>(P, skeys, n);
        else
            k_hash_insert<2><<<(n + per_wg - 1) / per_wg, WG, 0, s>>>(P, skeys, n);
    }
    const int tiles = ((int)H + SCAN_TILE - 1) / SCAN_TILE;
    const int gb = grid_for(P.block_cap, 2048);
    const int gs = grid_for(2ll * (1 << P.dim) * P.block_cap, 8192);  // k_block_setup: 2^(d+1) lanes per block
    // without the key order, Phi is slot order and the compaction also writes
    // the work items
    const bool items = det == nullptr;
    k_compact_count<<<tiles, WG, 0, s>>>(P, (int)H, partials, tiles, items);
    if (det) {
        // compaction in slot order into the alternate tables, then the blocks
        // sorted by key and gathered into the block tables
        DevParams Pa = P;
        Pa.b_keys = det->keys;
        Pa.b_mask = det->mask;
        Pa.b_start = det->start;
        Pa.b_count = det->count;
        k_compact_write<<<tiles, WG, 0, s>>>(Pa, (int)H, partials, tiles, det->slot, false);
        const int kb = P.blk_bits + (P.n_inst > 1 ? 6 : 0);
        const uint32_t sentinel = kb >= 32 ? 0xFFFFFFFFu : ((1u << kb) - 1u);
        if (P.dim == 3)
            k_det_keys<3><<<gb, WG, 0, s>>>(P, det->keys, det->k[1], sentinel);
        else
            k_det_keys<2><<<gb, WG, 0, s>>>(P, det->keys, det->k[1], sentinel);
        uint32_t *ko = nullptr, *vo = nullptr;
        hipError_t e = radix_sort(det->k[1], det->k[0], det->k[1], det->v[0], det->v[1], P.block_cap, kb, det->hist,
                                  partials, &ko, &vo, s);
        if (e != hipSuccess) return e;
        k_det_apply<<<gb, WG, 0, s>>>(P, *det, vo);
    } else {
        k_compact_write<<<tiles, WG, 0, s>>>(P, (int)H, partials, tiles, nullptr, true);
    }
    if (P.dim == 3)
        k_block_setup<3><<<gs, WG, 0, s>>>(P);
    else
        k_block_setup<2><<<gs, WG, 0, s>>>(P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // no grid clear: the second P2G pass writes every node of every active block
    return items ? hipSuccess : launch_work_items(P, partials, s);
}

// Work items: exclusive scan of the per-block chunk counts, then the items.
hipError_t launch_work_items(const DevParams& P, unsigned* partials, hipStream_t s) {
    hipError_t e = scan_exclusive(P.b_chunks, P.b_chunk_off, P.block_cap, &P.ctr->nb, partials,
                                  (unsigned*)&P.ctr->n_work, s);
    if (e != hipSuccess) return e;
    k_work_write<<<grid_for(P.block_cap, 2048), WG, 0, s>>>(P);
    return hipGetLastError();
}

hipError_t launch_build_dense(const DevParams& P, const uint32_t* skeys, int n, int n_blocks, unsigned* partials,
                              hipStream_t s) {
    const int gb = grid_for(n_blocks);
    k_dense_clear_seg<<<gb, WG, 0, s>>>(P, n_blocks);
    if (n > 0) {
        if (P.dim == 3)
            k_dense_segments<3><<<(n + WG - 1) / WG, WG, 0, s>>>(P, skeys, n);
        else
            k_dense_segments<2><<<(n + WG - 1) / WG, WG, 0, s>>>(P, skeys, n);
    }
    if (P.dim == 3)
        k_dense_setup<3><<<gb, WG, 0, s>>>(P, n_blocks);
    else
        k_dense_setup<2><<<gb, WG, 0, s>>>(P, n_blocks);
    hipError_t e = scan_exclusive(P.b_chunks, P.b_chunk_off, n_blocks, nullptr, partials,
                                  (unsigned*)&P.ctr->n_work, s);
    if (e != hipSuccess) return e;
    k_work_write<<<gb, WG, 0, s>>>(P);
    const long long NPB = P.dim == 3 ? 64 : 16;
    if (P.dim == 3)
        k_grid_clear<3><<<grid_for((long long)n_blocks * NPB, 65536), WG, 0, s>>>(P, (long long)n_blocks * NPB);
    else
        k_grid_clear<2><<<grid_for((long long)n_blocks * NPB, 65536), WG, 0, s>>>(P, (long long)n_blocks * NPB);
    return hipGetLastError();
}

hipError_t launch_copy_active(const DevParams& P, uint64_t* keys, uint64_t* masks, int cap, hipStream_t s) {
    k_copy_active<<<grid_for(cap, 2048), WG, 0, s>>>(P, keys, masks, cap);
    return hipGetLastError();
}

}  // namespace mpmx
