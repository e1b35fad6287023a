// Incremental re-sort of the particles by owner block: the alternative to the
// full radix sort (sort.hip) for a build that follows a build of the same
// number of particles on the same context.
//
// The particle at position i of a step's G2P output belongs to the owner
// segment [b_start, b_start + b_count) of the previous build that contains i,
// and a step moves a particle by a fraction of a cell, so nearly all particles
// keep their owner block.  What the later stages need is a grouping, not a
// global order: each owner block's particles contiguous, base cells ascending
// inside the block.  The new layout keeps the previous blocks in their
// previous order and appends the blocks that had no slot before:
//   count    one wave per previous block: the particles whose new key has the
//            block's owner part ("stayers") are counted per base cell, the
//            others ("movers") per block;
//   list     the movers of each block are written, in segment order, at the
//            block's exclusive prefix of the mover counts;
//            (inside mpm_step the G2P that wrote the positions does count and
//            list itself, see k_g2p: stayer counts per block and cell and
//            their sum, the owner part of each block from the build before,
//            movers appended in any order; both passes are then skipped)
//   route    one thread per mover: its new block is looked up in the previous
//            hash table and the block's per-cell mover count and particle
//            count incremented, or, for a block without a previous slot, a
//            slot of a second hash table is claimed (the claiming thread
//            appends it to a list) and counted; the mover's target (entry
//            or slot) is recorded for the placement;
//   new      one wave per listed slot: the second table's blocks become the
//            entries after the previous blocks, in claim order;
//   totals   (only without the G2P's counting) particles per entry = stayers
//            + movers; then an exclusive scan over the entries gives each
//            entry's first position;
//   place    one wave per entry: first positions of its cells (a wave scan of
//            stayers + movers per cell); for a previous block each stayer
//            then takes the next position of its cell from an LDS counter (an
//            atomic, so stayers of one cell land in any order); then one
//            thread per mover: movers go after the stayers of their cell, each
//            taking the position its atomic decrement of the cell's mover
//            count names (which leaves the counts at zero for the next build);
//            the stayer pass also clears the tables the route has finished
//            with: the block hash for the insertion that follows and the
//            second table's keys for the next build.
// Cost: two reads of the new keys and one write of keys and values, against
// 2-4 full read/write passes of the radix sort.  The per-block kernels only
// stream keys; the dependent lookups of the few movers run one per thread, so
// their latencies overlap instead of stalling a block's wave.
#include <algorithm>

#include "internal.h"

namespace mpmx {

namespace {

// Lanes whose value v (its low BITS bits) equals this lane's, among lanes with
// `valid` set.  Every lane of the wave must call it.
template <int BITS>
__device__ __forceinline__ unsigned long long match_bits(unsigned v, bool valid) {
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool bit = (v >> b) & 1u;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// 64-bit block key (Eq. 22, instance folded in) of the owner part of a sort key.
template <int DIM>
__device__ __forceinline__ uint64_t owner_block_key(const DevParams& P, uint32_t owner) {
    const uint32_t bl = owner & ((1u << P.blk_bits) - 1u);
    const int inst = (int)(owner >> P.blk_bits);
    int bc[3];
    linear_to_block<DIM>(P, bl, bc);
    return block_key<DIM>(P, bc[0], bc[1], bc[2], inst);
}

// Second table: same size, hash and probing as the block table.  *claimed is
// set for the one caller whose CAS stored the key.
__device__ int nh_insert(const DevParams& P, uint64_t K, bool* claimed) {
    unsigned s = (unsigned)mix64(K) & P.h_mask_bits;
    *claimed = false;
    for (int r = 0; r < P.n_probe; ++r) {
        const uint64_t cur = __hip_atomic_load(&P.nh_keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == K) return (int)s;
        if (cur == EMPTY_KEY) {
            const uint64_t old = atomicCAS((unsigned long long*)&P.nh_keys[s], (unsigned long long)EMPTY_KEY,
                                           (unsigned long long)K);
            *claimed = old == EMPTY_KEY;
            if (old == EMPTY_KEY || old == K) return (int)s;
        }
        s = (s + 1) & P.h_mask_bits;
    }
    return -1;
}

}  // namespace

constexpr int RS_BATCH = 8;  // 64-particle chunks of a segment whose keys are loaded together

// count: one wave per previous block e (its segment of the previous order);
// the block's mover count goes to rs_cnt[e] (rs_cnt and rs_start serve the
// mover list first, the entry scan later).
template <int DIM>
__global__ __launch_bounds__(WG) void k_rs_count(DevParams P, const uint32_t* __restrict__ keys_new) {
    constexpr int CB = 2 * DIM, NC = 1 << CB;
    __shared__ unsigned cnt[WG / 64][64];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int nb = min(P.ctr->nb, P.block_cap);
    const int stride = gridDim.x * (WG / 64);
    int s_n = 0, c_n = 0;
    auto fetch = [&](int e) {  // the wave's next block, loaded while the current one is counted
        c_n = 0;
        if (e < nb) {
            asm volatile("" : "+v"(e));  // same in every lane; keeps the values in vector registers
            s_n = P.b_start[e];
            c_n = P.b_count[e];
        }
    };
    fetch(blockIdx.x * (WG / 64) + w);
    for (int e = blockIdx.x * (WG / 64) + w; e < nb; e += stride) {
        const int s = s_n, c = c_n;
        fetch(e + stride);
        cnt[w][lane] = 0u;
        // owner part of the block's sort key, stored by the previous build (a
        // block that only held stencil nodes may still receive movers)
        const uint32_t owner = P.rs_oldblk[e];
        unsigned n_mov = 0u;
        if (c > 0) {
            const int end = s + c;
            for (int i0 = s; i0 < end; i0 += 64 * RS_BATCH) {
                uint32_t k[RS_BATCH];
#pragma unroll
                for (int r = 0; r < RS_BATCH; ++r) {
                    const int i = i0 + r * 64 + lane;
                    k[r] = i < end ? keys_new[i] : 0u;
                }
#pragma unroll
                for (int r = 0; r < RS_BATCH; ++r) {
                    if (i0 + r * 64 >= end) break;  // uniform
                    const int i = i0 + r * 64 + lane;
                    const bool valid = i < end;
                    const bool stay = valid && (k[r] >> CB) == owner;
                    const uint32_t cell = k[r] & (NC - 1);
                    const unsigned long long m = match_bits<CB>(cell, stay);
                    if (stay && (m & lt) == 0ull) cnt[w][cell] += (unsigned)__popcll(m);  // one leader per cell
                    n_mov += (unsigned)__popcll(__ballot(valid && !stay));
                }
            }
        }
        if (lane < NC) P.rs_stay[(size_t)e * NC + lane] = cnt[w][lane];
        if (lane == 0) P.rs_cnt[e] = n_mov;
    }
}

// list: one wave per previous block with movers; rs_start[e] is its offset in
// the mover list (exclusive scan of the counts, total in rs_n_mov).
template <int DIM>
__global__ __launch_bounds__(WG) void k_rs_list(DevParams P, const uint32_t* __restrict__ keys_new,
                                                uint32_t* __restrict__ movers, int n) {
    constexpr int CB = 2 * DIM;
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int nb = min(P.ctr->nb, P.block_cap);
    for (int e = blockIdx.x * (WG / 64) + w; e < nb; e += gridDim.x * (WG / 64)) {
        if (P.rs_cnt[e] == 0u) continue;
        const int s = P.b_start[e], end = s + P.b_count[e];
        const uint32_t owner = P.rs_oldblk[e];
        unsigned slot0 = P.rs_start[e];
        for (int i0 = s; i0 < end; i0 += 64 * RS_BATCH) {
            uint32_t k[RS_BATCH];
#pragma unroll
            for (int r = 0; r < RS_BATCH; ++r) {
                const int i = i0 + r * 64 + lane;
                k[r] = i < end ? keys_new[i] : 0u;
            }
#pragma unroll
            for (int r = 0; r < RS_BATCH; ++r) {
                if (i0 + r * 64 >= end) break;  // uniform
                const int i = i0 + r * 64 + lane;
                const bool mover = i < end && (k[r] >> CB) != owner;
                const unsigned long long mv = __ballot(mover);
                const unsigned slot = slot0 + (unsigned)__popcll(mv & lt);
                if (mover && slot < (unsigned)n) movers[slot] = (uint32_t)i;
                slot0 += (unsigned)__popcll(mv);
            }
        }
    }
}

// route: one thread per mover.
// Target of a mover, recorded by the route for the placement: its previous
// entry, or (RS_TGT_NEW | slot) a slot of the second table, or RS_TGT_NONE.
constexpr uint32_t RS_TGT_NEW = 0x80000000u;
constexpr uint32_t RS_TGT_NONE = 0xFFFFFFFFu;

template <int DIM>
__global__ __launch_bounds__(WG) void k_rs_route(DevParams P, const uint32_t* __restrict__ keys_new,
                                                 const uint32_t* __restrict__ movers, uint32_t* __restrict__ tgt,
                                                 int n) {
    constexpr int CB = 2 * DIM, NC = 1 << CB;
    const int m = min(P.ctr->rs_n_mov, n);
    for (int t = blockIdx.x * WG + threadIdx.x; t < m; t += gridDim.x * WG) {
        const uint32_t k = keys_new[movers[t]];
        const uint32_t cell = k & (NC - 1);
        const uint64_t K = owner_block_key<DIM>(P, k >> CB);
        const int phi = hash_lookup(P, K);
        uint32_t target = RS_TGT_NONE;
        if (phi >= 0) {
            atomicAdd(&P.rs_in[(size_t)phi * NC + cell], 1u);
            atomicAdd(&P.rs_cnt[phi], 1u);
            target = (uint32_t)phi;
        } else {
            bool claimed;
            const int slot = nh_insert(P, K, &claimed);
            if (slot >= 0) {
                atomicAdd(&P.nh_cnt[(size_t)slot * NC + cell], 1u);
                P.nh_owner[slot] = k >> CB;  // the same value from every mover of the block
                if (claimed) {
                    // the slot joins the list of new blocks (claim order)
                    const int j = atomicAdd(&P.ctr->rs_n_new, 1);
                    if (j < P.block_cap) P.rs_new[j] = (uint32_t)slot;
                }
                target = RS_TGT_NEW | (uint32_t)slot;
            } else {
                raise_flag(P.ctr, MPM_FLAG_OVERFLOW);
            }
        }
        tgt[t] = target;
    }
}

// new: one wave per block that the route claimed in the second table, in claim
// order; block j becomes entry nb + j, with its mover counts (cleared in the
// table) as the entry's row and their sum as its particle count.
template <int DIM>
__global__ __launch_bounds__(WG) void k_rs_new_write(DevParams P) {
    constexpr int NC = 1 << (2 * DIM);
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int nb = min(P.ctr->nb, P.block_cap);
    const int max_ent = 2 * P.block_cap;
    const int n_new = P.ctr->rs_n_new;
    const int listed = min(n_new, P.block_cap);
    bool over = n_new > listed;
    for (int j = blockIdx.x * (WG / 64) + w; j < listed; j += gridDim.x * (WG / 64)) {
        const uint32_t slot = P.rs_new[j];
        const int e = nb + j;
        uint32_t* src = &P.nh_cnt[(size_t)slot * NC];
        const unsigned c = lane < NC ? src[lane] : 0u;
        if (lane < NC) src[lane] = 0u;
        const unsigned tot = wave_incl_scan(c);
        if (e < max_ent) {
            if (lane < NC) P.rs_in[(size_t)e * NC + lane] = c;
            if (lane == 63) {
                P.nh_idx[slot] = e;
                P.rs_oldblk[e] = P.nh_owner[slot];
                P.rs_cnt[e] = tot;
            }
        } else {
            if (lane == 0) P.nh_idx[slot] = -1;
            over = true;
        }
    }
    if (over) raise_flag(P.ctr, MPM_FLAG_OVERFLOW);
    if (blockIdx.x == 0 && threadIdx.x == 0) P.ctr->rs_n_ent = min(nb + listed, max_ent);
}

// Particles of entry e in base cell `lane` (0 for lanes >= NC).
template <int DIM>
__device__ __forceinline__ unsigned entry_cell_count(const DevParams& P, int e, int nb, int lane) {
    constexpr int NC = 1 << (2 * DIM);
    if (lane >= NC) return 0u;
    const unsigned st = e < nb ? P.rs_stay[(size_t)e * NC + lane] : 0u;
    return st + P.rs_in[(size_t)e * NC + lane];
}

// totals: particles per entry (one wave per entry), when no G2P counted the
// stayers (the route has added the movers of the previous blocks to counts
// that this pass replaces).
template <int DIM>
__global__ __launch_bounds__(WG) void k_rs_entry_count(DevParams P) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int nb = min(P.ctr->nb, P.block_cap);
    const int ne = P.ctr->rs_n_ent;
    for (int e = blockIdx.x * (WG / 64) + w; e < ne; e += gridDim.x * (WG / 64)) {
        const unsigned tot = wave_incl_scan(entry_cell_count<DIM>(P, e, nb, lane));
        if (lane == 63) P.rs_cnt[e] = tot;
    }
}

constexpr int RS_STAGE = 768;  // particles of a block whose output is staged in LDS (larger: direct stores);
                                // 25 KB of LDS per workgroup, six workgroups per compute unit
constexpr uint32_t RS_EMPTY = 0xFFFFFFFFu;  // staging slot left to a mover (indices are < 2^30)

// place, stayers: one wave per entry.  The wave first turns the entry's cell
// counts (stayers and movers) and its first position into the first position
// of every cell (rs_off); for a previous block it then walks the block's
// segment in the previous order and places the stayers.  The block's output
// range (stayers and the movers that join it) is staged in LDS and written out
// contiguously; the metadata of the wave's next entry is loaded while the
// current one is placed.
// KEYS: the sorted keys are written too (keys_out); without them the staging
// holds values only, half the LDS.
template <int DIM, bool KEYS>
__global__ __launch_bounds__(WG) void k_rs_place(DevParams P, const uint32_t* __restrict__ keys_new,
                                                 uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                                 int n, unsigned H) {
    constexpr int CB = 2 * DIM, NC = 1 << CB;
    __shared__ unsigned run[WG / 64][64];
    __shared__ uint32_t sk[WG / 64][KEYS ? RS_STAGE : 1], sv[WG / 64][RS_STAGE];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int nb = min(P.ctr->nb, P.block_cap);
    const int ne = P.ctr->rs_n_ent;
    const int stride = gridDim.x * (WG / 64);
    int s_n = 0, c_n = 0;
    unsigned base_n = 0u, tot_n = 0u, st_n = 0u, in_n = 0u;
    uint32_t owner_n = 0u;
    auto fetch = [&](int e) {
        c_n = 0;
        if (e < ne) {
            asm volatile("" : "+v"(e));  // same in every lane; keeps the values in vector registers
            const bool prev = e < nb;
            s_n = prev ? P.b_start[e] : 0;
            c_n = prev ? P.b_count[e] : 0;
            owner_n = P.rs_oldblk[e];
            base_n = P.rs_start[e];
            tot_n = P.rs_cnt[e];
            st_n = prev && lane < NC ? P.rs_stay[(size_t)e * NC + lane] : 0u;
            in_n = lane < NC ? P.rs_in[(size_t)e * NC + lane] : 0u;
        }
    };
    bool bad = false;
    fetch(blockIdx.x * (WG / 64) + w);
    for (int e = blockIdx.x * (WG / 64) + w; e < ne; e += stride) {
        const int s = s_n, c = c_n;
        const uint32_t owner = owner_n;
        const unsigned base = base_n, tot = tot_n, cv = st_n + in_n;
        fetch(e + stride);
        const unsigned off = base + wave_incl_scan(cv) - cv;
        if (lane < NC) P.rs_off[(size_t)e * NC + lane] = off;
        if (c <= 0) continue;
        const bool staged = tot <= (unsigned)RS_STAGE;
        if (staged)
            for (unsigned j = lane; j < tot; j += 64) sv[w][j] = RS_EMPTY;
        run[w][lane] = off;
        const int end = s + c;
        for (int i0 = s; i0 < end; i0 += 64 * RS_BATCH) {
            uint32_t k[RS_BATCH];
#pragma unroll
            for (int r = 0; r < RS_BATCH; ++r) {
                const int i = i0 + r * 64 + lane;
                k[r] = i < end ? keys_new[i] : 0u;
            }
#pragma unroll
            for (int r = 0; r < RS_BATCH; ++r) {
                if (i0 + r * 64 >= end) break;  // uniform
                const int i = i0 + r * 64 + lane;
                const bool stay = i < end && (k[r] >> CB) == owner;
                const uint32_t cell = k[r] & (NC - 1);
                if (stay) {
                    // next position of the cell: an LDS atomic on its counter
                    // (lanes hitting one counter are served one after another,
                    // so any order of them is a valid placement)
                    const unsigned pos = atomicAdd(&run[w][cell], 1u);
                    if (staged && pos - base < tot) {
                        if (KEYS) sk[w][pos - base] = k[r];
                        sv[w][pos - base] = (uint32_t)i;
                    } else if (!staged && pos < (unsigned)n) {
                        if (KEYS) keys_out[pos] = k[r];
                        vals_out[pos] = (uint32_t)i;
                    } else {
                        bad = true;
                    }
                }
            }
        }
        if (staged) {
            for (unsigned j = lane; j < tot; j += 64) {
                const uint32_t v = sv[w][j];
                if (v != RS_EMPTY && base + j < (unsigned)n) {
                    if (KEYS) keys_out[base + j] = sk[w][j];
                    vals_out[base + j] = v;
                }
            }
        }
    }
    if (bad) raise_flag(P.ctr, MPM_FLAG_OVERFLOW);
    // The tables the route has finished with are cleared here, behind the
    // placement's latency-bound work: the block hash for the insertion that
    // follows (Algorithm 5's initialisation) and the second table's keys for
    // the next re-sort.  (The movers' placement reads the route's recorded
    // targets, not the tables.)
    for (long long t = (long long)blockIdx.x * WG + threadIdx.x; t < (long long)H; t += (long long)gridDim.x * WG) {
        P.nh_keys[t] = EMPTY_KEY;
        P.h_keys[t] = EMPTY_KEY;
        P.h_mask[t] = 0ull;
        P.h_start[t] = -1;
        P.h_end[t] = -1;
        P.h_entry[t] = -1;
    }
}

// place, movers: one thread per mover, after the stayers of its cell.
template <int DIM>
__global__ __launch_bounds__(WG) void k_rs_place_movers(DevParams P, const uint32_t* __restrict__ keys_new,
                                                        const uint32_t* __restrict__ movers,
                                                        const uint32_t* __restrict__ tgt,
                                                        uint32_t* __restrict__ keys_out,
                                                        uint32_t* __restrict__ vals_out, int n) {
    constexpr int CB = 2 * DIM, NC = 1 << CB;
    const int m = min(P.ctr->rs_n_mov, n);
    const int ne = P.ctr->rs_n_ent;
    const int nb = min(P.ctr->nb, P.block_cap);
    bool bad = false;
    for (int t = blockIdx.x * WG + threadIdx.x; t < m; t += gridDim.x * WG) {
        const uint32_t i = movers[t];
        const uint32_t k = keys_new[i];
        const uint32_t cell = k & (NC - 1);
        const uint32_t target = tgt[t];  // the route's lookup, so no table is probed again
        const bool prev = (target & RS_TGT_NEW) == 0u;
        int e2 = -1;
        if (prev) {
            e2 = (int)target < nb ? (int)target : -1;
        } else if (target != RS_TGT_NONE) {
            e2 = P.nh_idx[target & ~RS_TGT_NEW];
            if (e2 >= ne) e2 = -1;
        }
        if (e2 < 0) {
            bad = true;
            continue;
        }
        const size_t r = (size_t)e2 * NC + cell;
        // the cell's movers still to place, this one included: the last of
        // them takes the first position after the stayers (the decrement and
        // the loads of the cell's offsets are in flight together)
        const unsigned left = atomicSub(&P.rs_in[r], 1u);
        const unsigned b0 = P.rs_off[r] + (prev ? P.rs_stay[r] : 0u);
        const unsigned pos = b0 + left - 1u;
        if (left != 0u && pos < (unsigned)n) {
            if (keys_out) keys_out[pos] = k;
            vals_out[pos] = i;
        } else {
            bad = true;
        }
    }
    if (bad) raise_flag(P.ctr, MPM_FLAG_OVERFLOW);
}

// Initial state of the buffers the re-sort expects between builds.
template <int DIM>
__global__ __launch_bounds__(WG) void k_rs_init(DevParams P, unsigned H) {
    constexpr int NC = 1 << (2 * DIM);
    const long long rows = 2ll * P.block_cap * NC;
    const long long hrows = (long long)H * NC;
    const long long all = rows > hrows ? rows : hrows;
    for (long long t = (long long)blockIdx.x * WG + threadIdx.x; t < all; t += (long long)gridDim.x * WG) {
        if (t < rows) P.rs_in[t] = 0u;
        if (t < hrows) P.nh_cnt[t] = 0u;
        if (t < (long long)H) {
            P.nh_keys[t] = EMPTY_KEY;
            P.nh_idx[t] = -1;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) P.ctr->rs_n_new = 0;
}

namespace {
int grid_for_waves(long long waves) {
    const long long g = (waves + WG / 64 - 1) / (WG / 64);
    return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}
}  // namespace

hipError_t launch_resort_init(const DevParams& P, unsigned H, hipStream_t s) {
    if (P.dim == 3)
        k_rs_init<3><<<4096, WG, 0, s>>>(P, H);
    else
        k_rs_init<2><<<4096, WG, 0, s>>>(P, H);
    return hipGetLastError();
}

// counted: the G2P that wrote keys_new already stored the stayer counts per
// previous block and cell, the owner part of each previous block and the
// mover list (in any order) with its length; count and list are skipped.
hipError_t launch_resort(const DevParams& P, const uint32_t* keys_new, uint32_t* keys_out, uint32_t* vals_out,
                         uint32_t* movers, uint32_t* tgt, int n, unsigned H, unsigned* partials, hipStream_t s,
                         bool counted) {
    const int gw = grid_for_waves(P.block_cap);
    const int ge = grid_for_waves(2ll * P.block_cap);
    const int gm = (int)std::min<long long>(((long long)n + WG - 1) / WG, 2048);  // grid-stride over the movers
    hipError_t e = hipSuccess;
    if (!counted) {
        if (P.dim == 3)
            k_rs_count<3><<<gw, WG, 0, s>>>(P, keys_new);
        else
            k_rs_count<2><<<gw, WG, 0, s>>>(P, keys_new);
        e = scan_exclusive(P.rs_cnt, P.rs_start, P.block_cap, &P.ctr->nb, partials, (unsigned*)&P.ctr->rs_n_mov,
                           s);
        if (e != hipSuccess) return e;
        if (P.dim == 3)
            k_rs_list<3><<<gw, WG, 0, s>>>(P, keys_new, movers, n);
        else
            k_rs_list<2><<<gw, WG, 0, s>>>(P, keys_new, movers, n);
    }
    if (P.dim == 3)
        k_rs_route<3><<<gm, WG, 0, s>>>(P, keys_new, movers, tgt, n);
    else
        k_rs_route<2><<<gm, WG, 0, s>>>(P, keys_new, movers, tgt, n);
    const int gn = 256;  // workgroups, grid-stride over the new blocks (a few hundred per step)
    if (P.dim == 3)
        k_rs_new_write<3><<<gn, WG, 0, s>>>(P);
    else
        k_rs_new_write<2><<<gn, WG, 0, s>>>(P);
    if (!counted) {
        if (P.dim == 3)
            k_rs_entry_count<3><<<ge, WG, 0, s>>>(P);
        else
            k_rs_entry_count<2><<<ge, WG, 0, s>>>(P);
    }
    e = scan_exclusive(P.rs_cnt, P.rs_start, 2 * P.block_cap, &P.ctr->rs_n_ent, partials, nullptr, s);
    if (e != hipSuccess) return e;
    if (P.dim == 3) {
        if (keys_out)
            k_rs_place<3, true><<<ge, WG, 0, s>>>(P, keys_new, keys_out, vals_out, n, H);
        else
            k_rs_place<3, false><<<ge, WG, 0, s>>>(P, keys_new, keys_out, vals_out, n, H);
        k_rs_place_movers<3><<<gm, WG, 0, s>>>(P, keys_new, movers, tgt, keys_out, vals_out, n);
    } else {
        if (keys_out)
            k_rs_place<2, true><<<ge, WG, 0, s>>>(P, keys_new, keys_out, vals_out, n, H);
        else
            k_rs_place<2, false><<<ge, WG, 0, s>>>(P, keys_new, keys_out, vals_out, n, H);
        k_rs_place_movers<2><<<gm, WG, 0, s>>>(P, keys_new, movers, tgt, keys_out, vals_out, n);
    }
    return hipGetLastError();
}

}  // namespace mpmx
