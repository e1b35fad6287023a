// Scan-based active set (the paper's first construction, Methods 3.2 and
// Algorithms 1-4, here on the GPU): the alternative to the hash table of
// Algorithms 5-6.  It yields the same active blocks and node masks, with the
// compact index Phi in ascending block-key order.
//
//   k_sb_bbox   bounding box of the owner blocks of all particles: each of a
//               fixed number of workgroups reduces its share (wave shuffles,
//               then LDS) and writes one partial box, no atomics;
//   k_sb_box    one workgroup reduces the partial boxes; the mask domain is the
//               box grown by one block on each upper side (a stencil spills
//               only upward), its extents and volume m, all on the device (no
//               host read-back);
//   k_sb_zero   occupancy of the m blocks of the domain <- 0;
//   k_sb_occ    per owner block, the 64-bit occupancy of its base cells (lanes
//               of a wave with the same owner merged by ballot, one atomicOr);
//               from sorted keys it also records each owner segment's first and
//               one-past-last sorted position;
//   k_sb_flag   per block of the domain: active iff the OR over itself and its
//               2^d - 1 lower neighbours of the dilated occupancy (own part for
//               itself, spill part for the neighbours) is non-zero, a gather
//               with no atomics;
//   scan        exclusive scan of the flags -> compact index (Eq. 18);
//   k_sb_write  keys (Eq. 22) and node masks of the flagged blocks, in the
//               domain's order: i slowest, k fastest, which is ascending key
//               order (Eq. 22 packs i highest);
//   step build  (k_sb_write_blocks, k_sb_block_setup) the same into the
//               context's block tables, owner segments, upper and lower
//               neighbours looked up in the domain instead of the hash table.
//
// The scratch (accumulators, occupancy, flags, Phi, segment bounds, scan
// partials) is passed in as an SbScratch: the context's own, allocated at
// create for the whole potential domain, or a fixed static device array.
#include <climits>

#include "internal.h"
#include "../../include/mpm.h"

namespace mpmx {

// Node masks of a block from its occupied base cells (bit i + 4 j + 16 k for
// cell or node (i, j, k)).  Along one axis a base cell at local index l covers
// nodes l, l+1, l+2: those below 4 stay in the block, those at 4 and 5 are
// nodes 0 and 1 of the upper neighbour.
__device__ __forceinline__ uint64_t sb_axis(uint64_t o, int shift, uint64_t lane_mask, bool spill) {
    // o holds 4 positions along the axis at strides of `shift` bits; lane_mask
    // selects position 0 of every row.
    const uint64_t p0 = o & lane_mask, p1 = (o >> shift) & lane_mask, p2 = (o >> (2 * shift)) & lane_mask,
                   p3 = (o >> (3 * shift)) & lane_mask;
    uint64_t q0, q1, q2, q3;
    if (!spill) {  // nodes 0..3 of the block
        q0 = p0;
        q1 = p0 | p1;
        q2 = p0 | p1 | p2;
        q3 = p1 | p2 | p3;
    } else {  // nodes 0..1 of the upper neighbour (4 and 5 of this block's frame)
        q0 = p2 | p3;
        q1 = p3;
        q2 = 0;
        q3 = 0;
    }
    return q0 | (q1 << shift) | (q2 << (2 * shift)) | (q3 << (3 * shift));
}

template <int DIM>
__device__ __forceinline__ uint64_t sb_node_mask(uint64_t occ, int d) {
    if (DIM == 2) {
        uint64_t o = sb_axis(occ, 1, 0x1111ull, d & 1);
        return sb_axis(o, 4, 0x000Full, (d >> 1) & 1);
    }
    uint64_t o = sb_axis(occ, 1, 0x1111111111111111ull, d & 1);
    o = sb_axis(o, 4, 0x000F000F000F000Full, (d >> 1) & 1);
    return sb_axis(o, 16, 0x000000000000FFFFull, (d >> 2) & 1);
}

// Owner block coordinates and base cell of particle i, from a sorted key or,
// with x != nullptr, from its position (the binning arithmetic of k_bin: base
// node floor(x/dx - 1/2) in float64, clamped into the grid).
template <int DIM>
__device__ __forceinline__ void sb_owner(const DevParams& P, const float* __restrict__ x,
                                         const uint32_t* __restrict__ keys, int n, int i, int* bc, int* cell) {
    if (x) {
        int b[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double f = floor(index_arg(x[(size_t)a * n + i], P.inv_dx));
            if (!(f == f)) f = 0.0;
            f = fmin(fmax(f, 0.0), (double)(P.cells[a] - 2));
            b[a] = (int)f;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) bc[a] = b[a] >> 2;
        *cell = DIM == 3 ? ((b[0] & 3) | ((b[1] & 3) << 2) | ((b[2] & 3) << 4)) : ((b[0] & 3) | ((b[1] & 3) << 2));
        return;
    }
    const uint32_t k = keys[i];
    linear_to_block<DIM>(P, (k >> (2 * DIM)) & ((1u << P.blk_bits) - 1u), bc);
    *cell = (int)(k & ((1u << (2 * DIM)) - 1u));
}

// Domain index of block coordinates c (box-relative), i slowest, k fastest.
__device__ __forceinline__ long long sb_index(const SbBox& B, int c0, int c1, int c2) {
    return ((long long)c0 * B.ext[1] + c1) * B.ext[2] + c2;
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_bbox(DevParams P, const float* __restrict__ x,
                                                const uint32_t* __restrict__ keys, int n, int* __restrict__ bbp) {
    __shared__ int red[WG / 64][6];
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {-1, -1, -1};
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        int bc[3], cell;
        sb_owner<DIM>(P, x, keys, n, i, bc, &cell);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            lo[a] = min(lo[a], bc[a]);
            hi[a] = max(hi[a], bc[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int m = 32; m >= 1; m >>= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], m));
            hi[a] = max(hi[a], __shfl_xor(hi[a], m));
        }
    }
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            red[w][a] = lo[a];
            red[w][3 + a] = hi[a];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int t = threadIdx.x;
        int v = red[0][t];
        for (int q = 1; q < WG / 64; ++q) v = t < 3 ? min(v, red[q][t]) : max(v, red[q][t]);
        bbp[blockIdx.x * 8 + t] = v;
    }
}

// The bounding box from the partial boxes, and the extents of the mask domain;
// volume 0 when there is no particle or when it exceeds max_m (then too_big is
// set and nothing further is done).  The active-block total is set by the
// scan that follows.
template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_box(DevParams P, const int* __restrict__ bbp, int parts, SbBox* box,
                                               long long max_m) {
    __shared__ int red[WG / 64][6];
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {-1, -1, -1};
    for (int q = threadIdx.x; q < parts; q += WG) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], bbp[q * 8 + a]);
            hi[a] = max(hi[a], bbp[q * 8 + 3 + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int m = 32; m >= 1; m >>= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], m));
            hi[a] = max(hi[a], __shfl_xor(hi[a], m));
        }
    }
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            red[w][a] = lo[a];
            red[w][3 + a] = hi[a];
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int a = 0; a < 3; ++a) {
        box->lo[a] = red[0][a];
        box->hi[a] = red[0][3 + a];
        for (int q = 1; q < WG / 64; ++q) {
            box->lo[a] = min(box->lo[a], red[q][a]);
            box->hi[a] = max(box->hi[a], red[q][3 + a]);
        }
    }
    box->too_big = 0;
    long long m = 1;
    for (int a = 0; a < 3; ++a) {
        if (a >= DIM) {
            box->lo[a] = 0;
            box->ext[a] = 1;
            continue;
        }
        if (box->hi[a] < 0) {  // no particle
            m = 0;
            box->lo[a] = 0;
            box->ext[a] = 0;
            continue;
        }
        // owners lo..hi plus the upper neighbour, inside the potential domain
        box->ext[a] = min(box->hi[a] + 1, P.nblk[a] - 1) - box->lo[a] + 1;
        m *= box->ext[a];
    }
    if (m > max_m) {
        box->too_big = 1;
        m = 0;
    }
    box->m = (int)m;
}

__global__ __launch_bounds__(WG) void k_sb_zero(const SbBox* __restrict__ box, uint64_t* __restrict__ occ) {
    const int m = box->m;
    for (int t = blockIdx.x * WG + threadIdx.x; t < m; t += gridDim.x * WG) occ[t] = 0ull;
}

// Occupancy of each owner block's base cells; from sorted keys (x == nullptr)
// also the first and one-past-last sorted position of each owner segment.
template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_occ(DevParams P, const float* __restrict__ x,
                                               const uint32_t* __restrict__ keys, int n,
                                               const SbBox* __restrict__ box, uint64_t* __restrict__ occ,
                                               int* __restrict__ seg_lo, int* __restrict__ seg_hi) {
    const SbBox B = *box;
    if (B.m == 0) return;
    const int lane = __lane_id();
    for (int i0 = blockIdx.x * WG + (threadIdx.x & ~63); i0 < n; i0 += gridDim.x * WG) {
        const int i = i0 + lane;
        const bool valid = i < n;
        long long idx = -1;
        uint64_t bit = 0ull;
        if (valid) {
            int bc[3], cell;
            sb_owner<DIM>(P, x, keys, n, i, bc, &cell);
            idx = sb_index(B, bc[0] - B.lo[0], bc[1] - B.lo[1], bc[2] - B.lo[2]);
            bit = 1ull << cell;
            if (!x) {  // owner segment bounds of the sorted order
                const uint32_t seg = keys[i] >> (2 * DIM);
                if (i == 0 || (keys[i - 1] >> (2 * DIM)) != seg) seg_lo[idx] = i;
                if (i == n - 1 || (keys[i + 1] >> (2 * DIM)) != seg) seg_hi[idx] = i + 1;
            }
        }
        unsigned long long pending = __ballot(valid);
        while (pending) {  // one round per distinct owner block in the wave
            const int leader = __ffsll((long long)pending) - 1;
            const long long own = __shfl(idx, leader);
            const bool mine = valid && idx == own;
            const uint64_t mk = wave_or64(mine ? bit : 0ull);
            if (lane == leader) atomicOr((unsigned long long*)&occ[own], (unsigned long long)mk);
            pending &= ~__ballot(mine);
        }
    }
}

// Node mask of domain block (c0, c1, c2): its own dilated occupancy and the
// spills of its lower neighbours.
template <int DIM>
__device__ __forceinline__ uint64_t sb_mask_at(const SbBox& B, const uint64_t* __restrict__ occ, int c0, int c1,
                                               int c2) {
    constexpr int NB = 1 << DIM;
    uint64_t acc = 0ull;
#pragma unroll
    for (int d = 0; d < NB; ++d) {
        const int a0 = c0 - (d & 1), a1 = c1 - ((d >> 1) & 1), a2 = c2 - ((d >> 2) & 1);
        if (a0 < 0 || a1 < 0 || a2 < 0) continue;
        const uint64_t o = occ[sb_index(B, a0, a1, a2)];
        if (o) acc |= sb_node_mask<DIM>(o, d);
    }
    return acc;
}

__device__ __forceinline__ void sb_coords(const SbBox& B, int t, int* c) {
    c[2] = t % B.ext[2];
    const int r = t / B.ext[2];
    c[1] = r % B.ext[1];
    c[0] = r / B.ext[1];
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_flag(const SbBox* __restrict__ box, const uint64_t* __restrict__ occ,
                                                unsigned* __restrict__ flag) {
    const SbBox B = *box;
    for (int t = blockIdx.x * WG + threadIdx.x; t < B.m; t += gridDim.x * WG) {
        int c[3];
        sb_coords(B, t, c);
        flag[t] = sb_mask_at<DIM>(B, occ, c[0], c[1], c[2]) != 0ull ? 1u : 0u;
    }
}

// Keys and masks of the flagged blocks into caller arrays (the first cap).
template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_write(DevParams P, const SbBox* __restrict__ box,
                                                 const uint64_t* __restrict__ occ, const unsigned* __restrict__ flag,
                                                 const unsigned* __restrict__ phi, uint64_t* __restrict__ keys_out,
                                                 uint64_t* __restrict__ masks_out, int cap) {
    const SbBox B = *box;
    for (int t = blockIdx.x * WG + threadIdx.x; t < B.m; t += gridDim.x * WG) {
        if (!flag[t]) continue;
        const unsigned p = phi[t];
        if (p >= (unsigned)cap) continue;
        int c[3];
        sb_coords(B, t, c);
        keys_out[p] = block_key<DIM>(P, B.lo[0] + c[0], B.lo[1] + c[1], B.lo[2] + c[2], 0);
        masks_out[p] = sb_mask_at<DIM>(B, occ, c[0], c[1], c[2]);
    }
}

// Step build: the flagged blocks into the context's block tables in Phi order,
// with their owner segments; the block count and the capacity check.
template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_write_blocks(DevParams P, const SbBox* __restrict__ box,
                                                        const uint64_t* __restrict__ occ,
                                                        const unsigned* __restrict__ flag,
                                                        const unsigned* __restrict__ phi,
                                                        const int* __restrict__ seg_lo,
                                                        const int* __restrict__ seg_hi) {
    const SbBox B = *box;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.ctr->n_touched = (int)B.total;
        P.ctr->nb = min((int)B.total, P.block_cap);
        P.ctr->n_work = 0;
        if ((int)B.total > P.block_cap) raise_flag(P.ctr, MPM_FLAG_OVERFLOW);
    }
    for (int t = blockIdx.x * WG + threadIdx.x; t < B.m; t += gridDim.x * WG) {
        if (!flag[t]) continue;
        const unsigned p = phi[t];
        if (p >= (unsigned)P.block_cap) continue;
        int c[3];
        sb_coords(B, t, c);
        P.b_keys[p] = block_key<DIM>(P, B.lo[0] + c[0], B.lo[1] + c[1], B.lo[2] + c[2], 0);
        P.b_mask[p] = sb_mask_at<DIM>(B, occ, c[0], c[1], c[2]);
        const bool owns = occ[t] != 0ull;
        const int st = owns ? seg_lo[t] : -1;
        P.b_start[p] = st;
        P.b_count[p] = owns ? seg_hi[t] - st : 0;
    }
}

// Compact index of the domain block at box-relative c, -1 outside the domain
// or inactive (or past the capacity).
__device__ __forceinline__ int sb_phi_at(const DevParams& P, const SbBox& B, const unsigned* __restrict__ flag,
                                         const unsigned* __restrict__ phi, int c0, int c1, int c2) {
    if (c0 < 0 || c1 < 0 || c2 < 0 || c0 >= B.ext[0] || c1 >= B.ext[1] || c2 >= B.ext[2]) return -1;
    const long long t = sb_index(B, c0, c1, c2);
    if (!flag[t]) return -1;
    const unsigned p = phi[t];
    return p < (unsigned)P.block_cap ? (int)p : -1;
}

// Upper and lower neighbours (as k_block_setup, looked up in the domain) and
// the chunk count of each block.
template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_block_setup(DevParams P, const SbBox* __restrict__ box,
                                                       const unsigned* __restrict__ flag,
                                                       const unsigned* __restrict__ phi) {
    constexpr int NB = 1 << DIM;
    const SbBox B = *box;
    const int nb = P.ctr->nb;
    for (int b = blockIdx.x * WG + threadIdx.x; b < nb; b += gridDim.x * WG) {
        int bc[3], inst;
        unblock_key<DIM>(P, P.b_keys[b], bc, &inst);
        const int c0 = bc[0] - B.lo[0], c1 = bc[1] - B.lo[1], c2 = bc[2] - B.lo[2];
        P.b_nbr[b * NB] = b;
#pragma unroll
        for (int d = 1; d < NB; ++d)
            P.b_nbr[b * NB + d] = sb_phi_at(P, B, flag, phi, c0 + (d & 1), c1 + ((d >> 1) & 1), c2 + ((d >> 2) & 1));
        if (P.b_lo) {
            P.b_lo[b * NB] = P.b_count[b] > 0 ? b : -1;
#pragma unroll
            for (int d = 1; d < NB; ++d) {
                const int lo = sb_phi_at(P, B, flag, phi, c0 - (d & 1), c1 - ((d >> 1) & 1), c2 - ((d >> 2) & 1));
                P.b_lo[b * NB + d] = (lo >= 0 && P.b_count[lo] > 0) ? lo : -1;
            }
        }
        P.b_chunks[b] = (unsigned)((P.b_count[b] + P.chunk - 1) / P.chunk);
    }
}

namespace {
int sb_grid(long long items, int cap_wgs) {
    long long g = (items + WG - 1) / WG;
    if (g < 1) g = 1;
    if (g > cap_wgs) g = cap_wgs;
    return (int)g;
}

// Bounding box, domain, occupancy, flags and their scan: the part shared by
// the query and the step build.  x != nullptr: bins the positions on the fly;
// else reads sorted keys.
hipError_t sb_mark(const DevParams& P, const float* x, const uint32_t* keys, int n, const SbScratch& S,
                   hipStream_t s) {
    const int gp = sb_grid(n, 4096);
    const int gm = sb_grid(S.max_m, 8192);
    if (P.dim == 3) {
        k_sb_bbox<3><<<SB_BBOX_WGS, WG, 0, s>>>(P, x, keys, n, S.bbp);
        k_sb_box<3><<<1, WG, 0, s>>>(P, S.bbp, SB_BBOX_WGS, S.box, S.max_m);
        k_sb_zero<<<gm, WG, 0, s>>>(S.box, S.occ);
        if (n > 0) k_sb_occ<3><<<gp, WG, 0, s>>>(P, x, keys, n, S.box, S.occ, S.seg_lo, S.seg_hi);
        k_sb_flag<3><<<gm, WG, 0, s>>>(S.box, S.occ, S.flag);
    } else {
        k_sb_bbox<2><<<SB_BBOX_WGS, WG, 0, s>>>(P, x, keys, n, S.bbp);
        k_sb_box<2><<<1, WG, 0, s>>>(P, S.bbp, SB_BBOX_WGS, S.box, S.max_m);
        k_sb_zero<<<gm, WG, 0, s>>>(S.box, S.occ);
        if (n > 0) k_sb_occ<2><<<gp, WG, 0, s>>>(P, x, keys, n, S.box, S.occ, S.seg_lo, S.seg_hi);
        k_sb_flag<2><<<gm, WG, 0, s>>>(S.box, S.occ, S.flag);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan_exclusive(S.flag, S.phi, (int)S.max_m, &S.box->m, S.partials, &S.box->total, s);
}
}  // namespace

size_t sb_scratch_bytes(long long max_m) {
    // segment bounds (2 x i32 per block) are allocated by the step build's owner
    return sb_scratch_size(max_m);
}

SbScratch sb_carve(void* base, long long max_m, int* seg_lo, int* seg_hi) {
    SbScratch S{};
    char* p = (char*)base;
    S.box = (SbBox*)p;
    p += 256;
    S.bbp = (int*)p;
    p += (size_t)SB_BBOX_WGS * 8 * sizeof(int);
    S.occ = (uint64_t*)p;
    p += (size_t)max_m * 8;
    S.flag = (unsigned*)p;
    p += (size_t)max_m * 4;
    S.phi = (unsigned*)p;
    p += (size_t)max_m * 4;
    S.partials = (unsigned*)p;
    S.max_m = max_m;
    S.seg_lo = seg_lo;
    S.seg_hi = seg_hi;
    return S;
}

hipError_t launch_scan_active(const DevParams& P, const float* x, int n, const SbScratch& S, uint64_t* keys_out,
                              uint64_t* masks_out, int cap, hipStream_t s) {
    hipError_t e = sb_mark(P, x, nullptr, n, S, s);
    if (e != hipSuccess || cap <= 0) return e;
    const int gm = sb_grid(S.max_m, 8192);
    if (P.dim == 3)
        k_sb_write<3><<<gm, WG, 0, s>>>(P, S.box, S.occ, S.flag, S.phi, keys_out, masks_out, cap);
    else
        k_sb_write<2><<<gm, WG, 0, s>>>(P, S.box, S.occ, S.flag, S.phi, keys_out, masks_out, cap);
    return hipGetLastError();
}

hipError_t launch_build_scan(const DevParams& P, const uint32_t* skeys, int n, const SbScratch& S,
                             unsigned* partials, hipStream_t s) {
    hipError_t e = sb_mark(P, nullptr, skeys, n, S, s);
    if (e != hipSuccess) return e;
    const int gm = sb_grid(S.max_m, 8192);
    const int gb = sb_grid(P.block_cap, 2048);
    if (P.dim == 3) {
        k_sb_write_blocks<3><<<gm, WG, 0, s>>>(P, S.box, S.occ, S.flag, S.phi, S.seg_lo, S.seg_hi);
        k_sb_block_setup<3><<<gb, WG, 0, s>>>(P, S.box, S.flag, S.phi);
    } else {
        k_sb_write_blocks<2><<<gm, WG, 0, s>>>(P, S.box, S.occ, S.flag, S.phi, S.seg_lo, S.seg_hi);
        k_sb_block_setup<2><<<gb, WG, 0, s>>>(P, S.box, S.flag, S.phi);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_work_items(P, partials, s);
}

}  // namespace mpmx
