// Scan-based active set (the paper's first construction, Algorithms 1-4, here on
// the GPU): an alternative to the hash table of Algorithms 5-6 that yields the
// same active blocks and node masks, used to check one against the other and
// to compare their cost.
//
//   k_sb_bbox   bounding box of the owner blocks of all particles (wave min/max,
//               one atomic per wave and axis);
//   host        reads the box back; the mask domain is the box grown by one
//               block on each upper side (the stencil spills only upward);
//   k_sb_occ    per owner block, the 64-bit occupancy of its base cells (lanes
//               of a wave with the same owner merged by ballot, one atomicOr);
//   k_sb_mask   per block of the domain, its node mask: the OR over itself and
//               its 2^d - 1 lower neighbours of the dilated occupancy (own part
//               for itself, spill part for the neighbours), a gather with no
//               atomics; flag = mask != 0;
//   scan        exclusive scan of the flags -> compact index (Eq. 18);
//   k_sb_write  keys (Eq. 22) and masks of the flagged blocks, in the domain's
//               x-fastest order.
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

template <int DIM>
__device__ __forceinline__ void sb_owner(const DevParams& P, uint32_t key, int* bc) {
    const uint32_t bl = (key >> (2 * DIM)) & ((1u << P.blk_bits) - 1u);
    bc[0] = (int)(bl % (uint32_t)P.nblk[0]);
    const uint32_t r = bl / (uint32_t)P.nblk[0];
    bc[1] = DIM == 3 ? (int)(r % (uint32_t)P.nblk[1]) : (int)r;
    bc[2] = DIM == 3 ? (int)(r / (uint32_t)P.nblk[1]) : 0;
}

__global__ __launch_bounds__(64) void k_sb_init(int* bb) {
    if (threadIdx.x < 3) {
        bb[threadIdx.x] = INT_MAX;
        bb[3 + threadIdx.x] = -1;
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_bbox(DevParams P, const uint32_t* __restrict__ keys, int n,
                                                int* __restrict__ bb) {
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {-1, -1, -1};
    for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
        int bc[3];
        sb_owner<DIM>(P, keys[i], bc);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            lo[a] = min(lo[a], bc[a]);
            hi[a] = max(hi[a], bc[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        for (int m = 32; m >= 1; m >>= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], m));
            hi[a] = max(hi[a], __shfl_xor(hi[a], m));
        }
    }
    if (__lane_id() == 0) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (hi[a] >= 0) {
                atomicMin(&bb[a], lo[a]);
                atomicMax(&bb[3 + a], hi[a]);
            }
        }
    }
}

__global__ __launch_bounds__(WG) void k_sb_zero(uint64_t* __restrict__ a, long long m) {
    for (long long i = (long long)blockIdx.x * WG + threadIdx.x; i < m; i += (long long)gridDim.x * WG) a[i] = 0ull;
}

struct SbBox {
    int lo[3], ext[3];
};

template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_occ(DevParams P, const uint32_t* __restrict__ keys, int n, SbBox B,
                                               uint64_t* __restrict__ occ) {
    constexpr int NC = 1 << (2 * DIM);
    const int lane = __lane_id();
    const int i = blockIdx.x * WG + threadIdx.x;
    const bool valid = i < n;
    uint32_t idx = 0xFFFFFFFFu;
    uint64_t bit = 0ull;
    if (valid) {
        const uint32_t k = keys[i];
        int bc[3];
        sb_owner<DIM>(P, k, bc);
        idx = (uint32_t)(bc[0] - B.lo[0]) +
              (uint32_t)B.ext[0] * ((uint32_t)(bc[1] - B.lo[1]) + (uint32_t)B.ext[1] * (uint32_t)(bc[2] - B.lo[2]));
        bit = 1ull << (k & (NC - 1));
    }
    unsigned long long pending = __ballot(valid);
    while (pending) {  // one round per distinct owner block in the wave
        const int leader = __ffsll((long long)pending) - 1;
        const uint32_t own = (uint32_t)__shfl((int)idx, leader);
        const bool mine = valid && idx == own;
        const uint64_t m = wave_or64(mine ? bit : 0ull);
        if (lane == leader) atomicOr((unsigned long long*)&occ[own], (unsigned long long)m);
        pending &= ~__ballot(mine);
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_mask(SbBox B, long long m, const uint64_t* __restrict__ occ,
                                                uint64_t* __restrict__ mask, unsigned* __restrict__ flag) {
    constexpr int NB = 1 << DIM;
    for (long long t = (long long)blockIdx.x * WG + threadIdx.x; t < m; t += (long long)gridDim.x * WG) {
        const int b0 = (int)(t % B.ext[0]);
        const long long r = t / B.ext[0];
        const int b1 = (int)(r % B.ext[1]);
        const int b2 = (int)(r / B.ext[1]);
        uint64_t acc = 0ull;
#pragma unroll
        for (int d = 0; d < NB; ++d) {
            const int c0 = b0 - (d & 1), c1 = b1 - ((d >> 1) & 1), c2 = b2 - ((d >> 2) & 1);
            if (c0 < 0 || c1 < 0 || c2 < 0) continue;
            const uint64_t o = occ[(long long)c0 + (long long)B.ext[0] * (c1 + (long long)B.ext[1] * c2)];
            if (o) acc |= sb_node_mask<DIM>(o, d);
        }
        mask[t] = acc;
        flag[t] = acc != 0ull ? 1u : 0u;
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_sb_write(DevParams P, SbBox B, long long m, const uint64_t* __restrict__ mask,
                                                 const unsigned* __restrict__ phi, uint64_t* __restrict__ keys_out,
                                                 uint64_t* __restrict__ masks_out, int cap) {
    for (long long t = (long long)blockIdx.x * WG + threadIdx.x; t < m; t += (long long)gridDim.x * WG) {
        const uint64_t mk = mask[t];
        if (mk == 0ull) continue;
        const unsigned p = phi[t];
        if (p >= (unsigned)cap) continue;
        const int b0 = (int)(t % B.ext[0]);
        const long long r = t / B.ext[0];
        const int b1 = (int)(r % B.ext[1]);
        const int b2 = (int)(r / B.ext[1]);
        keys_out[p] = block_key<DIM>(P, B.lo[0] + b0, B.lo[1] + b1, B.lo[2] + b2, 0);
        masks_out[p] = mk;
    }
}

namespace {
template <typename T>
hipError_t sb_alloc(T** p, size_t count) {
    *p = nullptr;
    return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}
template <typename T>
void sb_free(T* p) {
    if (p) (void)hipFree((void*)p);
}
}  // namespace

// Synchronous: bins x into a scratch key array, reads the bounding box back,
// allocates the mask domain, and returns the number of active blocks in
// *n_blocks (the first min(*n_blocks, cap) are written).
hipError_t launch_scan_active(const DevParams& P, const float* x, int n, uint64_t* keys_out, uint64_t* masks_out,
                              int cap, int* n_blocks, hipStream_t s) {
    *n_blocks = 0;
    if (n == 0) return hipSuccess;
    uint32_t* keys = nullptr;
    int* bb = nullptr;
    uint64_t *occ = nullptr, *mask = nullptr;
    unsigned *flag = nullptr, *phi = nullptr, *partials = nullptr, *total = nullptr;
    hipError_t e = sb_alloc(&keys, (size_t)n);
    if (e == hipSuccess) e = sb_alloc(&bb, 8);
    if (e == hipSuccess) e = launch_bin(P, x, nullptr, n, keys, s);
    if (e == hipSuccess) {
        k_sb_init<<<1, 64, 0, s>>>(bb);
        const int g = std::min((n + WG - 1) / WG, 4096);
        if (P.dim == 3)
            k_sb_bbox<3><<<g, WG, 0, s>>>(P, keys, n, bb);
        else
            k_sb_bbox<2><<<g, WG, 0, s>>>(P, keys, n, bb);
        e = hipGetLastError();
    }
    int hb[6] = {0, 0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hb, bb, sizeof(hb), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    SbBox B{};
    long long m = 0;
    if (e == hipSuccess) {
        m = 1;
        for (int a = 0; a < 3; ++a) {
            if (a >= P.dim) {
                B.lo[a] = 0;
                B.ext[a] = 1;
                continue;
            }
            B.lo[a] = hb[a];
            // owners lo..hi plus the upper neighbour, inside the potential domain
            B.ext[a] = std::min(hb[3 + a] + 1, P.nblk[a] - 1) - hb[a] + 1;
            m *= B.ext[a];
        }
        if (m <= 0 || m > (long long)INT_MAX) e = hipErrorInvalidValue;
    }
    if (e == hipSuccess) e = sb_alloc(&occ, (size_t)m);
    if (e == hipSuccess) e = sb_alloc(&mask, (size_t)m);
    if (e == hipSuccess) e = sb_alloc(&flag, (size_t)m);
    if (e == hipSuccess) e = sb_alloc(&phi, (size_t)m);
    if (e == hipSuccess) e = sb_alloc(&partials, (size_t)scan_partials_size((int)m));
    if (e == hipSuccess) e = sb_alloc(&total, 1);
    if (e == hipSuccess) {
        const int gm = (int)std::min<long long>((m + WG - 1) / WG, 8192);
        k_sb_zero<<<gm, WG, 0, s>>>(occ, m);
        if (P.dim == 3) {
            k_sb_occ<3><<<(n + WG - 1) / WG, WG, 0, s>>>(P, keys, n, B, occ);
            k_sb_mask<3><<<gm, WG, 0, s>>>(B, m, occ, mask, flag);
        } else {
            k_sb_occ<2><<<(n + WG - 1) / WG, WG, 0, s>>>(P, keys, n, B, occ);
            k_sb_mask<2><<<gm, WG, 0, s>>>(B, m, occ, mask, flag);
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = scan_exclusive(flag, phi, (int)m, nullptr, partials, total, s);
        if (e == hipSuccess && cap > 0) {
            if (P.dim == 3)
                k_sb_write<3><<<gm, WG, 0, s>>>(P, B, m, mask, phi, keys_out, masks_out, cap);
            else
                k_sb_write<2><<<gm, WG, 0, s>>>(P, B, m, mask, phi, keys_out, masks_out, cap);
            e = hipGetLastError();
        }
    }
    unsigned count = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&count, total, sizeof(count), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) *n_blocks = (int)count;
    (void)hipStreamSynchronize(s);
    sb_free(keys);
    sb_free(bb);
    sb_free(occ);
    sb_free(mask);
    sb_free(flag);
    sb_free(phi);
    sb_free(partials);
    sb_free(total);
    return e;
}

}  // namespace mpmx
