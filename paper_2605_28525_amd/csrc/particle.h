// Device helpers shared by the forward and adjoint transfer kernels: the
// (4+2)^d node tile of an owner block, the per-particle frame (base node,
// t = s - b, u = 1 - t), quadratic B-spline weights, and a cyclic Jacobi
// eigen-solver for symmetric 3x3 (2x2) matrices.
#pragma once

#include "internal.h"

namespace mpmx {

constexpr int P2G_ORDER_STAGE = 1024; // sort permutation entries staged per P2G block

template <int DIM>
struct Tile {
    static constexpr int E = BLK + 2;                       // 6 nodes per axis
    static constexpr int N = DIM == 3 ? E * E * E : E * E;  // 216 / 36
    static constexpr int NB = 1 << DIM;                     // blocks touched
    static constexpr int NPB = 1 << (2 * DIM);              // nodes per block
    // Padded LDS layout of a scatter tile written by one lane per base cell:
    // node (I, J, K) at I + SY J + SZ K.  For a fixed stencil offset the 64
    // lanes of a wave (cells i, j, k in 0..3) then hit 64 distinct banks
    // modulo 64, and 32 distinct banks within each half-wave modulo 32.
    static constexpr int SY = DIM == 3 ? 12 : E;
    static constexpr int SZ = DIM == 3 ? 80 : 0;
    static constexpr int NP = DIM == 3 ? E * SZ : E * E;   // padded size
    static __device__ __forceinline__ int pad(int I, int J, int K) { return I + SY * J + SZ * K; }

    // Layout of a tile in the HBM tile store, grouped by the block each node
    // belongs to: part d (d = dx + 2 dy + 4 dz) holds the nodes of the upper
    // neighbour d, local indices 0..3 along an axis where d's bit is clear and
    // 4..5 (spilled) where it is set, x fastest.  The gather of a block then
    // reads each part it needs whole and contiguous.  Part sizes are 4 or 2
    // per axis, so the index arithmetic is shifts and masks; the part offsets
    // are packed 8 bits each (3D: 0, 64, 96, 128, 144, 176, 192, 208; 2D: 0,
    // 16, 24, 32).
    static constexpr uint64_t PART_OFFS = DIM == 3 ? 0xD0C0B09080604000ull : 0x20181000ull;
    static __device__ __forceinline__ int part_off(int d) { return (int)((PART_OFFS >> (8 * d)) & 255u); }
    static __device__ __forceinline__ int part_lx(int d, int a) { return ((d >> a) & 1) ? 1 : 2; }  // log2 extent
    // store position of node (I, J, K) of the 6^d tile
    static __device__ __forceinline__ int store_index(int I, int J, int K) {
        const int d = (I >> 2) | ((J >> 2) << 1) | (DIM == 3 ? ((K >> 2) << 2) : 0);
        const int lx = part_lx(d, 0), ly = part_lx(d, 1);
        return part_off(d) + (I & 3) + (((J & 3) + ((K & 3) << ly)) << lx);
    }
    // node (I, J, K) of the tile at store position t
    static __device__ __forceinline__ void store_node(int t, int* I, int* J, int* K) {
        int d = 0;
#pragma unroll
        for (int q = 1; q < NB; ++q) d += t >= part_off(q) ? 1 : 0;
        const int i = t - part_off(d), lx = part_lx(d, 0), ly = part_lx(d, 1);
        *I = (i & ((1 << lx) - 1)) + ((d & 1) << 2);
        *J = ((i >> lx) & ((1 << ly) - 1)) + (((d >> 1) & 1) << 2);
        *K = DIM == 3 ? (i >> (lx + ly)) + (((d >> 2) & 1) << 2) : 0;
    }
};

// Per-axis base offset within the owner block, t and u, for one particle.
template <int DIM>
__device__ __forceinline__ void particle_frame(const DevParams& P, const float* xp, const int* org, int* lb, float* t,
                                               float* u) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double s = index_arg(xp[a], P.inv_dx);
        double f = floor(s);
        f = fmin(fmax(f, 0.0), (double)(P.cells[a] - 2));  // keeps indices in range for flagged particles
        const double td = s - f;
        t[a] = fminf(fmaxf((float)td, 0.f), 1.f);
        u[a] = fminf(fmaxf((float)(1.0 - td), 0.f), 1.f);
        lb[a] = min(max((int)f - org[a], 0), BLK - 1);
    }
}

// The same offsets for a particle whose base node is known (P2G's lanes own
// one base cell each, the sort key's cell, which the binning took from the
// same float64 floor and clamp): t = s - base without recomputing the floor.
template <int DIM>
__device__ __forceinline__ void particle_frame_at(const DevParams& P, const float* xp, const double* base, float* t,
                                                  float* u) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double td = index_arg(xp[a], P.inv_dx) - base[a];
        t[a] = fminf(fmaxf((float)td, 0.f), 1.f);
        u[a] = fminf(fmaxf((float)(1.0 - td), 0.f), 1.f);
    }
}

template <int DIM>
__device__ __forceinline__ void bspline(const float* t, const float* u, float inv_dx, float (*w)[3], float (*dw)[3]) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        w[a][0] = 0.5f * u[a] * u[a];
        w[a][1] = 0.5f + t[a] * u[a];
        w[a][2] = 0.5f * t[a] * t[a];
        dw[a][0] = -u[a] * inv_dx;
        dw[a][1] = (u[a] - t[a]) * inv_dx;
        dw[a][2] = t[a] * inv_dx;
    }
}


// second derivative (in xi) of the 1D quadratic B-spline at the three stencil
// nodes: +1, -2, +1 (times inv_dx^2)
__device__ __forceinline__ void bspline_dd(float inv_dx2, float* ddw) {
    ddw[0] = inv_dx2;
    ddw[1] = -2.f * inv_dx2;
    ddw[2] = inv_dx2;
}

// ---------------------------------------------------------------------------
// constitutive update: Hencky strain from the eigen-decomposition of
// F F^T - I (cyclic Jacobi), Drucker-Prager return map, Kirchhoff stress.
template <int DIM>
__device__ __forceinline__ void jacobi_sym(float (*A)[3], float (*U)[3]) {
    constexpr int SWEEPS = DIM == 3 ? 4 : 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) U[a][b] = a == b ? 1.f : 0.f;
#pragma unroll
    for (int sw = 0; sw < SWEEPS; ++sw) {
#pragma unroll
        for (int pr = 0; pr < (DIM == 3 ? 3 : 1); ++pr) {
            const int p = pr == 2 ? 1 : 0;
            const int q = pr == 0 ? 1 : 2;
            const float apq = A[p][q];
            if (apq != 0.f) {
                // rotation angle with hardware reciprocal / square root (about
                // 1 ulp): any rotation that zeroes a_pq to that accuracy and
                // keeps c^2 + s^2 = 1 to float precision serves the iteration
                float th = (A[q][q] - A[p][p]) * (0.5f * __builtin_amdgcn_rcpf(apq));
                th = fminf(fmaxf(th, -1e18f), 1e18f);
                const float t = copysignf(__builtin_amdgcn_rcpf(fabsf(th) + __builtin_amdgcn_sqrtf(th * th + 1.f)), th);
                const float c = __builtin_amdgcn_rsqf(t * t + 1.f);
                const float sn = t * c;
                A[p][p] -= t * apq;
                A[q][q] += t * apq;
                A[p][q] = A[q][p] = 0.f;
                if (DIM == 3) {
                    const int r = 3 - p - q;
                    const float arp = A[r][p], arq = A[r][q];
                    A[r][p] = A[p][r] = c * arp - sn * arq;
                    A[r][q] = A[q][r] = sn * arp + c * arq;
                }
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    const float urp = U[r][p], urq = U[r][q];
                    U[r][p] = c * urp - sn * urq;
                    U[r][q] = sn * urp + c * urq;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Placement of a block's particles in the G2P output.
//
// The sort lists a block's particles cell by cell.  The next step's P2G gives
// each base cell of a block to one lane and walks that cell's particles, so
// cell-major storage would make its loads stride by the particles per cell
// (a few cache lines per wave instruction, each used in part).  G2P therefore
// stores a block's particles rank-major: the first particle of every non-empty
// cell (cells in order), then every second particle, and so on for ranks below
// IL_ROUNDS; particles of higher rank follow cell by cell.  The radix sort is
// stable, so a cell that keeps its particles hands them back to its P2G lane
// in the same rank order, and consecutive lanes load consecutive addresses;
// the incremental re-sort may permute a cell's particles among its ranks,
// which keeps a wave's loads inside the block's range of the set.
constexpr int IL_ROUNDS = 32;

template <int DIM>
struct Interleave {
    static constexpr int NC = 1 << (2 * DIM);
    unsigned long long mask[IL_ROUNDS];  // cells holding more than j particles
    int R[IL_ROUNDS + 1];                // particles of rank < j
    int cs[NC], ce[NC];                  // cell ranges in sorted order
    int op[NC];                          // rank >= IL_ROUNDS particles of the cells before
    int st;                              // first sorted position of the block
};

constexpr int IL_BATCH = 8;  // 64-key chunks of a segment whose loads are issued together

// Lanes whose value v (its low BITS bits) equals this lane's, among lanes with
// `valid` set.  Every lane of the wave must call it.
template <int BITS>
__device__ __forceinline__ unsigned long long lanes_matching(unsigned v, bool valid) {
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const bool bit = (v >> b) & 1u;
        const unsigned long long bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Workgroup-cooperative set-up for the owner segment [st, en) (every thread
// calls it; blockDim.x is a multiple of 64; ends with a barrier).  The keys of
// the segment are sorted by base cell, so a cell's range starts after the
// particles of all lower cells: the cells are counted (keys loaded in batches,
// one wave-wide match per 64 keys, one LDS add per distinct cell) and the
// ranges follow from an exclusive scan of the counts.  Optionally the first
// `stage_max` entries of another per-particle array (`stage_src[st ..]`) are
// copied to LDS (`stage_dst`) by the same batched loads.  With `cell_first`
// (the first sorted position of each base cell, which an incremental re-sort
// leaves per block) the counts are taken from it and no key is read.
template <int DIM>
__device__ void interleave_setup(Interleave<DIM>& L, const uint32_t* __restrict__ skeys, int st, int en,
                                 const uint32_t* __restrict__ stage_src = nullptr, uint32_t* stage_dst = nullptr,
                                 int stage_max = 0, const uint32_t* __restrict__ cell_first = nullptr) {
    constexpr int NC = Interleave<DIM>::NC;
    const int stage_end = stage_dst ? min(en, st + stage_max) : st;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    if (cell_first) {
        // the cell table and the first batch of the staged array are loaded
        // together, then further batches (IL_BATCH loads in flight per lane)
        int first = 0, next = 0;
        if (threadIdx.x < NC) {
            first = (int)cell_first[threadIdx.x];
            next = threadIdx.x + 1 < NC ? (int)cell_first[threadIdx.x + 1] : en;
        }
        for (int i0 = st + wave * 64 * IL_BATCH; i0 < stage_end; i0 += n_waves * 64 * IL_BATCH) {
            uint32_t v[IL_BATCH];
#pragma unroll
            for (int r = 0; r < IL_BATCH; ++r) {
                const int i = i0 + r * 64 + lane;
                v[r] = i < stage_end ? stage_src[i] : 0u;
            }
#pragma unroll
            for (int r = 0; r < IL_BATCH; ++r) {
                const int i = i0 + r * 64 + lane;
                if (i < stage_end) stage_dst[i - st] = v[r];
            }
        }
        if (threadIdx.x < NC) L.ce[threadIdx.x] = next - first;
        if (threadIdx.x == 0) L.st = st;
    } else {
        for (int c = threadIdx.x; c < NC; c += blockDim.x) L.ce[c] = 0;  // per-cell counts first
        if (threadIdx.x == 0) L.st = st;
    }
    __syncthreads();
    for (int i0 = st + wave * 64 * IL_BATCH; !cell_first && i0 < en; i0 += n_waves * 64 * IL_BATCH) {
        uint32_t k[IL_BATCH], v[IL_BATCH];
#pragma unroll
        for (int r = 0; r < IL_BATCH; ++r) {
            const int i = i0 + r * 64 + lane;
            k[r] = i < en ? skeys[i] : 0u;
            v[r] = i < stage_end ? stage_src[i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < IL_BATCH; ++r) {
            const int i = i0 + r * 64 + lane;
            if (i < stage_end) stage_dst[i - st] = v[r];
        }
#pragma unroll
        for (int r = 0; r < IL_BATCH; ++r) {
            if (i0 + r * 64 >= en) break;  // uniform
            const bool valid = i0 + r * 64 + lane < en;
            const uint32_t c = k[r] & (NC - 1);
            const unsigned long long m = lanes_matching<2 * DIM>(c, valid);
            if (valid && (m & lt) == 0ull) atomicAdd(&L.ce[c], __popcll(m));
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int cnt = lane < NC ? L.ce[lane] : 0;
        const int first = st + (int)wave_incl_scan((unsigned)cnt) - cnt;
        if (lane < NC) {
            L.cs[lane] = first;
            L.ce[lane] = first + cnt;
        }
        const int ovf = max(cnt - IL_ROUNDS, 0);
        const int inc = (int)wave_incl_scan((unsigned)ovf);
        if (lane < NC) L.op[lane] = inc - ovf;
        // ranks at or beyond the largest count are never looked up, and
        // R[IL_ROUNDS] only when some cell overflows (then no early exit)
        int acc = 0;
        for (int j = 0; j < IL_ROUNDS; ++j) {
            const unsigned long long m = __ballot(cnt > j);
            if (m == 0ull) break;
            if (lane == 0) {
                L.mask[j] = m;
                L.R[j] = acc;
            }
            acc += __popcll(m);
        }
        if (lane == 0) L.R[IL_ROUNDS] = acc;
    }
    __syncthreads();
}

// Output position of the particle of rank j in base cell c.
template <int DIM>
__device__ __forceinline__ int interleave_pos_cj(const Interleave<DIM>& L, int c, int j) {
    if (j < IL_ROUNDS) return L.st + L.R[j] + __popcll(L.mask[j] & ((1ull << c) - 1ull));
    return L.st + L.R[IL_ROUNDS] + L.op[c] + (j - IL_ROUNDS);
}

// Output position of the particle at sorted position i (sort key `key`).
template <int DIM>
__device__ __forceinline__ int interleave_pos(const Interleave<DIM>& L, int i, uint32_t key) {
    const int c = (int)(key & (Interleave<DIM>::NC - 1));
    return interleave_pos_cj<DIM>(L, c, i - L.cs[c]);
}

}  // namespace mpmx
