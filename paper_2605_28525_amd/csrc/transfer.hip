// P2G, grid update and G2P on the compact block storage (Methods 3.1,
// Eqs. 6-17), with quadratic B-spline weights.
//
// Work is organised by owner block: a work item is a run of at most CHUNK
// particles (contiguous in sorted order) whose base nodes lie in one block.
// Their 3^d stencils cover a (4+2)^d node tile anchored at that block's origin,
// which spans the block and its upper neighbours (2^d blocks).
//
//   P2G: one wave per owner block accumulates the mass and momentum of the
//        block's particles into an LDS tile and stores the tile to its own slot
//        in HBM; a second pass gives each node the sum of the (at most 2^d)
//        tiles that cover it (inside mpm_step it also applies the grid
//        update).  No global atomics, and node sums do not depend on
//        scheduling.  (The dense baseline flushes its tiles with global float
//        atomics instead, at most 4 per non-zero tile node.)
//   G2P: a workgroup stages the tile's updated nodal velocities in LDS, then each
//        thread gathers its 3^d nodes, updates the particle and writes it to its
//        output position (structure-of-arrays, coalesced; the layout P2G
//        recorded for the next P2G's lanes).
//
// Weights: with s = x/dx - 1/2 in float64, b = floor(s), t = s - b and u = 1 - t
// (both rounded once to float32, so small weights keep their relative accuracy)
//   w = (u^2/2, 1/2 + t u, t^2/2),  dw/dxi = (-u, u - t, t).
#include <stdlib.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "particle.h"

namespace mpmx {

// ---------------------------------------------------------------------------
// P2G, one wave64 per owner block and one lane per base cell.
//
// Inside a block the sorted order groups particles by the local index of their
// base node (the low 2d bits of the sort key), and every particle with the same
// base node scatters to the same 3^d nodes.  A lane therefore sums its cell's
// particles into 27 x 4 registers and adds them to the LDS tile once per cell,
// not once per particle; the tile then goes to HBM as above.
template <int DIM>
__global__ __launch_bounds__(64) void k_p2g_cell(DevParams P, const float* __restrict__ x,
                                                 const float* __restrict__ v, const float* __restrict__ C,
                                                 const float* __restrict__ tau, int n,
                                                 const uint32_t* __restrict__ order,
                                                 const uint32_t* __restrict__ skeys, uint32_t* __restrict__ osrc) {
    using T = Tile<DIM>;
    constexpr int NS = DIM == 3 ? 6 : 3;
    constexpr int NC = T::NPB;  // base cells per block
    constexpr int NK = DIM == 3 ? 27 : 9;
    __shared__ float tile[4][T::NP];
    __shared__ Interleave<DIM> il;  // cell ranges and the G2P output layout of the block
    __shared__ uint32_t ord[P2G_ORDER_STAGE];
    __shared__ int nbr[T::NB];  // compact indices of the blocks the tile covers
    const int lane = threadIdx.x;
    const int nb = min(P.ctr->nb, P.block_cap);
    const float dx = P.dxf, inv_dx = P.inv_dxf;
    // The count, first sorted position and key of the next block are loaded
    // while the current one is processed (a dense grid has no key table: its
    // key is the linear block index).
    int cnt_n = 0, st_n = 0, ent_n = -1;
    uint64_t key_n = 0;
    auto fetch_meta = [&](int bb) {
        if (bb < nb) {
            // the same in every lane; hidden so that the values stay in vector
            // registers and nothing waits for them before they are used
            asm volatile("" : "+v"(bb));
            cnt_n = P.b_count[bb];
            st_n = P.b_start[bb];
            key_n = P.dense ? (uint64_t)bb : P.b_keys[bb];
            ent_n = P.b_entry ? P.b_entry[bb] : -1;
        }
    };
    fetch_meta(blockIdx.x);
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int cnt = cnt_n, st = st_n, ent = ent_n;
        const uint64_t key = key_n;
        fetch_meta(b + gridDim.x);
        if (cnt <= 0) continue;
        const int en = st + cnt;
        const int nbv = lane < T::NB ? P.b_nbr[(size_t)b * T::NB + lane] : -1;
        for (int t = lane; t < 4 * T::NP; t += 64) (&tile[0][0])[t] = 0.f;
        int bc[3], inst = 0;
        if (P.dense)
            linear_to_block<DIM>(P, (uint32_t)key, bc);
        else
            unblock_key<DIM>(P, key, bc, &inst);
        const InstMat mat = material(P, inst);
        // the lanes accumulate per unit particle mass (m_p is uniform in a
        // block); the merge into the tile scales by m_p
        const float mp = mat.p_mass;
        const float dtv = mat.dt * mat.p_vol0 / mp;
        const int org[3] = {bc[0] * BLK, bc[1] * BLK, bc[2] * BLK};
        // cell ranges of the block and its G2P output layout (rank-major over
        // the base cells), with the block's permutation staged in LDS by the
        // same loads; each lane records where G2P will store its cell's
        // particles as it visits them (osrc)
        // after an incremental re-sort the block's cell ranges are its entry's
        // row of first positions; otherwise they are counted from the keys
        interleave_setup<DIM>(il, skeys, st, en, order, ord, P2G_ORDER_STAGE,
                              ent >= 0 ? P.rs_off + (size_t)ent * NC : nullptr);
        if (lane < T::NB) nbr[lane] = nbv;
        float acc[NK][4];
#pragma unroll
        for (int k = 0; k < NK; ++k) acc[k][0] = acc[k][1] = acc[k][2] = acc[k][3] = 0.f;
        int lb[3] = {lane & 3, (lane >> 2) & 3, DIM == 3 ? (lane >> 4) & 3 : 0};
        const double base[3] = {(double)(org[0] + lb[0]), (double)(org[1] + lb[1]), (double)(org[2] + lb[2])};
        const int c0 = lane < NC ? il.cs[lane] : 0, c1 = lane < NC ? il.ce[lane] : 0;
        const bool has = c1 > c0;
        // The walk over the lane's particles, with the source index read from
        // the LDS copy of the permutation when the block fits it (the usual
        // case) and from HBM otherwise: one uniform choice per block, so each
        // variant uses one kind of load and the loads of the next particle stay
        // in flight across the accumulation of the current one.
        auto walk = [&](auto staged) {
            constexpr bool STAGED = decltype(staged)::value;
            auto src = [&](int i) -> uint32_t {
                if constexpr (STAGED)
                    return ord[i - st];
                else
                    return order[i];
            };
            // Software pipeline: the loads of particle i+1 are issued before the
            // 3^d-node accumulation of particle i and consumed one iteration
            // later.  They are issued on every iteration (the last one reloads
            // its own particle), so the number of loads in flight never depends
            // on the path taken and the wait for them lands after the
            // accumulation, not before it.
            // Two register sets take turns (A holds particle i while the loads
            // of particle i + 1 land in B, and the other way round), so no
            // copies move a prefetched particle into place.
            float xa[3], va[3], Ca[9], ta[6], xb[3], vb[3], Cb[9], tb[6];
            auto load_into = [&](float* xs, float* vs, float* Cs, float* ts, uint32_t q) {
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    xs[a] = x[(size_t)a * n + q];
                    vs[a] = v[(size_t)a * n + q];
                }
#pragma unroll
                for (int k = 0; k < DIM * DIM; ++k) Cs[k] = C[(size_t)k * n + q];
#pragma unroll
                for (int k = 0; k < NS; ++k) ts[k] = tau[(size_t)k * n + q];
            };
            auto process = [&](const float* xp, const float* vp, const float* Cp, const float* tp, uint32_t qp,
                               int i) {
                float t[3] = {0, 0, 0}, u[3] = {1, 1, 1};
                particle_frame_at<DIM>(P, xp, base, t, u);
                float wt[3][3], dw[3][3];
                bspline<DIM>(t, u, inv_dx, wt, dw);
                // per unit mass: m v -> v, A = m C -> C, G = dt V0 tau / m
                float mv[3], A[3][3], G[3][3];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    mv[a] = vp[a];
#pragma unroll
                    for (int bb = 0; bb < DIM; ++bb) A[a][bb] = Cp[a * DIM + bb];
                }
                if (DIM == 3) {
                    G[0][0] = dtv * tp[0];
                    G[1][1] = dtv * tp[1];
                    G[2][2] = dtv * tp[2];
                    G[0][1] = G[1][0] = dtv * tp[3];
                    G[1][2] = G[2][1] = dtv * tp[4];
                    G[0][2] = G[2][0] = dtv * tp[5];
                } else {
                    G[0][0] = dtv * tp[0];
                    G[1][1] = dtv * tp[1];
                    G[0][1] = G[1][0] = dtv * tp[2];
                }
                float dxn[3][3];
#pragma unroll
                for (int a = 0; a < DIM; ++a)
#pragma unroll
                    for (int k = 0; k < 3; ++k) dxn[a][k] = ((float)k - 0.5f - t[a]) * dx;
                // Tensor-product factorisation.  The momentum contribution of the
                // particle to node (kx, ky, kz) is
                //   w_x w_y w_z (m v + A dx) - G grad w,   A = m_p C_p, G = dt V0 tau_p,
                // which regroups as w_x b + (w_z w_y) h with
                //   b(ky, kz) = w_z Y(ky) + w_y Z(kz),
                //   Y(ky) = w_y (m v + A_1 dx_y) - G_1 dw_y,  Z(kz) = w_z dx_z A_2 - G_2 dw_z,
                //   h(kx) = (w_x dx_x) A_0 - dw_x G_0
                // (columns A_j, G_j): two fused multiply-adds per node and momentum
                // component, one for the mass w_x (w_z w_y).
                float h[3][3], wd[3];
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    wd[kx] = wt[0][kx] * dxn[0][kx];
#pragma unroll
                    for (int q = 0; q < DIM; ++q) h[kx][q] = wd[kx] * A[q][0] - dw[0][kx] * G[q][0];
                }
                if (DIM == 3) {
                    float Z[3][3];
#pragma unroll
                    for (int kz = 0; kz < 3; ++kz) {
                        const float wzd = wt[2][kz] * dxn[2][kz];
#pragma unroll
                        for (int q = 0; q < 3; ++q) Z[kz][q] = wzd * A[q][2] - G[q][2] * dw[2][kz];
                    }
#pragma unroll
                    for (int ky = 0; ky < 3; ++ky) {
                        const float wy = wt[1][ky];
                        float Y[3];
#pragma unroll
                        for (int q = 0; q < 3; ++q) Y[q] = wy * (mv[q] + A[q][1] * dxn[1][ky]) - G[q][1] * dw[1][ky];
#pragma unroll
                        for (int kz = 0; kz < 3; ++kz) {
                            const float wz = wt[2][kz];
                            const float wzy = wz * wy;
                            float be[3];
#pragma unroll
                            for (int q = 0; q < 3; ++q) be[q] = wz * Y[q] + wy * Z[kz][q];

#pragma unroll
                            for (int kx = 0; kx < 3; ++kx) {
                                const int k = kx + 3 * (ky + 3 * kz);
                                const float wx = wt[0][kx];
#pragma unroll
                                for (int q = 0; q < 3; ++q) acc[k][q] = fmaf(wx, be[q], fmaf(wzy, h[kx][q], acc[k][q]));
                                acc[k][3] = fmaf(wx, wzy, acc[k][3]);
                            }
                        }
                    }
                } else {
                    // 2D: the same with no z axis (w_z = 1, Z = 0)
#pragma unroll
                    for (int ky = 0; ky < 3; ++ky) {
                        const float wy = wt[1][ky];
                        float Y[2];
#pragma unroll
                        for (int q = 0; q < 2; ++q) Y[q] = wy * (mv[q] + A[q][1] * dxn[1][ky]) - G[q][1] * dw[1][ky];
#pragma unroll
                        for (int kx = 0; kx < 3; ++kx) {
                            const int k = kx + 3 * ky;
                            const float wx = wt[0][kx];
#pragma unroll
                            for (int q = 0; q < 2; ++q) acc[k][q] = fmaf(wx, Y[q], fmaf(wy, h[kx][q], acc[k][q]));
                            acc[k][3] = fmaf(wx, wy, acc[k][3]);
                        }
                    }
                }
                // the G2P output position of this particle records its source
                osrc[interleave_pos_cj<DIM>(il, lane, i - c0)] = qp;
            };
            uint32_t qa = 0, qb = 0;
            if (has) {
                qa = src(c0);
                load_into(xa, va, Ca, ta, qa);
            }
            for (int i = c0; i < c1; i += 2) {
                qb = src(min(i + 1, c1 - 1));
                load_into(xb, vb, Cb, tb, qb);
                process(xa, va, Ca, ta, qa, i);
                qa = src(min(i + 2, c1 - 1));
                load_into(xa, va, Ca, ta, qa);
                if (i + 1 < c1) process(xb, vb, Cb, tb, qb, i + 1);
            }
        };
        if (cnt <= P2G_ORDER_STAGE)
            walk(std::true_type{});
        else
            walk(std::false_type{});
        // Merge the cell sums (per unit mass, scaled by m_p here) into the
        // tile.  For a fixed offset k, distinct
        // cells address distinct nodes, so each offset is a conflict-free
        // read-add-write; the barrier orders successive offsets, which may hit
        // the same node from neighbouring cells.
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int kx = k % 3, ky = (k / 3) % 3, kz = DIM == 3 ? k / 9 : 0;
            const int idx = T::pad(lb[0] + kx, lb[1] + ky, DIM == 3 ? lb[2] + kz : 0);
            if (has) {
                tile[0][idx] = fmaf(mp, acc[k][0], tile[0][idx]);
                tile[1][idx] = fmaf(mp, acc[k][1], tile[1][idx]);
                if (DIM == 3) tile[2][idx] = fmaf(mp, acc[k][2], tile[2][idx]);
                tile[3][idx] = fmaf(mp, acc[k][3], tile[3][idx]);
            }
            __syncthreads();
        }
        __syncthreads();
        if (!P.dense) {
            // sparse grid: the whole tile goes to the block's slot of the tile
            // store (coalesced plain stores); k_p2g_gather sums the tiles that
            // cover each node.  A fixed number of stores per lane (the last
            // node repeated by the lanes past the end) keeps the count of
            // memory operations in flight static, so the wait for the next
            // block's metadata does not also wait for these stores.
#pragma unroll
            for (int r = 0; r < (T::N + 63) / 64; ++r) {
                const int t = min(lane + 64 * r, T::N - 1);
                int I, J, K;
                T::store_node(t, &I, &J, &K);
                const int tp = T::pad(I, J, K);
                P.tiles[(size_t)b * T::N + t] =
                    make_float4(tile[0][tp], tile[1][tp], DIM == 3 ? tile[2][tp] : 0.f, tile[3][tp]);
            }
            __syncthreads();
            continue;
        }
        for (int t = lane; t < T::N; t += 64) {
            const int I = t % T::E;
            const int J = (t / T::E) % T::E;
            const int K = DIM == 3 ? t / (T::E * T::E) : 0;
            const int tp = T::pad(I, J, K);
            const float m = tile[3][tp], p0 = tile[0][tp], p1 = tile[1][tp], p2 = DIM == 3 ? tile[2][tp] : 0.f;
            if (m != 0.f || p0 != 0.f || p1 != 0.f || p2 != 0.f) {
                const int d = (I >> 2) | ((J >> 2) << 1) | ((K >> 2) << 2);
                const int phi = nbr[d];
                if (phi >= 0) {
                    const int l = (I & 3) + BLK * ((J & 3) + BLK * (K & 3));
                    float* g = reinterpret_cast<float*>(&P.grid[(size_t)phi * T::NPB + l]);
                    atomicAdd(g + 0, p0);
                    atomicAdd(g + 1, p1);
                    if (DIM == 3) atomicAdd(g + 2, p2);
                    atomicAdd(g + 3, m);
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// grid update with boundary conditions

// Terrain heights a node's condition reads: at (i, j) and its four axis
// neighbours (clamped to the heightmap), as h[0] (i, j), h[1] (i-1), h[2]
// (i+1), h[3] (j-1), h[4] (j+1).  Loaded unconditionally, so that a caller
// can issue them long before the node's velocity is known.
__device__ __forceinline__ void terrain_heights(const DevParams& P, int i, int j, float* h) {
    const int nx = P.cells[0] + 1, ny = P.cells[1] + 1;
    const int ic = min(max(i, 0), nx - 1), jc = min(max(j, 0), ny - 1);
    const int il = max(ic - 1, 0), ih = min(ic + 1, nx - 1);
    const int jl = max(jc - 1, 0), jh = min(jc + 1, ny - 1);
    const float* H = P.heightmap;
    h[0] = H[(size_t)ic * ny + jc];
    h[1] = H[(size_t)il * ny + jc];
    h[2] = H[(size_t)ih * ny + jc];
    h[3] = H[(size_t)ic * ny + jl];
    h[4] = H[(size_t)ic * ny + jh];
}

// Coulomb friction against the terrain level set (the node below the surface
// height h[0], normal from central differences of the heights).
__device__ __forceinline__ void terrain_bc(const DevParams& P, int i, int j, int k, const float* h, float* vel) {
    const int nx = P.cells[0] + 1, ny = P.cells[1] + 1;
    if (!((double)k * P.dx <= (double)h[0])) return;
    const int il = max(i - 1, 0), ih = min(i + 1, nx - 1);
    const int jl = max(j - 1, 0), jh = min(j + 1, ny - 1);
    const float hx = (h[2] - h[1]) / ((float)(ih - il) * P.dxf);
    const float hy = (h[4] - h[3]) / ((float)(jh - jl) * P.dxf);
    const float inv = 1.f / sqrtf(hx * hx + hy * hy + 1.f);
    const float n0 = -hx * inv, n1 = -hy * inv, n2 = inv;
    const float vn = vel[0] * n0 + vel[1] * n1 + vel[2] * n2;
    if (vn >= 0.f) return;
    const float t0 = vel[0] - vn * n0, t1 = vel[1] - vn * n1, t2 = vel[2] - vn * n2;
    const float tn = sqrtf(t0 * t0 + t1 * t1 + t2 * t2);
    if (tn <= -P.mu_terrain * vn) {
        vel[0] = vel[1] = vel[2] = 0.f;
    } else {
        const float sc = 1.f + P.mu_terrain * vn / tn;
        vel[0] = t0 * sc;
        vel[1] = t1 * sc;
        vel[2] = t2 * sc;
    }
}

// Eqs. 8-12 for one node: v = p / m + dt g, then the terrain and wall
// conditions; records the pre-condition velocity u where an adjoint context
// keeps it.  gv = (p, m); h: the node's terrain heights (3D with terrain).
template <int DIM>
__device__ __forceinline__ float4 node_update(const DevParams& P, size_t s, const int* node, float dtn, float4 gv,
                                              const float* h) {
    const float m = gv.w;
    float vel[3] = {0.f, 0.f, 0.f};
    if (m > 0.f) {
        vel[0] = gv.x / m + dtn * P.g[0];
        vel[1] = gv.y / m + dtn * P.g[1];
        if (DIM == 3) vel[2] = gv.z / m + dtn * P.g[2];
        if (P.grid_u) P.grid_u[s] = make_float4(vel[0], vel[1], vel[2], m);
        if (DIM == 3 && P.has_terrain && node[0] <= P.cells[0] && node[1] <= P.cells[1])
            terrain_bc(P, node[0], node[1], node[2], h, vel);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool on = side == 0 ? node[a] < P.bound : node[a] > P.cells[a] - P.bound;
                if (!on) continue;
                const int kind = P.bc[a][side];
                if (kind == MPM_BC_STICKY) {
                    vel[0] = vel[1] = vel[2] = 0.f;
                } else if (kind == MPM_BC_SLIP) {
                    vel[a] = 0.f;
                } else if (kind == MPM_BC_SEPARATE) {
                    vel[a] = side == 0 ? fmaxf(vel[a], 0.f) : fminf(vel[a], 0.f);
                }
            }
        }
    } else if (P.grid_u) {
        P.grid_u[s] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return make_float4(vel[0], vel[1], vel[2], m);
}

// What the update of node `lane` of compact block b needs besides the node's
// mass and momentum: its grid coordinates, the block instance's time step and
// the terrain heights around it (all issued at once; the heights unconditionally).
template <int DIM>
__device__ __forceinline__ void node_update_inputs(const DevParams& P, int b, int lane, int* node, float* dtn,
                                                   float* h) {
    int bc[3], inst;
    block_coords<DIM>(P, b, bc, &inst);
    *dtn = P.n_inst > 1 ? P.inst[inst].dt : P.dt;
    node[0] = bc[0] * BLK + (lane & 3);
    node[1] = bc[1] * BLK + ((lane >> 2) & 3);
    node[2] = DIM == 3 ? bc[2] * BLK + ((lane >> 4) & 3) : 0;
    if (DIM == 3 && P.has_terrain) terrain_heights(P, node[0], node[1], h);
}

// P2G, second pass on a sparse grid: node n of block b receives the tile
// entries that cover it, from b's own tile and from the tiles of the lower
// neighbours b - d (d in {0,1}^d) whose 6-node tiles reach n (local index < 2
// on every axis where d is set).  One wave per block, one lane per node; each
// tile node is read once in total, and the sum is written (no atomics).
// UPDATE (inside mpm_step): the node's grid update follows at once and the
// velocity is written instead of the momentum; the block key, time step and
// terrain heights the update needs are loaded beside the tile reads, so the
// wave's chain of dependent loads is no longer than the gather's own.
template <int DIM, bool UPDATE>
__global__ __launch_bounds__(WG) void k_p2g_gather(DevParams P) {
    using T = Tile<DIM>;
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int nb = min(P.ctr->nb, P.block_cap);
    const int I = lane & 3, J = (lane >> 2) & 3, K = DIM == 3 ? (lane >> 4) & 3 : 0;
    for (int b = blockIdx.x * (WG / 64) + w; b < nb; b += gridDim.x * (WG / 64)) {
        int src[T::NB];  // the block and its lower neighbours that own particles, else -1
#pragma unroll
        for (int d = 0; d < T::NB; ++d) src[d] = P.b_lo[(size_t)b * T::NB + d];
        int node[3] = {0, 0, 0};
        float dtn = P.dt, h[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        if (UPDATE) node_update_inputs<DIM>(P, b, lane, node, &dtn, h);
        float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int d = 0; d < T::NB; ++d) {
            const int dx = d & 1, dy = (d >> 1) & 1, dz = (d >> 2) & 1;
            const bool reach = (!dx || I < 2) && (!dy || J < 2) && (DIM == 2 || !dz || K < 2);
            if (src[d] >= 0 && reach && lane < T::NPB) {
                const int t = T::store_index(I + 4 * dx, J + 4 * dy, K + 4 * dz);
                const float4 g = P.tiles[(size_t)src[d] * T::N + t];
                sum.x += g.x;
                sum.y += g.y;
                sum.z += g.z;
                sum.w += g.w;
            }
        }
        if (lane < T::NPB) {
            const size_t s = (size_t)b * T::NPB + lane;
            P.grid[s] = UPDATE ? node_update<DIM>(P, s, node, dtn, sum, h) : sum;
        }
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_grid_update(DevParams P, long long n_nodes_host) {
    constexpr int NPB = Tile<DIM>::NPB;
    const long long n_nodes = n_nodes_host >= 0 ? n_nodes_host : (long long)P.ctr->nb * NPB;
    for (long long s = (long long)blockIdx.x * WG + threadIdx.x; s < n_nodes; s += (long long)gridDim.x * WG) {
        const float4 gv = P.grid[s];
        float4 out = make_float4(0.f, 0.f, 0.f, gv.w);
        if (gv.w > 0.f || P.grid_u) {
            const int b = (int)(s / NPB), l = (int)(s % NPB);
            int bc[3], inst;
            block_coords<DIM>(P, b, bc, &inst);
            const float dtn = P.n_inst > 1 ? P.inst[inst].dt : P.dt;
            const int node[3] = {bc[0] * BLK + (l & 3), bc[1] * BLK + ((l >> 2) & 3),
                                 DIM == 3 ? bc[2] * BLK + (l >> 4) : 0};
            float h[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            if (DIM == 3 && P.has_terrain && gv.w > 0.f) terrain_heights(P, node[0], node[1], h);
            out = node_update<DIM>(P, (size_t)s, node, dtn, gv, h);
        }
        P.grid[s] = out;
    }
}

// C = A B for symmetric A, B that commute (polynomials in one matrix), so C
// is symmetric: upper triangle computed, mirrored.
template <int DIM>
__device__ __forceinline__ void sym_mul(const float (*A)[3], const float (*B)[3], float (*C)[3]) {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = a; b < DIM; ++b) {
            float s2 = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s2 += A[a][c] * B[c][b];
            C[a][b] = s2;
            C[b][a] = s2;
        }
}

constexpr float SERIES_MAX_NORM2 = 1.f / 64.f;  // |F F^T - I|_F^2 limit of the series path

// Eigen path: Jacobi on M = F F^T - I, Hencky strain and return map on the
// principal values, tau = U diag(sigma) U^T, F_new = U diag(exp(eps' - eps)) U^T F.
template <int DIM>
__device__ __forceinline__ void constitutive_eigen(int model, const InstMat& P, const float (*Ft)[3], float (*M)[3],
                                                float (*Fn)[3], float* tau6) {
    float U[3][3];
    jacobi_sym<DIM>(M, U);
    float eps[3], e2[3];
    float tr = 0.f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        // Hencky strain 0.5 ln(1 + delta) via the hardware log2 (absolute error
        // ~1e-7, below the float32 resolution of F itself)
        eps[a] = (0.5f * 0.69314718f) * __builtin_amdgcn_logf(1.f + fmaxf(M[a][a], -0.999999f));
        tr += eps[a];
    }
    bool plastic = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) e2[a] = eps[a];
    if (model == MPM_MODEL_DP) {
        if (tr > 0.f) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) e2[a] = 0.f;
            plastic = true;
        } else {
            float dev[3], nd2 = 0.f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                dev[a] = eps[a] - tr / (float)DIM;
                nd2 += dev[a] * dev[a];
            }
            const float nd = sqrtf(nd2);
            const float dg = nd + P.dp_coef * tr * P.alpha;
            if (dg > 0.f) {
                const float sc = dg * __builtin_amdgcn_rcpf(nd);
#pragma unroll
                for (int a = 0; a < DIM; ++a) e2[a] = eps[a] - sc * dev[a];
                plastic = true;
            }
        }
    }
    float tr2 = 0.f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) tr2 += e2[a];
    float sig[3], gam[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        sig[a] = 2.f * P.mu * e2[a] + P.lam * tr2;
        gam[a] = __builtin_amdgcn_exp2f((e2[a] - eps[a]) * 1.44269504f) - 1.f;
    }
    float T[3][3], W[3][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float st = 0.f, sw = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                st += U[a][c] * sig[c] * U[b][c];
                sw += U[a][c] * gam[c] * U[b][c];
            }
            T[a][b] = st;
            W[a][b] = sw;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s = Ft[a][b];
            if (plastic) {
#pragma unroll
                for (int c = 0; c < DIM; ++c) s += W[a][c] * Ft[c][b];
            }
            Fn[a][b] = s;
        }
    if (DIM == 3) {
        tau6[0] = T[0][0];
        tau6[1] = T[1][1];
        tau6[2] = T[2][2];
        tau6[3] = T[0][1];
        tau6[4] = T[1][2];
        tau6[5] = T[0][2];
    } else {
        tau6[0] = T[0][0];
        tau6[1] = T[1][1];
        tau6[2] = T[0][1];
    }
}


template <int DIM>
__device__ __forceinline__ unsigned constitutive(int model, const InstMat& P, const float (*Ft)[3], float (*Fn)[3],
                                                 float* tau6) {
    unsigned flags = 0;
    float det;
    if (DIM == 3)
        det = Ft[0][0] * (Ft[1][1] * Ft[2][2] - Ft[1][2] * Ft[2][1]) -
              Ft[0][1] * (Ft[1][0] * Ft[2][2] - Ft[1][2] * Ft[2][0]) +
              Ft[0][2] * (Ft[1][0] * Ft[2][1] - Ft[1][1] * Ft[2][0]);
    else
        det = Ft[0][0] * Ft[1][1] - Ft[0][1] * Ft[1][0];
    if (!(det > 0.f)) flags |= MPM_FLAG_INVERTED;
    // M = F F^T - I = H + H^T + H H^T with H = F - I
    float Hm[3][3], M[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Hm[a][b] = (a < DIM && b < DIM) ? Ft[a][b] - (a == b ? 1.f : 0.f) : 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            float s = Hm[a][b] + Hm[b][a];
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += Hm[a][c] * Hm[b][c];
            M[a][b] = s;
        }
    float nrm2 = 0.f;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) nrm2 += M[a][b] * M[a][b];
    if (nrm2 > SERIES_MAX_NORM2) {
        constitutive_eigen<DIM>(model, P, Ft, M, Fn, tau6);
        return flags;
    }
    // Series path (|M|_F <= 1/8): every quantity is a polynomial in the
    // symmetric M, so no eigenvectors are needed.  Hencky strain
    // E = log(I + M) / 2 by its Taylor series to degree 7 (truncation below
    // 1e-7 relative at |M| = 1/8); the return map acts on dev(E) as a matrix;
    // tau = 2 mu E' + lambda tr(E') I; F_new = expm(E' - E) F with expm - I to
    // degree 5 (|E' - E| <= |E|).
    // log(I + M) = sum_{k=1..7} (-1)^(k+1) M^k / k, evaluated as
    // (M - M^2/2 + M^3/3) + M^3 (-M/4 + M^2/5 - M^3/6 + M^4/7)
    // (Paterson-Stockmeyer: four matrix products instead of six)
    float Q[3][3], L[3][3], M2[3][3], M3[3][3], M4[3][3];
    sym_mul<DIM>(M, M, M2);
    sym_mul<DIM>(M2, M, M3);
    sym_mul<DIM>(M2, M2, M4);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            Q[a][b] = -0.25f * M[a][b] + M2[a][b] * (1.f / 5.f) - M3[a][b] * (1.f / 6.f) + M4[a][b] * (1.f / 7.f);
    float E[3][3];
    sym_mul<DIM>(M3, Q, L);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) E[a][b] = M[a][b] - 0.5f * M2[a][b] + M3[a][b] * (1.f / 3.f) + L[a][b];
    float tr = 0.f;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) E[a][b] *= 0.5f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) tr += E[a][a];
    // D = E' - E
    float Dm[3][3];
    bool plastic = false;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Dm[a][b] = 0.f;
    if (model == MPM_MODEL_DP) {
        if (tr > 0.f) {
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) Dm[a][b] = -E[a][b];
            plastic = true;
        } else {
            float nd2 = 0.f;
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) {
                    const float dv = E[a][b] - (a == b ? tr / (float)DIM : 0.f);
                    nd2 += dv * dv;
                }
            const float nd = sqrtf(nd2);
            const float dg = nd + P.dp_coef * tr * P.alpha;
            if (dg > 0.f) {
                const float sc = -dg * __builtin_amdgcn_rcpf(nd);
#pragma unroll
                for (int a = 0; a < DIM; ++a)
#pragma unroll
                    for (int b = 0; b < DIM; ++b) Dm[a][b] = sc * (E[a][b] - (a == b ? tr / (float)DIM : 0.f));
                plastic = true;
            }
        }
    }
    float tr2 = 0.f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) tr2 += E[a][a] + Dm[a][a];
    float T[3][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) T[a][b] = 2.f * P.mu * (E[a][b] + Dm[a][b]) + (a == b ? P.lam * tr2 : 0.f);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) Fn[a][b] = Ft[a][b];
    if (plastic) {
        float G[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Q[a][b] = (a == b ? 1.f : 0.f) + Dm[a][b] * 0.2f;
#pragma unroll
        for (int c = 4; c >= 2; --c) {
            sym_mul<DIM>(Dm, Q, L);
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) Q[a][b] = (a == b ? 1.f : 0.f) + L[a][b] * (1.f / (float)c);
        }
        sym_mul<DIM>(Dm, Q, G);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                float s2 = 0.f;
#pragma unroll
                for (int c = 0; c < DIM; ++c) s2 += G[a][c] * Ft[c][b];
                Fn[a][b] += s2;
            }
    }
    if (DIM == 3) {
        tau6[0] = T[0][0];
        tau6[1] = T[1][1];
        tau6[2] = T[2][2];
        tau6[3] = T[0][1];
        tau6[4] = T[1][2];
        tau6[5] = T[0][2];
    } else {
        tau6[0] = T[0][0];
        tau6[1] = T[1][1];
        tau6[2] = T[0][1];
    }
    return flags;
}

struct G2PIn {
    const float* x;
    const float* F;
    const uint32_t* id;
    const uint32_t* inst;
};
struct G2POut {
    float* x;
    float* v;
    float* C;
    float* F;
    float* tau;
    uint32_t* id;
    uint32_t* inst;
    uint32_t* keys;    // optional: the sort key of each new position (the next step's binning)
    uint32_t* movers;  // optional (with keys): the next incremental re-sort's counting, see k_g2p
};

// GS threads per workgroup, work items of at most g2p_max_items(GS) particles.
//
// With out.keys the kernel also bins each new position (the next build's
// sort key).  With out.movers as well it does the counting of the next
// incremental re-sort for the block of each item: the particles whose new key
// keeps the block's owner ("stayers") are counted per base cell in LDS and
// the counts stored to the block's row of rs_stay and their sum to rs_cnt
// (added, for blocks split over several items, to what the build cleared);
// the others ("movers") are appended to out.movers at a position claimed once
// per wave from the counter rs_n_mov.
template <int DIM, int GS>
__global__ __launch_bounds__(GS) void k_g2p(DevParams P, G2PIn in, G2POut out, int n,
                                            const uint32_t* __restrict__ osrc) {
    using T = Tile<DIM>;
    constexpr int NS = DIM == 3 ? 6 : 3;
    constexpr int DD = DIM * DIM;
    constexpr int VSY = 20, VSZ = DIM == 3 ? 120 : 0;  // padded float4 tile: row / plane strides
    __shared__ float4 vt[DIM == 3 ? 6 * VSZ : 6 * VSY];
    constexpr int MAXI = g2p_max_items(GS);
    __shared__ float xs[DIM][MAXI];
    __shared__ float fs[DD][MAXI];
    constexpr int NC = 1 << (2 * DIM);
    __shared__ unsigned scnt[NC];  // stayers per base cell of the current item's block
    if (threadIdx.x < NC) scnt[threadIdx.x] = 0u;
    const int n_work = min(P.ctr->n_work, P.work_cap);
    const float dx = P.dxf, inv_dx = P.inv_dxf;
    const float cscale = 4.f * inv_dx * inv_dx;  // D_p^{-1} = (4/dx^2) I for quadratic B-splines
    // Software pipeline over the items w, w + G, w + 2G, ... of a workgroup
    // (G workgroups).  While item w is computed, later items are being
    // gathered: the work record of item w + 2G and the source indices, tile
    // slots and block key of item w + G are loaded after phase 0, the particle
    // data, grid tile and material of item w + G after phase 1.  Each load is
    // consumed at least one compute phase after it was issued, so the
    // dependent chain record -> indices -> data stays off the critical path.
    // Every lane issues every load (indices past an item or the tile are
    // clamped into range and the values are discarded), so the number of
    // loads in flight does not depend on the lane's position in the item.
    constexpr int PER = MAXI / GS;                 // particles per thread
    constexpr int TPER = (T::N + GS - 1) / GS;     // tile nodes per thread
    const int tid = threadIdx.x;
    const int G = gridDim.x;
    struct Rec {
        int blk, s, e;  // raw record; the item length is formed where it is used
    };
    uint32_t pq[PER];
    int pphi[TPER];
    uint64_t pkey = 0;
    unsigned pch = 0;
    float px[PER][DIM], pF[PER][DD];
    uint32_t pid[PER], pin[PER];
    float4 pt[TPER];
    InstMat pmat;
    auto fetch_rec = [&](int i) {
        i = min(i, n_work - 1);  // past the end: the last record, never computed
        // The record is the same in every lane; the empty asm hides that, so
        // the values stay in vector registers and no read-first-lane right
        // after the loads waits for them.
        asm volatile("" : "+v"(i));
        Rec r;
        r.blk = P.w_block[i];
        r.s = P.w_start[i];
        r.e = P.w_end[i];
        return r;
    };
    auto fetch_index = [&](const Rec& R) {
        const int RL = min(R.e - R.s, MAXI);
#pragma unroll
        for (int k = 0; k < PER; ++k) pq[k] = osrc[R.s + min(tid + k * GS, RL - 1)];
#pragma unroll
        for (int k = 0; k < TPER; ++k) {
            const int t = min(tid + k * GS, T::N - 1);
            const int I = t % T::E, J = (t / T::E) % T::E, K = DIM == 3 ? t / (T::E * T::E) : 0;
            const int d = (I >> 2) | ((J >> 2) << 1) | ((K >> 2) << 2);
            pphi[k] = P.b_nbr[R.blk * T::NB + d];
        }
        // block key (sparse grids); a dense grid has no key table and reads a
        // discarded word of the neighbour table instead, so that the load is
        // unconditional and its value is not needed before the next item
        const uint64_t* kp = P.dense ? reinterpret_cast<const uint64_t*>(P.b_nbr + (size_t)R.blk * T::NB)
                                     : P.b_keys + R.blk;
        pkey = *kp;
        pch = P.b_chunks[R.blk];  // work items of the block
    };
    auto fetch_data = [&]() {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const size_t q = pq[k];
#pragma unroll
            for (int a = 0; a < DIM; ++a) px[k][a] = in.x[(size_t)a * n + q];
#pragma unroll
            for (int j = 0; j < DD; ++j) pF[k][j] = in.F[(size_t)j * n + q];
            pid[k] = in.id ? in.id[q] : (uint32_t)q;
            pin[k] = in.inst ? in.inst[q] : 0u;
        }
#pragma unroll
        for (int k = 0; k < TPER; ++k) {
            const int t = min(tid + k * GS, T::N - 1);
            const int I = t % T::E, J = (t / T::E) % T::E, K = DIM == 3 ? t / (T::E * T::E) : 0;
            const int l = (I & 3) + BLK * ((J & 3) + BLK * (K & 3));
            // a missing neighbour block (slot < 0) is zeroed when staged
            pt[k] = P.grid[(size_t)max(pphi[k], 0) * T::NPB + l];
        }
        int bc[3], inst = 0;
        if (!P.dense) unblock_key<DIM>(P, pkey, bc, &inst);
        pmat = material(P, inst);
    };
    int w = blockIdx.x;
    if (w >= n_work) return;
    Rec cur = fetch_rec(w);
    fetch_index(cur);
    fetch_data();
    Rec nxt = fetch_rec(w + G);
    while (w < n_work) {
        const int s = cur.s, L = min(cur.e - cur.s, MAXI);
        const uint64_t key = P.dense ? (uint64_t)cur.blk : pkey;
        const unsigned chunks = pch;
        const InstMat mat = pmat;
        // phase 0: stage the gathered item in LDS; ids travel with the
        // particles (output positions s .. s+L-1 are contiguous, so every
        // store coalesces; osrc named the input particle of each)
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int r = tid + k * GS;
            if (r < L) {
#pragma unroll
                for (int a = 0; a < DIM; ++a) xs[a][r] = px[k][a];
#pragma unroll
                for (int j = 0; j < DD; ++j) fs[j][r] = pF[k][j];
                if (out.id) out.id[s + r] = pid[k];
                if (out.inst) out.inst[s + r] = pin[k];
            }
        }
#pragma unroll
        for (int k = 0; k < TPER; ++k) {
            const int t = tid + k * GS;
            if (t < T::N) {
                const int I = t % T::E, J = (t / T::E) % T::E, K = DIM == 3 ? t / (T::E * T::E) : 0;
                vt[I + VSY * J + VSZ * K] = pphi[k] >= 0 ? pt[k] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        __syncthreads();
        fetch_index(nxt);
        const Rec nn = fetch_rec(w + 2 * G);
        int org[3], inst = 0;
        if (P.dense)
            linear_to_block<DIM>(P, (uint32_t)key, org);
        else
            unblock_key<DIM>(P, key, org, &inst);
        // owner part of the block's sort key (stayers keep it)
        const uint32_t own =
            ((uint32_t)inst << P.blk_bits) |
            (DIM == 3 ? ((uint32_t)org[2] * (uint32_t)P.nblk[1] + (uint32_t)org[1]) * (uint32_t)P.nblk[0] +
                            (uint32_t)org[0]
                      : (uint32_t)org[1] * (uint32_t)P.nblk[0] + (uint32_t)org[0]);
#pragma unroll
        for (int a = 0; a < 3; ++a) org[a] *= BLK;
        const float dt = mat.dt;
        // phase 1: grid gather, new position, velocity and affine matrix,
        // F_trial = (I + dt grad v) F (Eq. 17) kept in LDS
#pragma unroll 1
        for (int r = threadIdx.x; r < L; r += GS) {
            float xp[3] = {0, 0, 0};
#pragma unroll
            for (int a = 0; a < DIM; ++a) xp[a] = xs[a][r];
            int lb[3] = {0, 0, 0};
            float t[3] = {0, 0, 0}, u[3] = {1, 1, 1};
            particle_frame<DIM>(P, xp, org, lb, t, u);
            float wt[3][3], dw[3][3];
            bspline<DIM>(t, u, inv_dx, wt, dw);
            float dxn[3][3];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k) dxn[a][k] = ((float)k - 0.5f - t[a]) * dx;
            // Tensor-product factorisation, one axis at a time.  Along x, per
            // (ky, kz) row: S0 = sum w_x v, S1 = sum w_x dx_x v, S2 = sum dw_x v.
            // Along y, per kz plane: U0 = sum w_y S0, U1 = sum w_y dx_y S0,
            // U2 = sum dw_y S0, U3 = sum w_y S1, U4 = sum w_y S2.  Along z:
            // v_p = sum w_z U0, B = sum [w_z U3 | w_z U1 | w_z dx_z U0],
            // grad v = sum [w_z U4 | w_z U2 | dw_z U0].
            float vp[3] = {0, 0, 0}, B[3][3] = {{0}}, gv[3][3] = {{0}};
#pragma unroll
            for (int kz = 0; kz < (DIM == 3 ? 3 : 1); ++kz) {
                float U0[3] = {0, 0, 0}, U1[3] = {0, 0, 0}, U2[3] = {0, 0, 0}, U3[3] = {0, 0, 0}, U4[3] = {0, 0, 0};
#pragma unroll
                for (int ky = 0; ky < 3; ++ky) {
                    float S0[3] = {0, 0, 0}, S1[3] = {0, 0, 0}, S2[3] = {0, 0, 0};
#pragma unroll
                    for (int kx = 0; kx < 3; ++kx) {
                        const int idx = (lb[0] + kx) + VSY * (lb[1] + ky) + (DIM == 3 ? VSZ * (lb[2] + kz) : 0);
                        const float4 g = vt[idx];
                        const float vn[3] = {g.x, g.y, g.z};
                        const float wx = wt[0][kx], wdx = wt[0][kx] * dxn[0][kx], dwx = dw[0][kx];
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            S0[a] += wx * vn[a];
                            S1[a] += wdx * vn[a];
                            S2[a] += dwx * vn[a];
                        }
                    }
                    const float wy = wt[1][ky], wyd = wt[1][ky] * dxn[1][ky], dwy = dw[1][ky];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        U0[a] += wy * S0[a];
                        U1[a] += wyd * S0[a];
                        U2[a] += dwy * S0[a];
                        U3[a] += wy * S1[a];
                        U4[a] += wy * S2[a];
                    }
                    // keep the LDS gathers of one row in flight at a time
                    // (bounds register pressure, hence raises occupancy), and
                    // finish the row's sums here: without the empty asm the
                    // compiler sinks the B and grad v terms below the stores
                    // of x and v, which keeps all 27 nodal velocities live
                    // (215 instead of 150 VGPRs: two waves per SIMD, not three)
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int a = 0; a < DIM; ++a)
                        asm volatile("" : "+v"(U0[a]), "+v"(U1[a]), "+v"(U2[a]), "+v"(U3[a]), "+v"(U4[a]));
                }
                const float wz = DIM == 3 ? wt[2][kz] : 1.f;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    vp[a] += wz * U0[a];
                    B[a][0] += wz * U3[a];
                    B[a][1] += wz * U1[a];
                    gv[a][0] += wz * U4[a];
                    gv[a][1] += wz * U2[a];
                }
                if (DIM == 3) {
                    const float wzd = wz * dxn[2][kz], dwz = dw[2][kz];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        B[a][2] += wzd * U0[a];
                        gv[a][2] += dwz * U0[a];
                    }
                }
            }
            const size_t o = (size_t)(s + r);
            bool finite = true;
            float xn[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                xn[a] = xp[a] + dt * vp[a];
                finite = finite && isfinite(xn[a]) && isfinite(vp[a]);
                out.x[(size_t)a * n + o] = xn[a];
                out.v[(size_t)a * n + o] = vp[a];
            }
            if (out.keys) {
                // the next build's binning of the position just written (the
                // same float64 arithmetic as k_bin on the stored float32 value);
                // every particle of an item shares the owner block's instance
                unsigned bad = 0;
                const uint32_t nk = bin_key<DIM>(P, xn, (uint32_t)inst, &bad);
                out.keys[o] = nk;
                if (bad) raise_flag(P.ctr, bad);
                if (out.movers) {
                    const bool stay = (nk >> (2 * DIM)) == own;
                    if (stay) atomicAdd(&scnt[nk & (NC - 1)], 1u);
                    // movers of the wave's active lanes: one claim per wave
                    const unsigned long long mv = __ballot(!stay);
                    if (mv) {
                        const int leader = __ffsll((long long)mv) - 1;
                        const int lane = __lane_id();
                        unsigned base = 0u;
                        if (lane == leader) base = atomicAdd((unsigned*)&P.ctr->rs_n_mov, (unsigned)__popcll(mv));
                        base = (unsigned)__shfl((int)base, leader);
                        if (!stay) {
                            const unsigned slot = base + (unsigned)__popcll(mv & ((1ull << lane) - 1ull));
                            if (slot < (unsigned)n) out.movers[slot] = (uint32_t)o;
                        }
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) out.C[(size_t)(a * DIM + b) * n + o] = cscale * B[a][b];
            float Fp[3][3];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) Fp[a][b] = fs[a * DIM + b][r];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) {
                    float s2 = 0.f;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) s2 += gv[a][c] * Fp[c][b];
                    fs[a * DIM + b][r] = Fp[a][b] + dt * s2;
                }
            if (!finite) raise_flag(P.ctr, MPM_FLAG_NAN);
        }
        // no barrier: phase 2 reads only the trial F its own thread wrote
        fetch_data();  // in flight during phase 2
        // phase 2: constitutive update (its register live range is separate)
#pragma unroll 1
        for (int r = threadIdx.x; r < L; r += GS) {
            const size_t o = (size_t)(s + r);
            float Ft[3][3], Fn[3][3], tau6[6];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) Ft[a][b] = fs[a * DIM + b][r];
            unsigned flags = constitutive<DIM>(P.model, mat, Ft, Fn, tau6);
            bool finite = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) out.F[(size_t)(a * DIM + b) * n + o] = Fn[a][b];
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                finite = finite && isfinite(tau6[k]);
                out.tau[(size_t)k * n + o] = tau6[k];
            }
            if (!finite) flags |= MPM_FLAG_NAN;
            if (flags) raise_flag(P.ctr, flags);
        }
        __syncthreads();
        if (out.movers && threadIdx.x < 64) {
            // the first wave stores the item's stayer counts and their sum
            // (the particles of the block's entry, before the movers arrive)
            const unsigned c = threadIdx.x < NC ? scnt[threadIdx.x] : 0u;
            if (threadIdx.x < NC) {
                unsigned* row = P.rs_stay + (size_t)cur.blk * NC + threadIdx.x;
                if (chunks == 1u)
                    *row = c;
                else if (c)
                    atomicAdd(row, c);
                scnt[threadIdx.x] = 0u;  // ordered before the next item's counting by the barrier of its phase 0
            }
            const unsigned tot = wave_incl_scan(c);
            if (threadIdx.x == 63) {
                if (chunks == 1u)
                    P.rs_cnt[cur.blk] = tot;
                else if (tot)
                    atomicAdd(&P.rs_cnt[cur.blk], tot);
            }
        }
        w += G;
        cur = nxt;
        nxt = nn;
    }
}

hipError_t launch_p2g(const DevParams& P, const float* x, const float* v, const float* C, const float* tau, int n,
                      const uint32_t* order, const uint32_t* skeys, uint32_t* osrc, int grid_blocks, hipStream_t s,
                      bool update) {
    const int g = P.dense ? 65536 : grid_blocks * 4;
    if (P.dim == 3)
        k_p2g_cell<3><<<g, 64, 0, s>>>(P, x, v, C, tau, n, order, skeys, osrc);
    else
        k_p2g_cell<2><<<g, 64, 0, s>>>(P, x, v, C, tau, n, order, skeys, osrc);
    if (!P.dense) {
        const int gg = (int)std::min<long long>(((long long)P.block_cap + 3) / 4, 16384);  // one wave per block
        if (P.dim == 3) {
            if (update)
                k_p2g_gather<3, true><<<gg, WG, 0, s>>>(P);
            else
                k_p2g_gather<3, false><<<gg, WG, 0, s>>>(P);
        } else {
            if (update)
                k_p2g_gather<2, true><<<gg, WG, 0, s>>>(P);
            else
                k_p2g_gather<2, false><<<gg, WG, 0, s>>>(P);
        }
    }
    return hipGetLastError();
}

hipError_t launch_grid_update(const DevParams& P, long long n_nodes_host, int grid_blocks, hipStream_t s) {
    if (P.dim == 3)
        k_grid_update<3><<<grid_blocks, WG, 0, s>>>(P, n_nodes_host);
    else
        k_grid_update<2><<<grid_blocks, WG, 0, s>>>(P, n_nodes_host);
    return hipGetLastError();
}

hipError_t launch_g2p(const DevParams& P, const float* x_in, const float* F_in, const uint32_t* id_in,
                      const uint32_t* inst_in, float* x_out, float* v_out, float* C_out, float* F_out, float* tau_out,
                      uint32_t* id_out, uint32_t* inst_out, int n, const uint32_t* osrc, int block_size,
                      int grid_blocks, hipStream_t s, uint32_t* keys_out, uint32_t* movers_out) {
    G2PIn in{x_in, F_in, id_in, inst_in};
    G2POut out{x_out, v_out, C_out, F_out, tau_out, id_out, inst_out, keys_out, keys_out ? movers_out : nullptr};
    if (g2p_max_items(block_size) < P.chunk) return hipErrorInvalidValue;  // work items must fit the LDS staging
    switch (block_size * 4 + P.dim) {
        case 64 * 4 + 3: k_g2p<3, 64><<<grid_blocks, 64, 0, s>>>(P, in, out, n, osrc); break;
        case 128 * 4 + 3: k_g2p<3, 128><<<grid_blocks, 128, 0, s>>>(P, in, out, n, osrc); break;
        case 256 * 4 + 3: k_g2p<3, 256><<<grid_blocks, 256, 0, s>>>(P, in, out, n, osrc); break;
        case 64 * 4 + 2: k_g2p<2, 64><<<grid_blocks, 64, 0, s>>>(P, in, out, n, osrc); break;
        case 128 * 4 + 2: k_g2p<2, 128><<<grid_blocks, 128, 0, s>>>(P, in, out, n, osrc); break;
        case 256 * 4 + 2: k_g2p<2, 256><<<grid_blocks, 256, 0, s>>>(P, in, out, n, osrc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mpmx
