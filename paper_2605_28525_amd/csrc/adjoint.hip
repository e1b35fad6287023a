// Reverse mode of the explicit step: hand-written adjoints of G2P (with the
// Hencky / Drucker-Prager constitutive map), the grid update and P2G.
//
// Per step, with the forward recomputed from the step's input state:
//   k_g2p_adj      per particle (sorted order): recomputes v_p, B_p, grad v and
//                  F_trial from the staged grid tile, back-propagates the
//                  output adjoints through the constitutive map (Daleckii-Krein
//                  form on the eigen-decomposition of F F^T, with closed-form
//                  divided differences), and writes x_bar (partial), F_bar, and
//                  the per-particle (v'_bar, B_bar, W_bar) that the grid needs;
//                  accumulates dL/dE and dL/dphi.
//   k_scatter_adj  v_bar_n = sum_p N v'_bar + N B_bar (x_n - x_p) + W_bar grad N,
//                  one wave per owner block, one lane per base cell, like P2G.
//   k_grid_adj     u_bar = (boundary Jacobian) v_bar; p_bar = u_bar / m,
//                  m_bar = -u_bar . (u - dt g) / m.
//   k_p2g_adj      per particle gather of (p_bar, m_bar): v_bar, C_bar, tau_bar
//                  and the position terms (shape-function gradient and Hessian).
#include <math.h>

#include <algorithm>

#include "internal.h"
#include "particle.h"

namespace mpmx {

// x / sinh(x), smooth through 0
__device__ __forceinline__ float x_over_sinh(float x) {
    if (fabsf(x) < 1e-2f) return 1.f - x * x * (1.f / 6.f);
    return x / sinhf(x);
}
// sinh(beta x / 2) / sinh(x), smooth through 0
__device__ __forceinline__ float sinh_ratio(float beta, float x) {
    const float hb = 0.5f * beta;
    if (fabsf(x) < 1e-2f) return hb * (1.f + (hb * hb - 1.f) * x * x * (1.f / 6.f));
    return sinhf(hb * x) / sinhf(x);
}

// Adjoint of (F^E, tau) = Z(F_trial).  Inputs: Ft (F_trial), Fe_bar (full),
// tau_bar as stored components; outputs: Ft_bar, dL/dE, dL/dalpha.
template <int DIM>
__device__ void constitutive_adj(const DevParams& P, const float (*Ft)[3], const float (*Fe_bar)[3],
                                 const float* tau_bar_c, float (*Ft_bar)[3], float* E_bar, float* a_bar) {
    float Hm[3][3], M[3][3], U[3][3];
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
    jacobi_sym<DIM>(M, U);
    float lam[3] = {1.f, 1.f, 1.f}, eps[3] = {0.f, 0.f, 0.f};
    float tr = 0.f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        lam[a] = fmaxf(1.f + M[a][a], 1e-6f);
        eps[a] = 0.5f * logf(lam[a]);
        tr += eps[a];
    }
    // return map, its Jacobian J = d eps'/d eps, d eps'/d alpha, and kappa with
    // eps'_i - eps'_j = kappa (eps_i - eps_j)
    float e2[3], J[3][3], da[3] = {0.f, 0.f, 0.f}, kappa = 1.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        e2[a] = eps[a];
#pragma unroll
        for (int b = 0; b < 3; ++b) J[a][b] = a == b ? 1.f : 0.f;
    }
    if (P.model == MPM_MODEL_DP) {
        float dev[3], nd2 = 0.f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            dev[a] = eps[a] - tr / (float)DIM;
            nd2 += dev[a] * dev[a];
        }
        const float nd = sqrtf(nd2);
        const float dg = nd + P.dp_coef * tr * P.alpha;
        if (tr > 0.f) {
            kappa = 0.f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                e2[a] = 0.f;
#pragma unroll
                for (int b = 0; b < 3; ++b) J[a][b] = 0.f;
            }
        } else if (dg > 0.f) {
            const float ca = P.dp_coef * P.alpha;
            kappa = -ca * tr / nd;
            float nh[3];
#pragma unroll
            for (int a = 0; a < DIM; ++a) nh[a] = dev[a] / nd;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                e2[a] = tr / (float)DIM - ca * tr * nh[a];
                da[a] = -P.dp_coef * tr * nh[a];
#pragma unroll
                for (int b = 0; b < DIM; ++b) {
                    const float pdev = (a == b ? 1.f : 0.f) - 1.f / (float)DIM;
                    J[a][b] = 1.f / (float)DIM - ca * (nh[a] + tr * (pdev - nh[a] * nh[b]) / nd);
                }
            }
        }
    }
    float tr2 = 0.f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) tr2 += e2[a];
    const float c0 = e2[0] - kappa * eps[0];
    const float beta = kappa - 1.f;
    float t[3], h[3], Jt[3][3], Jh[3][3];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        t[i] = 2.f * P.mu * e2[i] + P.lam * tr2;
        h[i] = expf(e2[i] - eps[i]);
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            float cj = 0.f;
#pragma unroll
            for (int k = 0; k < DIM; ++k) cj += ((i == k ? 2.f * P.mu : 0.f) + P.lam) * J[k][j];
            Jt[i][j] = cj / (2.f * lam[j]);
            Jh[i][j] = h[i] * (J[i][j] - (i == j ? 1.f : 0.f)) / (2.f * lam[j]);
        }
    // symmetric adjoint of tau from stored components
    float Yt_s[3][3], Hb[3][3];
    if (DIM == 3) {
        Yt_s[0][0] = tau_bar_c[0];
        Yt_s[1][1] = tau_bar_c[1];
        Yt_s[2][2] = tau_bar_c[2];
        Yt_s[0][1] = Yt_s[1][0] = 0.5f * tau_bar_c[3];
        Yt_s[1][2] = Yt_s[2][1] = 0.5f * tau_bar_c[4];
        Yt_s[0][2] = Yt_s[2][0] = 0.5f * tau_bar_c[5];
    } else {
        Yt_s[0][0] = tau_bar_c[0];
        Yt_s[1][1] = tau_bar_c[1];
        Yt_s[0][1] = Yt_s[1][0] = 0.5f * tau_bar_c[2];
    }
    // H_bar = Fe_bar Ft^T (symmetrised); Ft_bar = H Fe_bar with H = U diag(h) U^T
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += Fe_bar[a][c] * Ft[b][c];
            Hb[a][b] = s;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = a + 1; b < DIM; ++b) Hb[a][b] = Hb[b][a] = 0.5f * (Hb[a][b] + Hb[b][a]);
    float Hmat[3][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += U[a][c] * h[c] * U[b][c];
            Hmat[a][b] = s;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += Hmat[a][c] * Fe_bar[c][b];
            Ft_bar[a][b] = s;
        }
    // rotate into the eigenbasis: Y = U^T Ybar U
    float Yt[3][3], Yh[3][3], tmp1[3][3], tmp2[3][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s1 = 0.f, s2 = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                s1 += Yt_s[a][c] * U[c][b];
                s2 += Hb[a][c] * U[c][b];
            }
            tmp1[a][b] = s1;
            tmp2[a][b] = s2;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s1 = 0.f, s2 = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                s1 += U[c][a] * tmp1[c][b];
                s2 += U[c][a] * tmp2[c][b];
            }
            Yt[a][b] = s1;
            Yh[a][b] = s2;
        }
    float S[3][3];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < DIM; ++i) s += Jt[i][j] * Yt[i][i] + Jh[i][j] * Yh[i][i];
        S[j][j] = s;
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            if (i == j) continue;
            const float x = eps[i] - eps[j], mid = 0.5f * (eps[i] + eps[j]);
            const float Kt = P.mu * kappa * expf(-2.f * mid) * x_over_sinh(x);
            const float Kh = expf(c0 + (beta - 2.f) * mid) * sinh_ratio(beta, x);
            S[i][j] = Kt * Yt[i][j] + Kh * Yh[i][j];
        }
    // b_bar = U S U^T; Ft_bar += 2 b_bar Ft
    float bb[3][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += S[a][c] * U[b][c];
            tmp1[a][b] = s;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += U[a][c] * tmp1[c][b];
            bb[a][b] = s;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = a + 1; b < DIM; ++b) bb[a][b] = bb[b][a] = 0.5f * (bb[a][b] + bb[b][a]);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) s += bb[a][c] * Ft[c][b];
            Ft_bar[a][b] += 2.f * s;
        }
    // parameters: tau is proportional to E; alpha enters eps' (plastic branch)
    float eb = 0.f, ab = 0.f;
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        eb += Yt[i][i] * t[i];
        float cda = 0.f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) cda += ((i == k ? 2.f * P.mu : 0.f) + P.lam) * da[k];
        ab += Yt[i][i] * cda + Yh[i][i] * h[i] * da[i];
    }
    *E_bar = eb / P.E;
    *a_bar = ab;
}

struct OutBar {
    const float* x;
    const float* v;
    const float* C;
    const float* F;
    const float* tau;
};

// shape-function value, gradient and Hessian at stencil offset (kx, ky, kz)
template <int DIM>
__device__ __forceinline__ void shape_k(const float (*wt)[3], const float (*dw)[3], const float* ddw, int kx, int ky,
                                        int kz, float* N, float* G, float (*Hs)[3]) {
    const int k[3] = {kx, ky, kz};
    float w[3] = {1.f, 1.f, 1.f}, d[3] = {0.f, 0.f, 0.f}, dd[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        w[a] = wt[a][k[a]];
        d[a] = dw[a][k[a]];
        dd[a] = ddw[k[a]];
    }
    *N = w[0] * w[1] * w[2];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        float g = d[a];
#pragma unroll
        for (int e = 0; e < DIM; ++e)
            if (e != a) g *= w[e];
        G[a] = g;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float hh;
            if (a == b) {
                hh = dd[a];
#pragma unroll
                for (int e = 0; e < DIM; ++e)
                    if (e != a) hh *= w[e];
            } else {
                hh = d[a] * d[b];
#pragma unroll
                for (int e = 0; e < DIM; ++e)
                    if (e != a && e != b) hh *= w[e];
            }
            Hs[a][b] = hh;
        }
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_g2p_adj(DevParams P, const float* __restrict__ x, const float* __restrict__ F,
                                                OutBar ob, float* __restrict__ x_bar, float* __restrict__ F_bar, int n,
                                                const uint32_t* __restrict__ order,
                                                const uint32_t* __restrict__ skeys) {
    using T = Tile<DIM>;
    constexpr int NS = DIM == 3 ? 6 : 3;
    constexpr int DD = DIM * DIM;
    __shared__ float4 vt[T::N];
    __shared__ int nbr[T::NB];
    __shared__ int org[3];
    __shared__ float red[2][WG / 64];
    __shared__ Interleave<DIM> il;
    const int n_work = min(P.ctr->n_work, P.work_cap);
    const float dt = P.dt, dx = P.dxf, inv_dx = P.inv_dxf;
    const float bscale = 4.f * inv_dx * inv_dx;
    float accE = 0.f, accA = 0.f;
    for (int w = blockIdx.x; w < n_work; w += gridDim.x) {
        const int blk = P.w_block[w], s = P.w_start[w], e = P.w_end[w];
        if (threadIdx.x < T::NB) nbr[threadIdx.x] = P.b_nbr[blk * T::NB + threadIdx.x];
        if (threadIdx.x == 0) {
            int bc[3];
            block_coords<DIM>(P, blk, bc);
            org[0] = bc[0] * BLK;
            org[1] = bc[1] * BLK;
            org[2] = bc[2] * BLK;
        }
        interleave_setup<DIM>(il, skeys, P.b_start[blk], P.b_start[blk] + P.b_count[blk]);
        for (int t = threadIdx.x; t < T::N; t += WG) {
            const int I = t % T::E, J = (t / T::E) % T::E, K = DIM == 3 ? t / (T::E * T::E) : 0;
            const int d = (I >> 2) | ((J >> 2) << 1) | ((K >> 2) << 2);
            const int phi = nbr[d];
            const int l = (I & 3) + BLK * ((J & 3) + BLK * (K & 3));
            vt[t] = phi >= 0 ? P.grid[(size_t)phi * T::NPB + l] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();
#pragma unroll 1
        for (int i = s + (int)threadIdx.x; i < e; i += WG) {
            const size_t q = order[i];
            const size_t o = (size_t)interleave_pos<DIM>(il, i, skeys[i]);  // where G2P stored it
            float xp[3] = {0, 0, 0}, Fp[3][3];
#pragma unroll
            for (int a = 0; a < DIM; ++a) xp[a] = x[(size_t)a * n + q];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) Fp[a][b] = F[(size_t)(a * DIM + b) * n + q];
            int lb[3] = {0, 0, 0};
            float tt[3] = {0, 0, 0}, uu[3] = {1, 1, 1};
            particle_frame<DIM>(P, xp, org, lb, tt, uu);
            float wt[3][3], dw[3][3], ddw[3], dxn[3][3];
            bspline<DIM>(tt, uu, inv_dx, wt, dw);
            bspline_dd(inv_dx * inv_dx, ddw);
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k) dxn[a][k] = ((float)k - 0.5f - tt[a]) * dx;
            // forward recompute: grad v
            float W[3][3] = {{0}};
#pragma unroll
            for (int kz = 0; kz < (DIM == 3 ? 3 : 1); ++kz)
#pragma unroll
                for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                    for (int kx = 0; kx < 3; ++kx) {
                        const int idx = (lb[0] + kx) + T::E * ((lb[1] + ky) + (DIM == 3 ? T::E * (lb[2] + kz) : 0));
                        const float4 g4 = vt[idx];
                        const float vn[3] = {g4.x, g4.y, g4.z};
                        float N, G[3], Hs[3][3];
                        shape_k<DIM>(wt, dw, ddw, kx, ky, kz, &N, G, Hs);
#pragma unroll
                        for (int a = 0; a < DIM; ++a)
#pragma unroll
                            for (int b = 0; b < DIM; ++b) W[a][b] += vn[a] * G[b];
                    }
            float Ft[3][3];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) {
                    float s2 = 0.f;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) s2 += W[a][c] * Fp[c][b];
                    Ft[a][b] = Fp[a][b] + dt * s2;
                }
            // output adjoints at the particle's G2P output position o
            float xbo[3] = {0, 0, 0}, vbo[3] = {0, 0, 0}, Cbo[3][3] = {{0}}, Fbo[3][3] = {{0}}, tbo[6] = {0};
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                xbo[a] = ob.x[(size_t)a * n + o];
                vbo[a] = ob.v[(size_t)a * n + o];
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) {
                    Cbo[a][b] = ob.C[(size_t)(a * DIM + b) * n + o];
                    Fbo[a][b] = ob.F[(size_t)(a * DIM + b) * n + o];
                }
#pragma unroll
            for (int k = 0; k < NS; ++k) tbo[k] = ob.tau[(size_t)k * n + o];
            float Ftb[3][3], eb, ab;
            constitutive_adj<DIM>(P, Ft, Fbo, tbo, Ftb, &eb, &ab);
            accE += eb;
            accA += ab;
            // F_trial = (I + dt W) F
            float Fb[3][3], Wb[3][3];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) {
                    float s1 = Ftb[a][b], s2 = 0.f;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        s1 += dt * W[c][a] * Ftb[c][b];
                        s2 += Ftb[a][c] * Fp[b][c];
                    }
                    Fb[a][b] = s1;
                    Wb[a][b] = dt * s2;
                }
            float vpb[3], Bb[3][3], xb[3];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                vpb[a] = vbo[a] + dt * xbo[a];
                xb[a] = xbo[a];
#pragma unroll
                for (int b = 0; b < DIM; ++b) Bb[a][b] = bscale * Cbo[a][b];
            }
            // position adjoint through the weights of the gather
#pragma unroll
            for (int kz = 0; kz < (DIM == 3 ? 3 : 1); ++kz)
#pragma unroll
                for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                    for (int kx = 0; kx < 3; ++kx) {
                        const int idx = (lb[0] + kx) + T::E * ((lb[1] + ky) + (DIM == 3 ? T::E * (lb[2] + kz) : 0));
                        const float4 g4 = vt[idx];
                        const float vn[3] = {g4.x, g4.y, g4.z};
                        float N, G[3], Hs[3][3];
                        shape_k<DIM>(wt, dw, ddw, kx, ky, kz, &N, G, Hs);
                        const float dd[3] = {dxn[0][kx], dxn[1][ky], DIM == 3 ? dxn[2][kz] : 0.f};
                        float s1 = 0.f, s2 = 0.f, BtV[3] = {0, 0, 0}, WtV[3] = {0, 0, 0};
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            s1 += vn[a] * vpb[a];
#pragma unroll
                            for (int b = 0; b < DIM; ++b) {
                                s2 += vn[a] * Bb[a][b] * dd[b];
                                BtV[b] += Bb[a][b] * vn[a];
                                WtV[b] += Wb[a][b] * vn[a];
                            }
                        }
#pragma unroll
                        for (int c = 0; c < DIM; ++c) {
                            float hv = 0.f;
#pragma unroll
                            for (int b = 0; b < DIM; ++b) hv += Hs[b][c] * WtV[b];
                            xb[c] += G[c] * (s1 + s2) - N * BtV[c] + hv;
                        }
                    }
#pragma unroll
            for (int a = 0; a < DIM; ++a) x_bar[(size_t)a * n + q] = xb[a];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) F_bar[(size_t)(a * DIM + b) * n + q] = Fb[a][b];
            float* sc = P.adj_scratch;
#pragma unroll
            for (int a = 0; a < DIM; ++a) sc[(size_t)a * n + i] = vpb[a];
#pragma unroll
            for (int k = 0; k < DD; ++k) {
                sc[(size_t)(DIM + k) * n + i] = Bb[k / DIM][k % DIM];
                sc[(size_t)(DIM + DD + k) * n + i] = Wb[k / DIM][k % DIM];
            }
        }
        __syncthreads();
    }
    // parameter gradients: wave reduction, then one atomic per workgroup that
    // had an item (same-address float atomics serialise in L2: thousands of
    // empty workgroups adding zeros made the reverse sweep 1.8x slower)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        accE += __shfl_xor(accE, o);
        accA += __shfl_xor(accA, o);
    }
    if (__lane_id() == 0) {
        red[0][threadIdx.x >> 6] = accE;
        red[1][threadIdx.x >> 6] = accA;
    }
    __syncthreads();
    if (threadIdx.x == 0 && (int)blockIdx.x < n_work) {
        float se = 0.f, sa = 0.f;
#pragma unroll
        for (int k = 0; k < WG / 64; ++k) {
            se += red[0][k];
            sa += red[1][k];
        }
        atomicAdd(&P.param_bar[0], se);
        atomicAdd(&P.param_bar[1], sa * P.dalpha_dphi);
    }
}

// v_bar_n = sum_p N v'_bar + N B_bar (x_n - x_p) + W_bar grad N; same block /
// cell organisation as the forward P2G (one wave per owner block, one lane per
// base cell, register sums merged into an LDS tile offset by offset).
template <int DIM>
__global__ __launch_bounds__(64) void k_scatter_adj(DevParams P, const float* __restrict__ x, int n,
                                                    const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ skeys) {
    using T = Tile<DIM>;
    constexpr int NC = T::NPB;
    constexpr int NK = DIM == 3 ? 27 : 9;
    constexpr int DD = DIM * DIM;
    __shared__ float tile[3][T::NP];
    __shared__ int cs[NC], ce[NC];
    const int lane = threadIdx.x;
    const int nb = min(P.ctr->nb, P.block_cap);
    const float dx = P.dxf, inv_dx = P.inv_dxf;
    const float* sc = P.adj_scratch;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int cnt = P.b_count[b];
        if (cnt <= 0) continue;
        const int st = P.b_start[b], en = st + cnt;
        for (int t = lane; t < 3 * T::NP; t += 64) (&tile[0][0])[t] = 0.f;
        for (int c = lane; c < NC; c += 64) cs[c] = ce[c] = 0;
        int bc[3];
        block_coords<DIM>(P, b, bc);
        const int org[3] = {bc[0] * BLK, bc[1] * BLK, bc[2] * BLK};
        __syncthreads();
        for (int i = st + lane; i < en; i += 64) {
            const uint32_t c = skeys[i] & (NC - 1);
            if (i == st || (skeys[i - 1] & (NC - 1)) != c) cs[c] = i;
            if (i == en - 1 || (skeys[i + 1] & (NC - 1)) != c) ce[c] = i + 1;
        }
        __syncthreads();
        float acc[NK][3];
#pragma unroll
        for (int k = 0; k < NK; ++k) acc[k][0] = acc[k][1] = acc[k][2] = 0.f;
        int lb[3] = {lane & 3, (lane >> 2) & 3, DIM == 3 ? (lane >> 4) & 3 : 0};
        bool has = false;
        if (lane < NC) {
            const int c0 = cs[lane], c1 = ce[lane];
            has = c1 > c0;
            for (int i = c0; i < c1; ++i) {
                const size_t q = order[i];
                float xp[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < DIM; ++a) xp[a] = x[(size_t)a * n + q];
                float vb[3] = {0, 0, 0}, A[3][3] = {{0}}, G[3][3] = {{0}};
#pragma unroll
                for (int a = 0; a < DIM; ++a) vb[a] = sc[(size_t)a * n + i];
#pragma unroll
                for (int k = 0; k < DD; ++k) {
                    A[k / DIM][k % DIM] = sc[(size_t)(DIM + k) * n + i];
                    G[k / DIM][k % DIM] = -sc[(size_t)(DIM + DD + k) * n + i];
                }
                float tt[3] = {0, 0, 0}, uu[3] = {1, 1, 1};
                particle_frame<DIM>(P, xp, org, lb, tt, uu);
                float wt[3][3], dw[3][3], dxn[3][3];
                bspline<DIM>(tt, uu, inv_dx, wt, dw);
#pragma unroll
                for (int a = 0; a < DIM; ++a)
#pragma unroll
                    for (int k = 0; k < 3; ++k) dxn[a][k] = ((float)k - 0.5f - tt[a]) * dx;
#pragma unroll
                for (int kz = 0; kz < (DIM == 3 ? 3 : 1); ++kz)
#pragma unroll
                    for (int ky = 0; ky < 3; ++ky) {
                        const float wz = DIM == 3 ? wt[2][kz] : 1.f;
                        const float al = wt[1][ky] * wz;
                        const float gy = dw[1][ky] * wz;
                        const float gz = DIM == 3 ? wt[1][ky] * dw[2][kz] : 0.f;
                        const float dy = dxn[1][ky], dz = DIM == 3 ? dxn[2][kz] : 0.f;
                        float be[3];
#pragma unroll
                        for (int a = 0; a < DIM; ++a)
                            be[a] = al * (vb[a] + A[a][1] * dy + (DIM == 3 ? A[a][2] * dz : 0.f)) - G[a][1] * gy -
                                    (DIM == 3 ? G[a][2] * gz : 0.f);
#pragma unroll
                        for (int kx = 0; kx < 3; ++kx) {
                            const int k = kx + 3 * (ky + 3 * kz);
                            const float wx = wt[0][kx];
                            const float ca = al * wx * dxn[0][kx], cg = al * dw[0][kx];
#pragma unroll
                            for (int a = 0; a < DIM; ++a) acc[k][a] += wx * be[a] + A[a][0] * ca - G[a][0] * cg;
                        }
                    }
            }
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int kx = k % 3, ky = (k / 3) % 3, kz = DIM == 3 ? k / 9 : 0;
            const int idx = T::pad(lb[0] + kx, lb[1] + ky, DIM == 3 ? lb[2] + kz : 0);
            if (has) {
#pragma unroll
                for (int a = 0; a < DIM; ++a) tile[a][idx] += acc[k][a];
            }
            __syncthreads();
        }
        for (int t = lane; t < T::N; t += 64) {
            const int I = t % T::E;
            const int J = (t / T::E) % T::E;
            const int K = DIM == 3 ? t / (T::E * T::E) : 0;
            const int tp = T::pad(I, J, K);
            const float p0 = tile[0][tp], p1 = tile[1][tp], p2 = DIM == 3 ? tile[2][tp] : 0.f;
            if (p0 != 0.f || p1 != 0.f || p2 != 0.f) {
                const int d = (I >> 2) | ((J >> 2) << 1) | ((K >> 2) << 2);
                const int phi = P.b_nbr[(size_t)b * T::NB + d];
                if (phi >= 0) {
                    const int l = (I & 3) + BLK * ((J & 3) + BLK * (K & 3));
                    float* g = reinterpret_cast<float*>(&P.grid_bar[(size_t)phi * T::NPB + l]);
                    atomicAdd(g + 0, p0);
                    atomicAdd(g + 1, p1);
                    if (DIM == 3) atomicAdd(g + 2, p2);
                }
            }
        }
        __syncthreads();
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_grid_adj(DevParams P, long long n_nodes_host) {
    constexpr int NPB = Tile<DIM>::NPB;
    const long long n_nodes = n_nodes_host >= 0 ? n_nodes_host : (long long)P.ctr->nb * NPB;
    for (long long s = (long long)blockIdx.x * WG + threadIdx.x; s < n_nodes; s += (long long)gridDim.x * WG) {
        const float4 gb = P.grid_bar[s];
        const float4 gu = P.grid_u[s];
        const float m = gu.w;
        float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
        if (m > 0.f) {
            float ub[3] = {gb.x, gb.y, gb.z};
            const float u[3] = {gu.x, gu.y, gu.z};
            const int b = (int)(s / NPB), l = (int)(s % NPB);
            int bc[3];
            block_coords<DIM>(P, b, bc);
            const int node[3] = {bc[0] * BLK + (l & 3), bc[1] * BLK + ((l >> 2) & 3),
                                 DIM == 3 ? bc[2] * BLK + (l >> 4) : 0};
            // Jacobian of the wall projections (diagonal 0/1), applied to the adjoint
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const bool on = side == 0 ? node[a] < P.bound : node[a] > P.cells[a] - P.bound;
                    if (!on) continue;
                    const int kind = P.bc[a][side];
                    if (kind == MPM_BC_STICKY) {
                        ub[0] = ub[1] = ub[2] = 0.f;
                    } else if (kind == MPM_BC_SLIP) {
                        ub[a] = 0.f;
                    } else if (kind == MPM_BC_SEPARATE) {
                        if (side == 0 ? u[a] < 0.f : u[a] > 0.f) ub[a] = 0.f;
                    }
                }
            }
            const float inv = 1.f / m;
            float mb = 0.f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) mb -= ub[a] * (u[a] - P.dt * P.g[a]);
            out = make_float4(ub[0] * inv, ub[1] * inv, DIM == 3 ? ub[2] * inv : 0.f, mb * inv);
        }
        P.grid_bar[s] = out;
    }
}

struct PIn {
    const float* x;
    const float* v;
    const float* C;
    const float* tau;
};
struct PBar {
    float* x;
    float* v;
    float* C;
    float* tau;
};

template <int DIM>
__global__ __launch_bounds__(WG) void k_p2g_adj(DevParams P, PIn in, PBar bar, int n,
                                                const uint32_t* __restrict__ order) {
    using T = Tile<DIM>;
    constexpr int NS = DIM == 3 ? 6 : 3;
    __shared__ float4 gt[T::N];
    __shared__ int nbr[T::NB];
    __shared__ int org[3];
    const int n_work = min(P.ctr->n_work, P.work_cap);
    const float mp = P.p_mass, dtv = P.dt * P.p_vol0;
    const float dx = P.dxf, inv_dx = P.inv_dxf;
    for (int w = blockIdx.x; w < n_work; w += gridDim.x) {
        const int blk = P.w_block[w], s = P.w_start[w], e = P.w_end[w];
        if (threadIdx.x < T::NB) nbr[threadIdx.x] = P.b_nbr[blk * T::NB + threadIdx.x];
        if (threadIdx.x == 0) {
            int bc[3];
            block_coords<DIM>(P, blk, bc);
            org[0] = bc[0] * BLK;
            org[1] = bc[1] * BLK;
            org[2] = bc[2] * BLK;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < T::N; t += WG) {
            const int I = t % T::E, J = (t / T::E) % T::E, K = DIM == 3 ? t / (T::E * T::E) : 0;
            const int d = (I >> 2) | ((J >> 2) << 1) | ((K >> 2) << 2);
            const int phi = nbr[d];
            const int l = (I & 3) + BLK * ((J & 3) + BLK * (K & 3));
            gt[t] = phi >= 0 ? P.grid_bar[(size_t)phi * T::NPB + l] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();
#pragma unroll 1
        for (int i = s + (int)threadIdx.x; i < e; i += WG) {
            const size_t q = order[i];
            float xp[3] = {0, 0, 0}, vp[3] = {0, 0, 0}, Cp[3][3] = {{0}}, tau[3][3] = {{0}};
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                xp[a] = in.x[(size_t)a * n + q];
                vp[a] = in.v[(size_t)a * n + q];
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) Cp[a][b] = in.C[(size_t)(a * DIM + b) * n + q];
            if (DIM == 3) {
                tau[0][0] = in.tau[q];
                tau[1][1] = in.tau[(size_t)n + q];
                tau[2][2] = in.tau[2 * (size_t)n + q];
                tau[0][1] = tau[1][0] = in.tau[3 * (size_t)n + q];
                tau[1][2] = tau[2][1] = in.tau[4 * (size_t)n + q];
                tau[0][2] = tau[2][0] = in.tau[5 * (size_t)n + q];
            } else {
                tau[0][0] = in.tau[q];
                tau[1][1] = in.tau[(size_t)n + q];
                tau[0][1] = tau[1][0] = in.tau[2 * (size_t)n + q];
            }
            int lb[3] = {0, 0, 0};
            float tt[3] = {0, 0, 0}, uu[3] = {1, 1, 1};
            particle_frame<DIM>(P, xp, org, lb, tt, uu);
            float wt[3][3], dw[3][3], ddw[3], dxn[3][3];
            bspline<DIM>(tt, uu, inv_dx, wt, dw);
            bspline_dd(inv_dx * inv_dx, ddw);
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int k = 0; k < 3; ++k) dxn[a][k] = ((float)k - 0.5f - tt[a]) * dx;
            float vb[3] = {0, 0, 0}, Cb[3][3] = {{0}}, tb[3][3] = {{0}}, xb[3] = {0, 0, 0};
#pragma unroll
            for (int kz = 0; kz < (DIM == 3 ? 3 : 1); ++kz)
#pragma unroll
                for (int ky = 0; ky < 3; ++ky)
#pragma unroll
                    for (int kx = 0; kx < 3; ++kx) {
                        const int idx = (lb[0] + kx) + T::E * ((lb[1] + ky) + (DIM == 3 ? T::E * (lb[2] + kz) : 0));
                        const float4 g4 = gt[idx];
                        const float pb[3] = {g4.x, g4.y, g4.z};
                        const float mb = g4.w;
                        float N, G[3], Hs[3][3];
                        shape_k<DIM>(wt, dw, ddw, kx, ky, kz, &N, G, Hs);
                        const float dd[3] = {dxn[0][kx], dxn[1][ky], DIM == 3 ? dxn[2][kz] : 0.f};
                        // mom = v + C dxn ; tau p_bar
                        float pm = 0.f, CtP[3] = {0, 0, 0}, tP[3] = {0, 0, 0};
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            float ma = vp[a];
#pragma unroll
                            for (int b = 0; b < DIM; ++b) {
                                ma += Cp[a][b] * dd[b];
                                CtP[b] += Cp[a][b] * pb[a];
                                tP[b] += tau[a][b] * pb[a];
                            }
                            pm += pb[a] * ma;
                        }
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            vb[a] += mp * N * pb[a];
#pragma unroll
                            for (int b = 0; b < DIM; ++b) {
                                Cb[a][b] += mp * N * pb[a] * dd[b];
                                tb[a][b] -= dtv * pb[a] * G[b];
                            }
                        }
#pragma unroll
                        for (int c = 0; c < DIM; ++c) {
                            float ht = 0.f;
#pragma unroll
                            for (int b = 0; b < DIM; ++b) ht += Hs[b][c] * tP[b];
                            xb[c] += mb * mp * G[c] + mp * G[c] * pm - N * mp * CtP[c] - dtv * ht;
                        }
                    }
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                bar.v[(size_t)a * n + q] = vb[a];
                bar.x[(size_t)a * n + q] += xb[a];
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) bar.C[(size_t)(a * DIM + b) * n + q] = Cb[a][b];
            if (DIM == 3) {
                bar.tau[q] = tb[0][0];
                bar.tau[(size_t)n + q] = tb[1][1];
                bar.tau[2 * (size_t)n + q] = tb[2][2];
                bar.tau[3 * (size_t)n + q] = tb[0][1] + tb[1][0];
                bar.tau[4 * (size_t)n + q] = tb[1][2] + tb[2][1];
                bar.tau[5 * (size_t)n + q] = tb[0][2] + tb[2][0];
            } else {
                bar.tau[q] = tb[0][0];
                bar.tau[(size_t)n + q] = tb[1][1];
                bar.tau[2 * (size_t)n + q] = tb[0][1] + tb[1][0];
            }
        }
        __syncthreads();
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_grid_bar_clear(DevParams P, long long n_nodes_host) {
    constexpr int NPB = Tile<DIM>::NPB;
    const long long n_nodes = n_nodes_host >= 0 ? n_nodes_host : (long long)P.ctr->nb * NPB;
    for (long long s = (long long)blockIdx.x * WG + threadIdx.x; s < n_nodes; s += (long long)gridDim.x * WG)
        P.grid_bar[s] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_g2p_adj(const DevParams& P, const float* x, const float* F, const float* const* out_bar, float* x_bar,
                          float* F_bar, int n, const uint32_t* order, const uint32_t* skeys, int grid_blocks,
                          hipStream_t s) {
    OutBar ob{out_bar[0], out_bar[1], out_bar[2], out_bar[3], out_bar[4]};
    if (P.dim == 3)
        k_g2p_adj<3><<<grid_blocks, WG, 0, s>>>(P, x, F, ob, x_bar, F_bar, n, order, skeys);
    else
        k_g2p_adj<2><<<grid_blocks, WG, 0, s>>>(P, x, F, ob, x_bar, F_bar, n, order, skeys);
    return hipGetLastError();
}

hipError_t launch_scatter_adj(const DevParams& P, const float* x, int n, const uint32_t* order, const uint32_t* skeys,
                              int grid_blocks, hipStream_t s) {
    const long long nodes = (long long)P.block_cap * (P.dim == 3 ? 64 : 16);
    const int gc = (int)std::min<long long>((nodes + WG - 1) / WG, P.dense ? 65536 : 8192);
    if (P.dim == 3) {
        k_grid_bar_clear<3><<<gc, WG, 0, s>>>(P, P.dense ? nodes : -1);
        k_scatter_adj<3><<<P.dense ? 65536 : grid_blocks * 4, 64, 0, s>>>(P, x, n, order, skeys);
    } else {
        k_grid_bar_clear<2><<<gc, WG, 0, s>>>(P, P.dense ? nodes : -1);
        k_scatter_adj<2><<<P.dense ? 65536 : grid_blocks * 4, 64, 0, s>>>(P, x, n, order, skeys);
    }
    return hipGetLastError();
}

hipError_t launch_grid_adj(const DevParams& P, long long n_nodes_host, int grid_blocks, hipStream_t s) {
    if (P.dim == 3)
        k_grid_adj<3><<<grid_blocks, WG, 0, s>>>(P, n_nodes_host);
    else
        k_grid_adj<2><<<grid_blocks, WG, 0, s>>>(P, n_nodes_host);
    return hipGetLastError();
}

hipError_t launch_p2g_adj(const DevParams& P, const float* const* in, float* const* in_bar, int n,
                          const uint32_t* order, int grid_blocks, hipStream_t s) {
    PIn pin{in[0], in[1], in[2], in[3]};
    PBar pb{in_bar[0], in_bar[1], in_bar[2], in_bar[3]};
    if (P.dim == 3)
        k_p2g_adj<3><<<grid_blocks, WG, 0, s>>>(P, pin, pb, n, order);
    else
        k_p2g_adj<2><<<grid_blocks, WG, 0, s>>>(P, pin, pb, n, order);
    return hipGetLastError();
}

}  // namespace mpmx
