// C ABI of the sparse-grid MPM step: context management, argument checks and
// the per-step call sequence.  Everything a step needs is allocated once at
// mpm_create (capacity-bounded); the step itself never allocates, and the
// only host synchronisation points are mpm_get_status, mpm_active_count and
// the optional Algorithm-7 rebuild (MPM_FLAG_SYNC_REBUILD).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "internal.h"

using namespace mpmx;

struct mpm_ctx {
    mpm_params prm;
    int dim = 3;
    int nblk[3] = {1, 1, 1};
    long long n_blocks_total = 0;
    int key_bits = 0;
    int block_cap = 0;
    int H_log2 = 0;
    int work_cap = 0;
    int chunk = 512;
    int max_particles = 0;
    bool dense = false;
    int persistent_wgs = 2048;
    // sort
    uint32_t *k0 = nullptr, *k1 = nullptr, *v0 = nullptr, *v1 = nullptr;
    unsigned* hist = nullptr;
    unsigned* partials = nullptr;
    // hash
    uint64_t *h_keys = nullptr, *h_mask = nullptr;
    int *h_vals = nullptr, *h_start = nullptr, *h_end = nullptr;
    // blocks
    uint64_t *b_keys = nullptr, *b_mask = nullptr;
    int *b_nbr = nullptr, *b_start = nullptr, *b_count = nullptr;
    unsigned *b_chunks = nullptr, *b_chunk_off = nullptr;
    // work
    int *w_block = nullptr, *w_start = nullptr, *w_end = nullptr;
    float4* grid = nullptr;
    float4* grid_u = nullptr;
    float4* grid_bar = nullptr;
    float* adj_scratch = nullptr;
    bool adjoint = false;
    float* heightmap = nullptr;
    DevCounters* ctr = nullptr;
    DevParams P{};
    bool built = false;
    int built_n = -1;
    uint32_t* order = nullptr;
    uint32_t* skeys = nullptr;
};

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

int bits_for(long long v) {
    int b = 0;
    while ((1ll << b) <= v) ++b;
    return b;
}

void free_capacity_buffers(mpm_ctx* c) {
    dfree(c->h_keys);
    dfree(c->h_mask);
    dfree(c->h_vals);
    dfree(c->h_start);
    dfree(c->h_end);
    dfree(c->b_keys);
    dfree(c->b_mask);
    dfree(c->b_nbr);
    dfree(c->b_start);
    dfree(c->b_count);
    dfree(c->b_chunks);
    dfree(c->b_chunk_off);
    dfree(c->w_block);
    dfree(c->w_start);
    dfree(c->w_end);
    dfree(c->grid);
    dfree(c->grid_u);
    dfree(c->grid_bar);
    dfree(c->partials);
}

void free_all(mpm_ctx* c) {
    free_capacity_buffers(c);
    dfree(c->k0);
    dfree(c->k1);
    dfree(c->v0);
    dfree(c->v1);
    dfree(c->hist);
    dfree(c->heightmap);
    dfree(c->adj_scratch);
    dfree(c->ctr);
}

void fill_material(mpm_ctx* c) {
    const double E = c->prm.E, nu = c->prm.nu;
    const double mu = E / (2.0 * (1.0 + nu));
    const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double sphi = sin(c->prm.friction_deg * M_PI / 180.0);
    c->P.mu = (float)mu;
    c->P.lam = (float)lam;
    c->P.alpha = (float)(sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi));
    c->P.dp_coef = (float)((c->dim * lam + 2.0 * mu) / (2.0 * mu));
    c->P.dt = c->prm.dt;
    c->P.E = c->prm.E;
    const double phi = c->prm.friction_deg * M_PI / 180.0;
    c->P.dalpha_dphi = (float)(sqrt(2.0 / 3.0) * 6.0 * cos(phi) / ((3.0 - sphi) * (3.0 - sphi)) * (M_PI / 180.0));
}

void fill_params(mpm_ctx* c) {
    DevParams& P = c->P;
    const mpm_params& q = c->prm;
    P.dim = c->dim;
    for (int a = 0; a < 3; ++a) {
        P.cells[a] = a < c->dim ? q.cells[a] : 0;
        P.nblk[a] = c->nblk[a];
        P.g[a] = q.gravity[a];
        P.bc[a][0] = a < c->dim ? q.bc[a][0] : MPM_BC_NONE;
        P.bc[a][1] = a < c->dim ? q.bc[a][1] : MPM_BC_NONE;
    }
    P.dense = c->dense ? 1 : 0;
    P.dx = q.dx;
    P.inv_dx = 1.0 / q.dx;
    P.dxf = (float)q.dx;
    P.inv_dxf = (float)(1.0 / q.dx);
    P.model = q.model;
    P.p_mass = q.p_mass;
    P.p_vol0 = q.p_vol0;
    P.bound = q.bound > 0 ? q.bound : 3;
    P.heightmap = c->heightmap;
    P.mu_terrain = q.mu_terrain;
    P.has_terrain = c->heightmap != nullptr;
    P.h_keys = c->h_keys;
    P.h_mask = c->h_mask;
    P.h_vals = c->h_vals;
    P.h_start = c->h_start;
    P.h_end = c->h_end;
    P.h_mask_bits = (unsigned)((1u << c->H_log2) - 1u);
    P.n_probe = 1 << c->H_log2;
    P.b_keys = c->b_keys;
    P.b_mask = c->b_mask;
    P.b_nbr = c->b_nbr;
    P.b_start = c->b_start;
    P.b_count = c->b_count;
    P.b_chunks = c->b_chunks;
    P.b_chunk_off = c->b_chunk_off;
    P.block_cap = c->block_cap;
    P.w_block = c->w_block;
    P.w_start = c->w_start;
    P.w_end = c->w_end;
    P.work_cap = c->work_cap;
    P.chunk = c->chunk;
    P.grid = c->grid;
    P.ctr = c->ctr;
    P.grid_u = c->grid_u;
    P.grid_bar = c->grid_bar;
    P.adj_scratch = c->adj_scratch;
    P.param_bar = nullptr;
    fill_material(c);
}

// (Re)allocate every buffer whose size depends on block_cap or H.
int alloc_capacity_buffers(mpm_ctx* c) {
    free_capacity_buffers(c);
    const int NB = 1 << c->dim, NPB = 1 << (2 * c->dim);
    const size_t H = (size_t)1 << c->H_log2;
    const size_t cap = (size_t)c->block_cap;
    c->work_cap = c->block_cap + c->max_particles / c->chunk + 1;
    int scan_n = std::max({radix_hist_size(c->max_particles), (int)H, c->block_cap, 1});
    hipError_t e = hipSuccess;
    if (!c->dense) {
        e = e ? e : dalloc(&c->h_keys, H);
        e = e ? e : dalloc(&c->h_mask, H);
        e = e ? e : dalloc(&c->h_vals, H);
        e = e ? e : dalloc(&c->h_start, H);
        e = e ? e : dalloc(&c->h_end, H);
        e = e ? e : dalloc(&c->b_keys, cap);
        e = e ? e : dalloc(&c->b_mask, cap);
    }
    e = e ? e : dalloc(&c->b_nbr, cap * NB);
    e = e ? e : dalloc(&c->b_start, cap);
    e = e ? e : dalloc(&c->b_count, cap);
    e = e ? e : dalloc(&c->b_chunks, cap);
    e = e ? e : dalloc(&c->b_chunk_off, cap);
    e = e ? e : dalloc(&c->w_block, (size_t)c->work_cap);
    e = e ? e : dalloc(&c->w_start, (size_t)c->work_cap);
    e = e ? e : dalloc(&c->w_end, (size_t)c->work_cap);
    e = e ? e : dalloc(&c->grid, cap * NPB);
    if (c->adjoint) {
        e = e ? e : dalloc(&c->grid_u, cap * NPB);
        e = e ? e : dalloc(&c->grid_bar, cap * NPB);
    }
    e = e ? e : dalloc(&c->partials, (size_t)scan_partials_size(scan_n));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_capacity_buffers(c);
        return MPM_ERR_NOMEM;
    }
    fill_params(c);
    return MPM_OK;
}

bool particles_ok(const mpm_ctx* c, const mpm_particles* p, bool need_state) {
    if (!p || p->n < 0 || p->n > c->max_particles || !p->x) return false;
    if (need_state && (!p->v || !p->C || !p->F || !p->tau)) return false;
    return true;
}

int hip_status(hipError_t e) { return e == hipSuccess ? MPM_OK : MPM_ERR_HIP; }

int build_once(mpm_ctx* c, const mpm_particles* p, hipStream_t s) {
    const int n = p->n;
    hipError_t e = launch_bin(c->P, p->x, n, c->k1, s);
    if (e != hipSuccess) return MPM_ERR_HIP;
    uint32_t *ko = c->k1, *vo = c->v0;
    if (n > 0) {
        e = radix_sort(c->k1, c->k0, c->k1, c->v0, c->v1, n, c->key_bits, c->hist, c->partials, &ko, &vo, s);
        if (e != hipSuccess) return MPM_ERR_HIP;
    }
    c->skeys = ko;
    c->order = vo;
    if (c->dense)
        e = launch_build_dense(c->P, ko, n, (int)c->n_blocks_total, c->partials, s);
    else
        e = launch_build_sparse(c->P, ko, n, 1u << c->H_log2, c->partials, s);
    return hip_status(e);
}

int first_flag_code(unsigned f) {
    if (f & MPM_FLAG_OVERFLOW) return MPM_ERR_OVERFLOW;
    if (f & MPM_FLAG_DOMAIN) return MPM_ERR_DOMAIN;
    if (f & MPM_FLAG_INVERTED) return MPM_ERR_INVERTED;
    if (f & MPM_FLAG_NAN) return MPM_ERR_NAN;
    return MPM_OK;
}

int read_counters(mpm_ctx* c, hipStream_t s, DevCounters* out) {
    if (hipStreamSynchronize(s) != hipSuccess) return MPM_ERR_HIP;
    if (hipMemcpy(out, c->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost) != hipSuccess) return MPM_ERR_HIP;
    return MPM_OK;
}

}  // namespace

namespace mpmx {
__global__ void k_clear_flags(DevCounters* c) { c->flags = 0u; }
hipError_t launch_clear_flags(DevCounters* c, hipStream_t s) {
    k_clear_flags<<<1, 1, 0, s>>>(c);
    return hipGetLastError();
}
}  // namespace mpmx

extern "C" {

const char* mpm_status_string(int status) {
    switch (status) {
        case MPM_OK: return "MPM_OK";
        case MPM_ERR_ARG: return "MPM_ERR_ARG: invalid argument";
        case MPM_ERR_HIP: return "MPM_ERR_HIP: HIP runtime call failed";
        case MPM_ERR_NOMEM: return "MPM_ERR_NOMEM: device allocation failed";
        case MPM_ERR_OVERFLOW: return "MPM_ERR_OVERFLOW: hash table or block capacity exceeded";
        case MPM_ERR_DOMAIN: return "MPM_ERR_DOMAIN: particle support outside the grid";
        case MPM_ERR_INVERTED: return "MPM_ERR_INVERTED: deformation gradient with det <= 0";
        case MPM_ERR_NAN: return "MPM_ERR_NAN: non-finite value";
        case MPM_ERR_STATE: return "MPM_ERR_STATE: call out of order";
        default: return "unknown status";
    }
}

int mpm_create(const mpm_params* q, mpm_ctx** out) {
    if (!out) return MPM_ERR_ARG;
    *out = nullptr;
    if (!q) return MPM_ERR_ARG;
    if (q->dim != 2 && q->dim != 3) return MPM_ERR_ARG;
    if (!(q->dx > 0.0) || !(q->dt > 0.f) || q->max_particles < 1 || q->max_particles > (1 << 30)) return MPM_ERR_ARG;
    if (q->model != MPM_MODEL_ELASTIC && q->model != MPM_MODEL_DP) return MPM_ERR_ARG;
    if (!(q->E > 0.f) || !(q->nu >= 0.f && q->nu < 0.5f) || !(q->p_mass > 0.f) || !(q->p_vol0 > 0.f)) return MPM_ERR_ARG;
    if (q->grid_mode != MPM_GRID_SPARSE && q->grid_mode != MPM_GRID_DENSE) return MPM_ERR_ARG;
    if (q->heightmap && q->dim != 3) return MPM_ERR_ARG;
    if (q->heightmap && (q->flags & MPM_FLAG_ADJOINT)) return MPM_ERR_ARG;
    if (q->bound < 0 || q->block_capacity < 0 || q->hash_capacity_log2 < 0 || q->hash_capacity_log2 > 30)
        return MPM_ERR_ARG;
    for (int a = 0; a < q->dim; ++a) {
        if (q->cells[a] < 4 || q->cells[a] > (1 << 20)) return MPM_ERR_ARG;
        for (int sd = 0; sd < 2; ++sd)
            if (q->bc[a][sd] < MPM_BC_NONE || q->bc[a][sd] > MPM_BC_SEPARATE) return MPM_ERR_ARG;
    }
    mpm_ctx* c = new (std::nothrow) mpm_ctx();
    if (!c) return MPM_ERR_NOMEM;
    c->prm = *q;
    c->prm.heightmap = nullptr;
    c->dim = q->dim;
    c->dense = q->grid_mode == MPM_GRID_DENSE;
    c->adjoint = (q->flags & MPM_FLAG_ADJOINT) != 0;
    c->max_particles = q->max_particles;
    long long total = 1;
    for (int a = 0; a < 3; ++a) {
        c->nblk[a] = a < c->dim ? (q->cells[a] + 1 + BLK - 1) / BLK : 1;
        total *= c->nblk[a];
    }
    c->n_blocks_total = total;
    c->key_bits = bits_for(total - 1) + 2 * c->dim;
    if (c->key_bits > 32 || total > (1ll << 30)) {
        delete c;
        return MPM_ERR_ARG;
    }
    if (c->dense) {
        c->block_cap = (int)total;
    } else {
        long long def = std::max(4096ll, 2ll * q->max_particles / (1 << (2 * c->dim)) + 4096ll);
        long long cap = q->block_capacity > 0 ? q->block_capacity : def;
        c->block_cap = (int)std::min(cap, total + 0ll);
    }
    {
        int hl = q->hash_capacity_log2;
        if (hl == 0) {
            hl = 10;
            while ((1ll << hl) < 2ll * c->block_cap) ++hl;
        }
        c->H_log2 = hl;
    }
    if (const char* ch = getenv("MPMX_CHUNK")) {
        int v = atoi(ch);
        if (v >= 32 && v <= 512) c->chunk = v;
    }
    if (const char* pw = getenv("MPMX_WGS")) {
        int v = atoi(pw);
        if (v >= 1 && v <= 1 << 20) c->persistent_wgs = v;
    }
    hipError_t e = hipSuccess;
    const size_t np = (size_t)q->max_particles;
    e = e ? e : dalloc(&c->k0, np);
    e = e ? e : dalloc(&c->k1, np);
    e = e ? e : dalloc(&c->v0, np);
    e = e ? e : dalloc(&c->v1, np);
    e = e ? e : dalloc(&c->hist, (size_t)radix_hist_size(q->max_particles));
    e = e ? e : dalloc(&c->ctr, 1);
    if (c->adjoint) e = e ? e : dalloc(&c->adj_scratch, np * (size_t)(c->dim + 2 * c->dim * c->dim));
    if (e == hipSuccess && q->heightmap) {
        const size_t hn = (size_t)(q->cells[0] + 1) * (size_t)(q->cells[1] + 1);
        e = dalloc(&c->heightmap, hn);
        if (e == hipSuccess) e = hipMemcpy(c->heightmap, q->heightmap, hn * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(c->ctr, 0, sizeof(DevCounters));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_all(c);
        delete c;
        return MPM_ERR_NOMEM;
    }
    int st = alloc_capacity_buffers(c);
    if (st != MPM_OK) {
        free_all(c);
        delete c;
        return st;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        free_all(c);
        delete c;
        return MPM_ERR_HIP;
    }
    *out = c;
    return MPM_OK;
}

int mpm_destroy(mpm_ctx* c) {
    if (!c) return MPM_ERR_ARG;
    (void)hipDeviceSynchronize();
    free_all(c);
    delete c;
    return MPM_OK;
}

int mpm_set_material(mpm_ctx* c, float E, float nu, float friction_deg, float dt) {
    if (!c || !(E > 0.f) || !(nu >= 0.f && nu < 0.5f) || !(dt > 0.f)) return MPM_ERR_ARG;
    c->prm.E = E;
    c->prm.nu = nu;
    c->prm.friction_deg = friction_deg;
    c->prm.dt = dt;
    fill_material(c);
    return MPM_OK;
}

int mpm_sparse_build(mpm_ctx* c, const mpm_particles* p, void* stream) {
    if (!c || !particles_ok(c, p, false)) return MPM_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    int st = build_once(c, p, s);
    if (st != MPM_OK) return st;
    if (!c->dense && (c->prm.flags & MPM_FLAG_SYNC_REBUILD)) {
        // Algorithm 7: on overflow, double the table (and the block capacity)
        // and insert again until nothing overflows.
        for (int attempt = 0; attempt < 24; ++attempt) {
            DevCounters h;
            st = read_counters(c, s, &h);
            if (st != MPM_OK) return st;
            if (!(h.flags & MPM_FLAG_OVERFLOW)) break;
            const long long want = std::max<long long>(2ll * c->block_cap, (long long)h.n_touched);
            c->block_cap = (int)std::min<long long>(want, c->n_blocks_total);
            if (c->H_log2 < 30) ++c->H_log2;
            while ((1ll << c->H_log2) < 2ll * c->block_cap && c->H_log2 < 30) ++c->H_log2;
            st = alloc_capacity_buffers(c);
            if (st != MPM_OK) return st;
            unsigned keep = h.flags & ~MPM_FLAG_OVERFLOW;
            if (hipMemcpyAsync(&c->ctr->flags, &keep, sizeof(unsigned), hipMemcpyHostToDevice, s) != hipSuccess)
                return MPM_ERR_HIP;
            if (hipStreamSynchronize(s) != hipSuccess) return MPM_ERR_HIP;
            st = build_once(c, p, s);
            if (st != MPM_OK) return st;
        }
    }
    c->built = true;
    c->built_n = p->n;
    return MPM_OK;
}

int mpm_p2g(mpm_ctx* c, const mpm_particles* p, void* stream) {
    if (!c || !particles_ok(c, p, true)) return MPM_ERR_ARG;
    if (!c->built || p->n != c->built_n) return MPM_ERR_STATE;
    if (p->n == 0) return MPM_OK;
    const int wgs = std::min(c->persistent_wgs, c->work_cap);
    return hip_status(launch_p2g(c->P, p->x, p->v, p->C, p->tau, p->n, c->order, c->skeys, wgs, (hipStream_t)stream));
}

int mpm_grid_update(mpm_ctx* c, void* stream) {
    if (!c) return MPM_ERR_ARG;
    if (!c->built) return MPM_ERR_STATE;
    const long long NPB = 1ll << (2 * c->dim);
    const long long nodes = (long long)c->block_cap * NPB;
    long long wgs = (nodes + WG - 1) / WG;
    wgs = std::min<long long>(wgs, c->dense ? 65536 : 8192);
    return hip_status(launch_grid_update(c->P, c->dense ? nodes : -1, (int)std::max(1ll, wgs), (hipStream_t)stream));
}

int mpm_g2p(mpm_ctx* c, const mpm_particles* in, const mpm_particles* out, void* stream) {
    if (!c || !particles_ok(c, in, false) || !out || !out->x || !out->v || !out->C || !out->F || !out->tau ||
        !in->F || out->n != in->n)
        return MPM_ERR_ARG;
    if (in->x == out->x || in->F == out->F) return MPM_ERR_ARG;
    if (!c->built || in->n != c->built_n) return MPM_ERR_STATE;
    if (in->n == 0) return MPM_OK;
    const int wgs = std::min(c->persistent_wgs, c->work_cap);
    return hip_status(launch_g2p(c->P, in->x, in->F, in->id, out->x, out->v, out->C, out->F, out->tau, out->id, in->n,
                                 c->order, wgs, (hipStream_t)stream));
}

int mpm_step(mpm_ctx* c, const mpm_particles* a, const mpm_particles* b, int n_steps, void* stream) {
    if (!c || !a || !b || n_steps < 0 || a->n != b->n) return MPM_ERR_ARG;
    const mpm_particles* cur = a;
    const mpm_particles* nxt = b;
    for (int k = 0; k < n_steps; ++k) {
        int st = mpm_sparse_build(c, cur, stream);
        if (st == MPM_OK) st = mpm_p2g(c, cur, stream);
        if (st == MPM_OK) st = mpm_grid_update(c, stream);
        if (st == MPM_OK) st = mpm_g2p(c, cur, nxt, stream);
        if (st != MPM_OK) return st;
        std::swap(cur, nxt);
    }
    return MPM_OK;
}

int mpm_g2p_adj(mpm_ctx* c, const mpm_particles* in, const mpm_particles* ob, const mpm_particles* ib,
                float* param_bar, void* stream) {
    if (!c || !particles_ok(c, in, false) || !in->F || !ob || !ib || !param_bar) return MPM_ERR_ARG;
    if (!ob->x || !ob->v || !ob->C || !ob->F || !ob->tau || !ib->x || !ib->F) return MPM_ERR_ARG;
    if (ob->n != in->n || ib->n != in->n) return MPM_ERR_ARG;
    if (!c->adjoint || !c->built || in->n != c->built_n) return MPM_ERR_STATE;
    if (in->n == 0) return MPM_OK;
    DevParams P = c->P;
    P.param_bar = param_bar;
    const float* obp[5] = {ob->x, ob->v, ob->C, ob->F, ob->tau};
    const int wgs = std::min(c->persistent_wgs, c->work_cap);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_g2p_adj(P, in->x, in->F, obp, ib->x, ib->F, in->n, c->order, wgs, s);
    if (e == hipSuccess) e = launch_scatter_adj(P, in->x, in->n, c->order, c->skeys, wgs, s);
    return hip_status(e);
}

int mpm_grid_update_adj(mpm_ctx* c, void* stream) {
    if (!c) return MPM_ERR_ARG;
    if (!c->adjoint || !c->built) return MPM_ERR_STATE;
    const long long NPB = 1ll << (2 * c->dim);
    const long long nodes = (long long)c->block_cap * NPB;
    long long wgs = std::min<long long>((nodes + WG - 1) / WG, c->dense ? 65536 : 8192);
    return hip_status(launch_grid_adj(c->P, c->dense ? nodes : -1, (int)std::max(1ll, wgs), (hipStream_t)stream));
}

int mpm_p2g_adj(mpm_ctx* c, const mpm_particles* in, const mpm_particles* ib, void* stream) {
    if (!c || !particles_ok(c, in, true) || !ib || ib->n != in->n) return MPM_ERR_ARG;
    if (!ib->x || !ib->v || !ib->C || !ib->tau) return MPM_ERR_ARG;
    if (!c->adjoint || !c->built || in->n != c->built_n) return MPM_ERR_STATE;
    if (in->n == 0) return MPM_OK;
    const float* inp[4] = {in->x, in->v, in->C, in->tau};
    float* ibp[4] = {ib->x, ib->v, ib->C, ib->tau};
    const int wgs = std::min(c->persistent_wgs, c->work_cap);
    return hip_status(launch_p2g_adj(c->P, inp, ibp, in->n, c->order, wgs, (hipStream_t)stream));
}

int mpm_step_adj(mpm_ctx* c, const mpm_particles* in, const mpm_particles* ob, const mpm_particles* ib,
                 float* param_bar, void* stream) {
    if (!c) return MPM_ERR_ARG;
    if (!c->adjoint) return MPM_ERR_STATE;
    int st = mpm_sparse_build(c, in, stream);
    if (st == MPM_OK) st = mpm_p2g(c, in, stream);
    if (st == MPM_OK) st = mpm_grid_update(c, stream);
    if (st == MPM_OK) st = mpm_g2p_adj(c, in, ob, ib, param_bar, stream);
    if (st == MPM_OK) st = mpm_grid_update_adj(c, stream);
    if (st == MPM_OK) st = mpm_p2g_adj(c, in, ib, stream);
    return st;
}

int mpm_get_status(mpm_ctx* c, void* stream, uint32_t* flags) {
    if (!c) return MPM_ERR_ARG;
    DevCounters h;
    int st = read_counters(c, (hipStream_t)stream, &h);
    if (st != MPM_OK) return st;
    if (flags) *flags = h.flags;
    return first_flag_code(h.flags);
}

int mpm_clear_status(mpm_ctx* c, void* stream) {
    if (!c) return MPM_ERR_ARG;
    return hip_status(launch_clear_flags(c->ctr, (hipStream_t)stream));
}

int mpm_active_count(mpm_ctx* c, void* stream, int* n_blocks, int* n_touched) {
    if (!c) return MPM_ERR_ARG;
    DevCounters h;
    int st = read_counters(c, (hipStream_t)stream, &h);
    if (st != MPM_OK) return st;
    if (n_blocks) *n_blocks = h.nb;
    if (n_touched) *n_touched = h.n_touched;
    return MPM_OK;
}

int mpm_get_active(mpm_ctx* c, uint64_t* keys, uint64_t* masks, int capacity, void* stream) {
    if (!c || !keys || !masks || capacity < 0) return MPM_ERR_ARG;
    if (c->dense) return MPM_ERR_STATE;
    if (!c->built) return MPM_ERR_STATE;
    if (capacity == 0) return MPM_OK;
    return hip_status(launch_copy_active(c->P, keys, masks, capacity, (hipStream_t)stream));
}

int mpm_get_grid(mpm_ctx* c, float* out, int capacity_blocks, void* stream) {
    if (!c || !out || capacity_blocks < 0) return MPM_ERR_ARG;
    if (!c->built) return MPM_ERR_STATE;
    const size_t nblk = (size_t)std::min(capacity_blocks, c->block_cap);
    const size_t bytes = nblk * ((size_t)1 << (2 * c->dim)) * sizeof(float4);
    if (bytes == 0) return MPM_OK;
    return hip_status(hipMemcpyAsync(out, c->grid, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

int mpm_get_order(mpm_ctx* c, uint32_t* order, int n, void* stream) {
    if (!c || !order || n < 0) return MPM_ERR_ARG;
    if (!c->built || n != c->built_n) return MPM_ERR_STATE;
    if (n == 0) return MPM_OK;
    return hip_status(
        hipMemcpyAsync(order, c->order, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

}  // extern "C"
