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
#include <vector>

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
    int p2g_wgs = 8192;     // persistent workgroups of the P2G launch
    int g2p_wgs = 8192;     // persistent workgroups of the G2P launch
    int g2p_block = 256;    // threads per G2P workgroup (work items of at most g2p_max_items of it)
    int n_inst = 1;
    int blk_bits = 0;
    InstMat* inst = nullptr;  // device table of per-instance constants (ensembles)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
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
    float4* tiles = nullptr;
    int* b_lo = nullptr;
    float4* grid_u = nullptr;
    float4* grid_bar = nullptr;
    float* adj_scratch = nullptr;
    bool adjoint = false;
    float* heightmap = nullptr;
    DevCounters* ctr = nullptr;
    DevParams P{};
    bool built = false;
    int built_n = -1;
    // incremental re-sort: the block segments, hash table and sorted keys of
    // the last build (for seg_n particles) are intact and may seed the next sort
    bool seg_valid = false;
    int seg_n = -1;
    uint32_t *rs_stay = nullptr, *rs_in = nullptr, *rs_off = nullptr, *rs_oldblk = nullptr;
    unsigned *rs_cnt = nullptr, *rs_start = nullptr;
    uint64_t* nh_keys = nullptr;
    uint32_t* nh_cnt = nullptr;
    int* nh_idx = nullptr;
    uint32_t* nh_owner = nullptr;
    uint32_t* rs_new = nullptr;
    int* h_entry = nullptr;
    int* b_entry = nullptr;
    uint32_t* order = nullptr;
    uint32_t* skeys = nullptr;
    uint32_t* osrc = nullptr;  // G2P output position -> input index (the spare sort value buffer)
    uint32_t* movers = nullptr;  // incremental re-sort: particles that changed owner block
    // scan-based construction (MPM_FLAG_SCAN_BUILD): mask-domain scratch for
    // every block of the potential domain, allocated at create
    bool scan_build = false;
    void* sb_mem = nullptr;
    int* sb_seg = nullptr;
    SbScratch sb{};
    // ascending-key Phi order (MPM_FLAG_DETERMINISTIC_ORDER, hash builds)
    bool det_order = false;
    DetTables det{};
    // Reverse-mode tape: for each step of a recorded segment, what its adjoint
    // reads from the step's build and transfers (block and work tables, both
    // grids, counters, sorted keys and order).
    struct TapeSlot {
        uint64_t* b_keys = nullptr;
        int *b_nbr = nullptr, *b_start = nullptr, *b_count = nullptr;
        int *w_block = nullptr, *w_start = nullptr, *w_end = nullptr;
        float4 *grid = nullptr, *grid_u = nullptr;
        uint32_t *order = nullptr, *skeys = nullptr;
    };
    std::vector<TapeSlot> tape;
    DevCounters* tape_ctr = nullptr;  // one per slot
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
    dfree(c->tiles);
    dfree(c->b_lo);
    dfree(c->grid_u);
    dfree(c->grid_bar);
    dfree(c->partials);
    dfree(c->rs_stay);
    dfree(c->rs_in);
    dfree(c->rs_off);
    dfree(c->rs_oldblk);
    dfree(c->rs_cnt);
    dfree(c->rs_start);
    dfree(c->nh_keys);
    dfree(c->nh_cnt);
    dfree(c->nh_idx);
    dfree(c->nh_owner);
    dfree(c->rs_new);
    dfree(c->h_entry);
    dfree(c->b_entry);
    dfree(c->det.keys);
    dfree(c->det.mask);
    dfree(c->det.start);
    dfree(c->det.count);
    dfree(c->det.slot);
    for (int j = 0; j < 2; ++j) {
        dfree(c->det.k[j]);
        dfree(c->det.v[j]);
    }
    dfree(c->det.hist);
    c->seg_valid = false;
}

void free_tape(mpm_ctx* c) {
    for (auto& t : c->tape) {
        dfree(t.b_keys);
        dfree(t.b_nbr);
        dfree(t.b_start);
        dfree(t.b_count);
        dfree(t.w_block);
        dfree(t.w_start);
        dfree(t.w_end);
        dfree(t.grid);
        dfree(t.grid_u);
        dfree(t.order);
        dfree(t.skeys);
    }
    c->tape.clear();
    dfree(c->tape_ctr);
}

void free_all(mpm_ctx* c) {
    free_tape(c);
    free_capacity_buffers(c);
    dfree(c->k0);
    dfree(c->k1);
    dfree(c->v0);
    dfree(c->v1);
    dfree(c->hist);
    dfree(c->heightmap);
    dfree(c->adj_scratch);
    dfree(c->inst);
    dfree(c->ctr);
    dfree(c->movers);
    if (c->sb_mem) (void)hipFree(c->sb_mem);
    c->sb_mem = nullptr;
    dfree(c->sb_seg);
}

void release_graph(mpm_ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

// Material constants of one simulation: Lame parameters, the Drucker-Prager
// cone coefficient alpha = sqrt(2/3) 2 sin(phi) / (3 - sin(phi)) and its
// derivative in degrees, and (d lambda + 2 mu) / (2 mu).
InstMat make_instmat(int dim, double E, double nu, double friction_deg, float dt, float p_mass, float p_vol0) {
    InstMat m{};
    const double mu = E / (2.0 * (1.0 + nu));
    const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double phi = friction_deg * M_PI / 180.0;
    const double sphi = sin(phi);
    m.mu = (float)mu;
    m.lam = (float)lam;
    m.alpha = (float)(sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi));
    m.dp_coef = (float)((dim * lam + 2.0 * mu) / (2.0 * mu));
    m.dt = dt;
    m.p_mass = p_mass;
    m.p_vol0 = p_vol0;
    m.E = (float)E;
    m.dalpha_dphi = (float)(sqrt(2.0 / 3.0) * 6.0 * cos(phi) / ((3.0 - sphi) * (3.0 - sphi)) * (M_PI / 180.0));
    return m;
}

void fill_material(mpm_ctx* c) {
    const InstMat m = make_instmat(c->dim, c->prm.E, c->prm.nu, c->prm.friction_deg, c->prm.dt, c->prm.p_mass,
                                   c->prm.p_vol0);
    c->P.mu = m.mu;
    c->P.lam = m.lam;
    c->P.alpha = m.alpha;
    c->P.dp_coef = m.dp_coef;
    c->P.dt = m.dt;
    c->P.E = m.E;
    c->P.dalpha_dphi = m.dalpha_dphi;
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
    P.tiles = c->tiles;
    P.b_lo = c->b_lo;
    P.ctr = c->ctr;
    P.grid_u = c->grid_u;
    P.grid_bar = c->grid_bar;
    P.adj_scratch = c->adj_scratch;
    P.param_bar = nullptr;
    P.n_inst = c->n_inst;
    P.blk_bits = c->blk_bits;
    P.inst = c->inst;
    P.rs_stay = c->rs_stay;
    P.rs_in = c->rs_in;
    P.rs_off = c->rs_off;
    P.rs_cnt = c->rs_cnt;
    P.rs_start = c->rs_start;
    P.rs_oldblk = c->rs_oldblk;
    P.nh_keys = c->nh_keys;
    P.nh_cnt = c->nh_cnt;
    P.nh_idx = c->nh_idx;
    P.nh_owner = c->nh_owner;
    P.rs_new = c->rs_new;
    P.h_entry = c->h_entry;
    P.b_entry = c->b_entry;
    fill_material(c);
}

// (Re)allocate every buffer whose size depends on block_cap or H.
int alloc_capacity_buffers(mpm_ctx* c) {
    free_tape(c);  // sized by the capacities
    free_capacity_buffers(c);
    const int NB = 1 << c->dim, NPB = 1 << (2 * c->dim);
    const size_t H = (size_t)1 << c->H_log2;
    const size_t cap = (size_t)c->block_cap;
    // room for the smallest work-item size mpm_set_tuning accepts
    c->work_cap = c->block_cap + c->max_particles / MIN_CHUNK + 1;
    // (the hash compaction keeps two tile sums per tile of the table)
    int scan_n = std::max({radix_hist_size(c->max_particles), radix_hist_size(c->block_cap), (int)(2 * H),
                           2 * c->block_cap, 1});
    // the incremental re-sort serves hash-built sparse contexts whose particle
    // order may depend on earlier builds
    const bool resort = !c->dense && !c->adjoint && !c->scan_build && !c->det_order;
    const bool hashed = !c->dense && !c->scan_build;
    hipError_t e = hipSuccess;
    if (hashed) {
        e = e ? e : dalloc(&c->h_keys, H);
        e = e ? e : dalloc(&c->h_mask, H);
        e = e ? e : dalloc(&c->h_vals, H);
        e = e ? e : dalloc(&c->h_start, H);
        e = e ? e : dalloc(&c->h_end, H);
    }
    if (!c->dense) {
        e = e ? e : dalloc(&c->b_keys, cap);
        e = e ? e : dalloc(&c->b_mask, cap);
    }
    if (hashed && c->det_order) {
        e = e ? e : dalloc(&c->det.keys, cap);
        e = e ? e : dalloc(&c->det.mask, cap);
        e = e ? e : dalloc(&c->det.start, cap);
        e = e ? e : dalloc(&c->det.count, cap);
        e = e ? e : dalloc(&c->det.slot, cap);
        for (int j = 0; j < 2; ++j) {
            e = e ? e : dalloc(&c->det.k[j], cap);
            e = e ? e : dalloc(&c->det.v[j], cap);
        }
        e = e ? e : dalloc(&c->det.hist, (size_t)radix_hist_size(c->block_cap));
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
    if (!c->dense) {
        const size_t tile_nodes = c->dim == 3 ? 216 : 36;
        e = e ? e : dalloc(&c->tiles, cap * tile_nodes);
        e = e ? e : dalloc(&c->b_lo, cap * NB);
    }
    if (c->adjoint) {
        e = e ? e : dalloc(&c->grid_u, cap * NPB);
        e = e ? e : dalloc(&c->grid_bar, cap * NPB);
    }
    e = e ? e : dalloc(&c->partials, (size_t)scan_partials_size(scan_n));
    if (resort) {
        e = e ? e : dalloc(&c->rs_stay, cap * NPB);
        e = e ? e : dalloc(&c->rs_in, 2 * cap * NPB);
        e = e ? e : dalloc(&c->rs_off, 2 * cap * NPB);
        e = e ? e : dalloc(&c->rs_oldblk, 2 * cap);
        e = e ? e : dalloc(&c->rs_cnt, 2 * cap);
        e = e ? e : dalloc(&c->rs_start, 2 * cap);
        e = e ? e : dalloc(&c->nh_keys, H);
        e = e ? e : dalloc(&c->nh_cnt, H * NPB);
        e = e ? e : dalloc(&c->nh_idx, H);
        e = e ? e : dalloc(&c->nh_owner, H);
        e = e ? e : dalloc(&c->rs_new, cap);
        e = e ? e : dalloc(&c->h_entry, H);
        e = e ? e : dalloc(&c->b_entry, cap);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_capacity_buffers(c);
        return MPM_ERR_NOMEM;
    }
    fill_params(c);
    if (resort) {
        // zeroed mover counters and an empty second table, as every re-sort leaves them
        e = launch_resort_init(c->P, (unsigned)H, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_capacity_buffers(c);
            return MPM_ERR_HIP;
        }
    }
    return MPM_OK;
}

bool particles_ok(const mpm_ctx* c, const mpm_particles* p, bool need_state) {
    if (!p || p->n < 0 || p->n > c->max_particles) return false;
    if (p->n == 0) return true;  // an empty set needs no arrays
    if (!p->x) return false;
    if (c->n_inst > 1 && !p->inst) return false;
    if (need_state && (!p->v || !p->C || !p->F || !p->tau)) return false;
    return true;
}

int hip_status(hipError_t e) { return e == hipSuccess ? MPM_OK : MPM_ERR_HIP; }

// Buffer that the binning of the next build writes (and that a G2P which
// bins its output writes instead): the key buffer the sorted keys of the
// current build do not occupy when the next build re-sorts incrementally, else
// k1 (free once P2G has read the sorted keys).
uint32_t* next_bin_buffer(const mpm_ctx* c, bool next_reuse) {
    if (next_reuse) return c->skeys == c->k0 ? c->k1 : c->k0;
    return c->k1;
}

// Whether a build of n particles following the last one re-sorts incrementally.
bool would_reuse(const mpm_ctx* c, int n) {
    return c->seg_valid && c->seg_n == n &&
           !(c->prm.flags & (MPM_FLAG_FULL_SORT | MPM_FLAG_DETERMINISTIC_ORDER | MPM_FLAG_SCAN_BUILD));
}

// One build.  `reuse`: the previous build's segments, hash table and sorted
// keys (same particle count) seed an incremental re-sort instead of the full
// radix sort; the new sorted keys then take the previous ones' buffer.
// `keys_ready`: the binning was already done (by the G2P that wrote these
// positions) into next_bin_buffer(c, reuse).
int build_once(mpm_ctx* c, const mpm_particles* p, hipStream_t s, bool reuse, bool keys_ready = false) {
    const int n = p->n;
    hipError_t e;
    uint32_t *ko = c->k1, *vo = c->v0;
    if (reuse && n > 0) {
        uint32_t* prev = c->skeys;
        uint32_t* fresh = prev == c->k0 ? c->k1 : c->k0;
        vo = c->order;
        if (!keys_ready) {
            e = launch_bin(c->P, p->x, p->inst, n, fresh, s);
            if (e != hipSuccess) return MPM_ERR_HIP;
        }
        // keys_ready: the G2P that binned also counted stayers and listed movers.
        // The sorted keys are not written: P2G reads each block's cell ranges
        // from the re-sort's table, and the next re-sort reads no previous key,
        // so the previous keys' buffer holds the movers' targets instead.
        e = launch_resort(c->P, fresh, nullptr, vo, c->movers, prev, n, 1u << c->H_log2, c->partials, s,
                          keys_ready);
        if (e != hipSuccess) return MPM_ERR_HIP;
        ko = prev;
    } else {
        if (!keys_ready) {
            e = launch_bin(c->P, p->x, p->inst, n, c->k1, s);
            if (e != hipSuccess) return MPM_ERR_HIP;
        }
        if (n > 0) {
            e = radix_sort(c->k1, c->k0, c->k1, c->v0, c->v1, n, c->key_bits, c->hist, c->partials, &ko, &vo, s);
            if (e != hipSuccess) return MPM_ERR_HIP;
        }
    }
    c->skeys = ko;
    c->order = vo;
    c->osrc = vo == c->v0 ? c->v1 : c->v0;
    if (c->dense)
        e = launch_build_dense(c->P, ko, n, (int)c->n_blocks_total, c->partials, s);
    else if (c->scan_build)
        e = launch_build_scan(c->P, ko, n, c->sb, c->partials, s);
    else
        e = launch_build_sparse(c->P, ko, n, 1u << c->H_log2, c->partials, s, reuse && n > 0,
                                c->det_order ? &c->det : nullptr);
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

// Points the context's build tables, grids and counters at tape slot j.
void bind_slot(mpm_ctx* c, int j) {
    const mpm_ctx::TapeSlot& t = c->tape[(size_t)j];
    c->P.b_keys = t.b_keys;
    c->P.b_nbr = t.b_nbr;
    c->P.b_start = t.b_start;
    c->P.b_count = t.b_count;
    c->P.w_block = t.w_block;
    c->P.w_start = t.w_start;
    c->P.w_end = t.w_end;
    c->P.grid = t.grid;
    c->P.grid_u = t.grid_u;
    c->P.ctr = c->tape_ctr + j;
}

// Checks shared by the tape calls: a sparse adjoint context with a tape of at
// least n_steps slots, n_steps + 1 distinct sets of one size.
int tape_args_ok(const mpm_ctx* c, const mpm_particles* states, int n_steps) {
    if (!c || !states || n_steps < 0) return MPM_ERR_ARG;
    if (!c->adjoint || c->dense || (c->prm.flags & MPM_FLAG_SYNC_REBUILD)) return MPM_ERR_STATE;
    if ((size_t)n_steps > c->tape.size()) return MPM_ERR_STATE;
    for (int j = 0; j <= n_steps; ++j) {
        if (!particles_ok(c, &states[j], true) || states[j].n != states[0].n) return MPM_ERR_ARG;
        if (j > 0 && states[0].n > 0 && (states[j].x == states[j - 1].x || states[j].F == states[j - 1].F))
            return MPM_ERR_ARG;
    }
    return MPM_OK;
}

}  // namespace

namespace {
// The build behind mpm_sparse_build; keys_ready as for build_once (a rebuild
// after an overflow bins again).
int sparse_build(mpm_ctx* c, const mpm_particles* p, hipStream_t s, bool keys_ready) {
    const bool reuse = would_reuse(c, p->n);
    c->built = false;
    c->seg_valid = false;
    int st = build_once(c, p, s, reuse, keys_ready);
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
            st = build_once(c, p, s, false);
            if (st != MPM_OK) return st;
        }
    }
    c->built = true;
    c->built_n = p->n;
    c->seg_valid = c->rs_in != nullptr;
    c->seg_n = p->n;
    return MPM_OK;
}
}  // namespace

namespace mpmx {
__global__ void k_clear_flags(DevCounters* c) { c->flags = 0u; }
hipError_t launch_clear_flags(DevCounters* c, hipStream_t s) {
    k_clear_flags<<<1, 1, 0, s>>>(c);
    return hipGetLastError();
}
// ORs the status flags of the tape slots [0, n) into the context's counters
// and clears them.
__global__ void k_merge_tape_flags(DevCounters* dst, DevCounters* slots, int n) {
    unsigned f = 0u;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        f |= slots[i].flags;
        slots[i].flags = 0u;
    }
    if (f) atomicOr(&dst->flags, f);
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
    if (!(q->dx > 0.0) || !(q->dt > 0.f) || q->max_particles < 1 || q->max_particles >= (1 << 30)) return MPM_ERR_ARG;
    if (q->model != MPM_MODEL_ELASTIC && q->model != MPM_MODEL_DP) return MPM_ERR_ARG;
    if (!(q->E > 0.f) || !(q->nu >= 0.f && q->nu < 0.5f) || !(q->p_mass > 0.f) || !(q->p_vol0 > 0.f)) return MPM_ERR_ARG;
    if (q->grid_mode != MPM_GRID_SPARSE && q->grid_mode != MPM_GRID_DENSE) return MPM_ERR_ARG;
    if (q->heightmap && q->dim != 3) return MPM_ERR_ARG;
    if (q->heightmap && (q->flags & MPM_FLAG_ADJOINT)) return MPM_ERR_ARG;
    if (q->bound < 0 || q->block_capacity < 0 || q->hash_capacity_log2 < 0 || q->hash_capacity_log2 > 30)
        return MPM_ERR_ARG;
    if (q->n_instances < 0 || q->n_instances > MAX_INSTANCES) return MPM_ERR_ARG;
    const int n_inst = std::max(1, q->n_instances);
    if ((q->flags & MPM_FLAG_DETERMINISTIC_ORDER) && q->grid_mode != MPM_GRID_SPARSE) return MPM_ERR_ARG;
    if ((q->flags & MPM_FLAG_SCAN_BUILD) &&
        (q->grid_mode != MPM_GRID_SPARSE || n_inst > 1 || (q->flags & MPM_FLAG_ADJOINT)))
        return MPM_ERR_ARG;
    if (n_inst > 1) {
        if (!q->instances || q->grid_mode != MPM_GRID_SPARSE || (q->flags & MPM_FLAG_ADJOINT)) return MPM_ERR_ARG;
        for (int i = 0; i < n_inst; ++i) {
            const mpm_instance& m = q->instances[i];
            if (!(m.E > 0.f) || !(m.nu >= 0.f && m.nu < 0.5f) || !(m.dt > 0.f) || !(m.p_mass > 0.f) ||
                !(m.p_vol0 > 0.f))
                return MPM_ERR_ARG;
        }
    }
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
    c->scan_build = (q->flags & MPM_FLAG_SCAN_BUILD) != 0;
    c->det_order = (q->flags & MPM_FLAG_DETERMINISTIC_ORDER) != 0;
    c->max_particles = q->max_particles;
    long long total = 1;
    for (int a = 0; a < 3; ++a) {
        c->nblk[a] = a < c->dim ? (q->cells[a] + 1 + BLK - 1) / BLK : 1;
        total *= c->nblk[a];
    }
    c->n_blocks_total = total;
    c->n_inst = n_inst;
    c->blk_bits = bits_for(total - 1);
    // sort key: instance | linear block | local cell, all in 32 bits
    c->key_bits = (n_inst > 1 ? bits_for(n_inst - 1) : 0) + c->blk_bits + 2 * c->dim;
    bool fits = c->key_bits <= 32 && total <= (1ll << 30);
    if (n_inst > 1)  // ensemble block keys hold 19-bit biased coordinates (block -1 .. nblk)
        for (int a = 0; a < c->dim; ++a) fits = fits && c->nblk[a] < (int)ENS_KEY_BIAS - 1;
    if (!fits) {
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
        if (v >= MIN_CHUNK && v <= MAX_CHUNK) c->chunk = v;
    }
    if (const char* pw = getenv("MPMX_WGS")) {
        int v = atoi(pw);
        if (v >= 1 && v <= 1 << 20) c->p2g_wgs = c->g2p_wgs = v;
    }
    hipError_t e = hipSuccess;
    const size_t np = (size_t)q->max_particles;
    e = e ? e : dalloc(&c->k0, np);
    e = e ? e : dalloc(&c->k1, np);
    e = e ? e : dalloc(&c->v0, np);
    e = e ? e : dalloc(&c->v1, np);
    e = e ? e : dalloc(&c->hist, (size_t)radix_hist_size(q->max_particles));
    if (!c->dense && !c->adjoint && !c->scan_build && !c->det_order) e = e ? e : dalloc(&c->movers, np);
    e = e ? e : dalloc(&c->ctr, 1);
    if (c->adjoint) e = e ? e : dalloc(&c->adj_scratch, np * (size_t)(c->dim + 2 * c->dim * c->dim));
    if (e == hipSuccess && q->heightmap) {
        const size_t hn = (size_t)(q->cells[0] + 1) * (size_t)(q->cells[1] + 1);
        e = dalloc(&c->heightmap, hn);
        if (e == hipSuccess) e = hipMemcpy(c->heightmap, q->heightmap, hn * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(c->ctr, 0, sizeof(DevCounters));
    if (e == hipSuccess && c->scan_build) {
        const long long mm = c->n_blocks_total;
        e = hipMalloc(&c->sb_mem, sb_scratch_bytes(mm));
        if (e == hipSuccess) e = dalloc(&c->sb_seg, (size_t)(2 * mm));
        if (e == hipSuccess) c->sb = sb_carve(c->sb_mem, mm, c->sb_seg, c->sb_seg + mm);
    }
    if (e == hipSuccess && n_inst > 1) {
        InstMat host[MAX_INSTANCES];
        for (int i = 0; i < n_inst; ++i) {
            const mpm_instance& m = q->instances[i];
            host[i] = make_instmat(c->dim, m.E, m.nu, m.friction_deg, m.dt, m.p_mass, m.p_vol0);
        }
        e = dalloc(&c->inst, (size_t)n_inst);
        if (e == hipSuccess) e = hipMemcpy(c->inst, host, n_inst * sizeof(InstMat), hipMemcpyHostToDevice);
    }
    c->prm.instances = nullptr;
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
    release_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    free_all(c);
    delete c;
    return MPM_OK;
}

int mpm_set_material(mpm_ctx* c, float E, float nu, float friction_deg, float dt) {
    if (!c || !(E > 0.f) || !(nu >= 0.f && nu < 0.5f) || !(dt > 0.f)) return MPM_ERR_ARG;
    if (c->n_inst > 1) return MPM_ERR_STATE;
    c->prm.E = E;
    c->prm.nu = nu;
    c->prm.friction_deg = friction_deg;
    c->prm.dt = dt;
    fill_material(c);
    return MPM_OK;
}


int mpm_sparse_build(mpm_ctx* c, const mpm_particles* p, void* stream) {
    if (!c || !particles_ok(c, p, false)) return MPM_ERR_ARG;
    return sparse_build(c, p, (hipStream_t)stream, false);
}

namespace {
// mpm_p2g; with `update` (sparse grids) P2G's second pass also applies the grid
// update, so the grid holds velocities afterwards.
int p2g_impl(mpm_ctx* c, const mpm_particles* p, hipStream_t s, bool update) {
    if (!c || !particles_ok(c, p, true)) return MPM_ERR_ARG;
    if (!c->built || p->n != c->built_n) return MPM_ERR_STATE;
    if (p->n == 0) return MPM_OK;
    const int wgs = std::min(c->p2g_wgs, c->work_cap);
    return hip_status(
        launch_p2g(c->P, p->x, p->v, p->C, p->tau, p->n, c->order, c->skeys, c->osrc, wgs, s, update));
}
}  // namespace

int mpm_p2g(mpm_ctx* c, const mpm_particles* p, void* stream) {
    return p2g_impl(c, p, (hipStream_t)stream, false);
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

namespace {
// mpm_g2p; with keys_out, the kernel also bins the positions it writes (the
// next build then skips its binning pass).
int g2p_impl(mpm_ctx* c, const mpm_particles* in, const mpm_particles* out, hipStream_t s, uint32_t* keys_out,
             uint32_t* movers_out) {
    if (!c || !particles_ok(c, in, false) || !out || out->n != in->n) return MPM_ERR_ARG;
    if (in->n > 0) {
        if (!out->x || !out->v || !out->C || !out->F || !out->tau || !in->F) return MPM_ERR_ARG;
        if (in->x == out->x || in->F == out->F) return MPM_ERR_ARG;
        if (c->n_inst > 1 && (!out->inst || out->inst == in->inst)) return MPM_ERR_ARG;
    }
    if (!c->built || in->n != c->built_n) return MPM_ERR_STATE;
    if (in->n == 0) return MPM_OK;
    const int wgs = std::min(c->g2p_wgs, c->work_cap);
    return hip_status(launch_g2p(c->P, in->x, in->F, in->id, in->inst, out->x, out->v, out->C, out->F, out->tau,
                                 out->id, out->inst, in->n, c->osrc, c->g2p_block, wgs, s, keys_out, movers_out));
}
}  // namespace

int mpm_g2p(mpm_ctx* c, const mpm_particles* in, const mpm_particles* out, void* stream) {
    return g2p_impl(c, in, out, (hipStream_t)stream, nullptr, nullptr);
}

int mpm_step(mpm_ctx* c, const mpm_particles* a, const mpm_particles* b, int n_steps, void* stream) {
    if (!c || !a || !b || n_steps < 0 || a->n != b->n) return MPM_ERR_ARG;
    if (!particles_ok(c, a, true) || !particles_ok(c, b, true)) return MPM_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const mpm_particles* cur = a;
    const mpm_particles* nxt = b;
    bool keys_ready = false;  // the previous step's G2P binned the positions it wrote
    for (int k = 0; k < n_steps; ++k) {
        int st = sparse_build(c, cur, s, keys_ready);
        // on a sparse grid the grid update runs inside P2G's second pass (the
        // grid between the two is not visible to the caller here; reverse-mode
        // contexts keep the separate calls their tape repeats); with zero
        // particles the grid update still runs on its own
        const bool fuse_update = !c->dense && !c->adjoint && cur->n > 0;
        if (st == MPM_OK) st = p2g_impl(c, cur, s, fuse_update);
        if (st == MPM_OK && !fuse_update) st = mpm_grid_update(c, stream);
        // Between two steps of this call nothing else touches the positions,
        // so G2P bins them as it writes them.  Not in reverse-mode contexts,
        // whose tape records each build as mpm_sparse_build makes it.
        keys_ready = k + 1 < n_steps && !c->adjoint && cur->n > 0;
        const bool next_reuse = would_reuse(c, nxt->n);
        uint32_t* keys_out = keys_ready ? next_bin_buffer(c, next_reuse) : nullptr;
        // with an incremental re-sort next, G2P also does its counting
        uint32_t* movers_out = keys_ready && next_reuse ? c->movers : nullptr;
        if (st == MPM_OK) st = g2p_impl(c, cur, nxt, s, keys_out, movers_out);
        if (st != MPM_OK) return st;
        std::swap(cur, nxt);
    }
    return MPM_OK;
}

int mpm_g2p_adj(mpm_ctx* c, const mpm_particles* in, const mpm_particles* ob, const mpm_particles* ib,
                float* param_bar, void* stream) {
    if (!c || !particles_ok(c, in, false) || !ob || !ib || !param_bar) return MPM_ERR_ARG;
    if (in->n > 0 && (!in->F || !ob->x || !ob->v || !ob->C || !ob->F || !ob->tau || !ib->x || !ib->F))
        return MPM_ERR_ARG;
    if (ob->n != in->n || ib->n != in->n) return MPM_ERR_ARG;
    if (!c->adjoint || !c->built || in->n != c->built_n) return MPM_ERR_STATE;
    if (in->n == 0) return MPM_OK;
    DevParams P = c->P;
    P.param_bar = param_bar;
    const float* obp[5] = {ob->x, ob->v, ob->C, ob->F, ob->tau};
    const int wgs = std::min(c->g2p_wgs, c->work_cap);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_g2p_adj(P, in->x, in->F, obp, ib->x, ib->F, in->n, c->order, c->skeys, wgs, s);
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
    if (in->n > 0 && (!ib->x || !ib->v || !ib->C || !ib->tau)) return MPM_ERR_ARG;
    if (!c->adjoint || !c->built || in->n != c->built_n) return MPM_ERR_STATE;
    if (in->n == 0) return MPM_OK;
    const float* inp[4] = {in->x, in->v, in->C, in->tau};
    float* ibp[4] = {ib->x, ib->v, ib->C, ib->tau};
    const int wgs = std::min(c->g2p_wgs, c->work_cap);
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

int mpm_tape_reserve(mpm_ctx* c, int n_slots) {
    if (!c || n_slots < 0) return MPM_ERR_ARG;
    if (!c->adjoint || c->dense) return MPM_ERR_STATE;
    if (hipDeviceSynchronize() != hipSuccess) return MPM_ERR_HIP;  // no work may still use the old slots
    free_tape(c);
    if (n_slots == 0) return MPM_OK;
    const size_t NB = (size_t)1 << c->dim, NPB = (size_t)1 << (2 * c->dim);
    const size_t cap = (size_t)c->block_cap, wc = (size_t)c->work_cap, np = (size_t)c->max_particles;
    hipError_t e = dalloc(&c->tape_ctr, (size_t)n_slots);
    if (e == hipSuccess) e = hipMemset(c->tape_ctr, 0, (size_t)n_slots * sizeof(DevCounters));
    c->tape.resize((size_t)n_slots);
    for (auto& t : c->tape) {
        e = e ? e : dalloc(&t.b_keys, cap);
        e = e ? e : dalloc(&t.b_nbr, cap * NB);
        e = e ? e : dalloc(&t.b_start, cap);
        e = e ? e : dalloc(&t.b_count, cap);
        e = e ? e : dalloc(&t.w_block, wc);
        e = e ? e : dalloc(&t.w_start, wc);
        e = e ? e : dalloc(&t.w_end, wc);
        e = e ? e : dalloc(&t.grid, cap * NPB);
        e = e ? e : dalloc(&t.grid_u, cap * NPB);
        e = e ? e : dalloc(&t.order, np);
        e = e ? e : dalloc(&t.skeys, np);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_tape(c);
        return MPM_ERR_NOMEM;
    }
    return MPM_OK;
}

int mpm_tape_forward(mpm_ctx* c, const mpm_particles* states, int n_steps, void* stream) {
    int st = tape_args_ok(c, states, n_steps);
    if (st != MPM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const DevParams saved = c->P;
    const size_t bytes = (size_t)states[0].n * sizeof(uint32_t);
    for (int j = 0; j < n_steps && st == MPM_OK; ++j) {
        bind_slot(c, j);
        st = mpm_sparse_build(c, &states[j], stream);
        if (st == MPM_OK && bytes &&
            (hipMemcpyAsync(c->tape[(size_t)j].order, c->order, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
             hipMemcpyAsync(c->tape[(size_t)j].skeys, c->skeys, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess))
            st = MPM_ERR_HIP;
        if (st == MPM_OK) st = mpm_p2g(c, &states[j], stream);
        if (st == MPM_OK) st = mpm_grid_update(c, stream);
        if (st == MPM_OK) st = mpm_g2p(c, &states[j], &states[j + 1], stream);
    }
    // the context's own tables were not written: no build is current
    c->P = saved;
    c->built = false;
    c->seg_valid = false;
    if (n_steps > 0) {
        k_merge_tape_flags<<<1, 64, 0, s>>>(c->ctr, c->tape_ctr, n_steps);
        if (st == MPM_OK && hipGetLastError() != hipSuccess) st = MPM_ERR_HIP;
    }
    return st;
}

int mpm_tape_adjoint(mpm_ctx* c, const mpm_particles* states, int n_steps, const mpm_particles* bar,
                     const mpm_particles* spare, float* param_bar, void* stream) {
    int st = tape_args_ok(c, states, n_steps);
    if (st != MPM_OK) return st;
    if (!bar || !spare || !param_bar || bar->n != states[0].n || spare->n != states[0].n) return MPM_ERR_ARG;
    const mpm_particles* sets[2] = {bar, spare};
    if (states[0].n > 0) {
        for (const mpm_particles* q : sets)
            if (!q->x || !q->v || !q->C || !q->F || !q->tau) return MPM_ERR_ARG;
        if (bar->x == spare->x) return MPM_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const DevParams saved = c->P;
    uint32_t* const saved_order = c->order;
    uint32_t* const saved_skeys = c->skeys;
    const mpm_particles* ob = bar;
    const mpm_particles* ib = spare;
    for (int j = n_steps - 1; j >= 0 && st == MPM_OK; --j) {
        bind_slot(c, j);
        c->order = c->tape[(size_t)j].order;
        c->skeys = c->tape[(size_t)j].skeys;
        c->built = true;
        c->built_n = states[j].n;
        st = mpm_g2p_adj(c, &states[j], ob, ib, param_bar, stream);
        if (st == MPM_OK) st = mpm_grid_update_adj(c, stream);
        if (st == MPM_OK) st = mpm_p2g_adj(c, &states[j], ib, stream);
        std::swap(ob, ib);
    }
    c->P = saved;
    c->order = saved_order;
    c->skeys = saved_skeys;
    c->built = false;
    c->seg_valid = false;
    if (st == MPM_OK && ob != bar) {
        // an odd number of steps leaves the result in `spare`
        const int d = c->dim, ns = d == 3 ? 6 : 3;
        const size_t n = (size_t)states[0].n * sizeof(float);
        const float* src[5] = {spare->x, spare->v, spare->C, spare->F, spare->tau};
        float* dst[5] = {bar->x, bar->v, bar->C, bar->F, bar->tau};
        const size_t planes[5] = {(size_t)d, (size_t)d, (size_t)(d * d), (size_t)(d * d), (size_t)ns};
        for (int f = 0; f < 5 && st == MPM_OK; ++f)
            if (n && hipMemcpyAsync(dst[f], src[f], planes[f] * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
                st = MPM_ERR_HIP;
    }
    if (n_steps > 0) {
        k_merge_tape_flags<<<1, 64, 0, s>>>(c->ctr, c->tape_ctr, n_steps);
        if (st == MPM_OK && hipGetLastError() != hipSuccess) st = MPM_ERR_HIP;
    }
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

int mpm_scan_active(mpm_ctx* c, const mpm_particles* p, uint64_t* keys, uint64_t* masks, int capacity,
                    int* n_blocks, void* stream) {
    if (!c || !n_blocks || capacity < 0 || (capacity > 0 && (!keys || !masks))) return MPM_ERR_ARG;
    if (c->P.n_inst > 1 || !particles_ok(c, p, false)) return MPM_ERR_ARG;
    *n_blocks = 0;
    if (!c->sb_mem) return MPM_ERR_STATE;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_scan_active(c->P, p->x, p->n, c->sb, keys, masks, capacity, s);
    SbBox box{};
    if (e == hipSuccess) e = hipMemcpyAsync(&box, c->sb.box, sizeof(SbBox), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return MPM_ERR_HIP;
    *n_blocks = (int)box.total;
    return MPM_OK;
}

int mpm_scan_active_static(mpm_ctx* c, const mpm_particles* p, uint64_t* keys, uint64_t* masks, int capacity,
                           int* n_blocks, void* stream) {
    if (!c || !n_blocks || capacity < 0 || (capacity > 0 && (!keys || !masks))) return MPM_ERR_ARG;
    if (c->P.n_inst > 1 || !particles_ok(c, p, false)) return MPM_ERR_ARG;
    *n_blocks = 0;
    SbBox box{};
    if (launch_scan_active_static(c->P, p->x, p->n, keys, masks, capacity, &box, (hipStream_t)stream) !=
        hipSuccess)
        return MPM_ERR_HIP;
    if (box.too_big) return MPM_ERR_OVERFLOW;
    *n_blocks = (int)box.total;
    return MPM_OK;
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
        hipMemcpyAsync(order, c->osrc, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

int mpm_graph_release(mpm_ctx* c) {
    if (!c) return MPM_ERR_ARG;
    release_graph(c);
    return MPM_OK;
}

int mpm_graph_capture(mpm_ctx* c, const mpm_particles* a, const mpm_particles* b, int n_steps, void* stream) {
    if (!c || !a || !b || n_steps < 2 || (n_steps & 1)) return MPM_ERR_ARG;
    if (c->prm.flags & MPM_FLAG_SYNC_REBUILD) return MPM_ERR_STATE;
    release_graph(c);
    // Record on a private stream (the caller's may be the legacy default
    // stream, which cannot be captured); the graph is replayed on the
    // caller's stream.  Work already queued on `stream` is waited for first.
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return MPM_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MPM_ERR_HIP;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPM_ERR_HIP;
    const int st = mpm_step(c, a, b, n_steps, c->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != MPM_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return st != MPM_OK ? st : MPM_ERR_HIP;
    }
    c->graph = g;
    if (hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        c->graph_exec = nullptr;
        release_graph(c);
        return MPM_ERR_HIP;
    }
    return MPM_OK;
}

int mpm_graph_launch(mpm_ctx* c, int times, void* stream) {
    if (!c || times < 0) return MPM_ERR_ARG;
    if (!c->graph_exec) return MPM_ERR_STATE;
    for (int i = 0; i < times; ++i)
        if (hipGraphLaunch(c->graph_exec, (hipStream_t)stream) != hipSuccess) return MPM_ERR_HIP;
    return MPM_OK;
}

int mpm_set_tuning(mpm_ctx* c, int chunk, int g2p_block, int p2g_workgroups, int g2p_workgroups) {
    if (!c) return MPM_ERR_ARG;
    if (chunk != 0 && (chunk < MIN_CHUNK || chunk > MAX_CHUNK)) return MPM_ERR_ARG;
    if (g2p_block != 0 && g2p_block != 64 && g2p_block != 128 && g2p_block != 256) return MPM_ERR_ARG;
    if (p2g_workgroups < 0 || p2g_workgroups > (1 << 20) || g2p_workgroups < 0 || g2p_workgroups > (1 << 20))
        return MPM_ERR_ARG;
    const int new_chunk = chunk ? chunk : c->chunk;
    const int new_block = g2p_block ? g2p_block : c->g2p_block;
    if (new_chunk > g2p_max_items(new_block)) return MPM_ERR_ARG;
    if (new_chunk != c->chunk) {
        c->chunk = c->P.chunk = new_chunk;
        c->built = false;  // work items of the last build used the old size
    }
    c->g2p_block = new_block;
    if (p2g_workgroups) c->p2g_wgs = p2g_workgroups;
    if (g2p_workgroups) c->g2p_wgs = g2p_workgroups;
    return MPM_OK;
}

int mpm_autotune(mpm_ctx* c, const mpm_particles* a, const mpm_particles* b, int* chosen, void* stream) {
    if (!c || !particles_ok(c, a, true) || !b || b->n != a->n) return MPM_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    // (G2P workgroup size, particles per work item) pairs, persistent workgroup counts
    static const int shapes[][2] = {{64, 64},   {64, 128},  {128, 128}, {128, 256},
                                    {256, 256}, {256, 512}, {256, 768}};
    static const int wgs[] = {1024, 2048, 4096, 8192};
    constexpr int NS = 7, NW = 4, REPS = 5;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int st = MPM_OK;
    for (int i = 0; i < 4 && st == MPM_OK; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) st = MPM_ERR_HIP;
    double p2g_ms[NW] = {0}, g2p_ms[NS][NW] = {{0}};
    // Every trial reads a and writes b, so a is left as it was.  P2G does not
    // depend on the G2P shape: its time per workgroup count is summed over
    // the shapes.
    for (int si = 0; si < NS && st == MPM_OK; ++si) {
        for (int wi = 0; wi < NW && st == MPM_OK; ++wi) {
            c->g2p_block = shapes[si][0];
            c->chunk = c->P.chunk = shapes[si][1];
            c->p2g_wgs = c->g2p_wgs = wgs[wi];
            for (int r = 0; r <= REPS && st == MPM_OK; ++r) {
                st = mpm_sparse_build(c, a, s);
                if (st == MPM_OK && hipEventRecord(ev[0], s) != hipSuccess) st = MPM_ERR_HIP;
                if (st == MPM_OK) st = mpm_p2g(c, a, s);
                if (st == MPM_OK && hipEventRecord(ev[1], s) != hipSuccess) st = MPM_ERR_HIP;
                if (st == MPM_OK) st = mpm_grid_update(c, s);
                if (st == MPM_OK && hipEventRecord(ev[2], s) != hipSuccess) st = MPM_ERR_HIP;
                if (st == MPM_OK) {
                    // G2P as inside mpm_step: it also bins and counts for the
                    // next build (which the next trial's build ignores)
                    const bool next_reuse = would_reuse(c, b->n);
                    uint32_t* keys_out = !c->adjoint && a->n > 0 ? next_bin_buffer(c, next_reuse) : nullptr;
                    uint32_t* movers_out = keys_out && next_reuse ? c->movers : nullptr;
                    st = g2p_impl(c, a, b, s, keys_out, movers_out);
                }
                if (st == MPM_OK && hipEventRecord(ev[3], s) != hipSuccess) st = MPM_ERR_HIP;
                if (st == MPM_OK && hipEventSynchronize(ev[3]) != hipSuccess) st = MPM_ERR_HIP;
                if (st != MPM_OK || r == 0) continue;  // the first repetition warms up
                float t_p2g = 0.f, t_g2p = 0.f;
                if (hipEventElapsedTime(&t_p2g, ev[0], ev[1]) != hipSuccess ||
                    hipEventElapsedTime(&t_g2p, ev[2], ev[3]) != hipSuccess)
                    st = MPM_ERR_HIP;
                p2g_ms[wi] += t_p2g;
                g2p_ms[si][wi] += t_g2p;
            }
        }
    }
    for (int i = 0; i < 4; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (st != MPM_OK) return st;
    int best_p2g = 0, best_s = 0, best_w = 0;
    for (int wi = 1; wi < NW; ++wi)
        if (p2g_ms[wi] < p2g_ms[best_p2g]) best_p2g = wi;
    for (int si = 0; si < NS; ++si)
        for (int wi = 0; wi < NW; ++wi)
            if (g2p_ms[si][wi] < g2p_ms[best_s][best_w]) best_s = si, best_w = wi;
    c->g2p_block = shapes[best_s][0];
    c->chunk = c->P.chunk = shapes[best_s][1];
    c->p2g_wgs = wgs[best_p2g];
    c->g2p_wgs = wgs[best_w];
    c->built = false;
    if (chosen) {
        chosen[0] = c->chunk;
        chosen[1] = c->g2p_block;
        chosen[2] = c->p2g_wgs;
        chosen[3] = c->g2p_wgs;
    }
    return MPM_OK;
}

}  // extern "C"
