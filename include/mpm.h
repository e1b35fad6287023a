/*
 * mpm.h -- C ABI of the sparse-grid explicit material point method step
 * (HIP, gfx950).
 *
 * One explicit step (Methods 3.1 of "Unified sparse framework for large-scale
 * simulations using the material point method") on a background grid whose
 * storage is restricted to the active nodes A = union_p S(p) (Eqs. 4-5):
 *
 *   mpm_sparse_build   active-node indexing: the active blocks of B^d nodes
 *                      (B = 4), their compact indices Phi and the compact node
 *                      map phi(n) = Phi(b(n)) B^d + l(n) (Methods 3.2-3.3,
 *                      Algorithms 1 and 5-7, Eqs. 18, 22-25);
 *   mpm_p2g            particle-to-grid transfer onto the compact storage
 *                      (Eqs. 6-7 mass and APIC momentum, Eq. 9 internal force);
 *   mpm_grid_update    nodal velocity normalisation and explicit Euler update
 *                      (Eqs. 8, 10-12) followed by boundary conditions;
 *   mpm_g2p            grid-to-particle APIC gather, position, affine matrix
 *                      and deformation-gradient update (Eqs. 13-17) and the
 *                      constitutive update (Hencky elasticity or a
 *                      Drucker-Prager return map on Hencky strain);
 *   mpm_step           n_steps x (build; p2g; grid update; g2p).
 *
 * Conventions
 * -----------
 * - All particle arrays are DEVICE pointers owned by the caller, float32,
 *   structure-of-arrays and component-major with plane stride n:
 *     x[a*n + p], v[a*n + p]               a < d
 *     C[(r*d + c)*n + p], F[(r*d + c)*n + p] row-major d x d
 *     tau[k*n + p]  Kirchhoff stress, 2D (xx, yy, xy), 3D (xx, yy, zz, xy, yz, xz)
 *     id[p]         optional uint32 particle identity carried along (may be NULL)
 * - Nodes sit at x_n = n * dx, n = (i, j[, k]) with 0 <= n_a <= cells[a]
 *   (Eq. 3).  A particle's support is the 3^d stencil from its base node
 *   floor(x/dx - 1/2); every stencil node must lie inside the grid, otherwise the
 *   step raises MPM_FLAG_DOMAIN (positions are clamped so no access leaves the
 *   grid).
 * - The library REORDERS particles: mpm_g2p reads the input set through the
 *   sort permutation of the last build and writes the output set in sorted
 *   (block-key) order; id[] travels with each particle.
 * - stream is a hipStream_t (NULL = the default stream).  Every call only
 *   enqueues work on it, except where stated ("synchronises").
 * - Every call returns an MPM_* status and never aborts.  Argument errors are
 *   reported synchronously.  Conditions found on the device (hash overflow,
 *   domain exit, inverted deformation, non-finite values) are latched in a
 *   sticky device status word read by mpm_get_status.
 * - One context per stream; a context is not thread-safe across host threads.
 */
#ifndef MPM_H
#define MPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_ctx mpm_ctx;

/* return codes */
#define MPM_OK            0
#define MPM_ERR_ARG       1   /* invalid argument (null pointer, size, capacity) */
#define MPM_ERR_HIP       2   /* a HIP runtime call failed */
#define MPM_ERR_NOMEM     3   /* device allocation failed */
#define MPM_ERR_OVERFLOW  4   /* hash table or block capacity exceeded */
#define MPM_ERR_DOMAIN    5   /* a particle support left the grid */
#define MPM_ERR_INVERTED  6   /* a trial deformation gradient has det <= 0 */
#define MPM_ERR_NAN       7   /* a non-finite value was produced */
#define MPM_ERR_STATE     8   /* call out of order (e.g. p2g before a build) */

/* bits of the sticky device status word */
#define MPM_FLAG_OVERFLOW 1u
#define MPM_FLAG_DOMAIN   2u
#define MPM_FLAG_INVERTED 4u
#define MPM_FLAG_NAN      8u

/* boundary condition of one grid face (nodes within `bound` of the face) */
#define MPM_BC_NONE     0   /* no constraint */
#define MPM_BC_STICKY   1   /* v = 0 */
#define MPM_BC_SLIP     2   /* normal component set to 0 */
#define MPM_BC_SEPARATE 3   /* normal component may only point away from the face */

/* constitutive models */
#define MPM_MODEL_ELASTIC 0   /* Hencky (logarithmic-strain) elasticity */
#define MPM_MODEL_DP      1   /* cohesionless Drucker-Prager return map on Hencky strain */

/* grid storage */
#define MPM_GRID_SPARSE 0     /* active blocks only (the method) */
#define MPM_GRID_DENSE  1     /* every block of the potential domain (baseline) */

/* flags */
#define MPM_FLAG_SYNC_REBUILD 1  /* mpm_sparse_build synchronises and, on overflow,
                                    doubles the table and block capacity and rebuilds
                                    (Algorithm 7) until it fits */
#define MPM_FLAG_ADJOINT      2  /* allocate the reverse-mode buffers (pre-boundary
                                    nodal velocity, grid adjoint, per-particle
                                    scratch); the grid update then also records u.
                                    Walls only: not allowed with a heightmap. */
#define MPM_FLAG_FULL_SORT    4  /* sort from scratch on every build.  By default a
                                    sparse build of a context without MPM_FLAG_ADJOINT
                                    that follows a build of the same number of
                                    particles re-sorts incrementally: particles that
                                    keep their owner block stay in its range, the
                                    others are routed through the previous build's
                                    hash table.  Either way each owner block's
                                    particles are contiguous with base cells
                                    ascending; block order and the order of the
                                    particles inside a cell differ between the
                                    two (the re-sort's order inside a cell is not
                                    fixed from run to run). */
#define MPM_FLAG_DETERMINISTIC_ORDER 8
                                 /* Phi in ascending order of the Eq. 22 block key
                                    (lexicographic (i, j, k), instance first in an
                                    ensemble) instead of hash-slot order, and the
                                    particle order a fixed function of the input
                                    order (every build sorts from scratch, as with
                                    MPM_FLAG_FULL_SORT).  Two runs from the same
                                    input then give the same Phi and bit-identical
                                    grids and particles.  Sparse grid only. */
#define MPM_FLAG_SCAN_BUILD  16  /* mpm_sparse_build constructs the active set by the
                                    scan-based method (Methods 3.2, Algorithms 1-4)
                                    instead of the hash table: a block mask over the
                                    bounding box of the owner blocks (grown by one
                                    block upward), an exclusive scan of its flags
                                    and compaction (Eq. 18), all on the device.
                                    Every build sorts from scratch; Phi comes out in
                                    ascending key order.  Allocates at create a mask
                                    domain for every block of the potential grid
                                    (24 bytes per block).  Sparse grid, one
                                    simulation, no MPM_FLAG_ADJOINT. */

/* Material and time step of one instance of an ensemble (see n_instances). */
typedef struct mpm_instance {
    float E, nu;             /* Young's modulus (Pa) and Poisson ratio */
    float friction_deg;      /* Drucker-Prager friction angle (degrees) */
    float dt;                /* time step of this instance */
    float p_mass, p_vol0;    /* particle mass and initial volume */
} mpm_instance;

typedef struct mpm_params {
    int dim;                 /* 2 or 3 */
    double dx;               /* grid spacing h (Eq. 3), metres */
    int cells[3];            /* cells per axis; nodes per axis = cells + 1 */
    float gravity[3];        /* body force per unit mass g (Eq. 10) */
    float dt;                /* time step (Eqs. 11-17) */
    int bound;               /* wall thickness in nodes (default 3 when 0) */
    int bc[3][2];            /* MPM_BC_* per axis, [0] low face, [1] high face */
    const float* heightmap;  /* HOST pointer, (cells[0]+1) x (cells[1]+1) node heights,
                                x-major (h[i*(cells[1]+1) + j]); 3D only, z up; copied at
                                create; NULL = no terrain */
    float mu_terrain;        /* Coulomb friction of the terrain */
    int model;               /* MPM_MODEL_* */
    float E, nu;             /* Young's modulus (Pa) and Poisson ratio */
    float friction_deg;      /* Drucker-Prager friction angle (degrees) */
    float p_mass;            /* particle mass m_p (kg) */
    float p_vol0;            /* initial particle volume V0_p */
    int max_particles;       /* capacity of every per-particle buffer */
    int block_capacity;      /* max active blocks (0 = default) */
    int hash_capacity_log2;  /* log2 H of the block hash table (0 = default) */
    int grid_mode;           /* MPM_GRID_* */
    int flags;               /* MPM_FLAG_SYNC_REBUILD ... */
    int n_instances;         /* 0 or 1: one simulation.  2..64: an ensemble of independent
                                simulations on identical potential grids, sharing every
                                buffer; each particle names its instance in inst[] and each
                                instance has its own material and dt (instances[]).  The
                                instance id is folded into the sort key and into the block
                                key (then m = 19 bits per coordinate, bias 2^18, instance in
                                bits 57-62); the instance, block and cell bits together must
                                fit 32 bits.  Sparse grid only, no adjoint. */
    const mpm_instance* instances;  /* HOST pointer, n_instances entries, copied at create */
} mpm_params;

typedef struct mpm_particles {
    int n;                   /* number of particles (<= max_particles); with n = 0 the
                                array pointers may be NULL */
    float* x;
    float* v;
    float* C;
    float* F;
    float* tau;
    uint32_t* id;            /* optional */
    uint32_t* inst;          /* instance of each particle (ensembles; NULL = instance 0),
                                permuted with the particle like id */
} mpm_particles;

/* Create a context: validates *params, copies the heightmap, allocates every
 * device buffer (nothing is allocated by later calls except on an Algorithm-7
 * rebuild).  On success *out owns them; returns MPM_ERR_ARG / MPM_ERR_NOMEM /
 * MPM_ERR_HIP otherwise and leaves *out NULL. */
int mpm_create(const mpm_params* params, mpm_ctx** out);

/* Free a context and all its device memory (synchronises the device). */
int mpm_destroy(mpm_ctx* ctx);

/* Human-readable name of an MPM_* return code (static storage). */
const char* mpm_status_string(int status);

/* Active-node indexing (Methods 3.3, Algorithms 5-6, Eqs. 22-25, with the
 * block layout of Methods 3.2): bins the particles by base node, sorts them by
 * 4^d-block key, inserts every block touched by a stencil into the open-
 * addressing table (packed key, Eq. 22; 64-bit mixer, Eq. 23; slot h & (H-1),
 * Eq. 24; linear probing, Eq. 25), records the node-level active mask of each
 * block, and compacts the occupied slots into Phi in [0, n_blocks) by a prefix
 * scan.  The active set (blocks and node masks) is a pure function of the
 * positions.  The particle order is one in which each owner block's particles
 * are contiguous with their base cells ascending; after a build of the same
 * number of particles it is derived incrementally from that build's order
 * (see MPM_FLAG_FULL_SORT).  If more blocks are touched than block_capacity,
 * or a probe sequence finds no slot, MPM_FLAG_OVERFLOW is latched (with
 * MPM_FLAG_SYNC_REBUILD the call rebuilds instead, Algorithm 7, sorting from
 * scratch).  In MPM_GRID_DENSE mode Phi is the linear block index of the whole
 * domain. */
int mpm_sparse_build(mpm_ctx* ctx, const mpm_particles* p, void* stream);

/* P2G onto the compact storage (Eqs. 6, 7, 9): sets every node of the active
 * blocks to m_n and p_n = sum_p N m_p [v_p + C_p (x_n - x_p)]
 * - dt sum_p V0_p tau_p grad N_n (zero where no particle reaches).  Requires a
 * build of the same positions; one call per build (on a dense grid the sums
 * accumulate into the grid that the build cleared). */
int mpm_p2g(mpm_ctx* ctx, const mpm_particles* p, void* stream);

/* Grid update (Eqs. 8, 10-12): v_n = p_n / m_n + dt g where m_n > 0, else 0,
 * then boundary conditions (terrain level set with Coulomb friction, then the
 * walls).  Operates on the storage filled by mpm_p2g. */
int mpm_grid_update(mpm_ctx* ctx, void* stream);

/* G2P (Eqs. 13-17) and the constitutive update.  Reads `in` through the sort
 * permutation of the last build and writes the advanced state to `out`
 * grouped by owner block in the build's particle order; inside a block's range the
 * particles are stored rank-major over the block's cells (first particle of
 * each occupied cell, then the second, ... up to rank 31, then the rest cell
 * by cell), which makes the next step's P2G loads contiguous.
 * mpm_get_order gives the resulting permutation.  `in` and `out` must not
 * overlap and must have the same n. */
int mpm_g2p(mpm_ctx* ctx, const mpm_particles* in, const mpm_particles* out, void* stream);

/* n_steps explicit steps ping-ponging between a and b: step 0 reads a and
 * writes b, step 1 reads b and writes a, ...  The final state is in a when
 * n_steps is even and in b when it is odd.  Between two steps of one call,
 * G2P also bins the positions it writes (the float64 arithmetic of the build's
 * binning on the same float32 values), so the next build skips its binning
 * pass, and on a sparse grid P2G's second pass applies the grid update (the
 * momenta between the two are never stored); the results are those of the
 * four calls made one after the other (contexts with MPM_FLAG_ADJOINT bin in
 * every build and keep the separate grid update). */
int mpm_step(mpm_ctx* ctx, const mpm_particles* a, const mpm_particles* b, int n_steps, void* stream);

/* Synchronises `stream` and returns the sticky MPM_FLAG_* word in *flags;
 * the return code is MPM_OK when no flag is set, else the MPM_ERR_* of the
 * lowest flag set. */
int mpm_get_status(mpm_ctx* ctx, void* stream, uint32_t* flags);

/* Clears the sticky status word (enqueued). */
int mpm_clear_status(mpm_ctx* ctx, void* stream);

/* Synchronises `stream` and reports the number of active blocks of the last
 * build (n_blocks) and the number of occupied hash slots before the capacity
 * check (n_touched, > n_blocks only on overflow). */
int mpm_active_count(mpm_ctx* ctx, void* stream, int* n_blocks, int* n_touched);

/* Copies, for compact blocks 0..min(n_blocks, capacity)-1 in Phi order, the
 * packed block key of Eq. 22 (m = 21, bias 2^20; 2D packs (i, j) in the low
 * 42 bits) into keys[] and the node-level active mask (bit l(n) =
 * i_l + 4 (j_l + 4 k_l) set iff node n is in A) into masks[].  Device pointers
 * owned by the caller.  Sparse mode only.  In an ensemble the keys use the
 * ensemble packing (instance in bits 57-62, m = 19, bias 2^18). */
int mpm_get_active(mpm_ctx* ctx, uint64_t* keys, uint64_t* masks, int capacity, void* stream);

/* Scan-based construction of the same active set (Methods 3.2, Algorithms
 * 1-4: block mask over the bounding box of the particles' owner blocks, grown
 * by one block on each upper side, then an exclusive scan of the flags and
 * compaction), for checking the active set or comparing the two
 * constructions.  Bins p->x itself; independent of any earlier build and
 * leaves the context's build tables untouched.  Writes the Eq. 22 keys and
 * node masks (same formats as mpm_get_active) of the first
 * min(*n_blocks, capacity) blocks, in ascending key order, to the caller's
 * device arrays keys[] and masks[] (may be NULL when capacity is 0), and the
 * number of active blocks to the host int *n_blocks.  Synchronises `stream`.
 * Uses the mask-domain scratch of a context created with MPM_FLAG_SCAN_BUILD
 * (MPM_ERR_STATE otherwise; nothing is allocated).  MPM_ERR_ARG for an
 * ensemble context or bad arguments. */
int mpm_scan_active(mpm_ctx* ctx, const mpm_particles* p, uint64_t* keys, uint64_t* masks, int capacity,
                    int* n_blocks, void* stream);

/* Allocation-free form of mpm_scan_active, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, outputs and synchronisation as
 * mpm_scan_active, on any one-simulation context (MPM_FLAG_SCAN_BUILD not
 * needed): the scratch is a static device array holding a mask domain of at
 * most 1,048,576 blocks (16 MiB on each device the library runs on, resident
 * until the process ends); no device memory is allocated or freed.  Returns
 * MPM_ERR_OVERFLOW, with *n_blocks = 0 and nothing written, when the bounding
 * box of the owner blocks grown by one block exceeds that.  Every call on a
 * device shares that device's array: calls that overlap on one device (other
 * streams, other host threads) race. */
int mpm_scan_active_static(mpm_ctx* ctx, const mpm_particles* p, uint64_t* keys, uint64_t* masks, int capacity,
                           int* n_blocks, void* stream);

/* Copies the compact grid, 4 floats per node, blocks 0..min(n_blocks,
 * capacity)-1 in Phi order, nodes in l(n) order within a block: after mpm_p2g
 * (p_x, p_y, p_z, m); after mpm_grid_update (v_x, v_y, v_z, m) (2D: z = 0).
 * Device pointer owned by the caller, capacity * 4^d * 4 floats. */
int mpm_get_grid(mpm_ctx* ctx, float* out, int capacity_blocks, void* stream);

/* Writes the particle permutation of mpm_g2p for the last build: order[i] =
 * index in the input set of the particle that mpm_g2p writes to position i
 * (recorded by mpm_p2g, so valid once mpm_p2g has run on the build).  Device
 * pointer owned by the caller, n entries. */
int mpm_get_order(mpm_ctx* ctx, uint32_t* order, int n, void* stream);

/* ---- reverse mode (contexts created with MPM_FLAG_ADJOINT) -------------
 * The adjoints are those of the discrete step above (not in the paper; they
 * differentiate P2G, the grid update with wall boundaries, G2P and the
 * constitutive map, with the active set held fixed).  Adjoint particle sets use
 * the same SoA layout as states: x_bar, v_bar, C_bar, F_bar (full d x d) and
 * tau_bar for the stored stress components.  Output-side adjoints are in the
 * step's output order (the sorted order written by mpm_g2p); input-side
 * adjoints are in the input order, so the in_bar of one step is the out_bar of
 * the step before it.  param_bar is a DEVICE float[2] accumulator
 * (dL/dE in 1/Pa, dL/dphi per degree) that the caller zeroes.
 *
 * mpm_g2p_adj: needs mpm_sparse_build, mpm_p2g and mpm_grid_update of `in` on
 *   this context; writes in_bar->x (partial) and in_bar->F, and records the
 *   grid adjoint of the nodal velocities.
 * mpm_grid_update_adj: turns it into the adjoints of nodal momentum and mass.
 * mpm_p2g_adj: writes in_bar->v, C, tau and adds the rest of in_bar->x.
 * mpm_step_adj: build + p2g + grid update of `in`, then the three adjoints. */
int mpm_g2p_adj(mpm_ctx* ctx, const mpm_particles* in, const mpm_particles* out_bar, const mpm_particles* in_bar,
                float* param_bar, void* stream);
int mpm_grid_update_adj(mpm_ctx* ctx, void* stream);
int mpm_p2g_adj(mpm_ctx* ctx, const mpm_particles* in, const mpm_particles* in_bar, void* stream);
int mpm_step_adj(mpm_ctx* ctx, const mpm_particles* in, const mpm_particles* out_bar, const mpm_particles* in_bar,
                 float* param_bar, void* stream);

/* Tape for checkpointed reverse mode (sparse contexts with MPM_FLAG_ADJOINT,
 * without MPM_FLAG_SYNC_REBUILD).  The adjoint of a step reads what the step's
 * own build, P2G and grid update produced (block and work tables, nodal
 * velocities before and after the boundary conditions, sorted keys and
 * order).  mpm_step_adj recomputes them; a tape keeps them instead, one slot
 * per step of a segment, so that the reverse sweep runs only the three
 * adjoint transfers per step.  A slot holds 2 x 4^d x 16 B of grid plus about
 * 80 B of tables per block of capacity and 8 B per particle of capacity
 * (about 28 MB for 262,144 particles at the default block capacity).
 *
 * mpm_tape_reserve: allocates n_slots slots (0 frees them; synchronises the
 *   device).  A capacity change (the overflow rebuild) frees them.
 * mpm_tape_forward: states[0 .. n_steps] are n_steps + 1 caller-owned sets of
 *   one size, consecutive ones distinct; runs n_steps steps, step j from
 *   states[j] to states[j+1] (as mpm_step on that pair), keeping slot j.
 *   n_steps <= n_slots.  Afterwards no build is current (mpm_p2g etc. need a
 *   new mpm_sparse_build).
 * mpm_tape_adjoint: the reverse sweep over the same steps and the same sets,
 *   unchanged since mpm_tape_forward: on entry `bar` holds dL/d(states[n_steps])
 *   (in that set's order), on return dL/d(states[0]) (in states[0]'s order);
 *   `spare` is scratch of the same layout; param_bar accumulates as for
 *   mpm_step_adj.  Status flags raised in the slots are merged into the
 *   context's own (mpm_get_status). */
int mpm_tape_reserve(mpm_ctx* ctx, int n_slots);
int mpm_tape_forward(mpm_ctx* ctx, const mpm_particles* states, int n_steps, void* stream);
int mpm_tape_adjoint(mpm_ctx* ctx, const mpm_particles* states, int n_steps, const mpm_particles* bar,
                     const mpm_particles* spare, float* param_bar, void* stream);

/* ---- graphs and tuning -------------------------------------------------------
 * mpm_graph_capture records n_steps (even, >= 2) of mpm_step(a, b) into a HIP
 * graph held by the context (replacing any previous one).  It first waits for
 * the work queued on `stream`, records on a private stream and executes
 * nothing.  mpm_graph_launch replays the graph `times` times on `stream`; each
 * replay advances a by n_steps (the state ends in a).  The step needs no host
 * synchronisation, so one graph holds whole steps.  The graph keeps the
 * particle pointers, material and launch shape it was recorded with: a, b must
 * stay allocated, and mpm_set_material / mpm_set_tuning do not change it.
 * Returns MPM_ERR_STATE with MPM_FLAG_SYNC_REBUILD (that rebuild needs the
 * host).  mpm_graph_release frees the graph (mpm_destroy does too). */
int mpm_graph_capture(mpm_ctx* ctx, const mpm_particles* a, const mpm_particles* b, int n_steps, void* stream);
int mpm_graph_launch(mpm_ctx* ctx, int times, void* stream);
int mpm_graph_release(mpm_ctx* ctx);

/* Launch shape of the transfer kernels: particles per work item `chunk`
 * (64..768, used by G2P and the reverse kernels), G2P workgroup size
 * `g2p_block` (64, 128 or 256; chunk <= 2 g2p_block, or 3 g2p_block at 256)
 * and the persistent workgroup counts of the P2G and G2P launches.  0 keeps a
 * value.  Takes effect on the next build; a captured graph keeps the shape it
 * was recorded with.  MPM_ERR_ARG for values out of range. */
int mpm_set_tuning(mpm_ctx* ctx, int chunk, int g2p_block, int p2g_workgroups, int g2p_workgroups);

/* Autotuner: for every candidate launch shape ((g2p_block, chunk) in {(64,
 * 64), (64, 128), (128, 128), (128, 256), (256, 256), (256, 512), (256, 768)}
 * x persistent workgroups in {1024, 2048, 4096, 8192}) runs one warm-up and 5 timed steps
 * that read a and write b (a is left unchanged; b ends one step ahead of a;
 * G2P as inside mpm_step, binning and counting for a next build),
 * keeps the fastest P2G workgroup count and the fastest G2P shape, and
 * reports them in chosen[4] = {chunk, g2p_block, p2g_workgroups,
 * g2p_workgroups} (host ints, may be NULL).  Synchronises the stream. */
int mpm_autotune(mpm_ctx* ctx, const mpm_particles* a, const mpm_particles* b, int* chosen, void* stream);

/* Replaces the material constants (E, nu, friction angle) and dt of a live
 * context without reallocating. */
int mpm_set_material(mpm_ctx* ctx, float E, float nu, float friction_deg, float dt);

#ifdef __cplusplus
}
#endif

#endif /* MPM_H */
