/*
 * mibh.h - C ABI of an MI355X (gfx950) Barnes-Hut force step.
 *
 * The method is the GPU tree-code of Bedorf, Gaburov & Portegies Zwart,
 * "Bonsai: A GPU Tree-Code" (arXiv:1204.2280): every part of one force
 * evaluation runs on the GPU with no host<->device traffic (Abstract,
 * Introduction), in the parts the Results section times separately - sorting
 * along a Morton curve, moving particle properties, tree construction,
 * multipole moments and the tree traverse with a Barnes (1994) / vector-
 * machine (Barnes 1990) opening criterion theta.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers on the context's device; the
 *     caller owns them.  Host pointers are named h_* or are plain outputs.
 *   - Arrays are C-contiguous float32: positions and accelerations are
 *     [n][3] (x, y, z interleaved), masses and potentials are [n].
 *   - All work is enqueued on the stream given to mibh_create; calls return
 *     once enqueued unless they say "synchronises".
 *   - Every call returns a mibh_status; no exception crosses the ABI.  On an
 *     error the thread-local message is available from mibh_last_error().
 *   - Device-side conditions (non-finite input, capacity overflow) are
 *     recorded in device memory and reported by the next synchronising call
 *     (mibh_sync, mibh_stats, mibh_energy).
 *   - The library never allocates device memory: the caller passes one
 *     workspace of mibh_workspace_bytes() bytes at mibh_create.
 *   - Calls on one context are not thread-safe; contexts are independent.
 */
#ifndef MIBH_H
#define MIBH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mibh_ctx mibh_ctx;

typedef enum {
    MIBH_OK = 0,
    MIBH_EINVAL = -1,      /* bad argument: null pointer, n out of range, theta <= 0, ... */
    MIBH_ENOMEM = -2,      /* workspace smaller than mibh_workspace_bytes() */
    MIBH_EHIP = -3,        /* a HIP runtime call failed */
    MIBH_ESTATE = -4,      /* calls out of order (e.g. forces before build_tree) */
    MIBH_EOVERFLOW = -5,   /* a device-side capacity was exceeded (results invalid) */
    MIBH_ENONFINITE = -6   /* a position or mass was NaN/Inf, or a mass was negative */
} mibh_status;

/* Per-particle accumulation of the walk's float32 interaction terms.
 * MIBH_PLAIN: plain float32.  Within one evaluation of the interaction lists
 * (a full list's flush, or the group's end) each lane sums at most 16 tiles of
 * terms and the 64 lanes are folded by a six-level tree; a particle's totals
 * of successive evaluations are then added.
 * MIBH_KAHAN: the same, with those totals of successive evaluations added with
 * Kahan compensation (the long sums of a particle with long lists).
 * MIBH_KAHAN_TERM: every term compensated as it is added to its lane's sum, and
 * the evaluations' totals as in MIBH_KAHAN (for measurement; the walk runs
 * 8 group particles per pass instead of 16).
 * All three walk the same lists: counts are identical, forces differ by
 * rounding only. */
enum { MIBH_PLAIN = 0, MIBH_KAHAN = 1, MIBH_KAHAN_TERM = 2 };

/* Parameters of the method and of the walk kernel. */
typedef struct {
    int32_t ncrit;      /* leaf capacity: a cell splits iff it holds more than ncrit
                           particles and is above level 20 (default 16) */
    int32_t group_cap;  /* groups are the largest cells with <= group_cap particles;
                           1 <= ncrit <= group_cap <= 64 (default 64) */
    float eps2;         /* Plummer softening length squared (default 0) */
    float G;            /* gravitational constant (default 1) */
    int32_t precision;  /* MIBH_PLAIN, MIBH_KAHAN or MIBH_KAHAN_TERM accumulation (default plain) */
    int32_t walk_waves; /* waves of the persistent walk launch; 0 = 4096 (16 per CU of a
                           256-CU MI355X) */
    int32_t pc_cap;     /* per-wave particle-cell list entries (in LDS) before an evaluation
                           flush, 128 <= pc_cap <= 1024 (default 1024) */
    int32_t pp_cap;     /* per-wave particle-particle list entries (in LDS) before a flush,
                           128 <= pp_cap <= 512 (default 512) */
    int32_t max_systems; /* most independent systems one batched build may hold,
                            1 <= max_systems <= 256 (default 1) */
    int32_t anchor_up;  /* 0: every group's traversal starts at its root.
                           1..4 (default 3): the groups below each ancestor cell
                           anchor_up levels above them share one traversal with the
                           ancestor's particle box: the cells it accepts are accepted by
                           every such group, the cells it surely opens (its box's
                           farthest point inside the opening radius) are opened by every
                           such group, and each group traverses only the rest.  Same
                           lists and counts as 0, summed in another order, by every walk
                           (any queue order; active walks build the lists of their
                           groups' anchors only).  Adds 8 bytes per particle, 16 per cell and a pool of
                           (16 >> (anchor_up - 1)) words per particle to the workspace. */
} mibh_params;

/* Fills the defaults listed above. */
void mibh_default_params(mibh_params *p);

/* Bytes of device workspace a context needs for up to n_max particles with
 * these parameters (NULL = defaults).  Returns 0 if the arguments are invalid
 * (n_max < 1 or >= 2^31, or invalid parameters). */
size_t mibh_workspace_bytes(int64_t n_max, const mibh_params *p);

/* Creates a context on the current HIP device.  d_workspace must hold at
 * least mibh_workspace_bytes(n_max, p) bytes, 256-byte aligned, and stay
 * valid until mibh_destroy; stream is a hipStream_t (NULL = null stream).
 * Errors: EINVAL (bad parameters or pointers), ENOMEM (workspace too small),
 * EHIP. */
mibh_status mibh_create(const mibh_params *p, int64_t n_max, void *d_workspace,
                        size_t workspace_bytes, void *stream, mibh_ctx **out);

/* Frees the host-side context (the workspace stays the caller's). */
mibh_status mibh_destroy(mibh_ctx *ctx);

/* Tree construction: bounding cube, 60-bit Morton keys, stable radix sort,
 * reorder of positions and masses, breadth-first sparse octree and groups
 * (the sorting / moving / tree-construction parts of the Results section).
 * d_pos [n][3] and d_mass [n] must stay valid and unchanged until the next
 * build_tree; 1 <= n <= n_max.  Errors: EINVAL.  Non-finite inputs are
 * flagged on the device (ENONFINITE at the next synchronising call). */
mibh_status mibh_build_tree(mibh_ctx *ctx, const float *d_pos, const float *d_mass, int64_t n);

/* Batched tree construction for nsys independent systems (an ensemble): system
 * s is particles [h_offsets[s], h_offsets[s+1]) of d_pos/d_mass, gets its own
 * root cube, octree and groups, and interacts only with itself; one
 * compute_forces call then walks the groups of all systems in one persistent
 * launch.  h_offsets is a host array of nsys+1 values, 0 = h_offsets[0] <
 * h_offsets[1] < ... < h_offsets[nsys] = n <= n_max (no empty system), read
 * before the call returns.  1 <= nsys <= max_systems.  mibh_build_tree is the
 * nsys = 1 case.  Cells and groups of all systems share one breadth-first
 * numbering; the level-0 cells are the systems' roots in system order.
 * Errors: EINVAL. */
mibh_status mibh_build_tree_batch(mibh_ctx *ctx, const float *d_pos, const float *d_mass,
                                  const int64_t *h_offsets, int nsys);

/* Multipole moments of every cell (the "tree-properties"): float64 mass,
 * centre of mass and second moments, reduced bottom-up level by level, then
 * the float32 monopole + traceless quadrupole used by the walk.
 * Errors: ESTATE if no tree was built. */
mibh_status mibh_compute_multipoles(mibh_ctx *ctx);

/* Tree traverse for all groups with opening parameter theta > 0 (the MAC of
 * the Results section), particle-cell and particle-particle interactions in
 * float32, results written in the caller's particle order: d_acc [n][3],
 * d_pot [n] (potential, negative; self term excluded).
 * Errors: EINVAL (theta not finite or <= 0, null outputs), ESTATE. */
mibh_status mibh_compute_forces(mibh_ctx *ctx, float theta, float *d_acc, float *d_pot);

/* Refit (block time steps, the paper's Discussion section: between
 * rebuilds only the multipole moments are recomputed).  The particles of the
 * last build_tree take new positions and masses d_pos [n][3], d_mass [n]
 * (input order, the same n particles); the sorted order, cells and groups
 * are kept and the particles are moved into that order again.  Call
 * compute_multipoles next: it recomputes every cell's moments, delta and
 * l' (MIBH_EXPORT_LSIDE), so a cell whose particles left its cube is opened
 * from further away.  Non-finite input or negative masses are reported by the
 * next synchronising call.  Errors: ESTATE before build_tree, EINVAL. */
mibh_status mibh_refit(mibh_ctx *ctx, const float *d_pos, const float *d_mass);

/* compute_forces for the groups that hold at least one particle with
 * d_active[i] != 0 (uint8 [n], input order, device memory): the walk visits
 * only those groups (the paper's block time steps, Results section: the
 * traverse time falls with the number of active particles).  Each visited
 * group's interaction lists are those of a full walk (its whole box), but only
 * its active particles are evaluated: acc and pot are written for the active
 * particles and left untouched for every other particle; MIBH_EXPORT_COUNTS is
 * updated for the visited groups only, and MIBH_EXPORT_QUEUE lists the visited
 * groups first, in Morton order.
 * Errors: as compute_forces, EINVAL for a null mask. */
mibh_status mibh_compute_forces_active(mibh_ctx *ctx, float theta, const uint8_t *d_active, float *d_acc,
                                       float *d_pot);

/* build_tree + compute_multipoles + compute_forces in order. */
mibh_status mibh_forces(mibh_ctx *ctx, const float *d_pos, const float *d_mass, int64_t n,
                        float theta, float *d_acc, float *d_pot);

/* The force step for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same result as mibh_forces with default parameters (ncrit 16, groups of
 * <= 64, eps2 0, G 1, plain float32 accumulation) except anchor_up = 0 (every
 * group's traversal starts at the root; no anchor buffers), bit for bit, for
 * 1 <= n <= mibh_static_n_max() (32768) particles; larger n gives EINVAL.
 * Inputs and outputs are the caller's device arrays, laid out as for
 * mibh_forces; work is enqueued on `stream` (a hipStream_t, NULL: the null
 * stream) and the call does not synchronise.  The workspace is a file-scope
 * device array of mibh_static_bytes() (40 MiB) that every GPU the library
 * runs on holds from module load until the process ends; the call allocates
 * nothing (no hipMalloc, no host allocation).  All calls on one GPU share that
 * array and the host state that describes it: calls that overlap on one GPU
 * (two streams, or a second call before the first has finished on its
 * stream) race and give undefined results; calls from several host threads
 * are serialised while they enqueue, not while they run.  Device-side
 * conditions (non-finite input, negative mass) leave acc/pot unwritten and are
 * not reported by this call.  Errors: EINVAL (null pointer, n out of range,
 * theta <= 0 or non-finite), EHIP. */
mibh_status mibh_forces_static(const float *d_pos, const float *d_mass, int64_t n, float theta, float *d_acc,
                               float *d_pot, void *stream);
size_t mibh_static_bytes(void);
int64_t mibh_static_n_max(void);

/* Graph capture of one whole step: build (batched, as mibh_build_tree_batch),
 * multipoles and forces are captured from the context's stream into a HIP graph
 * and instantiated; nothing runs during the capture.  mibh_graph_launch replays
 * it on the context's stream with the captured pointers, offsets and theta
 * (the inputs may change in place between replays).  The step holds no
 * allocation, memset or synchronisation, so the whole step is one graph launch.
 * The context's stream must not be the null stream.
 * Errors: EINVAL, EHIP; graph_launch: ESTATE if nothing was captured. */
mibh_status mibh_graph_capture(mibh_ctx *ctx, const float *d_pos, const float *d_mass,
                               const int64_t *h_offsets, int nsys, float theta, float *d_acc,
                               float *d_pot);
mibh_status mibh_graph_launch(mibh_ctx *ctx);

/* Changes the stream later calls enqueue on (hipStream_t; NULL = null stream). */
mibh_status mibh_set_stream(mibh_ctx *ctx, void *stream);

/* Synchronises: waits for the context's stream and reports device flags
 * (ENONFINITE, EOVERFLOW) raised since the last build_tree. */
mibh_status mibh_sync(mibh_ctx *ctx);

/* Per-step statistics; synchronises. */
typedef struct {
    int64_t n, ncells, ngroups, nleaves;
    int32_t depth;         /* deepest cell level */
    int32_t root_k;        /* root cube side of system 0 is 2^root_k */
    int32_t nsys;          /* systems of the current tree */
    uint64_t sum_pc;       /* sum over particles of their group's particle-cell count */
    uint64_t sum_pp;       /* sum over particles of their group's particle-particle count */
    uint32_t flags;        /* device flags: 1 non-finite, 2 negative mass, 4 stack, 8 cell capacity */
    uint32_t anchors;      /* shared-prefix walk (anchor_up > 0): anchor cells of the last walk */
    uint32_t anchor_fallbacks; /* of those, anchors whose lists did not fit their room (their
                                  groups walked from the root: same results, slower) */
} mibh_stats_t;
mibh_status mibh_stats(mibh_ctx *ctx, mibh_stats_t *out);

/* Total energies in float64 with a fixed-shape (deterministic) reduction:
 * W = 1/2 sum m phi over the last compute_forces, T = 1/2 sum m |v|^2 for
 * d_vel [n][3] (NULL: T = 0).  Synchronises.  Errors: ESTATE. */
mibh_status mibh_energy(mibh_ctx *ctx, const float *d_vel, double *T, double *W);

/* Shared-time-step integration.  The paper integrates every step on the GPU
 * with no host traffic (Introduction, Results section) but does not name its
 * integrator; this library uses the kick-drift-kick leapfrog (second order,
 * time-reversible) on float32 state, each update one fused multiply-add.
 *
 * mibh_kick_drift: v <- v + dt_kick a, then, if dt_drift != 0,
 * x <- x + dt_drift v with the updated v, for n particles (device arrays
 * [n][3], updated in place; a as written by compute_forces, G included).
 * Enqueues one kernel.  Errors: EINVAL (null pointer, n out of range,
 * non-finite step).
 *
 * mibh_leapfrog: nsteps steps of size dt (negative dt integrates backwards):
 * forces at the initial positions, then per step kick(dt/2) + drift(dt),
 * forces (a full rebuild: shared time steps), kick(dt/2).  d_acc and d_pot
 * [n][3], [n] receive the forces of the final positions.  With
 * log_every > 0, h_log (host, log_cap >= nsteps/log_every + 1 rows) gets
 * rows (t, T, W) in float64 (mibh_energy) at step 0 and every log_every
 * steps, *nlog the number of rows; each row synchronises.  Synchronises at
 * its end and returns ENONFINITE or EOVERFLOW when any build or walk of the
 * run met that condition (a walk after such a build leaves acc/pot unwritten,
 * so the state is then void); the next build does not hide it.  Errors: as
 * mibh_forces and mibh_energy, EINVAL for a short log. */
mibh_status mibh_kick_drift(mibh_ctx *ctx, float *d_pos, float *d_vel, const float *d_acc, int64_t n,
                            float dt_kick, float dt_drift);
mibh_status mibh_leapfrog(mibh_ctx *ctx, float *d_pos, float *d_vel, const float *d_mass, int64_t n,
                          float theta, float dt, int nsteps, int log_every, float *d_acc, float *d_pot,
                          double *h_log, int log_cap, int *nlog);

/* Block time steps (the paper's Results and Discussion sections: the walk
 * visits only the particles that are due, the tree is refitted between
 * rebuilds and rebuilt when the walk slows down).  The paper names no scheme;
 * this one is hierarchical kick-drift-kick:
 *   - particle i steps with dt_max / 2^r_i, r_i in 0..max_level, the smallest
 *     r with dt_max / 2^r <= eta sqrt(eps / |a_i|) (r = 0 for a = 0);
 *   - a clock ticks in dt_max / 2^max_level; every particle drifts every
 *     tick; at tick s the particles with 2^(max_level - r_i) dividing s are
 *     due; if any is, the tree is refitted (mibh_refit) or rebuilt, the
 *     groups holding a due particle are walked (mibh_compute_forces_active),
 *     and each due
 *     particle gets its closing half kick, a new level (a larger step only
 *     where the tick is a boundary of it) and its opening half kick;
 *   - after each walk the walked groups' work count * (1 + n_pc + n_pp) is
 *     summed against the same groups' work at their first walk after the last
 *     build (the initial walk of every particle sets all of them); when the
 *     ratio exceeds 1 + rebuild_tol the next tick with a due particle rebuilds
 *     (rebuild_tol < 0: every tick rebuilds; with max_level 0 this is the
 *     shared-step mibh_leapfrog).
 * mibh_block_run starts from synchronised velocities, runs nbig steps of
 * dt_max and returns synchronised velocities, d_acc/d_pot at the final
 * positions and, when d_level is not NULL, the levels of the last step (uint8
 * [n]).  h_log (host, >= nbig + 1 rows, NULL: none) gets (t, T, W) in float64
 * at every multiple of dt_max.  Synchronises once per tick, and stops with
 * ENONFINITE or EOVERFLOW at the first tick whose build, refit or walk met
 * that condition (stats then hold the ticks run so far).  Errors: EINVAL
 * (parameters, pointers, n), as mibh_forces. */
typedef struct {
    float dt_max;       /* largest step */
    int32_t max_level;  /* 0..20: steps dt_max / 2^r, r <= max_level */
    float eta, eps;     /* step criterion dt = eta * sqrt(eps / |a|) */
    float rebuild_tol;  /* rebuild when the walked groups' work grows beyond (1 + rebuild_tol) */
} mibh_block_params;
typedef struct {
    int64_t substeps, rebuilds;     /* ticks run; rebuilds after the first build */
    int64_t active_updates;         /* sum over ticks of the particles due */
    int64_t groups_walked;          /* sum over ticks of the groups walked */
} mibh_block_stats;
mibh_status mibh_block_run(mibh_ctx *ctx, float *d_pos, float *d_vel, const float *d_mass, int64_t n,
                           float theta, const mibh_block_params *bp, int nbig, float *d_acc, float *d_pot,
                           uint8_t *d_level, mibh_block_stats *stats, double *h_log, int log_cap, int *nlog);

/* Neighbour search and SPH density on the current tree (the paper's
 * Discussion section: the tree serves neighbour search and smoothed particle
 * hydrodynamics).  Gather form: the neighbours of particle i are the j (i
 * included) with d2 <= r_i * r_i, d = x_j - x_i, d2 = (dx*dx + dy*dy) + dz*dz,
 * every operation float32 and rounded.  Needs compute_multipoles (it uses the
 * cells' particle boxes).  All arrays are device memory in input order.
 *
 * mibh_neighbor_count: d_count[i] = number of neighbours within d_radius[i]
 * (float32 [n], finite, >= 0).
 *
 * mibh_neighbor_list: the same counts, d_offset [n+1] their exclusive prefix
 * sums (d_offset[n] = *total), and, when *total <= capacity, d_index
 * [capacity] the neighbours' input indices, those of particle i in
 * d_index[d_offset[i] .. d_offset[i+1]) (order unspecified).  Synchronises
 * once (to read the total).  Errors: EOVERFLOW when *total > capacity (the
 * counts, offsets and *total are written), EINVAL, ESTATE.
 *
 * mibh_sph_density: d_rho[i] = sum over the neighbours within 2 h_i of
 * m_j W(|x_j - x_i|, h_i), W the cubic spline of Monaghan & Lattanzio (1985)
 * (W = (1 - 3/2 q^2 + 3/4 q^3)/(pi h^3) for q = r/h < 1, (2 - q)^3/(4 pi h^3)
 * for 1 <= q < 2), float32; d_count[i] the number of those neighbours; d_h
 * float32 [n], > 0. */
mibh_status mibh_neighbor_count(mibh_ctx *ctx, const float *d_radius, uint32_t *d_count);
mibh_status mibh_neighbor_list(mibh_ctx *ctx, const float *d_radius, uint32_t *d_count, uint32_t *d_offset,
                               uint32_t *d_index, int64_t capacity, int64_t *total);
mibh_status mibh_sph_density(mibh_ctx *ctx, const float *d_h, float *d_rho, uint32_t *d_count);

/* Device-to-device copy of an internal array of the current tree (for tests
 * and tools).  bytes must be at least the size reported by mibh_export_bytes.
 *   MIBH_EXPORT_KEYS    uint64 [n]        sorted Morton keys
 *   MIBH_EXPORT_PERM    uint32 [n]        sorted position -> input index
 *   MIBH_EXPORT_CELLS   uint32 [ncells][4] first, count, child_first (0 = leaf),
 *                                         system << 16 | level << 8 | nchild
 *   MIBH_EXPORT_GROUPS  uint32 [ngroups][2] first, system << 16 | level << 8 | count
 *   MIBH_EXPORT_COUNTS  uint32 [ngroups][2] particle-cell count, particle-particle count
 *   MIBH_EXPORT_MULTIPOLES float64 [ncells][10] M, com x y z, S xx yy zz xy xz yz
 *   MIBH_EXPORT_DELTA   float64 [ncells]  |com - geometric centre|
 *   MIBH_EXPORT_MAC     float32 [ncells][4] com x y z (float32), r_open^2
 *   MIBH_EXPORT_QUAD    float32 [ncells][8] M, Qxx Qyy Qzz, Qxy Qxz Qyz, 0
 *   MIBH_EXPORT_SPOS    float32 [n][4]    sorted x y z m
 *   MIBH_EXPORT_FEATURES float32 [ngroups][8] work-estimator features (mibh_group_features)
 *   MIBH_EXPORT_PREDICTIONS float32 [ngroups] estimator output of the last compute_forces
 *                                         with MIBH_ORDER_ESTIMATOR
 *   MIBH_EXPORT_QUEUE   uint32 [ngroups]  group indices in the order the last walk took them
 *                                         (ESTATE when that walk used Morton order)
 *   MIBH_EXPORT_LSIDE   float64 [ncells]  l' = max(cell side, 2 * largest per-axis distance of
 *                                         a particle from the cell's geometric centre); the
 *                                         MAC uses r_open = l'/theta + delta (l' = side unless
 *                                         particles moved out of their cells: mibh_refit)
 * Synchronises (it reads the current sizes).  Errors: EINVAL, ESTATE. */
enum {
    MIBH_EXPORT_KEYS = 0, MIBH_EXPORT_PERM, MIBH_EXPORT_CELLS, MIBH_EXPORT_GROUPS,
    MIBH_EXPORT_COUNTS, MIBH_EXPORT_MULTIPOLES, MIBH_EXPORT_DELTA, MIBH_EXPORT_MAC,
    MIBH_EXPORT_QUAD, MIBH_EXPORT_SPOS, MIBH_EXPORT_FEATURES, MIBH_EXPORT_PREDICTIONS, MIBH_EXPORT_QUEUE,
    MIBH_EXPORT_LSIDE
};
mibh_status mibh_export_bytes(mibh_ctx *ctx, int what, size_t *bytes);
mibh_status mibh_export(mibh_ctx *ctx, int what, void *d_dst, size_t bytes);

/* Stage timing with HIP events on the context's stream, for the sections the
 * paper times separately (Results section, Fig. 1): sorting (bounding cube,
 * keys, radix sort), moving (reorder), tree construction (octree, groups),
 * multipole moments, MAC preparation and the tree traverse (walk kernel).
 * mibh_profile_begin(ctx, max_steps) starts recording one set of events per
 * step (a step ends at compute_forces) for up to max_steps steps; stages a
 * step skips (a compute_forces on an existing tree) are empty;
 * mibh_profile_read synchronises, writes ms[step][MIBH_NSTAGES] for the
 * recorded steps, sets *nsteps and stops recording.  Errors: EINVAL, EHIP. */
enum {
    MIBH_STAGE_SORT = 0, MIBH_STAGE_MOVE, MIBH_STAGE_BUILD, MIBH_STAGE_MULTIPOLES, MIBH_STAGE_MACPREP,
    MIBH_STAGE_WALK, MIBH_NSTAGES
};
mibh_status mibh_profile_begin(mibh_ctx *ctx, int max_steps);
mibh_status mibh_profile_read(mibh_ctx *ctx, float *ms, int max_steps, int *nsteps);

/* Learned work estimator (not part of the paper's method; it never changes
 * the results, only the order in which the walk's persistent waves take the
 * groups).
 * An MLP 8 -> 64 -> 64 -> 1 with ReLU, float16 weights and float32
 * arithmetic predicts y = log2(1 + n_pc + n_pp) of a group from its features:
 * log2(count)/6, log2(bounding extent/L)/24, log2(|box centre - system com|/L)/24,
 * log2(density relative to the system mean)/32, theta, level/20,
 * log2(system particles)/24, log2(theta)  (L: the system's root cube side).
 * Weights: MIBH_MLP_PARAMS float16 values, layout W1[64][8], b1[64], W2[64][64],
 * b2[64], w3[64], b3.  Device pointers; all calls enqueue on `stream`. */
#define MIBH_MLP_FEATURES 8
#define MIBH_MLP_PARAMS 4801
enum { MIBH_ORDER_MORTON = 0, MIBH_ORDER_ESTIMATOR = 1, MIBH_ORDER_EXACT = 2 };

/* Features of every group of the current tree for this theta into d_feat
 * [ngroups][8] (NULL: the context's own buffer, see MIBH_EXPORT_FEATURES).
 * Errors: ESTATE before compute_multipoles, EINVAL. */
mibh_status mibh_group_features(mibh_ctx *ctx, float theta, float *d_feat);

/* Order of the walk's group queue in compute_forces (the default is MORTON).
 * MORTON: the groups in Morton order.  ESTIMATOR and EXACT: longest
 * processing time first, a stable counting sort by floor(4 log2 work),
 * heaviest bucket first and Morton order within a bucket, where work is
 * count * 2^y predicted with the float16 weights d_w16 (kept by pointer, read
 * at every compute_forces) or count * (1 + n_pc + n_pp) from the exact counts
 * of the previous walk of the same tree (MORTON when the tree is new).  The
 * order never changes the results.  Errors: EINVAL. */
mibh_status mibh_set_queue_order(mibh_ctx *ctx, int mode, const void *d_w16);

/* y[r] = MLP(x[r]) for rows r < rows (x: float32 [rows][8], y: float32 [rows]). */
mibh_status mibh_mlp_forward(const void *d_w16, const float *d_x, int64_t rows, float *d_y, void *stream);

/* Gradient of the mean squared error (1/B) sum_b (MLP(x[idx[b]]) - t[idx[b]])^2 over
 * the B = batch sampled rows idx (int32 [batch]) with respect to the MIBH_MLP_PARAMS
 * parameters, into d_grad (float32 [4801]); d_loss (float32 [1], nullable) gets the
 * loss.  d_scratch holds mibh_mlp_scratch_bytes(batch) bytes.  Deterministic. */
size_t mibh_mlp_scratch_bytes(int batch);
mibh_status mibh_mlp_gradient(const void *d_w16, const float *d_x, const float *d_t, const int32_t *d_idx,
                              int batch, float *d_grad, float *d_loss, void *d_scratch, size_t scratch_bytes,
                              void *stream);

/* One Adam step (step >= 1) on float32 master weights d_w32 with moments d_m,
 * d_v (all float32 [4801]); writes the float16 copy d_w16. */
mibh_status mibh_mlp_adam(float *d_w32, void *d_w16, const float *d_grad, float *d_m, float *d_v, int step,
                          float lr, float beta1, float beta2, float eps, void *stream);

/* Throughput probe, not part of the method: the rate that plain (non-packed)
 * float32 fused multiply-adds reach on the running GPU, against which the
 * walk's algorithmic flop rate is compared.  Launches `blocks` waves of 64
 * lanes on `stream`; lane l of wave w starts 32 accumulators at
 * v_j = ((64 w + l) mod 256) / 256 + j / 32 and applies v_j <- fma(a, b, v_j)
 * `iters` times, then stores them to d_out[(64 w + l) * 32 + j] (caller-owned
 * device memory of 2048 * blocks floats).  Work: 64 * blocks * iters * 64
 * flops.  Errors: EINVAL (null d_out, blocks outside [1, 2^20], iters < 0),
 * EHIP. */
mibh_status mibh_fma_probe(float *d_out, int32_t blocks, int32_t iters, float a, float b, void *stream);

/* Human-readable status name, and the calling thread's last error message. */
const char *mibh_status_string(mibh_status s);
const char *mibh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MIBH_H */
