// Internal definitions shared by the HIP kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mibh {

constexpr int KEY_LEVELS = 20;          // 20 bits per axis, 60-bit keys, levels 0..20
constexpr int NCOUNTERS = 22;           // per-block counters of the build: levels 0..20, groups

constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_PASSES = 8;          // 64 bits in 8-bit digits (bits 60..63 are zero)
// Sort tiles of 512 threads x 8 keys: longer runs of each digit per tile, so
// the scatter's stores coalesce better (eight passes at N = 2^22: 256 x 8
// 475 us, 512 x 8 405 us, 512 x 6 or x 10 432 us, 768 x 8 468 us, 1024 x 8 421 us).
#ifndef MIBH_SORT_THREADS
#define MIBH_SORT_THREADS 512
#endif
constexpr int SORT_THREADS = MIBH_SORT_THREADS;  // a multiple of RADIX, <= 1024
#ifndef MIBH_SORT_ITEMS
#define MIBH_SORT_ITEMS 8
#endif
constexpr int SORT_ITEMS = MIBH_SORT_ITEMS;  // keys per thread per tile
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;

// particles per build block (tree construction at N = 2^22: 256 175 us, 512 150 us, 1024 162 us)
#ifndef MIBH_BUILD_THREADS
#define MIBH_BUILD_THREADS 512
#endif
constexpr int BUILD_THREADS = MIBH_BUILD_THREADS;
constexpr int MAX_WINDOW = 64;          // largest ncrit and group_cap (a build wave's window reach)
constexpr int BBOX_BLOCKS = 1024;
constexpr int ENERGY_BLOCKS = 1024;
constexpr int ENERGY_THREADS = 256;

// Walk: one wave per workgroup; cell stack bound (see walk kernel): every
// traversal step pushes at most 64*8 children and at most one step's pushes
// per level are on the stack at any time, so 1 + 20*512 entries suffice.
constexpr unsigned STACK_CAP = 21u * 512u;

enum : unsigned {
    FLAG_NONFINITE = 1u,
    FLAG_NEGMASS = 2u,
    FLAG_STACK = 4u,
    FLAG_CELLCAP = 8u,
};

// Per-system root cube: corner lo (x, y, z) and side 2^k.
struct SysCube {
    float lo[3];
    int k;
};

constexpr int MAX_SYSTEMS = 256;        // systems per batch (one extra 8-bit sort pass)
constexpr int MLP_IN = 8, MLP_H = 64;   // work estimator 8 -> 64 -> 64 -> 1
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 4801
constexpr int BBOX_MIN_BLOCKS = 16;     // bounding-box blocks per system at least

// Device-resident per-context state, rewritten by every build (zeroed once
// when the context is created).
struct Header {
    unsigned nsys;          // systems in the current batch (1 for a single system)
    unsigned flags;         // conditions met since the current build started
    unsigned sticky;        // flags of the earlier builds since the drivers last cleared it
    unsigned n;
    unsigned ncells;
    unsigned ngroups;
    unsigned lvl_begin[24]; // cells of level l are [lvl_begin[l], lvl_begin[l+1]), l = 0..20
    // Heads of the walks' group queues (one per XCD, 256 bytes apart).  Every
    // wave of a walk increments them, so they sit on cache lines of their own:
    // sharing a line with the fields above, which every wave reads, made the
    // walk 1.8 times slower.
    alignas(256) unsigned walk_head[8 * 64];
    // Shared-prefix walk: heads of the anchor pass's queues (as walk_head), then
    // the allocation head of the anchor-list pool and the number of anchors.
    alignas(256) unsigned prefix_head[8 * 64];
    alignas(256) unsigned long long pool_head;
    unsigned anchor_count;
    unsigned anchor_fail;  // anchors whose lists did not fit
    unsigned pool_pad[60];
};

// Group queues of the persistent walks.  gfx950 deals the workgroups of a
// launch to its 8 XCDs in turn (workgroup i to XCD i mod 8), and each XCD has
// its own L2.  Queue q holds the slots [q n / 8, (q + 1) n / 8) of the
// processing order (Morton order by default), so the waves of one XCD walk
// neighbouring groups, whose cells they then share in that XCD's L2.  A wave
// takes slots from its XCD's queue, then from the following queues in turn as
// each runs empty, and stops when all are empty.
constexpr unsigned WALK_QUEUES = 8;
constexpr unsigned QUEUE_STRIDE = 64;  // words between queue heads

struct QueueCursor {
    unsigned q, tried;  // queue in use, queues found empty
};

__device__ __forceinline__ QueueCursor queue_start() { return QueueCursor{blockIdx.x % WALK_QUEUES, 0u}; }

// Next slot for the calling wave, or n when every queue is empty.  Every lane
// calls it (lane 0 adds 1, the others 0), so no lane-dependent branch is
// needed around it.
__device__ __forceinline__ unsigned queue_next(unsigned *heads, unsigned n, QueueCursor &qc) {
    while (qc.tried < WALK_QUEUES) {
        const unsigned lo = (unsigned)((unsigned long long)n * qc.q / WALK_QUEUES);
        const unsigned hi = (unsigned)((unsigned long long)n * (qc.q + 1u) / WALK_QUEUES);
        const unsigned s = __builtin_amdgcn_readfirstlane(
            atomicAdd(heads + QUEUE_STRIDE * qc.q, __lane_id() == 0 ? 1u : 0u));
        if (s < hi - lo) return lo + s;
        qc.tried++;
        qc.q = (qc.q + 1u) % WALK_QUEUES;
    }
    return n;
}

// Walk queue order by predicted or measured work: quarter-octave buckets of
// log2(work), heaviest first, Morton order within a bucket.
constexpr int ORDER_BUCKETS = 128;
constexpr int ORDER_BLOCKS = 256;

// Walk: LDS capacities per wave (one wave per workgroup).
constexpr unsigned WALK_LSTACK = 512;   // cell stack in LDS (spills to the global stack)
// Shared-prefix walk: per-wave scratch for an anchor cell's lists: the cells it
// accepts (F), then the cells left for each group, raw and sorted by level (S).
constexpr unsigned PREFIX_F_CAP = 3072;
constexpr unsigned PREFIX_S_CAP = 512;  // a seed of <= 512 cells fits the walk's LDS ring and keeps
                                        // the stack within STACK_CAP
constexpr unsigned PREFIX_SCRATCH = PREFIX_F_CAP + 2 * PREFIX_S_CAP;
// Pool words per particle for all anchors' lists: 16 >> (anchor_up - 1), as
// anchors get fewer and larger with their height (at N = 2^22 in a Plummer
// sphere the lists take about 0.8 words per particle at height 3); capped at
// 2^32 - 1 words, the reach of a 32-bit offset.  Anchors that find no room
// leave their groups to walk from the root.
constexpr unsigned PREFIX_POOL_WORDS_1 = 16;
constexpr unsigned PREFIX_STEP = 4;     // stack cells per lane in one step of an anchor's traversal
constexpr unsigned PREFIX_RING = 4096;  // LDS stack ring of the anchor-list pass
constexpr unsigned WALK_PC_LDS = 1024;  // particle-cell list
constexpr unsigned WALK_PP_LDS = 512;   // particle-particle list
static_assert(WALK_PC_LDS % 64 == 0 && WALK_PP_LDS % 64 == 0, "lists hold whole 64-entry tiles");
// A list's last tile is padded with a massless source this far away (its
// terms are exact zeros): the cell at index cap_cells (cmac, ceval) and the
// particle at index n_max (spos), one entry past the cells and particles.
constexpr float WALK_FAR = 1.0e18f;

// Device pointers carved from the caller's workspace.
struct Buffers {
    Header *hdr;
    SysCube *cube;          // [max_systems]
    uint32_t *sys_off;      // [max_systems + 1] first particle of each system (input = sorted order)
    uint8_t *sys8;          // [n] system of each input particle (batches only)
    float *bbox_part;       // [max_systems][bbox blocks per system][8]
    uint64_t *keys[2];
    uint32_t *vals[2];
    uint32_t *hist;         // [RADIX][ntiles]
    uint32_t *btot;         // [RADIX]
    float4 *ppack;          // input x, y, z, m packed by the keys kernel (one line per gather)
    float4 *spos;           // sorted x, y, z, m
    int8_t *cl;             // common leading octal digits with the previous key (-1 at 0)
    uchar4 *lvinfo;         // per particle: first level started, leaf level, group level, group start
    uint32_t *blkcnt;       // [NCOUNTERS][nblk]
    uint32_t *ctot;         // [NCOUNTERS]
    uint4 *topo;            // cells: first, count, child_first, system<<16 | level<<8 | nchild
    double *mp;             // cells: [10] M, com xyz, S xx yy zz xy xz yz
    double *delta;          // cells: |com - centre|
    float *cbox;            // cells: [6] bounding box of the cell's particles (min xyz, max xyz)
    double *lside;          // cells: l' = max(side, 2 * largest per-axis distance of a particle from the centre)
    float4 *cmac;           // cells: com32 xyz, r_open^2
    float4 *ceval;          // cells: [2] (M, Qxx, Qyy, Qzz), (Qxy, Qxz, Qyz, 0)
    uint2 *groups;          // first, system<<16 | level<<8 | count
    uint2 *gcounts;         // n_pc, n_pp
    uint32_t *wstack;       // per walk wave: STACK_CAP (spill of the LDS stack)
    float *feat;            // work estimator: group features [n][8]
    float *pred;            // work estimator: predicted log2(1 + n_pc + n_pp) per group
    uint8_t *level;         // block time steps: level of every particle (input order)
    uint8_t *active;        // block time steps: particle due at the current tick
    uint32_t *gref;         // block time steps: work of a group at its first walk after a build (0: none)
    unsigned long long *bsum;  // block time steps: [0] work now, [1] reference work, [2] due particles
    uint32_t *qorder;       // walk queue: groups in processing order (work-ordered modes)
    uint32_t *anchor;       // shared-prefix walk: anchor cell of each group
    uint32_t *alist;        // shared-prefix walk: the anchor cells, each once
    uint4 *arec;            // shared-prefix walk, per cell: pool offset, |F|, |S|, 1 if the lists are valid
                            // (2 while claimed, before the lists are built)
    uint32_t *pool;         // shared-prefix walk: the anchors' F and S lists
    uint32_t *pscr;         // shared-prefix walk: PREFIX_SCRATCH words per walk wave
    unsigned long long pool_cap;  // words of the pool
    uint32_t *ohist;        // [ORDER_BUCKETS][ORDER_BLOCKS] bucket counts of the queue order
    double *epart;          // energy partials [ENERGY_BLOCKS][2]
    unsigned cap_cells, n_max, ntiles_max, nblk_max;
    unsigned walk_waves, pc_cap, pp_cap, max_systems;
};

// System of sorted or input position i: the s with sys_off[s] <= i < sys_off[s+1].
__device__ __forceinline__ unsigned system_of(const uint32_t *__restrict__ sys_off, unsigned nsys, unsigned i) {
    unsigned lo = 0, hi = nsys;  // sys_off[lo] <= i < sys_off[hi]
    while (hi - lo > 1) {
        const unsigned mid = (lo + hi) >> 1;
        if (sys_off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Host launchers (kernels live in the .hip files).
hipError_t launch_bbox(const Buffers &b, const float *pos, const float *mass, unsigned n, unsigned nsys,
                       hipStream_t s);
hipError_t launch_keys(const Buffers &b, const float *pos, const float *mass, unsigned n, unsigned nsys,
                       hipStream_t s);
hipError_t launch_sort(const Buffers &b, unsigned n, unsigned nsys, hipStream_t s);
// buffer (0 or 1) that holds the sorted keys and permutation after launch_sort
inline int sorted_buffer(unsigned nsys) { return nsys > 1 ? (SORT_PASSES + 1) & 1 : SORT_PASSES & 1; }
hipError_t launch_reorder(const Buffers &b, unsigned n, unsigned nsys, hipStream_t s);
hipError_t launch_build(const Buffers &b, unsigned n, unsigned nsys, int ncrit, int gcap, hipStream_t s);
hipError_t launch_multipoles(const Buffers &b, unsigned nsys, hipStream_t s);
// theta: the float32 opening angle widened to float64
hipError_t launch_mac_prep(const Buffers &b, unsigned nsys, double theta, hipStream_t s);
// order: the queue (NULL: groups in Morton order); qlen: device count of queue
// entries to walk (NULL: every group)
// anchor_up > 0: groups share the traversal of their ancestor anchor_up levels up
hipError_t launch_walk(const Buffers &b, unsigned n, unsigned nsys, float eps2, float G, int precision,
                       const uint32_t *order, const uint32_t *qlen, const uint8_t *active, float *acc, float *pot,
                       int anchor_up, hipStream_t s);
hipError_t launch_features(const Buffers &b, float theta, float *feat, hipStream_t s);
hipError_t launch_mlp_forward(const void *w16, const float *x, unsigned rows, const Header *hdr, float *y,
                              hipStream_t s);
size_t mlp_scratch_bytes(unsigned batch);
hipError_t launch_mlp_grad(const void *w16, const float *x, const float *target, const int *idx, unsigned batch,
                           float *grad, float *loss, void *scratch, hipStream_t s);
hipError_t launch_adam(float *w32, void *w16, const float *grad, float *m, float *v, int step, float lr,
                       float beta1, float beta2, float eps, hipStream_t s);
// Writes b.qorder: the groups ordered by work, heaviest first; mode 1: work
// predicted by the estimator (b.pred), 2: exact counts of the last walk; mode
// 3: groups holding a particle with active[input index] != 0 first (their
// number, after the call, is b.ohist[ORDER_BLOCKS]), in Morton order.
hipError_t launch_queue_order(const Buffers &b, int mode, const uint8_t *active, unsigned nsys, hipStream_t s);
// Packs input (x, y, z, m) into b.ppack and flags non-finite or negative values.
hipError_t launch_pack(const Buffers &b, const float *pos, const float *mass, unsigned n, hipStream_t s);
// v <- v + dt_kick a, then (dt_drift != 0) x <- x + dt_drift v, for n particles
hipError_t launch_kick_drift(float *pos, float *vel, const float *acc, unsigned n, float dt_kick, float dt_drift,
                             hipStream_t s);
// block time steps
enum : int { BLOCK_CLOSE = 1, BLOCK_LEVEL = 2, BLOCK_OPEN = 4 };
hipError_t launch_block_active(const uint8_t *level, unsigned n, unsigned tick, int R, uint8_t *active,
                               unsigned long long *nactive, hipStream_t s);
hipError_t launch_block_kick(float *vel, const float *acc, uint8_t *level, unsigned n, unsigned tick, int R,
                             float dt_max, int flags, double eta, double eps, hipStream_t s);
hipError_t launch_rebuild_check(const Buffers &b, const uint32_t *qlen, unsigned long long *sums, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, unsigned n, uint32_t v, hipStream_t s);
// neighbour search (mode 0 counts, 1 lists, 2 SPH density); needs the cell boxes of compute_multipoles
hipError_t launch_neighbors(const Buffers &b, int mode, const float *radius, uint32_t *count, const uint32_t *offset,
                            uint32_t *index, float *rho, unsigned nsys, hipStream_t s);
// exclusive scan of n counts into out[0..n], out[n] = total; tmp holds (n + 1023) / 1024 words
hipError_t launch_scan_u32(const uint32_t *in, unsigned n, uint32_t *out, uint32_t *tmp, hipStream_t s);
hipError_t launch_energy(const Buffers &b, const float *mass, const float *pot, const float *vel,
                         unsigned n, double *d_out2, hipStream_t s);

}  // namespace mibh
