// Host side of the C ABI declared in include/mibh.h: workspace layout,
// argument checks, launch sequencing on the caller's stream.
#include "mibh.h"
#include "mibh_device.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

using namespace mibh;

// queue mode of a walk over the groups holding an active particle (internal)
constexpr int ORDER_ACTIVE = 3;
// the neighbour-list offset scan keeps its tile sums in the queue-order counts
constexpr int SCAN_MAX_TILES = ORDER_BUCKETS * ORDER_BLOCKS;

struct mibh_ctx {
    mibh_params p;
    int64_t n_max;
    int nsys;                 // systems of the current tree
    int order;                // walk queue order: MIBH_ORDER_*
    int last_order;           // order the last walk used (Morton when exact counts were missing)
    const void *est_w16;      // estimator weights (float16, caller-owned)
    int counts_valid;         // gcounts belong to the current tree
    hipGraph_t graph;         // captured step (mibh_graph_capture)
    hipGraphExec_t graph_exec;
    int graph_nsys;
    int64_t graph_n;
    const float *graph_pos, *graph_mass;
    float *graph_acc, *graph_pot;
    hipStream_t stream;
    int device;
    Buffers b;
    int state;  // 0 nothing, 1 tree built, 2 multipoles, 3 forces
    int64_t n;
    const float *pos, *mass;
    float *acc, *pot;
    double *h_energy;  // pinned 8 words: mibh_energy's two sums, or the block driver's counters
    double *d_energy;  // 2 doubles in the workspace
    // stage events: MIBH_NSTAGES + 1 per profiled step
    hipEvent_t *events;
    int prof_max, prof_step;
    int prof_last;            // last stage recorded in the current step (-2: none)
};

namespace {

thread_local char g_err[512] = "";

mibh_status fail(mibh_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

mibh_status hip_fail(hipError_t e, const char *where) {
    return fail(MIBH_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(call, where)                         \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

constexpr size_t ALIGN = 256;
constexpr int DEFAULT_WALK_WAVES = 4096;  // 16 per compute unit on 256 CUs

size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// System offsets travel to the device as a kernel argument, so a captured
// graph holds them by value and no host staging buffer is needed.
struct SysOffsets {
    unsigned nsys;
    unsigned off[MAX_SYSTEMS + 1];
};

__global__ void k_set_offsets(SysOffsets o, uint32_t *__restrict__ sys_off) {
    for (unsigned i = threadIdx.x; i <= o.nsys; i += blockDim.x) sys_off[i] = o.off[i];
}

bool params_valid(const mibh_params &p) {
    return p.ncrit >= 1 && p.group_cap >= p.ncrit && p.group_cap <= 64 && p.eps2 >= 0.0f &&
           p.max_systems >= 1 && p.max_systems <= MAX_SYSTEMS &&
           isfinite(p.eps2) && isfinite(p.G) && (p.precision == MIBH_PLAIN || p.precision == MIBH_KAHAN || p.precision == MIBH_KAHAN_TERM) &&
           p.walk_waves >= 0 && p.walk_waves <= (1 << 20) && p.pc_cap >= 128 && p.pp_cap >= 128 &&
           p.pc_cap <= (int)WALK_PC_LDS && p.pp_cap <= (int)WALK_PP_LDS && p.anchor_up >= 0 && p.anchor_up <= 4;
}

// Assigns every buffer of the layout from `base` (nullptr: sizing only) and
// returns the total bytes.
size_t layout(int64_t n_max, const mibh_params &p, char *base, Buffers *b) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *ptr = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return ptr;
    };
    const size_t n = (size_t)n_max;
    const size_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    const size_t nblk = (n + BUILD_THREADS - 1) / BUILD_THREADS;
    // leaves are disjoint and non-empty (<= n); internal cells hold > ncrit
    // particles each and every particle has at most 20 internal ancestors
    const size_t cap_cells = n + (20 * n) / (size_t)(p.ncrit + 1) + 2;
    const size_t waves = p.walk_waves ? (size_t)p.walk_waves : DEFAULT_WALK_WAVES;
    const size_t nsys = (size_t)p.max_systems;
    const size_t bbox_blocks = nsys * (size_t)std::max(BBOX_MIN_BLOCKS, BBOX_BLOCKS / (int)nsys);
    Buffers t;
    t.hdr = (Header *)take(sizeof(Header));
    t.cube = (SysCube *)take(sizeof(SysCube) * nsys);
    t.sys_off = (uint32_t *)take(4 * (nsys + 1));
    t.sys8 = (uint8_t *)take(nsys > 1 ? n : 1);
    t.bbox_part = (float *)take(sizeof(float) * 8 * std::max(bbox_blocks, (size_t)BBOX_BLOCKS));
    t.keys[0] = (uint64_t *)take(8 * n);
    t.keys[1] = (uint64_t *)take(8 * n);
    t.vals[0] = (uint32_t *)take(4 * n);
    t.vals[1] = (uint32_t *)take(4 * n);
    t.hist = (uint32_t *)take(4 * RADIX * ntiles);
    t.btot = (uint32_t *)take(4 * RADIX);
    t.ppack = (float4 *)take(16 * n);
    t.spos = (float4 *)take(16 * (n + 1));  // + the padding particle
    t.cl = (int8_t *)take(n);
    t.lvinfo = (uchar4 *)take(4 * n);
    t.blkcnt = (uint32_t *)take(4 * NCOUNTERS * nblk);
    t.ctot = (uint32_t *)take(4 * NCOUNTERS);
    t.topo = (uint4 *)take(16 * cap_cells);
    t.mp = (double *)take(80 * cap_cells);
    t.delta = (double *)take(8 * cap_cells);
    t.cbox = (float *)take(24 * cap_cells);
    t.lside = (double *)take(8 * cap_cells);
    t.cmac = (float4 *)take(16 * (cap_cells + 1));   // + the padding cell
    t.ceval = (float4 *)take(32 * (cap_cells + 1));
    t.groups = (uint2 *)take(8 * n);
    t.gcounts = (uint2 *)take(8 * n);
    t.wstack = (uint32_t *)take(4 * (size_t)STACK_CAP * waves);
    t.feat = (float *)take(4 * (size_t)MLP_IN * n);
    t.pred = (float *)take(4 * n);
    t.level = (uint8_t *)take(4 * ((n + 3) / 4));
    t.active = (uint8_t *)take(4 * ((n + 3) / 4));
    t.gref = (uint32_t *)take(4 * n);
    t.bsum = (unsigned long long *)take(8 * 4);
    t.qorder = (uint32_t *)take(4 * n);
    const bool shared_walk = p.anchor_up > 0;
    t.anchor = shared_walk ? (uint32_t *)take(4 * n) : nullptr;
    t.alist = shared_walk ? (uint32_t *)take(4 * n) : nullptr;
    t.arec = shared_walk ? (uint4 *)take(16 * cap_cells) : nullptr;
    const size_t pool_words =
        shared_walk ? std::min<size_t>((size_t)(PREFIX_POOL_WORDS_1 >> (p.anchor_up - 1)) * n, 0xffffffffull) : 0;
    t.pool = shared_walk ? (uint32_t *)take(4 * pool_words) : nullptr;
    t.pscr = shared_walk ? (uint32_t *)take(4 * (size_t)PREFIX_SCRATCH * waves) : nullptr;
    t.pool_cap = pool_words;
    t.ohist = (uint32_t *)take(4 * ORDER_BUCKETS * ORDER_BLOCKS);
    t.epart = (double *)take(8 * 2 * ENERGY_BLOCKS + 16);
    t.cap_cells = (unsigned)cap_cells;
    t.n_max = (unsigned)n_max;
    t.ntiles_max = (unsigned)ntiles;
    t.nblk_max = (unsigned)nblk;
    t.walk_waves = (unsigned)waves;
    t.pc_cap = (unsigned)p.pc_cap;
    t.pp_cap = (unsigned)p.pp_cap;
    t.max_systems = (unsigned)p.max_systems;
    if (b) *b = t;
    return off;
}

mibh_status check_ctx(mibh_ctx *ctx) {
    if (!ctx) return fail(MIBH_EINVAL, "null context");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return MIBH_OK;
}

mibh_status read_header(mibh_ctx *ctx, Header *h) {
    HIP_TRY(hipMemcpyAsync(h, ctx->b.hdr, sizeof(Header), hipMemcpyDeviceToHost, ctx->stream),
            "hipMemcpyAsync(header)");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return MIBH_OK;
}

mibh_status flags_status(unsigned flags) {
    if (flags & (FLAG_NONFINITE | FLAG_NEGMASS))
        return fail(MIBH_ENONFINITE, "input has a non-finite position or mass, or a negative mass");
    if (flags & (FLAG_STACK | FLAG_CELLCAP)) return fail(MIBH_EOVERFLOW, "device capacity exceeded (flags %u)", flags);
    return MIBH_OK;
}

// Drivers running many builds: clears the sticky flags once the driver's first
// build has moved the flags of earlier calls into them (stream order).
hipError_t clear_sticky(mibh_ctx *ctx) {
    return launch_fill_u32(&ctx->b.hdr->sticky, 1u, 0u, ctx->stream);
}

// Every condition met by any build since clear_sticky (syncs).
mibh_status driver_flags(mibh_ctx *ctx) {
    Header h;
    mibh_status st = read_header(ctx, &h);
    if (st) return st;
    return flags_status(h.flags | h.sticky);
}

}  // namespace

extern "C" {

void mibh_default_params(mibh_params *p) {
    if (!p) return;
    p->ncrit = 16;
    p->group_cap = 64;
    p->eps2 = 0.0f;
    p->G = 1.0f;
    p->precision = MIBH_PLAIN;
    p->walk_waves = 0;
    p->pc_cap = (int32_t)WALK_PC_LDS;
    p->pp_cap = (int32_t)WALK_PP_LDS;
    p->max_systems = 1;
    p->anchor_up = 3;
}

size_t mibh_workspace_bytes(int64_t n_max, const mibh_params *pp) {
    mibh_params p;
    if (pp) p = *pp; else mibh_default_params(&p);
    if (n_max < 1 || n_max >= ((int64_t)1 << 31) || !params_valid(p)) return 0;
    return layout(n_max, p, nullptr, nullptr);
}

mibh_status mibh_create(const mibh_params *pp, int64_t n_max, void *d_workspace, size_t workspace_bytes,
                        void *stream, mibh_ctx **out) {
    if (!out) return fail(MIBH_EINVAL, "null output pointer");
    *out = nullptr;
    mibh_params p;
    if (pp) p = *pp; else mibh_default_params(&p);
    if (!params_valid(p)) return fail(MIBH_EINVAL, "invalid parameters");
    if (n_max < 1 || n_max >= ((int64_t)1 << 31)) return fail(MIBH_EINVAL, "n_max out of range");
    if (!d_workspace || ((uintptr_t)d_workspace % ALIGN) != 0)
        return fail(MIBH_EINVAL, "workspace must be non-null and 256-byte aligned");
    const size_t need = layout(n_max, p, nullptr, nullptr);
    if (workspace_bytes < need)
        return fail(MIBH_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
    mibh_ctx *c = new (std::nothrow) mibh_ctx();
    if (!c) return fail(MIBH_ENOMEM, "host allocation failed");
    c->p = p;
    c->n_max = n_max;
    c->stream = (hipStream_t)stream;
    c->state = 0;
    c->n = 0;
    c->pos = c->mass = nullptr;
    c->acc = c->pot = nullptr;
    c->events = nullptr;
    c->prof_max = c->prof_step = 0;
    c->prof_last = -2;
    c->nsys = 1;
    c->order = c->last_order = MIBH_ORDER_MORTON;
    c->est_w16 = nullptr;
    c->counts_valid = 0;
    c->graph = nullptr;
    c->graph_exec = nullptr;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetDevice");
    }
    layout(n_max, p, (char *)d_workspace, &c->b);
    c->d_energy = c->b.epart + 2 * ENERGY_BLOCKS;
    e = hipHostMalloc((void **)&c->h_energy, 8 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipHostMalloc");
    }
    // flags and sticky flags start clear (the workspace arrives uninitialised)
    e = launch_fill_u32(reinterpret_cast<uint32_t *>(c->b.hdr), (unsigned)(sizeof(Header) / 4), 0u, c->stream);
    if (e != hipSuccess) {
        (void)hipHostFree(c->h_energy);
        delete c;
        return hip_fail(e, "header fill");
    }
    *out = c;
    return MIBH_OK;
}

static void free_events(mibh_ctx *ctx) {
    if (!ctx->events) return;
    for (int i = 0; i < ctx->prof_max * (MIBH_NSTAGES + 1); i++)
        if (ctx->events[i]) (void)hipEventDestroy(ctx->events[i]);
    free(ctx->events);
    ctx->events = nullptr;
    ctx->prof_max = ctx->prof_step = 0;
}

// Records the event that ends stage `stage` (stage -1: the step's start).
static mibh_status mark(mibh_ctx *ctx, int stage) {
    if (!ctx->events || ctx->prof_step >= ctx->prof_max) return MIBH_OK;
    // stages that this step skipped (a walk of an existing tree) end here: zero length
    for (int s = ctx->prof_last + 1; s <= stage; s++) {
        hipEvent_t e = ctx->events[ctx->prof_step * (MIBH_NSTAGES + 1) + s + 1];
        HIP_TRY(hipEventRecord(e, ctx->stream), "hipEventRecord");
    }
    if (stage > ctx->prof_last) ctx->prof_last = stage;
    return MIBH_OK;
}

mibh_status mibh_destroy(mibh_ctx *ctx) {
    if (!ctx) return MIBH_OK;
    (void)hipSetDevice(ctx->device);
    free_events(ctx);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->h_energy) (void)hipHostFree(ctx->h_energy);
    delete ctx;
    return MIBH_OK;
}

mibh_status mibh_build_tree_batch(mibh_ctx *ctx, const float *d_pos, const float *d_mass,
                                  const int64_t *h_offsets, int nsys) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!d_pos || !d_mass || !h_offsets) return fail(MIBH_EINVAL, "null input pointer");
    if (nsys < 1 || nsys > ctx->p.max_systems)
        return fail(MIBH_EINVAL, "nsys = %d outside [1, max_systems = %d]", nsys, ctx->p.max_systems);
    if (h_offsets[0] != 0) return fail(MIBH_EINVAL, "offsets[0] must be 0");
    for (int s = 0; s < nsys; s++)
        if (h_offsets[s + 1] <= h_offsets[s]) return fail(MIBH_EINVAL, "system %d is empty or offsets decrease", s);
    const int64_t n = h_offsets[nsys];
    if (n > ctx->n_max) return fail(MIBH_EINVAL, "n = %lld > n_max = %lld", (long long)n, (long long)ctx->n_max);
    SysOffsets o;
    o.nsys = (unsigned)nsys;
    for (int s = 0; s <= nsys; s++) o.off[s] = (unsigned)h_offsets[s];
    const unsigned un = (unsigned)n, us = (unsigned)nsys;
    hipStream_t s = ctx->stream;
    if ((st = mark(ctx, -1))) return st;
    hipLaunchKernelGGL(k_set_offsets, dim3(1), dim3(256), 0, s, o, ctx->b.sys_off);
    HIP_TRY(hipGetLastError(), "set_offsets");
    HIP_TRY(launch_bbox(ctx->b, d_pos, d_mass, un, us, s), "bbox");
    HIP_TRY(launch_keys(ctx->b, d_pos, d_mass, un, us, s), "keys");
    HIP_TRY(launch_sort(ctx->b, un, us, s), "sort");
    if ((st = mark(ctx, MIBH_STAGE_SORT))) return st;
    HIP_TRY(launch_reorder(ctx->b, un, us, s), "reorder");
    if ((st = mark(ctx, MIBH_STAGE_MOVE))) return st;
    HIP_TRY(launch_build(ctx->b, un, us, ctx->p.ncrit, ctx->p.group_cap, s), "build");
    if ((st = mark(ctx, MIBH_STAGE_BUILD))) return st;
    ctx->n = n;
    ctx->nsys = nsys;
    ctx->counts_valid = 0;
    ctx->pos = d_pos;
    ctx->mass = d_mass;
    ctx->state = 1;
    return MIBH_OK;
}

mibh_status mibh_build_tree(mibh_ctx *ctx, const float *d_pos, const float *d_mass, int64_t n) {
    if (ctx && (n < 1 || n > ctx->n_max))
        return fail(MIBH_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)ctx->n_max);
    const int64_t off[2] = {0, n};
    return mibh_build_tree_batch(ctx, d_pos, d_mass, off, 1);
}

mibh_status mibh_compute_multipoles(mibh_ctx *ctx) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (ctx->state < 1) return fail(MIBH_ESTATE, "compute_multipoles before build_tree");
    if ((st = mark(ctx, MIBH_STAGE_BUILD))) return st;  // no-op after a build in this step
    HIP_TRY(launch_multipoles(ctx->b, (unsigned)ctx->nsys, ctx->stream), "multipoles");
    if ((st = mark(ctx, MIBH_STAGE_MULTIPOLES))) return st;
    ctx->state = 2;
    return MIBH_OK;
}

// The force step on the current tree: every group (active == nullptr) or the
// groups holding a particle with active[input index] != 0.
static mibh_status forces_impl(mibh_ctx *ctx, float theta, const uint8_t *d_active, float *d_acc, float *d_pot) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (ctx->state < 2) return fail(MIBH_ESTATE, "compute_forces before compute_multipoles");
    if (!(theta > 0.0f) || !isfinite(theta)) return fail(MIBH_EINVAL, "theta must be finite and > 0");
    if (!d_acc || !d_pot) return fail(MIBH_EINVAL, "null output pointer");

    if ((st = mark(ctx, MIBH_STAGE_MULTIPOLES))) return st;  // no-op after compute_multipoles in this step
    HIP_TRY(launch_mac_prep(ctx->b, (unsigned)ctx->nsys, (double)theta, ctx->stream), "mac_prep");
    int mode = d_active ? ORDER_ACTIVE : ctx->order;
    if (mode == MIBH_ORDER_EXACT && !ctx->counts_valid) mode = MIBH_ORDER_MORTON;  // no walk of this tree yet
    if (mode == MIBH_ORDER_ESTIMATOR) {
        HIP_TRY(launch_features(ctx->b, theta, ctx->b.feat, ctx->stream), "features");
        HIP_TRY(launch_mlp_forward(ctx->est_w16, ctx->b.feat, 0, ctx->b.hdr, ctx->b.pred, ctx->stream), "estimator");
    }
    if (mode != MIBH_ORDER_MORTON)
        HIP_TRY(launch_queue_order(ctx->b, mode, d_active, (unsigned)ctx->nsys, ctx->stream), "queue order");
    if ((st = mark(ctx, MIBH_STAGE_MACPREP))) return st;
    HIP_TRY(launch_walk(ctx->b, (unsigned)ctx->n, (unsigned)ctx->nsys, ctx->p.eps2, ctx->p.G, ctx->p.precision,
                        mode == MIBH_ORDER_MORTON ? nullptr : ctx->b.qorder,
                        d_active ? ctx->b.ohist + ORDER_BLOCKS : nullptr, d_active, d_acc, d_pot, ctx->p.anchor_up,
                        ctx->stream),
            "walk");
    ctx->last_order = mode;
    if ((st = mark(ctx, MIBH_STAGE_WALK))) return st;
    ctx->counts_valid = 1;
    if (ctx->events && ctx->prof_step < ctx->prof_max) {
        ctx->prof_step++;
        ctx->prof_last = -2;
    }
    ctx->acc = d_acc;
    ctx->pot = d_pot;
    ctx->state = 3;
    return MIBH_OK;
}

mibh_status mibh_compute_forces(mibh_ctx *ctx, float theta, float *d_acc, float *d_pot) {
    return forces_impl(ctx, theta, nullptr, d_acc, d_pot);
}

mibh_status mibh_compute_forces_active(mibh_ctx *ctx, float theta, const uint8_t *d_active, float *d_acc,
                                       float *d_pot) {
    if (!d_active) return fail(MIBH_EINVAL, "null active mask");
    return forces_impl(ctx, theta, d_active, d_acc, d_pot);
}

mibh_status mibh_refit(mibh_ctx *ctx, const float *d_pos, const float *d_mass) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (ctx->state < 1) return fail(MIBH_ESTATE, "refit before build_tree");
    if (!d_pos || !d_mass) return fail(MIBH_EINVAL, "null input pointer");
    if ((st = mark(ctx, MIBH_STAGE_SORT))) return st;  // a refit has no sorting or tree construction
    HIP_TRY(launch_pack(ctx->b, d_pos, d_mass, (unsigned)ctx->n, ctx->stream), "pack");
    HIP_TRY(launch_reorder(ctx->b, (unsigned)ctx->n, (unsigned)ctx->nsys, ctx->stream), "reorder");
    if ((st = mark(ctx, MIBH_STAGE_BUILD))) return st;
    ctx->pos = d_pos;
    ctx->mass = d_mass;
    ctx->state = 1;
    return MIBH_OK;
}

mibh_status mibh_forces(mibh_ctx *ctx, const float *d_pos, const float *d_mass, int64_t n, float theta,
                        float *d_acc, float *d_pot) {
    if (!(theta > 0.0f) || !isfinite(theta)) return fail(MIBH_EINVAL, "theta must be finite and > 0");
    if (!d_acc || !d_pot) return fail(MIBH_EINVAL, "null output pointer");
    mibh_status st = mibh_build_tree(ctx, d_pos, d_mass, n);
    if (st) return st;
    if ((st = mibh_compute_multipoles(ctx))) return st;
    return mibh_compute_forces(ctx, theta, d_acc, d_pot);
}

mibh_status mibh_kick_drift(mibh_ctx *ctx, float *d_pos, float *d_vel, const float *d_acc, int64_t n,
                            float dt_kick, float dt_drift) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!d_pos || !d_vel || !d_acc) return fail(MIBH_EINVAL, "null pointer");
    if (n < 1 || n > ctx->n_max)
        return fail(MIBH_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)ctx->n_max);
    if (!isfinite(dt_kick) || !isfinite(dt_drift)) return fail(MIBH_EINVAL, "time steps must be finite");
    HIP_TRY(launch_kick_drift(d_pos, d_vel, d_acc, (unsigned)n, dt_kick, dt_drift, ctx->stream), "kick_drift");
    return MIBH_OK;
}

mibh_status mibh_leapfrog(mibh_ctx *ctx, float *d_pos, float *d_vel, const float *d_mass, int64_t n, float theta,
                          float dt, int nsteps, int log_every, float *d_acc, float *d_pot, double *h_log,
                          int log_cap, int *nlog) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!d_pos || !d_vel || !d_mass || !d_acc || !d_pot) return fail(MIBH_EINVAL, "null pointer");
    if (!isfinite(dt)) return fail(MIBH_EINVAL, "dt must be finite");
    if (nsteps < 0 || log_every < 0) return fail(MIBH_EINVAL, "nsteps and log_every must be >= 0");
    const int need = log_every > 0 ? nsteps / log_every + 1 : 0;
    if (need > 0 && (!h_log || log_cap < need))
        return fail(MIBH_EINVAL, "energy log needs %d entries, capacity %d", need, log_cap);
    int k = 0;
    if (nlog) *nlog = 0;
    auto record = [&](int step) -> mibh_status {
        double T = 0.0, W = 0.0;
        mibh_status s2 = mibh_energy(ctx, d_vel, &T, &W);
        if (s2) return s2;
        h_log[3 * k] = (double)step * (double)dt;
        h_log[3 * k + 1] = T;
        h_log[3 * k + 2] = W;
        k++;
        if (nlog) *nlog = k;
        return MIBH_OK;
    };
    const float half = 0.5f * dt;
    if ((st = mibh_forces(ctx, d_pos, d_mass, n, theta, d_acc, d_pot))) return st;
    HIP_TRY(clear_sticky(ctx), "sticky flags");
    if (log_every > 0 && (st = record(0))) return st;
    for (int s = 1; s <= nsteps; s++) {
        HIP_TRY(launch_kick_drift(d_pos, d_vel, d_acc, (unsigned)n, half, dt, ctx->stream), "kick_drift");
        if ((st = mibh_forces(ctx, d_pos, d_mass, n, theta, d_acc, d_pot))) return st;
        HIP_TRY(launch_kick_drift(d_pos, d_vel, d_acc, (unsigned)n, half, 0.0f, ctx->stream), "kick");
        if (log_every > 0 && s % log_every == 0 && (st = record(s))) return st;
    }
    // a walk skips its work after a flagged build, so a flag of any step voids the run
    return driver_flags(ctx);
}

mibh_status mibh_block_run(mibh_ctx *ctx, float *d_pos, float *d_vel, const float *d_mass, int64_t n,
                           float theta, const mibh_block_params *bp, int nbig, float *d_acc, float *d_pot,
                           uint8_t *d_level, mibh_block_stats *stats, double *h_log, int log_cap, int *nlog) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!bp || !d_pos || !d_vel || !d_mass || !d_acc || !d_pot) return fail(MIBH_EINVAL, "null pointer");
    const int R = bp->max_level;
    if (R < 0 || R > 20) return fail(MIBH_EINVAL, "max_level %d outside [0, 20]", R);
    if (!(bp->dt_max > 0.0f) || !isfinite(bp->dt_max)) return fail(MIBH_EINVAL, "dt_max must be finite and > 0");
    if (!(bp->eta > 0.0f) || !(bp->eps > 0.0f) || !isfinite(bp->eta) || !isfinite(bp->eps))
        return fail(MIBH_EINVAL, "eta and eps must be finite and > 0");
    if (!isfinite(bp->rebuild_tol)) return fail(MIBH_EINVAL, "rebuild_tol must be finite");
    if (nbig < 0) return fail(MIBH_EINVAL, "nbig must be >= 0");
    if (h_log && log_cap < nbig + 1) return fail(MIBH_EINVAL, "energy log needs %d rows", nbig + 1);
    if (n < 1 || n > ctx->n_max)
        return fail(MIBH_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)ctx->n_max);
    const unsigned un = (unsigned)n, nsub = 1u << R;
    const float dt_min = ldexpf(bp->dt_max, -R);
    const double eta = bp->eta, eps = bp->eps;
    hipStream_t s = ctx->stream;
    mibh_block_stats stt = {0, 0, 0, 0};
    int k = 0;
    if (nlog) *nlog = 0;
    unsigned long long *h_cnt = reinterpret_cast<unsigned long long *>(ctx->h_energy);
    auto record = [&](int big) -> mibh_status {
        double T = 0.0, W = 0.0;
        mibh_status s2 = mibh_energy(ctx, d_vel, &T, &W);
        if (s2) return s2;
        h_log[3 * k] = (double)big * (double)bp->dt_max;
        h_log[3 * k + 1] = T;
        h_log[3 * k + 2] = W;
        k++;
        if (nlog) *nlog = k;
        return MIBH_OK;
    };
    auto reset_refs = [&]() -> hipError_t { return launch_fill_u32(ctx->b.gref, un, 0u, s); };

    // forces at the start, every particle due: the walk also gives every group its reference work
    auto walk_and_check = [&]() -> mibh_status {
        mibh_status s2 = forces_impl(ctx, theta, ctx->b.active, d_acc, d_pot);
        if (s2) return s2;
        HIP_TRY(launch_rebuild_check(ctx->b, ctx->b.ohist + ORDER_BLOCKS, ctx->b.bsum, s), "rebuild check");
        return MIBH_OK;
    };
    if ((st = mibh_build_tree(ctx, d_pos, d_mass, n))) return st;
    HIP_TRY(clear_sticky(ctx), "sticky flags");
    if ((st = mibh_compute_multipoles(ctx))) return st;
    HIP_TRY(reset_refs(), "gref");
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->b.active), (un + 3u) / 4u, 0x01010101u, s), "due");
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->b.bsum), 8u, 0u, s), "counters");
    if ((st = walk_and_check())) return st;
    if (h_log && (st = record(0))) return st;
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->b.level), (un + 3u) / 4u, 0u, s), "levels");
    HIP_TRY(launch_block_kick(d_vel, d_acc, ctx->b.level, un, 0u, R, bp->dt_max,
                              nbig > 0 ? BLOCK_LEVEL | BLOCK_OPEN : BLOCK_LEVEL, eta, eps, s),
            "kick");
    bool rebuild = bp->rebuild_tol < 0.0f;  // negative: every tick rebuilds, the first one too
    for (int big = 0; big < nbig; big++) {
        for (unsigned tick = 1; tick <= nsub; tick++) {
            HIP_TRY(launch_kick_drift(d_pos, d_vel, d_acc, un, 0.0f, dt_min, s), "drift");
            HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->b.bsum), 8u, 0u, s), "counters");
            HIP_TRY(launch_block_active(ctx->b.level, un, tick, R, ctx->b.active, ctx->b.bsum + 2, s), "due");
            HIP_TRY(hipMemcpyAsync(&h_cnt[2], ctx->b.bsum + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
                    "hipMemcpyAsync(due)");
            HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
            stt.substeps++;
            if (h_cnt[2] == 0) continue;  // nobody is due: the particles only drift (a pending rebuild waits)
            stt.active_updates += (int64_t)h_cnt[2];
            if (rebuild) {
                if ((st = mibh_build_tree(ctx, d_pos, d_mass, n))) return st;
                HIP_TRY(reset_refs(), "gref");
                stt.rebuilds++;
                rebuild = false;
            } else if ((st = mibh_refit(ctx, d_pos, d_mass))) {
                return st;
            }
            if ((st = mibh_compute_multipoles(ctx))) return st;
            if ((st = walk_and_check())) return st;
            HIP_TRY(hipMemcpyAsync(h_cnt, ctx->b.bsum, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
                    "hipMemcpyAsync(counters)");
            HIP_TRY(hipMemcpyAsync(&h_cnt[3], ctx->b.ohist + ORDER_BLOCKS, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                   s),
                    "hipMemcpyAsync(groups)");
            HIP_TRY(hipMemcpyAsync(&h_cnt[4], &ctx->b.hdr->flags, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, s),
                    "hipMemcpyAsync(flags)");
            HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
            {  // the walk skipped its work after a flagged build or refit: stop here
                const unsigned *fl = reinterpret_cast<const unsigned *>(&h_cnt[4]);
                if ((st = flags_status(fl[0] | fl[1]))) {
                    if (stats) *stats = stt;
                    return st;
                }
            }
            const unsigned long long work_now = h_cnt[0], work_ref = h_cnt[1];
            stt.groups_walked += (int64_t)(uint32_t)h_cnt[3];
            rebuild = bp->rebuild_tol < 0.0f ||
                      (work_ref > 0 && (double)work_now > (1.0 + (double)bp->rebuild_tol) * (double)work_ref);
            if (tick == nsub) {  // every particle is due: synchronised velocities in between the kicks
                HIP_TRY(launch_block_kick(d_vel, d_acc, ctx->b.level, un, tick, R, bp->dt_max, BLOCK_CLOSE, eta, eps,
                                          s),
                        "kick");
                if (h_log && (st = record(big + 1))) return st;
                if (big + 1 < nbig)
                    HIP_TRY(launch_block_kick(d_vel, d_acc, ctx->b.level, un, tick, R, bp->dt_max,
                                              BLOCK_LEVEL | BLOCK_OPEN, eta, eps, s),
                            "kick");
            } else {
                HIP_TRY(launch_block_kick(d_vel, d_acc, ctx->b.level, un, tick, R, bp->dt_max,
                                          BLOCK_CLOSE | BLOCK_LEVEL | BLOCK_OPEN, eta, eps, s),
                        "kick");
            }
        }
    }
    if (d_level) HIP_TRY(hipMemcpyAsync(d_level, ctx->b.level, un, hipMemcpyDeviceToDevice, s), "levels out");
    if (stats) *stats = stt;
    return driver_flags(ctx);  // syncs
}

static mibh_status neighbors_check(mibh_ctx *ctx, const void *radius, const void *out) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (ctx->state < 2) return fail(MIBH_ESTATE, "neighbour search before compute_multipoles");
    if (!radius || !out) return fail(MIBH_EINVAL, "null pointer");
    return MIBH_OK;
}

mibh_status mibh_neighbor_count(mibh_ctx *ctx, const float *d_radius, uint32_t *d_count) {
    mibh_status st = neighbors_check(ctx, d_radius, d_count);
    if (st) return st;
    HIP_TRY(launch_neighbors(ctx->b, 0, d_radius, d_count, nullptr, nullptr, nullptr, (unsigned)ctx->nsys,
                             ctx->stream),
            "neighbors");
    return MIBH_OK;
}

mibh_status mibh_neighbor_list(mibh_ctx *ctx, const float *d_radius, uint32_t *d_count, uint32_t *d_offset,
                               uint32_t *d_index, int64_t capacity, int64_t *total) {
    mibh_status st = neighbors_check(ctx, d_radius, d_count);
    if (st) return st;
    if (!d_offset || !total || (capacity > 0 && !d_index)) return fail(MIBH_EINVAL, "null pointer");
    if ((int64_t)ctx->n > (int64_t)SCAN_MAX_TILES * 1024)
        return fail(MIBH_EINVAL, "too many particles for the offset scan");
    HIP_TRY(launch_neighbors(ctx->b, 0, d_radius, d_count, nullptr, nullptr, nullptr, (unsigned)ctx->nsys,
                             ctx->stream),
            "neighbors");
    HIP_TRY(launch_scan_u32(d_count, (unsigned)ctx->n, d_offset, ctx->b.ohist, ctx->stream), "scan");
    uint32_t *h_tot = reinterpret_cast<uint32_t *>(ctx->h_energy);
    HIP_TRY(hipMemcpyAsync(h_tot, d_offset + ctx->n, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream),
            "hipMemcpyAsync(total)");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    *total = (int64_t)*h_tot;
    if (*total > capacity)
        return fail(MIBH_EOVERFLOW, "%lld neighbours, capacity %lld", (long long)*total, (long long)capacity);
    HIP_TRY(launch_neighbors(ctx->b, 1, d_radius, d_count, d_offset, d_index, nullptr, (unsigned)ctx->nsys,
                             ctx->stream),
            "neighbors");
    return MIBH_OK;
}

mibh_status mibh_sph_density(mibh_ctx *ctx, const float *d_h, float *d_rho, uint32_t *d_count) {
    mibh_status st = neighbors_check(ctx, d_h, d_rho);
    if (st) return st;
    if (!d_count) return fail(MIBH_EINVAL, "null count pointer");
    HIP_TRY(launch_neighbors(ctx->b, 2, d_h, d_count, nullptr, nullptr, d_rho, (unsigned)ctx->nsys, ctx->stream),
            "density");
    return MIBH_OK;
}

mibh_status mibh_sync(mibh_ctx *ctx) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (ctx->state < 1) {
        HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        return MIBH_OK;
    }
    Header h;
    if ((st = read_header(ctx, &h))) return st;
    return flags_status(h.flags);
}

mibh_status mibh_stats(mibh_ctx *ctx, mibh_stats_t *out) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!out) return fail(MIBH_EINVAL, "null output pointer");
    if (ctx->state < 1) return fail(MIBH_ESTATE, "stats before build_tree");
    Header h;
    if ((st = read_header(ctx, &h))) return st;
    memset(out, 0, sizeof(*out));
    out->n = ctx->n;
    out->ncells = h.ncells;
    out->ngroups = h.ngroups;
    SysCube c0;
    HIP_TRY(hipMemcpy(&c0, ctx->b.cube, sizeof(SysCube), hipMemcpyDeviceToHost), "hipMemcpy(cube)");
    out->root_k = c0.k;
    out->nsys = ctx->nsys;
    out->flags = h.flags;
    if (ctx->p.anchor_up > 0) {
        out->anchors = h.anchor_count;
        out->anchor_fallbacks = h.anchor_fail;
    }
    int depth = 0;
    for (int l = 0; l <= KEY_LEVELS; l++)
        if (h.lvl_begin[l + 1] > h.lvl_begin[l]) depth = l;
    out->depth = depth;
    // leaves and interaction counts from the exported arrays (host side, exact integers)
    const size_t ncell = h.ncells <= ctx->b.cap_cells ? h.ncells : ctx->b.cap_cells;
    uint4 *topo = (uint4 *)malloc(ncell * sizeof(uint4) + 1);
    uint2 *grp = (uint2 *)malloc((size_t)h.ngroups * sizeof(uint2) + 1);
    uint2 *cnt = (uint2 *)malloc((size_t)h.ngroups * sizeof(uint2) + 1);
    if (!topo || !grp || !cnt) {
        free(topo); free(grp); free(cnt);
        return fail(MIBH_ENOMEM, "host allocation failed");
    }
    hipError_t e = hipMemcpy(topo, ctx->b.topo, ncell * sizeof(uint4), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(grp, ctx->b.groups, (size_t)h.ngroups * sizeof(uint2), hipMemcpyDeviceToHost);
    if (e == hipSuccess && ctx->state >= 3)
        e = hipMemcpy(cnt, ctx->b.gcounts, (size_t)h.ngroups * sizeof(uint2), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        free(topo); free(grp); free(cnt);
        return hip_fail(e, "hipMemcpy(stats)");
    }
    for (size_t c = 0; c < ncell; c++) out->nleaves += (topo[c].w & 255u) == 0;
    if (ctx->state >= 3)
        for (size_t g = 0; g < h.ngroups; g++) {
            const uint64_t gn = grp[g].y & 255u;
            out->sum_pc += gn * cnt[g].x;
            out->sum_pp += gn * cnt[g].y;
        }
    free(topo); free(grp); free(cnt);
    return flags_status(h.flags);
}

mibh_status mibh_energy(mibh_ctx *ctx, const float *d_vel, double *T, double *W) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (ctx->state < 3) return fail(MIBH_ESTATE, "energy before compute_forces");
    if (!T || !W) return fail(MIBH_EINVAL, "null output pointer");
    HIP_TRY(launch_energy(ctx->b, ctx->mass, ctx->pot, d_vel, (unsigned)ctx->n, ctx->d_energy, ctx->stream),
            "energy");
    HIP_TRY(hipMemcpyAsync(ctx->h_energy, ctx->d_energy, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
            "hipMemcpyAsync(energy)");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    *T = ctx->h_energy[0];
    *W = ctx->h_energy[1];
    Header h;
    if ((st = read_header(ctx, &h))) return st;
    return flags_status(h.flags);
}

mibh_status mibh_export_bytes(mibh_ctx *ctx, int what, size_t *bytes) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!bytes) return fail(MIBH_EINVAL, "null output pointer");
    if (ctx->state < 1) return fail(MIBH_ESTATE, "export before build_tree");
    Header h;
    if ((st = read_header(ctx, &h))) return st;
    const size_t n = (size_t)ctx->n;
    const size_t nc = h.ncells <= ctx->b.cap_cells ? h.ncells : ctx->b.cap_cells, ng = h.ngroups;
    switch (what) {
        case MIBH_EXPORT_KEYS: *bytes = 8 * n; break;
        case MIBH_EXPORT_PERM: *bytes = 4 * n; break;
        case MIBH_EXPORT_CELLS: *bytes = 16 * nc; break;
        case MIBH_EXPORT_GROUPS: *bytes = 8 * ng; break;
        case MIBH_EXPORT_COUNTS: *bytes = 8 * ng; break;
        case MIBH_EXPORT_MULTIPOLES: *bytes = 80 * nc; break;
        case MIBH_EXPORT_DELTA: *bytes = 8 * nc; break;
        case MIBH_EXPORT_MAC: *bytes = 16 * nc; break;
        case MIBH_EXPORT_QUAD: *bytes = 32 * nc; break;
        case MIBH_EXPORT_SPOS: *bytes = 16 * n; break;
        case MIBH_EXPORT_FEATURES: *bytes = 4 * (size_t)MLP_IN * ng; break;
        case MIBH_EXPORT_PREDICTIONS: *bytes = 4 * ng; break;
        case MIBH_EXPORT_QUEUE: *bytes = 4 * ng; break;
        case MIBH_EXPORT_LSIDE: *bytes = 8 * nc; break;
        default: return fail(MIBH_EINVAL, "unknown export %d", what);
    }
    return MIBH_OK;
}

mibh_status mibh_export(mibh_ctx *ctx, int what, void *d_dst, size_t bytes) {
    size_t need = 0;
    mibh_status st = mibh_export_bytes(ctx, what, &need);
    if (st) return st;
    if (!d_dst) return fail(MIBH_EINVAL, "null destination");
    if (bytes < need) return fail(MIBH_EINVAL, "destination too small: %zu < %zu", bytes, need);
    if ((what == MIBH_EXPORT_COUNTS || what == MIBH_EXPORT_MAC || what == MIBH_EXPORT_QUEUE) && ctx->state < 3)
        return fail(MIBH_ESTATE, "export of walk data before compute_forces");
    if (what == MIBH_EXPORT_QUEUE && ctx->last_order == MIBH_ORDER_MORTON)
        return fail(MIBH_ESTATE, "the last walk took the groups in Morton order");
    if ((what == MIBH_EXPORT_MULTIPOLES || what == MIBH_EXPORT_DELTA || what == MIBH_EXPORT_QUAD ||
         what == MIBH_EXPORT_LSIDE) &&
        ctx->state < 2)
        return fail(MIBH_ESTATE, "export of multipoles before compute_multipoles");
    const void *src = nullptr;
    switch (what) {
        case MIBH_EXPORT_KEYS: src = ctx->b.keys[sorted_buffer((unsigned)ctx->nsys)]; break;
        case MIBH_EXPORT_PERM: src = ctx->b.vals[sorted_buffer((unsigned)ctx->nsys)]; break;
        case MIBH_EXPORT_CELLS: src = ctx->b.topo; break;
        case MIBH_EXPORT_GROUPS: src = ctx->b.groups; break;
        case MIBH_EXPORT_COUNTS: src = ctx->b.gcounts; break;
        case MIBH_EXPORT_MULTIPOLES: src = ctx->b.mp; break;
        case MIBH_EXPORT_DELTA: src = ctx->b.delta; break;
        case MIBH_EXPORT_MAC: src = ctx->b.cmac; break;
        case MIBH_EXPORT_QUAD: src = ctx->b.ceval; break;
        case MIBH_EXPORT_SPOS: src = ctx->b.spos; break;
        case MIBH_EXPORT_FEATURES: src = ctx->b.feat; break;
        case MIBH_EXPORT_PREDICTIONS: src = ctx->b.pred; break;
        case MIBH_EXPORT_QUEUE: src = ctx->b.qorder; break;
        case MIBH_EXPORT_LSIDE: src = ctx->b.lside; break;
    }
    if (need) HIP_TRY(hipMemcpyAsync(d_dst, src, need, hipMemcpyDeviceToDevice, ctx->stream), "hipMemcpyAsync(export)");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return MIBH_OK;
}

mibh_status mibh_graph_capture(mibh_ctx *ctx, const float *d_pos, const float *d_mass, const int64_t *h_offsets,
                               int nsys, float theta, float *d_acc, float *d_pot) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!ctx->stream) return fail(MIBH_EINVAL, "graph capture needs a non-null stream");
    if (!(theta > 0.0f) || !isfinite(theta)) return fail(MIBH_EINVAL, "theta must be finite and > 0");
    if (!d_acc || !d_pot) return fail(MIBH_EINVAL, "null output pointer");
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    hipEvent_t *saved = ctx->events;  // no stage events inside a graph
    ctx->events = nullptr;
    HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    st = mibh_build_tree_batch(ctx, d_pos, d_mass, h_offsets, nsys);
    if (!st) st = mibh_compute_multipoles(ctx);
    if (!st) st = mibh_compute_forces(ctx, theta, d_acc, d_pot);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    ctx->events = saved;
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        ctx->state = 0;
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        ctx->state = 0;
        return hip_fail(e, "hipGraphInstantiate");
    }
    ctx->graph = g;
    ctx->graph_nsys = nsys;
    ctx->graph_n = h_offsets[nsys];
    ctx->graph_pos = d_pos;
    ctx->graph_mass = d_mass;
    ctx->graph_acc = d_acc;
    ctx->graph_pot = d_pot;
    ctx->state = 0;  // capture enqueued no work
    return MIBH_OK;
}

mibh_status mibh_graph_launch(mibh_ctx *ctx) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!ctx->graph_exec) return fail(MIBH_ESTATE, "no captured graph");
    HIP_TRY(hipGraphLaunch(ctx->graph_exec, ctx->stream), "hipGraphLaunch");
    ctx->nsys = ctx->graph_nsys;
    ctx->n = ctx->graph_n;
    ctx->pos = ctx->graph_pos;
    ctx->mass = ctx->graph_mass;
    ctx->acc = ctx->graph_acc;
    ctx->pot = ctx->graph_pot;
    ctx->state = 3;
    return MIBH_OK;
}

mibh_status mibh_group_features(mibh_ctx *ctx, float theta, float *d_feat) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (ctx->state < 2) return fail(MIBH_ESTATE, "features before compute_multipoles");
    if (!(theta > 0.0f) || !isfinite(theta)) return fail(MIBH_EINVAL, "theta must be finite and > 0");
    HIP_TRY(launch_features(ctx->b, theta, d_feat ? d_feat : ctx->b.feat, ctx->stream), "features");
    return MIBH_OK;
}

mibh_status mibh_set_queue_order(mibh_ctx *ctx, int mode, const void *d_w16) {
    if (!ctx) return fail(MIBH_EINVAL, "null context");
    if (mode < MIBH_ORDER_MORTON || mode > MIBH_ORDER_EXACT) return fail(MIBH_EINVAL, "unknown queue order %d", mode);
    if (mode == MIBH_ORDER_ESTIMATOR && !d_w16) return fail(MIBH_EINVAL, "estimator weights needed");
    ctx->order = mode;
    ctx->est_w16 = d_w16;
    return MIBH_OK;
}

mibh_status mibh_mlp_forward(const void *d_w16, const float *d_x, int64_t rows, float *d_y, void *stream) {
    if (!d_w16 || !d_x || !d_y) return fail(MIBH_EINVAL, "null pointer");
    if (rows < 1 || rows >= ((int64_t)1 << 31)) return fail(MIBH_EINVAL, "rows out of range");
    HIP_TRY(launch_mlp_forward(d_w16, d_x, (unsigned)rows, nullptr, d_y, (hipStream_t)stream), "mlp_forward");
    return MIBH_OK;
}

size_t mibh_mlp_scratch_bytes(int batch) { return batch < 1 ? 0 : mlp_scratch_bytes((unsigned)batch); }

mibh_status mibh_mlp_gradient(const void *d_w16, const float *d_x, const float *d_t, const int32_t *d_idx, int batch,
                              float *d_grad, float *d_loss, void *d_scratch, size_t scratch_bytes, void *stream) {
    if (!d_w16 || !d_x || !d_t || !d_idx || !d_grad || !d_scratch) return fail(MIBH_EINVAL, "null pointer");
    if (batch < 1 || batch > (1 << 24)) return fail(MIBH_EINVAL, "batch out of range");
    if (scratch_bytes < mlp_scratch_bytes((unsigned)batch)) return fail(MIBH_ENOMEM, "scratch too small");
    HIP_TRY(launch_mlp_grad(d_w16, d_x, d_t, d_idx, (unsigned)batch, d_grad, d_loss, d_scratch, (hipStream_t)stream),
            "mlp_gradient");
    return MIBH_OK;
}

mibh_status mibh_mlp_adam(float *d_w32, void *d_w16, const float *d_grad, float *d_m, float *d_v, int step, float lr,
                          float beta1, float beta2, float eps, void *stream) {
    if (!d_w32 || !d_w16 || !d_grad || !d_m || !d_v) return fail(MIBH_EINVAL, "null pointer");
    if (step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(MIBH_EINVAL, "invalid Adam hyper-parameters");
    HIP_TRY(launch_adam(d_w32, d_w16, d_grad, d_m, d_v, step, lr, beta1, beta2, eps, (hipStream_t)stream), "adam");
    return MIBH_OK;
}

mibh_status mibh_set_stream(mibh_ctx *ctx, void *stream) {
    if (!ctx) return fail(MIBH_EINVAL, "null context");
    ctx->stream = (hipStream_t)stream;
    return MIBH_OK;
}

mibh_status mibh_profile_begin(mibh_ctx *ctx, int max_steps) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (max_steps < 1 || max_steps > 100000) return fail(MIBH_EINVAL, "max_steps out of range");
    free_events(ctx);
    const int ne = max_steps * (MIBH_NSTAGES + 1);
    ctx->events = (hipEvent_t *)calloc(ne, sizeof(hipEvent_t));
    if (!ctx->events) return fail(MIBH_ENOMEM, "host allocation failed");
    ctx->prof_max = max_steps;
    ctx->prof_step = 0;
    ctx->prof_last = -2;
    for (int i = 0; i < ne; i++) {
        hipError_t e = hipEventCreate(&ctx->events[i]);
        if (e != hipSuccess) {
            free_events(ctx);
            return hip_fail(e, "hipEventCreate");
        }
    }
    return MIBH_OK;
}

mibh_status mibh_profile_read(mibh_ctx *ctx, float *ms, int max_steps, int *nsteps) {
    mibh_status st = check_ctx(ctx);
    if (st) return st;
    if (!ms || !nsteps) return fail(MIBH_EINVAL, "null output pointer");
    if (!ctx->events) return fail(MIBH_EINVAL, "profiling was not started");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    const int ns = ctx->prof_step < max_steps ? ctx->prof_step : max_steps;
    for (int k = 0; k < ns; k++)
        for (int s = 0; s < MIBH_NSTAGES; s++) {
            float t = 0.0f;
            hipEvent_t *e = ctx->events + k * (MIBH_NSTAGES + 1);
            HIP_TRY(hipEventElapsedTime(&t, e[s], e[s + 1]), "hipEventElapsedTime");
            ms[k * MIBH_NSTAGES + s] = t;
        }
    *nsteps = ns;
    free_events(ctx);
    return MIBH_OK;
}

}  // extern "C"

namespace mibh {
// float32 fused multiply-add throughput probe (probe_kernel.hip): out[64 * blocks * 32]
hipError_t launch_fma_probe(float *out, unsigned blocks, unsigned iters, float a, float b, hipStream_t s);
}  // namespace mibh

extern "C" {

mibh_status mibh_fma_probe(float *d_out, int32_t blocks, int32_t iters, float a, float b, void *stream) {
    if (!d_out) return fail(MIBH_EINVAL, "null pointer");
    if (blocks < 1 || blocks > (1 << 20) || iters < 0) return fail(MIBH_EINVAL, "blocks or iters out of range");
    HIP_TRY(launch_fma_probe(d_out, (unsigned)blocks, (unsigned)iters, a, b, (hipStream_t)stream), "fma_probe");
    return MIBH_OK;
}

}  // extern "C"

// --------------------------------------------------------------------------
// The force step without allocation (mibh_forces_static).  Its workspace is
// the file-scope device array `scratch`; every GPU the library runs on holds
// its own copy from module load until the process ends.  Host code never
// passes the array's name to a kernel or copy: at the first call on a device
// (that device current) hipGetSymbolAddress gives that device's address,
// which is kept per device and carved like a caller's workspace.
// --------------------------------------------------------------------------
namespace {

constexpr int64_t STATIC_N_MAX = 32768;       // particles per call at most
constexpr int STATIC_WALK_WAVES = 512;        // persistent walk waves (spill stacks are per wave)
constexpr size_t STATIC_BYTES = 40ull << 20;  // >= the layout of (STATIC_N_MAX, STATIC_WALK_WAVES)
constexpr int STATIC_DEVICES = 64;

struct StaticSlot {
    std::mutex mu;
    bool ready;
    mibh_ctx ctx;
};
StaticSlot g_static[STATIC_DEVICES];

}  // namespace

static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

extern "C" {

size_t mibh_static_bytes(void) { return STATIC_BYTES; }

int64_t mibh_static_n_max(void) { return STATIC_N_MAX; }

mibh_status mibh_forces_static(const float *d_pos, const float *d_mass, int64_t n, float theta, float *d_acc,
                               float *d_pot, void *stream) {
    if (!d_pos || !d_mass || !d_acc || !d_pot) return fail(MIBH_EINVAL, "null pointer");
    if (n < 1 || n > STATIC_N_MAX)
        return fail(MIBH_EINVAL, "n = %lld outside [1, %lld], the limit of the static workspace", (long long)n,
                    (long long)STATIC_N_MAX);
    if (!(theta > 0.0f) || !isfinite(theta)) return fail(MIBH_EINVAL, "theta must be finite and > 0");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= STATIC_DEVICES) return fail(MIBH_EINVAL, "device %d beyond the static slots", dev);
    StaticSlot &slot = g_static[dev];
    std::lock_guard<std::mutex> lock(slot.mu);
    mibh_ctx *c = &slot.ctx;
    if (!slot.ready) {
        mibh_default_params(&c->p);
        c->p.walk_waves = STATIC_WALK_WAVES;
        c->p.anchor_up = 0;  // the walk from the root: no anchor buffers in the static workspace
        const size_t need = layout(STATIC_N_MAX, c->p, nullptr, nullptr);
        if (need > STATIC_BYTES)
            return fail(MIBH_ENOMEM, "static workspace too small: %zu < %zu bytes", STATIC_BYTES, need);
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr || ((uintptr_t)ptr % ALIGN) != 0) return fail(MIBH_EHIP, "static workspace address not aligned");
        c->n_max = STATIC_N_MAX;
        c->device = dev;
        c->nsys = 1;
        c->order = c->last_order = MIBH_ORDER_MORTON;
        c->est_w16 = nullptr;
        c->counts_valid = 0;
        c->graph = nullptr;
        c->graph_exec = nullptr;
        c->h_energy = nullptr;  // this entry point never synchronises
        c->events = nullptr;
        c->prof_max = c->prof_step = 0;
        c->prof_last = -2;
        layout(STATIC_N_MAX, c->p, (char *)ptr, &c->b);
        c->d_energy = c->b.epart + 2 * ENERGY_BLOCKS;
        // flags start clear: a kernel fill, also on a stream being captured
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(c->b.hdr), (unsigned)(sizeof(Header) / 4), 0u,
                                (hipStream_t)stream),
                "header fill");
        slot.ready = true;
    }
    c->stream = (hipStream_t)stream;
    c->state = 0;
    return mibh_forces(c, d_pos, d_mass, n, theta, d_acc, d_pot);
}

const char *mibh_status_string(mibh_status s) {
    switch (s) {
        case MIBH_OK: return "MIBH_OK";
        case MIBH_EINVAL: return "MIBH_EINVAL";
        case MIBH_ENOMEM: return "MIBH_ENOMEM";
        case MIBH_EHIP: return "MIBH_EHIP";
        case MIBH_ESTATE: return "MIBH_ESTATE";
        case MIBH_EOVERFLOW: return "MIBH_EOVERFLOW";
        case MIBH_ENONFINITE: return "MIBH_ENONFINITE";
    }
    return "MIBH_UNKNOWN";
}

const char *mibh_last_error(void) { return g_err; }

}  // extern "C"
