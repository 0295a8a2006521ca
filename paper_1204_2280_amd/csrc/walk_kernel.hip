// Group tree walk ("tree-traverse", the >90% part of a step in the paper's
// Results section) on gfx950.
//
// One wave64 per group (the vector-machine idea of Barnes 1990: one
// interaction list shared by a group of nearby particles), persistent waves
// pulling groups from eight queues, one per XCD, each an atomic head on a
// cache line of its own over one eighth of the processing order: the groups
// in Morton order (the waves of an XCD then walk spatial neighbours, whose
// cells they share in that XCD's L2) or a work-ordered permutation, heaviest
// groups first.  A wave whose queue is empty takes groups from the others.
//
// Traversal: lanes hold up to 64 candidate cells popped from a per-wave stack
// kept in LDS (circular, spilling its bottom to a per-wave global stack when
// full); each lane applies the opening test of Barnes (1994) for the group's
// bounding box (float32, fixed operation order); ballots + mbcnt compact
// accepted cells into the particle-cell list, opened leaves into the
// particle-particle list (expanded to particle indices) and opened internal
// cells' children onto the stack.  Lanes pop in stack order and push in lane
// order, so stack levels never decrease towards the top; then at most one
// step's pushes (<= 64*8) per level are on the stack at any time, which bounds
// it by 1 + 20*512 entries.  Both lists live in LDS and are evaluated in whole
// 64-entry tiles when they fill (the remainder stays), the last partial tile at
// the end of the group.
//
// Evaluation: groups average ~20 particles, so lanes run over the list
// entries (64 sources per tile) and a wave-uniform loop runs over the group's
// particles, 16 at a time; each lane keeps 16 x 4 partial sums, folded across
// lanes by a 63-shuffle transposed reduction (lane l receives the total of
// accumulator bitrev6(l)) when a full list is flushed, and once for both lists
// at the end of the group.  An active walk (block time
// steps) evaluates only the group's active particles, packed into the first
// lanes; its lists are still built from the whole group's box.  No
// floating-point atomics: results are bitwise reproducible run to run.
#include "mibh_device.h"

namespace mibh {

namespace {

__device__ __forceinline__ unsigned lane64() { return __lane_id(); }

__device__ __forceinline__ unsigned rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ unsigned uniform(unsigned v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ unsigned bitrev6(unsigned l) {
    return ((l & 1u) << 5) | ((l & 2u) << 3) | ((l & 4u) << 1) | ((l & 8u) >> 1) | ((l & 16u) >> 3) |
           ((l & 32u) >> 5);
}

// Exclusive prefix sum over the wave of small per-lane values (0 <= v < 2^BITS),
// from BITS ballots; *total gets the wave total.
template <int BITS = 4>
__device__ __forceinline__ unsigned small_excl_scan(unsigned v, unsigned *total) {
    unsigned r = 0, t = 0;
#pragma unroll
    for (int b = 0; b < BITS; b++) {
        const unsigned long long m = __ballot((v >> b) & 1u);
        r += rank_below(m) << b;
        t += (unsigned)__popcll(m) << b;
    }
    *total = t;
    return r;
}

// Inclusive prefix sum over the wave, in lane order, of unsigned per-lane
// values whose sums do not overflow: Hillis-Steele steps inside each row of 16
// lanes (DPP row shifts 1, 2, 4, 8; a lane with no source lane adds 0), then the
// row totals carried across rows by the GFX9 row broadcasts (lane 15 into rows 1
// and 3, lane 31 into rows 2 and 3).  Six DPP steps (a move and an add each,
// where the compiler does not fuse them) against two ballots and a shift-add
// per bit for a ballot scan; the whole wave must be active.
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v) {
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Sums each of the NV per-lane values v[0..NV) (NV = 64 or 32) over the wave.
// With NV = 64 lane l gets the total of v[bitrev6(l)]; with NV = 32 lanes l and
// l ^ 1 both get the total of v[bitrev6(l) & 31].  Stage with offset o pairs
// v[2p], v[2p+1]: lanes whose bit o is clear keep the pair sum of v[2p], the
// others of v[2p+1].  The offsets 32 and 16 are the gfx950 half/row swaps
// (v_permlane32_swap exchanges the upper half of its first operand with the
// lower half of its second, so one swap and one add finish a pair); the others
// use shuffles, and for NV = 32 a last shuffle adds the two lanes of a pair.
template <int NV>
__device__ __forceinline__ float transpose_reduce(float (&v)[NV]) {
    static_assert(NV == 64 || NV == 32, "64 or 32 values");
    const unsigned ln = lane64();
#pragma unroll
    for (int p = 0; p < NV / 2; p++) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * p]), __float_as_uint(v[2 * p + 1]),
                                                        false, false);
        v[p] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int p = 0; p < NV / 4; p++) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[2 * p]), __float_as_uint(v[2 * p + 1]),
                                                        false, false);
        v[p] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int s = 2; (NV >> s) >= 2; s++) {
        const int o = 32 >> s;
        const int len = NV >> s;
        const bool hi = (ln & (unsigned)o) != 0;
#pragma unroll
        for (int p = 0; p < len / 2; p++) {
            const float keep = hi ? v[2 * p + 1] : v[2 * p];
            const float send = hi ? v[2 * p] : v[2 * p + 1];
            v[p] = keep + __shfl_xor(send, o, 64);
        }
    }
    return NV == 64 ? v[0] : v[0] + __shfl_xor(v[0], 1, 64);
}

// The opening test, float32 with every operation rounded (no contraction):
// d_a = max(max(bmin_a - c_a, c_a - bmax_a), 0), d2 = (dx dx + dy dy) + dz dz,
// accept iff d2 > r_open^2.  The inputs are finite (the walk refuses others),
// so fmaxf (one v_max_f32) gives the maxima; where it may pick -0 instead of
// +0 the square is +0 all the same.
__device__ __forceinline__ bool mac_accept(float3 bmin, float3 bmax, float4 m) {
#pragma clang fp contract(off)
    const float dx = fmaxf(fmaxf(bmin.x - m.x, m.x - bmax.x), 0.0f);
    const float dy = fmaxf(fmaxf(bmin.y - m.y, m.y - bmax.y), 0.0f);
    const float dz = fmaxf(fmaxf(bmin.z - m.z, m.z - bmax.z), 0.0f);
    const float d2 = (dx * dx + dy * dy) + dz * dz;
    return d2 > m.w;
}

// The opening test's distance taken to the box's farthest point instead of its
// nearest: d_a = max(max(bmax_a - c_a, c_a - bmin_a), 0), same operation order.
// For any box B' inside [bmin, bmax] each rounded step of the nearest-point
// distance of B' is at most the same step here, so d2(B') <= far_d2: a cell with
// far_d2 <= r_open^2 is opened for every group inside the box.
__device__ __forceinline__ float far_d2(float3 bmin, float3 bmax, float4 m) {
#pragma clang fp contract(off)
    const float dx = fmaxf(fmaxf(bmax.x - m.x, m.x - bmin.x), 0.0f);
    const float dy = fmaxf(fmaxf(bmax.y - m.y, m.y - bmin.y), 0.0f);
    const float dz = fmaxf(fmaxf(bmax.z - m.z, m.z - bmin.z), 0.0f);
    return (dx * dx + dy * dy) + dz * dz;
}

template <bool KAHAN>
__device__ __forceinline__ void add(float &s, float &c, float x) {
    if (KAHAN) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    } else {
        s += x;
    }
}

struct WalkArgs {
    Header *hdr;
    const uint4 *topo;
    const float4 *cmac;
    const float4 *ceval;
    const float4 *spos;
    const uint32_t *perm;
    const uint2 *groups;
    uint2 *gcounts;
    uint32_t *wstack;
    const uint32_t *order;   // queue order (NULL: Morton order)
    const uint32_t *qlen;    // number of queue entries to walk (NULL: all groups)
    const uint8_t *active;   // per input particle, nonzero = evaluate it (NULL: every particle)
    unsigned *head;          // heads of the group queues (one per XCD)
    float *acc, *pot;
    float eps2, G;
    unsigned pc_cap, pp_cap;
    unsigned dcell, dpart;   // padding cell and particle (massless, far)
    // shared-prefix walk
    const float *cbox;       // cells' particle boxes
    const uint32_t *anchor;  // anchor cell of each group
    const uint4 *arec;       // per anchor cell: pool offset, |F|, |S|, valid
    const uint32_t *pool;    // the anchors' lists
};

// Accumulation modes (the library's precision parameter):
//   0 plain float32;
//   1 compensated across flushes: within one evaluation of the lists each lane
//     sums its <= 16 tiles in plain float32 and the lanes are folded by a
//     six-level tree, and the per-particle totals of successive evaluations
//     (one per flush of a full list, one at the end of the group) are added
//     with Kahan compensation: the long sums of a particle are the ones across
//     evaluations, while those inside one are short and pairwise;
//   2 compensated per term: every term is added to its lane's sum with Kahan
//     compensation, and the evaluations' totals as in mode 1.
// Group particles per evaluation pass: 16 (64 sums per lane), or 8 per term
// compensated (32 sums and 32 compensations), so that every mode keeps 64
// accumulator registers per lane.
template <int PREC> constexpr int chunk_of() { return PREC == 2 ? 8 : 16; }
// Slot of a lane's reduced value for chunk c in the per-group result array
// (256 floats: 4 chunks x 64 values, or 8 chunks x 32 values).
template <int PREC> __device__ __forceinline__ unsigned res_slot(unsigned c, unsigned ln) {
    return chunk_of<PREC>() == 8 ? c * 32u + (ln >> 1) : c * 64u + ln;
}
// Evaluates the particle-cell entries `fl` (`nfl`, an anchor's shared cells in
// the pool, or none) and `pcl` (`npcl`, in LDS) and the particle-particle
// entries `ppl` (`nppl`), all whole 64-entry tiles (a list's last tile is padded
// with the massless far cell or particle), for all `gn` group particles and
// adds the results into s_res (one value per lane per chunk): one reduction per
// chunk covers all the lists.  Whole tiles need no per-lane test or substitute
// in the tile loops.
template <int PREC>
__device__ void evaluate(const WalkArgs &a, const uint32_t *fl, unsigned nfl, const uint32_t *pcl, unsigned npcl,
                         const uint32_t *ppl, unsigned nppl, unsigned gn, float px, float py, float pz, float *s_res,
                         float *s_cmp) {
    constexpr int CHUNK = chunk_of<PREC>();
    constexpr int NV = 4 * CHUNK;
    constexpr bool TERM = PREC == 2;
    const unsigned ln = lane64();
    const float eps2 = a.eps2;
    for (unsigned c0 = 0; c0 < gn; c0 += CHUNK) {
        const unsigned cn = min((unsigned)CHUNK, gn - c0);
        float xi[CHUNK], yi[CHUNK], zi[CHUNK];
#pragma unroll
        for (int ii = 0; ii < CHUNK; ii++) {
            const unsigned src = c0 + min((unsigned)ii, cn - 1);
            xi[ii] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(px), src));
            yi[ii] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(py), src));
            zi[ii] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pz), src));
        }
        float v[NV], cv[NV];
#pragma unroll
        for (int j = 0; j < NV; j++) { v[j] = 0.0f; cv[j] = 0.0f; }
        // particle-cell tiles: the shared list in the pool (fl), then the
        // group's own list in LDS (pcl), one loop over both
        const uint32_t *lst = fl;
        unsigned nl = nfl;
#pragma unroll 1
        for (int seg = 0; seg < 2; seg++, lst = pcl, nl = npcl)
        for (unsigned t0 = 0; t0 < nl; t0 += 64) {
            // The particle count of the chunk is taken as new in every tile, so
            // that its 16 comparisons are made in place (scalar compares) instead
            // of being kept as 16 lane masks across the loop: 32 scalar registers
            // more than the wave can hold, spilled to vector-register lanes and
            // read back in every tile.
            unsigned cn_t = cn;
            asm volatile("" : "+s"(cn_t));
            const unsigned e = lst[t0 + ln];
            const float4 m = a.cmac[e], q0 = a.ceval[2 * (size_t)e], q1 = a.ceval[2 * (size_t)e + 1];
#pragma unroll
            for (int ii = 0; ii < CHUNK; ii++) {
                if ((unsigned)ii < cn_t) {
                    // R = x - com; r2 = R.R + eps2
                    const float Rx = xi[ii] - m.x, Ry = yi[ii] - m.y, Rz = zi[ii] - m.z;
                    const float r2 = fmaf(Rz, Rz, fmaf(Ry, Ry, fmaf(Rx, Rx, eps2)));
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const float rinv2 = rinv * rinv;
                    const float r3 = rinv * rinv2;
                    const float r5 = r3 * rinv2;
                    // Q R with Q = (xx, yy, zz | xy, xz, yz)
                    const float QRx = fmaf(q0.y, Rx, fmaf(q1.x, Ry, q1.y * Rz));
                    const float QRy = fmaf(q1.x, Rx, fmaf(q0.z, Ry, q1.z * Rz));
                    const float QRz = fmaf(q1.y, Rx, fmaf(q1.z, Ry, q0.w * Rz));
                    const float RQR = fmaf(Rx, QRx, fmaf(Ry, QRy, Rz * QRz));
                    const float Mr3 = q0.x * r3;
                    const float u = RQR * r5;
                    // a = -M R/r^3 + Q R/r^5 - (5/2)(RQR) R/r^7 ; phi = -(M/r + RQR/(2 r^5))
                    const float coef = fmaf(2.5f * u, rinv2, Mr3);
                    if (TERM) {
                        add<true>(v[4 * ii + 0], cv[4 * ii + 0], fmaf(QRx, r5, -coef * Rx));
                        add<true>(v[4 * ii + 1], cv[4 * ii + 1], fmaf(QRy, r5, -coef * Ry));
                        add<true>(v[4 * ii + 2], cv[4 * ii + 2], fmaf(QRz, r5, -coef * Rz));
                        add<true>(v[4 * ii + 3], cv[4 * ii + 3], -fmaf(0.5f, u, q0.x * rinv));
                    } else {  // the term goes into the sum as two fused multiply-adds
                        v[4 * ii + 0] = fmaf(-coef, Rx, fmaf(QRx, r5, v[4 * ii + 0]));
                        v[4 * ii + 1] = fmaf(-coef, Ry, fmaf(QRy, r5, v[4 * ii + 1]));
                        v[4 * ii + 2] = fmaf(-coef, Rz, fmaf(QRz, r5, v[4 * ii + 2]));
                        v[4 * ii + 3] = fmaf(-q0.x, rinv, fmaf(-0.5f, u, v[4 * ii + 3]));
                    }
                }
            }
        }
        for (unsigned t0 = 0; t0 < nppl; t0 += 64) {
            unsigned cn_t = cn;  // in place in every tile, as above
            asm volatile("" : "+s"(cn_t));
            const float4 s = a.spos[ppl[t0 + ln]];
#pragma unroll
            for (int ii = 0; ii < CHUNK; ii++) {
                if ((unsigned)ii < cn_t) {
                    const float dx = s.x - xi[ii], dy = s.y - yi[ii], dz = s.z - zi[ii];
                    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    float rinv = __builtin_amdgcn_rsqf(r2 + eps2);
                    rinv = r2 > 0.0f ? rinv : 0.0f;  // self and coincident pairs contribute nothing
                    const float mr = s.w * rinv;
                    const float mr3 = mr * rinv * rinv;
                    add<TERM>(v[4 * ii + 0], cv[4 * ii + 0], mr3 * dx);
                    add<TERM>(v[4 * ii + 1], cv[4 * ii + 1], mr3 * dy);
                    add<TERM>(v[4 * ii + 2], cv[4 * ii + 2], mr3 * dz);
                    add<TERM>(v[4 * ii + 3], cv[4 * ii + 3], -mr);
                }
            }
        }
        if (TERM) {
#pragma unroll
            for (int j = 0; j < NV; j++) v[j] = v[j] - cv[j];
        }
        const float r = transpose_reduce<NV>(v);
        const unsigned slot = res_slot<PREC>(c0 / CHUNK, ln);
        if (PREC) add<true>(s_res[slot], s_cmp[slot], r);
        else s_res[slot] += r;
    }
}

// Evaluates the list's whole 64-entry tiles, moves the remaining entries to
// the front and returns their number.
template <int PREC, bool PC>
__device__ unsigned flush_list(const WalkArgs &a, uint32_t *list, unsigned n, unsigned gn, float px, float py,
                               float pz, float *s_res, float *s_cmp) {
    const unsigned ne = n & ~63u;
    __syncthreads();  // list entries written by other lanes are visible
    if (ne) {
        if (PC) evaluate<PREC>(a, nullptr, 0u, list, ne, list, 0u, gn, px, py, pz, s_res, s_cmp);
        else evaluate<PREC>(a, nullptr, 0u, list, 0u, list, ne, gn, px, py, pz, s_res, s_cmp);
    }
    const unsigned r = n - ne;
    if (r) {
        const unsigned ln = lane64();
        const unsigned v = ln < r ? list[ne + ln] : 0u;
        __syncthreads();
        if (ln < r) list[ln] = v;
        __syncthreads();
    }
    return r;
}

template <int PREC, bool SHARED>
__global__ __launch_bounds__(64, 4) void k_walk(WalkArgs a) {
    constexpr unsigned MASK = WALK_LSTACK - 1;
    static_assert((WALK_LSTACK & MASK) == 0 && WALK_LSTACK >= 512, "stack ring must hold one step's pushes");
    static_assert(PREFIX_S_CAP <= WALK_LSTACK, "an anchor's cells left fit the empty ring");
    __shared__ uint32_t s_stk[WALK_LSTACK];
    // the compensated walks' compensations take 768 more bytes of LDS: their
    // particle-cell list is shorter by as much, so 16 waves still fit a CU
    constexpr unsigned PC_LDS = PREC ? WALK_PC_LDS - 192 : WALK_PC_LDS;
    __shared__ uint32_t s_pc[PC_LDS];
    __shared__ uint32_t s_pp[WALK_PP_LDS];
    __shared__ float s_res[256];
    __shared__ float s_cmp[PREC ? 256 : 64];
    __shared__ uint32_t s_idx[64];  // group particle evaluated in each lane
    __shared__ uint32_t s_perm[64];  // caller's index of each group particle
    const unsigned ln = lane64();
    uint32_t *gstk = a.wstack + (size_t)blockIdx.x * STACK_CAP;
    if (a.hdr->flags & (FLAG_NONFINITE | FLAG_NEGMASS | FLAG_CELLCAP)) return;
    // particles a lane may add to the particle-particle list per round, so that
    // a round (<= 64 * per_round) fits after a flush leaves < 64 entries
    const unsigned per_round = max(1u, (a.pp_cap - 64u) >> 6);  // < 16 since pp_cap <= 1024
    static_assert(WALK_PP_LDS <= 1024, "per-round counts must fit the 4-bit prefix sums");
    const unsigned ngroups = a.qlen ? uniform(*a.qlen) : uniform(a.hdr->ngroups);
    const unsigned pc_cap = min(a.pc_cap, PC_LDS);
    QueueCursor qc = queue_start();
    for (;;) {
        // Every lane executes the queue atomic (only lane 0 adds 1) so that no
        // lane-dependent branch sits inside this loop: the compiler may split a
        // loop on a loop-invariant divergent condition, which would separate
        // lane 0 from the cross-lane operations of the other lanes.
        const unsigned slot = queue_next(a.head, ngroups, qc);
        if (slot >= ngroups) break;
        const unsigned g = a.order ? uniform(a.order[slot]) : slot;
        const uint2 gr = a.groups[g];
        // the anchor's record (its lists' place in the pool) is read now, so that
        // it arrives while the group's box is formed
        const uint4 rec = SHARED ? a.arec[uniform(a.anchor[g])] : make_uint4(0u, 0u, 0u, 0u);
        const unsigned gf = uniform(gr.x), gn = uniform(gr.y & 255u), glev = uniform((gr.y >> 8) & 255u);
        const unsigned root = uniform(gr.y >> 16);  // level-0 cells are the systems' roots, in system order
        const unsigned gl = min(ln, gn - 1);
        const float4 p0 = a.spos[gf + gl];
        // each lane's particle in the caller's order, kept in LDS for the results
        const unsigned pm = a.perm[gf + gl];
        float3 bmin = make_float3(p0.x, p0.y, p0.z), bmax = bmin;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            bmin.x = fminf(bmin.x, __shfl_xor(bmin.x, o, 64));
            bmin.y = fminf(bmin.y, __shfl_xor(bmin.y, o, 64));
            bmin.z = fminf(bmin.z, __shfl_xor(bmin.z, o, 64));
            bmax.x = fmaxf(bmax.x, __shfl_xor(bmax.x, o, 64));
            bmax.y = fmaxf(bmax.y, __shfl_xor(bmax.y, o, 64));
            bmax.z = fmaxf(bmax.z, __shfl_xor(bmax.z, o, 64));
        }
        // The particles evaluated: all of the group's, or only its active ones
        // (an active walk), packed into the first `ge` lanes.  The interaction
        // lists are the whole group's either way (its box above).
        const bool due = ln < gn && (!a.active || a.active[pm] != 0);
        const unsigned long long dm = __ballot(due);
        const unsigned ge = (unsigned)__popcll(dm);
        if (due) s_idx[rank_below(dm)] = ln;
        s_perm[ln] = pm;
        __syncthreads();
        const unsigned pv = s_idx[ln];
        const unsigned pj = ln < ge ? pv : 0u;
        float4 p;
        p.x = __shfl(p0.x, pj, 64);
        p.y = __shfl(p0.y, pj, 64);
        p.z = __shfl(p0.z, pj, 64);
        p.w = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            s_res[c * 64 + ln] = 0.0f;
            if (PREC) s_cmp[c * 64 + ln] = 0.0f;
        }

        // logical stack = global spill [0, gtop) followed by the LDS ring [sb, st)
        unsigned sb = 0, st = 0, gtop = 0;
        unsigned npc = 0, npp = 0, tot_pc = 0, tot_pp = 0;
        bool overflow = false;
        bool seeded = false;
        unsigned f_off = 0, f_n = 0;  // the shared accepted cells, whole tiles in the pool
        if (SHARED) {
            // the lists shared by the groups below this group's anchor cell: its
            // accepted cells are evaluated in place, from the pool, with the
            // group's own lists at its end, and the stack starts with the cells
            // left (sorted by level, shallowest at the bottom, so that stack levels
            // never decrease towards the top), in the LDS ring, which is empty here
            // and holds all of them (<= PREFIX_S_CAP)
            seeded = uniform(rec.w) == 1u;
            if (seeded) {
                const unsigned off = uniform(rec.x), nf = uniform(rec.y), ns = uniform(rec.z);
                const unsigned nfp = (nf + 63u) & ~63u;
                for (unsigned i = ln; i < ns; i += 64) s_stk[i] = a.pool[off + nfp + i];
                st = ns;
                f_off = off;
                f_n = nfp;
                tot_pc += nf;
            }
        }
        if (!seeded) {
            // The root is an ancestor of every group, so the walk always opens it:
            // its children (the root itself when it is a leaf) start the stack, in
            // the order its opening would push them.
            const uint4 tr = a.topo[root];
            const unsigned rn = uniform(tr.w & 255u);
            st = rn ? rn : 1u;
            const unsigned first = rn ? tr.z + min(ln, rn - 1) : root;
            if (ln < st) s_stk[ln] = first;
        }
        __threadfence_block();
        __syncthreads();
        while (st != sb || gtop > 0) {
            if (st == sb) {  // LDS part empty: refill from the top of the global spill
                const unsigned k = min(gtop, WALK_LSTACK / 2);
                __threadfence_block();
                for (unsigned i = ln; i < k; i += 64) s_stk[(sb - k + i) & MASK] = gstk[gtop - k + i];
                sb -= k;
                gtop -= k;
                __syncthreads();
            }
            const unsigned m = min(st - sb, 64u);
            const bool valid = ln < m;
            const unsigned c = valid ? s_stk[(st - m + ln) & MASK] : 0u;
            st -= m;
            const uint4 t = a.topo[c];
            const float4 mc = a.cmac[c];
            const unsigned lvl = (t.w >> 8) & 255u, nch = t.w & 255u;
            const bool anc = t.x <= gf && gf < t.x + t.y && lvl <= glev;
            // The opening test is taken in every lane and combined without
            // short-circuit: were it skipped for ancestors, the compiler would
            // issue the cell's MAC load only after its topology had arrived,
            // two dependent round trips per step instead of one.
            const bool far = mac_accept(bmin, bmax, mc);
            const bool accept = valid & !anc & far;
            const bool opened = valid && !accept;
            const bool leaf = opened && nch == 0;
            const bool push = opened && nch != 0;

            // accepted cells -> particle-cell list
            const unsigned long long am = __ballot(accept);
            const unsigned na = (unsigned)__popcll(am);
            if (npc + na > pc_cap)
                npc = flush_list<PREC, true>(a, s_pc, npc, ge, p.x, p.y, p.z, s_res, s_cmp);
            if (accept) s_pc[npc + rank_below(am)] = c;
            npc += na;
            tot_pc += na;

            // One prefix sum gives the list offsets of both the opened leaves'
            // particles (low half; leaves of 32 or more particles count 0 here
            // and go by rounds below) and the opened internal cells' children
            // (high half): sums stay below 64 * 32 and 64 * 8.
            unsigned rem = leaf ? t.y : 0u, src = t.x;
            const unsigned nc = push ? nch : 0u;
            const bool big = __ballot(rem > 31u) != 0;
            const unsigned packed = (big ? 0u : rem) | (nc << 16);
            const unsigned incl = wave_incl_scan(packed);
            const unsigned excl = incl - packed;
            const unsigned both = uniform(__builtin_amdgcn_readlane(incl, 63));

            // opened leaves -> particle-particle list: whole leaves in one round
            // when every leaf holds fewer than 32 particles and they fit after a
            // flush, else in rounds of at most per_round particles per lane
            if (!big && (both & 0xffffu)) {
                const unsigned sum = both & 0xffffu;
                const unsigned off = excl & 0xffffu;
                if (sum + 63u <= a.pp_cap) {
                    if (npp + sum > a.pp_cap)
                        npp = flush_list<PREC, false>(a, s_pp, npp, ge, p.x, p.y, p.z, s_res, s_cmp);
                    for (unsigned j = 0; j < rem; j++) s_pp[npp + off + j] = src + j;
                    npp += sum;
                    tot_pp += sum;
                    rem = 0;
                }
            }
            while (__ballot(rem > 0)) {
                const unsigned take = min(rem, per_round);
                unsigned sum;
                const unsigned off = small_excl_scan(take, &sum);
                if (npp + sum > a.pp_cap)
                    npp = flush_list<PREC, false>(a, s_pp, npp, ge, p.x, p.y, p.z, s_res, s_cmp);
                for (unsigned j = 0; j < take; j++) s_pp[npp + off + j] = src + j;
                npp += sum;
                tot_pp += sum;
                rem -= take;
                src += take;
            }

            // opened internal cells -> children onto the stack
            const unsigned nsum = both >> 16;
            const unsigned off = excl >> 16;
            const unsigned used = st - sb;
            if (used + nsum > WALK_LSTACK) {  // spill the bottom of the LDS ring
                const unsigned need = used + nsum - WALK_LSTACK;
                const unsigned sp = min(used, max(need, WALK_LSTACK / 2));
                if (gtop + sp > STACK_CAP) {
                    overflow = true;
                    break;
                }
                for (unsigned i = ln; i < sp; i += 64) gstk[gtop + i] = s_stk[(sb + i) & MASK];
                sb += sp;
                gtop += sp;
                __syncthreads();
            }
            for (unsigned j = 0; j < nc; j++) s_stk[(st + off + j) & MASK] = t.z + j;
            st += nsum;
            __syncthreads();
        }
        if (overflow) {
            atomicOr(&a.hdr->flags, FLAG_STACK);
            continue;
        }
        if (f_n + npc + npp) {
            // both lists' last tiles padded with the massless far cell and
            // particle (npc <= pc_cap and npp <= pp_cap, so the padded lists
            // stay within their LDS arrays, whole tiles long)
            const unsigned npc_t = (npc + 63u) & ~63u, npp_t = (npp + 63u) & ~63u;
            if (npc + ln < npc_t) s_pc[npc + ln] = a.dcell;
            if (npp + ln < npp_t) s_pp[npp + ln] = a.dpart;
            __syncthreads();  // list entries written by other lanes are visible
            evaluate<PREC>(a, f_n ? a.pool + f_off : nullptr, f_n, s_pc, npc_t, s_pp, npp_t, ge, p.x, p.y, p.z,
                           s_res, s_cmp);
        }

        // results back to the caller's order
        constexpr int CHUNK = chunk_of<PREC>();
        constexpr bool HALF = CHUNK == 8;
        // value held by this lane: bitrev6(ln) (64 per chunk) or its low five
        // bits (32 per chunk, lanes ln and ln ^ 1 alike: the even one stores)
        const unsigned idx = HALF ? (bitrev6(ln) & 31u) : bitrev6(ln);
        const unsigned comp = idx & 3u;
        for (unsigned c = 0; c * CHUNK < ge; c++) {
            const unsigned pi = c * CHUNK + (idx >> 2) + ((HALF && (ln & 1u)) ? 64u : 0u);
            if (pi < ge) {
                const unsigned slot = res_slot<PREC>(c, ln);
                float val = s_res[slot];
                if (PREC) val = val - s_cmp[slot];
                val *= a.G;
                const size_t orig = s_perm[s_idx[pi]];
                if (comp < 3) a.acc[3 * orig + comp] = val;
                else a.pot[orig] = val;
            }
        }
        a.gcounts[g] = make_uint2(tot_pc, tot_pp);  // same value from every lane
    }
}

// --------------------------------------------------------------------------
// Shared-prefix walk: the groups below one anchor cell A (the ancestor `up`
// levels above each group) share the part of their traversals that A's
// particle box decides for all of them.  From the root, with A's box:
//   * a cell that is an ancestor-or-self of A, or whose opening radius reaches
//     the farthest point of A's box, is opened by every group inside A: its
//     children are visited, and a leaf among them is left to each group (it
//     lands in the group's particle-particle list);
//   * a cell A's box accepts (the group MAC with A's box) is accepted by every
//     group inside A: the group's box lies inside A's, so its rounded distance
//     is no smaller; such a cell is never an ancestor of a group (it would
//     either contain A, and ancestors of A are opened, or lie inside A, with
//     its centre of mass inside A's box at distance 0);
//   * any other cell is left to each group.
// Each group then starts with the cells left (S) on its stack and walks on as
// usual, and evaluates the accepted cells (F, whole tiles in the pool) in place
// with its own lists at its end: the same cells are accepted and opened as in
// a walk from the root, and summed in another order.
// --------------------------------------------------------------------------

// Anchor of every group: the cell at level max(level - up, 0) that holds the
// group's first particle (cells of one level are numbered in particle order).
// The anchor's record is cleared here; k_walk_claim then lists each anchor once.
__global__ __launch_bounds__(256) void k_walk_anchor(const Header *__restrict__ hdr, const uint2 *__restrict__ groups,
                                                     const uint4 *__restrict__ topo, int up,
                                                     uint32_t *__restrict__ anchor, uint4 *__restrict__ arec) {
    if (hdr->flags & (FLAG_NONFINITE | FLAG_NEGMASS | FLAG_CELLCAP)) return;
    const unsigned ng = hdr->ngroups;
    for (unsigned g = blockIdx.x * 256u + threadIdx.x; g < ng; g += gridDim.x * 256u) {
        const uint2 gr = groups[g];
        const int glev = (int)((gr.y >> 8) & 255u);
        const int lev = glev > up ? glev - up : 0;
        unsigned lo = hdr->lvl_begin[lev], hi = hdr->lvl_begin[lev + 1];  // topo[lo].x <= gr.x
        while (hi - lo > 1) {
            const unsigned mid = lo + (hi - lo) / 2;
            if (topo[mid].x <= gr.x) lo = mid; else hi = mid;
        }
        anchor[g] = lo;
        arec[lo] = make_uint4(0u, 0u, 0u, 0u);
    }
}

// Anchor list: the anchors of the groups the walk visits (every group, or the
// queue's first *qlen entries), each once, appended by the one group that claims
// it (a compare-and-swap of the record's valid word from 0 to 2).  Only entries
// whose anchor differs from the previous entry's try: in Morton order an
// anchor's groups are contiguous unless groups of deeper levels sit between
// them, so few entries compete.
__global__ __launch_bounds__(256) void k_walk_claim(const Header *__restrict__ hdr,
                                                    const uint32_t *__restrict__ anchor, const uint32_t *order,
                                                    const uint32_t *qlen, uint4 *__restrict__ arec,
                                                    uint32_t *__restrict__ alist, unsigned *__restrict__ acount) {
    if (hdr->flags & (FLAG_NONFINITE | FLAG_NEGMASS | FLAG_CELLCAP)) return;
    const unsigned ng = hdr->ngroups;
    const unsigned nq = qlen ? min(*qlen, ng) : ng;
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < nq; i += gridDim.x * 256u) {
        const unsigned A = anchor[order ? order[i] : i];
        const bool starts = i == 0 || anchor[order ? order[i - 1] : i - 1] != A;
        if (starts && atomicCAS(&arec[A].w, 0u, 2u) == 0u) alist[atomicAdd(acount, 1u)] = A;
    }
}

// F and S of anchor cell A into this wave's scratch (F at pf, S sorted by level
// at pf + PREFIX_F_CAP + PREFIX_S_CAP).  False when a list outgrows its room or
// the stack its bound (the groups then walk from the root).  A step takes up to
// PREFIX_STEP cells per lane off the stack: the pass is bound by the dependent
// round trips of its longest traversal, not by its arithmetic.
__device__ bool anchor_lists(const WalkArgs &a, unsigned A, uint32_t *s_stk, uint32_t *gstk, uint32_t *pf,
                             unsigned *nf_out, unsigned *ns_out) {
    constexpr unsigned K = PREFIX_STEP, RING = PREFIX_RING, MASK = RING - 1;
    static_assert((RING & MASK) == 0 && RING >= 2 * 64 * 8 * K, "ring must hold one step's pushes");
    const unsigned ln = lane64();
    uint32_t *praw = pf + PREFIX_F_CAP, *pseed = praw + PREFIX_S_CAP;
    const uint4 ta = a.topo[A];
    const unsigned af = uniform(ta.x), alev = uniform((ta.w >> 8) & 255u), root = uniform(ta.w >> 16);
    const float *cb = a.cbox + 6 * (size_t)A;
    const float3 bmin = make_float3(cb[0], cb[1], cb[2]), bmax = make_float3(cb[3], cb[4], cb[5]);
    const uint4 tr = a.topo[root];
    const unsigned rn = uniform(tr.w & 255u);
    unsigned sb = 0, st = rn ? rn : 1u, gtop = 0, nf = 0, ns = 0;
    bool ok = true;
    const unsigned first = rn ? tr.z + min(ln, rn - 1) : root;
    if (ln < st) s_stk[ln] = first;
    __syncthreads();
    while (st != sb || gtop > 0) {
        if (st == sb) {  // LDS part empty: refill from the top of the global spill
            const unsigned k = min(gtop, RING / 2);
            __threadfence_block();
            for (unsigned i = ln; i < k; i += 64) s_stk[(sb - k + i) & MASK] = gstk[gtop - k + i];
            sb -= k;
            gtop -= k;
            __syncthreads();
        }
        const unsigned m = min(st - sb, 64u * K);
        unsigned c[K];
        uint4 t[K];
        float4 mc[K];
#pragma unroll
        for (unsigned k = 0; k < K; k++) {
            const unsigned i = k * 64u + ln;
            c[k] = i < m ? s_stk[(st - m + i) & MASK] : 0u;
        }
#pragma unroll
        for (unsigned k = 0; k < K; k++) {
            t[k] = a.topo[c[k]];
            mc[k] = a.cmac[c[k]];
        }
        st -= m;
        unsigned nc[K], nsum = 0;
#pragma unroll
        for (unsigned k = 0; k < K; k++) {
            const bool valid = k * 64u + ln < m;
            const unsigned lvl = (t[k].w >> 8) & 255u, nch = t[k].w & 255u;
            const bool anc = t[k].x <= af && af < t[k].x + t[k].y && lvl <= alev;
            // both tests in every lane, no short-circuit: the MAC loads then go
            // out with the topology loads (see the group walk)
            const bool reach = !(far_d2(bmin, bmax, mc[k]) > mc[k].w);
            const bool far = mac_accept(bmin, bmax, mc[k]);
            const bool open = valid & (anc | reach);
            const bool accept = valid & !open & far;
            const bool left = valid && !accept && (!open || nch == 0);
            const unsigned long long am = __ballot(accept);
            const unsigned na = (unsigned)__popcll(am);
            const unsigned long long lm = __ballot(left);
            const unsigned nl = (unsigned)__popcll(lm);
            if (nf + na > PREFIX_F_CAP || ns + nl > PREFIX_S_CAP) ok = false;
            if (ok && accept) pf[nf + rank_below(am)] = c[k];
            if (ok && left) praw[ns + rank_below(lm)] = c[k];
            nf += na;
            ns += nl;
            nc[k] = open ? nch : 0u;
            unsigned tk;
            const unsigned o = small_excl_scan(nc[k], &tk);
            nc[k] |= (nsum + o) << 8;  // this lane's first push slot above st, with its count
            nsum += tk;
        }
        if (!ok) break;
        const unsigned used = st - sb;
        if (used + nsum > RING) {  // spill the bottom of the LDS ring
            const unsigned need = used + nsum - RING;
            const unsigned sp = min(used, max(need, RING / 2));
            if (gtop + sp > STACK_CAP) {
                ok = false;
                break;
            }
            for (unsigned i = ln; i < sp; i += 64) gstk[gtop + i] = s_stk[(sb + i) & MASK];
            sb += sp;
            gtop += sp;
            __syncthreads();
        }
#pragma unroll
        for (unsigned k = 0; k < K; k++) {
            const unsigned cnt = nc[k] & 255u, off = nc[k] >> 8;
            for (unsigned j = 0; j < cnt; j++) s_stk[(st + off + j) & MASK] = t[k].z + j;
        }
        st += nsum;
        __syncthreads();
    }
    __threadfence_block();
    if (ok) {  // S by level, shallowest first: a counting pass over the levels
        unsigned cell[PREFIX_S_CAP / 64], lv[PREFIX_S_CAP / 64];
#pragma unroll
        for (unsigned k = 0; k < PREFIX_S_CAP / 64; k++) {
            const unsigned i = k * 64 + ln;
            cell[k] = i < ns ? praw[i] : 0u;
            lv[k] = i < ns ? (a.topo[cell[k]].w >> 8) & 255u : 255u;
        }
        unsigned pos = 0;
        for (unsigned l = 0; l <= (unsigned)KEY_LEVELS; l++) {
#pragma unroll
            for (unsigned k = 0; k < PREFIX_S_CAP / 64; k++) {
                const bool h = lv[k] == l;
                const unsigned long long hm = __ballot(h);
                if (h) pseed[pos + rank_below(hm)] = cell[k];
                pos += (unsigned)__popcll(hm);
            }
        }
        __threadfence_block();
    }
    *nf_out = nf;
    *ns_out = ns;
    return ok;
}

// One pass over the anchor list (persistent waves, per-XCD queues as in the
// walk; one anchor per queue slot): a wave builds its anchor's lists, stores
// them in the pool and their place in arec[anchor] (valid word 1; all zero when
// they did not fit, and the anchor's groups walk from the root).
__global__ __launch_bounds__(64) void k_walk_prefix(WalkArgs a, unsigned *__restrict__ prefix_head,
                                                    const unsigned *__restrict__ acount,
                                                    const uint32_t *__restrict__ alist,
                                                    unsigned long long *__restrict__ pool_head,
                                                    uint4 *__restrict__ arec, uint32_t *__restrict__ pool,
                                                    unsigned long long pool_cap,
                                                    uint32_t *__restrict__ pscr, unsigned *__restrict__ nfail) {
    __shared__ uint32_t s_stk[PREFIX_RING];
    const unsigned ln = lane64();
    uint32_t *gstk = a.wstack + (size_t)blockIdx.x * STACK_CAP;
    uint32_t *pf = pscr + (size_t)blockIdx.x * PREFIX_SCRATCH;
    if (a.hdr->flags & (FLAG_NONFINITE | FLAG_NEGMASS | FLAG_CELLCAP)) return;
    const unsigned nanchor = uniform(*acount);
    QueueCursor qc = queue_start();
    for (;;) {
        const unsigned slot = queue_next(prefix_head, nanchor, qc);
        if (slot >= nanchor) break;
        const unsigned A = uniform(alist[slot]);
        unsigned nf, ns;
        bool ok = anchor_lists(a, A, s_stk, gstk, pf, &nf, &ns);
        nf = uniform(nf);
        ns = uniform(ns);
        // F takes whole 64-entry tiles in the pool (padded with the massless far
        // cell): the groups evaluate it in place
        const unsigned nfp = (nf + 63u) & ~63u;
        unsigned long long off64 = 0;
        if (ok) {  // every lane calls the atomic (lane 0 adds), see queue_next
            off64 = atomicAdd(pool_head, ln == 0 ? (unsigned long long)(nfp + ns) : 0ull);
            off64 = ((unsigned long long)uniform((unsigned)(off64 >> 32)) << 32) | uniform((unsigned)off64);
            ok = off64 + nfp + ns <= pool_cap;
        }
        if (!ok) atomicAdd(nfail, ln == 0 ? 1u : 0u);  // ok is wave-uniform
        const unsigned off = (unsigned)off64;  // < 2^32 when ok
        if (ok) {
            for (unsigned i = ln; i < nfp; i += 64) pool[off + i] = i < nf ? pf[i] : a.dcell;
            const uint32_t *pseed = pf + PREFIX_F_CAP + PREFIX_S_CAP;
            for (unsigned i = ln; i < ns; i += 64) pool[off + nfp + i] = pseed[i];
        }
        // every lane stores the same record: no lane-dependent branch in this loop
        arec[A] = ok ? make_uint4(off, nf, ns, 1u) : make_uint4(0u, 0u, 0u, 0u);
    }
}

}  // namespace

hipError_t launch_walk(const Buffers &b, unsigned n, unsigned nsys, float eps2, float G, int precision,
                       const uint32_t *order, const uint32_t *qlen, const uint8_t *active, float *acc, float *pot,
                       int anchor_up, hipStream_t s) {
    (void)n;
    WalkArgs a;
    a.hdr = b.hdr;
    a.topo = b.topo;
    a.cmac = b.cmac;
    a.ceval = b.ceval;
    a.spos = b.spos;
    a.perm = b.vals[sorted_buffer(nsys)];
    a.groups = b.groups;
    a.gcounts = b.gcounts;
    a.wstack = b.wstack;
    a.order = order;
    a.qlen = qlen;
    a.active = active;
    a.head = b.hdr->walk_head;
    a.acc = acc;
    a.pot = pot;
    a.eps2 = eps2;
    a.G = G;
    a.pc_cap = b.pc_cap;
    a.pp_cap = b.pp_cap;
    a.dcell = b.cap_cells;
    a.dpart = b.n_max;
    a.cbox = b.cbox;
    a.anchor = b.anchor;
    a.arec = b.arec;
    a.pool = b.pool;
    const bool shared = anchor_up > 0 && b.anchor;
    if (shared) {
        const unsigned grid = min((b.n_max + 255u) / 256u, 2048u);
        hipLaunchKernelGGL(k_walk_anchor, dim3(grid), dim3(256), 0, s, b.hdr, b.groups, b.topo, anchor_up, b.anchor,
                           b.arec);
        hipLaunchKernelGGL(k_walk_claim, dim3(grid), dim3(256), 0, s, b.hdr, b.anchor, order, qlen, b.arec, b.alist,
                           &b.hdr->anchor_count);
        hipLaunchKernelGGL(k_walk_prefix, dim3(b.walk_waves), dim3(64), 0, s, a, b.hdr->prefix_head,
                           &b.hdr->anchor_count, b.alist, &b.hdr->pool_head, b.arec, b.pool, b.pool_cap, b.pscr,
                           &b.hdr->anchor_fail);
    }
    if (precision == 2) {
        if (shared) hipLaunchKernelGGL((k_walk<2, true>), dim3(b.walk_waves), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_walk<2, false>), dim3(b.walk_waves), dim3(64), 0, s, a);
    } else if (precision == 1) {
        if (shared) hipLaunchKernelGGL((k_walk<1, true>), dim3(b.walk_waves), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_walk<1, false>), dim3(b.walk_waves), dim3(64), 0, s, a);
    } else {
        if (shared) hipLaunchKernelGGL((k_walk<0, true>), dim3(b.walk_waves), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_walk<0, false>), dim3(b.walk_waves), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Queue order: a stable counting sort of the groups by work bucket, heaviest
// bucket first.  work = count * 2^prediction (estimator) or
// count * (1 + n_pc + n_pp) (exact counts of the last walk); bucket =
// floor(4 log2 work), clamped to ORDER_BUCKETS values.  Block b owns a
// contiguous slice of the groups; the blocks' bucket counts, scanned
// bucket-major (heaviest first) then block-minor, place every group, and ranks
// inside a block are taken tile by tile in group order, so groups of equal
// bucket keep their Morton order.  Integer counts only: the order is the same
// on every run.
// --------------------------------------------------------------------------
namespace {

constexpr int ORDER_THREADS = 256;
constexpr int ORDER_SCAN_THREADS = 1024;
constexpr unsigned ORDER_SKIP = FLAG_NONFINITE | FLAG_NEGMASS | FLAG_CELLCAP;  // the walk does nothing then

struct OrderArgs {
    const Header *hdr;
    unsigned n_max;
    const uint2 *groups;
    const float *pred;       // mode 1
    const uint2 *counts;     // mode 2
    const uint32_t *perm;    // mode 3: sorted position -> input index
    const uint8_t *active;   // mode 3: per input particle, nonzero = active
    int mode;
};

// Queue bucket of group g: 0 for the heaviest work (modes 1, 2), or 0 for a
// group holding an active particle and 1 otherwise (mode 3).
__device__ __forceinline__ unsigned work_bucket(const OrderArgs &o, unsigned g) {
    const uint2 gr = o.groups[g];
    if (o.mode == 3) {
        bool any = false;
        for (unsigned k = gr.x; k < gr.x + (gr.y & 255u); k++) any = any || o.active[o.perm[k]] != 0;
        return any ? 0u : 1u;
    }
    const float gn = (float)(gr.y & 255u);
    const float *pred = o.pred;
    const uint2 *counts = o.counts;
    const int mode = o.mode;
    float l2;
    if (mode == 1) {
        const float p = pred[g];
        l2 = log2f(gn) + (isfinite(p) ? fminf(fmaxf(p, 0.0f), 40.0f) : 0.0f);
    } else {
        const uint2 c = counts[g];
        l2 = log2f(gn * (float)(1u + c.x + c.y));
    }
    const int b = min(max((int)floorf(4.0f * l2), 0), ORDER_BUCKETS - 1);
    return (unsigned)(ORDER_BUCKETS - 1 - b);
}

__device__ __forceinline__ void order_slice(const Header *hdr, unsigned n_max, unsigned *beg, unsigned *end) {
    const unsigned ng = min(hdr->ngroups, n_max);
    const unsigned chunk = (ng + ORDER_BLOCKS - 1) / ORDER_BLOCKS;
    *beg = min(ng, blockIdx.x * chunk);
    *end = min(ng, *beg + chunk);
}

__global__ __launch_bounds__(ORDER_THREADS) void k_order_hist(OrderArgs o, uint32_t *__restrict__ ohist) {
    __shared__ unsigned s_h[ORDER_BUCKETS];
    if (o.hdr->flags & ORDER_SKIP) return;
    const unsigned t = threadIdx.x;
    if (t < ORDER_BUCKETS) s_h[t] = 0;
    __syncthreads();
    unsigned beg, end;
    order_slice(o.hdr, o.n_max, &beg, &end);
    for (unsigned g = beg + t; g < end; g += ORDER_THREADS) atomicAdd(&s_h[work_bucket(o, g)], 1u);
    __syncthreads();
    if (t < ORDER_BUCKETS) ohist[t * ORDER_BLOCKS + blockIdx.x] = s_h[t];
}

// Exclusive prefix sum, in place, of ohist[ORDER_BUCKETS][ORDER_BLOCKS] read
// as one row-major sequence.  It skips with the histogram and scatter kernels:
// run on a table the histogram did not refill, it would scan the previous
// prefix sums again, and the queue length it leaves (ohist[ORDER_BLOCKS] in the
// active mode) would exceed the number of groups.
__global__ __launch_bounds__(ORDER_SCAN_THREADS) void k_order_scan(const Header *__restrict__ hdr,
                                                                   uint32_t *__restrict__ ohist) {
    constexpr int PER = ORDER_BUCKETS * ORDER_BLOCKS / ORDER_SCAN_THREADS;
    static_assert(PER * ORDER_SCAN_THREADS == ORDER_BUCKETS * ORDER_BLOCKS, "scan covers the table");
    __shared__ unsigned s_w[ORDER_SCAN_THREADS / 64];
    if (hdr->flags & ORDER_SKIP) return;
    const unsigned t = threadIdx.x, ln = lane64(), w = t >> 6;
    unsigned v[PER], sum = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        v[i] = ohist[t * PER + i];
        sum += v[i];
    }
    unsigned x = sum;  // inclusive scan over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(x, o, 64);
        x += ln >= (unsigned)o ? y : 0u;
    }
    if (ln == 63) s_w[w] = x;
    __syncthreads();
    unsigned run = x - sum;
    for (unsigned i = 0; i < w; i++) run += s_w[i];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        ohist[t * PER + i] = run;
        run += v[i];
    }
}

__global__ __launch_bounds__(ORDER_THREADS) void k_order_scatter(OrderArgs o, const uint32_t *__restrict__ ohist,
                                                                 uint32_t *__restrict__ order) {
    constexpr int NW = ORDER_THREADS / 64;
    static_assert(NW * ORDER_BUCKETS == 2 * ORDER_THREADS, "two counters per thread to clear");
    __shared__ unsigned s_base[ORDER_BUCKETS];
    __shared__ unsigned s_wcnt[NW][ORDER_BUCKETS];
    if (o.hdr->flags & ORDER_SKIP) return;
    const unsigned t = threadIdx.x, w = t >> 6;
    if (t < ORDER_BUCKETS) s_base[t] = ohist[t * ORDER_BLOCKS + blockIdx.x];
    unsigned beg, end;
    order_slice(o.hdr, o.n_max, &beg, &end);
    // No branch below depends on the thread alone (see the walk's queue loop).
    for (unsigned t0 = beg; t0 < end; t0 += ORDER_THREADS) {
        (&s_wcnt[0][0])[t] = 0;
        (&s_wcnt[0][0])[t + ORDER_THREADS] = 0;
        __syncthreads();
        const unsigned g = t0 + t;
        const bool valid = g < end;
        const unsigned d = valid ? work_bucket(o, g) : 0u;
        // lanes of this wave with the same bucket
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 7; bit++) {
            static_assert(ORDER_BUCKETS <= 128, "7-bit buckets");
            const unsigned long long m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        const unsigned rank = rank_below(peers), cnt = (unsigned)__popcll(peers);
        const bool leader = valid && rank == 0;
        if (leader) s_wcnt[w][d] = cnt;
        __syncthreads();
        if (valid) {
            unsigned pos = s_base[d] + rank;
            for (unsigned w2 = 0; w2 < w; w2++) pos += s_wcnt[w2][d];
            order[pos] = g;
        }
        __syncthreads();
        if (leader) atomicAdd(&s_base[d], cnt);
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_queue_order(const Buffers &b, int mode, const uint8_t *active, unsigned nsys, hipStream_t s) {
    OrderArgs o;
    o.hdr = b.hdr;
    o.n_max = b.n_max;
    o.groups = b.groups;
    o.pred = b.pred;
    o.counts = b.gcounts;
    o.perm = b.vals[sorted_buffer(nsys)];
    o.active = active;
    o.mode = mode;
    hipLaunchKernelGGL(k_order_hist, dim3(ORDER_BLOCKS), dim3(ORDER_THREADS), 0, s, o, b.ohist);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(ORDER_SCAN_THREADS), 0, s, b.hdr, b.ohist);
    hipLaunchKernelGGL(k_order_scatter, dim3(ORDER_BLOCKS), dim3(ORDER_THREADS), 0, s, o, b.ohist, b.qorder);
    return hipGetLastError();
}

}  // namespace mibh
