// Neighbour search and SPH density on the tree: the paper's Discussion notes
// that its tree serves neighbour search and makes smoothed particle
// hydrodynamics straightforward.  Definitions taken (gather form):
//   * the neighbours of particle i are the j (i included) with
//     d2 <= r_i * r_i, d = x_j - x_i, d2 = (dx*dx + dy*dy) + dz*dz, every
//     operation float32 and rounded (no contraction), so that any
//     implementation decides every pair alike;
//   * rho_i = sum over the neighbours within r_i = 2 h_i of m_j W(|d|, h_i),
//     W the cubic spline of Monaghan & Lattanzio (1985).
//
// One wave64 per group, persistent waves on the walk's per-XCD group queues.  The
// traversal opens a cell when the gap between the group's bounding box and
// the cell's particle box (both float32, from the multipole pass) is within
// the group's largest radius, with a relative margin of 1e-5 on the squared
// radius: the float32 gap can differ from the exact one by a few ulps, and the
// margin makes the test a superset of the pairs the exact predicate admits.
// Opened leaves put their particles on a candidate list in LDS; tiles of 64
// candidates (one per lane) are tested against the group's particles 8 at a
// time (positions broadcast from their lanes into scalar registers: 16 at a
// time needed more scalar registers than a wave holds).  Counts go to the
// lane of their particle by a select (no lane-dependent branch inside a loop
// that holds cross-lane operations); list entries are placed by ballot ranks;
// densities are summed per lane, reduced across the wave by three transposed
// stages and three butterflies, and moved to their particle's lane.
#include "mibh_device.h"

namespace mibh {

namespace {

constexpr unsigned NGB_LSTACK = 512;   // LDS part of the cell stack (spills to the global stack)
constexpr unsigned NGB_LIST = 512;     // candidate list
constexpr int NGB_CHUNK = 8;          // group particles per pass over the list
constexpr float NGB_FAR = 1.0e18f;

__device__ __forceinline__ unsigned lane64() { return __lane_id(); }
__device__ __forceinline__ unsigned uniform(unsigned v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// exclusive prefix sum of small per-lane values (0 <= v < 16); *total = wave total
template <int BITS = 4>
__device__ __forceinline__ unsigned small_scan(unsigned v, unsigned *total) {
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

__device__ __forceinline__ float readlane_f(float v, unsigned l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Bits 0..K-1 of x in reverse order.
template <int K> __device__ __forceinline__ unsigned bitrev_k(unsigned x) {
    unsigned r = 0;
#pragma unroll
    for (int b = 0; b < K; b++) r |= ((x >> b) & 1u) << (K - 1 - b);
    return r;
}

// Sum over the wave of v[0..2^K): lane l ends with the total of
// v[bitrev_k<K>(l >> (6 - K))]; the particle of value p thus sits on the
// lanes bitrev_k<K>(p) << (6 - K) ... + 2^(6-K) - 1.
template <int K>
__device__ __forceinline__ float reduce_pow2(float (&v)[1 << K]) {
    const unsigned ln = lane64();
#pragma unroll
    for (int s = 0; s < K; s++) {
        const int o = 32 >> s;
        const int len = (1 << K) >> s;
        const bool hi = (ln & (unsigned)o) != 0;
#pragma unroll
        for (int p = 0; p < len / 2; p++) {
            const float keep = hi ? v[2 * p + 1] : v[2 * p];
            const float send = hi ? v[2 * p] : v[2 * p + 1];
            v[p] = keep + __shfl_xor(send, o, 64);
        }
    }
    float r = v[0];
#pragma unroll
    for (int o = 32 >> K; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
    return r;
}

// float32 squared distance, each operation rounded
__device__ __forceinline__ float dist2(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
    const float dx = bx - ax, dy = by - ay, dz = bz - az;
    return (dx * dx + dy * dy) + dz * dz;
}

// cubic spline W(r, h) with sig = 1/(pi h^3), ih = 1/h
__device__ __forceinline__ float spline(float r, float ih, float sig) {
    const float q = r * ih;
    const float t = 2.0f - q;
    const float inner = fmaf(0.75f * q, q * q, fmaf(-1.5f, q * q, 1.0f));
    const float outer = 0.25f * t * t * t;
    return sig * (q < 1.0f ? inner : (q < 2.0f ? outer : 0.0f));
}

struct NgbArgs {
    Header *hdr;
    unsigned *head;
    const uint4 *topo;
    const float *cbox;
    const float4 *spos;
    const uint32_t *perm;
    const uint2 *groups;
    const float *radius;     // per input particle: radius (count, list) or h (density)
    float scale;             // search radius = scale * radius (2 for density)
    uint32_t *wstack;
    uint32_t *count;         // per input particle
    const uint32_t *offset;  // list: first slot of each input particle
    uint32_t *index;         // list: neighbour input indices
    float *rho;              // density
};

enum { NGB_COUNT = 0, NGB_LISTS = 1, NGB_DENSITY = 2 };

// Tests the candidates list[0..nlist) against the group's particles.
template <int MODE>
__device__ void ngb_eval(const NgbArgs &a, const uint32_t *list, unsigned nlist, unsigned gn, float px, float py,
                         float pz, float pr2, float ph, unsigned &cnt, unsigned obase, unsigned ocap, float &rho) {
    const unsigned ln = lane64();
    for (unsigned c0 = 0; c0 < gn; c0 += NGB_CHUNK) {
        const unsigned cn = min((unsigned)NGB_CHUNK, gn - c0);
        float xi[NGB_CHUNK], yi[NGB_CHUNK], zi[NGB_CHUNK], r2i[NGB_CHUNK], ihi[NGB_CHUNK], sgi[NGB_CHUNK];
#pragma unroll
        for (int ii = 0; ii < NGB_CHUNK; ii++) {
            const unsigned src = c0 + min((unsigned)ii, cn - 1);
            xi[ii] = readlane_f(px, src);
            yi[ii] = readlane_f(py, src);
            zi[ii] = readlane_f(pz, src);
            // a padding particle (ii >= cn) admits nothing
            r2i[ii] = (unsigned)ii < cn ? readlane_f(pr2, src) : -1.0f;
            if (MODE == NGB_DENSITY) {
                const float h = readlane_f(ph, src);
                ihi[ii] = 1.0f / h;
                sgi[ii] = ihi[ii] * ihi[ii] * ihi[ii] * 0.318309886183790672f;  // 1 / (pi h^3)
            }
        }
        float acc[NGB_CHUNK];
#pragma unroll
        for (int ii = 0; ii < NGB_CHUNK; ii++) acc[ii] = 0.0f;
        for (unsigned t0 = 0; t0 < nlist; t0 += 64) {
            const unsigned k = t0 + ln;
            const bool valid = k < nlist;
            const unsigned e = valid ? list[k] : 0u;
            float4 s = a.spos[e];
            if (!valid) s = make_float4(NGB_FAR, NGB_FAR, NGB_FAR, 0.0f);
            const unsigned oj = MODE == NGB_LISTS ? a.perm[e] : 0u;
#pragma unroll
            for (int ii = 0; ii < NGB_CHUNK; ii++) {
                const float d2 = dist2(xi[ii], yi[ii], zi[ii], s.x, s.y, s.z);
                const bool in = d2 <= r2i[ii];
                const unsigned long long m = __ballot(in);
                const unsigned nin = (unsigned)__popcll(m);
                if (MODE == NGB_LISTS) {
                    const unsigned base = __builtin_amdgcn_readlane(obase + cnt, c0 + ii);
                    const unsigned cap = __builtin_amdgcn_readlane(ocap, c0 + ii);
                    const unsigned slot = base + rank_below(m);
                    if (in && slot < cap) a.index[slot] = oj;
                }
                if (MODE == NGB_DENSITY) {
                    const float r = d2 > 0.0f ? d2 * __builtin_amdgcn_rsqf(d2) : 0.0f;
                    acc[ii] += in ? s.w * spline(r, ihi[ii], sgi[ii]) : 0.0f;
                }
                cnt += ln == c0 + (unsigned)ii ? nin : 0u;
            }
        }
        if (MODE == NGB_DENSITY) {
            constexpr int K = NGB_CHUNK == 16 ? 4 : 3;
            static_assert((1 << K) == NGB_CHUNK, "chunk of 8 or 16");
            const float tot = reduce_pow2<K>(acc);
            const unsigned p = ln - c0;
            const float mine = __shfl(tot, (int)(bitrev_k<K>(p & (NGB_CHUNK - 1u)) << (6 - K)), 64);
            rho += ln >= c0 && ln < c0 + cn ? mine : 0.0f;
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(64, 4) void k_neighbors(NgbArgs a) {
    constexpr unsigned MASK = NGB_LSTACK - 1;
    __shared__ uint32_t s_stk[NGB_LSTACK];
    __shared__ uint32_t s_list[NGB_LIST];
    const unsigned ln = lane64();
    uint32_t *gstk = a.wstack + (size_t)blockIdx.x * STACK_CAP;
    if (a.hdr->flags & (FLAG_NONFINITE | FLAG_NEGMASS | FLAG_CELLCAP)) return;
    constexpr unsigned per_round = NGB_LIST >> 6;  // 8 particles per lane: a round always fits an empty list
    const unsigned ngroups = uniform(a.hdr->ngroups);
    QueueCursor qc = queue_start();
    for (;;) {
        // every lane takes part in the queue atomic (see the walk's queue loop)
        const unsigned g = queue_next(a.head, ngroups, qc);
        if (g >= ngroups) break;
        const uint2 gr = a.groups[g];
        const unsigned gf = uniform(gr.x), gn = uniform(gr.y & 255u);
        const unsigned root = uniform(gr.y >> 16);
        const unsigned mine = gf + min(ln, gn - 1);
        const float4 p = a.spos[mine];
        const unsigned oi = a.perm[mine];
        const float hr = a.radius[oi];
        const float rr = a.scale * hr;
        const float pr2 = rr * rr;
        float bmin[3] = {p.x, p.y, p.z}, bmax[3] = {p.x, p.y, p.z};
        float rmax = rr;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int d = 0; d < 3; d++) {
                bmin[d] = fminf(bmin[d], __shfl_xor(bmin[d], o, 64));
                bmax[d] = fmaxf(bmax[d], __shfl_xor(bmax[d], o, 64));
            }
            rmax = fmaxf(rmax, __shfl_xor(rmax, o, 64));
        }
        const float open2 = rmax * rmax * (1.0f + 1.0e-5f);
        unsigned cnt = 0;
        float rho = 0.0f;
        const unsigned obase = MODE == NGB_LISTS ? a.offset[oi] : 0u;
        const unsigned ocap = MODE == NGB_LISTS ? a.offset[oi] + a.count[oi] : 0u;

        // The root holds every particle, so every search opens it: its
        // children (the root itself when it is a leaf) start the stack.
        const uint4 tr = a.topo[root];
        const unsigned rn = uniform(tr.w & 255u);
        unsigned sb = 0, st = rn ? rn : 1u, gtop = 0, nl = 0;
        bool overflow = false;
        const unsigned first = rn ? tr.z + min(ln, rn - 1) : root;
        if (ln < st) s_stk[ln] = first;
        __syncthreads();
        while (st != sb || gtop > 0) {
            if (st == sb) {  // refill the LDS part of the stack from the global spill
                const unsigned k = min(gtop, NGB_LSTACK / 2);
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
            const unsigned nch = t.w & 255u;
            bool open = false;
            if (valid) {
#pragma clang fp contract(off)
                float gap2 = 0.0f;
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    const float u = a.cbox[6 * (size_t)c + d] - bmax[d];
                    const float w = bmin[d] - a.cbox[6 * (size_t)c + 3 + d];
                    const float gp = fmaxf(fmaxf(u, w), 0.0f);
                    gap2 = gap2 + gp * gp;
                }
                open = gap2 <= open2;
            }
            // opened leaves -> candidate list: whole leaves in one round when
            // each holds fewer than 32 particles and they fit an empty list,
            // else in rounds; the list is evaluated when a round does not fit
            unsigned rem = open && nch == 0 ? t.y : 0u, src = t.x;
            if (__ballot(rem > 0) && !__ballot(rem > 31u)) {
                unsigned sum;
                const unsigned off = small_scan<5>(rem, &sum);
                if (sum <= NGB_LIST) {
                    if (nl + sum > NGB_LIST) {
                        __syncthreads();
                        ngb_eval<MODE>(a, s_list, nl, gn, p.x, p.y, p.z, pr2, hr, cnt, obase, ocap, rho);
                        nl = 0;
                        __syncthreads();
                    }
                    for (unsigned j = 0; j < rem; j++) s_list[nl + off + j] = src + j;
                    nl += sum;
                    rem = 0;
                }
            }
            while (__ballot(rem > 0)) {
                const unsigned take = min(rem, per_round);
                unsigned sum;
                const unsigned off = small_scan(take, &sum);
                if (nl + sum > NGB_LIST) {
                    __syncthreads();
                    ngb_eval<MODE>(a, s_list, nl, gn, p.x, p.y, p.z, pr2, hr, cnt, obase, ocap, rho);
                    nl = 0;
                    __syncthreads();
                }
                for (unsigned j = 0; j < take; j++) s_list[nl + off + j] = src + j;
                nl += sum;
                rem -= take;
                src += take;
            }
            // opened internal cells -> children onto the stack
            unsigned nsum;
            const unsigned nc = open && nch != 0 ? nch : 0u;
            const unsigned off = small_scan(nc, &nsum);
            const unsigned used = st - sb;
            if (used + nsum > NGB_LSTACK) {  // spill the bottom of the LDS ring
                const unsigned need = used + nsum - NGB_LSTACK;
                const unsigned sp = min(used, max(need, NGB_LSTACK / 2));
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
        if (!overflow && nl > 0) {
            __syncthreads();
            ngb_eval<MODE>(a, s_list, nl, gn, p.x, p.y, p.z, pr2, hr, cnt, obase, ocap, rho);
        }
        if (overflow) {
            atomicOr(&a.hdr->flags, FLAG_STACK);
            continue;
        }
        if (ln < gn) {
            if (MODE != NGB_LISTS) a.count[oi] = cnt;
            if (MODE == NGB_DENSITY) a.rho[oi] = rho;
        }
    }
}

// Exclusive scan of n counts into off[0..n] (off[n] = total) in tiles of 1024:
// tile sums, one block scanning the tile sums, tiles scanned with their offset.
constexpr unsigned SCAN_TILE = 1024;

__global__ __launch_bounds__(256) void k_scan_tiles(const uint32_t *__restrict__ in, unsigned n,
                                                    uint32_t *__restrict__ tsum) {
    __shared__ unsigned s[4];
    const unsigned b = blockIdx.x * SCAN_TILE;
    unsigned v = 0;
    for (unsigned i = threadIdx.x; i < SCAN_TILE; i += 256) v += b + i < n ? in[b + i] : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63u) == 0u) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) tsum[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *__restrict__ tsum, unsigned ntiles) {
    __shared__ unsigned s_w[16];
    const unsigned t = threadIdx.x, ln = lane64(), w = t >> 6;
    const unsigned per = (ntiles + 1023u) / 1024u;
    unsigned sum = 0;
    for (unsigned i = 0; i < per; i++) sum += t * per + i < ntiles ? tsum[t * per + i] : 0u;
    unsigned x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(x, o, 64);
        x += ln >= (unsigned)o ? y : 0u;
    }
    if (ln == 63) s_w[w] = x;
    __syncthreads();
    unsigned run = x - sum;
    for (unsigned i = 0; i < w; i++) run += s_w[i];
    for (unsigned i = 0; i < per; i++) {
        if (t * per + i < ntiles) {
            const unsigned v = tsum[t * per + i];
            tsum[t * per + i] = run;
            run += v;
        }
    }
}

__global__ __launch_bounds__(SCAN_TILE) void k_scan_apply(const uint32_t *__restrict__ in, unsigned n,
                                                           const uint32_t *__restrict__ tsum,
                                                           uint32_t *__restrict__ out) {
    __shared__ unsigned s_w[SCAN_TILE / 64];
    const unsigned t = threadIdx.x, ln = lane64(), w = t >> 6;
    const unsigned i = blockIdx.x * SCAN_TILE + t;
    const unsigned v = i < n ? in[i] : 0u;
    unsigned x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(x, o, 64);
        x += ln >= (unsigned)o ? y : 0u;
    }
    if (ln == 63) s_w[w] = x;
    __syncthreads();
    unsigned run = tsum[blockIdx.x] + x - v;
    for (unsigned k = 0; k < w; k++) run += s_w[k];
    if (i < n) out[i] = run;
    if (i == n - 1) out[n] = run + v;
}

}  // namespace

hipError_t launch_neighbors(const Buffers &b, int mode, const float *radius, uint32_t *count, const uint32_t *offset,
                            uint32_t *index, float *rho, unsigned nsys, hipStream_t s) {
    NgbArgs a;
    a.hdr = b.hdr;
    a.head = b.hdr->walk_head;
    a.topo = b.topo;
    a.cbox = b.cbox;
    a.spos = b.spos;
    a.perm = b.vals[sorted_buffer(nsys)];
    a.groups = b.groups;
    a.radius = radius;
    a.scale = mode == NGB_DENSITY ? 2.0f : 1.0f;
    a.wstack = b.wstack;
    a.count = count;
    a.offset = offset;
    a.index = index;
    a.rho = rho;
    hipError_t e = launch_fill_u32(b.hdr->walk_head, WALK_QUEUES * QUEUE_STRIDE, 0u, s);
    if (e != hipSuccess) return e;
    if (mode == NGB_COUNT)
        hipLaunchKernelGGL(k_neighbors<NGB_COUNT>, dim3(b.walk_waves), dim3(64), 0, s, a);
    else if (mode == NGB_LISTS)
        hipLaunchKernelGGL(k_neighbors<NGB_LISTS>, dim3(b.walk_waves), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL(k_neighbors<NGB_DENSITY>, dim3(b.walk_waves), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t *in, unsigned n, uint32_t *out, uint32_t *tmp, hipStream_t s) {
    const unsigned ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(SCAN_TILE), 0, s, in, n, tmp, out);
    return hipGetLastError();
}

}  // namespace mibh
