// Tree pipeline of the force step on gfx950: bounding cube, Morton keys,
// stable LSD radix sort, reorder ("moving"), breadth-first sparse octree and
// groups ("tree-construction"), float64 multipole moments and the per-theta
// opening radii.  The paper's parts are named in its Results section; the
// kernels here are this library's own design for CDNA4 (wave64 ballots,
// LDS-staged windows, no host synchronisation inside a step).
#include "mibh_device.h"

#include <math.h>

namespace mibh {

// --------------------------------------------------------------------------
// wave64 helpers
// --------------------------------------------------------------------------

__device__ __forceinline__ unsigned lane64() { return __lane_id(); }

// Number of set bits of mask in lanes below this one.
__device__ __forceinline__ unsigned rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Lanes (among those in `active`) holding the same 8-bit digit as this lane.
__device__ __forceinline__ unsigned long long match_digit(unsigned d, unsigned long long active) {
    unsigned long long m = active;
#pragma unroll
    for (int b = 0; b < RADIX_BITS; b++) {
        const bool bit = (d >> b) & 1u;
        const unsigned long long v = __ballot(bit);
        m &= bit ? v : ~v;
    }
    return m;
}

// Inclusive scan over the 64 lanes of a wave.
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned y = __shfl_up(v, o, 64);
        if (lane64() >= (unsigned)o) v += y;
    }
    return v;
}

// Exclusive scan of a block of NT threads (NT multiple of 64, <= 1024).
template <int NT>
__device__ __forceinline__ unsigned block_excl_scan(unsigned v, unsigned *s_wave, unsigned *total) {
    const unsigned w = threadIdx.x >> 6;
    const unsigned inc = wave_incl_scan(v);
    if (lane64() == 63) s_wave[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned run = 0;
        for (int i = 0; i < NT / 64; i++) {
            unsigned t = s_wave[i];
            s_wave[i] = run;
            run += t;
        }
        s_wave[NT / 64] = run;
    }
    __syncthreads();
    const unsigned r = s_wave[w] + inc - v;
    *total = s_wave[NT / 64];
    __syncthreads();
    return r;
}

// Morton bit spreading: bit b of v (20 bits) moves to bit 3b.
__device__ __forceinline__ uint64_t spread3(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Inverse of spread3: gathers bits 0, 3, 6, ... into a dense integer.
__device__ __forceinline__ uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

// Number of leading octal digits two 60-bit keys share (0..20).
__device__ __forceinline__ int shared_digits(uint64_t a, uint64_t b) {
    const uint64_t x = a ^ b;
    if (x == 0) return KEY_LEVELS;
    return (__clzll((long long)x) - 4) / 3;
}

// First index j > i whose key differs from key i in the first `lev` octal
// digits (n if none): galloping search over the sorted keys.
__device__ __forceinline__ unsigned run_end(const uint64_t *__restrict__ keys, unsigned n, unsigned i,
                                            int lev) {
    // n is the end of i's system: keys of different systems are never compared
    if (lev == 0) return n;
    const int sh = 3 * (KEY_LEVELS - lev);
    const uint64_t p = keys[i] >> sh;
    unsigned lo = i, step = 1, hi = i + 1;
    while (hi < n && (keys[hi] >> sh) == p) {
        lo = hi;
        step <<= 1;
        hi = (n - i > step) ? i + step : n;
    }
    if (hi > n) hi = n;
    while (hi - lo > 1) {
        const unsigned mid = lo + (hi - lo) / 2;
        if ((keys[mid] >> sh) == p) lo = mid; else hi = mid;
    }
    return hi;
}

// --------------------------------------------------------------------------
// Bounding cube, one per system (grid row y = system)
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_bbox_partial(const float *__restrict__ pos,
                                                      const float *__restrict__ mass,
                                                      const uint32_t *__restrict__ sys_off,
                                                      float *__restrict__ part) {
    const unsigned sys = blockIdx.y;
    const unsigned b0 = sys_off[sys], b1 = sys_off[sys + 1];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    unsigned flags = 0;
    for (unsigned i = b0 + blockIdx.x * 256u + threadIdx.x; i < b1; i += gridDim.x * 256u) {
        const size_t b = (size_t)i * 3;
        const float x[3] = {pos[b], pos[b + 1], pos[b + 2]};
        const float m = mass[i];
        if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(m))) flags |= FLAG_NONFINITE;
        if (m < 0.0f) flags |= FLAG_NEGMASS;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            mn[a] = fminf(mn[a], x[a]);
            mx[a] = fmaxf(mx[a], x[a]);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
        }
        flags |= __shfl_xor(flags, o, 64);
    }
    __shared__ float s[4][8];
    const unsigned w = threadIdx.x >> 6;
    if (lane64() == 0) {
        for (int a = 0; a < 3; a++) { s[w][a] = mn[a]; s[w][3 + a] = mx[a]; }
        s[w][6] = __uint_as_float(flags);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 4; v++) {
            for (int a = 0; a < 3; a++) {
                s[0][a] = fminf(s[0][a], s[v][a]);
                s[0][3 + a] = fmaxf(s[0][3 + a], s[v][3 + a]);
            }
            s[0][6] = __uint_as_float(__float_as_uint(s[0][6]) | __float_as_uint(s[v][6]));
        }
        float *o = part + ((size_t)sys * gridDim.x + blockIdx.x) * 8;
        for (int a = 0; a < 7; a++) o[a] = s[0][a];
    }
}

// Root cube of each system (one block per system): corner = per-axis minimum,
// side 2^k with 2^k > largest extent (frexp of the float64 extent), k = 0 for a
// zero extent.  Block 0 also resets the header.
__global__ __launch_bounds__(256) void k_bbox_final(const float *__restrict__ part, unsigned nblocks,
                                                    unsigned n, unsigned nsys, Header *__restrict__ hdr,
                                                    SysCube *__restrict__ cube) {
    const unsigned sys = blockIdx.x;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    unsigned flags = 0;
    for (unsigned b = threadIdx.x; b < nblocks; b += 256) {
        const float *p = part + ((size_t)sys * nblocks + b) * 8;
        for (int a = 0; a < 3; a++) {
            mn[a] = fminf(mn[a], p[a]);
            mx[a] = fmaxf(mx[a], p[3 + a]);
        }
        flags |= __float_as_uint(p[6]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        for (int a = 0; a < 3; a++) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
        }
        flags |= __shfl_xor(flags, o, 64);
    }
    __shared__ float s[4][8];
    const unsigned w = threadIdx.x >> 6;
    if (lane64() == 0) {
        for (int a = 0; a < 3; a++) { s[w][a] = mn[a]; s[w][3 + a] = mx[a]; }
        s[w][6] = __uint_as_float(flags);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 4; v++) {
            for (int a = 0; a < 3; a++) {
                s[0][a] = fminf(s[0][a], s[v][a]);
                s[0][3 + a] = fmaxf(s[0][3 + a], s[v][3 + a]);
            }
            s[0][6] = __uint_as_float(__float_as_uint(s[0][6]) | __float_as_uint(s[v][6]));
        }
        flags = __float_as_uint(s[0][6]);
        double ext = 0.0;
        for (int a = 0; a < 3; a++) {
            const double e = (double)s[0][3 + a] - (double)s[0][a];
            if (e > ext) ext = e;
        }
        int k = 0;
        if (ext > 0.0) frexp(ext, &k);
        if (flags & FLAG_NONFINITE) {  // keep every later index computation tame
            k = 0;
            for (int a = 0; a < 3; a++) s[0][a] = 0.0f;
        }
        for (int a = 0; a < 3; a++) cube[sys].lo[a] = s[0][a];
        cube[sys].k = k;
        if (flags) atomicOr(&hdr->flags, flags);
    }
}

// Header reset, before the per-system reductions of one build.  The flags of
// the previous build move into the sticky word, so that a driver running many
// steps still sees a condition that one of its earlier builds met.
__global__ void k_header_reset(unsigned n, unsigned nsys, Header *__restrict__ hdr, float4 *__restrict__ cmac,
                               float4 *__restrict__ ceval, float4 *__restrict__ spos, unsigned cap_cells,
                               unsigned n_max) {
    if (threadIdx.x == 0) {
        // the walk's padding cell and particle: massless, far away
        cmac[cap_cells] = make_float4(WALK_FAR, WALK_FAR, WALK_FAR, 0.0f);
        ceval[2 * (size_t)cap_cells] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        ceval[2 * (size_t)cap_cells + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        spos[n_max] = make_float4(WALK_FAR, WALK_FAR, WALK_FAR, 0.0f);
        hdr->nsys = nsys;
        hdr->sticky |= hdr->flags;
        hdr->flags = 0;
        hdr->n = n;
        hdr->ncells = 0;
        hdr->ngroups = 0;
        for (int l = 0; l < 24; l++) hdr->lvl_begin[l] = 0;
    }
    if (threadIdx.x < WALK_QUEUES) hdr->walk_head[QUEUE_STRIDE * threadIdx.x] = 0;
}

hipError_t launch_bbox(const Buffers &b, const float *pos, const float *mass, unsigned n, unsigned nsys,
                       hipStream_t s) {
    const unsigned per = max((unsigned)BBOX_MIN_BLOCKS, (unsigned)BBOX_BLOCKS / nsys);
    hipLaunchKernelGGL(k_header_reset, dim3(1), dim3(64), 0, s, n, nsys, b.hdr, b.cmac, b.ceval, b.spos, b.cap_cells,
                       b.n_max);
    hipLaunchKernelGGL(k_bbox_partial, dim3(per, nsys), dim3(256), 0, s, pos, mass, b.sys_off, b.bbox_part);
    hipLaunchKernelGGL(k_bbox_final, dim3(nsys), dim3(256), 0, s, b.bbox_part, per, n, nsys, b.hdr, b.cube);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Morton keys: q_a = min(floor((x_a - lo_a) 2^(20-k)), 2^20 - 1), bits of
// q_x, q_y, q_z at 3b+2, 3b+1, 3b.
// --------------------------------------------------------------------------

// Also packs (x, y, z, m) of every particle into one float4, so that the
// reorder gathers one 16-byte record per particle instead of two.
__global__ __launch_bounds__(256) void k_keys(const float *__restrict__ pos, const float *__restrict__ mass,
                                              unsigned n, unsigned nsys, const uint32_t *__restrict__ sys_off,
                                              const SysCube *__restrict__ cube, uint64_t *__restrict__ keys,
                                              uint8_t *__restrict__ sys8, float4 *__restrict__ ppack) {
    const unsigned i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    const unsigned sys = nsys > 1 ? system_of(sys_off, nsys, i) : 0u;
    const SysCube c = cube[sys];
    const double s = ldexp(1.0, KEY_LEVELS - c.k);
    const float x[3] = {pos[(size_t)i * 3], pos[(size_t)i * 3 + 1], pos[(size_t)i * 3 + 2]};
    ppack[i] = make_float4(x[0], x[1], x[2], mass[i]);
    uint64_t q[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double f = floor(((double)x[a] - (double)c.lo[a]) * s);
        if (!(f >= 0.0)) f = 0.0;
        if (f > 1048575.0) f = 1048575.0;
        q[a] = (uint64_t)f;
    }
    keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    if (nsys > 1) sys8[i] = (uint8_t)sys;
}

// Refit input: packs (x, y, z, m) like the keys kernel and records non-finite
// values and negative masses in the header flags (the build does this in its
// bounding-box pass).
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ pos, const float *__restrict__ mass,
                                              unsigned n, Header *__restrict__ hdr, float4 *__restrict__ ppack) {
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const float4 p = make_float4(pos[(size_t)i * 3], pos[(size_t)i * 3 + 1], pos[(size_t)i * 3 + 2], mass[i]);
        ppack[i] = p;
        unsigned f = 0;
        if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z) || !isfinite(p.w)) f |= FLAG_NONFINITE;
        if (p.w < 0.0f) f |= FLAG_NEGMASS;
        if (f) atomicOr(&hdr->flags, f);
    }
}

hipError_t launch_pack(const Buffers &b, const float *pos, const float *mass, unsigned n, hipStream_t s) {
    const unsigned grid = min((n + 255u) / 256u, 8192u);
    hipLaunchKernelGGL(k_pack, dim3(grid), dim3(256), 0, s, pos, mass, n, b.hdr, b.ppack);
    return hipGetLastError();
}

hipError_t launch_keys(const Buffers &b, const float *pos, const float *mass, unsigned n, unsigned nsys,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_keys, dim3((n + 255) / 256), dim3(256), 0, s, pos, mass, n, nsys, b.sys_off, b.cube,
                       b.keys[0], b.sys8, b.ppack);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Stable LSD radix sort of (key, index), 8-bit digits, reduce-then-scan:
// per-tile digit histograms -> per-digit scan over tiles -> stable scatter.
// Ranks inside a tile come from wave64 digit matching (8 ballots) processed
// in key order, so equal digits keep their input order.
// --------------------------------------------------------------------------

// Digit of an element: 8 key bits at `shift`, or (shift < 0) the element's
// system, looked up by its original index (the last pass of a batch).
__device__ __forceinline__ unsigned radix_digit(uint64_t key, uint32_t val, int shift,
                                                const uint8_t *__restrict__ sys8) {
    return shift >= 0 ? (unsigned)(key >> shift) & (RADIX - 1) : (unsigned)sys8[val];
}

// AGG: equal digits of a wave are matched first (8 ballots) and their leader
// adds their number, one LDS atomic per distinct digit instead of per element:
// cheaper where digits are concentrated (the high digits of clustered keys,
// the system digit), where per-element atomics collide on one counter.
template <bool AGG>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                             const uint32_t *__restrict__ vals,
                                                             const uint8_t *__restrict__ sys8,
                                                             unsigned n, int shift,
                                                             uint32_t *__restrict__ hist,
                                                             unsigned ntiles) {
    __shared__ uint32_t h[SORT_THREADS / 64][RADIX];
    const unsigned w = threadIdx.x >> 6, ln = lane64();
    for (unsigned j = threadIdx.x; j < (SORT_THREADS / 64) * RADIX; j += SORT_THREADS) (&h[0][0])[j] = 0;
    __syncthreads();
    const unsigned base = blockIdx.x * SORT_TILE + w * (64 * SORT_ITEMS);
#pragma unroll
    for (int t = 0; t < SORT_ITEMS; t++) {
        const unsigned idx = base + t * 64 + ln;
        const bool valid = idx < n;
        const unsigned d = valid ? radix_digit(shift >= 0 ? keys[idx] : 0ull, shift >= 0 ? 0u : vals[idx], shift,
                                               sys8)
                                 : 0u;
        if (AGG) {
            const unsigned long long peers = match_digit(d, __ballot(valid));
            if (valid && ln == (unsigned)(__ffsll((long long)peers) - 1)) atomicAdd(&h[w][d], (unsigned)__popcll(peers));
        } else if (valid) {
            atomicAdd(&h[w][d], 1u);  // integer counts: the order of the adds does not matter
        }
    }
    __syncthreads();
    for (unsigned d = threadIdx.x; d < RADIX; d += SORT_THREADS) {
        unsigned s = 0;
        for (int v = 0; v < SORT_THREADS / 64; v++) s += h[v][d];
        hist[(size_t)d * ntiles + blockIdx.x] = s;
    }
}

// One block per digit: exclusive scan of its row over tiles; row total to btot.
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t *__restrict__ hist, unsigned ntiles,
                                                    uint32_t *__restrict__ btot) {
    __shared__ unsigned s_wave[256 / 64 + 1];
    uint32_t *row = hist + (size_t)blockIdx.x * ntiles;
    const unsigned per = (ntiles + 255) / 256;
    const unsigned b = threadIdx.x * per, e = min(b + per, ntiles);
    unsigned sum = 0;
    for (unsigned j = b; j < e; j++) sum += row[j];
    unsigned total;
    unsigned run = block_excl_scan<256>(sum, s_wave, &total);
    for (unsigned j = b; j < e; j++) {
        const unsigned v = row[j];
        row[j] = run;
        run += v;
    }
    if (threadIdx.x == 0) btot[blockIdx.x] = total;
}

// Ranks every element of the tile (digit, then input order), stages the tile
// in LDS in that order and writes it out from there: consecutive threads then
// write consecutive addresses of each digit's run.
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint8_t *__restrict__ sys8, unsigned n, int shift,
    const uint32_t *__restrict__ hist, const uint32_t *__restrict__ btot, unsigned ntiles) {
    constexpr int NW = SORT_THREADS / 64;
    static_assert(SORT_THREADS % RADIX == 0, "the first RADIX threads look after one digit each");
    __shared__ uint32_t wcnt[NW][RADIX];
    __shared__ uint32_t gshift[RADIX];  // output position of tile position i of digit d: gshift[d] + i
    __shared__ unsigned s_wave[NW + 1];
    __shared__ uint64_t s_key[SORT_TILE];  // the indices (as 32-bit words), then the keys
    const unsigned w = threadIdx.x >> 6, ln = lane64();
    const bool owner = threadIdx.x < (unsigned)RADIX;
    const unsigned dt = owner ? threadIdx.x : 0u;  // the digit this thread looks after
    unsigned total;
    // start of digit dt's run of this tile in the output
    const unsigned gstart = block_excl_scan<SORT_THREADS>(owner ? btot[dt] : 0u, s_wave, &total) +
                            (owner ? hist[(size_t)dt * ntiles + blockIdx.x] : 0u);
    if (owner)
        for (int v = 0; v < NW; v++) wcnt[v][dt] = 0;
    __syncthreads();
    const unsigned base = blockIdx.x * SORT_TILE + w * (64 * SORT_ITEMS);
    uint64_t key[SORT_ITEMS];
    uint32_t val[SORT_ITEMS], rank[SORT_ITEMS];
#pragma unroll
    for (int t = 0; t < SORT_ITEMS; t++) {
        const unsigned idx = base + t * 64 + ln;
        const bool valid = idx < n;
        key[t] = valid ? kin[idx] : 0ull;
        val[t] = valid ? (vin ? vin[idx] : idx) : 0u;
        const unsigned d = valid ? radix_digit(key[t], val[t], shift, sys8) : 0u;
        const unsigned long long peers = match_digit(d, __ballot(valid));
        const unsigned before = wcnt[w][d];
        rank[t] = before + rank_below(peers);
        if (valid && ln == (unsigned)(__ffsll((long long)peers) - 1)) wcnt[w][d] = before + __popcll(peers);
    }
    __syncthreads();
    {
        // tile position of the first element of digit dt from wave v: digits
        // before dt, then waves before v
        unsigned run = 0;
        if (owner)
            for (int v = 0; v < NW; v++) {
                const unsigned c = wcnt[v][dt];
                wcnt[v][dt] = run;
                run += c;
            }
        const unsigned lstart = block_excl_scan<SORT_THREADS>(run, s_wave, &total);
        if (owner) {
            for (int v = 0; v < NW; v++) wcnt[v][dt] += lstart;
            gshift[dt] = gstart - lstart;  // modulo 2^32; gshift + i >= 0 for the tile positions of dt
        }
    }
    __syncthreads();
    // the indices, then the keys, through the same LDS (a third less LDS, three
    // blocks per CU instead of two: sorting 402 -> 395 us at N = 2^22); each
    // thread keeps the indices of its tile positions between the two phases,
    // since the system pass needs an element's index for its digit
    unsigned lpos[SORT_ITEMS];
    uint32_t *s_val = reinterpret_cast<uint32_t *>(s_key);
#pragma unroll
    for (int t = 0; t < SORT_ITEMS; t++) {
        const unsigned idx = base + t * 64 + ln;
        const unsigned d = idx < n ? radix_digit(key[t], val[t], shift, sys8) : 0u;
        lpos[t] = wcnt[w][d] + rank[t];
    }
    const unsigned cnt = min((unsigned)SORT_TILE, n - blockIdx.x * SORT_TILE);
    uint32_t vpos[SORT_ITEMS];  // the index at tile position threadIdx.x + t * SORT_THREADS
    // phase 1: the indices
#pragma unroll
    for (int t = 0; t < SORT_ITEMS; t++)
        if (base + t * 64 + ln < n) s_val[lpos[t]] = val[t];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < SORT_ITEMS; t++) {
        const unsigned i = threadIdx.x + t * SORT_THREADS;
        vpos[t] = i < cnt ? s_val[i] : 0u;
    }
    __syncthreads();
    // phase 2: the keys; position i's output slot from its digit
#pragma unroll
    for (int t = 0; t < SORT_ITEMS; t++)
        if (base + t * 64 + ln < n) s_key[lpos[t]] = key[t];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < SORT_ITEMS; t++) {
        const unsigned i = threadIdx.x + t * SORT_THREADS;
        if (i < cnt) {
            const uint64_t k = s_key[i];
            const uint32_t v = vpos[t];
            const unsigned p = gshift[radix_digit(k, v, shift, sys8)] + i;
            kout[p] = k;
            vout[p] = v;
        }
    }
}

#ifndef MIBH_HIST_AGG_SHIFT
#define MIBH_HIST_AGG_SHIFT 48  // passes over key bits 48.. (and the system pass) match digits first
                                // (sorting at 2^22: 404 us without, 401 us with, 439 us for every pass)
#endif

// 8 passes over the 60-bit keys; a batch adds a last pass by system, which
// gathers each system's particles (in key order) into its input range.
hipError_t launch_sort(const Buffers &b, unsigned n, unsigned nsys, hipStream_t s) {
    const unsigned ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    const int passes = SORT_PASSES + (nsys > 1 ? 1 : 0);
    for (int pass = 0; pass < passes; pass++) {
        const int src = pass & 1, dst = src ^ 1;
        const int shift = pass < SORT_PASSES ? pass * RADIX_BITS : -1;
        if (shift < 0 || shift >= MIBH_HIST_AGG_SHIFT)
            hipLaunchKernelGGL(k_radix_hist<true>, dim3(ntiles), dim3(SORT_THREADS), 0, s, b.keys[src], b.vals[src],
                               b.sys8, n, shift, b.hist, ntiles);
        else
            hipLaunchKernelGGL(k_radix_hist<false>, dim3(ntiles), dim3(SORT_THREADS), 0, s, b.keys[src], b.vals[src],
                               b.sys8, n, shift, b.hist, ntiles);
        hipLaunchKernelGGL(k_radix_scan, dim3(RADIX), dim3(256), 0, s, b.hist, ntiles, b.btot);
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(SORT_THREADS), 0, s, b.keys[src],
                           pass == 0 ? (const uint32_t *)nullptr : b.vals[src], b.keys[dst], b.vals[dst],
                           b.sys8, n, shift, b.hist, b.btot, ntiles);
    }
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Moving: gather (x, y, z, m) into key order; shared digits with the previous key.
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_reorder(const float4 *__restrict__ ppack,
                                                 const uint64_t *__restrict__ keys,
                                                 const uint32_t *__restrict__ perm, unsigned n, unsigned nsys,
                                                 const uint32_t *__restrict__ sys_off,
                                                 float4 *__restrict__ spos, int8_t *__restrict__ cl) {
    const unsigned k = blockIdx.x * 256u + threadIdx.x;
    if (k >= n) return;
    spos[k] = ppack[perm[k]];
    // a system's first particle opens cells at every level, like particle 0
    const bool start = k == 0 || (nsys > 1 && sys_off[system_of(sys_off, nsys, k)] == k);
    cl[k] = start ? (int8_t)-1 : (int8_t)shared_digits(keys[k - 1], keys[k]);
}

hipError_t launch_reorder(const Buffers &b, unsigned n, unsigned nsys, hipStream_t s) {
    const int sb = sorted_buffer(nsys);
    hipLaunchKernelGGL(k_reorder, dim3((n + 255) / 256), dim3(256), 0, s, b.ppack, b.keys[sb], b.vals[sb],
                       n, nsys, b.sys_off, b.spos, b.cl);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Octree and groups, particle-parallel.
//
// With cl(i) the number of leading octal digits keys i-1 and i share, the
// level-l cell containing particle i starts at i iff cl(i) < l, and it holds
// more than w particles iff some window of w+1 consecutive particles around i
// has all its w inner cl values >= l.  So
//   lstar_w(i) = max over windows [a, a+w] containing i of min cl(a+1..a+w)
// is the deepest level whose cell around i holds more than w particles.  The
// leaf of i is at level min(lstar_ncrit + 1, 20) (0 if lstar < 0), its group at
// min(lstar_gcap + 1, 20); particle i starts the cells of levels
// cl(i)+1 .. leaf(i).  Cell numbers are per-level ranks, which gives the
// breadth-first order (level, then key).
// --------------------------------------------------------------------------

// Value at position `pos` (0..127, or 0..191 with three registers) of an array
// held as consecutive 64-lane registers r0, r1, r2: lane pos & 63 of register
// pos >> 6.  Every lane passes its own position; the lane index is shared by the
// shuffles, the register is picked afterwards.
__device__ __forceinline__ int wave_at3(int r0, int r1, int r2, unsigned pos) {
    const int lane = (int)(pos & 63u);
    const int v0 = __shfl(r0, lane, 64), v1 = __shfl(r1, lane, 64), v2 = __shfl(r2, lane, 64);
    return pos < 64u ? v0 : pos < 128u ? v1 : v2;
}
__device__ __forceinline__ int wave_at2(int r0, int r1, unsigned pos) {
    const int lane = (int)(pos & 63u);
    const int v0 = __shfl(r0, lane, 64), v1 = __shfl(r1, lane, 64);
    return pos < 64u ? v0 : v1;
}

__global__ __launch_bounds__(BUILD_THREADS) void k_build_count(
    const int8_t *__restrict__ cl, const uint64_t *__restrict__ keys, unsigned n, unsigned nsys,
    const uint32_t *__restrict__ sys_off, int ncrit, int gcap, uchar4 *__restrict__ lvinfo,
    uint32_t *__restrict__ blkcnt, unsigned nblk) {
    constexpr int NW = BUILD_THREADS / 64;
    __shared__ uint32_t s_cnt[NW][NCOUNTERS];
    const unsigned base = blockIdx.x * BUILD_THREADS;
    const unsigned i = base + threadIdx.x;
    const bool valid = i < n;
    // Each wave on its own, in registers: the cl values of positions wb - 64 ..
    // wb + 127 (wb = the wave's first particle; -1 outside the particles) cover
    // every window that contains one of the wave's particles (ncrit, gcap <= 64).
    // This replaced doubling tables in LDS with 13 block barriers (tree
    // construction at N = 2^22: 148 -> 139 us).
    static_assert(MAX_WINDOW <= 64, "windows reach at most one wave width either side");
    const unsigned ln_ = lane64();
    const long long wb = (long long)base + (long long)(threadIdx.x & ~63u);
    int t[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        const long long j = wb - 64 + 64 * r + ln_;
        t[r] = (j >= 0 && j < (long long)n) ? (int)cl[j] : -1;
    }
    const int ci = t[1];
    // Minima by doubling: after step k, t[r] at lane l is the minimum of the 2^k
    // values from position 64 r + l on (positions past 191 are never asked for).
    const int kn = 31 - __clz(ncrit), kg = 31 - __clz(gcap), kmax = max(kn, kg);
    int tn[3] = {t[0], t[1], t[2]}, tg[3] = {t[0], t[1], t[2]};
    for (int k = 0; k < kmax; k++) {
        const unsigned sh = 1u << k;
        const int src = (int)((ln_ + sh) & 63u);
        const bool wrap = ln_ + sh >= 64u;
        const int a0 = __shfl(t[0], src, 64), a1 = __shfl(t[1], src, 64), a2 = __shfl(t[2], src, 64);
        t[0] = min(t[0], wrap ? a1 : a0);
        t[1] = min(t[1], wrap ? a2 : a1);
        t[2] = min(t[2], wrap ? t[2] : a2);
        if (k + 1 == kn) { tn[0] = t[0]; tn[1] = t[1]; tn[2] = t[2]; }
        if (k + 1 == kg) { tg[0] = t[0]; tg[1] = t[1]; tg[2] = t[2]; }
    }
    // Window minima for the window starts a = wb - 64 + 64 r + lane (r = 0, 1):
    // min cl[a+1 .. a+w] = min(T[a+1], T[a+1+w-2^k]); a start's position is its
    // array position, so a+1 sits at 64 r + lane + 1.
    int mn[2], mg[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const unsigned p = 64u * r + ln_ + 1u;
        mn[r] = min(wave_at3(tn[0], tn[1], tn[2], p), wave_at3(tn[0], tn[1], tn[2], p + (unsigned)(ncrit - (1 << kn))));
        mg[r] = min(wave_at3(tg[0], tg[1], tg[2], p), wave_at3(tg[0], tg[1], tg[2], p + (unsigned)(gcap - (1 << kg))));
    }
    // ln = max of the window minima over the starts tl - w .. tl (tl = the
    // particle's start position, 64 + lane), maxima by doubling over the 128 starts.
    int ln, lg;
    {
        const int kn2 = 31 - __clz(ncrit + 1), kg2 = 31 - __clz(gcap + 1), kmax2 = max(kn2, kg2);
        int un[2] = {mn[0], mn[1]}, ug[2] = {mg[0], mg[1]};
        int vn[2] = {mn[0], mn[1]}, vg[2] = {mg[0], mg[1]};  // the tables at kn2 and kg2
        for (int k = 0; k < kmax2; k++) {
            const unsigned sh = 1u << k;
            const int src = (int)((ln_ + sh) & 63u);
            const bool wrap = ln_ + sh >= 64u;
            const int b0 = __shfl(un[0], src, 64), b1 = __shfl(un[1], src, 64);
            const int c0 = __shfl(ug[0], src, 64), c1 = __shfl(ug[1], src, 64);
            un[0] = max(un[0], wrap ? b1 : b0);
            un[1] = max(un[1], wrap ? un[1] : b1);
            ug[0] = max(ug[0], wrap ? c1 : c0);
            ug[1] = max(ug[1], wrap ? ug[1] : c1);
            if (k + 1 == kn2) { vn[0] = un[0]; vn[1] = un[1]; }
            if (k + 1 == kg2) { vg[0] = ug[0]; vg[1] = ug[1]; }
        }
        const unsigned tl = 64u + ln_;
        ln = max(wave_at2(vn[0], vn[1], tl - (unsigned)ncrit), wave_at2(vn[0], vn[1], tl - (1u << kn2) + 1u));
        lg = max(wave_at2(vg[0], vg[1], tl - (unsigned)gcap), wave_at2(vg[0], vg[1], tl - (1u << kg2) + 1u));
    }
    const int leaf = ln < 0 ? 0 : min(ln + 1, KEY_LEVELS);
    const int glev = lg < 0 ? 0 : min(lg + 1, KEY_LEVELS);
    const int clo = ci + 1;
    bool gstart;
    unsigned oversized = 0;
    if (lg >= KEY_LEVELS && valid) {
        // a run of more than gcap identical keys: cut into chunks of gcap from its start
        oversized = 1;
        unsigned start = i;
        if (ci >= KEY_LEVELS) {
            const uint64_t key = keys[i];
            // first index of the run lies in [start of i's system, i]
            unsigned lo = nsys > 1 ? sys_off[system_of(sys_off, nsys, i)] : 0u, hi = i;
            while (lo < hi) {
                const unsigned mid = lo + (hi - lo) / 2;
                if (keys[mid] < key) lo = mid + 1; else hi = mid;
            }
            start = lo;
        }
        gstart = ((i - start) % (unsigned)gcap) == 0;
    } else {
        gstart = ci < glev;
    }
    if (valid) lvinfo[i] = make_uchar4((unsigned char)clo, (unsigned char)leaf, (unsigned char)glev,
                                       (unsigned char)((gstart ? 1 : 0) | (oversized << 1)));
    // Padding threads start no cell (first level 1 > leaf level 0) and no
    // group, so the ballot loops below need no per-lane validity branch; the
    // wave-uniform counts are stored by every lane.
    const int c_lo = valid ? clo : 1, c_hi = valid ? leaf : 0;
    const bool g_st = valid && gstart;
    const unsigned w = threadIdx.x >> 6;
    for (int l = 0; l <= KEY_LEVELS; l++) {
        const unsigned long long b = __ballot(c_lo <= l && l <= c_hi);
        s_cnt[w][l] = (uint32_t)__popcll(b);
    }
    {
        const unsigned long long b = __ballot(g_st);
        s_cnt[w][NCOUNTERS - 1] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    if (threadIdx.x < NCOUNTERS) {
        uint32_t s = 0;
        for (int v = 0; v < NW; v++) s += s_cnt[v][threadIdx.x];
        blkcnt[(size_t)threadIdx.x * nblk + blockIdx.x] = s;
    }
}

// One block per counter: exclusive scan over blocks, totals to ctot.
__global__ __launch_bounds__(1024) void k_build_scan(uint32_t *__restrict__ blkcnt, unsigned nblk,
                                                     uint32_t *__restrict__ ctot) {
    __shared__ unsigned s_wave[1024 / 64 + 1];
    uint32_t *row = blkcnt + (size_t)blockIdx.x * nblk;
    const unsigned per = (nblk + 1023) / 1024;
    const unsigned b = threadIdx.x * per, e = min(b + per, nblk);
    unsigned sum = 0;
    for (unsigned j = b; j < e; j++) sum += row[j];
    unsigned total;
    unsigned run = block_excl_scan<1024>(sum, s_wave, &total);
    for (unsigned j = b; j < e; j++) {
        const unsigned v = row[j];
        row[j] = run;
        run += v;
    }
    if (threadIdx.x == 0) ctot[blockIdx.x] = total;
}

// Cell ends searched at the end of a block.  A cell whose end lies beyond its
// first particle's wave contains that wave's last particle, so a wave defers at
// most one cell per level: 16 waves x 21 levels fit (the inline search below
// is only a guard).
constexpr unsigned BUILD_PENDING = 512;
static_assert(BUILD_PENDING >= (BUILD_THREADS / 64) * (KEY_LEVELS + 1), "one deferred cell per wave and level");

__global__ __launch_bounds__(BUILD_THREADS) void k_build_write(
    const uchar4 *__restrict__ lvinfo, const uint64_t *__restrict__ keys, unsigned n, unsigned nsys,
    const uint32_t *__restrict__ sys_off, int gcap, const uint32_t *__restrict__ blkcnt,
    const uint32_t *__restrict__ ctot, unsigned nblk, Header *__restrict__ hdr, uint4 *__restrict__ topo,
    uint2 *__restrict__ groups, unsigned cap_cells) {
    constexpr int NW = BUILD_THREADS / 64;
    __shared__ uint32_t s_base[NCOUNTERS];   // first cell number of each level; 0 for groups
    __shared__ uint32_t s_blk[NCOUNTERS];    // this block's offset within each level
    __shared__ uint32_t s_wpre[NW][NCOUNTERS];
    // cells whose end lies beyond their wave: record (cell, first, child_first,
    // system | level word) and (system end, group + 1 or 0), searched at the end
    __shared__ uint4 s_prec[BUILD_PENDING];
    __shared__ uint2 s_pext[BUILD_PENDING];
    __shared__ unsigned s_np;
    if (threadIdx.x == 0) s_np = 0;
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int l = 0; l <= KEY_LEVELS; l++) {
            s_base[l] = run;
            run += ctot[l];
        }
        s_base[NCOUNTERS - 1] = 0;
        if (blockIdx.x == 0) {
            for (int l = 0; l <= KEY_LEVELS; l++) hdr->lvl_begin[l] = s_base[l];
            hdr->lvl_begin[KEY_LEVELS + 1] = run;
            hdr->ncells = run;
            hdr->ngroups = ctot[NCOUNTERS - 1];
            if (run > cap_cells) atomicOr(&hdr->flags, FLAG_CELLCAP);
        }
    }
    if (threadIdx.x < NCOUNTERS) s_blk[threadIdx.x] = blkcnt[(size_t)threadIdx.x * nblk + blockIdx.x];
    const unsigned i = blockIdx.x * BUILD_THREADS + threadIdx.x;
    const bool valid = i < n;
    // padding threads: first level 1 > leaf level 0 and no group start
    const uchar4 info = valid ? lvinfo[i] : make_uchar4(1, 0, 0, 0);
    const int clo = info.x, leaf = info.y, glev = info.z;
    const bool gstart = (info.w & 1) != 0;
    const unsigned w = threadIdx.x >> 6;
    for (int c = 0; c < NCOUNTERS; c++) {
        const bool pred = c < NCOUNTERS - 1 ? (clo <= c && c <= leaf) : gstart;
        const unsigned long long b = __ballot(pred);
        s_wpre[w][c] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    if (threadIdx.x < NCOUNTERS) {
        uint32_t run = 0;
        for (int v = 0; v < NW; v++) {
            const uint32_t t = s_wpre[v][threadIdx.x];
            s_wpre[v][threadIdx.x] = run;
            run += t;
        }
    }
    __syncthreads();
    // the system of this particle and its end: runs never cross systems
    const unsigned sys = (nsys > 1 && valid) ? system_of(sys_off, nsys, i) : 0u;
    const unsigned send = nsys > 1 ? (valid ? sys_off[sys + 1] : n) : n;
    // cells, deepest level first so that each cell knows its first child's number.
    // A level-l cell starting at i ends at the first j > i with cl(j) < l (or
    // where the particles end): the wave finds it from a ballot of those
    // boundaries when it lies inside the wave, else by searching the keys.
    // Ends found by searching the keys are deferred to the end of the kernel,
    // where the block's threads take one search each: a particle that starts
    // large cells at many levels (the first particles of the big cells) would
    // otherwise run its searches one after the other, the kernel's longest path.
    const int ci = clo - 1;
    const unsigned ln = lane64();
    unsigned next = 0, gend = 0, gpend = 0;
    for (int l = KEY_LEVELS; l >= 0; l--) {
        const bool pred = clo <= l && l <= leaf;
        const unsigned long long b = __ballot(pred);
        if (b == 0) continue;
        const unsigned long long bnd = __ballot(!valid || ci < l);
        if (pred) {
            const unsigned idx = s_base[l] + s_blk[l] + s_wpre[w][l] + rank_below(b);
            const unsigned long long after = ln < 63 ? bnd >> (ln + 1) : 0ull;
            const unsigned cf = l < leaf ? next : 0u;
            const unsigned word = (sys << 16) | ((unsigned)l << 8);
            const unsigned k = after ? BUILD_PENDING : atomicAdd(&s_np, 1u);
            if (k < BUILD_PENDING) {
                s_prec[k] = make_uint4(idx, i, cf, word);
                s_pext[k] = make_uint2(send, 0u);
                if (l == glev) gpend = k + 1;
            } else {  // end inside the wave, or no room left to defer
                const unsigned end = after ? i + (unsigned)__ffsll((long long)after) : run_end(keys, send, i, l);
                if (idx < cap_cells) topo[idx] = make_uint4(i, end - i, cf, word);
                if (l == glev) gend = end;
            }
            next = idx;
        }
    }
    {
        const unsigned long long b = __ballot(gstart);
        if (gstart) {
            const unsigned g = s_blk[NCOUNTERS - 1] + s_wpre[w][NCOUNTERS - 1] + rank_below(b);
            const unsigned gword = (sys << 16) | ((unsigned)glev << 8);
            if (info.w & 2) {
                groups[g] = make_uint2(i, gword | min((unsigned)gcap, run_end(keys, send, i, KEY_LEVELS) - i));
            } else if (gend == 0 && gpend) {
                s_pext[gpend - 1].y = g + 1;  // written with its cell's end below
            } else {
                groups[g] = make_uint2(i, gword | ((gend ? gend : run_end(keys, send, i, glev)) - i));
            }
        }
    }
    __syncthreads();
    const unsigned np = min(s_np, BUILD_PENDING);
    for (unsigned k = threadIdx.x; k < np; k += BUILD_THREADS) {
        const uint4 r = s_prec[k];
        const uint2 e = s_pext[k];
        const unsigned end = run_end(keys, e.x, r.y, (int)((r.w >> 8) & 255u));
        if (r.x < cap_cells) topo[r.x] = make_uint4(r.y, end - r.y, r.z, r.w);
        if (e.y) groups[e.y - 1] = make_uint2(r.y, r.w | (end - r.y));
    }
}

// Children of an internal cell are the consecutive next-level cells that start inside it.
__global__ __launch_bounds__(256) void k_build_nchild(const Header *__restrict__ hdr,
                                                      uint4 *__restrict__ topo, unsigned cap_cells) {
    if (hdr->flags & FLAG_CELLCAP) return;  // cell numbers beyond the capacity were never written
    const unsigned nc = min(hdr->ncells, cap_cells);
    for (unsigned c = blockIdx.x * 256u + threadIdx.x; c < nc; c += gridDim.x * 256u) {
        const uint4 t = topo[c];
        if (t.z == 0) continue;
        const unsigned l = (t.w >> 8) & 255u;
        const unsigned lend = min(hdr->lvl_begin[l + 2], nc);
        const unsigned end = t.x + t.y;
        unsigned nch = 0;
        for (unsigned k = t.z; k < lend && nch < 8; k++) {
            if (topo[k].x < end) nch++;
            else break;
        }
        reinterpret_cast<unsigned *>(topo)[4 * (size_t)c + 3] = (t.w & 0xffff0000u) | (l << 8) | nch;
    }
}

hipError_t launch_build(const Buffers &b, unsigned n, unsigned nsys, int ncrit, int gcap, hipStream_t s) {
    const unsigned nblk = (n + BUILD_THREADS - 1) / BUILD_THREADS;
    const uint64_t *keys = b.keys[sorted_buffer(nsys)];
    hipLaunchKernelGGL(k_build_count, dim3(nblk), dim3(BUILD_THREADS), 0, s, b.cl, keys, n, nsys, b.sys_off,
                       ncrit, gcap, b.lvinfo, b.blkcnt, nblk);
    hipLaunchKernelGGL(k_build_scan, dim3(NCOUNTERS), dim3(1024), 0, s, b.blkcnt, nblk, b.ctot);
    hipLaunchKernelGGL(k_build_write, dim3(nblk), dim3(BUILD_THREADS), 0, s, b.lvinfo, keys, n, nsys, b.sys_off,
                       gcap, b.blkcnt, b.ctot, nblk, b.hdr, b.topo, b.groups, b.cap_cells);
    const unsigned grid = min((b.cap_cells + 255u) / 256u, 4096u);
    hipLaunchKernelGGL(k_build_nchild, dim3(grid), dim3(256), 0, s, b.hdr, b.topo, b.cap_cells);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Multipole moments, float64: one launch for the leaves of every level (they
// depend on particles only), then one per level for its internal cells, from
// the deepest up.
//   leaf:     M = sum m, com = (sum fma(m, x, .)) / M, S_ab = sum fma(m d_a, d_b, .)
//   internal: M = sum M_c, com = (sum fma(M_c, com_c, .)) / M,
//             S_ab = sum (S_c,ab + (M_c e_a) e_b), e = com_c - com
//   Q = 3 S - tr(S) I, delta = |com - geometric centre|
//   box = float32 min/max of the cell's particles (children's boxes for an
//   internal cell); l' = max(l, 2 max_a max(centre_a - min_a, max_a - centre_a)):
//   the side of the smallest cube about the geometric centre that holds the
//   particles, never below the cell side.  A freshly built cell holds its
//   particles, so l' = l; after a refit (particles moved, tree kept) l' grows
//   with the particles that left their cells.
// The operation order is fixed and nothing is contracted except the explicit
// fma calls, so every run gives the same bits.
// --------------------------------------------------------------------------

constexpr unsigned LEAF_REGS = 16;  // leaves up to this size are summed from registers

// Side and geometric centre of cell t (level from its record, corner from the
// key prefix of its first particle).
__device__ __forceinline__ double cell_geometry(const uint4 &t, const SysCube *__restrict__ cube,
                                                const uint64_t *__restrict__ keys, double centre[3]) {
#pragma clang fp contract(off)
    const int lev = (int)((t.w >> 8) & 255u);
    const SysCube cb3 = cube[t.w >> 16];
    const double lo[3] = {(double)cb3.lo[0], (double)cb3.lo[1], (double)cb3.lo[2]};
    const double l = ldexp(1.0, cb3.k - lev);
    const uint64_t pre = keys[t.x] >> (3 * (KEY_LEVELS - lev));
    const double q[3] = {(double)compact3(pre >> 2), (double)compact3(pre >> 1), (double)compact3(pre)};
    for (int a = 0; a < 3; a++) {
        const double corner = lo[a] + q[a] * l;
        centre[a] = corner + 0.5 * l;
    }
    return l;
}

// Writes cell c's moments and the quantities derived from them.
__device__ __forceinline__ void store_cell(unsigned c, double l, const double centre[3], double M,
                                           const double com[3], const double S[6], const float bn[3],
                                           const float bx[3], double *__restrict__ mp, double *__restrict__ delta,
                                           float *__restrict__ cbox, double *__restrict__ lside,
                                           float4 *__restrict__ cmac, float4 *__restrict__ ceval) {
#pragma clang fp contract(off)
    double *o = mp + 10 * (size_t)c;
    o[0] = M;
    o[1] = com[0];
    o[2] = com[1];
    o[3] = com[2];
    for (int s = 0; s < 6; s++) o[4 + s] = S[s];
    const double tr = (S[0] + S[1]) + S[2];
    const double Q0 = 3.0 * S[0] - tr, Q1 = 3.0 * S[1] - tr, Q2 = 3.0 * S[2] - tr;
    const double dx = com[0] - centre[0], dy = com[1] - centre[1], dz = com[2] - centre[2];
    delta[c] = sqrt((dx * dx + dy * dy) + dz * dz);
    double reach = 0.0;
    for (int a = 0; a < 3; a++) {
        reach = fmax(reach, centre[a] - (double)bn[a]);
        reach = fmax(reach, (double)bx[a] - centre[a]);
        cbox[6 * (size_t)c + a] = bn[a];
        cbox[6 * (size_t)c + 3 + a] = bx[a];
    }
    lside[c] = fmax(l, 2.0 * reach);
    cmac[c] = make_float4((float)com[0], (float)com[1], (float)com[2], 0.0f);
    ceval[2 * (size_t)c] = make_float4((float)M, (float)Q0, (float)Q1, (float)Q2);
    ceval[2 * (size_t)c + 1] = make_float4((float)(3.0 * S[3]), (float)(3.0 * S[4]), (float)(3.0 * S[5]), 0.0f);
}

// Every leaf of every level.
__global__ __launch_bounds__(256) void k_multipole_leaves(
    const Header *__restrict__ hdr, const SysCube *__restrict__ cube, const uint4 *__restrict__ topo,
    const float4 *__restrict__ spos, const uint64_t *__restrict__ keys, double *__restrict__ mp,
    double *__restrict__ delta, float *__restrict__ cbox, double *__restrict__ lside, float4 *__restrict__ cmac,
    float4 *__restrict__ ceval, unsigned cap_cells) {
#pragma clang fp contract(off)
    if (hdr->flags & FLAG_CELLCAP) return;
    const unsigned nc = min(hdr->ncells, cap_cells);
    for (unsigned c = blockIdx.x * 256u + threadIdx.x; c < nc; c += gridDim.x * 256u) {
        const uint4 t = topo[c];
        if ((t.w & 255u) != 0) continue;
        double centre[3];
        const double l = cell_geometry(t, cube, keys, centre);
        double M = 0.0, cm[3] = {0.0, 0.0, 0.0}, com[3];
        double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        float bn[3], bx[3];
        if (t.y <= LEAF_REGS) {
            // a leaf of up to LEAF_REGS particles: all loads in flight at once,
            // both passes from registers (same operations in the same order)
            float4 pr[LEAF_REGS];
#pragma unroll
            for (int j = 0; j < LEAF_REGS; j++)
                pr[j] = (unsigned)j < t.y ? spos[t.x + j] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            bn[0] = bx[0] = pr[0].x;
            bn[1] = bx[1] = pr[0].y;
            bn[2] = bx[2] = pr[0].z;
#pragma unroll
            for (int j = 1; j < LEAF_REGS; j++) {
                if ((unsigned)j < t.y) {
                    bn[0] = fminf(bn[0], pr[j].x);
                    bx[0] = fmaxf(bx[0], pr[j].x);
                    bn[1] = fminf(bn[1], pr[j].y);
                    bx[1] = fmaxf(bx[1], pr[j].y);
                    bn[2] = fminf(bn[2], pr[j].z);
                    bx[2] = fmaxf(bx[2], pr[j].z);
                }
            }
#pragma unroll
            for (int j = 0; j < LEAF_REGS; j++) {
                if ((unsigned)j < t.y) {
                    const double m = (double)pr[j].w;
                    M = M + m;
                    cm[0] = fma(m, (double)pr[j].x, cm[0]);
                    cm[1] = fma(m, (double)pr[j].y, cm[1]);
                    cm[2] = fma(m, (double)pr[j].z, cm[2]);
                }
            }
            for (int a = 0; a < 3; a++) com[a] = M > 0.0 ? cm[a] / M : centre[a];
            // the second pass converts the particles to float64 again instead of
            // keeping 16 x 4 float64 values live across the divisions (128 registers)
#pragma unroll
            for (int j = 0; j < LEAF_REGS; j++)
                asm volatile("" : "+v"(pr[j].x), "+v"(pr[j].y), "+v"(pr[j].z), "+v"(pr[j].w));
#pragma unroll
            for (int j = 0; j < LEAF_REGS; j++) {
                if ((unsigned)j < t.y) {
                    const double m = (double)pr[j].w;
                    const double dx = (double)pr[j].x - com[0], dy = (double)pr[j].y - com[1],
                                 dz = (double)pr[j].z - com[2];
                    S[0] = fma(m * dx, dx, S[0]);
                    S[1] = fma(m * dy, dy, S[1]);
                    S[2] = fma(m * dz, dz, S[2]);
                    S[3] = fma(m * dx, dy, S[3]);
                    S[4] = fma(m * dx, dz, S[4]);
                    S[5] = fma(m * dy, dz, S[5]);
                }
            }
        } else {
            {
                const float4 p0 = spos[t.x];
                bn[0] = bx[0] = p0.x;
                bn[1] = bx[1] = p0.y;
                bn[2] = bx[2] = p0.z;
            }
            for (unsigned j = t.x; j < t.x + t.y; j++) {
                const float4 p = spos[j];
                bn[0] = fminf(bn[0], p.x);
                bx[0] = fmaxf(bx[0], p.x);
                bn[1] = fminf(bn[1], p.y);
                bx[1] = fmaxf(bx[1], p.y);
                bn[2] = fminf(bn[2], p.z);
                bx[2] = fmaxf(bx[2], p.z);
                const double m = (double)p.w;
                M = M + m;
                cm[0] = fma(m, (double)p.x, cm[0]);
                cm[1] = fma(m, (double)p.y, cm[1]);
                cm[2] = fma(m, (double)p.z, cm[2]);
            }
            for (int a = 0; a < 3; a++) com[a] = M > 0.0 ? cm[a] / M : centre[a];
            for (unsigned j = t.x; j < t.x + t.y; j++) {
                const float4 p = spos[j];
                const double m = (double)p.w;
                const double dx = (double)p.x - com[0], dy = (double)p.y - com[1], dz = (double)p.z - com[2];
                S[0] = fma(m * dx, dx, S[0]);
                S[1] = fma(m * dy, dy, S[1]);
                S[2] = fma(m * dz, dz, S[2]);
                S[3] = fma(m * dx, dy, S[3]);
                S[4] = fma(m * dx, dz, S[4]);
                S[5] = fma(m * dy, dz, S[5]);
            }
        }
        store_cell(c, l, centre, M, com, S, bn, bx, mp, delta, cbox, lside, cmac, ceval);
    }
}

// The internal cells of level lev (their children, at level lev + 1, are
// done).  The up to 8 children's moments and boxes are loaded together, one
// round trip per cell instead of one per child, then combined in child order.
// One wave per workgroup: about one cell in five of a level is internal, and
// the cell code holds many registers (two waves per SIMD), so small
// workgroups spread a level's internal cells over more compute units.
constexpr unsigned MP_INTERNAL_THREADS = 64;
#ifndef MP_INTERNAL_GRID
#define MP_INTERNAL_GRID 1024u  // workgroups per level launch (grid-stride over the level's cells; 8192 and 256 were slower)
#endif

__global__ __launch_bounds__(MP_INTERNAL_THREADS) void k_multipole_internal(
    int lev, const Header *__restrict__ hdr, const SysCube *__restrict__ cube, const uint4 *__restrict__ topo,
    const uint64_t *__restrict__ keys, double *__restrict__ mp, double *__restrict__ delta,
    float *__restrict__ cbox, double *__restrict__ lside, float4 *__restrict__ cmac, float4 *__restrict__ ceval,
    unsigned cap_cells) {
#pragma clang fp contract(off)
    if (hdr->flags & FLAG_CELLCAP) return;
    const unsigned nc = min(hdr->ncells, cap_cells);
    const unsigned cb = min(hdr->lvl_begin[lev], nc), ce = min(hdr->lvl_begin[lev + 1], nc);
    for (unsigned c = cb + blockIdx.x * MP_INTERNAL_THREADS + threadIdx.x; c < ce;
         c += gridDim.x * MP_INTERNAL_THREADS) {
        const uint4 t = topo[c];
        const unsigned nch = t.w & 255u;
        if (nch == 0) continue;
        double2 cm2[8][5];  // child moments: M, com xyz, S xx yy zz xy xz yz
        float2 cb2[8][3];   // child boxes: min xyz, max xyz
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if ((unsigned)j < nch) {
                const double2 *pm = reinterpret_cast<const double2 *>(mp + 10 * (size_t)(t.z + j));
                const float2 *pb = reinterpret_cast<const float2 *>(cbox + 6 * (size_t)(t.z + j));
#pragma unroll
                for (int a = 0; a < 5; a++) cm2[j][a] = pm[a];
#pragma unroll
                for (int a = 0; a < 3; a++) cb2[j][a] = pb[a];
            }
        }
        double centre[3];
        const double l = cell_geometry(t, cube, keys, centre);
        float bn[3] = {cb2[0][0].x, cb2[0][0].y, cb2[0][1].x}, bx[3] = {cb2[0][1].y, cb2[0][2].x, cb2[0][2].y};
#pragma unroll
        for (int j = 1; j < 8; j++) {
            if ((unsigned)j < nch) {
                bn[0] = fminf(bn[0], cb2[j][0].x);
                bn[1] = fminf(bn[1], cb2[j][0].y);
                bn[2] = fminf(bn[2], cb2[j][1].x);
                bx[0] = fmaxf(bx[0], cb2[j][1].y);
                bx[1] = fmaxf(bx[1], cb2[j][2].x);
                bx[2] = fmaxf(bx[2], cb2[j][2].y);
            }
        }
        double M = 0.0, cm[3] = {0.0, 0.0, 0.0}, com[3];
        double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if ((unsigned)j < nch) {
                const double Mc = cm2[j][0].x;
                M = M + Mc;
                cm[0] = fma(Mc, cm2[j][0].y, cm[0]);
                cm[1] = fma(Mc, cm2[j][1].x, cm[1]);
                cm[2] = fma(Mc, cm2[j][1].y, cm[2]);
            }
        }
        for (int a = 0; a < 3; a++) com[a] = M > 0.0 ? cm[a] / M : centre[a];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if ((unsigned)j < nch) {
                const double Mc = cm2[j][0].x;
                const double ex = cm2[j][0].y - com[0], ey = cm2[j][1].x - com[1], ez = cm2[j][1].y - com[2];
                S[0] = S[0] + (cm2[j][2].x + (Mc * ex) * ex);
                S[1] = S[1] + (cm2[j][2].y + (Mc * ey) * ey);
                S[2] = S[2] + (cm2[j][3].x + (Mc * ez) * ez);
                S[3] = S[3] + (cm2[j][3].y + (Mc * ex) * ey);
                S[4] = S[4] + (cm2[j][4].x + (Mc * ex) * ez);
                S[5] = S[5] + (cm2[j][4].y + (Mc * ey) * ez);
            }
        }
        store_cell(c, l, centre, M, com, S, bn, bx, mp, delta, cbox, lside, cmac, ceval);
    }
}

hipError_t launch_multipoles(const Buffers &b, unsigned nsys, hipStream_t s) {
    const uint64_t *keys = b.keys[sorted_buffer(nsys)];
    // up to one thread per cell at N = 2^22 (multipoles 210 us with 2048 blocks, 204 us with 4096)
    const unsigned grid = min((b.cap_cells + 255u) / 256u, 4096u);
    hipLaunchKernelGGL(k_multipole_leaves, dim3(grid), dim3(256), 0, s, b.hdr, b.cube, b.topo, b.spos, keys, b.mp,
                       b.delta, b.cbox, b.lside, b.cmac, b.ceval, b.cap_cells);
    // level KEY_LEVELS holds leaves only
    const unsigned igrid = min((b.cap_cells + MP_INTERNAL_THREADS - 1u) / MP_INTERNAL_THREADS, MP_INTERNAL_GRID);
    for (int lev = KEY_LEVELS - 1; lev >= 0; lev--)
        hipLaunchKernelGGL(k_multipole_internal, dim3(igrid), dim3(MP_INTERNAL_THREADS), 0, s, lev, b.hdr, b.cube,
                           b.topo, keys, b.mp, b.delta, b.cbox, b.lside, b.cmac, b.ceval, b.cap_cells);
    return hipGetLastError();
}

// r_open = l'/theta + delta in float64 (a correctly rounded division; for a
// fresh cell l' = 2^(k - level) and the quotient is the exact scaling of
// fl(1/theta)), squared in float64, rounded once to float32.
__global__ __launch_bounds__(256) void k_mac_prep(Header *__restrict__ hdr, const double *__restrict__ lside,
                                                  const double *__restrict__ delta, double theta,
                                                  float4 *__restrict__ cmac, unsigned cap_cells) {
#pragma clang fp contract(off)
    if (hdr->flags & FLAG_CELLCAP) return;
    const unsigned nc = min(hdr->ncells, cap_cells);
    if (blockIdx.x == 0 && threadIdx.x < WALK_QUEUES) {  // queues of the walk that follows
        hdr->walk_head[QUEUE_STRIDE * threadIdx.x] = 0;
        hdr->prefix_head[QUEUE_STRIDE * threadIdx.x] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr->pool_head = 0;
        hdr->anchor_count = 0;
        hdr->anchor_fail = 0;
    }
    for (unsigned c = blockIdx.x * 256u + threadIdx.x; c < nc; c += gridDim.x * 256u) {
        const double ro = lside[c] / theta + delta[c];
        cmac[c].w = (float)(ro * ro);
    }
}

hipError_t launch_mac_prep(const Buffers &b, unsigned nsys, double theta, hipStream_t s) {
    (void)nsys;
    const unsigned grid = min((b.cap_cells + 255u) / 256u, 4096u);
    hipLaunchKernelGGL(k_mac_prep, dim3(grid), dim3(256), 0, s, b.hdr, b.lside, b.delta, theta, b.cmac,
                       b.cap_cells);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Energies: W = 1/2 sum m phi, T = 1/2 sum m v^2 in float64; every block sums
// a fixed strided set, then one block sums the partials in a fixed order.
// --------------------------------------------------------------------------

__global__ __launch_bounds__(ENERGY_THREADS) void k_energy_partial(const float *__restrict__ mass,
                                                                   const float *__restrict__ pot,
                                                                   const float *__restrict__ vel,
                                                                   unsigned n, double *__restrict__ part) {
    double w = 0.0, t = 0.0;
    for (unsigned i = blockIdx.x * ENERGY_THREADS + threadIdx.x; i < n; i += ENERGY_BLOCKS * ENERGY_THREADS) {
        const double m = (double)mass[i];
        w += m * (double)pot[i];
        if (vel) {
            const double vx = vel[3 * (size_t)i], vy = vel[3 * (size_t)i + 1], vz = vel[3 * (size_t)i + 2];
            t += m * (vx * vx + vy * vy + vz * vz);
        }
    }
    __shared__ double sw[ENERGY_THREADS], st[ENERGY_THREADS];
    sw[threadIdx.x] = w;
    st[threadIdx.x] = t;
    __syncthreads();
    for (int o = ENERGY_THREADS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) {
            sw[threadIdx.x] += sw[threadIdx.x + o];
            st[threadIdx.x] += st[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sw[0];
        part[2 * blockIdx.x + 1] = st[0];
    }
}

__global__ __launch_bounds__(ENERGY_THREADS) void k_energy_final(const double *__restrict__ part,
                                                                 double *__restrict__ out) {
    __shared__ double sw[ENERGY_THREADS], st[ENERGY_THREADS];
    double w = 0.0, t = 0.0;
    for (int b = threadIdx.x; b < ENERGY_BLOCKS; b += ENERGY_THREADS) {
        w += part[2 * b];
        t += part[2 * b + 1];
    }
    sw[threadIdx.x] = w;
    st[threadIdx.x] = t;
    __syncthreads();
    for (int o = ENERGY_THREADS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) {
            sw[threadIdx.x] += sw[threadIdx.x + o];
            st[threadIdx.x] += st[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = 0.5 * st[0];
        out[1] = 0.5 * sw[0];
    }
}

hipError_t launch_energy(const Buffers &b, const float *mass, const float *pot, const float *vel,
                         unsigned n, double *d_out2, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_partial, dim3(ENERGY_BLOCKS), dim3(ENERGY_THREADS), 0, s, mass, pot, vel, n,
                       b.epart);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(ENERGY_THREADS), 0, s, b.epart, d_out2);
    return hipGetLastError();
}

}  // namespace mibh
