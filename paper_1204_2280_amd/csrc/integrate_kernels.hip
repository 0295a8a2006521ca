// Shared-time-step leapfrog (kick-drift-kick) around the force step: the
// paper's code integrates its particles every step on the GPU with nothing
// sent back to the host (Introduction; Results section); the integrator is
// not specified there, and a second-order, time-reversible leapfrog is the
// reading taken here.
//
// One fused kernel serves both halves of a step: v <- v + dt_kick a, then
// x <- x + dt_drift v with the updated v, each update one fused multiply-add
// (one rounding) on the float32 state.  It is HBM-bound: a kick reads 24 bytes
// (velocity, acceleration) and writes 12 per particle; the drift adds 12 read
// and 12 written (the position).
#include "mibh_device.h"

namespace mibh {

namespace {

__global__ __launch_bounds__(256) void k_kick_drift(float *__restrict__ pos, float *__restrict__ vel,
                                                    const float *__restrict__ acc, unsigned n3, float dt_kick,
                                                    float dt_drift, int drift) {
    for (unsigned j = blockIdx.x * 256u + threadIdx.x; j < n3; j += gridDim.x * 256u) {
        const float v = fmaf(dt_kick, acc[j], vel[j]);
        vel[j] = v;
        if (drift) pos[j] = fmaf(dt_drift, v, pos[j]);
    }
}

}  // namespace

hipError_t launch_kick_drift(float *pos, float *vel, const float *acc, unsigned n, float dt_kick, float dt_drift,
                             hipStream_t s) {
    const unsigned n3 = 3u * n;
    const unsigned grid = min((n3 + 255u) / 256u, 8192u);
    hipLaunchKernelGGL(k_kick_drift, dim3(grid), dim3(256), 0, s, pos, vel, acc, n3, dt_kick, dt_drift,
                       dt_drift != 0.0f ? 1 : 0);
    return hipGetLastError();
}

}  // namespace mibh

// --------------------------------------------------------------------------
// Block time steps (the paper's Results and Discussion sections: the walk
// visits only the particles that are due, the tree is refitted between
// rebuilds).  The paper names no scheme; the one used here:
//   * particle i steps with dt_max / 2^r_i, r_i in 0..R, the smallest r with
//     dt_max / 2^r <= eta sqrt(eps / |a_i|) (r = 0 for a = 0), taken in
//     float64 as the smallest r with 16^r >= dt_max^4 |a|^2 / (eta^4 eps^2);
//   * the global clock ticks in dt_max / 2^R; every particle drifts every
//     tick; particle i is due at tick s iff 2^(R - r_i) divides s, and a due
//     particle gets its closing half kick (old level), a new level (no larger
//     step than the tick's alignment allows) and its opening half kick;
//   * hierarchical kick-drift-kick; each update one fused multiply-add.
// --------------------------------------------------------------------------
namespace mibh {

namespace {

__device__ __forceinline__ unsigned block_level(float ax, float ay, float az, double dt_max, double eta, double eps,
                                                int R) {
#pragma clang fp contract(off)
    const double a2 = ((double)ax * (double)ax + (double)ay * (double)ay) + (double)az * (double)az;
    if (!(a2 > 0.0)) return 0u;
    const double q = ((dt_max * dt_max) * (dt_max * dt_max)) * a2 / (((eta * eta) * (eta * eta)) * (eps * eps));
    unsigned r = 0;
    double p = 1.0;
    while ((int)r < R && p < q) {
        p *= 16.0;
        r++;
    }
    return r;
}

// sum over the wave, in every lane
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// smallest level whose steps start at tick s (s > 0), R for s odd
__device__ __forceinline__ unsigned aligned_level(unsigned tick, int R) {
    if (tick == 0) return 0u;
    const int tz = __builtin_ctz(tick);
    return (unsigned)(tz >= R ? 0 : R - tz);
}

__global__ __launch_bounds__(256) void k_block_active(const uint8_t *__restrict__ level, unsigned n, unsigned tick,
                                                      int R, uint8_t *__restrict__ active,
                                                      unsigned long long *__restrict__ nactive) {
    unsigned cnt = 0;
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const bool due = (tick & ((1u << (R - level[i])) - 1u)) == 0u;
        active[i] = due ? 1 : 0;
        cnt += due ? 1u : 0u;
    }
    // one atomic per block: the per-wave sums meet in LDS first
    __shared__ unsigned long long s_part[4];
    const unsigned long long tot = wave_sum(cnt);
    if ((threadIdx.x & 63u) == 0u) s_part[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(nactive, (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]));
}

__global__ __launch_bounds__(256) void k_block_kick(float *__restrict__ vel, const float *__restrict__ acc,
                                                    uint8_t *__restrict__ level, unsigned n, unsigned tick, int R,
                                                    float half_max, int flags, double dt_max, double eta,
                                                    double eps) {
    const unsigned rmin = aligned_level(tick, R);
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        unsigned r = level[i];
        if ((tick & ((1u << (R - r)) - 1u)) != 0u) continue;  // not due
        const float ax = acc[3 * (size_t)i], ay = acc[3 * (size_t)i + 1], az = acc[3 * (size_t)i + 2];
        float vx = vel[3 * (size_t)i], vy = vel[3 * (size_t)i + 1], vz = vel[3 * (size_t)i + 2];
        if (flags & BLOCK_CLOSE) {
            const float h = ldexpf(half_max, -(int)r);
            vx = fmaf(h, ax, vx);
            vy = fmaf(h, ay, vy);
            vz = fmaf(h, az, vz);
        }
        if (flags & BLOCK_LEVEL) {
            r = max(block_level(ax, ay, az, dt_max, eta, eps, R), rmin);
            level[i] = (uint8_t)r;
        }
        if (flags & BLOCK_OPEN) {
            const float h = ldexpf(half_max, -(int)r);
            vx = fmaf(h, ax, vx);
            vy = fmaf(h, ay, vy);
            vz = fmaf(h, az, vz);
        }
        vel[3 * (size_t)i] = vx;
        vel[3 * (size_t)i + 1] = vy;
        vel[3 * (size_t)i + 2] = vz;
    }
}

// Work of the groups just walked (queue entries [0, *qlen)), work =
// count * (1 + n_pc + n_pp): a group's first walk after a build stores its
// reference; later walks add (now, reference) to the sums.  After a build or
// refit with a flagged condition the walk and its queue were skipped (the
// queue and its length are stale), so this kernel skips too.
__global__ __launch_bounds__(256) void k_rebuild_check(const Header *__restrict__ hdr,
                                                       const uint32_t *__restrict__ order,
                                                       const uint32_t *__restrict__ qlen,
                                                       const uint2 *__restrict__ groups,
                                                       const uint2 *__restrict__ counts,
                                                       uint32_t *__restrict__ gref,
                                                       unsigned long long *__restrict__ sums) {
    if (hdr->flags & (FLAG_NONFINITE | FLAG_NEGMASS | FLAG_CELLCAP)) return;
    const unsigned nq = min(*qlen, hdr->ngroups);
    unsigned long long now_sum = 0, ref_sum = 0;
    for (unsigned j = blockIdx.x * 256u + threadIdx.x; j < nq; j += gridDim.x * 256u) {
        const unsigned g = order[j];
        const uint2 c = counts[g];
        const unsigned now = (groups[g].y & 255u) * (1u + c.x + c.y);
        const unsigned ref = gref[g];
        if (ref == 0u) {
            gref[g] = now;
        } else {
            now_sum += now;
            ref_sum += ref;
        }
    }
    // one pair of atomics per block: the per-wave sums meet in LDS first
    __shared__ unsigned long long s_part[2][4];
    now_sum = wave_sum(now_sum);
    ref_sum = wave_sum(ref_sum);
    if ((threadIdx.x & 63u) == 0u) {
        s_part[0][threadIdx.x >> 6] = now_sum;
        s_part[1][threadIdx.x >> 6] = ref_sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&sums[0], (s_part[0][0] + s_part[0][1]) + (s_part[0][2] + s_part[0][3]));
        atomicAdd(&sums[1], (s_part[1][0] + s_part[1][1]) + (s_part[1][2] + s_part[1][3]));
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, unsigned n, uint32_t v) {
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) p[i] = v;
}

}  // namespace

hipError_t launch_block_active(const uint8_t *level, unsigned n, unsigned tick, int R, uint8_t *active,
                               unsigned long long *nactive, hipStream_t s) {
    const unsigned grid = min((n + 255u) / 256u, 1024u);
    hipLaunchKernelGGL(k_block_active, dim3(grid), dim3(256), 0, s, level, n, tick, R, active, nactive);
    return hipGetLastError();
}

hipError_t launch_block_kick(float *vel, const float *acc, uint8_t *level, unsigned n, unsigned tick, int R,
                             float dt_max, int flags, double eta, double eps, hipStream_t s) {
    const unsigned grid = min((n + 255u) / 256u, 4096u);
    hipLaunchKernelGGL(k_block_kick, dim3(grid), dim3(256), 0, s, vel, acc, level, n, tick, R, 0.5f * dt_max, flags,
                       (double)dt_max, eta, eps);
    return hipGetLastError();
}

hipError_t launch_rebuild_check(const Buffers &b, const uint32_t *qlen, unsigned long long *sums, hipStream_t s) {
    hipLaunchKernelGGL(k_rebuild_check, dim3(256), dim3(256), 0, s, b.hdr, b.qorder, qlen, b.groups, b.gcounts,
                       b.gref, sums);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, unsigned n, uint32_t v, hipStream_t s) {
    const unsigned grid = max(1u, min((n + 255u) / 256u, 4096u));
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace mibh
