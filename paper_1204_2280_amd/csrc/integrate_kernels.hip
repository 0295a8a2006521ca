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
