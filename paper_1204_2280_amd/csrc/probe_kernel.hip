// Throughput probe for the walk's roofline (not part of the method).
//
// The walk is bound by float32 vector arithmetic.  The chip's published peak
// counts two flops per lane of a packed fused multiply-add every cycle; this
// build never emits packed float32 instructions, so the rate that ordinary
// fused multiply-adds actually reach on the running chip is measured here:
// every lane adds a * b to 32 independent accumulators per iteration
// (v <- fma(a, b, v), 64 flops), with a and b held in vector registers (the
// accumulate form with only vector-register operands is the fastest float32
// form measured on gfx950; an operand from a scalar register halves the
// rate), and enough waves to fill every SIMD.  The result is a measured
// ceiling that the walk's algorithmic flop rate is set against.
#include <hip/hip_runtime.h>

namespace mibh {

namespace {

constexpr int PROBE_ACC = 32;

__global__ __launch_bounds__(64) void k_fma_probe(float *__restrict__ out, unsigned iters, float a, float b) {
    const unsigned id = blockIdx.x * 64u + threadIdx.x;
    float v[PROBE_ACC];
#pragma unroll
    for (int j = 0; j < PROBE_ACC; j++) v[j] = (float)(id & 255u) * (1.0f / 256.0f) + (float)j * (1.0f / 32.0f);
    float va = a, vb = b;
    asm volatile("" : "+v"(va), "+v"(vb));  // operands in vector registers
    for (unsigned t = 0; t < iters; t++) {
#pragma unroll
        for (int j = 0; j < PROBE_ACC; j++) v[j] = fmaf(va, vb, v[j]);
    }
#pragma unroll
    for (int j = 0; j < PROBE_ACC; j++) out[(size_t)id * PROBE_ACC + j] = v[j];
}

}  // namespace

hipError_t launch_fma_probe(float *out, unsigned blocks, unsigned iters, float a, float b, hipStream_t s) {
    k_fma_probe<<<blocks, 64, 0, s>>>(out, iters, a, b);
    return hipGetLastError();
}

}  // namespace mibh
