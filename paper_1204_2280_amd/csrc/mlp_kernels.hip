// Learned work estimator for the group walk: a multilayer perceptron
// 8 -> 64 -> 64 -> 1 (ReLU) mapping a group's geometry to
// log2(1 + n_pc + n_pp), the length of its interaction lists.  Weights are
// stored in float16, arithmetic accumulates in float32.  Training kernels
// (forward, backward, Adam) run on the GPU; the backward pass is
// deterministic (per-block outer products summed in a fixed order, then a
// fixed-order sum over blocks).  The prediction orders the walk's group
// queue, heaviest predicted work first.
#include "mibh_device.h"

#include <hip/hip_fp16.h>

namespace mibh {

// parameter layout: W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int OFF_W1 = 0, OFF_B1 = MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H,
              OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H;
static_assert(OFF_B3 + 1 == MLP_NPARAM, "parameter layout");

// --------------------------------------------------------------------------
// Features of each group (one thread per group): particle count, bounding
// extent and distance to the system's centre of mass (in root-cube units),
// local density relative to the system's mean, theta, group level, system
// size.  All are O(1) by construction so that no data-dependent
// normalisation is needed.  The group's box is gathered 8 particles per round
// with the indices clamped to the group's last particle (a repeated particle
// leaves a minimum or maximum unchanged), so each round issues its 8 loads at
// once and a group of n particles takes ceil(n / 8) round trips.
// --------------------------------------------------------------------------

constexpr unsigned FEAT_BATCH = 8;

__global__ __launch_bounds__(256) void k_features(const Header *__restrict__ hdr, const SysCube *__restrict__ cube,
                                                  const uint2 *__restrict__ groups, const uint4 *__restrict__ topo,
                                                  const float4 *__restrict__ spos, const double *__restrict__ mp,
                                                  float theta, float *__restrict__ feat) {
    const unsigned ng = hdr->ngroups;
    for (unsigned g = blockIdx.x * 256u + threadIdx.x; g < ng; g += gridDim.x * 256u) {
        const uint2 gr = groups[g];
        const unsigned gf = gr.x, gn = gr.y & 255u, glev = (gr.y >> 8) & 255u, sys = gr.y >> 16;
        float3 bmin = make_float3(INFINITY, INFINITY, INFINITY), bmax = make_float3(-INFINITY, -INFINITY, -INFINITY);
        for (unsigned j0 = 0; j0 < gn; j0 += FEAT_BATCH) {
            float4 p[FEAT_BATCH];
#pragma unroll
            for (unsigned u = 0; u < FEAT_BATCH; u++) p[u] = spos[gf + min(j0 + u, gn - 1u)];
#pragma unroll
            for (unsigned u = 0; u < FEAT_BATCH; u++) {
                bmin.x = fminf(bmin.x, p[u].x); bmin.y = fminf(bmin.y, p[u].y); bmin.z = fminf(bmin.z, p[u].z);
                bmax.x = fmaxf(bmax.x, p[u].x); bmax.y = fmaxf(bmax.y, p[u].y); bmax.z = fmaxf(bmax.z, p[u].z);
            }
        }
        const float L = ldexpf(1.0f, cube[sys].k);
        const float ext = fmaxf(fmaxf(bmax.x - bmin.x, bmax.y - bmin.y), bmax.z - bmin.z);
        const double *root = mp + 10 * (size_t)sys;  // level-0 cell of system sys
        const float cx = 0.5f * (bmin.x + bmax.x) - (float)root[1];
        const float cy = 0.5f * (bmin.y + bmax.y) - (float)root[2];
        const float cz = 0.5f * (bmin.z + bmax.z) - (float)root[3];
        const float dist = sqrtf(cx * cx + cy * cy + cz * cz);
        const float nsys_particles = (float)topo[sys].y;
        const float e = fmaxf(ext, L * 9.5367431640625e-07f) / L;  // at least one finest cell
        float *f = feat + (size_t)g * MLP_IN;
        f[0] = log2f((float)gn) / 6.0f;
        f[1] = log2f(ext / L + 5.9604645e-08f) / 24.0f;
        f[2] = log2f(dist / L + 5.9604645e-08f) / 24.0f;
        f[3] = log2f(((float)gn / nsys_particles) / (e * e * e)) / 32.0f;
        f[4] = theta;
        f[5] = (float)glev / 20.0f;
        f[6] = log2f(nsys_particles) / 24.0f;
        f[7] = log2f(theta);
    }
}

// --------------------------------------------------------------------------
// Forward pass, one row per thread; weights converted once into LDS and read
// back as wave-uniform (broadcast) loads.  The hidden layers run as outer
// products: hidden unit j of the first layer is computed on its own, then
// added into the 64 second-layer sums, whose weights W2[.][j] sit transposed
// in LDS (16 broadcast loads of 4).  Each sum keeps the order of its dot
// product (bias first, then j = 0..63), so the predictions equal those of
// plain dot products bit for bit.  A fully unrolled first layer made the
// compiler keep 488 registers (one wave per SIMD); this form takes 221 (two
// waves per SIMD; bounds asking for three or four waves make it spill).
// --------------------------------------------------------------------------

__device__ __forceinline__ void load_weights(const __half *__restrict__ w16, float *s_w) {
    for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) s_w[i] = __half2float(w16[i]);
    __syncthreads();
}

// LDS image for the forward pass: W1, b1 as stored, W2 transposed, b2, w3, b3.
static_assert(OFF_W2 % 4 == 0, "float4 reads of the transposed second layer");
constexpr int FWD_W2T = OFF_W2;

__device__ __forceinline__ void load_weights_fwd(const __half *__restrict__ w16, float *s_w) {
    for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) {
        int d = i;
        if (i >= OFF_W2 && i < OFF_B2) {  // W2[r][c] -> W2T[c][r]
            const int r = (i - OFF_W2) / MLP_H, c = (i - OFF_W2) % MLP_H;
            d = FWD_W2T + c * MLP_H + r;
        }
        s_w[d] = __half2float(w16[i]);
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_fwd(const __half *__restrict__ w16, const float *__restrict__ x,
                                                 unsigned rows, const Header *__restrict__ hdr,
                                                 float *__restrict__ y) {
    __shared__ __align__(16) float s_w[MLP_NPARAM];
    load_weights_fwd(w16, s_w);
    const unsigned nrows = hdr ? hdr->ngroups : rows;
    for (unsigned r = blockIdx.x * 256u + threadIdx.x; r < nrows; r += gridDim.x * 256u) {
        float xi[MLP_IN], h2[MLP_H];
#pragma unroll
        for (int k = 0; k < MLP_IN; k++) xi[k] = x[(size_t)r * MLP_IN + k];
#pragma unroll
        for (int i = 0; i < MLP_H; i++) h2[i] = s_w[OFF_B2 + i];
#pragma nounroll
        for (int j = 0; j < MLP_H; j++) {
            float a = s_w[OFF_B1 + j];
#pragma unroll
            for (int k = 0; k < MLP_IN; k++) a = fmaf(s_w[OFF_W1 + j * MLP_IN + k], xi[k], a);
            const float h1j = fmaxf(a, 0.0f);
            const float4 *col = reinterpret_cast<const float4 *>(s_w + FWD_W2T + j * MLP_H);
#pragma unroll
            for (int q = 0; q < MLP_H / 4; q++) {
                const float4 w = col[q];
                h2[4 * q] = fmaf(w.x, h1j, h2[4 * q]);
                h2[4 * q + 1] = fmaf(w.y, h1j, h2[4 * q + 1]);
                h2[4 * q + 2] = fmaf(w.z, h1j, h2[4 * q + 2]);
                h2[4 * q + 3] = fmaf(w.w, h1j, h2[4 * q + 3]);
            }
        }
        float out = s_w[OFF_B3];
#pragma unroll
        for (int i = 0; i < MLP_H; i++) out = fmaf(s_w[OFF_W3 + i], fmaxf(h2[i], 0.0f), out);
        y[r] = out;
    }
}

// --------------------------------------------------------------------------
// Backward pass of the mean squared error over a batch of sampled rows,
// 64 samples per block: every sample's activations and deltas go to LDS, then
// thread t sums row t of each weight gradient over the 64 samples in sample
// order.  Partial gradients per block are summed over blocks in block order.
// --------------------------------------------------------------------------

constexpr int GS = 64;  // samples per block

__global__ __launch_bounds__(GS) void k_mlp_grad(const __half *__restrict__ w16, const float *__restrict__ x,
                                                 const float *__restrict__ target, const int *__restrict__ idx,
                                                 unsigned batch, float *__restrict__ partial,
                                                 float *__restrict__ loss_part) {
    __shared__ float s_w[MLP_NPARAM];
    __shared__ float s_x[GS][MLP_IN];
    __shared__ float s_h1[GS][MLP_H + 1];
    __shared__ float s_h2[GS][MLP_H + 1];
    __shared__ float s_d2[GS][MLP_H + 1];
    __shared__ float s_d1[GS][MLP_H + 1];
    __shared__ float s_dy[GS], s_e2[GS];
    load_weights(w16, s_w);
    const unsigned t = threadIdx.x;
    const unsigned s = blockIdx.x * GS + t;
    const bool valid = s < batch;
    const int row = valid ? idx[s] : 0;
    float xi[MLP_IN];
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) {
        xi[k] = valid ? x[(size_t)row * MLP_IN + k] : 0.0f;
        s_x[t][k] = xi[k];
    }
    // forward, keeping activations
    for (int i = 0; i < MLP_H; i++) {
        float a = s_w[OFF_B1 + i];
        for (int k = 0; k < MLP_IN; k++) a = fmaf(s_w[OFF_W1 + i * MLP_IN + k], xi[k], a);
        s_h1[t][i] = fmaxf(a, 0.0f);
    }
    float y = s_w[OFF_B3];
    for (int i = 0; i < MLP_H; i++) {
        float a = s_w[OFF_B2 + i];
        for (int j = 0; j < MLP_H; j++) a = fmaf(s_w[OFF_W2 + i * MLP_H + j], s_h1[t][j], a);
        const float h = fmaxf(a, 0.0f);
        s_h2[t][i] = h;
        y = fmaf(s_w[OFF_W3 + i], h, y);
    }
    const float err = valid ? y - target[row] : 0.0f;
    const float dy = 2.0f * err / (float)batch;
    s_dy[t] = dy;
    s_e2[t] = err * err;
    for (int i = 0; i < MLP_H; i++) s_d2[t][i] = s_h2[t][i] > 0.0f ? dy * s_w[OFF_W3 + i] : 0.0f;
    for (int j = 0; j < MLP_H; j++) {
        float a = 0.0f;
        for (int i = 0; i < MLP_H; i++) a = fmaf(s_w[OFF_W2 + i * MLP_H + j], s_d2[t][i], a);
        s_d1[t][j] = s_h1[t][j] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    // weight gradients, row t, summed over the block's samples in order
    float *out = partial + (size_t)blockIdx.x * MLP_NPARAM;
    for (int j = 0; j < MLP_H; j++) {
        float a = 0.0f;
        for (int q = 0; q < GS; q++) a = fmaf(s_d2[q][t], s_h1[q][j], a);
        out[OFF_W2 + t * MLP_H + j] = a;
    }
    for (int k = 0; k < MLP_IN; k++) {
        float a = 0.0f;
        for (int q = 0; q < GS; q++) a = fmaf(s_d1[q][t], s_x[q][k], a);
        out[OFF_W1 + t * MLP_IN + k] = a;
    }
    float b1 = 0.0f, b2 = 0.0f, w3 = 0.0f;
    for (int q = 0; q < GS; q++) {
        b1 += s_d1[q][t];
        b2 += s_d2[q][t];
        w3 = fmaf(s_dy[q], s_h2[q][t], w3);
    }
    out[OFF_B1 + t] = b1;
    out[OFF_B2 + t] = b2;
    out[OFF_W3 + t] = w3;
    if (t == 0) {
        float b3 = 0.0f, l = 0.0f;
        for (int q = 0; q < GS; q++) {
            b3 += s_dy[q];
            l += s_e2[q];
        }
        out[OFF_B3] = b3;
        loss_part[blockIdx.x] = l;
    }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partial, unsigned nblk,
                                                    const float *__restrict__ loss_part, unsigned batch,
                                                    float *__restrict__ grad, float *__restrict__ loss) {
    for (unsigned p = blockIdx.x * 256u + threadIdx.x; p < (unsigned)MLP_NPARAM; p += gridDim.x * 256u) {
        float a = 0.0f;
        for (unsigned b = 0; b < nblk; b++) a += partial[(size_t)b * MLP_NPARAM + p];
        grad[p] = a;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        float l = 0.0f;
        for (unsigned b = 0; b < nblk; b++) l += loss_part[b];
        *loss = l / (float)batch;
    }
}

// Adam (Kingma & Ba 2015) on float32 master weights; float16 copies for the kernels.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w32, __half *__restrict__ w16,
                                              const float *__restrict__ grad, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float beta1, float beta2,
                                              float eps, float corr1, float corr2) {
    for (unsigned p = blockIdx.x * 256u + threadIdx.x; p < (unsigned)MLP_NPARAM; p += gridDim.x * 256u) {
        const float g = grad[p];
        const float mp = beta1 * m[p] + (1.0f - beta1) * g;
        const float vp = beta2 * v[p] + (1.0f - beta2) * g * g;
        m[p] = mp;
        v[p] = vp;
        const float w = w32[p] - lr * (mp / corr1) / (sqrtf(vp / corr2) + eps);
        w32[p] = w;
        w16[p] = __float2half(w);
    }
}

hipError_t launch_features(const Buffers &b, float theta, float *feat, hipStream_t s) {
    const unsigned grid = min((b.n_max + 255u) / 256u, 2048u);
    hipLaunchKernelGGL(k_features, dim3(grid), dim3(256), 0, s, b.hdr, b.cube, b.groups, b.topo, b.spos, b.mp, theta,
                       feat);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const void *w16, const float *x, unsigned rows, const Header *hdr, float *y,
                              hipStream_t s) {
    const unsigned grid = min(max((rows + 255u) / 256u, 1u), 1024u);
    hipLaunchKernelGGL(k_mlp_fwd, dim3(hdr ? 1024u : grid), dim3(256), 0, s, (const __half *)w16, x, rows, hdr, y);
    return hipGetLastError();
}

size_t mlp_scratch_bytes(unsigned batch) {
    const size_t nblk = (batch + GS - 1) / GS;
    return nblk * MLP_NPARAM * sizeof(float) + nblk * sizeof(float) + 256;
}

hipError_t launch_mlp_grad(const void *w16, const float *x, const float *target, const int *idx, unsigned batch,
                           float *grad, float *loss, void *scratch, hipStream_t s) {
    const unsigned nblk = (batch + GS - 1) / GS;
    float *partial = (float *)scratch;
    float *loss_part = partial + (size_t)nblk * MLP_NPARAM;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(GS), 0, s, (const __half *)w16, x, target, idx, batch, partial,
                       loss_part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, partial, nblk, loss_part,
                       batch, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *w32, void *w16, const float *grad, float *m, float *v, int step, float lr,
                       float beta1, float beta2, float eps, hipStream_t s) {
    const float corr1 = 1.0f - powf(beta1, (float)step), corr2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, w32, (__half *)w16, grad, m, v, lr,
                       beta1, beta2, eps, corr1, corr2);
    return hipGetLastError();
}

}  // namespace mibh
