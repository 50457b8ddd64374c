// mlp.hip -- training and scoring kernels of the learned class selector (gfx950).
//
// The selector is a 19 -> 64 (ReLU) -> 16 network over block features (see
// kernels_common.h). Training minimises the mean cross-entropy between softmax(scores) and
// the class exhaustive search picks, with Adam. Gradients are reduced deterministically:
// every workgroup sums the contributions of its samples in a fixed order into its own
// partial gradient, and a second launch adds the partials in workgroup order.
#include "kernels_common.h"

namespace pcomp {

constexpr uint32_t kChunk = 64;  // samples staged in LDS at once (one wavefront's)

// Scores of n samples, in the selector's exact order of operations.
__global__ __launch_bounds__(kThreads) void mlp_scores_kernel(const float *__restrict__ prm,
                                                              const float *__restrict__ X, uint64_t n,
                                                              float *__restrict__ S) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    float x[kMlpIn], s[kMlpOut];
#pragma unroll
    for (int q = 0; q < kMlpIn; q++) x[q] = X[kMlpIn * i + q];
    mlp_scores([&](int k) { return prm[k]; }, x, s);
#pragma unroll
    for (int k = 0; k < kMlpOut; k++) S[kMlpOut * i + k] = s[k];
}

// Per-workgroup partial loss sum and gradient of kThreads samples (one per thread).
// part: [gridDim.x][kMlpParams + 1] floats, the last one the loss sum.
__global__ __launch_bounds__(kThreads) void mlp_grad_partial_kernel(const float *__restrict__ prm,
                                                                    const float *__restrict__ X,
                                                                    const uint8_t *__restrict__ Y, uint64_t n,
                                                                    float inv_n, float *__restrict__ part) {
    __shared__ float s_x[kChunk][kMlpIn + 1];
    __shared__ float s_h[kChunk][kMlpHid + 1];
    __shared__ float s_da[kChunk][kMlpHid + 1];
    __shared__ float s_ds[kChunk][kMlpOut + 1];
    __shared__ float s_loss[kThreads];
    const uint32_t tid = threadIdx.x;
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + tid;
    const bool live = i < n;

    // forward and backward of this thread's sample, down to the hidden pre-activations
    float x[kMlpIn], h[kMlpHid], s[kMlpOut];
#pragma unroll
    for (int q = 0; q < kMlpIn; q++) x[q] = live ? X[kMlpIn * i + q] : 0.0f;
#pragma unroll
    for (int k = 0; k < kMlpOut; k++) s[k] = prm[kMlpB2 + k];
#pragma unroll
    for (int j = 0; j < kMlpHid; j++) {
        float a = prm[kMlpB1 + j];
#pragma unroll
        for (int q = 0; q < kMlpIn; q++) a = __builtin_fmaf(prm[kMlpW1 + j * kMlpIn + q], x[q], a);
        h[j] = a > 0.0f ? a : 0.0f;
#pragma unroll
        for (int k = 0; k < kMlpOut; k++) s[k] = __builtin_fmaf(prm[kMlpW2 + k * kMlpHid + j], h[j], s[k]);
    }
    const int y = live ? (int)Y[i] : 0;
    float m = s[0];
#pragma unroll
    for (int k = 1; k < kMlpOut; k++) m = s[k] > m ? s[k] : m;
    float z = 0.0f, sy = 0.0f;
#pragma unroll
    for (int k = 0; k < kMlpOut; k++) sy = (k == y) ? s[k] - m : sy;
#pragma unroll
    for (int k = 0; k < kMlpOut; k++) {
        s[k] = __expf(s[k] - m);
        z += s[k];
    }
    s_loss[tid] = live ? (__logf(z) - sy) : 0.0f;  // log-sum-exp minus the label's score
    // dL/ds_k = (p_k - [k == y]) / n
    const float rz = 1.0f / z;
#pragma unroll
    for (int k = 0; k < kMlpOut; k++) s[k] = live ? (s[k] * rz - (k == y ? 1.0f : 0.0f)) * inv_n : 0.0f;

    // accumulate the parameter gradients over the workgroup's samples, kChunk at a time;
    // thread tid owns parameters tid, tid + kThreads, ...
    constexpr int kPer = (kMlpParams + kThreads - 1) / kThreads;
    float acc[kPer];
#pragma unroll
    for (int r = 0; r < kPer; r++) acc[r] = 0.0f;
    for (uint32_t c = 0; c < kThreads / kChunk; c++) {
        if (tid / kChunk == c) {
            const uint32_t r = tid % kChunk;
#pragma unroll
            for (int q = 0; q < kMlpIn; q++) s_x[r][q] = x[q];
#pragma unroll
            for (int k = 0; k < kMlpOut; k++) s_ds[r][k] = s[k];
#pragma unroll
            for (int j = 0; j < kMlpHid; j++) {
                // dL/da_j = (sum_k dL/ds_k W2[k][j]) for an active unit, else 0
                float g = 0.0f;
#pragma unroll
                for (int k = 0; k < kMlpOut; k++) g = __builtin_fmaf(s[k], prm[kMlpW2 + k * kMlpHid + j], g);
                s_h[r][j] = h[j];
                s_da[r][j] = h[j] > 0.0f ? g : 0.0f;
            }
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < kPer; rr++) {
            const int p = (int)tid + rr * (int)kThreads;
            if (p >= kMlpParams) break;
            float a = acc[rr];
            if (p < kMlpB1) {  // W1[j][q]: sum of da_j x_q
                const int j = p / kMlpIn, q = p % kMlpIn;
                for (uint32_t r = 0; r < kChunk; r++) a = __builtin_fmaf(s_da[r][j], s_x[r][q], a);
            } else if (p < kMlpW2) {  // b1[j]
                const int j = p - kMlpB1;
                for (uint32_t r = 0; r < kChunk; r++) a += s_da[r][j];
            } else if (p < kMlpB2) {  // W2[k][j]: sum of ds_k h_j
                const int k = (p - kMlpW2) / kMlpHid, j = (p - kMlpW2) % kMlpHid;
                for (uint32_t r = 0; r < kChunk; r++) a = __builtin_fmaf(s_ds[r][k], s_h[r][j], a);
            } else {  // b2[k]
                const int k = p - kMlpB2;
                for (uint32_t r = 0; r < kChunk; r++) a += s_ds[r][k];
            }
            acc[rr] = a;
        }
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.x * (kMlpParams + 1);
#pragma unroll
    for (int rr = 0; rr < kPer; rr++) {
        const int p = (int)tid + rr * (int)kThreads;
        if (p < kMlpParams) out[p] = acc[rr];
    }
    if (tid == 0) {
        float l = 0.0f;
        for (uint32_t t = 0; t < kThreads; t++) l += s_loss[t];
        out[kMlpParams] = l;
    }
}

// grad[p] = sum over workgroups (in order) of the partials; loss = their loss sums / n.
__global__ __launch_bounds__(kThreads) void mlp_grad_reduce_kernel(const float *__restrict__ part, uint32_t n_part,
                                                                   float inv_n, float *__restrict__ grad,
                                                                   float *__restrict__ loss) {
    const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
    if (p > (uint32_t)kMlpParams) return;
    float a = 0.0f;
    for (uint32_t w = 0; w < n_part; w++) a += part[(size_t)w * (kMlpParams + 1) + p];
    if (p < (uint32_t)kMlpParams)
        grad[p] = a;
    else if (loss)
        *loss = a * inv_n;
}

// Adam (Kingma & Ba 2015, Algorithm 1) with bias correction; step counts from 1.
__global__ __launch_bounds__(kThreads) void mlp_adam_kernel(float *__restrict__ prm, const float *__restrict__ grad,
                                                            float *__restrict__ m, float *__restrict__ v,
                                                            float lr, float b1, float b2, float eps, float c1,
                                                            float c2) {
    const uint32_t p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= (uint32_t)kMlpParams) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    prm[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

uint64_t mlp_ws_bytes(uint64_t n) {
    const uint64_t parts = (n + kThreads - 1) / kThreads;
    return 4 * (parts ? parts : 1) * (kMlpParams + 1);
}

int launch_mlp_scores(const float *prm, const float *X, uint64_t n, float *S, hipStream_t st) {
    if (n) mlp_scores_kernel<<<(uint32_t)((n + kThreads - 1) / kThreads), kThreads, 0, st>>>(prm, X, n, S);
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

int launch_mlp_loss_grad(const float *prm, const float *X, const uint8_t *Y, uint64_t n, float *grad, float *loss,
                         void *ws, hipStream_t st) {
    const uint32_t parts = (uint32_t)((n + kThreads - 1) / kThreads);
    const float inv_n = 1.0f / (float)n;
    float *part = (float *)ws;
    mlp_grad_partial_kernel<<<parts, kThreads, 0, st>>>(prm, X, Y, n, inv_n, part);
    mlp_grad_reduce_kernel<<<(kMlpParams + 1 + kThreads - 1) / kThreads, kThreads, 0, st>>>(part, parts, inv_n,
                                                                                           grad, loss);
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

int launch_mlp_adam(float *prm, const float *grad, float *m, float *v, uint32_t step, float lr, float b1, float b2,
                    float eps, hipStream_t st) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    mlp_adam_kernel<<<(kMlpParams + kThreads - 1) / kThreads, kThreads, 0, st>>>(prm, grad, m, v, lr, b1, b2, eps,
                                                                                c1, c2);
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

}  // namespace pcomp
