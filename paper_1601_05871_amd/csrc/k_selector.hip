// Inference of the learned (variant, block size) selector: a 3-layer FP32
// MLP, features -> 64 -> 64 -> classes, ReLU between layers.  One wavefront
// per feature row, weights staged in LDS (the second and third layers
// transposed so that lane j reads consecutive words), lane j computes hidden
// unit j; every sum runs in a fixed order with fmaf, so the result is
// deterministic.
#include "flame_internal.h"

namespace flame {

constexpr int kF = FLAME_SEL_FEATURES, kH = FLAME_SEL_HIDDEN, kC = FLAME_SEL_CLASSES;

__global__ __launch_bounds__(64) void k_selector(const float *__restrict__ w, const float *__restrict__ feat,
                                                 int64_t count, float *__restrict__ logits) {
    __shared__ float W1[kH][kF];
    __shared__ float b1[kH];
    __shared__ float W2t[kH][kH];  // [k][j] = W2[j][k]
    __shared__ float b2[kH];
    __shared__ float W3t[kH][kC];  // [k][j] = W3[j][k]
    __shared__ float b3[kC];
    __shared__ float h1[kH], h2[kH], x[kF];
    const int j = threadIdx.x;
    const float *pW1 = w, *pb1 = pW1 + kH * kF, *pW2 = pb1 + kH, *pb2 = pW2 + kH * kH, *pW3 = pb2 + kH,
                *pb3 = pW3 + kC * kH;
    for (int e = j; e < kH * kF; e += 64) W1[e / kF][e % kF] = pW1[e];
    for (int e = j; e < kH * kH; e += 64) W2t[e % kH][e / kH] = pW2[e];
    for (int e = j; e < kC * kH; e += 64) W3t[e % kH][e / kH] = pW3[e];
    b1[j] = pb1[j];
    b2[j] = pb2[j];
    if (j < kC) b3[j] = pb3[j];
    __syncthreads();
    for (int64_t row = blockIdx.x; row < count; row += gridDim.x) {
        if (j < kF) x[j] = feat[row * kF + j];
        __syncthreads();
        float a = b1[j];
#pragma unroll
        for (int k = 0; k < kF; ++k) a = fmaf(W1[j][k], x[k], a);
        h1[j] = fmaxf(a, 0.0f);
        __syncthreads();
        a = b2[j];
#pragma unroll 8
        for (int k = 0; k < kH; ++k) a = fmaf(W2t[k][j], h1[k], a);
        h2[j] = fmaxf(a, 0.0f);
        __syncthreads();
        if (j < kC) {
            a = b3[j];
#pragma unroll 8
            for (int k = 0; k < kH; ++k) a = fmaf(W3t[k][j], h2[k], a);
            logits[row * kC + j] = a;
        }
        __syncthreads();
    }
}

int launch_selector(const float *w, const float *feat, int64_t count, float *logits, hipStream_t s) {
    if (count <= 0) return FLAME_OK;
    const unsigned grid = (unsigned)std::min<int64_t>(count, 4096);
    hipLaunchKernelGGL(k_selector, dim3(grid), dim3(64), 0, s, w, feat, count, logits);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
