// Measurement probes: the matrix-core and HBM rates that the roofline
// fractions of the factorization are read against, measured on the device
// itself (the datasheet peaks are the reference; these show what a plain
// loop reaches on the same chip and clock).
//
//   MFMA probes: every wavefront runs kChains independent accumulation chains
//   of one MFMA instruction (FP64 16x16x4, FP32 16x16x4, BF16 16x16x32) for
//   `iters` rounds of kUnroll steps; operands stay in registers, so the loop
//   is bound by the matrix cores only (the unrolled body keeps the copies of
//   the accumulators between loop iterations, which the compiler inserts at
//   the back edge, to one per kUnroll * kChains instructions).  The accumulators are written out once so the work is
//   not removed.  Four wavefronts per workgroup, wg_per_cu workgroups per CU.
//   Copy probe: a grid-stride copy of `bytes` bytes in 16-byte units (reads
//   and writes `bytes` each).
#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kChains = 4;
constexpr int kUnroll = 16;

template <int KIND>
__global__ __launch_bounds__(256) void k_probe_mfma(int64_t iters, float *__restrict__ sink) {
    const int lane = threadIdx.x & 63;
    if constexpr (KIND == FLAME_PROBE_MFMA_F64) {
        d4 acc[kChains];
        for (int c = 0; c < kChains; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
        double a = 1.0 + lane * 1e-3, b = 1.0 - lane * 1e-3;
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        }
        double s = 0.0;
        for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
        sink[blockIdx.x * 256 + threadIdx.x] = (float)s;
    } else if constexpr (KIND == FLAME_PROBE_MFMA_F32) {
        f4 acc[kChains];
        for (int c = 0; c < kChains; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
        float a = 1.0f + lane * 1e-3f, b = 1.0f - lane * 1e-3f;
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        }
        float s = 0.f;
        for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
        sink[blockIdx.x * 256 + threadIdx.x] = s;
    } else {
        f4 acc[kChains];
        for (int c = 0; c < kChains; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
        bf16x8 a, b;
        for (int e = 0; e < 8; ++e) {
            a[e] = (__bf16)(1.0f + (lane + e) * 1e-3f);
            b[e] = (__bf16)(1.0f - (lane + e) * 1e-3f);
        }
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
        }
        float s = 0.f;
        for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
        sink[blockIdx.x * 256 + threadIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void k_probe_copy(int64_t units, const uint4 *__restrict__ src,
                                                    uint4 *__restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < units; i += stride) dst[i] = src[i];
}

}  // namespace

}  // namespace flame

using namespace flame;

extern "C" int flame_probe(int32_t kind, int64_t work, int32_t wg_per_cu, void *buf, int64_t buf_bytes,
                           int32_t reps, double *rate, void *stream) {
    if (kind < FLAME_PROBE_MFMA_F64 || kind > FLAME_PROBE_COPY) return -1;
    if (work <= 0) return -2;
    if (wg_per_cu < 0 || wg_per_cu > 8) return -3;
    if (buf == nullptr) return -4;
    if (reps <= 0) return -6;
    if (rate == nullptr) return -7;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    FLAME_HIP(hipGetDevice(&dev));
    FLAME_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int grid = cus * (wg_per_cu == 0 ? 2 : wg_per_cu);
    double flops_or_bytes = 0.0;
    if (kind == FLAME_PROBE_COPY) {
        // src = first half of buf, dst = second half; work = bytes copied
        if (buf_bytes < 2 * work || (work % 16) != 0) return -5;
        flops_or_bytes = 2.0 * (double)work;  // read + write
    } else {
        if (buf_bytes < (int64_t)grid * 256 * (int64_t)sizeof(float)) return -5;
        const double per = (kind == FLAME_PROBE_MFMA_BF16) ? 2.0 * 16 * 16 * 32 : 2.0 * 16 * 16 * 4;
        flops_or_bytes = per * kChains * kUnroll * (double)work * (double)grid * 4.0;  // 4 wavefronts per workgroup
    }
    hipEvent_t e0, e1;
    FLAME_HIP(hipEventCreate(&e0));
    FLAME_HIP(hipEventCreate(&e1));
    float best = 0.f;
    for (int r = 0; r <= reps; ++r) {  // the first run is a warm-up
        FLAME_HIP(hipEventRecord(e0, s));
        if (kind == FLAME_PROBE_COPY) {
            const int64_t units = work / 16;
            const uint4 *src = static_cast<const uint4 *>(buf);
            uint4 *dst = reinterpret_cast<uint4 *>(static_cast<char *>(buf) + work);
            hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)grid), dim3(256), 0, s, units, src, dst);
        } else if (kind == FLAME_PROBE_MFMA_F64) {
            hipLaunchKernelGGL(k_probe_mfma<FLAME_PROBE_MFMA_F64>, dim3((unsigned)grid), dim3(256), 0, s, work,
                               static_cast<float *>(buf));
        } else if (kind == FLAME_PROBE_MFMA_F32) {
            hipLaunchKernelGGL(k_probe_mfma<FLAME_PROBE_MFMA_F32>, dim3((unsigned)grid), dim3(256), 0, s, work,
                               static_cast<float *>(buf));
        } else {
            hipLaunchKernelGGL(k_probe_mfma<FLAME_PROBE_MFMA_BF16>, dim3((unsigned)grid), dim3(256), 0, s, work,
                               static_cast<float *>(buf));
        }
        FLAME_CHECK_LAUNCH();
        FLAME_HIP(hipEventRecord(e1, s));
        FLAME_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        FLAME_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r > 0 && (best == 0.f || ms < best)) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // TFLOP/s for the MFMA probes, GB/s for the copy
    *rate = (kind == FLAME_PROBE_COPY) ? flops_or_bytes / (best * 1e-3) / 1e9 : flops_or_bytes / (best * 1e-3) / 1e12;
    return FLAME_OK;
}
