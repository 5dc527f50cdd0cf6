// Wavefront-level helpers of the diagonal-block factorization (the CHOL step
// of Fig. "dense-chol"): reading one lane's value and a full-precision
// reciprocal.
#pragma once

#include <hip/hip_runtime.h>

namespace flame {

__device__ __forceinline__ double rdlane(double v, int l) {
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
    int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 1 / s to full precision: hardware reciprocal estimate and two Newton steps
// (exact when s is a power of two).
__device__ __forceinline__ double recip(double s) {
    double r = __builtin_amdgcn_rcp(s);
    r = __builtin_fma(__builtin_fma(-s, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-s, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ float recip(float s) {
    float r = __builtin_amdgcn_rcpf(s);
    r = __builtin_fmaf(__builtin_fmaf(-s, r, 1.0f), r, r);
    return r;
}

}  // namespace flame
