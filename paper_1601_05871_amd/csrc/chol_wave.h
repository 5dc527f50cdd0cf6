// Wavefront-level building blocks of the diagonal-block factorization
// (the CHOL step of Fig. "dense-chol", unblocked, b = 1 inside the block):
// lane broadcasts, a full-precision reciprocal and the column-per-lane
// factorization of an S x S block held in registers.
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

// Unguarded S x S wave factorization (column-per-lane registers, as in
// chol_wave_regs with w = S) without branches: a pivot that is not > 0 is
// recorded and the remaining arithmetic runs on (meaningless) values, so the
// whole sequence is one basic block and the next pivot's square root and
// reciprocal overlap the previous pivot's row updates.  Returns the first bad
// local pivot (1-based) or 0; *rinv = 1 / U(lane, lane).
// FENCE: keep pivots from being interleaved by the instruction scheduler
// (bounds the number of broadcast values in flight, for large S).
template <typename T, int S, bool FENCE = false>
__device__ __forceinline__ int chol_wave_full(T (&a)[S], int lane, T *rinv) {
    int bad = 0;
    T myinv = T(1);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const T djj = rdlane(a[j], j);
        bad = (bad == 0 && !(djj > T(0))) ? j + 1 : bad;
        const T sq = sqrt(djj);
        const T inv = recip(sq);
        myinv = (lane == j) ? inv : myinv;
        a[j] = (lane == j) ? sq : (lane > j ? a[j] * inv : a[j]);
#pragma unroll
        for (int i = j + 1; i < S; ++i) {
            const T uji = rdlane(a[j], i);
            a[i] = a[i] - uji * a[j];
        }
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
    }
    *rinv = myinv;
    return bad;
}

}  // namespace flame
