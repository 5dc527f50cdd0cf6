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

// Unguarded S x S wave factorization: lane c holds column c (a[i] = A(i, c)
// for i <= c; the entries below the diagonal may hold anything: they are never
// read into an entry on or above it), branch-free, one basic block.
//
// The elimination runs square-root free: pivot j subtracts
// A(j, i) A(j, c) / d_j from A(i, c) (d_j the current A(j, j)), so the
// dependent chain from one pivot to the next holds a reciprocal and a few
// multiply-adds, not a square root.  The row scaling U(j, c) = A(j, c) / s_j,
// s_j = sqrt(d_j), is applied once at the end, for all rows at once.  No
// per-row lane masks are kept alive across pivots (they would not fit in
// scalar registers).  A pivot that is not > 0 is recorded and the arithmetic
// runs on (meaningless) values.  Returns the first bad local pivot (1-based)
// or 0; *rinv = 1 / U(lane, lane).
// FENCE: keep pivots from being interleaved by the instruction scheduler
// (bounds the number of broadcast values in flight, for large S).
// Lane I of this lane's row of 16 (DPP row_newbcast: a register move, no
// scalar round trip).
template <int I>
__device__ __forceinline__ double row_bcast(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + I, 0xF, 0xF, false);
}
template <int I>
__device__ __forceinline__ float row_bcast(float v) {
    return __builtin_amdgcn_update_dpp(0.0f, v, 0x150 + I, 0xF, 0xF, false);
}

// Pivot J of the square-root-free elimination in row-broadcast form, then
// the next pivots (compile-time recursion: DPP lane selects are immediates).
template <int J, int I, int S, typename T>
__device__ __forceinline__ void row_update(T (&a)[S], T t) {
    if constexpr (I < S) {
        a[I] = a[I] - row_bcast<I>(a[J]) * t;
        row_update<J, I + 1, S>(a, t);
    }
}
template <int J, int S, typename T>
__device__ __forceinline__ void pivots_dpp(T (&a)[S], int lane, int &bad, T &dme) {
    if constexpr (J < S) {
        const T d = row_bcast<J>(a[J]);
        bad = (bad == 0 && !(d > T(0))) ? J + 1 : bad;
        dme = (lane == J) ? d : dme;
        const T t = a[J] * recip(d);
        row_update<J, J + 1, S>(a, t);
        pivots_dpp<J + 1, S>(a, lane, bad, dme);
    }
}
template <int J, int S, typename T>
__device__ __forceinline__ void scale_dpp(T (&a)[S], int lane, T sme, T ime) {
    if constexpr (J < S) {
        // the broadcast runs with every lane active: inside a branch (as an
        // operand of ?:) the source lane J would be masked off and read as 0
        const T inv_j = row_bcast<J>(ime);
        const T scaled = a[J] * inv_j;
        a[J] = (lane == J) ? sme : scaled;
        scale_dpp<J + 1, S>(a, lane, sme, ime);
    }
}

// The same factorization for S <= 16 with the broadcasts of row j done by DPP
// row_newbcast inside each row of 16 lanes (lanes 0..S-1 hold the block; the
// other rows compute on their own, discarded, values).  The caller reads the
// result of lanes 0..S-1 only.
template <typename T, int S>
__device__ __forceinline__ int chol_row16(T (&a)[S], int lane, T *rinv) {
    static_assert(S <= 16, "one DPP row");
    asm volatile("" : "+v"(lane));
    int bad = 0;
    T dme = T(1);
    pivots_dpp<0, S>(a, lane, bad, dme);
    const T sme = sqrt(dme);
    const T ime = recip(sme);
    scale_dpp<0, S>(a, lane, sme, ime);
    *rinv = ime;
    return bad;
}

template <typename T, int S, bool FENCE = false>
__device__ __forceinline__ int chol_wave_full(T (&a)[S], int lane, T *rinv) {
    // the lane compares below are recomputed at each use: hoisted out of a
    // caller's loop they would be 2 S scalar registers kept alive (and spilled)
    asm volatile("" : "+v"(lane));
    int bad = 0;
    T dme = T(1);  // this lane's pivot d_lane
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const T d = rdlane(a[j], j);
        bad = (bad == 0 && !(d > T(0))) ? j + 1 : bad;
        dme = (lane == j) ? d : dme;
        const T t = a[j] * recip(d);  // A(j, c) / d_j (lanes c <= j: unused)
#pragma unroll
        for (int i = j + 1; i < S; ++i) a[i] = a[i] - rdlane(a[j], i) * t;
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
    }
    const T sme = sqrt(dme);
    const T ime = recip(sme);
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const T inv_j = rdlane(ime, j);
        a[j] = (lane == j) ? sme : a[j] * inv_j;
    }
    *rinv = ime;
    return bad;
}

}  // namespace flame
