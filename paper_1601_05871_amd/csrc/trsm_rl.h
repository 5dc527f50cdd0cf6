#pragma once

#include <hip/hip_runtime.h>

namespace flame {

// Matrix-core panel solve X := U^{-T} X (TRSM step of Fig. "dense-chol") for
// b <= 16 NB, as device functions shared by the panel kernel and the batched
// kernel.
//
// The solve blocked by 16 rows (U padded with the identity to a multiple of
// 16).  Each workgroup first forms the inverses D_s = U_ss^{-1} of the 16 x 16
// diagonal blocks in LDS (16 lanes per block, one lane per column, back
// substitution).  Then each wavefront owns 16 columns of X, keeps all of its
// row blocks in registers and runs the right-looking loop
//   X_s = D_s^T R_s;   R_t -= U(s, t)^T X_s  for t > s
// on matrix cores (FP64 v_mfma_f64_16x16x4f64 or FP32 v_mfma_f32_16x16x4f32),
// fully unrolled over the eight row blocks so that the loads of U are
// independent of the arithmetic and can be issued early.  Placement as in the
// trailing update: FP64 lane (r, g) item v holds row r, column g + 4v of a
// 16 x 16 block; FP32 lane (r, g) item v holds row 4g + v, column r (the two
// MFMAs return their results transposed to each other, so the operands are
// passed in swapped order).
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct TrsmAcc;
template <>
struct TrsmAcc<double> {
    typedef d4v type;
};
template <>
struct TrsmAcc<float> {
    typedef f4v type;
};

// U(i, j) with rows / columns >= b read as the identity
template <typename T>
__device__ __forceinline__ T u_pad(const T *__restrict__ U, int64_t ldu, int b, int i, int j) {
    const T v = U[(int64_t)min(i, b - 1) + (int64_t)min(j, b - 1) * ldu];
    return (i < b && j < b) ? v : (i == j ? T(1) : T(0));
}

// acc += A B with A[i][k] = a-operand, B[k][j] = b-operand over one k slot;
// rowop / colop: the per-lane operand that indexes the result's rows / columns
// in this precision's placement.
__device__ __forceinline__ d4v mma_rc(double rowop, double colop, d4v acc) {
    // FP64 result D[g + 4v][r] in lane (r, g): pass the column operand first
    return __builtin_amdgcn_mfma_f64_16x16x4f64(colop, rowop, acc, 0, 0, 0);
}
__device__ __forceinline__ f4v mma_rc(float rowop, float colop, f4v acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(rowop, colop, acc, 0, 0, 0);
}

// (1) D_s = U_ss^{-1} for the NB diagonal 16 x 16 blocks into Ds (all threads
// of the workgroup).  The blocks are first copied into Ds with coalesced
// loads (eight per thread, all issued before the LDS stores), then each of
// NB * 16 threads solves one column U_ss D(:, t) = e_t by back substitution
// from LDS into registers, and the columns replace the blocks in Ds.
// Opaque (for callers inside a loop, like the batched kernel): the lane
// indices are hidden from the compiler, so that the addresses and the unit
// vectors are formed at each call, not hoisted out of the caller's loop into
// registers that stay live (and spill) across it.
template <typename T, int NB, bool Opaque = false>
__device__ __forceinline__ void trsm_inverses(int b, const T *__restrict__ U, int64_t ldu, T (*Ds)[16][17]) {
    int tid = threadIdx.x;
    if constexpr (Opaque) asm volatile("" : "+v"(tid));
    constexpr int PER = (NB * 256 + 255) / 256;
    T v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;  // element (i, j) of block sb, i fastest
        const int sb = min(e >> 8, NB - 1), i = e & 15, j = (e >> 4) & 15;
        v[q] = U[(int64_t)min(16 * sb + i, b - 1) + (int64_t)min(16 * sb + j, b - 1) * ldu];
    }
    asm volatile("" ::: "memory");  // the loads stay ahead of the stores below
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + 256 * q;
        const int sb = e >> 8, i = e & 15, j = (e >> 4) & 15;
        if (sb < NB) {
            const int gi = 16 * sb + i, gj = 16 * sb + j;
            Ds[sb][i][j] = (gi < b && gj < b) ? v[q] : (gi == gj ? T(1) : T(0));
        }
    }
    __syncthreads();
    T d[16];
    const int sb = tid >> 4;
    int t = tid & 15;  // column t of D_sb
    if constexpr (Opaque) asm volatile("" : "+v"(t));
    if (sb < NB) {
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            T acc = (i == t) ? T(1) : T(0);
#pragma unroll
            for (int k = i + 1; k < 16; ++k) acc -= Ds[sb][i][k] * d[k];
            d[i] = acc / Ds[sb][i][i];  // rows below the diagonal come out 0
        }
    }
    __syncthreads();
    if (sb < NB) {
#pragma unroll
        for (int i = 0; i < 16; ++i) Ds[sb][i][t] = d[i];
    }
}

// (2) One wavefront solves the 16 columns c0 .. c0 + 15 of X (b x m; columns
// >= m are skipped) with the inverses in Ds; Rt: this wavefront's 16 x 17
// LDS scratch.
template <typename T, int NB, bool Opaque = false>
__device__ __forceinline__ void trsm_cols(int b, int64_t m, const T *__restrict__ U, int64_t ldu,
                                          T *__restrict__ X, int64_t ldx, int64_t c0, T (*Ds)[16][17],
                                          T (*Rt)[17]) {
    typedef typename TrsmAcc<T>::type acc_t;
    constexpr bool F64 = sizeof(T) == 8;
    const int lane = threadIdx.x & 63;
    int r = lane & 15;
    if constexpr (Opaque) asm volatile("" : "+v"(r));
    const int g = lane >> 4;
    const int nblk = (b + 15) >> 4;
    // (2) right-looking solve of this wavefront's 16 columns.  Accumulator
    // item v of lane (r, g) is element (arow(v), acol(v)) of a 16 x 16 block.
    auto arow = [&](int v) { return F64 ? r : 4 * g + v; };
    auto acol = [&](int v) { return F64 ? g + 4 * v : r; };
    int64_t colc[4];
    bool colok[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t col = c0 + acol(v);
        colok[v] = col < m;
        colc[v] = min(col, m - 1);
    }
    // all loads first (clamped addresses, unconditional): the barrier keeps
    // the compiler from sinking each load into the masking select below,
    // which would give one branch and one full memory wait per load
    T xin[NB][4];
#pragma unroll
    for (int t = 0; t < NB; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) xin[t][v] = X[(int64_t)min(16 * t + arow(v), b - 1) + colc[v] * ldx];
    asm volatile("" ::: "memory");
    acc_t acc[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * t + arow(v);
            acc[t][v] = (row < b && colok[v]) ? xin[t][v] : T(0);
        }
    }
    // U(s, t) operands of row block s (all t > s), loaded one row block ahead
    // of their use: the barrier keeps each set of loads at its issue point,
    // so their latency overlaps the previous block's products
    T un[NB][4];
#pragma unroll
    for (int t = 1; t < NB; ++t)
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) un[t][t4] = u_pad(U, ldu, b, 4 * g + t4, 16 * t + r);
#pragma unroll
    for (int s = 0; s < NB; ++s) {
        T uc[NB][4];
#pragma unroll
        for (int t = s + 1; t < NB; ++t)
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) uc[t][t4] = un[t][t4];
        if (s + 1 < NB) {
#pragma unroll
            for (int t = s + 2; t < NB; ++t)
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) un[t][t4] = u_pad(U, ldu, b, 16 * (s + 1) + 4 * g + t4, 16 * t + r);
        }
        asm volatile("" ::: "memory");
        if (s < nblk) {
            // X_s = D_s^T R_s: R_s through LDS into operand layout
#pragma unroll
            for (int v = 0; v < 4; ++v) Rt[arow(v)][acol(v)] = acc[s][v];
            acc_t xs = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                const int k = 4 * g + t4;  // both operands: k slot (g, t4)
                xs = mma_rc(Ds[s][k][r], Rt[k][r], xs);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Rt[arow(v)][acol(v)] = -xs[v];
                if (16 * s + arow(v) < b && colok[v]) X[(int64_t)(16 * s + arow(v)) + colc[v] * ldx] = xs[v];
            }
            // R_t -= U(s-rows, t-cols)^T X_s
#pragma unroll
            for (int t = s + 1; t < NB; ++t) {
                if (t < nblk) {
#pragma unroll
                    for (int t4 = 0; t4 < 4; ++t4) {
                        const int k = 4 * g + t4;
                        acc[t] = mma_rc(uc[t][t4], Rt[k][r], acc[t]);
                    }
                }
            }
        }
    }
}

}  // namespace flame
