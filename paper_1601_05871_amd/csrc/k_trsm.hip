// TRSM step of the loop body (Fig. "dense-chol"): A12 := triu(A11)^{-T} A12,
// i.e. solve U^T X = A12 for X with U = triu(A11) (b x b, b <= 256) and
// A12 b x m.  (The figure prints triu(A11)^{-1}; only the transposed solve
// reproduces A = U^T U.)
//
// Orders above 128 are solved as two row halves joined by a GEMM update.
#include "flame_internal.h"

namespace flame {

// ---- matrix-core panel solve (b <= 128) -------------------------------------
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
constexpr int kTrsmNb = 8;  // row blocks of 16 per kernel: b <= 128

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

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_trsm_rl(int b, int64_t m, const T *__restrict__ U, int64_t ldu,
                                                 T *__restrict__ X, int64_t ldx, const int32_t *__restrict__ info,
                                                 int64_t u_step, int64_t x_step) {
    typedef typename TrsmAcc<T>::type acc_t;
    constexpr bool F64 = sizeof(T) == 8;
    // blockIdx.y selects one of several independent solves (U and X advanced
    // by u_step and x_step elements)
    U += (int64_t)blockIdx.y * u_step;
    X += (int64_t)blockIdx.y * x_step;
    __shared__ T Ds[NB][16][17];  // inverses of the diagonal blocks, [block][k][col]
    __shared__ T Rt[4][16][17];   // per wavefront: one block, [row][col]
    if (info != nullptr && *info != 0) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15;
    const int g = lane >> 4;
    const int nblk = (b + 15) >> 4;
    // (1) inverses of the 16 x 16 diagonal blocks (U read from global memory /
    // L2: no LDS copy, so that the kernel fits beside two trailing-update
    // workgroups on one CU)
    for (int ct = tid; ct < NB * 16; ct += 256) {
        const int sb = ct >> 4, t = ct & 15;  // column t of D_sb: U_ss D(:, t) = e_t
        T v[16];
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            T acc = (i == t) ? T(1) : T(0);
#pragma unroll
            for (int k = i + 1; k < 16; ++k) acc -= u_pad(U, ldu, b, 16 * sb + i, 16 * sb + k) * v[k];
            v[i] = acc / u_pad(U, ldu, b, 16 * sb + i, 16 * sb + i);  // rows below the diagonal come out 0
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Ds[sb][i][t] = v[i];
    }
    __syncthreads();

    // (2) right-looking solve of this wavefront's 16 columns.  Accumulator
    // item v of lane (r, g) is element (arow(v), acol(v)) of a 16 x 16 block.
    auto arow = [&](int v) { return F64 ? r : 4 * g + v; };
    auto acol = [&](int v) { return F64 ? g + 4 * v : r; };
    const int64_t c0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    int64_t colc[4];
    bool colok[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t col = c0 + acol(v);
        colok[v] = col < m;
        colc[v] = min(col, m - 1);
    }
    acc_t acc[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * t + arow(v);
            const T x = X[(int64_t)min(row, b - 1) + colc[v] * ldx];
            acc[t][v] = (row < b && colok[v]) ? x : T(0);
        }
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) {
        if (s < nblk) {
            // X_s = D_s^T R_s: R_s through LDS into operand layout
#pragma unroll
            for (int v = 0; v < 4; ++v) Rt[wave][arow(v)][acol(v)] = acc[s][v];
            acc_t xs = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                const int k = 4 * g + t4;  // both operands: k slot (g, t4)
                xs = mma_rc(Ds[s][k][r], Rt[wave][k][r], xs);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Rt[wave][arow(v)][acol(v)] = -xs[v];
                if (16 * s + arow(v) < b && colok[v]) X[(int64_t)(16 * s + arow(v)) + colc[v] * ldx] = xs[v];
            }
            // R_t -= U(s-rows, t-cols)^T X_s
#pragma unroll
            for (int t = s + 1; t < NB; ++t) {
                if (t < nblk) {
#pragma unroll
                    for (int t4 = 0; t4 < 4; ++t4) {
                        const int k = 4 * g + t4;
                        acc[t] = mma_rc(u_pad(U, ldu, b, 16 * s + k, 16 * t + r), Rt[wave][k][r], acc[t]);
                    }
                }
            }
        }
    }
}

template <typename T>
int launch_trsm_panel(int b, int64_t m, const T *U, int64_t ldu, T *X, int64_t ldx, const int32_t *info,
                      hipStream_t s) {
    if (b <= 0 || m <= 0) return FLAME_OK;
    if (b > 16 * kTrsmNb) {
        // two row halves: X_top := U_tt^{-T} X_top; X_bot -= U_tb^T X_top;
        // X_bot := U_bb^{-T} X_bot.  (One kernel over all sixteen row blocks
        // needs ~300 registers per lane, which keeps it off the CUs the
        // concurrent trailing update occupies; the split runs faster there.)
        const int b1 = 16 * kTrsmNb, b2 = b - b1;
        int rc = launch_trsm_panel<T>(b1, m, U, ldu, X, ldx, info, s);
        if (rc) return rc;
        rc = launch_gemm_tn(sizeof(T) == 8 ? Prec::F64 : Prec::F32, sizeof(T) == 8, false, b2, m, b1,
                            U + (int64_t)b1 * ldu, ldu, X, ldx, X + b1, ldx, info, s);
        if (rc) return rc;
        return launch_trsm_panel<T>(b2, m, U + b1 + (int64_t)b1 * ldu, ldu, X + b1, ldx, info, s);
    }
    const int tr = trace_begin(FLAME_KC_TRSM, s);
    hipLaunchKernelGGL((k_trsm_rl<T, kTrsmNb>), dim3((unsigned)((m + 63) / 64)), dim3(256), 0, s, b, m, U, ldu, X,
                       ldx, info, (int64_t)0, (int64_t)0);
    FLAME_CHECK_LAUNCH();
    const double db = (double)b, dm = (double)m;
    trace_end(tr, s, db * db * dm, (db * (db + 1) / 2 + 2 * db * dm) * (double)sizeof(T));
    return FLAME_OK;
}

// Inverses of the diagonal blocks of U (order <= 128 each, `nblk` blocks of
// order bs starting at U(0, 0), the last one min(bs, n - o)): Dt_q = U_qq^{-T},
// bs x bs column-major at Dt + q bs^2.  Dt must hold the identity on entry.
int launch_diag_inverse_t(int64_t n, int bs, const double *U, int64_t ldu, double *Dt, hipStream_t s) {
    const int64_t nblk = (n + bs - 1) / bs;
    const int64_t full = n / bs;  // blocks of order bs
    if (full > 0) {
        hipLaunchKernelGGL((k_trsm_rl<double, kTrsmNb>), dim3((unsigned)((bs + 63) / 64), (unsigned)full), dim3(256), 0, s, bs, (int64_t)bs,
                           U, ldu, Dt, (int64_t)bs, nullptr, (int64_t)bs * (ldu + 1), (int64_t)bs * bs);
        FLAME_CHECK_LAUNCH();
    }
    if (nblk > full) {
        const int64_t o = full * bs;
        const int last = (int)(n - o);
        hipLaunchKernelGGL((k_trsm_rl<double, kTrsmNb>), dim3((unsigned)((last + 63) / 64), 1u), dim3(256), 0, s, last, (int64_t)last,
                           U + o + o * ldu, ldu, Dt + full * (int64_t)bs * bs, (int64_t)bs, nullptr, (int64_t)0,
                           (int64_t)0);
        FLAME_CHECK_LAUNCH();
    }
    return FLAME_OK;
}

template int launch_trsm_panel<double>(int, int64_t, const double *, int64_t, double *, int64_t, const int32_t *,
                                       hipStream_t);
template int launch_trsm_panel<float>(int, int64_t, const float *, int64_t, float *, int64_t, const int32_t *,
                                      hipStream_t);

}  // namespace flame
