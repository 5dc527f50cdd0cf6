// TRSM step of the loop body (Fig. "dense-chol"): A12 := triu(A11)^{-T} A12,
// i.e. solve U^T X = A12 for X with U = triu(A11) (b x b, b <= 256) and
// A12 b x m.  (The figure prints triu(A11)^{-1}; only the transposed solve
// reproduces A = U^T U.)
//
// Columns of A12 are independent: one lane owns one column.  Rows are taken in
// chunks of 32 held in registers; inside a chunk the solve is a forward
// substitution, and each finished chunk immediately updates the rows below it
// (right-looking over chunks).  U is only ever addressed with wave-uniform
// indices, so its entries come in through scalar loads shared by the wave.
#include "flame_internal.h"

namespace flame {

constexpr int TCH = 32;  // rows per register chunk

template <typename T>
__global__ __launch_bounds__(64) void k_trsm_panel(int b, int64_t m, const T *__restrict__ U, int64_t ldu,
                                                   T *__restrict__ X, int64_t ldx,
                                                   const int32_t *__restrict__ info) {
    if (info != nullptr && *info != 0) return;
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool active = c < m;
    T *xc = X + (active ? c : 0) * ldx;
    for (int r0 = 0; r0 < b; r0 += TCH) {
        const int w = min(TCH, b - r0);
        T x[TCH];
#pragma unroll
        for (int i = 0; i < TCH; ++i) x[i] = (active && i < w) ? xc[r0 + i] : T(0);
        // forward substitution with the chunk's diagonal block of U^T
#pragma unroll
        for (int t = 0; t < TCH; ++t) {
            if (t < w) {
                const T *ut = U + r0 + (int64_t)(r0 + t) * ldu;  // column r0 + t of U
                T acc = x[t];
#pragma unroll
                for (int q = 0; q < t; ++q) acc = acc - ut[q] * x[q];
                x[t] = acc / ut[t];
            }
        }
        if (active) {
#pragma unroll
            for (int i = 0; i < TCH; ++i)
                if (i < w) xc[r0 + i] = x[i];
        }
        // rows below the chunk: x_r -= sum_q U(r0 + q, r) x_q
        for (int r = r0 + w; r < b; ++r) {
            const T *ur = U + r0 + (int64_t)r * ldu;  // column r of U, rows r0 ..
            T v = active ? xc[r] : T(0);
#pragma unroll
            for (int q = 0; q < TCH; ++q)
                if (q < w) v = v - ur[q] * x[q];
            if (active) xc[r] = v;
        }
    }
}

// ---- FP64 matrix-core panel solve (b <= 128) -------------------------------
// The solve blocked by 16 rows (U padded with the identity to a multiple of
// 16).  Each workgroup first forms the inverses D_s = U_ss^{-1} of the 16 x 16
// diagonal blocks in LDS (16 lanes per block, one lane per column, back
// substitution).  Then each wavefront owns 16 columns of X, keeps all of its
// row blocks in registers and runs the right-looking loop
//   X_s = D_s^T R_s;   R_t -= U(s, t)^T X_s  for t > s
// on FP64 matrix cores, fully unrolled over the eight row blocks so that the
// loads of U are independent of the arithmetic and can be issued early.  MFMA
// placement as in the trailing update: lane (r, g) holds row r, columns
// g + 4v of a 16 x 16 block.
typedef double d4v __attribute__((ext_vector_type(4)));
constexpr int kTrsmNb = 8;  // row blocks of 16: b <= 128

// U(i, j) with rows / columns >= b read as the identity
__device__ __forceinline__ double u_pad(const double *__restrict__ U, int64_t ldu, int b, int i, int j) {
    const double v = U[(int64_t)min(i, b - 1) + (int64_t)min(j, b - 1) * ldu];
    return (i < b && j < b) ? v : (i == j ? 1.0 : 0.0);
}

__global__ __launch_bounds__(256) void k_trsm_rl(int b, int64_t m, const double *__restrict__ U, int64_t ldu,
                                                 double *__restrict__ X, int64_t ldx,
                                                 const int32_t *__restrict__ info, int64_t u_step, int64_t x_step) {
    // blockIdx.y selects one of several independent solves (U and X advanced
    // by u_step and x_step elements)
    U += (int64_t)blockIdx.y * u_step;
    X += (int64_t)blockIdx.y * x_step;
    constexpr int NB = kTrsmNb;
    __shared__ double Ub[NB][16][17];  // diagonal blocks of U, [block][row][col]
    __shared__ double Ds[NB][16][17];  // their inverses, [block][k][col]
    __shared__ double Rt[4][16][17];   // per wavefront: one block in operand layout
    if (info != nullptr && *info != 0) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15;
    const int g = lane >> 4;
    const int nblk = (b + 15) >> 4;
    // (1) diagonal blocks and their inverses
    for (int idx = tid; idx < NB * 256; idx += 256) {
        const int sb = idx >> 8, i = (idx >> 4) & 15, j = idx & 15;
        Ub[sb][i][j] = u_pad(U, ldu, b, 16 * sb + i, 16 * sb + j);
    }
    __syncthreads();
    if (tid < NB * 16) {
        const int sb = tid >> 4, t = tid & 15;  // column t of D_sb: U_ss D(:, t) = e_t
        double v[16];
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            double acc = (i == t) ? 1.0 : 0.0;
#pragma unroll
            for (int k = i + 1; k < 16; ++k) acc -= Ub[sb][i][k] * v[k];
            v[i] = acc / Ub[sb][i][i];  // rows below the diagonal come out 0
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Ds[sb][i][t] = v[i];
    }
    __syncthreads();

    // (2) right-looking solve of this wavefront's 16 columns
    const int64_t c0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    int64_t colc[4];
    bool colok[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t col = c0 + g + 4 * v;
        colok[v] = col < m;
        colc[v] = min(col, m - 1);
    }
    d4v acc[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int row = 16 * t + r;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double x = X[(int64_t)min(row, b - 1) + colc[v] * ldx];
            acc[t][v] = (row < b && colok[v]) ? x : 0.0;
        }
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) {
        if (s < nblk) {
            // X_s = D_s^T R_s: R_s through LDS into operand layout
#pragma unroll
            for (int v = 0; v < 4; ++v) Rt[wave][r][g + 4 * v] = acc[s][v];
            d4v xs = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                const int k = 4 * g + t4;
                xs = __builtin_amdgcn_mfma_f64_16x16x4f64(Rt[wave][k][r], Ds[s][k][r], xs, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Rt[wave][r][g + 4 * v] = -xs[v];
                if (16 * s + r < b && colok[v]) X[(int64_t)(16 * s + r) + colc[v] * ldx] = xs[v];
            }
            // R_t -= U(s-rows, t-cols)^T X_s
#pragma unroll
            for (int t = s + 1; t < NB; ++t) {
                if (t < nblk) {
#pragma unroll
                    for (int t4 = 0; t4 < 4; ++t4) {
                        const int k = 4 * g + t4;
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Rt[wave][k][r],
                                                                      u_pad(U, ldu, b, 16 * s + k, 16 * t + r), acc[t],
                                                                      0, 0, 0);
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
    if constexpr (sizeof(T) == 8) {
        if (b > 16 * kTrsmNb) {
            // two row halves: X_top := U_tt^{-T} X_top; X_bot -= U_tb^T X_top;
            // X_bot := U_bb^{-T} X_bot
            const int b1 = 16 * kTrsmNb, b2 = b - b1;
            int rc = launch_trsm_panel<T>(b1, m, U, ldu, X, ldx, info, s);
            if (rc) return rc;
            rc = launch_gemm_tn(Prec::F64, true, false, b2, m, b1, U + (int64_t)b1 * ldu, ldu, X, ldx, X + b1, ldx,
                                info, s);
            if (rc) return rc;
            return launch_trsm_panel<T>(b2, m, U + b1 + (int64_t)b1 * ldu, ldu, X + b1, ldx, info, s);
        }
    }
    const int tr = trace_begin(FLAME_KC_TRSM, s);
    if constexpr (sizeof(T) == 8) {
        const int64_t blocks = (m + 63) / 64;
        hipLaunchKernelGGL(k_trsm_rl, dim3((unsigned)blocks), dim3(256), 0, s, b, m, U, ldu, X, ldx, info, (int64_t)0,
                           (int64_t)0);
    } else {
        const int64_t blocks = (m + 63) / 64;
        hipLaunchKernelGGL(k_trsm_panel<T>, dim3((unsigned)blocks), dim3(64), 0, s, b, m, U, ldu, X, ldx, info);
    }
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
        hipLaunchKernelGGL(k_trsm_rl, dim3((unsigned)((bs + 63) / 64), (unsigned)full), dim3(256), 0, s, bs, (int64_t)bs,
                           U, ldu, Dt, (int64_t)bs, nullptr, (int64_t)bs * (ldu + 1), (int64_t)bs * bs);
        FLAME_CHECK_LAUNCH();
    }
    if (nblk > full) {
        const int64_t o = full * bs;
        const int last = (int)(n - o);
        hipLaunchKernelGGL(k_trsm_rl, dim3((unsigned)((last + 63) / 64), 1u), dim3(256), 0, s, last, (int64_t)last,
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
