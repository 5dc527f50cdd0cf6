// TRSM step of the loop body (Fig. "dense-chol"): A12 := triu(A11)^{-T} A12,
// i.e. solve U^T X = A12 for X with U = triu(A11) (b x b, b <= 256) and
// A12 b x m.  (The figure prints triu(A11)^{-1}; only the transposed solve
// reproduces A = U^T U.)
//
// Orders above 128 are solved as two row halves joined by a GEMM update.
#include "flame_internal.h"
#include "trsm_rl.h"

namespace flame {

// Panel kernel: each workgroup forms the inverses, then each of its four
// wavefronts solves 16 columns.
constexpr int kTrsmNb = 8;  // row blocks of 16 per kernel: b <= 128

// At most 256 registers per lane (two workgroups per CU): a TRSM workgroup
// then fits on a CU beside one trailing-update workgroup (the concurrent
// remainder update leaves such CUs), not only on empty ones (n = 16384:
// 32.4 -> 32.0 ms; 210 registers, no spills).
template <typename T, int NB>
__global__ __launch_bounds__(256, 2) void k_trsm_rl(int b, int64_t m, const T *__restrict__ U, int64_t ldu,
                                                 T *__restrict__ X, int64_t ldx, const int32_t *__restrict__ info,
                                                 int64_t u_step, int64_t x_step) {
    // blockIdx.y selects one of several independent solves (U and X advanced
    // by u_step and x_step elements)
    U += (int64_t)blockIdx.y * u_step;
    X += (int64_t)blockIdx.y * x_step;
    __shared__ T Ds[NB][16][17];  // inverses of the diagonal blocks, [block][k][col]
    __shared__ T Rt[4][16][17];   // per wavefront: one block, [row][col]
    if (info != nullptr && *info != 0) return;
    const int wave = threadIdx.x >> 6;
    // U is read from global memory / L2 (no LDS copy), so that the kernel fits
    // beside the trailing-update workgroups on a CU
    trsm_inverses<T, NB>(b, U, ldu, Ds);
    __syncthreads();
    trsm_cols<T, NB>(b, m, U, ldu, X, ldx, ((int64_t)blockIdx.x * 4 + wave) * 16, Ds, Rt[wave]);
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
