// LU without pivoting (flame_lu), right-looking at block 64 (the kernels are in
// k_lu.hip):
//   A11 := L\U(A11)                      k_lu_lds (LDS, one workgroup)
//   P1 := -(L11^{-1})^T, P2 := -U11^{-1}  k_lu_inv
//   A12 := L11^{-1} A12                  T := 0 - P1^T A12, A12 := T
//   A21 := A21 U11^{-1}, kept transposed: S := A21^T, S' := 0 - P2^T S
//                                        (= U11^{-T} A21^T)
//   A22 := A22 - A21 A12 = A22 - S'^T A12
//   A21 := S'^T
// The three products are the matrix-core trailing-update kernel (C -= X^T Y).
#include <algorithm>

#include "flame_internal.h"

namespace flame {

int lu_factor(int64_t n, double *A, int64_t lda, int32_t *info, hipStream_t s) {
    constexpr int kB = 64;
    int rc = launch_zero_i32(info, 1, s);
    if (rc || n == 0) return rc;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    // P1, P2 (kB x kB); T (kB x n); S, S' (kB x n)
    const size_t doubles = 2 * (size_t)kB * kB + 3 * (size_t)kB * (size_t)n;
    void *ws = nullptr;
    rc = ctx_workspace(ctx, kWsLu, doubles * sizeof(double), &ws);
    if (rc) return rc;
    double *P1 = static_cast<double *>(ws), *P2 = P1 + kB * kB;
    double *T = P2 + kB * kB, *S = T + (size_t)kB * n, *S2 = S + (size_t)kB * n;
    for (int64_t k = 0; k < n; k += kB) {
        const int64_t bk = std::min<int64_t>(kB, n - k), m = n - k - bk;
        double *A11 = A + k + k * lda, *A12 = A + k + (k + bk) * lda, *A21 = A + (k + bk) + k * lda;
        double *A22 = A + (k + bk) + (k + bk) * lda;
        rc = launch_lu_lds((int)bk, A11, lda, info, k, s);
        if (rc) return rc;
        if (m == 0) break;
        rc = launch_lu_inv((int)bk, A11, lda, P1, P2, info, s);
        // A12 := L11^{-1} A12
        if (!rc) rc = launch_fill0(bk, m, T, kB, s);
        if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, bk, m, bk, P1, kB, A12, lda, T, kB, info, s);
        if (!rc) rc = launch_scaled_copy(bk, m, T, kB, A12, lda, 1.0, info, s);
        // A21^T := U11^{-T} A21^T
        if (!rc) rc = launch_transpose_copy(m, bk, A21, lda, S, kB, info, s);
        if (!rc) rc = launch_fill0(bk, m, S2, kB, s);
        if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, bk, m, bk, P2, kB, S, kB, S2, kB, info, s);
        // A22 -= A21 A12
        if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, m, m, bk, S2, kB, A12, lda, A22, lda, info, s);
        // A21 := (A21^T)^T (skipped after a breakdown: A21 keeps what it held)
        if (!rc) rc = launch_transpose_copy(bk, m, S2, kB, A21, lda, info, s);
        if (rc) return rc;
    }
    return FLAME_OK;
}

}  // namespace flame
