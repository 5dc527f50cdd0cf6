// LU without pivoting (flame_lu), right-looking at block 64 (the kernels are in
// k_lu.hip):
//   A11 := L\U(A11),                     k_lu_diag (LDS, one workgroup,
//   P1 := -(L11^{-1})^T, P2 := -U11^{-1}  one launch)
//   S := A21^T, T := 0, S' := 0          one launch
//   A12 := L11^{-1} A12                  T := 0 - P1^T A12
//   A21 := A21 U11^{-1}, kept transposed: S' := 0 - P2^T S
//                                        (= U11^{-T} A21^T)
//   A22 := A22 - A21 A12 = A22 - S'^T T
//   A12 := T, A21 := S'^T                after the products
// The products are the matrix-core trailing-update kernel (C -= X^T Y).
#include <algorithm>

#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kB = 64;
constexpr int64_t kLookN = 2048;
constexpr int64_t kWbSideN = 4096;
constexpr int kSideCus = 16;  // compute units the side stream's product leaves to the next step's chain
// The side stream takes the rest of A22 only while more than kLookN rows
// remain beyond the next step's: below that the product is shorter than what
// the second stream costs (events, a third launch), and one product on the
// main stream is faster (n = 2048: 4.4 ms against 5.0 ms with the split).
// The write-backs of A12 and A21 join the side stream while fewer than
// kWbSideN rows remain beyond the next step's: there the step's chain is the
// longer path; above it the side stream's product is, and they stay on the
// main stream.

// A12 := T and A21 := S2^T (skipped after a breakdown).
int write_back(int64_t bk, int64_t m, const double *T, const double *S2, double *A12, double *A21, int64_t lda,
               const int32_t *info, hipStream_t s) {
    int rc = launch_scaled_copy(bk, m, T, kB, A12, lda, 1.0, info, s);
    if (!rc) rc = launch_transpose_copy(bk, m, S2, kB, A21, lda, info, s);
    return rc;
}

int lu_steps(int64_t n, double *A, int64_t lda, int32_t *info, hipStream_t s, hipStream_t side, double *P1,
             double *P2, double *const Tbuf[2], double *S, double *const S2buf[2], hipEvent_t ev_next,
             hipEvent_t ev_rest, bool *side_pending) {
    int rc = FLAME_OK;
    for (int64_t k = 0, step = 0; k < n; k += kB, ++step) {
        const int64_t bk = std::min<int64_t>(kB, n - k), m = n - k - bk;
        double *A11 = A + k + k * lda, *A12 = A + k + (k + bk) * lda, *A21 = A + (k + bk) + k * lda;
        double *A22 = A + (k + bk) + (k + bk) * lda;
        double *T = Tbuf[step & 1], *S2 = S2buf[step & 1];
        // the step's chain: it reads only what the previous step's first
        // products (main stream) updated
        rc = launch_lu_diag((int)bk, A11, lda, info, k, m > 0 ? P1 : nullptr, m > 0 ? P2 : nullptr, s);
        if (rc) return rc;
        if (m == 0) break;
        // S := A21^T, and T, S2 := 0 for the products below (one launch)
        rc = launch_transpose_copy(m, bk, A21, lda, S, kB, info, s, T, S2);
        // T := L11^{-1} A12 and S2 := U11^{-T} A21^T
        if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, bk, m, bk, P1, kB, A12, lda, T, kB, info, s);
        if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, bk, m, bk, P2, kB, S, kB, S2, kB, info, s);
        if (rc) return rc;
        // A22 -= A21 A12 = S2^T T (the previous step's side product covered
        // part of A22 too); A12 := T and A21 := S2^T are results only (no
        // later step reads them), written back after the products (skipped
        // after a breakdown: A12 and A21 keep what they held)
        if (*side_pending) FLAME_HIP(hipStreamWaitEvent(s, ev_rest, 0));
        *side_pending = false;
        const int64_t nb2 = std::min<int64_t>(kB, m), far = m - nb2;
        if (far <= kLookN) {  // all of A22 on the main stream
            rc = launch_gemm_tn(Prec::F64, true, false, m, m, bk, S2, kB, T, kB, A22, lda, info, s);
            if (!rc) rc = write_back(bk, m, T, S2, A12, A21, lda, info, s);
            if (rc) return rc;
            continue;
        }
        // first the next step's rows and columns (main stream) ...
        rc = launch_gemm_tn(Prec::F64, true, false, nb2, m, bk, S2, kB, T, kB, A22, lda, info, s);
        if (!rc)
            rc = launch_gemm_tn(Prec::F64, true, false, far, nb2, bk, S2 + nb2 * kB, kB, T, kB, A22 + nb2, lda, info,
                                s);
        if (rc) return rc;
        // ... then the rest on the side stream, beside the next step's chain;
        // the write-backs join whichever stream has the shorter path (on the
        // main stream before the side stream starts: while the side product
        // runs, the main stream has few compute units)
        const bool wb_side = far < kWbSideN;
        if (!wb_side) rc = write_back(bk, m, T, S2, A12, A21, lda, info, s);
        if (rc) return rc;
        FLAME_HIP(hipEventRecord(ev_next, s));
        FLAME_HIP(hipStreamWaitEvent(side, ev_next, 0));
        rc = launch_gemm_tn(Prec::F64, true, false, far, far, bk, S2 + nb2 * kB, kB, T + nb2 * kB, kB,
                            A22 + nb2 + nb2 * lda, lda, info, side, kSideCus);
        if (!rc && wb_side) rc = write_back(bk, m, T, S2, A12, A21, lda, info, side);
        if (rc) return rc;
        FLAME_HIP(hipEventRecord(ev_rest, side));
        *side_pending = true;
    }
    return FLAME_OK;
}

}  // namespace

// Lookahead of one step: step k's product for the rows and columns of step
// k + 1 runs first on the main stream, the rest of A22 on the side stream
// while the main stream runs step k + 1's chain (diagonal block, panel
// solves), which reads only those rows and columns; step k + 1's own
// products wait for the side stream.  The panel solves' results T and S'
// alternate between two buffers each, so step k + 1's chain never overwrites
// what the side stream still reads; the side stream also writes them back to
// A12 and A21, off the chain.
int lu_factor(int64_t n, double *A, int64_t lda, int32_t *info, hipStream_t s) {
    int rc = launch_zero_i32(info, 1, s);
    if (rc || n == 0) return rc;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    // P1, P2 (kB x kB); T twice, S, S' twice (kB x n each)
    const size_t doubles = 2 * (size_t)kB * kB + 5 * (size_t)kB * (size_t)n;
    void *ws = nullptr;
    rc = ctx_workspace(ctx, kWsLu, doubles * sizeof(double), &ws);
    if (rc) return rc;
    double *P1 = static_cast<double *>(ws), *P2 = P1 + kB * kB;
    double *const Tbuf[2] = {P2 + kB * kB, P2 + kB * kB + (size_t)kB * n};
    double *S = Tbuf[1] + (size_t)kB * n;
    double *const S2buf[2] = {S + (size_t)kB * n, S + 2 * (size_t)kB * n};
    hipStream_t side = ctx_side_stream(ctx);
    hipEvent_t ev_next = ctx_event(ctx, 2);  // main: the next step's rows and columns updated
    hipEvent_t ev_rest = ctx_event(ctx, 3);  // side: the rest of A22 updated
    bool side_pending = false;
    rc = lu_steps(n, A, lda, info, s, side, P1, P2, Tbuf, S, S2buf, ev_next, ev_rest, &side_pending);
    // the side stream's last product joins the caller's stream (also after an error)
    if (side_pending) FLAME_HIP(hipStreamWaitEvent(s, ev_rest, 0));
    return rc;
}

}  // namespace flame
