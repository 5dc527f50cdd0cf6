// Complex Hermitian factorization A = U^H U (dtype FLAME_Z64 of flame_factor):
// the right-looking loop of Fig. "dense-chol" with its update read literally
// as the Hermitian rank-k update,
//   A11 := Chol(A11);  A12 := triu(A11)^{-H} A12;  A22 := A22 - A12^H A12,
// on complex data (the conclusion lists complex data among the extensions).
//
// The matrix is kept in two real planes (real and imaginary parts, column-
// major, ld = n) for the whole factorization, split from and merged back into
// the caller's interleaved upper triangle.  Every complex product
// C -= P^H Q is then four real matrix-core products of the trailing-update
// kernel (launch_gemm_tn, C -= X^T Y), since
//   P^H Q = (Pr^T Qr + Pi^T Qi) + i (Pr^T Qi - Pi^T Qr),
// the last one with a negated copy of Pi.  The HERK of each iteration is one
// such product (upper triangle only); the panel solve goes by diagonal blocks
// of 64: V = -U_ss^{-1}, X_s := -V^H X_s = U_ss^{-H} X_s in place by the
// fused complex product, and X_t -= U_st^H X_s for the blocks below.
// Diagonal blocks of the outer loop (nb) are factored by the same loop at
// block 64, whose diagonal blocks go to the LDS kernel k_zchol_lds; it forms
// each 64-block's V in the same launch, kept for the outer panel solve.
#include <algorithm>

#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kZB = 64;  // inner block (LDS kernels)
constexpr int kSlots = 8;  // inverses kept, one per 64-block of an outer block (nb <= 512)

struct ZWork {
    double *R, *I;  // planes, ld = n
    int64_t ld;
    double *Pn;       // negated imaginary operand, up to nb x n
    double *Vr, *Vi;  // V = -U_ss^{-1} of the outer block's 64-blocks, kSlots x (kZB x kZB)
};

// C -= P^H Q; P is K x M (ldp), Q is K x N (ldq), C is M x N (ldc), each given
// by its planes.  upper: only i <= j of C is written (the HERK: four real
// products on the LDS-staged trailing-update kernel); otherwise the fused
// complex product k_zgemm_h.
int zgemm_h(bool upper, int64_t M, int64_t N, int64_t K, const double *Pr, const double *Pi, int64_t ldp,
            const double *Qr, const double *Qi, int64_t ldq, double *Cr, double *Ci, int64_t ldc, double *Pn,
            const int32_t *info, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return FLAME_OK;
    // the panel solve's products (at most nb rows of C): one fused pass,
    // the four real products sharing their operand loads
    if (!upper) return launch_zgemm_h(false, M, N, K, Pr, Pi, ldp, Qr, Qi, ldq, Cr, Ci, ldc, info, s);
    int rc = launch_gemm_tn(Prec::F64, true, upper, M, N, K, Pr, ldp, Qr, ldq, Cr, ldc, info, s);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, upper, M, N, K, Pi, ldp, Qi, ldq, Cr, ldc, info, s);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, upper, M, N, K, Pr, ldp, Qi, ldq, Ci, ldc, info, s);
    if (!rc) rc = launch_scaled_copy(K, M, Pi, ldp, Pn, K, -1.0, info, s);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, upper, M, N, K, Pn, K, Qr, ldq, Ci, ldc, info, s);
    return rc;
}

// X := triu(U)^{-H} X for the b x b block U at (k, k) and the b x m panel X
// at (k, c0) of the planes.  The negated inverse of the 64-block s is in slot
// slot0 + s already: the diagonal-block kernel formed it with the factor.
int ztrsm(const ZWork &w, int64_t k, int64_t b, int64_t c0, int64_t m, const int32_t *info, hipStream_t s,
          int slot0) {
    const int64_t ld = w.ld;
    for (int64_t s0 = 0; s0 < b; s0 += kZB) {
        const int64_t bs = std::min<int64_t>(kZB, b - s0);
        const int64_t xs = (k + s0) + c0 * ld;         // X_s
        const int ib = (int)(s0 / kZB);
        double *Vr = w.Vr + (int64_t)(slot0 + ib) * kZB * kZB, *Vi = w.Vi + (int64_t)(slot0 + ib) * kZB * kZB;
        // X_s := -V^H X_s = U_ss^{-H} X_s, in place
        int rc = launch_zgemm_h_inplace(bs, m, bs, Vr, Vi, kZB, w.R + xs, w.I + xs, ld, info, s);
        if (rc) return rc;
        const int64_t rest = b - s0 - bs;
        if (rest > 0) {
            // X_t -= U(s, t)^H X_s for the rows of the blocks below
            const int64_t ust = (k + s0) + (k + s0 + bs) * ld;
            const int64_t xt = (k + s0 + bs) + c0 * ld;
            rc = zgemm_h(false, rest, m, bs, w.R + ust, w.I + ust, ld, w.R + xs, w.I + xs, ld, w.R + xt, w.I + xt,
                         ld, w.Pn, info, s);
            if (rc) return rc;
        }
    }
    return FLAME_OK;
}

// Chol of the n x n diagonal block at (k, k) of the planes, by the loop at
// block nb (<= kZB: the LDS kernel, which also forms the 64-block's negated
// inverse); the inverses go to the slots from slot_base (one per 64-block).
int zpotrf_block(const ZWork &w, int64_t k, int64_t n, int64_t nb, int32_t *info, int64_t info_base,
                 hipStream_t s, int slot_base) {
    const int64_t ld = w.ld;
    if (n <= kZB)
        return launch_zchol_lds((int)n, w.R + k + k * ld, w.I + k + k * ld, ld, info, info_base,
                                w.Vr + (int64_t)slot_base * kZB * kZB, w.Vi + (int64_t)slot_base * kZB * kZB, kZB, s);
    for (int64_t k0 = 0; k0 < n; k0 += nb) {
        const int64_t bk = std::min<int64_t>(nb, n - k0);
        const int64_t m = n - k0 - bk;
        int rc = zpotrf_block(w, k + k0, bk, kZB, info, info_base + k0, s, slot_base + (int)(k0 / kZB));
        if (rc) return rc;
        if (m == 0) break;
        rc = ztrsm(w, k + k0, bk, k + k0 + bk, m, info, s, slot_base + (int)(k0 / kZB));
        if (rc) return rc;
        // A22 -= A12^H A12 (upper)
        const int64_t a12 = (k + k0) + (k + k0 + bk) * ld, a22 = (k + k0 + bk) + (k + k0 + bk) * ld;
        rc = zgemm_h(true, m, m, bk, w.R + a12, w.I + a12, ld, w.R + a12, w.I + a12, ld, w.R + a22, w.I + a22, ld,
                     w.Pn, info, s);
        if (rc) return rc;
    }
    return FLAME_OK;
}

// C -= P^H P for the upper triangle of the M x N block C at (i0, i0) of the
// trailing matrix (the HERK's rows i0 .. i0 + M, columns from i0), P the K x n
// panel (planes, ld w.ld) with its imaginary part negated in Pn (ld K): four
// real products on the trailing-update kernel.
int herk_part(const ZWork &w, int64_t a12, int64_t a22, const double *Pn, int64_t i0, int64_t M, int64_t N,
              int64_t K, const int32_t *info, hipStream_t s, int reserve_cus) {
    const int64_t ld = w.ld;
    const double *Pr = w.R + a12 + i0 * ld, *Pi = w.I + a12 + i0 * ld, *Pni = Pn + i0 * K;
    double *Cr = w.R + a22 + i0 + i0 * ld, *Ci = w.I + a22 + i0 + i0 * ld;
    int rc = launch_gemm_tn(Prec::F64, true, true, M, N, K, Pr, ld, Pr, ld, Cr, ld, info, s, reserve_cus);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, true, M, N, K, Pi, ld, Pi, ld, Cr, ld, info, s, reserve_cus);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, true, M, N, K, Pr, ld, Pi, ld, Ci, ld, info, s, reserve_cus);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, true, M, N, K, Pni, K, Pr, ld, Ci, ld, info, s, reserve_cus);
    return rc;
}

constexpr int64_t kLookN = 2048;  // side stream only while more rows than this remain beyond the next block
constexpr int kSideCus = 16;

// The outer loop at block nb with one block of lookahead: the HERK's rows of
// the next block first (main stream), the rest of the trailing matrix on the
// side stream beside the next block's chain (its diagonal block and panel
// solve, which read only those rows); the next block's HERK waits for it.
// The negated imaginary panel alternates between two buffers.
int zfactor_outer(const ZWork &w, int64_t n, int64_t nb, double *const Pnb[2], int32_t *info, hipStream_t s,
                  hipStream_t side, hipEvent_t ev_next, hipEvent_t ev_rest, bool *side_pending) {
    const int64_t ld = w.ld;
    for (int64_t k0 = 0, step = 0; k0 < n; k0 += nb, ++step) {
        const int64_t bk = std::min<int64_t>(nb, n - k0), m = n - k0 - bk;
        int rc = zpotrf_block(w, k0, bk, kZB, info, k0, s, 0);
        if (rc) return rc;
        if (m == 0) break;
        // the diagonal-block kernels formed the inverses of all its 64-blocks
        rc = ztrsm(w, k0, bk, k0 + bk, m, info, s, 0);
        if (rc) return rc;
        // A22 -= A12^H A12 (upper); the previous block's side part covered
        // rows of it too
        if (*side_pending) FLAME_HIP(hipStreamWaitEvent(s, ev_rest, 0));
        *side_pending = false;
        const int64_t a12 = k0 + (k0 + bk) * ld, a22 = (k0 + bk) + (k0 + bk) * ld;
        double *Pn = Pnb[step & 1];
        rc = launch_scaled_copy(bk, m, w.I + a12, ld, Pn, bk, -1.0, info, s);
        if (rc) return rc;
        const int64_t nb2 = std::min<int64_t>(nb, m), far = m - nb2;
        if (far <= kLookN) {
            rc = herk_part(w, a12, a22, Pn, 0, m, m, bk, info, s, 0);
            if (rc) return rc;
            continue;
        }
        rc = herk_part(w, a12, a22, Pn, 0, nb2, m, bk, info, s, 0);
        if (rc) return rc;
        FLAME_HIP(hipEventRecord(ev_next, s));
        FLAME_HIP(hipStreamWaitEvent(side, ev_next, 0));
        rc = herk_part(w, a12, a22, Pn, nb2, far, far, bk, info, side, kSideCus);
        if (rc) return rc;
        FLAME_HIP(hipEventRecord(ev_rest, side));
        *side_pending = true;
    }
    return FLAME_OK;
}

}  // namespace

int zfactor(int64_t n, void *A, int64_t lda, int nb, int32_t *info, hipStream_t s) {
    int rc = launch_zero_i32(info, 1, s);
    if (rc || n == 0) return rc;
    nb = std::max(kZB, std::min(nb, 512)) / kZB * kZB;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    const size_t plane = (size_t)n * (size_t)n;
    const size_t doubles =
        2 * plane + 3 * (size_t)nb * (size_t)n + 2 * (size_t)kSlots * kZB * kZB;
    void *ws = nullptr;
    rc = ctx_workspace(ctx, kWsComplex, doubles * sizeof(double), &ws);
    if (rc) return rc;
    double *p = static_cast<double *>(ws);
    ZWork w;
    w.R = p;
    w.I = p + plane;
    w.ld = n;
    w.Pn = p + 2 * plane;
    w.Vr = w.Pn + (size_t)nb * n;
    w.Vi = w.Vr + (size_t)kSlots * kZB * kZB;
    double *const Pnb[2] = {w.Vi + (size_t)kSlots * kZB * kZB, w.Vi + (size_t)kSlots * kZB * kZB + (size_t)nb * n};
    hipStream_t side = ctx_side_stream(ctx);
    hipEvent_t ev_next = ctx_event(ctx, 2);  // main: the next block's rows updated
    hipEvent_t ev_rest = ctx_event(ctx, 3);  // side: the rest of the trailing matrix updated
    bool side_pending = false;
    rc = launch_z_split(n, A, lda, w.R, w.I, n, s);
    if (!rc) rc = zfactor_outer(w, n, nb, Pnb, info, s, side, ev_next, ev_rest, &side_pending);
    // the side stream's last part joins the caller's stream (also after an error)
    if (side_pending) FLAME_HIP(hipStreamWaitEvent(s, ev_rest, 0));
    if (!rc) rc = launch_z_merge(n, w.R, w.I, n, A, lda, s);
    return rc;
}

}  // namespace flame
