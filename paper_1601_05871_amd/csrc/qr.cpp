// Householder QR (flame_qr), A = Q R for m x n, m >= n: the right-looking
// partitioned loop of Fig. "dense-chol" with QR's steps (the conclusion names
// QR among the factorizations the pattern carries over to), blocked twice:
//
//   for each outer block of 128 columns (the rows below it: V, T, the update):
//     for each panel of 32 columns inside it:
//       factor the panel into reflectors              k_qr_panel
//       G(:, panel) := -V^T V_panel                   matrix-core product
//       T(:, panel) from G and tau                    k_qr_t
//       C := (I - V_p T_pp^T V_p^T) C for the block's columns right of the
//            panel (three matrix-core products, below)
//     A2 := (I - V T^T V^T) A2 for the columns right of the block
//
// Q^T C = C - V T^T V^T C goes as
//   W  := 0 - V^T C        (K = rows of C: split over K)
//   Y  := 0 - T^T W        (= T^T V^T C)
//   C  := C - (V^T)^T Y    (K = block width)
// with V kept twice, as columns (Vs, for V^T C) and as rows (Vt, for V Y), so
// that every product is the trailing-update kernel's C -= X^T Y.
#include <algorithm>

#include "flame_internal.h"

namespace flame {

int qr_panel_rows();
int launch_qr_panel(int64_t m, int b, double *A, int64_t lda, double *tau, double *Vs, int64_t ldvs, double *Vt,
                    int64_t ldvt, int64_t ro, double *xch, int32_t *info, hipStream_t s);
int launch_qr_t(int j0, int j1, const double *G, int64_t ldg, const double *tau, double *T, int64_t ldt,
                const int32_t *info, hipStream_t s);

namespace {

constexpr int kIB = 32;   // panel
constexpr int kOB = 128;  // outer block

struct QrWork {
    double *Vs;  // m x kOB, ld ldvs
    int64_t ldvs;
    double *Vt;  // kOB x m, ld kOB
    double *W, *Y;  // kOB x n, ld kOB
    double *G, *T;  // kOB x kOB
    double *xch;
    double *split;  // split-K partial products
};

// C -= X^T Y with a long K: the largest multiple of 32 of K split over
// slices (one launch), the rest as a plain product.
int gemm_long(int64_t M, int64_t N, int64_t K, const double *X, int64_t ldx, const double *Y, int64_t ldy, double *C,
              int64_t ldc, double *split, const int32_t *info, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return FLAME_OK;
    const int64_t Km = K / 32 * 32;
    int rc = FLAME_OK;
    if (Km > 0) rc = launch_gemm_splitk<double>(false, M, N, Km, X, ldx, Y, ldy, C, ldc, split, info, s);
    if (!rc && K > Km)
        rc = launch_gemm_tn(Prec::F64, true, false, M, N, K - Km, X + Km, ldx, Y + Km, ldy, C, ldc, info, s);
    return rc;
}

// C := (I - V T^T V^T) C for the mr x nc block C, kb reflectors: V (mr x kb)
// at V (ld ldv), its rows at Vt (ld kOB), T (kb x kb) at Tb (ld kOB).
int apply_qt(const QrWork &w, int64_t mr, int64_t nc, int kb, const double *V, const double *Vt, const double *Tb,
             double *C, int64_t ldc, const int32_t *info, hipStream_t s) {
    if (nc <= 0) return FLAME_OK;
    int rc = launch_fill0(kb, nc, w.W, kOB, s);
    if (!rc) rc = gemm_long(kb, nc, mr, V, w.ldvs, C, ldc, w.W, kOB, w.split, info, s);
    if (!rc) rc = launch_fill0(kb, nc, w.Y, kOB, s);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, kb, nc, kb, Tb, kOB, w.W, kOB, w.Y, kOB, info, s);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, mr, nc, kb, Vt, kOB, w.Y, kOB, C, ldc, info, s);
    return rc;
}

}  // namespace

int qr_factor(int64_t m, int64_t n, double *A, int64_t lda, double *tau, int32_t *info, hipStream_t s) {
    int rc = launch_zero_i32(info, 1, s);
    if (rc || n == 0) return rc;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    const int64_t pmax = (m + qr_panel_rows() - 1) / qr_panel_rows();
    const int64_t ldvs = (m + 1) / 2 * 2;  // even: 16-byte aligned columns
    const size_t xch = (size_t)kIB * pmax * kIB + (size_t)kIB * kIB;
    const size_t doubles = (size_t)ldvs * kOB + (size_t)kOB * (size_t)m + 2 * (size_t)kOB * (size_t)n +
                           2 * (size_t)kOB * kOB + xch;
    void *ws = nullptr;
    rc = ctx_workspace(ctx, kWsQr, doubles * sizeof(double), &ws);
    if (rc) return rc;
    void *split = nullptr;
    rc = ctx_workspace(ctx, kWsSplit, splitk_workspace_bytes(), &split);
    if (rc) return rc;
    QrWork w;
    w.Vs = static_cast<double *>(ws);
    w.ldvs = ldvs;
    w.Vt = w.Vs + (size_t)ldvs * kOB;
    w.W = w.Vt + (size_t)kOB * m;
    w.Y = w.W + (size_t)kOB * n;
    w.G = w.Y + (size_t)kOB * n;
    w.T = w.G + (size_t)kOB * kOB;
    w.xch = w.T + (size_t)kOB * kOB;
    w.split = static_cast<double *>(split);
    for (int64_t k = 0; k < n; k += kOB) {
        const int nbk = (int)std::min<int64_t>(kOB, n - k);
        const int64_t mk = m - k;
        for (int i0 = 0; i0 < nbk; i0 += kIB) {
            const int bi = std::min(kIB, nbk - i0);
            const int64_t mi = mk - i0;
            double *Ap = A + (k + i0) + (k + i0) * lda;
            rc = launch_qr_panel(mi, bi, Ap, lda, tau + k + i0, w.Vs + (int64_t)i0 * ldvs, ldvs, w.Vt + i0, kOB, i0,
                                 w.xch, info, s);
            // G(0:i0+bi, i0:i0+bi) := -V^T V_p over the rows where V_p is not zero
            if (!rc) rc = launch_fill0(i0 + bi, bi, w.G + (int64_t)i0 * kOB, kOB, s);
            if (!rc)
                rc = gemm_long(i0 + bi, bi, mi, w.Vs + i0, ldvs, w.Vs + i0 + (int64_t)i0 * ldvs, ldvs,
                               w.G + (int64_t)i0 * kOB, kOB, w.split, info, s);
            if (!rc) rc = launch_qr_t(i0, i0 + bi, w.G, kOB, tau + k, w.T, kOB, info, s);
            // the block's columns right of the panel
            if (!rc)
                rc = apply_qt(w, mi, nbk - i0 - bi, bi, w.Vs + i0 + (int64_t)i0 * ldvs, w.Vt + i0 + (int64_t)i0 * kOB,
                              w.T + i0 + (int64_t)i0 * kOB, Ap + (int64_t)bi * lda, lda, info, s);
            if (rc) return rc;
        }
        // the columns right of the block
        rc = apply_qt(w, mk, n - k - nbk, nbk, w.Vs, w.Vt, w.T, A + k + (k + nbk) * lda, lda, info, s);
        if (rc) return rc;
    }
    return FLAME_OK;
}

}  // namespace flame
