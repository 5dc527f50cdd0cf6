// Householder QR (flame_qr), A = Q R for m x n, m >= n: the right-looking
// partitioned loop of Fig. "dense-chol" with QR's steps (the conclusion names
// QR among the factorizations the pattern carries over to), blocked twice:
//
//   for each outer block of 128 columns (the rows below it: V, T, the update):
//     for each panel of 32 columns inside it:
//       factor the panel into reflectors                   k_qr_panel
//       V^T V_p and V_p^T C (C: the block's columns right
//         of the panel), as slices of one launch           k_qr_skinny
//       T's new columns from the Gram slices and tau       k_qr_gt
//       Y := T_pp^T V_p^T C from the slices                k_qr_wy
//       C -= V_p Y                                         matrix cores
//     the next block's columns: the same with the block's V and T
//     the columns beyond it (side stream, one block ahead):
//       W := 0 - V^T C (split over K), Y := 0 - T^T W, C -= V Y
//
// Q^T C = (I - V T V^T)^T C = C - V T^T V^T C; V is kept twice, as columns
// (Vs, for V^T C) and as rows (Vt, for V Y), so that the large products are
// the trailing-update kernel's C -= X^T Y.
#include <algorithm>

#include "flame_internal.h"

namespace flame {

int qr_panel_rows();
int launch_qr_fill_empty(int64_t count, double *p, hipStream_t s);
int launch_qr_panel(int64_t m, int b, double *A, int64_t lda, double *tau, double *Vs, int64_t ldvs, double *Vt,
                    int64_t ldvt, int64_t ro, double *xch, double *xnext, int32_t *info, hipStream_t s);
int launch_qr_zero2(int64_t rows, int64_t cols, double *d0, double *d1, int64_t ldd, hipStream_t s);
int qr_slices(int64_t K, int smax, int64_t *kc);
int launch_qr_skinny(int S1, int M1, int N1, int64_t K1, int64_t kc1, const double *X1, int64_t ldx1,
                     const double *Y1, int64_t ldy1, double *part1, int S2, int M2, int N2, int64_t K2, int64_t kc2,
                     const double *X2, int64_t ldx2, const double *Y2, int64_t ldy2, double *part2,
                     const int32_t *info, hipStream_t s);
int launch_qr_gt(int S, int j0, int j1, const double *part, const double *tau, double *T, int64_t ldt,
                 const int32_t *info, hipStream_t s);
int launch_qr_wy(int S, int kb, int nc, const double *part, const double *T, int64_t ldt, double *Y,
                 const int32_t *info, hipStream_t s);

namespace {

constexpr int kIB = 32;        // panel
constexpr int kOB = 128;       // outer block
constexpr int kSideCus = 16;   // compute units the side stream's large product leaves to the panels
constexpr int kSlices = 128;   // K slices of a skinny product at most
constexpr int kGramSlices = 32;  // (k_qr_gt adds at most 32)

struct QrBuf {  // one outer block's reflectors (two of them: the side stream reads one while the next is built)
    double *Vs;  // m x kOB, ld ldvs
    double *Vt;  // kOB x m, ld kOB
    double *T;   // kOB x kOB
};

struct QrWork {
    QrBuf buf[2];
    int64_t ldvs;
    double *W[2], *Y[2];  // kOB x n, ld kOB: [0] main stream, [1] side stream
    double *split;        // split-K partial products of the side stream
    double *part;         // skinny-product slices (main stream)
    double *gpart;        // Gram slices of a panel (main stream)
    double *xch[2];  // panel exchange slots, alternate panels
    int64_t nxch;
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
// at V (ld ldvs), its rows at Vt (ld kOB), T (kb x kb) at Tb (ld kOB).
// nc <= kOB (main stream): Y := T^T V^T C from the slices of the skinny
// product V^T C, then C -= (V^T)^T Y.
int apply_qt_narrow(const QrWork &w, int64_t mr, int64_t nc, int kb, const double *V, const double *Vt,
                    const double *Tb, double *C, int64_t ldc, const int32_t *info, hipStream_t s) {
    if (nc <= 0) return FLAME_OK;
    int64_t kc = 0;
    const int S = qr_slices(mr, kSlices, &kc);
    int rc = launch_qr_skinny(S, kb, (int)nc, mr, kc, V, w.ldvs, C, ldc, w.part, 0, 0, 0, 0, 0, nullptr, 0, nullptr,
                              0, nullptr, info, s);
    if (!rc) rc = launch_qr_wy(S, kb, (int)nc, w.part, Tb, kOB, w.Y[0], info, s);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, mr, nc, kb, Vt, kOB, w.Y[0], kOB, C, ldc, info, s);
    return rc;
}

// The same for any nc (side stream): W := 0 - V^T C (split over K),
// Y := 0 - T^T W, C -= (V^T)^T Y.
int apply_qt_wide(const QrWork &w, int64_t mr, int64_t nc, int kb, const double *V, const double *Vt,
                  const double *Tb, double *C, int64_t ldc, const int32_t *info, hipStream_t s, int reserve_cus) {
    if (nc <= 0) return FLAME_OK;
    int rc = launch_qr_zero2(kb, nc, w.W[1], w.Y[1], kOB, s);
    if (!rc) rc = gemm_long(kb, nc, mr, V, w.ldvs, C, ldc, w.W[1], kOB, w.split, info, s);
    if (!rc) rc = launch_gemm_tn(Prec::F64, true, false, kb, nc, kb, Tb, kOB, w.W[1], kOB, w.Y[1], kOB, info, s);
    if (!rc)
        rc = launch_gemm_tn(Prec::F64, true, false, mr, nc, kb, Vt, kOB, w.Y[1], kOB, C, ldc, info, s, reserve_cus);
    return rc;
}

}  // namespace

static int qr_blocks(const QrWork &w, int64_t m, int64_t n, double *A, int64_t lda, double *tau, int32_t *info,
                     hipStream_t s, hipStream_t side, hipEvent_t ev_next, hipEvent_t ev_rest, bool *side_pending);

// Lookahead of one block: block k's update of the columns beyond block k + 1
// runs on the side stream while the main stream updates block k + 1's
// columns and factors its panels; before block k + 1's own updates the main
// stream waits for it.  The reflectors of consecutive blocks live in
// alternate buffers, so block k + 1's panels never overwrite what the side
// stream still reads.
int qr_factor(int64_t m, int64_t n, double *A, int64_t lda, double *tau, int32_t *info, hipStream_t s) {
    int rc = launch_zero_i32(info, 1, s);
    if (rc || n == 0) return rc;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    const int64_t pmax = (m + qr_panel_rows() - 1) / qr_panel_rows();
    const int64_t ldvs = (m + 1) / 2 * 2;  // even: 16-byte aligned columns
    const size_t xch = (size_t)kIB * pmax * kIB + (size_t)kIB * kIB;
    const size_t per_buf = (size_t)ldvs * kOB + (size_t)kOB * (size_t)m + (size_t)kOB * kOB;
    const size_t part = (size_t)kSlices * kOB * kOB, gpart = (size_t)kGramSlices * kOB * kIB;
    const size_t doubles = 2 * per_buf + 4 * (size_t)kOB * (size_t)n + part + gpart + 2 * xch;
    void *ws = nullptr;
    rc = ctx_workspace(ctx, kWsQr, doubles * sizeof(double), &ws);
    if (rc) return rc;
    void *split = nullptr;
    rc = ctx_workspace(ctx, kWsQrSplit, splitk_workspace_bytes(), &split);
    if (rc) return rc;
    QrWork w;
    double *p = static_cast<double *>(ws);
    for (int b = 0; b < 2; ++b) {
        w.buf[b].Vs = p;
        w.buf[b].Vt = p + (size_t)ldvs * kOB;
        w.buf[b].T = w.buf[b].Vt + (size_t)kOB * m;
        p += per_buf;
    }
    w.ldvs = ldvs;
    for (int q = 0; q < 2; ++q) {
        w.W[q] = p;
        w.Y[q] = p + (size_t)kOB * n;
        p += 2 * (size_t)kOB * n;
    }
    w.part = p;
    w.gpart = p + part;
    w.xch[0] = w.gpart + gpart;
    w.xch[1] = w.xch[0] + xch;
    w.nxch = (int64_t)xch;
    rc = launch_qr_fill_empty(2 * w.nxch, w.xch[0], s);
    if (rc) return rc;
    w.split = static_cast<double *>(split);
    hipStream_t side = ctx_side_stream(ctx);
    hipEvent_t ev_next = ctx_event(ctx, 2);  // main: the next block's columns updated, V and T final
    hipEvent_t ev_rest = ctx_event(ctx, 3);  // side: the columns beyond the next block updated
    bool side_pending = false;
    rc = qr_blocks(w, m, n, A, lda, tau, info, s, side, ev_next, ev_rest, &side_pending);
    // the side stream's last update joins the caller's stream (also after an error)
    if (side_pending) FLAME_HIP(hipStreamWaitEvent(s, ev_rest, 0));
    return rc;
}

static int qr_blocks(const QrWork &w, int64_t m, int64_t n, double *A, int64_t lda, double *tau, int32_t *info,
                     hipStream_t s, hipStream_t side, hipEvent_t ev_next, hipEvent_t ev_rest, bool *side_pending) {
    const int64_t ldvs = w.ldvs;
    int rc = FLAME_OK;
    int64_t np = 0;  // panels so far (which exchange buffer)
    for (int64_t k = 0, blk = 0; k < n; k += kOB, ++blk) {
        const QrBuf &B = w.buf[blk & 1];
        const int nbk = (int)std::min<int64_t>(kOB, n - k);
        const int64_t mk = m - k;
        for (int i0 = 0; i0 < nbk; i0 += kIB) {
            const int bi = std::min(kIB, nbk - i0);
            const int64_t mi = mk - i0;
            double *Ap = A + (k + i0) + (k + i0) * lda;
            rc = launch_qr_panel(mi, bi, Ap, lda, tau + k + i0, B.Vs + (int64_t)i0 * ldvs, ldvs, B.Vt + i0, kOB, i0,
                                 w.xch[np & 1], w.xch[(np + 1) & 1], info, s);
            ++np;
            // in one launch: V^T V_p (rows i0..: V_p is zero above) and, for
            // the block's columns right of the panel, V_p^T C
            const int64_t nc = nbk - i0 - bi;
            const double *Vp = B.Vs + i0 + (int64_t)i0 * ldvs;
            double *Cp = Ap + (int64_t)bi * lda;
            int64_t kc = 0, kcw = 0;
            const int S = qr_slices(mi, kGramSlices, &kc);
            const int Sw = nc > 0 ? qr_slices(mi, kSlices, &kcw) : 0;
            if (!rc)
                rc = launch_qr_skinny(S, i0 + bi, bi, mi, kc, B.Vs + i0, ldvs, Vp, ldvs, w.gpart, Sw, bi, (int)nc, mi,
                                      kcw, Vp, ldvs, Cp, lda, w.part, info, s);
            // T's new columns, then C := (I - V_p T_pp^T V_p^T) C
            if (!rc) rc = launch_qr_gt(S, i0, i0 + bi, w.gpart, tau + k, B.T, kOB, info, s);
            if (!rc && nc > 0)
                rc = launch_qr_wy(Sw, bi, (int)nc, w.part, B.T + i0 + (int64_t)i0 * kOB, kOB, w.Y[0], info, s);
            if (!rc && nc > 0)
                rc = launch_gemm_tn(Prec::F64, true, false, mi, nc, bi, B.Vt + i0 + (int64_t)i0 * kOB, kOB, w.Y[0],
                                    kOB, Cp, lda, info, s);
            if (rc) return rc;
        }
        const int64_t rest = n - k - nbk;
        if (rest == 0) break;
        // the previous block's side update covered these columns too
        if (*side_pending) FLAME_HIP(hipStreamWaitEvent(s, ev_rest, 0));
        *side_pending = false;
        const int64_t nn = std::min<int64_t>(kOB, rest), far = rest - nn;
        double *C = A + k + (k + nbk) * lda;
        rc = apply_qt_narrow(w, mk, nn, nbk, B.Vs, B.Vt, B.T, C, lda, info, s);
        if (rc) return rc;
        if (far > 0) {
            FLAME_HIP(hipEventRecord(ev_next, s));
            FLAME_HIP(hipStreamWaitEvent(side, ev_next, 0));
            rc = apply_qt_wide(w, mk, far, nbk, B.Vs, B.Vt, B.T, C + nn * lda, lda, info, side, kSideCus);
            if (rc) return rc;
            FLAME_HIP(hipEventRecord(ev_rest, side));
            *side_pending = true;
        }
    }
    return FLAME_OK;
}

}  // namespace flame
