// flame_solve: A X = B with A = U^T U, and FP64 iterative refinement against
// the original matrix A0 (for factors computed with low-precision trailing
// updates).  Every step runs on the GPU; only eta crosses to the host.
#include <cmath>
#include <vector>

#include "flame_internal.h"

using namespace flame;

namespace {

constexpr int kTb = 128;     // row block of the single-launch solves
constexpr int kFastRhs = 8;  // right-hand sides handled column by column

template <typename T>
int plain_solve(int64_t n, int64_t nrhs, const T *U, int64_t ldu, T *B, int64_t ldb, hipStream_t s) {
    int rc = launch_trsv_fwd<T>(n, nrhs, U, ldu, B, ldb, s);
    if (rc) return rc;
    return launch_trsv_bwd<T>(n, nrhs, U, ldu, B, ldb, s);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// FP64 workspace of the single-launch path, carved from one slot.
struct FastWs {
    double *Dt = nullptr;       // nblk blocks of 128 x 128: U_qq^{-T}
    double *b0 = nullptr;       // n x nrhs copy of the right-hand sides
    double *r = nullptr;        // n x nrhs residual / correction
    double *rowsums = nullptr;  // n
    double *eta = nullptr;      // nrhs + 1
    double *part = nullptr;     // residual partials
    int32_t *flags = nullptr;   // nblk
    int32_t *err = nullptr;     // 1
};

int fast_ws(int64_t n, int64_t nrhs, bool refine, FastWs *w) {
    const int64_t nblk = (n + kTb - 1) / kTb;
    size_t off[8], total = 0;
    const size_t sizes[8] = {
        (size_t)nblk * kTb * kTb * sizeof(double),
        refine ? (size_t)n * nrhs * sizeof(double) : 0,
        refine ? (size_t)n * nrhs * sizeof(double) : 0,
        refine ? (size_t)n * sizeof(double) : 0,
        refine ? (size_t)(nrhs + 1) * sizeof(double) : 0,
        refine ? residual_workspace_doubles(n, nrhs) * sizeof(double) : 0,
        (size_t)nblk * sizeof(int32_t),
        sizeof(int32_t),
    };
    for (int k = 0; k < 8; ++k) {
        off[k] = total;
        total += align256(sizes[k]);
    }
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    void *base = nullptr;
    int rc = ctx_workspace(ctx, kWsSolve, total, &base);
    if (rc) return rc;
    char *b = static_cast<char *>(base);
    w->Dt = reinterpret_cast<double *>(b + off[0]);
    w->b0 = reinterpret_cast<double *>(b + off[1]);
    w->r = reinterpret_cast<double *>(b + off[2]);
    w->rowsums = reinterpret_cast<double *>(b + off[3]);
    w->eta = reinterpret_cast<double *>(b + off[4]);
    w->part = reinterpret_cast<double *>(b + off[5]);
    w->flags = reinterpret_cast<int32_t *>(b + off[6]);
    w->err = reinterpret_cast<int32_t *>(b + off[7]);
    return FLAME_OK;
}

// Inverses of the 128 x 128 diagonal blocks (once per call) and a cleared
// error flag.
int fast_prepare(int64_t n, const double *U, int64_t ldu, const FastWs &w, hipStream_t s) {
    const int64_t nblk = (n + kTb - 1) / kTb;
    int rc = launch_identity_blocks(nblk, kTb, w.Dt, s);
    if (rc) return rc;
    rc = launch_diag_inverse_t(n, kTb, U, ldu, w.Dt, s);
    if (rc) return rc;
    return launch_zero_i32(w.err, 1, s);
}

int fast_solve(int64_t n, int64_t nrhs, const double *U, int64_t ldu, double *B, int64_t ldb, const FastWs &w,
               hipStream_t s) {
    for (int64_t c = 0; c < nrhs; ++c) {
        int rc = launch_trsv1(true, n, U, ldu, w.Dt, B + c * ldb, w.flags, w.err, s);
        if (rc) return rc;
        rc = launch_trsv1(false, n, U, ldu, w.Dt, B + c * ldb, w.flags, w.err, s);
        if (rc) return rc;
    }
    return FLAME_OK;
}

}  // namespace

extern "C" int flame_solve(int32_t dtype, int64_t n, int64_t nrhs, const void *U, int64_t ldu, void *B, int64_t ldb,
                           const flame_refine_t *refine, flame_solve_report_t *report, void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (n < 0) return -2;
    if (nrhs < 0 || nrhs > 65535 * 8) return -3;
    if (U == nullptr && n > 0) return -4;
    if (ldu < (n > 1 ? n : 1)) return -5;
    if (B == nullptr && n > 0 && nrhs > 0) return -6;
    if (ldb < (n > 1 ? n : 1)) return -7;
    if (refine != nullptr) {
        if (dtype != FLAME_F64) return FLAME_ERR_UNSUPPORTED;
        if ((refine->A0 == nullptr && n > 0) || refine->lda0 < (n > 1 ? n : 1) || refine->max_iter < 0 ||
            !(refine->tol >= 0.0))
            return -8;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 0 || nrhs == 0) {
        if (report) {
            report->iters = 0;
            report->eta_max = 0.0;
        }
        return FLAME_OK;
    }
    const bool fast = dtype == FLAME_F64 && nrhs <= kFastRhs;
    if (refine == nullptr) {
        if (fast) {
            FastWs w;
            int rc = fast_ws(n, nrhs, false, &w);
            if (rc) return rc;
            const double *Ud = static_cast<const double *>(U);
            rc = fast_prepare(n, Ud, ldu, w, s);
            if (rc) return rc;
            return fast_solve(n, nrhs, Ud, ldu, static_cast<double *>(B), ldb, w, s);
        }
        if (dtype == FLAME_F64)
            return plain_solve<double>(n, nrhs, static_cast<const double *>(U), ldu, static_cast<double *>(B), ldb, s);
        return plain_solve<float>(n, nrhs, static_cast<const float *>(U), ldu, static_cast<float *>(B), ldb, s);
    }

    const double *Ud = static_cast<const double *>(U);
    double *X = static_cast<double *>(B);
    double eta_h = INFINITY;
    int32_t err_h = 0;
    int it = 0;
    if (fast) {
        // single-launch solves, tiled residual
        FastWs w;
        int rc = fast_ws(n, nrhs, true, &w);
        if (rc) return rc;
        rc = fast_prepare(n, Ud, ldu, w, s);
        if (rc) return rc;
        rc = launch_copy_cols(n, nrhs, X, ldb, w.b0, n, s);
        if (rc) return rc;
        rc = fast_solve(n, nrhs, Ud, ldu, X, ldb, w, s);
        if (rc) return rc;
        for (;; ++it) {
            rc = launch_residual_tiled(n, nrhs, refine->A0, refine->lda0, X, ldb, w.b0, n, w.r, n,
                                       it == 0 ? w.rowsums : nullptr, w.part, s);
            if (rc) return rc;
            rc = launch_eta_full(n, nrhs, w.r, n, X, ldb, w.b0, n, w.rowsums, w.eta, s);
            if (rc) return rc;
            FLAME_HIP(hipMemcpyAsync(&eta_h, w.eta + nrhs, sizeof(double), hipMemcpyDeviceToHost, s));
            FLAME_HIP(hipMemcpyAsync(&err_h, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            FLAME_HIP(hipStreamSynchronize(s));
            if (err_h != 0) return FLAME_ERR_HIP;  // a solve gave up waiting (results are NaN)
            if (eta_h <= refine->tol || it >= refine->max_iter) break;
            rc = fast_solve(n, nrhs, Ud, ldu, w.r, n, w, s);
            if (rc) return rc;
            rc = launch_axpy_cols(n, nrhs, w.r, n, X, ldb, s);
            if (rc) return rc;
        }
    } else {
        // workspace: b (copy of the right-hand sides), r / d, row sums, eta
        DevCtx *ctx = ctx_for_current_device();
        if (ctx == nullptr) return FLAME_ERR_HIP;
        const size_t colbytes = (size_t)n * sizeof(double);
        const size_t need = 2 * colbytes * (size_t)nrhs + colbytes + (size_t)(nrhs + 1) * sizeof(double) + 256;
        void *ws = nullptr;
        int rc = ctx_workspace(ctx, kWsSolve, need, &ws);
        if (rc) return rc;
        double *b0 = static_cast<double *>(ws);
        double *r = b0 + (size_t)n * nrhs;
        double *rowsums = r + (size_t)n * nrhs;
        double *eta = rowsums + n;
        rc = launch_copy_cols(n, nrhs, X, ldb, b0, n, s);
        if (rc) return rc;
        rc = plain_solve<double>(n, nrhs, Ud, ldu, X, ldb, s);
        if (rc) return rc;
        for (;; ++it) {
            rc = launch_residual(n, nrhs, refine->A0, refine->lda0, X, ldb, b0, n, r, n, rowsums, it == 0, s);
            if (rc) return rc;
            rc = launch_eta_full(n, nrhs, r, n, X, ldb, b0, n, rowsums, eta, s);
            if (rc) return rc;
            FLAME_HIP(hipMemcpyAsync(&eta_h, eta + nrhs, sizeof(double), hipMemcpyDeviceToHost, s));
            FLAME_HIP(hipStreamSynchronize(s));
            if (eta_h <= refine->tol || it >= refine->max_iter) break;
            rc = plain_solve<double>(n, nrhs, Ud, ldu, r, n, s);
            if (rc) return rc;
            rc = launch_axpy_cols(n, nrhs, r, n, X, ldb, s);
            if (rc) return rc;
        }
    }
    if (report) {
        report->iters = it;
        report->eta_max = eta_h;
    }
    return (eta_h <= refine->tol) ? FLAME_OK : FLAME_ERR_NOT_CONVERGED;
}
