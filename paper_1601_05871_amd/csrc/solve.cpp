// flame_solve: A X = B with A = U^T U, and FP64 iterative refinement against
// the original matrix A0 (for factors computed with low-precision trailing
// updates).  Every step runs on the GPU; only eta crosses to the host.
#include <cmath>
#include <vector>

#include "flame_internal.h"

using namespace flame;

namespace {

template <typename T>
int plain_solve(int64_t n, int64_t nrhs, const T *U, int64_t ldu, T *B, int64_t ldb, hipStream_t s) {
    int rc = launch_trsv_fwd<T>(n, nrhs, U, ldu, B, ldb, s);
    if (rc) return rc;
    return launch_trsv_bwd<T>(n, nrhs, U, ldu, B, ldb, s);
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
    if (refine == nullptr) {
        if (dtype == FLAME_F64)
            return plain_solve<double>(n, nrhs, static_cast<const double *>(U), ldu, static_cast<double *>(B), ldb, s);
        return plain_solve<float>(n, nrhs, static_cast<const float *>(U), ldu, static_cast<float *>(B), ldb, s);
    }

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
    const double *Ud = static_cast<const double *>(U);
    double *X = static_cast<double *>(B);

    rc = launch_copy_cols(n, nrhs, X, ldb, b0, n, s);
    if (rc) return rc;
    rc = plain_solve<double>(n, nrhs, Ud, ldu, X, ldb, s);
    if (rc) return rc;
    double eta_h = INFINITY;
    int it = 0;
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
    if (report) {
        report->iters = it;
        report->eta_max = eta_h;
    }
    return (eta_h <= refine->tol) ? FLAME_OK : FLAME_ERR_NOT_CONVERGED;
}
