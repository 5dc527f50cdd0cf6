// flame_solve: A X = B with A = U^T U, and FP64 refinement against the
// original matrix A0 for factors computed with low-precision trailing
// updates.  flame_solve_mixed: the whole mixed-precision solve (scaling,
// low-precision factorization with shifted retries, refinement).  Every step
// runs on the GPU; only eta and info cross to the host.
//
// Refinement methods (the paper factors A to solve SPD systems, using the
// factor as a preconditioner; how the low-precision factor is corrected is
// not in the paper):
//   IR   classical iterative refinement, x += (U^T U)^{-1} (b - A0 x).  Each
//        step multiplies the error by about ||I - (U^T U)^{-1} A0||, so it
//        converges only while kappa(A0) u_low is well below 1.
//   CG   conjugate gradients on A0 x = b with the preconditioner M = U^T U
//        (A0 and M are SPD), started from the current x.  The recursive
//        residual decides when to look at the true one: when its eta reaches
//        tol the true residual b - A0 x is formed; if that eta is still above
//        tol the iteration restarts from it.
//   AUTO IR while eta at least halves per step, then CG from the current x.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "flame_internal.h"

using namespace flame;

namespace {

constexpr int kTb = 128;  // row block of the single-launch solves
// Right-hand sides solved column by column with the one-column kernels (n =
// 16384: 1.63 ms per column for both directions); from 3 columns on the
// matrix-core chain solves are faster (4.3 ms for 16 columns, 11.5 ms for 64).
constexpr int kColumnRhs = 2;
// Right-hand sides of the tiled residual (more use the row-block product).
constexpr int kTiledRhs = 8;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Named buffers carved from one workspace slot.
class Carver {
   public:
    size_t add(size_t bytes) {
        const size_t o = total_;
        total_ += align256(bytes);
        return o;
    }
    size_t total() const { return total_ == 0 ? 256 : total_; }

   private:
    size_t total_ = 0;
};

struct SolveWs {
    bool fast = false;   // nrhs <= kColumnRhs: column-by-column solves
    bool tiled = false;  // nrhs <= kTiledRhs: tiled residual
    // FP64 solves
    double *Dt = nullptr;      // nblk blocks of 128 x 128: U_qq^{-T}
    int32_t *flags = nullptr;  // nblk, or one per row block and column chunk of the chain solves
    int32_t *err = nullptr;    // 1
    double *part = nullptr;    // partials of the tiled residual
    // refinement
    double *b0 = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;  // n x nrhs each
    double *rowsums = nullptr;                                                      // n
    double *eta = nullptr;                                                          // nrhs + 1
    double *rho = nullptr, *rho_old = nullptr, *pq = nullptr;                       // nrhs each
};

int solve_ws(int64_t n, int64_t nrhs, bool f64, bool refine, bool cg, SolveWs *w) {
    const int64_t nblk = (n + kTb - 1) / kTb;
    const bool fast = f64 && nrhs <= kColumnRhs;
    const bool tiled = f64 && nrhs <= kTiledRhs;
    const size_t col = (size_t)n * (size_t)nrhs * sizeof(double);
    Carver c;
    const size_t oDt = f64 ? c.add((size_t)nblk * kTb * kTb * sizeof(double)) : 0;
    const size_t nflags = fast ? (size_t)nblk : (size_t)trsm_chain_flags(n, nrhs);
    const size_t oFl = f64 ? c.add(nflags * sizeof(int32_t)) : 0;
    const size_t oEr = f64 ? c.add(sizeof(int32_t)) : 0;
    const size_t oPa = (tiled && refine) ? c.add(residual_workspace_doubles(n, nrhs) * sizeof(double)) : 0;
    const size_t oB0 = refine ? c.add(col) : 0;
    const size_t oR = refine ? c.add(col) : 0;
    const size_t oZ = cg ? c.add(col) : 0;
    const size_t oP = cg ? c.add(col) : 0;
    const size_t oQ = cg ? c.add(col) : 0;
    const size_t oRs = refine ? c.add((size_t)n * sizeof(double)) : 0;
    const size_t oEt = refine ? c.add((size_t)(nrhs + 1) * sizeof(double)) : 0;
    const size_t oRho = cg ? c.add((size_t)nrhs * sizeof(double)) : 0;
    const size_t oRho2 = cg ? c.add((size_t)nrhs * sizeof(double)) : 0;
    const size_t oPq = cg ? c.add((size_t)nrhs * sizeof(double)) : 0;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    void *base = nullptr;
    int rc = ctx_workspace(ctx, kWsSolve, c.total(), &base);
    if (rc) return rc;
    char *b = static_cast<char *>(base);
    auto D = [&](size_t o) { return reinterpret_cast<double *>(b + o); };
    w->fast = fast;
    w->tiled = tiled;
    if (f64) {
        w->Dt = D(oDt);
        w->flags = reinterpret_cast<int32_t *>(b + oFl);
        w->err = reinterpret_cast<int32_t *>(b + oEr);
    }
    if (tiled && refine) w->part = D(oPa);
    if (refine) {
        w->b0 = D(oB0);
        w->r = D(oR);
        w->rowsums = D(oRs);
        w->eta = D(oEt);
    }
    if (cg) {
        w->z = D(oZ);
        w->p = D(oP);
        w->q = D(oQ);
        w->rho = D(oRho);
        w->rho_old = D(oRho2);
        w->pq = D(oPq);
    }
    return FLAME_OK;
}

// Inverses of the 128 x 128 diagonal blocks (once per call) and a cleared
// error flag, for the single-launch solves.
int fast_prepare(int64_t n, const double *U, int64_t ldu, const SolveWs &w, hipStream_t s) {
    const int64_t nblk = (n + kTb - 1) / kTb;
    int rc = launch_identity_blocks(nblk, kTb, w.Dt, s);
    if (rc) return rc;
    rc = launch_diag_inverse_t(n, kTb, U, ldu, w.Dt, s);
    if (rc) return rc;
    return launch_zero_i32(w.err, 1, s);
}

// X := (U^T U)^{-1} X in place.
template <typename T>
int apply_inverse(int64_t n, int64_t nrhs, const T *U, int64_t ldu, T *X, int64_t ldx, const SolveWs &w,
                  hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        if (w.fast) {
            for (int64_t c = 0; c < nrhs; ++c) {
                int rc = launch_trsv1(true, n, U, ldu, w.Dt, X + c * ldx, w.flags, w.err, s);
                if (rc) return rc;
                rc = launch_trsv1(false, n, U, ldu, w.Dt, X + c * ldx, w.flags, w.err, s);
                if (rc) return rc;
            }
            return FLAME_OK;
        }
        int rc = launch_trsm_chain(true, n, nrhs, U, ldu, w.Dt, X, ldx, w.flags, w.err, s);
        if (rc) return rc;
        return launch_trsm_chain(false, n, nrhs, U, ldu, w.Dt, X, ldx, w.flags, w.err, s);
    }
    int rc = launch_trsv_fwd<T>(n, nrhs, U, ldu, X, ldx, s);
    if (rc) return rc;
    return launch_trsv_bwd<T>(n, nrhs, U, ldu, X, ldx, s);
}

// R := B - A0 X (B != nullptr) or R := A0 X (B == nullptr); row sums of |A0|
// when rowsums != nullptr.
int apply_a0(int64_t n, int64_t nrhs, const double *A0, int64_t lda0, const double *X, int64_t ldx, const double *B,
             double *R, double *rowsums, const SolveWs &w, hipStream_t s) {
    if (w.tiled) return launch_residual_tiled(n, nrhs, A0, lda0, X, ldx, B, n, R, n, rowsums, w.part, s);
    if (B != nullptr) return launch_symm(n, nrhs, -1.0, A0, lda0, X, ldx, 1.0, B, n, R, n, rowsums, s);
    return launch_symm(n, nrhs, 1.0, A0, lda0, X, ldx, 0.0, nullptr, n, R, n, rowsums, s);
}

// eta of the residual in w.r for the iterate X, read back to the host.
int eta_to_host(int64_t n, int64_t nrhs, const double *X, int64_t ldx, const SolveWs &w, double *eta_h,
                hipStream_t s) {
    int rc = launch_eta_full(n, nrhs, w.r, n, X, ldx, w.b0, n, w.rowsums, w.eta, s);
    if (rc) return rc;
    int32_t err_h = 0;
    FLAME_HIP(hipMemcpyAsync(eta_h, w.eta + nrhs, sizeof(double), hipMemcpyDeviceToHost, s));
    FLAME_HIP(hipMemcpyAsync(&err_h, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FLAME_HIP(hipStreamSynchronize(s));
    if (err_h != 0) return FLAME_ERR_HIP;  // a single-launch solve gave up waiting (results are NaN)
    return FLAME_OK;
}

int refine_solve(int64_t n, int64_t nrhs, const double *U, int64_t ldu, double *X, int64_t ldx,
                 const flame_refine_t &ref, flame_solve_report_t *report, hipStream_t s) {
    const bool may_cg = ref.method != FLAME_REFINE_IR;
    SolveWs w;
    int rc = solve_ws(n, nrhs, true, true, may_cg, &w);
    if (rc) return rc;
    rc = fast_prepare(n, U, ldu, w, s);
    if (rc) return rc;
    rc = launch_copy_cols(n, nrhs, X, ldx, w.b0, n, s);
    if (rc) return rc;
    rc = apply_inverse<double>(n, nrhs, U, ldu, X, ldx, w, s);
    if (rc) return rc;
    rc = apply_a0(n, nrhs, ref.A0, ref.lda0, X, ldx, w.b0, w.r, w.rowsums, w, s);
    if (rc) return rc;
    double eta = INFINITY, eta_prev = INFINITY;
    rc = eta_to_host(n, nrhs, X, ldx, w, &eta, s);
    if (rc) return rc;
    int method = (ref.method == FLAME_REFINE_CG) ? FLAME_REFINE_CG : FLAME_REFINE_IR;
    bool cg_first = true;  // the next CG step starts a new direction sequence from w.r
    int it = 0;
    while (eta > ref.tol && it < ref.max_iter) {
        if (method == FLAME_REFINE_IR && ref.method == FLAME_REFINE_AUTO && it > 0 && !(eta <= 0.5 * eta_prev)) {
            method = FLAME_REFINE_CG;
            cg_first = true;
        }
        eta_prev = eta;
        ++it;
        if (method == FLAME_REFINE_IR) {
            // x += (U^T U)^{-1} r; r = b - A0 x
            rc = apply_inverse<double>(n, nrhs, U, ldu, w.r, n, w, s);
            if (rc) return rc;
            rc = launch_axpy_cols(n, nrhs, w.r, n, X, ldx, s);
            if (rc) return rc;
            rc = apply_a0(n, nrhs, ref.A0, ref.lda0, X, ldx, w.b0, w.r, nullptr, w, s);
            if (rc) return rc;
            rc = eta_to_host(n, nrhs, X, ldx, w, &eta, s);
            if (rc) return rc;
            continue;
        }
        // one preconditioned CG step: z = M^{-1} r, rho = r.z, p = z + beta p,
        // q = A0 p, alpha = rho / p.q, x += alpha p, r -= alpha q
        rc = launch_copy_cols(n, nrhs, w.r, n, w.z, n, s);
        if (rc) return rc;
        rc = apply_inverse<double>(n, nrhs, U, ldu, w.z, n, w, s);
        if (rc) return rc;
        rc = launch_dot_cols(n, nrhs, w.r, n, w.z, n, w.rho, s);
        if (rc) return rc;
        rc = launch_cg_direction(n, nrhs, w.z, n, w.p, n, w.rho, w.rho_old, cg_first, s);
        if (rc) return rc;
        rc = apply_a0(n, nrhs, ref.A0, ref.lda0, w.p, n, nullptr, w.q, nullptr, w, s);
        if (rc) return rc;
        rc = launch_dot_cols(n, nrhs, w.p, n, w.q, n, w.pq, s);
        if (rc) return rc;
        rc = launch_cg_step(n, nrhs, X, ldx, w.r, n, w.p, n, w.q, n, w.rho, w.pq, s);
        if (rc) return rc;
        std::swap(w.rho, w.rho_old);
        cg_first = false;
        rc = eta_to_host(n, nrhs, X, ldx, w, &eta, s);
        if (rc) return rc;
        if (eta <= ref.tol) {
            // the recursive residual says done: check the true one
            rc = apply_a0(n, nrhs, ref.A0, ref.lda0, X, ldx, w.b0, w.r, nullptr, w, s);
            if (rc) return rc;
            rc = eta_to_host(n, nrhs, X, ldx, w, &eta, s);
            if (rc) return rc;
            cg_first = true;  // continue (if needed) from the true residual
        }
    }
    if (report) {
        report->iters = it;
        report->method = method;
        report->eta_max = eta;
    }
    return (eta <= ref.tol) ? FLAME_OK : FLAME_ERR_NOT_CONVERGED;
}

void report_clear(flame_solve_report_t *report) {
    if (report == nullptr) return;
    report->iters = 0;
    report->method = FLAME_REFINE_IR;
    report->eta_max = 0.0;
    report->shift = 0.0;
    report->factor_info = 0;
    report->attempts = 0;
}

int check_refine(const flame_refine_t *refine, int64_t n) {
    if ((refine->A0 == nullptr && n > 0) || refine->lda0 < (n > 1 ? n : 1) || refine->max_iter < 0 ||
        !(refine->tol >= 0.0) || refine->method < FLAME_REFINE_IR || refine->method > FLAME_REFINE_AUTO)
        return -8;
    return 0;
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
        const int rc = check_refine(refine, n);
        if (rc) return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    report_clear(report);
    if (n == 0 || nrhs == 0) return FLAME_OK;
    if (refine != nullptr)
        return refine_solve(n, nrhs, static_cast<const double *>(U), ldu, static_cast<double *>(B), ldb, *refine,
                            report, s);
    SolveWs w;
    int rc = solve_ws(n, nrhs, dtype == FLAME_F64, false, false, &w);
    if (rc) return rc;
    if (dtype == FLAME_F64) {
        const double *Ud = static_cast<const double *>(U);
        rc = fast_prepare(n, Ud, ldu, w, s);
        if (rc) return rc;
        // asynchronous: a solve whose bounded wait gave up writes NaN
        return apply_inverse<double>(n, nrhs, Ud, ldu, static_cast<double *>(B), ldb, w, s);
    }
    return apply_inverse<float>(n, nrhs, static_cast<const float *>(U), ldu, static_cast<float *>(B), ldb, w, s);
}

extern "C" int flame_solve_mixed(int64_t n, int64_t nrhs, const double *A0, int64_t lda0, double *W, int64_t ldw,
                                 double *B, int64_t ldb, const flame_mixed_opts_t *opts, flame_solve_report_t *report,
                                 void *stream) {
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return -1;
    if (nrhs < 0 || nrhs > 65535 * 8) return -2;
    if (A0 == nullptr && n > 0) return -3;
    if (lda0 < (n > 1 ? n : 1)) return -4;
    if (W == nullptr && n > 0) return -5;
    if (ldw < (n > 1 ? n : 1)) return -6;
    if (B == nullptr && n > 0 && nrhs > 0) return -7;
    if (ldb < (n > 1 ? n : 1)) return -8;
    if (opts == nullptr) return -9;
    const flame_mixed_opts_t &o = *opts;
    if (o.trail < FLAME_TRAIL_NATIVE || o.trail > FLAME_TRAIL_BF16 || o.nb < 0 || o.nb > 512 ||
        o.method < FLAME_REFINE_IR || o.method > FLAME_REFINE_AUTO || o.max_iter < 0 || !(o.tol >= 0.0) ||
        (o.scale != 0 && o.scale != 1) || o.max_shifts < 0 || o.max_shifts > 64 || !(o.shift >= 0.0) ||
        o.reserved != 0)
        return -9;
    hipStream_t s = static_cast<hipStream_t>(stream);
    report_clear(report);
    if (n == 0) return FLAME_OK;

    // workspace: scaling vector, breakdown column, factor info
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    void *base = nullptr;
    int rc = ctx_workspace(ctx, kWsMixed, align256((size_t)n * sizeof(double)) + 256, &base);
    if (rc) return rc;
    double *d = static_cast<double *>(base);
    int32_t *ints = reinterpret_cast<int32_t *>(static_cast<char *>(base) + align256((size_t)n * sizeof(double)));
    int32_t *bad = ints, *info = ints + 1;

    if (o.scale) {
        rc = launch_diag_scale(n, A0, lda0, d, bad, s);
        if (rc) return rc;
        int32_t bad_h = 0;
        FLAME_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FLAME_HIP(hipStreamSynchronize(s));
        if (bad_h != 0x7fffffff) {
            // A0 has a diagonal entry that is not positive: not SPD
            if (report) report->factor_info = bad_h;
            return FLAME_ERR_BREAKDOWN;
        }
    }
    // unit roundoff of the trailing products
    const double u = (o.trail == FLAME_TRAIL_BF16) ? std::ldexp(1.0, -8)
                     : (o.trail == FLAME_TRAIL_F32) ? std::ldexp(1.0, -24)
                                                    : std::ldexp(1.0, -53);
    // first shift: a small multiple of u relative to the (unit) diagonal
    const double mu1 = (o.shift > 0.0) ? o.shift : 2.0 * u;
    flame_opts_t fo{};
    fo.variant = FLAME_VAR_RIGHT;
    fo.nb = o.nb;
    fo.trail = o.trail;
    double mu = 0.0;
    int32_t info_h = 0;
    int attempt = 0;
    for (;; ++attempt) {
        rc = launch_scale_copy_upper(n, A0, lda0, W, ldw, o.scale ? d : nullptr, mu, s);
        if (rc) return rc;
        rc = flame_factor(FLAME_F64, n, W, ldw, &fo, info, stream);
        if (rc) return rc;
        FLAME_HIP(hipMemcpyAsync(&info_h, info, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FLAME_HIP(hipStreamSynchronize(s));
        if (info_h == 0 || attempt >= o.max_shifts) break;
        mu = (mu == 0.0) ? mu1 : 4.0 * mu;  // Higham & Pranesh: shift, then grow it on a further breakdown
    }
    if (report) {
        report->shift = mu;
        report->factor_info = info_h;
        report->attempts = attempt + 1;
    }
    if (info_h != 0) return FLAME_ERR_BREAKDOWN;
    if (o.scale) {
        rc = launch_unscale_cols(n, W, ldw, d, s);
        if (rc) return rc;
    }
    if (nrhs == 0) return FLAME_OK;
    flame_refine_t ref{};
    ref.A0 = A0;
    ref.lda0 = lda0;
    ref.tol = o.tol;
    ref.max_iter = o.max_iter;
    ref.method = o.method;
    flame_solve_report_t rep{};
    rc = refine_solve(n, nrhs, W, ldw, B, ldb, ref, &rep, s);
    if (report) {
        report->iters = rep.iters;
        report->method = rep.method;
        report->eta_max = rep.eta_max;
    }
    return rc;
}
