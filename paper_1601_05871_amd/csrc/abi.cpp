// C ABI entry points (include/flame.h): host-side argument checks, option
// defaults, dispatch.  Nothing is enqueued when a check fails.
#include <cmath>
#include <cstring>

#include "flame_internal.h"

using namespace flame;

namespace {

constexpr int kMaxNb = 512;     // block size of the factorization loops
constexpr int kMaxBlockOp = 256;  // order of the exposed block operations
// Block size when neither the caller nor the selector names one: the RIGHT
// loop then runs 512 while more than 8192 columns remain, 256 down to 6144
// and 128 in the tail (the schedule measured fastest at n = 16384).
constexpr int kDefaultNb = 512;

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// Fills defaults; returns 0 or -5 (bad option field).
int normalize_opts(const flame_opts_t *in, int32_t dtype, int64_t n, flame_opts_t *o) {
    if (in != nullptr)
        *o = *in;
    else
        std::memset(o, 0, sizeof(*o));
    if (o->variant < FLAME_VAR_AUTO || o->variant > FLAME_VAR_BY_BLOCKS) return -5;
    if (o->nb < 0 || o->nb > kMaxNb) return -5;
    if (o->trail < FLAME_TRAIL_NATIVE || o->trail > FLAME_TRAIL_BF16) return -5;
    if (o->lookahead < -1 || o->lookahead > 2) return -5;
    if (o->graph < 0 || o->graph > 1) return -5;
    if ((o->flags & ~(FLAME_OPT_FIXED_NB | FLAME_OPT_LOWER)) != 0) return -5;
    if (o->reserved[0] != 0 || o->reserved[1] != 0) return -5;
    if (o->variant == FLAME_VAR_AUTO) choose_variant(dtype, n, 1, o);
    if (o->nb == 0) o->nb = kDefaultNb;
    return 0;
}

// dtype FLAME_Z64: the complex Hermitian factorization (zfactor.cpp), the
// right-looking loop only, native precision, run without graph capture.
int factor_complex(int64_t n, void *A, int64_t lda, const flame_opts_t *opts, int32_t *info, void *stream) {
    flame_opts_t o;
    if (opts != nullptr)
        o = *opts;
    else
        std::memset(&o, 0, sizeof(o));
    if (o.variant < FLAME_VAR_AUTO || o.variant > FLAME_VAR_BY_BLOCKS) return -5;
    if (o.nb < 0 || o.nb > kMaxNb) return -5;
    if (o.trail < FLAME_TRAIL_NATIVE || o.trail > FLAME_TRAIL_BF16) return -5;
    if (o.lookahead < -1 || o.lookahead > 2) return -5;
    if (o.graph < 0 || o.graph > 1) return -5;
    if ((o.flags & ~(FLAME_OPT_FIXED_NB | FLAME_OPT_LOWER)) != 0) return -5;
    if (o.reserved[0] != 0 || o.reserved[1] != 0) return -5;
    if ((o.variant != FLAME_VAR_AUTO && o.variant != FLAME_VAR_RIGHT) || o.trail != FLAME_TRAIL_NATIVE)
        return FLAME_ERR_UNSUPPORTED;
    const int nb = o.nb == 0 ? 256 : o.nb;
    hipStream_t s = as_stream(stream);
    if ((o.flags & FLAME_OPT_LOWER) == 0) return zfactor(n, A, lda, nb, info, s);
    // lower storage (A = L L^H): the swapped triangles hold conj(A)'s upper
    // triangle, whose factor U_c gives L = U_c^T once swapped back
    int rc = launch_swap_triangles<zdouble>(n, static_cast<zdouble *>(A), lda, s);
    if (!rc) rc = zfactor(n, A, lda, nb, info, s);
    if (!rc) rc = launch_swap_triangles<zdouble>(n, static_cast<zdouble *>(A), lda, s);
    return rc;
}

}  // namespace

extern "C" {

int flame_factor(int32_t dtype, int64_t n, void *A, int64_t lda, const flame_opts_t *opts, int32_t *info,
                 void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32 && dtype != FLAME_Z64) return -1;
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return -2;
    if (A == nullptr && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (info == nullptr) return -6;
    if (dtype == FLAME_Z64) return factor_complex(n, A, lda, opts, info, stream);
    flame_opts_t o;
    int rc = normalize_opts(opts, dtype, n, &o);
    if (rc) return rc;
    if (o.trail != FLAME_TRAIL_NATIVE && (dtype != FLAME_F64 || o.variant != FLAME_VAR_RIGHT))
        return FLAME_ERR_UNSUPPORTED;
    if (o.variant == FLAME_VAR_BY_BLOCKS && dtype != FLAME_F64) return FLAME_ERR_UNSUPPORTED;
    if ((o.flags & FLAME_OPT_LOWER) == 0) return factor_dispatch(dtype, n, A, lda, o, info, as_stream(stream));
    // lower storage: the transpose's upper triangle, factored as usual
    hipStream_t s = as_stream(stream);
    o.flags &= ~FLAME_OPT_LOWER;
    rc = dtype == FLAME_F64 ? launch_swap_triangles<double>(n, static_cast<double *>(A), lda, s)
                            : launch_swap_triangles<float>(n, static_cast<float *>(A), lda, s);
    if (rc) return rc;
    rc = factor_dispatch(dtype, n, A, lda, o, info, s);
    if (rc) return rc;
    return dtype == FLAME_F64 ? launch_swap_triangles<double>(n, static_cast<double *>(A), lda, s)
                              : launch_swap_triangles<float>(n, static_cast<float *>(A), lda, s);
}

int flame_lu(int32_t dtype, int64_t n, void *A, int64_t lda, int32_t *info, void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return -2;
    if (A == nullptr && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (info == nullptr) return -5;
    if (dtype != FLAME_F64) return FLAME_ERR_UNSUPPORTED;
    return lu_factor(n, static_cast<double *>(A), lda, info, as_stream(stream));
}

int flame_qr(int32_t dtype, int64_t m, int64_t n, void *A, int64_t lda, void *tau, int32_t *info, void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (m < 0 || m > ((int64_t)1 << 31) - 1) return -2;
    if (n < 0 || n > m) return -3;
    if (A == nullptr && n > 0) return -4;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (tau == nullptr && n > 0) return -6;
    if (info == nullptr) return -7;
    if (dtype != FLAME_F64 || m > 131072) return FLAME_ERR_UNSUPPORTED;
    return qr_factor(m, n, static_cast<double *>(A), lda, static_cast<double *>(tau), info, as_stream(stream));
}

int flame_op_chol(int32_t dtype, int64_t n, void *A, int64_t lda, int32_t *info, int64_t info_base, void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (n < 0 || n > kMaxBlockOp) return -2;
    if (A == nullptr && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (info == nullptr) return -5;
    if (dtype == FLAME_F64)
        return launch_chol_block<double>((int)n, static_cast<double *>(A), lda, info, info_base, as_stream(stream));
    return launch_chol_block<float>((int)n, static_cast<float *>(A), lda, info, info_base, as_stream(stream));
}

int flame_op_trsm(int32_t dtype, int64_t b, int64_t m, const void *U, int64_t ldu, void *X, int64_t ldx,
                  void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (b < 0 || b > kMaxBlockOp) return -2;
    if (m < 0) return -3;
    if (U == nullptr && b > 0) return -4;
    if (ldu < (b > 1 ? b : 1)) return -5;
    if (X == nullptr && b > 0 && m > 0) return -6;
    if (ldx < (b > 1 ? b : 1)) return -7;
    if (dtype == FLAME_F64)
        return launch_trsm_panel<double>((int)b, m, static_cast<const double *>(U), ldu, static_cast<double *>(X),
                                         ldx, nullptr, as_stream(stream));
    return launch_trsm_panel<float>((int)b, m, static_cast<const float *>(U), ldu, static_cast<float *>(X), ldx,
                                    nullptr, as_stream(stream));
}

int flame_op_gemm_tn(int32_t dtype, int32_t trail, int32_t upper, int64_t mr, int64_t nc, int64_t k, const void *X,
                     int64_t ldx, const void *Y, int64_t ldy, void *C, int64_t ldc, void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (trail < FLAME_TRAIL_NATIVE || trail > FLAME_TRAIL_BF16) return -2;
    if (dtype == FLAME_F32 && trail != FLAME_TRAIL_NATIVE) return -2;
    if (mr < 0) return -3;
    if (nc < 0) return -4;
    if (k < 0) return -5;
    const bool any = mr > 0 && nc > 0;
    if (X == nullptr && any && k > 0) return -6;
    if (ldx < (k > 1 ? k : 1)) return -7;
    if (Y == nullptr && any && k > 0) return -8;
    if (ldy < (k > 1 ? k : 1)) return -9;
    if (C == nullptr && any) return -10;
    if (ldc < (mr > 1 ? mr : 1)) return -11;
    if (!any) return FLAME_OK;
    Prec p = Prec::F64;
    bool cd = true;
    if (dtype == FLAME_F32) {
        p = Prec::F32;
        cd = false;
    } else if (trail == FLAME_TRAIL_F32) {
        p = Prec::F32;
    } else if (trail == FLAME_TRAIL_BF16) {
        p = Prec::BF16;
    }
    return launch_gemm_tn(p, cd, upper != 0, mr, nc, k, X, ldx, Y, ldy, C, ldc, nullptr, as_stream(stream));
}

const char *flame_status_string(int status) {
    if (status < 0) return "invalid argument (the negated status is its 1-based position)";
    switch (status) {
        case FLAME_OK:
            return "success";
        case FLAME_ERR_HIP:
            return hipGetErrorString(last_hip_error());
        case FLAME_ERR_NOMEM:
            return "device workspace allocation failed";
        case FLAME_ERR_NOT_CONVERGED:
            return "iterative refinement did not reach the tolerance";
        case FLAME_ERR_UNSUPPORTED:
            return "unsupported combination of arguments";
        case FLAME_ERR_BREAKDOWN:
            return "the factorization broke down (not positive definite at the precision used)";
        default:
            return "unknown status";
    }
}

const char *flame_version(void) { return "flame-mi355x 0.1 (gfx950)"; }

}  // extern "C"
