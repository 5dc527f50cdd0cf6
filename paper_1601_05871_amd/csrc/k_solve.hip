// Triangular solves with the factor and the FP64 residual used by iterative
// refinement.  The paper's use of the factor is the solution of SPD systems
// (as a preconditioner); A X = B with A = U^T U is solved as U^T Y = B
// (forward substitution) and U X = Y (back substitution).
//
// Both solves are blocked by `kSolveBlock` rows: a diagonal-block kernel (one
// lane per right-hand side) and an update of the remaining rows with the
// panel of U just used, so U is streamed from HBM once per solve.
#include "flame_internal.h"

namespace flame {

constexpr int kSolveBlock = 128;

// X := triu(U)^{-1} X for a w x w diagonal block (w <= 128), back
// substitution, one lane per column of X.
template <typename T>
__global__ __launch_bounds__(64) void k_trsm_upper_n(int w, int64_t nrhs, const T *__restrict__ U, int64_t ldu,
                                                     T *__restrict__ X, int64_t ldx) {
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= nrhs) return;
    T *xc = X + c * ldx;
    for (int t = w - 1; t >= 0; --t) {
        T acc = xc[t];
        for (int q = t + 1; q < w; ++q) acc = acc - U[t + (int64_t)q * ldu] * xc[q];
        xc[t] = acc / U[t + (int64_t)t * ldu];
    }
}

// Y(i, c) -= sum_q P(i, q) Z(q, c): P is M x w (column-major, ld ldp), Z is
// w x nrhs.  One thread per row i, loop over the right-hand sides.
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_n(int64_t M, int w, int64_t nrhs, const T *__restrict__ P,
                                                int64_t ldp, const T *__restrict__ Z, int64_t ldz,
                                                T *__restrict__ Y, int64_t ldy) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M) return;
    for (int64_t c = blockIdx.y; c < nrhs; c += gridDim.y) {
        T acc = 0;
        for (int q = 0; q < w; ++q) acc += P[i + (int64_t)q * ldp] * Z[q + c * ldz];
        Y[i + c * ldy] -= acc;
    }
}

template <typename T>
int launch_trsv_fwd(int64_t n, int64_t nrhs, const T *U, int64_t ldu, T *B, int64_t ldb, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    const Prec p = sizeof(T) == 8 ? Prec::F64 : Prec::F32;
    for (int64_t j0 = 0; j0 < n; j0 += kSolveBlock) {
        const int64_t w = std::min<int64_t>(kSolveBlock, n - j0);
        int rc = launch_trsm_panel<T>((int)w, nrhs, U + j0 + j0 * ldu, ldu, B + j0, ldb, nullptr, s);
        if (rc) return rc;
        const int64_t rest = n - j0 - w;
        if (rest > 0) {
            // B(j0+w:n, :) -= U(j0:j0+w, j0+w:n)^T B(j0:j0+w, :)
            rc = launch_gemm_tn(p, sizeof(T) == 8, false, rest, nrhs, w, U + j0 + (j0 + w) * ldu, ldu, B + j0, ldb,
                                B + j0 + w, ldb, nullptr, s);
            if (rc) return rc;
        }
    }
    return FLAME_OK;
}

template <typename T>
int launch_trsv_bwd(int64_t n, int64_t nrhs, const T *U, int64_t ldu, T *B, int64_t ldb, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    const int64_t nblk = (n + kSolveBlock - 1) / kSolveBlock;
    for (int64_t bi = nblk - 1; bi >= 0; --bi) {
        const int64_t j0 = bi * kSolveBlock;
        const int64_t w = std::min<int64_t>(kSolveBlock, n - j0);
        hipLaunchKernelGGL(k_trsm_upper_n<T>, dim3((unsigned)((nrhs + 63) / 64)), dim3(64), 0, s, (int)w, nrhs,
                           U + j0 + j0 * ldu, ldu, B + j0, ldb);
        FLAME_CHECK_LAUNCH();
        if (j0 > 0) {
            // B(0:j0, :) -= U(0:j0, j0:j0+w) B(j0:j0+w, :)
            const unsigned gy = (unsigned)std::min<int64_t>(nrhs, 64);
            hipLaunchKernelGGL(k_gemv_n<T>, dim3((unsigned)((j0 + 255) / 256), gy), dim3(256), 0, s, j0, (int)w,
                               nrhs, U + j0 * ldu, ldu, B + j0, ldb, B, ldb);
            FLAME_CHECK_LAUNCH();
        }
    }
    return FLAME_OK;
}

template int launch_trsv_fwd<double>(int64_t, int64_t, const double *, int64_t, double *, int64_t, hipStream_t);
template int launch_trsv_fwd<float>(int64_t, int64_t, const float *, int64_t, float *, int64_t, hipStream_t);
template int launch_trsv_bwd<double>(int64_t, int64_t, const double *, int64_t, double *, int64_t, hipStream_t);
template int launch_trsv_bwd<float>(int64_t, int64_t, const float *, int64_t, float *, int64_t, hipStream_t);

// ---- residual R = B - A0 X, A0 symmetric from its upper triangle ------------
// The row-block symmetric product of k_refine.hip (R = B - A0 X, |A0| row
// sums with it when asked for).
int launch_residual(int64_t n, int64_t nrhs, const double *A0, int64_t lda0, const double *X, int64_t ldx,
                    const double *B, int64_t ldb, double *R, int64_t ldr, double *rowsums, bool want_rowsums,
                    hipStream_t s) {
    return launch_symm(n, nrhs, -1.0, A0, lda0, X, ldx, 1.0, B, ldb, R, ldr, want_rowsums ? rowsums : nullptr, s);
}

// eta[c] = ||r_c||_inf / (||A0||_inf ||x_c||_inf + ||b_c||_inf); eta[nrhs] =
// max over c.  One workgroup, deterministic reductions.
__global__ __launch_bounds__(256) void k_eta(int64_t n, int64_t nrhs, const double *__restrict__ R, int64_t ldr,
                                             const double *__restrict__ X, int64_t ldx, const double *__restrict__ B,
                                             int64_t ldb, const double *__restrict__ rowsums,
                                             double *__restrict__ eta) {
    __shared__ double red[3][256];
    __shared__ double anorm;
    const int tid = threadIdx.x;
    double m = 0.0;
    for (int64_t i = tid; i < n; i += 256) m = fmax(m, rowsums[i]);
    red[0][tid] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) red[0][tid] = fmax(red[0][tid], red[0][tid + st]);
        __syncthreads();
    }
    if (tid == 0) anorm = red[0][0];
    __syncthreads();
    double emax = 0.0;
    for (int64_t c = 0; c < nrhs; ++c) {
        double mr = 0.0, mx = 0.0, mb = 0.0;
        for (int64_t i = tid; i < n; i += 256) {
            mr = fmax(mr, fabs(R[i + c * ldr]));
            mx = fmax(mx, fabs(X[i + c * ldx]));
            mb = fmax(mb, fabs(B[i + c * ldb]));
        }
        __syncthreads();
        red[0][tid] = mr;
        red[1][tid] = mx;
        red[2][tid] = mb;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st) {
                red[0][tid] = fmax(red[0][tid], red[0][tid + st]);
                red[1][tid] = fmax(red[1][tid], red[1][tid + st]);
                red[2][tid] = fmax(red[2][tid], red[2][tid + st]);
            }
            __syncthreads();
        }
        if (tid == 0) {
            const double den = anorm * red[1][0] + red[2][0];
            const double e = den > 0.0 ? red[0][0] / den : (red[0][0] > 0.0 ? INFINITY : 0.0);
            eta[c] = e;
            emax = fmax(emax, e);
        }
    }
    if (tid == 0) eta[nrhs] = emax;
}

int launch_eta_full(int64_t n, int64_t nrhs, const double *R, int64_t ldr, const double *X, int64_t ldx,
                    const double *B, int64_t ldb, const double *rowsums, double *eta, hipStream_t s) {
    hipLaunchKernelGGL(k_eta, dim3(1), dim3(256), 0, s, n, nrhs, R, ldr, X, ldx, B, ldb, rowsums, eta);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

__global__ void k_axpy_cols(int64_t n, int64_t nrhs, const double *__restrict__ D, int64_t ldd,
                            double *__restrict__ X, int64_t ldx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n) X[i + c * ldx] += D[i + c * ldd];
}

int launch_axpy_cols(int64_t n, int64_t nrhs, const double *D, int64_t ldd, double *X, int64_t ldx,
                     hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, s, n, nrhs, D,
                       ldd, X, ldx);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

__global__ void k_copy_cols(int64_t n, const double *__restrict__ S, int64_t lds, double *__restrict__ D,
                            int64_t ldd) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n) D[i + c * ldd] = S[i + c * lds];
}

int launch_copy_cols(int64_t n, int64_t nrhs, const double *S, int64_t lds, double *D, int64_t ldd,
                     hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, s, n, S, lds,
                       D, ldd);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
