// Kernels of the FP64 refinement methods and of the mixed-precision solve
// driver: the symmetric product with many right-hand sides, per-column dot
// products and the conjugate-gradient vector updates, and the diagonal
// scaling (with an optional shift) applied before a low-precision
// factorization.  All arithmetic here is FP64.
#include "flame_internal.h"

namespace flame {

// ---- R := beta B + alpha A0 X, A0 symmetric from its upper triangle ----------
// Workgroup (I, c): rows 64 I .. 64 I + 63 of R, right-hand sides 64 c .. 64 c
// + 63.  The row block of the symmetric matrix is walked in 64-column chunks:
// chunk J comes from the upper tile (I, J) when I <= J (element (i, j) at
// A0[i + j lda0]) and from the transposed upper tile (J, I) otherwise, loaded
// so that consecutive lanes read consecutive addresses either way.  Wavefront
// w holds the 64 rows x 16 right-hand sides w*16 .. w*16+15 in registers; each
// chunk is 64 FP64 multiply-adds per right-hand side per row, the X operand a
// wave-uniform LDS broadcast.  Grid y = 0 also forms the |A0| row sums.  The
// order of the additions is fixed (chunk by chunk, column by column), so
// results are deterministic.
constexpr int kSymmRows = 64;
constexpr int kSymmRhs = 64;

__global__ __launch_bounds__(256) void k_symm_rows(int64_t n, int64_t nrhs, double alpha,
                                                   const double *__restrict__ A0, int64_t lda0,
                                                   const double *__restrict__ X, int64_t ldx, double beta,
                                                   const double *__restrict__ B, int64_t ldb, double *__restrict__ R,
                                                   int64_t ldr, double *__restrict__ rowsums) {
    __shared__ double As[kSymmRows][kSymmRows + 1];  // [j][r]: element (row r, column j) of the chunk
    __shared__ double Xs[kSymmRows][kSymmRhs];       // [j][c]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kSymmRows;
    const int64_t c0 = (int64_t)blockIdx.y * kSymmRhs;
    const bool sums = (rowsums != nullptr) && blockIdx.y == 0;
    double acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;
    double asum = 0.0;
    const int64_t nchunks = (n + kSymmRows - 1) / kSymmRows;
    for (int64_t J = 0; J < nchunks; ++J) {
        const int64_t j0 = J * kSymmRows;
        __syncthreads();
        // 64 x 64 chunk of the symmetric matrix: 16 elements per thread
#pragma unroll 4
        for (int e = 0; e < 16; ++e) {
            const int idx = tid + 256 * e;
            const int a = idx & 63, b = idx >> 6;  // a: fastest-varying (coalesced) index
            double v = 0.0;
            if ((int64_t)blockIdx.x <= J) {
                // upper tile: row i0 + a, column j0 + b
                const int64_t gi = i0 + a, gj = j0 + b;
                if (gi < n && gj < n) v = (gi <= gj) ? A0[gi + gj * lda0] : A0[gj + gi * lda0];
                As[b][a] = v;
            } else {
                // mirrored: element (row i0 + b, column j0 + a) = A0[j0 + a + (i0 + b) lda0]
                const int64_t gi = i0 + b, gj = j0 + a;
                if (gi < n && gj < n) v = A0[gj + gi * lda0];
                As[a][b] = v;
            }
        }
        for (int idx = tid; idx < kSymmRows * kSymmRhs; idx += 256) {
            const int j = idx & 63, c = idx >> 6;
            const int64_t gj = j0 + j, gc = c0 + c;
            Xs[j][c] = (gj < n && gc < nrhs) ? X[gj + gc * ldx] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int j = 0; j < kSymmRows; ++j) {
            const double a = As[j][lane];
            if (sums && wave == 0) asum += fabs(a);
#pragma unroll
            for (int c = 0; c < 16; ++c) acc[c] = fma(a, Xs[j][wave * 16 + c], acc[c]);
        }
    }
    const int64_t gi = i0 + lane;
    if (gi < n) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int64_t gc = c0 + wave * 16 + c;
            if (gc < nrhs) {
                const double bv = (B != nullptr) ? beta * B[gi + gc * ldb] : 0.0;
                R[gi + gc * ldr] = bv + alpha * acc[c];
            }
        }
        if (sums && wave == 0) rowsums[gi] = asum;
    }
}

int launch_symm(int64_t n, int64_t nrhs, double alpha, const double *A0, int64_t lda0, const double *X, int64_t ldx,
                double beta, const double *B, int64_t ldb, double *R, int64_t ldr, double *rowsums, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    const int tr = trace_begin(FLAME_KC_OTHER, s);
    hipLaunchKernelGGL(k_symm_rows, dim3((unsigned)((n + kSymmRows - 1) / kSymmRows),
                                         (unsigned)((nrhs + kSymmRhs - 1) / kSymmRhs)),
                       dim3(256), 0, s, n, nrhs, alpha, A0, lda0, X, ldx, beta, B, ldb, R, ldr, rowsums);
    FLAME_CHECK_LAUNCH();
    const double dn = (double)n;
    trace_end(tr, s, 2.0 * dn * dn * (double)nrhs, 4.0 * dn * (dn + 1) + 24.0 * dn * (double)nrhs);
    return FLAME_OK;
}

// ---- per-column dot products -------------------------------------------------
// out[c] = sum_i X(i, c) Y(i, c); one workgroup per column, a fixed reduction
// order (strided partial sums, then a tree), so results are deterministic.
__global__ __launch_bounds__(256) void k_dot_cols(int64_t n, const double *__restrict__ X, int64_t ldx,
                                                  const double *__restrict__ Y, int64_t ldy,
                                                  double *__restrict__ out) {
    __shared__ double red[256];
    const int64_t c = blockIdx.x;
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int64_t i = tid; i < n; i += 256) s = fma(X[i + c * ldx], Y[i + c * ldy], s);
    red[tid] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) out[c] = red[0];
}

int launch_dot_cols(int64_t n, int64_t nrhs, const double *X, int64_t ldx, const double *Y, int64_t ldy, double *out,
                    hipStream_t s) {
    if (nrhs <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_dot_cols, dim3((unsigned)nrhs), dim3(256), 0, s, n, X, ldx, Y, ldy, out);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

// ---- conjugate-gradient updates (per column) -------------------------------
// P := Z + beta P with beta = rho / rho_old (0 on the first step or when
// rho_old is 0: a converged column keeps a zero direction).
__global__ void k_cg_direction(int64_t n, const double *__restrict__ Z, int64_t ldz, double *__restrict__ P,
                               int64_t ldp, const double *__restrict__ rho, const double *__restrict__ rho_old,
                               int first) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i >= n) return;
    double b = 0.0;
    if (!first && rho_old[c] != 0.0) b = rho[c] / rho_old[c];
    P[i + c * ldp] = first ? Z[i + c * ldz] : fma(b, P[i + c * ldp], Z[i + c * ldz]);
}

// X += alpha P, R -= alpha Q with alpha = rho / (p^T q) (0 when p^T q is not
// positive: the direction is zero or the operator is not positive definite).
__global__ void k_cg_step(int64_t n, double *__restrict__ X, int64_t ldx, double *__restrict__ R, int64_t ldr,
                          const double *__restrict__ P, int64_t ldp, const double *__restrict__ Q, int64_t ldq,
                          const double *__restrict__ rho, const double *__restrict__ pq) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i >= n) return;
    const double a = (pq[c] > 0.0) ? rho[c] / pq[c] : 0.0;
    X[i + c * ldx] = fma(a, P[i + c * ldp], X[i + c * ldx]);
    R[i + c * ldr] = fma(-a, Q[i + c * ldq], R[i + c * ldr]);
}

int launch_cg_direction(int64_t n, int64_t nrhs, const double *Z, int64_t ldz, double *P, int64_t ldp,
                        const double *rho, const double *rho_old, bool first, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_cg_direction, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, s, n, Z, ldz,
                       P, ldp, rho, rho_old, first ? 1 : 0);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_cg_step(int64_t n, int64_t nrhs, double *X, int64_t ldx, double *R, int64_t ldr, const double *P,
                   int64_t ldp, const double *Q, int64_t ldq, const double *rho, const double *pq, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_cg_step, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, s, n, X, ldx, R,
                       ldr, P, ldp, Q, ldq, rho, pq);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

// ---- diagonal scaling ---------------------------------------------------------
// d[j] = 1 / sqrt(A0(j, j)); a diagonal entry that is not > 0 (NaN included)
// records its 1-based column in *bad (the smallest such column wins).
__global__ void k_diag_scale(int64_t n, const double *__restrict__ A0, int64_t lda0, double *__restrict__ d,
                             int32_t *__restrict__ bad) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double a = A0[j + j * lda0];
    if (!(a > 0.0)) {
        atomicMin(bad, (int32_t)(j + 1));
        d[j] = 1.0;
        return;
    }
    d[j] = 1.0 / sqrt(a);
}

__global__ void k_fill_i32(int32_t *p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

int launch_diag_scale(int64_t n, const double *A0, int64_t lda0, double *d, int32_t *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, bad, (int32_t)0x7fffffff);
    FLAME_CHECK_LAUNCH();
    if (n <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_diag_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, A0, lda0, d, bad);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

// W(i, j) := d_i A0(i, j) d_j + (i == j ? mu : 0) on the upper triangle
// (d == nullptr: no scaling).  One workgroup per column, rows 0..j.
__global__ __launch_bounds__(256) void k_scale_copy_upper(int64_t n, const double *__restrict__ A0, int64_t lda0,
                                                          double *__restrict__ W, int64_t ldw,
                                                          const double *__restrict__ d, double mu) {
    const int64_t j = blockIdx.x;
    const double dj = d ? d[j] : 1.0;
    const double *a = A0 + j * lda0;
    double *w = W + j * ldw;
    for (int64_t i = threadIdx.x; i <= j; i += 256) {
        double v = a[i] * (d ? d[i] : 1.0) * dj;
        if (i == j) v += mu;
        w[i] = v;
    }
}

int launch_scale_copy_upper(int64_t n, const double *A0, int64_t lda0, double *W, int64_t ldw, const double *d,
                            double mu, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    const int tr = trace_begin(FLAME_KC_OTHER, s);
    hipLaunchKernelGGL(k_scale_copy_upper, dim3((unsigned)n), dim3(256), 0, s, n, A0, lda0, W, ldw, d, mu);
    FLAME_CHECK_LAUNCH();
    const double dn = (double)n;
    trace_end(tr, s, 0.0, 8.0 * dn * (dn + 1));
    return FLAME_OK;
}

// U(i, j) := U(i, j) / d_j on the upper triangle: the factor of the scaled
// matrix D A0 D (+ mu I) becomes a factor of A0 (+ mu D^{-2}).
__global__ __launch_bounds__(256) void k_unscale_cols(int64_t n, double *__restrict__ U, int64_t ldu,
                                                      const double *__restrict__ d) {
    const int64_t j = blockIdx.x;
    const double inv = 1.0 / d[j];
    double *u = U + j * ldu;
    for (int64_t i = threadIdx.x; i <= j; i += 256) u[i] *= inv;
}

int launch_unscale_cols(int64_t n, double *U, int64_t ldu, const double *d, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    const int tr = trace_begin(FLAME_KC_OTHER, s);
    hipLaunchKernelGGL(k_unscale_cols, dim3((unsigned)n), dim3(256), 0, s, n, U, ldu, d);
    FLAME_CHECK_LAUNCH();
    const double dn = (double)n;
    trace_end(tr, s, 0.0, 8.0 * dn * (dn + 1));
    return FLAME_OK;
}

}  // namespace flame
