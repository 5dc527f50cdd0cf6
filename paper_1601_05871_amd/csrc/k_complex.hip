// Complex Hermitian factorization A = U^H U (the loop of Fig. "dense-chol"
// with its HERK update taken literally; complex data is one of the
// extensions the conclusion lists): the kernels of the steps that are not a
// plain real product.  The driver (zfactor.cpp) keeps the matrix as two real
// planes, real and imaginary parts, so that the Hermitian update and the
// off-diagonal products of the panel solve run as real matrix-core products
// (launch_gemm_tn); the kernels here split and merge the planes, factor a
// diagonal block of order <= 64 and form the inverse of a diagonal block of
// U for the panel solve.
#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kZ = 64;  // order of the diagonal blocks factored in LDS

// planes := upper triangle of the interleaved complex A (one workgroup per
// column); the strictly lower part of the planes is not written
__global__ __launch_bounds__(256) void k_z_split(int64_t n, const double *__restrict__ A, int64_t lda,
                                                 double *__restrict__ R, double *__restrict__ I, int64_t ld) {
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i <= j; i += 256) {
        const double *a = A + 2 * (i + j * lda);
        R[i + j * ld] = a[0];
        I[i + j * ld] = a[1];
    }
}

// upper triangle of the interleaved A := planes; the diagonal's imaginary
// part is written 0 (U has a real diagonal)
__global__ __launch_bounds__(256) void k_z_merge(int64_t n, const double *__restrict__ R,
                                                 const double *__restrict__ I, int64_t ld, double *__restrict__ A,
                                                 int64_t lda) {
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i <= j; i += 256) {
        double *a = A + 2 * (i + j * lda);
        a[0] = R[i + j * ld];
        a[1] = (i == j) ? 0.0 : I[i + j * ld];
    }
}

// dst := scale * src (rows x cols), one workgroup per column; skipped if
// *info != 0 (after a breakdown the panel keeps what it held)
__global__ __launch_bounds__(256) void k_scaled_copy(int64_t rows, const double *__restrict__ src, int64_t lds,
                                                     double *__restrict__ dst, int64_t ldd, double scale,
                                                     const int32_t *__restrict__ info) {
    if (info != nullptr && *info != 0) return;
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i < rows; i += 256) dst[i + j * ldd] = scale * src[i + j * lds];
}

__global__ __launch_bounds__(256) void k_fill0(int64_t rows, double *__restrict__ dst, int64_t ldd) {
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i < rows; i += 256) dst[i + j * ldd] = 0.0;
}

// A := Chol(A) for the n x n (n <= 64) diagonal block held in the planes
// (upper triangle), one workgroup.  Thread (c, g) (c = tid % 64,
// g = tid / 64) keeps elements (g + 4 k, c), k < 16, real and imaginary
// parts, in registers for the whole factorization; step j goes through LDS
// only for the pivot and row j of U (double-buffered by step parity, two
// barriers per step): the pivot's owner publishes re A(j,j) (its imaginary
// part is not read); every thread reads it, row j's owners divide their
// element by its square root and publish U(j, :); every thread updates its
// elements (i, c), j < i <= c, with conj(U(j,i)) U(j,c) (selects, no
// per-element branch).  A pivot that is not > 0: *info = info_base + j + 1
// and every thread leaves (the planes then hold nothing of this block's
// result).  Then V := -U^{-1} into the planes Vr, Vi (ldv), zero below the
// diagonal, from U as the registers hold it (the panel solves' operand: one
// launch for both).  U is padded to 64 with the identity and W = U^{-1}
// formed by doubling: the four 16 x 16 diagonal blocks by back substitution
// (a thread per column, no barriers), then pairs of blocks of order h = 16
// and 32 joined by W(lo, hi) = -W(lo, lo) U(lo, hi) W(hi, hi), the inner
// product kept in W's unused lower triangle; U and W in LDS, [row][column].
// Skips if *info != 0 on entry.
__global__ __launch_bounds__(256) void k_zchol_lds(int n, double *__restrict__ R, double *__restrict__ I, int64_t ld,
                                                   int32_t *__restrict__ info, int64_t info_base,
                                                   double *__restrict__ Vr, double *__restrict__ Vi, int64_t ldv) {
    __shared__ double rowr[2][kZ], rowi[2][kZ], pivb[2];
    __shared__ double ur[kZ][kZ + 1], ui[kZ][kZ + 1];
    __shared__ double wr[kZ][kZ + 1], wi[kZ][kZ + 1];
    if (*info != 0) return;
    const int tid = threadIdx.x, c = tid & (kZ - 1), g = tid >> 6;
    double ar[16], ai[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int i = g + 4 * k;
        const bool in = i <= c && c < n;
        ar[k] = in ? R[i + (int64_t)c * ld] : 0.0;
        ai[k] = in ? I[i + (int64_t)c * ld] : 0.0;
    }
    // j = 4 kj + r with kj unrolled: the registers holding row j are
    // ar[kj], ai[kj], compile-time indices (run-time ones would put the
    // arrays in scratch)
#pragma unroll
    for (int kj = 0; kj < 16; ++kj)
    for (int r = 0; r < 4; ++r) {
        const int j = 4 * kj + r;
        if (j >= n) break;
        const int b = j & 1;
        const bool rowown = g == r;
        if (rowown && c == j) pivb[b] = ar[kj];
        __syncthreads();
        const double d = pivb[b];
        if (!(d > 0.0)) {
            if (tid == 0) *info = (int32_t)(info_base + j + 1);
            return;
        }
        const double sq = sqrt(d);
        if (rowown) {  // row j of U: A(j, c) / sqrt(d) for c > j, sqrt(d) on the diagonal
            const double rs = 1.0 / sq;
            double ur = ar[kj] * rs, ui = ai[kj] * rs;
            if (c == j) {
                ur = sq;
                ui = 0.0;
            }
            ar[kj] = (c >= j) ? ur : ar[kj];
            ai[kj] = (c >= j) ? ui : ai[kj];
            rowr[b][c] = ur;
            rowi[b][c] = ui;
        }
        __syncthreads();
        const double yr = rowr[b][c], yi = rowi[b][c];
        const bool cu = c > j && c < n;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int i = g + 4 * k;
            const double xr = rowr[b][i], xi = rowi[b][i];
            const bool up = cu && i > j && i <= c;
            ar[k] = up ? ar[k] - (xr * yr + xi * yi) : ar[k];
            ai[k] = up ? ai[k] - (xr * yi - xi * yr) : ai[k];
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int i = g + 4 * k;
        const bool in = i <= c && c < n;
        if (in) {
            R[i + (int64_t)c * ld] = ar[k];
            I[i + (int64_t)c * ld] = ai[k];
        }
        ur[i][c] = in ? ar[k] : (i == c ? 1.0 : 0.0);
        ui[i][c] = in ? ai[k] : 0.0;
    }
    for (int e = tid; e < kZ * kZ; e += 256) {
        const int r = e & (kZ - 1), cc = e >> 6;
        wr[r][cc] = 0.0;
        wi[r][cc] = 0.0;
    }
    __syncthreads();
    if (tid < kZ) {  // the diagonal 16-blocks: block b, column j of it, rows j .. 0
        const int b = tid >> 4, j = tid & 15, c = 16 * b + j;
        for (int i = j; i >= 0; --i) {
            const int r = 16 * b + i;
            double sr = (i == j) ? 1.0 : 0.0, si = 0.0;
            for (int k = i + 1; k <= j; ++k) {
                const int q = 16 * b + k;
                sr -= ur[r][q] * wr[q][c] - ui[r][q] * wi[q][c];
                si -= ur[r][q] * wi[q][c] + ui[r][q] * wr[q][c];
            }
            const double d = ur[r][r];  // real diagonal
            wr[r][c] = sr / d;
            wi[r][c] = si / d;
        }
    }
    __syncthreads();
    for (int h = 16; h < kZ; h *= 2) {
        const int outs = (kZ / (2 * h)) * h * h;  // pairs x h^2
        for (int e = tid; e < outs; e += 256) {   // T = U(lo, hi) W(hi, hi), into W(hi, lo)'s place
            const int p = e / (h * h), q = e % (h * h), i = q % h, j = q / h;
            const int lo = 2 * h * p, hi = lo + h;
            double sr = 0.0, si = 0.0;
            for (int k = 0; k <= j; ++k) {
                const double a = ur[lo + i][hi + k], b = ui[lo + i][hi + k];
                const double x = wr[hi + k][hi + j], y = wi[hi + k][hi + j];
                sr += a * x - b * y;
                si += a * y + b * x;
            }
            wr[hi + i][lo + j] = sr;
            wi[hi + i][lo + j] = si;
        }
        __syncthreads();
        for (int e = tid; e < outs; e += 256) {  // W(lo, hi) = -W(lo, lo) T
            const int p = e / (h * h), q = e % (h * h), i = q % h, j = q / h;
            const int lo = 2 * h * p, hi = lo + h;
            double sr = 0.0, si = 0.0;
            for (int k = i; k < h; ++k) {
                const double a = wr[lo + i][lo + k], b = wi[lo + i][lo + k];
                const double x = wr[hi + k][lo + j], y = wi[hi + k][lo + j];
                sr += a * x - b * y;
                si += a * y + b * x;
            }
            wr[lo + i][hi + j] = -sr;
            wi[lo + i][hi + j] = -si;
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += 256) {
        const int i = e % n, c = e / n;
        Vr[i + (int64_t)c * ldv] = i <= c ? -wr[i][c] : 0.0;
        Vi[i + (int64_t)c * ldv] = i <= c ? -wi[i][c] : 0.0;
    }
}

typedef double zd4 __attribute__((ext_vector_type(4)));

// acc += x^T y over one k slot: lane (r, g) of the result holds element
// (r, g + 4 v) of the 16 x 16 block in item v, r from x's columns (C's rows),
// g + 4 v from y's columns.
__device__ __forceinline__ zd4 zmma(double x, double y, zd4 acc) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(y, x, acc, 0, 0, 0);
}

// C -= P^H Q on planes, in one pass: per k slot the four real products
//   C_re -= Pr^T Qr + Pi^T Qi,   C_im -= Pr^T Qi - Pi^T Qr
// share the operands each lane loads.  P is K x M (ldp), Q is K x N (ldq),
// C is M x N (ldc).  A workgroup takes a 64 x 64 tile of C, each wavefront
// 32 x 32 of it (2 x 2 blocks of 16 x 16, real and imaginary accumulators);
// operands straight from global memory, k = kc + 4 g + t in step t of a
// 16-k chunk, rows, columns and k beyond the matrices clamped or zeroed.
// upper: only i <= j of C is written (tiles entirely below skipped).
// Skips if *info != 0.
// INPLACE: C and Q are the same (M <= 64, one row of workgroup tiles, so each
// workgroup owns its columns) and C := -P^H Q is written over it: no
// wavefront leaves early, and all of them have read their Q before any
// writes C (a barrier between).
template <bool INPLACE>
__global__ __launch_bounds__(256) void k_zgemm_h(int64_t M, int64_t N, int64_t K, const double *Pr, const double *Pi,
                                                 int64_t ldp, const double *Qr, const double *Qi, int64_t ldq,
                                                 double *Cr, double *Ci, int64_t ldc, int upper,
                                                 const int32_t *__restrict__ info) {
    if (*info != 0) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * 64 + (wave >> 1) * 32;
    const int64_t col0 = (int64_t)blockIdx.y * 64 + (wave & 1) * 32;
    if (!INPLACE) {
        if (row0 >= M || col0 >= N) return;
        if (upper && row0 > col0 + 31) return;
    }
    zd4 are[2][2], aim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) are[a][b] = aim[a][b] = zd4{0.0, 0.0, 0.0, 0.0};
    const double *pr[2], *pi[2], *qr[2], *qi[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int64_t pc = min(row0 + 16 * a + r, M - 1), qc = min(col0 + 16 * a + r, N - 1);
        pr[a] = Pr + pc * ldp;
        pi[a] = Pi + pc * ldp;
        qr[a] = Qr + qc * ldq;
        qi[a] = Qi + qc * ldq;
    }
    for (int64_t kc = 0; kc < K; kc += 16) {
        double xr[2][4], xi[2][4], yr[2][4], yi[2][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t k = kc + 4 * g + t;
            const bool ok = k < K;
            const int64_t kk = ok ? k : K - 1;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                xr[a][t] = ok ? -pr[a][kk] : 0.0;
                xi[a][t] = ok ? pi[a][kk] : 0.0;
                yr[a][t] = qr[a][kk];
                yi[a][t] = qi[a][kk];
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    are[a][b] = zmma(xr[a][t], yr[b][t], are[a][b]);   // - Pr^T Qr
                    are[a][b] = zmma(-xi[a][t], yi[b][t], are[a][b]);  // - Pi^T Qi
                    aim[a][b] = zmma(xr[a][t], yi[b][t], aim[a][b]);   // - Pr^T Qi
                    aim[a][b] = zmma(xi[a][t], yr[b][t], aim[a][b]);   // + Pi^T Qr
                }
    }
    if (INPLACE) __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = row0 + 16 * a + r, j = col0 + 16 * b + g + 4 * v;
                if (i < M && j < N && (!upper || i <= j)) {
                    if (INPLACE) {
                        Cr[i + j * ldc] = are[a][b][v];
                        Ci[i + j * ldc] = aim[a][b][v];
                    } else {
                        Cr[i + j * ldc] += are[a][b][v];
                        Ci[i + j * ldc] += aim[a][b][v];
                    }
                }
            }
}

unsigned cols_grid(int64_t cols) { return (unsigned)std::max<int64_t>(1, cols); }

}  // namespace

int launch_z_split(int64_t n, const void *A, int64_t lda, double *R, double *I, int64_t ld, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_z_split, dim3(cols_grid(n)), dim3(256), 0, s, n, static_cast<const double *>(A), lda, R, I,
                       ld);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_z_merge(int64_t n, const double *R, const double *I, int64_t ld, void *A, int64_t lda, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_z_merge, dim3(cols_grid(n)), dim3(256), 0, s, n, R, I, ld, static_cast<double *>(A), lda);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_scaled_copy(int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst, int64_t ldd,
                       double scale, const int32_t *info, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_scaled_copy, dim3(cols_grid(cols)), dim3(256), 0, s, rows, src, lds, dst, ldd, scale, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_fill0(int64_t rows, int64_t cols, double *dst, int64_t ldd, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_fill0, dim3(cols_grid(cols)), dim3(256), 0, s, rows, dst, ldd);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_zgemm_h(bool upper, int64_t M, int64_t N, int64_t K, const double *Pr, const double *Pi, int64_t ldp,
                   const double *Qr, const double *Qi, int64_t ldq, double *Cr, double *Ci, int64_t ldc,
                   const int32_t *info, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return FLAME_OK;
    const dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
    hipLaunchKernelGGL(k_zgemm_h<false>, grid, dim3(256), 0, s, M, N, K, Pr, Pi, ldp, Qr, Qi, ldq, Cr, Ci, ldc,
                       upper ? 1 : 0, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_zgemm_h_inplace(int64_t M, int64_t N, int64_t K, const double *Pr, const double *Pi, int64_t ldp,
                           double *Xr, double *Xi, int64_t ldx, const int32_t *info, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return FLAME_OK;
    if (M > 64) return FLAME_ERR_UNSUPPORTED;
    const dim3 grid(1u, (unsigned)((N + 63) / 64));
    hipLaunchKernelGGL(k_zgemm_h<true>, grid, dim3(256), 0, s, M, N, K, Pr, Pi, ldp, Xr, Xi, ldx, Xr, Xi, ldx, 0,
                       info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_zchol_lds(int n, double *R, double *I, int64_t ld, int32_t *info, int64_t info_base, double *Vr,
                     double *Vi, int64_t ldv, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    if (n > kZ || ldv < n) return FLAME_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_zchol_lds, dim3(1), dim3(256), 0, s, n, R, I, ld, info, info_base, Vr, Vi, ldv);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
