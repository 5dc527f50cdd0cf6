// LU without pivoting, A = L U (L unit lower, U upper), by the partitioned
// loop of Fig. "dense-chol" carried over to LU (the conclusion names LU among
// the factorizations the pattern extends to):
//   A11 := LU(A11);  A12 := L11^{-1} A12;  A21 := A21 U11^{-1};
//   A22 := A22 - A21 A12.
// The kernels of the steps that are not a plain product: the diagonal block
// (order <= 64) factored in LDS, the negated inverses of its two triangles in
// the operand layout of the trailing-update kernel, and a tiled transpose
// (the driver, lu.cpp, keeps A21 transposed while it is solved and used).
#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kL = 64;

// A := L\U for the n x n (n <= 64) block, one workgroup, the block in LDS
// ([column][row], padded).  Step j: pivot A(j,j) (zero or not finite:
// *info = info_base + j + 1, stop), column below divided by it, then
// A(r,c) -= A(r,j) A(j,c) for r, c > j, the 256 threads on (column, row
// group) pairs.  Skips if *info != 0 on entry.
__global__ __launch_bounds__(256) void k_lu_lds(int n, double *__restrict__ A, int64_t lda, int32_t *__restrict__ info,
                                                int64_t info_base) {
    __shared__ double a[kL][kL + 1];
    if (*info != 0) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < kL * kL; e += 256) {
        const int i = e & (kL - 1), j = e >> 6;
        if (i < n && j < n) a[j][i] = A[i + (int64_t)j * lda];
    }
    __syncthreads();
    const int cl = tid & (kL - 1), rg = tid >> 6;
    for (int j = 0; j < n; ++j) {
        const double piv = a[j][j];
        if (piv == 0.0 || !isfinite(piv)) {  // the same value in every thread: a uniform exit
            if (tid == 0) *info = (int32_t)(info_base + j + 1);
            return;
        }
        for (int r = j + 1 + tid; r < n; r += 256) a[j][r] = a[j][r] / piv;
        __syncthreads();
        const int c = j + 1 + cl;
        if (c < n) {
            const double ujc = a[c][j];
            for (int r = j + 1 + rg; r < n; r += 4) a[c][r] -= a[j][r] * ujc;
        }
        __syncthreads();
    }
    for (int e = tid; e < kL * kL; e += 256) {
        const int i = e & (kL - 1), j = e >> 6;
        if (i < n && j < n) A[i + (int64_t)j * lda] = a[j][i];
    }
}

// For the factored n x n block (L\U): P1 := -(L^{-1})^T and P2 := -U^{-1}
// (n x n each, ld kL, zero outside the triangles), so that the
// trailing-update kernel's C -= X^T Y gives C + L^{-1} Y with X = P1 and
// C + U^{-T} Y with X = P2.  512 threads: the first 256 form the columns of
// L^{-1} (forward substitution, L w = e_t, unit diagonal), the others those
// of U^{-1} (back substitution, U v = e_t), both row by row in lockstep, the
// sum over k of each row split over four threads (k mod 4) and combined after
// a barrier.  The block, the columns and the partial sums in LDS.
__global__ __launch_bounds__(512) void k_lu_inv(int n, const double *__restrict__ A, int64_t lda,
                                                double *__restrict__ P1, double *__restrict__ P2,
                                                const int32_t *__restrict__ info) {
    __shared__ double a[kL][kL + 1];   // [column][row]
    __shared__ double w[kL][kL + 1];   // [column t][row] of L^{-1}
    __shared__ double v[kL][kL + 1];   // [column t][row] of U^{-1}
    __shared__ double part[2][4][kL];  // partial sums [triangle][k mod 4][column]
    if (*info != 0) return;
    const int tid = threadIdx.x, t = tid & (kL - 1), q = (tid >> 6) & 3, up = tid >> 8;
    for (int e = tid; e < kL * kL; e += 512) {
        const int i = e & (kL - 1), j = e >> 6;
        if (i < n && j < n) a[j][i] = A[i + (int64_t)j * lda];
    }
    __syncthreads();
    for (int step = 0; step < n; ++step) {
        double s = 0.0;
        if (t < n) {
            if (!up) {  // row i of L w = e_t: w_i = delta - sum_{t <= k < i} L(i, k) w_k
                const int i = step;
                if (i > t)
                    for (int k = t + q; k < i; k += 4) s += a[k][i] * w[t][k];
            } else {  // row i of U v = e_t: v_i = (delta - sum_{i < k <= t} U(i, k) v_k) / U(i, i)
                const int i = n - 1 - step;
                if (i <= t)
                    for (int k = i + 1 + q; k <= t; k += 4) s += a[k][i] * v[t][k];
            }
        }
        part[up][q][t] = s;
        __syncthreads();
        if (q == 0 && t < n) {
            const double sum = (part[up][0][t] + part[up][1][t]) + (part[up][2][t] + part[up][3][t]);
            if (!up) {
                const int i = step;
                w[t][i] = (i < t) ? 0.0 : (((i == t) ? 1.0 : 0.0) - sum);
            } else {
                const int i = n - 1 - step;
                v[t][i] = (i > t) ? 0.0 : (((i == t) ? 1.0 : 0.0) - sum) / a[i][i];
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += 512) {
        const int i = e % n, c = e / n;
        P1[c + (int64_t)i * kL] = -w[c][i];  // P1(c, i) = -W(i, c)
        P2[i + (int64_t)c * kL] = -v[c][i];  // P2(i, c) = -V(i, c)
    }
}

// dst (cols x rows, ldd) := src^T (src rows x cols, lds), 64 x 64 tiles
// through LDS, grid (row tiles, column tiles); skipped if info && *info.
__global__ __launch_bounds__(256) void k_transpose_copy(int64_t rows, int64_t cols, const double *__restrict__ src,
                                                        int64_t lds, double *__restrict__ dst, int64_t ldd,
                                                        const int32_t *__restrict__ info) {
    __shared__ double tile[kL][kL + 1];
    if (info != nullptr && *info != 0) return;
    const int64_t r0 = (int64_t)blockIdx.x * kL, c0 = (int64_t)blockIdx.y * kL;
    const int tx = threadIdx.x & (kL - 1), ty = threadIdx.x >> 6;
    for (int k = ty; k < kL; k += 4) {
        const int64_t r = r0 + tx, c = c0 + k;
        if (r < rows && c < cols) tile[k][tx] = src[r + c * lds];
    }
    __syncthreads();
    for (int k = ty; k < kL; k += 4) {
        const int64_t dr = c0 + tx, dc = r0 + k;  // dst(dr, dc) = src(dc, dr)
        if (dr < cols && dc < rows) dst[dr + dc * ldd] = tile[tx][k];
    }
}

}  // namespace

int launch_lu_lds(int n, double *A, int64_t lda, int32_t *info, int64_t info_base, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    if (n > kL) return FLAME_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_lu_lds, dim3(1), dim3(256), 0, s, n, A, lda, info, info_base);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_lu_inv(int n, const double *A, int64_t lda, double *P1, double *P2, const int32_t *info, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    if (n > kL) return FLAME_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_lu_inv, dim3(1), dim3(512), 0, s, n, A, lda, P1, P2, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_transpose_copy(int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst, int64_t ldd,
                          const int32_t *info, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return FLAME_OK;
    const dim3 grid((unsigned)((rows + kL - 1) / kL), (unsigned)((cols + kL - 1) / kL));
    hipLaunchKernelGGL(k_transpose_copy, grid, dim3(256), 0, s, rows, cols, src, lds, dst, ldd, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
