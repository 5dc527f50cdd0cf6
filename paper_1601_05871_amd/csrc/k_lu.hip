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

// v of lane `lane` (uniform) for every lane.
__device__ __forceinline__ double lane_value(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// A := L\U for the n x n (n <= 64) block, one workgroup, the block in LDS
// ([column][row], padded), blocked by 16 columns.  For the panel of columns
// k0 .. k0 + 15:
//   wavefront 0 factors the panel A(k0:n, k0:k0+16) with a lane per row and
//     the row's 16 values in registers: step j takes the pivot row from lane
//     j (readlane; zero or not finite: *info = info_base + column, stop),
//     each row below divides its entry by the pivot and subtracts the
//     multiple of the pivot row (no barriers: one wavefront);
//   a thread per column forms U12 := L11^{-1} A12 (forward substitution);
//   all threads apply A22 -= L21 U12, pivot by pivot.
// Each entry sees the same operations in the same order as in the unblocked
// loop (a(r, c) -= l(r, j) u(j, c) for j ascending), only grouped by panel.
// Skips if *info != 0 on entry.
__global__ __launch_bounds__(256) void k_lu_lds(int n, double *__restrict__ A, int64_t lda, int32_t *__restrict__ info,
                                                int64_t info_base) {
    __shared__ double a[kL][kL + 1];
    __shared__ int s_bad;
    if (*info != 0) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < kL * kL; e += 256) {
        const int i = e & (kL - 1), j = e >> 6;
        if (i < n && j < n) a[j][i] = A[i + (int64_t)j * lda];
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += 16) {
        const int w = min(16, n - k0);  // panel width
        if (tid < 64) {                 // the panel: lane tid holds row k0 + tid
            const int r = k0 + tid;
            const bool live = r < n;
            double x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = (live && c < w) ? a[k0 + c][r] : 0.0;
            int bad = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < w && bad == 0) {  // uniform
                    double prow[16];
#pragma unroll
                    for (int c = j; c < 16; ++c) prow[c] = lane_value(x[c], j);
                    const double piv = prow[j];
                    if (piv == 0.0 || !isfinite(piv)) {
                        bad = k0 + j + 1;
                    } else if (tid > j && live) {
                        const double l = x[j] / piv;
                        x[j] = l;
#pragma unroll
                        for (int c = j + 1; c < 16; ++c) x[c] -= l * prow[c];
                    }
                }
            }
            if (live) {
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (c < w) a[k0 + c][r] = x[c];
            }
            if (tid == 0 && bad != 0) s_bad = bad;
        }
        __syncthreads();
        if (s_bad != 0) {  // uniform
            if (tid == 0) *info = (int32_t)(info_base + s_bad);
            return;
        }
        const int c0 = k0 + w, rest = n - c0;
        if (rest <= 0) break;
        if (tid < rest) {  // U12 := L11^{-1} A12, column c0 + tid
            const int c = c0 + tid;
            double y[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) y[i] = i < w ? a[c][k0 + i] : 0.0;
#pragma unroll
            for (int i = 1; i < 16; ++i)
#pragma unroll
                for (int k = 0; k < i; ++k) y[i] -= a[k0 + k][k0 + i] * y[k];  // L(k0 + i, k0 + k)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < w) a[c][k0 + i] = y[i];
        }
        __syncthreads();
        for (int e = tid; e < rest * rest; e += 256) {  // A22 -= L21 U12, pivot by pivot
            const int rr = c0 + e % rest, cc = c0 + e / rest;
            double v = a[cc][rr];
            for (int k = 0; k < w; ++k) v -= a[k0 + k][rr] * a[cc][k0 + k];
            a[cc][rr] = v;
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
// C + U^{-T} Y with X = P2.  The block is padded to 64 with the identity, and
// each inverse is formed by doubling: the four 16 x 16 diagonal blocks by
// substitution (a thread per column, no barriers), then pairs of blocks of
// order h = 16 and 32 joined by
//   W(hi, lo) = -W(hi, hi) L(hi, lo) W(lo, lo)     (W = L^{-1}, lower)
//   V(lo, hi) = -V(lo, lo) U(lo, hi) V(hi, hi)     (V = U^{-1}, upper)
// as two products each, the inner one kept in the inverse's other (unused)
// triangle.  512 threads: the first 256 form W, the others V.  In LDS,
// [row][column].
__global__ __launch_bounds__(512) void k_lu_inv(int n, const double *__restrict__ A, int64_t lda,
                                                double *__restrict__ P1, double *__restrict__ P2,
                                                const int32_t *__restrict__ info) {
    __shared__ double a[kL][kL + 1];
    __shared__ double w[kL][kL + 1];
    __shared__ double v[kL][kL + 1];
    if (*info != 0) return;
    const int tid = threadIdx.x, t = tid & 255;
    const bool up = tid >= 256;  // uniform per wavefront
    for (int e = tid; e < kL * kL; e += 512) {
        const int r = e & (kL - 1), c = e >> 6;
        a[r][c] = (r < n && c < n) ? A[r + (int64_t)c * lda] : (r == c ? 1.0 : 0.0);
        w[r][c] = 0.0;
        v[r][c] = 0.0;
    }
    __syncthreads();
    if (t < kL) {  // the diagonal 16-blocks: block b, column j of it
        const int b = t >> 4, j = t & 15, c = 16 * b + j;
        if (!up) {  // unit lower: rows j .. 15
            for (int i = j; i < 16; ++i) {
                const int r = 16 * b + i;
                double sum = (i == j) ? 1.0 : 0.0;
                for (int k = j; k < i; ++k) sum -= a[r][16 * b + k] * w[16 * b + k][c];
                w[r][c] = sum;
            }
        } else {  // upper: rows j .. 0
            for (int i = j; i >= 0; --i) {
                const int r = 16 * b + i;
                double sum = (i == j) ? 1.0 : 0.0;
                for (int k = i + 1; k <= j; ++k) sum -= a[r][16 * b + k] * v[16 * b + k][c];
                v[r][c] = sum / a[r][r];
            }
        }
    }
    __syncthreads();
    for (int h = 16; h < kL; h *= 2) {
        const int outs = (kL / (2 * h)) * h * h;  // pairs x h^2
        for (int e = t; e < outs; e += 256) {     // the inner products, into the other triangle
            const int p = e / (h * h), q = e % (h * h), i = q % h, j = q / h;
            const int lo = 2 * h * p, hi = lo + h;
            double sum = 0.0;
            if (!up) {
                for (int k = j; k < h; ++k) sum += a[hi + i][lo + k] * w[lo + k][lo + j];  // L(hi, lo) W(lo, lo)
                w[lo + i][hi + j] = sum;
            } else {
                for (int k = 0; k <= j; ++k) sum += a[lo + i][hi + k] * v[hi + k][hi + j];  // U(lo, hi) V(hi, hi)
                v[hi + i][lo + j] = sum;
            }
        }
        __syncthreads();
        for (int e = t; e < outs; e += 256) {
            const int p = e / (h * h), q = e % (h * h), i = q % h, j = q / h;
            const int lo = 2 * h * p, hi = lo + h;
            double sum = 0.0;
            if (!up) {
                for (int k = 0; k <= i; ++k) sum += w[hi + i][hi + k] * w[lo + k][hi + j];
                w[hi + i][lo + j] = -sum;
            } else {
                for (int k = i; k < h; ++k) sum += v[lo + i][lo + k] * v[hi + k][lo + j];
                v[lo + i][hi + j] = -sum;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += 512) {
        const int i = e % n, c = e / n;
        P1[c + (int64_t)i * kL] = i >= c ? -w[i][c] : 0.0;  // P1(c, i) = -W(i, c)
        P2[i + (int64_t)c * kL] = i <= c ? -v[i][c] : 0.0;  // P2(i, c) = -V(i, c)
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
