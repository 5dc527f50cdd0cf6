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
// The panel step of k_lu_diag wants 284 VGPRs: at 512 threads (two waves per
// SIMD, 256 registers each) it spills 132 bytes per lane to scratch, at 256 it
// does not, but the inverses then run on half as many threads; 512 is the
// faster of the two (n = 2048: 3.19 ms against 3.63 ms).
constexpr int kDiagThreads = 512;

// v of lane `lane` (uniform) for every lane.
__device__ __forceinline__ double lane_value(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// The diagonal block of one step, one workgroup of NT threads, the block in
// LDS ([column][row], padded to 64 with the identity):
//
// (1) A := L\U for the n x n (n <= 64) block, blocked by 16 columns.  For the
// panel of columns k0 .. k0 + 15:
//   wavefront 0 factors the panel A(k0:n, k0:k0+16) with a lane per row and
//     the row's 16 values in registers: step j takes the pivot row from lane
//     j (readlane; zero or not finite: *info = info_base + column, stop),
//     each row below divides its entry by the pivot and subtracts the
//     multiple of the pivot row (no barriers: one wavefront);
//   a thread per column forms U12 := L11^{-1} A12 (forward substitution);
//   all threads apply A22 -= L21 U12, pivot by pivot.
// Each entry sees the same operations in the same order as in the unblocked
// loop (a(r, c) -= l(r, j) u(j, c) for j ascending), only grouped by panel.
//
// (2) Unless P1 is null: P1 := -(L^{-1})^T and P2 := -U^{-1} (n x n each,
// ld kL, zero outside the triangles), so that the trailing-update kernel's
// C -= X^T Y gives C + L^{-1} Y with X = P1 and C + U^{-T} Y with X = P2.
// Each inverse is formed by doubling: the four 16 x 16 diagonal blocks by
// substitution (a thread per column, no barriers), then pairs of blocks of
// order h = 16 and 32 joined by
//   W(hi, lo) = -W(hi, hi) L(hi, lo) W(lo, lo)     (W = L^{-1}, lower)
//   V(lo, hi) = -V(lo, lo) U(lo, hi) V(hi, hi)     (V = U^{-1}, upper)
// as two products each, the inner one kept in the inverse's other (unused)
// triangle.  The first half of the threads form W, the others V
// ([row][column]).
// The factor is read from LDS where step (1) left it: one launch, one load.
//
// Skips if *info != 0 on entry; after a breakdown A keeps what it held.
template <int NT>
__global__ __launch_bounds__(NT) void k_lu_diag(int n, double *__restrict__ A, int64_t lda,
                                                 int32_t *__restrict__ info, int64_t info_base,
                                                 double *__restrict__ P1, double *__restrict__ P2) {
    __shared__ double a[kL][kL + 1];
    __shared__ double w[kL][kL + 1];
    __shared__ double v[kL][kL + 1];
    __shared__ int s_bad;
    if (*info != 0) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < kL * kL; e += NT) {
        const int i = e & (kL - 1), j = e >> 6;
        a[j][i] = (i < n && j < n) ? A[i + (int64_t)j * lda] : (i == j ? 1.0 : 0.0);
        w[j][i] = 0.0;
        v[j][i] = 0.0;
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += 16) {
        const int wd = min(16, n - k0);  // panel width
        if (tid < 64) {                  // the panel: lane tid holds row k0 + tid
            const int r = k0 + tid;
            const bool live = r < n;
            double x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = (live && c < wd) ? a[k0 + c][r] : 0.0;
            int bad = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < wd && bad == 0) {  // uniform
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
                    if (c < wd) a[k0 + c][r] = x[c];
            }
            if (tid == 0 && bad != 0) s_bad = bad;
        }
        __syncthreads();
        if (s_bad != 0) {  // uniform
            if (tid == 0) *info = (int32_t)(info_base + s_bad);
            return;
        }
        const int c0 = k0 + wd, rest = n - c0;
        if (rest <= 0) break;
        if (tid < rest) {  // U12 := L11^{-1} A12, column c0 + tid
            const int c = c0 + tid;
            double y[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) y[i] = i < wd ? a[c][k0 + i] : 0.0;
#pragma unroll
            for (int i = 1; i < 16; ++i)
#pragma unroll
                for (int k = 0; k < i; ++k) y[i] -= a[k0 + k][k0 + i] * y[k];  // L(k0 + i, k0 + k)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < wd) a[c][k0 + i] = y[i];
        }
        __syncthreads();
        for (int e = tid; e < rest * rest; e += NT) {  // A22 -= L21 U12, pivot by pivot
            const int rr = c0 + e % rest, cc = c0 + e / rest;
            double val = a[cc][rr];
            for (int k = 0; k < wd; ++k) val -= a[k0 + k][rr] * a[cc][k0 + k];
            a[cc][rr] = val;
        }
        __syncthreads();
    }
    for (int e = tid; e < kL * kL; e += NT) {
        const int i = e & (kL - 1), j = e >> 6;
        if (i < n && j < n) A[i + (int64_t)j * lda] = a[j][i];
    }
    if (P1 == nullptr) return;  // uniform
    // (2): a[c][r] holds L\U(r, c); the padding is the identity.
    const int t = tid % (NT / 2);
    const bool up = tid >= NT / 2;  // uniform per wavefront
    if (t < kL) {                // the diagonal 16-blocks: block b, column j of it
        const int b = t >> 4, j = t & 15, c = 16 * b + j;
        if (!up) {  // unit lower: rows j .. 15
            for (int i = j; i < 16; ++i) {
                const int r = 16 * b + i;
                double sum = (i == j) ? 1.0 : 0.0;
                for (int k = j; k < i; ++k) sum -= a[16 * b + k][r] * w[16 * b + k][c];
                w[r][c] = sum;
            }
        } else {  // upper: rows j .. 0
            for (int i = j; i >= 0; --i) {
                const int r = 16 * b + i;
                double sum = (i == j) ? 1.0 : 0.0;
                for (int k = i + 1; k <= j; ++k) sum -= a[16 * b + k][r] * v[16 * b + k][c];
                v[r][c] = sum / a[r][r];
            }
        }
    }
    __syncthreads();
    for (int h = 16; h < kL; h *= 2) {
        const int outs = (kL / (2 * h)) * h * h;  // pairs x h^2
        for (int e = t; e < outs; e += NT / 2) {     // the inner products, into the other triangle
            const int p = e / (h * h), q = e % (h * h), i = q % h, j = q / h;
            const int lo = 2 * h * p, hi = lo + h;
            double sum = 0.0;
            if (!up) {
                for (int k = j; k < h; ++k) sum += a[lo + k][hi + i] * w[lo + k][lo + j];  // L(hi, lo) W(lo, lo)
                w[lo + i][hi + j] = sum;
            } else {
                for (int k = 0; k <= j; ++k) sum += a[hi + k][lo + i] * v[hi + k][hi + j];  // U(lo, hi) V(hi, hi)
                v[hi + i][lo + j] = sum;
            }
        }
        __syncthreads();
        for (int e = t; e < outs; e += NT / 2) {
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
    for (int e = tid; e < n * n; e += NT) {
        const int i = e % n, c = e / n;
        P1[c + (int64_t)i * kL] = i >= c ? -w[i][c] : 0.0;  // P1(c, i) = -W(i, c)
        P2[i + (int64_t)c * kL] = i <= c ? -v[i][c] : 0.0;  // P2(i, c) = -V(i, c)
    }
}

// dst (cols x rows, ldd) := src^T, 64 x 64 tiles through LDS, grid (row
// tiles, column tiles); z1 and z2 (each null or cols x rows with ld ldd) are
// set to zero over the same tiles, which saves the fills of the products'
// scratch a launch each.  Skipped if info && *info.
__global__ __launch_bounds__(256) void k_transpose_copy(int64_t rows, int64_t cols, const double *__restrict__ src,
                                                        int64_t lds, double *__restrict__ dst, int64_t ldd,
                                                        double *__restrict__ z1, double *__restrict__ z2,
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
        if (dr < cols && dc < rows) {
            dst[dr + dc * ldd] = tile[tx][k];
            if (z1 != nullptr) z1[dr + dc * ldd] = 0.0;
            if (z2 != nullptr) z2[dr + dc * ldd] = 0.0;
        }
    }
}

}  // namespace

int launch_lu_diag(int n, double *A, int64_t lda, int32_t *info, int64_t info_base, double *P1, double *P2,
                   hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    if (n > kL) return FLAME_ERR_UNSUPPORTED;
    if ((P1 == nullptr) != (P2 == nullptr)) return FLAME_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_lu_diag<kDiagThreads>, dim3(1), dim3(kDiagThreads), 0, s, n, A, lda, info, info_base, P1, P2);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_transpose_copy(int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst, int64_t ldd,
                          const int32_t *info, hipStream_t s, double *z1, double *z2) {
    if (rows <= 0 || cols <= 0) return FLAME_OK;
    const dim3 grid((unsigned)((rows + kL - 1) / kL), (unsigned)((cols + kL - 1) / kL));
    hipLaunchKernelGGL(k_transpose_copy, grid, dim3(256), 0, s, rows, cols, src, lds, dst, ldd, z1, z2, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
