// Single-launch triangular solves and the tiled FP64 residual used by
// iterative refinement.
//
// Triangular solves (one right-hand side, row blocks of 128): workgroup i
// owns row block i.  For the forward solve U^T y = b it takes the finished
// blocks q < i as their flags appear, accumulates U(q, i)^T y_q, then applies
// the precomputed inverse of the diagonal block, y_i = U_ii^{-T} (b_i - sum),
// and publishes y_i.  The backward solve U x = y runs the blocks from the
// last one up.  U is read from HBM exactly once; the dependency chain per
// block is one 128 x 128 mat-vec and a flag.  Workgroups are dispatched in
// index order and wait only on lower indices, so the chain always makes
// progress; every wait is bounded (a wait that gives up sets *err, writes
// NaN over its block and lets the kernel finish).
#include "dev_sync.h"
#include "flame_internal.h"
#include "tile_map.h"

namespace flame {

constexpr int kTb = 128;                  // row block of the solves
constexpr long long kSpinLimit = 1LL << 26;  // s_sleep rounds before a wait gives up

__global__ void k_identity_blocks(int64_t nblk, int bs, double *__restrict__ Dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = nblk * bs * bs;
    if (i >= total) return;
    const int64_t e = i % ((int64_t)bs * bs);
    const int r = (int)(e % bs), c = (int)(e / bs);
    Dt[i] = (r == c) ? 1.0 : 0.0;
}

int launch_identity_blocks(int64_t nblk, int bs, double *Dt, hipStream_t s) {
    const int64_t total = nblk * bs * bs;
    if (total <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_identity_blocks, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, nblk, bs, Dt);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

// Waits (bounded) for a block's flag; false if it gave up or another wait
// did (*err).  The block itself is then read with device-scope loads.
__device__ __forceinline__ bool wait_flag(const int32_t *flag, int32_t *err) {
    return poll_at_least(flag, 1, err, 1, kSpinLimit);
}

// Publishes this workgroup's block: device-scope stores, completed by every
// wavefront before the barrier, then the flag.
__device__ __forceinline__ void publish(double *xi, int tid, int w, double v, bool bad, int32_t *flag) {
    if (tid < w) store_dev(xi + tid, bad ? __builtin_nan("") : v);
    wait_stores();
    __syncthreads();
    if (tid == 0) store_dev(flag, 1);
}

// U^T y = b in place on x (n x 1).  Thread (c, h): column c of the block,
// half h of the 128 rows of each contribution.  The operands that do not
// depend on earlier blocks (this block's inverse, the next U block) are
// loaded into registers before the wait.
__global__ __launch_bounds__(256) void k_trsv1_fwd(int64_t n, const double *__restrict__ U, int64_t ldu,
                                                   const double *__restrict__ Dt, double *x, int32_t *flags,
                                                   int32_t *err) {
    __shared__ double xs[kTb];
    __shared__ double part[2][kTb];
    __shared__ double rhs[kTb];
    __shared__ int bad;
    const int64_t i = blockIdx.x;
    const int64_t r0 = i * kTb;
    const int w = (int)min((int64_t)kTb, n - r0);
    const int tid = threadIdx.x;
    const int c = tid & (kTb - 1), h = tid >> 7;
    const int cc = min(c, w - 1);
    if (tid == 0) bad = 0;
    // d[k] = Dt_i(c, 64 h + k)
    const double *D = Dt + i * (int64_t)kTb * kTb + c + (int64_t)kTb * 64 * h;
    double d[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) d[k] = D[(int64_t)kTb * k];
    const double *Ucol = U + (r0 + cc) * ldu + 64 * h;  // column r0 + c of U, rows from 64 h
    double acc = 0.0;
    for (int64_t q = 0; q < i; ++q) {
        double u[64];
#pragma unroll
        for (int k = 0; k < 64; ++k) u[k] = Ucol[q * kTb + k];
        if (tid == 0 && !wait_flag(flags + q, err)) bad = 1;
        __syncthreads();
        if (tid < kTb) xs[tid] = load_dev(x + q * kTb + tid);  // block q < i is full
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 64; ++k) acc += u[k] * xs[64 * h + k];
    }
    part[h][c] = acc;
    __syncthreads();
    if (tid < kTb) rhs[tid] = (tid < w) ? x[r0 + tid] - (part[0][tid] + part[1][tid]) : 0.0;
    __syncthreads();
    double y = 0.0;  // y(c) = sum_k Dt_i(c, k) rhs(k); rhs is 0 past w
#pragma unroll
    for (int k = 0; k < 64; ++k) y += d[k] * rhs[64 * h + k];
    part[h][c] = y;
    __syncthreads();
    publish(x + r0, tid, w, part[0][tid & (kTb - 1)] + part[1][tid & (kTb - 1)], bad != 0, flags + i);
}

// U x = y in place on x; workgroup w handles row block nblk - 1 - w.
// Thread (r, h): row r of the block, half h of the 128 columns.
__global__ __launch_bounds__(256) void k_trsv1_bwd(int64_t n, const double *__restrict__ U, int64_t ldu,
                                                   const double *__restrict__ Dt, double *x, int32_t *flags,
                                                   int32_t *err) {
    __shared__ double xs[kTb];
    __shared__ double part[2][kTb];
    __shared__ double rhs[kTb];
    __shared__ int bad;
    const int64_t nblk = (n + kTb - 1) / kTb;
    const int64_t i = nblk - 1 - (int64_t)blockIdx.x;
    const int64_t r0 = i * kTb;
    const int w = (int)min((int64_t)kTb, n - r0);
    const int tid = threadIdx.x;
    const int r = tid & (kTb - 1), h = tid >> 7;
    const int64_t row = r0 + min(r, w - 1);
    if (tid == 0) bad = 0;
    // d[k] = Dt_i(64 h + k, r), i.e. U_ii^{-1}(r, 64 h + k)
    const double *D = Dt + i * (int64_t)kTb * kTb + (int64_t)kTb * r + 64 * h;
    double d[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) d[k] = D[k];
    double acc = 0.0;
    for (int64_t q = nblk - 1; q > i; --q) {
        double u[64];
        const int64_t c0 = q * kTb + 64 * h;
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            const int64_t col = c0 + k;
            const double v = U[row + min(col, n - 1) * ldu];
            u[k] = (col < n) ? v : 0.0;
        }
        const int wq = (int)min((int64_t)kTb, n - q * kTb);
        if (tid == 0 && !wait_flag(flags + q, err)) bad = 1;
        __syncthreads();
        if (tid < kTb) xs[tid] = (tid < wq) ? load_dev(x + q * kTb + tid) : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 64; ++k) acc += u[k] * xs[64 * h + k];
    }
    part[h][r] = acc;
    __syncthreads();
    if (tid < kTb) rhs[tid] = (tid < w) ? x[r0 + tid] - (part[0][tid] + part[1][tid]) : 0.0;
    __syncthreads();
    double y = 0.0;
#pragma unroll
    for (int k = 0; k < 64; ++k) y += d[k] * rhs[64 * h + k];
    part[h][r] = y;
    __syncthreads();
    publish(x + r0, tid, w, part[0][tid & (kTb - 1)] + part[1][tid & (kTb - 1)], bad != 0, flags + i);
}

int launch_trsv1(bool forward, int64_t n, const double *U, int64_t ldu, const double *Dt, double *x, int32_t *flags,
                 int32_t *err, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    const int64_t nblk = (n + kTb - 1) / kTb;
    int rc = launch_zero_i32(flags, nblk, s);
    if (rc) return rc;
    const int tr = trace_begin(FLAME_KC_OTHER, s);
    if (forward)
        hipLaunchKernelGGL(k_trsv1_fwd, dim3((unsigned)nblk), dim3(256), 0, s, n, U, ldu, Dt, x, flags, err);
    else
        hipLaunchKernelGGL(k_trsv1_bwd, dim3((unsigned)nblk), dim3(256), 0, s, n, U, ldu, Dt, x, flags, err);
    FLAME_CHECK_LAUNCH();
    const double dn = (double)n;
    trace_end(tr, s, dn * dn, 4.0 * dn * (dn + 1));
    return FLAME_OK;
}

// ---- residual R = B - A0 X through per-tile partials --------------------------
// Tile (I, J), I <= J, of the upper triangle of A0 (128 x 128, staged in LDS):
// threads 0..127 form row sums for block I (symmetric part of A0), threads
// 128..255 the transposed contribution to block J (I < J).  Partials
// P[I][J][k][r] (k < nrhs: A0 X, k = nrhs: |A0| row sums) are reduced in a
// fixed order by k_residual_reduce.
constexpr int kResMax = 8;

__global__ __launch_bounds__(256) void k_symv_tiles(int64_t n, int tn, int nrhs, const double *__restrict__ A,
                                                    int64_t lda, const double *__restrict__ X, int64_t ldx,
                                                    double *__restrict__ P) {
    __shared__ double As[kTb][kTb + 1];  // [column][row]
    __shared__ double xi[kResMax][kTb], xj[kResMax][kTb];
    int I, J;
    tile_of((int64_t)blockIdx.x, tn, tn, true, I, J);
    const int tid = threadIdx.x;
    const int64_t ri0 = (int64_t)I * kTb, cj0 = (int64_t)J * kTb;
    // the tile in two halves of 32 loads per thread, all issued before their
    // LDS stores (one load in flight at a time would leave the kernel
    // latency-bound)
    constexpr int kHalf = kTb * kTb / 512;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        double v[kHalf];
#pragma unroll
        for (int e = 0; e < kHalf; ++e) {
            const int idx = tid + 256 * (h * kHalf + e);
            const int c = idx >> 7, r = idx & (kTb - 1);
            v[e] = A[min(ri0 + r, n - 1) + min(cj0 + c, n - 1) * lda];
        }
#pragma unroll
        for (int e = 0; e < kHalf; ++e) {
            const int idx = tid + 256 * (h * kHalf + e);
            const int c = idx >> 7, r = idx & (kTb - 1);
            const int64_t gr = ri0 + r, gc = cj0 + c;
            As[c][r] = (gr < n && gc < n && gr <= gc) ? v[e] : 0.0;
        }
    }
    for (int idx = tid; idx < nrhs * kTb; idx += 256) {
        const int k = idx >> 7, r = idx & (kTb - 1);
        const int64_t gi = ri0 + r, gj = cj0 + r;
        xi[k][r] = (gi < n) ? X[gi + k * ldx] : 0.0;
        xj[k][r] = (gj < n) ? X[gj + k * ldx] : 0.0;
    }
    __syncthreads();
    const int nk = nrhs + 1;
    if (tid < kTb) {
        const int r = tid;
        double acc[kResMax];
#pragma unroll
        for (int k = 0; k < kResMax; ++k) acc[k] = 0.0;
        double asum = 0.0;
        for (int c = 0; c < kTb; ++c) {
            // symmetric element (r, c) of the tile: upper part, or its mirror on
            // a diagonal tile
            const double a = (I < J || r <= c) ? As[c][r] : As[r][c];
            asum += fabs(a);
#pragma unroll
            for (int k = 0; k < kResMax; ++k)
                if (k < nrhs) acc[k] += a * xj[k][c];
        }
        double *p = P + ((int64_t)I * tn + J) * nk * kTb;
#pragma unroll
        for (int k = 0; k < kResMax; ++k)
            if (k < nrhs) p[(int64_t)k * kTb + r] = acc[k];
        p[(int64_t)nrhs * kTb + r] = asum;
    } else if (I < J) {
        const int c = tid - kTb;
        double acc[kResMax];
#pragma unroll
        for (int k = 0; k < kResMax; ++k) acc[k] = 0.0;
        double asum = 0.0;
        for (int r = 0; r < kTb; ++r) {
            const double a = As[c][r];
            asum += fabs(a);
#pragma unroll
            for (int k = 0; k < kResMax; ++k)
                if (k < nrhs) acc[k] += a * xi[k][r];
        }
        double *p = P + ((int64_t)J * tn + I) * nk * kTb;
#pragma unroll
        for (int k = 0; k < kResMax; ++k)
            if (k < nrhs) p[(int64_t)k * kTb + c] = acc[k];
        p[(int64_t)nrhs * kTb + c] = asum;
    }
}

__global__ __launch_bounds__(256) void k_residual_reduce(int64_t n, int tn, int nrhs, const double *__restrict__ P,
                                                         const double *__restrict__ B, int64_t ldb,
                                                         double *__restrict__ R, int64_t ldr,
                                                         double *__restrict__ rowsums) {
    const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gi >= n) return;
    const int I = (int)(gi / kTb), r = (int)(gi % kTb);
    const int nk = nrhs + 1;
    for (int k = 0; k <= nrhs; ++k) {
        double y = 0.0;
        for (int J = 0; J < tn; ++J) y += P[(((int64_t)I * tn + J) * nk + k) * kTb + r];
        if (k < nrhs)
            R[gi + k * ldr] = (B != nullptr) ? B[gi + k * ldb] - y : y;
        else if (rowsums != nullptr)
            rowsums[gi] = y;
    }
}

size_t residual_workspace_doubles(int64_t n, int64_t nrhs) {
    const int64_t tn = (n + kTb - 1) / kTb;
    return (size_t)tn * tn * kTb * (size_t)(nrhs + 1);
}

int launch_residual_tiled(int64_t n, int64_t nrhs, const double *A0, int64_t lda0, const double *X, int64_t ldx,
                          const double *B, int64_t ldb, double *R, int64_t ldr, double *rowsums, double *part,
                          hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    if (nrhs > kResMax) return FLAME_ERR_UNSUPPORTED;
    const int tn = (int)((n + kTb - 1) / kTb);
    const int64_t ntiles = tile_count(tn, tn, true);
    const int tr = trace_begin(FLAME_KC_OTHER, s);
    hipLaunchKernelGGL(k_symv_tiles, dim3((unsigned)ntiles), dim3(256), 0, s, n, tn, (int)nrhs, A0, lda0, X, ldx,
                       part);
    FLAME_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_residual_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, tn, (int)nrhs, part,
                       B, ldb, R, ldr, rowsums);
    FLAME_CHECK_LAUNCH();
    const double dn = (double)n;
    trace_end(tr, s, 2.0 * dn * dn * (double)nrhs, 4.0 * dn * (dn + 1) + 24.0 * dn * (double)nrhs);
    return FLAME_OK;
}

}  // namespace flame
