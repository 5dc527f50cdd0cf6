// Lower storage (A = L L^T with L in the lower triangle of a column-major A):
// the kernels of the loop read and write the upper triangle, and the lower
// triangle of a column-major matrix is the upper triangle of its transpose,
// so flame_factor with FLAME_OPT_LOWER swaps the two strict triangles in
// place, factors, and swaps back: the factor U = L^T lands in the lower
// triangle and the caller's strictly upper triangle comes back untouched.
// Each workgroup swaps one pair of mirrored 64 x 64 tiles (or transposes a
// diagonal tile in place) through LDS, reading and writing whole columns.
#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kTs = 64;

template <typename T>
__global__ __launch_bounds__(256) void k_swap_triangles(int64_t n, T *A, int64_t lda) {
    __shared__ T lo[kTs][kTs + 1], up[kTs][kTs + 1];  // [column][row]
    const int64_t t = blockIdx.x;
    // tile pair t = I (I + 1) / 2 + J, J <= I: lower tile (I, J), upper tile (J, I)
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t r0 = I * kTs, c0 = J * kTs;
    const int tx = threadIdx.x & (kTs - 1), ty = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kTs / 4; ++k) {
        const int cc = ty + 4 * k, rr = tx;
        const int64_t gr = r0 + rr, gc = c0 + cc;  // lower tile element
        lo[cc][rr] = (gr < n && gc < n) ? A[gr + gc * lda] : T(0);
        const int64_t ur = c0 + rr, uc = r0 + cc;  // upper tile element
        up[cc][rr] = (ur < n && uc < n) ? A[ur + uc * lda] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTs / 4; ++k) {
        const int cc = ty + 4 * k, rr = tx;
        if (I == J) {  // diagonal tile: transpose in place, the diagonal stays
            const int64_t gr = r0 + rr, gc = c0 + cc;
            if (rr != cc && gr < n && gc < n) A[gr + gc * lda] = lo[rr][cc];
        } else {
            const int64_t gr = r0 + rr, gc = c0 + cc;  // new lower (gr, gc) = old upper (gc, gr)
            if (gr < n && gc < n) A[gr + gc * lda] = up[rr][cc];
            const int64_t ur = c0 + rr, uc = r0 + cc;  // new upper (ur, uc) = old lower (uc, ur)
            if (ur < n && uc < n) A[ur + uc * lda] = lo[rr][cc];
        }
    }
}

}  // namespace

template <typename T>
int launch_swap_triangles(int64_t n, T *A, int64_t lda, hipStream_t s) {
    if (n <= 1) return FLAME_OK;
    const int64_t nt = (n + kTs - 1) / kTs;
    const int64_t pairs = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_swap_triangles<T>, dim3((unsigned)pairs), dim3(256), 0, s, n, A, lda);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

template int launch_swap_triangles<double>(int64_t, double *, int64_t, hipStream_t);
template int launch_swap_triangles<float>(int64_t, float *, int64_t, hipStream_t);
template int launch_swap_triangles<zdouble>(int64_t, zdouble *, int64_t, hipStream_t);

}  // namespace flame
