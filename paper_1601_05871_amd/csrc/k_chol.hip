// CHOL step of the loop body (Fig. "dense-chol"): A11 := Chol(A11) for one
// diagonal block of order n <= 256, upper triangle, in place.
//
// Orders up to 128: one workgroup holds the block's upper triangle in LDS as
// 16 x 16 tiles (72 KB in FP64, so that the kernel fits on a CU beside one
// workgroup of the trailing update) and factors it with the band loop of
// chol_lds.h (per 16-row band: one elimination pass over diagonal block and
// row panel, then a matrix-core rank-16 update); U goes to A straight from
// registers.  Orders 129..256 take the same loop one level up (two
// LDS-resident blocks, the panel TRSM and the trailing update kernels in
// between).
#include "chol_lds.h"
#include "flame_internal.h"

namespace flame {

constexpr int kLdsN = 128;

template <typename T, int S>
__global__ __launch_bounds__(256) void k_chol_lds(int n, T *__restrict__ A, int64_t lda, int32_t *__restrict__ info,
                                                  int64_t info_base) {
    __shared__ T L[band_lds_size<kLdsN>()];              // the block's upper triangle in 16 x 16 tiles
    __shared__ int s_bad;
    if (info != nullptr && *info != 0) return;
    band_load<T, kLdsN>(n, A, lda, L);
    __syncthreads();
    const int bad = chol_lds_core2<T, kLdsN>(n, L, &s_bad, A, lda);
    if (bad != 0 && threadIdx.x == 0) *info = (int32_t)(info_base + bad);
}

template <typename T>
int launch_chol_block(int n, T *A, int64_t lda, int32_t *info, int64_t info_base, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    if (n > kLdsN) {
        // n in (128, 256]: the same loop one level up, with the LDS kernel on the
        // two diagonal blocks: Chol(A11); A12 := U11^{-T} A12; A22 -= A12^T A12;
        // Chol(A22)
        const int n1 = kLdsN, n2 = n - kLdsN;
        int rc = launch_chol_block<T>(n1, A, lda, info, info_base, s);
        if (rc) return rc;
        rc = launch_trsm_panel<T>(n1, n2, A, lda, A + (int64_t)n1 * lda, lda, info, s);
        if (rc) return rc;
        rc = launch_gemm_tn(sizeof(T) == 8 ? Prec::F64 : Prec::F32, sizeof(T) == 8, true, n2, n2, n1,
                            A + (int64_t)n1 * lda, lda, A + (int64_t)n1 * lda, lda, A + n1 + (int64_t)n1 * lda, lda,
                            info, s);
        if (rc) return rc;
        return launch_chol_block<T>(n2, A + n1 + (int64_t)n1 * lda, lda, info, info_base + n1, s);
    }
    const int tr = trace_begin(FLAME_KC_CHOL, s);
    hipLaunchKernelGGL((k_chol_lds<T, 16>), dim3(1), dim3(256), 0, s, n, A, lda, info, info_base);
    FLAME_CHECK_LAUNCH();
    const double dn = (double)n;
    trace_end(tr, s, dn * (dn + 1) * (2 * dn + 1) / 6.0, dn * (dn + 1) * (double)sizeof(T));
    return FLAME_OK;
}

template int launch_chol_block<double>(int, double *, int64_t, int32_t *, int64_t, hipStream_t);
template int launch_chol_block<float>(int, float *, int64_t, int32_t *, int64_t, hipStream_t);

// info[0 .. count) := 0 with a kernel (not a memset node: the loop may be
// captured into a graph).
__global__ void k_zero_i32(int32_t *p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

int launch_zero_i32(int32_t *p, int64_t count, hipStream_t s) {
    if (count <= 0) return FLAME_OK;
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
