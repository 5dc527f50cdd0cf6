// TRSM step of the loop body (Fig. "dense-chol"): A12 := triu(A11)^{-T} A12,
// i.e. solve U^T X = A12 for X with U = triu(A11) (b x b, b <= 256) and
// A12 b x m.  (The figure prints triu(A11)^{-1}; only the transposed solve
// reproduces A = U^T U.)
//
// Columns of A12 are independent: one lane owns one column.  Rows are taken in
// chunks of 64 held in registers; inside a chunk the solve is a forward
// substitution, and each finished chunk immediately updates the rows below it
// (right-looking over chunks).  U is only ever addressed with wave-uniform
// indices, so its entries come in through scalar loads shared by the wave.
#include "flame_internal.h"

namespace flame {

template <typename T>
__global__ __launch_bounds__(64) void k_trsm_panel(int b, int64_t m, const T *__restrict__ U, int64_t ldu,
                                                   T *__restrict__ X, int64_t ldx,
                                                   const int32_t *__restrict__ info) {
    if (info != nullptr && *info != 0) return;
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool active = c < m;
    T *xc = X + (active ? c : 0) * ldx;
    for (int r0 = 0; r0 < b; r0 += 64) {
        const int w = min(64, b - r0);
        T x[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) x[i] = (active && i < w) ? xc[r0 + i] : T(0);
        // forward substitution with the chunk's diagonal block of U^T
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            if (t < w) {
                const T *ut = U + r0 + (int64_t)(r0 + t) * ldu;  // column r0 + t of U
                T acc = x[t];
#pragma unroll
                for (int q = 0; q < t; ++q) acc = acc - ut[q] * x[q];
                x[t] = acc / ut[t];
            }
        }
        if (active) {
#pragma unroll
            for (int i = 0; i < 64; ++i)
                if (i < w) xc[r0 + i] = x[i];
        }
        // rows below the chunk: x_r -= sum_q U(r0 + q, r) x_q
        for (int r = r0 + w; r < b; ++r) {
            const T *ur = U + r0 + (int64_t)r * ldu;  // column r of U, rows r0 ..
            T v = active ? xc[r] : T(0);
#pragma unroll
            for (int q = 0; q < 64; ++q)
                if (q < w) v = v - ur[q] * x[q];
            if (active) xc[r] = v;
        }
    }
}

template <typename T>
int launch_trsm_panel(int b, int64_t m, const T *U, int64_t ldu, T *X, int64_t ldx, const int32_t *info,
                      hipStream_t s) {
    if (b <= 0 || m <= 0) return FLAME_OK;
    const int64_t blocks = (m + 63) / 64;
    const int tr = trace_begin(FLAME_KC_TRSM, s);
    hipLaunchKernelGGL(k_trsm_panel<T>, dim3((unsigned)blocks), dim3(64), 0, s, b, m, U, ldu, X, ldx, info);
    FLAME_CHECK_LAUNCH();
    const double db = (double)b, dm = (double)m;
    trace_end(tr, s, db * db * dm, (db * (db + 1) / 2 + 2 * db * dm) * (double)sizeof(T));
    return FLAME_OK;
}

template int launch_trsm_panel<double>(int, int64_t, const double *, int64_t, double *, int64_t, const int32_t *,
                                       hipStream_t);
template int launch_trsm_panel<float>(int, int64_t, const float *, int64_t, float *, int64_t, const int32_t *,
                                      hipStream_t);

}  // namespace flame
