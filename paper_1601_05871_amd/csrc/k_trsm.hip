// TRSM step of the loop body (Fig. "dense-chol"): A12 := triu(A11)^{-T} A12,
// i.e. solve U^T X = A12 for X with U = triu(A11) (b x b, b <= 256) and
// A12 b x m.  (The figure prints triu(A11)^{-1}; only the transposed solve
// reproduces A = U^T U.)
//
// Columns of A12 are independent: one lane owns one column.  Rows are taken in
// chunks of 32 held in registers; inside a chunk the solve is a forward
// substitution, and each finished chunk immediately updates the rows below it
// (right-looking over chunks).  U is only ever addressed with wave-uniform
// indices, so its entries come in through scalar loads shared by the wave.
#include "flame_internal.h"

namespace flame {

constexpr int TCH = 32;  // rows per register chunk

template <typename T>
__global__ __launch_bounds__(64) void k_trsm_panel(int b, int64_t m, const T *__restrict__ U, int64_t ldu,
                                                   T *__restrict__ X, int64_t ldx,
                                                   const int32_t *__restrict__ info) {
    if (info != nullptr && *info != 0) return;
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool active = c < m;
    T *xc = X + (active ? c : 0) * ldx;
    for (int r0 = 0; r0 < b; r0 += TCH) {
        const int w = min(TCH, b - r0);
        T x[TCH];
#pragma unroll
        for (int i = 0; i < TCH; ++i) x[i] = (active && i < w) ? xc[r0 + i] : T(0);
        // forward substitution with the chunk's diagonal block of U^T
#pragma unroll
        for (int t = 0; t < TCH; ++t) {
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
            for (int i = 0; i < TCH; ++i)
                if (i < w) xc[r0 + i] = x[i];
        }
        // rows below the chunk: x_r -= sum_q U(r0 + q, r) x_q
        for (int r = r0 + w; r < b; ++r) {
            const T *ur = U + r0 + (int64_t)r * ldu;  // column r of U, rows r0 ..
            T v = active ? xc[r] : T(0);
#pragma unroll
            for (int q = 0; q < TCH; ++q)
                if (q < w) v = v - ur[q] * x[q];
            if (active) xc[r] = v;
        }
    }
}

// ---- FP64 matrix-core panel solve -----------------------------------------
// The same solve blocked by 16 rows, each wavefront owning 16 columns of X:
//   R   = X_s - sum_{q < s} U(q, s)^T X_q   (16 x 16 blocks, MFMA)
//   X_s = D_s^{-T} R                        (D_s^{-1}: inverse of the 16 x 16
//                                            diagonal block of U, MFMA)
// The workgroup inverts the diagonal blocks once (back substitution, one lane
// per column) into LDS; the solved rows of each wavefront stay in LDS for the
// later blocks.  MFMA operand/output placement as in the trailing update:
// lane (r, g) holds row r, columns g + 4v of a 16 x 16 result.
typedef double d4v __attribute__((ext_vector_type(4)));

template <int NW, int BMAX>
__global__ __launch_bounds__(64 * NW) void k_trsm_mfma(int b, int64_t m, const double *__restrict__ U, int64_t ldu,
                                                      double *__restrict__ X, int64_t ldx,
                                                      const int32_t *__restrict__ info) {
    constexpr int P = 17;  // padded row length
    __shared__ double Xs[NW][BMAX][P];       // solved rows, [row][column] per wavefront
    __shared__ double Dv[BMAX / 16][16][P];  // D_s^{-1}, [k][i]
    __shared__ double Rt[NW][16][P];         // R of the current block, [row][column]
    if (info != nullptr && *info != 0) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15;
    const int g = lane >> 4;
    const int nblk = (b + 15) >> 4;
    // U(i, j) with rows/columns >= b read as the identity
    auto uat = [&](int i, int j) -> double {
        const bool in = (i < b) && (j < b);
        const double v = U[(int64_t)min(i, b - 1) + (int64_t)min(j, b - 1) * ldu];
        return in ? v : (i == j ? 1.0 : 0.0);
    };

    // (1) inverses of the diagonal blocks: wavefront w takes blocks w, w + NW, ..;
    //     lane t < 16 computes column t of D_s^{-1} (U D = I, back substitution)
    for (int sb = wave; sb < nblk; sb += NW) {
        const int o = 16 * sb;
        if (lane < 16) {
            const int t = lane;
            double v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = 0.0;
#pragma unroll
            for (int i = 15; i >= 0; --i) {
                if (i <= t) {
                    double acc = (i == t) ? 1.0 : 0.0;
#pragma unroll
                    for (int k = i + 1; k < 16; ++k)
                        if (k <= t) acc -= uat(o + i, o + k) * v[k];
                    v[i] = acc / uat(o + i, o + i);
                }
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) Dv[sb][i][t] = v[i];  // D(i, t), i.e. [k = i][column t]
        }
    }
    __syncthreads();

    const int64_t c0 = ((int64_t)blockIdx.x * NW + wave) * 16;  // this wavefront's first column
    const bool colok_any = c0 < m;
    for (int s = 0; s < nblk; ++s) {
        const int rs = 16 * s;
        // R = X_s (rows rs + r, columns c0 + g + 4v)
        d4v acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = c0 + g + 4 * v;
            const int row = rs + r;
            const double x = X[(int64_t)min(row, b - 1) + min(col, m - 1) * ldx];
            acc[v] = (row < b && col < m) ? x : 0.0;
        }
        // R -= U(q-rows, s-cols)^T X_q for q < s; k slot (g, t) <-> row 16q + 4g + t
        for (int q = 0; q < s; ++q) {
            const int kq = 16 * q + 4 * g;
            double uq[4], xq[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                uq[t] = uat(kq + t, rs + r);       // U(k, rs + i), i = r
                xq[t] = -Xs[wave][kq + t][r];      // X(k, column r), negated
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xq[t], uq[t], acc, 0, 0, 0);
        }
        // R to LDS as [row][column]
#pragma unroll
        for (int v = 0; v < 4; ++v) Rt[wave][r][g + 4 * v] = acc[v];
        __syncthreads();
        // X_s = D_s^{-T} R
        d4v xs = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * g + t;
            xs = __builtin_amdgcn_mfma_f64_16x16x4f64(Rt[wave][k][r], Dv[s][k][r], xs, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            Xs[wave][rs + r][g + 4 * v] = xs[v];
            const int64_t col = c0 + g + 4 * v;
            if (colok_any && rs + r < b && col < m) X[(int64_t)(rs + r) + col * ldx] = xs[v];
        }
        __syncthreads();
    }
}

template <typename T>
int launch_trsm_panel(int b, int64_t m, const T *U, int64_t ldu, T *X, int64_t ldx, const int32_t *info,
                      hipStream_t s) {
    if (b <= 0 || m <= 0) return FLAME_OK;
    const int tr = trace_begin(FLAME_KC_TRSM, s);
    if constexpr (sizeof(T) == 8) {
        if (b <= 128) {
            const int64_t blocks = (m + 63) / 64;
            hipLaunchKernelGGL((k_trsm_mfma<4, 128>), dim3((unsigned)blocks), dim3(256), 0, s, b, m, U, ldu, X, ldx,
                               info);
        } else {
            const int64_t blocks = (m + 31) / 32;
            hipLaunchKernelGGL((k_trsm_mfma<2, 256>), dim3((unsigned)blocks), dim3(128), 0, s, b, m, U, ldu, X, ldx,
                               info);
        }
    } else {
        const int64_t blocks = (m + 63) / 64;
        hipLaunchKernelGGL(k_trsm_panel<T>, dim3((unsigned)blocks), dim3(64), 0, s, b, m, U, ldu, X, ldx, info);
    }
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
