// CHOL step of the loop body (Fig. "dense-chol"): A11 := Chol(A11) for one
// diagonal block of order n <= 256, upper triangle, in place.
//
// One workgroup of four wavefronts walks the block in SB-column sub-blocks
// (the same right-looking loop one level down):
//   (a) wavefront 0 factors the SB x SB diagonal sub-block in registers: lane
//       c holds column c, the pivot and the row of U are broadcast with
//       v_readlane, so the unblocked loop (b = 1 in the figure) runs without a
//       barrier or an LDS round trip;
//   (b) every thread solves one column of the sub-block's row panel against the
//       fresh U (the TRSM step), U staged in LDS;
//   (c) the trailing block takes the rank-SB update (the HERK step) from the
//       panel, staged in LDS.
// SB = 32 keeps the unrolled register code of (a) and (b) small enough to stay
// in the instruction cache while the loop over sub-blocks repeats it.  The
// block lives in L2 between the steps (512 KiB at n = 256 in FP64).
#include "flame_internal.h"

namespace flame {

__device__ __forceinline__ double rdlane(double v, int l) {
    unsigned long long u = (unsigned long long)__double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
    int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

constexpr int SB = 32;  // sub-block order

// Unblocked right-looking Cholesky of a w x w (w <= SB) upper block held one
// column per lane: a[i] = A(i, lane) for i <= lane (other entries 0).  On
// return a[i] = U(i, lane) for i <= lane.  Returns 0, or the 1-based local
// column of the first pivot that is not > 0 (the rest is then unspecified).
template <typename T>
__device__ __forceinline__ int chol_wave_regs(T (&a)[SB], int w, int lane) {
    int bad = 0;
#pragma unroll
    for (int j = 0; j < SB; ++j) {
        if (j < w && bad == 0) {
            const T djj = rdlane(a[j], j);  // pivot A(j, j), uniform
            if (!(djj > T(0))) {
                bad = j + 1;
            } else {
                const T s = sqrt(djj);
                const T q = a[j] / s;  // U(j, c) = A(j, c) / U(j, j)
                a[j] = (lane == j) ? s : (lane > j ? q : a[j]);
#pragma unroll
                for (int i = j + 1; i < SB; ++i) {
                    if (i < w) {
                        const T uji = rdlane(a[j], i);  // U(j, i), uniform
                        a[i] = a[i] - uji * a[j];       // A(i, c) -= U(j, i) U(j, c)
                    }
                }
            }
        }
    }
    return bad;
}

template <typename T>
__global__ __launch_bounds__(256) void k_chol_block(int n, T *__restrict__ A, int64_t lda, int32_t *__restrict__ info,
                                                    int64_t info_base) {
    constexpr int RMAX = 256 - SB;  // widest trailing block
    __shared__ T Us[SB][SB + 1];    // U of the current diagonal sub-block, [row][col]
    __shared__ T Ps[SB][RMAX + 4];  // the sub-block's row panel after its TRSM, [row][col]
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (info != nullptr && *info != 0) return;  // an earlier block broke down

    for (int r0 = 0; r0 < n; r0 += SB) {
        const int w = min(SB, n - r0);
        const int rest = n - r0 - w;
        // (a) diagonal sub-block in the registers of wavefront 0
        if (wave == 0) {
            T a[SB];
            T *col = A + r0 + (int64_t)(r0 + (lane < w ? lane : 0)) * lda;
            // unconditional loads from clamped rows (no branch per element, so
            // they are all in flight at once); unused entries are zeroed
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const T v = col[min(i, w - 1)];
                a[i] = (lane < w && i <= lane) ? v : T(0);
            }
            const int bad = chol_wave_regs(a, w, lane);
            if (lane == 0) s_bad = bad;
            if (lane < w) {
#pragma unroll
                for (int i = 0; i < SB; ++i) {
                    if (i <= lane) col[i] = a[i];
                    Us[i][lane] = a[i];
                }
            }
        }
        __syncthreads();
        if (s_bad != 0) {
            if (tid == 0) *info = (int32_t)(info_base + r0 + s_bad);
            return;
        }
        if (rest > 0) {
            // (b) row panel: column c = r0 + w + tid, rows r0 .. r0 + w - 1
            if (tid < rest) {
                T x[SB];
                T *colc = A + r0 + (int64_t)(r0 + w + tid) * lda;
#pragma unroll
                for (int i = 0; i < SB; ++i) {
                    const T v = colc[min(i, w - 1)];
                    x[i] = (i < w) ? v : T(0);
                }
#pragma unroll
                for (int q = 0; q < SB; ++q) {
                    if (q < w) {
                        x[q] = x[q] / Us[q][q];
#pragma unroll
                        for (int t = q + 1; t < SB; ++t) x[t] = x[t] - Us[q][t] * x[q];
                    }
                }
#pragma unroll
                for (int i = 0; i < SB; ++i) {
                    if (i < w) colc[i] = x[i];
                    Ps[i][tid] = (i < w) ? x[i] : T(0);
                }
            }
            __syncthreads();
            // (c) trailing rest x rest upper block -= panel^T panel, 4 x 4 per thread
            const int nb4 = (rest + 3) >> 2;
            const int cnt = nb4 * (nb4 + 1) / 2;
            T *T0 = A + (r0 + w) + (int64_t)(r0 + w) * lda;
            for (int idx = tid; idx < cnt; idx += 256) {
                int bj = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
                while (bj * (bj + 1) / 2 > idx) --bj;
                while ((bj + 1) * (bj + 2) / 2 <= idx) ++bj;
                const int bi = idx - bj * (bj + 1) / 2;
                T acc[4][4];
#pragma unroll
                for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) acc[ii][jj] = T(0);
                for (int q = 0; q < w; ++q) {
                    T pi[4], pj[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        pi[e] = Ps[q][4 * bi + e];
                        pj[e] = Ps[q][4 * bj + e];
                    }
#pragma unroll
                    for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) acc[ii][jj] += pi[ii] * pj[jj];
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int j = 4 * bj + jj;
                    if (j < rest) {
#pragma unroll
                        for (int ii = 0; ii < 4; ++ii) {
                            const int i = 4 * bi + ii;
                            if (i <= j) T0[i + (int64_t)j * lda] -= acc[ii][jj];
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <typename T>
int launch_chol_block(int n, T *A, int64_t lda, int32_t *info, int64_t info_base, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    const int tr = trace_begin(FLAME_KC_CHOL, s);
    hipLaunchKernelGGL(k_chol_block<T>, dim3(1), dim3(256), 0, s, n, A, lda, info, info_base);
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
