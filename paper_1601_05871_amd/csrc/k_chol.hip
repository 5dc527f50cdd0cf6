// CHOL step of the loop body (Fig. "dense-chol"): A11 := Chol(A11) for one
// diagonal block of order n <= 256, upper triangle, in place.
//
// One workgroup of four wavefronts holds the block in LDS and walks it in
// S-column sub-blocks (the same right-looking loop one level down):
//   (a) wavefront 0 factors the S x S diagonal sub-block in registers: lane c
//       holds column c, the pivot and the row of U are broadcast with
//       v_readlane, so the unblocked loop (b = 1 in the figure) runs without a
//       barrier or an LDS round trip;
//   (b) every thread solves one column of the sub-block's row panel against the
//       fresh U (the TRSM step);
//   (c) the trailing block takes the rank-S update (the HERK step), 4 x 4
//       entries per thread.
// S = 16 keeps the unrolled register code small: the kernel runs as a single
// workgroup, so its code must stay in the instruction cache.  Blocks of order
// 129..256 take the same loop one level up (two LDS-resident blocks, the
// panel TRSM and the trailing update kernels in between).
#include "chol_wave.h"
#include "flame_internal.h"

namespace flame {

// LDS-resident form for n <= 128: the upper triangle is loaded into LDS once
// (packed column by column: 66 KB in FP64, so that the kernel fits on a CU
// beside one workgroup of the trailing update), padded with the identity to a
// multiple of the sub-block order S (so every sub-block is full and the
// unrolled register code needs no bounds guards), steps (a)-(c) run on LDS
// only, and the factor is written back once.  The padding stays the identity:
// its pivots are 1 and its coupling to the matrix is 0.
constexpr int kLdsN = 128;
constexpr int kPacked = kLdsN * (kLdsN + 1) / 2;  // upper triangle, packed by columns

// LDS position of element (i, c), i <= c, of the packed upper triangle
__device__ __forceinline__ int pk(int i, int c) { return c * (c + 1) / 2 + i; }

template <typename T, int S>
__global__ __launch_bounds__(256) void k_chol_lds(int n, T *__restrict__ A, int64_t lda, int32_t *__restrict__ info,
                                                  int64_t info_base) {
    constexpr int RMAX = kLdsN - S;       // widest trailing block
    __shared__ T L[kPacked];              // the block's upper triangle, packed columns
    __shared__ T Pt[S][RMAX + 4];         // the current panel rows, row-major
    __shared__ T rinv[S];                 // 1 / U(j, j) of the current sub-block
    __shared__ int s_bad;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (info != nullptr && *info != 0) return;
    const int np = (n + S - 1) / S * S;
    // load: all of this thread's loads first, then the LDS stores (lower
    // positions get a copy of an upper element, never used; padding rows and
    // columns >= n hold the identity)
    {
        constexpr int PER = kLdsN * kLdsN / 256;
        T v[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + 256 * e;
            const int col = idx >> 7, row = idx & (kLdsN - 1);
            v[e] = A[(int64_t)min(min(row, col), n - 1) + (int64_t)min(col, n - 1) * lda];
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = tid + 256 * e;
            const int col = idx >> 7, row = idx & (kLdsN - 1);
            if (row <= col && col < np)
                L[pk(row, col)] = (row < n && col < n) ? v[e] : (row == col ? T(1) : T(0));
        }
    }
    __syncthreads();

    // (a) of the first sub-block, then per sub-block: (b), and (c) with the
    // next diagonal block's share updated first by wavefront 0, which goes on
    // to factor it (the next (a)) while wavefronts 1-3 finish the update.
    auto diag = [&](int r0) {
        T a[S];
        // column r0 + c from row r0 (the entries read past the column's
        // diagonal belong to the next columns and are discarded)
        const T *colp = L + pk(r0, r0 + min(lane, S - 1));
#pragma unroll
        for (int i = 0; i < S; ++i) a[i] = colp[i];
        T ri;
        const int bad = chol_row16<T, S>(a, lane & 15, &ri);
        if (lane == 0) s_bad = bad;
        if (lane < S) {
            T *colw = L + pk(r0, r0 + lane);
#pragma unroll
            for (int i = 0; i < S; ++i)
                if (i <= lane) colw[i] = a[i];
            rinv[lane] = ri;
        }
    };
    // 4 x 4 tile idx (upper, column by column) of the trailing block at o
    auto tile_update = [&](int o, int idx) {
        int bj = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
        while (bj * (bj + 1) / 2 > idx) --bj;
        while ((bj + 1) * (bj + 2) / 2 <= idx) ++bj;
        const int bi = idx - bj * (bj + 1) / 2;
        T acc[4][4];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) acc[ii][jj] = T(0);
#pragma unroll 4
        for (int q = 0; q < S; ++q) {
            T pi[4], pj[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                pi[e] = Pt[q][4 * bi + e];
                pj[e] = Pt[q][4 * bj + e];
            }
#pragma unroll
            for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) acc[ii][jj] += pi[ii] * pj[jj];
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int ii = 0; ii < 4; ++ii)
                if (4 * bi + ii <= 4 * bj + jj) L[pk(o + 4 * bi + ii, o + 4 * bj + jj)] -= acc[ii][jj];
    };
    constexpr int kDiagTiles = (S / 4) * (S / 4 + 1) / 2;  // tiles of one S x S diagonal block

    if (wave == 0) diag(0);
    __syncthreads();
    for (int r0 = 0;; r0 += S) {
        if (__builtin_amdgcn_readfirstlane(s_bad) != 0) {  // uniform: a scalar branch
            if (tid == 0) *info = (int32_t)(info_base + r0 + s_bad);
            return;
        }
        const int rest = np - r0 - S;
        if (rest == 0) break;
        // (b) row panel: thread t owns column r0 + S + t
        if (tid < rest) {
            T x[S];
            T *colc = L + pk(r0, r0 + S + tid);
#pragma unroll
            for (int i = 0; i < S; ++i) x[i] = colc[i];
#pragma unroll
            for (int q = 0; q < S; ++q) {
                x[q] = x[q] * rinv[q];
#pragma unroll
                for (int t = q + 1; t < S; ++t) x[t] = x[t] - L[pk(r0 + q, r0 + t)] * x[q];
            }
#pragma unroll
            for (int i = 0; i < S; ++i) {
                colc[i] = x[i];
                Pt[i][tid] = x[i];
            }
        }
        __syncthreads();
        // (c) trailing update of the block at o = r0 + S in 4 x 4 tiles
        const int o = r0 + S;
        const int nb4 = rest >> 2;
        const int cnt = nb4 * (nb4 + 1) / 2;
        if (wave == 0) {
            if (lane < kDiagTiles) tile_update(o, lane);  // the next diagonal block
            __threadfence_block();                        // its LDS writes before the reads below
            diag(o);
        } else {
            for (int idx = kDiagTiles + tid - 64; idx < cnt; idx += 192) tile_update(o, idx);
        }
        __syncthreads();
    }
    // store the upper triangle
    for (int col = wave; col < n; col += 4)
        for (int row = lane; row <= col; row += 64) A[(int64_t)row + (int64_t)col * lda] = L[pk(row, col)];
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
