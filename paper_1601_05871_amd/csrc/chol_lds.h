// The LDS-resident factorization of a diagonal block of order <= NMAX
// (CHOL step of Fig. "dense-chol"), shared by the single-block kernel and the
// batched kernel.  The block's upper triangle is packed column by column in
// LDS (element (i, c), i <= c, at c (c + 1) / 2 + i), padded with the identity
// to a multiple of the sub-block order S, and factored right-looking in
// S-column sub-blocks:
//   (a) wavefront 0 factors the S x S diagonal sub-block in registers (one
//       column per lane, chol_row16);
//   (b) every thread solves one column of the sub-block's row panel against
//       the fresh U (the TRSM step);
//   (c) the trailing block takes the rank-S update (the HERK step) in 4 x 4
//       register tiles; the next diagonal sub-block's tiles are updated first
//       by wavefront 0, which then factors it (the next (a)) while wavefronts
//       1-3 finish the update.
// All functions are called by the whole workgroup (256 threads) with uniform
// control flow.
#pragma once

#include "chol_wave.h"

namespace flame {

// LDS position of element (i, c), i <= c, of a packed upper triangle
__device__ __forceinline__ int pk(int i, int c) { return c * (c + 1) / 2 + i; }

template <int NMAX>
constexpr int packed_size() {
    return NMAX * (NMAX + 1) / 2;
}

// Loads the upper triangle of the n x n block A (n <= NMAX) into L, padded
// with the identity up to np = n rounded up to S.  All loads are issued first,
// then the LDS stores.
template <typename T, int NMAX, int S>
__device__ __forceinline__ void chol_lds_load(int n, const T *__restrict__ A, int64_t lda, T *L) {
    constexpr int PER = NMAX * NMAX / 256;
    const int tid = threadIdx.x;
    const int np = (n + S - 1) / S * S;
    T v[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = tid + 256 * e;
        const int col = idx / NMAX, row = idx % NMAX;
        v[e] = A[(int64_t)min(min(row, col), n - 1) + (int64_t)min(col, n - 1) * lda];
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = tid + 256 * e;
        const int col = idx / NMAX, row = idx % NMAX;
        if (row <= col && col < np) L[pk(row, col)] = (row < n && col < n) ? v[e] : (row == col ? T(1) : T(0));
    }
}

// Writes the factored upper triangle (order n) back to A.
template <typename T>
__device__ __forceinline__ void chol_lds_store(int n, T *__restrict__ A, int64_t lda, const T *L) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int col = wave; col < n; col += 4)
        for (int row = lane; row <= col; row += 64) A[(int64_t)row + (int64_t)col * lda] = L[pk(row, col)];
}

// Factors the packed block of padded order np (a multiple of S) in place.
// Returns 0, or the 1-based position of the first pivot that is not > 0.
// Pt: S x (NMAX - S + 4) panel rows; rinv: S entries; s_bad: one int.
template <typename T, int S, int NMAX>
__device__ int chol_lds_core(int np, T *L, T (*Pt)[NMAX - S + 4], T *rinv, int *s_bad) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    auto diag = [&](int r0) {
        T a[S];
        // column r0 + c from row r0 (the entries read past the column's
        // diagonal belong to the next columns and are discarded)
        const T *colp = L + pk(r0, r0 + min(lane, S - 1));
#pragma unroll
        for (int i = 0; i < S; ++i) a[i] = colp[i];
        T ri;
        const int bad = chol_row16<T, S>(a, lane & 15, &ri);
        if (lane == 0) *s_bad = bad;
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
        const int bad = __builtin_amdgcn_readfirstlane(*s_bad);  // uniform: a scalar branch
        if (bad != 0) return r0 + bad;
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
                // one row of U at a time: all S (S - 1) / 2 LDS reads issued
                // up front would hold as many registers
                __builtin_amdgcn_sched_barrier(0);
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
    return 0;
}

}  // namespace flame
