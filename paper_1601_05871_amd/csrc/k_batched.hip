// Batched factorization: many independent matrices A_i := Chol(A_i) (upper,
// in place) of uneven orders in one persistent launch.
//
// Work distribution: the matrices are ordered by decreasing order n_i
// (counting sort on the device: histogram, scan, scatter), and a persistent
// grid of (CUs x resident workgroups) takes them from an atomic counter in
// that order, largest first, so the long factorizations start early and the
// small ones fill the tail (longest-processing-time-first scheduling).
//
// One workgroup (4 wavefronts) factors one matrix with the right-looking loop
// of Fig. "dense-chol" at block size kBB = 128, on the matrix in HBM / L2:
//   CHOL  the 128 x 128 diagonal block in LDS as 16 x 16 tiles, factored
//         band by band with matrix-core trailing updates (chol_lds.h), U11
//         stored as each band is done;
//   TRSM  the 128-row panel on matrix cores, 16 columns per wavefront
//         (trsm_rl.h);
//   SYRK  the upper 32 x 32 tiles of A22 are spread over the wavefronts; each
//         tile is a 2 x 2 set of 16 x 16 matrix-core products (FP64 or FP32
//         MFMA, K = 128) accumulated onto the tile of A22.
// The diagonal block's LDS tiles and the TRSM scratch share one union (73.7 KB
// in FP64), so two workgroups fit on a CU.  A matrix of order <= 128 is one
// CHOL step.
// A breakdown stops that matrix only (info[i] = first bad column, 1-based).
#include "chol_lds.h"
#include "flame_internal.h"
#include "trsm_rl.h"

namespace flame {

#ifndef FLAME_BATCH_BB
#define FLAME_BATCH_BB 128
#endif
constexpr int kBB = FLAME_BATCH_BB;  // block size inside a workgroup (64 or 128; 128 measured faster)
constexpr int kBatchMaxN = 1024;   // largest order accepted
constexpr int kBuckets = kBatchMaxN + 2;  // orders 0..1024, plus one for invalid entries

typedef double bd4 __attribute__((ext_vector_type(4)));
typedef float bf4 __attribute__((ext_vector_type(4)));

template <typename T>
struct BAcc;
template <>
struct BAcc<double> {
    typedef bd4 type;
};
template <>
struct BAcc<float> {
    typedef bf4 type;
};

// acc += x^T y for one k slot.  FP64: lane (r, g) item v of the result is
// element (r, g + 4v) of the 16 x 16 block; FP32: element (4g + v, r).
__device__ __forceinline__ bd4 mma(double x, double y, bd4 acc) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(y, x, acc, 0, 0, 0);
}
__device__ __forceinline__ bf4 mma(float x, float y, bf4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc, 0, 0, 0);
}

// Row and column (within a 16 x 16 block) of accumulator item v of lane (r, g).
template <typename T>
__device__ __forceinline__ int acc_row(int r, int g, int v) {
    return sizeof(T) == 8 ? r : 4 * g + v;
}
template <typename T>
__device__ __forceinline__ int acc_col(int r, int g, int v) {
    return sizeof(T) == 8 ? g + 4 * v : r;
}

// C := C - P^T P on the upper triangle of the m x m matrix C, P is kBB x m.
// Upper 32 x 32 tiles, column by column, are handed to the wavefronts in turn.
template <typename T>
__device__ void syrk_tiles(int m, const T *__restrict__ P, int64_t ldp, T *__restrict__ C, int64_t ldc, int wave,
                           int lane) {
    typedef typename BAcc<T>::type acc_t;
    const int r = lane & 15, g = lane >> 4;
    const int nt = (m + 31) >> 5;
    const int ntasks = nt * (nt + 1) / 2;
    for (int task = wave; task < ntasks; task += 4) {
        int J = (int)((sqrtf(8.0f * (float)task + 1.0f) - 1.0f) * 0.5f);
        while (J * (J + 1) / 2 > task) --J;
        while ((J + 1) * (J + 2) / 2 <= task) ++J;
        const int I = task - J * (J + 1) / 2;
        const int rb = 32 * I, cb = 32 * J;
        acc_t acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = rb + 16 * a + acc_row<T>(r, g, v);
                    const int j = cb + 16 * b + acc_col<T>(r, g, v);
                    acc[a][b][v] = C[(int64_t)min(i, m - 1) + (int64_t)min(j, m - 1) * ldc];
                }
        // operand columns (clamped; products of clamped columns are never stored)
        const T *xp[2], *yp[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            xp[a] = P + (int64_t)min(rb + 16 * a + r, m - 1) * ldp;
            yp[a] = P + (int64_t)min(cb + 16 * a + r, m - 1) * ldp;
        }
#pragma unroll
        for (int kc = 0; kc < kBB; kc += 16) {
            // lane (r, g) supplies k = kc + 4g + t in MFMA step t for both
            // operands, so the k slots agree whatever the hardware's order
            T x[2][4], y[2][4];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    x[a][t] = -xp[a][kc + 4 * g + t];
                    y[a][t] = yp[a][kc + 4 * g + t];
                }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) acc[a][b] = mma(x[a][t], y[b][t], acc[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = rb + 16 * a + acc_row<T>(r, g, v);
                    const int j = cb + 16 * b + acc_col<T>(r, g, v);
                    if (i <= j && j < m) C[(int64_t)i + (int64_t)j * ldc] = acc[a][b][v];
                }
    }
}

// Workgroup-shared scratch of factor_one: the diagonal block's tiles during
// CHOL, the TRSM inverses and per-wavefront staging afterwards.
template <typename T>
struct BatchLds {
    union {
        T L[band_lds_size<kBB>()];  // diagonal block, upper 16 x 16 tiles
        struct {
            T Ds[kBB / 16][16][17];  // inverses of the 16 x 16 diagonal blocks of U11
            T Rt[4][16][17];         // per wavefront TRSM scratch
        } t;
    };
    int s_bad;
};

// Factors one matrix with the whole workgroup; returns the info value.
template <typename T>
__device__ int factor_one(int n, T *__restrict__ A, int64_t lda, BatchLds<T> &sh) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    for (int k0 = 0; k0 < n; k0 += kBB) {
        const int bk = min(kBB, n - k0);
        const int m = n - k0 - bk;
        T *A11 = A + k0 + (int64_t)k0 * lda;
        // CHOL: the block's tiles in LDS, U11 stored to A11 band by band
        band_load<T, kBB>(bk, A11, lda, sh.L);
        __syncthreads();
        const int bad = chol_lds_core2<T, kBB>(bk, sh.L, &sh.s_bad, A11, lda);
        if (bad != 0) return k0 + bad;
        __syncthreads();  // U11 in memory for every wavefront; L free again
        if (m == 0) break;
        // TRSM: A12 := U11^{-T} A12 (bk == kBB here)
        T *A12 = A + k0 + (int64_t)(k0 + kBB) * lda;
        trsm_inverses<T, kBB / 16, true>(kBB, A11, lda, sh.t.Ds);
        __syncthreads();
        for (int c0 = 16 * wave; c0 < m; c0 += 64) {
            // keeps the U11 loads inside the loop (hoisted, they would not fit
            // in registers)
            asm volatile("" ::: "memory");
            trsm_cols<T, kBB / 16, true>(kBB, m, A11, lda, A12, lda, c0, sh.t.Ds, sh.t.Rt[wave]);
        }
        __syncthreads();
        // SYRK: A22 -= A12^T A12 (upper)
        syrk_tiles<T>(m, A12, lda, A + (k0 + kBB) + (int64_t)(k0 + kBB) * lda, lda, wave, lane);
        __syncthreads();
    }
    return 0;
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_batched(int32_t batch, const int32_t *__restrict__ ns, T *const *As,
                                                    const int32_t *__restrict__ ldas, int32_t *__restrict__ info,
                                                    const int32_t *__restrict__ order, int32_t *counter) {
    __shared__ BatchLds<T> sh;
    __shared__ int s_item;
    const int tid = threadIdx.x;
    // Every value that steers the loop is made wave-uniform (readfirstlane):
    // the branches around the barriers are then scalar, and every lane of a
    // wavefront takes the same path through them.
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (t >= batch) break;  // every wave of the workgroup leaves together
        const int i = __builtin_amdgcn_readfirstlane(order[t]);
        const int n = __builtin_amdgcn_readfirstlane(ns[i]);
        const int lda = __builtin_amdgcn_readfirstlane(ldas[i]);
        int res = -1;  // order out of range or lda < n: not touched
        if (n >= 0 && n <= kBatchMaxN && lda >= max(1, n)) res = factor_one<T>(n, As[i], (int64_t)lda, sh);
        if (tid == 0) info[i] = res;
        __syncthreads();
    }
}

// ---- ordering: counting sort by decreasing order ------------------------------
__device__ __forceinline__ int bucket_of(int n, int lda) {
    return (n < 0 || n > kBatchMaxN || lda < max(1, n)) ? kBatchMaxN + 1 : n;
}

__global__ void k_batch_hist(int32_t batch, const int32_t *__restrict__ ns, const int32_t *__restrict__ ldas,
                             int32_t *hist) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch) atomicAdd(hist + bucket_of(ns[i], ldas[i]), 1);
}

// start[b] = number of entries in buckets that come before b: invalid entries
// first (they finish at once), then orders from kBatchMaxN down to 0.
__global__ __launch_bounds__(256) void k_batch_scan(int32_t *hist) {
    constexpr int PER = (kBuckets + 255) / 256;
    __shared__ int part[256];
    const int tid = threadIdx.x;
    // position p in processing order: p = 0 is the invalid bucket, then
    // p = 1 + (kBatchMaxN - n)
    int loc[PER];
    int sum = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int p = tid * PER + e;
        const int b = (p == 0) ? kBatchMaxN + 1 : kBatchMaxN - (p - 1);
        loc[e] = (p < kBuckets) ? hist[b] : 0;
        sum += loc[e];
    }
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int v = (tid >= off) ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - sum;  // exclusive prefix of this thread's range
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int p = tid * PER + e;
        if (p < kBuckets) {
            const int b = (p == 0) ? kBatchMaxN + 1 : kBatchMaxN - (p - 1);
            hist[b] = run;
            run += loc[e];
        }
    }
}

__global__ void k_batch_scatter(int32_t batch, const int32_t *__restrict__ ns, const int32_t *__restrict__ ldas,
                                int32_t *start, int32_t *__restrict__ order) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch) order[atomicAdd(start + bucket_of(ns[i], ldas[i]), 1)] = i;
}

size_t batched_workspace_ints(int32_t batch) { return (size_t)batch + kBuckets + 1; }

template <typename T>
int launch_batched(int32_t batch, const int32_t *n, void *const *A, const int32_t *lda, int32_t *info, int32_t *ws,
                   hipStream_t s, bool traced) {
    if (batch <= 0) return FLAME_OK;
    int32_t *hist = ws;                  // kBuckets
    int32_t *counter = ws + kBuckets;    // 1
    int32_t *order = ws + kBuckets + 1;  // batch
    static int grid_cache[64] = {};
    int dev = 0;
    FLAME_HIP(hipGetDevice(&dev));
    int grid = (dev < 64) ? grid_cache[dev] : 0;
    if (grid == 0) {
        int cus = 0, per = 0;
        FLAME_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        FLAME_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batched<T>, 256, 0));
        grid = std::max(1, cus * std::max(1, per));
        if (dev < 64) grid_cache[dev] = grid;
    }
    int rc = launch_zero_i32(ws, kBuckets + 1, s);
    if (rc) return rc;
    const unsigned gb = (unsigned)((batch + 255) / 256);
    hipLaunchKernelGGL(k_batch_hist, dim3(gb), dim3(256), 0, s, batch, n, lda, hist);
    FLAME_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(256), 0, s, hist);
    FLAME_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_batch_scatter, dim3(gb), dim3(256), 0, s, batch, n, lda, hist, order);
    FLAME_CHECK_LAUNCH();
    const int tr = traced ? trace_begin(FLAME_KC_OTHER, s) : -1;
    hipLaunchKernelGGL(k_batched<T>, dim3((unsigned)std::min<int64_t>(grid, batch)), dim3(256), 0, s, batch, n,
                       reinterpret_cast<T *const *>(A), lda, info, order, counter);
    FLAME_CHECK_LAUNCH();
    trace_end(tr, s, 0.0, 0.0);
    return FLAME_OK;
}

template int launch_batched<double>(int32_t, const int32_t *, void *const *, const int32_t *, int32_t *, int32_t *,
                                    hipStream_t, bool);
template int launch_batched<float>(int32_t, const int32_t *, void *const *, const int32_t *, int32_t *, int32_t *,
                                   hipStream_t, bool);

}  // namespace flame
