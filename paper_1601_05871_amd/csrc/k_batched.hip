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
//         band by band with matrix-core trailing updates (chol_lds.h); U11
//         stored as each band is done and left in LDS;
//   TRSM  from LDS: the eight diagonal tiles of U11 inverted in place, then
//         each wavefront solves 16-column strips of the panel block by block
//         on matrix cores, reading U11's tiles from LDS;
//   SYRK  per 64-column block of A22, the panel's 64 columns staged in LDS;
//         each wavefront updates 16 rows x 64 columns of A22 (FP64 or FP32
//         MFMA, K = 128) with its own 16 panel columns in registers.
// LDS holds one union of the CHOL / TRSM tiles (73.7 KB in FP64) and the
// staged SYRK columns, so two workgroups fit on a CU.  A matrix of order
// <= 128 is one CHOL step.
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

// One matrix-core step acc += M^T A over a k slot, where the lane's memory
// operand is element (k, r) of a 16 x 16 block M and the lane's accumulator
// operand is item t of another accumulator of the same layout (FP64 operands
// in swapped roles, see below).  Both precisions keep a 16-column strip of a
// panel with lane r on column r and item v on row k_slot(g, v) of each 16-row
// block (FP64: g + 4 v, the transposed FP64 accumulator; FP32: 4 g + v, the
// FP32 accumulator as it is).
__device__ __forceinline__ bd4 mma_ma(double memop, double accop, bd4 acc) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(memop, accop, acc, 0, 0, 0);
}
__device__ __forceinline__ bf4 mma_ma(float memop, float accop, bf4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(memop, accop, acc, 0, 0, 0);
}

// D_s := U_ss^{-1} for the eight diagonal 16 x 16 tiles of the band layout,
// in place (128 threads: one per column of one tile, back substitution; the
// rows below the diagonal come out 0).
template <typename T>
__device__ __forceinline__ void inv_diag_lds(T *L) {
    int tid = threadIdx.x;
    // opaque to the compiler: otherwise the unit vectors below and the tile
    // positions are formed once per kernel and kept live (spilled) across the
    // persistent loop
    asm volatile("" : "+v"(tid));
    const int sb = tid >> 4, t = tid & 15;
    T *U = L + tile_base(sb, sb);
    T d[16];
    if (tid < 16 * (kBB / 16)) {
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            T acc = (i == t) ? T(1) : T(0);
#pragma unroll
            for (int k = i + 1; k < 16; ++k) acc -= U[tile_pos<T>(i, k, 0)] * d[k];
            d[i] = acc / U[tile_pos<T>(i, i, 0)];
        }
    }
    __syncthreads();
    if (tid < 16 * (kBB / 16)) {
#pragma unroll
        for (int i = 0; i < 16; ++i) U[tile_pos<T>(i, t, 0)] = d[i];
    }
    __syncthreads();
}

// X := U11^{-T} X for the 16 columns c0 .. c0 + 15 of the 128 x m panel X
// (columns >= m skipped), one wavefront.  U11's off-diagonal tiles and the
// inverses of its diagonal tiles are read from L (band layout).  Block by
// block, right-looking: X_s = D_s^T R_s, then R_t -= U(s, t)^T X_s for t > s;
// the strip stays in registers in the layout of mma_ma, so no product needs
// its operand transposed.
template <typename T>
__device__ __forceinline__ void trsm_strip_lds(int m, const T *L, T *__restrict__ X, int64_t ldx, int c0, int lane) {
    typedef typename BAcc<T>::type acc_t;
    constexpr int NB = kBB / 16;
    const int r = lane & 15, g = lane >> 4;
    const bool cok = c0 + r < m;
    T *__restrict__ xc = X + (int64_t)min(c0 + r, m - 1) * ldx;
    acc_t acc[NB];
#pragma unroll
    for (int s = 0; s < NB; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[s][v] = xc[16 * s + k_slot<T>(g, v)];
#pragma unroll
    for (int s = 0; s < NB; ++s) {
        // this block's LDS operands first, all at once; the compiler barrier
        // keeps later blocks' reads from being hoisted here (their registers
        // would not fit)
        T dm[4], um[NB][4];
        const T *D = L + tile_base(s, s);
#pragma unroll
        for (int t = 0; t < 4; ++t) dm[t] = D[tile_pos<T>(k_slot<T>(g, t), r, 0)];
#pragma unroll
        for (int q = s + 1; q < NB; ++q) {
            const T *U = L + tile_base(s, q);
            const int key = tile_key<T>(q - s);
#pragma unroll
            for (int t = 0; t < 4; ++t) um[q][t] = U[tile_pos<T>(k_slot<T>(g, t), r, key)];
        }
        asm volatile("" ::: "memory");
        acc_t xs = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int t = 0; t < 4; ++t) xs = mma_ma(dm[t], acc[s][t], xs);
        if (cok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) xc[16 * s + k_slot<T>(g, v)] = xs[v];
        }
        T nx[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) nx[t] = -xs[t];
#pragma unroll
        for (int q = s + 1; q < NB; ++q)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[q] = mma_ma(um[q][t], nx[t], acc[q]);
    }
}

// C := C - P^T P on the upper triangle of the m x m matrix C, P is kBB x m,
// by the whole workgroup.  For each 64-column block J of C the workgroup
// stages P(:, J) in LDS (column stride ys_stride, so that the operand reads
// below hit distinct banks); then for each 64-row block I <= J, wavefront w
// takes rows I + 16 w .. I + 16 w + 15 against the 16-column blocks of J that
// reach the diagonal and lie inside C, with its own 16 columns of P read from
// global memory into registers.  k slot of lane (r, g) in step e: 4 e + g, for
// both operands.
template <typename T>
constexpr int ys_stride() {
    return sizeof(T) == 8 ? kBB + 2 : kBB + 4;  // 2 mod 32 doubles / 4 mod 64 floats
}

// 16 (or 4) bytes per lane from global memory straight into LDS: lane l's
// bytes land at lds + 16 l (4 l); lds wavefront-uniform.
__device__ __forceinline__ void copy16_to_lds(const char *gsrc, char *lds) {
    __builtin_amdgcn_global_load_lds(gsrc, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}
__device__ __forceinline__ void copy4_to_lds(const char *gsrc, char *lds) {
    __builtin_amdgcn_global_load_lds(gsrc, (__attribute__((address_space(3))) void *)lds, 4, 0, 0);
}

// One wavefront: rows R0 .. R0 + 15 of C against its column blocks
// b0 .. b0 + NA - 1 of the staged block at column J0 (NA fixed, so that the
// products carry no per-block predicate).  The wavefront's panel columns
// R0 + r are negated into registers in two halves of k: xa (k < 64) arrives
// loaded by the previous item; xb (k >= 64) is loaded at the start and used
// in the second half, and xa is reloaded meanwhile with the next item's
// columns Rn + r.  Element e of a half is k = 4 e + g (+ 64).
template <typename T>
__device__ __forceinline__ void syrk_load_half(int m, const T *__restrict__ P, int64_t ldp, int R0, int k0, int lane,
                                               T (&x)[kBB / 8]) {
    const T *xp = P + (int64_t)min(R0 + (lane & 15), m - 1) * ldp + k0 + (lane >> 4);
#pragma unroll
    for (int e = 0; e < kBB / 8; ++e) x[e] = -xp[4 * e];
}

template <typename T, int NA>
__device__ __forceinline__ void syrk_rows(int m, const T *__restrict__ P, int64_t ldp, T (&xa)[kBB / 8], int Rn,
                                          T *__restrict__ C, int64_t ldc, const T *Y, int R0, int J0, int b0,
                                          int lane) {
    typedef typename BAcc<T>::type acc_t;
    constexpr int YS = ys_stride<T>();
    constexpr int H = kBB / 8;  // elements per half
    const int r = lane & 15, g = lane >> 4;
    T cv[NA][4];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = R0 + acc_row<T>(r, g, v), j = J0 + 16 * (b0 + a) + acc_col<T>(r, g, v);
            cv[a][v] = C[(int64_t)min(i, m - 1) + (int64_t)min(j, m - 1) * ldc];
        }
    T xb[H];
    syrk_load_half<T>(m, P, ldp, R0, kBB / 2, lane, xb);
    acc_t acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = acc_t{T(0), T(0), T(0), T(0)};
    const T *yb = Y + (16 * b0 + r) * YS + g;
    auto half = [&](const T(&x)[H], int kh) {
#pragma unroll
        for (int e0 = 0; e0 < H; e0 += 4) {
            // 16 k at a time: the chunk's LDS reads, then its products
            T y[4][NA];
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int a = 0; a < NA; ++a) y[e][a] = yb[16 * a * YS + kh + 4 * (e0 + e)];
            asm volatile("" ::: "memory");
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int a = 0; a < NA; ++a) acc[a] = mma(x[e0 + e], y[e][a], acc[a]);
        }
    };
    half(xa, 0);
    syrk_load_half<T>(m, P, ldp, Rn, 0, lane, xa);
    half(xb, kBB / 2);
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = R0 + acc_row<T>(r, g, v), j = J0 + 16 * (b0 + a) + acc_col<T>(r, g, v);
            if (i <= j && j < m) C[(int64_t)i + (int64_t)j * ldc] = cv[a][v] + acc[a][v];
        }
}

// A wavefront's items are (J, I) with I <= J in loop order; it is idle only
// on a diagonal item whose rows start at or beyond m, which can happen only in
// the last column block.  The panel columns of the next item are loaded while
// the current one computes.
template <typename T>
__device__ __forceinline__ void syrk_lds(int m, const T *__restrict__ P, int64_t ldp, T *__restrict__ C, int64_t ldc,
                                         T *Y, int wave, int lane) {
    constexpr int YS = ys_stride<T>();
    const int tid = threadIdx.x;
    const bool wide16 = ((reinterpret_cast<uintptr_t>(P) & 15) == 0) && ((ldp & 1) == 0);
    T xa[kBB / 8];
    syrk_load_half<T>(m, P, ldp, 16 * wave, 0, lane, xa);  // item (0, 0)
    for (int J0 = 0; J0 < m; J0 += 64) {
        if constexpr (sizeof(T) == 8) {
            // copies from global memory straight into LDS (no registers: the
            // wavefront holds the next item's panel columns meanwhile); wavefront
            // w copies columns 16 w .. 16 w + 15, 16 bytes per lane (one column
            // per copy) when every column starts 16-byte aligned, else 4
#pragma unroll 4
            for (int cc = 0; cc < 16; ++cc) {
                const int c = 16 * wave + cc;
                const char *src = reinterpret_cast<const char *>(P + (int64_t)min(J0 + c, m - 1) * ldp);
                char *dst = reinterpret_cast<char *>(Y + c * YS);
                if (wide16) {
                    copy16_to_lds(src + 16 * lane, dst);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) copy4_to_lds(src + 256 * q + 4 * lane, dst + 256 * q);
                }
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        } else {
            // thread (c, q) copies k = 32 q .. 32 q + 31 of column J0 + c
            const int c = tid >> 2, q = tid & 3;
            const T *src = P + (int64_t)min(J0 + c, m - 1) * ldp + 32 * q;
            T v[32];
#pragma unroll
            for (int i = 0; i < 32; ++i) v[i] = src[i];
            T *dst = Y + c * YS + 32 * q;
#pragma unroll
            for (int i = 0; i < 32; ++i) dst[i] = v[i];
        }
        __syncthreads();
        const int nb = min(4, (m - J0 + 15) >> 4);  // column blocks of J inside C
        for (int I0 = 0; I0 <= J0; I0 += 64) {
            const int R0 = I0 + 16 * wave;
            const int b0 = (I0 == J0) ? wave : 0;  // blocks left of b0: below the diagonal
            if (R0 < m && b0 < nb) {
                // next item: (J, I + 64), or (J + 64, 0) after the diagonal
                const int Rn = (I0 + 64 <= J0 ? I0 + 64 : 0) + 16 * wave;
                switch (nb - b0) {
                    case 1: syrk_rows<T, 1>(m, P, ldp, xa, Rn, C, ldc, Y, R0, J0, b0, lane); break;
                    case 2: syrk_rows<T, 2>(m, P, ldp, xa, Rn, C, ldc, Y, R0, J0, b0, lane); break;
                    case 3: syrk_rows<T, 3>(m, P, ldp, xa, Rn, C, ldc, Y, R0, J0, b0, lane); break;
                    default: syrk_rows<T, 4>(m, P, ldp, xa, Rn, C, ldc, Y, R0, J0, b0, lane); break;
                }
            }
        }
        __syncthreads();  // Y is restaged
    }
}

// Workgroup-shared scratch of factor_one: the diagonal block's tiles during
// CHOL and TRSM (all of U11 after CHOL, the diagonal tiles then replaced by
// their inverses), the staged SYRK operands afterwards.
template <typename T>
struct BatchLds {
    union {
        T L[band_lds_size<kBB>()];      // diagonal block, upper 16 x 16 tiles
        T Y[64 * ys_stride<T>()];       // SYRK: 64 staged columns of the panel
    };
    int s_bad;
    int s_item;
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
        // CHOL: the block's tiles in LDS, U11 stored to A11 band by band and
        // kept in L
        band_load<T, kBB>(bk, A11, lda, sh.L);
        __syncthreads();
        const int bad = chol_lds_core2<T, kBB, false, true>(bk, sh.L, &sh.s_bad, A11, lda);
        if (bad != 0) return k0 + bad;
        __syncthreads();  // U11 in L and in memory
        if (m == 0) break;
        // TRSM: A12 := U11^{-T} A12 (bk == kBB here)
        T *A12 = A + k0 + (int64_t)(k0 + kBB) * lda;
        inv_diag_lds<T>(sh.L);
        for (int c0 = 16 * wave; c0 < m; c0 += 64) trsm_strip_lds<T>(m, sh.L, A12, lda, c0, lane);
        __syncthreads();  // A12 in memory, L free
        // SYRK: A22 -= A12^T A12 (upper)
        syrk_lds<T>(m, A12, lda, A + (k0 + kBB) + (int64_t)(k0 + kBB) * lda, lda, sh.Y, wave, lane);
    }
    return 0;
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_batched(int32_t batch, const int32_t *__restrict__ ns, T *const *As,
                                                    const int32_t *__restrict__ ldas, int32_t *__restrict__ info,
                                                    const int32_t *__restrict__ order, int32_t *counter) {
    // one LDS object: with several, the compiler tags LDS accesses with alias
    // scopes and makes LDS reads wait for every copy into LDS still in flight
    __shared__ BatchLds<T> sh;
    const int tid = threadIdx.x;
    // Every value that steers the loop is made wave-uniform (readfirstlane):
    // the branches around the barriers are then scalar, and every lane of a
    // wavefront takes the same path through them.
    for (;;) {
        if (tid == 0) sh.s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(sh.s_item);
        __syncthreads();
        if (t >= batch) break;  // every wave of the workgroup leaves together
        const int i = __builtin_amdgcn_readfirstlane(order[t]);
        const int n = __builtin_amdgcn_readfirstlane(ns[i]);
        const int lda = __builtin_amdgcn_readfirstlane(ldas[i]);
        int res = -1;  // order out of range or lda < n: not touched
        if (n >= 0 && n <= kBatchMaxN && lda >= max(1, n)) {
            // the matrix pointer read as a global-memory pointer: a pointer of
            // unknown address space would make every access a flat one, and
            // flat accesses count on the LDS wait counter too (each LDS wait
            // would also wait for the global loads and stores in flight)
            typedef __attribute__((address_space(1))) T gT;
            gT *gA = static_cast<gT *const *>(static_cast<const void *>(As))[i];
            res = factor_one<T>(n, (T *)gA, (int64_t)lda, sh);
        }
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
