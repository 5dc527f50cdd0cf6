// Cholesky-by-blocks as a task DAG run by one persistent kernel (Fig.
// "sparse-chol" of the paper with dense 128 x 128 blocks; the dependence rule
// of the by-blocks section: a block operation may run as soon as the blocks it
// reads are final and the block it writes has received every earlier update).
//
// The matrix is a grid of nbt x nbt blocks of 128 (the last row / column of
// blocks ragged); a pattern names the blocks of the upper triangle that exist
// (all of them for a dense matrix).  For iteration k the paper's generators
// emit
//   CHOL(k):       A_kk := Chol(A_kk)
//   TRSM(k, j):    A_kj := triu(A_kk)^{-T} A_kj          for existing A_kj, j > k
//   UPD(k, i, j):  A_ij := A_ij - A_ki^T A_kj            for existing A_ki, A_kj
//                  and existing A_ij, k < i <= j (HERK when i = j, GEMM else);
// with a pattern that is not closed under this fill the update of a missing
// block is dropped, which is the block form of an incomplete factorization.
//
// Futures (the paper's per-block task dependences) are per-block counters in
// device memory: fin[i][j] = 1 once block (i, j) is final (after its CHOL or
// TRSM), upd[i][j] = updates applied to it so far.  A task records how many
// updates its output block must have received before it runs ("need"), so
// the updates of one block are applied in iteration order (deterministic
// results).  Tasks are listed in a static order in which every task comes
// after all the tasks it depends on, with one iteration of lookahead:
//   block of the list for iteration r (r >= 1):
//     CHOL(r), TRSM(r, *), UPD(r-1, r+1, *), UPD(r, r+1, *), UPD(r-1, >= r+2, *)
// so the diagonal and panel work of iteration r (and the updates of the next
// block row) come before the bulk of iteration r-1's updates.  Workgroups
// claim tasks in list order from an atomic counter and wait (bounded) for the
// task's futures; since every dependence points to an earlier task, the
// earliest unfinished task always belongs to a running workgroup whose
// dependences are complete, so the launch always progresses, whatever the
// number of resident workgroups.  A wait that gives up, or a breakdown, sets
// an abort flag that every workgroup polls, so all of them exit.
#include <algorithm>
#include <vector>

#include "chol_lds.h"
#include "dev_sync.h"
#include "flame_internal.h"
#include "trsm_rl.h"

namespace flame {

namespace {

constexpr int kT = 128;                        // block order
constexpr long long kDagSpin = 1LL << 26;      // s_sleep rounds before a wait gives up
constexpr int kLdsChol = band_lds_size<kT>();  // doubles of the CHOL block in LDS
constexpr int kLdsTrsm = 8 * 16 * 17 + 4 * 16 * 17;
constexpr int kStages = 4;                      // update: chunks of 16 k staged at once (3 in flight)
constexpr int kLdsDoubles = kLdsChol > kLdsTrsm ? kLdsChol : kLdsTrsm;

struct DagP {
    int64_t n;
    double *A;
    int64_t lda;
    int nbt;              // blocks per side
    const int4 *tasks;    // (type | k << 2, i, j, need)
    int64_t ntasks;
    int32_t *claim;       // next task to claim
    int32_t *abort_flag;  // 1: a wait gave up, 2: breakdown
    int32_t *fin;         // nbt x nbt
    int32_t *upd;         // nbt x nbt
    int32_t *info;
    int stage;            // 1: operand columns 16-byte aligned (A and lda): LDS-staged updates
    // block-sparse form (the incomplete factorization): A is a pool of
    // 128 x 128 tiles (leading dimension 128), block (i, j) at A + boff[i nbt + j]
    // (-1: missing), of order bstart[i + 1] - bstart[i] x bstart[j + 1] - bstart[j];
    // masks: per tile (in pool order) 128 columns x 128 bits, bit r of column c
    // set when (r, c) is in the pattern of the factor
    const int64_t *boff;
    const int32_t *bstart;
    const uint64_t *masks;
    const uint64_t *rowocc;  // per tile: 2 words, bit r set when row r has an entry of the pattern
    // breakdowns of the block-sparse form: max of INT32_MAX - column (so the
    // lowest column wins and 0 means none); independent blocks may break down
    // in any order, so a breakdown does not stop the launch
    int32_t *bad_enc;
};

// Waits (bounded) until *p >= want; false on abort or give-up (which sets
// the abort flag to 1).
__device__ __forceinline__ bool wait_at_least(const int32_t *p, int want, int32_t *abort_flag) {
    return poll_at_least(p, want, abort_flag, 1, kDagSpin);
}

// An update's result goes out with device-scope stores (store_dev), which
// write through to the device's coherence point: once every wavefront has
// waited for its stores and the workgroup has passed a barrier, the block is
// visible to every CU and the future is set without a release.  (A release
// at device scope writes back the XCD's whole L2; with a workgroup per CU
// publishing an update every few tens of microseconds those write-backs
// contend: a 128-block update took 59 us against 28 us this way.)

// C := C - X^T Y for one block (C M x N of a 128-grid, X and Y 128 x M / N,
// columns contiguous in k), upper part only when `diag`.  Wavefront w owns the
// 64 x 64 quarter (w / 2, w % 2) as 4 x 4 FP64 MFMA blocks (lane (r, g) of
// block (a, b) ends with row 16 a + r, columns 16 b + g + 4 v of the quarter);
// the accumulator starts from C and X enters negated.  Operand fragments
// straight from memory: the form for columns that are not 16-byte aligned.
__device__ __forceinline__ void block_update(const double *__restrict__ X, const double *__restrict__ Y, double *C,
                                             int64_t ld, int M, int N, bool diag) {
    typedef double d4_t __attribute__((ext_vector_type(4)));
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 15, g = lane >> 4;
    const int row0 = (wave >> 1) * 64, col0 = (wave & 1) * 64;
    if (diag && row0 > col0) return;  // this quarter lies below the diagonal (wave-uniform)
    if (row0 >= M || col0 >= N) return;
    d4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = min(row0 + 16 * a + r, M - 1), col = min(col0 + 16 * b + g + 4 * v, N - 1);
                acc[a][b][v] = C[row + (int64_t)col * ld];
            }
    // lane (r, g) reads k = kc + 4 g .. kc + 4 g + 3 of its X and Y columns;
    // MFMA e of the chunk takes element e of every lane, so both operands put
    // the same k in each (g, e) slot
    const double *xc[4], *yc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) xc[a] = X + (int64_t)min(row0 + 16 * a + r, M - 1) * ld + 4 * g;
#pragma unroll
    for (int b = 0; b < 4; ++b) yc[b] = Y + (int64_t)min(col0 + 16 * b + r, N - 1) * ld + 4 * g;
#pragma unroll 1
    for (int kc = 0; kc < kT; kc += 16) {
        double xa[4][4], yb[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) xa[a][e] = xc[a][kc + e];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) yb[b][e] = yc[b][kc + e];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[b][e], -xa[a][e], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + 16 * a + r, col = col0 + 16 * b + g + 4 * v;
                if (row < M && col < N && (!diag || row <= col)) store_dev(&C[row + (int64_t)col * ld], acc[a][b][v]);
            }
}

// 16 bytes per lane from global memory straight into LDS (lane l's bytes land
// at lds + 16 l; lds wavefront-uniform).
__device__ __forceinline__ void copy16_to_lds(const char *gsrc, char *lds) {
    __builtin_amdgcn_global_load_lds(gsrc, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}
// byte offset of 16-byte unit `unit` (k = 2 unit, 2 unit + 1 of the chunk) of
// operand column `col` in a staged chunk: units XOR-swizzled by (col mod 8) so
// that the 16 lanes reading one unit of 16 consecutive columns hit different
// banks
__device__ __forceinline__ int slab_off(int col, int unit) { return col * 128 + ((unit ^ (col & 7)) << 4); }

// LDS of the kernel, one object: a kernel with several LDS variables has
// their accesses tagged with alias scopes, and the compiler then makes every
// LDS read wait for all outstanding copies into LDS (which would serialize
// the update's copy pipeline below); the waits those copies need are explicit.
struct DagShared {
    union {
        double band[kLdsDoubles];                // CHOL block (band layout) or TRSM scratch
        char stage[kStages][2][kT * 128];        // update: [chunk mod kStages][X or Y][column x 128 bytes]
        double tile[kT * kT];                    // masked TRSM: the diagonal block's factor
    } u;
    double row[2][kT];                           // masked CHOL / TRSM: the row of the step (double-buffered)
    double piv[2];                               // masked CHOL: the pivot of the step
    double diag[kT];                             // masked TRSM: the diagonal of the block's factor
    int s_task, s_ok, s_bad;
};

// The same update with the operands staged through LDS, 16 k per chunk: the
// workgroup copies the chunk's 128 columns of X and of Y (128 bytes each)
// from global memory straight into LDS, three chunks ahead of the MFMAs
// (kStages buffers, one barrier per chunk), so every operand element is read
// once per workgroup with 16-byte loads and the copy latency is hidden behind
// the MFMAs of the chunks before.  Needs 16-byte aligned columns.  Called by
// the whole workgroup (barriers inside).
__device__ __forceinline__ void block_update_lds(const double *__restrict__ X, const double *__restrict__ Y,
                                                 double *C, int64_t ld, int M, int N, bool diag,
                                                 char (*stage)[2][kT * 128]) {
    typedef double d4_t __attribute__((ext_vector_type(4)));
    typedef double d2_t __attribute__((ext_vector_type(2)));
    typedef unsigned int u4_t __attribute__((ext_vector_type(4)));
    constexpr int kChunks = kT / 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 15, g = lane >> 4;
    const int row0 = (wave >> 1) * 64, col0 = (wave & 1) * 64;
    const bool active = row0 < M && col0 < N && !(diag && row0 > col0);  // wavefront-uniform
    // copies: wavefront w takes columns 8 w + 32 j + lane / 8 (j < 4) of each
    // operand; lane l's 16 bytes land in slot l % 8 of its column, so it
    // fetches the unit the swizzle puts there (8 copy instructions a chunk)
    const int unit = (lane & 7) ^ ((lane >> 3) & 7);
    const char *xg[4], *yg[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = 8 * wave + 32 * j + (lane >> 3);
        xg[j] = reinterpret_cast<const char *>(X + (int64_t)min(col, M - 1) * ld) + 16 * unit;
        yg[j] = reinterpret_cast<const char *>(Y + (int64_t)min(col, N - 1) * ld) + 16 * unit;
    }
    auto copy = [&](int c) {
        const int sb = c & (kStages - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            copy16_to_lds(xg[j] + 128 * c, &stage[sb][0][0] + (8 * wave + 32 * j) * 128);
            copy16_to_lds(yg[j] + 128 * c, &stage[sb][1][0] + (8 * wave + 32 * j) * 128);
        }
    };
    d4_t acc[4][4];
    if (active) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = min(row0 + 16 * a + r, M - 1), col = min(col0 + 16 * b + g + 4 * v, N - 1);
                    acc[a][b][v] = C[row + (int64_t)col * ld];
                }
    }
    // the C loads are issued before the copies (the vmcnt counts below
    // count copies only after them)
    asm volatile("" ::: "memory");
#pragma unroll
    for (int c = 0; c < kStages - 1; ++c) copy(c);
#pragma unroll 1
    for (int c = 0; c < kChunks; ++c) {
        // chunk c landed: at most the copies of the chunks after it (8
        // instructions each, up to two) still in flight
        if (c + 2 < kChunks)
            asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
        else if (c + 1 < kChunks)
            asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
        else
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        // every wavefront's part of chunk c is in LDS, and every wavefront is
        // done with chunk c - 1, whose buffer the copy of chunk c + 3 reuses
        __syncthreads();
        if (c + kStages - 1 < kChunks) copy(c + kStages - 1);
        if (active) {
            const char *xs = &stage[c & (kStages - 1)][0][0], *ys = &stage[c & (kStages - 1)][1][0];
            // lane (r, g) takes units 2 g and 2 g + 1 (k = 4 g .. 4 g + 3) of
            // its columns in turn; MFMA e of a unit takes element e of every
            // lane, so both operands put the same k in each (g, e) slot
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                d2_t fa[4], fb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    fa[a] = __builtin_bit_cast(d2_t, *reinterpret_cast<const u4_t *>(xs + slab_off(row0 + 16 * a + r, 2 * g + h)) ^
                                                         u4_t{0u, 0x80000000u, 0u, 0x80000000u});  // -X
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    fb[b] = __builtin_bit_cast(d2_t, *reinterpret_cast<const u4_t *>(ys + slab_off(col0 + 16 * b + r, 2 * g + h)));
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[b][0], fa[a][0], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[b][1], fa[a][1], acc[a][b], 0, 0, 0);
                    }
            }
        }
    }
    __syncthreads();  // the staging buffers are free again (the next task may overwrite the LDS)
    if (active) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = row0 + 16 * a + r, col = col0 + 16 * b + g + 4 * v;
                    if (row < M && col < N && (!diag || row <= col)) store_dev(&C[row + (int64_t)col * ld], acc[a][b][v]);
                }
    }
}

// The task bodies, inlined into the persistent loop: called by the whole
// workgroup; every LDS access goes to the kernel's own LDS array.
__device__ __forceinline__ void task_chol(double *A, int64_t lda, int b, double *lds, int *s_bad, int k,
                                          int32_t *info, int32_t *abort_flag) {
    band_load<double, kT>(b, A, lda, lds);
    __syncthreads();
    const int bad = chol_lds_core2<double, kT>(b, lds, s_bad, A, lda);
    if (bad != 0 && threadIdx.x == 0) {
        atomicCAS(info, 0, (int32_t)((int64_t)k * kT + bad));
        __hip_atomic_store(abort_flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ void task_trsm(const double *U, double *X, int64_t lda, int m, double *lds) {
    auto Ds = reinterpret_cast<double (*)[16][17]>(lds);
    auto Rt = reinterpret_cast<double (*)[17]>(lds + 8 * 16 * 17);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    trsm_inverses<double, 8>(kT, U, lda, Ds);
    __syncthreads();
    for (int c0 = 0; c0 < m; c0 += 64) trsm_cols<double, 8>(kT, m, U, lda, X, lda, c0 + 16 * wave, Ds, Rt + 16 * wave);
}

// ---- the incomplete factorization's block operations ------------------------
// Level(k) incomplete Cholesky drops every update whose target lies outside
// the pattern.  A dropped entry is never used as a multiplier, so it suffices
// to drop it when its row of U becomes final: the CHOL and TRSM of a block
// zero each row's entries outside the pattern as soon as the row is
// computed, before it updates the rows below; the HERK / GEMM updates write
// the whole block (their entries outside the pattern are dropped when that
// block's own rows become final).  The element form is kept: thread (c, h)
// holds column c, rows 64 h .. 64 h + 63 of the block in registers; row j is
// finalized by the 128 threads of half j / 64 and broadcast through LDS.
// Register indices are compile-time: row j of a thread's 64 is selected by
// comparison, not by indexing.

// Element 16 q + t of a thread's 64 values (t compile-time, q wave-uniform),
// read and written with constant indices only (the four candidates pass an
// empty asm first, so the choice is a select of register values, never a load
// through a chosen address, which would put the array in scratch memory).
__device__ __forceinline__ double pick16(const double (&v)[64], int q, int t) {
    double v0 = v[t], v1 = v[16 + t], v2 = v[32 + t], v3 = v[48 + t];
    asm volatile("" : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3));
    return q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3;
}
__device__ __forceinline__ void put16(double (&v)[64], int q, int t, double x) {
    v[t] = q == 0 ? x : v[t];
    v[16 + t] = q == 1 ? x : v[16 + t];
    v[32 + t] = q == 2 ? x : v[32 + t];
    v[48 + t] = q == 3 ? x : v[48 + t];
}

// Incomplete CHOL of the b x b diagonal tile (leading dimension 128, the
// whole 128 x 128 tile readable, zero below the diagonal and outside b);
// returns 0 or the 1-based position of the first pivot that is not > 0
// (uniform).  Writes the upper triangle.  Step j: the owners of row j
// publish the pivot and the row unscaled (v_c for c > j in the pattern, 0
// elsewhere); after one barrier every thread forms w = v_c / d for its column
// and subtracts v_r w from its rows r (the zeros leave finished rows alone),
// and the owners store u_jc = v_c / sqrt(d).  Row and pivot are
// double-buffered, so one barrier per step suffices.
__device__ __forceinline__ int task_chol_masked(double *A, int b, const uint64_t *mask, DagShared &sh) {
    const int tid = threadIdx.x, c = tid & (kT - 1);
    const int h = __builtin_amdgcn_readfirstlane(tid >> 7);
    const uint64_t m = mask[2 * c + h];  // bit i: row 64 h + i of column c in the pattern
    double a[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) a[i] = A[64 * h + i + (int64_t)c * kT];
    int bad = 0;
    for (int jq = 0; jq < kT / 16 && 16 * jq < b && bad == 0; ++jq) {
        const int jb = jq >> 2, q = jq & 3;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int j = 16 * jq + t;
            if (j < b && bad == 0) {
                const int buf = t & 1;
                if (h == jb) {
                    const double v = pick16(a, q, t);
                    if (c == j) sh.piv[buf] = v;
                    sh.row[buf][c] = (c > j && ((m >> (16 * q + t)) & 1)) ? v : 0.0;
                }
                __syncthreads();
                const double d = sh.piv[buf];
                if (__builtin_amdgcn_readfirstlane(d > 0.0 ? 1 : 0) == 0) {
                    bad = j + 1;
                } else {
                    const double p = sqrt(d);
                    const double vc = sh.row[buf][c];
                    const double w = vc / d;
                    if (h == jb) {
                        const double u = (c == j) ? p : vc / p;
                        put16(a, q, t, u);
                    }
#pragma unroll
                    for (int i = 0; i < 64; ++i) a[i] = __builtin_fma(-sh.row[buf][64 * h + i], w, a[i]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        const int r = 64 * h + i;
        if (r <= c && c < b) A[r + (int64_t)c * kT] = a[i];
    }
    return bad;
}

// Incomplete TRSM X := triu(U)^{-T} X for the bk x m tile X of the block row
// whose diagonal factor is U (tiles of leading dimension 128, readable whole,
// U zero below its diagonal and outside bk): forward substitution row by
// row, each row dropped outside the pattern as soon as it is computed.  U is
// copied to LDS with its diagonal moved aside, so the update of every row by
// the row just computed is unconditional (U's zeros leave the rows above it
// alone).
__device__ __forceinline__ void task_trsm_masked(const double *U, double *X, int bk, int m, const uint64_t *mask,
                                                 const uint64_t *occ, DagShared &sh) {
    (void)m;  // columns >= m are outside the pattern (mask bits 0)
    // rows of X without an entry of the pattern stay zero and update nothing:
    // their steps are skipped (the decision is uniform)
    const uint64_t occ0 = __builtin_amdgcn_readfirstlane((unsigned)(occ[0] & 0xffffffffu)) |
                          ((uint64_t)__builtin_amdgcn_readfirstlane((unsigned)(occ[0] >> 32)) << 32);
    const uint64_t occ1 = __builtin_amdgcn_readfirstlane((unsigned)(occ[1] & 0xffffffffu)) |
                          ((uint64_t)__builtin_amdgcn_readfirstlane((unsigned)(occ[1] >> 32)) << 32);
    const int tid = threadIdx.x, c = tid & (kT - 1);
    const int h = __builtin_amdgcn_readfirstlane(tid >> 7);
    typedef double d2_t __attribute__((ext_vector_type(2)));
    const d2_t *U2 = reinterpret_cast<const d2_t *>(U);
    d2_t *T2 = reinterpret_cast<d2_t *>(sh.u.tile);
#pragma unroll 4
    for (int e = tid; e < kT * kT / 2; e += 256) T2[e] = U2[e];
    const uint64_t mk = mask[2 * c + h];
    double x[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) x[i] = X[64 * h + i + (int64_t)c * kT];
    __syncthreads();
    double *Ut = sh.u.tile;
    if (tid < kT) {
        sh.diag[tid] = Ut[tid + tid * kT];
        Ut[tid + tid * kT] = 0.0;
    }
    __syncthreads();
    for (int rq = 0; rq < kT / 16 && 16 * rq < bk; ++rq) {
        const int rb = rq >> 2, q = rq & 3;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int r = 16 * rq + t;
            if (r < bk && (((rb ? occ1 : occ0) >> (16 * q + t)) & 1)) {
                const int buf = t & 1;
                if (h == rb) {
                    const double v = pick16(x, q, t);
                    const double u = ((mk >> (16 * q + t)) & 1) ? v / sh.diag[r] : 0.0;
                    put16(x, q, t, u);
                    sh.row[buf][c] = u;
                }
                __syncthreads();
                const double xr = sh.row[buf][c];
#pragma unroll
                for (int i = 0; i < 64; ++i) x[i] = __builtin_fma(-Ut[r + (64 * h + i) * kT], xr, x[i]);
            }
        }
    }
    // stored through the mask: a skipped (empty) row still holds what the rows
    // above it subtracted from it, and must leave as zeros
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        const int rr = 64 * h + i;
        if (rr < bk) X[rr + (int64_t)c * kT] = ((mk >> i) & 1) ? x[i] : 0.0;
    }
}

// Loop control is wave-uniform (readfirstlane) and thread 0 has ONE region
// per iteration, publish of the finished task followed by the next claim,
// with a barrier after it: with a claim region at the top of the loop and a
// publish region at its end, both on thread 0, the compiler may thread the
// one into the other across the back edge; the loop then has two entries and
// its structurized form lets the other lanes of wavefront 0 run ahead of
// thread 0 to the next barrier with the old task index.
template <bool SPARSE>
__global__ __launch_bounds__(256, 1) void k_by_blocks(DagP p) {
    __shared__ __attribute__((aligned(16))) DagShared sh;
    double *lds = sh.u.band;
    int &s_task = sh.s_task, &s_ok = sh.s_ok, &s_bad = sh.s_bad;
    const int tid = threadIdx.x;
    const int nbt = p.nbt;
    const int64_t lda = SPARSE ? kT : p.lda;
    if (tid == 0) s_task = atomicAdd(p.claim, 1);
    __syncthreads();
    for (;;) {
        const int t = __builtin_amdgcn_readfirstlane(s_task);
        if (t >= p.ntasks) break;
        const int4 d = p.tasks[t];
        const int type = __builtin_amdgcn_readfirstlane(d.x) & 3, k = __builtin_amdgcn_readfirstlane(d.x) >> 2;
        const int i = __builtin_amdgcn_readfirstlane(d.y), j = __builtin_amdgcn_readfirstlane(d.z);
        const int need = __builtin_amdgcn_readfirstlane(d.w);
        // wait for the futures of the task
        if (tid == 0) {
            bool ok = true;
            if (type == 0) {
                ok = wait_at_least(p.upd + (int64_t)k * nbt + k, need, p.abort_flag);
            } else if (type == 1) {
                ok = wait_at_least(p.fin + (int64_t)k * nbt + k, 1, p.abort_flag) &&
                     wait_at_least(p.upd + (int64_t)k * nbt + j, need, p.abort_flag);
            } else {
                ok = wait_at_least(p.fin + (int64_t)k * nbt + i, 1, p.abort_flag) &&
                     wait_at_least(p.fin + (int64_t)k * nbt + j, 1, p.abort_flag) &&
                     wait_at_least(p.upd + (int64_t)i * nbt + j, need, p.abort_flag);
            }
            s_ok = ok ? 1 : 0;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_ok) == 0) break;
        // every wavefront takes an acquire of its own before reading the blocks
        acquire_dev();
        auto blk = [&](int bi, int bj) {
            if constexpr (SPARSE)
                return p.A + p.boff[(int64_t)bi * nbt + bj];
            else
                return p.A + (int64_t)bi * kT + (int64_t)bj * kT * lda;
        };
        auto width = [&](int b) {
            if constexpr (SPARSE)
                return (int)(p.bstart[b + 1] - p.bstart[b]);
            else
                return (int)min((int64_t)kT, p.n - (int64_t)b * kT);
        };
        auto mask = [&](int bi, int bj) { return p.masks + (p.boff[(int64_t)bi * nbt + bj] / (kT * kT)) * (2 * kT); };
        if (SPARSE && type == 0) {
            const int bad = task_chol_masked(blk(k, k), width(k), mask(k, k), sh);
            if (bad != 0 && tid == 0) atomicMax(p.bad_enc, (int32_t)(0x7fffffff - (p.bstart[k] + bad)));
        } else if (SPARSE && type == 1) {
            task_trsm_masked(blk(k, k), blk(k, j), width(k), width(j), mask(k, j),
                             p.rowocc + (p.boff[(int64_t)k * nbt + j] / (kT * kT)) * 2, sh);
        } else if (type == 0)
            task_chol(blk(k, k), lda, width(k), lds, &s_bad, k, p.info, p.abort_flag);
        else if (type == 1)
            task_trsm(blk(k, k), blk(k, j), lda, width(j), lds);
        else if (SPARSE || p.stage)
            block_update_lds(blk(k, i), blk(k, j), blk(i, j), lda, width(i), width(j), i == j, sh.u.stage);
        else
            block_update(blk(k, i), blk(k, j), blk(i, j), lda, width(i), width(j), i == j);
        // publish: the block visible at device scope, then the future; then
        // the next claim (no claim once the launch is aborting).  An update
        // wrote through (store_dev): its stores complete, the future follows;
        // CHOL and TRSM wrote through the L2 and release it.
        if (type == 2)
            wait_stores();
        else
            __threadfence();
        __syncthreads();
        if (tid == 0) {
            if (type == 2)
                store_dev(p.upd + (int64_t)i * nbt + j, need + 1);
            else
                __hip_atomic_store(p.fin + (int64_t)k * nbt + (type == 0 ? k : j), 1, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            s_task = (load_dev(p.abort_flag) != 0) ? (int)p.ntasks : atomicAdd(p.claim, 1);
        }
        __syncthreads();
    }
}

__global__ void k_dag_abort_info(const int32_t *abort_flag, int32_t *info) {
    // a wait that gave up (not a breakdown): info = -1
    if (threadIdx.x == 0 && *abort_flag == 1 && *info == 0) *info = -1;
}

}  // namespace

// Task list of the by-blocks factorization (see the top of this file).
// pattern: nbt x nbt, row-major, nonzero = block (i, j) exists (only i <= j
// read; nullptr = dense).  Returns the tasks as (type | k << 2, i, j, need).
std::vector<int4> by_blocks_tasks(int nbt, const uint8_t *pattern) {
    auto ex = [&](int i, int j) -> bool { return i == j || pattern == nullptr || pattern[(int64_t)i * nbt + j] != 0; };
    // need(k, i, j): updates of block (i, j) from iterations before k (k for a
    // dense matrix)
    auto need_at = [&](int k, int i, int j) {
        if (pattern == nullptr) return k;
        int c = 0;
        for (int q = 0; q < k; ++q)
            if (ex(q, i) && ex(q, j)) ++c;
        return c;
    };
    std::vector<int4> out;
    auto chol = [&](int r) { out.push_back(int4{0 | (r << 2), r, r, need_at(r, r, r)}); };
    auto trsm = [&](int r) {
        for (int j = r + 1; j < nbt; ++j)
            if (ex(r, j)) out.push_back(int4{1 | (r << 2), r, j, need_at(r, r, j)});
    };
    auto upd_row = [&](int k, int i) {  // UPD(k, i, j >= i)
        if (k < 0 || i >= nbt || !ex(k, i)) return;
        for (int j = i; j < nbt; ++j)
            if (ex(k, j) && ex(i, j)) out.push_back(int4{2 | (k << 2), i, j, need_at(k, i, j)});
    };
    for (int r = 0; r < nbt; ++r) {
        chol(r);
        trsm(r);
        upd_row(r - 1, r + 1);
        upd_row(r, r + 1);
        for (int i = r + 2; i < nbt; ++i) upd_row(r - 1, i);
    }
    return out;
}

int launch_by_blocks(int64_t n, double *A, int64_t lda, const int4 *tasks, int64_t ntasks, int nbt, int32_t *ints,
                     int32_t *info, hipStream_t s) {
    // ints: claim, abort, fin[nbt^2], upd[nbt^2] (cleared here)
    const int64_t nints = 2 + 2 * (int64_t)nbt * nbt;
    int rc = launch_zero_i32(ints, nints, s);
    if (rc) return rc;
    rc = launch_zero_i32(info, 1, s);
    if (rc) return rc;
    if (n == 0 || ntasks == 0) return FLAME_OK;
    static int grid_cache[64] = {};
    int dev = 0;
    FLAME_HIP(hipGetDevice(&dev));
    int grid = (dev < 64) ? grid_cache[dev] : 0;
    if (grid == 0) {
        int cus = 0, per = 0;
        FLAME_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        FLAME_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_by_blocks<false>, 256, 0));
        grid = std::max(1, cus * std::max(1, per));
        if (dev < 64) grid_cache[dev] = grid;
    }
    DagP p;
    p.n = n;
    p.A = A;
    p.lda = lda;
    p.nbt = nbt;
    p.tasks = tasks;
    p.ntasks = ntasks;
    p.claim = ints;
    p.abort_flag = ints + 1;
    p.fin = ints + 2;
    p.upd = ints + 2 + (int64_t)nbt * nbt;
    p.info = info;
    p.stage = (((uintptr_t)A & 15) == 0 && (lda & 1) == 0) ? 1 : 0;
    p.boff = nullptr;
    p.bstart = nullptr;
    p.masks = nullptr;
    p.rowocc = nullptr;
    p.bad_enc = nullptr;
    const int tr = trace_begin(FLAME_KC_OTHER, s);
    hipLaunchKernelGGL(k_by_blocks<false>, dim3((unsigned)std::min<int64_t>(grid, ntasks)), dim3(256), 0, s, p);
    FLAME_CHECK_LAUNCH();
    const double dn = (double)n;
    trace_end(tr, s, dn * dn * dn / 3.0, 16.0 * dn * dn);
    hipLaunchKernelGGL(k_dag_abort_info, dim3(1), dim3(64), 0, s, p.abort_flag, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

// ---- level(k) incomplete Cholesky-by-blocks on a tile pool -----------------

namespace {

__global__ void k_zero_f64(double *p, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

// pool[map[e]] = vals[e] for the upper entries of A (map[e] < 0: lower, skipped)
__global__ void k_scatter_vals(int64_t nnz, const int64_t *__restrict__ map, const double *__restrict__ vals,
                               double *__restrict__ pool) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = map[e];
        if (o >= 0) pool[o] = vals[e];
    }
}

__global__ void k_gather_vals(int64_t nnz, const int64_t *__restrict__ map, const double *__restrict__ pool,
                              double *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = pool[map[e]];
}

// info: -1 when a wait gave up, else the lowest breakdown column, else 0
__global__ void k_ichol_info(const int32_t *abort_flag, const int32_t *bad_enc, int32_t *info) {
    if (threadIdx.x == 0) *info = (*abort_flag == 1) ? -1 : (*bad_enc > 0 ? 0x7fffffff - *bad_enc : 0);
}

unsigned grid_for(int64_t count) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 65536)); }

}  // namespace

// Zeroes the pool, scatters A's upper entries into it, runs the task DAG of
// the block pattern on it (masked CHOL / TRSM, staged updates) and sets info
// (-1: a wait gave up; else the lowest breakdown column).  ints: claim,
// abort, fin[nbt^2], upd[nbt^2], breakdown (cleared here).
int launch_ichol_dag(double *pool, int64_t pool_elems, const double *vals, int64_t nnz_a, const int64_t *amap,
                     const int64_t *boff, const int32_t *bstart, const uint64_t *masks, const uint64_t *rowocc, int nbt,
                     const int4 *tasks, int64_t ntasks, int32_t *ints, int32_t *info, hipStream_t s) {
    const int64_t nints = 3 + 2 * (int64_t)nbt * nbt;
    int rc = launch_zero_i32(ints, nints, s);
    if (rc) return rc;
    rc = launch_zero_i32(info, 1, s);
    if (rc) return rc;
    if (pool_elems > 0) {
        hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(pool_elems)), dim3(256), 0, s, pool, pool_elems);
        FLAME_CHECK_LAUNCH();
    }
    if (nnz_a > 0) {
        hipLaunchKernelGGL(k_scatter_vals, dim3(grid_for(nnz_a)), dim3(256), 0, s, nnz_a, amap, vals, pool);
        FLAME_CHECK_LAUNCH();
    }
    if (ntasks == 0) return FLAME_OK;
    int dev = 0, cus = 0, per = 0;
    FLAME_HIP(hipGetDevice(&dev));
    FLAME_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    FLAME_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_by_blocks<true>, 256, 0));
    const int64_t grid = std::max(1, cus * std::max(1, per));
    DagP p;
    p.n = 0;
    p.A = pool;
    p.lda = kT;
    p.nbt = nbt;
    p.tasks = tasks;
    p.ntasks = ntasks;
    p.claim = ints;
    p.abort_flag = ints + 1;
    p.fin = ints + 2;
    p.upd = ints + 2 + (int64_t)nbt * nbt;
    p.info = info;
    p.stage = 1;
    p.boff = boff;
    p.bstart = bstart;
    p.masks = masks;
    p.rowocc = rowocc;
    p.bad_enc = ints + 2 + 2 * (int64_t)nbt * nbt;
    const int tr = trace_begin(FLAME_KC_OTHER, s);
    hipLaunchKernelGGL(k_by_blocks<true>, dim3((unsigned)std::min<int64_t>(grid, ntasks)), dim3(256), 0, s, p);
    FLAME_CHECK_LAUNCH();
    trace_end(tr, s, 0.0, 0.0);
    hipLaunchKernelGGL(k_ichol_info, dim3(1), dim3(64), 0, s, p.abort_flag, p.bad_enc, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_gather_vals(int64_t nnz, const int64_t *map, const double *pool, double *out, hipStream_t s) {
    if (nnz <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_gather_vals, dim3(grid_for(nnz)), dim3(256), 0, s, nnz, map, pool, out);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
