// Triangular solves with many right-hand sides on matrix cores, one launch
// per direction:
//   forward   U^T Y = B:  Y_i = U_ii^{-T} (B_i - sum_{q < i} U_qi^T Y_q)
//   backward  U X = Y:    X_i = U_ii^{-1} (Y_i - sum_{q > i} U_iq X_q)
// over row blocks of 128, in place on B (n x nrhs).  The right-hand sides are
// cut into chunks of 16 RB columns solved side by side, each with its own
// flags.  One workgroup per (row block, chunk) forms the sum over the blocks
// already solved, in solving order, as their flags appear, applies the
// precomputed inverse of the diagonal block (Dt_i = U_ii^{-T}, 128 x 128,
// identity-padded) and publishes block i.  Workgroup index = (position of i
// in solving order) * chunks + chunk: workgroups are dispatched in index
// order (in order on each XCD) and wait only on blocks earlier in that
// order, so the lowest unfinished block of every chunk always progresses.
// Every wait is bounded: one that gives up sets *err and the block is
// published as NaN, so that the launch still finishes.  (Spreading a long
// sum over several workgroups that hand partial sums to the block's owner
// was measured slower: every hand-off costs a device-scope release and
// acquire, i.e. L2 write-back and invalidation.)
//
// Products on v_mfma_f64_16x16x4f64: wavefront w owns rows 32 w .. 32 w + 31
// of the block (two 16-row blocks) and the chunk's RB 16-column blocks.  The
// operand of U (or of Dt) is loaded straight into registers, lane (r, g)
// holding the 32 consecutive k = 32 g .. 32 g + 31 of row r of its 16-row
// block; the right-hand block goes through LDS.  Placement of the results as
// in the panel TRSM: lane (r, g) item v holds row r, column g + 4 v of a
// 16 x 16 block.
#include <algorithm>

#include "dev_sync.h"
#include "flame_internal.h"
#include "trsm_rl.h"

namespace flame {

namespace {

constexpr int kTc = 128;                  // row block
constexpr long long kSpinCap = 1LL << 26;  // s_sleep rounds before a wait gives up

// Waits (bounded) for a block's flag; false if it gave up or another wait
// did (*err).
__device__ __forceinline__ bool wait_set(const int32_t *flag, int32_t *err) {
    return poll_at_least(flag, 1, err, 1, kSpinCap);
}

// After the barrier behind thread 0's wait: every wavefront invalidates its
// view of device memory, so that its ordinary (batched) loads of the block
// published before the flag see it.
__device__ __forceinline__ void acquire_all() { acquire_dev(); }

// Operand of row block h of this wavefront for all 32 k slots, from a
// column-major matrix M: TRANS = false reads element (row, k) at
// M[row + k * ld] (stride ld along k), TRANS = true reads (row, k) at
// M[k + row * ld] (contiguous along k).  Rows >= rmax and k >= kmax read as 0.
template <bool TRANS>
__device__ __forceinline__ void load_op(const double *__restrict__ M, int64_t ld, int row, int kbase, int rmax,
                                        int kmax, double (&a)[32]) {
    const int rr = min(row, rmax - 1);
#pragma unroll
    for (int t = 0; t < 32; ++t) {
        const int k = kbase + t;
        const int kk = min(k, kmax - 1);
        const double v = TRANS ? M[(int64_t)kk + (int64_t)rr * ld] : M[(int64_t)rr + (int64_t)kk * ld];
        a[t] = (row < rmax && k < kmax) ? v : 0.0;
    }
}

template <bool FWD, int RB>
__global__ __launch_bounds__(256) void k_trsm_chain(int64_t n, int64_t nrhs_all, const double *__restrict__ U,
                                                    int64_t ldu, const double *__restrict__ Dt, double *X_all,
                                                    int64_t ldx, int32_t *flags_all, int nchunks, int32_t *err) {
    constexpr int R = 16 * RB;
    __shared__ double Ys[kTc][R + 1];  // right-hand block of the current product, [k][c]
    __shared__ int s_bad;
    const int nblk = (int)((n + kTc - 1) / kTc);
    const int chunk = blockIdx.x % nchunks;
    const int pos = blockIdx.x / nchunks;  // place of row block i in solving order
    const int nrhs = (int)min((int64_t)R, nrhs_all - (int64_t)chunk * R);
    double *X = X_all + (int64_t)chunk * R * ldx;
    int32_t *flags = flags_all + (int64_t)chunk * nblk;
    const int i = FWD ? pos : nblk - 1 - pos;
    const int64_t i0 = (int64_t)i * kTc;
    const int w = (int)min((int64_t)kTc, n - i0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int nq = pos;  // blocks in the sum: all earlier ones in solving order
    if (tid == 0) s_bad = 0;

    typedef double d4_t __attribute__((ext_vector_type(4)));
    d4_t acc[2][RB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int cb = 0; cb < RB; ++cb) acc[h][cb] = d4_t{0.0, 0.0, 0.0, 0.0};

    for (int jq = 0; jq < nq; ++jq) {
        const int q = FWD ? jq : nblk - 1 - jq;  // the jq-th block in solving order
        const int64_t q0 = (int64_t)q * kTc;
        const int wq = (int)min((int64_t)kTc, n - q0);
        // operand of U for this block pair (independent of the flag: issued first)
        double a[2][32];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = 32 * wave + 16 * h + r;  // row of block i
            if (FWD)  // A(row, k) = U(q0 + k, i0 + row): column i0 + row, contiguous in k
                load_op<true>(U + q0 + i0 * ldu, ldu, row, 32 * g, w, wq, a[h]);
            else  // A(row, k) = U(i0 + row, q0 + k): stride ldu in k
                load_op<false>(U + i0 + q0 * ldu, ldu, row, 32 * g, w, wq, a[h]);
        }
        if (tid == 0 && !wait_set(flags + q, err)) s_bad = 1;
        __syncthreads();
        acquire_all();
        {
            constexpr int PER = kTc * R / 256;
            double v[PER];
#pragma unroll
            for (int e = 0; e < PER; ++e) {  // all loads issued before the LDS stores
                const int idx = tid + 256 * e;
                const int k = idx % kTc, c = idx / kTc;
                v[e] = X[q0 + min(k, wq - 1) + (int64_t)min(c, nrhs - 1) * ldx];
            }
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int idx = tid + 256 * e;
                const int k = idx % kTc, c = idx / kTc;
                Ys[k][c] = (k < wq && c < nrhs) ? v[e] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 32; ++t) {
#pragma unroll
            for (int cb = 0; cb < RB; ++cb) {
                const double yv = Ys[32 * g + t][16 * cb + r];
#pragma unroll
                for (int h = 0; h < 2; ++h) acc[h][cb] = mma_rc(a[h][t], yv, acc[h][cb]);
            }
        }
    }

    // the operand of the diagonal block's inverse, Dt_i forward, Dt_i^T backward; Dt_i is 128 x 128
    // column-major and identity-padded past w
    const double *D = Dt + (int64_t)i * kTc * kTc;
    double da[2][32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int row = 32 * wave + 16 * h + r;
        if (FWD)  // A(row, k) = Dt_i(row, k)
            load_op<false>(D, kTc, row, 32 * g, kTc, kTc, da[h]);
        else  // A(row, k) = Dt_i(k, row)
            load_op<true>(D, kTc, row, 32 * g, kTc, kTc, da[h]);
    }
    // right-hand side of the diagonal solve, B_i - sum, into LDS (rows >= w: 0)
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int cb = 0; cb < RB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 32 * wave + 16 * h + r, col = 16 * cb + g + 4 * v;
                Ys[row][col] = (row < w && col < nrhs) ? X[i0 + row + (int64_t)col * ldx] - acc[h][cb][v] : 0.0;
            }
    __syncthreads();
    // block i = Dt_i (rhs) forward, Dt_i^T (rhs) backward
    d4_t y[2][RB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int cb = 0; cb < RB; ++cb) y[h][cb] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 32; ++t) {
#pragma unroll
        for (int cb = 0; cb < RB; ++cb) {
            const double rv = Ys[32 * g + t][16 * cb + r];
#pragma unroll
            for (int h = 0; h < 2; ++h) y[h][cb] = mma_rc(da[h][t], rv, y[h][cb]);
        }
    }
    __syncthreads();
    const bool bad = s_bad != 0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int cb = 0; cb < RB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 32 * wave + 16 * h + r, col = 16 * cb + g + 4 * v;
                if (row < w && col < nrhs) store_dev(&X[i0 + row + (int64_t)col * ldx], bad ? __builtin_nan("") : y[h][cb][v]);
            }
    // publish: the stores completed by every wavefront, then the flag
    wait_stores();
    __syncthreads();
    if (tid == 0) store_dev(flags + i, 1);
}

}  // namespace

// Columns per chunk: 64 (four 16-column blocks per workgroup) when there are
// more than 16 right-hand sides, else 16.
int chain_rb(int64_t nrhs) { return nrhs > 16 ? 4 : 1; }

int launch_trsm_chain(bool forward, int64_t n, int64_t nrhs, const double *U, int64_t ldu, const double *Dt,
                      double *X, int64_t ldx, int32_t *flags, int32_t *err, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return FLAME_OK;
    const int64_t nblk = (n + kTc - 1) / kTc;
    const int rb = chain_rb(nrhs);
    const int nchunks = (int)((nrhs + 16 * rb - 1) / (16 * rb));
    int e = launch_zero_i32(flags, nblk * nchunks, s);
    if (e) return e;
    const int tr = trace_begin(FLAME_KC_OTHER, s);
    const dim3 grid((unsigned)(nblk * nchunks));
    if (rb == 4) {
        if (forward)
            hipLaunchKernelGGL((k_trsm_chain<true, 4>), grid, dim3(256), 0, s, n, nrhs, U, ldu, Dt, X, ldx, flags,
                               nchunks, err);
        else
            hipLaunchKernelGGL((k_trsm_chain<false, 4>), grid, dim3(256), 0, s, n, nrhs, U, ldu, Dt, X, ldx, flags,
                               nchunks, err);
    } else {
        if (forward)
            hipLaunchKernelGGL((k_trsm_chain<true, 1>), grid, dim3(256), 0, s, n, nrhs, U, ldu, Dt, X, ldx, flags,
                               nchunks, err);
        else
            hipLaunchKernelGGL((k_trsm_chain<false, 1>), grid, dim3(256), 0, s, n, nrhs, U, ldu, Dt, X, ldx, flags,
                               nchunks, err);
    }
    FLAME_CHECK_LAUNCH();
    const double dn = (double)n;
    trace_end(tr, s, dn * dn * (double)nrhs, 4.0 * dn * (dn + 1) + 16.0 * dn * (double)nrhs);
    return FLAME_OK;
}

int trsm_chain_flags(int64_t n, int64_t nrhs) {
    const int rb = chain_rb(nrhs);
    return (int)(((n + kTc - 1) / kTc) * ((nrhs + 16 * rb - 1) / (16 * rb)));
}

}  // namespace flame
