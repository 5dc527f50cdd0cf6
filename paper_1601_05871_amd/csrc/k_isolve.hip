// Preconditioned conjugate gradients with the incomplete factor (the use of
// the factor the paper names in its introduction: a preconditioner for SPD
// solves): the sparse product A x, and z = (U^T U)^{-1} r with U the
// block-sparse incomplete factor held in a plan's tile pool.
//
// Triangular solves on the pool: one workgroup per block row i, in solving
// order (forward: U^T y = b, blocks 0 .. nbt - 1; backward: U x = y, blocks
// nbt - 1 .. 0).  The workgroup sums the products of the existing blocks of
// its block column (forward: U(q, i)^T y_q, q < i) or block row (backward:
// U(i, j) x_j, j > i) as their flags appear, then solves with its diagonal
// tile in LDS, row by row, and publishes its block (device-scope stores, then
// the flag: dev_sync.h).  Workgroups are dispatched in index order and wait
// only on earlier ones, so the chain progresses; every wait is bounded (a
// wait that gives up sets *err, the block is published as NaN).
#include "dev_sync.h"
#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kT = 128;
constexpr long long kSpin = 1LL << 26;

struct BsolveP {
    const double *pool;
    const int64_t *boff;   // nbt x nbt tile offsets (-1: missing)
    const int32_t *bstart; // nbt + 1
    int nbt;
    const int32_t *lptr;   // per block: its list of off-diagonal blocks (forward: q < i with (q, i); backward: j > i with (i, j))
    const int32_t *lblk;
    double *y;             // in: right-hand side (plan numbering); out: solution
    int32_t *flags;        // nbt, cleared before the launch
    int32_t *err;
};

template <bool FWD>
__global__ __launch_bounds__(256, 1) void k_bsolve(BsolveP p) {
    __shared__ double T[kT * kT];  // the diagonal tile, column-major, its diagonal moved to dg
    __shared__ double rhs[kT], out[kT], vin[kT], dg[kT], part[2][kT];
    __shared__ int s_bad;
    const int nbt = p.nbt;
    const int i = __builtin_amdgcn_readfirstlane(FWD ? (int)blockIdx.x : nbt - 1 - (int)blockIdx.x);
    const int r0 = __builtin_amdgcn_readfirstlane(p.bstart[i]);
    const int w = __builtin_amdgcn_readfirstlane(p.bstart[i + 1]) - r0;
    const int tid = threadIdx.x, c = tid & (kT - 1), h = tid >> 7;
    if (tid == 0) s_bad = 0;
    const double *D = p.pool + p.boff[(int64_t)i * nbt + i];
    for (int e = tid; e < w * kT; e += 256) T[e] = D[e];
    double acc = 0.0;
    const int e0 = __builtin_amdgcn_readfirstlane(p.lptr[i]), e1 = __builtin_amdgcn_readfirstlane(p.lptr[i + 1]);
    for (int e = e0; e < e1; ++e) {
        const int q = __builtin_amdgcn_readfirstlane(p.lblk[e]);
        const int q0 = __builtin_amdgcn_readfirstlane(p.bstart[q]);
        const int wq = __builtin_amdgcn_readfirstlane(p.bstart[q + 1]) - q0;
        if (tid == 0 && !poll_at_least(p.flags + q, 1, p.err, 1, kSpin)) s_bad = 1;
        __syncthreads();
        if (tid < kT) vin[tid] = (tid < wq) ? load_dev(p.y + q0 + tid) : 0.0;
        __syncthreads();
        if (FWD) {  // (U(q, i)^T y_q)(c) = sum_r U(q, i)(r, c) y_q(r), rows of half h
            const double *B = p.pool + p.boff[(int64_t)q * nbt + i] + (int64_t)c * kT + 64 * h;
#pragma unroll 8
            for (int r = 0; r < 64; ++r) acc = fma(B[r], vin[64 * h + r], acc);
        } else {  // (U(i, j) x_j)(c) = sum_col U(i, j)(c, col) x_j(col), columns of half h
            const double *B = p.pool + p.boff[(int64_t)i * nbt + q] + c + (int64_t)(64 * h) * kT;
#pragma unroll 8
            for (int col = 0; col < 64; ++col) acc = fma(B[(int64_t)col * kT], vin[64 * h + col], acc);
        }
        __syncthreads();  // vin is refilled by the next block
    }
    part[h][c] = acc;
    __syncthreads();
    if (tid < kT) {
        rhs[tid] = (tid < w) ? p.y[r0 + tid] - (part[0][tid] + part[1][tid]) : 0.0;
        dg[tid] = (tid < w) ? T[tid + tid * kT] : 1.0;
        if (tid < w) T[tid + tid * kT] = 0.0;
    }
    __syncthreads();
    // the diagonal solve: U zero below its diagonal (and on it, now), so the
    // update of every entry by the one just solved is unconditional
    for (int s = 0; s < w; ++s) {
        const int r = FWD ? s : w - 1 - s;
        const double v = rhs[r] / dg[r];
        if (tid < kT) {
            if (tid == r) out[r] = v;
            rhs[tid] = fma(-(FWD ? T[r + tid * kT] : T[tid + r * kT]), v, rhs[tid]);
        }
        __syncthreads();
    }
    const bool bad = s_bad != 0;
    if (tid < w) store_dev(p.y + r0 + tid, bad ? __builtin_nan("") : out[tid]);
    wait_stores();
    __syncthreads();
    if (tid == 0) store_dev(p.flags + i, 1);
}

// y = A x (sub = 0) or y = b - A x (sub = 1), CSR rows, one thread per row.
__global__ void k_spmv(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const double *__restrict__ v, const double *__restrict__ x, const double *__restrict__ b,
                       double *__restrict__ y, int sub) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) s = fma(v[e], x[ci[e]], s);
    y[i] = sub ? b[i] - s : s;
}

// dst[k] = src[order[k]] (gather = true) or dst[order[k]] = src[k]
__global__ void k_permute(int64_t n, const int64_t *__restrict__ order, const double *__restrict__ src,
                          double *__restrict__ dst, int gather) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (gather)
        dst[k] = src[order[k]];
    else
        dst[order[k]] = src[k];
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace

int launch_bsolve(bool forward, const double *pool, const int64_t *boff, const int32_t *bstart, int nbt,
                  const int32_t *lptr, const int32_t *lblk, double *y, int32_t *flags, int32_t *err, hipStream_t s) {
    if (nbt <= 0) return FLAME_OK;
    int rc = launch_zero_i32(flags, nbt, s);
    if (rc) return rc;
    BsolveP p{pool, boff, bstart, nbt, lptr, lblk, y, flags, err};
    if (forward)
        hipLaunchKernelGGL(k_bsolve<true>, dim3((unsigned)nbt), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL(k_bsolve<false>, dim3((unsigned)nbt), dim3(256), 0, s, p);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x, const double *b,
                double *y, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_spmv, dim3(blocks_for(n)), dim3(256), 0, s, n, rp, ci, v, x, b, y, b != nullptr ? 1 : 0);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_permute(int64_t n, const int64_t *order, const double *src, double *dst, bool gather, hipStream_t s) {
    if (n <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_permute, dim3(blocks_for(n)), dim3(256), 0, s, n, order, src, dst, gather ? 1 : 0);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
