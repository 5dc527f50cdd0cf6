// Householder QR (flame_qr): the kernels of the steps that are not plain
// products.  The loop (qr.cpp) is the partitioned loop of Fig. "dense-chol"
// carried over to QR (the conclusion names QR among the factorizations the
// pattern extends to): factor a panel of columns into reflectors, then apply
// their block form to the columns on its right on the matrix cores.
//
// k_qr_panel factors an m x b (b <= 32) panel with the reflector convention
// of LAPACK's geqrf (beta = -sign(alpha) ||[alpha; x]||, tau = (beta - alpha)
// / beta, v = [1; x / (alpha - beta)]).  The panel's rows are spread over
// several workgroups (512 rows each, one per thread, all b columns in
// registers), so a tall panel is read from HBM once.  Step j needs, from all
// rows r > j, the sums
//     d_c = sum_r A(r, j) A(r, c),   c >= j     (d_j = sigma = ||x||^2),
// and the pivot row A(j, :).  They determine everything else: with
// den = alpha - beta, the reflected column c has w_c = A(j, c) + d_c / den,
// and A(r, c) -= tau w_c A(r, j) / den.  So each step is one exchange between
// the workgroups: every workgroup publishes its partial sums (device-scope
// stores into slots that start out holding a marker value), then reads all
// of them and adds them in workgroup order, so that every workgroup derives
// the same scalars bit for bit.  One workgroup (m <= 512) skips the exchange.
//
// The rest serves the block form H_0 ... H_{k-1} = I - V T V^T (T upper
// triangular, T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) V(:, 0:j)^T v_j):
// k_qr_skinny forms products X^T Y with a long K as slices (the Gram columns
// V^T V_p of a panel, V^T C of a block), k_qr_gt adds the Gram slices and
// appends the panel's columns to T in block form, k_qr_wy adds the slices of
// V^T C and forms Y = T^T V^T C for the update C -= V Y.
#include <algorithm>
#include <cstdlib>

#include "dev_sync.h"
#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kQB = 32;                  // panel width
constexpr int kPT = 512;                 // panel kernel threads (two wavefronts per SIMD)
constexpr int kRpt = 1;                  // panel rows per thread
constexpr int kWgRows = kPT * kRpt;      // panel rows per workgroup
constexpr int kGroups = kPT / 32;        // half-wavefronts
constexpr int kOB = 128;                 // outer block (order of T)
constexpr int kGramMax = 32;             // K slices of the Gram product at most
constexpr long long kQrSpin = 1LL << 22; // sleep rounds before a wait gives up
// The empty-slot marker: a signalling NaN.  Arithmetic never produces one and
// published values are canonicalized (any NaN becomes the quiet NaN), so a
// slot holding it has not been written yet.
constexpr unsigned long long kEmpty = 0xFFF4A5A5A5A5A5A5ull;

struct QrPanelP {
    int64_t m;  // panel rows
    int b;      // panel columns (<= kQB)
    int P;      // workgroups (ceil(m / kWgRows))
    double *A;
    int64_t lda;
    double *tau;  // b scalars
    // explicit V (unit diagonal, zeros above) as columns of Vs (rows ro + r)
    // and as rows of Vt (Vt[c + (ro + r) ldvt]); rows 0..ro-1 written as zeros
    double *Vs;
    int64_t ldvs;
    double *Vt;
    int64_t ldvt;
    int64_t ro;
    double *xch;  // b * P * kQB partial sums, then b * kQB pivot-row values
    // the other exchange buffer, reset here for the next panel (whose
    // workgroups are no more than these), nreset doubles; none when P = 1
    double *xnext;
    int64_t nreset;
    long long spin_cap;  // bound of each wait in sleep rounds (< 0: give up at once)
    int32_t *info;
};

__device__ __forceinline__ double publishable(double v) {
    return v != v ? __longlong_as_double(0x7FF8000000000000ll) : v;
}

// Waits (bounded: cap sleep rounds) until *p holds a value; false when
// *stop is set or the wait gives up (then *stop := 1).  cap < 0: gives up at
// once (the host's way to exercise this path).
__device__ bool poll_slot(const double *p, int32_t *stop, double *out, long long cap) {
    if (cap < 0) {
        store_dev(stop, 1);
        return false;
    }
    long long spins = 0;
    for (;;) {
        const double v = load_dev(p);
        if ((unsigned long long)__double_as_longlong(v) != kEmpty) {
            *out = v;
            return true;
        }
        if (++spins > cap) {
            store_dev(stop, 1);
            return false;
        }
        if ((spins & 63) == 0 && load_dev(stop) != 0) return false;  // one load per round otherwise
        __builtin_amdgcn_s_sleep(1);
    }
}

// v of the lane whose index differs in bit log2(D) (D < 32: inside each half
// of the wavefront), through the swizzle's bit mode on the two halves.
template <int D>
__device__ __forceinline__ double xor_lane(double v) {
    constexpr int pat = 0x1F | (D << 10);
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), pat);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), pat);
    return __hiloint2double(hi, lo);
}

// One step of the halving sum over lanes: the lane keeps H of its 2 H
// values (the upper ones when its bit D is set), added to its partner's.
template <int H, int D>
__device__ __forceinline__ void halve(double *d, int lane) {
    const bool hi = (lane & D) != 0;
#pragma unroll
    for (int c = 0; c < H; ++c) {
        const double give = hi ? d[c] : d[c + H];
        const double keep = hi ? d[c + H] : d[c];
        d[c] = keep + xor_lane<D>(give);
    }
}

// Column c of the kGroups rows of an LDS table, added pairwise in a fixed
// order (every workgroup adds the same values the same way).
template <int LD>
__device__ __forceinline__ double sum_groups(const double (*t)[LD], int c) {
    double v[kGroups];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) v[g] = t[g][c];
#pragma unroll
    for (int w = 1; w < kGroups; w *= 2)
#pragma unroll
        for (int g = 0; g < kGroups; g += 2 * w) v[g] += v[g + w];
    return v[0];
}

// The panel step's live columns C0..31 (C0 = 16 once the first 16 are
// final): the thread's row's share of d_c = x A(r, c), summed over each
// half-wavefront by recursive halving into red[half-wavefront][c].
template <int C0>
__device__ __forceinline__ void step_sums(const double (&a)[kQB], double xm, int tid, int lane,
                                          double (*red)[kQB]) {
    constexpr int L = kQB - C0;
    double d[L];
#pragma unroll
    for (int c = 0; c < L; ++c) d[c] = xm * a[C0 + c];
    if constexpr (L == 32) {  // afterwards lane l holds column l & 31 of its half's 32 lanes
        halve<16, 16>(d, lane);
        halve<8, 8>(d, lane);
        halve<4, 4>(d, lane);
        halve<2, 2>(d, lane);
        halve<1, 1>(d, lane);
        red[tid >> 5][lane & (kQB - 1)] = d[0];
    } else {  // 16 columns: lane l holds column C0 + ((l >> 1) & 15), lanes l, l ^ 1 alike
        static_assert(L == 16, "32 or 16 live columns");
        halve<8, 16>(d, lane);
        halve<4, 8>(d, lane);
        halve<2, 4>(d, lane);
        halve<1, 2>(d, lane);
        d[0] += xor_lane<1>(d[0]);
        if ((lane & 1) == 0) red[tid >> 5][C0 + ((lane >> 1) & 15)] = d[0];
    }
}

// Column j of the row (a product with the j-th unit vector over the live
// columns: exact for finite values, no per-element select).
template <int C0>
__device__ __forceinline__ double pick_col(const double (&a)[kQB], int j) {
    double x = 0.0;
#pragma unroll
    for (int c = C0; c < kQB; ++c) x = fma(a[c], c == j ? 1.0 : 0.0, x);
    return x;
}

// The row's update over the live columns: A(r, c) mul_c - tw_c v.
template <int C0>
__device__ __forceinline__ void step_update(double (&a)[kQB], const double *mul, const double *tw, double v) {
#pragma unroll
    for (int c = C0; c < kQB; ++c) a[c] = fma(a[c], mul[c], -(tw[c] * v));
}

__global__ __launch_bounds__(256) void k_qr_fill_empty(int64_t count, double *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = __longlong_as_double((long long)kEmpty);
}

__global__ __launch_bounds__(kPT) void k_qr_panel(QrPanelP p) {
    __shared__ double red[kGroups][kQB];      // per half-wavefront column sums
    __shared__ double grp[kGroups][kQB + 1];  // workgroup partials added by groups of the grid
    __shared__ double prow[2][kQB];     // pivot row: [0] as held by its owner, [1] as used
    __shared__ double tws[kQB];         // tau w_c (0 for c <= j)
    __shared__ double mulv[kQB];        // 1, and 1 / (alpha - beta) at column j
    __shared__ double keep[kQB];        // 1, and 0 at column j
    __shared__ double sc[4];            // beta, tau, 1 / (alpha - beta), sigma
    __shared__ int s_bad;
    if (*p.info != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wg = blockIdx.x;
    for (int64_t e = (int64_t)wg * kPT + tid; e < p.nreset; e += (int64_t)p.P * kPT)
        p.xnext[e] = __longlong_as_double((long long)kEmpty);
    const int64_t r0 = (int64_t)wg * kWgRows + tid;
    double a[kRpt][kQB];
#pragma unroll
    for (int i = 0; i < kRpt; ++i) {
        const int64_t r = r0 + kPT * i;
#pragma unroll
        for (int c = 0; c < kQB; ++c) a[i][c] = (r < p.m && c < p.b) ? p.A[r + c * p.lda] : 0.0;
    }
    if (tid == 0) s_bad = 0;
    double *const xrow = p.xch + (int64_t)p.b * p.P * kQB;
    for (int j = 0; j < p.b; ++j) {
        // column j of this thread's row if it lies below the pivot, else 0;
        // the columns left of 16 are final once j >= 16: those steps work on
        // the live columns only (a uniform choice; a third tier at 24
        // measured no faster)
        static_assert(kRpt == 1, "one panel row per thread");
        const int64_t r = r0;
        const bool below = r > j && r < p.m;
        const bool late = j >= 16;
        const double x = late ? pick_col<16>(a[0], j) : pick_col<0>(a[0], j);
        const double xm = below ? x : 0.0;
        if (late) step_sums<16>(a[0], xm, tid, lane, red);
        else step_sums<0>(a[0], xm, tid, lane, red);
        if (wg == 0 && tid == j) {
#pragma unroll
            for (int c = 0; c < kQB; ++c) prow[0][c] = a[0][c];
        }
        __syncthreads();
        double s_c = 0.0, s_j = 0.0;  // d_c and sigma, for threads tid < kQB
        if (p.P == 1) {
            if (tid < kQB) {
                s_c = sum_groups(red, tid);
                s_j = sum_groups(red, j);
                prow[1][tid] = prow[0][tid];
            }
        } else {
            if (tid < kQB) {
                const double part = sum_groups(red, tid);
                store_dev(p.xch + ((int64_t)j * p.P + wg) * kQB + tid, publishable(part));
                if (wg == 0) store_dev(xrow + (int64_t)j * kQB + tid, publishable(prow[0][tid]));
            }
            // gather: thread (g, c) adds the partials of workgroups g, g + kGroups, ...
            const int c = tid & (kQB - 1), g = tid >> 5;
            double s = 0.0;
            bool ok = true;
            for (int q = g; q < p.P && ok; q += kGroups) {
                double v = 0.0;
                ok = poll_slot(p.xch + ((int64_t)j * p.P + q) * kQB + c, p.info, &v, p.spin_cap);
                s += v;
            }
            if (ok && g == 0) {
                double v = 0.0;
                ok = poll_slot(xrow + (int64_t)j * kQB + c, p.info, &v, p.spin_cap);
                prow[1][c] = v;
            }
            grp[g][c] = s;
            if (!ok) s_bad = 1;
            __syncthreads();
            if (s_bad) return;
            if (tid < kQB) {
                s_c = sum_groups(grp, tid);
                s_j = sum_groups(grp, j);
            }
        }
        if (tid < kQB) {  // the scalars of step j, the same in every thread and workgroup
            const double alpha = prow[1][j];
            double tw = 0.0, beta = alpha, tj = 0.0, den = 1.0;
            if (s_j != 0.0) {
                const double mag = sqrt(alpha * alpha + s_j);
                beta = alpha >= 0.0 ? -mag : mag;
                tj = (beta - alpha) / beta;
                den = 1.0 / (alpha - beta);  // the reflector's scale, as a reciprocal
                if (tid > j) tw = tj * (prow[1][tid] + s_c * den);
            }
            tws[tid] = tw;
            mulv[tid] = tid == j ? den : 1.0;
            keep[tid] = tid == j ? 0.0 : 1.0;
            if (tid == 0) {
                sc[0] = beta;
                sc[1] = tj;
                sc[2] = den;
                sc[3] = s_j;
                if (wg == 0) p.tau[j] = tj;
            }
        }
        __syncthreads();
        if (sc[3] == 0.0) continue;  // H_j = I (uniform: every thread reads the same value)
        const double beta = sc[0], den = sc[2];
        // below the pivot: A(r, c) -= tau w_c v_r (tau w_c = 0 for c <= j) and
        // A(r, j) := v_r, as A(r, c) mul_c - tau w_c v_r (mul_c = 1 except
        // mul_j = 1 / (alpha - beta)); the pivot row: A(j, c) -= tau w_c and
        // A(j, j) := beta, as A(j, c) keep_c - tau w_c + beta (1 - keep_c)
        if (below) {
            const double v = xm * den;
            if (late) step_update<16>(a[0], mulv, tws, v);
            else step_update<0>(a[0], mulv, tws, v);
        } else if (r == j) {
#pragma unroll
            for (int c = 0; c < kQB; ++c) a[0][c] = fma(a[0][c], keep[c], fma(beta, 1.0 - keep[c], -tws[c]));
        }
    }
#pragma unroll
    for (int i = 0; i < kRpt; ++i) {
        const int64_t r = r0 + kPT * i;
        if (r >= p.m) continue;
#pragma unroll
        for (int c = 0; c < kQB; ++c) {
            if (c < p.b) {
                p.A[r + c * p.lda] = a[i][c];
                const double v = r > c ? a[i][c] : (r == c ? 1.0 : 0.0);
                p.Vs[(p.ro + r) + c * p.ldvs] = v;
                p.Vt[c + (p.ro + r) * p.ldvt] = v;
            }
        }
    }
    if (wg == 0) {
        for (int64_t e = tid; e < p.ro * p.b; e += kPT) {
            const int64_t rr = e % p.ro, c = e / p.ro;
            p.Vs[rr + c * p.ldvs] = 0.0;
            p.Vt[c + rr * p.ldvt] = 0.0;
        }
    }
}

// Zeroes two rows x cols blocks of the same shape (ld ldd).
__global__ __launch_bounds__(256) void k_qr_zero2(int64_t rows, double *__restrict__ d0, double *__restrict__ d1,
                                                  int64_t ldd) {
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i < rows; i += 256) {
        d0[i + j * ldd] = 0.0;
        d1[i + j * ldd] = 0.0;
    }
}

// One skinny product X^T Y (X: K x M, Y: K x N, column-major), cut into
// slices of kc rows whose products go to part + s M N.
struct SkinnyJob {
    int M, N;  // <= kOB
    int64_t K, kc;
    const double *X;
    int64_t ldx;
    const double *Y;
    int64_t ldy;
    double *part;
};

// LDS of a skinny product: 32 staged rows of X and of Y (TM, TN <= 8).
struct SkinnyLds {
    double xs[32][kOB + 1];
    double ys[32][kOB + 1];
};

// Slice s of the skinny C = X^T Y (M, N <= 128, K long): X(K_s, :)^T Y(K_s, :)
// over the slice K_s of kc rows, stored at part + s M N (column-major, ld M);
// the caller adds the slices in order.  Rows staged through LDS 32 at a time,
// the next 32 loaded into registers while the current ones are used; thread
// (ti, tj) forms the outputs (ti + 16 a, tj + 16 b), a < TM, b < TN
// (16 TM >= M, 16 TN >= N).
template <int TM, int TN>
__device__ __forceinline__ void skinny_slice(const SkinnyJob &q, int64_t s, SkinnyLds &L) {
    const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
    const int kr = tid & 31, cg = tid >> 5;  // staging: row kr of the 32, columns cg + 8 u
    const int64_t k0 = s * q.kc, k1 = min(q.K, k0 + q.kc);
    double acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = 0.0;
    // two groups of 32 rows in flight in registers while one is used
    double xa[2 * TM], ya[2 * TN], xb[2 * TM], yb[2 * TN];
    auto fetch = [&](double *xr, double *yr, int64_t kb) {
        const int64_t k = kb + kr;
        const bool in = k < k1;
#pragma unroll
        for (int u = 0; u < 2 * TM; ++u) {
            const int i = cg + 8 * u;
            xr[u] = (in && i < q.M) ? q.X[k + i * q.ldx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 2 * TN; ++u) {
            const int j = cg + 8 * u;
            yr[u] = (in && j < q.N) ? q.Y[k + j * q.ldy] : 0.0;
        }
    };
    auto use = [&](const double *xr, const double *yr) {
#pragma unroll
        for (int u = 0; u < 2 * TM; ++u) L.xs[kr][cg + 8 * u] = xr[u];
#pragma unroll
        for (int u = 0; u < 2 * TN; ++u) L.ys[kr][cg + 8 * u] = yr[u];
        __syncthreads();
    };
    auto multiply = [&]() {
#pragma unroll 4
        for (int r = 0; r < 32; ++r) {
            double xv[TM], yv[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) xv[a] = L.xs[r][ti + 16 * a];
#pragma unroll
            for (int b = 0; b < TN; ++b) yv[b] = L.ys[r][tj + 16 * b];
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b) acc[a][b] += xv[a] * yv[b];
        }
        __syncthreads();
    };
    fetch(xa, ya, k0);
    fetch(xb, yb, k0 + 32);
    for (int64_t kb = k0; kb < k1; kb += 64) {
        use(xa, ya);
        fetch(xa, ya, kb + 64);
        multiply();
        if (kb + 32 < k1) {  // uniform
            use(xb, yb);
            fetch(xb, yb, kb + 96);
            multiply();
        }
    }
    double *dst = q.part + s * q.M * q.N;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int i = ti + 16 * a, j = tj + 16 * b;
            if (i < q.M && j < q.N) dst[i + (int64_t)j * q.M] = acc[a][b];
        }
}

// One or two skinny products in one launch: workgroups [0, S1) take the
// slices of the first, the others those of the second.
template <int TM1, int TN1, int TM2, int TN2>
__global__ __launch_bounds__(256) void k_qr_skinny(SkinnyJob q1, int S1, SkinnyJob q2,
                                                   const int32_t *__restrict__ info) {
    __shared__ SkinnyLds L;
    if (*info != 0) return;
    if ((int)blockIdx.x < S1) skinny_slice<TM1, TN1>(q1, blockIdx.x, L);
    else skinny_slice<TM2, TN2>(q2, blockIdx.x - S1, L);
}

// From the S partial products of V^T V_p (j1 x b, b = j1 - j0 <= kQB,
// j1 <= kOB: the Gram columns of the panel's reflectors j0..j1-1, added in
// slice order), columns j0..j1-1 of T (ld ldt), given columns 0..j0-1.  In
// block form, with T11 the first j0 columns and V = [V1 V2]:
//   T22 = the recurrence on the new columns alone,
//   T12 = -T11 (V1^T V2) T22.
// One workgroup.  T22: row i of T22 depends only on row i and on V2^T V2, so
// each row is formed by one thread from its own registers, no barriers; then
// the two products through LDS.
__global__ __launch_bounds__(1024) void k_qr_gt(int S, int j0, int j1, const double *__restrict__ part,
                                               const double *__restrict__ tau, double *__restrict__ T, int64_t ldt,
                                               const int32_t *__restrict__ info) {
    constexpr int kH = kOB - kQB;          // rows of T12 at most
    __shared__ double g[kOB][kQB + 1];     // V^T V_p (rows 0..j1-1)
    __shared__ double t22[kQB][kQB + 1];
    __shared__ double x[kH][kQB + 1];      // (V1^T V2) T22
    __shared__ double t11[kH][kH + 1];
    __shared__ double tv[kQB];
    if (*info != 0) return;
    const int tid = threadIdx.x, b = j1 - j0;
    // the slices (S <= kGramMax) of each element are all loaded before they
    // are added, in slice order
    for (int e = tid; e < j1 * b; e += 1024) {
        const int r = e % j1, c = e / j1;
        double v[kGramMax];
#pragma unroll
        for (int q = 0; q < kGramMax; ++q) v[q] = q < S ? part[(int64_t)q * j1 * b + e] : 0.0;
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < kGramMax; ++q) sum += v[q];
        g[r][c] = sum;
    }
    for (int e = tid; e < j0 * j0; e += 1024) {
        const int r = e % j0, c = e / j0;
        t11[r][c] = r <= c ? T[r + (int64_t)c * ldt] : 0.0;
    }
    if (tid < kQB) tv[tid] = tid < b ? tau[j0 + tid] : 0.0;
    __syncthreads();
    if (tid < kQB) {  // row i = tid of T22: T(i, c) = -tau_c sum_{l < c} T(i, l) (V2^T V2)(l, c)
        const int i = tid;
        double t[kQB];
#pragma unroll
        for (int c = 0; c < kQB; ++c) {
            double sum = 0.0;
#pragma unroll
            for (int l = 0; l < c; ++l) sum += t[l] * g[j0 + l][c];
            t[c] = c < b ? (c > i ? -tv[c] * sum : (c == i ? tv[c] : 0.0)) : 0.0;
        }
#pragma unroll
        for (int c = 0; c < kQB; ++c) t22[i][c] = t[c];
    }
    __syncthreads();
    if (j0 > 0) {
        // thread (r, h): row r, columns 8 h .. 8 h + 7, eight independent sums
        for (int e = tid; e < j0 * 4; e += 1024) {  // X = (V1^T V2) T22
            const int r = e % j0, h = e / j0;
            double acc[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] = 0.0;
            for (int l = 0; l < b; ++l) {
                const double gl = g[r][l];
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] += gl * t22[l][8 * h + c];
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) x[r][8 * h + c] = acc[c];
        }
        __syncthreads();
        for (int e = tid; e < j0 * 4; e += 1024) {  // T12 = -T11 X
            const int r = e % j0, h = e / j0;
            double acc[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] = 0.0;
            for (int l = r; l < j0; ++l) {
                const double tl = t11[r][l];
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] += tl * x[l][8 * h + c];
            }
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (8 * h + c < b) T[r + (int64_t)(j0 + 8 * h + c) * ldt] = -acc[c];
        }
    }
    // T22 and zeros below it (the rows up to kOB: the products read the whole block)
    for (int e = tid; e < (kOB - j0) * b; e += 1024) {
        const int r = e % (kOB - j0), c = e / (kOB - j0);
        T[(j0 + r) + (int64_t)(j0 + c) * ldt] = r < kQB ? t22[r][c] : 0.0;
    }
}

// Y := T^T V^T C for the product slices of V^T C (kb x nc, added in slice
// order): one workgroup per column j of Y (ld kOB); T (kb x kb, ld ldt,
// upper triangular).
__global__ __launch_bounds__(kOB) void k_qr_wy(int S, int kb, int nc, const double *__restrict__ part,
                                               const double *__restrict__ T, int64_t ldt, double *__restrict__ Y,
                                               const int32_t *__restrict__ info) {
    __shared__ double w[kOB];
    if (*info != 0) return;
    const int i = threadIdx.x, j = blockIdx.x;
    if (i < kb) {
        double sum = 0.0;
#pragma unroll 8
        for (int q = 0; q < S; ++q) sum += part[(int64_t)q * kb * nc + i + (int64_t)j * kb];
        w[i] = sum;
    }
    __syncthreads();
    if (i < kb) {
        double sum = 0.0;
        for (int l = 0; l <= i; ++l) sum += T[l + (int64_t)i * ldt] * w[l];
        Y[i + (int64_t)j * kOB] = sum;
    }
}

}  // namespace

int qr_panel_rows() { return kWgRows; }

int launch_qr_fill_empty(int64_t count, double *p, hipStream_t s) {
    if (count <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_qr_fill_empty, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, p);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

// xch must hold empty slots on entry (launch_qr_fill_empty once, then each
// panel resets xnext for the one after it).
int launch_qr_panel(int64_t m, int b, double *A, int64_t lda, double *tau, double *Vs, int64_t ldvs, double *Vt,
                    int64_t ldvt, int64_t ro, double *xch, double *xnext, int32_t *info, hipStream_t s) {
    if (m <= 0 || b <= 0) return FLAME_OK;
    if (b > kQB || m < b) return FLAME_ERR_UNSUPPORTED;
    QrPanelP p;
    p.m = m;
    p.b = b;
    p.P = (int)((m + kWgRows - 1) / kWgRows);
    p.A = A;
    p.lda = lda;
    p.tau = tau;
    p.Vs = Vs;
    p.ldvs = ldvs;
    p.Vt = Vt;
    p.ldvt = ldvt;
    p.ro = ro;
    p.xch = xch;
    p.xnext = xnext;
    p.nreset = p.P > 1 ? (int64_t)kQB * p.P * kQB + (int64_t)kQB * kQB : 0;
    // FLAME_QR_SPIN_CAP (environment): the waits' bound, for tests of the
    // give-up path; kQrSpin otherwise
    const char *cap = getenv("FLAME_QR_SPIN_CAP");
    p.spin_cap = (cap != nullptr && *cap != '\0') ? atoll(cap) : kQrSpin;
    p.info = info;
    const int tr = trace_begin(FLAME_KC_CHOL, s);
    hipLaunchKernelGGL(k_qr_panel, dim3((unsigned)p.P), dim3(kPT), 0, s, p);
    FLAME_CHECK_LAUNCH();
    trace_end(tr, s, 4.0 * (double)m * b * b, 8.0 * (double)m * b * 4);
    return FLAME_OK;
}

int launch_qr_zero2(int64_t rows, int64_t cols, double *d0, double *d1, int64_t ldd, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return FLAME_OK;
    hipLaunchKernelGGL(k_qr_zero2, dim3((unsigned)cols), dim3(256), 0, s, rows, d0, d1, ldd);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int qr_slices(int64_t K, int smax, int64_t *kc) {
    int S = (int)std::min<int64_t>(smax, std::max<int64_t>(1, (K + 127) / 128));
    int64_t c = ((K + S - 1) / S + 31) / 32 * 32;
    S = (int)((K + c - 1) / c);
    *kc = c;
    return S;
}

namespace {
int tiles16(int v) { return v <= 32 ? 2 : (v <= 64 ? 4 : 8); }

template <int TM1, int TN1, int TM2, int TN2>
void skinny_go(const SkinnyJob &q1, int S1, const SkinnyJob &q2, int S2, const int32_t *info, hipStream_t s) {
    hipLaunchKernelGGL((k_qr_skinny<TM1, TN1, TM2, TN2>), dim3((unsigned)(S1 + S2)), dim3(256), 0, s, q1, S1, q2,
                       info);
}
template <int TM1, int TN1, int TM2>
void skinny_tn2(int tn2, const SkinnyJob &q1, int S1, const SkinnyJob &q2, int S2, const int32_t *info,
                hipStream_t s) {
    if (tn2 == 2) skinny_go<TM1, TN1, TM2, 2>(q1, S1, q2, S2, info, s);
    else if (tn2 == 4) skinny_go<TM1, TN1, TM2, 4>(q1, S1, q2, S2, info, s);
    else skinny_go<TM1, TN1, TM2, 8>(q1, S1, q2, S2, info, s);
}
}  // namespace

// The Gram columns of a panel (M1 x N1, N1 <= 32) and, when S2 > 0, the
// product V_p^T C of its update (M2 = 32 x N2), in one launch; or one product
// alone (S2 = 0).  Shapes the driver uses: (M1 <= 128, N1 <= 32) with
// (32, <= 128), and (<= 128, <= 128) alone.
int launch_qr_skinny(int S1, int M1, int N1, int64_t K1, int64_t kc1, const double *X1, int64_t ldx1,
                     const double *Y1, int64_t ldy1, double *part1, int S2, int M2, int N2, int64_t K2, int64_t kc2,
                     const double *X2, int64_t ldx2, const double *Y2, int64_t ldy2, double *part2,
                     const int32_t *info, hipStream_t s) {
    if (M1 <= 0 || N1 <= 0 || S1 <= 0) return FLAME_OK;
    if (M1 > kOB || N1 > kOB || K1 <= 0) return FLAME_ERR_UNSUPPORTED;
    SkinnyJob q1{M1, N1, K1, kc1, X1, ldx1, Y1, ldy1, part1};
    SkinnyJob q2{M2, N2, K2, kc2, X2, ldx2, Y2, ldy2, part2};
    if (S2 > 0 && (M2 <= 0 || N2 <= 0)) S2 = 0;
    if (S2 > 0 && (N1 > kQB || M2 > kQB || N2 > kOB || K2 <= 0)) return FLAME_ERR_UNSUPPORTED;
    const int tm1 = tiles16(M1), tn1 = tiles16(N1);
    if (S2 > 0) {  // the panel's pair: TN1 = 2, TM2 = 2
        const int tn2 = tiles16(N2);
        if (tm1 == 2) skinny_tn2<2, 2, 2>(tn2, q1, S1, q2, S2, info, s);
        else if (tm1 == 4) skinny_tn2<4, 2, 2>(tn2, q1, S1, q2, S2, info, s);
        else skinny_tn2<8, 2, 2>(tn2, q1, S1, q2, S2, info, s);
    } else if (tn1 == 2) {  // one product (the second shape is not used)
        if (tm1 == 2) skinny_go<2, 2, 2, 2>(q1, S1, q2, 0, info, s);
        else if (tm1 == 4) skinny_go<4, 2, 2, 2>(q1, S1, q2, 0, info, s);
        else skinny_go<8, 2, 2, 2>(q1, S1, q2, 0, info, s);
    } else {
        skinny_go<8, 8, 2, 2>(q1, S1, q2, 0, info, s);
    }
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_qr_gt(int S, int j0, int j1, const double *part, const double *tau, double *T, int64_t ldt,
                 const int32_t *info, hipStream_t s) {
    if (j1 <= j0) return FLAME_OK;
    if (j0 < 0 || j1 > kOB || j1 - j0 > kQB) return FLAME_ERR_UNSUPPORTED;
    if (S > kGramMax) return FLAME_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_qr_gt, dim3(1), dim3(1024), 0, s, S, j0, j1, part, tau, T, ldt, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

int launch_qr_wy(int S, int kb, int nc, const double *part, const double *T, int64_t ldt, double *Y,
                 const int32_t *info, hipStream_t s) {
    if (kb <= 0 || nc <= 0) return FLAME_OK;
    if (kb > kOB) return FLAME_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_qr_wy, dim3((unsigned)nc), dim3(kOB), 0, s, S, kb, nc, part, T, ldt, Y, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
