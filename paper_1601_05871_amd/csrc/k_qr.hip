// Householder QR (flame_qr): the kernels of the steps that are not plain
// products.  The loop (qr.cpp) is the partitioned loop of Fig. "dense-chol"
// carried over to QR (the conclusion names QR among the factorizations the
// pattern extends to): factor a panel of columns into reflectors, then apply
// their block form to the columns on its right on the matrix cores.
//
// k_qr_panel factors an m x b (b <= 32) panel with the reflector convention
// of LAPACK's geqrf (beta = -sign(alpha) ||[alpha; x]||, tau = (beta - alpha)
// / beta, v = [1; x / (alpha - beta)]).  The panel's rows are spread over
// several workgroups (512 rows each, two per thread, all b columns in
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
// k_qr_t forms the upper triangular T of the block reflector
// H_0 ... H_{k-1} = I - V T V^T column by column (T(j, j) = tau_j,
// T(0:j, j) = -tau_j T(0:j, 0:j) V(:, 0:j)^T v_j) from the Gram matrix of V.
#include "dev_sync.h"
#include "flame_internal.h"

namespace flame {

namespace {

constexpr int kQB = 32;                  // panel width
constexpr int kRpt = 2;                  // panel rows per thread
constexpr int kWgRows = 256 * kRpt;      // panel rows per workgroup
constexpr int kOB = 128;                 // outer block (order of T)
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
    int32_t *info;
};

__device__ __forceinline__ double publishable(double v) {
    return v != v ? __longlong_as_double(0x7FF8000000000000ll) : v;
}

// Waits (bounded) until *p holds a value; false when *stop is set or the
// wait gives up (then *stop := 1).
__device__ bool poll_slot(const double *p, int32_t *stop, double *out) {
    long long spins = 0;
    for (;;) {
        const double v = load_dev(p);
        if ((unsigned long long)__double_as_longlong(v) != kEmpty) {
            *out = v;
            return true;
        }
        if (load_dev(stop) != 0) return false;
        if (++spins > kQrSpin) {
            store_dev(stop, 1);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

__global__ __launch_bounds__(256) void k_qr_fill_empty(int64_t count, double *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = __longlong_as_double((long long)kEmpty);
}

__global__ __launch_bounds__(256) void k_qr_panel(QrPanelP p) {
    __shared__ double red[4][kQB];      // per-wave column sums
    __shared__ double grp[8][kQB + 1];  // workgroup partials added by groups of the grid
    __shared__ double prow[2][kQB];     // pivot row: [0] as held by its owner, [1] as used
    __shared__ double tws[kQB];         // tau w_c (0 for c <= j)
    __shared__ double sc[4];            // beta, tau, alpha - beta, sigma
    __shared__ int s_bad;
    if (*p.info != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wg = blockIdx.x;
    const int64_t r0 = (int64_t)wg * kWgRows + tid;
    double a[kRpt][kQB];
#pragma unroll
    for (int i = 0; i < kRpt; ++i) {
        const int64_t r = r0 + 256 * i;
#pragma unroll
        for (int c = 0; c < kQB; ++c) a[i][c] = (r < p.m && c < p.b) ? p.A[r + c * p.lda] : 0.0;
    }
    if (tid == 0) s_bad = 0;
    double *const xrow = p.xch + (int64_t)p.b * p.P * kQB;
    for (int j = 0; j < p.b; ++j) {
        // column j of this thread's rows (selected without a dynamic index)
        double x[kRpt];
        bool below[kRpt];
#pragma unroll
        for (int i = 0; i < kRpt; ++i) {
            const int64_t r = r0 + 256 * i;
            below[i] = r > j && r < p.m;
            x[i] = 0.0;
#pragma unroll
            for (int c = 0; c < kQB; ++c)
                if (c == j) x[i] = a[i][c];
        }
        {
            double d[kQB];
#pragma unroll
            for (int c = 0; c < kQB; ++c) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < kRpt; ++i)
                    if (below[i]) s += x[i] * a[i][c];
                d[c] = s;
            }
            // wave sum by recursive halving: at distance 32 >> st the lane
            // keeps half of its columns (the upper half when that bit of its
            // index is set), added to its partner's; in the end it holds
            // column (lane >> 1) & 31
#pragma unroll
            for (int st = 0; st < 5; ++st) {
                const int h = 16 >> st, dist = 32 >> st;
                const bool hi = (lane & dist) != 0;
#pragma unroll
                for (int c = 0; c < h; ++c) {
                    const double give = hi ? d[c] : d[c + h];
                    const double keep = hi ? d[c + h] : d[c];
                    d[c] = keep + __shfl_xor(give, dist);
                }
            }
            d[0] += __shfl_xor(d[0], 1);
            if ((lane & 1) == 0) red[wave][(lane >> 1) & (kQB - 1)] = d[0];
        }
        if (wg == 0 && tid == j) {
#pragma unroll
            for (int c = 0; c < kQB; ++c) prow[0][c] = a[0][c];
        }
        __syncthreads();
        double s_c = 0.0, s_j = 0.0;  // d_c and sigma, for threads tid < kQB
        if (p.P == 1) {
            if (tid < kQB) {
                s_c = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
                s_j = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
                prow[1][tid] = prow[0][tid];
            }
        } else {
            if (tid < kQB) {
                const double part = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
                store_dev(p.xch + ((int64_t)j * p.P + wg) * kQB + tid, publishable(part));
                if (wg == 0) store_dev(xrow + (int64_t)j * kQB + tid, publishable(prow[0][tid]));
            }
            // gather: thread (g, c) adds the partials of workgroups g, g + 8, ...
            const int c = tid & (kQB - 1), g = tid >> 5;
            double s = 0.0;
            bool ok = true;
            for (int q = g; q < p.P && ok; q += 8) {
                double v = 0.0;
                ok = poll_slot(p.xch + ((int64_t)j * p.P + q) * kQB + c, p.info, &v);
                s += v;
            }
            if (ok && g == 0) {
                double v = 0.0;
                ok = poll_slot(xrow + (int64_t)j * kQB + c, p.info, &v);
                prow[1][c] = v;
            }
            grp[g][c] = s;
            if (!ok) s_bad = 1;
            __syncthreads();
            if (s_bad) return;
            if (tid < kQB) {
                s_c = ((grp[0][tid] + grp[1][tid]) + (grp[2][tid] + grp[3][tid])) +
                      ((grp[4][tid] + grp[5][tid]) + (grp[6][tid] + grp[7][tid]));
                s_j = ((grp[0][j] + grp[1][j]) + (grp[2][j] + grp[3][j])) +
                      ((grp[4][j] + grp[5][j]) + (grp[6][j] + grp[7][j]));
            }
        }
        if (tid < kQB) {  // the scalars of step j, the same in every thread and workgroup
            const double alpha = prow[1][j];
            double tw = 0.0, beta = alpha, tj = 0.0, den = 1.0;
            if (s_j != 0.0) {
                const double mag = sqrt(alpha * alpha + s_j);
                beta = alpha >= 0.0 ? -mag : mag;
                tj = (beta - alpha) / beta;
                den = alpha - beta;
                if (tid > j) tw = tj * (prow[1][tid] + s_c / den);
            }
            tws[tid] = tw;
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
#pragma unroll
        for (int i = 0; i < kRpt; ++i) {
            const int64_t r = r0 + 256 * i;
            if (below[i]) {
                const double v = x[i] / den;
#pragma unroll
                for (int c = 0; c < kQB; ++c) a[i][c] = c == j ? v : a[i][c] - tws[c] * v;
            } else if (r == j) {
#pragma unroll
                for (int c = 0; c < kQB; ++c) a[i][c] = c == j ? beta : a[i][c] - tws[c];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kRpt; ++i) {
        const int64_t r = r0 + 256 * i;
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
    if (wg == 0)
        for (int64_t e = tid; e < p.ro * p.b; e += 256) {
            const int64_t rr = e % p.ro, c = e / p.ro;
            p.Vs[rr + c * p.ldvs] = 0.0;
            p.Vt[c + rr * p.ldvt] = 0.0;
        }
}

// Columns j0..j1-1 of T (ld ldt, j1 <= kOB) from G = -V^T V (ld ldg) and tau,
// given columns 0..j0-1; one workgroup, T(0:j1, 0:j1) in LDS, thread i forms
// row i.
__global__ __launch_bounds__(kOB) void k_qr_t(int j0, int j1, const double *__restrict__ G, int64_t ldg,
                                              const double *__restrict__ tau, double *__restrict__ T, int64_t ldt,
                                              const int32_t *__restrict__ info) {
    __shared__ double t[kOB][kOB + 1];
    if (*info != 0) return;
    const int i = threadIdx.x;
    for (int l = 0; l < j0; ++l) t[i][l] = (i <= l) ? T[i + (int64_t)l * ldt] : 0.0;
    __syncthreads();
    for (int j = j0; j < j1; ++j) {
        const double tj = tau[j];
        double s = 0.0;
        for (int l = i; l < j; ++l) s += t[i][l] * G[l + (int64_t)j * ldg];  // V^T v_j = -G(:, j)
        t[i][j] = i < j ? tj * s : (i == j ? tj : 0.0);
        __syncthreads();
    }
    for (int j = j0; j < j1; ++j) T[i + (int64_t)j * ldt] = t[i][j];  // zero below the diagonal
}

}  // namespace

int qr_panel_rows() { return kWgRows; }

int launch_qr_panel(int64_t m, int b, double *A, int64_t lda, double *tau, double *Vs, int64_t ldvs, double *Vt,
                    int64_t ldvt, int64_t ro, double *xch, int32_t *info, hipStream_t s) {
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
    p.info = info;
    if (p.P > 1) {
        const int64_t count = (int64_t)b * p.P * kQB + (int64_t)b * kQB;
        hipLaunchKernelGGL(k_qr_fill_empty, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, xch);
        FLAME_CHECK_LAUNCH();
    }
    const int tr = trace_begin(FLAME_KC_CHOL, s);
    hipLaunchKernelGGL(k_qr_panel, dim3((unsigned)p.P), dim3(256), 0, s, p);
    FLAME_CHECK_LAUNCH();
    trace_end(tr, s, 4.0 * (double)m * b * b, 8.0 * (double)m * b * 4);
    return FLAME_OK;
}

int launch_qr_t(int j0, int j1, const double *G, int64_t ldg, const double *tau, double *T, int64_t ldt,
                const int32_t *info, hipStream_t s) {
    if (j1 <= j0) return FLAME_OK;
    if (j0 < 0 || j1 > kOB) return FLAME_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_qr_t, dim3(1), dim3(kOB), 0, s, j0, j1, G, ldg, tau, T, ldt, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
