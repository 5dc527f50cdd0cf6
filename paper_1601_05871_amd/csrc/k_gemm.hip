// HERK/SYRK (and GEMM) step of the loop body (Fig. "dense-chol"):
//   A22 := A22 - A12^T A12
// in the general form C := C - X^T Y (C M x N, X K x M, Y K x N, every column
// of X and Y contiguous in k).  Diagonal tiles of the upper triangle are the
// HERK of the by-blocks form, the others its GEMM; both are this kernel.
//
// Matrix-core mapping (gfx950, wave64):
//   - a workgroup of 4 wavefronts owns a 128 x 128 tile of C, each wavefront a
//     64 x 64 quarter = 4 x 4 blocks of 16 x 16 MFMA outputs kept in registers;
//   - MFMA A/B operands are read straight from HBM/L2 into registers: lane
//     (r = lane % 16, g = lane / 16) loads 32 contiguous bytes of column r of
//     X (resp. Y) at k offset g * VEC, so one load instruction reads 16 full
//     128-byte column segments.  MFMA step t then uses element t of every
//     lane: both operands assign the same k to the same (g, t) slot, so the
//     contraction is exact whatever the hardware's k order inside a slot;
//   - the next k-chunk is loaded while the current one is multiplied;
//   - the C tile is the accumulator (its column-major 4-row runs match the
//     MFMA output layout: lane holds rows 4g..4g+3 of column r): it is loaded
//     at the start, X is negated, and the tile is written back once.
// Precisions: F64 (v_mfma_f64_16x16x4_f64), F32 (v_mfma_f32_16x16x4_f32) and
// BF16 inputs (v_mfma_f32_16x16x32_bf16), FP32 accumulation for the latter
// two; with an FP64 C the FP32 sum is subtracted in FP64 at the end.
#include "flame_internal.h"
#include "tile_map.h"

namespace flame {

template <Prec P>
struct Tr;
template <>
struct Tr<Prec::F64> {
    using in_t = double;
    using acc_t = d4;
    static constexpr int VEC = 4;  // elements per 32-byte fragment
    static constexpr int NMF = 4;  // MFMAs per fragment
};
template <>
struct Tr<Prec::F32> {
    using in_t = float;
    using acc_t = f4;
    static constexpr int VEC = 8;
    static constexpr int NMF = 8;
};
template <>
struct Tr<Prec::BF16> {
    using in_t = uint16_t;
    using acc_t = f4;
    static constexpr int VEC = 16;
    static constexpr int NMF = 2;
};

union Frag {
    uint4 u[2];
    double d[4];
    float f[8];
    bf16x8 b[2];
};

struct GemmP {
    int64_t M, N, K;
    const void *X;
    int64_t ldx;
    const void *Y;
    int64_t ldy;
    void *C;
    int64_t ldc;
    const int32_t *info;
    int tm, tn;
    int64_t ntiles;
    int upper;
};

// One 32-byte fragment: column `col` of a K x ncols operand, k range
// [k, k + VEC).  Out-of-range columns and k are zero.
template <Prec P, bool VECLD>
__device__ __forceinline__ void load_frag(Frag &f, const typename Tr<P>::in_t *__restrict__ base, int64_t ld,
                                          int64_t col, int64_t ncols, int64_t k, int64_t K) {
    using in_t = typename Tr<P>::in_t;
    constexpr int VEC = Tr<P>::VEC;
    if (col >= ncols) {
        f.u[0] = make_uint4(0, 0, 0, 0);
        f.u[1] = make_uint4(0, 0, 0, 0);
        return;
    }
    const in_t *p = base + col * ld + k;
    if (VECLD && k + VEC <= K) {
        const uint4 *q = reinterpret_cast<const uint4 *>(p);
        f.u[0] = q[0];
        f.u[1] = q[1];
    } else {
        in_t tmp[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) tmp[e] = (k + e < K) ? p[e] : in_t(0);
        __builtin_memcpy(&f, tmp, sizeof(Frag));
    }
}

template <Prec P>
__device__ __forceinline__ void negate(Frag &f) {
    if constexpr (P == Prec::F64) {
#pragma unroll
        for (int e = 0; e < 4; ++e) f.d[e] = -f.d[e];
    } else if constexpr (P == Prec::F32) {
#pragma unroll
        for (int e = 0; e < 8; ++e) f.f[e] = -f.f[e];
    } else {
        f.u[0] ^= make_uint4(0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u);
        f.u[1] ^= make_uint4(0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u);
    }
}

template <Prec P>
__device__ __forceinline__ void mfma_frag(typename Tr<P>::acc_t &acc, const Frag &a, const Frag &b) {
    if constexpr (P == Prec::F64) {
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.d[t], b.d[t], acc, 0, 0, 0);
    } else if constexpr (P == Prec::F32) {
#pragma unroll
        for (int t = 0; t < 8; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.f[t], b.f[t], acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int t = 0; t < 2; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.b[t], b.b[t], acc, 0, 0, 0);
    }
}

// CT: element type of C.  CINIT: the accumulator starts from C (C's type is
// the accumulator's); otherwise it starts at zero and C - sum is formed in CT.
template <Prec P, typename CT, bool VECLD>
__global__ __launch_bounds__(256, 1) void k_gemm_tn(GemmP p) {
    using TR = Tr<P>;
    using in_t = typename TR::in_t;
    using acc_t = typename TR::acc_t;
    constexpr int VEC = TR::VEC;
    constexpr int CK = 4 * VEC;  // k per chunk
    constexpr bool CINIT = (P == Prec::F64 && sizeof(CT) == 8) || (P == Prec::F32 && sizeof(CT) == 4);

    if (p.info != nullptr && *p.info != 0) return;
    const int64_t t = xcd_remap((int64_t)blockIdx.x, p.ntiles);
    int I, J;
    tile_of(t, p.tm, p.tn, p.upper != 0, I, J);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int g = lane >> 4;
    const int64_t row0 = (int64_t)I * kTile + (wave >> 1) * 64;
    const int64_t col0 = (int64_t)J * kTile + (wave & 1) * 64;
    if (row0 >= p.M || col0 >= p.N) return;
    if (p.upper && row0 > col0 + 63) return;  // quarter entirely below the diagonal

    const in_t *__restrict__ X = static_cast<const in_t *>(p.X);
    const in_t *__restrict__ Y = static_cast<const in_t *>(p.Y);
    CT *__restrict__ C = static_cast<CT *>(p.C);
    const int64_t M = p.M, N = p.N, K = p.K, ldc = p.ldc;

    acc_t acc[4][4];
    // accumulator init (C tile, or zero)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0;
            if constexpr (CINIT) {
                const int64_t col = col0 + 16 * b + r;
                const int64_t row = row0 + 16 * a + 4 * g;
                if (col < N) {
                    const CT *cp = C + row + col * ldc;
                    if (VECLD && row + 3 < M) {
                        if constexpr (sizeof(CT) == 8) {
                            const double2 *q = reinterpret_cast<const double2 *>(cp);
                            double2 lo = q[0], hi = q[1];
                            acc[a][b][0] = lo.x;
                            acc[a][b][1] = lo.y;
                            acc[a][b][2] = hi.x;
                            acc[a][b][3] = hi.y;
                        } else {
                            float4 q = *reinterpret_cast<const float4 *>(cp);
                            acc[a][b][0] = q.x;
                            acc[a][b][1] = q.y;
                            acc[a][b][2] = q.z;
                            acc[a][b][3] = q.w;
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (row + v < M) acc[a][b][v] = cp[v];
                    }
                }
            }
        }

    Frag fa[4], fb[4];
    const int64_t kg = (int64_t)g * VEC;
#pragma unroll
    for (int a = 0; a < 4; ++a) load_frag<P, VECLD>(fa[a], X, p.ldx, row0 + 16 * a + r, M, kg, K);
#pragma unroll
    for (int b = 0; b < 4; ++b) load_frag<P, VECLD>(fb[b], Y, p.ldy, col0 + 16 * b + r, N, kg, K);

    for (int64_t k0 = 0; k0 < K; k0 += CK) {
        Frag na[4], nb[4];
        const bool more = k0 + CK < K;
        if (more) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
                load_frag<P, VECLD>(na[a], X, p.ldx, row0 + 16 * a + r, M, k0 + CK + kg, K);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                load_frag<P, VECLD>(nb[b], Y, p.ldy, col0 + 16 * b + r, N, k0 + CK + kg, K);
        }
        if constexpr (CINIT) {
#pragma unroll
            for (int a = 0; a < 4; ++a) negate<P>(fa[a]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) mfma_frag<P>(acc[a][b], fa[a], fb[b]);
        if (more) {
#pragma unroll
            for (int a = 0; a < 4; ++a) fa[a] = na[a];
#pragma unroll
            for (int b = 0; b < 4; ++b) fb[b] = nb[b];
        }
    }

    // write back (upper: only i <= j)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t col = col0 + 16 * b + r;
            const int64_t row = row0 + 16 * a + 4 * g;
            if (col >= N) continue;
            CT *cp = C + row + col * ldc;
            const bool full = (row + 3 < M) && (!p.upper || row + 3 <= col);
            if constexpr (CINIT) {
                if (VECLD && full) {
                    if constexpr (sizeof(CT) == 8) {
                        double2 *q = reinterpret_cast<double2 *>(cp);
                        q[0] = make_double2(acc[a][b][0], acc[a][b][1]);
                        q[1] = make_double2(acc[a][b][2], acc[a][b][3]);
                    } else {
                        *reinterpret_cast<float4 *>(cp) =
                            make_float4(acc[a][b][0], acc[a][b][1], acc[a][b][2], acc[a][b][3]);
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (row + v < M && (!p.upper || row + v <= col)) cp[v] = (CT)acc[a][b][v];
                }
            } else {
                if (VECLD && full) {
                    double2 *q = reinterpret_cast<double2 *>(cp);
                    double2 lo = q[0], hi = q[1];
                    lo.x -= (double)acc[a][b][0];
                    lo.y -= (double)acc[a][b][1];
                    hi.x -= (double)acc[a][b][2];
                    hi.y -= (double)acc[a][b][3];
                    q[0] = lo;
                    q[1] = hi;
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (row + v < M && (!p.upper || row + v <= col)) cp[v] = cp[v] - (CT)acc[a][b][v];
                }
            }
        }
}

template <Prec P, typename CT>
static int launch_t(const GemmP &p, bool vec, hipStream_t s) {
    const unsigned grid = (unsigned)p.ntiles;
    // algorithmic work: 2K flops per updated element; each operand element
    // read once (one panel when X and Y are the same), C read and written
    const double M = (double)p.M, N = (double)p.N, K = (double)p.K;
    const double elems = p.upper ? (M <= N ? M * (M + 1) / 2 + (N - M) * M : N * (N + 1) / 2) : M * N;
    const double esz = P == Prec::F64 ? 8.0 : (P == Prec::F32 ? 4.0 : 2.0);
    const double panel = (p.X == p.Y && p.M == p.N) ? K * M : K * (M + N);
    const int tr = trace_begin(FLAME_KC_GEMM, s);
    if (vec)
        hipLaunchKernelGGL((k_gemm_tn<P, CT, true>), dim3(grid), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL((k_gemm_tn<P, CT, false>), dim3(grid), dim3(256), 0, s, p);
    FLAME_CHECK_LAUNCH();
    trace_end(tr, s, 2.0 * K * elems, panel * esz + 2.0 * elems * (double)sizeof(CT));
    return FLAME_OK;
}

static bool aligned16(const void *q) { return ((uintptr_t)q & 15u) == 0; }

int launch_gemm_tn(Prec prec, bool c_is_double, bool upper, int64_t M, int64_t N, int64_t K, const void *X,
                   int64_t ldx, const void *Y, int64_t ldy, void *C, int64_t ldc, const int32_t *info,
                   hipStream_t s) {
    if (M <= 0 || N <= 0) return FLAME_OK;
    GemmP p;
    p.M = M;
    p.N = N;
    p.K = K;
    p.X = X;
    p.ldx = ldx;
    p.Y = Y;
    p.ldy = ldy;
    p.C = C;
    p.ldc = ldc;
    p.info = info;
    p.tm = (int)((M + kTile - 1) / kTile);
    p.tn = (int)((N + kTile - 1) / kTile);
    p.upper = upper ? 1 : 0;
    p.ntiles = tile_count(p.tm, p.tn, upper);
    if (p.ntiles <= 0) return FLAME_OK;
    const size_t esz = prec == Prec::F64 ? 8 : (prec == Prec::F32 ? 4 : 2);
    const int64_t vec_elems = 16 / (int64_t)esz;
    const size_t csz = c_is_double ? 8 : 4;
    const bool vec = aligned16(X) && aligned16(Y) && aligned16(C) && (ldx % vec_elems == 0) &&
                     (ldy % vec_elems == 0) && ((ldc * (int64_t)csz) % 16 == 0);
    switch (prec) {
        case Prec::F64:
            return launch_t<Prec::F64, double>(p, vec, s);
        case Prec::F32:
            return c_is_double ? launch_t<Prec::F32, double>(p, vec, s) : launch_t<Prec::F32, float>(p, vec, s);
        case Prec::BF16:
            return launch_t<Prec::BF16, double>(p, vec, s);
    }
    return FLAME_ERR_UNSUPPORTED;
}

// ---- low-precision copy of the panel ------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <Prec P>
__global__ void k_round_panel(int64_t rows, int64_t cols, const double *__restrict__ X, int64_t ldx,
                              void *__restrict__ Yv, int64_t ldy, const int32_t *__restrict__ info) {
    if (info != nullptr && *info != 0) return;
    const int64_t c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ldy; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (i < rows) ? X[i + c * ldx] : 0.0;  // pad rows up to ldy with zeros
        if constexpr (P == Prec::F32) {
            static_cast<float *>(Yv)[i + c * ldy] = (float)v;
        } else {
            static_cast<uint16_t *>(Yv)[i + c * ldy] = f32_to_bf16_rne((float)v);
        }
    }
}

int launch_round_panel(Prec p, int64_t rows, int64_t cols, const double *X, int64_t ldx, void *Y, int64_t ldy,
                       const int32_t *info, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return FLAME_OK;
    const unsigned gx = (unsigned)((ldy + 255) / 256);
    if (p == Prec::F32)
        hipLaunchKernelGGL(k_round_panel<Prec::F32>, dim3(gx, (unsigned)cols), dim3(256), 0, s, rows, cols, X, ldx,
                           Y, ldy, info);
    else
        hipLaunchKernelGGL(k_round_panel<Prec::BF16>, dim3(gx, (unsigned)cols), dim3(256), 0, s, rows, cols, X,
                           ldx, Y, ldy, info);
    FLAME_CHECK_LAUNCH();
    return FLAME_OK;
}

}  // namespace flame
