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
//   - the C tile is the accumulator: it is loaded at the start, X is negated,
//     and the tile is written back once (mfma_frag gives the element each
//     accumulator item holds; 16 lanes always cover 64 or 128 contiguous
//     bytes of one column of C).
// Precisions: F64 (v_mfma_f64_16x16x4_f64), F32 (v_mfma_f32_16x16x4_f32) and
// BF16 inputs (v_mfma_f32_16x16x32_bf16), FP32 accumulation for the latter
// two; with an FP64 C the FP32 sum is subtracted in FP64 at the end.
#include <algorithm>

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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

union Frag {
    u32x4 u[2];
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
    // split-K (k_gemm_lds only): nslices > 1 runs ntiles * nslices workgroups;
    // slice s covers k in [s kslice, min(K, (s + 1) kslice)) and writes
    // -X_s^T Y_s to W + s ldw N (nothing is read from C)
    int nslices;
    int64_t kslice;
    void *W;
    int64_t ldw;
    // compute units to leave free for concurrent kernels (0 = none).  With a
    // reservation k_gemm_lds launches 2 workgroups per remaining CU and each
    // walks work items blockIdx.x, + gridDim.x, ... (tiles x slices);
    // k_gemm_p8 launches one per remaining CU.
    int reserve_cus;
};

// One 32-byte fragment of a K x ncols operand: column `col` (already clamped
// to a valid column), k range [k, k + VEC) entirely inside [0, K).  No
// branches, so the compiler can keep many of these loads in flight.
template <Prec P, bool VECLD>
__device__ __forceinline__ void load_frag(Frag &f, const typename Tr<P>::in_t *__restrict__ base, int64_t ld,
                                          int64_t col, int64_t k) {
    using in_t = typename Tr<P>::in_t;
    constexpr int VEC = Tr<P>::VEC;
    const in_t *p = base + col * ld + k;
    if constexpr (VECLD) {
        const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
        f.u[0] = q[0];
        f.u[1] = q[1];
    } else {
        in_t tmp[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) tmp[e] = p[e];
        __builtin_memcpy(&f, tmp, sizeof(Frag));
    }
}

// The same for the last, partial k chunk: elements at k + e >= K are zero
// (their address is clamped to k = K - 1 and the value discarded).
template <Prec P>
__device__ __forceinline__ void load_frag_tail(Frag &f, const typename Tr<P>::in_t *__restrict__ base, int64_t ld,
                                               int64_t col, int64_t k, int64_t K) {
    using in_t = typename Tr<P>::in_t;
    constexpr int VEC = Tr<P>::VEC;
    const in_t *p = base + col * ld;
    in_t tmp[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int64_t kk = k + e;
        const in_t v = p[kk < K ? kk : K - 1];
        tmp[e] = (kk < K) ? v : in_t(0);
    }
    __builtin_memcpy(&f, tmp, sizeof(Frag));
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
        f.u[0] ^= u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
        f.u[1] ^= u32x4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    }
}

// acc += (fragment of X)^T (fragment of Y) over the fragment's k range.
// FP64: the 16x16x4 FP64 MFMA returns D[g + 4v][r] in lane r + 16g, item v,
// so Y is passed as the row operand and X as the column operand: lane
// (r, g) then holds (X^T Y)(row r, column g + 4v) of the 16 x 16 block, and
// 16 lanes with the same g cover 16 consecutive rows of one column of C.
// FP32 / BF16 MFMAs return D[4g + v][r]: X is the row operand and lane (r, g)
// holds (X^T Y)(row 4g + v, column r), four consecutive rows of one column.
template <Prec P>
__device__ __forceinline__ void mfma_frag(typename Tr<P>::acc_t &acc, const Frag &a, const Frag &b) {
    if constexpr (P == Prec::F64) {
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(b.d[t], a.d[t], acc, 0, 0, 0);
    } else if constexpr (P == Prec::F32) {
#pragma unroll
        for (int t = 0; t < 8; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.f[t], b.f[t], acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int t = 0; t < 2; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.b[t], b.b[t], acc, 0, 0, 0);
    }
}

// The same for one 16-byte half h of the fragments (the first or second half
// of the fragment's k range).
template <Prec P>
__device__ __forceinline__ void mfma_half(typename Tr<P>::acc_t &acc, const u32x4 &a, const u32x4 &b) {
    if constexpr (P == Prec::F64) {
        typedef double d2v __attribute__((ext_vector_type(2)));
        const d2v x = __builtin_bit_cast(d2v, a), y = __builtin_bit_cast(d2v, b);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(y[0], x[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(y[1], x[1], acc, 0, 0, 0);
    } else if constexpr (P == Prec::F32) {
        const f4 x = __builtin_bit_cast(f4, a), y = __builtin_bit_cast(f4, b);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x[t], y[t], acc, 0, 0, 0);
    } else {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                      acc, 0, 0, 0);
    }
}

__device__ __forceinline__ u32x4 negate_half(Prec P, u32x4 v) {
    if (P == Prec::F64) return v ^ u32x4{0u, 0x80000000u, 0u, 0x80000000u};
    return v ^ u32x4{0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u};
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

    // C element of accumulator item v of block (a, b) of this lane (see mfma_frag)
    auto crow = [&](int a, int v) -> int64_t {
        return (P == Prec::F64) ? row0 + 16 * a + r : row0 + 16 * a + 4 * g + v;
    };
    auto ccol = [&](int b, int v) -> int64_t {
        return (P == Prec::F64) ? col0 + 16 * b + g + 4 * v : col0 + 16 * b + r;
    };
    constexpr bool ROWRUN = (P != Prec::F64);  // items v are 4 consecutive rows

    acc_t acc[4][4];
    // accumulator init: the C tile (or zero).  Loads are unconditional from
    // clamped addresses; entries outside C are never stored.
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] = 0;
            if constexpr (CINIT) {
                if constexpr (ROWRUN) {
                    const int64_t col = min(ccol(b, 0), N - 1);
                    const int64_t row = crow(a, 0);
                    if (VECLD && row + 3 < M) {
                        float4 q = *reinterpret_cast<const float4 *>(C + row + col * ldc);
                        acc[a][b][0] = q.x;
                        acc[a][b][1] = q.y;
                        acc[a][b][2] = q.z;
                        acc[a][b][3] = q.w;
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[a][b][v] = C[min(row + v, M - 1) + col * ldc];
                    }
                } else {
                    const int64_t row = min(crow(a, 0), M - 1);
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[a][b][v] = C[row + min(ccol(b, v), N - 1) * ldc];
                }
            }
        }

    // operand columns, clamped into range: an out-of-range column only feeds
    // rows >= M or columns >= N of the product, which are never stored
    int64_t xcol[4], ycol[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) xcol[a] = min(row0 + 16 * a + r, M - 1);
#pragma unroll
    for (int b = 0; b < 4; ++b) ycol[b] = min(col0 + 16 * b + r, N - 1);
    const int64_t kg = (int64_t)g * VEC;
    const int64_t nfull = K / CK;

    auto load_chunk = [&](Frag(&fx)[4], Frag(&fy)[4], int64_t k0) {
#pragma unroll
        for (int a = 0; a < 4; ++a) load_frag<P, VECLD>(fx[a], X, p.ldx, xcol[a], k0 + kg);
#pragma unroll
        for (int b = 0; b < 4; ++b) load_frag<P, VECLD>(fy[b], Y, p.ldy, ycol[b], k0 + kg);
    };
    auto compute = [&](Frag(&fx)[4], Frag(&fy)[4]) {
        if constexpr (CINIT) {
#pragma unroll
            for (int a = 0; a < 4; ++a) negate<P>(fx[a]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) mfma_frag<P>(acc[a][b], fx[a], fy[b]);
    };

    // software pipeline with two register buffers used in turn (no copies,
    // so the loads of the next chunk stay in flight while this one multiplies)
    Frag fa[4], fb[4], ga[4], gb[4];
    if (nfull > 0) {
        load_chunk(fa, fb, 0);
        int64_t c = 0;
        for (; c + 2 < nfull; c += 2) {
            load_chunk(ga, gb, (c + 1) * CK);
            compute(fa, fb);
            load_chunk(fa, fb, (c + 2) * CK);
            compute(ga, gb);
        }
        if (c + 1 < nfull) {
            load_chunk(ga, gb, (c + 1) * CK);
            compute(fa, fb);
            compute(ga, gb);
        } else {
            compute(fa, fb);
        }
    }
    if (nfull * CK < K) {
        const int64_t k0 = nfull * CK + kg;
#pragma unroll
        for (int a = 0; a < 4; ++a) load_frag_tail<P>(fa[a], X, p.ldx, xcol[a], k0, K);
#pragma unroll
        for (int b = 0; b < 4; ++b) load_frag_tail<P>(fb[b], Y, p.ldy, ycol[b], k0, K);
        compute(fa, fb);
    }

    // write back (upper: only i <= j); the quarter is interior when all its
    // elements are stored
    const bool interior = (row0 + 64 <= M) && (col0 + 64 <= N) && (!p.upper || row0 + 63 <= col0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if constexpr (ROWRUN) {
                const int64_t col = ccol(b, 0), row = crow(a, 0);
                if (col >= N) continue;
                CT *cp = C + row + col * ldc;
                const bool full = (row + 3 < M) && (!p.upper || row + 3 <= col);
                if constexpr (CINIT) {
                    if (VECLD && full) {
                        *reinterpret_cast<float4 *>(cp) =
                            make_float4(acc[a][b][0], acc[a][b][1], acc[a][b][2], acc[a][b][3]);
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
            } else {
                const int64_t row = crow(a, 0);
                if (interior) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) C[row + ccol(b, v) * ldc] = (CT)acc[a][b][v];
                } else if (row < M) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t col = ccol(b, v);
                        if (col < N && (!p.upper || row <= col)) C[row + col * ldc] = (CT)acc[a][b][v];
                    }
                }
            }
        }
}

// ---- LDS-staged variant (K a multiple of the chunk, 16-byte aligned) ------
// Per k-chunk the workgroup stages the 128 columns of X and of Y it needs
// (128 bytes of each column: 16 FP64, 32 FP32 or 64 BF16 values) in LDS, so
// each operand element is read from L2 once per workgroup instead of once per
// wavefront.  The copies go from global memory straight into LDS
// (global_load_lds_dwordx4: 16 bytes per lane, no registers in between), and
// those of chunk c + 1 overlap the MFMAs of chunk c (two LDS buffers, one
// barrier per chunk).  Each column's eight 16-byte units are stored
// XOR-swizzled by (column mod 8) so that the 16 lanes reading one unit of 16
// consecutive columns hit different banks.  (Against copies staged through
// registers: n = 16384 FP64 factorization 32.0 -> 30.6 ms; the 32 registers
// the staging held had left the fragment reads of each chunk one at a time.)

// 16 bytes per lane from global memory straight into LDS: lane l's bytes land
// at lds + 16 l (lds wavefront-uniform).
__device__ __forceinline__ void copy16_to_lds(const char *g, char *lds) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}

__device__ __forceinline__ int slab_off(int col, int unit) { return col * 128 + ((unit ^ (col & 7)) << 4); }

// TM: tile order, 128 (wavefront blocks of 64 x 64) or 64 (32 x 32: four
// times the workgroups for launches with few tiles, a quarter of the serial
// MFMA chain per tile).
template <Prec P, typename CT, int TM>
__global__ __launch_bounds__(256, 2) void k_gemm_lds(GemmP p) {
    using TR = Tr<P>;
    using in_t = typename TR::in_t;
    using acc_t = typename TR::acc_t;
    constexpr int VEC = TR::VEC;
    constexpr int CK = 4 * VEC;  // k per chunk (128 bytes of a column)
    constexpr int WT = TM / 2;   // a wavefront's block of the tile: WT x WT
    constexpr int WB = WT / 16;  // 16 x 16 MFMA blocks per wavefront side
    constexpr int NJ = TM / 32;  // operand columns copied per thread and chunk
    static_assert(TM == 128 || TM == 64, "tile order");
    __shared__ __attribute__((aligned(16))) char lds[2][2][TM * 128];  // [buffer][X or Y]

    if (p.info != nullptr && *p.info != 0) return;
    const bool split = p.nslices > 1;
    const int64_t items = p.ntiles * (split ? p.nslices : 1);
    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
    int64_t bid = item;
    int64_t kbeg = 0;
    if (split) {
        const int64_t slice = bid / p.ntiles;
        bid -= slice * p.ntiles;
        kbeg = slice * p.kslice;
    }
    const int64_t t = xcd_remap(bid, p.ntiles);
    int I, J;
    tile_of(t, p.tm, p.tn, p.upper != 0, I, J);
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15;
    const int g = lane >> 4;
    const int64_t tr0 = (int64_t)I * TM, tc0 = (int64_t)J * TM;
    const int64_t row0 = tr0 + (wave >> 1) * WT;
    const int64_t col0 = tc0 + (wave & 1) * WT;
    const int64_t M = p.M, N = p.N;
    const int64_t K = split ? min(p.kslice, p.K - kbeg) : p.K;
    const int64_t ldc = split ? p.ldw : p.ldc;
    const bool active = (row0 < M) && (col0 < N) && !(p.upper && row0 > col0 + WT - 1);
    const char *__restrict__ Xb = static_cast<const char *>(p.X) + kbeg * (int64_t)sizeof(in_t);
    const char *__restrict__ Yb = static_cast<const char *>(p.Y) + kbeg * (int64_t)sizeof(in_t);
    const int64_t ldxb = p.ldx * (int64_t)sizeof(in_t), ldyb = p.ldy * (int64_t)sizeof(in_t);

    // copy assignment: wavefront w copies columns 8 w + 32 j .. 8 w + 32 j + 7
    // (j < NJ) of each operand, 1 KB per copy instruction; lane l's 16 bytes
    // land in slot l % 8 of column 8 w + 32 j + l / 8, so the lane fetches the
    // unit that the swizzle puts there: unit (l % 8) ^ (l / 8).
    const int unit = (tid & 7) ^ ((tid >> 3) & 7);
    const int ccol0 = tid >> 3;
    const int64_t chunk_bytes = CK * (int64_t)sizeof(in_t);  // 128
    const int64_t nch = K / CK;
    // byte offsets (from Xb / Yb) of this lane's NJ units of each operand
    int64_t xoff[NJ], yoff[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int col = ccol0 + 32 * j;
        xoff[j] = min(tr0 + col, M - 1) * ldxb + unit * 16;
        yoff[j] = min(tc0 + col, N - 1) * ldyb + unit * 16;
    }

    // C element of accumulator item v of block (a, b) (see mfma_frag)
#define FLAME_CROW(a, v) ((P == Prec::F64) ? row0 + 16 * (a) + r : row0 + 16 * (a) + 4 * g + (v))
#define FLAME_CCOL(b, v) ((P == Prec::F64) ? col0 + 16 * (b) + g + 4 * (v) : col0 + 16 * (b) + r)
    // CINIT: the accumulator starts from the C tile (same precision) and X is
    // negated; otherwise it starts at zero and C - X^T Y is formed at the end.
    constexpr bool CINIT = (P == Prec::F64 && sizeof(CT) == 8) || (P == Prec::F32 && sizeof(CT) == 4);
    CT *__restrict__ C = split ? static_cast<CT *>(p.W) + (kbeg / p.kslice) * p.ldw * N : static_cast<CT *>(p.C);
    acc_t acc[WB][WB];
    // one uniform branch around the whole (unconditional, clamped) tile load
    if (CINIT && !split) {
#pragma unroll
        for (int a = 0; a < WB; ++a)
#pragma unroll
            for (int b = 0; b < WB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[a][b][v] = C[min(FLAME_CROW(a, v), M - 1) + min(FLAME_CCOL(b, v), N - 1) * ldc];
    } else {
#pragma unroll
        for (int a = 0; a < WB; ++a)
#pragma unroll
            for (int b = 0; b < WB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[a][b][v] = 0;
    }

    const int xr = (wave >> 1) * WT + r, yr = (wave & 1) * WT + r;

// One chunk from LDS buffer `buf`: the two 16-byte halves of each lane's
// fragments are read and multiplied in turn (half the operand registers).
#define FLAME_COMPUTE(buf)                                                                            \
    {                                                                                                 \
        const char *xs_ = &lds[buf][0][0];                                                            \
        const char *ys_ = &lds[buf][1][0];                                                            \
        _Pragma("unroll") for (int h = 0; h < 2; ++h) {                                               \
            u32x4 fa_[WB], fb_[WB];                                                                   \
            _Pragma("unroll") for (int a = 0; a < WB; ++a) {                                          \
                fa_[a] = *reinterpret_cast<const u32x4 *>(xs_ + slab_off(xr + 16 * a, 2 * g + h));    \
                if constexpr (CINIT) fa_[a] = negate_half(P, fa_[a]);                                 \
            }                                                                                         \
            _Pragma("unroll") for (int b = 0; b < WB; ++b)                                            \
                fb_[b] = *reinterpret_cast<const u32x4 *>(ys_ + slab_off(yr + 16 * b, 2 * g + h));    \
            _Pragma("unroll") for (int a = 0; a < WB; ++a)                                            \
                _Pragma("unroll") for (int b = 0; b < WB; ++b) mfma_half<P>(acc[a][b], fa_[a], fb_[b]); \
        }                                                                                             \
    }

    // the wait for this wavefront's copies of chunk c + 1 and the barrier
    // come after the MFMAs of chunk c; the copies are unconditional (an
    // inactive wavefront's product is discarded)
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
#define FLAME_COPY(cidx, buf)                                                                             \
    {                                                                                                     \
        _Pragma("unroll") for (int j_ = 0; j_ < NJ; ++j_) {                                               \
            copy16_to_lds(Xb + xoff[j_] + (cidx) * chunk_bytes, &lds[buf][0][0] + (8 * wv + 32 * j_) * 128); \
            copy16_to_lds(Yb + yoff[j_] + (cidx) * chunk_bytes, &lds[buf][1][0] + (8 * wv + 32 * j_) * 128); \
        }                                                                                                 \
    }
    FLAME_COPY(0, 0)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    int64_t c = 0;
    for (; c + 1 < nch; ++c) {
        FLAME_COPY(c + 1, (int)((c + 1) & 1))
        FLAME_COMPUTE((int)(c & 1))
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
#undef FLAME_COPY

    FLAME_COMPUTE((int)(c & 1))
    if (active) {
        const bool interior = (row0 + WT <= M) && (col0 + WT <= N) && (!p.upper || row0 + WT - 1 <= col0);
#pragma unroll
        for (int a = 0; a < WB; ++a)
#pragma unroll
            for (int b = 0; b < WB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = FLAME_CROW(a, v), col = FLAME_CCOL(b, v);
                    if (interior || (row < M && col < N && (!p.upper || row <= col))) {
                        CT *cp = C + row + col * ldc;
                        if constexpr (CINIT)
                            *cp = (CT)acc[a][b][v];
                        else
                            *cp = *cp - (CT)acc[a][b][v];
                    }
                }
    }
#undef FLAME_COMPUTE
#undef FLAME_CROW
#undef FLAME_CCOL
    __syncthreads();  // the LDS buffers are refilled by the next item
    }
}

// ---- 8-wavefront persistent LDS-staged variant --------------------------------
// One workgroup of eight wavefronts per CU (two per SIMD, so the FP64 MFMA
// pipe always has a second wavefront to issue from), each wavefront a 64 x 32
// part of the 128 x 128 tile (wave grid 2 x 4).  The k-chunk is 256 bytes per
// column (32 FP64 / 64 FP32 / 128 BF16 values) and the two LDS buffers take
// 128 KiB; 16-byte units are XOR-swizzled by (column mod 16).  The workgroup
// is persistent: it walks tiles L, L + G, ... (G workgroups, L its
// XCD-remapped index, so that the 32 workgroups of an XCD work on 32
// consecutive tiles of the band order) and overlaps each tile's last chunk
// with the loads of the next tile's first chunk and C tile, so no tile
// prologue or epilogue is exposed.
constexpr int kSlab8Bytes = kTile * 256;
constexpr int64_t kPersistentWgs = 256;  // one per CU

__device__ __forceinline__ int slab8_off(int col, int unit) { return col * 256 + ((unit ^ (col & 15)) << 4); }

template <Prec P, typename CT>
__global__ __launch_bounds__(512, 1) void k_gemm_p8(GemmP p) {
    using TR = Tr<P>;
    using in_t = typename TR::in_t;
    using acc_t = typename TR::acc_t;
    constexpr int CK = 256 / (int)sizeof(in_t);  // k per chunk
    constexpr bool CINIT = (P == Prec::F64 && sizeof(CT) == 8) || (P == Prec::F32 && sizeof(CT) == 4);
    __shared__ __attribute__((aligned(16))) char lds[2][2][kSlab8Bytes];

    if (p.info != nullptr && *p.info != 0) return;
    const int64_t G = gridDim.x;
    int64_t tile = xcd_remap((int64_t)blockIdx.x, G);
    if (tile >= p.ntiles) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int r = lane & 15;
    const int g = lane >> 4;
    const int wr = wave >> 2, wc = wave & 3;  // 2 x 4 wave grid
    const int64_t M = p.M, N = p.N, K = p.K, ldc = p.ldc;
    const char *__restrict__ Xb = static_cast<const char *>(p.X);
    const char *__restrict__ Yb = static_cast<const char *>(p.Y);
    const int64_t ldxb = p.ldx * (int64_t)sizeof(in_t), ldyb = p.ldy * (int64_t)sizeof(in_t);
    CT *__restrict__ C = static_cast<CT *>(p.C);
    const int64_t nch = K / CK;
    constexpr int64_t chunk_bytes = 256;
    // copy assignment: unit q = tid + 512 j (j < 8) of the 2 x 2048 units of a
    // chunk: operand j / 4, column tid / 16 + 32 (j % 4), unit tid % 16
    const int unit = tid & 15;
    const int ccol0 = tid >> 4;
    int dofs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) dofs[j] = slab8_off(ccol0 + 32 * j, unit);
    const int xr = wr * 64 + r, yr = wc * 32 + r;

    // per-tile state
    int64_t tr0, tc0, row0, col0;
    int64_t xoff[4], yoff[4];
    auto set_tile = [&](int64_t tt) {
        int I, J;
        tile_of(tt, p.tm, p.tn, p.upper != 0, I, J);
        tr0 = (int64_t)I * kTile;
        tc0 = (int64_t)J * kTile;
        row0 = tr0 + wr * 64;
        col0 = tc0 + wc * 32;
    };
    auto set_offsets = [&]() {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = ccol0 + 32 * j;
            xoff[j] = min(tr0 + col, M - 1) * ldxb + unit * 16;
            yoff[j] = min(tc0 + col, N - 1) * ldyb + unit * 16;
        }
    };

#define FLAME_CROW(a, v) ((P == Prec::F64) ? row0 + 16 * (a) + r : row0 + 16 * (a) + 4 * g + (v))
#define FLAME_CCOL(b, v) ((P == Prec::F64) ? col0 + 16 * (b) + g + 4 * (v) : col0 + 16 * (b) + r)
#define FLAME_LOADC()                                                                                 \
    _Pragma("unroll") for (int a = 0; a < 4; ++a) _Pragma("unroll") for (int b = 0; b < 2; ++b)      \
        _Pragma("unroll") for (int v = 0; v < 4; ++v) cpre[a][b][v] =                                 \
            C[min(FLAME_CROW(a, v), M - 1) + min(FLAME_CCOL(b, v), N - 1) * ldc];
#define FLAME_FETCH1(j, cidx)                                                                         \
    stx[j] = *reinterpret_cast<const u32x4 *>(Xb + xoff[j] + (cidx) * chunk_bytes);                   \
    sty[j] = *reinterpret_cast<const u32x4 *>(Yb + yoff[j] + (cidx) * chunk_bytes);
#define FLAME_FETCH(cidx)                                                                             \
    {                                                                                                 \
        FLAME_FETCH1(0, cidx) FLAME_FETCH1(1, cidx) FLAME_FETCH1(2, cidx) FLAME_FETCH1(3, cidx)       \
    }
#define FLAME_PUT1(j, buf)                                                                            \
    *reinterpret_cast<u32x4 *>(&lds[buf][0][0] + dofs[j]) = stx[j];                                   \
    *reinterpret_cast<u32x4 *>(&lds[buf][1][0] + dofs[j]) = sty[j];
#define FLAME_PUT(buf)                                                                                \
    {                                                                                                 \
        FLAME_PUT1(0, buf) FLAME_PUT1(1, buf) FLAME_PUT1(2, buf) FLAME_PUT1(3, buf)                   \
    }
// lane (r, g) covers 16-byte units 4g .. 4g + 3 of each column, read and
// multiplied one unit at a time
#define FLAME_COMPUTE(buf)                                                                            \
    {                                                                                                 \
        const char *xs_ = &lds[buf][0][0];                                                            \
        const char *ys_ = &lds[buf][1][0];                                                            \
        _Pragma("unroll") for (int h = 0; h < 4; ++h) {                                               \
            u32x4 fa_[4], fb_[2];                                                                     \
            _Pragma("unroll") for (int a = 0; a < 4; ++a) {                                           \
                fa_[a] = *reinterpret_cast<const u32x4 *>(xs_ + slab8_off(xr + 16 * a, 4 * g + h));   \
                if constexpr (CINIT) fa_[a] = negate_half(P, fa_[a]);                                 \
            }                                                                                         \
            _Pragma("unroll") for (int b = 0; b < 2; ++b)                                             \
                fb_[b] = *reinterpret_cast<const u32x4 *>(ys_ + slab8_off(yr + 16 * b, 4 * g + h));   \
            _Pragma("unroll") for (int a = 0; a < 4; ++a)                                             \
                _Pragma("unroll") for (int b = 0; b < 2; ++b) mfma_half<P>(acc[a][b], fa_[a], fb_[b]); \
        }                                                                                             \
    }

    CT cpre[4][2][4];  // CINIT: the next tile's C; otherwise this tile's C
    acc_t acc[4][2];
    u32x4 stx[4], sty[4];

    set_tile(tile);
    set_offsets();
    if constexpr (CINIT) {
        FLAME_LOADC()
    }
    FLAME_FETCH(0)
    FLAME_PUT(0)
    __syncthreads();
    int buf = 0;
    for (;;) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[a][b][v] = CINIT ? cpre[a][b][v] : 0;
        const int64_t next = tile + G;
        const bool has_next = next < p.ntiles;
        const int64_t crow0 = row0, ccol0t = col0;
        for (int64_t c = 0; c < nch; ++c) {
            const bool last = (c + 1 == nch);
            if (!last) {
                FLAME_FETCH(c + 1)
            } else {
                if constexpr (!CINIT) {
                    FLAME_LOADC()  // this tile's C, for the epilogue
                }
                if (has_next) {
                    set_tile(next);
                    set_offsets();
                    FLAME_FETCH(0)
                    if constexpr (CINIT) {
                        FLAME_LOADC()  // the next tile's C, its accumulator start
                    }
                }
            }
            FLAME_COMPUTE(buf)
            __builtin_amdgcn_sched_barrier(0);
            if (!last || has_next) {
                FLAME_PUT(buf ^ 1)
            }
            __syncthreads();
            buf ^= 1;
        }
        // epilogue of the tile just finished (its row0 / col0 were saved)
        {
            const int64_t rw0 = crow0, cl0 = ccol0t;
            const bool active = (rw0 < M) && (cl0 < N) && !(p.upper && rw0 > cl0 + 31);
            if (active) {
                const bool interior = (rw0 + 64 <= M) && (cl0 + 32 <= N) && (!p.upper || rw0 + 63 <= cl0);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int64_t row = (P == Prec::F64) ? rw0 + 16 * a + r : rw0 + 16 * a + 4 * g + v;
                            const int64_t col = (P == Prec::F64) ? cl0 + 16 * b + g + 4 * v : cl0 + 16 * b + r;
                            if (interior || (row < M && col < N && (!p.upper || row <= col))) {
                                if constexpr (CINIT)
                                    C[row + col * ldc] = (CT)acc[a][b][v];
                                else
                                    C[row + col * ldc] = cpre[a][b][v] - (CT)acc[a][b][v];
                            }
                        }
            }
        }
        if (!has_next) break;
        tile = next;
    }
#undef FLAME_FETCH
#undef FLAME_FETCH1
#undef FLAME_PUT
#undef FLAME_PUT1
#undef FLAME_COMPUTE
#undef FLAME_LOADC
#undef FLAME_CROW
#undef FLAME_CCOL
}

// Launches with at most this many 128-tiles (about one per CU; no CU
// reservation, no split) run on 64-tiles: the products inside the 256- and
// 512-wide CHOL and TRSM steps and the panel-row updates of the tail
// (n = 16384: 35.5 -> 33.0 ms; at 512 and above the large panel-row updates
// lose more than the small ones gain: 38.7 ms)
#ifndef FLAME_SMALL_TILES
#define FLAME_SMALL_TILES 256
#endif
constexpr int64_t kSmallTiles = FLAME_SMALL_TILES;

template <Prec P, typename CT>
static int launch_t(const GemmP &p, bool vec, hipStream_t s) {
    constexpr int64_t CK = 4 * Tr<P>::VEC;
    constexpr int64_t CK8 = 2 * CK;
    // FP64 runs best as two 4-wavefront workgroups per CU (k_gemm_lds); the
    // FP32 / BF16 products alone as one persistent 8-wavefront workgroup
    // (k_gemm_p8).  Beside the CHOL/TRSM chain (a CU reservation) they also
    // take k_gemm_lds: k_gemm_p8 fills whole CUs and leaves the chain's panel
    // TRSM only the reserved ones
    const bool lds8_ok = P != Prec::F64 && p.reserve_cus == 0 && vec && p.K > 0 && (p.K % CK8) == 0;
    const bool lds_ok = vec && p.K > 0 && (p.K % CK) == 0;
    // algorithmic work: 2K flops per updated element; each operand element
    // read once (one panel when X and Y are the same), C read and written
    const double M = (double)p.M, N = (double)p.N, K = (double)p.K;
    const double elems = p.upper ? (M <= N ? M * (M + 1) / 2 + (N - M) * M : N * (N + 1) / 2) : M * N;
    const double esz = P == Prec::F64 ? 8.0 : (P == Prec::F32 ? 4.0 : 2.0);
    const double panel = (p.X == p.Y && p.M == p.N) ? K * M : K * (M + N);
    int64_t cus_left = kPersistentWgs;
    if (p.reserve_cus > 0) {
        static int cus_cache[64] = {};
        int dev = 0;
        FLAME_HIP(hipGetDevice(&dev));
        int cus = dev < 64 ? cus_cache[dev] : 0;
        if (cus == 0) {
            FLAME_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            if (dev < 64) cus_cache[dev] = cus;
        }
        // a multiple of the 8 XCDs, so that the persistent walk keeps each
        // workgroup on its XCD's contiguous tiles
        cus_left = std::max<int64_t>(8, (cus - p.reserve_cus) / 8 * 8);
    }
    const int tr = trace_begin(FLAME_KC_GEMM, s);
    if (lds8_ok)
        hipLaunchKernelGGL((k_gemm_p8<P, CT>), dim3((unsigned)std::min<int64_t>(p.ntiles, cus_left)), dim3(512), 0, s,
                           p);
    else if (lds_ok && p.reserve_cus == 0 && p.nslices <= 1 && p.ntiles <= kSmallTiles) {
        // few 128-tiles: 64-tiles, four times the workgroups
        GemmP q = p;
        q.tm = (int)((p.M + 63) / 64);
        q.tn = (int)((p.N + 63) / 64);
        q.ntiles = tile_count(q.tm, q.tn, p.upper != 0);
        hipLaunchKernelGGL((k_gemm_lds<P, CT, 64>), dim3((unsigned)q.ntiles), dim3(256), 0, s, q);
    } else if (lds_ok)
        hipLaunchKernelGGL((k_gemm_lds<P, CT, 128>),
                           dim3((unsigned)(p.reserve_cus > 0 ? std::min<int64_t>(p.ntiles, 2 * cus_left) : p.ntiles)),
                           dim3(256), 0, s, p);
    else if (vec)
        hipLaunchKernelGGL((k_gemm_tn<P, CT, true>), dim3((unsigned)p.ntiles), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL((k_gemm_tn<P, CT, false>), dim3((unsigned)p.ntiles), dim3(256), 0, s, p);
    FLAME_CHECK_LAUNCH();
    trace_end(tr, s, 2.0 * K * elems, panel * esz + 2.0 * elems * (double)sizeof(CT));
    return FLAME_OK;
}

static bool aligned16(const void *q) { return ((uintptr_t)q & 15u) == 0; }

int launch_gemm_tn(Prec prec, bool c_is_double, bool upper, int64_t M, int64_t N, int64_t K, const void *X,
                   int64_t ldx, const void *Y, int64_t ldy, void *C, int64_t ldc, const int32_t *info, hipStream_t s,
                   int reserve_cus) {
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
    p.nslices = 1;
    p.kslice = K;
    p.W = nullptr;
    p.ldw = 0;
    p.reserve_cus = reserve_cus;
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

// ---- split-K for the tall-K products of the left-looking and bordered loops --
template <typename CT>
__global__ void k_splitk_reduce(int64_t M, int64_t N, int upper, const CT *__restrict__ W, int64_t ldw, int S,
                                CT *__restrict__ C, int64_t ldc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= M || (upper && i > j)) return;
    CT acc = C[i + j * ldc];
    for (int s = 0; s < S; ++s) acc += W[i + j * ldw + (int64_t)s * ldw * N];  // fixed order
    C[i + j * ldc] = acc;
}

int splitk_slices(bool upper, int64_t M, int64_t N, int64_t K, int64_t *kslice) {
    constexpr int64_t kTargetWgs = 1024, kMinSliceK = 256;
    const int tm = (int)((M + kTile - 1) / kTile), tn = (int)((N + kTile - 1) / kTile);
    const int64_t tiles = tile_count(tm, tn, upper);
    if (tiles <= 0) return 1;
    int64_t S = std::min((kTargetWgs + tiles - 1) / tiles, K / kMinSliceK);
    if (S <= 1) return 1;
    const int64_t step = 32;  // a multiple of the k chunk of every precision
    int64_t ks = ((K + S - 1) / S + step - 1) / step * step;
    S = (K + ks - 1) / ks;
    *kslice = ks;
    return (int)S;
}

size_t splitk_workspace_bytes() { return (size_t)2048 * kTile * kTile * sizeof(double); }

template <typename CT>
int launch_gemm_splitk(bool upper, int64_t M, int64_t N, int64_t K, const CT *X, int64_t ldx, const CT *Y,
                       int64_t ldy, CT *C, int64_t ldc, CT *W, const int32_t *info, hipStream_t s) {
    constexpr Prec P = sizeof(CT) == 8 ? Prec::F64 : Prec::F32;
    int64_t ks = K;
    const int S = splitk_slices(upper, M, N, K, &ks);
    const bool vec = aligned16(X) && aligned16(Y) && (ldx % (16 / (int64_t)sizeof(CT)) == 0) &&
                     (ldy % (16 / (int64_t)sizeof(CT)) == 0) && (K % 32 == 0);
    if (S <= 1 || !vec || (size_t)S * M * N * sizeof(CT) > splitk_workspace_bytes())
        return launch_gemm_tn(P, sizeof(CT) == 8, upper, M, N, K, X, ldx, Y, ldy, C, ldc, info, s);
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
    p.nslices = S;
    p.kslice = ks;
    p.W = W;
    p.ldw = M;
    p.reserve_cus = 0;
    const double dM = (double)M, dN = (double)N, dK = (double)K;
    const double elems = upper ? (M <= N ? dM * (dM + 1) / 2 + (dN - dM) * dM : dN * (dN + 1) / 2) : dM * dN;
    const int tr = trace_begin(FLAME_KC_GEMM, s);
    hipLaunchKernelGGL((k_gemm_lds<P, CT, 128>), dim3((unsigned)(p.ntiles * S)), dim3(256), 0, s, p);
    FLAME_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_splitk_reduce<CT>, dim3((unsigned)((M + 255) / 256), (unsigned)N), dim3(256), 0, s, M, N,
                       p.upper, W, M, S, C, ldc);
    FLAME_CHECK_LAUNCH();
    trace_end(tr, s, 2.0 * dK * elems, dK * (dM + dN) * sizeof(CT) + (2.0 + S) * elems * sizeof(CT));
    return FLAME_OK;
}

template int launch_gemm_splitk<double>(bool, int64_t, int64_t, int64_t, const double *, int64_t, const double *,
                                        int64_t, double *, int64_t, double *, const int32_t *, hipStream_t);
template int launch_gemm_splitk<float>(bool, int64_t, int64_t, int64_t, const float *, int64_t, const float *,
                                       int64_t, float *, int64_t, float *, const int32_t *, hipStream_t);

// ---- low-precision copy of the panel ------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP64 -> BF16, one rounding to nearest even.  (float)x rounds once already,
// so rounding its result again to BF16 could round twice; instead x is first
// rounded to odd at FP32 precision (truncated toward zero, last bit set when
// inexact), which keeps the information the second rounding needs: with
// FP32's 24 bits >= BF16's 8 + 2, round-to-odd followed by
// round-to-nearest-even equals a direct round-to-nearest-even (Boldo and
// Melquiond, "When double rounding is odd").
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double x) {
    float f = (float)x;
    if (!__builtin_isnan(x) && (double)f != x) {
        uint32_t u = __float_as_uint(f);
        if (fabs((double)f) > fabs(x)) u -= 1u;  // one FP32 step toward zero (f != 0 here)
        f = __uint_as_float(u | 1u);
    }
    return f32_to_bf16_rne(f);
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
            static_cast<uint16_t *>(Yv)[i + c * ldy] = f64_to_bf16_rne(v);
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
