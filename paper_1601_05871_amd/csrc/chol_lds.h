// LDS-resident factorization of a diagonal block (CHOL step of Fig.
// "dense-chol"), unblocked inside in square-root-free form: the block's upper
// 16 x 16 tiles in LDS in matrix-core accumulator order, one elimination pass
// per 16-row band and a matrix-core update of the trailing tiles (described
// below, before chol_lds_core2).  Used by the single-block kernel (blocks of
// 128) and by the batched kernel (its diagonal blocks).
//
// All functions are called by the whole workgroup (256 threads) with uniform
// control flow.
#pragma once

#include "chol_wave.h"
#include "trsm_rl.h"

namespace flame {

// ---- one-pass band elimination + matrix-core update ------------------------
// Per 16-row sub-block [r0, r0 + 16):
//   (a) every wavefront eliminates the band: lanes 0..15 (row 0 of the
//       wavefront) hold the 16 columns of the diagonal sub-block, the other
//       48 lanes 48 columns of the row panel to its right, rows r0 .. r0 + 15
//       of each in registers.  The square-root-free elimination with pivot j
//       updates every such column with row j of the diagonal sub-block, which
//       is copied from row 0 to the three other rows of 16 lanes (permlane
//       swaps) and then read lane by lane through a DPP row broadcast fused
//       into the multiply-add.  Diagonal sub-block and row panel (the CHOL and
//       TRSM steps on the sub-block) come out of one pass; the four wavefronts
//       take 192 panel columns between them (and repeat the diagonal work).
//   (b) the trailing block takes the rank-16 update A22 -= P^T P on matrix
//       cores, 16 x 16 output tiles (stored in LDS in accumulator order),
//       P read from the band's tiles, where the elimination left it.
// Two barriers per sub-block.

// row 0's value (lanes 0..15) in all four rows of 16 lanes
__device__ __forceinline__ unsigned rep_row0_u32(unsigned x) {
    const auto a = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows 0 0 2 2
    const auto b = __builtin_amdgcn_permlane32_swap(a[0], a[0], false, false);
    return b[0];
}
__device__ __forceinline__ double rep_row0(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = rep_row0_u32((unsigned)u), hi = rep_row0_u32((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float rep_row0(float v) { return __uint_as_float(rep_row0_u32(__float_as_uint(v))); }

// lane I of this row of 16, all lanes active (bound_ctrl: no old value kept)
template <int I>
__device__ __forceinline__ double row_bcast_b(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + I, 0xF, 0xF, true);
}
template <int I>
__device__ __forceinline__ float row_bcast_b(float v) {
    return __builtin_amdgcn_update_dpp(0.0f, v, 0x150 + I, 0xF, 0xF, true);
}

// acc + (src of lane I of this row of 16) * mul as one v_fmac with a DPP row
// broadcast on src (the compiler does not form this for 64-bit operands).
// The compiler does not see the DPP read either: NOP adds the two wait states
// a DPP read of a VGPR written by one of the last two VALU instructions
// needs.  The statements are volatile, so they keep their order among
// themselves; within one pivot only the first read of the new broadcast row
// can follow its write that closely.
template <int I, bool NOP>
__device__ __forceinline__ double fmac_bcast(double acc, double src, double mul) {
    if constexpr (NOP)
        asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(src), "v"(mul), "i"(I));
    else
        asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(src), "v"(mul), "i"(I));
    return acc;
}
template <int I, bool NOP>
__device__ __forceinline__ float fmac_bcast(float acc, float src, float mul) {
    if constexpr (NOP)
        asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(src), "v"(mul), "i"(I));
    else
        asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(src), "v"(mul), "i"(I));
    return acc;
}

template <int I, typename T>
__device__ __forceinline__ void band_row_update(T (&a)[16], T rep, T nt) {
    if constexpr (I < 16) {
        a[I] = fmac_bcast<I, false>(a[I], rep, nt);
        band_row_update<I + 1>(a, rep, nt);
    }
}
// Pivot J: d_J read from lane J as a scalar (the serial chain: read, then
// the reciprocal and the multiplier nt = -A(J, col) / d_J), and row J of the
// diagonal sub-block copied into every row of 16 (rep, off that chain).
template <int J, typename T>
__device__ __forceinline__ void band_pivot_setup(const T (&a)[16], int c, int &bad, T &dme, T &rep, T &nt) {
    const T d = rdlane(a[J], J);
    bad = (bad == 0 && !(d > T(0))) ? J + 1 : bad;
    dme = (c == J) ? d : dme;
    nt = -(a[J] * recip(d));
    rep = rep_row0(a[J]);
}
// Pivot J's update: column J + 1 first, then pivot J + 1's set-up, then the
// other columns of pivot J.
template <int J, typename T>
__device__ __forceinline__ void band_pivots(T (&a)[16], int c, int &bad, T &dme, T rep, T nt) {
    if constexpr (J < 15) {
        a[J + 1] = fmac_bcast<J + 1, true>(a[J + 1], rep, nt);
        T rep1, nt1;
        band_pivot_setup<J + 1>(a, c, bad, dme, rep1, nt1);
        band_row_update<J + 2>(a, rep, nt);
        band_pivots<J + 1>(a, c, bad, dme, rep1, nt1);
    }
}
template <int J, typename T>
__device__ __forceinline__ void band_scale(T (&a)[16], bool diag_lane, int c, T sme, T ime) {
    if constexpr (J < 16) {
        const T inv_j = row_bcast_b<J>(ime);  // 1 / sqrt(d_J): every row holds the same d
        const T scaled = a[J] * inv_j;
        a[J] = (diag_lane && c == J) ? sme : scaled;
        band_scale<J + 1>(a, diag_lane, c, sme, ime);
    }
}

// LDS layout of the band factorization: the upper block triangle in 16 x 16
// tiles, tile (bi, bj), bi <= bj, at (bj (bj + 1) / 2 + bi) 256 elements; a
// tile is stored in the order of a matrix-core accumulator (item v of lane l
// in the run of 64 elements at 64 v), so that the update reads and writes a
// tile as 4 runs of 64.  FP64 accumulators hold (row l % 16, column
// l / 16 + 4 v), FP32 ones (row 4 (l / 16) + v, column l % 16).  Entries
// below the diagonal of a diagonal tile are never written or read as data.
//
// Inside each run the elements are permuted so that the three access
// patterns of the factorization hit distinct LDS banks (64 banks of 4 bytes):
//   (a) accumulator runs (the update's C tiles): any permutation inside a run
//       keeps these free of conflicts;
//   (b) operand reads of the update: lane (r, g) reads element (k, r) of one
//       tile for its k slot of a matrix-core step (FP64: k = g + 4 t in step
//       t; FP32: k = 4 g + t);
//   (c) the elimination: each 16-lane group reads (and writes) one column,
//       row by row, of its own tile, the four groups of a wavefront in four
//       different tiles.
// FP64 (64-bit accesses, 32 lanes at a time; 128-bit ones 16 at a time): the
// row index is XORed with h = 2 (column bits 2-3) + 8 (column bit 1), an even
// number, so rows 2 i and 2 i + 1 stay side by side and (c) reads a column as
// eight 128-bit pairs; in (b) each half-wavefront then covers 32 distinct
// banks pairs.  Unpermuted, 8 lanes shared a bank in (b) and 16 in (c).
// FP32 (32-bit accesses, 64 lanes at a time): (a) and (b) read consecutive
// addresses; for (c) bits 2-3 of the row index (the 16-element quarter of a
// run) are XORed with a key of the tile's distance d = bj - bi from the
// diagonal, 0 for d = 0, else 1 + (d - 1) mod 3, which puts the four groups
// (distances 0, 1 + 3 w, 2 + 3 w, 3 + 3 w in wavefront w) in different
// quarters (tabulated for d <= 15: blocks of up to 256).
template <int NMAX>
constexpr int band_lds_size() {
    return (NMAX / 16) * (NMAX / 16 + 1) / 2 * 256;
}
template <typename T>
__device__ __forceinline__ int tile_key(int d) {
    if constexpr (sizeof(T) == 8)
        return 0;
    else
        return (int)((0xE79E79E4u >> (2 * d)) & 3u);
}
__device__ __forceinline__ int tile_base(int bi, int bj) { return ((bj * (bj + 1)) >> 1) * 256 + bi * 256; }
// FP64: the XOR applied to row indices of column cc (even)
__device__ __forceinline__ int row_xor64(int cc) { return ((cc >> 2) << 1) | ((cc & 2) << 2); }
template <typename T>
__device__ __forceinline__ int tile_pos(int rr, int cc, int key) {
    if constexpr (sizeof(T) == 8)
        return (cc >> 2) * 64 + (cc & 3) * 16 + (rr ^ row_xor64(cc));
    else
        return (rr & 3) * 64 + (((rr >> 2) ^ key) << 4) + cc;
}
// the row of k slot (g, t) in the update's operand reads
template <typename T>
__device__ __forceinline__ int k_slot(int g, int t) {
    return sizeof(T) == 8 ? g + 4 * t : 4 * g + t;
}
// position of accumulator item v of lane l in a tile with this key
template <typename T>
__device__ __forceinline__ int acc_pos(int l, int v, int key) {
    if constexpr (sizeof(T) == 8)
        return tile_pos<T>(l & 15, (l >> 4) + 4 * v, key);
    else
        return tile_pos<T>(4 * (l >> 4) + v, l & 15, key);
}
template <typename T>
__device__ __forceinline__ int band_at(int row, int col) {
    return tile_base(row >> 4, col >> 4) + tile_pos<T>(row & 15, col & 15, tile_key<T>((col >> 4) - (row >> 4)));
}

// Workgroup barrier for LDS traffic only: outstanding global stores stay in
// flight (the kernels below never read back what they store).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Loads the upper triangle of the n x n block A (n <= NMAX, NMAX = 64 or 128)
// into the tiles of L, padded with the identity up to n rounded up to 16.  A
// full FP64 128-block with 16-byte aligned columns: wavefront w loads columns
// w, w + 4, ... as 16-byte row pairs (lane l: rows 2 l, 2 l + 1; the pair
// straddling the diagonal also stores its lower entry, which no one reads).
// Otherwise one element per thread through clamped addresses (256 / NMAX
// columns at a time).  All loads are issued before the LDS stores.
template <typename T, int NMAX>
__device__ __forceinline__ void band_load(int n, const T *__restrict__ A, int64_t lda, T *L) {
    static_assert(NMAX == 64 || NMAX == 128, "64 x 64 or 128 x 128 block");
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    constexpr int PER = 16 / (int)sizeof(T);  // rows per 16-byte load
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool wide = n == NMAX && ((lda & (PER - 1)) == 0) && (((uintptr_t)A & 15) == 0);
    if (wide && PER * 64 == NMAX) {
        // FP64: 64 lanes x 2 rows = one column per load; lanes below the
        // diagonal read the diagonal's pair again (same bytes, no traffic)
        const int row = PER * lane;
        u4 v[NMAX / 4];
#pragma unroll
        for (int e = 0; e < NMAX / 4; ++e) {
            const int col = 4 * e + wave;
            v[e] = *reinterpret_cast<const u4 *>(A + (int64_t)col * lda + min(row, col & ~(PER - 1)));
        }
#pragma unroll
        for (int e = 0; e < NMAX / 4; ++e) {
            const int col = 4 * e + wave;
            // rows (row, row + 1) stay side by side, in order (row_xor64 is even)
            if (row <= col) *reinterpret_cast<u4 *>(L + band_at<T>(row, col)) = v[e];
        }
        return;
    }
    constexpr int H = 256 / NMAX;  // columns per pass
    const int row = tid & (NMAX - 1), h = __builtin_amdgcn_readfirstlane(tid / NMAX);
    const int np = (n + 15) / 16 * 16;
    const int rc = min(row, n - 1);
    T v[NMAX / H];
#pragma unroll
    for (int e = 0; e < NMAX / H; ++e) v[e] = A[(int64_t)rc + (int64_t)min(H * e + h, n - 1) * lda];
#pragma unroll
    for (int e = 0; e < NMAX / H; ++e) {
        const int col = H * e + h;
        if (row <= col && col < np)
            L[band_at<T>(row, col)] = (row < n && col < n) ? v[e] : (row == col ? T(1) : T(0));
    }
}

// Rank-16 update A22 -= P^T P of M trailing tiles: tiles w, w + 4, ...,
// w + 4 (M - 1) of the column-by-column list of upper tiles (bi, bj) of the
// trailing block (tile indices relative to sb + 1); P, the 16 rows of the
// band, is read from the band's own tiles (sb, sb + 1 + bi).  All LDS reads
// are issued first, then the 4 M matrix-core steps (M independent chains),
// then the stores; no branch in between.  Called by one whole wavefront (w
// uniform).
template <typename T, int M>
__device__ __forceinline__ void band_update_tiles(T *L, int sb, int w) {
    typedef typename TrsmAcc<T>::type acc_t;
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    int bi[M], bj[M];
    {
        int ti = 0, tj = 0;  // wavefront-uniform walk over the tile list
        for (int idx = 0; idx < w; ++idx)
            if (++ti > tj) ti = 0, ++tj;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            bi[m] = ti;
            bj[m] = tj;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (++ti > tj) ti = 0, ++tj;
        }
    }
    const int o16 = sb + 1;
    acc_t acc[M];
    T x[M][4], y[M][4];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const T *t = L + tile_base(o16 + bi[m], o16 + bj[m]);
        const int kc = tile_key<T>(bj[m] - bi[m]);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[m][v] = t[acc_pos<T>(lane, v, kc)];
        // the band's tiles (sb, o16 + b) lie at distance 1 + b from the diagonal
        const T *pi = L + tile_base(sb, o16 + bi[m]);
        const T *pj = L + tile_base(sb, o16 + bj[m]);
        const int ki = tile_key<T>(1 + bi[m]), kj = tile_key<T>(1 + bj[m]);
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
            x[m][t4] = pi[tile_pos<T>(k_slot<T>(g, t4), r, ki)];
            y[m][t4] = pj[tile_pos<T>(k_slot<T>(g, t4), r, kj)];
        }
    }
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4)
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] = mma_rc(-x[m][t4], y[m][t4], acc[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        T *t = L + tile_base(o16 + bi[m], o16 + bj[m]);
        const int kc = tile_key<T>(bj[m] - bi[m]);
#pragma unroll
        for (int v = 0; v < 4; ++v) t[acc_pos<T>(lane, v, kc)] = acc[m][v];
    }
}

// Factors the n x n block whose upper triangle L holds (band_load layout,
// padded to np = n rounded up to 16, np <= NMAX <= 16 + 192) and writes U
// to the upper triangle of A (column-major, lda) straight from registers.
// Returns 0, or the 1-based position of the first pivot that is not > 0 (A
// then holds a partial result).  s_bad: one int.  TS (instrumentation): the cycle counter at the end of sub-block s's
// elimination in wavefront w goes to ts[8 s + w], after its phases to
// ts[8 s + 4 .. 8 s + 6] (thread 0).
// KEEP_DIAG: the diagonal 16 x 16 tiles of U also go back into their LDS
// tiles (wavefront 0, after the band's barrier: every wavefront reads the
// diagonal tile in its elimination), so that L ends up holding all of U in
// band layout.
template <typename T, int NMAX, bool TS = false, bool KEEP_DIAG = false>
__device__ int chol_lds_core2(int n, T *L, int *s_bad, T *__restrict__ A, int64_t lda,
                              unsigned long long *ts = nullptr) {
    static_assert(NMAX - 16 <= 192, "four wavefronts take 192 panel columns");
    const int np = (n + 15) / 16 * 16;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lrow = lane >> 4;
    // 16-byte stores of a panel column's 16 entries when every column start
    // is 16-byte aligned
    const bool wide = ((lda & (16 / (int64_t)sizeof(T) - 1)) == 0) && (((uintptr_t)A & 15) == 0);
    for (int r0 = 0;; r0 += 16) {
        const int rest = np - r0 - 16;
        // the lane compares below recomputed in every pass: hoisted out of the
        // loop they would be 32 scalar-register masks kept alive (and spilled)
        int c = lane & 15;
        asm volatile("" : "+v"(c));
        // (a) this lane's column: diagonal column r0 + c, or panel column pc
        const bool diag_lane = lrow == 0;
        const int pc = 48 * wave + 16 * (lrow - 1) + c;
        const bool pvalid = !diag_lane && pc < rest;
        const int col = (diag_lane || rest == 0) ? r0 + c : r0 + 16 + min(pc, rest - 1);
        T a[16];
        T *const acol = L + tile_base(r0 >> 4, col >> 4);  // this column's tile in the band
        const int akey = tile_key<T>((col >> 4) - (r0 >> 4));
        int bad = 0;
        T *__restrict__ out = A + (int64_t)r0 + (int64_t)col * lda;
        auto to_tile = [&]() {
            if constexpr (sizeof(T) == 8) {
                T *cp = acol + ((col & 15) >> 2) * 64 + ((col & 15) & 3) * 16;
                const int hx = row_xor64(col & 15);
#pragma unroll
                for (int i = 0; i < 16; i += 2) *reinterpret_cast<double2 *>(cp + (i ^ hx)) = double2{a[i], a[i + 1]};
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) acol[tile_pos<T>(i, col & 15, akey)] = a[i];
            }
        };
        // a wavefront whose 48 panel columns all lie beyond the band has no
        // work in this pass (wavefront 0 always has: the diagonal block)
        const bool active = wave == 0 || 48 * wave < rest;
        if (active) {
            // i > c on the diagonal: unused
            if constexpr (sizeof(T) == 8) {
                const T *cp = acol + ((col & 15) >> 2) * 64 + ((col & 15) & 3) * 16;  // row 0 before the XOR
                const int hx = row_xor64(col & 15);
#pragma unroll
                for (int i = 0; i < 16; i += 2) {
                    const double2 pr = *reinterpret_cast<const double2 *>(cp + (i ^ hx));
                    a[i] = pr.x;
                    a[i + 1] = pr.y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) a[i] = acol[tile_pos<T>(i, col & 15, akey)];
            }
            T dme = T(1), rep, nt;
            band_pivot_setup<0>(a, c, bad, dme, rep, nt);
            band_pivots<0>(a, c, bad, dme, rep, nt);
            const T sme = sqrt(dme);
            const T ime = recip(sme);
            band_scale<0>(a, diag_lane, c, sme, ime);
            if constexpr (TS) {
                if (lane == 0) ts[r0 / 2 + wave] = __builtin_amdgcn_s_memtime();
            }
            // U rows r0 .. r0 + 15 are final: straight to A; the panel also back
            // into its band tiles, where the update reads it
            if (diag_lane) {
                if (wave == 0) {
                    if (col < n) {
#pragma unroll
                        for (int i = 0; i < 16; ++i)
                            if (i <= c) out[i] = a[i];
                    }
                }
            } else if (pvalid) {
                to_tile();
                if (col < n) {
                    if (wide) {
                        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
#pragma unroll
                        for (int i = 0; i < 16; i += 16 / (int)sizeof(T)) {
                            u4 w;
                            __builtin_memcpy(&w, &a[i], 16);
                            *reinterpret_cast<u4 *>(out + i) = w;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 16; ++i) out[i] = a[i];
                    }
                }
            }
        }  // active
        if (tid == 0) *s_bad = bad;
        lds_barrier();
        // every wavefront has read the diagonal tile of this band: it can take U
        if constexpr (KEEP_DIAG) {
            if (diag_lane && wave == 0) to_tile();
        }
        if constexpr (TS) {
            if (tid == 0) ts[r0 / 2 + 4] = __builtin_amdgcn_s_memtime();
        }
        const int bad_u = __builtin_amdgcn_readfirstlane(*s_bad);  // uniform: a scalar branch
        if (bad_u != 0) return r0 + bad_u;
        if (rest == 0) break;
        // (b) rank-16 update of the trailing tiles (bi, bj), o / 16 <= bi <=
        // bj: wavefront w takes tiles w, w + 4, ... (band_update_tiles)
        {
            constexpr int kNb = NMAX / 16 - 1;
            constexpr int kMaxT = (kNb * (kNb + 1) / 2 + 3) / 4;
            static_assert(kMaxT <= 7, "tile counts dispatched below");
            const int nb16 = rest >> 4;
            const int cnt = nb16 * (nb16 + 1) / 2;
            const int mine = cnt > wave ? (cnt - wave + 3) / 4 : 0;  // wavefront-uniform
            const int sb = r0 >> 4;
            switch (mine) {
                case 1: band_update_tiles<T, 1>(L, sb, wave); break;
                case 2: band_update_tiles<T, 2>(L, sb, wave); break;
                case 3: band_update_tiles<T, 3>(L, sb, wave); break;
                case 4: band_update_tiles<T, 4>(L, sb, wave); break;
                case 5: band_update_tiles<T, 5>(L, sb, wave); break;
                case 6: band_update_tiles<T, 6>(L, sb, wave); break;
                case 7: band_update_tiles<T, 7>(L, sb, wave); break;
                default: break;
            }
        }
        if constexpr (TS) {
            if (tid == 0) ts[r0 / 2 + 5] = __builtin_amdgcn_s_memtime();
        }
        lds_barrier();
        if constexpr (TS) {
            if (tid == 0) ts[r0 / 2 + 6] = __builtin_amdgcn_s_memtime();
        }
    }
    return 0;
}

}  // namespace flame
