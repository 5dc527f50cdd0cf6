// Loop drivers: the FLAME partition/repartition loop of Fig. "dense-chol" and
// the two other loop invariants of A = U^T U, expressed as launches of the
// CHOL, TRSM and SYRK/GEMM kernels on column-major sub-views of A.
//
// Views at an iteration (A_TL is k x k, A11 is bk x bk, bk = min(b, n - k),
// m = n - k - bk), element (i, j) at A + i + j*lda:
//   A01 = A + k*lda          (k x bk)     A02 = A + (k+bk)*lda        (k x m)
//   A11 = A + k + k*lda      (bk x bk)    A12 = A + k + (k+bk)*lda    (bk x m)
//   A22 = A + (k+bk) + (k+bk)*lda (m x m)
// Sub-views are pointer offsets; nothing is repacked (the dense analogue of the
// paper's matrix views over a base matrix).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "flame_internal.h"

namespace flame {

namespace {

template <typename T>
struct Views {
    T *A;
    int64_t lda;
    T *at(int64_t i, int64_t j) const { return A + i + j * lda; }
};

template <typename T>
constexpr Prec native_prec() {
    return sizeof(T) == 8 ? Prec::F64 : Prec::F32;
}

template <typename T>
int gemm(bool upper, int64_t M, int64_t N, int64_t K, const T *X, int64_t ldx, const T *Y, int64_t ldy, T *C,
         int64_t ldc, const int32_t *info, hipStream_t s, int reserve_cus = 0) {
    return launch_gemm_tn(native_prec<T>(), sizeof(T) == 8, upper, M, N, K, X, ldx, Y, ldy, C, ldc, info, s,
                          reserve_cus);
}

// Compute units the remainder of the trailing update leaves to the next
// diagonal block's CHOL and TRSM when the two run concurrently (lookahead 2).
#ifndef FLAME_CHAIN_CUS
#define FLAME_CHAIN_CUS 16
#endif
constexpr int kChainCus = FLAME_CHAIN_CUS;

// Right-looking loop with lookahead: the block size drops to kTailNb for the
// last kTailN columns (measured at n = 16384, nb = 256: FP64 trailing
// products 40.5 -> 38.9 ms with 6144; with FP32/BF16 products the remainder
// update is cheaper and the crossover comes later).
#ifndef FLAME_TAIL_N
#define FLAME_TAIL_N 6144
#endif
constexpr int64_t kTailN = FLAME_TAIL_N;
constexpr int64_t kTailNMixed = 4096;
constexpr int64_t kTailNb = 128;
// Blocks above 256 (a trailing update with K = 512 runs at 61 TF/s against
// 53 at K = 256) drop to 256 for the last kMidN columns.
#ifndef FLAME_MID_N
#define FLAME_MID_N 8192
#endif
constexpr int64_t kMidN = FLAME_MID_N;
constexpr int64_t kMidNb = 256;
// While more than kEarlyN rows remain below the next panel, the remainder of
// the trailing update is launched before the update of the next panel rows
// (the two write disjoint rows and read only the current panel): the panel
// update then overlaps the long remainder instead of running alone.  Below
// that the chain of the next CHOL and TRSM is critical and the panel update
// keeps the whole GPU.
#ifndef FLAME_EARLY_N
#define FLAME_EARLY_N 8192
#endif
constexpr int64_t kEarlyN = FLAME_EARLY_N;

// Split-K form of C -= X^T Y for the tall-K products of the left-looking and
// bordered variants (K up to n, output only b rows): the K range is cut into
// slices computed by one launch, their partial products are then added to C
// in slice order (deterministic).
template <typename T>
int gemm_tallk(bool upper, int64_t M, int64_t N, int64_t K, const T *X, int64_t ldx, const T *Y, int64_t ldy, T *C,
               int64_t ldc, const int32_t *info, hipStream_t s) {
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    void *w = nullptr;
    int rc = ctx_workspace(ctx, kWsSplit, splitk_workspace_bytes(), &w);
    if (rc) return rc;
    return launch_gemm_splitk<T>(upper, M, N, K, X, ldx, Y, ldy, C, ldc, static_cast<T *>(w), info, s);
}

// ---- right-looking (the paper's loop) ------------------------------------
template <typename T>
int factor_right(int64_t n, T *A, int64_t lda, int nb, int lookahead, flame_trail_t trail, bool fixed_nb,
                 int32_t *info, hipStream_t s) {
    const bool rest_on_side = (lookahead == 2 || lookahead == 0);
    Views<T> V{A, lda};
    int rc;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    const bool mixed = (trail != FLAME_TRAIL_NATIVE);
    const Prec lp = (trail == FLAME_TRAIL_BF16) ? Prec::BF16 : Prec::F32;
    const int64_t ldw = ((int64_t)nb + 15) / 16 * 16;  // rows of the rounded panel copy (zero padded)
    void *W = nullptr;
    if (mixed) {
        const size_t esz = (lp == Prec::BF16) ? 2 : 4;
        rc = ctx_workspace(ctx, kWsFactor, (size_t)ldw * (size_t)std::max<int64_t>(n, 1) * esz, &W);
        if (rc) return rc;
    }
    const size_t wesz = (lp == Prec::BF16) ? 2 : 4;
    auto wcol = [&](int64_t j) { return static_cast<char *>(W) + (size_t)j * (size_t)ldw * wesz; };

    // trailing update of C (Mr x Nc, at A22 offset (i0, i0)..) from panel columns
    auto update = [&](int64_t k, int64_t bk, int64_t i0, int64_t Mr, int64_t j0, int64_t Nc, hipStream_t st,
                      int reserve = 0) -> int {
        // C = A22(i0 : i0+Mr, j0 : j0+Nc) with A22 at (k+bk, k+bk); X = A12(:, i0..), Y = A12(:, j0..)
        const int64_t base = k + bk;
        T *C = V.at(base + i0, base + j0);
        if (!mixed) {
            const T *X = V.at(k, base + i0);
            const T *Y = V.at(k, base + j0);
            return gemm<T>(true, Mr, Nc, bk, X, lda, Y, lda, C, lda, info, st, reserve);
        }
        return launch_gemm_tn(lp, true, true, Mr, Nc, ldw, wcol(i0), ldw, wcol(j0), ldw, C, lda, info, st, reserve);
    };

    rc = launch_zero_i32(info, 1, s);
    if (rc) return rc;
    if (n == 0) return FLAME_OK;

    if (lookahead < 0) {
        for (int64_t k = 0; k < n; k += nb) {
            const int64_t bk = std::min<int64_t>(nb, n - k);
            const int64_t m = n - k - bk;
            rc = launch_chol_block<T>((int)bk, V.at(k, k), lda, info, k, s);
            if (rc) return rc;
            if (m == 0) break;
            rc = launch_trsm_panel<T>((int)bk, m, V.at(k, k), lda, V.at(k, k + bk), lda, info, s);
            if (rc) return rc;
            if (mixed) {
                rc = launch_round_panel(lp, bk, m, reinterpret_cast<const double *>(V.at(k, k + bk)), lda, W, ldw,
                                        info, s);
                if (rc) return rc;
            }
            rc = update(k, bk, 0, m, 0, m, s);
            if (rc) return rc;
        }
        return FLAME_OK;
    }

    // Depth-1 lookahead.  The next iteration's CHOL and TRSM read only the
    // first bk2 rows of A22 (the next A11 and A12).  Those rows are updated
    // first, then the side stream factors them while the main stream applies
    // the rest of the update: the out-of-order execution that the by-blocks
    // task graph allows (CHOL of a later block needs only its own updates).
    hipStream_t side = ctx_side_stream(ctx);
    hipEvent_t ev_panel = ctx_event(ctx, 0);  // next panel rows updated (main)
    hipEvent_t ev_ready = ctx_event(ctx, 1);  // next CHOL + TRSM done (side)
    // Block size by position: nb while the trailing matrix is large (the
    // trailing update dominates), at most kMidNb once kMidN columns remain and
    // kTailNb once kTailN remain (the serial CHOL + TRSM chain dominates there
    // and costs less per column at the smaller block).
    const int64_t tail_n = mixed ? kTailNMixed : kTailN;
    auto nb_at = [&](int64_t k) -> int64_t {
        if (fixed_nb) return nb;
        const int64_t rest = n - k;
        if (rest <= tail_n) return std::min<int64_t>(nb, kTailNb);
        if (rest <= kMidN) return std::min<int64_t>(nb, kMidNb);
        return nb;
    };
    {
        const int64_t bk = std::min<int64_t>(nb_at(0), n);
        rc = launch_chol_block<T>((int)bk, V.at(0, 0), lda, info, 0, s);
        if (rc) return rc;
        if (n - bk > 0) {
            rc = launch_trsm_panel<T>((int)bk, n - bk, V.at(0, 0), lda, V.at(0, bk), lda, info, s);
            if (rc) return rc;
        }
    }
    for (int64_t k = 0, bk = 0; k < n; k += bk) {
        bk = std::min<int64_t>(nb_at(k), n - k);
        const int64_t m = n - k - bk;
        if (m == 0) break;
        if (mixed) {
            rc = launch_round_panel(lp, bk, m, reinterpret_cast<const double *>(V.at(k, k + bk)), lda, W, ldw, info,
                                    s);
            if (rc) return rc;
        }
        const int64_t k2 = k + bk;
        const int64_t bk2 = std::min<int64_t>(nb_at(k2), m);
        const int64_t m2 = m - bk2;
        const bool early = rest_on_side && m2 > kEarlyN;
        if (early) {
            // the rest of A22 (rows and columns [bk2, m)) first, on the second
            // stream, beside the panel-row update below
            FLAME_HIP(hipEventRecord(ev_panel, s));
            FLAME_HIP(hipStreamWaitEvent(side, ev_panel, 0));
            rc = update(k, bk, bk2, m2, bk2, m2, side, kChainCus);
            if (rc) return rc;
            FLAME_HIP(hipEventRecord(ev_ready, side));
        }
        // rows [0, bk2) of A22: the next A11 and A12
        rc = update(k, bk, 0, bk2, 0, m, s);
        if (rc) return rc;
        if (m2 == 0) {
            rc = launch_chol_block<T>((int)bk2, V.at(k2, k2), lda, info, k2, s);
            if (rc) return rc;
            continue;
        }
        if (!rest_on_side) {
            FLAME_HIP(hipEventRecord(ev_panel, s));
            FLAME_HIP(hipStreamWaitEvent(side, ev_panel, 0));
            rc = launch_chol_block<T>((int)bk2, V.at(k2, k2), lda, info, k2, side);
            if (rc) return rc;
            rc = launch_trsm_panel<T>((int)bk2, m2, V.at(k2, k2), lda, V.at(k2, k2 + bk2), lda, info, side);
            if (rc) return rc;
            FLAME_HIP(hipEventRecord(ev_ready, side));
            // the rest of A22: rows and columns [bk2, m)
            rc = update(k, bk, bk2, m2, bk2, m2, s);
            if (rc) return rc;
            FLAME_HIP(hipStreamWaitEvent(s, ev_ready, 0));
        } else {
            // the rest of A22 on the second stream (unless already launched);
            // the next CHOL and TRSM follow the panel rows on the main stream,
            // which dispatches them ahead of the remainder's workgroups
            if (!early) {
                FLAME_HIP(hipEventRecord(ev_panel, s));
                FLAME_HIP(hipStreamWaitEvent(side, ev_panel, 0));
                rc = update(k, bk, bk2, m2, bk2, m2, side, kChainCus);
                if (rc) return rc;
                FLAME_HIP(hipEventRecord(ev_ready, side));
            }
            rc = launch_chol_block<T>((int)bk2, V.at(k2, k2), lda, info, k2, s);
            if (rc) return rc;
            rc = launch_trsm_panel<T>((int)bk2, m2, V.at(k2, k2), lda, V.at(k2, k2 + bk2), lda, info, s);
            if (rc) return rc;
            FLAME_HIP(hipStreamWaitEvent(s, ev_ready, 0));
        }
    }
    return FLAME_OK;
}

// ---- left-looking ----------------------------------------------------------
template <typename T>
int factor_left(int64_t n, T *A, int64_t lda, int nb, int32_t *info, hipStream_t s) {
    Views<T> V{A, lda};
    int rc = launch_zero_i32(info, 1, s);
    if (rc) return rc;
    for (int64_t k = 0; k < n; k += nb) {
        const int64_t bk = std::min<int64_t>(nb, n - k);
        const int64_t m = n - k - bk;
        if (k > 0) {  // A11 -= A01^T A01
            rc = gemm_tallk<T>(true, bk, bk, k, V.at(0, k), lda, V.at(0, k), lda, V.at(k, k), lda, info, s);
            if (rc) return rc;
        }
        rc = launch_chol_block<T>((int)bk, V.at(k, k), lda, info, k, s);
        if (rc) return rc;
        if (m == 0) break;
        if (k > 0) {  // A12 -= A01^T A02
            rc = gemm_tallk<T>(false, bk, m, k, V.at(0, k), lda, V.at(0, k + bk), lda, V.at(k, k + bk), lda, info,
                               s);
            if (rc) return rc;
        }
        rc = launch_trsm_panel<T>((int)bk, m, V.at(k, k), lda, V.at(k, k + bk), lda, info, s);
        if (rc) return rc;
    }
    return FLAME_OK;
}

// ---- bordered -------------------------------------------------------------
template <typename T>
int factor_bordered(int64_t n, T *A, int64_t lda, int nb, int32_t *info, hipStream_t s) {
    Views<T> V{A, lda};
    int rc = launch_zero_i32(info, 1, s);
    if (rc) return rc;
    for (int64_t k = 0; k < n; k += nb) {
        const int64_t bk = std::min<int64_t>(nb, n - k);
        // A01 := triu(A00)^{-T} A01: forward substitution over 256-row chunks
        // of the k x k triangle (TRSM on the chunk, then GEMM on the rows
        // below); the chunk is independent of nb, so the chain of dependent
        // launches is k / 256 long whatever the block size
        constexpr int64_t kChunk = 256;
        for (int64_t r0 = 0; r0 < k; r0 += kChunk) {
            const int64_t w = std::min<int64_t>(kChunk, k - r0);
            rc = launch_trsm_panel<T>((int)w, bk, V.at(r0, r0), lda, V.at(r0, k), lda, info, s);
            if (rc) return rc;
            const int64_t below = k - r0 - w;
            if (below > 0) {
                rc = gemm<T>(false, below, bk, w, V.at(r0, r0 + w), lda, V.at(r0, k), lda, V.at(r0 + w, k), lda,
                             info, s);
                if (rc) return rc;
            }
        }
        if (k > 0) {  // A11 -= A01^T A01
            rc = gemm_tallk<T>(true, bk, bk, k, V.at(0, k), lda, V.at(0, k), lda, V.at(k, k), lda, info, s);
            if (rc) return rc;
        }
        rc = launch_chol_block<T>((int)bk, V.at(k, k), lda, info, k, s);
        if (rc) return rc;
    }
    return FLAME_OK;
}

template <typename T>
int factor_t(int64_t n, T *A, int64_t lda, const flame_opts_t &o, int32_t *info, hipStream_t s) {
    const int nb = o.nb;
    switch (o.variant) {
        case FLAME_VAR_RIGHT:
            return factor_right<T>(n, A, lda, nb, o.lookahead, (flame_trail_t)o.trail,
                                   (o.flags & FLAME_OPT_FIXED_NB) != 0, info, s);
        case FLAME_VAR_LEFT:
            return factor_left<T>(n, A, lda, nb, info, s);
        case FLAME_VAR_BORDERED:
            return factor_bordered<T>(n, A, lda, nb, info, s);
        case FLAME_VAR_BY_BLOCKS:
            if constexpr (sizeof(T) == 8) return by_blocks_factor(n, A, lda, nullptr, info, s);
            return FLAME_ERR_UNSUPPORTED;
        default:
            return FLAME_ERR_UNSUPPORTED;
    }
}

// ---- graph cache -----------------------------------------------------------
// The key holds every pointer a captured loop uses: the caller's (A, info,
// stream) and the library workspace the loop reads and writes (the rounded
// panel of the FP32/BF16 products, the split-K partials) with the generation
// of that buffer, so a graph is never replayed into a workspace that has been
// freed and replaced since its capture.
using GraphKey = std::tuple<int, int64_t, void *, int64_t, int32_t *, int, int, int, int, int, hipStream_t, int,
                            int, void *, uint64_t>;
constexpr int kKeyDev = 11, kKeySlot = 12, kKeyGen = 14;
std::mutex g_graph_mu;
std::map<GraphKey, hipGraphExec_t> g_graphs;

}  // namespace

void drop_factor_graphs() {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto &kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.clear();
}

int factor_dispatch(int32_t dtype, int64_t n, void *A, int64_t lda, const flame_opts_t &o, int32_t *info,
                    hipStream_t s) {
    auto run = [&](hipStream_t st) -> int {
        if (dtype == FLAME_F64) return factor_t<double>(n, static_cast<double *>(A), lda, o, info, st);
        return factor_t<float>(n, static_cast<float *>(A), lda, o, info, st);
    };
    if (o.graph != 1 || s == nullptr) return run(s);

    int dev = 0;
    FLAME_HIP(hipGetDevice(&dev));
    // The workspace is allocated (or grown) before the lookup and the capture:
    // no allocation happens inside a capture, and the key sees the buffer the
    // loop will use.
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    void *ws = nullptr;
    int slot = -1;
    if (o.variant == FLAME_VAR_LEFT || o.variant == FLAME_VAR_BORDERED) {
        slot = kWsSplit;
        int rc = ctx_workspace(ctx, slot, splitk_workspace_bytes(), &ws);
        if (rc) return rc;
    } else if (o.trail != FLAME_TRAIL_NATIVE) {
        slot = kWsFactor;
        const int64_t ldw = ((int64_t)o.nb + 15) / 16 * 16;
        int rc = ctx_workspace(ctx, slot, (size_t)ldw * (size_t)std::max<int64_t>(n, 1) * 4, &ws);
        if (rc) return rc;
    }
    const uint64_t ws_gen = slot >= 0 ? ctx_workspace_gen(ctx, slot) : 0;
    GraphKey key{dtype, n, A, lda, info, o.variant, o.nb, o.trail, o.lookahead, o.flags, s, dev, slot, ws, ws_gen};
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) {
            FLAME_HIP(hipGraphLaunch(it->second, s));
            return FLAME_OK;
        }
        // graphs of this device whose workspace has been replaced can never
        // be replayed again
        for (auto g = g_graphs.begin(); g != g_graphs.end();) {
            const int gslot = std::get<kKeySlot>(g->first);
            const bool stale = std::get<kKeyDev>(g->first) == dev && gslot >= 0 &&
                               std::get<kKeyGen>(g->first) != ctx_workspace_gen(ctx, gslot);
            if (stale) {
                (void)hipGraphExecDestroy(g->second);
                g = g_graphs.erase(g);
            } else {
                ++g;
            }
        }
    }
    FLAME_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = run(s);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc) {
        if (graph) hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) {
        set_last_hip_error(e);
        return FLAME_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
        set_last_hip_error(e);
        return FLAME_ERR_HIP;
    }
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        g_graphs[key] = exec;
    }
    FLAME_HIP(hipGraphLaunch(exec, s));
    return FLAME_OK;
}

}  // namespace flame
