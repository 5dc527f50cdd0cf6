// Learned selector (weights, feature rows, inference through the HIP MLP
// kernel), the exhaustive autotuner and its tuning table, and the choice used
// by FLAME_VAR_AUTO.
//
// The classes are the library's distinct ways of solving an SPD system (or a
// batch of them) of one order: the loop variants and block sizes of the
// FP64 / FP32 factorization followed by a plain solve, the batched persistent
// factorization, and the mixed-precision solve (FP32 or BF16 trailing
// products, FP64 refinement by IR-then-CG or by CG alone).  The paper picks
// its task granularity by hand; the selector learns the choice from timings
// of these programs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "flame_internal.h"

using namespace flame;

namespace {

constexpr int kF = FLAME_SEL_FEATURES, kC = FLAME_SEL_CLASSES;

// class -> program (see flame.h)
const flame_choice_t kClasses[kC] = {
    {0, FLAME_VAR_RIGHT, 512, FLAME_TRAIL_NATIVE, 0, 0, 0, 0},
    {1, FLAME_VAR_RIGHT, 256, FLAME_TRAIL_NATIVE, FLAME_OPT_FIXED_NB, 0, 0, 0},
    {2, FLAME_VAR_RIGHT, 128, FLAME_TRAIL_NATIVE, FLAME_OPT_FIXED_NB, 0, 0, 0},
    {3, FLAME_VAR_RIGHT, 64, FLAME_TRAIL_NATIVE, FLAME_OPT_FIXED_NB, 0, 0, 0},
    {4, FLAME_VAR_LEFT, 128, FLAME_TRAIL_NATIVE, 0, 0, 0, 0},
    {5, FLAME_VAR_LEFT, 256, FLAME_TRAIL_NATIVE, 0, 0, 0, 0},
    {6, FLAME_VAR_BORDERED, 256, FLAME_TRAIL_NATIVE, 0, 0, 0, 0},
    {7, FLAME_VAR_RIGHT, 0, FLAME_TRAIL_NATIVE, 0, 0, 1, 0},
    {8, FLAME_VAR_RIGHT, 0, FLAME_TRAIL_F32, 0, FLAME_REFINE_AUTO, 0, 0},
    {9, FLAME_VAR_RIGHT, 0, FLAME_TRAIL_BF16, 0, FLAME_REFINE_AUTO, 0, 0},
    {10, FLAME_VAR_RIGHT, 0, FLAME_TRAIL_F32, 0, FLAME_REFINE_CG, 0, 0},
    {11, FLAME_VAR_RIGHT, 0, FLAME_TRAIL_BF16, 0, FLAME_REFINE_CG, 0, 0},
};
constexpr int kFactorClasses = 7;  // classes 0..6: single-matrix factorization + plain solve

struct SelState {
    std::mutex mu;
    std::vector<float> weights;     // host copy; empty = not loaded
    std::map<int, bool> on_device;  // device -> weights uploaded to its workspace
    std::map<int, uint64_t> gen;    // device -> generation of the workspace holding them
    std::map<std::pair<int32_t, int64_t>, int32_t> table;  // autotuner: (dtype, n) -> factor class
};
SelState g_sel;

void features(int64_t n, int64_t batch, int32_t dtype, double kappa, float *f) {
    f[0] = (float)std::log2((double)std::max<int64_t>(n, 1));
    f[1] = (float)std::log2((double)std::max<int64_t>(batch, 1));
    f[2] = dtype == FLAME_F64 ? 1.0f : 0.0f;
    f[3] = dtype == FLAME_F32 ? 1.0f : 0.0f;
    f[4] = (float)std::log10(std::max(kappa, 1.0));
}

// Whether class c can run for this shape: the batched kernel takes orders up
// to 1024, the mixed-precision solve FP64 matrices.
bool feasible(int c, int64_t n, int32_t dtype) {
    if (kClasses[c].batched) return n <= 1024;
    if (kClasses[c].trail != FLAME_TRAIL_NATIVE) return dtype == FLAME_F64;
    return true;
}

// Workspace of the selector on the current device: weights, then room for
// `count` feature rows and logits.  Caller holds g_sel.mu.
int sel_buffers(int64_t count, float **w, float **feat, float **logits, hipStream_t *s) {
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    int dev = 0;
    FLAME_HIP(hipGetDevice(&dev));
    const size_t need = ((size_t)FLAME_SEL_NPARAM + (size_t)count * (kF + kC)) * sizeof(float);
    void *base = nullptr;
    int rc = ctx_workspace(ctx, kWsSelector, need, &base);
    if (rc) return rc;
    // a replaced workspace has lost the uploaded weights
    const uint64_t gen = ctx_workspace_gen(ctx, kWsSelector);
    if (g_sel.gen[dev] != gen) g_sel.on_device[dev] = false;
    g_sel.gen[dev] = gen;
    *s = ctx_aux_stream(ctx);
    *w = static_cast<float *>(base);
    *feat = *w + FLAME_SEL_NPARAM;
    *logits = *feat + (size_t)count * kF;
    if (!g_sel.on_device[dev]) {
        FLAME_HIP(hipMemcpyAsync(*w, g_sel.weights.data(), (size_t)FLAME_SEL_NPARAM * sizeof(float),
                                 hipMemcpyHostToDevice, *s));
        g_sel.on_device[dev] = true;
    }
    return FLAME_OK;
}

int logits_locked(const float *f, int64_t count, float *out) {
    float *w, *df, *dl;
    hipStream_t s;
    int rc = sel_buffers(count, &w, &df, &dl, &s);
    if (rc) return rc;
    FLAME_HIP(hipMemcpyAsync(df, f, (size_t)count * kF * sizeof(float), hipMemcpyHostToDevice, s));
    rc = launch_selector(w, df, count, dl, s);
    if (rc) return rc;
    FLAME_HIP(hipMemcpyAsync(out, dl, (size_t)count * kC * sizeof(float), hipMemcpyDeviceToHost, s));
    FLAME_HIP(hipStreamSynchronize(s));
    return FLAME_OK;
}

// argmax of the logits over the classes [0, upto) feasible for the shape
int argmax_feasible(const float *l, int upto, int64_t n, int32_t dtype) {
    int best = -1;
    for (int c = 0; c < upto; ++c) {
        if (!feasible(c, n, dtype)) continue;
        if (best < 0 || l[c] > l[best]) best = c;
    }
    return best;
}

}  // namespace

namespace flame {

void selector_forget_devices() {
    std::lock_guard<std::mutex> lk(g_sel.mu);
    g_sel.on_device.clear();
    g_sel.gen.clear();
}

// VAR_AUTO of flame_factor: the single-matrix factorization class the
// selector ranks highest (when its weights are loaded), else the autotuner's
// table for the nearest tuned order of this dtype, else class 0.
void choose_variant(int32_t dtype, int64_t n, int64_t batch, flame_opts_t *o) {
    int c = -1;
    {
        std::lock_guard<std::mutex> lk(g_sel.mu);
        if (!g_sel.weights.empty()) {
            float f[kF], l[kC];
            features(n, batch, dtype, 0.0, f);
            if (logits_locked(f, 1, l) == FLAME_OK) c = argmax_feasible(l, kFactorClasses, n, dtype);
        }
        if (c < 0) {
            double dist = std::numeric_limits<double>::infinity();
            for (const auto &kv : g_sel.table) {
                if (kv.first.first != dtype) continue;
                const double d = std::fabs(std::log2((double)std::max<int64_t>(kv.first.second, 1)) -
                                           std::log2((double)std::max<int64_t>(n, 1)));
                if (d < dist) {
                    dist = d;
                    c = kv.second;
                }
            }
            if (dist > 0.5) c = -1;
        }
    }
    if (c < 0) c = 0;
    o->variant = kClasses[c].variant;
    if (o->nb == 0) {
        o->nb = kClasses[c].nb;
        o->flags |= kClasses[c].flags;
    }
}

}  // namespace flame

namespace {

// ---- autotuner ------------------------------------------------------------------

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

__global__ void k_fill_ones(int64_t n, void *b, int f64) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (f64)
        static_cast<double *>(b)[i] = 1.0;
    else
        static_cast<float *>(b)[i] = 1.0f;
}

__global__ void k_batch_arrays(int32_t count, int32_t n, char *base, int64_t bytes, int32_t *ns, int32_t *ldas,
                               int64_t *ptrs) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    ns[i] = n;
    ldas[i] = n;
    ptrs[i] = reinterpret_cast<int64_t>(base + (int64_t)i * bytes);
}

constexpr size_t kBatchBytesCap = (size_t)2 << 30;  // replicas the batched candidate factors
constexpr float kLongRunMs = 2000.f;                // a warm-up this long is not repeated

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int flame_selector_load(const float *w, int64_t count) {
    if (w == nullptr && count == 0) {  // unload
        std::lock_guard<std::mutex> lk(g_sel.mu);
        g_sel.weights.clear();
        g_sel.on_device.clear();
        return FLAME_OK;
    }
    if (w == nullptr) return -1;
    if (count != FLAME_SEL_NPARAM) return -2;
    std::lock_guard<std::mutex> lk(g_sel.mu);
    g_sel.weights.assign(w, w + count);
    g_sel.on_device.clear();
    return FLAME_OK;
}

int flame_select_class(int32_t cls, flame_choice_t *choice) {
    if (cls < 0 || cls >= kC) return -1;
    if (choice == nullptr) return -2;
    *choice = kClasses[cls];
    return FLAME_OK;
}

int flame_select(int64_t n, int64_t batch, int32_t dtype, double kappa, flame_choice_t *choice) {
    if (n < 0) return -1;
    if (batch < 0) return -2;
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -3;
    if (!(kappa >= 0.0)) return -4;
    if (choice == nullptr) return -5;
    std::lock_guard<std::mutex> lk(g_sel.mu);
    if (g_sel.weights.empty()) return FLAME_ERR_UNSUPPORTED;
    float f[kF], l[kC];
    features(n, batch, dtype, kappa, f);
    int rc = logits_locked(f, 1, l);
    if (rc) return rc;
    *choice = kClasses[argmax_feasible(l, kC, n, dtype)];
    return FLAME_OK;
}

int flame_select_logits(const float *features_in, int64_t count, float *logits) {
    if (features_in == nullptr && count > 0) return -1;
    if (count < 0) return -2;
    if (logits == nullptr && count > 0) return -3;
    std::lock_guard<std::mutex> lk(g_sel.mu);
    if (g_sel.weights.empty()) return FLAME_ERR_UNSUPPORTED;
    if (count == 0) return FLAME_OK;
    return logits_locked(features_in, count, logits);
}

int flame_autotune(int32_t dtype, int64_t n, void *A, int64_t lda, int64_t batch, int32_t reps, double *times_ms,
                   void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return -2;
    if (A == nullptr && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (batch < 1) return -5;
    if (reps < 1) return -6;
    if (times_ms == nullptr) return -7;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int c = 0; c < kC; ++c) times_ms[c] = std::numeric_limits<double>::infinity();
    if (n == 0) return FLAME_OK;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    const size_t esz = dtype == FLAME_F64 ? 8 : 4;
    const size_t mat = (size_t)n * (size_t)n * esz;
    // the batched candidate factors `copies` replicas of A (at most 2 GiB)
    const int64_t copies =
        (n <= 1024) ? std::max<int64_t>(1, std::min<int64_t>(batch, (int64_t)(kBatchBytesCap / mat))) : 0;
    const size_t oW = 0, oB = up256(mat), oX = oB + up256((size_t)n * esz), oInfo = oX + up256((size_t)n * esz),
                 oNs = oInfo + up256((size_t)std::max<int64_t>(copies, 1) * 4), oLd = oNs + up256((size_t)copies * 4),
                 oPt = oLd + up256((size_t)copies * 4), oBat = oPt + up256((size_t)copies * 8);
    const size_t total = oBat + (size_t)copies * mat;
    void *base = nullptr;
    int rc = ctx_workspace(ctx, kWsTune, total, &base);
    if (rc) return rc;
    char *ws = static_cast<char *>(base);
    char *W = ws + oW;
    void *b0 = ws + oB, *x = ws + oX;
    int32_t *info = reinterpret_cast<int32_t *>(ws + oInfo);  // one per replica of the batched candidate
    Timer tm;
    FLAME_HIP(hipEventCreate(&tm.e0));
    FLAME_HIP(hipEventCreate(&tm.e1));
    hipLaunchKernelGGL(k_fill_ones, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, b0, dtype == FLAME_F64);
    FLAME_CHECK_LAUNCH();
    auto copy_matrix = [&](char *dst) -> int {
        FLAME_HIP(hipMemcpy2DAsync(dst, (size_t)n * esz, A, (size_t)lda * esz, (size_t)n * esz, (size_t)n,
                                   hipMemcpyDeviceToDevice, s));
        return FLAME_OK;
    };
    // one run of fn between events, after prep; FLAME_ERR_BREAKDOWN when the
    // run reports a breakdown or fails to converge
    auto timed = [&](auto &&prep, auto &&fn, bool check_info, float *ms_out) -> int {
        int r = prep();
        if (r) return r;
        FLAME_HIP(hipEventRecord(tm.e0, s));
        r = fn();
        FLAME_HIP(hipEventRecord(tm.e1, s));
        FLAME_HIP(hipEventSynchronize(tm.e1));
        if (r) return r;
        if (check_info) {
            int32_t ih = 0;
            FLAME_HIP(hipMemcpy(&ih, info, sizeof(int32_t), hipMemcpyDeviceToHost));
            if (ih != 0) return FLAME_ERR_BREAKDOWN;
        }
        FLAME_HIP(hipEventElapsedTime(ms_out, tm.e0, tm.e1));
        return FLAME_OK;
    };
    // median of `reps` timed runs after a warm-up (the warm-up alone when it is
    // long); a candidate that fails keeps +inf
    auto median_of = [&](auto &&prep, auto &&fn, bool check_info, double *out) -> int {
        std::vector<double> t;
        for (int r = 0; r <= reps; ++r) {
            float ms = 0.f;
            const int e = timed(prep, fn, check_info, &ms);
            if (e == FLAME_ERR_HIP || e == FLAME_ERR_NOMEM) return e;
            if (e) return FLAME_OK;
            if (r > 0) t.push_back(ms);
            if (r == 0 && ms > kLongRunMs) {
                t.push_back(ms);
                break;
            }
        }
        std::sort(t.begin(), t.end());
        *out = t[t.size() / 2];
        return FLAME_OK;
    };
    auto restore_rhs = [&]() -> int {
        FLAME_HIP(hipMemcpyAsync(x, b0, (size_t)n * esz, hipMemcpyDeviceToDevice, s));
        return FLAME_OK;
    };

    double solve_ms = std::numeric_limits<double>::infinity();  // charged to the batched candidate
    for (int c = 0; c < kC; ++c) {
        const flame_choice_t &k = kClasses[c];
        if (!feasible(c, n, dtype)) continue;
        int e = FLAME_OK;
        if (k.trail != FLAME_TRAIL_NATIVE) {
            flame_mixed_opts_t mo{};
            mo.trail = k.trail;
            mo.nb = k.nb;
            mo.method = k.method;
            mo.max_iter = 3000;
            mo.tol = 1e-13;
            mo.scale = 1;
            mo.max_shifts = 8;
            auto fn = [&]() -> int {
                const int r = flame_solve_mixed(n, 1, static_cast<const double *>(A), lda, (double *)W, n,
                                                (double *)x, n, &mo, nullptr, s);
                return (r == FLAME_OK || r == FLAME_ERR_HIP || r == FLAME_ERR_NOMEM) ? r : FLAME_ERR_BREAKDOWN;
            };
            e = median_of(restore_rhs, fn, false, &times_ms[c]);
        } else if (k.batched) {
            char *bat = ws + oBat;
            int32_t *ns = reinterpret_cast<int32_t *>(ws + oNs);
            int32_t *ldas = reinterpret_cast<int32_t *>(ws + oLd);
            int64_t *ptrs = reinterpret_cast<int64_t *>(ws + oPt);
            hipLaunchKernelGGL(k_batch_arrays, dim3((unsigned)((copies + 255) / 256)), dim3(256), 0, s,
                               (int32_t)copies, (int32_t)n, bat, (int64_t)mat, ns, ldas, ptrs);
            FLAME_CHECK_LAUNCH();
            flame_opts_t bo{};  // graph = 0: direct launch
            auto prep = [&]() -> int {
                for (int64_t i = 0; i < copies; ++i) {
                    const int r = copy_matrix(bat + (size_t)i * mat);
                    if (r) return r;
                }
                return FLAME_OK;
            };
            // info of the first replica stands for all (they are the same matrix)
            auto fn = [&]() -> int {
                return flame_batched_factor(dtype, (int32_t)copies, ns, reinterpret_cast<void *const *>(ptrs), ldas,
                                            info, &bo, s);
            };
            double t = std::numeric_limits<double>::infinity();
            e = median_of(prep, fn, true, &t);
            if (std::isfinite(t) && std::isfinite(solve_ms)) times_ms[c] = t / (double)copies + solve_ms;
        } else {
            flame_opts_t fo{};
            fo.variant = k.variant;
            fo.nb = k.nb;
            fo.flags = k.flags;
            auto prep = [&]() -> int {
                const int r = copy_matrix(W);
                if (r) return r;
                return restore_rhs();
            };
            auto fn = [&]() -> int {
                const int r = flame_factor(dtype, n, W, n, &fo, info, s);
                if (r) return r;
                return flame_solve(dtype, n, 1, W, n, x, n, nullptr, nullptr, s);
            };
            e = median_of(prep, fn, true, &times_ms[c]);
            if (e == FLAME_OK && c == 0 && std::isfinite(times_ms[0])) {
                // the plain solve alone, on the factor just computed
                auto fn2 = [&]() -> int { return flame_solve(dtype, n, 1, W, n, x, n, nullptr, nullptr, s); };
                e = median_of(restore_rhs, fn2, false, &solve_ms);
            }
        }
        if (e) return e;
    }
    int best = -1;
    for (int c = 0; c < kFactorClasses; ++c)
        if (std::isfinite(times_ms[c]) && (best < 0 || times_ms[c] < times_ms[best])) best = c;
    if (best >= 0) {
        std::lock_guard<std::mutex> lk(g_sel.mu);
        g_sel.table[{dtype, n}] = best;
    }
    return FLAME_OK;
}

}  // extern "C"
