// Learned selector (weights, feature rows, inference through the HIP MLP
// kernel), the exhaustive autotuner and its tuning table, and the choice used
// by FLAME_VAR_AUTO.
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

struct SelState {
    std::mutex mu;
    std::vector<float> weights;  // host copy; empty = not loaded
    std::map<int, bool> on_device;  // device -> weights uploaded to its workspace
    std::map<int, uint64_t> gen;    // device -> generation of the workspace holding them
    std::map<std::tuple<int32_t, int64_t, int64_t>, std::pair<int32_t, int32_t>> memo;  // (dtype, n, batch)
    std::map<std::pair<int32_t, int64_t>, int32_t> table;  // autotuner: (dtype, n) -> class
};
SelState g_sel;

void class_to_choice(int c, int32_t *variant, int32_t *nb) {
    *variant = 1 + c / 4;
    *nb = 32 << (c % 4);
}

void features(int64_t n, int64_t batch, int32_t dtype, double kappa, float *f) {
    f[0] = (float)std::log2((double)std::max<int64_t>(n, 1));
    f[1] = (float)std::log2((double)std::max<int64_t>(batch, 1));
    f[2] = dtype == FLAME_F64 ? 1.0f : 0.0f;
    f[3] = dtype == FLAME_F32 ? 1.0f : 0.0f;
    f[4] = (float)std::log10(std::max(kappa, 1.0));
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

int argmax(const float *l) {
    int best = 0;
    for (int c = 1; c < kC; ++c)
        if (l[c] > l[best]) best = c;
    return best;
}

}  // namespace

namespace flame {

void selector_forget_devices() {
    std::lock_guard<std::mutex> lk(g_sel.mu);
    g_sel.on_device.clear();
    g_sel.gen.clear();
}

void choose_variant(int32_t dtype, int64_t n, int64_t batch, int32_t *variant, int32_t *nb) {
    if (flame_select(n, batch, dtype, 0.0, variant, nb) == FLAME_OK) return;
    std::lock_guard<std::mutex> lk(g_sel.mu);
    // autotuner table: the tuned order of this dtype nearest to n (log scale)
    int best = -1;
    double dist = std::numeric_limits<double>::infinity();
    for (const auto &kv : g_sel.table) {
        if (kv.first.first != dtype) continue;
        const double d = std::fabs(std::log2((double)std::max<int64_t>(kv.first.second, 1)) -
                                   std::log2((double)std::max<int64_t>(n, 1)));
        if (d < dist) {
            dist = d;
            best = kv.second;
        }
    }
    if (best >= 0 && dist <= 0.5) {
        class_to_choice(best, variant, nb);
        return;
    }
    *variant = FLAME_VAR_RIGHT;
    *nb = 256;
}

}  // namespace flame

extern "C" {

int flame_selector_load(const float *w, int64_t count) {
    if (w == nullptr && count == 0) {  // unload
        std::lock_guard<std::mutex> lk(g_sel.mu);
        g_sel.weights.clear();
        g_sel.on_device.clear();
        g_sel.memo.clear();
        return FLAME_OK;
    }
    if (w == nullptr) return -1;
    if (count != FLAME_SEL_NPARAM) return -2;
    std::lock_guard<std::mutex> lk(g_sel.mu);
    g_sel.weights.assign(w, w + count);
    g_sel.on_device.clear();
    g_sel.memo.clear();
    return FLAME_OK;
}

int flame_select(int64_t n, int64_t batch, int32_t dtype, double kappa, int32_t *variant, int32_t *nb) {
    if (n < 0) return -1;
    if (batch < 0) return -2;
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -3;
    if (!(kappa >= 0.0)) return -4;
    if (variant == nullptr) return -5;
    if (nb == nullptr) return -6;
    std::lock_guard<std::mutex> lk(g_sel.mu);
    if (g_sel.weights.empty()) return FLAME_ERR_UNSUPPORTED;
    const auto key = std::make_tuple(dtype, n, batch);
    if (kappa == 0.0) {
        auto it = g_sel.memo.find(key);
        if (it != g_sel.memo.end()) {
            *variant = it->second.first;
            *nb = it->second.second;
            return FLAME_OK;
        }
    }
    float f[kF], l[kC];
    features(n, batch, dtype, kappa, f);
    int rc = logits_locked(f, 1, l);
    if (rc) return rc;
    class_to_choice(argmax(l), variant, nb);
    if (kappa == 0.0) g_sel.memo[key] = {*variant, *nb};
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

int flame_autotune(int32_t dtype, int64_t n, void *A, int64_t lda, int32_t reps, double *times_ms, void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (n < 0) return -2;
    if (A == nullptr && n > 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (reps < 1) return -5;
    if (times_ms == nullptr) return -6;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int c = 0; c < kC; ++c) times_ms[c] = std::numeric_limits<double>::infinity();
    if (n == 0) return FLAME_OK;
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    const size_t esz = dtype == FLAME_F64 ? 8 : 4;
    const size_t mat = (size_t)n * (size_t)n * esz;
    void *base = nullptr;
    int rc = ctx_workspace(ctx, kWsTune, mat + 256, &base);
    if (rc) return rc;
    char *W = static_cast<char *>(base);
    int32_t *info = nullptr;
    FLAME_HIP(hipMalloc(&info, sizeof(int32_t)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FLAME_HIP(hipEventCreate(&e0));
    FLAME_HIP(hipEventCreate(&e1));
    auto restore = [&]() -> int {
        FLAME_HIP(hipMemcpy2DAsync(W, (size_t)n * esz, A, (size_t)lda * esz, (size_t)n * esz, (size_t)n,
                                   hipMemcpyDeviceToDevice, s));
        return FLAME_OK;
    };
    int status = FLAME_OK;
    for (int c = 0; c < kC && status == FLAME_OK; ++c) {
        flame_opts_t o;
        std::memset(&o, 0, sizeof(o));
        int32_t v = 0, nb = 0;
        class_to_choice(c, &v, &nb);
        o.variant = v;
        o.nb = nb;
        std::vector<double> t;
        bool failed = false;
        for (int r = 0; r <= reps && !failed; ++r) {  // r == 0: warm-up
            if ((status = restore()) != FLAME_OK) break;
            FLAME_HIP(hipEventRecord(e0, s));
            int frc = flame_factor(dtype, n, W, n, &o, info, s);
            FLAME_HIP(hipEventRecord(e1, s));
            FLAME_HIP(hipEventSynchronize(e1));
            int32_t ih = 0;
            FLAME_HIP(hipMemcpy(&ih, info, sizeof(int32_t), hipMemcpyDeviceToHost));
            if (frc != FLAME_OK || ih != 0) {
                failed = true;
                break;
            }
            float ms = 0.0f;
            FLAME_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (r > 0) t.push_back(ms);
        }
        if (!failed && !t.empty()) {
            std::sort(t.begin(), t.end());
            times_ms[c] = t[t.size() / 2];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(info);
    if (status != FLAME_OK) return status;
    int best = 0;
    for (int c = 1; c < kC; ++c)
        if (times_ms[c] < times_ms[best]) best = c;
    if (std::isfinite(times_ms[best])) {
        std::lock_guard<std::mutex> lk(g_sel.mu);
        g_sel.table[{dtype, n}] = best;
    }
    return FLAME_OK;
}

}  // extern "C"
