// flame_batched_factor: argument checks, workspace, and the HIP-graph cache
// of the launch sequence (zero fill, sort by order, persistent factor).
#include <map>
#include <mutex>
#include <tuple>

#include "flame_internal.h"

using namespace flame;

static_assert(FLAME_NOALLOC_MAX_BATCH > 0, "");

namespace {

using BKey = std::tuple<int, int32_t, const void *, const void *, const void *, const void *, void *, hipStream_t, int>;
std::mutex g_bmu;
std::map<BKey, hipGraphExec_t> g_bgraphs;

int run_batched(int32_t dtype, int32_t batch, const int32_t *n, void *const *A, const int32_t *lda, int32_t *info,
                int32_t *ws, hipStream_t s) {
    if (dtype == FLAME_F64) return launch_batched<double>(batch, n, A, lda, info, ws, s);
    return launch_batched<float>(batch, n, A, lda, info, ws, s);
}

// ---- no-allocation variant ------------------------------------------------
// The sort workspace of the batched factorization in a fixed device array,
// one per GPU (each device holds its own copy until the process ends).  Its
// host-side name is not a device address: kernels get the address from
// hipGetSymbolAddress, taken once per device.
constexpr int32_t kNoAllocMaxBatch = FLAME_NOALLOC_MAX_BATCH;
constexpr size_t kScratchInts = (size_t)kNoAllocMaxBatch + 1024 + 2 + 64;  // order + histogram + counter (+ slack)
static __device__ __align__(256) int32_t scratch[kScratchInts];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device), or nullptr with *err set.
int32_t *scratch_for_device(int *err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_last_hip_error(e);
        *err = FLAME_ERR_HIP;
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *err = FLAME_ERR_UNSUPPORTED;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_last_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            *err = FLAME_ERR_HIP;
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<int32_t *>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

namespace flame {
void drop_batched_graphs() {
    std::lock_guard<std::mutex> lk(g_bmu);
    for (auto &kv : g_bgraphs) (void)hipGraphExecDestroy(kv.second);
    g_bgraphs.clear();
}
}  // namespace flame

extern "C" int flame_batched_factor(int32_t dtype, int32_t batch, const int32_t *n, void *const *A,
                                    const int32_t *lda, int32_t *info, const flame_opts_t *opts, void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (batch < 0) return -2;
    if (batch > 0 && n == nullptr) return -3;
    if (batch > 0 && A == nullptr) return -4;
    if (batch > 0 && lda == nullptr) return -5;
    if (batch > 0 && info == nullptr) return -6;
    int graph = 1;
    if (opts != nullptr) {
        if (opts->variant != FLAME_VAR_AUTO && opts->variant != FLAME_VAR_RIGHT) return -7;
        if (opts->graph < 0 || opts->graph > 1) return -7;
        if (opts->trail != FLAME_TRAIL_NATIVE) return -7;
        graph = opts->graph;
    }
    if (batch == 0) return FLAME_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevCtx *ctx = ctx_for_current_device();
    if (ctx == nullptr) return FLAME_ERR_HIP;
    void *w = nullptr;
    int rc = ctx_workspace(ctx, kWsBatched, batched_workspace_ints(batch) * sizeof(int32_t), &w);
    if (rc) return rc;
    int32_t *ws = static_cast<int32_t *>(w);
    if (graph == 0 || s == nullptr) return run_batched(dtype, batch, n, A, lda, info, ws, s);

    // The key holds every pointer the captured kernels use, the workspace
    // included (it only grows, so a cached graph's workspace is never too small).
    int dev = 0;
    FLAME_HIP(hipGetDevice(&dev));
    BKey key{dtype, batch, n, A, lda, info, w, s, dev};
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        auto it = g_bgraphs.find(key);
        if (it != g_bgraphs.end()) {
            FLAME_HIP(hipGraphLaunch(it->second, s));
            return FLAME_OK;
        }
    }
    FLAME_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = run_batched(dtype, batch, n, A, lda, info, ws, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        set_last_hip_error(e);
        return FLAME_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        set_last_hip_error(e);
        return FLAME_ERR_HIP;
    }
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        g_bgraphs[key] = exec;
    }
    FLAME_HIP(hipGraphLaunch(exec, s));
    return FLAME_OK;
}

extern "C" int flame_batched_factor_noalloc(int32_t dtype, int32_t batch, const int32_t *n, void *const *A,
                                            const int32_t *lda, int32_t *info, void *stream) {
    if (dtype != FLAME_F64 && dtype != FLAME_F32) return -1;
    if (batch < 0 || batch > kNoAllocMaxBatch) return -2;
    if (batch > 0 && n == nullptr) return -3;
    if (batch > 0 && A == nullptr) return -4;
    if (batch > 0 && lda == nullptr) return -5;
    if (batch > 0 && info == nullptr) return -6;
    if (batch == 0) return FLAME_OK;
    if (batched_workspace_ints(batch) > kScratchInts) return -2;
    int err = FLAME_OK;
    int32_t *ws = scratch_for_device(&err);
    if (ws == nullptr) return err;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == FLAME_F64) return launch_batched<double>(batch, n, A, lda, info, ws, s, false);
    return launch_batched<float>(batch, n, A, lda, info, ws, s, false);
}
