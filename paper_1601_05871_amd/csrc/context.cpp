// Per-device library state: a second stream for lookahead, events, a grow-only
// workspace.  Created lazily on the first call on a device and kept until the
// process ends.
#include <mutex>
#include <vector>

#include "flame_internal.h"

namespace flame {

static thread_local hipError_t g_last_hip = hipSuccess;
void set_last_hip_error(hipError_t e) { g_last_hip = e; }
hipError_t last_hip_error() { return g_last_hip; }

struct DevCtx {
    int device = -1;
    hipStream_t side = nullptr;
    hipStream_t aux = nullptr;  // selector inference (never captured)
    std::vector<hipEvent_t> events;
    void *ws[kWsSlots] = {};
    size_t ws_bytes[kWsSlots] = {};
    uint64_t ws_gen[kWsSlots] = {};  // bumped whenever a slot's buffer is replaced
    std::mutex mu;
};

static std::mutex g_mu;
static std::vector<DevCtx *> g_ctx;

DevCtx *ctx_for_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_ctx.size() <= dev) g_ctx.resize(dev + 1, nullptr);
    if (g_ctx[dev] == nullptr) {
        DevCtx *c = new DevCtx();
        c->device = dev;
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return nullptr;
        }
        c->events.resize(4, nullptr);
        for (auto &e : c->events) {
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                delete c;
                return nullptr;
            }
        }
        g_ctx[dev] = c;
    }
    return g_ctx[dev];
}

hipStream_t ctx_side_stream(DevCtx *c) { return c->side; }
hipStream_t ctx_aux_stream(DevCtx *c) { return c->aux; }
hipEvent_t ctx_event(DevCtx *c, int i) { return c->events[i]; }

int ctx_workspace(DevCtx *c, int slot, size_t bytes, void **out) {
    std::lock_guard<std::mutex> lk(c->mu);
    if (bytes > c->ws_bytes[slot]) {
        // The old buffer may still be in use by enqueued work on any stream.
        if (c->ws[slot] != nullptr) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) {
                set_last_hip_error(e);
                return FLAME_ERR_HIP;
            }
            hipFree(c->ws[slot]);
            c->ws[slot] = nullptr;
            c->ws_bytes[slot] = 0;
        }
        size_t want = (bytes + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
        hipError_t e = hipMalloc(&c->ws[slot], want);
        if (e != hipSuccess) {
            set_last_hip_error(e);
            c->ws[slot] = nullptr;
            return FLAME_ERR_NOMEM;
        }
        c->ws_bytes[slot] = want;
        c->ws_gen[slot] += 1;
    }
    *out = c->ws[slot];
    return FLAME_OK;
}

uint64_t ctx_workspace_gen(DevCtx *c, int slot) {
    std::lock_guard<std::mutex> lk(c->mu);
    return c->ws_gen[slot];
}

// Releases every device's state: waits for the device, then destroys the
// cached graphs, streams and events and frees the workspaces.  Contexts are
// re-created lazily by the next call.
int shutdown_all() {
    {
        // nothing to release (and no HIP call) if no device was ever used
        std::lock_guard<std::mutex> lk(g_mu);
        bool any = false;
        for (DevCtx *c : g_ctx) any = any || (c != nullptr);
        if (!any) return FLAME_OK;
    }
    int rc = FLAME_OK;
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    drop_factor_graphs();
    drop_batched_graphs();
    drop_dag_lists();
    selector_forget_devices();
    std::lock_guard<std::mutex> lk(g_mu);
    for (DevCtx *c : g_ctx) {
        if (c == nullptr) continue;
        if (hipSetDevice(c->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) rc = FLAME_ERR_HIP;
        for (auto &e : c->events)
            if (e) (void)hipEventDestroy(e);
        if (c->side) (void)hipStreamDestroy(c->side);
        if (c->aux) (void)hipStreamDestroy(c->aux);
        for (int k = 0; k < kWsSlots; ++k)
            if (c->ws[k]) (void)hipFree(c->ws[k]);
        delete c;
    }
    g_ctx.clear();
    if (have_cur) (void)hipSetDevice(cur);
    return rc;
}

}  // namespace flame

extern "C" int flame_shutdown(void) { return flame::shutdown_all(); }
