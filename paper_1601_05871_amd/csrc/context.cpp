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
    }
    *out = c->ws[slot];
    return FLAME_OK;
}

}  // namespace flame
