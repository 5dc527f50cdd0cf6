// Flags between the workgroups of one launch (the persistent solves and the
// by-blocks task DAG).
//
// gfx950 has one L2 per XCD, not coherent with the others for ordinary
// stores: a release at device scope writes back the XCD's whole L2 (every
// dirty line, also other workgroups'), an acquire invalidates it.  Both are
// costly when a launch publishes a block every few microseconds, and an
// acquire per spin of a wait also throws away what the other workgroups of
// the XCD have cached.  So:
//   - data that another workgroup waits for is written with device-scope
//     stores (store_dev), which go through to the device's coherence point;
//     once each wavefront has waited for its stores (wait_stores) and the
//     workgroup has passed a barrier, the flag is set with a device-scope
//     store of its own (no write-back needed);
//   - a waiting thread polls the flag with device-scope loads, which read the
//     coherence point, and invalidates its caches once, after the flag has
//     been seen (acquire_dev, by every wavefront that then reads the data
//     with ordinary loads; device-scope loads of the data need none).
#pragma once

#include <hip/hip_runtime.h>

namespace flame {

__device__ __forceinline__ int32_t load_dev(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_dev(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_dev(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_dev(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// This wavefront's stores (and loads) have completed.
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Invalidates this wavefront's view of device memory (acquire at device scope).
__device__ __forceinline__ void acquire_dev() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Waits (bounded) until *p >= want.  Gives up when *stop becomes nonzero
// (returns false) or after `cap` sleep rounds (sets *stop to `give_up_code`
// and returns false).  No acquire: the caller takes acquire_dev after the
// barrier that follows.
__device__ __forceinline__ bool poll_at_least(const int32_t *p, int32_t want, int32_t *stop, int32_t give_up_code,
                                              long long cap) {
    long long spins = 0;
    while (load_dev(p) < want) {
        if (load_dev(stop) != 0) return false;
        if (++spins > cap) {
            store_dev(stop, give_up_code);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

}  // namespace flame
