// Host-side helpers shared by the entry points: the last HIP error seen and a
// per-device cached workspace for calls that pass ws == NULL.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <mutex>
#include <vector>

#include "lhdm.h"

namespace lhdm {

inline thread_local int g_last_hip = 0;

inline void set_last_hip_error(int e) { g_last_hip = e; }

#define HIPCHK(expr)                              \
    do {                                          \
        hipError_t e__ = (expr);                  \
        if (e__ != hipSuccess) {                  \
            ::lhdm::set_last_hip_error((int)e__); \
            return LHDM_EHIP;                     \
        }                                         \
    } while (0)

struct CachedWs {
    int device = -1;
    void* ptr = nullptr;
    size_t bytes = 0;
};

inline std::mutex& ws_mutex() {
    static std::mutex mu;
    return mu;
}

inline std::vector<CachedWs>& ws_cache() {
    static std::vector<CachedWs> v;
    return v;
}

// Library-owned workspace of at least `bytes` on the current device.
inline int cached_workspace(size_t bytes, void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(ws_mutex());
    for (auto& c : ws_cache())
        if (c.device == dev) {
            if (c.bytes < bytes) {
                HIPCHK(hipDeviceSynchronize());
                HIPCHK(hipFree(c.ptr));
                c.ptr = nullptr;
                c.bytes = 0;
                HIPCHK(hipMalloc(&c.ptr, bytes));
                c.bytes = bytes;
            }
            *out = c.ptr;
            return 0;
        }
    CachedWs c;
    c.device = dev;
    HIPCHK(hipMalloc(&c.ptr, bytes));
    c.bytes = bytes;
    ws_cache().push_back(c);
    *out = c.ptr;
    return 0;
}

inline void release_workspaces() {
    std::lock_guard<std::mutex> lk(ws_mutex());
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) cur = 0;
    for (auto& c : ws_cache()) {
        if (!c.ptr) continue;
        (void)hipSetDevice(c.device);
        (void)hipDeviceSynchronize();
        (void)hipFree(c.ptr);
    }
    (void)hipSetDevice(cur);
    ws_cache().clear();
}

// Event timing of the dominant kernel (see lhdm_profile_enable).
struct KernelProfile {
    bool on = false;
    double ms = 0.0;
    long long launches = 0;
    double bytes = 0.0;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, double>> pending;   // (event index of the start, bytes)
    int next = 0;
};

inline KernelProfile& kprof() {
    static KernelProfile k;
    return k;
}

// Record the start event of a timed launch; returns the event slot or -1.
inline int kprof_begin(hipStream_t st) {
    KernelProfile& k = kprof();
    if (!k.on) return -1;
    if (k.pool.empty()) {
        k.pool.resize(2048);
        for (auto& e : k.pool)
            if (hipEventCreate(&e) != hipSuccess) {
                k.pool.clear();
                k.on = false;
                return -1;
            }
    }
    if (k.next + 2 > (int)k.pool.size()) return -1;   // drained at the next synchronisation
    const int i = k.next;
    k.next += 2;
    (void)hipEventRecord(k.pool[i], st);
    return i;
}

// Event slot for a launch that records its own start and stop events
// (hipExtLaunchKernelGGL: no separate event packets on the stream); -1 when off.
inline int kprof_slot() {
    KernelProfile& k = kprof();
    if (!k.on) return -1;
    if (k.pool.empty()) {
        k.pool.resize(2048);
        for (auto& e : k.pool)
            if (hipEventCreate(&e) != hipSuccess) {
                k.pool.clear();
                k.on = false;
                return -1;
            }
    }
    if (k.next + 2 > (int)k.pool.size()) return -1;
    const int i = k.next;
    k.next += 2;
    return i;
}
inline hipEvent_t kprof_event(int i) { return i < 0 ? nullptr : kprof().pool[i]; }
// Register a launch timed through slot i (from kprof_slot).
inline void kprof_commit(int i, double bytes) {
    if (i >= 0) kprof().pending.push_back({i, bytes});
}

inline void kprof_end(hipStream_t st, int i, double bytes) {
    KernelProfile& k = kprof();
    if (i < 0) return;
    (void)hipEventRecord(k.pool[i + 1], st);
    k.pending.push_back({i, bytes});
}

// Called once the stream has passed the recorded events (a wait for the end
// event is then immediate).
inline void kprof_drain() {
    KernelProfile& k = kprof();
    for (auto& pr : k.pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(k.pool[pr.first + 1]);
        if (hipEventElapsedTime(&ms, k.pool[pr.first], k.pool[pr.first + 1]) == hipSuccess) {
            k.ms += ms;
            k.launches += 1;
            k.bytes += pr.second;
        }
    }
    k.pending.clear();
    k.next = 0;
}

// kprof_drain once half of the event pool is taken: for waits on the host's
// critical path (two event calls per timed launch), the rest drained at the end.
inline void kprof_drain_if_half() {
    KernelProfile& k = kprof();
    if (!k.pending.empty() && 2 * k.next >= (int)k.pool.size()) kprof_drain();
}

}  // namespace lhdm
