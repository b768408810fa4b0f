// Plan objects behind the opaque mxs_plan handle, and helpers of the C ABI.
#pragma once

#include "mxs_internal.h"
#include "mxsten.h"

#include <stddef.h>

enum PlanKind { KIND_STENCIL2D = 1, KIND_STENCIL1D = 2, KIND_SOLVE = 3, KIND_CH = 4, KIND_WENO = 5, KIND_FN = 6 };

struct mxs_plan_s {
    int kind;
    explicit mxs_plan_s(int k) : kind(k) {}
    virtual ~mxs_plan_s() {}
    virtual mxs_status compute(hipStream_t) { return MXS_ERR_BAD_HANDLE; }
    virtual mxs_status swap() { return MXS_ERR_BAD_HANDLE; }
    virtual mxs_status rebind(const void *, void *) { return MXS_ERR_BAD_HANDLE; }
    virtual mxs_status autotune(hipStream_t) { return MXS_OK; }
    virtual void info(char *buf, int len) const;
};

namespace mxs {

// Device allocation owned by a plan.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) {
        o.ptr = nullptr;
        o.bytes = 0;
    }
    ~DevBuf();
    void reset();
    hipError_t alloc(size_t n);
    hipError_t upload(const void *src, size_t n);
};

// Memory-side cache (MALL) of the device, and the buffer written to flush it
// when layouts are timed on cold caches.
constexpr size_t kMallBytes = size_t(256) << 20;
constexpr size_t kFlushBytes = size_t(512) << 20;

mxs_status fail(mxs_status st, const char *fmt, ...);
mxs_status hip_fail(hipError_t e, const char *what);
void register_plan(const mxs_plan_s *p);
bool unregister_plan(const mxs_plan_s *p);
bool is_live(const mxs_plan_s *p);
bool ranges_overlap(const void *a, size_t abytes, const void *b, size_t bbytes);
size_t grid_bytes(int nx, int ny, long long ld, int dtype);
int device_lds_limit();
int device_cu_count();
bool valid_dtype(int d);

// Average time in seconds of `reps` calls of fn on stream s (after `warm`
// untimed calls); negative on a launch error.
template <class F> double time_launches(F &&fn, hipStream_t s, int warm, int reps) {
    for (int i = 0; i < warm; ++i)
        if (fn() != hipSuccess) return -1.0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double r = -1.0;
    if (hipEventRecord(e0, s) == hipSuccess) {
        bool ok = true;
        for (int i = 0; i < reps && ok; ++i) ok = fn() == hipSuccess;
        float ms = 0;
        if (ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            r = ms * 1e-3 / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
}

// Average time of single launches of fn, each started with the memory-side
// cache (MALL) holding other data: before every timed launch the stream
// reads flush (flush_bytes, larger than that cache; reads leave no dirty
// lines to be written back during the timed launch).  For plans whose
// data exceed the cache, so that each candidate layout meets the cold
// caches that back-to-back launches over many buffers meet.
template <class F>
double time_launches_cold(F &&fn, hipStream_t s, int warm, int reps, void *flush, size_t flush_bytes) {
    for (int i = 0; i < warm; ++i)
        if (fn() != hipSuccess) return -1.0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double total = 0.0;
    bool ok = true;
    for (int i = 0; i < reps && ok; ++i) {
        float ms = 0;
        ok = launch_cache_flush(flush, flush_bytes, s) == hipSuccess && hipEventRecord(e0, s) == hipSuccess &&
             fn() == hipSuccess && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        total += ms * 1e-3;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ok ? total / reps : -1.0;
}

}  // namespace mxs
