// Host-side internals shared by the operator sources: the context, error
// reporting, kernel launch with optional event timing, and workspace layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "gq.h"

struct gq_timing_rec {
    std::string name;
    hipEvent_t start;
    hipEvent_t stop;
};

struct gq_ctx {
    int device = 0;
    int num_cus = 256;
    size_t lds_per_cu = 160 * 1024;
    uint32_t *status_dev = nullptr;          // bit (1 << code) per device error
    int64_t wait_limit = int64_t(1) << 24;   // polls of a bounded device-side wait
    void *filter_scratch = nullptr;          // device address of gq_filter_noalloc's scratch
    std::string last_error;
    bool timing = false;
    std::vector<gq_timing_rec> pending;      // recorded, not yet collected
    std::map<std::string, std::pair<int64_t, double>> totals;
    std::vector<hipEvent_t> free_events;
};

gq_status gq_fail(gq_ctx *ctx, gq_status code, const char *fmt, ...);
hipEvent_t gq_take_event(gq_ctx *ctx);

#define GQ_CHECK_HIP(ctx, expr)                                                          \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return gq_fail((ctx), GQ_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

#define GQ_TRY(expr)                      \
    do {                                  \
        gq_status s_ = (expr);            \
        if (s_ != GQ_OK) return s_;       \
    } while (0)

// Launch `kernel` on `stream`; with timing on, bracket it with events that are
// recorded on that same stream and attributed to `name`.
template <typename Kernel, typename... Args>
gq_status gq_launch(gq_ctx *ctx, const char *name, Kernel kernel, dim3 grid, dim3 block, size_t shmem,
                    hipStream_t stream, Args... args)
{
    if (grid.x == 0) return GQ_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        e0 = gq_take_event(ctx);
        e1 = gq_take_event(ctx);
        if (!e0 || !e1) return gq_fail(ctx, GQ_ERR_HIP, "hipEventCreate failed");
        GQ_CHECK_HIP(ctx, hipEventRecord(e0, stream));
    }
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, args...);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return gq_fail(ctx, GQ_ERR_HIP, "launch of %s: %s", name, hipGetErrorString(err));
    if (ctx->timing) {
        GQ_CHECK_HIP(ctx, hipEventRecord(e1, stream));
        ctx->pending.push_back({name, e0, e1});
    }
    return GQ_OK;
}

// Workspace layout: the same sequence of take() calls computes the size (with
// base == nullptr) and hands out the pieces (with the caller's buffer).
struct gq_carver {
    char *base;
    size_t off = 0;
    explicit gq_carver(void *b) : base(static_cast<char *>(b)) {}
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// Fill `words` 32-bit words with zero (a kernel, so that it can be captured
// into a graph, unlike a memset node).
gq_status gq_zero(gq_ctx *ctx, void *p, size_t words, hipStream_t stream);

constexpr int64_t GQ_MAX_ROWS = 2147483647LL;
