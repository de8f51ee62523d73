// Context, status word, per-kernel event timing and the zero-fill kernel.
#include <cstdio>
#include <cstring>

#include "gq_device.h"
#include "gq_internal.h"
#include "gq_ops.h"

gq_status gq_fail(gq_ctx *ctx, gq_status code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

hipEvent_t gq_take_event(gq_ctx *ctx)
{
    if (!ctx->free_events.empty()) {
        hipEvent_t e = ctx->free_events.back();
        ctx->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

__global__ void gq_zero_kernel(uint32_t *p, size_t words)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0;
}

gq_status gq_zero(gq_ctx *ctx, void *p, size_t words, hipStream_t stream)
{
    if (words == 0) return GQ_OK;
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    return gq_launch(ctx, "gq_zero", gq_zero_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream,
                     static_cast<uint32_t *>(p), words);
}

extern "C" {

gq_status gq_ctx_create(int device, gq_ctx **out)
{
    if (!out) return GQ_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GQ_ERR_INVALID_ARG;
    gq_ctx *ctx = new gq_ctx();
    ctx->device = device;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return GQ_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->num_cus = prop.multiProcessorCount;
        ctx->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
    }
    if (hipMalloc(&ctx->status_dev, 256) != hipSuccess ||
        hipMemset(ctx->status_dev, 0, 256) != hipSuccess || gq_filter_scratch_setup(ctx) != GQ_OK) {
        if (ctx->status_dev) (void)hipFree(ctx->status_dev);
        (void)hipSetDevice(prev);
        delete ctx;
        return GQ_ERR_HIP;
    }
    (void)hipSetDevice(prev);
    *out = ctx;
    return GQ_OK;
}

void gq_ctx_destroy(gq_ctx *ctx)
{
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    for (auto &r : ctx->pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    if (ctx->status_dev) (void)hipFree(ctx->status_dev);
    delete ctx;
}

const char *gq_last_error(const gq_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

gq_status gq_status_word(gq_ctx *ctx, gq_stream stream, gq_status *out)
{
    if (!ctx || !out) return GQ_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t bits = 0;
    GQ_CHECK_HIP(ctx, hipMemcpyAsync(&bits, ctx->status_dev, sizeof bits, hipMemcpyDeviceToHost, s));
    GQ_CHECK_HIP(ctx, hipStreamSynchronize(s));
    *out = gq_status_of_bits(bits);
    if (bits) {
        GQ_TRY(gq_zero(ctx, ctx->status_dev, 1, s));
        GQ_CHECK_HIP(ctx, hipStreamSynchronize(s));
    }
    return GQ_OK;
}

gq_status gq_set_wait_limit(gq_ctx *ctx, int64_t polls)
{
    if (!ctx || polls < 0) return GQ_ERR_INVALID_ARG;
    ctx->wait_limit = polls == 0 ? (int64_t(1) << 24) : polls - 1;
    return GQ_OK;
}

gq_status gq_set_timing(gq_ctx *ctx, int enable)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    ctx->timing = enable != 0;
    return GQ_OK;
}

static gq_status collect(gq_ctx *ctx)
{
    if (ctx->pending.empty()) return GQ_OK;
    GQ_CHECK_HIP(ctx, hipDeviceSynchronize());
    for (auto &r : ctx->pending) {
        float ms = 0.f;
        GQ_CHECK_HIP(ctx, hipEventElapsedTime(&ms, r.start, r.stop));
        auto &t = ctx->totals[r.name];
        t.first += 1;
        t.second += ms;
        ctx->free_events.push_back(r.start);
        ctx->free_events.push_back(r.stop);
    }
    ctx->pending.clear();
    return GQ_OK;
}

gq_status gq_kernel_time(gq_ctx *ctx, const char *name, int64_t *launches, double *total_ms)
{
    if (!ctx || !name || !launches || !total_ms) return GQ_ERR_INVALID_ARG;
    GQ_TRY(collect(ctx));
    auto it = ctx->totals.find(name);
    *launches = it == ctx->totals.end() ? 0 : it->second.first;
    *total_ms = it == ctx->totals.end() ? 0.0 : it->second.second;
    return GQ_OK;
}

gq_status gq_reset_timing(gq_ctx *ctx)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    GQ_TRY(collect(ctx));
    ctx->totals.clear();
    return GQ_OK;
}

}  // extern "C"
