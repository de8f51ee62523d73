// Device-wide exclusive scan of uint32 counts (single pass, decoupled
// look-back).  Used to turn per-(bucket, tile) histograms laid out
// bucket-major into global output offsets.
#include "gq_device.h"
#include "gq_internal.h"
#include "gq_ops.h"

namespace {

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

__global__ __launch_bounds__(SC_THREADS) void scan_u32_kernel(uint32_t *data, int64_t n, uint32_t *tile_ctr,
                                                              uint64_t *status)
{
    __shared__ uint32_t smem[SC_THREADS / 64];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_goff;
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    const int64_t base = static_cast<int64_t>(t) * SC_TILE + static_cast<int64_t>(threadIdx.x) * SC_ITEMS;
    uint32_t v[SC_ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        v[i] = (base + i < n) ? data[base + i] : 0u;
        sum += v[i];
    }
    uint32_t total;
    const uint32_t pre = gq_block_exclusive_scan<SC_THREADS>(sum, &total, smem);
    if ((threadIdx.x >> 6) == 0) {
        const uint64_t g = gq_lookback(status, t, total);
        if (gq_lane() == 0) s_goff = g;
    }
    __syncthreads();
    uint32_t run = static_cast<uint32_t>(s_goff) + pre;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        if (base + i < n) data[base + i] = run;
        run += v[i];
    }
}

}  // namespace

size_t gq_scan_u32_workspace(int64_t n)
{
    gq_carver c(nullptr);
    const int64_t tiles = (n + SC_TILE - 1) / SC_TILE;
    c.take<uint32_t>(64);
    c.take<uint64_t>(static_cast<size_t>(tiles > 0 ? tiles : 1));
    return c.bytes();
}

gq_status gq_scan_u32(gq_ctx *ctx, uint32_t *data, int64_t n, void *ws, hipStream_t s)
{
    if (n <= 0) return GQ_OK;
    gq_carver c(ws);
    const int64_t tiles = (n + SC_TILE - 1) / SC_TILE;
    uint32_t *ctr = c.take<uint32_t>(64);
    uint64_t *status = c.take<uint64_t>(static_cast<size_t>(tiles));
    GQ_TRY(gq_zero(ctx, ws, c.off / 4, s));
    return gq_launch(ctx, "gq_scan", scan_u32_kernel, dim3(static_cast<uint32_t>(tiles)), dim3(SC_THREADS), 0, s,
                     data, n, ctr, status);
}
