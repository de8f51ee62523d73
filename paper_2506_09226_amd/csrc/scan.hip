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

gq_status gq_scan_u32(gq_ctx *ctx, uint32_t *data, int64_t n, void *ws, hipStream_t s, const char *name)
{
    if (n <= 0) return GQ_OK;
    gq_carver c(ws);
    const int64_t tiles = (n + SC_TILE - 1) / SC_TILE;
    uint32_t *ctr = c.take<uint32_t>(64);
    uint64_t *status = c.take<uint64_t>(static_cast<size_t>(tiles));
    GQ_TRY(gq_zero(ctx, ws, c.off / 4, s));
    return gq_launch(ctx, name, scan_u32_kernel, dim3(static_cast<uint32_t>(tiles)), dim3(SC_THREADS), 0, s,
                     data, n, ctr, status);
}

// ---------------------------------------------------------------------------
// Run offsets from per-tile bucket counts in TILE-MAJOR layout (the counts of
// one tile are contiguous, so a histogram kernel writes them, and a scatter
// kernel reads its tile's P offsets, as one coalesced row):
//
//   off[t*P + b] = start[b] + sum_{t' < t} cnt[t'*P + b],
//   start[b]     = sum_{b' < b} total[b'],   start[P] = sum of all counts.
//
// Four small kernels, every access coalesced across buckets: per-chunk column
// sums, a scan of those sums down each column, an exclusive scan of the bucket
// totals, and the final per-tile offsets.  A chunk is 32 to 256 tiles, sized
// for about 192 chunks: enough workgroups for the two column passes, and a
// short walk down each column for the one-workgroup scan between them.
// ---------------------------------------------------------------------------
namespace {

constexpr int TO_THREADS = 256;
constexpr int TO_MAX_P = 8192;
constexpr int TO_START_THREADS = 1024;

// Column loops load TO_BATCH counts into registers before using them, so a
// thread keeps that many independent loads in flight.
constexpr int TO_BATCH = 32;

int64_t to_chunk_tiles(int64_t ntiles)
{
    int64_t c = 32;
    while (c < 256 && c * 192 < ntiles) c *= 2;
    return c;
}

// Tiles that hold counts: all ntiles, or those the device row count reaches.
GQ_DEV int64_t to_live_tiles(int64_t ntiles, gq_tile_count live)
{
    if (!live.n_dev) return ntiles;
    int64_t n = *live.n_dev;
    n = n < 0 ? 0 : (n < live.n_bound ? n : live.n_bound);
    const int64_t t = (n + live.tile_rows - 1) / live.tile_rows;
    return t < ntiles ? t : ntiles;
}

__global__ __launch_bounds__(TO_THREADS) void to_chunk_sum_kernel(const uint32_t *__restrict__ cnt, int64_t ntiles,
                                                                  int P, int64_t chunk, uint32_t *__restrict__ csum,
                                                                  gq_tile_count live)
{
    ntiles = to_live_tiles(ntiles, live);
    const int64_t c = blockIdx.x;
    const int b = blockIdx.y * TO_THREADS + threadIdx.x;
    if (b >= P) return;
    const int64_t t0 = c * chunk;
    const int64_t t1 = t0 + chunk < ntiles ? t0 + chunk : ntiles;
    uint32_t s = 0;
    for (int64_t t = t0; t < t1; t += TO_BATCH) {
        uint32_t x[TO_BATCH];
#pragma unroll
        for (int i = 0; i < TO_BATCH; ++i) x[i] = t + i < t1 ? cnt[(t + i) * P + b] : 0u;
#pragma unroll
        for (int i = 0; i < TO_BATCH; ++i) s += x[i];
    }
    csum[c * P + b] = s;
}

__global__ __launch_bounds__(TO_THREADS) void to_chunk_scan_kernel(uint32_t *__restrict__ csum, int64_t nchunks,
                                                                   int P, uint32_t *__restrict__ total)
{
    const int b = blockIdx.x * TO_THREADS + threadIdx.x;
    if (b >= P) return;
    uint32_t run = 0;
    for (int64_t c = 0; c < nchunks; c += TO_BATCH) {
        uint32_t x[TO_BATCH];
#pragma unroll
        for (int i = 0; i < TO_BATCH; ++i) x[i] = c + i < nchunks ? csum[(c + i) * P + b] : 0u;
#pragma unroll
        for (int i = 0; i < TO_BATCH; ++i) {
            if (c + i < nchunks) csum[(c + i) * P + b] = run;
            run += x[i];
        }
    }
    total[b] = run;
}

// Exclusive scan of the P bucket totals (one workgroup; each thread owns
// P / 1024 consecutive buckets).
__global__ __launch_bounds__(TO_START_THREADS) void to_bucket_start_kernel(const uint32_t *__restrict__ total, int P,
                                                                           uint32_t *__restrict__ start)
{
    __shared__ uint32_t smem[TO_START_THREADS / 64];
    const int per = (P + TO_START_THREADS - 1) / TO_START_THREADS;
    const int b0 = threadIdx.x * per;
    uint32_t v = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < P) v += total[b0 + i];
    uint32_t all;
    uint32_t run = gq_block_exclusive_scan<TO_START_THREADS>(v, &all, smem);
    for (int i = 0; i < per; ++i)
        if (b0 + i < P) {
            start[b0 + i] = run;
            run += total[b0 + i];
        }
    if (threadIdx.x == 0) start[P] = all;
}

__global__ __launch_bounds__(TO_THREADS) void to_final_kernel(uint32_t *__restrict__ cnt, int64_t ntiles, int P,
                                                              int64_t chunk, const uint32_t *__restrict__ csum,
                                                              const uint32_t *__restrict__ start, gq_tile_count live)
{
    ntiles = to_live_tiles(ntiles, live);
    const int64_t c = blockIdx.x;
    const int b = blockIdx.y * TO_THREADS + threadIdx.x;
    if (b >= P) return;
    const int64_t t0 = c * chunk;
    const int64_t t1 = t0 + chunk < ntiles ? t0 + chunk : ntiles;
    uint32_t run = start[b] + csum[c * P + b];
    for (int64_t t = t0; t < t1; t += TO_BATCH) {
        uint32_t x[TO_BATCH];
#pragma unroll
        for (int i = 0; i < TO_BATCH; ++i) x[i] = t + i < t1 ? cnt[(t + i) * P + b] : 0u;
#pragma unroll
        for (int i = 0; i < TO_BATCH; ++i) {
            if (t + i < t1) cnt[(t + i) * P + b] = run;
            run += x[i];
        }
    }
}

}  // namespace

size_t gq_tile_offsets_workspace(int64_t ntiles, int P)
{
    gq_carver c(nullptr);
    const int64_t chunk = to_chunk_tiles(ntiles);
    const int64_t nchunks = (ntiles + chunk - 1) / chunk;
    c.take<uint32_t>(static_cast<size_t>((nchunks > 0 ? nchunks : 1) * P));
    c.take<uint32_t>(static_cast<size_t>(P));
    return c.bytes();
}

gq_status gq_tile_offsets(gq_ctx *ctx, uint32_t *cnt, int64_t ntiles, int P, uint32_t *start, void *ws,
                          hipStream_t s, const char *name, const gq_tile_count *live)
{
    const gq_tile_count lv = live ? *live : gq_tile_count{nullptr, 0, 1};
    if (live && live->tile_rows < 1) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_tile_offsets: bad tile rows");
    if (P < 1 || P > TO_MAX_P || ntiles < 1) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_tile_offsets: bad shape");
    gq_carver c(ws);
    const int64_t chunk = to_chunk_tiles(ntiles);
    const int64_t nchunks = (ntiles + chunk - 1) / chunk;
    uint32_t *csum = c.take<uint32_t>(static_cast<size_t>(nchunks * P));
    uint32_t *total = c.take<uint32_t>(static_cast<size_t>(P));
    const dim3 grid2(static_cast<uint32_t>(nchunks), static_cast<uint32_t>((P + TO_THREADS - 1) / TO_THREADS));
    const dim3 grid1(static_cast<uint32_t>((P + TO_THREADS - 1) / TO_THREADS));
    GQ_TRY(gq_launch(ctx, name, to_chunk_sum_kernel, grid2, dim3(TO_THREADS), 0, s,
                     static_cast<const uint32_t *>(cnt), ntiles, P, chunk, csum, lv));
    GQ_TRY(gq_launch(ctx, name, to_chunk_scan_kernel, grid1, dim3(TO_THREADS), 0, s, csum, nchunks, P, total));
    GQ_TRY(gq_launch(ctx, name, to_bucket_start_kernel, dim3(1), dim3(TO_START_THREADS), 0, s,
                     static_cast<const uint32_t *>(total), P, start));
    return gq_launch(ctx, name, to_final_kernel, grid2, dim3(TO_THREADS), 0, s, cnt, ntiles, P, chunk,
                     static_cast<const uint32_t *>(csum), static_cast<const uint32_t *>(start), lv);
}
