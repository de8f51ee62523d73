// Scan + filter: ordered stream compaction of a range predicate.
//
// One pass over the column.  A workgroup takes FT_GROUP consecutive tiles of
// FT_TILE rows with one dequeue.  Each tile is read with coalesced loads (wave
// w, step c reads rows c*256 + w*64 + lane) and each wave's ballot becomes one
// 64-bit word of the tile's bitmap in LDS.  The group's match count goes
// through a decoupled look-back over groups, which gives its global offset;
// then, tile by tile, each thread owns 32 consecutive rows of the bitmap, a
// block scan gives output slots, and the compacted row ids are staged in LDS
// and written out contiguously.
#include "gq_device.h"
#include "gq_internal.h"

namespace {

constexpr int FT_THREADS = 512;
constexpr int FT_ITEMS = 16;
constexpr int FT_TILE = FT_THREADS * FT_ITEMS;     // 8192 rows
constexpr int FT_RPT = FT_TILE / FT_THREADS;       // rows of a tile each thread owns in the write-out (16)
constexpr int FT_TPW = 64 / FT_RPT;                // threads per bitmap word
constexpr int FT_WORDS = FT_TILE / 64;              // 128 bitmap words
constexpr int FT_GROUP = 4;                         // tiles per dequeue

struct filter_ws {
    uint32_t *tile_ctr;
    uint64_t *status;
};

// A dequeue counter, then one look-back status word per group of FT_GROUP tiles.
filter_ws filter_layout(gq_carver &c, int64_t n)
{
    filter_ws w;
    const int64_t tiles = (n + FT_TILE - 1) / FT_TILE;
    const int64_t groups = (tiles + FT_GROUP - 1) / FT_GROUP;
    w.tile_ctr = c.take<uint32_t>(64);
    w.status = c.take<uint64_t>(static_cast<size_t>(groups > 0 ? groups : 1));
    return w;
}

template <typename T, bool HAS_SEL>
__global__ __launch_bounds__(FT_THREADS) void filter_kernel(const T *__restrict__ col,
                                                            const int32_t *__restrict__ sel_in,
                                                            int64_t n_bound, const int64_t *n_dev, int64_t lo,
                                                            int64_t hi, int32_t *__restrict__ out,
                                                            int64_t *n_out, uint32_t *tile_ctr, uint64_t *status)
{
    __shared__ uint64_t bits[FT_GROUP][FT_WORDS];
    __shared__ int32_t stage[FT_TILE];
    __shared__ uint32_t scan_smem[FT_THREADS / 64];
    __shared__ uint32_t s_group;
    __shared__ uint64_t s_goff;

    int64_t n = n_bound;
    if (n_dev) {
        const int64_t d = *n_dev;
        n = d < n_bound ? (d > 0 ? d : 0) : n_bound;
    }
    const int64_t ntiles = (n + FT_TILE - 1) / FT_TILE;
    const int64_t ngroups = (ntiles + FT_GROUP - 1) / FT_GROUP;
    if (ntiles == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = 0;
        return;
    }
    // One dequeue per group of FT_GROUP consecutive tiles (atomics on one
    // address serialize chip-wide).  The group is one unit of the look-back:
    // its bitmaps are built first, its match count is published, and only
    // then does it wait for its predecessors (groups are numbered in dequeue
    // order, so each predecessor is done or held by a running workgroup).
    if (threadIdx.x == 0) s_group = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const int64_t g = s_group;
    if (g >= ngroups) return;                              // same value in every thread
    const int64_t t0 = g * FT_GROUP;
    const int nt = static_cast<int>(ntiles - t0 < FT_GROUP ? ntiles - t0 : FT_GROUP);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t cnt = 0;                                      // this thread's matches over the group
    // the next tile's values are loaded while this tile's are tested
    T nv[FT_ITEMS];
    auto load_tile = [&](int i) {
        const int64_t base = (t0 + i) * FT_TILE;
#pragma unroll
        for (int c = 0; c < FT_ITEMS; ++c) {
            const int64_t e = base + c * FT_THREADS + wave * 64 + lane;
            nv[c] = 0;
            if (i < nt && e < n) nv[c] = col[HAS_SEL ? static_cast<int64_t>(sel_in[e]) : e];
        }
    };
    load_tile(0);
    for (int i = 0; i < nt; ++i) {
        const int64_t base = (t0 + i) * FT_TILE;
        T v[FT_ITEMS];
#pragma unroll
        for (int c = 0; c < FT_ITEMS; ++c) v[c] = nv[c];
        if (i + 1 < nt) load_tile(i + 1);
#pragma unroll
        for (int c = 0; c < FT_ITEMS; ++c) {
            const int64_t e = base + c * FT_THREADS + wave * 64 + lane;
            const int64_t x = static_cast<int64_t>(v[c]);
            const uint64_t b = gq_ballot(e < n && lo <= x && x < hi);
            if (lane == 0) bits[i][c * (FT_THREADS / 64) + wave] = b;
        }
    }
    __syncthreads();
    // thread i owns rows [FT_RPT i, FT_RPT i + FT_RPT) of every tile
    auto owned = [&](int i) {
        const uint64_t word = bits[i][threadIdx.x / FT_TPW] >> ((threadIdx.x % FT_TPW) * FT_RPT);
        return static_cast<uint32_t>(word) & static_cast<uint32_t>((1ull << FT_RPT) - 1);
    };
    for (int i = 0; i < nt; ++i) cnt += __popc(owned(i));
    uint32_t gtotal;
    (void)gq_block_exclusive_scan<FT_THREADS>(cnt, &gtotal, scan_smem);
    if (wave == 0) {
        const uint64_t go = gq_lookback(status, static_cast<uint32_t>(g), gtotal);
        if (lane == 0) s_goff = go;
    }
    __syncthreads();
    int64_t goff = static_cast<int64_t>(s_goff);
    for (int i = 0; i < nt; ++i) {
        const int64_t base = (t0 + i) * FT_TILE;
        uint32_t mine = owned(i);
        uint32_t total;
        uint32_t pos =
            gq_block_exclusive_scan_lds<FT_THREADS>(static_cast<uint32_t>(__popc(mine)), &total, scan_smem);
        const int64_t row0 = base + static_cast<int64_t>(threadIdx.x) * FT_RPT;
        while (mine) {
            const int k = __builtin_ctz(mine);
            mine &= mine - 1;
            const int64_t e = row0 + k;
            stage[pos++] = HAS_SEL ? sel_in[e] : static_cast<int32_t>(e);
        }
        gq_lds_barrier();                                  // (LDS only: the last tile's stores stay in flight)
        for (uint32_t k = threadIdx.x; k < total; k += FT_THREADS) out[goff + k] = stage[k];
        goff += total;
        gq_lds_barrier();                                  // stage[] is free for the next tile
    }
    if (g == ngroups - 1 && threadIdx.x == 0) *n_out = goff;
}

template <typename T, bool S>
gq_status launch_filter(gq_ctx *ctx, const void *col, const int32_t *sel_in, int64_t n, const int64_t *n_dev,
                        int64_t lo, int64_t hi, int32_t *out, int64_t *n_out, filter_ws w, hipStream_t s)
{
    const int64_t tiles = (n + FT_TILE - 1) / FT_TILE;
    const int64_t groups = (tiles + FT_GROUP - 1) / FT_GROUP;
    const uint32_t grid = static_cast<uint32_t>(groups > 0 ? groups : 1);
    return gq_launch(ctx, "gq_filter", filter_kernel<T, S>, dim3(grid), dim3(FT_THREADS), 0, s,
                     static_cast<const T *>(col), sel_in, n, n_dev, lo, hi, out, n_out, w.tile_ctr, w.status);
}

// Scratch of gq_filter_noalloc, one copy per GPU for the life of the
// process: the dequeue counter (64 words) and one look-back status word per
// group of FT_GROUP tiles, enough for the largest accepted input
// (GQ_MAX_ROWS rows: 65,536 groups), 512.25 KiB in all.
constexpr int64_t FT_SCRATCH_GROUPS =
    ((GQ_MAX_ROWS + FT_TILE - 1) / FT_TILE + FT_GROUP - 1) / FT_GROUP;
constexpr size_t FT_SCRATCH_WORDS = 32 + static_cast<size_t>(FT_SCRATCH_GROUPS);   // 8-byte words
__device__ __align__(256) uint64_t scratch[FT_SCRATCH_WORDS];

}  // namespace

// Device address of this library's filter scratch on the context's device
// (the device must be current).  Host code uses this address, never the
// array's name, which on the host is only a stand-in.
gq_status gq_filter_scratch_setup(gq_ctx *ctx)
{
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return gq_fail(ctx, GQ_ERR_HIP, "filter scratch address: %s", hipGetErrorString(e));
    ctx->filter_scratch = p;
    return GQ_OK;
}

extern "C" {

size_t gq_filter_workspace_bytes(int64_t n)
{
    if (n < 0) n = 0;
    gq_carver c(nullptr);
    filter_layout(c, n);
    return c.bytes();
}

gq_status gq_filter(gq_ctx *ctx, const void *col, int dtype, int64_t n, const int64_t *n_dev,
                    const int32_t *sel_in, int64_t lo, int64_t hi, int32_t *sel_out, int64_t *n_out_dev,
                    void *ws, size_t ws_bytes, gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if ((!col && n > 0) || !sel_out || !n_out_dev)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_filter: NULL column, output or count");
    if (n < 0 || n > GQ_MAX_ROWS) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_filter: n=%lld out of range", (long long)n);
    if (dtype != GQ_I32 && dtype != GQ_I64) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_filter: bad dtype %d", dtype);
    const size_t need = gq_filter_workspace_bytes(n);
    if (!ws || ws_bytes < need)
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_filter: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gq_carver c(ws);
    filter_ws w = filter_layout(c, n);
    GQ_TRY(gq_zero(ctx, ws, c.off / 4, s));     // tile counter + tile status words
    if (dtype == GQ_I32)
        return sel_in ? launch_filter<int32_t, true>(ctx, col, sel_in, n, n_dev, lo, hi, sel_out, n_out_dev, w, s)
                      : launch_filter<int32_t, false>(ctx, col, sel_in, n, n_dev, lo, hi, sel_out, n_out_dev, w, s);
    return sel_in ? launch_filter<int64_t, true>(ctx, col, sel_in, n, n_dev, lo, hi, sel_out, n_out_dev, w, s)
                  : launch_filter<int64_t, false>(ctx, col, sel_in, n, n_dev, lo, hi, sel_out, n_out_dev, w, s);
}

gq_status gq_filter_noalloc(gq_ctx *ctx, const void *col, int dtype, int64_t n, const int64_t *n_dev,
                            const int32_t *sel_in, int64_t lo, int64_t hi, int32_t *sel_out, int64_t *n_out_dev,
                            gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if ((!col && n > 0) || !sel_out || !n_out_dev)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_filter_noalloc: NULL column, output or count");
    if (n < 0 || n > GQ_MAX_ROWS)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_filter_noalloc: n=%lld outside [0, %lld]", (long long)n,
                       (long long)GQ_MAX_ROWS);
    if (dtype != GQ_I32 && dtype != GQ_I64)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_filter_noalloc: bad dtype %d", dtype);
    if (!ctx->filter_scratch) return gq_fail(ctx, GQ_ERR_HIP, "gq_filter_noalloc: no scratch on this device");
    gq_carver need(nullptr);
    filter_layout(need, n);
    if (need.bytes() > FT_SCRATCH_WORDS * sizeof(uint64_t))
        return gq_fail(ctx, GQ_ERR_CAPACITY, "gq_filter_noalloc: %lld rows need %zu scratch bytes, more than %zu",
                       (long long)n, need.bytes(), FT_SCRATCH_WORDS * sizeof(uint64_t));
    hipStream_t s = static_cast<hipStream_t>(stream);
    gq_carver c(ctx->filter_scratch);
    filter_ws w = filter_layout(c, n);
    GQ_TRY(gq_zero(ctx, ctx->filter_scratch, c.off / 4, s));   // a kernel: no memset node under capture
    if (dtype == GQ_I32)
        return sel_in ? launch_filter<int32_t, true>(ctx, col, sel_in, n, n_dev, lo, hi, sel_out, n_out_dev, w, s)
                      : launch_filter<int32_t, false>(ctx, col, sel_in, n, n_dev, lo, hi, sel_out, n_out_dev, w, s);
    return sel_in ? launch_filter<int64_t, true>(ctx, col, sel_in, n, n_dev, lo, hi, sel_out, n_out_dev, w, s)
                  : launch_filter<int64_t, false>(ctx, col, sel_in, n, n_dev, lo, hi, sel_out, n_out_dev, w, s);
}

}  // extern "C"
