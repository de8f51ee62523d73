// Radix hash partition (local half of a shuffle), stable.
//
//  1. hist:    one LDS histogram per tile of rows -> hist[t * P + b]
//              (tile-major: a tile's counts are one contiguous row)
//  2. offsets: column-wise scan turning counts into the output start of every
//              (tile, bucket) run, plus the bucket starts offsets[0..P].
//  3. scatter: per tile, each wave ranks its rows inside their bucket with
//              ballots (stable: rows keep input order), the block turns ranks
//              into tile-local positions, and every column is staged in LDS in
//              bucket order and written out as contiguous runs.  Each XCD
//              takes chunks of PT_XCD_CHUNK consecutive tiles, the chunks
//              dealt round the XCDs in order: the partial lines at the ends of
//              a tile's runs meet the next tile's in the same L2 (except at a
//              chunk's end), and the eight XCDs write neighbouring stretches
//              of each bucket.
#include <cstdlib>

#include "gq_device.h"
#include "gq_internal.h"
#include "gq_ops.h"

namespace {

constexpr int PT_THREADS = 256;
constexpr int PT_WAVES = PT_THREADS / 64;
constexpr int PT_MAX_LOG2P = 8;
constexpr int PT_MAX_COLS = 8;
constexpr uint32_t PT_XCD_CHUNK = 32;

// Tile of workgroup bid.  Workgroups go round the XCDs in launch order (XCD =
// bid % GQ_NUM_XCD); the i-th workgroup of an XCD works in that XCD's
// (i / PT_XCD_CHUNK)-th chunk.  Workgroups past the last whole round of chunks
// keep their own index.  A bijection on [0, nblocks).
GQ_DEV uint32_t part_tile_of(uint32_t bid, uint32_t nblocks)
{
    constexpr uint32_t ROUND = GQ_NUM_XCD * PT_XCD_CHUNK;
    const uint32_t full = nblocks / ROUND * ROUND;
    if (bid >= full) return bid;
    const uint32_t xcd = bid % GQ_NUM_XCD, local = bid / GQ_NUM_XCD;
    return ((local / PT_XCD_CHUNK) * GQ_NUM_XCD + xcd) * PT_XCD_CHUNK + local % PT_XCD_CHUNK;
}

struct part_cols {
    const void *in[PT_MAX_COLS];
    void *out[PT_MAX_COLS];
    int32_t bytes[PT_MAX_COLS];
    int32_t n;
};

// Bucket = LOG2P bits of fmix64(key) starting at bit `shift` (the public
// operator uses the top bits: shift = 64 - LOG2P).
template <int LOG2P>
GQ_DEV uint32_t bucket_of(int64_t key, int shift)
{
    if constexpr (LOG2P == 0) {
        (void)key;
        (void)shift;
        return 0;
    } else {
        return static_cast<uint32_t>((gq_fmix64(static_cast<uint64_t>(key)) >> shift) & ((1u << LOG2P) - 1));
    }
}

// LDS histogram of one tile, written as the tile's row hist[t * P + b].
template <int LOG2P, int ITEMS>
__global__ __launch_bounds__(PT_THREADS) void part_hist_kernel(const int64_t *__restrict__ key, int64_t n,
                                                               int shift, uint32_t *__restrict__ hist)
{
    constexpr int P = 1 << LOG2P;
    constexpr int TILE = PT_THREADS * ITEMS;
    __shared__ uint32_t h[P];
    for (int i = threadIdx.x; i < P; i += PT_THREADS) h[i] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * TILE;
    int64_t k[ITEMS];
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int64_t e = base + c * PT_THREADS + threadIdx.x;
        k[c] = (e < n) ? key[e] : 0;
    }
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int64_t e = base + c * PT_THREADS + threadIdx.x;
        if (e < n) atomicAdd(&h[bucket_of<LOG2P>(k[c], shift)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < P; b += PT_THREADS) hist[static_cast<int64_t>(blockIdx.x) * P + b] = h[b];
}

__global__ void part_offsets_kernel(const uint32_t *__restrict__ start, int P, int64_t *__restrict__ offsets)
{
    for (int b = threadIdx.x; b <= P; b += blockDim.x) offsets[b] = static_cast<int64_t>(start[b]);
}

template <int LOG2P, int ITEMS>
__global__ __launch_bounds__(PT_THREADS) void part_scatter_kernel(const int64_t *__restrict__ key, int64_t n,
                                                                  int shift, const uint32_t *__restrict__ gofs,
                                                                  int64_t ntiles,
                                                                  int64_t *__restrict__ key_out,
                                                                  int32_t *__restrict__ rowid_out, part_cols cols)
{
    constexpr int P = 1 << LOG2P;
    constexpr int TILE = PT_THREADS * ITEMS;
    constexpr int WROWS = TILE / PT_WAVES;            // rows per wave
    __shared__ uint32_t wcnt[PT_WAVES][P];            // per-wave running counts, then per-wave prefixes
    __shared__ uint32_t lstart[P];
    __shared__ uint32_t gstart[P];
    __shared__ uint32_t scan_smem[PT_WAVES];
    __shared__ uint8_t lbucket[TILE];
    __shared__ uint64_t stage[TILE];

    const uint32_t tile = part_tile_of(blockIdx.x, gridDim.x);
    const int64_t base = static_cast<int64_t>(tile) * TILE;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < PT_WAVES * P; i += PT_THREADS) (&wcnt[0][0])[i] = 0;

    // rows of this thread: base + wave*WROWS + c*64 + lane (wave-contiguous)
    const int64_t row0 = base + static_cast<int64_t>(wave) * WROWS + lane;
    int64_t k[ITEMS];
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int64_t e = row0 + c * 64;
        k[c] = (e < n) ? key[e] : 0;
    }
    __syncthreads();

    uint32_t pos[ITEMS];     // bucket << 16 | rank in (wave, bucket), then tile-local position
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const bool valid = row0 + c * 64 < n;
        const uint32_t b = bucket_of<LOG2P>(k[c], shift);
        uint64_t match = gq_ballot(valid);
#pragma unroll
        for (int bit = 0; bit < LOG2P; ++bit) {
            const bool set = (b >> bit) & 1u;
            const uint64_t bal = gq_ballot(set);
            match &= set ? bal : ~bal;
        }
        const uint32_t below = gq_mbcnt(match);
        const uint32_t cnt = static_cast<uint32_t>(__popcll(match));
        uint32_t old = 0;
        if (valid) old = wcnt[wave][b];
        if (valid && below == cnt - 1) wcnt[wave][b] = old + cnt;
        pos[c] = (b << 16) | (old + below);
    }
    __syncthreads();

    // per-bucket totals, per-wave exclusive prefixes, bucket starts in the tile
    uint32_t tot = 0;
    for (int b = threadIdx.x; b < P; b += PT_THREADS) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < PT_WAVES; ++w) {
            const uint32_t x = wcnt[w][b];
            wcnt[w][b] = run;
            run += x;
        }
        tot = run;                                   // P <= PT_THREADS: one bucket per thread
    }
    uint32_t all;
    const uint32_t excl = gq_block_exclusive_scan<PT_THREADS>(threadIdx.x < P ? tot : 0u, &all, scan_smem);
    if (threadIdx.x < P) {
        lstart[threadIdx.x] = excl;
        gstart[threadIdx.x] = gofs[static_cast<int64_t>(tile) * P + threadIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        if (row0 + c * 64 < n) {
            const uint32_t b = pos[c] >> 16;
            const uint32_t p = lstart[b] + wcnt[wave][b] + (pos[c] & 0xffffu);
            lbucket[p] = static_cast<uint8_t>(b);
            pos[c] = p;
        }
    }
    const int64_t rem = n - base;
    const uint32_t count = static_cast<uint32_t>(rem < TILE ? rem : TILE);

    // column 0 = key (in registers), 1..ncols = payload columns, last = row id.
    // The next column's loads are issued before the current column is written
    // out, and the barriers order LDS only, so loads and stores of neighbouring
    // columns overlap.
    const int ncol_total = 1 + cols.n + (rowid_out ? 1 : 0);
    auto load_col = [&](int ci, uint64_t *v) {
        const bool is_key = ci == 0;
        const bool is_rowid = ci == 1 + cols.n;
        const int width = is_key ? 8 : (is_rowid ? 4 : cols.bytes[ci - 1]);
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {
            const int64_t e = row0 + c * 64;
            uint64_t x = 0;
            if (e < n) {
                if (is_key) x = static_cast<uint64_t>(k[c]);
                else if (is_rowid) x = static_cast<uint32_t>(e);
                else if (width == 8) x = static_cast<const uint64_t *>(cols.in[ci - 1])[e];
                else x = static_cast<const uint32_t *>(cols.in[ci - 1])[e];
            }
            v[c] = x;
        }
    };
    uint64_t cur[ITEMS], nxt[ITEMS];
    load_col(0, cur);
    for (int ci = 0; ci < ncol_total; ++ci) {
        const bool is_key = ci == 0;
        const bool is_rowid = ci == 1 + cols.n;
        const int width = is_key ? 8 : (is_rowid ? 4 : cols.bytes[ci - 1]);
        gq_lds_barrier();                             // stage free (and lbucket ready)
        if (width == 8) {
#pragma unroll
            for (int c = 0; c < ITEMS; ++c)
                if (row0 + c * 64 < n) stage[pos[c]] = cur[c];
        } else {
            uint32_t *st32 = reinterpret_cast<uint32_t *>(stage);
#pragma unroll
            for (int c = 0; c < ITEMS; ++c)
                if (row0 + c * 64 < n) st32[pos[c]] = static_cast<uint32_t>(cur[c]);
        }
        if (ci + 1 < ncol_total) load_col(ci + 1, nxt);
        gq_lds_barrier();
        if (width == 8) {
            uint64_t *dst = is_key ? reinterpret_cast<uint64_t *>(key_out) : static_cast<uint64_t *>(cols.out[ci - 1]);
            for (uint32_t q = threadIdx.x; q < count; q += PT_THREADS) {
                const uint32_t b = lbucket[q];
                dst[gstart[b] + (q - lstart[b])] = stage[q];
            }
        } else {
            const uint32_t *st32 = reinterpret_cast<const uint32_t *>(stage);
            uint32_t *dst = is_rowid ? reinterpret_cast<uint32_t *>(rowid_out) : static_cast<uint32_t *>(cols.out[ci - 1]);
            for (uint32_t q = threadIdx.x; q < count; q += PT_THREADS) {
                const uint32_t b = lbucket[q];
                dst[gstart[b] + (q - lstart[b])] = st32[q];
            }
        }
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) cur[c] = nxt[c];
    }
}

// Rows per thread in the scatter (tile = 256 * items).  16 by default; the
// GQ_PARTITION_ITEMS environment variable (8, 16 or 32) overrides it.
int part_items()
{
    static int v = [] {
        const char *e = getenv("GQ_PARTITION_ITEMS");
        const int x = e ? atoi(e) : 16;
        return (x == 8 || x == 16 || x == 32) ? x : 16;
    }();
    return v;
}

constexpr int PT_MIN_TILE = PT_THREADS * 8;

struct part_ws {
    uint32_t *hist;
    uint32_t *start;
    void *scan_ws;
};

// The workspace is sized for the smallest tile, so it fits every choice.
part_ws part_layout(gq_carver &c, int64_t n, int log2p)
{
    part_ws w;
    const int64_t ntiles = n > 0 ? (n + PT_MIN_TILE - 1) / PT_MIN_TILE : 1;
    const int64_t cells = ntiles << log2p;
    w.hist = c.take<uint32_t>(static_cast<size_t>(cells));
    w.start = c.take<uint32_t>((size_t(1) << log2p) + 1);
    w.scan_ws = c.take<char>(gq_tile_offsets_workspace(ntiles, 1 << log2p));
    return w;
}

template <int LOG2P, int ITEMS>
gq_status run_partition_items(gq_ctx *ctx, const int64_t *key, int64_t n, int shift, const part_cols &cols,
                              int64_t *key_out, int32_t *rowid_out, int64_t *offsets, part_ws w, hipStream_t s,
                              const gq_part_names &nm)
{
    constexpr int P = 1 << LOG2P;
    constexpr int TILE = PT_THREADS * ITEMS;
    const int64_t ntiles = n > 0 ? (n + TILE - 1) / TILE : 1;
    const uint32_t grid = static_cast<uint32_t>(ntiles);
    GQ_TRY(gq_launch(ctx, nm.hist, part_hist_kernel<LOG2P, ITEMS>, dim3(grid), dim3(PT_THREADS), 0, s, key, n,
                     shift, w.hist));
    GQ_TRY(gq_tile_offsets(ctx, w.hist, ntiles, P, w.start, w.scan_ws, s, nm.scan));
    GQ_TRY(gq_launch(ctx, nm.offsets, part_offsets_kernel, dim3(1), dim3(256), 0, s,
                     static_cast<const uint32_t *>(w.start), P, offsets));
    if (n == 0) return GQ_OK;
    return gq_launch(ctx, nm.scatter, part_scatter_kernel<LOG2P, ITEMS>, dim3(grid), dim3(PT_THREADS),
                     0, s, key, n, shift, static_cast<const uint32_t *>(w.hist), ntiles, key_out, rowid_out,
                     cols);
}

template <int LOG2P>
gq_status run_partition(gq_ctx *ctx, const int64_t *key, int64_t n, int shift, const part_cols &cols,
                        int64_t *key_out, int32_t *rowid_out, int64_t *offsets, part_ws w, hipStream_t s,
                        const gq_part_names &nm, int items)
{
    switch (items > 0 ? items : part_items()) {
    case 8: return run_partition_items<LOG2P, 8>(ctx, key, n, shift, cols, key_out, rowid_out, offsets, w, s, nm);
    case 32: return run_partition_items<LOG2P, 32>(ctx, key, n, shift, cols, key_out, rowid_out, offsets, w, s, nm);
    default: return run_partition_items<LOG2P, 16>(ctx, key, n, shift, cols, key_out, rowid_out, offsets, w, s, nm);
    }
}

gq_status dispatch_partition(gq_ctx *ctx, const int64_t *key, int64_t n, int log2p, int shift, const part_cols &pc,
                             int64_t *key_out, int32_t *rowid_out, int64_t *offsets, part_ws w, hipStream_t s,
                             const gq_part_names &nm, int items = 0)
{
    switch (log2p) {
    case 0: return run_partition<0>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    case 1: return run_partition<1>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    case 2: return run_partition<2>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    case 3: return run_partition<3>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    case 4: return run_partition<4>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    case 5: return run_partition<5>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    case 6: return run_partition<6>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    case 7: return run_partition<7>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    default: return run_partition<8>(ctx, key, n, shift, pc, key_out, rowid_out, offsets, w, s, nm, items);
    }
}

}  // namespace

size_t gq_partition_bits_workspace(int64_t n, int log2p)
{
    gq_carver c(nullptr);
    part_layout(c, n < 0 ? 0 : n, log2p);
    return c.bytes();
}

gq_status gq_partition_bits(gq_ctx *ctx, const int64_t *key, int64_t n, int log2p, int shift, int ncols,
                            void *const *cols, const int32_t *col_bytes, int64_t *key_out, void *const *cols_out,
                            int64_t *offsets, void *ws, hipStream_t s, const gq_part_names &nm, int items)
{
    part_cols pc{};
    pc.n = ncols;
    for (int i = 0; i < ncols; ++i) {
        pc.in[i] = cols[i];
        pc.out[i] = cols_out[i];
        pc.bytes[i] = col_bytes[i];
    }
    gq_carver c(ws);
    part_ws w = part_layout(c, n, log2p);
    return dispatch_partition(ctx, key, n, log2p, shift, pc, key_out, nullptr, offsets, w, s, nm, items);
}

extern "C" {

size_t gq_radix_partition_workspace_bytes(int64_t n, int log2_fanout)
{
    if (n < 0) n = 0;
    if (log2_fanout < 0 || log2_fanout > PT_MAX_LOG2P) return 0;
    gq_carver c(nullptr);
    part_layout(c, n, log2_fanout);
    return c.bytes();
}

gq_status gq_radix_partition(gq_ctx *ctx, const int64_t *key, int64_t n, int log2_fanout, int ncols,
                             const void *const *cols, const int32_t *col_bytes, int64_t *key_out,
                             void *const *cols_out, int32_t *rowid_out, int64_t *offsets_dev, void *ws,
                             size_t ws_bytes, gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (n < 0 || n > GQ_MAX_ROWS)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_radix_partition: n=%lld out of range", (long long)n);
    if (!offsets_dev || (n > 0 && (!key || !key_out)))
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_radix_partition: NULL key, key_out or offsets");
    if (log2_fanout < 0 || log2_fanout > PT_MAX_LOG2P)
        return gq_fail(ctx, GQ_ERR_UNSUPPORTED, "gq_radix_partition: log2_fanout %d not in [0,%d]", log2_fanout,
                       PT_MAX_LOG2P);
    if (ncols < 0 || ncols > PT_MAX_COLS)
        return gq_fail(ctx, GQ_ERR_UNSUPPORTED, "gq_radix_partition: ncols %d not in [0,%d]", ncols, PT_MAX_COLS);
    part_cols pc{};
    pc.n = ncols;
    for (int i = 0; i < ncols; ++i) {
        if (!cols || !cols_out || !col_bytes || (n > 0 && (!cols[i] || !cols_out[i])) ||
            (col_bytes[i] != 4 && col_bytes[i] != 8))
            return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_radix_partition: bad column %d", i);
        pc.in[i] = cols[i];
        pc.out[i] = cols_out[i];
        pc.bytes[i] = col_bytes[i];
    }
    const size_t need = gq_radix_partition_workspace_bytes(n, log2_fanout);
    if (!ws || ws_bytes < need)
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_radix_partition: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gq_carver c(ws);
    part_ws w = part_layout(c, n, log2_fanout);
    static const gq_part_names names{"gq_partition_hist", "gq_partition_scan", "gq_partition_offsets",
                                     "gq_partition_scatter"};
    return dispatch_partition(ctx, key, n, log2_fanout, 64 - log2_fanout, pc, key_out, rowid_out, offsets_dev, w, s,
                              names);
}

}  // extern "C"
