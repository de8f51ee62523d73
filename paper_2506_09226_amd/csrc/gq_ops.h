// Internal operations shared between operator sources.
#pragma once

#include "gq_internal.h"

// In-place exclusive scan of n uint32 values (n >= 0); ws must hold
// gq_scan_u32_workspace(n) bytes and is zeroed by the call.
size_t gq_scan_u32_workspace(int64_t n);
gq_status gq_scan_u32(gq_ctx *ctx, uint32_t *data, int64_t n, void *ws, hipStream_t s, const char *name);

// Stable partition of n rows by the log2p (0..8) bits of fmix64(key) that
// start at bit `shift` (no row ids), with tiles of 256 * items rows (items 8,
// 16 or 32; 0 = the operator's default).  ws: gq_partition_bits_workspace(n, log2p).
size_t gq_partition_bits_workspace(int64_t n, int log2p);
// Kernel names of one use of the partition (for per-kernel timing).
struct gq_part_names {
    const char *hist, *scan, *offsets, *scatter;
};
gq_status gq_partition_bits(gq_ctx *ctx, const int64_t *key, int64_t n, int log2p, int shift, int ncols,
                            void *const *cols, const int32_t *col_bytes, int64_t *key_out, void *const *cols_out,
                            int64_t *offsets, void *ws, hipStream_t s, const gq_part_names &names, int items);

// In place: per-tile bucket counts cnt[t*P + b] (tile-major) become the output
// offsets of each (tile, bucket) run; start[0..P] receives the bucket starts
// (start[P] = total).  P <= 8192.  ws: gq_tile_offsets_workspace(ntiles, P).
size_t gq_tile_offsets_workspace(int64_t ntiles, int P);
// Optional: only the first ceil(min(*n_dev, n_bound) / tile_rows) of the
// ntiles tiles hold counts (the rows arrive as a device count); the rest are
// neither read nor written.
struct gq_tile_count {
    const int64_t *n_dev;
    int64_t n_bound;
    int64_t tile_rows;
};
gq_status gq_tile_offsets(gq_ctx *ctx, uint32_t *cnt, int64_t ntiles, int P, uint32_t *start, void *ws,
                          hipStream_t s, const char *name, const gq_tile_count *live = nullptr);

// Look up, on the current device (the context's), the device address of the
// filter's static scratch array used by gq_filter_noalloc.
gq_status gq_filter_scratch_setup(gq_ctx *ctx);
