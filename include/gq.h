/*
 * gq.h -- C ABI of the per-GPU relational hot path (MI355X / gfx950).
 *
 * The library implements, on one GPU's share of the data, the local
 * relational operators of a data-parallel SQL engine whose exchange steps
 * (shuffle, broadcast, all-reduce) are built from collective-communication
 * primitives (Wu et al., "Terabyte-Scale Analytics in the Blink of an Eye",
 * Sec. 2).  The paper runs these operators as tensor programs and states only
 * their semantics; the kernels behind this header are hand-written HIP.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory.  Every pointer argument named *_dev, every column, table,
 *    output and workspace pointer is DEVICE memory owned by the caller (e.g.
 *    from torch.empty(..., device="cuda")).  Arrays passed as "host array"
 *    are host memory read before the call returns.  The library never frees
 *    caller memory and never allocates memory that it hands back.
 *  - Streams.  gq_stream is a hipStream_t (NULL = the null stream).  Every
 *    operator is asynchronous and stream ordered; counts are written to
 *    device memory so that operators chain without host round trips.
 *  - Counts.  An input count is given as a host bound `n` (sizes the launch)
 *    plus an optional device scalar `n_dev` (int64); when `n_dev` is non-NULL
 *    the operator uses min(*n_dev, n) rows, read on the device.
 *  - Row ids are int32: tables have at most 2^31 - 1 rows.
 *  - Workspace.  Operators that need scratch memory take (ws, ws_bytes);
 *    the required size comes from the matching *_workspace_bytes() query.  A
 *    workspace must not be shared by calls that may run concurrently.
 *  - Errors.  Argument errors are detected on the host and returned
 *    synchronously (GQ_ERR_INVALID_ARG, GQ_ERR_WORKSPACE, GQ_ERR_UNSUPPORTED);
 *    nothing is launched then.  Data-dependent errors found by a kernel
 *    (duplicate or invalid build key, a full table) are recorded in a
 *    per-context device status word and read with gq_status_word(), which
 *    synchronizes the stream.  After such an error the outputs of that call
 *    are unspecified.  gq_last_error() returns a message for the last non-OK
 *    host-side status.
 *  - Results.  Filter, partition, probe and top-k outputs are deterministic
 *    and ordered.  Group output order is unspecified.  Every integer result
 *    is exact and independent of scheduling.
 */
#ifndef GQ_H
#define GQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gq_status;
#define GQ_OK                 0
#define GQ_ERR_INVALID_ARG    1  /* bad pointer, size or parameter            */
#define GQ_ERR_CAPACITY       2  /* a table or output capacity was exceeded   */
#define GQ_ERR_WORKSPACE      3  /* workspace missing or smaller than needed  */
#define GQ_ERR_DUPLICATE_KEY  4  /* two build rows carry the same key         */
#define GQ_ERR_HIP            5  /* a HIP runtime call failed                 */
#define GQ_ERR_UNSUPPORTED    6  /* parameter outside the supported range     */
#define GQ_ERR_INVALID_KEY    7  /* build key equal to the empty-slot marker  */
#define GQ_ERR_TIMEOUT        8  /* a bounded device-side wait ran out (see
                                    gq_set_wait_limit); outputs undefined     */

/* Column element types; the value is the element width in bytes. */
#define GQ_I32 4
#define GQ_I64 8

typedef void *gq_stream;                 /* hipStream_t */
typedef struct gq_ctx gq_ctx;            /* opaque, one per device */

/* ------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------ */

/* Create a context on HIP device `device` (allocates a few bytes of device
 * memory for the status word).  *out receives the context.
 * Errors: GQ_ERR_INVALID_ARG (out NULL, bad device), GQ_ERR_HIP. */
gq_status gq_ctx_create(int device, gq_ctx **out);

/* Destroy a context created by gq_ctx_create (NULL is ignored). */
void gq_ctx_destroy(gq_ctx *ctx);

/* Message for the last non-OK status returned on this context ("" if none).
 * The string is owned by the context and valid until its next call. */
const char *gq_last_error(const gq_ctx *ctx);

/* Synchronize `stream`, then read and clear the device status word: *out is
 * GQ_OK or one device-side error recorded since the last read, the first
 * present of GQ_ERR_TIMEOUT, GQ_ERR_DUPLICATE_KEY, GQ_ERR_INVALID_KEY,
 * GQ_ERR_CAPACITY, GQ_ERR_INVALID_ARG (a table whose header disagrees with
 * its given size).
 * Errors: GQ_ERR_INVALID_ARG, GQ_ERR_HIP. */
gq_status gq_status_word(gq_ctx *ctx, gq_stream stream, gq_status *out);

/* Bound of the device-side waits of kernels whose work items wait for
 * other work items (the batched form's build and probe items): at most
 * `polls` reads of the awaited counter, each after a short sleep.  polls = 0
 * restores the default (2^24 polls, far beyond any wait of a correct run).
 * A wait that runs out skips its item's work, raises GQ_ERR_TIMEOUT and lets
 * the kernel finish its queue and exit; the affected outputs are undefined.
 * A tiny bound (polls = 1) forces that path, for tests of the error
 * handling.  Errors: GQ_ERR_INVALID_ARG (polls < 0). */
gq_status gq_set_wait_limit(gq_ctx *ctx, int64_t polls);

/* Per-kernel timing with HIP events recorded on the stream each kernel is
 * launched on (off by default).  gq_kernel_time synchronizes the device and
 * returns, for the kernel named `name`, the number of timed launches and their
 * summed duration in milliseconds since the last reset.
 * Errors: GQ_ERR_INVALID_ARG, GQ_ERR_HIP. */
gq_status gq_set_timing(gq_ctx *ctx, int enable);
gq_status gq_kernel_time(gq_ctx *ctx, const char *name, int64_t *launches, double *total_ms);
gq_status gq_reset_timing(gq_ctx *ctx);

/* ------------------------------------------------------------------------
 * Scan + filter
 * Paper: Sec. 2.2 (the example plan filters both inputs of a join with
 * their predicates before the exchange and the join).
 * ------------------------------------------------------------------------ */

/* Workspace for gq_filter over at most n rows. */
size_t gq_filter_workspace_bytes(int64_t n);

/* sel_out = the row ids r with lo <= col[r] < hi, in ascending order of r
 * (when sel_in is NULL, r ranges over 0..n-1), or the entries r of sel_in
 * that satisfy the predicate, in sel_in's order.
 *   col        device, `dtype` (GQ_I32 or GQ_I64) elements, indexed by row id
 *   n          with sel_in NULL: rows of col; else: host bound on the length
 *              of sel_in, with n_dev (nullable) its device length
 *   sel_out    device int32, capacity >= n
 *   n_out_dev  device int64 scalar, receives the output length
 * Errors: GQ_ERR_INVALID_ARG (NULL col/sel_out/n_out_dev, n < 0 or > 2^31-1,
 * bad dtype), GQ_ERR_WORKSPACE. */
gq_status gq_filter(gq_ctx *ctx, const void *col, int dtype, int64_t n, const int64_t *n_dev,
                    const int32_t *sel_in, int64_t lo, int64_t hi,
                    int32_t *sel_out, int64_t *n_out_dev,
                    void *ws, size_t ws_bytes, gq_stream stream);

/* The same filter with no workspace argument and no allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Its scratch (a dequeue
 * counter and one look-back word per 32,768 rows, at most 512.25 KiB) is a
 * static device array of the library, one per GPU, held until the process
 * ends and located at context creation.  The call clears it with a kernel
 * (no memset node) and calls no allocating routine.  Every call on one GPU
 * shares that array: calls that may overlap on one GPU (other streams,
 * other threads, other contexts) race and give undefined results; serialize
 * them or use gq_filter with separate workspaces.
 * Arguments and output as gq_filter.  Errors: as gq_filter, plus
 * GQ_ERR_CAPACITY if n needs more scratch than the array holds (never for
 * n <= 2^31 - 1, the row limit) and GQ_ERR_HIP if the array could not be
 * located on this device. */
gq_status gq_filter_noalloc(gq_ctx *ctx, const void *col, int dtype, int64_t n, const int64_t *n_dev,
                            const int32_t *sel_in, int64_t lo, int64_t hi,
                            int32_t *sel_out, int64_t *n_out_dev, gq_stream stream);

/* ------------------------------------------------------------------------
 * Radix hash partition (the local half of a shuffle)
 * Paper: Sec. 2.2 (every process applies the same partitioning function to
 * its rows; the shuffle redistributes the partitions, keeping the total data
 * fixed) and Sec. 2.3 (sizes are exchanged first; each column is received
 * into one contiguous buffer at per-sender start offsets).
 * ------------------------------------------------------------------------ */

/* Workspace for partitioning n rows into 2^log2_fanout buckets. */
size_t gq_radix_partition_workspace_bytes(int64_t n, int log2_fanout);

/* bucket(r) = top log2_fanout bits of fmix64((uint64)key[r]), where fmix64 is
 * the 64-bit finalizer of MurmurHash3.  Rows are written bucket by bucket,
 * keeping their input order inside a bucket (stable), into contiguous
 * per-column output buffers:
 *   key_out[offsets[b] .. offsets[b+1])       keys of bucket b
 *   cols_out[c][same range]                   column c of the same rows
 *   rowid_out[same range]                     source row ids (nullable)
 *   offsets_dev                               device int64[P+1], offsets[0]=0,
 *                                             offsets[P]=n (exclusive prefix
 *                                             sums of the bucket sizes)
 *   key        device int64[n]
 *   cols       host array of `ncols` device pointers, column c has n
 *              elements of col_bytes[c] (4 or 8) bytes; cols_out likewise
 *   ncols      0..8
 *   log2_fanout 0..8 (1..256 buckets)
 * Errors: GQ_ERR_INVALID_ARG, GQ_ERR_UNSUPPORTED (fan-out or column count
 * outside the range), GQ_ERR_WORKSPACE. */
gq_status gq_radix_partition(gq_ctx *ctx, const int64_t *key, int64_t n, int log2_fanout,
                             int ncols, const void *const *cols, const int32_t *col_bytes,
                             int64_t *key_out, void *const *cols_out, int32_t *rowid_out,
                             int64_t *offsets_dev, void *ws, size_t ws_bytes, gq_stream stream);

/* ------------------------------------------------------------------------
 * Hash equi-join (build + probe)
 * Paper: Sec. 2.2 (a join of partitioned tables runs locally once both sides
 * are partitioned on the join key, after a broadcast or after shuffling both
 * sides) and Sec. 7.2 (each GPU builds a hash table of its local keys).
 * ------------------------------------------------------------------------ */

/* Bytes of a join hash table for m build keys at load factor <= load_factor
 * (0 < load_factor <= 0.9): a 256-byte header plus 2^L 16-byte slots,
 * 2^L >= max(64, m / load_factor).  Returns 0 for invalid arguments. */
size_t gq_join_table_bytes(int64_t m, double load_factor);

/* Workspace for gq_join_build of m keys into a table of table_bytes bytes
 * (a few hundred bytes for small tables; about 26 bytes per key for the
 * region build of large tables). */
size_t gq_join_build_workspace_bytes(int64_t m, size_t table_bytes);

/* Build an open-addressing table (linear probing; slot index = top L bits of
 * fmix64(key)) mapping the unique int64 key[i] to the int32 payload[i], for
 * i in 0..m-1, or for the rows listed in sel (nullable) of device length
 * min(*n_dev, m) when n_dev is given.  The table memory (device,
 * `table_bytes` from gq_join_table_bytes, 256-byte aligned) is fully
 * initialized here; its slot count is the largest power of two that fits.
 * Device-side errors: GQ_ERR_DUPLICATE_KEY, GQ_ERR_INVALID_KEY (key ==
 * INT64_MIN, the empty marker), GQ_ERR_CAPACITY.
 * Host errors: GQ_ERR_INVALID_ARG (table too small for m at load factor 0.9,
 * NULL pointers, bad m), GQ_ERR_WORKSPACE. */
gq_status gq_join_build(gq_ctx *ctx, const int64_t *key, const int32_t *payload, int64_t m,
                        const int64_t *n_dev, const int32_t *sel,
                        void *table, size_t table_bytes, void *ws, size_t ws_bytes, gq_stream stream);

/* Workspace for probing at most n rows. */
size_t gq_join_probe_workspace_bytes(int64_t n);

/* Inner equi-join of probe rows with a built table: for each probe row r
 * (r = sel[j] for j in 0..len-1, or r = j when sel is NULL), look fk[r] up;
 * a match emits (prow_out = r, payload_out = payload of the key).  Output
 * pairs are compacted in probe order; unmatched rows are dropped.
 *   n, n_dev   host bound / optional device length of the probe (of sel, or
 *              of fk when sel is NULL)
 *   prow_out, payload_out  device int32, capacity >= n
 *   n_out_dev  device int64 scalar, receives the number of pairs
 * Errors: GQ_ERR_INVALID_ARG, GQ_ERR_WORKSPACE. */
gq_status gq_join_probe(gq_ctx *ctx, const void *table, const int64_t *fk,
                        int64_t n, const int64_t *n_dev, const int32_t *sel,
                        int32_t *prow_out, int32_t *payload_out, int64_t *n_out_dev,
                        void *ws, size_t ws_bytes, gq_stream stream);

/* Workspace for gq_join_probe_partitioned of at most n rows (about 18 bytes
 * per row plus about 530 bytes per 4096 rows). */
size_t gq_join_probe_partitioned_workspace_bytes(int64_t n);

/* The same join as gq_join_probe, computed as a partitioned (radix) join:
 * the probes of each table region (4096 slots) are answered from an LDS copy
 * of that region.  Each tile of 4096 probe rows is split, stably, by the
 * region of its keys (fmix64 bits below the top log2_fanout, up to 256 ways);
 * one workgroup per region then loads the region into LDS and looks up that
 * region's rows of every tile; the results are put back in probe order tile
 * by tile.  Fast when the probe stream is in the order of a radix partition
 * by the top log2_fanout bits of the same hash (the output of
 * gq_radix_partition on fk), since then a tile's rows share those bits;
 * rows that do not are probed in device memory, so any order is correct.
 * Paper: Sec. 2.2 (a local join of inputs partitioned on the key) and the
 * Related Work section (single-GPU query processing, which cites
 * partitioned radix joins).
 *   table_bytes  the byte size given to gq_join_build for this table; it
 *                must match the table (checked on the device: a mismatch
 *                raises GQ_ERR_INVALID_ARG in the status word and leaves
 *                the output undefined)
 *   log2_fanout  radix bits of the partition the probe stream is in (0..16;
 *                0 when it is in no such order)
 * Tables with fewer than 2^20 slots (cache resident), or too large for 256
 * regions per partition bucket (more than 2^(log2_fanout + 20) slots), are
 * probed by gq_join_probe instead.
 * Output: identical to gq_join_probe's (pairs in probe order, *n_out_dev
 * their number).
 * Other arguments, errors and capacities as gq_join_probe; additionally
 * GQ_ERR_INVALID_ARG for table_bytes below a 64-slot table or log2_fanout
 * outside 0..16. */
gq_status gq_join_probe_partitioned(gq_ctx *ctx, const void *table, size_t table_bytes,
                                    const int64_t *fk, int64_t n, const int64_t *n_dev,
                                    const int32_t *sel, int log2_fanout,
                                    int32_t *prow_out, int32_t *payload_out, int64_t *n_out_dev,
                                    void *ws, size_t ws_bytes, gq_stream stream);

/* ------------------------------------------------------------------------
 * Group-by aggregate with exact fixed-point sums (+ float64 finalize)
 * Paper: Sec. 2.4 (exchange operators are injected before a group-by and for
 * the final aggregation) and Sec. 2.3 (the final aggregation of partial
 * results uses a reduction: sum, product, min, max or average).  The paper loads decimals as floating point; here money is an
 * exact integer in cents and the revenue sum is an exact 128-bit integer.
 * ------------------------------------------------------------------------ */

/* Input rows of a group-by.  Row j (0 <= j < len) reads its values at row
 * v = rowid[j] (v = j when rowid is NULL); its key is (key64, key32), each
 * part read at j or at v as flagged; a NULL key part is 0 for every row.
 *   revenue(v) = price[v] * (rev_scale - disc[v]) computed in 128 bits. */
typedef struct gq_groupby_in {
    int64_t n;                 /* host bound on the number of rows          */
    const int64_t *n_dev;      /* nullable device length (min with n)       */
    const int32_t *rowid;      /* nullable device int32[n]                  */
    const int64_t *key64;      /* nullable device int64                     */
    int32_t key64_by_rowid;    /* 1: key64[v], 0: key64[j]                  */
    const int32_t *key32;      /* nullable device int32                     */
    int32_t key32_by_rowid;    /* 1: key32[v], 0: key32[j]                  */
    const int64_t *qty;        /* device int64, read at v                   */
    const int64_t *price;      /* device int64, read at v                   */
    const int64_t *disc;       /* device int64, read at v                   */
    int64_t rev_scale;         /* e.g. 100 (percent)                        */
    const int32_t *filter;     /* nullable device int32 read at v: only rows */
    int64_t filter_lo;         /*   with filter_lo <= filter[v] < filter_hi  */
    int64_t filter_hi;         /*   are aggregated                           */
} gq_groupby_in;

/* Output groups, one entry per distinct key present, in unspecified order.
 * All arrays are device memory with room for `capacity` groups. */
typedef struct gq_groups {
    int64_t *key64;            /* nullable (required if the input has key64) */
    int32_t *key32;            /* nullable (required if the input has key32) */
    int64_t *count;            /* number of rows                            */
    int64_t *sum_qty;          /* sum of qty, wrapping int64                 */
    uint64_t *sum_rev_lo;      /* low 64 bits of the int128 revenue sum     */
    int64_t *sum_rev_hi;       /* high 64 bits (two's complement)           */
    double *avg_qty;           /* (double)sum_qty / (double)count, last      */
    double *avg_rev;           /* (double)sum_rev / (double)count, last      */
    int64_t *n_groups;         /* device int64 scalar: number of groups     */
    int64_t capacity;          /* room in each array                        */
} gq_groups;

/* Workspace for a group-by of at most n rows into at most max_groups groups.
 * has_key64 / has_key32 say which key parts the input carries. */
size_t gq_groupby_workspace_bytes(int64_t n, int64_t max_groups, int has_key64, int has_key32);

/* Aggregate count, sum(qty) and the exact sum of revenue per key, then the
 * float64 averages (computed last, from the exact integers).  max_groups
 * sizes the internal tables (it must match the workspace query) and must be
 * <= out->capacity.
 * Device-side error: GQ_ERR_CAPACITY when more than max_groups distinct keys
 * occur.  Host errors: GQ_ERR_INVALID_ARG, GQ_ERR_WORKSPACE. */
gq_status gq_groupby_agg(gq_ctx *ctx, const gq_groupby_in *in, int64_t max_groups,
                         const gq_groups *out, void *ws, size_t ws_bytes, gq_stream stream);

/* ------------------------------------------------------------------------
 * Top-k
 * The paper's query plans end by gathering the partial results of every GPU
 * (Sec. 4.4, whose exchange counts leave that final gather out); a top-k is
 * the local half of an ORDER BY ... LIMIT k before such a gather.
 * ------------------------------------------------------------------------ */

/* Workspace for top-k over at most n rows. */
size_t gq_topk_workspace_bytes(int64_t n, int k);

/* The k selected rows with the largest (descending=1) or smallest
 * (descending=0) val; equal values are ordered by ascending row id; if fewer
 * than k rows are selected all of them are returned.  Output sorted.
 *   val        device int64, indexed by row id
 *   sel        nullable device int32 row ids (NULL: rows 0..n-1)
 *   n, n_dev   host bound / optional device length of the selection
 *   k          1..2048
 *   val_out    device int64[k], rowid_out device int32[k]
 *   n_out_dev  device int64 scalar: min(k, selected rows)
 * Errors: GQ_ERR_INVALID_ARG, GQ_ERR_UNSUPPORTED (k > 2048),
 * GQ_ERR_WORKSPACE. */
gq_status gq_topk(gq_ctx *ctx, const int64_t *val, const int32_t *sel, int64_t n,
                  const int64_t *n_dev, int k, int descending,
                  int64_t *val_out, int32_t *rowid_out, int64_t *n_out_dev,
                  void *ws, size_t ws_bytes, gq_stream stream);

/* ------------------------------------------------------------------------
 * Batched join + aggregate: many independent instances in one persistent
 * launch.  Each instance is the filter -> join -> group-by -> averages
 * pipeline above on its own tables (the per-GPU body of the engine run on
 * many small queries at once).
 * ------------------------------------------------------------------------ */

typedef struct gq_instance {
    const int64_t *dim_key;    /* device int64[m], unique                   */
    const int32_t *dim_attr;   /* device int32[m], the group key            */
    int64_t m;
    const int64_t *fk;         /* device fact columns, n rows each          */
    const int32_t *date;
    const int64_t *qty, *price, *disc;
    int64_t n;
    int64_t date_lo, date_hi;  /* filter date_lo <= date < date_hi          */
    int64_t rev_scale;         /* revenue = price * (rev_scale - disc)      */
    gq_groups out;             /* key32 required; capacity >= groups, <= 2^24 */
} gq_instance;

typedef struct gq_tuning {
    double load_factor;        /* hash-table load factor (0, 0.9]           */
    int32_t probe_tile;        /* fact rows per probe work item (multiple of 4096) */
    int32_t build_tile;        /* keys per build work item (multiple of 256) */
    int32_t init_tile;         /* slots per table-fill work item            */
    int32_t lag;               /* probe items of instance i follow the build
                                  items of instance i + lag in the queue    */
    int32_t fanout;            /* probe fan-out, 1..64: the probe tiles of
                                  `fanout` consecutive instances are
                                  interleaved in the queue (1: one instance's
                                  tiles after another's, so every workgroup
                                  probes the same table; more: several tables
                                  probed at once)                           */
} gq_tuning;

/* Defaults: load factor 0.5, 8192-row probe tiles, 4096-key build tiles,
 * 16384-slot fill tiles, lag 2, fan-out 1. */
gq_tuning gq_default_tuning(void);

/* Workspace for gq_batch_join_agg (0 for invalid arguments).  It holds every
 * instance's hash table and group table. */
size_t gq_batch_workspace_bytes(const gq_instance *inst, int n_inst, const gq_tuning *tuning);

/* Run every instance of the host array inst[0..n_inst) in one persistent
 * kernel.  tuning NULL = gq_default_tuning() (autotuning is the separate,
 * timed and cached gq_batch_autotune below, so that a plain call never
 * spends seconds searching).  Each instance's out receives its groups
 * (unordered) and n_groups, exactly as gq_groupby_agg would.  ws must be
 * 256-byte aligned.
 *   inst_status_dev  nullable device int32[n_inst]: receives, per instance,
 *                    GQ_OK or that instance's own device-side error
 *                    (GQ_ERR_DUPLICATE_KEY, GQ_ERR_INVALID_KEY,
 *                    GQ_ERR_CAPACITY, GQ_ERR_TIMEOUT; precedence as in
 *                    gq_status_word).  An error of one instance leaves the
 *                    other instances' outputs exact.
 * Device-side errors of any instance are also recorded in the context's
 * status word.  A foreign key equal to INT64_MIN (the empty-slot marker)
 * matches no build key.  Host errors: GQ_ERR_INVALID_ARG, GQ_ERR_WORKSPACE. */
gq_status gq_batch_join_agg(gq_ctx *ctx, const gq_instance *inst, int n_inst, const gq_tuning *tuning,
                            gq_status *inst_status_dev, void *ws, size_t ws_bytes, gq_stream stream);

/* Autotuner: searches the tunings by coordinate descent over five axes
 * (load factor 0.2..0.7, probe tile 8K..512K rows, lag 1..512, probe fan-out
 * 1..16, build tile 1K..64K keys): from a starting point each axis in turn is
 * swept with the others fixed, each point timed on the stream (a warm-up run,
 * then one timed run), and its best value kept, for up to two rounds.  The
 * fastest tuning goes to *best (its time in *best_ms).  cache_path (nullable)
 * names a text file: a tuning already stored for the same workload signature
 * (device compute units and LDS; per instance m, n, date range and group
 * capacity) is returned without timing; a new result is appended.
 * Synchronizes the stream.  ws must hold
 * gq_batch_autotune_workspace_bytes(inst, n_inst). */
size_t gq_batch_autotune_workspace_bytes(const gq_instance *inst, int n_inst);
gq_status gq_batch_autotune(gq_ctx *ctx, const gq_instance *inst, int n_inst, const char *cache_path,
                            gq_tuning *best, double *best_ms, void *ws, size_t ws_bytes, gq_stream stream);

/* ------------------------------------------------------------------------
 * Served queries: a request loop over tables resident in HBM.
 * The paper's queries are interactive and recurring over data kept resident
 * in HBM (Sec. 4.2); the server admits queries by their memory footprint,
 * batches queries of one template that arrive while others run, and runs a
 * batch as one shared scan of the fact columns (continuous batching).
 * Scheduling: stream 0 takes the oldest waiting query; further streams take
 * only the short templates (FILTER_AGG, FILTER_TOPK), so long joins never
 * share the GPU with each other.  A template's waiting queries become one
 * shared-scan batch once there are enough of them for the shared scan to be
 * cheaper than running them one by one (JOIN_AGG: 2, FILTER_AGG and
 * JOIN2_AGG: 4; FILTER_TOPK: never, its plain form is cheaper); otherwise
 * the query runs alone as the plain operator chain.
 * ------------------------------------------------------------------------ */

#define GQ_QUERY_FILTER_AGG   1   /* date < date_hi, group by disc (key64)          */
#define GQ_QUERY_JOIN_AGG     2   /* + join fk = dim1 key, group by dim1 attr (key32) */
#define GQ_QUERY_JOIN2_AGG    3   /* + join fk = dim1, fk2 = dim2, group by dim2 attr */
#define GQ_QUERY_FILTER_TOPK  4   /* date < date_hi, top-k price (desc, ties by row) */

typedef struct gq_server_tables {
    const int64_t *fk, *fk2;   /* device fact columns, n rows each          */
    const int32_t *date;
    const int64_t *qty, *price, *disc;
    int64_t n;
    const void *dim1_table;    /* join tables from gq_join_build; payload = */
    size_t dim1_table_bytes;   /*   the dimension attribute                 */
    const void *dim2_table;
    size_t dim2_table_bytes;
} gq_server_tables;

typedef struct gq_server_cfg {
    gq_server_tables tables;   /* resident; must outlive the server         */
    void *pool;                /* device memory for query workspaces        */
    size_t pool_bytes;         /*   (caller-owned, 256-byte aligned)        */
    int32_t streams;           /* batches in flight at once, 1..8 (above:
                                  stream 0 any template, others short ones) */
    int32_t max_batch;         /* queries per shared-scan batch, 1..16      */
    int32_t serial;            /* 1: each query alone with the plain
                                  operators, one at a time, arrival order   */
} gq_server_cfg;

typedef struct gq_query {
    int32_t kind;              /* GQ_QUERY_*                                 */
    int32_t k;                 /* top-k size (FILTER_TOPK, 1..256)          */
    int64_t date_hi;           /* keep fact rows with date < date_hi        */
    int64_t max_groups;        /* aggregate templates: groups bound         */
    gq_groups groups;          /* aggregate outputs (device, caller-owned)  */
    int64_t *topk_val;         /* FILTER_TOPK outputs (device, k entries)   */
    int32_t *topk_row;
    int64_t *topk_n;
} gq_query;

typedef struct gq_server gq_server;

/* Start a server on the device of `ctx` (the caller's context, which also
 * receives the message of a failed create).  The server creates a scheduler
 * thread and, per HIP stream, its own context, so that every batch in flight
 * has its own device status word.
 * Errors: GQ_ERR_INVALID_ARG, GQ_ERR_HIP. */
gq_status gq_server_create(gq_ctx *ctx, const gq_server_cfg *cfg, gq_server **out);

/* Queue a query; *ticket identifies it.  The query's output buffers must stay
 * valid until gq_server_wait returns for the ticket.  Thread-safe.
 * Errors: GQ_ERR_INVALID_ARG (bad query), GQ_ERR_CAPACITY (its workspace can
 * never fit the pool), GQ_ERR_UNSUPPORTED (max_groups > 512 for FILTER_AGG or
 * JOIN2_AGG in batched mode, k > 256). */
gq_status gq_server_submit(gq_server *srv, const gq_query *q, uint64_t *ticket);

/* Block until the query has finished on the device; *latency_s = seconds from
 * submit to completion (re-runs included); *query_status = the query's own
 * result: GQ_OK, a launch error (GQ_ERR_HIP), or a device-side error of its
 * kernels, read from its batch's status word when the batch retires
 * (GQ_ERR_CAPACITY: more groups than its output capacity holds, the output
 * then being undefined).  Error handling inside the server: a shared batch
 * that reports an error runs each of its queries again alone, so that only
 * the failing query reports it; a query whose groups overflow max_groups
 * runs again with twice the bound, up to groups.capacity, so its status is
 * GQ_ERR_CAPACITY only when the output arrays themselves are too small.  The
 * caller's recovery is then to submit again with larger output arrays (and
 * max_groups).  Each ticket can be waited for once.  Thread-safe. */
gq_status gq_server_wait(gq_server *srv, uint64_t ticket, gq_status *query_status, double *latency_s);

/* Counters: queries finished, batches launched, largest batch, queries run
 * again after an error (any pointer may be NULL). */
gq_status gq_server_stats(gq_server *srv, int64_t *done, int64_t *batches, int64_t *max_batch_seen,
                          int64_t *reruns);

/* Finish every queued query, stop the scheduler, release its contexts. */
void gq_server_destroy(gq_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* GQ_H */
