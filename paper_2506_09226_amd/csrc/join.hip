// Hash equi-join: open-addressing build and ordered probe.
//
// Table: a 256-byte header then 2^L slots of 16 bytes {int64 key, int32
// payload, int32 unused}; EMPTY key = INT64_MIN.  The home slot of a key is
// the TOP L bits of fmix64(key): the same hash bits that pick a key's radix
// partition, so a probe stream that was partitioned by that hash touches one
// contiguous slice of the table at a time.  Linear probing, wrapping.
//
// Build, small tables: a fill kernel writes header and EMPTY slots; an insert
// kernel claims slots with a 64-bit compare-and-swap in device memory and then
// stores the payload (the probe runs in a later kernel, so it sees the store).
//
// Build, large tables (device-memory CAS runs at only ~10 G/s on MI355X): the
// build rows are sorted by the region of their home slot, a region being
// 4096 consecutive slots: the partition operator by the top 8 hash bits,
// then, for more than 256 regions, one workgroup per bucket splitting it by
// the remaining region bits; one workgroup per region inserts its keys into an LDS copy of the
// region with LDS compare-and-swap and writes the region out linearly.  A key
// whose probe runs past its region's last slot goes to an overflow list and is
// inserted afterwards by device CAS from the first slot of the next region,
// which is exactly where linear probing would continue; the table is the same
// valid linear-probing table either way.
//
// Probe: a tile of probe rows is looked up with one 16-byte load per slot
// visited; matches become a tile bitmap (ballots) and are compacted in probe
// order exactly like the filter: block scan + decoupled look-back + LDS stage.
// The partitioned probe (further below) gives the same output with the table
// reads kept in each XCD's L2.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "gq_device.h"
#include "gq_internal.h"
#include "gq_ops.h"

namespace {

constexpr uint64_t JT_MAGIC = 0x6a6f696e74626c31ull;   // "join tbl1"
constexpr int64_t JT_EMPTY = INT64_MIN;
constexpr size_t JT_HEADER = 256;

struct jt_header {
    uint64_t magic;
    uint32_t log2_slots;
    uint32_t unused;
    uint64_t slots;
};

struct alignas(16) jt_slot {
    int64_t key;
    int32_t payload;
    int32_t unused;
};

int jt_log2_slots(int64_t m, double lf)
{
    double want = static_cast<double>(m) / lf;
    int L = 6;
    while (L < 40 && static_cast<double>(1ull << L) < want) ++L;
    return L;
}

__global__ void jt_init_kernel(void *table, int log2_slots)
{
    const uint64_t slots = 1ull << log2_slots;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        jt_header *h = static_cast<jt_header *>(table);
        h->magic = JT_MAGIC;
        h->log2_slots = static_cast<uint32_t>(log2_slots);
        h->unused = 0;
        h->slots = slots;
    }
    jt_slot *s = reinterpret_cast<jt_slot *>(static_cast<char *>(table) + JT_HEADER);
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < slots; i += stride) {
        jt_slot e;
        e.key = JT_EMPTY;
        e.payload = 0;
        e.unused = 0;
        s[i] = e;
    }
}

__global__ __launch_bounds__(256) void jt_insert_kernel(void *table, int log2_slots, const int64_t *__restrict__ key,
                                                        const int32_t *__restrict__ payload, int64_t m_bound,
                                                        const int64_t *n_dev, const int32_t *__restrict__ sel,
                                                        uint32_t *status)
{
    int64_t m = m_bound;
    if (n_dev) {
        const int64_t d = *n_dev;
        m = d < m_bound ? (d > 0 ? d : 0) : m_bound;
    }
    jt_slot *slots = reinterpret_cast<jt_slot *>(static_cast<char *>(table) + JT_HEADER);
    const uint64_t mask = (1ull << log2_slots) - 1;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += stride) {
        const int64_t r = sel ? static_cast<int64_t>(sel[i]) : i;
        const int64_t k = key[r];
        const int32_t p = payload[r];
        if (k == JT_EMPTY) {
            gq_raise(status, GQ_ERR_INVALID_KEY);
            continue;
        }
        uint64_t s = gq_fmix64(static_cast<uint64_t>(k)) >> (64 - log2_slots);
        uint64_t probes = 0;
        for (; probes <= mask; ++probes) {
            unsigned long long *kp = reinterpret_cast<unsigned long long *>(&slots[s].key);
            const unsigned long long prev =
                atomicCAS(kp, static_cast<unsigned long long>(JT_EMPTY), static_cast<unsigned long long>(k));
            if (prev == static_cast<unsigned long long>(JT_EMPTY)) {
                slots[s].payload = p;
                break;
            }
            if (prev == static_cast<unsigned long long>(k)) {
                gq_raise(status, GQ_ERR_DUPLICATE_KEY);
                break;
            }
            s = (s + 1) & mask;
        }
        if (probes > mask) gq_raise(status, GQ_ERR_CAPACITY);
    }
}

constexpr int JR_BITS = 12;                         // 4096 slots per region (64 KiB)
constexpr int JR_SLOTS = 1 << JR_BITS;
constexpr int JR_MAX_REGION_BITS = 16;              // two 8-bit levels at most
constexpr int64_t JR_MIN_KEYS = 1 << 18;            // below this the CAS build is used

// Second level of the region sort.  The first level is a radix partition by
// the top JS_HIGH bits of the hash; workgroup b takes that partition's bucket
// b and splits it by the next g - JS_HIGH bits, so that the keys end up
// ordered by region (the top g bits) and roff[r] is the first key of region
// r.  It counts its bucket's sub-buckets first (one read of the keys), which
// gives both the region starts and the output cursors, then moves the bucket
// tile by tile: a tile's rows are grouped by sub-bucket in LDS and each group
// is written at its cursor as one run.  Rows keep no particular order inside
// a region; the region kernel's inserts do not depend on it.
constexpr int JS_HIGH = 8;                           // bits of the first level
constexpr int JS_THREADS = 1024;
constexpr int JS_ITEMS = 8;
constexpr int JS_TILE = JS_THREADS * JS_ITEMS;

GQ_DEV uint32_t js_sub(int64_t k, int g, uint32_t smask)
{
    return static_cast<uint32_t>(gq_fmix64(static_cast<uint64_t>(k)) >> (64 - g)) & smask;
}

__global__ __launch_bounds__(JS_THREADS) void jt_split_kernel(const int64_t *__restrict__ k1,
                                                              const int32_t *__restrict__ p1,
                                                              const int64_t *__restrict__ bstart, int64_t m, int g,
                                                              int64_t *__restrict__ k2, int32_t *__restrict__ p2,
                                                              int64_t *__restrict__ roff)
{
    __shared__ uint32_t cnt[1 << JS_HIGH];           // sub-bucket sizes, then a tile's counts
    __shared__ uint32_t tstart[1 << JS_HIGH];        // a tile's sub-bucket starts in the stage
    __shared__ int64_t cur[1 << JS_HIGH];            // output cursor of each sub-bucket
    __shared__ uint32_t scan_smem[JS_THREADS / 64];
    __shared__ uint8_t lsub[JS_TILE];
    __shared__ int64_t sk[JS_TILE];
    __shared__ int32_t sp[JS_TILE];
    const int sb = g - JS_HIGH;                      // 1..8 sub-bucket bits
    const uint32_t S = 1u << sb, smask = S - 1;
    const int tid = threadIdx.x;
    const int64_t b0 = bstart[blockIdx.x], b1 = bstart[blockIdx.x + 1];

    for (uint32_t i = tid; i < S; i += JS_THREADS) cnt[i] = 0;
    __syncthreads();
    for (int64_t i0 = b0; i0 < b1; i0 += 2 * JS_TILE) {
        int64_t kk[2 * JS_ITEMS];
#pragma unroll
        for (int c = 0; c < 2 * JS_ITEMS; ++c) {
            const int64_t e = i0 + c * JS_THREADS + tid;
            kk[c] = e < b1 ? k1[e] : 0;
        }
#pragma unroll
        for (int c = 0; c < 2 * JS_ITEMS; ++c)
            if (i0 + c * JS_THREADS + tid < b1) atomicAdd(&cnt[js_sub(kk[c], g, smask)], 1u);
    }
    __syncthreads();
    uint32_t total;
    const uint32_t excl = gq_block_exclusive_scan<JS_THREADS>(static_cast<uint32_t>(tid) < S ? cnt[tid] : 0u,
                                                              &total, scan_smem);
    if (static_cast<uint32_t>(tid) < S) {
        cur[tid] = b0 + excl;
        roff[(static_cast<int64_t>(blockIdx.x) << sb) + tid] = b0 + excl;
        cnt[tid] = 0;
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) roff[static_cast<int64_t>(gridDim.x) << sb] = m;

    int64_t k[JS_ITEMS];
    int32_t p[JS_ITEMS];
    auto load_tile = [&](int64_t i0) {
#pragma unroll
        for (int c = 0; c < JS_ITEMS; ++c) {
            const int64_t e = i0 + c * JS_THREADS + tid;
            const bool v = e < b1;
            k[c] = v ? k1[e] : 0;
            p[c] = v ? p1[e] : 0;
        }
    };
    if (b0 < b1) load_tile(b0);
    __syncthreads();
    for (int64_t i0 = b0; i0 < b1; i0 += JS_TILE) {
        uint32_t l[JS_ITEMS], rank[JS_ITEMS];
#pragma unroll
        for (int c = 0; c < JS_ITEMS; ++c) {
            l[c] = js_sub(k[c], g, smask);
            if (i0 + c * JS_THREADS + tid < b1) rank[c] = atomicAdd(&cnt[l[c]], 1u);
        }
        gq_lds_barrier();
        uint32_t tot;
        const uint32_t st = gq_block_exclusive_scan_lds<JS_THREADS>(
            static_cast<uint32_t>(tid) < S ? cnt[tid] : 0u, &tot, scan_smem);
        if (static_cast<uint32_t>(tid) < S) tstart[tid] = st;
        gq_lds_barrier();
#pragma unroll
        for (int c = 0; c < JS_ITEMS; ++c) {
            if (i0 + c * JS_THREADS + tid < b1) {
                const uint32_t q = tstart[l[c]] + rank[c];
                sk[q] = k[c];
                sp[q] = p[c];
                lsub[q] = static_cast<uint8_t>(l[c]);
            }
        }
        const int64_t next = i0 + JS_TILE;
        if (next < b1) load_tile(next);              // in flight while this tile is written
        gq_lds_barrier();
        const uint32_t count = static_cast<uint32_t>(b1 - i0 < JS_TILE ? b1 - i0 : JS_TILE);
        for (uint32_t q = tid; q < count; q += JS_THREADS) {
            const uint32_t x = lsub[q];
            const int64_t dst = cur[x] + (q - tstart[x]);
            k2[dst] = sk[q];
            p2[dst] = sp[q];
        }
        gq_lds_barrier();
        if (static_cast<uint32_t>(tid) < S) {
            cur[tid] += cnt[tid];
            cnt[tid] = 0;
        }
        gq_lds_barrier();
    }
}

// A persistent grid walks the regions; the barriers between a region's phases
// order LDS only, so one region's table stores drain while the next region's
// keys load.  A thread's keys of a region (up to JR_BATCH, a region holding
// about 2048 * load factor keys) are loaded together, and the next region's
// are loaded before the current region is written out.
constexpr int JR_THREADS = 256;
constexpr int JR_BATCH = 8;                          // keys per thread loaded together

__global__ __launch_bounds__(JR_THREADS) void jt_region_kernel(void *table, int L, const int64_t *__restrict__ keys,
                                                               const int32_t *__restrict__ pay,
                                                               const int64_t *__restrict__ roff, int64_t nregions,
                                                               int64_t *__restrict__ ovf_key,
                                                               int32_t *__restrict__ ovf_pay, uint32_t *ovf_cnt,
                                                               int64_t ovf_cap, uint32_t *status)
{
    __shared__ unsigned long long sk[JR_SLOTS];
    __shared__ int32_t sp[JR_SLOTS];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        jt_header *h = static_cast<jt_header *>(table);
        h->magic = JT_MAGIC;
        h->log2_slots = static_cast<uint32_t>(L);
        h->unused = 0;
        h->slots = 1ull << L;
    }
    int64_t k[JR_BATCH];
    int32_t p[JR_BATCH];
    bool v[JR_BATCH];
    auto load_batch = [&](int64_t i0, int64_t end) {
#pragma unroll
        for (int c = 0; c < JR_BATCH; ++c) {
            const int64_t i = i0 + c * JR_THREADS + threadIdx.x;
            v[c] = i < end;
            k[c] = v[c] ? keys[i] : 0;
            p[c] = v[c] ? pay[i] : 0;
        }
    };
    int64_t region = blockIdx.x;
    int64_t r0 = 0, r1 = 0;
    if (region < nregions) {
        r0 = roff[region];
        r1 = roff[region + 1];
        load_batch(r0, r1);
    }
    for (; region < nregions; region += gridDim.x) {
        gq_lds_barrier();                             // the previous region is read out of LDS
        for (int j = threadIdx.x; j < JR_SLOTS; j += JR_THREADS) {
            sk[j] = static_cast<unsigned long long>(JT_EMPTY);
            sp[j] = 0;
        }
        gq_lds_barrier();
        for (int64_t i0 = r0;;) {
#pragma unroll
            for (int c = 0; c < JR_BATCH; ++c) {
                if (!v[c]) continue;
                if (k[c] == JT_EMPTY) {
                    gq_raise(status, GQ_ERR_INVALID_KEY);
                    continue;
                }
                uint32_t loc =
                    static_cast<uint32_t>(gq_fmix64(static_cast<uint64_t>(k[c])) >> (64 - L)) & (JR_SLOTS - 1);
                while (true) {
                    const unsigned long long prev = atomicCAS(&sk[loc], static_cast<unsigned long long>(JT_EMPTY),
                                                              static_cast<unsigned long long>(k[c]));
                    if (prev == static_cast<unsigned long long>(JT_EMPTY)) {
                        sp[loc] = p[c];
                        break;
                    }
                    if (prev == static_cast<unsigned long long>(k[c])) {
                        gq_raise(status, GQ_ERR_DUPLICATE_KEY);
                        break;
                    }
                    if (++loc == JR_SLOTS) {             // continue in the next region, later
                        const uint32_t idx = atomicAdd(ovf_cnt, 1u);
                        if (idx < ovf_cap) {
                            ovf_key[idx] = k[c];
                            ovf_pay[idx] = p[c];
                        } else {
                            gq_raise(status, GQ_ERR_CAPACITY);
                        }
                        break;
                    }
                }
            }
            i0 += JR_THREADS * JR_BATCH;
            if (i0 >= r1) break;
            load_batch(i0, r1);                          // a region with more keys than one batch
        }
        const int64_t next = region + gridDim.x;         // the next region's keys: in flight meanwhile
        if (next < nregions) {
            r0 = roff[next];
            r1 = roff[next + 1];
            load_batch(r0, r1);
        }
        gq_lds_barrier();
        jt_slot *slots = reinterpret_cast<jt_slot *>(static_cast<char *>(table) + JT_HEADER) +
                         (static_cast<uint64_t>(region) << JR_BITS);
        for (int j = threadIdx.x; j < JR_SLOTS; j += JR_THREADS) {
            jt_slot e;
            e.key = static_cast<int64_t>(sk[j]);
            e.payload = sp[j];
            e.unused = 0;
            slots[j] = e;
        }
    }
}

__global__ __launch_bounds__(256) void jt_overflow_kernel(void *table, int L, const int64_t *__restrict__ ovf_key,
                                                          const int32_t *__restrict__ ovf_pay,
                                                          const uint32_t *ovf_cnt, int64_t ovf_cap, uint32_t *status)
{
    const int64_t cnt = *ovf_cnt;
    const int64_t n = cnt < ovf_cap ? cnt : ovf_cap;
    jt_slot *slots = reinterpret_cast<jt_slot *>(static_cast<char *>(table) + JT_HEADER);
    const uint64_t mask = (1ull << L) - 1;
    const int g = L - JR_BITS;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t k = ovf_key[i];
        const uint64_t home_region = gq_fmix64(static_cast<uint64_t>(k)) >> (64 - g);
        uint64_t s = ((home_region + 1) << JR_BITS) & mask;
        uint64_t probes = 0;
        for (; probes <= mask; ++probes) {
            unsigned long long *kp = reinterpret_cast<unsigned long long *>(&slots[s].key);
            const unsigned long long prev =
                atomicCAS(kp, static_cast<unsigned long long>(JT_EMPTY), static_cast<unsigned long long>(k));
            if (prev == static_cast<unsigned long long>(JT_EMPTY)) {
                slots[s].payload = ovf_pay[i];
                break;
            }
            if (prev == static_cast<unsigned long long>(k)) {
                gq_raise(status, GQ_ERR_DUPLICATE_KEY);
                break;
            }
            s = (s + 1) & mask;
        }
        if (probes > mask) gq_raise(status, GQ_ERR_CAPACITY);
    }
}

int table_log2_from_bytes(size_t table_bytes)
{
    int L = 6;
    while (L < 40 && JT_HEADER + (size_t(2) << L) * sizeof(jt_slot) <= table_bytes) ++L;
    return L;
}

// Which build a call takes: "region" for large tables built from whole
// columns, "cas" otherwise.  GQ_JOIN_BUILD=cas|region forces one (testing).
bool use_region_build(int64_t m, int L, bool has_sel_or_count)
{
    const int g = L - JR_BITS;
    if (has_sel_or_count || g < 1 || g > JR_MAX_REGION_BITS) return false;
    const char *e = getenv("GQ_JOIN_BUILD");
    if (e && strcmp(e, "cas") == 0) return false;
    if (e && strcmp(e, "region") == 0) return true;
    return m >= JR_MIN_KEYS;
}

struct build_ws {
    int64_t *k1, *k2;
    int32_t *p1, *p2;
    int64_t *offsets;
    int64_t *roff;
    void *part_ws;
    int64_t *ovf_key;
    int32_t *ovf_pay;
    uint32_t *ovf_cnt;
    int64_t ovf_cap;
};

build_ws build_layout(gq_carver &c, int64_t m)
{
    build_ws w{};
    const size_t rows = static_cast<size_t>(m > 0 ? m : 1);
    w.ovf_cnt = c.take<uint32_t>(64);
    w.k1 = c.take<int64_t>(rows);
    w.k2 = c.take<int64_t>(rows);
    w.p1 = c.take<int32_t>(rows);
    w.p2 = c.take<int32_t>(rows);
    w.offsets = c.take<int64_t>(257);
    w.roff = c.take<int64_t>((size_t(1) << JR_MAX_REGION_BITS) + 1);
    w.part_ws = c.take<char>(gq_partition_bits_workspace(m, 8));
    w.ovf_cap = m / 8 + 1024;
    w.ovf_key = c.take<int64_t>(static_cast<size_t>(w.ovf_cap));
    w.ovf_pay = c.take<int32_t>(static_cast<size_t>(w.ovf_cap));
    return w;
}

gq_status region_build(gq_ctx *ctx, const int64_t *key, const int32_t *payload, int64_t m, void *table, int L,
                       void *ws, hipStream_t s)
{
    gq_carver c(ws);
    build_ws w = build_layout(c, m);
    const int g = L - JR_BITS;
    const int32_t pbytes = 4;
    static const gq_part_names nm{"gq_join_build_part_hist", "gq_join_build_part_scan", "gq_join_build_part_offsets",
                                  "gq_join_build_part_scatter"};
    GQ_TRY(gq_zero(ctx, w.ovf_cnt, 64, s));
    void *in[1] = {const_cast<int32_t *>(payload)};
    if (g <= JS_HIGH) {                             // one pass: its bucket starts are the region starts
        void *out[1] = {w.p2};
        GQ_TRY(gq_partition_bits(ctx, key, m, g, 64 - g, 1, in, &pbytes, w.k2, out, w.roff, w.part_ws, s, nm, 8));
    } else {                                        // the top JS_HIGH bits, then each bucket by the rest
        void *out[1] = {w.p1};
        GQ_TRY(gq_partition_bits(ctx, key, m, JS_HIGH, 64 - JS_HIGH, 1, in, &pbytes, w.k1, out, w.offsets, w.part_ws,
                                 s, nm, 8));
        GQ_TRY(gq_launch(ctx, "gq_join_build_split", jt_split_kernel, dim3(1u << JS_HIGH), dim3(JS_THREADS), 0, s,
                         static_cast<const int64_t *>(w.k1), static_cast<const int32_t *>(w.p1),
                         static_cast<const int64_t *>(w.offsets), m, g, w.k2, w.p2, w.roff));
    }
    const int64_t nregions = int64_t(1) << g;
    const uint32_t rgrid = static_cast<uint32_t>(std::min<int64_t>(nregions, int64_t(ctx->num_cus) * 3));
    GQ_TRY(gq_launch(ctx, "gq_join_build_regions", jt_region_kernel, dim3(rgrid), dim3(JR_THREADS), 0, s, table, L,
                     static_cast<const int64_t *>(w.k2), static_cast<const int32_t *>(w.p2),
                     static_cast<const int64_t *>(w.roff), nregions, w.ovf_key, w.ovf_pay, w.ovf_cnt, w.ovf_cap,
                     ctx->status_dev));
    return gq_launch(ctx, "gq_join_build_overflow", jt_overflow_kernel, dim3(64), dim3(256), 0, s, table, L,
                     static_cast<const int64_t *>(w.ovf_key), static_cast<const int32_t *>(w.ovf_pay),
                     static_cast<const uint32_t *>(w.ovf_cnt), w.ovf_cap, ctx->status_dev);
}

constexpr int JP_THREADS = 256;
constexpr int JP_ITEMS = 16;
constexpr int JP_TILE = JP_THREADS * JP_ITEMS;    // 4096 probes
constexpr int JP_WORDS = JP_TILE / 64;

struct probe_ws {
    uint32_t *tile_ctr;
    uint64_t *status;
};

probe_ws probe_layout(gq_carver &c, int64_t n)
{
    probe_ws w;
    const int64_t tiles = (n + JP_TILE - 1) / JP_TILE;
    w.tile_ctr = c.take<uint32_t>(64);
    w.status = c.take<uint64_t>(static_cast<size_t>(tiles > 0 ? tiles : 1));
    return w;
}

template <bool HAS_SEL>
__global__ __launch_bounds__(JP_THREADS) void jt_probe_kernel(const void *table, const int64_t *__restrict__ fk,
                                                              int64_t n_bound, const int64_t *n_dev,
                                                              const int32_t *__restrict__ sel,
                                                              int32_t *__restrict__ prow_out,
                                                              int32_t *__restrict__ pay_out, int64_t *n_out,
                                                              uint32_t *tile_ctr, uint64_t *lb_status)
{
    __shared__ uint64_t bits[JP_WORDS];
    __shared__ int32_t pay_elem[JP_TILE];
    __shared__ int32_t stage_row[JP_TILE];
    __shared__ int32_t stage_pay[JP_TILE];
    __shared__ uint32_t scan_smem[JP_THREADS / 64];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_goff;

    int64_t n = n_bound;
    if (n_dev) {
        const int64_t d = *n_dev;
        n = d < n_bound ? (d > 0 ? d : 0) : n_bound;
    }
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    const int64_t ntiles = (n + JP_TILE - 1) / JP_TILE;
    if (static_cast<int64_t>(t) >= ntiles) {
        if (t == 0 && threadIdx.x == 0) *n_out = 0;
        return;
    }
    const jt_header *hdr = static_cast<const jt_header *>(table);
    const int L = static_cast<int>(hdr->log2_slots);
    const uint64_t mask = (1ull << L) - 1;
    const jt_slot *slots = reinterpret_cast<const jt_slot *>(static_cast<const char *>(table) + JT_HEADER);
    const int64_t base = static_cast<int64_t>(t) * JP_TILE;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    int64_t k[JP_ITEMS];
#pragma unroll
    for (int c = 0; c < JP_ITEMS; ++c) {
        const int64_t e = base + c * JP_THREADS + wave * 64 + lane;
        k[c] = JT_EMPTY;
        if (e < n) k[c] = fk[HAS_SEL ? static_cast<int64_t>(sel[e]) : e];
    }
    uint64_t s[JP_ITEMS];
    int4 v[JP_ITEMS];
#pragma unroll
    for (int c = 0; c < JP_ITEMS; ++c) {
        s[c] = gq_fmix64(static_cast<uint64_t>(k[c])) >> (64 - L);
        v[c] = *reinterpret_cast<const int4 *>(&slots[s[c]]);
    }
#pragma unroll
    for (int c = 0; c < JP_ITEMS; ++c) {
        const int64_t e = base + c * JP_THREADS + wave * 64 + lane;
        bool hit = false;
        int32_t pay = 0;
        if (e < n && k[c] != JT_EMPTY) {
            int64_t sk = (static_cast<int64_t>(static_cast<uint32_t>(v[c].y)) << 32) | static_cast<uint32_t>(v[c].x);
            uint64_t probes = 0;
            while (sk != k[c] && sk != JT_EMPTY && probes < mask) {
                s[c] = (s[c] + 1) & mask;
                v[c] = *reinterpret_cast<const int4 *>(&slots[s[c]]);
                sk = (static_cast<int64_t>(static_cast<uint32_t>(v[c].y)) << 32) | static_cast<uint32_t>(v[c].x);
                ++probes;
            }
            hit = sk == k[c];
            pay = v[c].z;
        }
        const int elem = c * JP_THREADS + wave * 64 + lane;
        pay_elem[elem] = pay;
        const uint64_t b = gq_ballot(hit);
        if (lane == 0) bits[c * (JP_THREADS / 64) + wave] = b;
    }
    __syncthreads();

    // thread i owns tile elements [16 i, 16 i + 16)
    uint32_t mine = static_cast<uint32_t>(bits[threadIdx.x >> 2] >> ((threadIdx.x & 3) * 16)) & 0xffffu;
    uint32_t total;
    uint32_t pos = gq_block_exclusive_scan<JP_THREADS>(static_cast<uint32_t>(__popc(mine)), &total, scan_smem);
    if (wave == 0) {
        const uint64_t g = gq_lookback(lb_status, t, total);
        if (lane == 0) s_goff = g;
    }
    const int elem0 = threadIdx.x * JP_ITEMS;
    while (mine) {
        const int i = __builtin_ctz(mine);
        mine &= mine - 1;
        const int64_t e = base + elem0 + i;
        stage_row[pos] = HAS_SEL ? sel[e] : static_cast<int32_t>(e);
        stage_pay[pos] = pay_elem[elem0 + i];
        ++pos;
    }
    __syncthreads();
    const int64_t goff = static_cast<int64_t>(s_goff);
    for (uint32_t i = threadIdx.x; i < total; i += JP_THREADS) {
        prow_out[goff + i] = stage_row[i];
        pay_out[goff + i] = stage_pay[i];
    }
    if (static_cast<int64_t>(t) == ntiles - 1 && threadIdx.x == 0) *n_out = goff + total;
}


// ------------------------------------------------------------------------
// Partitioned probe: the probes of one table region are answered from an LDS
// copy of that region, and the output order is restored tile by tile.
//
// A region is 4096 consecutive table slots (64 KB).  Its id is the top
// rbits = L - 12 bits of fmix64(key), split as (high part, sub-region): the
// high part is the top H bits, which a probe stream radix-partitioned by H
// or more hash bits (the partition operator on the same hash) holds constant
// along long runs of rows; the sub-region is the next S = rbits - H <= 8 bits.
//   split:   tile t of 4096 probe rows takes the high part of its first row.
//            Its rows are regrouped (stable) in LDS into 2^S sub-region lists
//            plus a stray list (rows of another high part, e.g. where a tile
//            straddles two partition buckets), and written to pool positions
//            [4096 t, 4096 t + rows) as (key, index of the row in the tile),
//            with the list starts of the tile.  Strays are probed right here
//            against the table in device memory.  The tile range of each high
//            part is recorded (atomic min / max).
//   region:  a persistent grid takes regions in order from a counter.  For
//            region (v, u) a workgroup loads the 4096 slots into LDS, then
//            walks the tiles of high part v in batches of 256 (one per
//            thread), gathers the run of list u of every tile, and looks each
//            key up in LDS; a probe sequence that runs past the region's last
//            slot continues in device memory, exactly as linear probing does.
//            The payload, or -1 for a miss, goes to the entry's pool position.
//   compact: per tile, the results are put back in probe order in LDS (by
//            the stored in-tile index) and compacted exactly like the
//            ordered probe (block scan + decoupled look-back).
// The output is therefore identical to the ordered probe's.  Tables with
// fewer than 2^20 slots (cache resident) or whose regions the tile split
// cannot separate (rbits - H > 8) take the ordered probe instead.
// ------------------------------------------------------------------------
constexpr int JX_THREADS = 256;
constexpr int JX_ITEMS = 16;
constexpr int JX_TILE = JX_THREADS * JX_ITEMS;          // probe rows per split tile
constexpr int JX_RBITS = 12;                            // region = 4096 slots
constexpr int JX_REGION = 1 << JX_RBITS;
constexpr int JX_MAX_S = 8;                             // sub-region bits split per tile
constexpr int JX_MAX_H = 8;                             // high-part bits (bounds arrays)
constexpr int JX_LISTS = (1 << JX_MAX_S) + 1;           // sub-region lists + the stray list
constexpr int JX_STARTS = 260;                          // per tile: list starts (JX_LISTS + 1 used)
constexpr int JX_WIN = 2048;                            // region kernel: entries per window
constexpr uint32_t JX_HEAVY_RUN = 256;                  // a tile's run longer than this counts to its region's weight
constexpr int JX_MAX_REGIONS = 1 << (JX_MAX_H + JX_MAX_S);
constexpr int JX_PLAN_THREADS = 1024;

struct jx_geom {
    int L;                  // log2 table slots
    int H;                  // high-part bits
    int S;                  // sub-region bits
    int nregions;           // 2^(H + S)
};

struct jx_ws {
    uint32_t *ctr;          // [0] region counter, [16] heavy-run flag, [32] compaction tile counter
    uint32_t *hp_first;     // per high part: ntiles - first tile (0: none)
    uint32_t *hp_end;       // per high part: last tile + 1 (0: none)
    uint64_t *status;       // compaction look-back words, one per tile
    uint32_t *rw;           // per region: probe rows in its heavy runs (runs > JX_HEAVY_RUN rows)
    uint32_t *iprefix;      // per region: work items before it; [nregions] = all items
    int32_t *tile_hp;       // high part of each tile's lists, -1 for an empty tile
    uint16_t *starts;       // per tile: JX_STARTS list starts
    int64_t *skey;          // pool: probe keys
    uint16_t *sidx;         // pool: index of the probe row inside its tile
    int64_t *res;           // pool: payload of the match, -1 for none
    int64_t ntiles;
};

jx_ws jx_layout(gq_carver &c, int64_t n)
{
    jx_ws w;
    const int64_t rows = n > 0 ? n : 1;
    w.ntiles = (rows + JX_TILE - 1) / JX_TILE;
    w.ctr = c.take<uint32_t>(64);
    w.hp_first = c.take<uint32_t>(1 << JX_MAX_H);
    w.hp_end = c.take<uint32_t>(1 << JX_MAX_H);
    w.status = c.take<uint64_t>(static_cast<size_t>(w.ntiles));
    w.rw = c.take<uint32_t>(JX_MAX_REGIONS);
    w.iprefix = c.take<uint32_t>(JX_MAX_REGIONS + 1);
    w.tile_hp = c.take<int32_t>(static_cast<size_t>(w.ntiles));     // first word after the zeroed prefix
    w.starts = c.take<uint16_t>(static_cast<size_t>(w.ntiles) * JX_STARTS);
    w.skey = c.take<int64_t>(static_cast<size_t>(rows));
    w.sidx = c.take<uint16_t>(static_cast<size_t>(rows));
    w.res = c.take<int64_t>(static_cast<size_t>(rows));
    return w;
}

GQ_DEV int64_t jx_eff_n(int64_t bound, const int64_t *n_dev)
{
    if (!n_dev) return bound;
    const int64_t d = *n_dev;
    return d < bound ? (d > 0 ? d : 0) : bound;
}

// Linear probing in device memory from slot s; payload or -1.
GQ_DEV int64_t jx_probe_global(const jt_slot *slots, uint64_t mask, uint64_t s, int64_t k, uint64_t probes)
{
    for (; probes <= mask; ++probes) {
        const int4 v = *reinterpret_cast<const int4 *>(&slots[s]);
        const int64_t sk = (static_cast<int64_t>(static_cast<uint32_t>(v.y)) << 32) | static_cast<uint32_t>(v.x);
        if (sk == k) return static_cast<int64_t>(static_cast<uint32_t>(v.z));
        if (sk == JT_EMPTY) return -1;
        s = (s + 1) & mask;
    }
    return -1;
}

// Stable split of one tile.  Rows are wave-contiguous (wave w holds rows
// [1024 w, 1024 w + 1024) of the tile, item c its rows 64 c + lane); a row's
// place is its list's start in the tile, plus the rows of that list in
// earlier waves, plus the rows of that list already seen by its wave, plus
// its rank among its wave's lanes with the same list (S + 1 ballots).
constexpr int JX_SPLIT_THREADS = 512;
template <bool HAS_SEL, int ST>
__global__ __launch_bounds__(ST) void jx_split_kernel(const void *table, const int64_t *__restrict__ fk,
                                                              int64_t n_bound, const int64_t *n_dev,
                                                              const int32_t *__restrict__ sel, jx_geom gm, jx_ws w,
                                                              uint32_t *status)
{
    constexpr int ITEMS = JX_TILE / ST;                   // rows per thread
    constexpr int WAVES = ST / 64;
    constexpr int WROWS = JX_TILE / WAVES;
    constexpr int LPT = (JX_LISTS + ST - 1) / ST;         // lists per thread in the list scan
    __shared__ uint32_t wcnt[WAVES][JX_LISTS];            // per wave: running counts, then prefixes
    __shared__ uint32_t lstart[LPT * ST + 1];
    __shared__ uint32_t scan_smem[WAVES];
    __shared__ int64_t stage_k[JX_TILE];
    __shared__ uint16_t stage_i[JX_TILE];
    __shared__ int32_t s_hp;
    const int64_t n = jx_eff_n(n_bound, n_dev);
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * JX_TILE;
    const int64_t rows = n - base < JX_TILE ? n - base : JX_TILE;
    const bool bad_table = static_cast<const jt_header *>(table)->log2_slots != static_cast<uint32_t>(gm.L);
    if (rows <= 0 || bad_table) {                          // uniform: a tile past the end, or a wrong table size
        if (threadIdx.x == 0) {
            w.tile_hp[tile] = -1;
            if (bad_table) gq_raise(status, GQ_ERR_INVALID_ARG);
        }
        return;
    }
    const jt_slot *slots = reinterpret_cast<const jt_slot *>(static_cast<const char *>(table) + JT_HEADER);
    const uint64_t mask = (1ull << gm.L) - 1;
    const int rbits = gm.L - JX_RBITS;
    const uint32_t stray = 1u << gm.S;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < WAVES * JX_LISTS; i += ST) (&wcnt[0][0])[i] = 0;
    int32_t r[ITEMS];
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int q = wave * WROWS + c * 64 + lane;          // index in the tile
        r[c] = 0;
        if (q < rows) r[c] = HAS_SEL ? sel[base + q] : static_cast<int32_t>(base + q);
    }
    int64_t k[ITEMS];
    uint32_t reg[ITEMS];
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int q = wave * WROWS + c * 64 + lane;
        k[c] = q < rows ? fk[r[c]] : 0;
        reg[c] = static_cast<uint32_t>(gq_fmix64(static_cast<uint64_t>(k[c])) >> (64 - rbits));
    }
    if (threadIdx.x == 0) s_hp = static_cast<int32_t>(reg[0] >> gm.S);
    __syncthreads();
    const uint32_t hp = static_cast<uint32_t>(s_hp);
    uint32_t pos[ITEMS];                               // list << 16 | rank in (wave, list)
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int q = wave * WROWS + c * 64 + lane;
        const bool valid = q < rows;
        const uint32_t x = (reg[c] >> gm.S) == hp ? (reg[c] & (stray - 1)) : stray;
        uint64_t match = gq_ballot(valid);
        for (int bit = 0; bit <= gm.S; ++bit) {
            const bool set = (x >> bit) & 1u;
            const uint64_t bal = gq_ballot(valid && set);
            match &= set ? bal : ~bal;
        }
        const uint32_t below = gq_mbcnt(match);
        const uint32_t cnt = static_cast<uint32_t>(__popcll(match));
        uint32_t old = 0;
        if (valid) old = wcnt[wave][x];
        if (valid && below == cnt - 1) wcnt[wave][x] = old + cnt;
        pos[c] = (x << 16) | (old + below);
    }
    __syncthreads();
    // per list: prefix over waves; thread i owns lists LPT i .. LPT i + LPT - 1
    uint32_t tot[LPT];
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        const int x = LPT * threadIdx.x + j;
        uint32_t run = 0;
        if (x < JX_LISTS) {
#pragma unroll
            for (int v = 0; v < WAVES; ++v) {
                const uint32_t t = wcnt[v][x];
                wcnt[v][x] = run;
                run += t;
            }
        }
        tot[j] = run;
    }
#pragma unroll
    for (int j = 0; j < LPT; ++j) {                       // a heavy key's region: its long runs are weighed
        const int x = LPT * threadIdx.x + j;
        if (x < (1 << gm.S) && tot[j] > JX_HEAVY_RUN) {
            atomicAdd(&w.rw[(hp << gm.S) + x], tot[j]);
            __hip_atomic_store(&w.ctr[16], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < LPT; ++j) mine += tot[j];
    uint32_t all;
    uint32_t excl = gq_block_exclusive_scan<ST>(mine, &all, scan_smem);
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
        lstart[LPT * threadIdx.x + j] = excl;
        excl += tot[j];
    }
    if (threadIdx.x == 0) lstart[LPT * ST] = all;
    __syncthreads();
    for (uint32_t x = threadIdx.x; x <= stray + 1; x += ST)
        w.starts[tile * JX_STARTS + x] = static_cast<uint16_t>(lstart[x]);
    if (threadIdx.x == 0) {
        w.tile_hp[tile] = static_cast<int32_t>(hp);
        atomicMax(&w.hp_first[hp], static_cast<uint32_t>(w.ntiles - tile));
        atomicMax(&w.hp_end[hp], static_cast<uint32_t>(tile + 1));
    }
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int q = wave * WROWS + c * 64 + lane;
        if (q < rows) {
            const uint32_t x = pos[c] >> 16;
            const uint32_t p = lstart[x] + wcnt[wave][x] + (pos[c] & 0xffffu);
            stage_k[p] = k[c];
            stage_i[p] = static_cast<uint16_t>(q);
            if (x == stray) {                              // probed here, in device memory
                const uint64_t s = gq_fmix64(static_cast<uint64_t>(k[c])) >> (64 - gm.L);
                w.res[base + p] = k[c] == JT_EMPTY ? -1 : jx_probe_global(slots, mask, s, k[c], 0);
            }
        }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < static_cast<uint32_t>(rows); q += ST) {
        w.skey[base + q] = stage_k[q];
        w.sidx[base + q] = stage_i[q];
    }
}

// Work items of the region pass: a region whose heavy runs hold more than
// item_rows probe rows (a heavy key's region) becomes ceil(weight / item_rows)
// items over equal ranges of its high part's tiles; every other region is one
// item.  iprefix[r] = items before region r.  One workgroup.
__global__ __launch_bounds__(JX_PLAN_THREADS) void jx_plan_kernel(const uint32_t *__restrict__ rw, int nregions,
                                                                  uint32_t item_rows, const uint32_t *heavy,
                                                                  uint32_t *__restrict__ iprefix)
{
    __shared__ uint32_t scan_smem[JX_PLAN_THREADS / 64];
    if (*heavy == 0u) {                                    // no heavy run anywhere: one item per region
        if (threadIdx.x == 0) iprefix[nregions] = static_cast<uint32_t>(nregions);
        return;
    }
    const int per = (nregions + JX_PLAN_THREADS - 1) / JX_PLAN_THREADS;   // consecutive regions per thread
    const int r0 = static_cast<int>(threadIdx.x) * per;
    auto items = [&](int r) { return rw[r] > item_rows ? (rw[r] + item_rows - 1) / item_rows : 1u; };
    uint32_t mine = 0;
    for (int r = r0; r < r0 + per && r < nregions; ++r) mine += items(r);
    uint32_t total;
    uint32_t run = gq_block_exclusive_scan<JX_PLAN_THREADS>(mine, &total, scan_smem);
    for (int r = r0; r < r0 + per && r < nregions; ++r) {
        iprefix[r] = run;
        run += items(r);
    }
    if (threadIdx.x == 0) iprefix[nregions] = total;
}

// Region probes from LDS (see above).  Persistent: work items (a region, or
// one tile range of a heavy region) come from w.ctr[0].  RT threads: a batch
// is RT tiles, a window gives each thread JX_WIN / RT entries.
constexpr int JR_THREADS_PROBE = 512;
template <int RT>
__global__ __launch_bounds__(RT) void jx_region_kernel(const void *table, jx_geom gm, jx_ws w)
{
    using map_t = std::conditional_t<(RT <= 256), uint8_t, uint16_t>;
    __shared__ __align__(16) int64_t lkey[JX_REGION];
    __shared__ int32_t lpay[JX_REGION];
    __shared__ map_t map[JX_WIN];                         // window entry -> batch tile (thread)
    __shared__ int32_t b_at[RT];                          // pool position of each batch tile's run
    __shared__ uint32_t b_pos[RT];                        // exclusive prefix of the runs' lengths
    __shared__ uint32_t scan_smem[RT / 64];
    __shared__ int64_t s_item;
    if (static_cast<const jt_header *>(table)->log2_slots != static_cast<uint32_t>(gm.L)) return;   // uniform
    const jt_slot *slots = reinterpret_cast<const jt_slot *>(static_cast<const char *>(table) + JT_HEADER);
    const uint64_t mask = (1ull << gm.L) - 1;
    const uint32_t nitems = static_cast<uint32_t>(gq_uniform(w.iprefix[gm.nregions]));   // written by the plan pass
    // As in every persistent loop here, a barrier opens each pass so the
    // thread-0 dequeue never merges with thread-0 work of the previous pass.
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = static_cast<int64_t>(atomicAdd(&w.ctr[0], 1u));
        __syncthreads();
        const uint32_t wi = static_cast<uint32_t>(gq_uniform(s_item));
        if (wi >= nitems) break;                           // same value in every thread
        int64_t item = wi;                                 // the region (with no split region, the item itself)
        uint32_t part = 0, nparts = 1;                     // this item's share of the region's tiles
        if (nitems != static_cast<uint32_t>(gm.nregions)) {
            item = 0;                                      // last r with iprefix[r] <= wi
            for (int64_t hi = gm.nregions - 1; item < hi;) {
                const int64_t mid = (item + hi + 1) >> 1;
                if (w.iprefix[mid] <= wi) item = mid;
                else hi = mid - 1;
            }
            part = wi - w.iprefix[item];
            nparts = w.iprefix[item + 1] - w.iprefix[item];
        }
        const uint32_t hp = static_cast<uint32_t>(item) >> gm.S;
        const uint32_t sub = static_cast<uint32_t>(item) & ((1u << gm.S) - 1);
        const jt_slot *rs = slots + (static_cast<uint64_t>(item) << JX_RBITS);
        for (int j = threadIdx.x; j < JX_REGION; j += RT) {
            const int4 v = *reinterpret_cast<const int4 *>(&rs[j]);
            lkey[j] = (static_cast<int64_t>(static_cast<uint32_t>(v.y)) << 32) | static_cast<uint32_t>(v.x);
            lpay[j] = v.z;
        }
        const uint32_t first_c = w.hp_first[hp], end = w.hp_end[hp];
        const int64_t hp_lo = gq_uniform(first_c ? w.ntiles - static_cast<int64_t>(first_c) : 0);
        const int64_t hp_hi = gq_uniform(static_cast<int64_t>(end));
        const int64_t span = hp_hi > hp_lo ? (hp_hi - hp_lo + nparts - 1) / nparts : 0;
        const int64_t t_lo = hp_lo + static_cast<int64_t>(part) * span;
        const int64_t t_hi = t_lo + span < hp_hi ? t_lo + span : hp_hi;
        // the run of list `sub` in tile t (length 0 if t is not a tile of this high part)
        auto run_of = [&](int64_t t, uint32_t &len, int32_t &at) {
            len = 0;
            at = 0;
            if (t < t_hi) {
                const int32_t thp = w.tile_hp[t];
                const uint32_t a = w.starts[t * JX_STARTS + sub], b = w.starts[t * JX_STARTS + sub + 1];
                if (thp == static_cast<int32_t>(hp)) {
                    len = b - a;
                    at = static_cast<int32_t>(t * JX_TILE + a);
                }
            }
        };
        uint32_t len;
        int32_t at;
        run_of(t_lo + threadIdx.x, len, at);
        // Communication inside the item goes through LDS only, so its barriers
        // order LDS alone: the region's loads, the next batch's run lookups
        // and the result stores stay in flight across them.
        gq_lds_barrier();                                  // the region is in LDS
        for (int64_t t0 = t_lo; t0 < t_hi; t0 += RT) {
            uint32_t nlen;
            int32_t nat;
            run_of(t0 + RT + threadIdx.x, nlen, nat);      // next batch, in flight meanwhile
            uint32_t total;
            const uint32_t pos = gq_block_exclusive_scan_lds<RT>(len, &total, scan_smem);
            b_at[threadIdx.x] = at;
            b_pos[threadIdx.x] = pos;
            const uint32_t ntot = static_cast<uint32_t>(gq_uniform(total));
            for (uint32_t w0 = 0; w0 < ntot; w0 += JX_WIN) {
                gq_lds_barrier();                          // previous window done with map; b_* written
                const uint32_t a = pos > w0 ? pos : w0;
                const uint32_t e = (pos + len < w0 + JX_WIN) ? pos + len : w0 + JX_WIN;
                for (uint32_t j = a; j < e; ++j) map[j - w0] = static_cast<map_t>(threadIdx.x);
                gq_lds_barrier();
                const uint32_t cnt = ntot - w0 < JX_WIN ? ntot - w0 : JX_WIN;
                constexpr int PER = JX_WIN / RT;
                int64_t k[PER];
                int32_t pa[PER];
#pragma unroll
                for (int c = 0; c < PER; ++c) {
                    const uint32_t q = c * RT + threadIdx.x;
                    pa[c] = -1;
                    k[c] = JT_EMPTY;
                    if (q < cnt) {
                        const int i = map[q];
                        pa[c] = b_at[i] + static_cast<int32_t>(w0 + q - b_pos[i]);
                        k[c] = w.skey[pa[c]];
                    }
                }
                // A probe step reads the aligned group of four slots that holds
                // the current slot (two 16-byte LDS reads).  The first step of
                // all PER probes is issued together; the few probes not settled
                // by it walk on one by one.  Payloads are read after all probes.
                int32_t hs[PER];                       // slot of the match, -1 none, -2 ran past the region
                uint32_t sl[PER];
                longlong2 q0[PER], q1[PER];
#pragma unroll
                for (int c = 0; c < PER; ++c) {
                    const uint64_t home = gq_fmix64(static_cast<uint64_t>(k[c])) >> (64 - gm.L);
                    sl[c] = static_cast<uint32_t>(home) & (JX_REGION - 1);
                    const uint32_t g = sl[c] & ~3u;
                    q0[c] = *reinterpret_cast<const longlong2 *>(&lkey[g]);
                    q1[c] = *reinterpret_cast<const longlong2 *>(&lkey[g + 2]);
                }
#pragma unroll
                for (int c = 0; c < PER; ++c) {
                    hs[c] = -1;
                    if (pa[c] < 0 || k[c] == JT_EMPTY) continue;
                    while (true) {
                        const uint32_t g = sl[c] & ~3u;
                        const int64_t v[4] = {q0[c].x, q0[c].y, q1[c].x, q1[c].y};
                        uint32_t eq = 0, em = 0;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            eq |= (v[j] == k[c] ? 1u : 0u) << j;
                            em |= (v[j] == JT_EMPTY ? 1u : 0u) << j;
                        }
                        const uint32_t stop = (eq | em) & (~0u << (sl[c] & 3u)) & 0xfu;
                        if (stop) {
                            const uint32_t j = static_cast<uint32_t>(__builtin_ctz(stop));
                            if ((eq >> j) & 1u) hs[c] = static_cast<int32_t>(g + j);
                            break;
                        }
                        sl[c] = g + 4;
                        if (sl[c] == JX_REGION) {
                            hs[c] = -2;
                            break;
                        }
                        q0[c] = *reinterpret_cast<const longlong2 *>(&lkey[sl[c]]);
                        q1[c] = *reinterpret_cast<const longlong2 *>(&lkey[sl[c] + 2]);
                    }
                }
#pragma unroll
                for (int c = 0; c < PER; ++c) {
                    if (pa[c] < 0) continue;
                    int64_t out = hs[c] >= 0 ? static_cast<int64_t>(static_cast<uint32_t>(lpay[hs[c]])) : -1;
                    if (hs[c] == -2) {                       // continue in device memory, as linear probing does
                        const uint64_t home = gq_fmix64(static_cast<uint64_t>(k[c])) >> (64 - gm.L);
                        out = jx_probe_global(slots, mask, ((static_cast<uint64_t>(item) + 1) << JX_RBITS) & mask,
                                              k[c], JX_REGION - (static_cast<uint32_t>(home) & (JX_REGION - 1)));
                    }
                    w.res[pa[c]] = out;
                }
            }
            gq_lds_barrier();                              // b_at / b_pos / map free for the next batch
            len = nlen;
            at = nat;
        }
    }
}

// Per tile: results back in probe order in LDS (payload words plus a hit
// bitmap, scattered by the stored in-tile index), then the ordered compaction
// of the matches (block scan + decoupled look-back).  Only the in-tile index
// of each match is staged; its row id is read from the selection as it is
// written out.  Persistent: a workgroup takes tiles in increasing order from
// a counter and issues the loads of its next tile before it compacts the
// current one; its barriers order LDS only, so those loads stay in flight.
// Look-back cannot deadlock: the smallest unfinished tile is always some
// workgroup's current tile, and it waits only on smaller tiles.
template <bool HAS_SEL, int CT>
__global__ __launch_bounds__(CT) void jx_compact_kernel(jx_ws w, int64_t n_bound, const int64_t *n_dev,
                                                                const int32_t *__restrict__ sel,
                                                                int32_t *__restrict__ prow_out,
                                                                int32_t *__restrict__ pay_out, int64_t *n_out)
{
    constexpr int CI = JX_TILE / CT;                      // tile elements per thread (16 or 8)
    // LDS index x is stored at x + x / CI: a thread's CI consecutive elements
    // then start CI + 1 words after its neighbour's, on another bank
    __shared__ int32_t pay[JX_TILE + JX_TILE / CI];       // payloads in probe order; then the staged payloads
    __shared__ uint16_t stage_i[JX_TILE + JX_TILE / CI];  // in-tile index of each staged match
    auto pad = [](uint32_t x) { return x + x / CI; };
    __shared__ uint32_t hitw[JX_TILE / 32];               // hit bitmap in probe order
    __shared__ uint32_t scan_smem[CT / 64];
    __shared__ uint32_t s_next;
    __shared__ uint64_t s_goff;
    const int64_t n = jx_eff_n(n_bound, n_dev);
    const int64_t ntiles = (n + JX_TILE - 1) / JX_TILE;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (ntiles == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = 0;
        return;
    }
    auto load_tile = [&](int64_t t, uint16_t *ix, int64_t *rv) {
#pragma unroll
        for (int c = 0; c < CI; ++c) {
            const int64_t p = t * JX_TILE + c * CT + threadIdx.x;             // pool position
            ix[c] = 0;
            rv[c] = -1;
            if (t < ntiles && p < n) {
                ix[c] = static_cast<uint16_t>(w.sidx[p] & (JX_TILE - 1));
                rv[c] = w.res[p];
            }
        }
    };
    if (threadIdx.x == 0) s_next = atomicAdd(&w.ctr[32], 1u);
    __syncthreads();
    int64_t t = static_cast<int64_t>(gq_uniform(s_next));
    uint16_t ix[CI];
    int64_t rv[CI];
    load_tile(t, ix, rv);
    while (t < ntiles) {
        // a barrier opens each pass, so thread-0 work of consecutive passes
        // (the count store below, the dequeue here) is never merged
        gq_lds_barrier();
        const int64_t base = t * JX_TILE;
        uint32_t nxt = 0;
        if (threadIdx.x == 0) nxt = atomicAdd(&w.ctr[32], 1u);  // the next tile, dequeued early
        if (threadIdx.x < JX_TILE / 32) hitw[threadIdx.x] = 0;
        // every thread has read s_next (the current tile) and finished the
        // last tile's LDS reads; hitw is clear
        gq_lds_barrier();
        if (threadIdx.x == 0) s_next = nxt;
#pragma unroll
        for (int c = 0; c < CI; ++c) {
            const int64_t p = base + c * CT + threadIdx.x;
            if (p < n) {
                pay[pad(ix[c])] = static_cast<int32_t>(rv[c]);
                if (rv[c] >= 0) atomicOr(&hitw[ix[c] >> 5], 1u << (ix[c] & 31));
            }
        }
        const int64_t tn = static_cast<int64_t>(gq_uniform(s_next));
        gq_lds_barrier();
        load_tile(tn, ix, rv);                             // next tile: in flight meanwhile
        if (wave == 0) {                                   // the tile's match count, published at once
            const uint32_t c = __popc(hitw[lane]) + __popc(hitw[lane + 64]);
            gq_lookback_publish(w.status, static_cast<uint32_t>(t), gq_wave_sum(c));
        }
        // thread i owns probe-order elements [CI i, CI i + CI)
        const int elem0 = threadIdx.x * CI;
        const uint32_t mine = (hitw[elem0 >> 5] >> (elem0 & 31)) & ((1u << CI) - 1u);
        int32_t my_pay[CI];
#pragma unroll
        for (int i = 0; i < CI; ++i) my_pay[i] = pay[pad(elem0 + i)];
        uint32_t total;
        uint32_t pos = gq_block_exclusive_scan_lds<CT>(static_cast<uint32_t>(__popc(mine)), &total, scan_smem);
        if (wave == 0) {
            const uint64_t g = gq_lookback_wait(w.status, static_cast<uint32_t>(t), total);
            if (lane == 0) s_goff = g;
        }
        // the scan's barriers ordered every read of pay[] before these writes
#pragma unroll
        for (int i = 0; i < CI; ++i) {
            if (mine & (1u << i)) {
                stage_i[pad(pos)] = static_cast<uint16_t>(elem0 + i);
                pay[pad(pos)] = my_pay[i];
                ++pos;
            }
        }
        gq_lds_barrier();
        const int64_t goff = static_cast<int64_t>(s_goff);
        const uint32_t tot = static_cast<uint32_t>(gq_uniform(total));
        for (uint32_t i0 = 0; i0 < tot; i0 += CT * 4) {
            int32_t rw[4], py[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t i = i0 + c * CT + threadIdx.x;
                rw[c] = 0;
                py[c] = 0;
                if (i < tot) {
                    const int64_t e = base + stage_i[pad(i)];
                    rw[c] = HAS_SEL ? sel[e] : static_cast<int32_t>(e);
                    py[c] = pay[pad(i)];
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t i = i0 + c * CT + threadIdx.x;
                if (i < tot) {
                    prow_out[goff + i] = rw[c];
                    pay_out[goff + i] = py[c];
                }
            }
        }
        if (t == ntiles - 1 && threadIdx.x == 0) *n_out = goff + tot;
        t = tn;
    }
}

}  // namespace

extern "C" {

size_t gq_join_table_bytes(int64_t m, double load_factor)
{
    if (m < 0 || !(load_factor > 0.0) || load_factor > 0.9) return 0;
    const int L = jt_log2_slots(m, load_factor);
    return JT_HEADER + (size_t(1) << L) * sizeof(jt_slot);
}

size_t gq_join_build_workspace_bytes(int64_t m, size_t table_bytes)
{
    if (m < 0) m = 0;
    const int L = table_log2_from_bytes(table_bytes);
    if (!use_region_build(m, L, false)) return 256;
    gq_carver c(nullptr);
    build_layout(c, m);
    return c.bytes();
}

gq_status gq_join_build(gq_ctx *ctx, const int64_t *key, const int32_t *payload, int64_t m, const int64_t *n_dev,
                        const int32_t *sel, void *table, size_t table_bytes, void *ws, size_t ws_bytes,
                        gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (m < 0 || m > GQ_MAX_ROWS) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_build: m=%lld", (long long)m);
    if (!table || (m > 0 && (!key || !payload)))
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_build: NULL key, payload or table");
    if (reinterpret_cast<uintptr_t>(table) % 256 != 0)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_build: table must be 256-byte aligned");
    if (table_bytes < JT_HEADER + 64 * sizeof(jt_slot))
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_build: table of %zu bytes is too small", table_bytes);
    const int L = table_log2_from_bytes(table_bytes);
    if (static_cast<double>(m) > 0.9 * static_cast<double>(1ull << L))
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_build: %lld keys exceed load factor 0.9 of %llu slots",
                       (long long)m, (unsigned long long)(1ull << L));
    const bool region = use_region_build(m, L, sel != nullptr || n_dev != nullptr);
    const size_t need = gq_join_build_workspace_bytes(m, table_bytes);
    if (region && (!ws || ws_bytes < need))
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_join_build: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (region) return region_build(ctx, key, payload, m, table, L, ws, s);
    const uint64_t slots = 1ull << L;
    uint64_t blocks = (slots + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    GQ_TRY(gq_launch(ctx, "gq_join_build_init", jt_init_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, table,
                     L));
    if (m == 0) return GQ_OK;
    uint64_t ib = (static_cast<uint64_t>(m) + 255) / 256;
    if (ib > 65536) ib = 65536;
    return gq_launch(ctx, "gq_join_build_insert", jt_insert_kernel, dim3(static_cast<uint32_t>(ib)), dim3(256), 0, s, table,
                     L, key, payload, m, n_dev, sel, ctx->status_dev);
}

size_t gq_join_probe_workspace_bytes(int64_t n)
{
    if (n < 0) n = 0;
    gq_carver c(nullptr);
    probe_layout(c, n);
    return c.bytes();
}

gq_status gq_join_probe(gq_ctx *ctx, const void *table, const int64_t *fk, int64_t n, const int64_t *n_dev,
                        const int32_t *sel, int32_t *prow_out, int32_t *payload_out, int64_t *n_out_dev, void *ws,
                        size_t ws_bytes, gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (n < 0 || n > GQ_MAX_ROWS) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_probe: n=%lld", (long long)n);
    if (!table || (!fk && n > 0) || !prow_out || !payload_out || !n_out_dev)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_probe: NULL table, fk, output or count");
    const size_t need = gq_join_probe_workspace_bytes(n);
    if (!ws || ws_bytes < need)
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_join_probe: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gq_carver c(ws);
    probe_ws w = probe_layout(c, n);
    GQ_TRY(gq_zero(ctx, ws, c.off / 4, s));
    const int64_t tiles = (n + JP_TILE - 1) / JP_TILE;
    const uint32_t grid = static_cast<uint32_t>(tiles > 0 ? tiles : 1);
    if (sel)
        return gq_launch(ctx, "gq_join_probe", jt_probe_kernel<true>, dim3(grid), dim3(JP_THREADS), 0, s, table, fk,
                         n, n_dev, sel, prow_out, payload_out, n_out_dev, w.tile_ctr, w.status);
    return gq_launch(ctx, "gq_join_probe", jt_probe_kernel<false>, dim3(grid), dim3(JP_THREADS), 0, s, table, fk, n,
                     n_dev, sel, prow_out, payload_out, n_out_dev, w.tile_ctr, w.status);
}

size_t gq_join_probe_partitioned_workspace_bytes(int64_t n)
{
    if (n < 0) n = 0;
    gq_carver c(nullptr);
    jx_layout(c, n);
    return c.bytes();
}

gq_status gq_join_probe_partitioned(gq_ctx *ctx, const void *table, size_t table_bytes, const int64_t *fk,
                                    int64_t n, const int64_t *n_dev, const int32_t *sel, int log2_fanout,
                                    int32_t *prow_out, int32_t *payload_out, int64_t *n_out_dev, void *ws,
                                    size_t ws_bytes, gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (n < 0 || n > GQ_MAX_ROWS)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_probe_partitioned: n=%lld", (long long)n);
    if (!table || (!fk && n > 0) || !prow_out || !payload_out || !n_out_dev)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_probe_partitioned: NULL table, fk, output or count");
    if (table_bytes < JT_HEADER + 64 * sizeof(jt_slot))
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_probe_partitioned: table of %zu bytes is too small",
                       table_bytes);
    if (log2_fanout < 0 || log2_fanout > 16)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_probe_partitioned: log2_fanout=%d", log2_fanout);
    const size_t need = gq_join_probe_partitioned_workspace_bytes(n);
    if (!ws || ws_bytes < need)
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_join_probe_partitioned: workspace %zu < %zu bytes", ws_bytes,
                       need);
    jx_geom gm{};
    gm.L = table_log2_from_bytes(table_bytes);
    const int rbits = gm.L - JX_RBITS;
    gm.H = std::min(std::min(log2_fanout, JX_MAX_H), std::max(rbits, 0));
    gm.S = rbits - gm.H;
    gm.nregions = rbits > 0 ? 1 << rbits : 1;
    // cache-resident tables, or regions the tile split cannot separate: the ordered probe
    if (rbits < 8 || gm.S > JX_MAX_S)
        return gq_join_probe(ctx, table, fk, n, n_dev, sel, prow_out, payload_out, n_out_dev, ws, ws_bytes, stream);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gq_carver c(ws);
    jx_ws w = jx_layout(c, n);
    // counters, tile bounds and look-back words (the prefix up to the tile table)
    GQ_TRY(gq_zero(ctx, ws, static_cast<size_t>(reinterpret_cast<char *>(w.tile_hp) - static_cast<char *>(ws)) / 4, s));
    const uint32_t tiles = static_cast<uint32_t>(w.ntiles);
    // 512-thread split workgroups: 86 VGPRs and 51 KB of LDS, 16 waves per CU
    // (256-thread ones at 144 VGPRs fit 12)
    if (sel)
        GQ_TRY(gq_launch(ctx, "gq_join_probe_split", jx_split_kernel<true, JX_SPLIT_THREADS>, dim3(tiles),
                         dim3(JX_SPLIT_THREADS), 0, s, table, fk, n, n_dev, sel, gm, w, ctx->status_dev));
    else
        GQ_TRY(gq_launch(ctx, "gq_join_probe_split", jx_split_kernel<false, JX_SPLIT_THREADS>, dim3(tiles),
                         dim3(JX_SPLIT_THREADS), 0, s, table, fk, n, n_dev, sel, gm, w, ctx->status_dev));
    // a region with more rows in heavy runs than 4x the mean region (and at
    // least 65,536) is split into items of that many rows
    const int64_t item_rows = std::max<int64_t>(65536, 4 * (n / gm.nregions));
    GQ_TRY(gq_launch(ctx, "gq_join_probe_plan", jx_plan_kernel, dim3(1), dim3(JX_PLAN_THREADS), 0, s,
                     static_cast<const uint32_t *>(w.rw), gm.nregions,
                     static_cast<uint32_t>(std::min<int64_t>(item_rows, 1ll << 31)),
                     static_cast<const uint32_t *>(w.ctr + 16), w.iprefix));
    // two 512-thread, 57-KB-LDS workgroups per CU (16 waves; with 256-thread
    // workgroups at 163 VGPRs only 12 waves fit)
    const uint32_t grid = static_cast<uint32_t>(ctx->num_cus) * 2;
    GQ_TRY(gq_launch(ctx, "gq_join_probe_regions", jx_region_kernel<JR_THREADS_PROBE>, dim3(grid),
                     dim3(JR_THREADS_PROBE), 0, s, table, gm, w));
    // persistent compaction: four workgroups per CU (122 VGPRs)
    const uint32_t cgrid = static_cast<uint32_t>(std::min<int64_t>(w.ntiles, static_cast<int64_t>(ctx->num_cus) * 4));
    if (sel)
        return gq_launch(ctx, "gq_join_probe_compact", jx_compact_kernel<true, JX_THREADS>, dim3(cgrid),
                         dim3(JX_THREADS), 0, s, w, n, n_dev, sel, prow_out, payload_out, n_out_dev);
    return gq_launch(ctx, "gq_join_probe_compact", jx_compact_kernel<false, JX_THREADS>, dim3(cgrid),
                     dim3(JX_THREADS), 0, s, w, n, n_dev, sel, prow_out, payload_out, n_out_dev);
}
}  // extern "C"
