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
// build rows are radix-partitioned (stable LSD passes of the partition
// operator) by the region of their home slot, a region being 4096 consecutive
// slots; one workgroup per region inserts its keys into an LDS copy of the
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
constexpr int JR_MAX_REGION_BITS = 16;              // two 8-bit partition passes at most
constexpr int64_t JR_MIN_KEYS = 1 << 18;            // below this the CAS build is used

// Start offset of every region in the region-sorted keys: roff[r] = first i
// with region(keys[i]) >= r, roff[2^g] = m.  Each entry is written once, by
// the element at which the region sequence steps past it.
__global__ __launch_bounds__(256) void jt_region_bounds_kernel(const int64_t *__restrict__ keys, int64_t m, int g,
                                                               int64_t *__restrict__ roff)
{
    const int64_t nr = int64_t(1) << g;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i <= m;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t prev =
            i == 0 ? -1 : static_cast<int64_t>(gq_fmix64(static_cast<uint64_t>(keys[i - 1])) >> (64 - g));
        const int64_t cur = i == m ? nr : static_cast<int64_t>(gq_fmix64(static_cast<uint64_t>(keys[i])) >> (64 - g));
        for (int64_t r = prev + 1; r <= cur; ++r) roff[r] = i;
    }
}

// A persistent grid walks the regions; the barriers between a region's phases
// order LDS only, so one region's table stores drain while the next region's
// keys load.
__global__ __launch_bounds__(256) void jt_region_kernel(void *table, int L, const int64_t *__restrict__ keys,
                                                        const int32_t *__restrict__ pay,
                                                        const int64_t *__restrict__ roff, int64_t nregions,
                                                        int64_t *__restrict__ ovf_key, int32_t *__restrict__ ovf_pay,
                                                        uint32_t *ovf_cnt, int64_t ovf_cap, uint32_t *status)
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
    for (int64_t region = blockIdx.x; region < nregions; region += gridDim.x) {
        gq_lds_barrier();                             // the previous region is read out of LDS
        for (int j = threadIdx.x; j < JR_SLOTS; j += blockDim.x) {
            sk[j] = static_cast<unsigned long long>(JT_EMPTY);
            sp[j] = 0;
        }
        gq_lds_barrier();
        const int64_t r0 = roff[region], r1 = roff[region + 1];
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const int64_t k = keys[i];
            const int32_t p = pay[i];
            if (k == JT_EMPTY) {
                gq_raise(status, GQ_ERR_INVALID_KEY);
                continue;
            }
            uint32_t loc = static_cast<uint32_t>(gq_fmix64(static_cast<uint64_t>(k)) >> (64 - L)) & (JR_SLOTS - 1);
            while (true) {
                const unsigned long long prev =
                    atomicCAS(&sk[loc], static_cast<unsigned long long>(JT_EMPTY), static_cast<unsigned long long>(k));
                if (prev == static_cast<unsigned long long>(JT_EMPTY)) {
                    sp[loc] = p;
                    break;
                }
                if (prev == static_cast<unsigned long long>(k)) {
                    gq_raise(status, GQ_ERR_DUPLICATE_KEY);
                    break;
                }
                if (++loc == JR_SLOTS) {                 // continue in the next region, later
                    const uint32_t idx = atomicAdd(ovf_cnt, 1u);
                    if (idx < ovf_cap) {
                        ovf_key[idx] = k;
                        ovf_pay[idx] = p;
                    } else {
                        gq_raise(status, GQ_ERR_CAPACITY);
                    }
                    break;
                }
            }
        }
        gq_lds_barrier();
        jt_slot *slots = reinterpret_cast<jt_slot *>(static_cast<char *>(table) + JT_HEADER) +
                         (static_cast<uint64_t>(region) << JR_BITS);
        for (int j = threadIdx.x; j < JR_SLOTS; j += blockDim.x) {
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
    if (g <= 8) {
        void *in[1] = {const_cast<int32_t *>(payload)};
        void *out[1] = {w.p2};
        GQ_TRY(gq_partition_bits(ctx, key, m, g, 64 - g, 1, in, &pbytes, w.k2, out, w.offsets, w.part_ws, s, nm, 8));
    } else {                                        // LSD: low digit first, both passes stable
        const int d1 = g / 2, d2 = g - d1;
        void *in1[1] = {const_cast<int32_t *>(payload)};
        void *out1[1] = {w.p1};
        GQ_TRY(gq_partition_bits(ctx, key, m, d1, 64 - g, 1, in1, &pbytes, w.k1, out1, w.offsets, w.part_ws, s, nm, 8));
        void *in2[1] = {w.p1};
        void *out2[1] = {w.p2};
        GQ_TRY(gq_partition_bits(ctx, w.k1, m, d2, 64 - d2, 1, in2, &pbytes, w.k2, out2, w.offsets, w.part_ws, s, nm, 8));
    }
    uint64_t bb = (static_cast<uint64_t>(m) + 256) / 256;
    if (bb > 8192) bb = 8192;
    GQ_TRY(gq_launch(ctx, "gq_join_build_bounds", jt_region_bounds_kernel, dim3(static_cast<uint32_t>(bb)), dim3(256),
                     0, s, static_cast<const int64_t *>(w.k2), m, g, w.roff));
    const int64_t nregions = int64_t(1) << g;
    const uint32_t rgrid = static_cast<uint32_t>(std::min<int64_t>(nregions, int64_t(ctx->num_cus) * 3));
    GQ_TRY(gq_launch(ctx, "gq_join_build_regions", jt_region_kernel, dim3(rgrid), dim3(256), 0, s, table, L,
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
// Partitioned probe.  The probe rows are split into 8 lists by hash bits
// 55..57, the three bits just below the top six (so a probe stream already
// in the order of a radix partition into 64 or more buckets walks, in each
// list, one 1/512 slice of the table at a time); the workgroups on XCD x
// probe list x, so each XCD's L2 holds the table slice its list is reading,
// and the table is read from HBM about once instead of one line per probe.
//   split:   tile t of 4096 probe rows is regrouped by list (stable) in LDS
//            and written to pool positions [4096 t, 4096 t + rows) as
//            (key, index of the row inside the tile); the run of list x in
//            tile t is chunk (x, t).  No atomics: the pool is dense over [0, n).
//   probe:   a persistent grid of 8 G workgroups; workgroup b probes list
//            b mod 8 (its XCD, as workgroups are dispatched round-robin over
//            the XCDs), taking tiles in groups of 4 with stride 4 G, so the
//            G workgroups of one XCD sweep one window of consecutive tiles;
//            each entry's payload, or -1 for a miss, goes to its pool
//            position.  The assignment is static: no atomics, and every
//            chunk is probed once whatever the dispatch order.
//   compact: per tile, the results are put back in probe order in LDS (by
//            the stored in-tile index) and compacted exactly like the
//            ordered probe (block scan + decoupled look-back).
// The output is therefore identical to the ordered probe's.
// ------------------------------------------------------------------------
constexpr int JX_LISTS = 8;
constexpr int JX_SHIFT = 55;
constexpr int JX_THREADS = 256;
constexpr int JX_ITEMS = 16;
constexpr int JX_TILE = JX_THREADS * JX_ITEMS;          // probe rows per split tile / probe round
constexpr int JX_GROUP = 4;                             // consecutive tiles of one list per probe step
constexpr int JX_PITEMS = 8;                            // probe entries per thread per round

struct jx_chunk {
    uint32_t off, len;
};

struct jx_ws {
    uint32_t *ctr;          // [32] compaction tile counter
    jx_chunk *chunks;       // chunk (x, t) at chunks[x * ntiles + t]
    int64_t *skey;          // pool: probe keys
    uint16_t *sidx;         // pool: index of the probe row inside its tile
    int64_t *res;           // pool: payload of the match, -1 for none
    uint64_t *status;       // compaction look-back words, one per tile
    int64_t ntiles;
};

jx_ws jx_layout(gq_carver &c, int64_t n)
{
    jx_ws w;
    const int64_t rows = n > 0 ? n : 1;
    w.ntiles = (rows + JX_TILE - 1) / JX_TILE;
    w.ctr = c.take<uint32_t>(64);
    w.status = c.take<uint64_t>(static_cast<size_t>(w.ntiles));
    w.chunks = c.take<jx_chunk>(static_cast<size_t>(JX_LISTS * w.ntiles));
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

GQ_DEV uint32_t jx_list(int64_t key) { return static_cast<uint32_t>(gq_fmix64(static_cast<uint64_t>(key)) >> JX_SHIFT) & 7u; }

// Stable split of one tile: a row's place is its list's start in the tile,
// plus the rows of that list in earlier (step, wave) groups, plus its rank
// among the lanes of its wave with the same list (three ballots, one per
// list bit).
template <bool HAS_SEL>
__global__ __launch_bounds__(JX_THREADS) void jx_split_kernel(const int64_t *__restrict__ fk, int64_t n_bound,
                                                              const int64_t *n_dev, const int32_t *__restrict__ sel,
                                                              jx_ws w)
{
    constexpr int WAVES = JX_THREADS / 64;
    __shared__ uint32_t grp[JX_ITEMS * WAVES][JX_LISTS];   // per (step, wave): count, then exclusive prefix
    __shared__ uint32_t start[JX_LISTS + 1];
    __shared__ int64_t stage_k[JX_TILE];
    __shared__ uint16_t stage_i[JX_TILE];
    const int64_t n = jx_eff_n(n_bound, n_dev);
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * JX_TILE;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t k[JX_ITEMS];
    int32_t r[JX_ITEMS];
#pragma unroll
    for (int c = 0; c < JX_ITEMS; ++c) {
        const int64_t e = base + c * JX_THREADS + threadIdx.x;
        r[c] = 0;
        if (e < n) r[c] = HAS_SEL ? sel[e] : static_cast<int32_t>(e);
    }
#pragma unroll
    for (int c = 0; c < JX_ITEMS; ++c) {
        const int64_t e = base + c * JX_THREADS + threadIdx.x;
        k[c] = e < n ? fk[r[c]] : 0;
    }
    uint32_t rank[JX_ITEMS];
    uint8_t lst[JX_ITEMS];
#pragma unroll
    for (int c = 0; c < JX_ITEMS; ++c) {
        const int64_t e = base + c * JX_THREADS + threadIdx.x;
        const bool valid = e < n;
        const uint32_t x = valid ? jx_list(k[c]) : 0u;
        const uint64_t act = gq_ballot(valid);
        const uint64_t b0 = gq_ballot(valid && (x & 1u)), b1 = gq_ballot(valid && (x & 2u)),
                       b2 = gq_ballot(valid && (x & 4u));
        const uint64_t peers = act & ((x & 1u) ? b0 : ~b0) & ((x & 2u) ? b1 : ~b1) & ((x & 4u) ? b2 : ~b2);
        rank[c] = gq_mbcnt(peers);
        lst[c] = static_cast<uint8_t>(x);
        if (lane < JX_LISTS) {
            const uint32_t l = static_cast<uint32_t>(lane);
            const uint64_t ml = act & ((l & 1u) ? b0 : ~b0) & ((l & 2u) ? b1 : ~b1) & ((l & 4u) ? b2 : ~b2);
            grp[c * WAVES + wave][l] = static_cast<uint32_t>(__popcll(ml));
        }
    }
    __syncthreads();
    if (threadIdx.x < JX_LISTS) {                     // per list: prefix over (step, wave) in row order
        uint32_t run = 0;
        for (int g = 0; g < JX_ITEMS * WAVES; ++g) {
            const uint32_t c = grp[g][threadIdx.x];
            grp[g][threadIdx.x] = run;
            run += c;
        }
        start[threadIdx.x] = run;                    // list total, turned into a start below
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int x = 0; x < JX_LISTS; ++x) {
            const uint32_t c = start[x];
            start[x] = run;
            run += c;
        }
        start[JX_LISTS] = run;
    }
    __syncthreads();
    if (threadIdx.x < JX_LISTS) {                     // every chunk is written, empty ones too
        jx_chunk ch;
        ch.off = static_cast<uint32_t>(base) + start[threadIdx.x];
        ch.len = start[threadIdx.x + 1] - start[threadIdx.x];
        w.chunks[static_cast<int64_t>(threadIdx.x) * w.ntiles + tile] = ch;
    }
#pragma unroll
    for (int c = 0; c < JX_ITEMS; ++c) {
        const int64_t e = base + c * JX_THREADS + threadIdx.x;
        if (e < n) {
            const uint32_t x = lst[c];
            const uint32_t q = start[x] + grp[c * WAVES + wave][x] + rank[c];
            stage_k[q] = k[c];
            stage_i[q] = static_cast<uint16_t>(c * JX_THREADS + threadIdx.x);
        }
    }
    __syncthreads();
    const uint32_t total = start[JX_LISTS];
    for (uint32_t q = threadIdx.x; q < total; q += JX_THREADS) {
        w.skey[base + q] = stage_k[q];
        w.sidx[base + q] = stage_i[q];
    }
}

__global__ __launch_bounds__(JX_THREADS) void jx_probe_kernel(const void *table, jx_ws w, int per_list)
{
    __shared__ uint32_t c_off[JX_GROUP], c_end[JX_GROUP + 1];
    const jt_header *hdr = static_cast<const jt_header *>(table);
    const int L = static_cast<int>(hdr->log2_slots);
    const uint64_t mask = (1ull << L) - 1;
    const jt_slot *slots = reinterpret_cast<const jt_slot *>(static_cast<const char *>(table) + JT_HEADER);
    const uint32_t x = blockIdx.x % JX_LISTS;
    const int64_t stride = static_cast<int64_t>(per_list) * JX_GROUP;
    for (int64_t t0 = static_cast<int64_t>(blockIdx.x / JX_LISTS) * JX_GROUP; t0 < w.ntiles; t0 += stride) {
        const uint32_t ng = static_cast<uint32_t>(w.ntiles - t0 < JX_GROUP ? w.ntiles - t0 : JX_GROUP);
        __syncthreads();                                  // the previous group is done with c_off / c_end
        if (threadIdx.x < ng) {
            const jx_chunk ch = w.chunks[static_cast<int64_t>(x) * w.ntiles + t0 + threadIdx.x];
            c_off[threadIdx.x] = ch.off;
            c_end[threadIdx.x + 1] = ch.len;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            c_end[0] = 0;
            for (uint32_t j = 1; j <= ng; ++j) c_end[j] += c_end[j - 1];
        }
        __syncthreads();
        uint32_t e1 = c_end[1], e2 = c_end[2], e3 = c_end[3];
        const uint32_t total = c_end[ng];
        for (uint32_t r0 = 0; r0 < total; r0 += JX_THREADS * JX_PITEMS) {
            int64_t k[JX_PITEMS];
            int64_t at[JX_PITEMS];
            uint64_t s[JX_PITEMS];
            int4 v[JX_PITEMS];
#pragma unroll
            for (int c = 0; c < JX_PITEMS; ++c) {
                const uint32_t q = r0 + c * JX_THREADS + threadIdx.x;
                k[c] = JT_EMPTY;
                at[c] = -1;
                if (q < total) {
                    const uint32_t j = (q >= e1 ? 1u : 0u) + (ng > 2 && q >= e2 ? 1u : 0u) + (ng > 3 && q >= e3 ? 1u : 0u);
                    at[c] = static_cast<int64_t>(c_off[j]) + (q - c_end[j]);
                    k[c] = w.skey[at[c]];
                }
            }
#pragma unroll
            for (int c = 0; c < JX_PITEMS; ++c) {
                s[c] = gq_fmix64(static_cast<uint64_t>(k[c])) >> (64 - L);
                v[c] = *reinterpret_cast<const int4 *>(&slots[s[c]]);
            }
#pragma unroll
            for (int c = 0; c < JX_PITEMS; ++c) {
                if (at[c] < 0) continue;
                int64_t out = -1;
                if (k[c] != JT_EMPTY) {
                    int64_t sk = (static_cast<int64_t>(static_cast<uint32_t>(v[c].y)) << 32) |
                                 static_cast<uint32_t>(v[c].x);
                    uint64_t probes = 0;
                    while (sk != k[c] && sk != JT_EMPTY && probes < mask) {
                        s[c] = (s[c] + 1) & mask;
                        v[c] = *reinterpret_cast<const int4 *>(&slots[s[c]]);
                        sk = (static_cast<int64_t>(static_cast<uint32_t>(v[c].y)) << 32) | static_cast<uint32_t>(v[c].x);
                        ++probes;
                    }
                    if (sk == k[c]) out = static_cast<int64_t>(static_cast<uint32_t>(v[c].z));
                }
                w.res[at[c]] = out;
            }
        }
    }
}

// Per tile: results back in probe order (one 8-byte LDS word per entry,
// scattered by the in-tile index), then the ordered compaction of the matches.
template <bool HAS_SEL>
__global__ __launch_bounds__(JX_THREADS) void jx_compact_kernel(jx_ws w, int64_t n_bound, const int64_t *n_dev,
                                                                const int32_t *__restrict__ sel,
                                                                int32_t *__restrict__ prow_out,
                                                                int32_t *__restrict__ pay_out, int64_t *n_out)
{
    __shared__ int64_t by_idx[JX_TILE];                   // payload or -1 in probe order; then the staged pairs
    __shared__ uint32_t scan_smem[JX_THREADS / 64];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_goff;
    const int64_t n = jx_eff_n(n_bound, n_dev);
    if (threadIdx.x == 0) s_tile = atomicAdd(&w.ctr[32], 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    const int64_t ntiles = (n + JX_TILE - 1) / JX_TILE;
    if (static_cast<int64_t>(t) >= ntiles) {
        if (t == 0 && threadIdx.x == 0) *n_out = 0;
        return;
    }
    const int64_t base = static_cast<int64_t>(t) * JX_TILE;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t rows = n - base < JX_TILE ? n - base : JX_TILE;
    // thread i owns probe-order elements [16 i, 16 i + 16): their rows, loaded now
    const int elem0 = threadIdx.x * JX_ITEMS;
    int32_t my_row[JX_ITEMS];
#pragma unroll
    for (int i = 0; i < JX_ITEMS; ++i) {
        const int64_t e = base + elem0 + i;
        my_row[i] = e < n ? (HAS_SEL ? sel[e] : static_cast<int32_t>(e)) : 0;
    }
#pragma unroll
    for (int c = 0; c < JX_ITEMS; ++c) {
        const int64_t p = base + c * JX_THREADS + threadIdx.x;     // pool position
        if (p < n) by_idx[w.sidx[p]] = w.res[p];
    }
    __syncthreads();
    uint32_t mine = 0;
    int32_t my_pay[JX_ITEMS];
#pragma unroll
    for (int i = 0; i < JX_ITEMS; ++i) {
        const int64_t rv = elem0 + i < rows ? by_idx[elem0 + i] : -1;
        mine |= rv >= 0 ? (1u << i) : 0u;
        my_pay[i] = static_cast<int32_t>(rv);
    }
    uint32_t total;
    uint32_t pos = gq_block_exclusive_scan<JX_THREADS>(static_cast<uint32_t>(__popc(mine)), &total, scan_smem);
    if (wave == 0) {
        const uint64_t g = gq_lookback(w.status, t, total);
        if (lane == 0) s_goff = g;
    }
    int32_t *stage_row = reinterpret_cast<int32_t *>(by_idx);
    int32_t *stage_pay = stage_row + JX_TILE;
#pragma unroll
    for (int i = 0; i < JX_ITEMS; ++i) {
        if (mine & (1u << i)) {
            stage_row[pos] = my_row[i];
            stage_pay[pos] = my_pay[i];
            ++pos;
        }
    }
    __syncthreads();
    const int64_t goff = static_cast<int64_t>(s_goff);
    for (uint32_t i = threadIdx.x; i < total; i += JX_THREADS) {
        prow_out[goff + i] = stage_row[i];
        pay_out[goff + i] = stage_pay[i];
    }
    if (static_cast<int64_t>(t) == ntiles - 1 && threadIdx.x == 0) *n_out = goff + total;
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

gq_status gq_join_probe_partitioned(gq_ctx *ctx, const void *table, const int64_t *fk, int64_t n,
                                    const int64_t *n_dev, const int32_t *sel, int32_t *prow_out,
                                    int32_t *payload_out, int64_t *n_out_dev, void *ws, size_t ws_bytes,
                                    gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (n < 0 || n > GQ_MAX_ROWS)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_probe_partitioned: n=%lld", (long long)n);
    if (!table || (!fk && n > 0) || !prow_out || !payload_out || !n_out_dev)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_join_probe_partitioned: NULL table, fk, output or count");
    const size_t need = gq_join_probe_partitioned_workspace_bytes(n);
    if (!ws || ws_bytes < need)
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_join_probe_partitioned: workspace %zu < %zu bytes", ws_bytes,
                       need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gq_carver c(ws);
    jx_ws w = jx_layout(c, n);
    // counters and look-back words (the prefix of the workspace up to the chunk table)
    GQ_TRY(gq_zero(ctx, ws, static_cast<size_t>(reinterpret_cast<char *>(w.chunks) - static_cast<char *>(ws)) / 4, s));
    const uint32_t tiles = static_cast<uint32_t>(w.ntiles);
    if (sel)
        GQ_TRY(gq_launch(ctx, "gq_join_probe_split", jx_split_kernel<true>, dim3(tiles), dim3(JX_THREADS), 0, s, fk,
                         n, n_dev, sel, w));
    else
        GQ_TRY(gq_launch(ctx, "gq_join_probe_split", jx_split_kernel<false>, dim3(tiles), dim3(JX_THREADS), 0, s,
                         fk, n, n_dev, sel, w));
    const int per_list = ctx->num_cus / 2;                  // 4 workgroups per CU in all
    GQ_TRY(gq_launch(ctx, "gq_join_probe_lists", jx_probe_kernel, dim3(static_cast<uint32_t>(per_list * JX_LISTS)),
                     dim3(JX_THREADS), 0, s, table, w, per_list));
    if (sel)
        return gq_launch(ctx, "gq_join_probe_compact", jx_compact_kernel<true>, dim3(tiles), dim3(JX_THREADS), 0, s,
                         w, n, n_dev, sel, prow_out, payload_out, n_out_dev);
    return gq_launch(ctx, "gq_join_probe_compact", jx_compact_kernel<false>, dim3(tiles), dim3(JX_THREADS), 0, s, w,
                     n, n_dev, sel, prow_out, payload_out, n_out_dev);
}
}  // extern "C"
