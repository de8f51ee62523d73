// Batched join + aggregate: many independent instances in ONE persistent launch.
//
// Instance i: filter date_lo <= date < date_hi over its fact rows, equi-join
// fk with its dimension keys (unique) carrying the dimension attribute, group
// by that attribute; per group count, sum(qty), exact 128-bit sum of
// price * (rev_scale - disc) and the float64 averages.
//
// Work queue (built on the host, consumed in order through one atomic
// counter by a persistent grid):
//   L_i  instance whose table fits one LDS region: build the whole table in
//        LDS and write it out (one item)
//   I_i  table-initialisation tiles of a larger instance (fill EMPTY)
//   B_i  build tiles of a larger instance (device compare-and-swap); they
//        wait until all I_i items of the instance are done
//   P_i  probe tiles: fused filter -> probe -> LDS aggregation, merged into
//        the instance's global group table at the end of the tile; they wait
//        until the instance's table is complete.  The last P_i item to finish
//        compacts the instance's groups into its output.
// Queue order interleaves instances (the build items of instance i+1 come
// before the probe items of instance i), so device-CAS builds overlap the
// bandwidth-bound probes of other instances.  An item only ever waits for
// items that were dequeued before it, which are held by running workgroups
// that never wait on later items: the wait always ends.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "gq_device.h"
#include "gq_internal.h"

namespace {

constexpr int BT_THREADS = 512;               // 84 VGPRs: three workgroups (24 waves) per CU
constexpr int BT_TILE_GRAIN = 256;            // build and fill tiles are multiples of this
constexpr int BT_LDS_GROUP_SLOTS = 1024;
constexpr int BT_REGION_SLOTS = 4096;              // tables up to this size are built in LDS
constexpr int64_t BT_EMPTY = INT64_MIN;

enum : int32_t { K_LDS_BUILD = 0, K_INIT = 1, K_BUILD = 2, K_PROBE = 3 };

struct bt_slot {
    int64_t key;
    int32_t payload;
    int32_t unused;
};

struct bt_inst {                   // device copy of one instance
    const int64_t *dim_key;
    const int32_t *dim_attr;
    const int64_t *fk;
    const int32_t *date;
    const int64_t *qty, *price, *disc;
    int64_t m, n;
    int64_t date_lo, date_hi, rev_scale;
    bt_slot *table;
    int32_t log2_slots;
    int32_t init_items, build_items, probe_items;
    // group table (global, per instance)
    uint32_t *gstate;
    int32_t *gkey;
    uint64_t *gcnt, *gsq, *glo;
    int64_t *ghi;
    uint64_t gmask;
    uint32_t *counters;            // [0] init done, [1] build done, [2] probe done,
                                   // [3] this instance's error bits (1 << gq_status)
    gq_groups out;
};

// An error of instance I: recorded in its own bits and in the context word.
GQ_DEV void inst_raise(const bt_inst &I, uint32_t *status, int code)
{
    gq_raise(status, code);
    gq_raise(&I.counters[3], code);
}

struct bt_seg {                    // a run of consecutive work items of one kind
    int64_t first_item;
    int32_t kind, inst;
    int64_t first_tile, ntiles;
};

GQ_DEV uint32_t load_acquire(const uint32_t *p)
{
    return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *ctr >= target, for at most `limit` polls (each after a short
// sleep).  Returns false, in every thread, when the bound ran out: the
// caller then skips its work (its inputs are incomplete) and reports
// GQ_ERR_TIMEOUT, so the kernel still drains its queue and exits.  Every
// wait here is for items dequeued earlier, so the bound is only reached
// through a bug, or when the host sets a tiny bound to test this path.
GQ_DEV bool wait_for(const uint32_t *ctr, uint32_t target, int64_t limit, uint32_t *s_ok)
{
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        for (int64_t polls = 0; load_acquire(ctr) < target; ++polls) {
            if (polls >= limit) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        *s_ok = ok;
    }
    __syncthreads();
    return gq_uniform(*s_ok) != 0;
}

GQ_DEV void signal_done(uint32_t *ctr)
{
    __syncthreads();                                     // every thread's work is issued
    if (threadIdx.x == 0) {
        __threadfence();                                 // ...and visible device-wide
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

GQ_DEV uint64_t key_hash(int64_t k) { return gq_fmix64(static_cast<uint64_t>(k)); }

// ---------------------------------------------------------------- groups
// LDS group table of a probe tile.  A slot is one 64-bit word, 0 = empty,
// else (key << 32) | 1, claimed and published by a single compare-and-swap.
// Revenue sums are kept split: lo[] sums the low 32 bits (unsigned) and hi[]
// the high 32 bits (signed) of each row's revenue, so no accumulation needs a
// returned value; the slot's revenue is hi * 2^32 + lo (exact for < 2^31 rows).
struct bt_lds {
    uint64_t word[BT_LDS_GROUP_SLOTS];
    uint32_t cnt[BT_LDS_GROUP_SLOTS];
    uint64_t sq[BT_LDS_GROUP_SLOTS];
    uint64_t lo[BT_LDS_GROUP_SLOTS];
    int64_t hi[BT_LDS_GROUP_SLOTS];
};

GQ_DEV void lds_clear(bt_lds &T)
{
    for (int s = threadIdx.x; s < BT_LDS_GROUP_SLOTS; s += BT_THREADS) {
        T.word[s] = 0;
        T.cnt[s] = 0;
        T.sq[s] = 0;
        T.lo[s] = 0;
        T.hi[s] = 0;
    }
}

GQ_DEV uint64_t group_hash(int32_t k) { return gq_fmix64(static_cast<uint64_t>(static_cast<uint32_t>(k)) * 0x9E3779B97F4A7C15ull); }

// find-or-claim in the LDS group table (wave-uniform loop); -1 when 64 probes fail
GQ_DEV int lds_group(bt_lds &T, bool active, int32_t key)
{
    uint32_t s = static_cast<uint32_t>(group_hash(key)) & (BT_LDS_GROUP_SLOTS - 1);
    const unsigned long long want = (static_cast<unsigned long long>(static_cast<uint32_t>(key)) << 32) | 1ull;
    int probes = 0, found = -1;
    bool done = !active;
    while (__any(!done)) {
        if (!done) {
            unsigned long long *wp = reinterpret_cast<unsigned long long *>(&T.word[s]);
            unsigned long long w = __hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (w == 0ull) {
                w = atomicCAS(wp, 0ull, want);            // claim only an empty slot
                if (w == 0ull) w = want;
            }
            if (w == want) {
                found = static_cast<int>(s);
                done = true;
            } else if (++probes >= 64) {
                done = true;
            } else {
                s = (s + 1) & (BT_LDS_GROUP_SLOTS - 1);
            }
        }
    }
    return found;
}

// one row into LDS slot s (revenue known to fit 64 bits)
GQ_DEV void lds_add_row(bt_lds &T, int s, int64_t qty, int64_t rev)
{
    atomicAdd(&T.cnt[s], 1u);
    atomicAdd(reinterpret_cast<unsigned long long *>(&T.sq[s]), static_cast<unsigned long long>(qty));
    atomicAdd(reinterpret_cast<unsigned long long *>(&T.lo[s]),
              static_cast<unsigned long long>(static_cast<uint32_t>(static_cast<uint64_t>(rev))));
    const int64_t high = rev >> 32;
    if (high) atomicAdd(reinterpret_cast<unsigned long long *>(&T.hi[s]), static_cast<unsigned long long>(high));
}

GQ_DEV gq_i128 split_total(uint64_t lo_sum, int64_t hi_sum)
{
    const __int128 v = static_cast<__int128>(hi_sum) * (static_cast<__int128>(1) << 32) + static_cast<__int128>(lo_sum);
    gq_i128 r;
    r.lo = static_cast<uint64_t>(v);
    r.hi = static_cast<int64_t>(v >> 64);
    return r;
}

GQ_DEV void add128(uint64_t *lo, int64_t *hi, gq_i128 v)
{
    const unsigned long long old =
        atomicAdd(reinterpret_cast<unsigned long long *>(lo), static_cast<unsigned long long>(v.lo));
    const int64_t h = v.hi + ((old + v.lo < old) ? 1 : 0);
    if (h) atomicAdd(reinterpret_cast<unsigned long long *>(hi), static_cast<unsigned long long>(h));
}

// find-or-claim in an instance's global group table (wave-uniform loop)
GQ_DEV int64_t global_group(const bt_inst &I, bool active, int32_t key, uint32_t *status)
{
    uint64_t s = group_hash(key) & I.gmask;
    uint64_t probes = 0;
    int64_t found = -1;
    bool done = !active;
    while (__any(!done)) {
        if (!done) {
            const uint32_t st = atomicCAS(&I.gstate[s], 0u, 1u);
            if (st == 0u) {
                __hip_atomic_store(&I.gkey[s], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&I.gstate[s], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                found = static_cast<int64_t>(s);
                done = true;
            } else if (st == 2u) {
                (void)__hip_atomic_load(&I.gstate[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (__hip_atomic_load(&I.gkey[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == key) {
                    found = static_cast<int64_t>(s);
                    done = true;
                } else if (++probes > I.gmask) {
                    inst_raise(I, status, GQ_ERR_CAPACITY);
                    done = true;
                } else {
                    s = (s + 1) & I.gmask;
                }
            }
        }
    }
    return found;
}

GQ_DEV void global_add(const bt_inst &I, int64_t s, uint64_t cnt, uint64_t sq, gq_i128 rev)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(&I.gcnt[s]), static_cast<unsigned long long>(cnt));
    atomicAdd(reinterpret_cast<unsigned long long *>(&I.gsq[s]), static_cast<unsigned long long>(sq));
    add128(&I.glo[s], &I.ghi[s], rev);
}

// ---------------------------------------------------------------- items
__device__ void item_lds_build(const bt_inst &I, uint32_t *status, unsigned long long *sk, int32_t *sp)
{
    const int L = I.log2_slots;
    const int S = 1 << L;
    for (int j = threadIdx.x; j < S; j += BT_THREADS) {
        sk[j] = static_cast<unsigned long long>(BT_EMPTY);
        sp[j] = 0;
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < I.m; i += BT_THREADS) {
        const int64_t k = I.dim_key[i];
        if (k == BT_EMPTY) {
            inst_raise(I, status, GQ_ERR_INVALID_KEY);
            continue;
        }
        uint32_t s = static_cast<uint32_t>(key_hash(k) >> (64 - L));
        for (int p = 0; p < S; ++p) {
            const unsigned long long prev =
                atomicCAS(&sk[s], static_cast<unsigned long long>(BT_EMPTY), static_cast<unsigned long long>(k));
            if (prev == static_cast<unsigned long long>(BT_EMPTY)) {
                sp[s] = I.dim_attr[i];
                break;
            }
            if (prev == static_cast<unsigned long long>(k)) {
                inst_raise(I, status, GQ_ERR_DUPLICATE_KEY);
                break;
            }
            s = (s + 1) & (S - 1);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < S; j += BT_THREADS) {
        bt_slot e;
        e.key = static_cast<int64_t>(sk[j]);
        e.payload = sp[j];
        e.unused = 0;
        I.table[j] = e;
    }
}

__device__ void item_init(const bt_inst &I, int64_t tile, int init_tile)
{
    const int64_t S = int64_t(1) << I.log2_slots;
    const int64_t a = tile * init_tile, b = (a + init_tile < S) ? a + init_tile : S;
    for (int64_t j = a + threadIdx.x; j < b; j += BT_THREADS) {
        bt_slot e;
        e.key = BT_EMPTY;
        e.payload = 0;
        e.unused = 0;
        I.table[j] = e;
    }
}

// Build tile: keys in groups of BT_BUILD_ITEMS per thread, so their first
// compare-and-swap attempts (one slot each, usually a free one at load
// factor <= 0.9) are in flight together; collisions then walk on one by one.
constexpr int BT_BUILD_ITEMS = 4;

__device__ void item_build(const bt_inst &I, int64_t tile, int build_tile, uint32_t *status)
{
    const int L = I.log2_slots;
    const uint64_t mask = (1ull << L) - 1;
    const int64_t a = tile * build_tile, b = (a + build_tile < I.m) ? a + build_tile : I.m;
    for (int64_t i0 = a; i0 < b; i0 += BT_THREADS * BT_BUILD_ITEMS) {
        int64_t k[BT_BUILD_ITEMS];
        int32_t pay[BT_BUILD_ITEMS];
        bool valid[BT_BUILD_ITEMS];
#pragma unroll
        for (int c = 0; c < BT_BUILD_ITEMS; ++c) {
            const int64_t i = i0 + c * BT_THREADS + threadIdx.x;
            valid[c] = i < b;
            k[c] = valid[c] ? I.dim_key[i] : 0;
            pay[c] = valid[c] ? I.dim_attr[i] : 0;
        }
        uint64_t s[BT_BUILD_ITEMS];
        unsigned long long prev[BT_BUILD_ITEMS];
#pragma unroll
        for (int c = 0; c < BT_BUILD_ITEMS; ++c) {
            if (valid[c] && k[c] == BT_EMPTY) {
                inst_raise(I, status, GQ_ERR_INVALID_KEY);
                valid[c] = false;
            }
            s[c] = key_hash(k[c]) >> (64 - L);
            prev[c] = valid[c] ? atomicCAS(reinterpret_cast<unsigned long long *>(&I.table[s[c]].key),
                                           static_cast<unsigned long long>(BT_EMPTY),
                                           static_cast<unsigned long long>(k[c]))
                               : 0ull;
        }
#pragma unroll
        for (int c = 0; c < BT_BUILD_ITEMS; ++c) {
            if (!valid[c]) continue;
            uint64_t p = 0;
            while (true) {
                if (prev[c] == static_cast<unsigned long long>(BT_EMPTY)) {
                    I.table[s[c]].payload = pay[c];
                    break;
                }
                if (prev[c] == static_cast<unsigned long long>(k[c])) {
                    inst_raise(I, status, GQ_ERR_DUPLICATE_KEY);
                    break;
                }
                if (++p > mask) {
                    inst_raise(I, status, GQ_ERR_CAPACITY);
                    break;
                }
                s[c] = (s[c] + 1) & mask;
                prev[c] = atomicCAS(reinterpret_cast<unsigned long long *>(&I.table[s[c]].key),
                                    static_cast<unsigned long long>(BT_EMPTY), static_cast<unsigned long long>(k[c]));
            }
        }
    }
}

// Fused filter -> probe -> aggregate over one tile of fact rows, walked in
// chunks of 8 rows per thread; groups accumulate in LDS for the whole tile
// and are merged into the instance's global group table at its end.  Each
// chunk runs in phases over its 8 rows (dates; foreign keys of the kept
// rows; table slots; value columns of the matches; LDS aggregation), so a
// phase's loads are all in flight together.
constexpr int BT_CHUNK_ITEMS = 4;
constexpr int BT_CHUNK = BT_THREADS * BT_CHUNK_ITEMS;

__device__ void item_probe(const bt_inst &I, int64_t tile, int tile_rows, bt_lds &T, uint32_t *status)
{
    const int L = I.log2_slots;
    const uint64_t mask = (1ull << L) - 1;
    lds_clear(T);
    __syncthreads();
    const int64_t t0 = tile * tile_rows;
    const int64_t t1 = t0 + tile_rows < I.n ? t0 + tile_rows : I.n;
    for (int64_t base = t0; base < t1; base += BT_CHUNK) {
        bool pass[BT_CHUNK_ITEMS];
        int64_t k[BT_CHUNK_ITEMS];
#pragma unroll
        for (int c = 0; c < BT_CHUNK_ITEMS; ++c) {
            const int64_t r = base + c * BT_THREADS + threadIdx.x;
            const int32_t d = r < t1 ? I.date[r] : 0;
            pass[c] = r < t1 && I.date_lo <= d && d < I.date_hi;
        }
#pragma unroll
        for (int c = 0; c < BT_CHUNK_ITEMS; ++c) {
            const int64_t r = base + c * BT_THREADS + threadIdx.x;
            k[c] = pass[c] ? I.fk[r] : BT_EMPTY;
            pass[c] = pass[c] && k[c] != BT_EMPTY;      // the empty-slot marker is no key: it never matches
        }
        uint64_t s[BT_CHUNK_ITEMS];
        int4 v[BT_CHUNK_ITEMS];
#pragma unroll
        for (int c = 0; c < BT_CHUNK_ITEMS; ++c) {
            s[c] = key_hash(k[c]) >> (64 - L);
            if (pass[c]) v[c] = *reinterpret_cast<const int4 *>(&I.table[s[c]]);
        }
        bool hit[BT_CHUNK_ITEMS];
        int32_t g[BT_CHUNK_ITEMS];
#pragma unroll
        for (int c = 0; c < BT_CHUNK_ITEMS; ++c) {
            hit[c] = false;
            g[c] = 0;
            if (pass[c]) {
                int64_t sk = (static_cast<int64_t>(static_cast<uint32_t>(v[c].y)) << 32) | static_cast<uint32_t>(v[c].x);
                uint64_t p = 0;
                while (sk != k[c] && sk != BT_EMPTY && p < mask) {
                    s[c] = (s[c] + 1) & mask;
                    v[c] = *reinterpret_cast<const int4 *>(&I.table[s[c]]);
                    sk = (static_cast<int64_t>(static_cast<uint32_t>(v[c].y)) << 32) | static_cast<uint32_t>(v[c].x);
                    ++p;
                }
                hit[c] = sk == k[c];
                g[c] = v[c].z;
            }
        }
        int64_t q[BT_CHUNK_ITEMS], pr[BT_CHUNK_ITEMS], ds[BT_CHUNK_ITEMS];
#pragma unroll
        for (int c = 0; c < BT_CHUNK_ITEMS; ++c) {
            const int64_t r = base + c * BT_THREADS + threadIdx.x;
            q[c] = hit[c] ? I.qty[r] : 0;
            pr[c] = hit[c] ? I.price[r] : 0;
            ds[c] = hit[c] ? I.disc[r] : 0;
        }
#pragma unroll
        for (int c = 0; c < BT_CHUNK_ITEMS; ++c) {
            const gq_i128 rev = hit[c] ? gq_revenue(pr[c], I.rev_scale, ds[c]) : gq_i128{0, 0};
            const bool fits = rev.hi == (static_cast<int64_t>(rev.lo) >> 63);
            const int slot = lds_group(T, hit[c] && fits, g[c]);
            if (hit[c] && fits && slot >= 0) lds_add_row(T, slot, q[c], static_cast<int64_t>(rev.lo));
            // a full LDS table or a revenue wider than 64 bits goes to the global table
            const bool spill = hit[c] && (!fits || slot < 0);
            const int64_t gs = global_group(I, spill, g[c], status);
            if (spill && gs >= 0) global_add(I, gs, 1, static_cast<uint64_t>(q[c]), rev);
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < BT_LDS_GROUP_SLOTS; s += BT_THREADS) {
        const uint64_t w = T.word[s];
        const bool occ = w != 0ull;
        const int32_t key = static_cast<int32_t>(static_cast<uint32_t>(w >> 32));
        const int64_t gs = global_group(I, occ, key, status);
        if (occ && gs >= 0) global_add(I, gs, T.cnt[s], T.sq[s], split_total(T.lo[s], T.hi[s]));
    }
}

// Compact an instance's global group table into its output (one workgroup).
__device__ void emit_groups(const bt_inst &I, uint32_t *status)
{
    const uint64_t slots = I.gmask + 1;
    for (uint64_t b = 0; b < slots; b += BT_THREADS) {
        const uint64_t s = b + threadIdx.x;
        const bool occ = s < slots && load_acquire(&I.gstate[s]) == 2u;
        const uint64_t mk = gq_ballot(occ);
        unsigned long long base = 0;
        if (mk && gq_lane() == 0)
            base = atomicAdd(reinterpret_cast<unsigned long long *>(I.out.n_groups),
                             static_cast<unsigned long long>(__popcll(mk)));
        base = __shfl(base, 0, 64);
        if (occ) {
            const int64_t idx = static_cast<int64_t>(base + gq_mbcnt(mk));
            if (idx >= I.out.capacity) {
                inst_raise(I, status, GQ_ERR_CAPACITY);
                continue;
            }
            const uint64_t cnt = __hip_atomic_load(&I.gcnt[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t sq = __hip_atomic_load(&I.gsq[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t lo = __hip_atomic_load(&I.glo[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t hi = __hip_atomic_load(&I.ghi[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int32_t key = __hip_atomic_load(&I.gkey[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (I.out.key32) I.out.key32[idx] = key;
            if (I.out.key64) I.out.key64[idx] = key;
            I.out.count[idx] = static_cast<int64_t>(cnt);
            I.out.sum_qty[idx] = static_cast<int64_t>(sq);
            I.out.sum_rev_lo[idx] = lo;
            I.out.sum_rev_hi[idx] = hi;
            const double c = static_cast<double>(static_cast<int64_t>(cnt));
            I.out.avg_qty[idx] = static_cast<double>(static_cast<int64_t>(sq)) / c;
            I.out.avg_rev[idx] = gq_i128_to_double(lo, hi) / c;
        }
    }
}

__global__ __launch_bounds__(BT_THREADS) void batch_kernel(const bt_inst *__restrict__ insts,
                                                           const bt_seg *__restrict__ segs, int nsegs,
                                                           int64_t total_items, uint32_t *work_ctr, int init_tile,
                                                           int build_tile, int probe_tile, int64_t wait_limit,
                                                           uint32_t *status)
{
    // one LDS buffer serves either use: the probe aggregation table or the
    // region copy of a table being built (never both within one item)
    constexpr size_t BUILD_BYTES = BT_REGION_SLOTS * (sizeof(unsigned long long) + sizeof(int32_t));
    constexpr size_t LDS_BYTES = sizeof(bt_lds) > BUILD_BYTES ? sizeof(bt_lds) : BUILD_BYTES;
    __shared__ __align__(16) char lds_buf[LDS_BYTES];
    bt_lds &T = *reinterpret_cast<bt_lds *>(lds_buf);
    unsigned long long *sk = reinterpret_cast<unsigned long long *>(lds_buf);
    int32_t *sp = reinterpret_cast<int32_t *>(lds_buf + BT_REGION_SLOTS * sizeof(unsigned long long));
    __shared__ int64_t s_item;
    __shared__ uint32_t s_last, s_ok;
    // Each pass starts with a barrier that every thread executes, so the
    // thread-0 dequeue below is never fused with the thread-0 tail of the
    // previous item (signal_done): fused, the two would form one divergent
    // path around the loop head, and the other lanes could re-read the old
    // item before thread 0 fetched the next one.
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = static_cast<int64_t>(atomicAdd(work_ctr, 1u));
        __syncthreads();
        const int64_t item = gq_uniform(s_item);
        if (item >= total_items) break;
        int lo = 0, hi = nsegs - 1;                        // last segment with first_item <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (segs[mid].first_item <= item) lo = mid;
            else hi = mid - 1;
        }
        const bt_seg sg = segs[lo];
        const bt_inst &I = insts[sg.inst];
        const int64_t tile = sg.first_tile + (item - sg.first_item);
        if (sg.kind == K_LDS_BUILD) {
            item_lds_build(I, status, sk, sp);
            signal_done(&I.counters[1]);
        } else if (sg.kind == K_INIT) {
            item_init(I, tile, init_tile);
            signal_done(&I.counters[0]);
        } else if (sg.kind == K_BUILD) {
            if (wait_for(&I.counters[0], static_cast<uint32_t>(I.init_items), wait_limit, &s_ok))
                item_build(I, tile, build_tile, status);
            else if (threadIdx.x == 0)
                inst_raise(I, status, GQ_ERR_TIMEOUT);
            signal_done(&I.counters[1]);
        } else {
            if (wait_for(&I.counters[1], static_cast<uint32_t>(I.build_items), wait_limit, &s_ok))
                item_probe(I, tile, probe_tile, T, status);
            else if (threadIdx.x == 0)
                inst_raise(I, status, GQ_ERR_TIMEOUT);
            __syncthreads();
            if (threadIdx.x == 0) {
                __threadfence();
                const uint32_t prev =
                    __hip_atomic_fetch_add(&I.counters[2], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                s_last = (prev + 1 == static_cast<uint32_t>(I.probe_items)) ? 1u : 0u;
            }
            __syncthreads();
            if (gq_uniform(s_last)) {
                __threadfence();
                emit_groups(I, status);
            }
        }
    }
}

// zero-probe instances still need their (empty) output count
__global__ void batch_zero_counts_kernel(const bt_inst *insts, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        *insts[i].out.n_groups = 0;
}

// Each instance's error bits as one status code (the same precedence as the
// context's status word), once the batch kernel has finished.
__global__ void batch_status_kernel(const bt_inst *insts, int n, int32_t *inst_status)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        inst_status[i] = gq_status_of_bits(insts[i].counters[3]);
}

}  // namespace

// --------------------------------------------------------------------------
// host
// --------------------------------------------------------------------------
namespace {

uint64_t pow2_at_least(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct bt_plan {
    std::vector<bt_inst> insts;
    std::vector<bt_seg> segs;
    bt_inst *insts_dev = nullptr;  // where the workspace holds the descriptors
    bt_seg *segs_dev = nullptr;    //   and the segment table
    int64_t total_items = 0;
    size_t bytes = 0;              // workspace bytes
    size_t zero_bytes = 0;         // prefix to clear (counters, group tables)
};

bool valid_tuning(const gq_tuning &t)
{
    return t.load_factor > 0.0 && t.load_factor <= 0.9 && t.probe_tile >= 4096 && t.probe_tile % 4096 == 0 &&
           t.probe_tile <= (1 << 22) && t.build_tile >= BT_TILE_GRAIN && t.build_tile % BT_TILE_GRAIN == 0 &&
           t.init_tile >= BT_TILE_GRAIN && t.init_tile % BT_TILE_GRAIN == 0 && t.lag >= 0 && t.lag <= 1024 &&
           t.fanout >= 1 && t.fanout <= 64;
}

// Lay the workspace out: [work counter | per-instance counters | group tables]
// (cleared) then [descriptors | segments | join tables].
bt_plan make_plan(const gq_instance *in, int n, const gq_tuning &t, char *base)
{
    bt_plan pl;
    gq_carver c(base);
    uint32_t *work = c.take<uint32_t>(64);
    (void)work;
    std::vector<uint32_t *> ctrs(n);
    for (int i = 0; i < n; ++i) ctrs[i] = c.take<uint32_t>(4);
    pl.insts.resize(n);
    for (int i = 0; i < n; ++i) {
        bt_inst &I = pl.insts[i];
        const int64_t cap = in[i].out.capacity;
        const uint64_t gslots = pow2_at_least(static_cast<uint64_t>(cap > 32 ? 2 * cap : 64));
        I.gstate = c.take<uint32_t>(gslots);
        I.gkey = c.take<int32_t>(gslots);
        I.gcnt = c.take<uint64_t>(gslots);
        I.gsq = c.take<uint64_t>(gslots);
        I.glo = c.take<uint64_t>(gslots);
        I.ghi = c.take<int64_t>(gslots);
        I.gmask = gslots - 1;
        I.counters = ctrs[i];
    }
    pl.zero_bytes = c.off;
    pl.insts_dev = c.take<bt_inst>(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        bt_inst &I = pl.insts[i];
        const gq_instance &s = in[i];
        I.dim_key = s.dim_key;
        I.dim_attr = s.dim_attr;
        I.fk = s.fk;
        I.date = s.date;
        I.qty = s.qty;
        I.price = s.price;
        I.disc = s.disc;
        I.m = s.m;
        I.n = s.n;
        I.date_lo = s.date_lo;
        I.date_hi = s.date_hi;
        I.rev_scale = s.rev_scale;
        I.out = s.out;
        int L = 6;
        while (static_cast<double>(1ull << L) < static_cast<double>(s.m) / t.load_factor) ++L;
        I.log2_slots = L;
        I.table = c.take<bt_slot>(size_t(1) << L);
        const int64_t slots = int64_t(1) << L;
        const bool lds = slots <= BT_REGION_SLOTS;
        I.init_items = lds ? 0 : static_cast<int32_t>((slots + t.init_tile - 1) / t.init_tile);
        I.build_items = lds ? 1 : static_cast<int32_t>((s.m + t.build_tile - 1) / t.build_tile);
        I.probe_items = static_cast<int32_t>((s.n + t.probe_tile - 1) / t.probe_tile);
    }
    // queue order: setup (init + build) of instance i, then probes of instance i - lag
    auto push = [&](int kind, int i, int64_t cnt) {
        if (cnt <= 0) return;
        bt_seg sg;
        sg.first_item = pl.total_items;
        sg.kind = kind;
        sg.inst = i;
        sg.first_tile = 0;
        sg.ntiles = cnt;
        pl.segs.push_back(sg);
        pl.total_items += cnt;
    };
    auto push_setup = [&](int i) {
        const bt_inst &I = pl.insts[i];
        if (I.init_items == 0) push(K_LDS_BUILD, i, 1);
        else {
            push(K_INIT, i, I.init_items);
            push(K_BUILD, i, I.build_items);
        }
    };
    // probe items: instances in groups of `fanout`; the probe tiles of a
    // group's instances are interleaved one by one (fanout 1: instance after
    // instance), so that many instances' probes are in flight together or
    // one instance's table is probed by every workgroup at once
    auto push_probes = [&](int g0, int g1) {
        if (g1 - g0 == 1) {
            push(K_PROBE, g0, pl.insts[g0].probe_items);
            return;
        }
        int32_t most = 0;
        for (int i = g0; i < g1; ++i) most = std::max(most, pl.insts[i].probe_items);
        for (int32_t tile = 0; tile < most; ++tile)
            for (int i = g0; i < g1; ++i)
                if (tile < pl.insts[i].probe_items) {
                    bt_seg sg;
                    sg.first_item = pl.total_items;
                    sg.kind = K_PROBE;
                    sg.inst = i;
                    sg.first_tile = tile;
                    sg.ntiles = 1;
                    pl.segs.push_back(sg);
                    pl.total_items += 1;
                }
    };
    const int F = std::max(1, t.fanout);
    for (int i = 0; i < n + t.lag; ++i) {
        if (i < n) push_setup(i);
        const int j = i - t.lag;
        if (j >= 0 && j < n && (j % F == F - 1 || j == n - 1)) push_probes(j - j % F, j + 1);
    }
    // the segment table goes last: its length depends on the fan-out
    pl.segs_dev = c.take<bt_seg>(pl.segs.size() + 1);
    pl.bytes = c.bytes();
    return pl;
}

}  // namespace

extern "C" {

gq_tuning gq_default_tuning(void)
{
    gq_tuning t;
    t.load_factor = 0.5;
    t.probe_tile = 8192;
    t.build_tile = 4096;
    t.init_tile = 16384;
    t.lag = 2;
    t.fanout = 1;
    return t;
}

size_t gq_batch_workspace_bytes(const gq_instance *inst, int n_inst, const gq_tuning *tuning)
{
    if (!inst || n_inst < 1) return 0;
    const gq_tuning t = tuning ? *tuning : gq_default_tuning();
    if (!valid_tuning(t)) return 0;
    return make_plan(inst, n_inst, t, nullptr).bytes;
}

gq_status gq_batch_join_agg(gq_ctx *ctx, const gq_instance *inst, int n_inst, const gq_tuning *tuning,
                            gq_status *inst_status_dev, void *ws, size_t ws_bytes, gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (!inst || n_inst < 1) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_batch_join_agg: no instances");
    const gq_tuning t = tuning ? *tuning : gq_default_tuning();
    if (!valid_tuning(t)) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_batch_join_agg: invalid tuning");
    for (int i = 0; i < n_inst; ++i) {
        const gq_instance &s = inst[i];
        if (s.m < 0 || s.n < 0 || s.m > GQ_MAX_ROWS || s.n > GQ_MAX_ROWS || (s.m > 0 && (!s.dim_key || !s.dim_attr)) ||
            (s.n > 0 && (!s.fk || !s.date || !s.qty || !s.price || !s.disc)) || !s.out.count || !s.out.sum_qty ||
            !s.out.sum_rev_lo || !s.out.sum_rev_hi || !s.out.avg_qty || !s.out.avg_rev || !s.out.n_groups ||
            !s.out.key32 || s.out.capacity < 1 || s.out.capacity > (int64_t(1) << 24))
            return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_batch_join_agg: bad instance %d", i);
    }
    const size_t need = gq_batch_workspace_bytes(inst, n_inst, &t);
    if (!ws || ws_bytes < need)
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_batch_join_agg: workspace %zu < %zu bytes", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_batch_join_agg: workspace must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    bt_plan pl = make_plan(inst, n_inst, t, base);
    gq_carver c(base);
    uint32_t *work = c.take<uint32_t>(64);
    bt_inst *d_insts = pl.insts_dev;
    bt_seg *d_segs = pl.segs_dev;
    GQ_TRY(gq_zero(ctx, ws, pl.zero_bytes / 4, s));
    GQ_CHECK_HIP(ctx, hipMemcpyAsync(d_insts, pl.insts.data(), sizeof(bt_inst) * n_inst, hipMemcpyHostToDevice, s));
    if (!pl.segs.empty())
        GQ_CHECK_HIP(ctx, hipMemcpyAsync(d_segs, pl.segs.data(), sizeof(bt_seg) * pl.segs.size(),
                                         hipMemcpyHostToDevice, s));
    GQ_TRY(gq_launch(ctx, "gq_batch_zero", batch_zero_counts_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, s,
                     static_cast<const bt_inst *>(d_insts), n_inst));
    if (pl.total_items > 0) {
        // three 48 KiB-LDS workgroups fit a CU
        const uint32_t grid = static_cast<uint32_t>(std::min<int64_t>(pl.total_items, int64_t(ctx->num_cus) * 3));
        const int nsegs = static_cast<int>(pl.segs.size());
        GQ_TRY(gq_launch(ctx, "gq_batch", batch_kernel, dim3(grid), dim3(BT_THREADS), 0, s,
                         static_cast<const bt_inst *>(d_insts), static_cast<const bt_seg *>(d_segs), nsegs,
                         pl.total_items, work, t.init_tile, t.build_tile, t.probe_tile, ctx->wait_limit,
                         ctx->status_dev));
    }
    if (!inst_status_dev) return GQ_OK;
    return gq_launch(ctx, "gq_batch_status", batch_status_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, s,
                     static_cast<const bt_inst *>(d_insts), n_inst, static_cast<int32_t *>(inst_status_dev));
}

}  // extern "C"

// --------------------------------------------------------------------------
// Autotuner: run the batch once per candidate tuning (after one warm-up run),
// time each on the stream with events, keep the fastest.  Results are
// identical for every candidate (integer sums are order independent).  A
// text cache (one line per workload signature) skips the search next time.
// --------------------------------------------------------------------------
namespace {

// What the fastest tuning depends on: the device (compute units, LDS) and,
// per instance, the table and probe sizes, the filter range and the group
// capacity (which sizes the group tables).
uint64_t batch_signature(const gq_ctx *ctx, const gq_instance *in, int n)
{
    uint64_t h = 0x9E3779B97F4A7C15ull ^ static_cast<uint64_t>(n);
    auto mix = [&h](uint64_t v) {
        h = (h ^ v) * 0xff51afd7ed558ccdull;
        h ^= h >> 29;
    };
    mix(static_cast<uint64_t>(ctx->num_cus));
    mix(static_cast<uint64_t>(ctx->lds_per_cu));
    for (int i = 0; i < n; ++i) {
        mix(static_cast<uint64_t>(in[i].m));
        mix(static_cast<uint64_t>(in[i].n));
        mix(static_cast<uint64_t>(in[i].date_lo));
        mix(static_cast<uint64_t>(in[i].date_hi));
        mix(static_cast<uint64_t>(in[i].out.capacity));
    }
    return h;
}

// The search space, one axis per tuning field.  The search is coordinate
// descent: from a starting point, each axis in turn is swept with the others
// fixed and its best value kept, for two rounds; each axis reaches beyond the
// values that win on the MI355X, so the winner lies inside the grid.
constexpr double TUNE_LF[] = {0.2, 0.25, 0.3, 0.4, 0.5, 0.6, 0.7};
constexpr int TUNE_TILE[] = {8192, 16384, 32768, 65536, 131072, 262144, 524288};
constexpr int TUNE_LAG[] = {1, 2, 4, 8, 16, 32, 64, 128, 256, 512};
constexpr int TUNE_FANOUT[] = {1, 2, 4, 8, 16};
constexpr int TUNE_BUILD[] = {1024, 4096, 16384, 65536};
constexpr int TUNE_ROUNDS = 2;

gq_tuning tune_start()
{
    gq_tuning t = gq_default_tuning();
    t.probe_tile = 65536;
    t.lag = 4;
    return t;
}

bool same_tuning(const gq_tuning &a, const gq_tuning &b)
{
    return a.load_factor == b.load_factor && a.probe_tile == b.probe_tile && a.build_tile == b.build_tile &&
           a.init_tile == b.init_tile && a.lag == b.lag && a.fanout == b.fanout;
}

// The points one sweep of axis `axis` visits from `base`.
std::vector<gq_tuning> axis_points(const gq_tuning &base, int axis)
{
    std::vector<gq_tuning> v;
    auto add = [&](gq_tuning t) { v.push_back(t); };
    gq_tuning t = base;
    switch (axis) {
    case 0: for (double x : TUNE_LF) { t.load_factor = x; add(t); } break;
    case 1: for (int x : TUNE_TILE) { t.probe_tile = x; add(t); } break;
    case 2: for (int x : TUNE_LAG) { t.lag = x; add(t); } break;
    case 3: for (int x : TUNE_FANOUT) { t.fanout = x; add(t); } break;
    default: for (int x : TUNE_BUILD) { t.build_tile = x; add(t); } break;
    }
    return v;
}
constexpr int TUNE_AXES = 5;

bool cache_lookup(const char *path, uint64_t sig, gq_tuning *t, double *ms)
{
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        unsigned long long s;
        gq_tuning x = gq_default_tuning();
        double m;
        if (sscanf(line, "%llx %lf %d %d %d %d %d %lf", &s, &x.load_factor, &x.probe_tile, &x.build_tile,
                   &x.init_tile, &x.lag, &x.fanout, &m) == 8 &&
            s == sig && valid_tuning(x)) {
            *t = x;
            *ms = m;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, uint64_t sig, const gq_tuning &t, double ms)
{
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%llx %.3f %d %d %d %d %d %.4f\n", static_cast<unsigned long long>(sig), t.load_factor, t.probe_tile,
            t.build_tile, t.init_tile, t.lag, t.fanout, ms);
    fclose(f);
}

}  // namespace

extern "C" {

size_t gq_batch_autotune_workspace_bytes(const gq_instance *inst, int n_inst)
{
    // the largest point: the lowest load factor (largest tables) with the
    // longest segment table (smallest tiles, widest fan-out, smallest builds)
    size_t best = 0;
    for (double lf : TUNE_LF) {
        gq_tuning t = tune_start();
        t.load_factor = lf;
        t.probe_tile = TUNE_TILE[0];
        t.fanout = TUNE_FANOUT[sizeof(TUNE_FANOUT) / sizeof(TUNE_FANOUT[0]) - 1];
        t.build_tile = TUNE_BUILD[0];
        best = std::max(best, gq_batch_workspace_bytes(inst, n_inst, &t));
    }
    return best;
}

gq_status gq_batch_autotune(gq_ctx *ctx, const gq_instance *inst, int n_inst, const char *cache_path,
                            gq_tuning *best, double *best_ms, void *ws, size_t ws_bytes, gq_stream stream)
{
    if (!ctx || !best || !best_ms) return GQ_ERR_INVALID_ARG;
    if (!inst || n_inst < 1) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_batch_autotune: no instances");
    const uint64_t sig = batch_signature(ctx, inst, n_inst);
    if (cache_lookup(cache_path, sig, best, best_ms)) return GQ_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    GQ_CHECK_HIP(ctx, hipEventCreate(&e0));
    GQ_CHECK_HIP(ctx, hipEventCreate(&e1));
    gq_status rc = GQ_OK;
    // one warm-up run, then the time of one run, on the caller's stream
    auto time_of = [&](const gq_tuning &t, double *ms_out) -> gq_status {
        GQ_TRY(gq_batch_join_agg(ctx, inst, n_inst, &t, nullptr, ws, ws_bytes, stream));
        GQ_CHECK_HIP(ctx, hipEventRecord(e0, s));
        GQ_TRY(gq_batch_join_agg(ctx, inst, n_inst, &t, nullptr, ws, ws_bytes, stream));
        GQ_CHECK_HIP(ctx, hipEventRecord(e1, s));
        GQ_CHECK_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        GQ_CHECK_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        *ms_out = ms;
        return GQ_OK;
    };
    gq_tuning bt = tune_start();
    double bms = 1e30;
    rc = time_of(bt, &bms);
    for (int round = 0; round < TUNE_ROUNDS && rc == GQ_OK; ++round) {
        bool moved = false;
        for (int axis = 0; axis < TUNE_AXES && rc == GQ_OK; ++axis) {
            const gq_tuning from = bt;
            for (const gq_tuning &t : axis_points(from, axis)) {
                if (same_tuning(t, from)) continue;
                double ms = 0.0;
                rc = time_of(t, &ms);
                if (rc != GQ_OK) break;
                if (ms < bms) {
                    bms = ms;
                    bt = t;
                    moved = true;
                }
            }
        }
        if (!moved) break;                               // a full round changed nothing
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != GQ_OK) return rc;
    *best = bt;
    *best_ms = bms;
    cache_store(cache_path, sig, bt, bms);
    return GQ_OK;
}

}  // extern "C"
