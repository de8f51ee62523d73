// Group-by aggregate with exact fixed-point sums, then the float64 finalize.
//
// Per key (key64, key32): count, sum(qty) (wrapping int64) and the exact
// 128-bit sum of price * (rev_scale - disc).  Device-wide atomics on MI355X
// run at a few tens of G/s for the whole chip while LDS atomics run far
// faster, so every row is aggregated in LDS:
//
//  small path (max_groups <= GB_SMALL_GROUPS): a persistent grid; each
//    workgroup aggregates its share of the rows into a private LDS table and
//    merges it into one global table at the end (a few atomics per group per
//    workgroup); a finalize kernel compacts the global table.
//
//  large path: the rows are hash-partitioned by key into P buckets (hist ->
//    scan -> LDS-staged scatter of key and value columns), chosen so that a
//    bucket's groups fit one LDS table; one workgroup per bucket aggregates it
//    in LDS and writes its groups out directly.  A bucket whose keys overflow
//    its LDS table sends the extra keys to a global fallback table (correct,
//    slower), compacted by the same finalize kernel.
//
// Table protocol (LDS and global alike): a per-slot state word 0 = empty,
// 1 = being claimed, 2 = key published.  A lane claims a slot with a CAS
// 0 -> 1, writes the key and publishes state 2; a lane that sees state 1
// retries the same slot on its next pass of a wave-uniform loop, so the
// claiming lane always finishes first.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "gq_device.h"
#include "gq_internal.h"
#include "gq_ops.h"

namespace {

constexpr int GB_THREADS = 256;
constexpr int GB_SMALL_SLOTS = 1024;
constexpr int64_t GB_SMALL_GROUPS = 512;
constexpr int GB_ITEMS = 16;
constexpr int GB_TILE = GB_THREADS * GB_ITEMS;       // rows per hist/scatter tile
constexpr int GB_MAX_LOG2P = 10;
constexpr int GB_BUCKET_THREADS = 1024;
constexpr int GB_LDS_PROBES = 64;

struct gb_args {
    int64_t n_bound;
    const int64_t *n_dev;
    const int32_t *rowid;
    const int64_t *key64;
    int32_t key64_by_rowid;
    const int32_t *key32;
    int32_t key32_by_rowid;
    const int64_t *qty;
    const int64_t *price;
    const int64_t *disc;
    int64_t rev_scale;
    const int32_t *filter;          // nullable: rows need flo <= filter[v] < fhi
    int64_t flo, fhi;
};

GQ_DEV int64_t eff_n(int64_t bound, const int64_t *n_dev)
{
    if (!n_dev) return bound;
    const int64_t d = *n_dev;
    return d < bound ? (d > 0 ? d : 0) : bound;
}

GQ_DEV uint64_t gb_hash(int64_t k64, int32_t k32)
{
    return gq_fmix64(static_cast<uint64_t>(k64) ^
                     (static_cast<uint64_t>(static_cast<uint32_t>(k32)) * 0x9E3779B97F4A7C15ull));
}

// Value row of input row j and whether it passes the optional row filter.
GQ_DEV int64_t value_row(const gb_args &a, int64_t j) { return a.rowid ? static_cast<int64_t>(a.rowid[j]) : j; }

GQ_DEV bool row_pass(const gb_args &a, int64_t v)
{
    if (!a.filter) return true;
    const int64_t f = a.filter[v];
    return a.flo <= f && f < a.fhi;
}

template <bool K64, bool K32>
struct gb_row {
    int64_t k64;
    int32_t k32;
    int64_t qty;
    gq_i128 rev;
};

template <bool K64, bool K32>
GQ_DEV gb_row<K64, K32> load_row(const gb_args &a, int64_t j)
{
    gb_row<K64, K32> r;
    const int64_t v = a.rowid ? static_cast<int64_t>(a.rowid[j]) : j;
    r.k64 = K64 ? a.key64[a.key64_by_rowid ? v : j] : 0;
    r.k32 = K32 ? a.key32[a.key32_by_rowid ? v : j] : 0;
    r.qty = a.qty[v];
    r.rev = gq_revenue(a.price[v], a.rev_scale, a.disc[v]);
    return r;
}

// ----------------------------------------------------------------- LDS table
template <int SLOTS, bool K64, bool K32>
struct lds_table {
    uint32_t state[SLOTS];
    uint32_t cnt[SLOTS];
    int32_t k32[K32 ? SLOTS : 1];
    int64_t k64[K64 ? SLOTS : 1];
    uint64_t sq[SLOTS];
    uint64_t lo[SLOTS];
    int64_t hi[SLOTS];
};

template <int SLOTS>
GQ_DEV uint32_t lds_home(uint64_t h)
{
    // bits 8..39 of the hash, scaled to [0, SLOTS); the top bits pick buckets
    return static_cast<uint32_t>((static_cast<uint64_t>(static_cast<uint32_t>(h >> 8)) * SLOTS) >> 32);
}

template <int SLOTS, bool K64, bool K32>
GQ_DEV void lds_init(lds_table<SLOTS, K64, K32> &T)
{
    for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) {
        T.state[s] = 0;
        T.cnt[s] = 0;
        T.sq[s] = 0;
        T.lo[s] = 0;
        T.hi[s] = 0;
    }
}

// Find or claim the slot of a key; -1 if absent after GB_LDS_PROBES slots
// (the table is then treated as full for that key).  Wave-uniform loop.
template <int SLOTS, bool K64, bool K32>
GQ_DEV int lds_find(lds_table<SLOTS, K64, K32> &T, bool active, uint64_t h, int64_t k64, int32_t k32)
{
    uint32_t s = lds_home<SLOTS>(h);
    int probes = 0, found = -1;
    bool done = !active;
    while (__any(!done)) {
        if (!done) {
            const uint32_t st = atomicCAS(&T.state[s], 0u, 1u);
            if (st == 0u) {
                if (K64) T.k64[s] = k64;
                if (K32) T.k32[s] = k32;
                __threadfence_block();
                atomicExch(&T.state[s], 2u);
                found = static_cast<int>(s);
                done = true;
            } else if (st == 2u) {
                const bool eq = (!K64 || T.k64[s] == k64) && (!K32 || T.k32[s] == k32);
                if (eq) {
                    found = static_cast<int>(s);
                    done = true;
                } else if (++probes >= GB_LDS_PROBES) {
                    done = true;
                } else {
                    s = (s + 1 == SLOTS) ? 0 : s + 1;
                }
            }
        }
    }
    return found;
}

template <int SLOTS, bool K64, bool K32>
GQ_DEV void lds_add(lds_table<SLOTS, K64, K32> &T, int s, uint32_t cnt, uint64_t qty, gq_i128 rev)
{
    atomicAdd(&T.cnt[s], cnt);
    atomicAdd(reinterpret_cast<unsigned long long *>(&T.sq[s]), static_cast<unsigned long long>(qty));
    const unsigned long long old =
        atomicAdd(reinterpret_cast<unsigned long long *>(&T.lo[s]), static_cast<unsigned long long>(rev.lo));
    const int64_t hadd = rev.hi + ((old + rev.lo < old) ? 1 : 0);
    if (hadd) atomicAdd(reinterpret_cast<unsigned long long *>(&T.hi[s]), static_cast<unsigned long long>(hadd));
}

// -------------------------------------------------------------- global table
struct gtable {
    uint32_t *state;
    int64_t *k64;
    int32_t *k32;
    uint64_t *cnt;
    uint64_t *sq;
    uint64_t *lo;
    int64_t *hi;
    uint64_t mask;
};

template <bool K64, bool K32>
GQ_DEV int64_t g_find(const gtable &g, bool active, uint64_t h, int64_t k64, int32_t k32, uint32_t *status)
{
    uint64_t s = h & g.mask;
    uint64_t probes = 0;
    int64_t found = -1;
    bool done = !active;
    while (__any(!done)) {
        if (!done) {
            const uint32_t st = atomicCAS(&g.state[s], 0u, 1u);
            if (st == 0u) {
                if (K64) __hip_atomic_store(&g.k64[s], k64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (K32) __hip_atomic_store(&g.k32[s], k32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&g.state[s], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                found = static_cast<int64_t>(s);
                done = true;
            } else if (st == 2u) {
                (void)__hip_atomic_load(&g.state[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                const bool eq =
                    (!K64 || __hip_atomic_load(&g.k64[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == k64) &&
                    (!K32 || __hip_atomic_load(&g.k32[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == k32);
                if (eq) {
                    found = static_cast<int64_t>(s);
                    done = true;
                } else if (++probes > g.mask) {
                    gq_raise(status, GQ_ERR_CAPACITY);
                    done = true;
                } else {
                    s = (s + 1) & g.mask;
                }
            }
        }
    }
    return found;
}

GQ_DEV void g_add(const gtable &g, int64_t s, uint64_t cnt, uint64_t qty, gq_i128 rev)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(&g.cnt[s]), static_cast<unsigned long long>(cnt));
    atomicAdd(reinterpret_cast<unsigned long long *>(&g.sq[s]), static_cast<unsigned long long>(qty));
    const unsigned long long old =
        atomicAdd(reinterpret_cast<unsigned long long *>(&g.lo[s]), static_cast<unsigned long long>(rev.lo));
    const int64_t hadd = rev.hi + ((old + rev.lo < old) ? 1 : 0);
    if (hadd) atomicAdd(reinterpret_cast<unsigned long long *>(&g.hi[s]), static_cast<unsigned long long>(hadd));
}

// Append one finished group to the output (idx from the caller's counter).
GQ_DEV void emit_group(const gq_groups &out, int64_t idx, int64_t k64, int32_t k32, uint64_t cnt, uint64_t sq,
                       uint64_t lo, int64_t hi, uint32_t *status)
{
    if (idx >= out.capacity) {
        gq_raise(status, GQ_ERR_CAPACITY);
        return;
    }
    if (out.key64) out.key64[idx] = k64;
    if (out.key32) out.key32[idx] = k32;
    out.count[idx] = static_cast<int64_t>(cnt);
    out.sum_qty[idx] = static_cast<int64_t>(sq);
    out.sum_rev_lo[idx] = lo;
    out.sum_rev_hi[idx] = hi;
    const double c = static_cast<double>(static_cast<int64_t>(cnt));
    out.avg_qty[idx] = static_cast<double>(static_cast<int64_t>(sq)) / c;
    out.avg_rev[idx] = gq_i128_to_double(lo, hi) / c;
}

// ------------------------------------------------------------- small path
template <bool K64, bool K32>
__global__ __launch_bounds__(GB_THREADS) void gb_small_kernel(gb_args a, gtable g, uint32_t *status)
{
    __shared__ lds_table<GB_SMALL_SLOTS, K64, K32> T;
    lds_init(T);
    __syncthreads();
    const int64_t n = eff_n(a.n_bound, a.n_dev);
    const int64_t step = static_cast<int64_t>(gridDim.x) * GB_TILE;
    for (int64_t j0 = static_cast<int64_t>(blockIdx.x) * GB_TILE; j0 < n; j0 += step) {
#pragma unroll 4
        for (int c = 0; c < GB_ITEMS; ++c) {
            const int64_t j = j0 + c * GB_THREADS + threadIdx.x;
            bool active = j < n && row_pass(a, value_row(a, j));
            gb_row<K64, K32> r{};
            if (active) r = load_row<K64, K32>(a, j);
            const uint64_t h = gb_hash(r.k64, r.k32);
            const int s = lds_find(T, active, h, r.k64, r.k32);
            if (active && s >= 0) lds_add(T, s, 1u, static_cast<uint64_t>(r.qty), r.rev);
            const bool spill = active && s < 0;
            const int64_t gs = g_find<K64, K32>(g, spill, h, r.k64, r.k32, status);
            if (spill && gs >= 0) g_add(g, gs, 1u, static_cast<uint64_t>(r.qty), r.rev);
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < GB_SMALL_SLOTS; s += GB_THREADS) {
        const bool occ = T.state[s] == 2u;
        const int64_t k64 = (K64 && occ) ? T.k64[s] : 0;
        const int32_t k32 = (K32 && occ) ? T.k32[s] : 0;
        const int64_t gs = g_find<K64, K32>(g, occ, gb_hash(k64, k32), k64, k32, status);
        if (occ && gs >= 0) {
            gq_i128 rv;
            rv.lo = T.lo[s];
            rv.hi = T.hi[s];
            g_add(g, gs, T.cnt[s], T.sq[s], rv);
        }
    }
}

// Compact the occupied slots of a global table into the output.
template <bool K64, bool K32>
__global__ __launch_bounds__(256) void gb_table_emit_kernel(gtable g, gq_groups out, uint32_t *status)
{
    const uint64_t slots = g.mask + 1;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t b = static_cast<uint64_t>(blockIdx.x) * blockDim.x; b < slots; b += stride) {
        const uint64_t s = b + threadIdx.x;
        const bool occ = s < slots && g.state[s] == 2u;
        const uint64_t m = gq_ballot(occ);
        if (!m) continue;
        unsigned long long basei = 0;
        if (gq_lane() == 0)
            basei = atomicAdd(reinterpret_cast<unsigned long long *>(out.n_groups),
                              static_cast<unsigned long long>(__popcll(m)));
        basei = __shfl(basei, 0, 64);
        if (occ)
            emit_group(out, static_cast<int64_t>(basei + gq_mbcnt(m)), K64 ? g.k64[s] : 0, K32 ? g.k32[s] : 0,
                       g.cnt[s], g.sq[s], g.lo[s], g.hi[s], status);
    }
}

// -------------------------------------------------------------- large path
//
// Partitioned rows are AoS records of 32 bytes (key64 or key32, qty, price,
// disc) or 64 bytes (composite key), written whole from registers: every
// record covers whole 32-byte memory sectors, so scattered short runs cost no
// partial-sector write amplification and need no LDS staging.
// A record is stored and loaded as whole 16-byte vectors (padding included),
// so each 32-byte sector is written completely by one store pair.
template <bool K64, bool K32>
struct gb_rec {
    static constexpr int VECS = (K64 && K32) ? 4 : 2;   // 16-byte vectors per record
    uint4 v[VECS];
};

template <bool K64, bool K32>
GQ_DEV gb_rec<K64, K32> make_rec(int64_t k64, int32_t k32, int64_t qty, int64_t price, int64_t disc)
{
    gb_rec<K64, K32> r;
    const uint64_t kw = K64 ? static_cast<uint64_t>(k64) : static_cast<uint64_t>(static_cast<uint32_t>(k32));
    r.v[0] = make_uint4(static_cast<uint32_t>(kw), static_cast<uint32_t>(kw >> 32), static_cast<uint32_t>(qty),
                        static_cast<uint32_t>(static_cast<uint64_t>(qty) >> 32));
    r.v[1] = make_uint4(static_cast<uint32_t>(price), static_cast<uint32_t>(static_cast<uint64_t>(price) >> 32),
                        static_cast<uint32_t>(disc), static_cast<uint32_t>(static_cast<uint64_t>(disc) >> 32));
    if constexpr (K64 && K32) {
        r.v[2] = make_uint4(static_cast<uint32_t>(k32), 0u, 0u, 0u);
        r.v[3] = make_uint4(0u, 0u, 0u, 0u);
    }
    return r;
}

GQ_DEV int64_t u64_of(uint32_t lo, uint32_t hi)
{
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

template <bool K64, bool K32>
GQ_DEV void read_rec(const gb_rec<K64, K32> *recs, int64_t i, int64_t &k64, int32_t &k32, int64_t &qty,
                     int64_t &price, int64_t &disc)
{
    const uint4 *p = reinterpret_cast<const uint4 *>(recs + i);
    const uint4 a = p[0], b = p[1];
    k64 = K64 ? u64_of(a.x, a.y) : 0;
    k32 = K32 ? static_cast<int32_t>(K64 ? p[2].x : a.x) : 0;
    qty = u64_of(a.z, a.w);
    price = u64_of(b.x, b.y);
    disc = u64_of(b.z, b.w);
}

template <bool K64, bool K32>
GQ_DEV void load_key(const gb_args &a, int64_t j, int64_t &k64, int32_t &k32)
{
    int64_t v = j;
    if (a.rowid && ((K64 && a.key64_by_rowid) || (K32 && a.key32_by_rowid))) v = a.rowid[j];
    k64 = K64 ? a.key64[a.key64_by_rowid ? v : j] : 0;
    k32 = K32 ? a.key32[a.key32_by_rowid ? v : j] : 0;
}

// LDS histogram of one tile of rows, written as the tile's row hist[t * P + b].
template <bool K64, bool K32>
__global__ __launch_bounds__(GB_THREADS) void gb_hist_kernel(gb_args a, int log2p, int items,
                                                             uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[1 << GB_MAX_LOG2P];
    const int P = 1 << log2p;
    for (int i = threadIdx.x; i < P; i += GB_THREADS) h[i] = 0;
    __syncthreads();
    const int64_t n = eff_n(a.n_bound, a.n_dev);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GB_THREADS * items;
#pragma unroll 4
    for (int c = 0; c < items; ++c) {
        const int64_t j = base + c * GB_THREADS + threadIdx.x;
        if (j < n && row_pass(a, value_row(a, j))) {
            int64_t k64;
            int32_t k32;
            load_key<K64, K32>(a, j, k64, k32);
            atomicAdd(&h[static_cast<uint32_t>(gb_hash(k64, k32) >> (64 - log2p))], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < P; b += GB_THREADS) hist[static_cast<int64_t>(blockIdx.x) * P + b] = h[b];
}

// Scatter rows to their buckets: rank inside (bucket, tile) by an LDS atomic
// (order inside a bucket is irrelevant to sums), then write each record whole
// to gofs[b, t] + rank.
template <bool K64, bool K32>
__global__ __launch_bounds__(GB_THREADS) void gb_scatter_kernel(gb_args a, int log2p,
                                                                const uint32_t *__restrict__ gofs, int64_t ntiles,
                                                                gb_rec<K64, K32> *__restrict__ recs)
{
    constexpr int PMAX = 1 << GB_MAX_LOG2P;
    __shared__ uint32_t lcnt[PMAX];
    __shared__ uint32_t gstart[PMAX];
    const int P = 1 << log2p;
    const uint32_t tile = gq_xcd_tile(blockIdx.x, gridDim.x);
    const int64_t n = eff_n(a.n_bound, a.n_dev);
    const int64_t base = static_cast<int64_t>(tile) * GB_TILE;
    if (base >= n) return;                          // whole block: uniform
    for (int b = threadIdx.x; b < P; b += GB_THREADS) {
        lcnt[b] = 0;
        gstart[b] = gofs[static_cast<int64_t>(tile) * P + b];
    }
    __syncthreads();
    gb_rec<K64, K32> r[GB_ITEMS];
    uint32_t dst[GB_ITEMS];
    bool keep[GB_ITEMS];
#pragma unroll
    for (int c = 0; c < GB_ITEMS; ++c) {
        const int64_t j = base + c * GB_THREADS + threadIdx.x;
        const int64_t v = j < n ? value_row(a, j) : 0;
        keep[c] = j < n && row_pass(a, v);
        if (keep[c]) {
            int64_t k64 = 0;
            int32_t k32 = 0;
            if (K64) k64 = a.key64[a.key64_by_rowid ? v : j];
            if (K32) k32 = a.key32[a.key32_by_rowid ? v : j];
            r[c] = make_rec<K64, K32>(k64, k32, a.qty[v], a.price[v], a.disc[v]);
            const uint32_t b = static_cast<uint32_t>(gb_hash(k64, k32) >> (64 - log2p));
            dst[c] = (b << 20) | atomicAdd(&lcnt[b], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < GB_ITEMS; ++c) {
        if (keep[c]) {
            const uint32_t b = dst[c] >> 20;
            uint4 *d = reinterpret_cast<uint4 *>(recs + static_cast<int64_t>(gstart[b]) + (dst[c] & 0xfffffu));
#pragma unroll
            for (int q = 0; q < gb_rec<K64, K32>::VECS; ++q) d[q] = r[c].v[q];
        }
    }
}

// Staged variant: records are placed in LDS in bucket order and written out
// as contiguous runs (consecutive threads store consecutive 16-byte vectors).
constexpr int GB_STAGED_ITEMS = 8;                  // 2048-row tiles: 64 KiB of 32-byte records

template <bool K64, bool K32>
__global__ __launch_bounds__(GB_THREADS) void gb_scatter_staged_kernel(gb_args a, int log2p,
                                                                       const uint32_t *__restrict__ gofs,
                                                                       int64_t ntiles,
                                                                       gb_rec<K64, K32> *__restrict__ recs)
{
    constexpr int PMAX = 1 << GB_MAX_LOG2P;
    constexpr int ITEMS = (K64 && K32) ? GB_STAGED_ITEMS / 2 : GB_STAGED_ITEMS;
    constexpr int TILE = GB_THREADS * ITEMS;
    constexpr int VECS = gb_rec<K64, K32>::VECS;
    __shared__ uint32_t lcnt[PMAX];
    __shared__ uint32_t lstart[PMAX];
    __shared__ uint32_t gstart[PMAX];
    __shared__ uint32_t scan_smem[GB_THREADS / 64];
    __shared__ uint16_t lbucket[TILE];
    __shared__ uint4 stage[TILE * VECS];
    const int P = 1 << log2p;
    const uint32_t tile = gq_xcd_tile(blockIdx.x, gridDim.x);
    const int64_t n = eff_n(a.n_bound, a.n_dev);
    const int64_t base = static_cast<int64_t>(tile) * TILE;
    if (base >= n) return;                          // whole block: uniform
    for (int b = threadIdx.x; b < P; b += GB_THREADS) lcnt[b] = 0;
    __syncthreads();
    gb_rec<K64, K32> r[ITEMS];
    uint32_t pos[ITEMS];
    bool keep[ITEMS];
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int64_t j = base + c * GB_THREADS + threadIdx.x;
        const int64_t v = j < n ? value_row(a, j) : 0;
        keep[c] = j < n && row_pass(a, v);
        if (keep[c]) {
            int64_t k64 = 0;
            int32_t k32 = 0;
            if (K64) k64 = a.key64[a.key64_by_rowid ? v : j];
            if (K32) k32 = a.key32[a.key32_by_rowid ? v : j];
            r[c] = make_rec<K64, K32>(k64, k32, a.qty[v], a.price[v], a.disc[v]);
            const uint32_t b = static_cast<uint32_t>(gb_hash(k64, k32) >> (64 - log2p));
            pos[c] = (b << 16) | atomicAdd(&lcnt[b], 1u);
        }
    }
    __syncthreads();
    const int per = (P + GB_THREADS - 1) / GB_THREADS;
    uint32_t local = 0;
    for (int i = 0; i < per; ++i) {
        const int b = threadIdx.x * per + i;
        if (b < P) local += lcnt[b];
    }
    uint32_t all;
    uint32_t run = gq_block_exclusive_scan<GB_THREADS>(local, &all, scan_smem);
    for (int i = 0; i < per; ++i) {
        const int b = threadIdx.x * per + i;
        if (b < P) {
            lstart[b] = run;
            run += lcnt[b];
            gstart[b] = gofs[static_cast<int64_t>(tile) * P + b];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        if (keep[c]) {
            const uint32_t b = pos[c] >> 16;
            const uint32_t q = lstart[b] + (pos[c] & 0xffffu);
            lbucket[q] = static_cast<uint16_t>(b);
#pragma unroll
            for (int x = 0; x < VECS; ++x) stage[q * VECS + x] = r[c].v[x];
        }
    }
    __syncthreads();
    const uint32_t count = all;                      // rows of this tile that pass the filter
    uint4 *out = reinterpret_cast<uint4 *>(recs);
    for (uint32_t e = threadIdx.x; e < count * VECS; e += GB_THREADS) {
        const uint32_t q = e / VECS, x = e % VECS;
        const uint32_t b = lbucket[q];
        out[(static_cast<int64_t>(gstart[b]) + (q - lstart[b])) * VECS + x] = stage[e];
    }
}

// Which scatter: "direct" (records written from registers) or "staged" (LDS,
// contiguous runs).  GQ_GROUPBY_SCATTER overrides the default.
bool gb_staged()
{
    static const bool v = [] {
        const char *e = getenv("GQ_GROUPBY_SCATTER");
        return !(e && strcmp(e, "direct") == 0);
    }();
    return v;
}

int gb_items(bool k64, bool k32)
{
    if (!gb_staged()) return GB_ITEMS;
    return (k64 && k32) ? GB_STAGED_ITEMS / 2 : GB_STAGED_ITEMS;
}

template <bool K64, bool K32>
struct bucket_slots {
    static constexpr int value = K64 ? 3072 : 4096;
};

template <bool K64, bool K32>
__global__ __launch_bounds__(GB_BUCKET_THREADS) void gb_bucket_kernel(const gb_rec<K64, K32> *__restrict__ recs,
                                                                      const uint32_t *__restrict__ start,
                                                                      int64_t rev_scale,
                                                                      gtable g, gq_groups out, uint32_t *status)
{
    constexpr int SLOTS = bucket_slots<K64, K32>::value;
    __shared__ lds_table<SLOTS, K64, K32> T;
    __shared__ uint32_t scan_smem[GB_BUCKET_THREADS / 64];
    __shared__ unsigned long long s_base;
    const int b = static_cast<int>(blockIdx.x);
    const int64_t r0 = start[b], r1 = start[b + 1];
    lds_init(T);
    __syncthreads();
    for (int64_t i0 = r0; i0 < r1; i0 += GB_BUCKET_THREADS) {
        const int64_t i = i0 + threadIdx.x;
        const bool active = i < r1;
        int64_t k64 = 0, q = 0;
        int32_t k32 = 0;
        gq_i128 rev{0, 0};
        if (active) {
            int64_t price, disc;
            read_rec<K64, K32>(recs, i, k64, k32, q, price, disc);
            rev = gq_revenue(price, rev_scale, disc);
        }
        const uint64_t h = gb_hash(k64, k32);
        const int s = lds_find(T, active, h, k64, k32);
        if (active && s >= 0) lds_add(T, s, 1u, static_cast<uint64_t>(q), rev);
        const bool spill = active && s < 0;
        const int64_t gs = g_find<K64, K32>(g, spill, h, k64, k32, status);
        if (spill && gs >= 0) g_add(g, gs, 1u, static_cast<uint64_t>(q), rev);
    }
    __syncthreads();
    // emit: each thread owns SLOTS / GB_BUCKET_THREADS consecutive slots
    constexpr int PER = SLOTS / GB_BUCKET_THREADS;
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) mine += T.state[threadIdx.x * PER + i] == 2u ? 1u : 0u;
    uint32_t total;
    uint32_t pre = gq_block_exclusive_scan<GB_BUCKET_THREADS>(mine, &total, scan_smem);
    if (threadIdx.x == 0)
        s_base = total ? atomicAdd(reinterpret_cast<unsigned long long *>(out.n_groups),
                                   static_cast<unsigned long long>(total))
                       : 0ull;
    __syncthreads();
    int64_t idx = static_cast<int64_t>(s_base) + pre;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int s = threadIdx.x * PER + i;
        if (T.state[s] == 2u) {
            emit_group(out, idx, K64 ? T.k64[s] : 0, K32 ? T.k32[s] : 0, T.cnt[s], T.sq[s], T.lo[s], T.hi[s],
                       status);
            ++idx;
        }
    }
}

// ------------------------------------------------------------------ host
uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct gb_plan {
    bool small;
    int log2p;
    int items;              // rows per thread of a hist/scatter tile
    int64_t ntiles;
    uint64_t gslots;
};

gb_plan make_plan(int64_t n, int64_t max_groups, bool k64, bool k32)
{
    gb_plan pl{};
    pl.small = max_groups <= GB_SMALL_GROUPS;
    pl.gslots = next_pow2(static_cast<uint64_t>(max_groups > 32 ? 2 * max_groups : 64));
    pl.items = gb_items(k64, k32);
    const int64_t tile = static_cast<int64_t>(GB_THREADS) * pl.items;
    pl.ntiles = n > 0 ? (n + tile - 1) / tile : 1;
    if (!pl.small) {
        const int64_t per_bucket = (k64 ? 3072 : 4096) / 2;
        const uint64_t want = static_cast<uint64_t>((max_groups + per_bucket - 1) / per_bucket);
        int l = 1;
        while ((1ull << l) < want && l < GB_MAX_LOG2P) ++l;
        pl.log2p = l;
    }
    return pl;
}

struct gb_ws {
    gtable g;
    uint32_t *hist;
    uint32_t *start;
    void *scan_ws;
    void *recs;             // partitioned rows, 32- or 64-byte records
    size_t zero_bytes;      // prefix of the workspace to clear (the table)
};

gb_ws gb_layout(gq_carver &c, const gb_plan &pl, int64_t n, bool k64, bool k32)
{
    gb_ws w{};
    const size_t S = pl.gslots;
    w.g.state = c.take<uint32_t>(S);
    w.g.k64 = c.take<int64_t>(k64 ? S : 1);
    w.g.k32 = c.take<int32_t>(k32 ? S : 1);
    w.g.cnt = c.take<uint64_t>(S);
    w.g.sq = c.take<uint64_t>(S);
    w.g.lo = c.take<uint64_t>(S);
    w.g.hi = c.take<int64_t>(S);
    w.g.mask = S - 1;
    w.zero_bytes = c.off;
    if (!pl.small) {
        const int64_t cells = pl.ntiles << pl.log2p;
        w.hist = c.take<uint32_t>(static_cast<size_t>(cells));
        w.start = c.take<uint32_t>((size_t(1) << pl.log2p) + 1);
        w.scan_ws = c.take<char>(gq_tile_offsets_workspace(pl.ntiles, 1 << pl.log2p));
        const size_t rows = static_cast<size_t>(n > 0 ? n : 1);
        w.recs = c.take<char>(rows * ((k64 && k32) ? 64 : 32));
    }
    return w;
}

template <bool K64, bool K32>
gq_status run_groupby(gq_ctx *ctx, const gb_args &a, const gb_plan &pl, const gb_ws &w, const gq_groups &out,
                      hipStream_t s)
{
    const uint32_t emit_blocks =
        static_cast<uint32_t>(std::min<uint64_t>((pl.gslots + 255) / 256, 4096));
    if (pl.small) {
        int64_t tiles = pl.ntiles;
        int64_t blocks = static_cast<int64_t>(ctx->num_cus) * 2;
        if (blocks > tiles) blocks = tiles;
        if (blocks < 1) blocks = 1;
        GQ_TRY(gq_launch(ctx, "gq_groupby_local", gb_small_kernel<K64, K32>, dim3(static_cast<uint32_t>(blocks)),
                         dim3(GB_THREADS), 0, s, a, w.g, ctx->status_dev));
        return gq_launch(ctx, "gq_groupby_emit", gb_table_emit_kernel<K64, K32>, dim3(emit_blocks), dim3(256), 0, s,
                         w.g, out, ctx->status_dev);
    }
    const uint32_t grid = static_cast<uint32_t>(pl.ntiles);
    const int P = 1 << pl.log2p;
    GQ_TRY(gq_launch(ctx, "gq_groupby_hist", gb_hist_kernel<K64, K32>, dim3(grid), dim3(GB_THREADS), 0, s, a,
                     pl.log2p, pl.items, w.hist));
    GQ_TRY(gq_tile_offsets(ctx, w.hist, pl.ntiles, P, w.start, w.scan_ws, s, "gq_groupby_scan"));
    auto *recs = static_cast<gb_rec<K64, K32> *>(w.recs);
    if (pl.items == GB_ITEMS)
        GQ_TRY(gq_launch(ctx, "gq_groupby_scatter", gb_scatter_kernel<K64, K32>, dim3(grid), dim3(GB_THREADS), 0, s,
                         a, pl.log2p, static_cast<const uint32_t *>(w.hist), pl.ntiles, recs));
    else
        GQ_TRY(gq_launch(ctx, "gq_groupby_scatter", gb_scatter_staged_kernel<K64, K32>, dim3(grid), dim3(GB_THREADS),
                         0, s, a, pl.log2p, static_cast<const uint32_t *>(w.hist), pl.ntiles, recs));
    GQ_TRY(gq_launch(ctx, "gq_groupby_bucket", gb_bucket_kernel<K64, K32>, dim3(static_cast<uint32_t>(P)),
                     dim3(GB_BUCKET_THREADS), 0, s, static_cast<const gb_rec<K64, K32> *>(recs),
                     static_cast<const uint32_t *>(w.start), a.rev_scale, w.g, out, ctx->status_dev));
    return gq_launch(ctx, "gq_groupby_emit", gb_table_emit_kernel<K64, K32>, dim3(emit_blocks), dim3(256), 0, s, w.g,
                     out, ctx->status_dev);
}

}  // namespace

extern "C" {

size_t gq_groupby_workspace_bytes(int64_t n, int64_t max_groups, int has_key64, int has_key32)
{
    if (n < 0) n = 0;
    if (max_groups < 1) max_groups = 1;
    gb_plan pl = make_plan(n, max_groups, has_key64 != 0, has_key32 != 0);
    gq_carver c(nullptr);
    gb_layout(c, pl, n, has_key64 != 0, has_key32 != 0);
    return c.bytes();
}

gq_status gq_groupby_agg(gq_ctx *ctx, const gq_groupby_in *in, int64_t max_groups, const gq_groups *out, void *ws,
                         size_t ws_bytes, gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (!in || !out) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_groupby_agg: NULL input or output");
    const int64_t n = in->n;
    if (n < 0 || n > GQ_MAX_ROWS) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_groupby_agg: n=%lld", (long long)n);
    if (max_groups < 1 || max_groups > out->capacity)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_groupby_agg: max_groups %lld not in [1, capacity %lld]",
                       (long long)max_groups, (long long)out->capacity);
    const bool k64 = in->key64 != nullptr, k32 = in->key32 != nullptr;
    if (n > 0 && (!in->qty || !in->price || !in->disc))
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_groupby_agg: NULL value column");
    if (!out->count || !out->sum_qty || !out->sum_rev_lo || !out->sum_rev_hi || !out->avg_qty || !out->avg_rev ||
        !out->n_groups || (k64 && !out->key64) || (k32 && !out->key32))
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_groupby_agg: NULL output array");
    const size_t need = gq_groupby_workspace_bytes(n, max_groups, k64, k32);
    if (!ws || ws_bytes < need)
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_groupby_agg: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gb_plan pl = make_plan(n, max_groups, k64, k32);
    gq_carver c(ws);
    gb_ws w = gb_layout(c, pl, n, k64, k32);
    GQ_TRY(gq_zero(ctx, ws, w.zero_bytes / 4, s));
    GQ_TRY(gq_zero(ctx, out->n_groups, 2, s));
    gb_args a{n,       in->n_dev, in->rowid, in->key64,     in->key64_by_rowid, in->key32, in->key32_by_rowid,
              in->qty, in->price, in->disc,  in->rev_scale, in->filter,         in->filter_lo, in->filter_hi};
    if (k64 && k32) return run_groupby<true, true>(ctx, a, pl, w, *out, s);
    if (k64) return run_groupby<true, false>(ctx, a, pl, w, *out, s);
    if (k32) return run_groupby<false, true>(ctx, a, pl, w, *out, s);
    return run_groupby<false, false>(ctx, a, pl, w, *out, s);
}

}  // extern "C"
