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
//    tile offsets -> LDS-staged scatter of narrow 16- or 24-byte records),
//    P chosen so that a bucket's groups fit one LDS table; one workgroup per
//    bucket aggregates it in LDS and writes its groups out directly.  A
//    bucket whose keys overflow its LDS table sends the extra keys to a
//    global fallback table (correct, slower), compacted by the same finalize
//    kernel; rows too wide for a narrow record reach it through a side list.
//
// Table protocol (LDS and global alike): a per-slot state word 0 = empty,
// 1 = being claimed, 2 = key published.  A lane claims a slot with a CAS
// 0 -> 1, writes the key and publishes state 2; a lane that sees state 1
// retries the same slot on its next pass of a wave-uniform loop, so the
// claiming lane always finishes first.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "gq_device.h"
#include "gq_internal.h"
#include "gq_ops.h"

namespace {

constexpr int GB_THREADS = 256;
constexpr int GB_SMALL_SLOTS = 1024;
constexpr int64_t GB_SMALL_GROUPS = 512;
constexpr int GB_ITEMS = 16;
constexpr int GB_TILE = GB_THREADS * GB_ITEMS;       // rows per small-path pass
constexpr int GB_SMALL_BATCH = 8;                    // rows per thread whose loads overlap
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
// Every table has one key word per slot, claimed by a single
// compare-and-swap.  Without key64 it is the 32-bit key32 itself
// (LDS_EMPTY32 = empty), so a claim publishes the whole key at once.  With
// key64 it is the 64-bit key64 (LDS_EMPTY64 = empty); a composite key's key32
// sits in a second word (LDS_EMPTY32 until the claiming lane writes it), so a
// slot whose key64 matches and whose key32 is still empty is being claimed,
// and a lookup reads it again.  A row whose key part equals an empty marker
// never enters an LDS table: it goes to the global table, which has its own
// claiming state.
constexpr uint64_t LDS_EMPTY64 = 0x8000000000000000ull;
constexpr uint32_t LDS_EMPTY32 = 0x80000000u;

template <int SLOTS, bool K64, bool K32>
struct lds_table {
    alignas(16) std::conditional_t<K64, uint64_t, uint32_t> word[SLOTS];
    int32_t k32[(K64 && K32) ? SLOTS : 1];
    uint32_t cnt[SLOTS];
    uint64_t sq[SLOTS];
    uint64_t lo[SLOTS];
    int64_t hi[SLOTS];
};

template <int SLOTS, bool K64, bool K32>
GQ_DEV bool lds_occupied(const lds_table<SLOTS, K64, K32> &T, int s)
{
    if constexpr (K64) return T.word[s] != LDS_EMPTY64;
    else return T.word[s] != LDS_EMPTY32;
}

template <int SLOTS, bool K64, bool K32>
GQ_DEV int32_t lds_key32(const lds_table<SLOTS, K64, K32> &T, int s)
{
    if constexpr (K64) return K32 ? T.k32[s] : 0;
    else return static_cast<int32_t>(T.word[s]);
}

template <int SLOTS, bool K64, bool K32>
GQ_DEV int64_t lds_key64(const lds_table<SLOTS, K64, K32> &T, int s)
{
    if constexpr (K64) return static_cast<int64_t>(T.word[s]);
    else return 0;
}

template <int SLOTS>
GQ_DEV uint32_t lds_home(uint64_t h)
{
    // bits 8..39 of the hash, scaled to [0, SLOTS); the top bits pick buckets
    return static_cast<uint32_t>((static_cast<uint64_t>(static_cast<uint32_t>(h >> 8)) * SLOTS) >> 32);
}

// Slot s back to empty (its sums to zero).
template <int SLOTS, bool K64, bool K32>
GQ_DEV void lds_clear_slot(lds_table<SLOTS, K64, K32> &T, int s)
{
    if constexpr (K64) T.word[s] = LDS_EMPTY64;
    else T.word[s] = LDS_EMPTY32;
    if constexpr (K64 && K32) T.k32[s] = static_cast<int32_t>(LDS_EMPTY32);
    T.cnt[s] = 0;
    T.sq[s] = 0;
    T.lo[s] = 0;
    T.hi[s] = 0;
}

template <int SLOTS, bool K64, bool K32>
GQ_DEV void lds_init(lds_table<SLOTS, K64, K32> &T)
{
    for (int s = threadIdx.x; s < SLOTS; s += blockDim.x) {
        if constexpr (K64) T.word[s] = LDS_EMPTY64;
        else T.word[s] = LDS_EMPTY32;
        if constexpr (K64 && K32) T.k32[s] = static_cast<int32_t>(LDS_EMPTY32);
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
    if constexpr (!K64) {
        // Linear probing over groups of four slots.  A lookup reads its group
        // and the next one together (two 16-byte loads), looks for the key in
        // both, and a missing key claims the first empty slot of the first
        // group that has one with one compare-and-swap (re-reading from that
        // group if another lane took the slot first).  A key therefore sits
        // in the first group from its home group that had room when it
        // arrived, and slots never empty again, so a lookup may stop at the
        // first group with an empty slot.  The wave-uniform loop runs as long
        // as the longest chain of the wave; reading two groups at a time
        // makes a second round rare (about 1% of keys overflow their home
        // group at the tables' load, which would otherwise give most waves
        // a lane that needs one).
        if (static_cast<uint32_t>(k32) == LDS_EMPTY32) done = true;   // the marker: the global table takes the row
        const uint32_t want = static_cast<uint32_t>(k32);
        constexpr uint32_t NG = SLOTS / 4;
        constexpr int LIMIT = GB_LDS_PROBES / 4;      // groups from the home group a key may sit in
        uint32_t g = s >> 2;                          // probes = distance of g from the home group
        while (__any(!done)) {
            if (!done) {
                const uint32_t g2 = (g + 1 == NG) ? 0 : g + 1;
                const bool two = probes + 1 < LIMIT;      // g2 is within the limit too
                // each word is read whole, which is all the claim protocol
                // needs (a word only ever goes from empty to a key)
                typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                typedef const volatile __attribute__((address_space(3))) u32x4 lds_u32x4;
                const u32x4 wa = *(lds_u32x4 *)(&T.word[4 * g]);
                const u32x4 wb = *(lds_u32x4 *)(&T.word[4 * g2]);
                const uint32_t w[8] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w};
                int hit1 = -1, empty1 = -1, hit2 = -1, empty2 = -1;
#pragma unroll
                for (int i = 3; i >= 0; --i) {
                    if (w[i] == want) hit1 = i;
                    if (w[i] == LDS_EMPTY32) empty1 = i;
                    if (w[4 + i] == want) hit2 = i;
                    if (w[4 + i] == LDS_EMPTY32) empty2 = i;
                }
                if (!two) hit2 = empty2 = -1;
                if (hit1 >= 0) {
                    found = static_cast<int>(4 * g) + hit1;
                    done = true;
                } else if (empty1 >= 0) {
                    const uint32_t prev = atomicCAS(&T.word[4 * g + empty1], LDS_EMPTY32, want);
                    if (prev == LDS_EMPTY32 || prev == want) {  // claimed, or the key arrived there meanwhile
                        found = static_cast<int>(4 * g) + empty1;
                        done = true;
                    }                                         // else: the slot went to another key; read again
                } else if (hit2 >= 0) {                       // the first group is full
                    found = static_cast<int>(4 * g2) + hit2;
                    done = true;
                } else if (empty2 >= 0) {
                    const uint32_t prev = atomicCAS(&T.word[4 * g2 + empty2], LDS_EMPTY32, want);
                    if (prev == LDS_EMPTY32 || prev == want) {
                        found = static_cast<int>(4 * g2) + empty2;
                        done = true;
                    } else {                                  // read again from the second group
                        g = g2;
                        probes += 1;
                    }
                } else if ((probes += two ? 2 : 1) >= LIMIT) {
                    done = true;                              // every group within the limit is full
                } else {
                    const uint32_t last = two ? g2 : g;
                    g = (last + 1 == NG) ? 0 : last + 1;
                }
            }
        }
    } else {
        // The same groups of four slots for tables keyed by key64: the four
        // key64 words (and key32 words) of a group are read together; a slot
        // with this key64 and an empty key32 is being claimed, so the group
        // is read again; with no match and no claim in progress the first
        // empty slot is claimed with one compare-and-swap of its key64 word,
        // and the claiming lane then writes the key32 word.
        if (K64 && (static_cast<uint64_t>(k64) == LDS_EMPTY64 ||
                    (K32 && static_cast<uint32_t>(k32) == LDS_EMPTY32)))
            done = true;                             // a marker value: the global table takes the row
        uint32_t g = s >> 2;
        while (__any(!done)) {
            if (!done) {
                unsigned long long *gp = reinterpret_cast<unsigned long long *>(&T.word[4 * g]);
                unsigned long long w[4];
                uint32_t x[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = __hip_atomic_load(gp + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    x[i] = K32 ? __hip_atomic_load(reinterpret_cast<uint32_t *>(&T.k32[4 * g + i]), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP)
                               : 0u;
                const unsigned long long want = static_cast<unsigned long long>(k64);
                int hit = -1, empty = -1;
                bool claiming = false;
#pragma unroll
                for (int i = 3; i >= 0; --i) {
                    if (w[i] == want) {
                        if (!K32 || x[i] == static_cast<uint32_t>(k32)) hit = i;
                        else if (x[i] == LDS_EMPTY32) claiming = true;
                    }
                    if (w[i] == LDS_EMPTY64) empty = i;
                }
                if (hit >= 0) {
                    found = static_cast<int>(4 * g) + hit;
                    done = true;
                } else if (claiming) {
                    // read the group again on the next pass
                } else if (empty >= 0) {
                    const int sl = static_cast<int>(4 * g) + empty;
                    if (atomicCAS(gp + empty, static_cast<unsigned long long>(LDS_EMPTY64), want) == LDS_EMPTY64) {
                        if (K32)
                            __hip_atomic_store(reinterpret_cast<uint32_t *>(&T.k32[sl]), static_cast<uint32_t>(k32),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        found = sl;
                        done = true;
                    }                                         // else: taken meanwhile; read again
                } else if (++probes >= GB_LDS_PROBES / 4) {
                    done = true;
                } else {
                    g = (g + 1 == SLOTS / 4) ? 0 : g + 1;
                }
            }
        }
    }
    return found;
}

// Accumulate one narrow row into slot s with no returned values: the
// revenue's low 32 bits (unsigned) and high 32 bits (signed) go to separate
// 64-bit sums, lo[s] and hi[s], exact for up to 2^31 rows per slot
// (|sum of highs| <= 2^62, sum of lows < 2^63).  The value is
// hi[s] * 2^32 + lo[s]; lds_split_total() recombines it.  The LDS atomic
// unit bounds the bucket pass, so a zero high half issues no atomic.
template <int SLOTS, bool K64, bool K32>
GQ_DEV void lds_add_split(lds_table<SLOTS, K64, K32> &T, int s, int64_t qty, int64_t rev)
{
    atomicAdd(&T.cnt[s], 1u);
    atomicAdd(reinterpret_cast<unsigned long long *>(&T.sq[s]), static_cast<unsigned long long>(qty));
    atomicAdd(reinterpret_cast<unsigned long long *>(&T.lo[s]),
              static_cast<unsigned long long>(static_cast<uint32_t>(static_cast<uint64_t>(rev))));
    const int64_t high = rev >> 32;
    if (high) atomicAdd(reinterpret_cast<unsigned long long *>(&T.hi[s]), static_cast<unsigned long long>(high));
}

GQ_DEV gq_i128 lds_split_total(uint64_t lo_sum, int64_t hi_sum)
{
    const __int128 v = static_cast<__int128>(hi_sum) * (static_cast<__int128>(1) << 32) + static_cast<__int128>(lo_sum);
    gq_i128 r;
    r.lo = static_cast<uint64_t>(v);
    r.hi = static_cast<int64_t>(v >> 64);
    return r;
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
    uint32_t *used;         // groups claimed so far (0: the table's emit has nothing to write)
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
                // the claimer zeroes the sums: only the state words start cleared
                if (K64) __hip_atomic_store(&g.k64[s], k64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (K32) __hip_atomic_store(&g.k32[s], k32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&g.cnt[s], uint64_t{0}, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&g.sq[s], uint64_t{0}, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&g.lo[s], uint64_t{0}, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&g.hi[s], int64_t{0}, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&g.state[s], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                atomicAdd(g.used, 1u);
                found = static_cast<int64_t>(s);
                done = true;
            } else if (st >= 2u) {                      // published (2) or taken (3)
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

// Find-only lookup in the global table (wave-uniform loop); -1 if absent.
template <bool K64, bool K32>
GQ_DEV int64_t g_lookup(const gtable &g, bool active, uint64_t h, int64_t k64, int32_t k32)
{
    uint64_t s = h & g.mask;
    uint64_t probes = 0;
    int64_t found = -1;
    bool done = !active;
    while (__any(!done)) {
        if (!done) {
            const uint32_t st = __hip_atomic_load(&g.state[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (st == 0u) {
                done = true;
            } else if (st >= 2u) {
                const bool eq =
                    (!K64 || __hip_atomic_load(&g.k64[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == k64) &&
                    (!K32 || __hip_atomic_load(&g.k32[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == k32);
                if (eq) {
                    found = static_cast<int64_t>(s);
                    done = true;
                } else if (++probes > g.mask) {
                    done = true;
                } else {
                    s = (s + 1) & g.mask;
                }
            }
        }
    }
    return found;
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
        // groups of 8 rows per thread: row ids, then keys and values, all in
        // flight together before the LDS work
        for (int c0 = 0; c0 < GB_ITEMS; c0 += GB_SMALL_BATCH) {
            int64_t v[GB_SMALL_BATCH];
            bool act[GB_SMALL_BATCH];
#pragma unroll
            for (int c = 0; c < GB_SMALL_BATCH; ++c) {
                const int64_t j = j0 + (c0 + c) * GB_THREADS + threadIdx.x;
                act[c] = j < n;
                v[c] = act[c] ? value_row(a, j) : 0;
            }
            if (a.filter) {
#pragma unroll
                for (int c = 0; c < GB_SMALL_BATCH; ++c) act[c] = act[c] && row_pass(a, v[c]);
            }
            int64_t k64[GB_SMALL_BATCH], qv[GB_SMALL_BATCH], pv[GB_SMALL_BATCH], dv[GB_SMALL_BATCH];
            int32_t k32[GB_SMALL_BATCH];
#pragma unroll
            for (int c = 0; c < GB_SMALL_BATCH; ++c) {
                const int64_t j = j0 + (c0 + c) * GB_THREADS + threadIdx.x;
                k64[c] = qv[c] = pv[c] = dv[c] = 0;
                k32[c] = 0;
                if (act[c]) {
                    k64[c] = K64 ? a.key64[a.key64_by_rowid ? v[c] : j] : 0;
                    k32[c] = K32 ? a.key32[a.key32_by_rowid ? v[c] : j] : 0;
                    qv[c] = a.qty[v[c]];
                    pv[c] = a.price[v[c]];
                    dv[c] = a.disc[v[c]];
                }
            }
#pragma unroll
            for (int c = 0; c < GB_SMALL_BATCH; ++c) {
                const gq_i128 rev = gq_revenue(pv[c], a.rev_scale, dv[c]);
                const uint64_t h = gb_hash(k64[c], k32[c]);
                const int s = lds_find(T, act[c], h, k64[c], k32[c]);
                if (act[c] && s >= 0) lds_add(T, s, 1u, static_cast<uint64_t>(qv[c]), rev);
                const bool spill = act[c] && s < 0;
                const int64_t gs = g_find<K64, K32>(g, spill, h, k64[c], k32[c], status);
                if (spill && gs >= 0) g_add(g, gs, 1u, static_cast<uint64_t>(qv[c]), rev);
            }
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < GB_SMALL_SLOTS; s += GB_THREADS) {
        const bool occ = lds_occupied(T, s);
        const int64_t k64 = occ ? lds_key64(T, s) : 0;
        const int32_t k32 = occ ? lds_key32(T, s) : 0;
        const int64_t gs = g_find<K64, K32>(g, occ, gb_hash(k64, k32), k64, k32, status);
        if (occ && gs >= 0) {
            gq_i128 rv;
            rv.lo = T.lo[s];
            rv.hi = T.hi[s];
            g_add(g, gs, T.cnt[s], T.sq[s], rv);
        }
    }
}

// Compact the occupied (state 2) slots of a global table into the output.
// Workgroup w owns one contiguous range of slots: it counts them, takes its
// output range with one atomic on the group counter (many atomics on one
// address serialize), then writes its groups in slot order.
template <bool K64, bool K32>
__global__ __launch_bounds__(256) void gb_table_emit_kernel(gtable g, gq_groups out, uint32_t *status)
{
    __shared__ uint32_t scan_smem[256 / 64];
    __shared__ unsigned long long s_base;
    if (*g.used == 0u) return;                       // nothing was claimed: no slot to scan
    const uint64_t slots = g.mask + 1;
    const uint64_t per = (slots + gridDim.x - 1) / gridDim.x;
    const uint64_t s0 = static_cast<uint64_t>(blockIdx.x) * per;
    const uint64_t s1 = s0 + per < slots ? s0 + per : slots;
    uint32_t mine = 0;
    for (uint64_t s = s0 + threadIdx.x; s < s1; s += 256) mine += g.state[s] == 2u ? 1u : 0u;
    uint32_t total;
    (void)gq_block_exclusive_scan<256>(mine, &total, scan_smem);
    if (total == 0) return;                          // same value for the whole workgroup
    if (threadIdx.x == 0)
        s_base = atomicAdd(reinterpret_cast<unsigned long long *>(out.n_groups),
                           static_cast<unsigned long long>(total));
    __syncthreads();
    int64_t idx = static_cast<int64_t>(s_base);
    for (uint64_t b = s0; b < s1; b += 256) {
        const uint64_t s = b + threadIdx.x;
        const bool occ = s < s1 && g.state[s] == 2u;
        uint32_t step;
        const uint32_t pre = gq_block_exclusive_scan<256>(occ ? 1u : 0u, &step, scan_smem);
        if (occ)
            emit_group(out, idx + pre, K64 ? g.k64[s] : 0, K32 ? g.k32[s] : 0, g.cnt[s], g.sq[s], g.lo[s], g.hi[s],
                       status);
        idx += step;
    }
}

// -------------------------------------------------------------- large path
//
// Rows are hash-partitioned by key into P buckets (any P in [2, GB_MAX_P]:
// the high 32 hash bits scaled to P), then one workgroup per bucket
// aggregates it in an LDS table.  A partitioned row is a narrow record of
// 8-byte words holding the key, qty as int32 and the revenue
// price * (rev_scale - disc) as int64:
//   key32 only       2 words  {k32 | qty32, rev64}
//   key64 (+ key32)  3 words  {k64, k32 | qty32, rev64}
// A row whose qty or revenue needs more bits (a wide row) is written with
// qty 0 and revenue 0, so it still counts one row in its bucket, and its row
// index goes to a side list.  A side kernel adds the full values of those
// rows to the global table with a count of 0; a bucket whose LDS group also
// has an entry there folds it in when it writes the group out and marks the
// entry taken (state 3).  With no wide rows the side list stays empty.
constexpr int GB_MAX_P = 1024;                      // buckets of the tile-staged scatter
constexpr int GB_MAX_P_WIDE = 8192;                 // buckets of the two-level scatter
constexpr int64_t GB_CUS = 256;                     // compute units of the MI355X
// Records per thread of a bucket-pass step (loaded one step ahead): four
// 16-byte records, or two of the wider key64 records, which keeps a
// 1024-thread workgroup's threads within their 128 registers (with four,
// the composite-key form spilled 14 registers to scratch).
template <bool K64>
struct bucket_items {
    static constexpr int value = K64 ? 2 : 4;
};
constexpr int GB_COMBINE_LANES = 8;                 // lanes on one slot above which a wave sums them first

template <bool K64, bool K32>
struct gb_fmt {
    static constexpr int WORDS = K64 ? 3 : 2;
    static constexpr int ITEMS = 8;                      // rows per thread of a hist/scatter tile
    static constexpr int TILE = GB_THREADS * ITEMS;
};

GQ_DEV uint32_t gb_bucket(uint64_t h, int P)
{
    return static_cast<uint32_t>(((h >> 32) * static_cast<uint64_t>(P)) >> 32);
}

GQ_DEV uint64_t pack2(uint32_t lo, uint32_t hi) { return (static_cast<uint64_t>(hi) << 32) | lo; }

GQ_DEV bool is_narrow(int64_t qty, const gq_i128 &rev)
{
    return qty == static_cast<int64_t>(static_cast<int32_t>(qty)) &&
           rev.hi == (static_cast<int64_t>(rev.lo) >> 63);
}

template <bool K64, bool K32>
GQ_DEV void make_words(uint64_t *w, int64_t k64, int32_t k32, int32_t q32, int64_t rev)
{
    if constexpr (!K64) {
        w[0] = pack2(static_cast<uint32_t>(k32), static_cast<uint32_t>(q32));
        w[1] = static_cast<uint64_t>(rev);
    } else {
        w[0] = static_cast<uint64_t>(k64);
        w[1] = pack2(K32 ? static_cast<uint32_t>(k32) : 0u, static_cast<uint32_t>(q32));
        w[2] = static_cast<uint64_t>(rev);
    }
}

template <bool K64, bool K32>
GQ_DEV void read_words(const uint64_t *__restrict__ recs, int64_t i, int64_t &k64, int32_t &k32, int64_t &qty,
                       int64_t &rev)
{
    if constexpr (!K64) {
        const uint4 v = reinterpret_cast<const uint4 *>(recs)[i];
        k64 = 0;
        k32 = static_cast<int32_t>(v.x);
        qty = static_cast<int32_t>(v.y);
        rev = static_cast<int64_t>(pack2(v.z, v.w));
    } else {
        const uint64_t *p = recs + i * 3;
        const uint64_t b = p[1];
        k64 = static_cast<int64_t>(p[0]);
        k32 = K32 ? static_cast<int32_t>(static_cast<uint32_t>(b)) : 0;
        qty = static_cast<int32_t>(static_cast<uint32_t>(b >> 32));
        rev = static_cast<int64_t>(p[2]);
    }
}

// The key of a record held in registers (the word layout of make_words).
template <bool K64, bool K32>
GQ_DEV void key_of_words(const uint64_t *w, int64_t &k64, int32_t &k32)
{
    if constexpr (!K64) {
        k64 = 0;
        k32 = static_cast<int32_t>(static_cast<uint32_t>(w[0]));
    } else {
        k64 = static_cast<int64_t>(w[0]);
        k32 = K32 ? static_cast<int32_t>(static_cast<uint32_t>(w[1])) : 0;
    }
}

template <bool K64, bool K32>
GQ_DEV void load_key(const gb_args &a, int64_t j, int64_t &k64, int32_t &k32)
{
    int64_t v = j;
    if (a.rowid && ((K64 && a.key64_by_rowid) || (K32 && a.key32_by_rowid))) v = a.rowid[j];
    k64 = K64 ? a.key64[a.key64_by_rowid ? v : j] : 0;
    k32 = K32 ? a.key32[a.key32_by_rowid ? v : j] : 0;
}

// LDS histogram of one chunk of rows (chunk_rows rows from chunk * chunk_rows),
// written as the chunk's row hist[chunk * P + b].
template <bool K64, bool K32, int PMAX>
__global__ __launch_bounds__(GB_THREADS) void gb_hist_kernel(gb_args a, int P, int64_t chunk_rows,
                                                             uint32_t *__restrict__ hist)
{
    constexpr int ITEMS = gb_fmt<K64, K32>::ITEMS;
    constexpr int TILE = gb_fmt<K64, K32>::TILE;
    __shared__ uint32_t h[PMAX];
    for (int i = threadIdx.x; i < P; i += GB_THREADS) h[i] = 0;
    __syncthreads();
    const int64_t n = eff_n(a.n_bound, a.n_dev);
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * chunk_rows;
    if (c0 >= n) return;                                   // past the row count: no counts (the scan skips it)
    const int64_t c1 = c0 + chunk_rows < n ? c0 + chunk_rows : n;
    // a tile's keys are loaded together, and the next tile's while this
    // tile's rows are counted (the row id is read only to filter)
    bool nv[ITEMS];
    int64_t nk64[ITEMS];
    int32_t nk32[ITEMS];
    auto load_tile = [&](int64_t base) {
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {
            const int64_t j = base + c * GB_THREADS + threadIdx.x;
            nv[c] = j < c1 && (!a.filter || row_pass(a, value_row(a, j)));
            nk64[c] = 0;
            nk32[c] = 0;
            if (nv[c]) load_key<K64, K32>(a, j, nk64[c], nk32[c]);
        }
    };
    load_tile(c0);
    for (int64_t base = c0; base < c1; base += TILE) {
        bool v[ITEMS];
        int64_t k64[ITEMS];
        int32_t k32[ITEMS];
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {
            v[c] = nv[c];
            k64[c] = nk64[c];
            k32[c] = nk32[c];
        }
        if (base + TILE < c1) load_tile(base + TILE);
#pragma unroll
        for (int c = 0; c < ITEMS; ++c)
            if (v[c]) atomicAdd(&h[gb_bucket(gb_hash(k64[c], k32[c]), P)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < P; b += GB_THREADS) hist[static_cast<int64_t>(blockIdx.x) * P + b] = h[b];
}

// Scatter of 2048-row tiles: rank each row inside its bucket with an LDS
// atomic (the order inside a bucket does not matter to sums), stage the
// records in LDS in bucket order, then write them out as contiguous runs
// starting at the tile's offset gofs[t * P + b] in each bucket.
// Persistent: XCD x (workgroups b with b mod 8 = x) takes one contiguous
// eighth of the tiles, in order, from its own counter (xctr[32 x], one
// 128-byte line per counter), so a
// bucket's runs from neighbouring tiles reach one L2 close together in time
// and leave it as whole lines.  The row ids, directly indexed keys and bucket
// offsets of a workgroup's next tile are loaded while it scatters the current
// one; the barriers order LDS only, so those loads stay in flight.
template <bool K64, bool K32>
__global__ __launch_bounds__(GB_THREADS) void gb_scatter_kernel(gb_args a, int P, const uint32_t *__restrict__ gofs,
                                                                uint64_t *__restrict__ recs,
                                                                uint32_t *__restrict__ side, uint32_t *side_cnt,
                                                                uint32_t *xctr)
{
    constexpr int ITEMS = gb_fmt<K64, K32>::ITEMS;
    constexpr int TILE = gb_fmt<K64, K32>::TILE;
    constexpr int W = gb_fmt<K64, K32>::WORDS;
    constexpr int GPER = GB_MAX_P / GB_THREADS;
    __shared__ uint32_t s_next;
    __shared__ uint32_t lpos[GB_MAX_P];          // counts -> local starts -> (global - local) starts
    __shared__ uint32_t scan_smem[GB_THREADS / 64];
    __shared__ uint16_t lbucket[TILE];
    __shared__ uint64_t stage[TILE * W];
    const int64_t n = eff_n(a.n_bound, a.n_dev);
    const int64_t nt = (n + TILE - 1) / TILE;
    const uint32_t xcd = blockIdx.x % GQ_NUM_XCD;
    const int64_t r0 = nt * xcd / GQ_NUM_XCD, r1 = nt * (xcd + 1) / GQ_NUM_XCD;
    auto prefetch = [&](int64_t t, int32_t *pv, int64_t *pk64, int32_t *pk32, uint32_t *pgo) {
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {
            const int64_t j = t * TILE + c * GB_THREADS + threadIdx.x;
            pv[c] = 0;
            pk64[c] = 0;
            pk32[c] = 0;
            if (t < r1 && j < n) {
                pv[c] = a.rowid ? __builtin_nontemporal_load(&a.rowid[j]) : static_cast<int32_t>(j);
                if (K64 && !a.key64_by_rowid) pk64[c] = __builtin_nontemporal_load(&a.key64[j]);
                if (K32 && !a.key32_by_rowid) pk32[c] = __builtin_nontemporal_load(&a.key32[j]);
            }
        }
#pragma unroll
        for (int i = 0; i < GPER; ++i) {
            const int b = threadIdx.x + i * GB_THREADS;
            pgo[i] = (t < r1 && b < P) ? gofs[t * P + b] : 0u;
        }
    };
    if (threadIdx.x == 0) s_next = atomicAdd(&xctr[32 * xcd], 1u);
    __syncthreads();
    int64_t t = r0 + static_cast<int64_t>(gq_uniform(s_next));
    int32_t v[ITEMS];
    int64_t k64[ITEMS];
    int32_t k32[ITEMS];
    uint32_t go[GPER];
    prefetch(t, v, k64, k32, go);
    while (t < r1) {
        gq_lds_barrier();                               // opens each pass (thread-0 work never merges across passes)
        const int64_t base = t * TILE;
        uint32_t nxt = 0;
        if (threadIdx.x == 0) nxt = atomicAdd(&xctr[32 * xcd], 1u);   // the next tile, dequeued early
        // every thread has read s_next (the current tile) and finished the
        // last tile's LDS reads
        gq_lds_barrier();
        if (threadIdx.x == 0) s_next = nxt;
        for (int b = threadIdx.x; b < P; b += GB_THREADS) lpos[b] = 0;
        int64_t qv[ITEMS], pv[ITEMS], dv[ITEMS];
        bool keep[ITEMS];
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {               // this tile's value gathers
            const int64_t j = base + c * GB_THREADS + threadIdx.x;
            keep[c] = j < n && (!a.filter || row_pass(a, v[c]));
            qv[c] = pv[c] = dv[c] = 0;
            if (keep[c]) {
                if (K64 && a.key64_by_rowid) k64[c] = a.key64[v[c]];
                if (K32 && a.key32_by_rowid) k32[c] = a.key32[v[c]];
                qv[c] = __builtin_nontemporal_load(&a.qty[v[c]]);
                pv[c] = __builtin_nontemporal_load(&a.price[v[c]]);
                dv[c] = __builtin_nontemporal_load(&a.disc[v[c]]);
            }
        }
        int32_t nv[ITEMS];
        int64_t nk64[ITEMS];
        int32_t nk32[ITEMS];
        uint32_t ngo[GPER];
        gq_lds_barrier();                               // lpos cleared; s_next set
        const int64_t tn = r0 + static_cast<int64_t>(gq_uniform(s_next));
        prefetch(tn, nv, nk64, nk32, ngo);              // the next tile: in flight meanwhile
        uint64_t w[ITEMS][W];
        uint32_t pos[ITEMS];
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {
            if (keep[c]) {
                const int64_t j = base + c * GB_THREADS + threadIdx.x;
                const gq_i128 rev = gq_revenue(pv[c], a.rev_scale, dv[c]);
                const bool nar = is_narrow(qv[c], rev);
                if (!nar) side[atomicAdd(side_cnt, 1u)] = static_cast<uint32_t>(j);
                make_words<K64, K32>(w[c], k64[c], k32[c], nar ? static_cast<int32_t>(qv[c]) : 0,
                                     nar ? static_cast<int64_t>(rev.lo) : 0);
                const uint32_t b = gb_bucket(gb_hash(k64[c], k32[c]), P);
                pos[c] = (b << 16) | atomicAdd(&lpos[b], 1u);
            }
        }
        gq_lds_barrier();
        const int per = (P + GB_THREADS - 1) / GB_THREADS;
        uint32_t local = 0;
        for (int i = 0; i < per; ++i) {
            const int b = threadIdx.x * per + i;
            if (b < P) local += lpos[b];
        }
        uint32_t all;
        uint32_t run = gq_block_exclusive_scan_lds<GB_THREADS>(local, &all, scan_smem);
        for (int i = 0; i < per; ++i) {
            const int b = threadIdx.x * per + i;
            if (b < P) {
                const uint32_t c = lpos[b];
                lpos[b] = run;
                run += c;
            }
        }
        gq_lds_barrier();
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {
            if (keep[c]) {
                const uint32_t b = pos[c] >> 16;
                const uint32_t q = lpos[b] + (pos[c] & 0xffffu);
                lbucket[q] = static_cast<uint16_t>(b);
#pragma unroll
                for (int x = 0; x < W; ++x) stage[q * W + x] = w[c][x];
            }
        }
        gq_lds_barrier();
#pragma unroll
        for (int i = 0; i < GPER; ++i) {
            const int b = threadIdx.x + i * GB_THREADS;
            if (b < P) lpos[b] = go[i] - lpos[b];
        }
        gq_lds_barrier();
        const uint32_t words = all * W;                  // rows of this tile that pass the filter
        for (uint32_t e = threadIdx.x; e < words; e += GB_THREADS) {
            const uint32_t q = e / W, x = e - q * W;
            const uint32_t row = q + lpos[lbucket[q]];  // global row position in the bucket array
            recs[static_cast<int64_t>(row) * W + x] = stage[e];
        }
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {
            v[c] = nv[c];
            k64[c] = nk64[c];
            k32[c] = nk32[c];
        }
#pragma unroll
        for (int i = 0; i < GPER; ++i) go[i] = ngo[i];
        t = tn;
    }
}

// Scatter of 16-byte records (tables without key64) by regions: workgroup r
// takes the r-th of gridDim.x contiguous ranges of hist chunks, and the
// region's share of each bucket is one contiguous stretch of the output that
// only this workgroup writes, front to back.  It therefore keeps the open end
// of every stretch in LDS and writes whole aligned 128-byte lines (eight
// records) only: per tile, each row takes the next place of its bucket with
// an LDS atomic; a line that the tile completes is written from the line
// buffer (its older records) and straight from the threads' registers (its
// new ones), all within one phase of the tile, so its pieces meet in L2 and
// leave it as one line; new records past the last complete line wait in the
// buffer.  Only the first and last line of a region's stretch in a bucket
// are written in part.  Row ids and direct keys are loaded two tiles ahead
// and the value gathers one tile ahead, so a single workgroup per CU keeps
// its loads in flight behind the LDS work (the barriers order LDS only).
constexpr int GL_THREADS = 512;
constexpr int GL_ITEMS = 8;
constexpr int GL_TILE = GL_THREADS * GL_ITEMS;      // rows per tile
constexpr int GL_LINE = 8;                          // records per written line (128 bytes)
constexpr int64_t GL_CHUNK_ROWS = 8 * GL_TILE;      // rows per hist chunk

template <bool K32>
__global__ __launch_bounds__(GL_THREADS) void gb_scatter_lines_kernel(gb_args a, int P, int64_t chunk_rows,
                                                                       const uint32_t *__restrict__ gofs,
                                                                       uint4 *__restrict__ recs,
                                                                       uint32_t *__restrict__ side, uint32_t *side_cnt)
{
    constexpr int GPER = GB_MAX_P / GL_THREADS;
    constexpr uint32_t LMASK = ~static_cast<uint32_t>(GL_LINE - 1);
    __shared__ uint4 lbuf[GB_MAX_P * GL_LINE];       // open line of each bucket, by position mod GL_LINE
    __shared__ uint32_t cnt[GB_MAX_P];               // this tile's rows per bucket
    __shared__ uint32_t cur[GB_MAX_P];               // output position of the bucket's next record
    __shared__ uint32_t lo[GB_MAX_P];                // first position held in the bucket's line buffer
    const int64_t n = eff_n(a.n_bound, a.n_dev);
    const int64_t nch = (n + chunk_rows - 1) / chunk_rows;
    const int64_t c0 = nch * blockIdx.x / gridDim.x, c1 = nch * (blockIdx.x + 1) / gridDim.x;
    if (c0 >= c1) return;                            // same for the whole workgroup
    const int64_t row0 = c0 * chunk_rows;
    const int64_t row1 = c1 * chunk_rows < n ? c1 * chunk_rows : n;
#pragma unroll
    for (int i = 0; i < GPER; ++i) {
        const int b = threadIdx.x + i * GL_THREADS;
        if (b < P) {
            const uint32_t g = gofs[c0 * P + b];
            cur[b] = g;
            lo[b] = g;
            cnt[b] = 0;
        }
    }
    auto load_ids = [&](int64_t base, int32_t *v, int32_t *k) {
#pragma unroll
        for (int c = 0; c < GL_ITEMS; ++c) {
            const int64_t j = base + c * GL_THREADS + threadIdx.x;
            v[c] = 0;
            k[c] = 0;
            if (j < row1) {
                v[c] = a.rowid ? __builtin_nontemporal_load(&a.rowid[j]) : static_cast<int32_t>(j);
                if (K32 && !a.key32_by_rowid) k[c] = __builtin_nontemporal_load(&a.key32[j]);
            }
        }
    };
    auto load_vals = [&](int64_t base, const int32_t *v, int32_t *k, int64_t *q, int64_t *p, int64_t *d,
                         bool *keep) {
#pragma unroll
        for (int c = 0; c < GL_ITEMS; ++c) {
            const int64_t j = base + c * GL_THREADS + threadIdx.x;
            keep[c] = j < row1 && (!a.filter || row_pass(a, v[c]));
            q[c] = p[c] = d[c] = 0;
            if (keep[c]) {
                if (K32 && a.key32_by_rowid) k[c] = a.key32[v[c]];
                q[c] = __builtin_nontemporal_load(&a.qty[v[c]]);
                p[c] = __builtin_nontemporal_load(&a.price[v[c]]);
                d[c] = __builtin_nontemporal_load(&a.disc[v[c]]);
            }
        }
    };
    int32_t v0[GL_ITEMS], k0[GL_ITEMS], v1[GL_ITEMS], k1[GL_ITEMS];
    int64_t q0[GL_ITEMS], p0[GL_ITEMS], d0[GL_ITEMS];
    bool keep0[GL_ITEMS];
    load_ids(row0, v0, k0);
    load_vals(row0, v0, k0, q0, p0, d0, keep0);
    load_ids(row0 + GL_TILE, v1, k1);
    for (int64_t base = row0; base < row1; base += GL_TILE) {
        int64_t q1[GL_ITEMS], p1[GL_ITEMS], d1[GL_ITEMS];
        bool keep1[GL_ITEMS];
        load_vals(base + GL_TILE, v1, k1, q1, p1, d1, keep1);      // the next tile's gathers
        int32_t v2[GL_ITEMS], k2[GL_ITEMS];
        load_ids(base + 2 * GL_TILE, v2, k2);                       // and the ids of the one after
        gq_lds_barrier();                                           // the last tile's write-out is done
#pragma unroll
        for (int i = 0; i < GPER; ++i) {
            const int b = threadIdx.x + i * GL_THREADS;
            if (b < P) {
                cur[b] += cnt[b];
                cnt[b] = 0;
            }
        }
        gq_lds_barrier();
        uint4 rec[GL_ITEMS];
        uint32_t bk[GL_ITEMS], rank[GL_ITEMS];
#pragma unroll
        for (int c = 0; c < GL_ITEMS; ++c) {
            if (keep0[c]) {
                const int64_t j = base + c * GL_THREADS + threadIdx.x;
                const gq_i128 rev = gq_revenue(p0[c], a.rev_scale, d0[c]);
                const bool nar = is_narrow(q0[c], rev);
                if (!nar) side[atomicAdd(side_cnt, 1u)] = static_cast<uint32_t>(j);
                const uint64_t r = nar ? rev.lo : 0ull;
                rec[c] = make_uint4(static_cast<uint32_t>(k0[c]), nar ? static_cast<uint32_t>(q0[c]) : 0u,
                                    static_cast<uint32_t>(r), static_cast<uint32_t>(r >> 32));
                bk[c] = gb_bucket(gb_hash(0, k0[c]), P);
                rank[c] = atomicAdd(&cnt[bk[c]], 1u);
            }
        }
        gq_lds_barrier();
        // a line that this tile completes: its older records leave the buffer
#pragma unroll
        for (int i = 0; i < GPER; ++i) {
            const int b = threadIdx.x + i * GL_THREADS;
            const uint32_t k = b < P ? cnt[b] : 0u;
            if (k) {
                const uint32_t g = cur[b];
                const uint32_t cut = (g + k) & LMASK;
                if ((g & LMASK) < cut) {
                    for (uint32_t x = lo[b]; x < g; ++x) recs[x] = lbuf[b * GL_LINE + (x & (GL_LINE - 1))];
                    lo[b] = cut;
                }
            }
        }
        gq_lds_barrier();                                           // the buffers are read
        // the new records: complete lines to the output, the rest to the buffer
#pragma unroll
        for (int c = 0; c < GL_ITEMS; ++c) {
            if (keep0[c]) {
                const uint32_t b = bk[c];
                const uint32_t g = cur[b];
                const uint32_t x = g + rank[c];
                const uint32_t cut = (g + cnt[b]) & LMASK;
                if (x < cut) recs[x] = rec[c];
                else lbuf[b * GL_LINE + (x & (GL_LINE - 1))] = rec[c];
            }
        }
#pragma unroll
        for (int c = 0; c < GL_ITEMS; ++c) {
            k0[c] = k1[c];
            q0[c] = q1[c];
            p0[c] = p1[c];
            d0[c] = d1[c];
            keep0[c] = keep1[c];
            v1[c] = v2[c];
            k1[c] = k2[c];
        }
    }
    gq_lds_barrier();
    // the open end of every stretch
#pragma unroll
    for (int i = 0; i < GPER; ++i) {
        const int b = threadIdx.x + i * GL_THREADS;
        if (b < P) {
            const uint32_t g = cur[b] + cnt[b];
            for (uint32_t x = lo[b]; x < g; ++x) recs[x] = lbuf[b * GL_LINE + (x & (GL_LINE - 1))];
        }
    }
}

// Full values of the wide rows into the global table (count 0: their rows
// were counted by their narrow records).
template <bool K64, bool K32>
__global__ __launch_bounds__(256) void gb_side_kernel(gb_args a, const uint32_t *__restrict__ side,
                                                      const uint32_t *side_cnt, gtable g, uint32_t *status)
{
    const uint32_t cnt = *side_cnt;
    for (uint32_t i0 = blockIdx.x * 256u; i0 < cnt; i0 += gridDim.x * 256u) {
        const uint32_t i = i0 + threadIdx.x;
        const bool active = i < cnt;
        gb_row<K64, K32> r{};
        if (active) r = load_row<K64, K32>(a, side[i]);
        const uint64_t h = gb_hash(r.k64, r.k32);
        const int64_t gs = g_find<K64, K32>(g, active, h, r.k64, r.k32, status);
        if (active && gs >= 0) g_add(g, gs, 0u, static_cast<uint64_t>(r.qty), r.rev);
    }
}

// Large fan-outs (P > GB_MAX_P buckets, up to GB_MAX_P_WIDE) in two levels,
// each a tile-staged scatter with runs long enough to fill cache lines:
//   level 1  the rows go to P1 = GB_P1 super-buckets (the scatter above, with
//            P1 buckets): super-bucket s = the buckets [s P2, (s + 1) P2) of
//            the full fan-out P = P1 P2, since floor(floor(x P1 P2) / P2) =
//            floor(x P1) for the scaled hash x in [0, 1);
//   level 2  each super-bucket's records are cut into tiles of GB_T2 records
//            (a tile never straddles two super-buckets), every tile is counted
//            by sub-bucket, a per-super-bucket column scan gives each (tile,
//            sub-bucket) run its place, and the tile is staged in LDS by
//            sub-bucket and written out as runs.
// The bucket pass then reads buckets b = s P2 + sub as usual.
constexpr int GB_P1 = 128;                          // super-buckets of level 1
constexpr int GB_T2 = 2048;                         // records per level-2 tile
constexpr int GB_MAX_P2 = GB_MAX_P_WIDE / GB_P1;    // 64

// Level-2 tiles of each super-bucket: tpre[s] = tiles before super-bucket s,
// tpre[P1] = all tiles.  One workgroup of 256 threads (P1 <= 256).
__global__ __launch_bounds__(256) void gb_tiles2_kernel(const uint32_t *__restrict__ startA, int P1,
                                                        uint32_t *__restrict__ tpre)
{
    __shared__ uint32_t scan_smem[256 / 64];
    const int sb = threadIdx.x;
    uint32_t nt = 0;
    if (sb < P1) nt = (startA[sb + 1] - startA[sb] + GB_T2 - 1) / GB_T2;
    uint32_t total;
    const uint32_t excl = gq_block_exclusive_scan<256>(nt, &total, scan_smem);
    if (sb < P1) tpre[sb] = excl;
    if (threadIdx.x == 0) tpre[P1] = total;
}

// The super-bucket of level-2 tile g: the last s with tpre[s] <= g.
GQ_DEV int gb_super_of(const uint32_t *tpre, int P1, uint32_t g)
{
    int lo = 0, hi = P1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tpre[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Per level-2 tile: its records counted by sub-bucket -> hist2[g * P2 + sub].
// Grid: an upper bound on the tile count; surplus workgroups exit.
template <bool K64, bool K32>
__global__ __launch_bounds__(GB_THREADS) void gb_hist2_kernel(const uint64_t *__restrict__ recs1,
                                                              const uint32_t *__restrict__ startA,
                                                              const uint32_t *__restrict__ tpre, int P1, int P,
                                                              int P2, uint32_t *__restrict__ hist2)
{
    __shared__ uint32_t h[GB_MAX_P2];
    const uint32_t g = blockIdx.x;
    if (g >= tpre[P1]) return;                          // same value for the whole workgroup
    for (int i = threadIdx.x; i < P2; i += GB_THREADS) h[i] = 0;
    __syncthreads();
    const int sb = gb_super_of(tpre, P1, g);
    const int64_t r0 = static_cast<int64_t>(startA[sb]) + static_cast<int64_t>(g - tpre[sb]) * GB_T2;
    const int64_t r1 = r0 + GB_T2 < static_cast<int64_t>(startA[sb + 1]) ? r0 + GB_T2 : startA[sb + 1];
    for (int64_t i = r0 + threadIdx.x; i < r1; i += GB_THREADS) {
        int64_t k64, q, rv;
        int32_t k32;
        read_words<K64, K32>(recs1, i, k64, k32, q, rv);
        const uint32_t b = gb_bucket(gb_hash(k64, k32), P);
        atomicAdd(&h[b - static_cast<uint32_t>(sb) * P2], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P2; i += GB_THREADS) hist2[static_cast<int64_t>(g) * P2 + i] = h[i];
}

// One workgroup per super-bucket s: the counts of its tiles become the output
// position of every (tile, sub-bucket) run (in place), and start[s P2 + sub]
// the start of every bucket (start[P] = all records).  Thread (q, col) sums,
// then writes, column col over the q-th quarter of s's tiles.
__global__ __launch_bounds__(256) void gb_scan2_kernel(uint32_t *__restrict__ hist2,
                                                       const uint32_t *__restrict__ startA,
                                                       const uint32_t *__restrict__ tpre, int P1, int P2,
                                                       uint32_t *__restrict__ start)
{
    __shared__ uint32_t part[4][GB_MAX_P2];
    __shared__ uint32_t colbase[GB_MAX_P2];
    const int sb = blockIdx.x;
    const int col = threadIdx.x & (GB_MAX_P2 - 1), q = threadIdx.x / GB_MAX_P2;
    const int64_t t0 = tpre[sb], nt = static_cast<int64_t>(tpre[sb + 1]) - t0;
    const int64_t a = t0 + nt * q / 4, b = t0 + nt * (q + 1) / 4;
    uint32_t sum = 0;
    if (col < P2) {
#pragma unroll 8
        for (int64_t t = a; t < b; ++t) sum += hist2[t * P2 + col];
    }
    part[q][col] = sum;
    __syncthreads();
    if (threadIdx.x < GB_MAX_P2) {                      // one wave: the columns' totals, scanned
        const uint32_t tot = col < P2 ? part[0][col] + part[1][col] + part[2][col] + part[3][col] : 0u;
        const uint32_t inc = gq_wave_inclusive_scan(tot);
        const uint32_t base = startA[sb] + inc - tot;
        colbase[col] = base;
        if (col < P2) start[sb * P2 + col] = base;
        if (sb == P1 - 1 && col == 0) start[P1 * P2] = startA[P1];
    }
    __syncthreads();
    if (col < P2) {
        uint32_t run = colbase[col];
        for (int p = 0; p < q; ++p) run += part[p][col];
        for (int64_t t = a; t < b; ++t) {
            const uint32_t c = hist2[t * P2 + col];
            hist2[t * P2 + col] = run;
            run += c;
        }
    }
}

// Per level-2 tile: its records ranked by sub-bucket (LDS atomics; the order
// inside a bucket does not matter to sums), staged in LDS in sub-bucket
// order and written out as runs at the positions the scan gave.
template <bool K64, bool K32>
__global__ __launch_bounds__(GB_THREADS) void gb_scatter2_kernel(const uint64_t *__restrict__ recs1,
                                                                 const uint32_t *__restrict__ startA,
                                                                 const uint32_t *__restrict__ tpre,
                                                                 const uint32_t *__restrict__ off2, int P1, int P,
                                                                 int P2, uint64_t *__restrict__ recs)
{
    constexpr int W = gb_fmt<K64, K32>::WORDS;
    constexpr int ITEMS = GB_T2 / GB_THREADS;
    __shared__ uint32_t cnt[GB_MAX_P2];
    __shared__ uint32_t lstart[GB_MAX_P2];
    __shared__ uint32_t delta[GB_MAX_P2];
    __shared__ uint8_t lsub[GB_T2];
    __shared__ uint64_t stage[GB_T2 * W];
    const uint32_t g = blockIdx.x;
    if (g >= tpre[P1]) return;                          // same value for the whole workgroup
    const int sb = gb_super_of(tpre, P1, g);
    const int64_t r0 = static_cast<int64_t>(startA[sb]) + static_cast<int64_t>(g - tpre[sb]) * GB_T2;
    const int64_t rem = static_cast<int64_t>(startA[sb + 1]) - r0;
    const int rows = static_cast<int>(rem < GB_T2 ? rem : GB_T2);
    for (int i = threadIdx.x; i < P2; i += GB_THREADS) cnt[i] = 0;
    uint64_t w[ITEMS][W];
    uint32_t pos[ITEMS];
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int i = c * GB_THREADS + threadIdx.x;
#pragma unroll
        for (int x = 0; x < W; ++x) w[c][x] = i < rows ? recs1[(r0 + i) * W + x] : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int i = c * GB_THREADS + threadIdx.x;
        if (i < rows) {
            int64_t k64;
            int32_t k32;
            key_of_words<K64, K32>(w[c], k64, k32);
            const uint32_t sub = gb_bucket(gb_hash(k64, k32), P) - static_cast<uint32_t>(sb) * P2;
            pos[c] = (sub << 16) | atomicAdd(&cnt[sub], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < GB_MAX_P2) {
        const uint32_t x = threadIdx.x < static_cast<uint32_t>(P2) ? cnt[threadIdx.x] : 0u;
        const uint32_t ex = gq_wave_inclusive_scan(x) - x;
        lstart[threadIdx.x] = ex;
        if (threadIdx.x < static_cast<uint32_t>(P2))
            delta[threadIdx.x] = off2[static_cast<int64_t>(g) * P2 + threadIdx.x] - ex;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < ITEMS; ++c) {
        const int i = c * GB_THREADS + threadIdx.x;
        if (i < rows) {
            const uint32_t sub = pos[c] >> 16;
            const uint32_t qd = lstart[sub] + (pos[c] & 0xffffu);
            lsub[qd] = static_cast<uint8_t>(sub);
#pragma unroll
            for (int x = 0; x < W; ++x) stage[qd * W + x] = w[c][x];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * W; e += GB_THREADS) {
        const int qd = e / W, x = e - qd * W;
        recs[(static_cast<int64_t>(qd) + delta[lsub[qd]]) * W + x] = stage[e];
    }
}

template <bool K64, bool K32>
struct bucket_slots {
    static constexpr int value = K64 ? 3072 : 4096;
};

// A partial group of one chunk of a split bucket (exact int128 revenue).
struct gb_part {
    int64_t k64;
    int32_t k32;
    uint32_t cnt;
    uint64_t sq;
    uint64_t lo;
    int64_t hi;
};

// Sums of several rows into slot s (the split form of lds_add_split).
template <int SLOTS, bool K64, bool K32>
GQ_DEV void lds_add_sums(lds_table<SLOTS, K64, K32> &T, int s, uint32_t cnt, uint64_t qty, uint64_t lo_sum,
                         int64_t hi_sum)
{
    atomicAdd(&T.cnt[s], cnt);
    atomicAdd(reinterpret_cast<unsigned long long *>(&T.sq[s]), static_cast<unsigned long long>(qty));
    atomicAdd(reinterpret_cast<unsigned long long *>(&T.lo[s]), static_cast<unsigned long long>(lo_sum));
    if (hi_sum) atomicAdd(reinterpret_cast<unsigned long long *>(&T.hi[s]), static_cast<unsigned long long>(hi_sum));
}

// Chunks of the bucket pass.  A bucket of at most chunk_rows rows is one
// chunk; a larger one (a bucket holding a heavy key) is cut into
// ceil(rows / chunk_rows) chunks, each aggregated by its own workgroup.
// cstart[b] = number of chunks before bucket b.  order[] lists the chunks in
// the order the bucket pass takes them: the chunks of split buckets first
// (the longest work, so none of it is left for the end), then the buckets of
// one chunk.  One workgroup of GB_BUCKET_THREADS threads; P <= GB_MAX_P_WIDE.
__global__ __launch_bounds__(GB_BUCKET_THREADS) void gb_chunks_kernel(const uint32_t *__restrict__ start, int P,
                                                                      int64_t chunk_rows, uint32_t *__restrict__ cstart,
                                                                      uint32_t *__restrict__ order,
                                                                      uint32_t *__restrict__ sfirst)
{
    __shared__ uint32_t scan_smem[GB_BUCKET_THREADS / 64];
    constexpr int PER = GB_MAX_P_WIDE / GB_BUCKET_THREADS;
    uint32_t nch[PER];
    uint32_t mine = 0, msplit = 0, mone = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = threadIdx.x * PER + i;
        nch[i] = 0;
        if (b < P) {
            const int64_t rows = static_cast<int64_t>(start[b + 1]) - static_cast<int64_t>(start[b]);
            nch[i] = rows > chunk_rows ? static_cast<uint32_t>((rows + chunk_rows - 1) / chunk_rows) : 1u;
        }
        mine += nch[i];
        msplit += nch[i] > 1 ? nch[i] : 0u;
        mone += nch[i] == 1 ? 1u : 0u;
    }
    uint32_t total, nsplit, none;
    uint32_t run = gq_block_exclusive_scan<GB_BUCKET_THREADS>(mine, &total, scan_smem);
    uint32_t srun = gq_block_exclusive_scan<GB_BUCKET_THREADS>(msplit, &nsplit, scan_smem);
    uint32_t orun = gq_block_exclusive_scan<GB_BUCKET_THREADS>(mone, &none, scan_smem);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = threadIdx.x * PER + i;
        if (b < P) {
            cstart[b] = run;
            if (nch[i] > 1) {
                for (uint32_t j = 0; j < nch[i]; ++j) order[srun + j] = run + j;
                sfirst[b] = srun;
                srun += nch[i];
            } else if (nch[i] == 1) {
                order[nsplit + orun] = run;
                ++orun;
            }
        }
        run += nch[i];
    }
    if (threadIdx.x == 0) cstart[P] = total;
}

// Persistent: one workgroup per CU takes chunks from a queue (order[], via a
// counter) until none is left, and aggregates each chunk's rows in an LDS
// table.  A bucket that is one chunk writes its groups out directly.  Each
// chunk of a split bucket writes its partial groups to its own stretch of
// the workspace and counts itself done; the bucket's last chunk to finish
// folds the other chunks' partial groups into its LDS table and writes the
// bucket's groups out.  (If a chunk of the bucket sent rows to the global
// table, because its LDS table was full, every partial goes to the global
// table instead, so that no key is emitted from two places; the table's emit
// pass writes those.)  The next chunk is taken when a chunk starts, and its
// first records are loaded during the current chunk's last step, so they
// arrive while the current chunk writes its groups.  When more than
// GB_COMBINE_LANES lanes of a wave update the same slot, they are summed
// across the wave first and added by one lane, so a heavy key costs one LDS
// update per wave rather than one per row.
template <bool K64, bool K32>
__global__ __launch_bounds__(GB_BUCKET_THREADS) void gb_bucket_kernel(const uint64_t *__restrict__ recs,
                                                                      const uint32_t *__restrict__ start,
                                                                      const uint32_t *__restrict__ cstart,
                                                                      const uint32_t *__restrict__ order,
                                                                      const uint32_t *__restrict__ sfirst, int P,
                                                                      int64_t chunk_rows, const uint32_t *side_cnt,
                                                                      uint32_t *qctr, uint32_t *bdone, uint32_t *bspill,
                                                                      uint32_t *pcnt, gb_part *part, gtable g,
                                                                      gq_groups out, uint32_t *status)
{
    constexpr int SLOTS = bucket_slots<K64, K32>::value;
    __shared__ lds_table<SLOTS, K64, K32> T;
    __shared__ uint32_t scan_smem[GB_BUCKET_THREADS / 64];
    __shared__ unsigned long long s_base;
    __shared__ uint32_t s_item, s_spill, s_last;
    const uint32_t total = cstart[P];
    // rows [r0, r1) of queue item `item`, its bucket, and whether that is split
    auto geom = [&](uint32_t item, int64_t &r0, int64_t &r1, int &bk, bool &split) {
        const uint32_t ch = order[item];
        int b = 0;                                   // the bucket of chunk ch: last b with cstart[b] <= ch
        for (int hi = P - 1; b < hi;) {
            const int mid = (b + hi + 1) >> 1;
            if (cstart[mid] <= ch) b = mid;
            else hi = mid - 1;
        }
        split = cstart[b + 1] - cstart[b] > 1;
        bk = b;
        const int64_t b0 = start[b], b1 = start[b + 1];
        r0 = split ? b0 + static_cast<int64_t>(ch - cstart[b]) * chunk_rows : b0;
        r1 = split ? (r0 + chunk_rows < b1 ? r0 + chunk_rows : b1) : b1;
    };
    constexpr int ITEMS = bucket_items<K64>::value;
    constexpr int STEP = GB_BUCKET_THREADS * ITEMS;
    // the records of the next step are loaded while this step's are aggregated
    int64_t nk64[ITEMS], nq[ITEMS], nrv[ITEMS];
    int32_t nk32[ITEMS];
    auto load_step = [&](int64_t i0, int64_t end) {
#pragma unroll
        for (int c = 0; c < ITEMS; ++c) {
            const int64_t i = i0 + c * GB_BUCKET_THREADS + threadIdx.x;
            nk64[c] = nq[c] = nrv[c] = 0;
            nk32[c] = 0;
            if (i < end) read_words<K64, K32>(recs, i, nk64[c], nk32[c], nq[c], nrv[c]);
        }
    };
    if (threadIdx.x == 0) s_item = atomicAdd(qctr, 1u);
    __syncthreads();
    uint32_t item = s_item;
    if (item >= total) return;                       // same for the whole workgroup
    int64_t r0, r1;
    int bk;
    bool split;
    geom(item, r0, r1, bk, split);
    bool have = false;                               // n*[] hold the first step of this item
    const bool merge = *side_cnt != 0u;              // same value for every thread
    lds_init(T);                                     // once: each chunk leaves the table empty
    while (true) {
        if (!have) load_step(r0, r1);
        if (threadIdx.x == 0) s_spill = 0;
        __syncthreads();                             // the table is clear; every thread has read s_item
        if (threadIdx.x == 0) s_item = atomicAdd(qctr, 1u);
        __syncthreads();
        const uint32_t nitem = s_item;
        int64_t nr0 = 0, nr1 = 0;
        int nbk = 0;
        bool nsplit = false;
        if (nitem < total) geom(nitem, nr0, nr1, nbk, nsplit);
        bool have_next = false;
        for (int64_t i0 = r0; i0 < r1; i0 += STEP) {
            int64_t k64[ITEMS], q[ITEMS], rv[ITEMS];
            int32_t k32[ITEMS];
#pragma unroll
            for (int c = 0; c < ITEMS; ++c) {
                k64[c] = nk64[c];
                k32[c] = nk32[c];
                q[c] = nq[c];
                rv[c] = nrv[c];
            }
            if (i0 + STEP < r1) {
                load_step(i0 + STEP, r1);
            } else if (nitem < total) {              // the next item's first step
                load_step(nr0, nr1);
                have_next = true;
            }
#pragma unroll
            for (int c = 0; c < ITEMS; ++c) {
                const int64_t i = i0 + c * GB_BUCKET_THREADS + threadIdx.x;
                const bool active = i < r1;
                gq_i128 rev;
                rev.lo = static_cast<uint64_t>(rv[c]);
                rev.hi = rv[c] >> 63;
                const uint64_t h = gb_hash(k64[c], k32[c]);
                const int s = lds_find(T, active, h, k64[c], k32[c]);
                bool mine = active && s >= 0;
                const uint64_t am = gq_ballot(mine);
                if (am) {
                    // the slot of the first updating lane, summed over every lane that updates it
                    const int lead = __builtin_ctzll(am);
                    const int sl = __builtin_amdgcn_readlane(s, lead);
                    const bool in = mine && s == sl;
                    const uint64_t same = gq_ballot(in);
                    // worth the cross-lane sums only for a key that fills much of
                    // the wave (a few equal lanes cost less as plain LDS atomics)
                    if (__popcll(same) > GB_COMBINE_LANES) {
                        const uint32_t cn = static_cast<uint32_t>(__popcll(same));
                        const uint64_t sq = gq_wave_sum<uint64_t>(in ? static_cast<uint64_t>(q[c]) : 0ull);
                        const uint64_t lo = gq_wave_sum<uint64_t>(
                            in ? static_cast<uint64_t>(static_cast<uint32_t>(static_cast<uint64_t>(rv[c]))) : 0ull);
                        const int64_t hs = gq_wave_sum<int64_t>(in ? (rv[c] >> 32) : 0);
                        if (gq_lane() == lead) lds_add_sums(T, sl, cn, sq, lo, hs);
                        mine = mine && !in;
                    }
                }
                if (mine) lds_add_split(T, s, q[c], rv[c]);
                const bool spill = active && s < 0;
                if (spill) s_spill = 1u;
                const int64_t gs = g_find<K64, K32>(g, spill, h, k64[c], k32[c], status);
                if (spill && gs >= 0) g_add(g, gs, 1u, static_cast<uint64_t>(q[c]), rev);
            }
        }
        __syncthreads();
        bool emit = !split;
        if (split) {
            // this chunk's partial groups to its stretch of the workspace
            constexpr int PER = SLOTS / GB_BUCKET_THREADS;
            uint32_t mine = 0;
#pragma unroll
            for (int i = 0; i < PER; ++i) mine += lds_occupied(T, threadIdx.x * PER + i) ? 1u : 0u;
            uint32_t all;
            uint32_t pre = gq_block_exclusive_scan<GB_BUCKET_THREADS>(mine, &all, scan_smem);
            gb_part *dst = part + static_cast<size_t>(item) * SLOTS;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int s = threadIdx.x * PER + i;
                if (lds_occupied(T, s)) {
                    const gq_i128 tot = lds_split_total(T.lo[s], T.hi[s]);
                    dst[pre++] = gb_part{lds_key64(T, s), lds_key32(T, s), T.cnt[s], T.sq[s], tot.lo, tot.hi};
                }
            }
            __syncthreads();                         // every partial is written
            if (threadIdx.x == 0) {
                pcnt[item] = all;
                if (s_spill) atomicOr(&bspill[bk], 1u);
                __threadfence();                     // partials, count and spill flag before the done count
                const uint32_t nch = cstart[bk + 1] - cstart[bk];
                s_last = (atomicAdd(&bdone[bk], 1u) + 1 == nch) ? 1u : 0u;
            }
            __syncthreads();
            if (s_last) {                            // the bucket's last chunk: every other chunk is done
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const bool to_global = __hip_atomic_load(&bspill[bk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
                const uint32_t nch = cstart[bk + 1] - cstart[bk];
                const uint32_t first = sfirst[bk];
                for (uint32_t j = 0; j < nch; ++j) {
                    const uint32_t it = first + j;
                    if (it == item && !to_global) continue;    // its own groups are in the LDS table
                    const uint32_t cntj = __hip_atomic_load(&pcnt[it], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const gb_part *src = part + static_cast<size_t>(it) * SLOTS;
                    for (uint32_t e0 = 0; e0 < cntj; e0 += GB_BUCKET_THREADS) {
                        const uint32_t e = e0 + threadIdx.x;
                        const bool act = e < cntj;
                        gb_part pe{};
                        if (act) pe = src[e];
                        const uint64_t h = gb_hash(pe.k64, pe.k32);
                        const gq_i128 rev{pe.lo, pe.hi};
                        // into the LDS table (unless the bucket goes to the global table)
                        int sl = to_global ? -1 : lds_find(T, act, h, pe.k64, pe.k32);
                        if (act && sl >= 0) {
                            // the int128 sum as split halves: low 32 bits, then the rest
                            // (|rev >> 32| < rows * 2^31 fits the 64-bit high sum)
                            const int64_t hi32 = static_cast<int64_t>((static_cast<uint64_t>(pe.hi) << 32) | (pe.lo >> 32));
                            lds_add_sums(T, sl, pe.cnt, pe.sq, pe.lo & 0xffffffffull, hi32);
                        }
                        const bool gl = act && sl < 0;
                        const int64_t gs = g_find<K64, K32>(g, gl, h, pe.k64, pe.k32, status);
                        if (gl && gs >= 0) g_add(g, gs, pe.cnt, pe.sq, rev);
                    }
                }
                emit = !to_global;
                __syncthreads();                     // the folded table is complete
            }
        }
        if (emit) {
            // emit: each thread owns SLOTS / GB_BUCKET_THREADS consecutive slots
            constexpr int PER = SLOTS / GB_BUCKET_THREADS;
            uint32_t mine = 0;
#pragma unroll
            for (int i = 0; i < PER; ++i) mine += lds_occupied(T, threadIdx.x * PER + i) ? 1u : 0u;
            uint32_t all;
            uint32_t pre = gq_block_exclusive_scan<GB_BUCKET_THREADS>(mine, &all, scan_smem);
            if (threadIdx.x == 0)
                s_base = all ? atomicAdd(reinterpret_cast<unsigned long long *>(out.n_groups),
                                         static_cast<unsigned long long>(all))
                             : 0ull;
            __syncthreads();
            int64_t idx = static_cast<int64_t>(s_base) + pre;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int s = threadIdx.x * PER + i;
                const bool occ = lds_occupied(T, s);
                const int64_t k64 = occ ? lds_key64(T, s) : 0;
                const int32_t k32 = occ ? lds_key32(T, s) : 0;
                uint64_t cnt = occ ? T.cnt[s] : 0, sq = occ ? T.sq[s] : 0;
                const gq_i128 tot = lds_split_total(occ ? T.lo[s] : 0, occ ? T.hi[s] : 0);
                uint64_t lo = tot.lo;
                int64_t hi = tot.hi;
                if (merge) {
                    const int64_t gs = g_lookup<K64, K32>(g, occ, gb_hash(k64, k32), k64, k32);
                    if (occ && gs >= 0) {
                        cnt += g.cnt[gs];
                        sq += g.sq[gs];
                        const uint64_t l2 = lo + g.lo[gs];
                        hi += g.hi[gs] + (l2 < lo ? 1 : 0);
                        lo = l2;
                        __hip_atomic_store(&g.state[gs], 3u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                if (occ) {
                    emit_group(out, idx, k64, k32, cnt, sq, lo, hi, status);
                    ++idx;
                    lds_clear_slot(T, s);            // the table is empty again for the next chunk
                }
            }
        } else {
            constexpr int PER = SLOTS / GB_BUCKET_THREADS;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int s = threadIdx.x * PER + i;
                if (lds_occupied(T, s)) lds_clear_slot(T, s);
            }
        }
        if (nitem >= total) break;                   // same for the whole workgroup
        item = nitem;
        r0 = nr0;
        r1 = nr1;
        bk = nbk;
        split = nsplit;
        have = have_next;
        __syncthreads();                             // the table is read out before it is cleared
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
    int P;                  // buckets of the large path
    bool wide;              // P > GB_MAX_P: two levels (GB_P1 super-buckets, then P / GB_P1 each)
    int P2;                 // sub-buckets per super-bucket (wide)
    int64_t tiles2;         // level-2 tiles, an upper bound (wide)
    int64_t ntiles;         // hist/scatter tiles (of level 1 when wide)
    int64_t chunk_rows;     // rows per hist/scatter workgroup
    int words;              // 8-byte words per partitioned record
    uint64_t gslots;
    int64_t bucket_chunk;   // rows per workgroup of a split bucket
    int64_t bucket_grid;    // bucket-pass workgroups: P plus the most extra chunks n rows can need
    int64_t split_max;      // the most chunks that split buckets can have
};

int groupby_fill_percent()
{
    static const int v = [] {
        const char *e = getenv("GQ_GROUPBY_FILL");
        const int x = e ? atoi(e) : 40;
        return (x >= 10 && x <= 90) ? x : 40;
    }();
    return v;
}

gb_plan make_plan(int64_t n, int64_t max_groups, bool k64, bool k32)
{
    (void)k32;
    gb_plan pl{};
    pl.small = max_groups <= GB_SMALL_GROUPS;
    pl.gslots = next_pow2(static_cast<uint64_t>(max_groups > 32 ? 2 * max_groups : 64));
    // hist chunks: one tile of the tile scatter (key64 records), or a chunk
    // of the region scatter (16-byte records)
    const int64_t tile = static_cast<int64_t>(GB_THREADS) * 8;        // gb_fmt<>::TILE
    pl.chunk_rows = (!pl.small && !k64) ? GL_CHUNK_ROWS : tile;
    pl.ntiles = n > 0 ? (n + pl.chunk_rows - 1) / pl.chunk_rows : 1;
    pl.words = k64 ? 3 : 2;
    if (!pl.small) {
        // about 40% of a bucket's LDS table for the expected groups: the
        // bucket pass waits on the longest probe chain of 64 lanes, so short
        // chains pay for the extra buckets (GQ_GROUPBY_FILL=<percent>, 10..90,
        // overrides it for measurements)
        const int64_t per_bucket = (k64 ? 3072 : 4096) * groupby_fill_percent() / 100;
        int64_t P = (max_groups + per_bucket - 1) / per_bucket;
        // one 1024-thread workgroup per bucket and one per CU at a time: a
        // whole number of rounds over the CUs leaves no idle tail
        if (P > GB_CUS) P = (P + GB_CUS - 1) / GB_CUS * GB_CUS;
        pl.P = static_cast<int>(std::min<int64_t>(std::max<int64_t>(P, 2), GB_MAX_P_WIDE));
        pl.wide = pl.P > GB_MAX_P;
        // a bucket with more than 4x the mean rows (and at least 64K) holds a
        // heavy key: it is split into chunks of that many rows
        const int64_t mean = (n + pl.P - 1) / pl.P;
        pl.bucket_chunk = std::max<int64_t>(4 * mean, 65536);
        pl.bucket_chunk = (pl.bucket_chunk + 4095) / 4096 * 4096;
        pl.bucket_grid = pl.P + n / pl.bucket_chunk;
        // a split bucket has more than bucket_chunk rows and at most
        // 2 rows / bucket_chunk chunks
        pl.split_max = 2 * (n / pl.bucket_chunk) + 1;
        if (pl.wide) {                      // P is a multiple of GB_CUS, so of GB_P1
            pl.P2 = pl.P / GB_P1;
            pl.tiles2 = (n + GB_T2 - 1) / GB_T2 + GB_P1;
        }
    }
    return pl;
}

struct gb_ws {
    gtable g;
    uint32_t *side_cnt;
    uint32_t *hist;
    uint32_t *start;
    uint32_t *cstart;       // chunks of the bucket pass before each bucket
    uint32_t *order;        // the bucket pass's chunk queue
    uint32_t *sfirst;       // queue position of a split bucket's first chunk
    uint32_t *bdone;        // chunks of each bucket finished
    uint32_t *bspill;       // a chunk of the bucket sent rows to the global table
    uint32_t *pcnt;         // partial groups of each split chunk
    void *part;             // the partial groups (split chunks only)
    void *scan_ws;
    uint64_t *recs;         // partitioned rows, narrow records
    uint32_t *side;         // row indices of wide rows
    uint32_t *startA;       // two levels: super-bucket starts (level 1)
    uint32_t *tpre;         //   level-2 tiles before each super-bucket
    uint32_t *hist2;        //   level-2 counts, then run positions, per (tile, sub-bucket)
    uint64_t *recs1;        //   level-1 records, in super-bucket order
    size_t zero_bytes;      // prefix of the workspace to clear (table, side count)
};

gb_ws gb_layout(gq_carver &c, const gb_plan &pl, int64_t n, bool k64, bool k32)
{
    gb_ws w{};
    const size_t S = pl.gslots;
    w.g.state = c.take<uint32_t>(S);
    // [0] wide rows; [32 (x + 1)] the scatter's tile counter of XCD x;
    // [32 (GQ_NUM_XCD + 1)] the bucket pass's queue counter; one 128-byte
    // line each
    w.side_cnt = c.take<uint32_t>(32 * (GQ_NUM_XCD + 2));
    w.g.used = c.take<uint32_t>(32);
    if (!pl.small) {                        // per bucket: chunks finished, a chunk spilled
        w.bdone = c.take<uint32_t>(static_cast<size_t>(pl.P));
        w.bspill = c.take<uint32_t>(static_cast<size_t>(pl.P));
    }
    w.zero_bytes = c.off;                   // the state words and counters start at zero
    w.g.k64 = c.take<int64_t>(k64 ? S : 1);
    w.g.k32 = c.take<int32_t>(k32 ? S : 1);
    w.g.cnt = c.take<uint64_t>(S);
    w.g.sq = c.take<uint64_t>(S);
    w.g.lo = c.take<uint64_t>(S);
    w.g.hi = c.take<int64_t>(S);
    w.g.mask = S - 1;
    if (!pl.small) {
        const size_t rows = static_cast<size_t>(n > 0 ? n : 1);
        const int P1 = pl.wide ? GB_P1 : pl.P;              // buckets of the tile-staged scatter
        w.hist = c.take<uint32_t>(static_cast<size_t>(pl.ntiles) * static_cast<size_t>(P1));
        w.start = c.take<uint32_t>(static_cast<size_t>(pl.P) + 1);
        w.cstart = c.take<uint32_t>(static_cast<size_t>(pl.P) + 1);
        w.order = c.take<uint32_t>(static_cast<size_t>(pl.bucket_grid));
        w.sfirst = c.take<uint32_t>(static_cast<size_t>(pl.P));
        w.pcnt = c.take<uint32_t>(static_cast<size_t>(pl.split_max));
        w.part = c.take<char>(static_cast<size_t>(pl.split_max) * static_cast<size_t>(k64 ? 3072 : 4096) *
                              sizeof(gb_part));
        w.scan_ws = c.take<char>(gq_tile_offsets_workspace(pl.ntiles, P1));
        w.recs = c.take<uint64_t>(rows * static_cast<size_t>(pl.words));
        w.side = c.take<uint32_t>(rows);
        if (pl.wide) {
            w.startA = c.take<uint32_t>(GB_P1 + 1);
            w.tpre = c.take<uint32_t>(GB_P1 + 1);
            w.hist2 = c.take<uint32_t>(static_cast<size_t>(pl.tiles2) * static_cast<size_t>(pl.P2));
            w.recs1 = c.take<uint64_t>(rows * static_cast<size_t>(pl.words));
        }
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
    const int P1 = pl.wide ? GB_P1 : pl.P;              // buckets of the tile-staged scatter
    uint32_t *start1 = pl.wide ? w.startA : w.start;
    uint64_t *recs1 = pl.wide ? w.recs1 : w.recs;
    GQ_TRY(gq_launch(ctx, "gq_groupby_hist", gb_hist_kernel<K64, K32, GB_MAX_P>, dim3(grid), dim3(GB_THREADS), 0, s,
                     a, P1, pl.chunk_rows, w.hist));
    const gq_tile_count live{a.n_dev, a.n_bound, pl.chunk_rows};     // tiles past the device row count are idle
    GQ_TRY(gq_tile_offsets(ctx, w.hist, pl.ntiles, P1, start1, w.scan_ws, s, "gq_groupby_scan", &live));
    // XCD x scatters the x-th eighth of the tiles with the workgroups b of
    // b mod 8 = x, so the grid is a whole number of rounds over the eight
    // XCDs (at least one workgroup each, even for fewer than 8 tiles); a
    // workgroup whose range is empty exits at once
    if constexpr (K64) {
        int64_t sgrid = std::min<int64_t>(grid, static_cast<int64_t>(ctx->num_cus) * 2);
        sgrid = (sgrid + GQ_NUM_XCD - 1) / GQ_NUM_XCD * GQ_NUM_XCD;
        GQ_TRY(gq_launch(ctx, "gq_groupby_scatter", gb_scatter_kernel<K64, K32>, dim3(static_cast<uint32_t>(sgrid)),
                         dim3(GB_THREADS), 0, s, a, P1, static_cast<const uint32_t *>(w.hist), recs1, w.side,
                         w.side_cnt, w.side_cnt + 32));
    } else {
        // one region per CU (a workgroup takes most of a CU's LDS)
        const int64_t rgrid = std::min<int64_t>(grid, static_cast<int64_t>(ctx->num_cus));
        GQ_TRY(gq_launch(ctx, "gq_groupby_scatter", gb_scatter_lines_kernel<K32>,
                         dim3(static_cast<uint32_t>(rgrid)), dim3(GL_THREADS), 0, s, a, P1, pl.chunk_rows,
                         static_cast<const uint32_t *>(w.hist), reinterpret_cast<uint4 *>(recs1), w.side,
                         w.side_cnt));
    }
    if (pl.wide) {                                      // level 2: each super-bucket by its sub-buckets
        GQ_TRY(gq_launch(ctx, "gq_groupby_tiles2", gb_tiles2_kernel, dim3(1), dim3(256), 0, s,
                         static_cast<const uint32_t *>(w.startA), GB_P1, w.tpre));
        const uint32_t g2 = static_cast<uint32_t>(pl.tiles2);
        GQ_TRY(gq_launch(ctx, "gq_groupby_hist2", gb_hist2_kernel<K64, K32>, dim3(g2), dim3(GB_THREADS), 0, s,
                         static_cast<const uint64_t *>(w.recs1), static_cast<const uint32_t *>(w.startA),
                         static_cast<const uint32_t *>(w.tpre), GB_P1, pl.P, pl.P2, w.hist2));
        GQ_TRY(gq_launch(ctx, "gq_groupby_scan2", gb_scan2_kernel, dim3(GB_P1), dim3(256), 0, s, w.hist2,
                         static_cast<const uint32_t *>(w.startA), static_cast<const uint32_t *>(w.tpre), GB_P1, pl.P2,
                         w.start));
        GQ_TRY(gq_launch(ctx, "gq_groupby_scatter2", gb_scatter2_kernel<K64, K32>, dim3(g2), dim3(GB_THREADS), 0, s,
                         static_cast<const uint64_t *>(w.recs1), static_cast<const uint32_t *>(w.startA),
                         static_cast<const uint32_t *>(w.tpre), static_cast<const uint32_t *>(w.hist2), GB_P1, pl.P,
                         pl.P2, w.recs));
    }
    GQ_TRY(gq_launch(ctx, "gq_groupby_side", gb_side_kernel<K64, K32>, dim3(64), dim3(256), 0, s, a,
                     static_cast<const uint32_t *>(w.side), static_cast<const uint32_t *>(w.side_cnt), w.g,
                     ctx->status_dev));
    GQ_TRY(gq_launch(ctx, "gq_groupby_chunks", gb_chunks_kernel, dim3(1), dim3(GB_BUCKET_THREADS), 0, s,
                     static_cast<const uint32_t *>(w.start), pl.P, pl.bucket_chunk, w.cstart, w.order, w.sfirst));
    // one workgroup per CU (its LDS table takes most of a CU), each taking
    // chunks from the queue
    const int64_t bgrid = std::min<int64_t>(pl.bucket_grid, static_cast<int64_t>(ctx->num_cus));
    GQ_TRY(gq_launch(ctx, "gq_groupby_bucket", gb_bucket_kernel<K64, K32>, dim3(static_cast<uint32_t>(bgrid)),
                     dim3(GB_BUCKET_THREADS), 0, s, static_cast<const uint64_t *>(w.recs),
                     static_cast<const uint32_t *>(w.start), static_cast<const uint32_t *>(w.cstart),
                     static_cast<const uint32_t *>(w.order), static_cast<const uint32_t *>(w.sfirst), pl.P,
                     pl.bucket_chunk, static_cast<const uint32_t *>(w.side_cnt), w.side_cnt + 32 * (GQ_NUM_XCD + 1),
                     w.bdone, w.bspill, w.pcnt, static_cast<gb_part *>(w.part), w.g, out, ctx->status_dev));
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
