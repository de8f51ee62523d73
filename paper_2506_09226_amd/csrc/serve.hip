// Shared-scan execution of a batch of queries of one template (the served
// form) and the plain per-query execution (the serial baseline).
//
// Templates over resident tables: a fact table (fk, fk2, date, qty, price,
// disc) and two dimension hash tables built by gq_join_build (payload = the
// dimension attribute).  Every query keeps the fact rows with date < date_hi.
//   FILTER_AGG   group by disc
//   JOIN_AGG     join fk with dim1, group by the dim1 attribute
//   JOIN2_AGG    join fk with dim1 and fk2 with dim2, group by the dim2 attribute
//   FILTER_TOPK  the k rows with the largest price (ties by row id)
// Aggregates: count, sum(qty), exact 128-bit sum of price * (100 - disc) and
// the float64 averages.
//
// A batch of Q queries of one template reads the fact columns once: each row
// is tested against every query's threshold and aggregated into per-query
// LDS tables (or offered to per-query top-k buffers); dimension probes are
// done once per row for the whole batch.  JOIN_AGG (about a million groups)
// shares the filter and the probe, then runs one filtered group-by per query.
#include <algorithm>
#include <cstring>
#include <vector>

#include "gq_device.h"
#include "gq_internal.h"
#include "gq_serve.h"

namespace {

constexpr int SV_THREADS = 256;
constexpr int SV_ITEMS = 16;
constexpr int SV_TILE = SV_THREADS * SV_ITEMS;
constexpr int SV_SLOTS = 64;                         // LDS group slots per query
constexpr int64_t SV_EMPTY = INT64_MIN;

struct sv_table {                                     // view of a join table built by gq_join_build
    const int4 *slots;
    int L;
};

GQ_DEV bool sv_lookup(const sv_table &t, int64_t k, int32_t &payload)
{
    if (k == SV_EMPTY) return false;                  // the empty-slot marker is no key: it never matches
    const uint64_t mask = (1ull << t.L) - 1;
    uint64_t s = gq_fmix64(static_cast<uint64_t>(k)) >> (64 - t.L);
    for (uint64_t p = 0; p <= mask; ++p) {
        const int4 v = t.slots[s];
        const int64_t sk = (static_cast<int64_t>(static_cast<uint32_t>(v.y)) << 32) | static_cast<uint32_t>(v.x);
        if (sk == k) {
            payload = v.z;
            return true;
        }
        if (sk == SV_EMPTY) return false;
        s = (s + 1) & mask;
    }
    return false;
}

// ------------------------------------------------------------ group tables
struct sv_gtable {                   // per query, global, 2^k slots
    uint32_t *state;
    int64_t *key;
    uint64_t *cnt, *sq, *lo;
    int64_t *hi;
    uint64_t mask;
};

struct sv_lds {
    uint32_t state[SV_MAX_BATCH][SV_SLOTS];
    int64_t key[SV_MAX_BATCH][SV_SLOTS];
    uint32_t cnt[SV_MAX_BATCH][SV_SLOTS];
    uint64_t sq[SV_MAX_BATCH][SV_SLOTS];
    uint64_t lo[SV_MAX_BATCH][SV_SLOTS];
    int64_t hi[SV_MAX_BATCH][SV_SLOTS];
};

GQ_DEV void add128(uint64_t *lo, int64_t *hi, gq_i128 v)
{
    const unsigned long long old =
        atomicAdd(reinterpret_cast<unsigned long long *>(lo), static_cast<unsigned long long>(v.lo));
    const int64_t h = v.hi + ((old + v.lo < old) ? 1 : 0);
    if (h) atomicAdd(reinterpret_cast<unsigned long long *>(hi), static_cast<unsigned long long>(h));
}

// find-or-claim a key in query q's LDS table (wave-uniform loop); -1 if full
GQ_DEV int lds_slot(sv_lds &T, int q, bool active, int64_t key)
{
    uint32_t s = static_cast<uint32_t>(gq_fmix64(static_cast<uint64_t>(key))) & (SV_SLOTS - 1);
    int probes = 0, found = -1;
    bool done = !active;
    while (__any(!done)) {
        if (!done) {
            uint32_t st = __hip_atomic_load(&T.state[q][s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (st == 0u) st = atomicCAS(&T.state[q][s], 0u, 1u);   // claim only an empty slot
            if (st == 0u) {
                T.key[q][s] = key;
                __threadfence_block();
                atomicExch(&T.state[q][s], 2u);
                found = static_cast<int>(s);
                done = true;
            } else if (st == 2u) {
                if (T.key[q][s] == key) {
                    found = static_cast<int>(s);
                    done = true;
                } else if (++probes >= SV_SLOTS) {
                    done = true;
                } else {
                    s = (s + 1) & (SV_SLOTS - 1);
                }
            }
        }
    }
    return found;
}

GQ_DEV int64_t global_slot(const sv_gtable &g, bool active, int64_t key, uint32_t *status)
{
    uint64_t s = gq_fmix64(static_cast<uint64_t>(key)) & g.mask;
    uint64_t probes = 0;
    int64_t found = -1;
    bool done = !active;
    while (__any(!done)) {
        if (!done) {
            const uint32_t st = atomicCAS(&g.state[s], 0u, 1u);
            if (st == 0u) {
                __hip_atomic_store(&g.key[s], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&g.state[s], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                found = static_cast<int64_t>(s);
                done = true;
            } else if (st == 2u) {
                (void)__hip_atomic_load(&g.state[s], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (__hip_atomic_load(&g.key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == key) {
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

GQ_DEV void global_add(const sv_gtable &g, int64_t s, uint64_t cnt, uint64_t sq, gq_i128 rev)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(&g.cnt[s]), static_cast<unsigned long long>(cnt));
    atomicAdd(reinterpret_cast<unsigned long long *>(&g.sq[s]), static_cast<unsigned long long>(sq));
    add128(&g.lo[s], &g.hi[s], rev);
}

struct sv_outs {                      // output descriptors of a batch's queries, passed by value
    gq_serve_query_out o[SV_MAX_BATCH];
};

struct sv_batch {                     // kernel view of a batch
    int nq;
    int64_t hi[SV_MAX_BATCH];         // date_hi per level, descending
    sv_gtable g[SV_MAX_BATCH];        // one table per level
    int32_t qidx[SV_MAX_BATCH];       // output slot of the query at each level
};

// Number of queries (levels) that keep a row with this date: hi is sorted in
// descending order, so they are levels 0 .. L-1.
GQ_DEV int row_level(const sv_batch &b, int64_t date)
{
    int L = 0;
    for (int l = 0; l < b.nq; ++l) L += date < b.hi[l] ? 1 : 0;
    return L;
}

// FILTER_AGG (key = disc) and JOIN2_AGG (key = dim2 attribute): one pass over
// the fact rows for the whole batch; each kept row is aggregated once, into
// the table of its level L-1 (the most selective query that keeps it).
template <bool JOIN2>
__global__ __launch_bounds__(SV_THREADS) void sv_agg_kernel(gq_serve_tables t, sv_table d1, sv_table d2,
                                                            sv_batch b, uint32_t *status)
{
    __shared__ sv_lds T;
    for (int i = threadIdx.x; i < SV_MAX_BATCH * SV_SLOTS; i += SV_THREADS) {
        (&T.state[0][0])[i] = 0;
        (&T.cnt[0][0])[i] = 0;
        (&T.sq[0][0])[i] = 0;
        (&T.lo[0][0])[i] = 0;
        (&T.hi[0][0])[i] = 0;
    }
    __syncthreads();
    const int64_t n = t.n;
    const int64_t step = static_cast<int64_t>(gridDim.x) * SV_TILE;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * SV_TILE; base < n; base += step) {
        int32_t date[SV_ITEMS];
#pragma unroll
        for (int c = 0; c < SV_ITEMS; ++c) {
            const int64_t r = base + c * SV_THREADS + threadIdx.x;
            date[c] = r < n ? t.date[r] : 0;
        }
#pragma unroll
        for (int c = 0; c < SV_ITEMS; ++c) {
            const int64_t r = base + c * SV_THREADS + threadIdx.x;
            int level = r < n ? row_level(b, date[c]) : 0;
            int64_t key = 0, qty = 0;
            gq_i128 rev{0, 0};
            if (level > 0) {
                if (JOIN2) {
                    int32_t p1 = 0, p2 = 0;
                    if (!(sv_lookup(d1, t.fk[r], p1) && sv_lookup(d2, t.fk2[r], p2))) level = 0;
                    key = p2;
                } else {
                    key = t.disc[r];
                }
                if (level > 0) {
                    qty = t.qty[r];
                    rev = gq_revenue(t.price[r], 100, t.disc[r]);
                }
            }
            const int q = level > 0 ? level - 1 : 0;
            const int s = lds_slot(T, q, level > 0, key);
            if (level > 0 && s >= 0) {
                atomicAdd(&T.cnt[q][s], 1u);
                atomicAdd(reinterpret_cast<unsigned long long *>(&T.sq[q][s]), static_cast<unsigned long long>(qty));
                add128(&T.lo[q][s], &T.hi[q][s], rev);
            }
            const bool spill = level > 0 && s < 0;
            const int64_t gs = global_slot(b.g[q], spill, key, status);
            if (spill && gs >= 0) global_add(b.g[q], gs, 1, static_cast<uint64_t>(qty), rev);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SV_MAX_BATCH * SV_SLOTS; i += SV_THREADS) {
        const int q = i / SV_SLOTS, s = i % SV_SLOTS;
        const bool occ = q < b.nq && T.state[q][s] == 2u;
        const int64_t key = occ ? T.key[q][s] : 0;
        const int64_t gs = global_slot(b.g[q < b.nq ? q : 0], occ, key, status);
        if (occ && gs >= 0) {
            gq_i128 rv;
            rv.lo = T.lo[q][s];
            rv.hi = T.hi[q][s];
            global_add(b.g[q], gs, T.cnt[q][s], T.sq[q][s], rv);
        }
    }
}

// Block l produces the query at level l: the sum of level tables l .. nq-1,
// merged in an LDS table and written to that query's output.
constexpr int SV_EMIT_SLOTS = 2 * SV_MAX_AGG_GROUPS;

__global__ __launch_bounds__(256) void sv_emit_kernel(sv_batch b, sv_outs outs, uint32_t *status)
{
    __shared__ uint32_t st[SV_EMIT_SLOTS];
    __shared__ int64_t ky[SV_EMIT_SLOTS];
    __shared__ uint64_t cn[SV_EMIT_SLOTS], sq[SV_EMIT_SLOTS], lo[SV_EMIT_SLOTS];
    __shared__ int64_t hi[SV_EMIT_SLOTS];
    __shared__ uint32_t scan_smem[4];
    const int l = blockIdx.x;
    for (int i = threadIdx.x; i < SV_EMIT_SLOTS; i += 256) {
        st[i] = 0;
        cn[i] = sq[i] = lo[i] = 0;
        hi[i] = 0;
    }
    __syncthreads();
    for (int lv = l; lv < b.nq; ++lv) {
        const sv_gtable g = b.g[lv];
        const uint64_t slots = g.mask + 1;
        for (uint64_t base = 0; base < slots; base += 256) {
            const uint64_t s = base + threadIdx.x;
            const bool occ = s < slots && g.state[s] == 2u;
            const int64_t key = occ ? g.key[s] : 0;
            uint32_t e = static_cast<uint32_t>(gq_fmix64(static_cast<uint64_t>(key))) & (SV_EMIT_SLOTS - 1);
            bool done = !occ;
            int found = -1, probes = 0;
            while (__any(!done)) {
                if (!done) {
                    const uint32_t x = atomicCAS(&st[e], 0u, 1u);
                    if (x == 0u) {
                        ky[e] = key;
                        __threadfence_block();
                        atomicExch(&st[e], 2u);
                        found = static_cast<int>(e);
                        done = true;
                    } else if (x == 2u) {
                        if (ky[e] == key) {
                            found = static_cast<int>(e);
                            done = true;
                        } else if (++probes >= SV_EMIT_SLOTS) {
                            gq_raise(status, GQ_ERR_CAPACITY);
                            done = true;
                        } else {
                            e = (e + 1) & (SV_EMIT_SLOTS - 1);
                        }
                    }
                }
            }
            if (occ && found >= 0) {
                atomicAdd(reinterpret_cast<unsigned long long *>(&cn[found]),
                          static_cast<unsigned long long>(g.cnt[s]));
                atomicAdd(reinterpret_cast<unsigned long long *>(&sq[found]),
                          static_cast<unsigned long long>(g.sq[s]));
                gq_i128 v;
                v.lo = g.lo[s];
                v.hi = g.hi[s];
                add128(&lo[found], &hi[found], v);
            }
        }
        __syncthreads();
    }
    // compact: each thread owns SV_EMIT_SLOTS / 256 consecutive slots
    constexpr int PER = SV_EMIT_SLOTS / 256;
    uint32_t mine = 0;
    for (int i = 0; i < PER; ++i) mine += st[threadIdx.x * PER + i] == 2u ? 1u : 0u;
    uint32_t total;
    uint32_t idx = gq_block_exclusive_scan<256>(mine, &total, scan_smem);
    const gq_groups &out = outs.o[b.qidx[l]].groups;
    for (int i = 0; i < PER; ++i) {
        const int s = threadIdx.x * PER + i;
        if (st[s] != 2u) continue;
        if (idx >= out.capacity) {
            gq_raise(status, GQ_ERR_CAPACITY);
            ++idx;
            continue;
        }
        if (out.key64) out.key64[idx] = ky[s];
        if (out.key32) out.key32[idx] = static_cast<int32_t>(ky[s]);
        out.count[idx] = static_cast<int64_t>(cn[s]);
        out.sum_qty[idx] = static_cast<int64_t>(sq[s]);
        out.sum_rev_lo[idx] = lo[s];
        out.sum_rev_hi[idx] = hi[s];
        const double c = static_cast<double>(static_cast<int64_t>(cn[s]));
        out.avg_qty[idx] = static_cast<double>(static_cast<int64_t>(sq[s])) / c;
        out.avg_rev[idx] = gq_i128_to_double(lo[s], hi[s]) / c;
        ++idx;
    }
    if (threadIdx.x == 0) *out.n_groups = total;
}

__global__ void sv_zero_counts_kernel(sv_outs outs, int nq, int topk)
{
    const int q = threadIdx.x;
    if (q >= nq) return;
    if (topk) *outs.o[q].topk_n = 0;
    else *outs.o[q].groups.n_groups = 0;
}

// ------------------------------------------------------------ top-k batch
constexpr int SV_TK_CAP = 512;                        // per-query LDS candidates
constexpr int SV_TK_BATCH = 8;                        // queries per top-k batch kernel
constexpr int SV_TK_MAX_K = SV_TK_CAP - SV_THREADS;   // 256

struct sv_tk_lds {
    uint64_t ok[SV_TK_BATCH][SV_TK_CAP];
    uint32_t rk[SV_TK_BATCH][SV_TK_CAP];
    uint32_t count[SV_TK_BATCH];
    uint64_t th_ok[SV_TK_BATCH];
    uint32_t th_rk[SV_TK_BATCH];
    uint32_t has_th[SV_TK_BATCH];
};

GQ_DEV bool better(uint64_t aok, uint32_t ark, uint64_t bok, uint32_t brk)
{
    return aok > bok || (aok == bok && ark > brk);
}

// sort query q's buffer best-first, keep the best k, set its threshold
GQ_DEV void tk_compact(sv_tk_lds &L, int q, int k)
{
    const int cnt = static_cast<int>(L.count[q]);
    int size = 64;
    while (size < cnt) size <<= 1;
    for (int i = cnt + threadIdx.x; i < size; i += SV_THREADS) {
        L.ok[q][i] = 0;
        L.rk[q][i] = 0;
    }
    __syncthreads();
    for (int kk = 2; kk <= size; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < size / 2; i += SV_THREADS) {
                const int lo = 2 * j * (i / j) + (i % j), hi = lo + j;
                const bool best_first = (lo & kk) == 0;
                const uint64_t aok = L.ok[q][lo], bok = L.ok[q][hi];
                const uint32_t ark = L.rk[q][lo], brk = L.rk[q][hi];
                if (best_first ? better(bok, brk, aok, ark) : better(aok, ark, bok, brk)) {
                    L.ok[q][lo] = bok;
                    L.ok[q][hi] = aok;
                    L.rk[q][lo] = brk;
                    L.rk[q][hi] = ark;
                }
            }
            __syncthreads();
        }
    if (threadIdx.x == 0 && cnt >= k) {
        L.count[q] = static_cast<uint32_t>(k);
        L.th_ok[q] = L.ok[q][k - 1];
        L.th_rk[q] = L.rk[q][k - 1];
        L.has_th[q] = 1;
    }
    __syncthreads();
}

// Stage 1: each block streams a chunk of rows; every row is offered to every
// query of the batch that selects it; the block's best k per query go to
// cand[(q * gridDim.x + block) * k ...].
__global__ __launch_bounds__(SV_THREADS) void sv_topk_local_kernel(gq_serve_tables t, sv_batch b, int k,
                                                                   int64_t chunk, uint64_t *cand_ok,
                                                                   uint32_t *cand_rk, uint32_t *cand_cnt)
{
    __shared__ sv_tk_lds L;
    if (threadIdx.x < SV_TK_BATCH) {
        L.count[threadIdx.x] = 0;
        L.has_th[threadIdx.x] = 0;
        L.th_ok[threadIdx.x] = 0;
        L.th_rk[threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t j1 = j0 + chunk < t.n ? j0 + chunk : t.n;
    for (int64_t s = j0; s < j1; s += SV_THREADS) {
        const int64_t r = s + threadIdx.x;
        const bool valid = r < j1;
        const int32_t date = valid ? t.date[r] : 0;
        const int64_t price = valid ? t.price[r] : 0;
        const uint64_t ok = static_cast<uint64_t>(price) ^ 0x8000000000000000ull;
        const uint32_t rk = 0x7fffffffu - static_cast<uint32_t>(r);
        for (int q = 0; q < b.nq; ++q) {
            if (valid && date < b.hi[q] && (!L.has_th[q] || better(ok, rk, L.th_ok[q], L.th_rk[q]))) {
                const uint32_t slot = atomicAdd(&L.count[q], 1u);
                L.ok[q][slot] = ok;
                L.rk[q][slot] = rk;
            }
        }
        __syncthreads();
        for (int q = 0; q < b.nq; ++q) {
            const uint32_t c = L.count[q];
            __syncthreads();
            if (c > static_cast<uint32_t>(SV_TK_CAP - SV_THREADS)) tk_compact(L, q, k);
        }
    }
    for (int q = 0; q < b.nq; ++q) {
        tk_compact(L, q, k);
        const uint32_t c = L.count[q] < static_cast<uint32_t>(k) ? L.count[q] : static_cast<uint32_t>(k);
        const int64_t o = (static_cast<int64_t>(q) * gridDim.x + blockIdx.x) * k;
        for (uint32_t i = threadIdx.x; i < c; i += SV_THREADS) {
            cand_ok[o + i] = L.ok[q][i];
            cand_rk[o + i] = L.rk[q][i];
        }
        if (threadIdx.x == 0) cand_cnt[q * gridDim.x + blockIdx.x] = c;
        __syncthreads();
    }
}

// Stage 2: block q merges query q's candidates from every stage-1 block.
__global__ __launch_bounds__(SV_THREADS) void sv_topk_merge_kernel(const uint64_t *cand_ok, const uint32_t *cand_rk,
                                                                   const uint32_t *cand_cnt, int nblocks, int k,
                                                                   sv_outs outs)
{
    __shared__ sv_tk_lds L;                                  // uses slot 0 only
    const int q = blockIdx.x;
    if (threadIdx.x == 0) {
        L.count[0] = 0;
        L.has_th[0] = 0;
        L.th_ok[0] = 0;
        L.th_rk[0] = 0;
    }
    __syncthreads();
    const int64_t total = static_cast<int64_t>(nblocks) * k;
    const int64_t o = static_cast<int64_t>(q) * nblocks * k;
    for (int64_t s = 0; s < total; s += SV_THREADS) {
        const int64_t j = s + threadIdx.x;
        if (j < total) {
            const int64_t blk = j / k, i = j % k;
            if (i < static_cast<int64_t>(cand_cnt[q * nblocks + blk])) {
                const uint64_t ok = cand_ok[o + j];
                const uint32_t rk = cand_rk[o + j];
                if (!L.has_th[0] || better(ok, rk, L.th_ok[0], L.th_rk[0])) {
                    const uint32_t slot = atomicAdd(&L.count[0], 1u);
                    L.ok[0][slot] = ok;
                    L.rk[0][slot] = rk;
                }
            }
        }
        __syncthreads();
        const uint32_t c = L.count[0];
        __syncthreads();
        if (c > static_cast<uint32_t>(SV_TK_CAP - SV_THREADS)) tk_compact(L, 0, k);
    }
    tk_compact(L, 0, k);
    const uint32_t c = L.count[0] < static_cast<uint32_t>(k) ? L.count[0] : static_cast<uint32_t>(k);
    for (uint32_t i = threadIdx.x; i < c; i += SV_THREADS) {
        outs.o[q].topk_val[i] = static_cast<int64_t>(L.ok[0][i] ^ 0x8000000000000000ull);
        outs.o[q].topk_row[i] = static_cast<int32_t>(0x7fffffffu - L.rk[0][i]);
    }
    if (threadIdx.x == 0) *outs.o[q].topk_n = c;
}

uint64_t pow2_at_least(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

sv_table table_view(const void *t)
{
    // the join table header stores log2(slots) at byte 8; slots start at 256
    sv_table v;
    v.slots = reinterpret_cast<const int4 *>(static_cast<const char *>(t) + 256);
    v.L = 0;
    return v;
}

}  // namespace

// --------------------------------------------------------------------------
// host side (internal to the library; used by the server)
// --------------------------------------------------------------------------
size_t gq_serve_batch_bytes(const gq_serve_tables &t, const gq_serve_query *q, int nq)
{
    if (nq < 1) return 0;
    gq_carver c(nullptr);
    const int kind = q[0].kind;
    if (kind == GQ_QUERY_FILTER_AGG || kind == GQ_QUERY_JOIN2_AGG) {
        for (int i = 0; i < nq; ++i) {
            const uint64_t S = pow2_at_least(static_cast<uint64_t>(std::max<int64_t>(64, 2 * q[i].max_groups)));
            c.take<uint32_t>(S);
            c.take<int64_t>(S);
            c.take<uint64_t>(S * 3);
            c.take<int64_t>(S);
        }
    } else if (kind == GQ_QUERY_FILTER_TOPK) {
        const int64_t blocks = 512;
        int k = 1;
        for (int i = 0; i < nq; ++i) k = std::max(k, q[i].k);
        c.take<uint64_t>(static_cast<size_t>(SV_TK_BATCH * blocks * k));
        c.take<uint32_t>(static_cast<size_t>(SV_TK_BATCH * blocks * k));
        c.take<uint32_t>(static_cast<size_t>(SV_TK_BATCH * blocks));
    } else {                                                   // JOIN_AGG
        const int64_t n = t.n;
        int64_t mg = 1;
        for (int i = 0; i < nq; ++i) mg = std::max(mg, q[i].max_groups);
        c.take<int32_t>(static_cast<size_t>(n));              // selection
        c.take<int64_t>(8);                                   // counts
        c.take<char>(gq_filter_workspace_bytes(n));
        c.take<int32_t>(static_cast<size_t>(n));              // probe rows
        c.take<int32_t>(static_cast<size_t>(n));              // dim1 attribute
        c.take<char>(gq_join_probe_workspace_bytes(n));
        c.take<char>(gq_groupby_workspace_bytes(n, mg, 0, 1));
    }
    return c.bytes();
}

static sv_outs outs_of(const gq_serve_query *q, int nq)
{
    sv_outs o{};
    for (int i = 0; i < nq; ++i) o.o[i] = q[i].out;
    return o;
}

gq_status gq_serve_batch(gq_ctx *ctx, const gq_serve_tables &t, const gq_serve_query *q, int nq, void *ws,
                         size_t ws_bytes, hipStream_t s)
{
    if (nq < 1 || nq > SV_MAX_BATCH) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "serve batch of %d queries", nq);
    const int kind = q[0].kind;
    for (int i = 1; i < nq; ++i)
        if (q[i].kind != kind) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "serve batch mixes templates");
    if (ws_bytes < gq_serve_batch_bytes(t, q, nq)) return gq_fail(ctx, GQ_ERR_WORKSPACE, "serve batch workspace");
    gq_carver c(ws);
    const sv_outs d_outs = outs_of(q, nq);
    int64_t max_hi = INT32_MIN;
    for (int i = 0; i < nq; ++i) max_hi = std::max(max_hi, q[i].date_hi);
    // three 40 KiB-LDS workgroups per CU; a persistent grid-stride loop over the rows
    const int nb = std::max(1, std::min<int>(ctx->num_cus * 3, static_cast<int>((t.n + SV_TILE - 1) / SV_TILE)));

    if (kind == GQ_QUERY_FILTER_AGG || kind == GQ_QUERY_JOIN2_AGG) {
        for (int i = 0; i < nq; ++i)
            if (q[i].max_groups > SV_MAX_AGG_GROUPS)
                return gq_fail(ctx, GQ_ERR_UNSUPPORTED, "serve aggregate: max_groups <= %d", SV_MAX_AGG_GROUPS);
        int order[SV_MAX_BATCH];
        for (int i = 0; i < nq; ++i) order[i] = i;
        std::stable_sort(order, order + nq, [&](int x, int y) { return q[x].date_hi > q[y].date_hi; });
        sv_batch b{};
        b.nq = nq;
        const size_t zero_from = c.off;
        for (int l = 0; l < nq; ++l) {
            const gq_serve_query &qq = q[order[l]];
            const uint64_t S = pow2_at_least(static_cast<uint64_t>(std::max<int64_t>(64, 2 * qq.max_groups)));
            b.hi[l] = qq.date_hi;
            b.qidx[l] = order[l];
            b.g[l].state = c.take<uint32_t>(S);
            b.g[l].key = c.take<int64_t>(S);
            uint64_t *v = c.take<uint64_t>(S * 3);
            b.g[l].cnt = v;
            b.g[l].sq = v + S;
            b.g[l].lo = v + 2 * S;
            b.g[l].hi = c.take<int64_t>(S);
            b.g[l].mask = S - 1;
        }
        GQ_TRY(gq_zero(ctx, static_cast<char *>(ws) + zero_from, (c.off - zero_from) / 4, s));
        sv_table d1 = table_view(t.dim1_table), d2 = table_view(t.dim2_table);
        d1.L = t.dim1_log2;
        d2.L = t.dim2_log2;
        if (kind == GQ_QUERY_JOIN2_AGG)
            GQ_TRY(gq_launch(ctx, "gq_serve_join2_agg", sv_agg_kernel<true>, dim3(nb), dim3(SV_THREADS), 0, s, t, d1,
                             d2, b, ctx->status_dev));
        else
            GQ_TRY(gq_launch(ctx, "gq_serve_filter_agg", sv_agg_kernel<false>, dim3(nb), dim3(SV_THREADS), 0, s, t,
                             d1, d2, b, ctx->status_dev));
        return gq_launch(ctx, "gq_serve_emit", sv_emit_kernel, dim3(nq), dim3(256), 0, s, b, d_outs,
                         ctx->status_dev);
    }
    if (kind == GQ_QUERY_FILTER_TOPK) {
        int k = 1;
        for (int i = 0; i < nq; ++i) k = std::max(k, q[i].k);
        if (k > SV_TK_MAX_K || nq > SV_TK_BATCH)
            return gq_fail(ctx, GQ_ERR_UNSUPPORTED, "serve top-k: k <= %d and <= %d queries", SV_TK_MAX_K,
                           SV_TK_BATCH);
        for (int i = 0; i < nq; ++i)
            if (q[i].k != k) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "serve top-k batch mixes k");
        const int blocks = 512;
        uint64_t *cok = c.take<uint64_t>(static_cast<size_t>(SV_TK_BATCH * blocks * k));
        uint32_t *crk = c.take<uint32_t>(static_cast<size_t>(SV_TK_BATCH * blocks * k));
        uint32_t *ccnt = c.take<uint32_t>(static_cast<size_t>(SV_TK_BATCH * blocks));
        sv_batch b{};
        b.nq = nq;
        for (int i = 0; i < nq; ++i) b.hi[i] = q[i].date_hi;
        int64_t chunk = (t.n + blocks - 1) / blocks;
        chunk = std::max<int64_t>(SV_THREADS, ((chunk + SV_THREADS - 1) / SV_THREADS) * SV_THREADS);
        GQ_TRY(gq_launch(ctx, "gq_serve_zero", sv_zero_counts_kernel, dim3(1), dim3(64), 0, s, d_outs, nq, 1));
        GQ_TRY(gq_launch(ctx, "gq_serve_topk_local", sv_topk_local_kernel, dim3(blocks), dim3(SV_THREADS), 0, s, t, b,
                         k, chunk, cok, crk, ccnt));
        return gq_launch(ctx, "gq_serve_topk_merge", sv_topk_merge_kernel, dim3(nq), dim3(SV_THREADS), 0, s,
                         static_cast<const uint64_t *>(cok), static_cast<const uint32_t *>(crk),
                         static_cast<const uint32_t *>(ccnt), blocks, k, d_outs);
    }
    // JOIN_AGG: shared filter (date < max_hi) and probe, one filtered group-by per query
    const int64_t n = t.n;
    int64_t mg = 1;
    for (int i = 0; i < nq; ++i) mg = std::max(mg, q[i].max_groups);
    int32_t *sel = c.take<int32_t>(static_cast<size_t>(n));
    int64_t *cnts = c.take<int64_t>(8);
    void *wf = c.take<char>(gq_filter_workspace_bytes(n));
    int32_t *prow = c.take<int32_t>(static_cast<size_t>(n));
    int32_t *attr = c.take<int32_t>(static_cast<size_t>(n));
    void *wp = c.take<char>(gq_join_probe_workspace_bytes(n));
    const size_t gbytes = gq_groupby_workspace_bytes(n, mg, 0, 1);
    void *wg = c.take<char>(gbytes);
    GQ_TRY(gq_filter(ctx, t.date, GQ_I32, n, nullptr, nullptr, INT32_MIN, max_hi, sel, &cnts[0], wf,
                     gq_filter_workspace_bytes(n), s));
    GQ_TRY(gq_join_probe(ctx, t.dim1_table, t.fk, n, &cnts[0], sel, prow, attr, &cnts[1], wp,
                         gq_join_probe_workspace_bytes(n), s));
    for (int i = 0; i < nq; ++i) {
        gq_groupby_in in{};
        in.n = n;
        in.n_dev = &cnts[1];
        in.rowid = prow;
        in.key32 = attr;
        in.qty = t.qty;
        in.price = t.price;
        in.disc = t.disc;
        in.rev_scale = 100;
        in.filter = t.date;
        in.filter_lo = INT32_MIN;
        in.filter_hi = q[i].date_hi;
        GQ_TRY(gq_groupby_agg(ctx, &in, q[i].max_groups, &q[i].out.groups, wg, gbytes, s));
    }
    return GQ_OK;
}

// --------------------------------------------------------------------------
// The plain per-operator form of one query (the serial baseline): the same
// operators a user would chain through the C ABI, one launch chain per query.
// --------------------------------------------------------------------------
namespace {

struct single_ws {
    int32_t *sel, *prow1, *pay1, *prow2, *pay2;
    int64_t *cnts;
    void *wf, *wp1, *wp2, *wg, *wt;
    size_t bf, bp, bg, bt;
};

single_ws single_layout(gq_carver &c, const gq_serve_tables &t, const gq_serve_query &q)
{
    single_ws w{};
    const int64_t n = t.n;
    const size_t rows = static_cast<size_t>(n > 0 ? n : 1);
    w.cnts = c.take<int64_t>(8);
    w.sel = c.take<int32_t>(rows);
    w.bf = gq_filter_workspace_bytes(n);
    w.wf = c.take<char>(w.bf);
    if (q.kind == GQ_QUERY_JOIN_AGG || q.kind == GQ_QUERY_JOIN2_AGG) {
        w.prow1 = c.take<int32_t>(rows);
        w.pay1 = c.take<int32_t>(rows);
        w.bp = gq_join_probe_workspace_bytes(n);
        w.wp1 = c.take<char>(w.bp);
    }
    if (q.kind == GQ_QUERY_JOIN2_AGG) {
        w.prow2 = c.take<int32_t>(rows);
        w.pay2 = c.take<int32_t>(rows);
        w.wp2 = c.take<char>(w.bp);
    }
    if (q.kind == GQ_QUERY_FILTER_TOPK) {
        w.bt = gq_topk_workspace_bytes(n, q.k);
        w.wt = c.take<char>(w.bt);
    } else {
        const bool k64 = q.kind == GQ_QUERY_FILTER_AGG;
        w.bg = gq_groupby_workspace_bytes(n, std::max<int64_t>(1, q.max_groups), k64, !k64);
        w.wg = c.take<char>(w.bg);
    }
    return w;
}

}  // namespace

size_t gq_serve_single_bytes(const gq_serve_tables &t, const gq_serve_query &q)
{
    gq_carver c(nullptr);
    single_layout(c, t, q);
    return c.bytes();
}

gq_status gq_serve_single(gq_ctx *ctx, const gq_serve_tables &t, const gq_serve_query &q, void *ws, size_t ws_bytes,
                          hipStream_t s)
{
    if (ws_bytes < gq_serve_single_bytes(t, q)) return gq_fail(ctx, GQ_ERR_WORKSPACE, "serve single workspace");
    gq_carver c(ws);
    single_ws w = single_layout(c, t, q);
    const int64_t n = t.n;
    GQ_TRY(gq_filter(ctx, t.date, GQ_I32, n, nullptr, nullptr, INT32_MIN, q.date_hi, w.sel, &w.cnts[0], w.wf, w.bf,
                     s));
    if (q.kind == GQ_QUERY_FILTER_TOPK)
        return gq_topk(ctx, t.price, w.sel, n, &w.cnts[0], q.k, 1, q.out.topk_val, q.out.topk_row, q.out.topk_n,
                       w.wt, w.bt, s);
    gq_groupby_in in{};
    in.n = n;
    in.qty = t.qty;
    in.price = t.price;
    in.disc = t.disc;
    in.rev_scale = 100;
    if (q.kind == GQ_QUERY_FILTER_AGG) {
        in.n_dev = &w.cnts[0];
        in.rowid = w.sel;
        in.key64 = t.disc;
        in.key64_by_rowid = 1;
    } else {
        GQ_TRY(gq_join_probe(ctx, t.dim1_table, t.fk, n, &w.cnts[0], w.sel, w.prow1, w.pay1, &w.cnts[1], w.wp1, w.bp,
                             s));
        if (q.kind == GQ_QUERY_JOIN_AGG) {
            in.n_dev = &w.cnts[1];
            in.rowid = w.prow1;
            in.key32 = w.pay1;
        } else {
            GQ_TRY(gq_join_probe(ctx, t.dim2_table, t.fk2, n, &w.cnts[1], w.prow1, w.prow2, w.pay2, &w.cnts[2], w.wp2,
                                 w.bp, s));
            in.n_dev = &w.cnts[2];
            in.rowid = w.prow2;
            in.key32 = w.pay2;
        }
    }
    return gq_groupby_agg(ctx, &in, std::max<int64_t>(1, q.max_groups), &q.out.groups, w.wg, w.bg, s);
}
