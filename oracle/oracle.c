/*
 * oracle.c -- plain, slow, obviously correct CPU reference of the relational
 * hot path (scan/filter, hash partition, equi-join, group-by aggregate, top-k).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file: it is used by the tests, by the smoke check and by the CPU-baseline leg
 * of the benchmark.  It shares no code, header or constant table with the HIP
 * kernels; the two meet only on the seeded synthetic inputs.
 *
 * Single-threaded, written for reading rather than speed.  Every function
 * computes the plain definition of its operator; where the paper fixes only
 * the semantics, the comment says which passage and which reading is used.
 *
 * Precision: all keys, row ids, counts and sums are exact integers; the
 * revenue sum is a two's-complement 128-bit integer (gcc __int128); averages
 * are float64, computed last from the exact integers.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Hash: the 64-bit finalizer of MurmurHash3 (A. Appleby, public domain).    */
/* The paper requires only that every process apply the same partitioning    */
/* function to the key (Sec. 2.2, shuffle description); the finalizer is the  */
/* reading taken for the unnamed "murmur-hash".                               */
/* ------------------------------------------------------------------------ */
uint64_t or_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

static uint64_t rotl64(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }

static uint64_t load_le64(const uint8_t *p)
{
    uint64_t v = 0;
    for (int i = 7; i >= 0; --i) v = (v << 8) | p[i];
    return v;
}

/* MurmurHash3_x64_128 (published algorithm, restated).  Present only so that
 * the tests can pin or_fmix64 against the published SMHasher verification
 * value of the full hash. */
void or_murmur3_x64_128(const void *key, int64_t len, uint32_t seed, uint64_t out[2])
{
    const uint8_t *data = (const uint8_t *)key;
    const uint64_t c1 = 0x87c37b91114253d5ULL, c2 = 0x4cf5ad432745937fULL;
    uint64_t h1 = seed, h2 = seed;
    int64_t nblocks = len / 16;
    for (int64_t i = 0; i < nblocks; ++i) {
        uint64_t k1 = load_le64(data + 16 * i), k2 = load_le64(data + 16 * i + 8);
        k1 *= c1; k1 = rotl64(k1, 31); k1 *= c2; h1 ^= k1;
        h1 = rotl64(h1, 27); h1 += h2; h1 = h1 * 5 + 0x52dce729;
        k2 *= c2; k2 = rotl64(k2, 33); k2 *= c1; h2 ^= k2;
        h2 = rotl64(h2, 31); h2 += h1; h2 = h2 * 5 + 0x38495ab5;
    }
    const uint8_t *tail = data + 16 * nblocks;
    int rem = (int)(len & 15);
    uint64_t k1 = 0, k2 = 0;
    for (int i = rem - 1; i >= 8; --i) k2 ^= (uint64_t)tail[i] << (8 * (i - 8));
    if (rem > 8) { k2 *= c2; k2 = rotl64(k2, 33); k2 *= c1; h2 ^= k2; }
    for (int i = (rem < 8 ? rem : 8) - 1; i >= 0; --i) k1 ^= (uint64_t)tail[i] << (8 * i);
    if (rem > 0) { k1 *= c1; k1 = rotl64(k1, 31); k1 *= c2; h1 ^= k1; }
    h1 ^= (uint64_t)len; h2 ^= (uint64_t)len;
    h1 += h2; h2 += h1;
    h1 = or_fmix64(h1); h2 = or_fmix64(h2);
    h1 += h2; h2 += h1;
    out[0] = h1; out[1] = h2;
}

/* ------------------------------------------------------------------------ */
/* Filter (Sec. 2.2, example plan: inputs are filtered before the join).     */
/* sel = [ r : lo <= col[r] < hi ] in ascending r, optionally restricted to   */
/* the rows listed in sel_in (kept in sel_in's order).                        */
/* ------------------------------------------------------------------------ */
int64_t or_filter(const void *col, int dtype_bytes, int64_t n, int64_t lo, int64_t hi,
                  const int32_t *sel_in, int64_t n_sel_in, int32_t *out)
{
    int64_t cnt = 0;
    int64_t m = sel_in ? n_sel_in : n;
    for (int64_t j = 0; j < m; ++j) {
        int64_t r = sel_in ? (int64_t)sel_in[j] : j;
        int64_t v = dtype_bytes == 4 ? (int64_t)((const int32_t *)col)[r]
                                     : ((const int64_t *)col)[r];
        if (lo <= v && v < hi) out[cnt++] = (int32_t)r;
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Hash partition (Sec. 2.2: every process applies the same partitioning     */
/* function; the receive buffer of a column is contiguous with start offsets */
/* that are exclusive prefix sums of the per-destination sizes).             */
/* bucket(k) = top log2p bits of fmix64(k).  Stable counting sort: rows keep */
/* their input order inside a bucket.  offsets has P+1 entries.              */
/* ------------------------------------------------------------------------ */
static int64_t bucket_of(int64_t key, int log2p)
{
    if (log2p == 0) return 0;
    return (int64_t)(or_fmix64((uint64_t)key) >> (64 - log2p));
}

int or_partition(const int64_t *key, int64_t n, int log2p, int ncols,
                 const void *const *cols, const int32_t *col_bytes,
                 int64_t *key_out, void *const *cols_out, int32_t *rowid_out,
                 int64_t *offsets)
{
    int64_t P = (int64_t)1 << log2p;
    int64_t *count = (int64_t *)calloc((size_t)P, sizeof(int64_t));
    int64_t *cursor = (int64_t *)malloc((size_t)P * sizeof(int64_t));
    if (!count || !cursor) { free(count); free(cursor); return -1; }
    for (int64_t i = 0; i < n; ++i) count[bucket_of(key[i], log2p)]++;
    offsets[0] = 0;
    for (int64_t b = 0; b < P; ++b) offsets[b + 1] = offsets[b] + count[b];
    for (int64_t b = 0; b < P; ++b) cursor[b] = offsets[b];
    for (int64_t i = 0; i < n; ++i) {
        int64_t d = cursor[bucket_of(key[i], log2p)]++;
        key_out[d] = key[i];
        if (rowid_out) rowid_out[d] = (int32_t)i;
        for (int c = 0; c < ncols; ++c) {
            int w = col_bytes[c];
            memcpy((char *)cols_out[c] + d * w, (const char *)cols[c] + i * w, (size_t)w);
        }
    }
    free(count);
    free(cursor);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Equi-join, local (Sec. 2.2: join locally once both sides are partitioned  */
/* on the key).  Inner join of probe rows (fk via sel) with a build side of   */
/* unique keys carrying an int32 payload.  Output pairs (probe row, payload)  */
/* in probe order; unmatched probe rows are dropped.  Sort-merge form.        */
/* Returns the pair count, -1 on a duplicate build key, -2 on no memory.      */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t key; int64_t idx; } kv_t;

static int cmp_kv(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

int64_t or_join_sortmerge(const int64_t *bkey, const int32_t *bpay, int64_t m,
                          const int64_t *fk, const int32_t *sel, int64_t n,
                          int32_t *prow_out, int32_t *pay_out)
{
    kv_t *b = (kv_t *)malloc((size_t)(m ? m : 1) * sizeof(kv_t));
    kv_t *p = (kv_t *)malloc((size_t)(n ? n : 1) * sizeof(kv_t));
    int64_t *match = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    if (!b || !p || !match) { free(b); free(p); free(match); return -2; }
    for (int64_t i = 0; i < m; ++i) { b[i].key = bkey[i]; b[i].idx = i; }
    qsort(b, (size_t)m, sizeof(kv_t), cmp_kv);
    for (int64_t i = 1; i < m; ++i)
        if (b[i].key == b[i - 1].key) { free(b); free(p); free(match); return -1; }
    for (int64_t j = 0; j < n; ++j) {
        int64_t r = sel ? (int64_t)sel[j] : j;
        p[j].key = fk[r]; p[j].idx = j;
        match[j] = -1;
    }
    qsort(p, (size_t)n, sizeof(kv_t), cmp_kv);
    int64_t ib = 0;
    for (int64_t jp = 0; jp < n; ++jp) {
        while (ib < m && b[ib].key < p[jp].key) ++ib;
        if (ib < m && b[ib].key == p[jp].key) match[p[jp].idx] = b[ib].idx;
    }
    int64_t cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (match[j] < 0) continue;
        prow_out[cnt] = sel ? sel[j] : (int32_t)j;
        pay_out[cnt] = bpay[match[j]];
        ++cnt;
    }
    free(b); free(p); free(match);
    return cnt;
}

/* Brute force: nested loops over probe rows and build rows (tiny inputs). */
int64_t or_join_nested(const int64_t *bkey, const int32_t *bpay, int64_t m,
                       const int64_t *fk, const int32_t *sel, int64_t n,
                       int32_t *prow_out, int32_t *pay_out)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = i + 1; k < m; ++k)
            if (bkey[i] == bkey[k]) return -1;
    int64_t cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t r = sel ? (int64_t)sel[j] : j;
        for (int64_t i = 0; i < m; ++i)
            if (bkey[i] == fk[r]) { prow_out[cnt] = (int32_t)r; pay_out[cnt] = bpay[i]; ++cnt; }
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Group-by aggregate (Sec. 2.2/2.4: aggregation after the join and the      */
/* final aggregation).  For input row j the value row is v = rowid[j] (or j); */
/* the key is (key64, key32), each read at j or at v as flagged (a missing    */
/* part is 0).  Per key: count, sum(qty) in wrapping int64, and the exact     */
/* 128-bit sum of price*(rev_scale - disc); then avg_qty = sum_qty/count and  */
/* avg_rev = sum_rev/count in float64, computed last.  Output in ascending     */
/* key order (key64 then key32).  Returns the group count, -1 if it exceeds   */
/* cap, -2 on no memory.                                                       */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t k64; int32_t k32; int64_t j; } gk_t;

static int cmp_gk(const void *a, const void *b)
{
    const gk_t *x = (const gk_t *)a, *y = (const gk_t *)b;
    if (x->k64 != y->k64) return x->k64 < y->k64 ? -1 : 1;
    if (x->k32 != y->k32) return x->k32 < y->k32 ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return 0;
}

typedef struct {
    int64_t n; const int32_t *rowid;
    const int64_t *key64; int key64_by_rowid;
    const int32_t *key32; int key32_by_rowid;
    const int64_t *qty, *price, *disc; int64_t rev_scale;
} or_gb_in;

typedef struct {
    int64_t *key64; int32_t *key32; int64_t *count; int64_t *sum_qty;
    uint64_t *sum_rev_lo; int64_t *sum_rev_hi; double *avg_qty; double *avg_rev;
    int64_t cap;
} or_gb_out;

static void gb_row(const or_gb_in *in, int64_t j, int64_t *k64, int32_t *k32, int64_t *v)
{
    *v = in->rowid ? (int64_t)in->rowid[j] : j;
    *k64 = in->key64 ? in->key64[in->key64_by_rowid ? *v : j] : 0;
    *k32 = in->key32 ? in->key32[in->key32_by_rowid ? *v : j] : 0;
}

static __int128 revenue(const or_gb_in *in, int64_t v)
{
    return (__int128)in->price[v] * ((__int128)in->rev_scale - (__int128)in->disc[v]);
}

static void gb_emit(const or_gb_in *in, or_gb_out *out, int64_t g, int64_t k64, int32_t k32,
                    int64_t cnt, int64_t sq, __int128 sr)
{
    (void)in;
    if (out->key64) out->key64[g] = k64;
    if (out->key32) out->key32[g] = k32;
    out->count[g] = cnt;
    out->sum_qty[g] = sq;
    out->sum_rev_lo[g] = (uint64_t)sr;
    out->sum_rev_hi[g] = (int64_t)(sr >> 64);
    out->avg_qty[g] = (double)sq / (double)cnt;
    out->avg_rev[g] = (double)sr / (double)cnt;
}

int64_t or_groupby_sort(const or_gb_in *in, or_gb_out *out)
{
    int64_t n = in->n;
    gk_t *a = (gk_t *)malloc((size_t)(n ? n : 1) * sizeof(gk_t));
    if (!a) return -2;
    for (int64_t j = 0; j < n; ++j) {
        int64_t v;
        gb_row(in, j, &a[j].k64, &a[j].k32, &v);
        a[j].j = j;
    }
    qsort(a, (size_t)n, sizeof(gk_t), cmp_gk);
    int64_t g = 0;
    for (int64_t s = 0; s < n;) {
        int64_t e = s;
        int64_t cnt = 0, sq = 0;
        __int128 sr = 0;
        while (e < n && a[e].k64 == a[s].k64 && a[e].k32 == a[s].k32) {
            int64_t k64, v; int32_t k32;
            gb_row(in, a[e].j, &k64, &k32, &v);
            cnt += 1;
            sq = (int64_t)((uint64_t)sq + (uint64_t)in->qty[v]);
            sr += revenue(in, v);
            ++e;
        }
        if (g >= out->cap) { free(a); return -1; }
        gb_emit(in, out, g, a[s].k64, a[s].k32, cnt, sq, sr);
        ++g;
        s = e;
    }
    free(a);
    return g;
}

/* Brute force: a linear list of groups searched for every row (tiny inputs);
 * groups come out in first-seen order. */
int64_t or_groupby_linear(const or_gb_in *in, or_gb_out *out)
{
    int64_t g = 0;
    int64_t *cnt = (int64_t *)calloc((size_t)(out->cap ? out->cap : 1), sizeof(int64_t));
    int64_t *sq = (int64_t *)calloc((size_t)(out->cap ? out->cap : 1), sizeof(int64_t));
    __int128 *sr = (__int128 *)calloc((size_t)(out->cap ? out->cap : 1), sizeof(__int128));
    int64_t *gk64 = (int64_t *)calloc((size_t)(out->cap ? out->cap : 1), sizeof(int64_t));
    int32_t *gk32 = (int32_t *)calloc((size_t)(out->cap ? out->cap : 1), sizeof(int32_t));
    if (!cnt || !sq || !sr || !gk64 || !gk32) { g = -2; goto done; }
    for (int64_t j = 0; j < in->n; ++j) {
        int64_t k64, v; int32_t k32;
        gb_row(in, j, &k64, &k32, &v);
        int64_t f = -1;
        for (int64_t q = 0; q < g; ++q)
            if (gk64[q] == k64 && gk32[q] == k32) { f = q; break; }
        if (f < 0) {
            if (g >= out->cap) { g = -1; goto done; }
            f = g++;
            gk64[f] = k64; gk32[f] = k32;
        }
        cnt[f] += 1;
        sq[f] = (int64_t)((uint64_t)sq[f] + (uint64_t)in->qty[v]);
        sr[f] += revenue(in, v);
    }
    for (int64_t q = 0; q < g; ++q) gb_emit(in, out, q, gk64[q], gk32[q], cnt[q], sq[q], sr[q]);
done:
    free(cnt); free(sq); free(sr); free(gk64); free(gk32);
    return g;
}

/* ------------------------------------------------------------------------ */
/* Top-k: the k selected rows with the largest (or smallest) value; equal     */
/* values are ordered by ascending row id; fewer than k rows -> all of them.   */
/* Full-sort form.  Returns the number of rows written.                        */
/* ------------------------------------------------------------------------ */
static int g_desc;

static int cmp_topk(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) {
        int less = x->key < y->key;
        return g_desc ? (less ? 1 : -1) : (less ? -1 : 1);
    }
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

int64_t or_topk_sort(const int64_t *val, const int32_t *sel, int64_t n, int64_t k, int descending,
                     int64_t *val_out, int32_t *rowid_out)
{
    kv_t *a = (kv_t *)malloc((size_t)(n ? n : 1) * sizeof(kv_t));
    if (!a) return -2;
    for (int64_t j = 0; j < n; ++j) {
        int64_t r = sel ? (int64_t)sel[j] : j;
        a[j].key = val[r]; a[j].idx = r;
    }
    g_desc = descending;
    qsort(a, (size_t)n, sizeof(kv_t), cmp_topk);
    int64_t out = n < k ? n : k;
    for (int64_t i = 0; i < out; ++i) { val_out[i] = a[i].key; rowid_out[i] = (int32_t)a[i].idx; }
    free(a);
    return out;
}

/* Brute force: k rounds of a linear scan for the best row not yet taken. */
int64_t or_topk_select(const int64_t *val, const int32_t *sel, int64_t n, int64_t k, int descending,
                       int64_t *val_out, int32_t *rowid_out)
{
    char *taken = (char *)calloc((size_t)(n ? n : 1), 1);
    if (!taken) return -2;
    int64_t out = n < k ? n : k;
    for (int64_t i = 0; i < out; ++i) {
        int64_t best = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (taken[j]) continue;
            if (best < 0) { best = j; continue; }
            int64_t rj = sel ? sel[j] : j, rb = sel ? sel[best] : best;
            int64_t vj = val[rj], vb = val[rb];
            int better = descending ? (vj > vb) : (vj < vb);
            if (better || (vj == vb && rj < rb)) best = j;
        }
        taken[best] = 1;
        int64_t rb = sel ? sel[best] : best;
        val_out[i] = val[rb];
        rowid_out[i] = (int32_t)rb;
    }
    free(taken);
    return out;
}
