// Top-k with ties broken by ascending row id.
//
// Every selected row gets a unique 96-bit order key (ok, rk): ok maps the
// int64 value to an unsigned word whose order is the requested order, and
// rk = 0x7fffffff - rowid ranks smaller row ids higher; the k rows with the
// largest keys are the answer, with no ties left to resolve.
//
// Stage 1 (many workgroups, one pass over the data): each workgroup streams a
// contiguous chunk of the selection; rows whose key beats the workgroup's
// current threshold are appended to an LDS candidate buffer; when the buffer
// could overflow, a radix selection cuts it to the best k and raises the
// threshold to (the leading digits of) the k-th key.  The workgroup's best k
// go to a candidate array.  Row ids are loaded two steps ahead and values one
// step ahead, and the per-step barriers order LDS only, so the loads stay in
// flight.  Stage 2 merges the candidate lists with the same buffer loop:
// first groups of lists in parallel (one workgroup per group, each keeping its
// best k), then one workgroup over the group results, which sorts its best k
// (bitonic) and writes the answer.
#include "gq_device.h"
#include "gq_internal.h"

namespace {

constexpr int TK_THREADS = 512;
constexpr int TK_STEP_ITEMS = 4;
constexpr int TK_STEP = TK_THREADS * TK_STEP_ITEMS;  // rows per step
constexpr int TK_CAP = 4096;                          // LDS candidates
constexpr int TK_MAX_K = TK_CAP - TK_STEP;            // 2048
constexpr uint64_t TK_SIGN = 0x8000000000000000ull;

struct tk_entry {
    uint64_t ok;
    uint32_t rk;
};

GQ_DEV bool tk_better(uint64_t aok, uint32_t ark, uint64_t bok, uint32_t brk)
{
    return aok > bok || (aok == bok && ark > brk);
}

struct tk_lds {
    uint64_t ok[TK_CAP];
    uint32_t rk[TK_CAP];
    uint32_t count;
    uint64_t th_ok;
    uint32_t th_rk;
    uint32_t has_th;
    uint32_t hist[2][256];          // digit counts of the selection, two passes in turn
    uint32_t sel_bin, sel_need, sel_cnt;
    uint32_t scan[TK_THREADS / 64];
};

// Bitonic sort, best first, of the first `size` (power of two) entries.
// Stage (k, j) compares entries lo and lo + j, where lo is the i-th index
// with bit j clear: i with a zero inserted at bit position log2(j) (shifts
// and masks, no integer division).
GQ_DEV void tk_sort(tk_lds &L, int size)
{
    for (int k = 2; k <= size; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < size / 2; i += TK_THREADS) {
                const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const int hi = lo + j;
                const bool best_first = (lo & k) == 0;
                const uint64_t aok = L.ok[lo], bok = L.ok[hi];
                const uint32_t ark = L.rk[lo], brk = L.rk[hi];
                const bool swap = best_first ? tk_better(bok, brk, aok, ark) : tk_better(aok, ark, bok, brk);
                if (swap) {
                    L.ok[lo] = bok;
                    L.ok[hi] = aok;
                    L.rk[lo] = brk;
                    L.rk[hi] = ark;
                }
            }
            gq_lds_barrier();
        }
    }
}

// Sort the first L.count entries, best first.  Block-wide.
GQ_DEV void tk_sort_count(tk_lds &L)
{
    const int cnt = static_cast<int>(L.count);
    int size = 64;
    while (size < cnt) size <<= 1;
    for (int i = cnt + threadIdx.x; i < size; i += TK_THREADS) {
        L.ok[i] = 0;            // (0, 0) ranks below every real entry (rk >= 1)
        L.rk[i] = 0;
    }
    gq_lds_barrier();
    tk_sort(L, size);
}

// Keep the best k entries of the buffer (in no particular order) and raise
// the threshold, by radix selection over the 96-bit keys (ok, then rk),
// eight bits at a time from the top.  A pass counts, among the entries that
// carry the digits chosen so far, how many take each value of the next digit;
// the chosen value is the one at which the count of better entries reaches
// the number still needed.  Once every entry carrying the chosen digits is
// needed, those entries and all better ones are exactly the best k.  The new
// threshold is the chosen digits followed by zero bits: no larger than the
// k-th best key, so no key that belongs in the best k is turned away later.
// Keys are unique (the row part differs), so the selection always ends.
// Block-wide; L.count must be the same in every thread on entry.
constexpr int TK_PER = TK_CAP / TK_THREADS;           // buffer entries per thread

GQ_DEV void tk_select(tk_lds &L, int k)
{
    const uint32_t cnt = L.count;
    if (cnt <= static_cast<uint32_t>(k)) return;
    uint64_t ok[TK_PER];
    uint32_t rk[TK_PER];
    uint32_t valid = 0;
#pragma unroll
    for (int i = 0; i < TK_PER; ++i) {
        const uint32_t e = threadIdx.x + i * TK_THREADS;
        const bool v = e < cnt;
        ok[i] = v ? L.ok[e] : 0;
        rk[i] = v ? L.rk[e] : 0;
        valid |= v ? (1u << i) : 0u;
    }
    for (int i = threadIdx.x; i < 256; i += TK_THREADS) L.hist[0][i] = 0;
    gq_lds_barrier();
    uint64_t p_ok = 0, m_ok = 0;                      // chosen digits and their mask
    uint32_t p_rk = 0, m_rk = 0;
    uint32_t need = static_cast<uint32_t>(k);
    for (int d = 0; d < 12; ++d) {
        uint32_t *h = L.hist[d & 1];
        const int sh = d < 8 ? 56 - 8 * d : 24 - 8 * (d - 8);
#pragma unroll
        for (int i = 0; i < TK_PER; ++i) {
            if (((valid >> i) & 1u) && (ok[i] & m_ok) == p_ok && (rk[i] & m_rk) == p_rk) {
                const uint32_t dig = d < 8 ? static_cast<uint32_t>(ok[i] >> sh) & 255u : (rk[i] >> sh) & 255u;
                atomicAdd(&h[dig], 1u);
            }
        }
        for (int i = threadIdx.x; i < 256; i += TK_THREADS) L.hist[(d + 1) & 1][i] = 0;
        gq_lds_barrier();
        if (threadIdx.x < 64) {                       // one wave finds the digit, from 255 down
            const uint32_t lane = threadIdx.x;
            uint32_t hb[4], sum = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                hb[j] = h[255 - 4 * lane - j];
                sum += hb[j];
            }
            const uint32_t incl = gq_wave_inclusive_scan(sum);
            uint32_t acc = incl - sum;
            if (acc < need && need <= incl) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (acc < need && need <= acc + hb[j]) {
                        L.sel_bin = 255 - 4 * lane - j;
                        L.sel_need = need - acc;
                        L.sel_cnt = hb[j];
                    }
                    acc += hb[j];
                }
            }
        }
        gq_lds_barrier();
        const uint32_t bin = L.sel_bin, c = L.sel_cnt;
        need = L.sel_need;
        if (d < 8) {
            p_ok |= static_cast<uint64_t>(bin) << sh;
            m_ok |= 255ull << sh;
        } else {
            p_rk |= bin << sh;
            m_rk |= 255u << sh;
        }
        if (c == need) break;                         // same in every thread
    }
    // the kept entries: chosen digits at least the prefix
    bool kp[TK_PER];
    uint32_t keep = 0;
#pragma unroll
    for (int i = 0; i < TK_PER; ++i) {
        const uint64_t a = ok[i] & m_ok;
        const uint32_t b = rk[i] & m_rk;
        kp[i] = ((valid >> i) & 1u) && (a > p_ok || (a == p_ok && b >= p_rk));
        keep += kp[i] ? 1u : 0u;
    }
    uint32_t total;
    uint32_t pos = gq_block_exclusive_scan_lds<TK_THREADS>(keep, &total, L.scan);
#pragma unroll
    for (int i = 0; i < TK_PER; ++i) {
        if (kp[i]) {
            L.ok[pos] = ok[i];
            L.rk[pos] = rk[i];
            ++pos;
        }
    }
    if (threadIdx.x == 0) {
        L.count = total;                              // k
        L.th_ok = p_ok;
        L.th_rk = p_rk;
        L.has_th = 1;
    }
    gq_lds_barrier();
}

GQ_DEV void tk_offer(tk_lds &L, bool valid, uint64_t ok, uint32_t rk, uint64_t th_ok, uint32_t th_rk, bool has_th)
{
    if (valid && (!has_th || tk_better(ok, rk, th_ok, th_rk))) {
        const uint32_t slot = atomicAdd(&L.count, 1u);
        L.ok[slot] = ok;
        L.rk[slot] = rk;
    }
}

GQ_DEV uint64_t tk_order(int64_t v, bool desc)
{
    const uint64_t u = static_cast<uint64_t>(v) ^ TK_SIGN;
    return desc ? u : ~u;
}

__global__ __launch_bounds__(TK_THREADS) void topk_stage1_kernel(const int64_t *__restrict__ val,
                                                                 const int32_t *__restrict__ sel, int64_t n_bound,
                                                                 const int64_t *n_dev, int k, int desc,
                                                                 int64_t chunk, uint64_t *__restrict__ cand_ok,
                                                                 uint32_t *__restrict__ cand_rk,
                                                                 uint32_t *__restrict__ cand_cnt)
{
    __shared__ tk_lds L;
    int64_t n = n_bound;
    if (n_dev) {
        const int64_t d = *n_dev;
        n = d < n_bound ? (d > 0 ? d : 0) : n_bound;
    }
    if (threadIdx.x == 0) {
        L.count = 0;
        L.has_th = 0;
        L.th_ok = 0;
        L.th_rk = 0;
    }
    gq_lds_barrier();
    // the chunk of each workgroup, from the device row count when there is one
    // (the host's chunk covers the bound and would leave workgroups idle)
    if (n_dev) {
        const int64_t per = (n + gridDim.x - 1) / gridDim.x;
        chunk = (per + TK_STEP - 1) / TK_STEP * TK_STEP;
        if (chunk < TK_STEP) chunk = TK_STEP;
    }
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * chunk;
    int64_t j1 = j0 + chunk;
    if (j1 > n) j1 = n;
    auto row_at = [&](int64_t j) -> int32_t {
        return j < j1 ? (sel ? __builtin_nontemporal_load(&sel[j]) : static_cast<int32_t>(j)) : 0;
    };
    // pipeline: r0/v0 = step s (offered now), r1/v1 = step s+1, r2 = step s+2
    int32_t r0[TK_STEP_ITEMS], r1[TK_STEP_ITEMS], r2[TK_STEP_ITEMS];
    int64_t v0[TK_STEP_ITEMS], v1[TK_STEP_ITEMS];
#pragma unroll
    for (int c = 0; c < TK_STEP_ITEMS; ++c) {
        r0[c] = row_at(j0 + c * TK_THREADS + threadIdx.x);
        r1[c] = row_at(j0 + TK_STEP + c * TK_THREADS + threadIdx.x);
    }
#pragma unroll
    for (int c = 0; c < TK_STEP_ITEMS; ++c) {
        const int64_t j = j0 + c * TK_THREADS + threadIdx.x;
        v0[c] = j < j1 ? __builtin_nontemporal_load(&val[r0[c]]) : 0;
    }
    for (int64_t s = j0; s < j1; s += TK_STEP) {
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) r2[c] = row_at(s + 2 * TK_STEP + c * TK_THREADS + threadIdx.x);
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) {
            const int64_t j = s + TK_STEP + c * TK_THREADS + threadIdx.x;
            v1[c] = j < j1 ? __builtin_nontemporal_load(&val[r1[c]]) : 0;
        }
        const uint64_t th_ok = L.th_ok;
        const uint32_t th_rk = L.th_rk;
        const bool has_th = L.has_th != 0;
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) {
            const int64_t j = s + c * TK_THREADS + threadIdx.x;
            tk_offer(L, j < j1, tk_order(v0[c], desc), 0x7fffffffu - static_cast<uint32_t>(r0[c]), th_ok, th_rk,
                     has_th);
        }
        gq_lds_barrier();
        const uint32_t cnt_now = L.count;      // same value in every thread
        gq_lds_barrier();
        if (cnt_now > static_cast<uint32_t>(TK_CAP - TK_STEP)) tk_select(L, k);
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) {
            r0[c] = r1[c];
            v0[c] = v1[c];
            r1[c] = r2[c];
        }
    }
    tk_select(L, k);
    const uint32_t cnt = L.count < static_cast<uint32_t>(k) ? L.count : static_cast<uint32_t>(k);
    for (uint32_t i = threadIdx.x; i < cnt; i += TK_THREADS) {
        cand_ok[static_cast<int64_t>(blockIdx.x) * k + i] = L.ok[i];
        cand_rk[static_cast<int64_t>(blockIdx.x) * k + i] = L.rk[i];
    }
    if (threadIdx.x == 0) cand_cnt[blockIdx.x] = cnt;
}

// Merge lists [blockIdx.x * per, +per) of up to k keys each (in any order)
// into the best k; the last level (out_ok == nullptr) sorts them and writes
// the answer.
__global__ __launch_bounds__(TK_THREADS) void topk_merge_kernel(const uint64_t *__restrict__ in_ok,
                                                                const uint32_t *__restrict__ in_rk,
                                                                const uint32_t *__restrict__ in_cnt, int nlists,
                                                                int per, int k, uint64_t *__restrict__ out_ok,
                                                                uint32_t *__restrict__ out_rk,
                                                                uint32_t *__restrict__ out_cnt, int desc,
                                                                int64_t *__restrict__ val_out,
                                                                int32_t *__restrict__ rowid_out, int64_t *n_out)
{
    __shared__ tk_lds L;
    if (threadIdx.x == 0) {
        L.count = 0;
        L.has_th = 0;
        L.th_ok = 0;
        L.th_rk = 0;
    }
    gq_lds_barrier();
    const int b0 = static_cast<int>(blockIdx.x) * per;
    const int b1 = b0 + per < nlists ? b0 + per : nlists;
    const int64_t base = static_cast<int64_t>(b0) * k;
    const int64_t total = b1 > b0 ? static_cast<int64_t>(b1 - b0) * k : 0;
    for (int64_t s = 0; s < total; s += TK_STEP) {
        bool valid[TK_STEP_ITEMS];
        uint64_t ok[TK_STEP_ITEMS];
        uint32_t rk[TK_STEP_ITEMS];
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) {
            const int64_t j = s + c * TK_THREADS + threadIdx.x;
            valid[c] = false;
            ok[c] = 0;
            rk[c] = 0;
            const uint32_t li = static_cast<uint32_t>(j) / static_cast<uint32_t>(k);    // total < 2^31
            if (j < total && static_cast<uint32_t>(j) - li * static_cast<uint32_t>(k) < in_cnt[b0 + li]) {
                valid[c] = true;
                ok[c] = in_ok[base + j];
                rk[c] = in_rk[base + j];
            }
        }
        const uint64_t th_ok = L.th_ok;
        const uint32_t th_rk = L.th_rk;
        const bool has_th = L.has_th != 0;
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) tk_offer(L, valid[c], ok[c], rk[c], th_ok, th_rk, has_th);
        gq_lds_barrier();
        const uint32_t cnt_now = L.count;      // same value in every thread
        gq_lds_barrier();
        if (cnt_now > static_cast<uint32_t>(TK_CAP - TK_STEP)) tk_select(L, k);
    }
    tk_select(L, k);
    const uint32_t cnt = L.count < static_cast<uint32_t>(k) ? L.count : static_cast<uint32_t>(k);
    if (out_ok) {
        for (uint32_t x = threadIdx.x; x < cnt; x += TK_THREADS) {
            out_ok[static_cast<int64_t>(blockIdx.x) * k + x] = L.ok[x];
            out_rk[static_cast<int64_t>(blockIdx.x) * k + x] = L.rk[x];
        }
        if (threadIdx.x == 0) out_cnt[blockIdx.x] = cnt;
        return;
    }
    tk_sort_count(L);                                   // the answer, best first
    for (uint32_t x = threadIdx.x; x < cnt; x += TK_THREADS) {
        const uint64_t o = L.ok[x];
        const uint64_t u = desc ? o : ~o;
        val_out[x] = static_cast<int64_t>(u ^ TK_SIGN);
        rowid_out[x] = static_cast<int32_t>(0x7fffffffu - L.rk[x]);
    }
    if (threadIdx.x == 0) *n_out = cnt;
}

constexpr int TK_MERGE_PER = 48;                      // lists per first-level merge workgroup

struct tk_ws {
    uint64_t *ok, *ok2;
    uint32_t *rk, *rk2;
    uint32_t *cnt, *cnt2;
    int blocks, groups;
    int64_t chunk;
};

tk_ws tk_layout(gq_carver &c, int64_t n, int k, int num_cus)
{
    tk_ws w;
    int64_t blocks = (n + 4 * TK_STEP - 1) / (4 * TK_STEP);     // at least 4 steps per block
    const int64_t maxb = static_cast<int64_t>(num_cus) * 2;    // two 512-thread workgroups fit a CU (95 VGPRs)
    if (blocks > maxb) blocks = maxb;
    if (blocks < 1) blocks = 1;
    int64_t chunk = (n + blocks - 1) / blocks;
    chunk = ((chunk + TK_STEP - 1) / TK_STEP) * TK_STEP;
    if (chunk < TK_STEP) chunk = TK_STEP;
    w.blocks = static_cast<int>(blocks);
    w.groups = blocks > 2 * TK_MERGE_PER ? static_cast<int>((blocks + TK_MERGE_PER - 1) / TK_MERGE_PER) : 0;
    w.chunk = chunk;
    w.ok = c.take<uint64_t>(static_cast<size_t>(blocks) * k);
    w.rk = c.take<uint32_t>(static_cast<size_t>(blocks) * k);
    w.cnt = c.take<uint32_t>(static_cast<size_t>(blocks));
    const size_t g = static_cast<size_t>(w.groups > 0 ? w.groups : 1);
    w.ok2 = c.take<uint64_t>(g * k);
    w.rk2 = c.take<uint32_t>(g * k);
    w.cnt2 = c.take<uint32_t>(g);
    return w;
}

int tk_num_cus_for_layout() { return 256; }

}  // namespace

extern "C" {

size_t gq_topk_workspace_bytes(int64_t n, int k)
{
    if (n < 0) n = 0;
    if (k < 1) k = 1;
    gq_carver c(nullptr);
    tk_layout(c, n, k, tk_num_cus_for_layout());
    return c.bytes();
}

gq_status gq_topk(gq_ctx *ctx, const int64_t *val, const int32_t *sel, int64_t n, const int64_t *n_dev, int k,
                  int descending, int64_t *val_out, int32_t *rowid_out, int64_t *n_out_dev, void *ws,
                  size_t ws_bytes, gq_stream stream)
{
    if (!ctx) return GQ_ERR_INVALID_ARG;
    if (n < 0 || n > GQ_MAX_ROWS) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_topk: n=%lld", (long long)n);
    if (k < 1) return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_topk: k=%d", k);
    if (k > TK_MAX_K) return gq_fail(ctx, GQ_ERR_UNSUPPORTED, "gq_topk: k=%d > %d", k, TK_MAX_K);
    if ((!val && n > 0) || !val_out || !rowid_out || !n_out_dev)
        return gq_fail(ctx, GQ_ERR_INVALID_ARG, "gq_topk: NULL value, output or count");
    const size_t need = gq_topk_workspace_bytes(n, k);
    if (!ws || ws_bytes < need)
        return gq_fail(ctx, GQ_ERR_WORKSPACE, "gq_topk: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gq_carver c(ws);
    tk_ws w = tk_layout(c, n, k, tk_num_cus_for_layout());
    GQ_TRY(gq_launch(ctx, "gq_topk_local", topk_stage1_kernel, dim3(static_cast<uint32_t>(w.blocks)),
                     dim3(TK_THREADS), 0, s, val, sel, n, n_dev, k, descending ? 1 : 0, w.chunk, w.ok, w.rk, w.cnt));
    const int d = descending ? 1 : 0;
    if (w.groups > 0) {
        GQ_TRY(gq_launch(ctx, "gq_topk_merge", topk_merge_kernel, dim3(static_cast<uint32_t>(w.groups)),
                         dim3(TK_THREADS), 0, s, static_cast<const uint64_t *>(w.ok),
                         static_cast<const uint32_t *>(w.rk), static_cast<const uint32_t *>(w.cnt), w.blocks,
                         TK_MERGE_PER, k, w.ok2, w.rk2, w.cnt2, d, val_out, rowid_out, n_out_dev));
        return gq_launch(ctx, "gq_topk_merge", topk_merge_kernel, dim3(1), dim3(TK_THREADS), 0, s,
                         static_cast<const uint64_t *>(w.ok2), static_cast<const uint32_t *>(w.rk2),
                         static_cast<const uint32_t *>(w.cnt2), w.groups, w.groups, k,
                         static_cast<uint64_t *>(nullptr), static_cast<uint32_t *>(nullptr),
                         static_cast<uint32_t *>(nullptr), d, val_out, rowid_out, n_out_dev);
    }
    return gq_launch(ctx, "gq_topk_merge", topk_merge_kernel, dim3(1), dim3(TK_THREADS), 0, s,
                     static_cast<const uint64_t *>(w.ok), static_cast<const uint32_t *>(w.rk),
                     static_cast<const uint32_t *>(w.cnt), w.blocks, w.blocks, k, static_cast<uint64_t *>(nullptr),
                     static_cast<uint32_t *>(nullptr), static_cast<uint32_t *>(nullptr), d, val_out, rowid_out,
                     n_out_dev);
}

}  // extern "C"
