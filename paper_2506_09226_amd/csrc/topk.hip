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
// could overflow it is bitonic-sorted, cut to the best k, and the k-th key
// becomes the new threshold.  The workgroup's best k go to a candidate array.
// Stage 2 (one workgroup) runs the same loop over the candidates and writes
// the final sorted answer.
#include "gq_device.h"
#include "gq_internal.h"

namespace {

constexpr int TK_THREADS = 256;
constexpr int TK_STEP_ITEMS = 8;
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
};

// Bitonic sort, best first, of the first `size` (power of two) entries.
GQ_DEV void tk_sort(tk_lds &L, int size)
{
    for (int k = 2; k <= size; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < size / 2; i += TK_THREADS) {
                const int lo = 2 * j * (i / j) + (i % j);
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
            __syncthreads();
        }
    }
}

// Sort the buffer, keep the best k, update the threshold.  Block-wide.
GQ_DEV void tk_compact(tk_lds &L, int k)
{
    const int cnt = static_cast<int>(L.count);
    int size = 64;
    while (size < cnt) size <<= 1;
    for (int i = cnt + threadIdx.x; i < size; i += TK_THREADS) {
        L.ok[i] = 0;            // (0, 0) ranks below every real entry (rk >= 1)
        L.rk[i] = 0;
    }
    __syncthreads();
    tk_sort(L, size);
    if (threadIdx.x == 0) {
        if (cnt >= k) {
            L.count = static_cast<uint32_t>(k);
            L.th_ok = L.ok[k - 1];
            L.th_rk = L.rk[k - 1];
            L.has_th = 1;
        }
    }
    __syncthreads();
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
    __syncthreads();
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * chunk;
    int64_t j1 = j0 + chunk;
    if (j1 > n) j1 = n;
    // software pipeline: the next step's rows are loaded before this step's
    // candidates are offered, so the loads overlap the LDS work and barriers
    int64_t v[TK_STEP_ITEMS], vn[TK_STEP_ITEMS];
    int32_t r[TK_STEP_ITEMS], rn[TK_STEP_ITEMS];
#pragma unroll
    for (int c = 0; c < TK_STEP_ITEMS; ++c) {
        const int64_t j = j0 + c * TK_THREADS + threadIdx.x;
        r[c] = 0;
        v[c] = 0;
        if (j < j1) {
            r[c] = sel ? sel[j] : static_cast<int32_t>(j);
            v[c] = val[r[c]];
        }
    }
    for (int64_t s = j0; s < j1; s += TK_STEP) {
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) {
            const int64_t j = s + TK_STEP + c * TK_THREADS + threadIdx.x;
            rn[c] = 0;
            vn[c] = 0;
            if (j < j1) {
                rn[c] = sel ? sel[j] : static_cast<int32_t>(j);
                vn[c] = val[rn[c]];
            }
        }
        const uint64_t th_ok = L.th_ok;
        const uint32_t th_rk = L.th_rk;
        const bool has_th = L.has_th != 0;
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) {
            const int64_t j = s + c * TK_THREADS + threadIdx.x;
            tk_offer(L, j < j1, tk_order(v[c], desc), 0x7fffffffu - static_cast<uint32_t>(r[c]), th_ok, th_rk,
                     has_th);
        }
        __syncthreads();
        const uint32_t cnt_now = L.count;      // same value in every thread
        __syncthreads();
        if (cnt_now > static_cast<uint32_t>(TK_CAP - TK_STEP)) tk_compact(L, k);
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) {
            v[c] = vn[c];
            r[c] = rn[c];
        }
    }
    tk_compact(L, k);
    const uint32_t cnt = L.count < static_cast<uint32_t>(k) ? L.count : static_cast<uint32_t>(k);
    for (uint32_t i = threadIdx.x; i < cnt; i += TK_THREADS) {
        cand_ok[static_cast<int64_t>(blockIdx.x) * k + i] = L.ok[i];
        cand_rk[static_cast<int64_t>(blockIdx.x) * k + i] = L.rk[i];
    }
    if (threadIdx.x == 0) cand_cnt[blockIdx.x] = cnt;
}

__global__ __launch_bounds__(TK_THREADS) void topk_stage2_kernel(const uint64_t *__restrict__ cand_ok,
                                                                 const uint32_t *__restrict__ cand_rk,
                                                                 const uint32_t *__restrict__ cand_cnt, int nblocks,
                                                                 int k, int desc, int64_t *__restrict__ val_out,
                                                                 int32_t *__restrict__ rowid_out, int64_t *n_out)
{
    __shared__ tk_lds L;
    if (threadIdx.x == 0) {
        L.count = 0;
        L.has_th = 0;
        L.th_ok = 0;
        L.th_rk = 0;
    }
    __syncthreads();
    // walk the candidate array block by block, k entries per source block
    const int64_t total = static_cast<int64_t>(nblocks) * k;
    for (int64_t s = 0; s < total; s += TK_STEP) {
        const uint64_t th_ok = L.th_ok;
        const uint32_t th_rk = L.th_rk;
        const bool has_th = L.has_th != 0;
#pragma unroll
        for (int c = 0; c < TK_STEP_ITEMS; ++c) {
            const int64_t j = s + c * TK_THREADS + threadIdx.x;
            bool valid = false;
            uint64_t ok = 0;
            uint32_t rk = 0;
            if (j < total) {
                const int64_t b = j / k, i = j % k;
                if (i < static_cast<int64_t>(cand_cnt[b])) {
                    valid = true;
                    ok = cand_ok[j];
                    rk = cand_rk[j];
                }
            }
            tk_offer(L, valid, ok, rk, th_ok, th_rk, has_th);
        }
        __syncthreads();
        const uint32_t cnt_now = L.count;      // same value in every thread
        __syncthreads();
        if (cnt_now > static_cast<uint32_t>(TK_CAP - TK_STEP)) tk_compact(L, k);
    }
    tk_compact(L, k);
    const uint32_t cnt = L.count < static_cast<uint32_t>(k) ? L.count : static_cast<uint32_t>(k);
    for (uint32_t i = threadIdx.x; i < cnt; i += TK_THREADS) {
        const uint64_t ok = L.ok[i];
        const uint64_t u = desc ? ok : ~ok;
        val_out[i] = static_cast<int64_t>(u ^ TK_SIGN);
        rowid_out[i] = static_cast<int32_t>(0x7fffffffu - L.rk[i]);
    }
    if (threadIdx.x == 0) *n_out = cnt;
}

struct tk_ws {
    uint64_t *ok;
    uint32_t *rk;
    uint32_t *cnt;
    int blocks;
    int64_t chunk;
};

tk_ws tk_layout(gq_carver &c, int64_t n, int k, int num_cus)
{
    tk_ws w;
    int64_t blocks = (n + 4 * TK_STEP - 1) / (4 * TK_STEP);     // at least 4 steps per block
    const int64_t maxb = static_cast<int64_t>(num_cus) * 3;
    if (blocks > maxb) blocks = maxb;
    if (blocks < 1) blocks = 1;
    int64_t chunk = (n + blocks - 1) / blocks;
    chunk = ((chunk + TK_STEP - 1) / TK_STEP) * TK_STEP;
    if (chunk < TK_STEP) chunk = TK_STEP;
    w.blocks = static_cast<int>(blocks);
    w.chunk = chunk;
    w.ok = c.take<uint64_t>(static_cast<size_t>(blocks) * k);
    w.rk = c.take<uint32_t>(static_cast<size_t>(blocks) * k);
    w.cnt = c.take<uint32_t>(static_cast<size_t>(blocks));
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
    return gq_launch(ctx, "gq_topk_merge", topk_stage2_kernel, dim3(1), dim3(TK_THREADS), 0, s,
                     static_cast<const uint64_t *>(w.ok), static_cast<const uint32_t *>(w.rk),
                     static_cast<const uint32_t *>(w.cnt), w.blocks, k, descending ? 1 : 0, val_out, rowid_out,
                     n_out_dev);
}

}  // extern "C"
