// Device-side primitives for gfx950 (wave64): hashing, wave ballots and
// prefix counts, block scans, decoupled look-back, XCD-aware tile mapping.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#define GQ_DEV __device__ __forceinline__

// 64-bit finalizer of MurmurHash3 (Appleby, public domain).  The partitioning
// function of the shuffle and the hash of every table.
GQ_DEV uint64_t gq_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

// Status-word bits set by kernels (bit = 1 << gq_status code).
GQ_DEV void gq_raise(uint32_t *status, int code) { atomicOr(status, 1u << code); }

// The status code reported for a set of error bits: the first present of
// timeout, duplicate key, invalid key, capacity, invalid argument (codes of
// gq.h), else 0 (GQ_OK).
__host__ __device__ inline int32_t gq_status_of_bits(uint32_t bits)
{
    const int32_t order[] = {8, 4, 7, 2, 1};
    for (int32_t c : order)
        if (bits & (1u << c)) return c;
    return 0;
}

GQ_DEV int gq_lane() { return __lane_id(); }

// Number of set bits of `mask` in lanes below the calling lane.
GQ_DEV uint32_t gq_mbcnt(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

GQ_DEV uint64_t gq_ballot(bool p) { return __ballot(p); }

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (a full __syncthreads() waits for them too).  For
// code whose threads communicate through LDS alone.
GQ_DEV void gq_lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A value every lane of the wave holds (read from LDS after a barrier, say),
// moved to a scalar register so that branches on it are scalar branches.
GQ_DEV int64_t gq_uniform(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(static_cast<uint64_t>(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(static_cast<uint64_t>(v) >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

template <typename T>
GQ_DEV T gq_wave_sum(T v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <typename T>
GQ_DEV T gq_wave_inclusive_scan(T v)
{
    const int lane = gq_lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    return v;
}

// Exclusive scan of one value per thread across a block of NT threads.
// `smem` holds NT/64 elements.  Returns the exclusive prefix, *total the sum.
// Contains two __syncthreads(): every thread of the block must call it.
template <int NT, typename T>
GQ_DEV T gq_block_exclusive_scan(T v, T *total, T *smem)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T inc = gq_wave_inclusive_scan(v);
    if (lane == 63) smem[wave] = inc;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        T s = smem[w];
        pre += (w < wave) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

// The same scan with LDS-only barriers (gq_lds_barrier): outstanding global
// loads and stores of the calling threads stay in flight across it.
template <int NT, typename T>
GQ_DEV T gq_block_exclusive_scan_lds(T v, T *total, T *smem)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T inc = gq_wave_inclusive_scan(v);
    if (lane == 63) smem[wave] = inc;
    gq_lds_barrier();
    T pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        T s = smem[w];
        pre += (w < wave) ? s : T(0);
        tot += s;
    }
    gq_lds_barrier();
    *total = tot;
    return pre + inc - v;
}

// ---------------------------------------------------------------------------
// Decoupled look-back over tiles processed in dynamic (atomic-counter) order.
// Tile status word: bits 62..63 = flag (0 empty, 1 aggregate, 2 inclusive),
// bits 0..61 = value.  Words are read and written with agent-scope atomics,
// which are coherent across the XCDs' separate L2 caches.
// ---------------------------------------------------------------------------
constexpr uint64_t GQ_LB_AGG = 1ull << 62;
constexpr uint64_t GQ_LB_INC = 2ull << 62;
constexpr uint64_t GQ_LB_VAL = (1ull << 62) - 1;

GQ_DEV uint64_t gq_atomic_load64(const uint64_t *p)
{
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

GQ_DEV void gq_atomic_store64(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishing and waiting, separately: a tile can publish its aggregate as
// soon as it is known and wait for its predecessors later.  Both are called
// by all 64 lanes of ONE wave, publish first.
GQ_DEV void gq_lookback_publish(uint64_t *status, uint32_t t, uint64_t agg)
{
    if (gq_lane() == 0) gq_atomic_store64(&status[t], (t == 0 ? GQ_LB_INC : GQ_LB_AGG) | agg);
}

GQ_DEV uint64_t gq_lookback_wait(uint64_t *status, uint32_t t, uint64_t agg);

// Called by all 64 lanes of ONE wave.  Publishes `agg` for tile `t`, waits for
// the predecessors and returns the exclusive prefix of tile t (same value in
// every lane).  Tiles are taken in increasing order from an atomic counter,
// so every predecessor belongs to a running or finished workgroup.
GQ_DEV uint64_t gq_lookback(uint64_t *status, uint32_t t, uint64_t agg)
{
    gq_lookback_publish(status, t, agg);
    return gq_lookback_wait(status, t, agg);
}

// The waiting half: the exclusive prefix of tile t, whose aggregate `agg`
// was published; then publishes t's inclusive value.
GQ_DEV uint64_t gq_lookback_wait(uint64_t *status, uint32_t t, uint64_t agg)
{
    const int lane = gq_lane();
    if (t == 0) return 0;
    uint64_t excl = 0;
    int64_t top = static_cast<int64_t>(t) - 1;        // window = [top-63, top]
    while (true) {
        const int64_t idx = top - lane;
        uint64_t s = (idx >= 0) ? gq_atomic_load64(&status[idx]) : GQ_LB_INC;
        const uint64_t flag = s >> 62;
        const uint64_t not_ready = gq_ballot(flag == 0);
        const uint64_t inc = gq_ballot(flag == 2);
        uint64_t upto;                                   // lanes [0, upto] contribute
        if (inc) {
            const int first = __builtin_ctzll(inc);
            const uint64_t need = (first == 63) ? ~0ull : ((2ull << first) - 1);
            if (not_ready & need) { __builtin_amdgcn_s_sleep(1); continue; }
            upto = static_cast<uint64_t>(first);
            uint64_t v = (static_cast<uint64_t>(lane) <= upto) ? (s & GQ_LB_VAL) : 0;
            excl += gq_wave_sum(v);
            break;
        }
        if (not_ready) { __builtin_amdgcn_s_sleep(1); continue; }
        excl += gq_wave_sum(s & GQ_LB_VAL);
        top -= 64;
    }
    if (lane == 0) gq_atomic_store64(&status[t], GQ_LB_INC | (excl + agg));
    return excl;
}

// ---------------------------------------------------------------------------
// XCD-aware static tile mapping.  Workgroups are dispatched round-robin over
// the 8 XCDs (block b runs on XCD b % 8); this maps blocks so that each XCD
// processes one contiguous range of tiles, which keeps neighbouring tiles'
// partial cache lines in the same L2.  A bijection of [0, nblocks).
// ---------------------------------------------------------------------------
constexpr uint32_t GQ_NUM_XCD = 8;

GQ_DEV uint32_t gq_xcd_tile(uint32_t bid, uint32_t nblocks)
{
    const uint32_t xcd = bid % GQ_NUM_XCD, local = bid / GQ_NUM_XCD;
    const uint32_t q = nblocks / GQ_NUM_XCD, r = nblocks % GQ_NUM_XCD;
    return (xcd < r) ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Two's complement 128-bit value held as (lo, hi).
struct gq_i128 {
    uint64_t lo;
    int64_t hi;
};

// price * (scale - disc), exact in 128 bits.
GQ_DEV gq_i128 gq_revenue(int64_t price, int64_t scale, int64_t disc)
{
    __int128 p = static_cast<__int128>(price);
    __int128 f = static_cast<__int128>(scale) - static_cast<__int128>(disc);
    __int128 r = p * f;
    gq_i128 out;
    out.lo = static_cast<uint64_t>(r);
    out.hi = static_cast<int64_t>(r >> 64);
    return out;
}

// Correctly rounded (nearest-even) conversion of a 128-bit integer to double:
// normalize the magnitude to 64 bits, fold the discarded bits into a sticky
// bit, convert (one rounding), scale by a power of two (exact).
GQ_DEV double gq_i128_to_double(uint64_t lo, int64_t hi)
{
    const bool neg = hi < 0;
    uint64_t mlo = lo, mhi = static_cast<uint64_t>(hi);
    if (neg) {
        mlo = ~mlo + 1;
        mhi = ~mhi + (mlo == 0 ? 1 : 0);
    }
    double d;
    if (mhi == 0) {
        d = static_cast<double>(mlo);
    } else {
        const int sh = 64 - __builtin_clzll(mhi);       // 1..64
        uint64_t top = (sh == 64) ? mhi : ((mhi << (64 - sh)) | (mlo >> sh));
        const uint64_t lost = (sh == 64) ? mlo : (mlo << (64 - sh));
        top |= (lost != 0) ? 1u : 0u;
        d = ldexp(static_cast<double>(top), sh);
    }
    return neg ? -d : d;
}
