// kern_util.h - small device helpers shared by the counting kernels.
#pragma once

#include "common.h"

namespace gsn {

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
constexpr int kNumQueues = 8;

__host__ __device__ inline uint32_t lds_align(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

// Pointers with their address space spelled out: global rows whose loads
// take a scalar base and a 32-bit lane offset, and LDS words addressed by
// absolute byte address (no per-access base add).
typedef __attribute__((address_space(1))) const uint32_t gbl_u32;
typedef __attribute__((address_space(1))) const uint8_t gbl_u8;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) const uint16_t lds_u16;

// Byte address of an LDS location.
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(size_t)(__attribute__((address_space(3))) const void *)p;
}

// A value the whole wavefront holds alike, moved to scalar registers (so a
// pointer built from it can serve as the scalar base of vector loads).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Fibonacci hash of a label into a table of 2^log2h slots.
__device__ __forceinline__ uint32_t label_hash(uint32_t k, int log2h) {
    return (k * 2654435769u) >> (32 - log2h);
}

// Exclusive scan of one u32 per thread over the work group (BLOCK a multiple
// of 64); ends with a barrier so wtot can be reused by the next call.
template <int BLOCK>
__device__ __forceinline__ uint32_t wg_excl_scan(uint32_t v, uint32_t *wtot, uint32_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wtot[wid] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) {
        uint32_t t = wtot[k];
        off += (k < wid) ? t : 0u;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return off + x - v;
}

// Exclusive scan of one u64 per thread over the work group. With TRAIL it
// ends with a barrier so that wtot can be reused at once; without, the
// caller puts a barrier between this call and the next write of wtot.
template <int BLOCK, bool TRAIL = true>
__device__ __forceinline__ uint64_t wg_excl_scan64(uint64_t v, uint64_t *wtot, uint64_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wtot[wid] = x;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) {
        uint64_t t = wtot[k];
        off += (k < wid) ? t : 0ull;
        tot += t;
    }
    total = tot;
    if (TRAIL) __syncthreads();
    return off + x - v;
}

// ---- exact weighted sums ----
// A tuple's weight term is x = +-(product of weight magnitudes) * 2^s, an
// integer below 2^87 (the scale s makes the smallest possible product an
// integer of 53 bits; the weight range check bounds the largest). Sums are
// signed 128-bit integers kept as (lo, hi) 64-bit words, two's complement.

// 128-bit two's complement add into a (lo, hi) pair of global words.
__device__ __forceinline__ void add128_words(unsigned long long *dst, __int128 v) {
    const unsigned long long lo = (unsigned long long)v;
    unsigned long long hi = (unsigned long long)((unsigned __int128)v >> 64);
    const unsigned long long old = atomicAdd(&dst[0], lo);
    if (old + lo < old) hi += 1;
    if (hi) atomicAdd(&dst[1], hi);
}

constexpr double kTwo63 = 9223372036854775808.0;

// Narrow terms (magnitude below 2^63) as one signed 64-bit integer.
__device__ __forceinline__ bool narrow_term(double x) { return x < kTwo63; }

// A term as a signed 128-bit integer: x = h * 2^32 + l with h = trunc(x 2^-32)
// and l = x - h 2^32, both exact (x is an integer, l < 2^32 is representable).
__device__ __forceinline__ __int128 wide_term(double x, bool neg) {
    const double h = trunc(__dmul_rn(x, 0x1.0p-32));
    const double l = __dsub_rn(x, __dmul_rn(h, 0x1.0p32));
    const __int128 v = ((__int128)(long long)h << 32) + (__int128)(long long)l;
    return neg ? -v : v;
}

// A positive term known to lie in [2^52, 2^63) -- the scale puts every
// product of weight magnitudes at or above 2^52, and narrow terms stay below
// 2^63 -- as a 64-bit integer: its significand shifted left by its exponent
// less 52 (0..10). Equal to the truncating conversion on that range, in four
// integer instructions.
__device__ __forceinline__ unsigned long long big_term_u64(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const uint32_t sh = (uint32_t)(b >> 52) - 1075u;
    return ((b & 0xFFFFFFFFFFFFFull) | 0x10000000000000ull) << sh;
}

// A narrow term into LDS sums: its low 32 bits and its arithmetic high part
// (term = high * 2^32 + low), each summed in 64 bits (room for 2^32 terms).
__device__ __forceinline__ void lds_term(unsigned long long *lo, unsigned long long *hi, long long t) {
    atomicAdd(lo, (unsigned long long)t & 0xFFFFFFFFull);
    atomicAdd(hi, (unsigned long long)(t >> 32));
}

// The 128-bit value of a pair of LDS sums.
__device__ __forceinline__ __int128 lds_sum128(unsigned long long lo, unsigned long long hi) {
    return ((__int128)(long long)hi << 32) + (__int128)lo;
}

// Lanes below this one with their bit set in the 64-bit wave mask.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Order LDS accesses of one wavefront (program order within the wave).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Largest k in [0, n) with pref[k] <= x, given pref[n] > x and pref non-decreasing.
__device__ __forceinline__ uint32_t upper_index(const uint32_t *pref, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (pref[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Hubs are handed out from eight label-range queues, one per slice of the
// hub range; a team (a work group, or one wavefront) starts on the queue of
// its own XCD (work groups are placed on the eight XCDs round-robin by block
// index) so nearby hubs share that XCD's L2, and moves on to the other queues
// once its own is empty. Each counter sits in a 256-byte line of its own so
// that the eight never contend for one line, and a team claims a run of
// consecutive hubs per atomic: the run is an eighth of the queue's remaining
// share per team, at most kMaxRun (guided self-scheduling), so the number of
// atomics grows with the log of the hub count rather than with the count,
// while the last hubs still go out one at a time.
constexpr int kQueueStride = 64;                       // u32 words between counters
constexpr int kQueueWords = kNumQueues * kQueueStride;  // words per queue set
constexpr uint32_t kMaxRun = 32;

struct HubCursor {
    uint32_t cur = 0, end = 0;  // unclaimed part of the current run
    uint32_t run = 0;           // length of the next claim (0: from the queue's full share)
    int qv = 0;                 // queues found empty
};

// Next hub of [h0, h1) for the calling thread (one per team), or kEmptyKey.
// teams: how many teams draw from these queues; max_run caps a claim (1 for
// hubs whose costs vary too much to hand out in runs).
__device__ __forceinline__ uint32_t next_hub_in(uint32_t *queue, uint32_t h0, uint32_t h1, uint32_t teams,
                                                HubCursor &c, uint32_t max_run = kMaxRun) {
    if (c.cur < c.end) return c.cur++;
    const int q0 = blockIdx.x % kNumQueues;
    const uint64_t n = (uint64_t)(h1 - h0);
    const uint64_t per_queue = (teams + kNumQueues - 1) / kNumQueues;
    while (c.qv < kNumQueues) {
        const int q = (q0 + c.qv) % kNumQueues;
        const uint64_t lo = h0 + n * q / kNumQueues, hi = h0 + n * (q + 1) / kNumQueues;
        if (c.run == 0)
            c.run = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(max_run, (hi - lo) / (8 * per_queue)));
        const uint32_t v = atomicAdd(&queue[q * kQueueStride], c.run);
        if (lo + v < hi) {
            const uint64_t first = lo + v, last = std::min<uint64_t>(first + c.run, hi);
            c.cur = (uint32_t)first + 1;
            c.end = (uint32_t)last;
            const uint64_t left = hi - last;
            c.run = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(max_run, left / (8 * per_queue)));
            return (uint32_t)first;
        }
        ++c.qv;
        c.run = 1;
    }
    return kEmptyKey;
}

// Make sure the cursor holds unclaimed hubs: false once every queue is
// empty, else the caller owns hubs [c.cur, c.end) (consecutive labels) and
// takes some of them by advancing c.cur.
__device__ __forceinline__ bool next_hub_run(uint32_t *queue, uint32_t h0, uint32_t h1, uint32_t teams,
                                             HubCursor &c) {
    if (c.cur < c.end) return true;
    const uint32_t v = next_hub_in(queue, h0, h1, teams, c);
    if (v == kEmptyKey) return false;
    c.cur = v;  // hand the first hub of the new run back
    return true;
}

}  // namespace gsn
