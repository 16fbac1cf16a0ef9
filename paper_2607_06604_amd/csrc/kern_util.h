// kern_util.h - small device helpers shared by the counting kernels.
#pragma once

#include "common.h"

namespace gsn {

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
constexpr int kNumQueues = 8;

__host__ __device__ inline uint32_t lds_align(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

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

// Exclusive scan of one u64 per thread over the work group; ends with a barrier.
template <int BLOCK>
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
    __syncthreads();
    return off + x - v;
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

// Position of the r-th set bit (r < popcount(w)).
__device__ __forceinline__ int select_bit(uint32_t w, int r) {
    int pos = 0, c;
    c = __popc(w & 0xFFFFu); if (r >= c) { r -= c; w >>= 16; pos += 16; }
    c = __popc(w & 0xFFu);   if (r >= c) { r -= c; w >>= 8;  pos += 8; }
    c = __popc(w & 0xFu);    if (r >= c) { r -= c; w >>= 4;  pos += 4; }
    c = __popc(w & 0x3u);    if (r >= c) { r -= c; w >>= 2;  pos += 2; }
    c = __popc(w & 0x1u);    if (r >= c) { pos += 1; }
    return pos;
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

// Next hub from eight label-range queues, starting at this work group's XCD
// (work groups are placed on the eight XCDs round-robin by block index).
// Called by one thread; *qv counts queues found empty. kEmptyKey when done.
__device__ __forceinline__ uint32_t next_hub(uint32_t *queue, uint32_t n, int *qv) {
    const int q0 = blockIdx.x % kNumQueues;
    while (*qv < kNumQueues) {
        const int q = (q0 + *qv) % kNumQueues;
        const uint64_t lo = (uint64_t)n * q / kNumQueues, hi = (uint64_t)n * (q + 1) / kNumQueues;
        const uint32_t v = atomicAdd(&queue[q], 1u);
        if (lo + v < hi) return (uint32_t)(lo + v);
        ++*qv;
    }
    return kEmptyKey;
}

}  // namespace gsn
