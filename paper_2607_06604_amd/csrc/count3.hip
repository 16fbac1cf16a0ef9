// count3.hip - binned triangle counts on the forward CSR (paper Sec. 2.2
// hub-and-spoke enumeration, Sec. 3.1 sorted-list intersection, Sec. 3.5.2
// one work group per hub with lanes on the inner loop).
//
// Every triangle {i < j < k} (labels) is found exactly once: at hub i, spoke
// j in N+(i), third vertex k in N+(i) and N+(j). The work group of a hub
// stages N+(i) in an LDS hash table (label -> bin of edge (i,k)), then
// streams the forward rows of all its spokes as one flat, coalesced sequence;
// each lane probes one candidate k. A hit has its three bins (ij from the
// spoke, ik from the table, jk from the row), which are sorted and ranked
// into an LDS histogram of 32-bit counters, flushed into the 64-bit result
// before any counter could wrap.
//
// Hubs are pulled from eight queues, one per XCD-sized slice of the label
// range; a work group starts on the queue of its own XCD (blockIdx % 8, the
// hardware's round-robin placement) so nearby hubs share that XCD's L2, and
// moves on to the other queues once its own is empty.
#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace gsn {
namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr int kQueues = 8;

struct C3Args {
    const uint64_t *rp;
    const uint32_t *col;
    const uint8_t *bin;
    const double *w;        // label-ordered weights (weighted)
    const uint32_t *perm;   // label -> original index (anchored)
    uint32_t n;
    int nb, nconf, log2h;
    uint32_t maxdeg;
    uint32_t anchor_lo, anchor_hi;
    double wmul;            // 2^wscale
    uint64_t flush_limit;   // flush LDS counters before this many increments
    uint32_t *queue;        // kQueues counters
    unsigned long long *hist;   // nconf
    unsigned long long *wsum;   // 2*nconf (lo, hi)
    unsigned long long *ntri;   // 1
};

// LDS layout of one work group (byte offsets).
struct Layout3 {
    uint32_t hkey, hbin, hslot, mstart, mpref, mbin, mw, mperm, hist, wlo, whi, tab, wtot, misc, total;
};

__host__ __device__ inline uint32_t align_up(uint32_t x, uint32_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline Layout3 layout3(int block, uint32_t H, uint32_t maxdeg, int nconf, int nb,
                                           bool weighted, bool anchored, bool lds_hist) {
    if (!lds_hist) nconf = 0;
    Layout3 L{};
    uint32_t o = 0;
    L.hkey = o;   o = align_up(o + 4 * H, 16);
    L.hbin = o;   o = align_up(o + H, 16);
    L.hslot = o;  o = align_up(o + 2 * (maxdeg + 1), 16);
    L.mstart = o; o = align_up(o + 8 * block, 16);
    L.mpref = o;  o = align_up(o + 4 * (block + 1), 16);
    L.mbin = o;   o = align_up(o + block, 16);
    L.mw = o;     if (weighted) o = align_up(o + 8 * block, 16);
    L.mperm = o;  if (anchored) o = align_up(o + 4 * block, 16);
    L.hist = o;   o = align_up(o + 4 * nconf, 16);
    L.wlo = o;    if (weighted) o = align_up(o + 8 * nconf, 16);
    L.whi = o;    if (weighted) o = align_up(o + 8 * nconf, 16);
    L.tab = o;    o = align_up(o + 8 * (nb + 1), 16);
    L.wtot = o;   o = align_up(o + 4 * (block / 64 + 1), 16);
    L.misc = o;   o = align_up(o + 16, 16);
    L.total = o;
    return L;
}

__device__ __forceinline__ uint32_t hash_slot(uint32_t k, int log2h) {
    return (k * 2654435769u) >> (32 - log2h);
}

// Exclusive block scan of u32 values (block a multiple of 64).
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wtot, uint32_t &total) {
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
    return off + x - v;
}

// 128-bit add into a (lo, hi) pair of global words.
__device__ __forceinline__ void add128(unsigned long long *dst, unsigned __int128 v) {
    unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    unsigned long long old = atomicAdd(&dst[0], lo);
    if (old + lo < old) hi += 1;
    if (hi) atomicAdd(&dst[1], hi);
}

template <int BLOCK, bool WEIGHTED, bool LDS_HIST>
__device__ void flush3(const C3Args &a, const Layout3 &L, unsigned char *sm) {
    if (!LDS_HIST) return;
    uint32_t *hist = (uint32_t *)(sm + L.hist);
    for (int b = threadIdx.x; b < a.nconf; b += BLOCK) {
        uint32_t v = hist[b];
        if (v) {
            atomicAdd(&a.hist[b], (unsigned long long)v);
            hist[b] = 0;
        }
        if (WEIGHTED) {
            unsigned long long *wlo = (unsigned long long *)(sm + L.wlo);
            unsigned long long *whi = (unsigned long long *)(sm + L.whi);
            unsigned long long lo = wlo[b], hi = whi[b];
            if (lo | hi) {
                unsigned __int128 V = ((unsigned __int128)hi << 32) + (unsigned __int128)lo;
                add128(&a.wsum[2 * b], V);
                wlo[b] = 0;
                whi[b] = 0;
            }
        }
    }
}

template <int BLOCK, bool WEIGHTED, bool ANCHORED, bool LDS_HIST>
__global__ __launch_bounds__(BLOCK) void k_count3(C3Args a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const uint32_t H = 1u << a.log2h, mask = H - 1;
    const Layout3 L = layout3(BLOCK, H, a.maxdeg, a.nconf, a.nb, WEIGHTED, ANCHORED, LDS_HIST);
    uint32_t *hkey = (uint32_t *)(sm + L.hkey);
    uint8_t *hbin = (uint8_t *)(sm + L.hbin);
    uint16_t *hslot = (uint16_t *)(sm + L.hslot);
    unsigned long long *mstart = (unsigned long long *)(sm + L.mstart);
    uint32_t *mpref = (uint32_t *)(sm + L.mpref);
    uint8_t *mbin = (uint8_t *)(sm + L.mbin);
    double *mw = (double *)(sm + L.mw);
    uint32_t *mperm = (uint32_t *)(sm + L.mperm);
    uint32_t *hist = (uint32_t *)(sm + L.hist);
    unsigned long long *wlo = (unsigned long long *)(sm + L.wlo);
    unsigned long long *whi = (unsigned long long *)(sm + L.whi);
    int *ta = (int *)(sm + L.tab);
    int *tb = ta + (a.nb + 1);
    uint32_t *wtot = (uint32_t *)(sm + L.wtot);
    uint32_t *s_hub = (uint32_t *)(sm + L.misc);
    unsigned long long *s_cnt = (unsigned long long *)(sm + L.misc + 8);
    const int tid = threadIdx.x;

    for (uint32_t s = tid; s < H; s += BLOCK) hkey[s] = kEmpty;
    if (LDS_HIST)
        for (int b = tid; b < a.nconf; b += BLOCK) {
            hist[b] = 0;
            if (WEIGHTED) { wlo[b] = 0; whi[b] = 0; }
        }
    for (int b = tid; b < a.nb; b += BLOCK) {
        ta[b] = rank_a(a.nb, b);
        tb[b] = rank_b(a.nb, b);
    }
    if (tid == 0) *s_cnt = 0;
    __syncthreads();

    unsigned long long mytri = 0;
    uint64_t acc = 0;   // upper bound on increments since the last flush (uniform)
    const int q0 = blockIdx.x % kQueues;
    int qv = 0;         // queues exhausted so far (thread 0)

    while (true) {
        if (tid == 0) {
            uint32_t hub = kEmpty;
            while (qv < kQueues) {
                const int q = (q0 + qv) % kQueues;
                const uint64_t lo = (uint64_t)a.n * q / kQueues, hi = (uint64_t)a.n * (q + 1) / kQueues;
                const uint32_t v = atomicAdd(&a.queue[q], 1u);
                if (lo + v < hi) { hub = (uint32_t)(lo + v); break; }
                ++qv;
            }
            *s_hub = hub;
        }
        __syncthreads();
        const uint32_t i = *s_hub;
        if (i == kEmpty) break;
        const uint64_t beg = a.rp[i];
        const uint32_t d = (uint32_t)(a.rp[i + 1] - beg);
        if (d < 2) { __syncthreads(); continue; }
        double wi = 0.0;
        uint32_t pi = 0;
        if (WEIGHTED) wi = a.w[i];
        if (ANCHORED) pi = a.perm[i];

        // stage N+(i): label -> bin of (i, k)
        for (uint32_t e = tid; e < d; e += BLOCK) {
            const uint32_t k = a.col[beg + e];
            uint32_t s = hash_slot(k, a.log2h);
            while (atomicCAS(&hkey[s], kEmpty, k) != kEmpty) s = (s + 1) & mask;
            hbin[s] = a.bin[beg + e];
            hslot[e] = (uint16_t)s;
        }
        __syncthreads();

        // spokes in chunks of BLOCK; the last spoke cannot close a triangle
        for (uint32_t c0 = 0; c0 + 1 < d; c0 += BLOCK) {
            const uint32_t sidx = c0 + tid;
            uint32_t len = 0;
            uint64_t st = 0;
            if (sidx + 1 < d) {
                const uint32_t j = a.col[beg + sidx];
                st = a.rp[j];
                len = (uint32_t)(a.rp[j + 1] - st);
                mbin[tid] = a.bin[beg + sidx];
                if (WEIGHTED) mw[tid] = a.w[j];
                if (ANCHORED) mperm[tid] = a.perm[j];
            }
            uint32_t total;
            const uint32_t pre = block_excl_scan<BLOCK>(len, wtot, total);
            mstart[tid] = st;
            mpref[tid] = pre;
            if (tid == 0) mpref[BLOCK] = total;
            if (acc + total >= a.flush_limit) {
                __syncthreads();
                flush3<BLOCK, WEIGHTED, LDS_HIST>(a, L, sm);
                acc = 0;
            }
            acc += total;
            __syncthreads();

            uint32_t sp = 0;
            for (uint32_t e0 = 0; e0 < total; e0 += BLOCK) {
                const uint32_t e = e0 + tid;
                if (e < total) {
                    while (mpref[sp + 1] <= e) ++sp;
                    const uint64_t pos = mstart[sp] + (e - mpref[sp]);
                    const uint32_t k = a.col[pos];
                    uint32_t h = hash_slot(k, a.log2h);
                    uint32_t key;
                    while ((key = hkey[h]) != k && key != kEmpty) h = (h + 1) & mask;
                    if (key == k) {
                        bool take = true;
                        if (ANCHORED) {
                            uint32_t m = min(pi, min(mperm[sp], a.perm[k]));
                            take = m >= a.anchor_lo && m < a.anchor_hi;
                        }
                        if (take) {
                            const int x = mbin[sp], y = hbin[h], z = a.bin[pos];
                            const int lo = min(x, min(y, z)), hi = max(x, max(y, z));
                            const int mid = x + y + z - lo - hi;
                            const int idx = ta[lo] + tb[mid] + hi;
                            if (LDS_HIST) atomicAdd(&hist[idx], 1u);
                            else atomicAdd(&a.hist[idx], 1ull);
                            ++mytri;
                            if (WEIGHTED) {
                                double p = wi, q = mw[sp], r = a.w[k], t;
                                if (p > q) { t = p; p = q; q = t; }
                                if (q > r) { t = q; q = r; r = t; }
                                if (p > q) { t = p; p = q; q = t; }
                                const double prod = __dmul_rn(__dmul_rn(p, q), r);
                                const unsigned long long ti =
                                    (unsigned long long)__dmul_rn(prod, a.wmul);
                                if (LDS_HIST) {
                                    atomicAdd(&wlo[idx], ti & 0xFFFFFFFFull);
                                    atomicAdd(&whi[idx], ti >> 32);
                                } else {
                                    add128(&a.wsum[2 * idx], (unsigned __int128)ti);
                                }
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        for (uint32_t e = tid; e < d; e += BLOCK) hkey[hslot[e]] = kEmpty;
        __syncthreads();
    }

    __syncthreads();
    flush3<BLOCK, WEIGHTED, LDS_HIST>(a, L, sm);
    if (mytri) atomicAdd(s_cnt, mytri);
    __syncthreads();
    if (tid == 0 && *s_cnt) atomicAdd(a.ntri, *s_cnt);
}

__global__ void k_zero_u64(unsigned long long *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int BLOCK, bool W, bool A, bool LH>
void launch3(Ctx &ctx, const C3Args &a, uint32_t lds) {
    const void *kern = reinterpret_cast<const void *>(&k_count3<BLOCK, W, A, LH>);
    if (lds > 65536)
        GS_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count3<BLOCK, W, A, LH>, BLOCK, lds));
    if (per_cu < 1) fail(GS_EUNSUPPORTED, "count kernel does not fit a compute unit");
    uint32_t grid = (uint32_t)ctx.n_cu * (uint32_t)per_cu;
    grid = (grid + kQueues - 1) / kQueues * kQueues;
    k_count3<BLOCK, W, A, LH><<<dim3(grid), dim3(BLOCK), lds, ctx.stream>>>(a);
    GS_HIP(hipGetLastError());
}

template <int BLOCK, bool LH>
void launch3_any(Ctx &ctx, const C3Args &a, uint32_t lds, bool w, bool an) {
    if (!w && !an) launch3<BLOCK, false, false, LH>(ctx, a, lds);
    else if (w && !an) launch3<BLOCK, true, false, LH>(ctx, a, lds);
    else if (!w && an) launch3<BLOCK, false, true, LH>(ctx, a, lds);
    else launch3<BLOCK, true, true, LH>(ctx, a, lds);
}

}  // namespace

void count3_run(Ctx &ctx, const Graph &g, uint64_t *hist, uint64_t *wsum, uint64_t *ntri,
                const gs_anchor_range *anchors) {
    const int nb = g.nbins;
    const int nconf = (int)n_configs(nb);
    const bool weighted = wsum != nullptr;
    bool anchored = anchors != nullptr;
    if (anchored && (anchors->lo > anchors->hi)) fail(GS_EINVAL, "anchor range lo > hi");
    const uint32_t maxdeg = g.max_deg;
    if (maxdeg > 16384) fail(GS_EUNSUPPORTED, "forward degree above 16384");
    uint32_t H = 64;
    int log2h = 6;
    while (H < 2 * maxdeg) { H <<= 1; ++log2h; }
    const int block = 256;
    // per-work-group LDS histograms while they fit; global atomics beyond
    bool lds_hist = nconf <= 8192;
    Layout3 L = layout3(block, H, maxdeg, nconf, nb, weighted, anchored, lds_hist);
    if ((int)L.total > ctx.max_lds && lds_hist) {
        lds_hist = false;
        L = layout3(block, H, maxdeg, nconf, nb, weighted, anchored, lds_hist);
    }
    if ((int)L.total > ctx.max_lds) fail(GS_EUNSUPPORTED, "LDS footprint too large for this degree");

    // device staging: hist | wsum | ntri | queues
    const size_t words = (size_t)nconf + 2 * (size_t)nconf + 1 + kQueues;
    unsigned long long *dv = (unsigned long long *)ctx.scratch_get(words * 8);
    C3Args a{};
    a.rp = g.row_ptr.as<uint64_t>();
    a.col = g.col.as<uint32_t>();
    a.bin = g.bin.as<uint8_t>();
    a.w = weighted ? g.weights.as<double>() : nullptr;
    a.perm = g.perm.as<uint32_t>();
    a.n = (uint32_t)g.n;
    a.nb = nb;
    a.nconf = nconf;
    a.log2h = log2h;
    a.maxdeg = maxdeg;
    a.anchor_lo = anchored ? (uint32_t)std::min<uint64_t>(anchors->lo, 0xFFFFFFFFull) : 0;
    a.anchor_hi = anchored ? (uint32_t)std::min<uint64_t>(anchors->hi, 0xFFFFFFFFull) : 0;
    a.wmul = std::ldexp(1.0, g.wscale);
    // GS_FLUSH_LIMIT lowers the flush threshold (exercises the flush path)
    const char *fl = getenv("GS_FLUSH_LIMIT");
    a.flush_limit = fl ? strtoull(fl, nullptr, 10) : 0xFFFFFFFFull;
    if (a.flush_limit < (uint64_t)block * (maxdeg + 1) || a.flush_limit > 0xFFFFFFFFull)
        a.flush_limit = 0xFFFFFFFFull;
    a.hist = dv;
    a.wsum = dv + nconf;
    a.ntri = dv + 3 * (size_t)nconf;
    a.queue = (uint32_t *)(dv + 3 * (size_t)nconf + 1);

    hipStream_t s = ctx.stream;
    GS_HIP(hipEventRecord(ctx.ev[0], s));
    k_zero_u64<<<64, 256, 0, s>>>(dv, words);
    GS_HIP(hipEventRecord(ctx.ev[2], s));
    if (g.n > 0) {
        if (lds_hist) launch3_any<256, true>(ctx, a, L.total, weighted, anchored);
        else launch3_any<256, false>(ctx, a, L.total, weighted, anchored);
    }
    GS_HIP(hipEventRecord(ctx.ev[3], s));
    std::vector<unsigned long long> h(3 * (size_t)nconf + 1);
    GS_HIP(hipMemcpyAsync(h.data(), dv, h.size() * 8, hipMemcpyDeviceToHost, s));
    GS_HIP(hipEventRecord(ctx.ev[1], s));
    GS_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < nconf; ++c) hist[c] = h[c];
    if (weighted)
        for (int c = 0; c < 2 * nconf; ++c) wsum[c] = h[nconf + c];
    *ntri = h[3 * (size_t)nconf];
    float ms = 0, kms = 0;
    GS_HIP(hipEventElapsedTime(&ms, ctx.ev[0], ctx.ev[1]));
    GS_HIP(hipEventElapsedTime(&kms, ctx.ev[2], ctx.ev[3]));
    ctx.t.count_ms = ms;
    ctx.t.kernel_ms = kms;
    ctx.t.kernel_launches = g.n > 0 ? 1 : 0;
    // merge-walk bytes: each hub-spoke step reads both forward half-lists,
    // 5 bytes per entry: 2.5 B x sum_i m_i^2 over full degrees m_i
    ctx.t.alg_bytes = (uint64_t)(2.5 * (double)g.sum_sq_deg);
}


}  // namespace gsn
