// count3.hip - binned triangle counts on the forward CSR (paper Sec. 2.2
// hub-and-spoke enumeration, Sec. 3.1 sorted-list intersection, Sec. 3.5.2
// one work group per hub with lanes on the inner loop, Sec. 3.5.3 tiles).
//
// Every triangle {i < j < k} (labels) is found exactly once: at hub i, spoke
// j in N+(i), third vertex k in N+(i) and N+(j). The work group of a hub
// stages N+(i) in an LDS hash table (label -> bin of edge (i,k)), then
// streams the forward rows of its spokes as one flat, coalesced sequence;
// each lane probes one candidate k. A hit has its three bins (ij from the
// spoke, ik from the table, jk from the row), which are sorted and ranked
// into an LDS histogram of 32-bit counters, flushed into the 64-bit result
// before any counter could wrap. Weighted counts add the exact integer
// t * 2^s of each triangle into 64-bit LDS halves, merged into 128-bit sums.
//
// A launch covers one tile: hubs in [h0, h1) and spokes in [s0, s1). A
// resident graph is a single tile; a host-tiled graph runs every (hub
// window, spoke window >= hub window) pair, so each spoke (i, j) -- and with
// it every triangle -- belongs to exactly one tile.
//
// Hubs are pulled from eight queues, one per slice of the tile's hub range;
// a work group starts on the queue of its own XCD so nearby hubs share that
// XCD's L2, and moves on to the other queues once its own is empty.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "kern_util.h"

namespace gsn {
namespace {

// One catalogue of a batched launch: its forward CSR, its first virtual hub
// index and where its counts go.
struct GDesc {
    const uint64_t *rp;
    const uint32_t *col;
    const uint8_t *bin;
    uint64_t v0;              // virtual hub index of label 0
    uint32_t n;
    uint32_t pad;
    unsigned long long *hist; // nconf
    unsigned long long *ntri; // 1
};

struct C3Args {
    const GDesc *gd;        // batched launch: ngraph descriptors (else null)
    int ngraph;
    uint32_t nvirt;         // batched launch: total hubs over all catalogues
    const uint64_t *rp;
    const uint32_t *hcol;   // hub rows (entry e of row i at rp[i] - hbase + e)
    const uint8_t *hbin;
    const uint32_t *scol;   // spoke rows (row j at rp[j] - sbase)
    const uint8_t *sbin;
    uint64_t hbase, sbase;
    uint32_t h0, h1, s0, s1;
    const double *w;        // label-ordered weights (weighted)
    const uint32_t *perm;   // label -> original index (anchored)
    const uint8_t *mark;    // anchored: hubs that can own an anchored triangle (nullable)
    int nb, nconf, log2h;
    int trunc;              // cut spoke rows at the hub row's largest label
    int packed;             // hash entries hold (label << 8 | bin): labels < 2^24 - 1
    int glog;               // > 0: spoke rows walked by groups of 2^glog lanes
    int lut;                // configuration index from an LDS table of nb^3 entries
    uint32_t maxdeg;
    uint32_t anchor_lo, anchor_hi;
    double wmul;            // 2^wscale
    uint64_t flush_limit;   // flush LDS counters before this many increments
    uint32_t *queue;        // kNumQueues counters
    unsigned long long *hist;   // nconf
    unsigned long long *wsum;   // 2*nconf (lo, hi)
    unsigned long long *ntri;   // 1
};

constexpr int kUnroll3 = 4;     // candidates per lane per pass
constexpr int kLutMaxBins = 16; // nb^3 u16 table up to 8 KB

struct TrueT { static constexpr bool value = true; };
struct FalseT { static constexpr bool value = false; };

// LDS layout of one work group (byte offsets).
struct Layout3 {
    uint32_t hkey, hbin, hslot, mstart, mpref, mbin, mw, mperm, hist, wlo, whi, tab, wtot, wflag, misc,
        lut, total;
};

__host__ __device__ inline Layout3 layout3(int block, uint32_t H, uint32_t maxdeg, int nconf, int nb,
                                           bool weighted, bool anchored, bool lds_hist, bool packed,
                                           bool lut) {
    if (!lds_hist) nconf = 0;
    Layout3 L{};
    uint32_t o = 0;
    L.mstart = o; o = lds_align(o + 8 * block, 16);
    L.mw = o;     if (weighted) o = lds_align(o + 8 * block, 16);
    L.wlo = o;    if (weighted) o = lds_align(o + 8 * nconf, 16);
    L.whi = o;    if (weighted) o = lds_align(o + 8 * nconf, 16);
    L.hkey = o;   o = lds_align(o + 4 * H, 16);
    L.mpref = o;  o = lds_align(o + 4 * (block + 1), 16);
    L.mperm = o;  if (anchored) o = lds_align(o + 4 * block, 16);
    L.hist = o;   o = lds_align(o + 4 * nconf, 16);
    L.tab = o;    o = lds_align(o + 8 * (nb + 1), 16);
    L.wtot = o;   o = lds_align(o + 8 * (block / 64 + 1), 16);
    L.wflag = o;  o = lds_align(o + 4 * block, 16);
    L.misc = o;   o = lds_align(o + 16, 16);
    L.hslot = o;  o = lds_align(o + 2 * (maxdeg + 1), 16);
    L.lut = o;    if (lut) o = lds_align(o + 2 * nb * nb * nb, 16);
    L.hbin = o;   if (!packed) o = lds_align(o + H, 16);
    L.mbin = o;   o = lds_align(o + block, 16);
    L.total = o;
    return L;
}

// 128-bit add into a (lo, hi) pair of global words.
__device__ __forceinline__ void add128(unsigned long long *dst, unsigned __int128 v) {
    unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    unsigned long long old = atomicAdd(&dst[0], lo);
    if (old + lo < old) hi += 1;
    if (hi) atomicAdd(&dst[1], hi);
}

template <int BLOCK, bool WEIGHTED, bool LDS_HIST>
__device__ void flush3(const C3Args &a, const Layout3 &L, unsigned char *sm,
                       unsigned long long *hout) {
    if (!LDS_HIST) return;
    uint32_t *hist = (uint32_t *)(sm + L.hist);
    for (int b = threadIdx.x; b < a.nconf; b += BLOCK) {
        uint32_t v = hist[b];
        if (v) {
            atomicAdd(&hout[b], (unsigned long long)v);
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

__device__ __forceinline__ uint32_t next_hub_in(uint32_t *queue, uint32_t h0, uint32_t h1, int *qv) {
    const int q0 = blockIdx.x % kNumQueues;
    const uint64_t n = (uint64_t)(h1 - h0);
    while (*qv < kNumQueues) {
        const int q = (q0 + *qv) % kNumQueues;
        const uint64_t lo = h0 + n * q / kNumQueues, hi = h0 + n * (q + 1) / kNumQueues;
        const uint32_t v = atomicAdd(&queue[q], 1u);
        if (lo + v < hi) return (uint32_t)(lo + v);
        ++*qv;
    }
    return kEmptyKey;
}

// Catalogue of virtual hub v: the last descriptor with v0 <= v.
__device__ __forceinline__ int graph_of(const GDesc *gd, int ng, uint32_t v) {
    int lo = 0, hi = ng;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (gd[mid].v0 <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Everything the candidate walk of one spoke chunk reads or updates.
struct Probe {
    const uint32_t *mpref;        // flat start of each compact spoke, [ncomp] = total
    const unsigned long long *mstart;  // row offset of each compact spoke in scol / sbin
    const uint8_t *mbin;          // bin of edge (hub, spoke)
    const double *mw;             // spoke weights
    const uint32_t *mperm;        // spoke original indices
    uint32_t *wflag;              // this wave's 64 LDS tags
    const uint32_t *hkey;         // hub hash
    const uint8_t *hbin;          // hub bins (unpacked hash)
    const uint16_t *lut;          // nb^3 configuration table
    const int *ta, *tb;           // rank tables
    uint32_t *hist;               // LDS counters (LDS_HIST)
    unsigned long long *hout;     // global counters (otherwise)
    unsigned long long *wlo, *whi, *wsum;
    const uint32_t *scol;
    const uint8_t *sbin;
    uint32_t mask, ncomp;
    int log2h, nb;
    double wi, wmul;
    const double *w;
    uint32_t pi;
    const uint32_t *perm;
    uint32_t anchor_lo, anchor_hi;
    int glog;                     // lanes per spoke group = 1 << glog (group walk)
};

// One candidate: probe the hub hash, bin and count a hit.
template <bool PACK, bool LUT, bool WEIGHTED, bool ANCHORED, bool LDS_HIST>
__device__ __forceinline__ void probe_one(const Probe &c, uint32_t k, uint32_t key, uint32_t hh, int s2,
                                          int z, unsigned long long &mytri) {
    const bool more = PACK ? (key != kEmptyKey && (key >> 8) != k) : (key != k && key != kEmptyKey);
    if (more) {
        do {
            hh = (hh + 1) & c.mask;
            key = c.hkey[hh];
        } while (PACK ? (key != kEmptyKey && (key >> 8) != k) : (key != k && key != kEmptyKey));
    }
    const bool hit = PACK ? key != kEmptyKey : key == k;
    if (!hit) return;
    if (ANCHORED) {
        const uint32_t mm = min(c.pi, min(c.mperm[s2], c.perm[k]));
        if (mm < c.anchor_lo || mm >= c.anchor_hi) return;
    }
    const int x = c.mbin[s2];
    const int y = PACK ? (int)(key & 0xFFu) : (int)c.hbin[hh];
    int idx;
    if (LUT) {
        idx = c.lut[(x * c.nb + y) * c.nb + z];
    } else {
        const int lo = min(x, min(y, z)), hi = max(x, max(y, z));
        const int mid = x + y + z - lo - hi;
        idx = c.ta[lo] + c.tb[mid] + hi;
    }
    if (LDS_HIST) atomicAdd(&c.hist[idx], 1u);
    else atomicAdd(&c.hout[idx], 1ull);
    ++mytri;
    if (WEIGHTED) {
        double p = c.wi, q = c.mw[s2], r = c.w[k], t;
        if (p > q) { t = p; p = q; q = t; }
        if (q > r) { t = q; q = r; r = t; }
        if (p > q) { t = p; p = q; q = t; }
        const double prod = __dmul_rn(__dmul_rn(p, q), r);
        const unsigned long long ti = (unsigned long long)__dmul_rn(prod, c.wmul);
        if (LDS_HIST) {
            atomicAdd(&c.wlo[idx], ti & 0xFFFFFFFFull);
            atomicAdd(&c.whi[idx], ti >> 32);
        } else {
            add128(&c.wsum[2 * idx], (unsigned __int128)ti);
        }
    }
}

// Spokes sfirst, sfirst + sstep, ... of a chunk, walked by groups of
// 2^glog lanes: group g of the wave takes every G-th of those spokes and
// reads its row 2^glog candidates at a time, U steps per pass with the loads
// of a pass issued back to back. Rows are padded to whole steps.
template <bool PACK, bool LUT, bool WEIGHTED, bool ANCHORED, bool LDS_HIST>
__device__ __forceinline__ void probe_groups(const Probe &c, uint32_t sfirst, uint32_t sstep,
                                             unsigned long long &mytri) {
    constexpr int U = kUnroll3;
    const uint32_t lane = threadIdx.x & 63;
    const int glog = c.glog;
    const uint32_t S = 1u << glog, G = 64u >> glog;
    const uint32_t sub = lane & (S - 1), gi = lane >> glog;
    const uint32_t ncomp = c.ncomp;
    uint32_t s = sfirst + gi * sstep;         // this group's spoke
    const uint32_t gstep = G * sstep;
    uint32_t off = 0, len = 0;
    uint64_t base = 0;
    if (s < ncomp) {
        len = c.mpref[s + 1] - c.mpref[s];
        base = c.mstart[s];
    }
    while (true) {
        uint32_t kk[U], key[U], hh[U], sp[U];
        uint8_t bz[U];
        bool ok[U];
        bool any = false;  // this lane has a candidate in this pass
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (off >= len && s < ncomp) {  // next spoke of this group
                s += gstep;
                off = 0;
                len = 0;
                if (s < ncomp) {
                    len = c.mpref[s + 1] - c.mpref[s];
                    base = c.mstart[s];
                }
            }
            const uint32_t e = off + sub;
            ok[u] = s < ncomp && e < len;
            sp[u] = ok[u] ? s : 0;
            const uint64_t pos = ok[u] ? base + e : c.mstart[0];  // in-bounds stand-in
            kk[u] = c.scol[pos];
            bz[u] = c.sbin[pos];
            off += S;
            any |= ok[u];
        }
        if (!__any(any)) break;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            hh[u] = label_hash(kk[u], c.log2h);
            key[u] = c.hkey[hh[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (ok[u]) probe_one<PACK, LUT, WEIGHTED, ANCHORED, LDS_HIST>(c, kk[u], key[u], hh[u], sp[u], bz[u], mytri);
    }
}

template <bool WEIGHTED, bool ANCHORED, bool LDS_HIST>
__device__ __forceinline__ void probe_groups_any(bool packed, bool lut, const Probe &c, uint32_t sfirst,
                                                 uint32_t sstep, unsigned long long &mytri) {
    if (packed) {
        if (lut) probe_groups<true, true, WEIGHTED, ANCHORED, LDS_HIST>(c, sfirst, sstep, mytri);
        else probe_groups<true, false, WEIGHTED, ANCHORED, LDS_HIST>(c, sfirst, sstep, mytri);
    } else {
        if (lut) probe_groups<false, true, WEIGHTED, ANCHORED, LDS_HIST>(c, sfirst, sstep, mytri);
        else probe_groups<false, false, WEIGHTED, ANCHORED, LDS_HIST>(c, sfirst, sstep, mytri);
    }
}

// Candidates [r0, r1) of the flat range of a spoke chunk, walked by one
// wavefront in windows of 64, U windows per pass with their loads issued back
// to back. The spokes starting inside a window tag their start positions in
// the wave's LDS flags; a ballot of the tags and a count of the tagged lanes
// below give every lane its spoke without a search.
template <bool PACK, bool LUT, bool WEIGHTED, bool ANCHORED, bool LDS_HIST>
__device__ __forceinline__ void probe_range(const Probe &c, uint32_t r0, uint32_t r1,
                                            unsigned long long &mytri) {
    constexpr int U = kUnroll3;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t ncomp = c.ncomp;
    c.wflag[lane] = 0;  // tags of earlier chunks must not match this one's
    wave_lds_sync();
    uint32_t base = upper_index(c.mpref, ncomp, r0);  // spoke holding r0
    for (uint32_t w0 = r0; w0 < r1; w0 += U * 64) {
        uint32_t kk[U], spk[U], key[U], hh[U];
        uint8_t bz[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t e0 = w0 + u * 64;
            const uint32_t cs = base + 1 + lane;
            const uint32_t p = cs < ncomp ? c.mpref[cs] - e0 : 0xFFFFFFFFu;
            if (p < 64) c.wflag[p] = e0 + 1;
            wave_lds_sync();
            const bool f = lane > 0 && c.wflag[lane] == e0 + 1;
            const uint64_t m = __ballot(f);
            const uint64_t at64 = __ballot(p == 64);
            const uint32_t sp = base + lanes_below(m) + (f ? 1u : 0u);
            base += (uint32_t)__popcll(m) + (at64 ? 1u : 0u);
            uint32_t e = e0 + lane;
            ok[u] = e < r1;
            const uint32_t sps = min(ok[u] ? sp : base, ncomp - 1);
            if (!ok[u]) e = c.mpref[sps];  // in-bounds stand-in, result dropped
            spk[u] = sps;
            const uint64_t pos = c.mstart[sps] + (e - c.mpref[sps]);
            kk[u] = c.scol[pos];
            bz[u] = c.sbin[pos];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            hh[u] = label_hash(kk[u], c.log2h);
            key[u] = c.hkey[hh[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // the first probe resolves almost always; chains are rare
            const bool more = PACK ? (key[u] != kEmptyKey && (key[u] >> 8) != kk[u])
                                   : (key[u] != kk[u] && key[u] != kEmptyKey);
            if (more) {
                uint32_t h = hh[u], kv;
                do {
                    h = (h + 1) & c.mask;
                    kv = c.hkey[h];
                } while (PACK ? (kv != kEmptyKey && (kv >> 8) != kk[u]) : (kv != kk[u] && kv != kEmptyKey));
                hh[u] = h;
                key[u] = kv;
            }
            const bool hit = PACK ? key[u] != kEmptyKey : key[u] == kk[u];
            if (!(hit && ok[u])) continue;
            const uint32_t k = kk[u];
            const int s2 = spk[u];
            if (ANCHORED) {
                const uint32_t mm = min(c.pi, min(c.mperm[s2], c.perm[k]));
                if (mm < c.anchor_lo || mm >= c.anchor_hi) continue;
            }
            const int x = c.mbin[s2];
            const int y = PACK ? (int)(key[u] & 0xFFu) : (int)c.hbin[hh[u]];
            const int z = bz[u];
            int idx;
            if (LUT) {
                idx = c.lut[(x * c.nb + y) * c.nb + z];
            } else {
                const int lo = min(x, min(y, z)), hi = max(x, max(y, z));
                const int mid = x + y + z - lo - hi;
                idx = c.ta[lo] + c.tb[mid] + hi;
            }
            if (LDS_HIST) atomicAdd(&c.hist[idx], 1u);
            else atomicAdd(&c.hout[idx], 1ull);
            ++mytri;
            if (WEIGHTED) {
                double p = c.wi, q = c.mw[s2], r = c.w[k], t;
                if (p > q) { t = p; p = q; q = t; }
                if (q > r) { t = q; q = r; r = t; }
                if (p > q) { t = p; p = q; q = t; }
                const double prod = __dmul_rn(__dmul_rn(p, q), r);
                const unsigned long long ti = (unsigned long long)__dmul_rn(prod, c.wmul);
                if (LDS_HIST) {
                    atomicAdd(&c.wlo[idx], ti & 0xFFFFFFFFull);
                    atomicAdd(&c.whi[idx], ti >> 32);
                } else {
                    add128(&c.wsum[2 * idx], (unsigned __int128)ti);
                }
            }
        }
    }
}

template <bool WEIGHTED, bool ANCHORED, bool LDS_HIST>
__device__ __forceinline__ void probe_any(bool packed, bool lut, const Probe &c, uint32_t r0,
                                          uint32_t r1, unsigned long long &mytri) {
    if (packed) {
        if (lut) probe_range<true, true, WEIGHTED, ANCHORED, LDS_HIST>(c, r0, r1, mytri);
        else probe_range<true, false, WEIGHTED, ANCHORED, LDS_HIST>(c, r0, r1, mytri);
    } else {
        if (lut) probe_range<false, true, WEIGHTED, ANCHORED, LDS_HIST>(c, r0, r1, mytri);
        else probe_range<false, false, WEIGHTED, ANCHORED, LDS_HIST>(c, r0, r1, mytri);
    }
}

template <int BLOCK, bool WEIGHTED, bool ANCHORED, bool LDS_HIST, bool BATCH>
__global__ __launch_bounds__(BLOCK) void k_count3(C3Args a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const uint32_t H = 1u << a.log2h, mask = H - 1;
    const Layout3 L = layout3(BLOCK, H, a.maxdeg, a.nconf, a.nb, WEIGHTED, ANCHORED, LDS_HIST, a.packed, a.lut);
    uint16_t *lut = (uint16_t *)(sm + L.lut);
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
    uint64_t *wtot64 = (uint64_t *)(sm + L.wtot);
    uint32_t *wflag = (uint32_t *)(sm + L.wflag) + (threadIdx.x & ~63u);  // this wave's 64 tags
    uint32_t *s_hub = (uint32_t *)(sm + L.misc);
    unsigned long long *s_cnt = (unsigned long long *)(sm + L.misc + 8);
    const int tid = threadIdx.x;

    for (uint32_t s = tid; s < H; s += BLOCK) hkey[s] = kEmptyKey;
    if (LDS_HIST)
        for (int b = tid; b < a.nconf; b += BLOCK) {
            hist[b] = 0;
            if (WEIGHTED) { wlo[b] = 0; whi[b] = 0; }
        }
    for (int b = tid; b < a.nb; b += BLOCK) {
        ta[b] = rank_a(a.nb, b);
        tb[b] = rank_b(a.nb, b);
    }
    if (a.lut)
        for (int t = tid; t < a.nb * a.nb * a.nb; t += BLOCK) {
            const int x = t / (a.nb * a.nb), y = (t / a.nb) % a.nb, z = t % a.nb;
            const int lo = min(x, min(y, z)), hi = max(x, max(y, z)), mid = x + y + z - lo - hi;
            lut[t] = (uint16_t)(rank_a(a.nb, lo) + rank_b(a.nb, mid) + hi);
        }
    if (tid == 0) *s_cnt = 0;
    __syncthreads();

    unsigned long long mytri = 0;
    uint64_t acc = 0;   // upper bound on increments since the last flush (uniform)
    int qv = 0;         // queues found empty (thread 0)
    int cur = -1;       // batched launch: catalogue whose counts the LDS holds
    int *s_g = (int *)(sm + L.misc + 4);
    // the CSR view of the current hub: the launch's tile, or one catalogue
    const uint64_t *rp = a.rp;
    const uint32_t *hcol = a.hcol, *scol = a.scol;
    const uint8_t *hbinp = a.hbin, *sbinp = a.sbin;
    uint64_t hbase = a.hbase, sbase = a.sbase;
    uint32_t s0 = a.s0, s1 = a.s1;
    unsigned long long *hout = a.hist, *tout = a.ntri;

    while (true) {
        if (tid == 0) {
            if (BATCH) {
                const uint32_t v = next_hub_in(a.queue, 0, a.nvirt, &qv);
                if (v != kEmptyKey) {
                    const int g = graph_of(a.gd, a.ngraph, v);
                    *s_g = g;
                    *s_hub = (uint32_t)(v - a.gd[g].v0);
                } else {
                    *s_hub = kEmptyKey;
                }
            } else {
                *s_hub = next_hub_in(a.queue, a.h0, a.h1, &qv);
            }
        }
        __syncthreads();
        const uint32_t i = *s_hub;
        if (i == kEmptyKey) break;
        if (BATCH) {
            const int g = *s_g;
            if (g != cur) {
                // a new catalogue: hand the previous one its counts first
                if (cur >= 0) {
                    flush3<BLOCK, WEIGHTED, LDS_HIST>(a, L, sm, hout);
                    if (mytri) atomicAdd(s_cnt, mytri);
                    mytri = 0;
                    acc = 0;
                    __syncthreads();
                    if (tid == 0 && *s_cnt) {
                        atomicAdd(tout, *s_cnt);
                        *s_cnt = 0;
                    }
                }
                cur = g;
                const GDesc &G = a.gd[g];
                rp = G.rp;
                hcol = scol = G.col;
                hbinp = sbinp = G.bin;
                hbase = sbase = 0;
                s0 = 0;
                s1 = G.n;
                hout = G.hist;
                tout = G.ntri;
            }
        }
        const uint64_t beg = rp[i] - hbase;
        const uint32_t d = (uint32_t)(rp[i + 1] - rp[i]);
        if (d < 2 || (ANCHORED && a.mark && !a.mark[i])) { __syncthreads(); continue; }
        const uint32_t kmax = hcol[beg + d - 1];  // largest label of N+(i)
        double wi = 0.0;
        uint32_t pi = 0;
        if (WEIGHTED) wi = a.w[i];
        if (ANCHORED) pi = a.perm[i];

        // stage N+(i): label -> bin of (i, k); packed as (label << 8 | bin)
        // when labels fit 24 bits, else label and bin in separate arrays
        for (uint32_t e = tid; e < d; e += BLOCK) {
            const uint32_t k = hcol[beg + e];
            const uint32_t v = a.packed ? ((k << 8) | hbinp[beg + e]) : k;
            uint32_t s = label_hash(k, a.log2h);
            while (atomicCAS(&hkey[s], kEmptyKey, v) != kEmptyKey) s = (s + 1) & mask;
            if (!a.packed) hbin[s] = hbinp[beg + e];
            hslot[e] = (uint16_t)s;
        }
        __syncthreads();

        // spokes in chunks of BLOCK; the last spoke cannot close a triangle;
        // spokes outside this tile's spoke range contribute nothing here
        for (uint32_t c0 = 0; c0 + 1 < d; c0 += BLOCK) {
            const uint32_t sidx = c0 + tid;
            uint32_t len = 0;
            uint64_t st = 0;
            uint8_t sb = 0;
            double sw = 0.0;
            uint32_t spm = 0;
            if (sidx + 1 < d) {
                const uint32_t j = hcol[beg + sidx];
                if (j >= s0 && j < s1) {
                    st = rp[j] - sbase;
                    len = (uint32_t)(rp[j + 1] - rp[j]);
                    // entries of N+(j) above the largest label of N+(i) cannot match
                    if (a.trunc && len > 16 && scol[st + len - 1] > kmax) {
                        uint32_t lo = 0, hi = len;  // first entry > kmax
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (scol[st + mid] <= kmax) lo = mid + 1;
                            else hi = mid;
                        }
                        len = lo;
                    }
                    sb = hbinp[beg + sidx];
                    if (WEIGHTED) sw = a.w[j];
                    if (ANCHORED) spm = a.perm[j];
                }
            }
            // one scan gives each non-empty spoke its compact index (high
            // word) and the flat start of its row (low word)
            uint64_t tot64;
            const uint64_t pre64 = wg_excl_scan64<BLOCK>(((uint64_t)(len > 0) << 32) | len, wtot64, tot64);
            const uint32_t total = (uint32_t)tot64, ncomp = (uint32_t)(tot64 >> 32);
            if (len > 0) {
                const uint32_t c = (uint32_t)(pre64 >> 32);
                mstart[c] = st;
                mpref[c] = (uint32_t)pre64;
                mbin[c] = sb;
                if (WEIGHTED) mw[c] = sw;
                if (ANCHORED) mperm[c] = spm;
            }
            if (tid == 0) mpref[ncomp] = total;
            if (acc + total >= a.flush_limit) {
                flush3<BLOCK, WEIGHTED, LDS_HIST>(a, L, sm, hout);
                acc = 0;
            }
            acc += total;
            __syncthreads();

            // each wave walks one contiguous quarter of the flat range
            if (total > 0) {
                constexpr int NW = BLOCK / 64;
                const uint32_t wid = tid >> 6;
                const uint32_t r0 = (uint32_t)((uint64_t)total * wid / NW);
                const uint32_t r1 = (uint32_t)((uint64_t)total * (wid + 1) / NW);
                Probe c;
                c.mpref = mpref; c.mstart = mstart; c.mbin = mbin; c.mw = mw; c.mperm = mperm;
                c.wflag = wflag; c.hkey = hkey; c.hbin = hbin; c.lut = lut; c.ta = ta; c.tb = tb;
                c.hist = hist; c.hout = hout; c.wlo = wlo; c.whi = whi; c.wsum = a.wsum;
                c.scol = scol; c.sbin = sbinp; c.mask = mask; c.ncomp = ncomp; c.log2h = a.log2h;
                c.nb = a.nb; c.wi = wi; c.wmul = a.wmul; c.w = a.w; c.pi = pi; c.perm = a.perm;
                c.anchor_lo = a.anchor_lo; c.anchor_hi = a.anchor_hi; c.glog = a.glog;
                if (a.glog > 0)
                    probe_groups_any<WEIGHTED, ANCHORED, LDS_HIST>(a.packed, a.lut, c, wid, NW, mytri);
                else if (r0 < r1)
                    probe_any<WEIGHTED, ANCHORED, LDS_HIST>(a.packed, a.lut, c, r0, r1, mytri);
            }
            __syncthreads();
        }
        for (uint32_t e = tid; e < d; e += BLOCK) hkey[hslot[e]] = kEmptyKey;
        __syncthreads();
    }

    __syncthreads();
    flush3<BLOCK, WEIGHTED, LDS_HIST>(a, L, sm, hout);
    if (mytri) atomicAdd(s_cnt, mytri);
    __syncthreads();
    if (tid == 0 && *s_cnt && tout) atomicAdd(tout, *s_cnt);
}

// ---------------------------------------------------------------------------
// Wave-per-hub variant for small degrees: every wavefront of a work group
// runs its own hub with its own LDS hash and spoke tables, so no work-group
// barrier is ever needed; the configuration table is shared. Unbatched, the
// work group's waves share one histogram that any wave may hand to global
// memory at any time by atomically exchanging each counter with zero (no
// increment is lost or counted twice); batched, each wave keeps its own
// histogram because neighbouring waves may be counting other catalogues.

struct Layout3w {
    uint32_t wlo, whi, acc, hist, tab, lut, shared_end;                  // work group
    uint32_t mstart, mw, hkey, mpref, mperm, wflag, whist, hslot, hbin, mbin, per_wave;  // per wave
    uint32_t total;
};

__host__ __device__ inline Layout3w layout3w(int nw, uint32_t H, uint32_t maxdeg, int nconf, int nb,
                                             bool weighted, bool anchored, bool lds_hist, bool packed,
                                             bool lut, bool batch) {
    const int nsh = (lds_hist && !batch) ? nconf : 0;  // shared counters
    const int nwv = (lds_hist && batch) ? nconf : 0;   // per-wave counters
    Layout3w L{};
    uint32_t o = 0;
    L.wlo = o;   if (weighted) o = lds_align(o + 8 * nsh, 16);
    L.whi = o;   if (weighted) o = lds_align(o + 8 * nsh, 16);
    L.acc = o;   o = lds_align(o + 16, 16);
    L.hist = o;  o = lds_align(o + 4 * nsh, 16);
    L.tab = o;   o = lds_align(o + 8 * (nb + 1), 16);
    L.lut = o;   if (lut) o = lds_align(o + 2 * nb * nb * nb, 16);
    L.shared_end = o;
    uint32_t q = 0;
    L.mstart = q; q = lds_align(q + 8 * 64, 16);
    L.mw = q;     if (weighted) q = lds_align(q + 8 * 64, 16);
    L.hkey = q;   q = lds_align(q + 4 * H, 16);
    L.mpref = q;  q = lds_align(q + 4 * 65, 16);
    L.mperm = q;  if (anchored) q = lds_align(q + 4 * 64, 16);
    L.wflag = q;  q = lds_align(q + 4 * 64, 16);
    L.whist = q;  q = lds_align(q + 4 * nwv, 16);
    L.hslot = q;  q = lds_align(q + 2 * (maxdeg + 1), 16);
    L.hbin = q;   if (!packed) q = lds_align(q + H, 16);
    L.mbin = q;   q = lds_align(q + 64, 16);
    L.per_wave = q;
    L.total = o + (uint32_t)nw * q;
    return L;
}

__device__ __forceinline__ uint64_t wave_excl_scan64(uint64_t v, uint64_t &total) {
    const int lane = threadIdx.x & 63;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NW, bool WEIGHTED, bool ANCHORED, bool LDS_HIST, bool BATCH>
__global__ __launch_bounds__(NW * 64) void k_count3w(C3Args a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const uint32_t H = 1u << a.log2h, mask = H - 1;
    const Layout3w L = layout3w(NW, H, a.maxdeg, a.nconf, a.nb, WEIGHTED, ANCHORED, LDS_HIST, a.packed, a.lut, BATCH);
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    uint16_t *lut = (uint16_t *)(sm + L.lut);
    int *ta = (int *)(sm + L.tab);
    int *tb = ta + (a.nb + 1);
    unsigned long long *s_acc = (unsigned long long *)(sm + L.acc);
    unsigned long long *wlo = (unsigned long long *)(sm + L.wlo);
    unsigned long long *whi = (unsigned long long *)(sm + L.whi);
    unsigned char *wb = sm + L.shared_end + wid * L.per_wave;
    uint32_t *hist = BATCH ? (uint32_t *)(wb + L.whist) : (uint32_t *)(sm + L.hist);
    uint32_t *hkey = (uint32_t *)(wb + L.hkey);
    uint8_t *hbin = (uint8_t *)(wb + L.hbin);
    uint16_t *hslot = (uint16_t *)(wb + L.hslot);
    unsigned long long *mstart = (unsigned long long *)(wb + L.mstart);
    uint32_t *mpref = (uint32_t *)(wb + L.mpref);
    uint8_t *mbin = (uint8_t *)(wb + L.mbin);
    double *mw = (double *)(wb + L.mw);
    uint32_t *mperm = (uint32_t *)(wb + L.mperm);
    uint32_t *wflag = (uint32_t *)(wb + L.wflag);

    for (uint32_t q = lane; q < H; q += 64) hkey[q] = kEmptyKey;
    if (LDS_HIST) {
        if (BATCH) {
            for (int b = lane; b < a.nconf; b += 64) hist[b] = 0;
        } else {
            for (int b = tid; b < a.nconf; b += NW * 64) {
                hist[b] = 0;
                if (WEIGHTED) { wlo[b] = 0; whi[b] = 0; }
            }
        }
    }
    for (int b = tid; b < a.nb; b += NW * 64) {
        ta[b] = rank_a(a.nb, b);
        tb[b] = rank_b(a.nb, b);
    }
    if (a.lut)
        for (int t = tid; t < a.nb * a.nb * a.nb; t += NW * 64) {
            const int x = t / (a.nb * a.nb), y = (t / a.nb) % a.nb, z = t % a.nb;
            const int lo = min(x, min(y, z)), hi = max(x, max(y, z)), mid = x + y + z - lo - hi;
            lut[t] = (uint16_t)(rank_a(a.nb, lo) + rank_b(a.nb, mid) + hi);
        }
    if (tid == 0) *s_acc = 0;
    __syncthreads();

    unsigned long long mytri = 0;
    uint64_t acc = 0;   // batched: increments since this wave's last flush
    int qv = 0;
    int cur = -1;
    const uint64_t *rp = a.rp;
    const uint32_t *hcol = a.hcol, *scol = a.scol;
    const uint8_t *hbinp = a.hbin, *sbinp = a.sbin;
    uint64_t hbase = a.hbase, sbase = a.sbase;
    uint32_t s0 = a.s0, s1 = a.s1;
    unsigned long long *hout = a.hist, *tout = a.ntri;

    // batched: hand this wave's counts to its catalogue
    auto flush_wave = [&]() {
        if (LDS_HIST)
            for (int b = lane; b < a.nconf; b += 64) {
                const uint32_t v = hist[b];
                if (v) {
                    atomicAdd(&hout[b], (unsigned long long)v);
                    hist[b] = 0;
                }
            }
        const unsigned long long t = wave_sum64(mytri);
        if (lane == 0 && t) atomicAdd(tout, t);
        mytri = 0;
    };
    // unbatched: any wave may move the shared counters to global memory
    auto flush_shared_exchange = [&]() {
        for (int b = lane; b < a.nconf; b += 64) {
            const uint32_t v = atomicExch(&hist[b], 0u);
            if (v) atomicAdd(&a.hist[b], (unsigned long long)v);
            if (WEIGHTED) {
                const unsigned long long lo = atomicExch(&wlo[b], 0ull);
                const unsigned long long hi = atomicExch(&whi[b], 0ull);
                if (lo | hi) add128(&a.wsum[2 * b], ((unsigned __int128)hi << 32) + (unsigned __int128)lo);
            }
        }
    };

    while (true) {
        uint32_t v = kEmptyKey;
        int g = 0;
        if (lane == 0) {
            if (BATCH) {
                v = next_hub_in(a.queue, 0, a.nvirt, &qv);
                if (v != kEmptyKey) {
                    g = graph_of(a.gd, a.ngraph, v);
                    v = (uint32_t)(v - a.gd[g].v0);
                }
            } else {
                v = next_hub_in(a.queue, a.h0, a.h1, &qv);
            }
        }
        const uint32_t i = __builtin_amdgcn_readfirstlane(v);
        if (i == kEmptyKey) break;
        if (BATCH) {
            g = __builtin_amdgcn_readfirstlane(g);
            if (g != cur) {
                if (cur >= 0) flush_wave();
                acc = 0;
                cur = g;
                const GDesc &G = a.gd[g];
                rp = G.rp;
                hcol = scol = G.col;
                hbinp = sbinp = G.bin;
                hbase = sbase = 0;
                s0 = 0;
                s1 = G.n;
                hout = G.hist;
                tout = G.ntri;
            }
        }
        const uint64_t beg = rp[i] - hbase;
        const uint32_t d = (uint32_t)(rp[i + 1] - rp[i]);
        if (d < 2 || (ANCHORED && a.mark && !a.mark[i])) continue;
        const uint32_t kmax = hcol[beg + d - 1];
        const double wi = WEIGHTED ? a.w[i] : 0.0;
        const uint32_t pi = ANCHORED ? a.perm[i] : 0;

        for (uint32_t e = lane; e < d; e += 64) {
            const uint32_t k = hcol[beg + e];
            const uint32_t val = a.packed ? ((k << 8) | hbinp[beg + e]) : k;
            uint32_t q = label_hash(k, a.log2h);
            while (atomicCAS(&hkey[q], kEmptyKey, val) != kEmptyKey) q = (q + 1) & mask;
            if (!a.packed) hbin[q] = hbinp[beg + e];
            hslot[e] = (uint16_t)q;
        }
        wave_lds_sync();

        for (uint32_t c0 = 0; c0 + 1 < d; c0 += 64) {
            const uint32_t sidx = c0 + lane;
            uint32_t len = 0;
            uint64_t st = 0;
            uint8_t sb = 0;
            double sw = 0.0;
            uint32_t spm = 0;
            if (sidx + 1 < d) {
                const uint32_t j = hcol[beg + sidx];
                if (j >= s0 && j < s1) {
                    st = rp[j] - sbase;
                    len = (uint32_t)(rp[j + 1] - rp[j]);
                    if (a.trunc && len > 16 && scol[st + len - 1] > kmax) {
                        uint32_t lo = 0, hi = len;
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (scol[st + mid] <= kmax) lo = mid + 1;
                            else hi = mid;
                        }
                        len = lo;
                    }
                    sb = hbinp[beg + sidx];
                    if (WEIGHTED) sw = a.w[j];
                    if (ANCHORED) spm = a.perm[j];
                }
            }
            uint64_t tot64;
            const uint64_t pre64 = wave_excl_scan64(((uint64_t)(len > 0) << 32) | len, tot64);
            const uint32_t total = (uint32_t)tot64, ncomp = (uint32_t)(tot64 >> 32);
            if (total == 0) continue;
            if (len > 0) {
                const uint32_t c = (uint32_t)(pre64 >> 32);
                mstart[c] = st;
                mpref[c] = (uint32_t)pre64;
                mbin[c] = sb;
                if (WEIGHTED) mw[c] = sw;
                if (ANCHORED) mperm[c] = spm;
            }
            if (lane == 0) mpref[ncomp] = total;
            wave_lds_sync();
            if (LDS_HIST) {
                if (BATCH) {
                    if (acc + total >= a.flush_limit) {
                        flush_wave();
                        acc = 0;
                    }
                    acc += total;
                } else {
                    // the group's increments since the start; the wave that
                    // crosses a multiple of 2^30 moves the shared counters out
                    unsigned long long old = 0;
                    if (lane == 0) old = atomicAdd(s_acc, (unsigned long long)total);
                    old = __shfl(old, 0, 64);
                    const unsigned long long lim = a.flush_limit >> 2;
                    if (old / lim != (old + total) / lim) flush_shared_exchange();
                }
            }
            Probe c;
            c.mpref = mpref; c.mstart = mstart; c.mbin = mbin; c.mw = mw; c.mperm = mperm;
            c.wflag = wflag; c.hkey = hkey; c.hbin = hbin; c.lut = lut; c.ta = ta; c.tb = tb;
            c.hist = hist; c.hout = BATCH ? hout : a.hist; c.wlo = wlo; c.whi = whi; c.wsum = a.wsum;
            c.scol = scol; c.sbin = sbinp; c.mask = mask; c.ncomp = ncomp; c.log2h = a.log2h;
            c.nb = a.nb; c.wi = wi; c.wmul = a.wmul; c.w = a.w; c.pi = pi; c.perm = a.perm;
            c.anchor_lo = a.anchor_lo; c.anchor_hi = a.anchor_hi; c.glog = a.glog;
            if (a.glog > 0) probe_groups_any<WEIGHTED, ANCHORED, LDS_HIST>(a.packed, a.lut, c, 0, 1, mytri);
            else probe_any<WEIGHTED, ANCHORED, LDS_HIST>(a.packed, a.lut, c, 0, total, mytri);
            wave_lds_sync();
        }
        for (uint32_t e = lane; e < d; e += 64) hkey[hslot[e]] = kEmptyKey;
        wave_lds_sync();
    }

    if (BATCH) {
        if (cur >= 0) flush_wave();
    } else {
        const unsigned long long t = wave_sum64(mytri);
        if (lane == 0 && t) atomicAdd(a.ntri, t);
        __syncthreads();
        if (LDS_HIST)
            for (int b = tid; b < a.nconf; b += NW * 64) {
                const uint32_t v = hist[b];
                if (v) atomicAdd(&a.hist[b], (unsigned long long)v);
                if (WEIGHTED) {
                    const unsigned long long lo = wlo[b], hi = whi[b];
                    if (lo | hi) add128(&a.wsum[2 * b], ((unsigned __int128)hi << 32) + (unsigned __int128)lo);
                }
            }
    }
}

__global__ void k_zero_u64(unsigned long long *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int B, bool W, bool A, bool LH, bool BATCH = false>
void launch3(Ctx &ctx, hipStream_t s, const C3Args &a, uint32_t lds) {
    const void *kern = reinterpret_cast<const void *>(&k_count3<B, W, A, LH, BATCH>);
    if (lds > 65536)
        GS_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count3<B, W, A, LH, BATCH>, B, lds));
    if (per_cu < 1) fail(GS_EUNSUPPORTED, "count kernel does not fit a compute unit");
    uint32_t grid = (uint32_t)ctx.n_cu * (uint32_t)per_cu;
    grid = (grid + kNumQueues - 1) / kNumQueues * kNumQueues;
    k_count3<B, W, A, LH, BATCH><<<dim3(grid), dim3(B), lds, s>>>(a);
    GS_HIP(hipGetLastError());
}

template <int B>
void launch3_b(Ctx &ctx, hipStream_t s, const C3Args &a, uint32_t lds, bool w, bool an, bool lh) {
    if (lh) {
        if (!w && !an) launch3<B, false, false, true>(ctx, s, a, lds);
        else if (w && !an) launch3<B, true, false, true>(ctx, s, a, lds);
        else if (!w && an) launch3<B, false, true, true>(ctx, s, a, lds);
        else launch3<B, true, true, true>(ctx, s, a, lds);
    } else {
        if (!w && !an) launch3<B, false, false, false>(ctx, s, a, lds);
        else if (w && !an) launch3<B, true, false, false>(ctx, s, a, lds);
        else if (!w && an) launch3<B, false, true, false>(ctx, s, a, lds);
        else launch3<B, true, true, false>(ctx, s, a, lds);
    }
}

constexpr uint32_t kWaveMaxDeg = 512;  // wave-per-hub kernel up to this forward degree

template <int NW, bool W, bool A, bool LH, bool BATCH>
void launch3w(Ctx &ctx, hipStream_t s, const C3Args &a, uint32_t lds) {
    const void *kern = reinterpret_cast<const void *>(&k_count3w<NW, W, A, LH, BATCH>);
    if (lds > 65536)
        GS_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count3w<NW, W, A, LH, BATCH>, NW * 64, lds));
    if (per_cu < 1) fail(GS_EUNSUPPORTED, "count kernel does not fit a compute unit");
    uint32_t grid = (uint32_t)ctx.n_cu * (uint32_t)per_cu;
    grid = (grid + kNumQueues - 1) / kNumQueues * kNumQueues;
    k_count3w<NW, W, A, LH, BATCH><<<dim3(grid), dim3(NW * 64), lds, s>>>(a);
    GS_HIP(hipGetLastError());
}

template <int NW, bool BATCH>
void launch3w_n(Ctx &ctx, hipStream_t s, const C3Args &a, uint32_t lds, bool w, bool an, bool lh) {
    if (BATCH) {
        if (lh) launch3w<NW, false, false, true, true>(ctx, s, a, lds);
        else launch3w<NW, false, false, false, true>(ctx, s, a, lds);
        return;
    }
    if (lh) {
        if (!w && !an) launch3w<NW, false, false, true, false>(ctx, s, a, lds);
        else if (w && !an) launch3w<NW, true, false, true, false>(ctx, s, a, lds);
        else if (!w && an) launch3w<NW, false, true, true, false>(ctx, s, a, lds);
        else launch3w<NW, true, true, true, false>(ctx, s, a, lds);
    } else {
        if (!w && !an) launch3w<NW, false, false, false, false>(ctx, s, a, lds);
        else if (w && !an) launch3w<NW, true, false, false, false>(ctx, s, a, lds);
        else if (!w && an) launch3w<NW, false, true, false, false>(ctx, s, a, lds);
        else launch3w<NW, true, true, false, false>(ctx, s, a, lds);
    }
}

// Lanes per spoke group from the mean forward row length (GS_GLOG / GS_MAP3
// override): short rows in small groups, long rows across the wavefront.
int group_log(double mean_row) {
    if (const char *em = getenv("GS_MAP3"))
        if (strcmp(em, "flat") == 0) return 0;
    if (const char *eg = getenv("GS_GLOG")) return std::max(0, std::min(6, atoi(eg)));
    if (mean_row < 24) return 3;
    if (mean_row < 64) return 4;
    if (mean_row < 160) return 5;
    return 6;
}

struct Plan3 {
    int nw = 0;           // > 0: wave-per-hub kernel with nw waves per group
    int block = 256;
    int trunc = 0;
    bool packed = true;
    bool lut = true;
    int log2h = 6;
    bool lds_hist = true;
    uint32_t lds = 0;
};

void launch3_any(Ctx &ctx, hipStream_t s, const C3Args &a, const Plan3 &P, bool w, bool an) {
    if (P.nw == 8) launch3w_n<8, false>(ctx, s, a, P.lds, w, an, P.lds_hist);
    else if (P.nw == 4) launch3w_n<4, false>(ctx, s, a, P.lds, w, an, P.lds_hist);
    else if (P.nw == 2) launch3w_n<2, false>(ctx, s, a, P.lds, w, an, P.lds_hist);
    else if (P.block == 512) launch3_b<512>(ctx, s, a, P.lds, w, an, P.lds_hist);
    else launch3_b<256>(ctx, s, a, P.lds, w, an, P.lds_hist);
}

// Work-group size and LDS plan: hash table at load factor <= 0.7, 512
// threads per hub for long rows (more waves per CU when LDS limits groups).
Plan3 plan3(const Ctx &ctx, uint32_t maxdeg, int nb, bool weighted, bool anchored, uint64_t max_n,
            bool batch = false) {
    Plan3 p;
    p.packed = max_n < (1ull << 24) - 1;
    p.lut = nb <= kLutMaxBins;
    const int nconf = (int)n_configs(nb);
    if (maxdeg > 16384) fail(GS_EUNSUPPORTED, "forward degree above 16384");
    // small degrees: one wavefront per hub (GS_KERNEL3=team|wave overrides)
    const char *ek = getenv("GS_KERNEL3");
    const bool wave = ek ? strcmp(ek, "wave") == 0 : maxdeg <= kWaveMaxDeg;
    if (wave) {
        p.nw = 4;
        if (const char *ew = getenv("GS_WAVES3")) p.nw = atoi(ew) == 8 ? 8 : (atoi(ew) == 2 ? 2 : 4);
        p.trunc = 0;
        if (const char *et = getenv("GS_TRUNC")) p.trunc = atoi(et) != 0;
        uint32_t H = 64;
        while ((uint64_t)H * 7 < (uint64_t)maxdeg * 10) { H <<= 1; ++p.log2h; }
        p.lds_hist = nconf <= 8192;
        Layout3w L = layout3w(p.nw, H, maxdeg, nconf, nb, weighted, anchored, p.lds_hist, p.packed, p.lut, batch);
        if ((int)L.total > ctx.max_lds && p.lds_hist) {
            p.lds_hist = false;
            L = layout3w(p.nw, H, maxdeg, nconf, nb, weighted, anchored, false, p.packed, p.lut, batch);
        }
        if ((int)L.total <= ctx.max_lds) {
            p.lds = L.total;
            p.block = 64 * p.nw;
            return p;
        }
        p.nw = 0;  // does not fit: team kernel
        p.log2h = 6;
    }
    if (const char *eb = getenv("GS_BLOCK3")) p.block = atoi(eb) == 512 ? 512 : 256;
    else p.block = maxdeg >= 1024 ? 512 : 256;
    // the per-spoke binary search pays off on long rows only
    if (const char *et = getenv("GS_TRUNC")) p.trunc = atoi(et) != 0;
    else p.trunc = maxdeg >= 1024;
    uint32_t H = 64;
    while ((uint64_t)H * 7 < (uint64_t)maxdeg * 10) { H <<= 1; ++p.log2h; }
    // per-work-group LDS histograms while they fit; global atomics beyond
    p.lds_hist = nconf <= 8192;
    Layout3 L = layout3(p.block, H, maxdeg, nconf, nb, weighted, anchored, p.lds_hist, p.packed, p.lut);
    if ((int)L.total > ctx.max_lds && p.lds_hist) {
        p.lds_hist = false;
        L = layout3(p.block, H, maxdeg, nconf, nb, weighted, anchored, false, p.packed, p.lut);
    }
    if ((int)L.total > ctx.max_lds) fail(GS_EUNSUPPORTED, "LDS footprint too large for this degree");
    p.lds = L.total;
    return p;
}

// Anchored counts: only hubs that are anchors or have an anchor in their
// forward row can own a triangle whose smallest original index is an anchor.
__global__ void k_mark_anchor_hubs(const uint64_t *__restrict__ rp, const uint32_t *__restrict__ col,
                                   const uint32_t *__restrict__ perm, uint32_t n, uint32_t lo,
                                   uint32_t hi, uint8_t *__restrict__ mark) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint8_t m = (perm[i] >= lo && perm[i] < hi) ? 1 : 0;
    for (uint64_t e = rp[i]; e < rp[i + 1] && !m; ++e) {
        const uint32_t p = perm[col[e]];
        m = (p >= lo && p < hi) ? 1 : 0;
    }
    mark[i] = m;
}

uint64_t flush_limit_for(uint32_t maxdeg, uint64_t per_chunk_factor) {
    // GS_FLUSH_LIMIT lowers the flush threshold (exercises the flush path)
    const char *fl = getenv("GS_FLUSH_LIMIT");
    uint64_t v = fl ? strtoull(fl, nullptr, 10) : 0xFFFFFFFFull;
    if (v < per_chunk_factor * (maxdeg + 1) || v > 0xFFFFFFFFull) v = 0xFFFFFFFFull;
    return v;
}

template <int B>
void launch3_batch(Ctx &ctx, hipStream_t s, const C3Args &a, const Plan3 &P) {
    if (P.lds_hist) launch3<B, false, false, true, true>(ctx, s, a, P.lds);
    else launch3<B, false, false, false, true>(ctx, s, a, P.lds);
}

}  // namespace

Batch3::~Batch3() {
    if (done) (void)hipEventDestroy(done);
}

void count3_batch_enqueue(Ctx &ctx, hipStream_t s, const Graph *const *gs, int ng, Batch3 &b) {
    if (ng < 1) fail(GS_EINVAL, "empty batch");
    const int nb = gs[0]->nbins;
    uint32_t maxdeg = 0;
    uint64_t nvirt = 0;
    for (int g = 0; g < ng; ++g) {
        if (!gs[g]) fail(GS_EINVAL, "null graph in batch");
        if (gs[g]->nbins != nb) fail(GS_EINVAL, "graphs of a batch must share nbins");
        if (gs[g]->n_windows != 1) fail(GS_EUNSUPPORTED, "batched counts need device-resident graphs");
        if (gs[g]->device != ctx.device) fail(GS_EINVAL, "graph on another device");
        maxdeg = std::max(maxdeg, gs[g]->max_deg);
        nvirt += (uint64_t)gs[g]->n;
    }
    if (nvirt >= 0xFFFFFFFFull) fail(GS_EUNSUPPORTED, "batch holds 2^32 or more points");
    const int nconf = (int)n_configs(nb);
    uint64_t max_n = 0;
    for (int g = 0; g < ng; ++g) max_n = std::max<uint64_t>(max_n, (uint64_t)gs[g]->n);
    const Plan3 P = plan3(ctx, maxdeg, nb, false, false, max_n, true);
    uint64_t sum_e = 0;
    for (int g = 0; g < ng; ++g) sum_e += gs[g]->n_edges;
    const int glog_sel = group_log(nvirt ? (double)sum_e / (double)nvirt : 0.0);
    b.ng = ng;
    b.nconf = nconf;
    const size_t per = (size_t)nconf + 1;
    const size_t words = (size_t)ng * per + kNumQueues / 2 + 1;
    b.dv.alloc(words * 8);
    unsigned long long *dv = b.dv.as<unsigned long long>();
    b.hostdesc.alloc(sizeof(GDesc) * ng);
    GDesc *hd = b.hostdesc.as<GDesc>();
    uint64_t v0 = 0;
    for (int g = 0; g < ng; ++g) {
        hd[g].rp = gs[g]->row_ptr.as<uint64_t>();
        hd[g].col = gs[g]->col.as<uint32_t>();
        hd[g].bin = gs[g]->bin.as<uint8_t>();
        hd[g].v0 = v0;
        hd[g].n = (uint32_t)gs[g]->n;
        hd[g].pad = 0;
        hd[g].hist = dv + (size_t)g * per;
        hd[g].ntri = dv + (size_t)g * per + nconf;
        v0 += (uint64_t)gs[g]->n;
    }
    b.gd.alloc(sizeof(GDesc) * ng);
    GS_HIP(hipMemcpyAsync(b.gd.p, hd, sizeof(GDesc) * ng, hipMemcpyHostToDevice, s));
    k_zero_u64<<<64, 256, 0, s>>>(dv, words);
    C3Args a{};
    a.gd = b.gd.as<GDesc>();
    a.ngraph = ng;
    a.nvirt = (uint32_t)nvirt;
    a.nb = nb;
    a.nconf = nconf;
    a.log2h = P.log2h;
    a.trunc = P.trunc;
    a.packed = P.packed;
    a.lut = P.lut;
    a.glog = glog_sel;
    a.maxdeg = maxdeg;
    a.flush_limit = flush_limit_for(maxdeg, P.block);
    a.queue = (uint32_t *)(dv + (size_t)ng * per);
    if (nvirt > 0) {
        if (P.nw == 8) launch3w_n<8, true>(ctx, s, a, P.lds, false, false, P.lds_hist);
        else if (P.nw == 4) launch3w_n<4, true>(ctx, s, a, P.lds, false, false, P.lds_hist);
        else if (P.nw == 2) launch3w_n<2, true>(ctx, s, a, P.lds, false, false, P.lds_hist);
        else if (P.block == 512) launch3_batch<512>(ctx, s, a, P);
        else launch3_batch<256>(ctx, s, a, P);
    }
    b.out.alloc(sizeof(unsigned long long) * (size_t)ng * per);
    GS_HIP(hipMemcpyAsync(b.out.p, dv, sizeof(unsigned long long) * (size_t)ng * per, hipMemcpyDeviceToHost, s));
    if (!b.done) GS_HIP(hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
    GS_HIP(hipEventRecord(b.done, s));
}

void count3_run(Ctx &ctx, const Graph &g, uint64_t *hist, uint64_t *wsum, uint64_t *ntri,
                const gs_anchor_range *anchors) {
    const int nb = g.nbins;
    const int nconf = (int)n_configs(nb);
    const bool weighted = wsum != nullptr;
    const bool anchored = anchors != nullptr;
    if (anchored && (anchors->lo > anchors->hi)) fail(GS_EINVAL, "anchor range lo > hi");
    const uint32_t maxdeg = g.max_deg;
    const Plan3 P = plan3(ctx, maxdeg, nb, weighted, anchored, (uint64_t)g.n);
    const int glog_sel = group_log(g.n ? (double)g.n_edges / (double)g.n : 0.0);
    const int W = g.n_windows;
    const int ntiles = W * (W + 1) / 2;

    // device staging: hist | wsum | ntri | queues (8 per tile)
    const size_t qwords = (size_t)ntiles * kNumQueues / 2 + 1;
    const size_t words = 3 * (size_t)nconf + 1 + qwords;
    unsigned long long *dv = (unsigned long long *)ctx.scratch_get(words * 8);
    C3Args a{};
    a.rp = g.row_ptr.as<uint64_t>();
    a.w = weighted ? g.weights.as<double>() : nullptr;
    a.perm = g.perm.as<uint32_t>();
    a.nb = nb;
    a.nconf = nconf;
    a.log2h = P.log2h;
    a.trunc = P.trunc;
    a.packed = P.packed;
    a.lut = P.lut;
    a.glog = glog_sel;
    a.maxdeg = maxdeg;
    a.anchor_lo = anchored ? (uint32_t)std::min<uint64_t>(anchors->lo, 0xFFFFFFFFull) : 0;
    a.anchor_hi = anchored ? (uint32_t)std::min<uint64_t>(anchors->hi, 0xFFFFFFFFull) : 0;
    a.wmul = std::ldexp(1.0, g.wscale);
    a.flush_limit = flush_limit_for(maxdeg, P.block);
    a.hist = dv;
    a.wsum = dv + nconf;
    a.ntri = dv + 3 * (size_t)nconf;
    uint32_t *queues = (uint32_t *)(dv + 3 * (size_t)nconf + 1);

    hipStream_t s = ctx.stream;
    GS_HIP(hipEventRecord(ctx.ev[0], s));
    k_zero_u64<<<64, 256, 0, s>>>(dv, words);
    GS_HIP(hipEventRecord(ctx.ev[2], s));
    DevBuf mark;
    if (anchored && W == 1 && g.n > 0) {
        mark.alloc((size_t)g.n);
        k_mark_anchor_hubs<<<(unsigned)((g.n + 255) / 256), 256, 0, s>>>(
            g.row_ptr.as<uint64_t>(), g.col.as<uint32_t>(), g.perm.as<uint32_t>(), (uint32_t)g.n,
            a.anchor_lo, a.anchor_hi, mark.as<uint8_t>());
        GS_HIP(hipGetLastError());
        a.mark = mark.as<uint8_t>();
    }
    if (g.n > 0 && W == 1) {
        a.hcol = a.scol = g.col.as<uint32_t>();
        a.hbin = a.sbin = g.bin.as<uint8_t>();
        a.hbase = a.sbase = 0;
        a.h0 = a.s0 = 0;
        a.h1 = a.s1 = (uint32_t)g.n;
        a.queue = queues;
        launch3_any(ctx, s, a, P, weighted, anchored);
    } else if (g.n > 0) {
        // host-tiled graph: spoke window S resident, hub windows H <= S
        // streamed through; copies of the next tile's windows overlap the
        // current tile's kernel on the copy stream
        uint64_t maxE = 1;
        for (int w = 0; w < W; ++w) maxE = std::max<uint64_t>(maxE, g.win_edge[w + 1] - g.win_edge[w]);
        DevBuf scol[2], sbin[2], hcol[2], hbin[2];
        for (int k = 0; k < 2; ++k) {
            scol[k].alloc(maxE * 4);
            sbin[k].alloc(maxE);
            hcol[k].alloc(maxE * 4);
            hbin[k].alloc(maxE);
        }
        struct Tile { int S, H, hslot; bool first_of_S, last_of_S; };
        std::vector<Tile> tiles;
        int hk = 0;
        for (int S = 0; S < W; ++S)
            for (int H = 0; H <= S; ++H)
                tiles.push_back(Tile{S, H, H == S ? -1 : (hk++ % 2), H == 0, H == S});
        hipEvent_t ev_sload[2], ev_sfree[2], ev_hload[2], ev_hfree[2];
        for (int k = 0; k < 2; ++k) {
            GS_HIP(hipEventCreateWithFlags(&ev_sload[k], hipEventDisableTiming));
            GS_HIP(hipEventCreateWithFlags(&ev_sfree[k], hipEventDisableTiming));
            GS_HIP(hipEventCreateWithFlags(&ev_hload[k], hipEventDisableTiming));
            GS_HIP(hipEventCreateWithFlags(&ev_hfree[k], hipEventDisableTiming));
        }
        hipStream_t cs = ctx.copy_stream;
        const uint32_t *hc = g.hcol.as<uint32_t>();
        const uint8_t *hb = g.hbin.as<uint8_t>();
        auto enqueue_load = [&](const Tile &t) {
            if (t.first_of_S) {
                const int k = t.S % 2;
                const uint64_t e0 = g.win_edge[t.S], ne = g.win_edge[t.S + 1] - e0;
                GS_HIP(hipStreamWaitEvent(cs, ev_sfree[k], 0));
                GS_HIP(hipMemcpyAsync(scol[k].p, hc + e0, ne * 4, hipMemcpyHostToDevice, cs));
                GS_HIP(hipMemcpyAsync(sbin[k].p, hb + e0, ne, hipMemcpyHostToDevice, cs));
                GS_HIP(hipEventRecord(ev_sload[k], cs));
            }
            if (t.hslot >= 0) {
                const int k = t.hslot;
                const uint64_t e0 = g.win_edge[t.H], ne = g.win_edge[t.H + 1] - e0;
                GS_HIP(hipStreamWaitEvent(cs, ev_hfree[k], 0));
                GS_HIP(hipMemcpyAsync(hcol[k].p, hc + e0, ne * 4, hipMemcpyHostToDevice, cs));
                GS_HIP(hipMemcpyAsync(hbin[k].p, hb + e0, ne, hipMemcpyHostToDevice, cs));
                GS_HIP(hipEventRecord(ev_hload[k], cs));
            }
        };
        enqueue_load(tiles[0]);
        for (size_t ti = 0; ti < tiles.size(); ++ti) {
            const Tile &t = tiles[ti];
            if (ti + 1 < tiles.size()) enqueue_load(tiles[ti + 1]);
            const int sk = t.S % 2;
            GS_HIP(hipStreamWaitEvent(s, ev_sload[sk], 0));
            C3Args b = a;
            b.scol = scol[sk].as<uint32_t>();
            b.sbin = sbin[sk].as<uint8_t>();
            b.sbase = g.win_edge[t.S];
            b.s0 = (uint32_t)g.win[t.S];
            b.s1 = (uint32_t)g.win[t.S + 1];
            if (t.hslot >= 0) {
                GS_HIP(hipStreamWaitEvent(s, ev_hload[t.hslot], 0));
                b.hcol = hcol[t.hslot].as<uint32_t>();
                b.hbin = hbin[t.hslot].as<uint8_t>();
            } else {
                b.hcol = b.scol;
                b.hbin = b.sbin;
            }
            b.hbase = g.win_edge[t.H];
            b.h0 = (uint32_t)g.win[t.H];
            b.h1 = (uint32_t)g.win[t.H + 1];
            b.queue = queues + ti * kNumQueues;
            launch3_any(ctx, s, b, P, weighted, anchored);
            if (t.hslot >= 0) GS_HIP(hipEventRecord(ev_hfree[t.hslot], s));
            if (t.last_of_S) GS_HIP(hipEventRecord(ev_sfree[sk], s));
        }
        GS_HIP(hipStreamSynchronize(s));
        GS_HIP(hipStreamSynchronize(cs));
        for (int k = 0; k < 2; ++k) {
            (void)hipEventDestroy(ev_sload[k]);
            (void)hipEventDestroy(ev_sfree[k]);
            (void)hipEventDestroy(ev_hload[k]);
            (void)hipEventDestroy(ev_hfree[k]);
        }
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
    ctx.t.kernel_launches = g.n > 0 ? (uint64_t)ntiles : 0;
    // merge-walk bytes: each hub-spoke step reads both forward half-lists,
    // 5 bytes per entry: 2.5 B x sum_i m_i^2 over full degrees m_i
    ctx.t.alg_bytes = g.stats_ready ? (uint64_t)(2.5 * (double)g.sum_sq_deg) : 0;
}

}  // namespace gsn
