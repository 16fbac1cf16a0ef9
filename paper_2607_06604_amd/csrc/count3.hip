// count3.hip - binned triangle counts on the forward CSR (paper Sec. 2.2
// hub-and-spoke enumeration, Sec. 3.1 sorted-list intersection, Sec. 3.5.2
// one work group per hub with lanes on the inner loop, Sec. 3.5.3 tiles).
//
// Every triangle {i < j < k} (labels) is found exactly once: at hub i, spoke
// j in N+(i), third vertex k in N+(i) and N+(j). The work group of a hub
// stages N+(i) in an LDS hash table (label -> bin of edge (i,k)) and cuts the
// forward rows of its spokes into steps of S = 2^glog consecutive entries,
// listed in an LDS step table; a group of S lanes takes one step and each of
// its lanes probes one candidate k. A hit has its three bins (ij from the
// step's spoke, ik from the table, jk from the row), which a configuration
// table turns into the LDS address of a 32-bit counter; the counters are
// flushed into the 64-bit result before any of them could wrap, and the
// triangle total is the sum of what was flushed. Weighted counts add the
// exact integer t * 2^s of each triangle into 64-bit LDS halves, merged into
// 128-bit sums.
//
// A launch covers one tile: hubs in [h0, h1) and spokes in [s0, s1). A
// resident graph is a single tile; a host-tiled graph runs every (hub
// window, spoke window >= hub window) pair, so each spoke (i, j) -- and with
// it every triangle -- belongs to exactly one tile.
//
// Hubs are pulled from eight queues, one per slice of the tile's hub range,
// in runs of consecutive hubs (next_hub_in).
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
    int packed;             // hash entries hold (bin << 24 | label): labels < 2^24 - 1
    int glog;               // entries per step = 2^glog
    int mode;               // hit counter addressing: kRank, kLut or kCube
    int kmax;               // hubs per group (1..kMaxGroup)
    int yshift;             // packed hash entries: bin << yshift | hub << 24 | label
    uint64_t group_cap;     // rows of a group (beyond the first hub) fit this many entries
    uint32_t maxdeg;
    uint32_t tmax;          // steps per table fill
    uint32_t tcap;          // table entries: tmax + padding of one pass
    uint32_t anchor_lo, anchor_hi;
    double wmul;            // 2^wscale
    int wgen;               // some weight is negative or some term may reach 2^63
    uint64_t flush_limit;   // flush LDS counters before this many increments
    uint32_t *queue;        // kQueueWords words
    unsigned long long *hist;   // nconf
    unsigned long long *wsum;   // 2*nconf (lo, hi)
    unsigned long long *ntri;   // 1
    unsigned long long *probes; // candidates probed (nullable)
    uint32_t *err;          // bit 1: LDS addressing
    uint64_t wspan;         // WIDE: entries a segment of spoke rows may span from its first row
    const uint16_t *cfg3;   // kLut / kCube: configuration index of ordered triple (x*nb + y)*nb + z
    const uint32_t *tiles;  // hub tiles of about equal cost: tile t = [tiles[t], tiles[t+1]) (or null)
    uint32_t ntiles;
};

constexpr int kUnroll3 = 4;              // steps per lane per pass
// Weighted unanchored counts (six wavefronts per SIMD at most: their LDS
// allows two groups per CU) keep more row loads in flight: 6 steps per pass
// (9.22 s on the 2e6-point weighted count against 9.44 with 5 and 9.56 with
// 4; 7 or 8 would spill, as would 6 with the anchored bookkeeping).
constexpr int kUnroll3W = 6;
__host__ __device__ constexpr int unroll3(bool weighted, bool anchored) {
    return weighted && !anchored ? kUnroll3W : kUnroll3;
}
constexpr int kLutMaxBins = 24;          // nb^3 u16 table up to 27 KB
constexpr int kCubeMaxBins = 16;         // nb^3 u32 counters up to 16 KB
constexpr int kMaxGroup = 4;             // hubs per group: two bits in a step entry

// How a hit finds its counter: the configuration index from the rank tables
// (kRank), an nb^3 table of counter addresses (kLut), or no index at all --
// one LDS counter per ordered bin triple (x, y, z), folded into
// configurations when the counters are flushed (kCube, unweighted only).
enum { kRank = 0, kLut = 1, kCube = 2 };
// Spoke rows of one hub are addressed by 32-bit offsets from the hub's
// first spoke row: byte offsets (loads with a scalar base) below 2^30
// entries, entry offsets with 64-bit addresses (WIDE launches) below 2^32.
constexpr uint64_t kNarrowSpan = 1ull << 30;
constexpr uint64_t kWideSpan = 1ull << 32;

// LDS layout of one work group (byte offsets). The configuration table and
// the counters come first so that their byte addresses fit 16 bits.
struct Layout3 {
    uint32_t cube, lut, hist, wlo, whi, hkey, hxb, tab, mw, mperm, rtab, wtot, misc, hbin, total;
};

__host__ __device__ inline Layout3 layout3(int block, uint32_t H, uint32_t maxdeg, uint32_t tcap, int nconf,
                                           int nb, bool weighted, bool anchored, bool lds_hist, bool packed,
                                           int mode) {
    if (!lds_hist) nconf = 0;
    Layout3 L{};
    uint32_t o = 0;
    // with the cube the configuration counters are only written while the
    // step table is idle (flushes), so they share its space
    const bool alias = mode == kCube && lds_hist;
    L.cube = o;   if (mode == kCube) o = lds_align(o + 4 * nb * nb * nb, 16);
    L.lut = o;    if (mode == kLut) o = lds_align(o + 2 * nb * nb * nb, 16);
    L.hist = o;   if (!alias) o = lds_align(o + 4 * nconf, 16);
    L.wlo = o;    if (weighted) o = lds_align(o + 8 * nconf, 16);
    L.whi = o;    if (weighted) o = lds_align(o + 8 * nconf, 16);
    L.hkey = o;   o = lds_align(o + 4 * H, 16);
    L.tab = o;    o = lds_align(o + std::max(8 * tcap, alias ? 4u * nconf : 0u), 16);
    if (alias) L.hist = L.tab;
    L.mw = o;     if (weighted) o = lds_align(o + 8 * block, 16);
    L.mperm = o;  if (anchored) o = lds_align(o + 4 * block, 16);
    L.rtab = o;   o = lds_align(o + 8 * (nb + 1), 16);
    L.wtot = o;   o = lds_align(o + 8 * (block / 64 + 1), 16);
    L.misc = o;   o = lds_align(o + 176, 16);
    L.hxb = o;    o = lds_align(o + maxdeg, 16);
    L.hbin = o;   if (!packed) o = lds_align(o + H, 16);
    L.total = o;
    return L;
}

// Fibonacci hash of a label below 2^24 in 24-bit arithmetic: the top log2h
// bits of k * A mod 2^24 with A = 2^24 / golden ratio (odd). Both factors fit
// 24 bits, so the multiply is the full-rate 24-bit one.
__device__ __forceinline__ uint32_t label_hash24(uint32_t k, int log2h) {
    return (((k & 0xFFFFFFu) * 0x9E3779u) & 0xFFFFFFu) >> (24 - log2h);
}

template <bool PACK>
__device__ __forceinline__ uint32_t hub_hash(uint32_t k, int log2h) {
    return PACK ? label_hash24(k, log2h) : label_hash(k, log2h);
}


__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Move the LDS counters into the 64-bit results (and their sum into the
// triangle total); the caller brackets it with barriers.
template <int BLOCK, bool WEIGHTED, bool LDS_HIST>
__device__ void flush3(const C3Args &a, const Layout3 &L, unsigned char *sm, unsigned long long *hout,
                       unsigned long long *tout) {
    if (!LDS_HIST) return;
    uint32_t *hist = (uint32_t *)(sm + L.hist);
    if (!WEIGHTED && a.mode == kCube) {
        // fold the ordered bin triples into their configurations (the
        // configuration counters share the idle step table: clear them first)
        for (int b = threadIdx.x; b < a.nconf; b += BLOCK) hist[b] = 0;
        __syncthreads();
        uint32_t *cube = (uint32_t *)(sm + L.cube);
        const int n3 = a.nb * a.nb * a.nb;
        for (int t = threadIdx.x; t < n3; t += BLOCK) {
            const uint32_t v = cube[t];
            if (v) {
                cube[t] = 0;
                atomicAdd(&hist[a.cfg3[t]], v);
            }
        }
        __syncthreads();
    }
    unsigned long long sum = 0;
    for (int b = threadIdx.x; b < a.nconf; b += BLOCK) {
        const uint32_t v = hist[b];
        if (v) {
            atomicAdd(&hout[b], (unsigned long long)v);
            hist[b] = 0;
            sum += v;
        }
        if (WEIGHTED) {
            unsigned long long *wlo = (unsigned long long *)(sm + L.wlo);
            unsigned long long *whi = (unsigned long long *)(sm + L.whi);
            const unsigned long long lo = wlo[b], hi = whi[b];
            if (lo | hi) {
                add128_words(&a.wsum[2 * b], lds_sum128(lo, hi));
                wlo[b] = 0;
                whi[b] = 0;
            }
        }
    }
    sum = wave_sum64(sum);
    if ((threadIdx.x & 63) == 0 && sum && tout) atomicAdd(tout, sum);
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

// What the walk over one step table reads or updates.
struct Walk {
    const uint2 *tab;             // steps: (row offset, entries | slot << 7 | x term << 17)
    const uint32_t *hkey;         // hub hash
    const uint8_t *hbin;          // hub bins per slot (unpacked hash)
    const int *ta, *tb;           // rank tables
    const double *mw;             // spoke weights (by spoke slot)
    const uint32_t *mperm;        // spoke original indices (by spoke slot)
    unsigned char *sm;            // LDS base
    unsigned long long *hout;     // global counters (!LDS_HIST)
    unsigned long long *wlo, *whi, *wsum;
    gbl_u32 *srow;                // spoke rows of this hub (32-bit offsets)
    gbl_u8 *sbrow;
    const double *w;
    const uint32_t *perm;
    const double *hw;             // weights of the group's hubs
    const uint32_t *hp;           // original indices of the group's hubs
    uint32_t mask, hist_addr;     // LDS byte address of counter 0
    uint32_t ys, qmask;           // packed keys: bin at bit ys, key bits below
    int log2h, nb, glog;
    double wmul;
    int wgen;
    uint32_t anchor_lo, anchor_hi;
};

// One hit: bins x (spoke, in the step's x term), y (hub table), z (row).
// The x term is the LDS address, in 2-byte units, of plane x of the
// ordered-triple counters (kCube) or of row x of the configuration table
// (kLut), whose entries are counter addresses (or indices); with kRank it is
// x itself.
template <int MODE, bool WEIGHTED, bool ANCHORED, bool LDS_HIST, bool WGEN>
__device__ __forceinline__ void count_hit(const Walk &c, uint32_t pk, double wk, uint32_t meta, uint32_t y,
                                          uint32_t z, uint32_t hub, unsigned long long &mytri) {
    // pk, wk: original index and weight of the third vertex (anchored / weighted)
    const uint32_t slot = (meta >> 7) & 1023u;
    if (ANCHORED) {
        const uint32_t mm = min(c.hp[hub], min(c.mperm[slot], pk));
        if (mm < c.anchor_lo || mm >= c.anchor_hi) return;
    }
    if (MODE == kCube) {
        // y, z < 256 and nb <= 16: 24-bit multiply
        const uint32_t addr = 2 * (meta >> 17) + 4 * ((y & 0xFFu) * ((uint32_t)c.nb & 0xFFu) + z);
        __hip_atomic_fetch_add((lds_u32 *)(size_t)addr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        return;
    }
    uint32_t addr, idx;
    if (MODE == kLut) {
        // y, z < 256 and nb <= 24: 24-bit multiply
        const uint32_t v = *(lds_u16 *)(size_t)(2 * ((meta >> 17) + (y & 0xFFu) * ((uint32_t)c.nb & 0xFFu) + z));
        addr = v;
        idx = LDS_HIST ? (v - c.hist_addr) >> 2 : v;
    } else {
        const int x = (int)(meta >> 17);
        const int lo = min(x, min((int)y, (int)z)), hi = max(x, max((int)y, (int)z));
        const int mid = x + (int)y + (int)z - lo - hi;
        idx = (uint32_t)(c.ta[lo] + c.tb[mid] + hi);
        addr = c.hist_addr + 4 * idx;
    }
    if (LDS_HIST) {
        __hip_atomic_fetch_add((lds_u32 *)(size_t)addr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        atomicAdd(&c.hout[idx], 1ull);
        ++mytri;
    }
    if (WEIGHTED && !WGEN) {
        // positive weights whose triangle terms stay below 2^63: the
        // product of the weights in ascending order as one 64-bit integer
        // (compare-and-swap: 32-bit selects, cheaper than float64 min / max
        // with their canonicalisations)
        double p = c.hw[hub], q = c.mw[slot], r = wk, t;
        if (p > q) { t = p; p = q; q = t; }
        if (q > r) { t = q; q = r; r = t; }
        if (p > q) { t = p; p = q; q = t; }
        const double prod = __dmul_rn(__dmul_rn(p, q), r);
        const unsigned long long ti = big_term_u64(__dmul_rn(prod, c.wmul));
        if (LDS_HIST) {
            atomicAdd(&c.wlo[idx], ti & 0xFFFFFFFFull);
            atomicAdd(&c.whi[idx], ti >> 32);
        } else {
            add128_words(&c.wsum[2 * idx], (__int128)ti);
        }
    }
    if (WEIGHTED && WGEN) {
        // any signs, any terms: magnitudes in ascending order multiplied left
        // to right, signed by the product of the signs; terms below 2^63 into
        // the LDS sums, wider ones into the global 128-bit sums
        const double w0 = c.hw[hub], w1 = c.mw[slot];
        const bool ng = (w0 < 0.0) ^ (w1 < 0.0) ^ (wk < 0.0);
        double p = fabs(w0), q = fabs(w1), r = fabs(wk), t;
        if (p > q) { t = p; p = q; q = t; }
        if (q > r) { t = q; q = r; r = t; }
        if (p > q) { t = p; p = q; q = t; }
        const double x = __dmul_rn(__dmul_rn(__dmul_rn(p, q), r), c.wmul);
        if (LDS_HIST && narrow_term(x)) {
            const long long m = (long long)big_term_u64(x);
            lds_term(&c.wlo[idx], &c.whi[idx], ng ? -m : m);
        } else {
            add128_words(&c.wsum[2 * idx], wide_term(x, ng));
        }
    }
}

// Steps [0, nsteps) of the table: lane group g (2^glog lanes) of the work
// group takes steps g, g + G, ... (G groups), U of them per pass with their
// row loads issued back to back; lane s of a group probes entry s of its
// step. The table is padded with empty steps past nsteps, and lanes past
// the end of a step load (and ignore) the row slack, so the loads need no
// branch.
template <int BLOCK, bool PACK, int MODE, bool WEIGHTED, bool ANCHORED, bool LDS_HIST, bool WIDE, bool WGEN>
__device__ __forceinline__ void walk3(const Walk &c, uint32_t nsteps, unsigned long long &mytri) {
    constexpr int U = unroll3(WEIGHTED, ANCHORED);
    const uint32_t glog = (uint32_t)c.glog;
    const uint32_t sub = threadIdx.x & ((1u << glog) - 1u);
    const uint32_t per = (uint32_t)BLOCK >> glog;
    const uint2 *tp = c.tab + (threadIdx.x >> glog);
    for (uint32_t base = 0; base < nsteps; base += U * per) {
        uint32_t kk[U], zz[U], meta[U], hub[U], hh[U], key[U];
        bool ok[U];
        // 1. row loads of all U steps (a slot past the table's end is skipped
        //    by the whole work group)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = false;
            kk[u] = zz[u] = meta[u] = hub[u] = 0;
            if (base + u * per < nsteps) {
                const uint2 e = tp[base + u * per];
                ok[u] = sub < (e.y & 127u);
                meta[u] = e.y;
                if (WIDE) {
                    const uint32_t pos = e.x + sub;
                    kk[u] = c.srow[pos];
                    zz[u] = c.sbrow[pos];
                } else {
                    // hub of the group in the top two bits
                    const uint32_t pos = (e.x & 0x3FFFFFFFu) + sub;
                    hub[u] = e.x >> 30;
                    kk[u] = *(gbl_u32 *)((gbl_u8 *)c.srow + (pos << 2));
                    zz[u] = c.sbrow[pos];
                }
            }
        }
        // 2. first probes of all U candidates
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (PACK) {
                hh[u] = label_hash24(kk[u] ^ (hub[u] << 22), c.log2h);
                kk[u] = (hub[u] << 24) | (kk[u] & 0xFFFFFFu);   // the key bits
            } else {
                hh[u] = label_hash(kk[u], c.log2h);
            }
            key[u] = c.hkey[hh[u]];
        }
        // 3. probe sequences to their ends: hit flag and the bin of (hub, k).
        //    Unweighted walks advance the U chains together (one LDS round
        //    trip per step of the longest chain: 6.95 -> 6.84 ms on a 1e6-point
        //    clustered count); weighted walks, six steps per pass, run them
        //    one after another (together: 9.22 -> 10.27 s on the 2e6-point
        //    weighted count).
        bool hit[U];
        uint32_t yy[U];
        if (!WEIGHTED) {
            bool live[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t kv = key[u];
                live[u] = ok[u] && (PACK ? ((kv ^ kk[u]) & c.qmask) != 0 : kv != kk[u]) && kv != kEmptyKey;
            }
            bool any = false;
#pragma unroll
            for (int u = 0; u < U; ++u) any |= live[u];
            while (any) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (live[u]) {
                        hh[u] = (hh[u] + 1) & c.mask;
                        key[u] = c.hkey[hh[u]];
                    }
                any = false;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t kv = key[u];
                    live[u] = live[u] && (PACK ? ((kv ^ kk[u]) & c.qmask) != 0 : kv != kk[u]) && kv != kEmptyKey;
                    any |= live[u];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t kv = key[u];
                hit[u] = ok[u] && kv != kEmptyKey && (PACK || kv == kk[u]);
                yy[u] = 0;
                if (PACK) {
                    yy[u] = kv >> c.ys;
                    kk[u] &= 0xFFFFFFu;
                } else if (hit[u]) {
                    yy[u] = c.hbin[hh[u]];
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                hit[u] = false;
                yy[u] = 0;
                if (!ok[u]) continue;
                const uint32_t q = kk[u];
                uint32_t h = hh[u], kv = key[u];
                if (PACK) {
                    while (((kv ^ q) & c.qmask) != 0 && kv != kEmptyKey) {
                        h = (h + 1) & c.mask;
                        kv = c.hkey[h];
                    }
                    hit[u] = kv != kEmptyKey;
                    yy[u] = kv >> c.ys;
                    kk[u] = q & 0xFFFFFFu;
                } else {
                    while (kv != q && kv != kEmptyKey) {
                        h = (h + 1) & c.mask;
                        kv = c.hkey[h];
                    }
                    hit[u] = kv == q;
                    if (hit[u]) yy[u] = c.hbin[h];
                }
            }
        }
        // 4. the third vertex's weight / original index, loaded for all hits
        //    at once, then the hits
        double wk[U];
        uint32_t pk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            wk[u] = 0.0;
            pk[u] = 0;
            if (WEIGHTED && hit[u]) wk[u] = c.w[kk[u]];
            if (ANCHORED && hit[u]) pk[u] = c.perm[kk[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (hit[u])
                count_hit<MODE, WEIGHTED, ANCHORED, LDS_HIST, WGEN>(c, pk[u], wk[u], meta[u], yy[u], zz[u],
                                                                    WIDE ? 0u : hub[u], mytri);
    }
}

template <int BLOCK, bool WEIGHTED, bool ANCHORED, bool LDS_HIST, bool WIDE, bool WGEN>
__device__ __forceinline__ void walk3_modes(bool packed, int mode, const Walk &c, uint32_t nsteps,
                                            unsigned long long &mytri) {
    // kCube only for unweighted counts into LDS (never selected otherwise)
    constexpr int CUBE = (!WEIGHTED && LDS_HIST) ? kCube : kLut;
    if (packed) {
        if (mode == kCube) walk3<BLOCK, true, CUBE, WEIGHTED, ANCHORED, LDS_HIST, WIDE, WGEN>(c, nsteps, mytri);
        else if (mode == kLut) walk3<BLOCK, true, kLut, WEIGHTED, ANCHORED, LDS_HIST, WIDE, WGEN>(c, nsteps, mytri);
        else walk3<BLOCK, true, kRank, WEIGHTED, ANCHORED, LDS_HIST, WIDE, WGEN>(c, nsteps, mytri);
    } else {
        if (mode == kCube) walk3<BLOCK, false, CUBE, WEIGHTED, ANCHORED, LDS_HIST, WIDE, WGEN>(c, nsteps, mytri);
        else if (mode == kLut) walk3<BLOCK, false, kLut, WEIGHTED, ANCHORED, LDS_HIST, WIDE, WGEN>(c, nsteps, mytri);
        else walk3<BLOCK, false, kRank, WEIGHTED, ANCHORED, LDS_HIST, WIDE, WGEN>(c, nsteps, mytri);
    }
}

// General weights (negative ones, or terms that may reach 2^63) take their
// own instance of the walk, so positive narrow weights keep the short one.
template <int BLOCK, bool WEIGHTED, bool ANCHORED, bool LDS_HIST, bool WIDE>
__device__ __forceinline__ void walk3_any(bool packed, int mode, const Walk &c, uint32_t nsteps,
                                          unsigned long long &mytri) {
    if (WEIGHTED && c.wgen) walk3_modes<BLOCK, WEIGHTED, ANCHORED, LDS_HIST, WIDE, true>(packed, mode, c, nsteps, mytri);
    else walk3_modes<BLOCK, WEIGHTED, ANCHORED, LDS_HIST, WIDE, false>(packed, mode, c, nsteps, mytri);
}

// Plain unbatched counts fit 64 VGPRs: eight wavefronts per SIMD.
// SEG (with WIDE): a hub's spoke rows may lie more than the segment span
// apart (graphs of 2^32 or more forward entries), so chunks whose rows spread
// that far go in segments. Weighted 768-thread groups run two per CU: six
// wavefronts per SIMD.
template <int BLOCK, bool WEIGHTED, bool ANCHORED, bool LDS_HIST, bool BATCH, bool WIDE, bool SEG = false>
__global__ __launch_bounds__(BLOCK, BLOCK == 768 ? 6 : (WEIGHTED || ANCHORED) ? 1 : 8) void k_count3(C3Args a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const uint32_t H = 1u << a.log2h, mask = H - 1;
    const Layout3 L = layout3(BLOCK, H, a.maxdeg, a.tcap, a.nconf, a.nb, WEIGHTED, ANCHORED, LDS_HIST,
                              a.packed, a.mode);
    uint16_t *lut = (uint16_t *)(sm + L.lut);
    uint32_t *cube = (uint32_t *)(sm + L.cube);
    uint32_t *hkey = (uint32_t *)(sm + L.hkey);
    uint8_t *hxb = (uint8_t *)(sm + L.hxb);
    uint8_t *hbin = (uint8_t *)(sm + L.hbin);
    uint2 *tab = (uint2 *)(sm + L.tab);
    double *mw = (double *)(sm + L.mw);
    uint32_t *mperm = (uint32_t *)(sm + L.mperm);
    uint32_t *hist = (uint32_t *)(sm + L.hist);
    unsigned long long *wlo = (unsigned long long *)(sm + L.wlo);
    unsigned long long *whi = (unsigned long long *)(sm + L.whi);
    int *ta = (int *)(sm + L.rtab);
    int *tb = ta + (a.nb + 1);
    uint64_t *wtot64 = (uint64_t *)(sm + L.wtot);
    // the current hub group: first hub and hub count, catalogue, row
    // bounds, largest label per row, hub weights, indices and marks
    uint32_t *s_hub = (uint32_t *)(sm + L.misc);
    int *s_g = (int *)(sm + L.misc + 8);
    uint64_t *s_rb = (uint64_t *)(sm + L.misc + 16);          // kMaxGroup + 1
    uint32_t *s_kmax = (uint32_t *)(sm + L.misc + 56);        // kMaxGroup
    double *s_hw = (double *)(sm + L.misc + 72);              // kMaxGroup
    uint32_t *s_hp = (uint32_t *)(sm + L.misc + 104);         // kMaxGroup
    uint8_t *s_mk = (uint8_t *)(sm + L.misc + 120);           // kMaxGroup
    const int tid = threadIdx.x;
    const uint32_t glog = (uint32_t)a.glog, S = 1u << glog;
    // the configuration table holds 16-bit LDS addresses
    const uint32_t smb = lds_addr(sm);
    if ((a.mode == kLut && smb + L.hist + 4 * (uint32_t)a.nconf > 0xFFFFu) ||
        (a.mode == kCube && smb + L.cube + 4 * (uint32_t)(a.nb * a.nb * a.nb) > 0xFFFFu)) {
        if (tid == 0) atomicOr(a.err, 2u);
        return;
    }

    for (uint32_t s = tid; s < H; s += BLOCK) hkey[s] = kEmptyKey;
    if (LDS_HIST)
        for (int b = tid; b < a.nconf; b += BLOCK) {
            hist[b] = 0;
            if (WEIGHTED) { wlo[b] = 0; whi[b] = 0; }
        }
    if (a.mode == kCube)
        for (int t = tid; t < a.nb * a.nb * a.nb; t += BLOCK) cube[t] = 0;
    for (int b = tid; b < a.nb; b += BLOCK) {
        ta[b] = rank_a(a.nb, b);
        tb[b] = rank_b(a.nb, b);
    }
    // table entry (x, y, z) at x*nb*nb + y*nb + z: the counter's absolute
    // LDS byte address, or its index when the counters are global
    if (a.mode == kLut)
        for (int t = tid; t < a.nb * a.nb * a.nb; t += BLOCK) {
            const uint32_t idx = a.cfg3[t];
            lut[t] = (uint16_t)(LDS_HIST ? smb + L.hist + 4 * idx : idx);
        }
    __syncthreads();

    unsigned long long mytri = 0;  // global counters: this thread's hits
    uint64_t acc = 0;   // candidates probed since the last flush: bounds the increments (uniform)
    uint64_t probed = 0;  // candidates probed in all (uniform)
    // thread 0's claimed hubs and tile claims live in LDS (no registers held
    // across the loop)
    HubCursor &cursor = *(HubCursor *)(sm + L.misc + 128);
    HubCursor &tcursor = *(HubCursor *)(sm + L.misc + 144);
    unsigned long long *s_seg = (unsigned long long *)(sm + L.misc + 160);   // WIDE: a segment's first row
    if (tid == 0) {
        cursor = HubCursor();
        tcursor = HubCursor();
    }
    int cur = -1;       // batched launch: catalogue whose counts the LDS holds
    // the CSR view of the current hub: the launch's tile, or one catalogue
    const uint64_t *rp = a.rp;
    const uint32_t *hcol = a.hcol, *scol = a.scol;
    const uint8_t *hbinp = a.hbin, *sbinp = a.sbin;
    uint64_t hbase = a.hbase, sbase = a.sbase;
    uint32_t s0 = a.s0, s1 = a.s1;
    unsigned long long *hout = a.hist, *tout = a.ntri;

    Walk c;
    c.tab = tab; c.hkey = hkey; c.hbin = hbin; c.ta = ta; c.tb = tb; c.mw = mw;
    c.mperm = mperm; c.sm = sm; c.wlo = wlo; c.whi = whi; c.wsum = a.wsum; c.w = a.w; c.perm = a.perm;
    c.mask = mask; c.hist_addr = smb + L.hist; c.log2h = a.log2h; c.nb = a.nb; c.glog = a.glog; c.wmul = a.wmul;
    c.wgen = a.wgen;
    c.anchor_lo = a.anchor_lo; c.anchor_hi = a.anchor_hi; c.hw = s_hw; c.hp = s_hp;
    c.ys = (uint32_t)a.yshift;
    c.qmask = (1u << a.yshift) - 1u;

    // hub groups: up to a.kmax consecutive hubs whose rows (contiguous in
    // the CSR) fit the table together; their spokes share one step table
    const uint32_t kmaxg = (uint32_t)a.kmax;
    while (true) {
        if (tid < 64) {
            // wavefront 0 forms the group: lane 0 owns the run of claimed
            // hubs, lanes 0..kmax load the row bounds of its next hubs
            uint32_t v0 = kEmptyKey, avail = 0;
            bool have = false;
            if (tid == 0) {
                if (a.tiles) {
                    // the queues hand out tiles; a tile's hubs go in order
                    have = cursor.cur < cursor.end;
                    while (!have) {
                        const uint32_t t = next_hub_in(a.queue, 0, a.ntiles, gridDim.x, tcursor, 1);
                        if (t == kEmptyKey) break;
                        cursor.cur = a.tiles[t];
                        cursor.end = a.tiles[t + 1];
                        have = cursor.cur < cursor.end;
                    }
                } else {
                    have = BATCH ? next_hub_run(a.queue, 0, a.nvirt, gridDim.x, cursor)
                                 : next_hub_run(a.queue, a.h0, a.h1, gridDim.x, cursor);
                }
            }
            if (have) {
                v0 = cursor.cur;
                avail = cursor.end - cursor.cur;
            }
            v0 = __shfl(v0, 0, 64);
            avail = __shfl(avail, 0, 64);
            if (v0 != kEmptyKey) {
                const uint64_t *grp = a.rp;
                uint32_t i0 = v0;
                int g = 0;
                if (BATCH) {
                    // a group stays inside one catalogue
                    g = graph_of(a.gd, a.ngraph, v0);
                    i0 = (uint32_t)(v0 - a.gd[g].v0);
                    grp = a.gd[g].rp;
                    avail = min(avail, a.gd[g].n - i0);
                }
                const uint32_t na = min(avail, kmaxg);
                const uint64_t r = tid <= na ? grp[i0 + tid] : 0;
                const uint64_t rn = __shfl_down(r, 1, 64);
                // rows of the first l + 1 hubs, and how many hubs fit
                const uint64_t span = __shfl(r, 0, 64);
                const bool fits = tid < na && (tid == 0 || rn - span <= a.group_cap);
                const uint32_t K = max(1u, (uint32_t)__popcll(__ballot(fits)));
                if (tid <= K) s_rb[tid] = r;
                if (tid < K) {
                    if (ANCHORED) s_hp[tid] = a.perm[i0 + tid];
                    if (ANCHORED) s_mk[tid] = a.mark ? a.mark[i0 + tid] : 1;
                    if (WEIGHTED) s_hw[tid] = a.w[i0 + tid];
                }
                if (tid == 0) {
                    s_hub[0] = i0;
                    s_hub[1] = K;
                    *s_g = g;
                    cursor.cur += K;
                }
            } else if (tid == 0) {
                s_hub[0] = kEmptyKey;
            }
        }
        __syncthreads();
        const uint32_t i0 = __builtin_amdgcn_readfirstlane(s_hub[0]);
        if (i0 == kEmptyKey) break;
        const uint32_t K = __builtin_amdgcn_readfirstlane(s_hub[1]);
        if (BATCH) {
            const int g = __builtin_amdgcn_readfirstlane(*s_g);
            if (g != cur) {
                // a new catalogue: hand the previous one its counts first
                if (cur >= 0) {
                    flush3<BLOCK, WEIGHTED, LDS_HIST>(a, L, sm, hout, tout);
                    acc = 0;
                    __syncthreads();
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
        // rows of the group: [rb0, rb0 + D) in the hub rows; hub k's row
        // starts at offset ofs(k) (ofs(k) = D for k >= K)
        const uint64_t rb0 = uniform64(s_rb[0]);
        const uint32_t D = (uint32_t)(uniform64(s_rb[K]) - rb0);
        uint32_t ofs1 = D, ofs2 = D, ofs3 = D;
        if (K > 1) ofs1 = (uint32_t)(uniform64(s_rb[1]) - rb0);
        if (K > 2) ofs2 = (uint32_t)(uniform64(s_rb[2]) - rb0);
        if (K > 3) ofs3 = (uint32_t)(uniform64(s_rb[3]) - rb0);
        const uint64_t beg = rb0 - hbase;
        // spokes of this tile have labels >= jlo; their rows are addressed
        // from rb = rp[jlo]
        const uint32_t jlo = max(i0 + 1, s0);
        if (D < 2 || jlo >= s1) { __syncthreads(); continue; }
        const uint64_t rb = uniform64(jlo == i0 + 1 ? s_rb[1] : rp[jlo]);
        // uniform: the row loads take these as their scalar base (a WIDE
        // launch re-bases them per segment of spokes below)
        c.srow = (gbl_u32 *)uniform64((uint64_t)(scol + (rb - sbase)));
        c.sbrow = (gbl_u8 *)uniform64((uint64_t)(sbinp + (rb - sbase)));
        c.hout = hout;

        // stage the group's rows: labels and bins in order, and (hub, label)
        // -> bin in the hash; the first spoke chunk's row bounds load along
        uint32_t st0 = 0, len0 = 0, j0 = 0;
        for (uint32_t e = tid; e < D; e += BLOCK) {
            const uint32_t k = hcol[beg + e];
            const uint32_t y = hbinp[beg + e];
            const uint32_t hk = (e >= ofs1) + (e >= ofs2) + (e >= ofs3);
            const uint32_t next = hk == 0 ? ofs1 : hk == 1 ? ofs2 : hk == 2 ? ofs3 : D;
            // the last entry of a hub's row is no spoke; it carries the row's
            // largest label
            if (e == (uint32_t)tid) j0 = k;
            if (e + 1 == next) s_kmax[hk] = k;
            else if (e == (uint32_t)tid && k >= s0 && k < s1) {
                const uint64_t rk = rp[k];
                st0 = (uint32_t)(rk - rb);
                len0 = (uint32_t)(rp[k + 1] - rk);
            }
            hxb[e] = (uint8_t)y;
            uint32_t s, v;
            if (a.packed) {
                s = label_hash24(k ^ (hk << 22), a.log2h);
                v = (y << c.ys) | (hk << 24) | k;
            } else {
                s = label_hash(k, a.log2h);
                v = k;
            }
            while (atomicCAS(&hkey[s], kEmptyKey, v) != kEmptyKey) s = (s + 1) & mask;
            if (!a.packed) hbin[s] = (uint8_t)y;
        }
        __syncthreads();

        // spokes in chunks of BLOCK entries, one per thread; spokes outside
        // the tile (or of hubs that own no anchored triangle) add nothing
        for (uint32_t c0 = 0; c0 < D; c0 += BLOCK) {
            const uint32_t sidx = c0 + tid;
            uint32_t len0c = 0, xv = 0, hk = 0;
            uint64_t rj = 0;   // first entry of the spoke's row
            bool pending = false;
            if (sidx < D) {
                hk = (sidx >= ofs1) + (sidx >= ofs2) + (sidx >= ofs3);
                const uint32_t next = hk == 0 ? ofs1 : hk == 1 ? ofs2 : hk == 2 ? ofs3 : D;
                const uint32_t j = c0 == 0 ? j0 : hcol[beg + sidx];
                if (sidx + 1 < next && j >= s0 && j < s1 && (!ANCHORED || s_mk[hk])) {
                    pending = true;
                    if (c0 == 0 && !WIDE) {
                        rj = rb + st0;
                        len0c = len0;
                    } else {
                        rj = rp[j];
                        len0c = (uint32_t)(rp[j + 1] - rj);
                    }
                    const uint32_t x = hxb[sidx];
                    // the x term: plane x's LDS address in 2-byte units (15
                    // bits: LDS addresses are even and below 2^16), or x
                    xv = a.mode == kCube ? (smb + L.cube + 4 * x * (uint32_t)(a.nb * a.nb)) >> 1
                         : a.mode == kLut ? (smb + L.lut + 2 * x * (uint32_t)(a.nb * a.nb)) >> 1
                                          : x;
                    if (WEIGHTED) mw[tid] = a.w[j];
                    if (ANCHORED) mperm[tid] = a.perm[j];
                }
            }
            // A WIDE launch addresses rows by 32-bit offsets: a chunk whose
            // rows all lie within the segment span of the hub's first spoke
            // row runs from it in one pass; otherwise (seg) the chunk's
            // spokes (rows ascending with the spoke) go in segments based at
            // the first row of each.
            const bool seg = SEG && WIDE && __syncthreads_or(pending && rj + len0c - rb >= a.wspan);
            uint64_t base = rb;
            while (true) {
                if (seg) {
                    if (tid == 0) *s_seg = ~0ull;
                    __syncthreads();
                    if (pending) atomicMin(s_seg, (unsigned long long)rj);
                    __syncthreads();
                    base = uniform64(*s_seg);
                    c.srow = (gbl_u32 *)uniform64((uint64_t)(scol + (base - sbase)));
                    c.sbrow = (gbl_u8 *)uniform64((uint64_t)(sbinp + (base - sbase)));
                }
                const bool mine = pending && (!seg || rj + len0c - base < a.wspan);
                pending = pending && !mine;
                uint32_t st = mine ? (uint32_t)(rj - base) : 0u, len = mine ? len0c : 0u;
                if (mine) {
                    // entries of N+(j) above the largest label of the hub's
                    // row cannot match
                    const uint32_t kmax = s_kmax[hk];
                    if (a.trunc && len > 16 && c.srow[st + len - 1] > kmax) {
                        uint32_t lo = 0, hi = len;  // first entry > kmax
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (c.srow[st + mid] <= kmax) lo = mid + 1;
                            else hi = mid;
                        }
                        len = lo;
                    }
                }
                const uint32_t ns = (len + S - 1) >> glog;
                // one scan: steps before this spoke (low word), candidates
                // (high); wtot is next written after a barrier below
                uint64_t tot64;
                const uint64_t pre = wg_excl_scan64<BLOCK, false>(((uint64_t)len << 32) | ns, wtot64, tot64);
                const uint32_t t0 = (uint32_t)pre, T = (uint32_t)tot64;
                acc += tot64 >> 32;
                probed += tot64 >> 32;
                if (T == 0) __syncthreads();   // (the fill barrier guards wtot otherwise)
                // the table holds tmax steps: fill and walk it as often as needed
                const uint32_t xhub = WIDE ? 0u : hk << 30;
                for (uint32_t w0 = 0; w0 < T; w0 += a.tmax) {
                    const uint32_t lo = max(t0, w0), hi = min(t0 + ns, w0 + a.tmax);
                    const uint32_t nfill = min(a.tmax, T - w0);
                    for (uint32_t s = lo; s < hi; ++s) {
                        const uint32_t r = (s - t0) << glog;
                        const uint32_t cnt = min(S, len - r);
                        tab[s - w0] = make_uint2((st + r) | xhub, cnt | ((uint32_t)tid << 7) | (xv << 17));
                    }
                    for (uint32_t s = tid; s < unroll3(WEIGHTED, ANCHORED) * (BLOCK >> glog); s += BLOCK)
                        tab[nfill + s] = make_uint2(0u, 0u);
                    __syncthreads();
                    walk3_any<BLOCK, WEIGHTED, ANCHORED, LDS_HIST, WIDE>(a.packed, a.mode, c, nfill, mytri);
                    __syncthreads();
                }
                if (!seg || !__syncthreads_or(pending)) break;
            }
            if (seg) {
                // the following chunks' rows are addressed from rb again
                c.srow = (gbl_u32 *)uniform64((uint64_t)(scol + (rb - sbase)));
                c.sbrow = (gbl_u8 *)uniform64((uint64_t)(sbinp + (rb - sbase)));
            }
        }
        // the barrier at the top of the loop orders this before the next
        // group's staging
        for (uint32_t q = tid; q < H; q += BLOCK) hkey[q] = kEmptyKey;
        // a group adds at most maxdeg^2 increments (rows of at most maxdeg
        // entries, at most maxdeg spokes): flush while the next one cannot
        // pass the limit (the walk's last barrier ordered every increment)
        if (acc + (uint64_t)a.maxdeg * a.maxdeg >= a.flush_limit) {
            flush3<BLOCK, WEIGHTED, LDS_HIST>(a, L, sm, hout, tout);
            acc = 0;
        }
    }

    __syncthreads();
    flush3<BLOCK, WEIGHTED, LDS_HIST>(a, L, sm, hout, tout);
    if (tid == 0 && a.probes && probed) atomicAdd(a.probes, (unsigned long long)probed);
    if (!LDS_HIST) {
        mytri = wave_sum64(mytri);
        if ((tid & 63) == 0 && mytri && tout) atomicAdd(tout, mytri);
    }
}

// Hub tiles balanced by the sum of squared forward degrees, handed out in
// guided order. The cost prefix runs over hubs (per 256-hub chunk, then over
// chunks); the hub range is cut into eight slices of equal cost (one per hub
// queue, so an XCD keeps to one slice of labels), and each slice into tiles
// whose cost shrinks geometrically: tile u of a slice ends at the cost
// fraction 1 - (1 - 1/(k P))^(u+1) (P teams per slice, k >= 4) until 1/64
// of the slice is left, which goes in k P equal tiles. Batched launches
// number hubs across catalogues (virtual hubs).
constexpr int kTileChunk = 256;
constexpr int kTileScanBlock = 1024;

__global__ __launch_bounds__(kTileChunk) void k_hub_cost(const uint64_t *__restrict__ rp,
                                                         const GDesc *__restrict__ gd, int ng, uint32_t h0,
                                                         uint32_t h1, unsigned long long *__restrict__ pre,
                                                         unsigned long long *__restrict__ chunk_tot) {
    __shared__ uint64_t wtot[kTileChunk / 64 + 1];
    const uint32_t v = h0 + blockIdx.x * kTileChunk + threadIdx.x;
    uint64_t c = 0;
    if (v < h1) {
        uint64_t d;
        if (gd) {
            const int g = graph_of(gd, ng, v);
            const uint32_t i = (uint32_t)(v - gd[g].v0);
            d = gd[g].rp[i + 1] - gd[g].rp[i];
        } else {
            d = rp[v + 1] - rp[v];
        }
        c = d * d;
    }
    uint64_t tot;
    const uint64_t ex = wg_excl_scan64<kTileChunk>(c, wtot, tot);
    if (v < h1) pre[v - h0] = ex + c;
    if (threadIdx.x == 0) chunk_tot[blockIdx.x] = tot;
}

// Cost fraction at the end of tile u of a slice with Tq tiles (see above).
__device__ __forceinline__ double tile_frac(uint32_t u, uint32_t tq, uint32_t kp, uint32_t tstar, double lq) {
    if (u + 1 >= tq) return 1.0;
    if (u + 1 <= tstar) return 1.0 - exp(lq * (double)(u + 1));
    const double r = exp(lq * (double)tstar);
    return 1.0 - r + r * (double)(u + 1 - tstar) / (double)kp;
}

// In-place inclusive scan of the chunk costs (one work group, a contiguous
// share per thread).
__global__ __launch_bounds__(kTileScanBlock) void k_chunk_scan(unsigned long long *__restrict__ chunk_tot,
                                                                uint32_t nchunk) {
    __shared__ uint64_t wtot[kTileScanBlock / 64 + 1];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (nchunk + kTileScanBlock - 1) / kTileScanBlock;
    const uint32_t b0 = min(nchunk, tid * per), b1 = min(nchunk, b0 + per);
    uint64_t run = 0;
    for (uint32_t b = b0; b < b1; ++b) run += chunk_tot[b];
    uint64_t total;
    run = wg_excl_scan64<kTileScanBlock>(run, wtot, total);
    for (uint32_t b = b0; b < b1; ++b) {
        run += chunk_tot[b];
        chunk_tot[b] = run;
    }
}

// Tile bounds, one thread per bound: the first hub whose inclusive cost
// exceeds the bound's cost target.
__global__ void k_tile_bounds(const unsigned long long *__restrict__ pre,
                              const unsigned long long *__restrict__ chunk_tot, uint32_t nchunk, uint32_t h0,
                              uint32_t h1, uint32_t tq, uint32_t kp, uint32_t tstar, double lq,
                              uint32_t *__restrict__ tiles) {
    const uint32_t T = 8 * tq;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > T) return;
    const uint64_t total = chunk_tot[nchunk - 1];
    uint32_t at;
    if (t == 0) {
        at = h0;
    } else if (t == T) {
        at = h1;
    } else if (total == 0) {
        at = (uint32_t)min<uint64_t>(h1, h0 + (uint64_t)(h1 - h0) * t / T);
    } else {
        // tile t - 1 ends at cost fraction (slice + its fraction) / 8
        const uint32_t sl = (t - 1) / tq, u = (t - 1) % tq;
        const double f = ((double)sl + tile_frac(u, tq, kp, tstar, lq)) / 8.0;
        const uint64_t target = (uint64_t)min((double)total, f * (double)total);
        uint32_t lo = 0, hi = nchunk;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (chunk_tot[mid] <= target) lo = mid + 1;
            else hi = mid;
        }
        if (lo >= nchunk) {
            at = h1;
        } else {
            const uint64_t base = lo ? chunk_tot[lo - 1] : 0;
            const uint32_t c0 = lo * kTileChunk, c1 = min(h1 - h0, c0 + kTileChunk);
            uint32_t a = c0, b = c1;
            while (a < b) {
                const uint32_t mid = (a + b) >> 1;
                if (base + pre[mid] <= target) a = mid + 1;
                else b = mid;
            }
            at = h0 + a;
        }
    }
    tiles[t] = at;
}

__global__ void k_zero_u64(unsigned long long *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int B, bool W, bool A, bool LH, bool BATCH = false, bool WIDE = false, bool SEG = false>
void launch3(Ctx &ctx, hipStream_t s, const C3Args &a, uint32_t lds) {
    const void *kern = reinterpret_cast<const void *>(&k_count3<B, W, A, LH, BATCH, WIDE, SEG>);
    if (lds > 65536)
        GS_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count3<B, W, A, LH, BATCH, WIDE, SEG>, B, lds));
    if (per_cu < 1) fail(GS_EUNSUPPORTED, "count kernel does not fit a compute unit");
    uint32_t grid = (uint32_t)ctx.n_cu * (uint32_t)per_cu;
    grid = (grid + kNumQueues - 1) / kNumQueues * kNumQueues;
    if (getenv("GS_PLAN_LOG")) fprintf(stderr, "count3 launch: %d groups per CU, grid %u\n", per_cu, grid);
    k_count3<B, W, A, LH, BATCH, WIDE, SEG><<<dim3(grid), dim3(B), lds, s>>>(a);
    GS_HIP(hipGetLastError());
}

template <int B, bool WIDE, bool SEG = false>
void launch3_bw(Ctx &ctx, hipStream_t s, const C3Args &a, uint32_t lds, bool w, bool an, bool lh) {
    if (lh) {
        if (!w && !an) launch3<B, false, false, true, false, WIDE, SEG>(ctx, s, a, lds);
        else if (w && !an) launch3<B, true, false, true, false, WIDE, SEG>(ctx, s, a, lds);
        else if (!w && an) launch3<B, false, true, true, false, WIDE, SEG>(ctx, s, a, lds);
        else launch3<B, true, true, true, false, WIDE, SEG>(ctx, s, a, lds);
    } else {
        if (!w && !an) launch3<B, false, false, false, false, WIDE, SEG>(ctx, s, a, lds);
        else if (w && !an) launch3<B, true, false, false, false, WIDE, SEG>(ctx, s, a, lds);
        else if (!w && an) launch3<B, false, true, false, false, WIDE, SEG>(ctx, s, a, lds);
        else launch3<B, true, true, false, false, WIDE, SEG>(ctx, s, a, lds);
    }
}

// Entries per step from the mean forward row length (GS_GLOG overrides):
// the largest power of two up to a fifth of a row, so that padding the last
// step of a row costs little and a row still takes several steps.
int group_log(double mean_row) {
    if (const char *eg = getenv("GS_GLOG")) return std::max(0, std::min(6, atoi(eg)));
    int g = 0;
    while (g < 6 && (double)(2u << g) * 5.0 <= mean_row) ++g;
    return g;
}

// Graphs of one shape share a tuned schedule: bin count, weighting, label
// width, and the scale (half powers of two) of the largest and the mean
// forward degree.
uint64_t tune_key(int nb, bool weighted, bool packed, uint32_t maxdeg, double mean_row) {
    const uint64_t lmax = (uint64_t)std::lround(2.0 * std::log2(std::max(1.0, (double)maxdeg)));
    const uint64_t lmean = (uint64_t)std::lround(2.0 * std::log2(std::max(1.0, mean_row)));
    return (uint64_t)nb | (uint64_t)weighted << 8 | (uint64_t)packed << 9 | lmax << 10 | lmean << 20;
}

// The tuned schedule of the nearest shape with the same bin count, weighting
// and label width, if its degree scales are within a factor two of key's.
Tune3 tuned_for(const Ctx &ctx, uint64_t key) {
    Tune3 best;
    long bestd = 5;
    for (const auto &kv : ctx.tuned) {
        if ((kv.first & 0x3FF) != (key & 0x3FF)) continue;
        const long dmax = std::labs((long)((kv.first >> 10) & 0x3FF) - (long)((key >> 10) & 0x3FF));
        const long dmean = std::labs((long)(kv.first >> 20) - (long)(key >> 20));
        if (dmax <= 2 && dmean <= 2 && dmax + dmean < bestd) {
            bestd = dmax + dmean;
            best = kv.second;
        }
    }
    return best;
}

struct Plan3 {
    int block = 256;
    int glog = 0;
    int hload = 5;
    int trunc = 0;
    bool packed = true;
    int mode = kLut;
    int log2h = 6;
    bool lds_hist = true;
    uint32_t tmax = 1024, tcap = 0;
    uint32_t lds = 0;
};

// Configuration index of every ordered bin triple (x, y, z) at
// (x*nb + y)*nb + z: the counter table and the cube fold read it.
std::vector<uint16_t> config_table(int nb) {
    std::vector<uint16_t> t;
    if (nb > kLutMaxBins) return t;
    t.resize((size_t)nb * nb * nb);
    for (int x = 0; x < nb; ++x)
        for (int y = 0; y < nb; ++y)
            for (int z = 0; z < nb; ++z) {
                const int lo = std::min(x, std::min(y, z)), hi = std::max(x, std::max(y, z));
                const int mid = x + y + z - lo - hi;
                t[((size_t)x * nb + y) * nb + z] = (uint16_t)(rank_a(nb, lo) + rank_b(nb, mid) + hi);
            }
    return t;
}

// Guided cost tiles for up to nhubs hubs (see k_tile_bounds): Tq tiles per
// slice for P = teams / 8 teams per slice. GS_TILES=0 turns them off (hubs
// then go out in runs of guided length by count).
struct TilePlan {
    uint32_t nchunk = 1, tq = 1, kp = 1, tstar = 0;
    double lq = 0;
    uint32_t T() const { return 8 * tq; }
};

bool tiles_enabled() {
    const char *e = getenv("GS_TILES");
    return !e || atoi(e) != 0;
}

TilePlan tile_plan(const Ctx &ctx, uint64_t nhubs) {
    TilePlan t;
    t.nchunk = (uint32_t)std::max<uint64_t>(1, (nhubs + kTileChunk - 1) / kTileChunk);
    // teams per slice (8 per CU over 8 slices), fewer for small graphs so
    // that tiles average at least ~8 hubs (a slice holds about 5.2 k P
    // tiles); k so that the first tiles hold about 32 hubs: the hubs that
    // an XCD's work groups count at once then span few enough labels for
    // their spoke rows to share that XCD's L2
    const uint32_t P = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(ctx.n_cu, nhubs / 1320));
    const uint64_t k = std::max<uint64_t>(4, std::min<uint64_t>(64, nhubs / (8ull * P * 32)));
    t.kp = (uint32_t)(k * P);
    t.lq = std::log1p(-1.0 / (double)t.kp);
    t.tstar = (uint32_t)std::ceil(std::log(64.0) / -t.lq);
    t.tq = t.tstar + t.kp;
    return t;
}

void enqueue_tiles(hipStream_t s, const TilePlan &tp, const uint64_t *rp, const GDesc *gd, int ng, uint32_t h0,
                   uint32_t h1, unsigned long long *pre, unsigned long long *chunk_tot, uint32_t *tiles) {
    const uint32_t nchunk = std::max<uint32_t>(1, (h1 - h0 + kTileChunk - 1) / kTileChunk);
    k_hub_cost<<<nchunk, kTileChunk, 0, s>>>(rp, gd, ng, h0, h1, pre, chunk_tot);
    GS_HIP(hipGetLastError());
    k_chunk_scan<<<1, kTileScanBlock, 0, s>>>(chunk_tot, nchunk);
    GS_HIP(hipGetLastError());
    k_tile_bounds<<<(tp.T() + 256) / 256, 256, 0, s>>>(pre, chunk_tot, nchunk, h0, h1, tp.tq, tp.kp, tp.tstar,
                                                        tp.lq, tiles);
    GS_HIP(hipGetLastError());
}

// Rows of 2^30 or more spoke entries take 64-bit addresses (GS_WIDE=1
// forces them, for tests).
bool wide_rows(uint64_t entries) {
    if (const char *ew = getenv("GS_WIDE"))
        if (atoi(ew) != 0) return true;
    return entries >= kNarrowSpan;
}

// Hubs per group and the packed key layout: groups need packed keys with
// room for the hub index (bins below 64) and 32-bit row offsets with two
// spare bits (GS_GROUP caps the group size, for tests).
void set_groups(C3Args &a, const Plan3 &P, int nb, bool wide, const Tune3 &tune) {
    a.yshift = P.packed && nb <= 64 ? 26 : 24;
    a.kmax = P.packed && nb <= 64 && !wide ? kMaxGroup : 1;
    if (tune.group > 0) a.kmax = std::min(a.kmax, tune.group);
    if (const char *eg = getenv("GS_GROUP")) a.kmax = std::max(1, std::min(a.kmax, atoi(eg)));
    a.group_cap = std::min<uint64_t>(a.maxdeg, (uint64_t)P.block);
}

void launch3_any(Ctx &ctx, hipStream_t s, const C3Args &a, const Plan3 &P, bool w, bool an, bool wide,
                 bool seg = false) {
    if (P.block == 768) {
        // weighted, unanchored, LDS counters only (plan3)
        if (!w || an || !P.lds_hist) fail(GS_EUNSUPPORTED, "768-thread plan outside weighted LDS counts");
        if (wide && seg) launch3<768, true, false, true, false, true, true>(ctx, s, a, P.lds);
        else if (wide) launch3<768, true, false, true, false, true>(ctx, s, a, P.lds);
        else launch3<768, true, false, true, false, false>(ctx, s, a, P.lds);
        return;
    }
    if (wide && seg) {
        if (P.block == 512) launch3_bw<512, true, true>(ctx, s, a, P.lds, w, an, P.lds_hist);
        else if (P.block == 128) launch3_bw<128, true, true>(ctx, s, a, P.lds, w, an, P.lds_hist);
        else launch3_bw<256, true, true>(ctx, s, a, P.lds, w, an, P.lds_hist);
    } else if (wide) {
        if (P.block == 512) launch3_bw<512, true>(ctx, s, a, P.lds, w, an, P.lds_hist);
        else if (P.block == 128) launch3_bw<128, true>(ctx, s, a, P.lds, w, an, P.lds_hist);
        else launch3_bw<256, true>(ctx, s, a, P.lds, w, an, P.lds_hist);
    } else {
        if (P.block == 512) launch3_bw<512, false>(ctx, s, a, P.lds, w, an, P.lds_hist);
        else if (P.block == 128) launch3_bw<128, false>(ctx, s, a, P.lds, w, an, P.lds_hist);
        else launch3_bw<256, false>(ctx, s, a, P.lds, w, an, P.lds_hist);
    }
}

// Work-group size and LDS plan: hash table at load factor <= 1/2 where it
// fits (<= 0.7 otherwise), 512 threads per hub for long rows.
// The schedule's LDS layout: among hash loads 1/2 and 0.7, the counter mode
// (or rank arithmetic) and a full or halved step table, the choice that
// fits the most wavefronts per CU, earlier choices first on ties. Tuned
// values and GS_* test overrides pin their parameter.
Plan3 plan3(const Ctx &ctx, uint32_t maxdeg, int nb, bool weighted, bool anchored, uint64_t max_n,
            double mean_row, const Tune3 &tune) {
    Plan3 p;
    p.glog = tune.glog >= 0 ? std::min(6, tune.glog) : group_log(mean_row);
    // GS_PACK=0 / GS_MODE3=rank|lut|cube / GS_TMAX force other paths (tests)
    p.packed = max_n < (1ull << 24) - 1;
    if (const char *ep = getenv("GS_PACK")) p.packed = p.packed && atoi(ep) != 0;
    const int nconf = (int)n_configs(nb);
    if (maxdeg > 16384) fail(GS_EUNSUPPORTED, "forward degree above 16384");
    // 768 threads only for weighted unanchored counts with LDS counters
    // (their LDS allows two groups of 512 per CU where the unweighted plan
    // fits three: two of 768 restore the wavefronts)
    const bool lds_hist_ok = nconf <= 8192;
    const bool w768 = weighted && !anchored && lds_hist_ok;
    bool block_pin = true;
    if (const char *eb = getenv("GS_BLOCK3")) {
        const int b = atoi(eb);
        p.block = b == 768 && w768 ? 768 : b == 512 || b == 768 ? 512 : b == 128 ? 128 : 256;
    } else if (tune.block > 0) {
        p.block = tune.block == 768 && w768 ? 768 : tune.block >= 512 ? 512 : 256;
    } else {
        p.block = maxdeg >= 1024 ? 512 : 256;
        block_pin = false;
    }
    int tmax_pin = tune.tmax > 0 ? tune.tmax : 0;
    if (const char *em = getenv("GS_TMAX")) tmax_pin = atoi(em);
    // the per-spoke binary search pays off on long rows only
    // cutting spoke rows at the hub row's largest label skips probes that
    // cannot match (in cell order a spoke's row runs past the hub's reach);
    // a binary search per spoke, so not for short rows
    if (const char *et = getenv("GS_TRUNC")) p.trunc = atoi(et) != 0;
    else if (tune.trunc >= 0) p.trunc = tune.trunc != 0;
    else p.trunc = maxdeg >= 32;
    // per-work-group LDS counters while they fit (lds_hist_ok); global
    // atomics beyond
    int want = nb <= kLutMaxBins ? kLut : kRank;
    bool mode_pin = false;
    if (tune.mode == kRank) want = kRank, mode_pin = true;
    if (tune.mode == kLut && nb <= kLutMaxBins) want = kLut, mode_pin = true;
    if (tune.mode == kCube && nb <= kCubeMaxBins && !weighted) want = kCube, mode_pin = true;
    if (const char *e = getenv("GS_MODE3")) {
        mode_pin = true;
        if (strcmp(e, "rank") == 0) want = kRank;
        else if (strcmp(e, "lut") == 0 && nb <= kLutMaxBins) want = kLut;
        else if (strcmp(e, "cube") == 0 && nb <= kCubeMaxBins && !weighted) want = kCube;
    }
    const int hload_pin = tune.hload;   // 5: load <= 1/2, 7: load <= 0.7
    int best_waves = -1;
    const int blocks[2] = {p.block, 768};
    const int nblocks = !block_pin && w768 && p.block == 512 ? 2 : 1;
    for (int bi = 0; bi < nblocks; ++bi) {
    const int blk = blocks[bi];
    for (int hl : {5, 7}) {
        if (hload_pin && hl != hload_pin) continue;
        uint32_t H = 64;
        int log2h = 6;
        while (hl == 5 ? H < 2 * maxdeg : (uint64_t)H * 7 < (uint64_t)maxdeg * 10) { H <<= 1; ++log2h; }
        for (int mi = 0; mi < 2; ++mi) {
            int mode0 = mi == 0 ? want : kRank;
            if (mi == 1 && (mode_pin || want == kRank)) continue;
            for (int tf = 0; tf < 2; ++tf) {
                if (tmax_pin && tf) continue;
                const uint32_t tmax = std::max<uint32_t>(
                    64, std::min<uint32_t>(1 << 16, tmax_pin ? (uint32_t)tmax_pin : (tf ? 1u : 2u) * blk));
                const uint32_t tcap = tmax + unroll3(weighted, anchored) * ((uint32_t)blk >> p.glog);
                for (int lh = lds_hist_ok; lh >= 0; --lh) {
                    // the cube lives in LDS; table entries hold 16-bit counter addresses
                    int mode = mode0;
                    if (mode == kCube && !lh) mode = nb <= kLutMaxBins ? kLut : kRank;
                    if (mode == kLut && lh && 4 * (uint64_t)nconf + 2 * (uint64_t)nb * nb * nb >= 65536) mode = kRank;
                    const Layout3 L = layout3(blk, H, maxdeg, tcap, nconf, nb, weighted, anchored, lh, p.packed,
                                              mode);
                    if ((int)L.total > ctx.max_lds) continue;
                    if (blk == 768 && !lh) continue;
                    const int groups = std::max(1, ctx.max_lds / (int)L.total);
                    const int waves = std::min(32, groups * blk / 64);
                    if (waves > best_waves) {
                        best_waves = waves;
                        p.block = blk;
                        p.lds_hist = lh;
                        p.mode = mode;
                        p.lds = L.total;
                        p.log2h = log2h;
                        p.tmax = tmax;
                        p.tcap = tcap;
                        p.hload = hl;
                    }
                    break;   // LDS counters preferred when they fit
                }
            }
        }
    }
    }
    if (best_waves < 0) fail(GS_EUNSUPPORTED, "LDS footprint too large for this degree");
    if (getenv("GS_PLAN_LOG"))
        fprintf(stderr, "count3 plan: maxdeg %u mean_row %.1f block %d glog %d mode %d packed %d H %u "
                        "tmax %u tcap %u lds_hist %d trunc %d lds %u waves/CU %d\n",
                maxdeg, mean_row, p.block, p.glog, p.mode, (int)p.packed, 1u << p.log2h, p.tmax, p.tcap,
                (int)p.lds_hist, p.trunc, p.lds, best_waves);
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
    if (P.lds_hist) launch3<B, false, false, true, true, false>(ctx, s, a, P.lds);
    else launch3<B, false, false, false, true, false>(ctx, s, a, P.lds);
}

}  // namespace

Batch3::~Batch3() {
    if (done) (void)hipEventDestroy(done);
}

namespace {
// Keep a batch buffer when it is large enough (a batch object serves one
// launch after another once the previous one has completed).
void grow(DevBuf &d, size_t n) {
    if (!d.p || d.cap < n) d.alloc(n);
    else d.bytes = n;
}
void grow(HostBuf &h, size_t n) {
    if (!h.p || h.bytes < n) h.alloc(n);
}
}  // namespace

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
    uint64_t sum_e = 0;
    for (int g = 0; g < ng; ++g) {
        sum_e += gs[g]->n_edges;
        if (gs[g]->n_edges >= kNarrowSpan) fail(GS_EUNSUPPORTED, "batched catalogue with 2^30 or more edges");
    }
    const double mean_row = nvirt ? (double)sum_e / (double)nvirt : 0.0;
    const bool packed = max_n < (1ull << 24) - 1;
    const Tune3 tune = tuned_for(ctx, tune_key(nb, false, packed, maxdeg, mean_row));
    const Plan3 P = plan3(ctx, maxdeg, nb, false, false, max_n, mean_row, tune);
    b.ng = ng;
    b.nconf = nconf;
    const size_t per = (size_t)nconf + 1;
    // device staging: counts per catalogue | error word | queues (256-byte
    // aligned) | configuration table
    const size_t qoff = ((size_t)ng * per + 1 + 31) / 32 * 32;
    const std::vector<uint16_t> cfg = config_table(nb);
    const size_t coff = qoff + kQueueWords / 2;
    // | hub tile bounds | block costs
    const bool use_tiles = tiles_enabled();
    const TilePlan tp = tile_plan(ctx, nvirt);
    const size_t toff = coff + (cfg.size() + 3) / 4;
    const size_t poff = toff + (tp.T() + 2) / 2;    // | hub cost prefix | chunk costs
    const size_t koff = poff + nvirt;
    const size_t words = use_tiles ? koff + tp.nchunk : toff;
    grow(b.dv, words * 8);
    unsigned long long *dv = b.dv.as<unsigned long long>();
    grow(b.hostdesc, sizeof(GDesc) * ng);
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
    grow(b.gd, sizeof(GDesc) * ng);
    GS_HIP(hipMemcpyAsync(b.gd.p, hd, sizeof(GDesc) * ng, hipMemcpyHostToDevice, s));
    k_zero_u64<<<64, 256, 0, s>>>(dv, words);
    if (!cfg.empty()) {
        // pinned staging that lives as long as the batch (the copy is async)
        grow(b.hostcfg, cfg.size() * 2);
        memcpy(b.hostcfg.p, cfg.data(), cfg.size() * 2);
        GS_HIP(hipMemcpyAsync(dv + coff, b.hostcfg.p, cfg.size() * 2, hipMemcpyHostToDevice, s));
    }
    C3Args a{};
    a.gd = b.gd.as<GDesc>();
    a.ngraph = ng;
    a.nvirt = (uint32_t)nvirt;
    a.nb = nb;
    a.nconf = nconf;
    a.log2h = P.log2h;
    a.trunc = P.trunc;
    a.packed = P.packed;
    a.mode = P.mode;
    a.glog = P.glog;
    a.maxdeg = maxdeg;
    a.tmax = P.tmax;
    a.tcap = P.tcap;
    a.flush_limit = flush_limit_for(maxdeg, P.block);
    a.queue = (uint32_t *)(dv + qoff);
    a.err = (uint32_t *)(dv + (size_t)ng * per);
    a.cfg3 = (const uint16_t *)(dv + coff);
    set_groups(a, P, nb, false, tune);
    if (nvirt > 0 && use_tiles) {
        enqueue_tiles(s, tp, nullptr, a.gd, ng, 0, (uint32_t)nvirt, dv + poff, dv + koff, (uint32_t *)(dv + toff));
        a.tiles = (uint32_t *)(dv + toff);
        a.ntiles = tp.T();
    }
    if (nvirt > 0) {
        if (P.block == 512) launch3_batch<512>(ctx, s, a, P);
        else if (P.block == 128) launch3_batch<128>(ctx, s, a, P);
        else launch3_batch<256>(ctx, s, a, P);
    }
    grow(b.out, sizeof(unsigned long long) * ((size_t)ng * per + 1));
    GS_HIP(hipMemcpyAsync(b.out.p, dv, sizeof(unsigned long long) * ((size_t)ng * per + 1), hipMemcpyDeviceToHost, s));
    if (!b.done) GS_HIP(hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
    GS_HIP(hipEventRecord(b.done, s));
}

void count3_run(Ctx &ctx, const Graph &g, uint64_t *hist, uint64_t *wsum, uint64_t *ntri,
                const gs_anchor_range *anchors, const Tune3 *force, uint32_t sample_lo, uint32_t sample_hi) {
    const int nb = g.nbins;
    const int nconf = (int)n_configs(nb);
    const bool weighted = wsum != nullptr;
    const bool anchored = anchors != nullptr;
    if (anchored && (anchors->lo > anchors->hi)) fail(GS_EINVAL, "anchor range lo > hi");
    const uint32_t maxdeg = g.max_deg;
    const double mean_row = g.n ? (double)g.n_edges / (double)g.n : 0.0;
    const bool packed = (uint64_t)g.n < (1ull << 24) - 1;
    const Tune3 tune = force ? *force : tuned_for(ctx, tune_key(nb, weighted, packed, maxdeg, mean_row));
    const Plan3 P = plan3(ctx, maxdeg, nb, weighted, anchored, (uint64_t)g.n, mean_row, tune);
    const int W = g.n_windows;
    const int ntiles = W * (W + 1) / 2;
    int kused = 1;          // hubs per group of the launches (reported in the timings)

    // device staging: hist | wsum | ntri | error word | probes | queue sets,
    // one per tile (256-byte aligned)
    const size_t qoff = (3 * (size_t)nconf + 3 + 31) / 32 * 32;
    const std::vector<uint16_t> cfg = config_table(nb);   // | configuration table
    const size_t coff = qoff + (size_t)ntiles * kQueueWords / 2;
    // | hub tile bounds | block costs
    const bool use_tiles = tiles_enabled();
    uint64_t max_hubs = 1;
    for (int w = 0; w < W; ++w) max_hubs = std::max<uint64_t>(max_hubs, W == 1 ? g.n : g.win[w + 1] - g.win[w]);
    const TilePlan tp = tile_plan(ctx, max_hubs);
    const size_t toff = coff + (cfg.size() + 3) / 4;
    const size_t poff = toff + (tp.T() + 2) / 2;    // | hub cost prefix | chunk costs
    const size_t koff = poff + max_hubs;
    const size_t words = use_tiles ? koff + tp.nchunk : toff;
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
    a.mode = P.mode;
    a.glog = P.glog;
    a.maxdeg = maxdeg;
    a.tmax = P.tmax;
    a.tcap = P.tcap;
    a.anchor_lo = anchored ? (uint32_t)std::min<uint64_t>(anchors->lo, 0xFFFFFFFFull) : 0;
    a.anchor_hi = anchored ? (uint32_t)std::min<uint64_t>(anchors->hi, 0xFFFFFFFFull) : 0;
    a.wmul = weighted ? std::ldexp(1.0, weight_scale(g, 3)) : 1.0;
    a.wgen = weighted && (g.wneg || wide_terms(g, 3));
    a.flush_limit = flush_limit_for(maxdeg, P.block);
    a.hist = dv;
    a.wsum = dv + nconf;
    a.ntri = dv + 3 * (size_t)nconf;
    a.err = (uint32_t *)(dv + 3 * (size_t)nconf + 1);
    // spoke-row segments of a WIDE launch: 2^32 entries (GS_WIDE_SPAN shrinks
    // it for tests; a segment always holds at least one whole row)
    a.wspan = kWideSpan;
    if (const char *es = getenv("GS_WIDE_SPAN")) a.wspan = std::max<uint64_t>(strtoull(es, nullptr, 10), 1);
    a.wspan = std::min<uint64_t>(kWideSpan, std::max<uint64_t>(a.wspan, (uint64_t)maxdeg + 1));
    a.probes = dv + 3 * (size_t)nconf + 2;
    a.cfg3 = (const uint16_t *)(dv + coff);
    uint32_t *queues = (uint32_t *)(dv + qoff);
    uint32_t *tbounds = (uint32_t *)(dv + toff);
    unsigned long long *hpre = dv + poff, *ctot = dv + koff;

    hipStream_t s = ctx.stream;
    GS_HIP(hipEventRecord(ctx.ev[0], s));
    k_zero_u64<<<64, 256, 0, s>>>(dv, words);
    if (!cfg.empty())
        GS_HIP(hipMemcpyAsync(dv + coff, cfg.data(), cfg.size() * 2, hipMemcpyHostToDevice, s));
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
        if (sample_hi > sample_lo) {
            a.h0 = std::min<uint32_t>(sample_lo, (uint32_t)g.n);
            a.h1 = std::min<uint32_t>(sample_hi, (uint32_t)g.n);
        }
        a.queue = queues;
        if (use_tiles) {
            const TilePlan t1 = tile_plan(ctx, a.h1 - a.h0);
            enqueue_tiles(s, t1, a.rp, nullptr, 0, a.h0, a.h1, hpre, ctot, tbounds);
            a.tiles = tbounds;
            a.ntiles = t1.T();
        }
        const bool wide = wide_rows(g.n_edges);
        set_groups(a, P, nb, wide, tune);
        kused = a.kmax;
        // spoke rows of one hub can lie 2^32 entries apart only in graphs
        // that large (GS_WIDE_SPAN forces segments, for tests)
        const bool seg = wide && (g.n_edges >= kWideSpan || getenv("GS_WIDE_SPAN") != nullptr);
        launch3_any(ctx, s, a, P, weighted, anchored, wide, seg);
    } else if (g.n > 0) {
        // host-tiled graph: spoke window S resident, hub windows H <= S
        // streamed through; copies of the next tile's windows overlap the
        // current tile's kernel on the copy stream
        uint64_t maxE = 1;
        for (int w = 0; w < W; ++w) maxE = std::max<uint64_t>(maxE, g.win_edge[w + 1] - g.win_edge[w]);
        DevBuf scol[2], sbin[2], hcol[2], hbin[2];
        for (int k = 0; k < 2; ++k) {
            scol[k].alloc((maxE + kRowSlack) * 4);
            sbin[k].alloc(maxE + kRowSlack);
            hcol[k].alloc((maxE + kRowSlack) * 4);
            hbin[k].alloc(maxE + kRowSlack);
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
            b.queue = queues + ti * kQueueWords;
            if (use_tiles) {
                const TilePlan tt = tile_plan(ctx, b.h1 - b.h0);
                enqueue_tiles(s, tt, a.rp, nullptr, 0, b.h0, b.h1, hpre, ctot, tbounds);
                b.tiles = tbounds;
                b.ntiles = tt.T();
            }
            const bool wide = wide_rows(maxE);
            set_groups(b, P, nb, wide, tune);
            kused = b.kmax;
            launch3_any(ctx, s, b, P, weighted, anchored, wide);
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
    std::vector<unsigned long long> h(3 * (size_t)nconf + 3);
    GS_HIP(hipMemcpyAsync(h.data(), dv, h.size() * 8, hipMemcpyDeviceToHost, s));
    GS_HIP(hipEventRecord(ctx.ev[1], s));
    GS_HIP(hipStreamSynchronize(s));
    if (h[3 * (size_t)nconf + 1] & 2) fail(GS_EUNSUPPORTED, "configuration table beyond 16-bit LDS addresses");
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
    ctx.t.probes = h[3 * (size_t)nconf + 2];
    ctx.t.table_log2 = P.log2h;
    ctx.t.block = P.block;
    ctx.t.group = kused;
    ctx.t.hash_load = P.hload;
    // merge-walk bytes: each hub-spoke step reads both forward half-lists,
    // 5 bytes per entry: 2.5 B x sum_i m_i^2 over full degrees m_i
    ctx.t.alg_bytes = g.stats_ready ? (uint64_t)(2.5 * (double)g.sum_sq_deg) : 0;
}

}  // namespace gsn

namespace gsn {

// Coordinate descent over the schedule on a centred run of hubs that takes a
// few milliseconds: each parameter in turn takes the value that times
// fastest (by more than 2%), the others held at their current best.
void tune3(Ctx &ctx, const Graph &g, bool weighted, gs_plan3 *out) {
    if (g.n_windows != 1) fail(GS_EUNSUPPORTED, "schedules are tuned on device-resident graphs");
    if (weighted && !(g.flags & GS_WEIGHTED)) fail(GS_EINVAL, "graph has no weights");
    const int nb = g.nbins;
    const size_t nconf = (size_t)n_configs(nb);
    const uint32_t n = (uint32_t)g.n;
    const double mean_row = g.n ? (double)g.n_edges / (double)g.n : 0.0;
    const bool packed = (uint64_t)g.n < (1ull << 24) - 1;
    const bool wide = wide_rows(g.n_edges);
    std::vector<uint64_t> hist(nconf), ws(weighted ? 2 * nconf : 0);
    uint64_t ntri = 0;
    int trials = 0;
    auto trial = [&](const Tune3 &t, uint32_t lo, uint32_t hi) {
        double best = 1e300;
        for (int r = 0; r < 2; ++r) {
            count3_run(ctx, g, hist.data(), weighted ? ws.data() : nullptr, &ntri, nullptr, &t, lo, hi);
            best = std::min(best, (double)ctx.t.kernel_ms);
            if (best > 100.0) break;   // long samples time steadily: once is enough
        }
        ++trials;
        return best;
    };

    // the built-in schedule, spelled out
    const Plan3 P0 = plan3(ctx, g.max_deg, nb, weighted, false, (uint64_t)g.n, mean_row, Tune3());
    Tune3 cur;
    cur.block = P0.block;
    cur.glog = P0.glog;
    cur.tmax = (int)P0.tmax;
    cur.mode = P0.mode;
    cur.hload = P0.hload;
    cur.trunc = P0.trunc;
    cur.group = packed && nb <= 64 && !wide ? kMaxGroup : 1;

    // the sample: every hub when a full count takes under ~30 ms, else a
    // centred hub run grown (or shrunk) to 10..40 ms but never below 64 hubs
    // per compute unit (short runs mistime the schedules: the launch tail and
    // the sample's own skew weigh too much)
    const uint64_t min_len = std::min<uint64_t>(n, (uint64_t)ctx.n_cu * 64);
    uint64_t len = std::max<uint64_t>(min_len, n / 16);
    uint32_t lo = 0, hi = n;
    double t0 = 0;
    for (int it = 0; it < 8 && n > 0; ++it) {
        lo = (uint32_t)((n - len) / 2);
        hi = (uint32_t)(lo + len);
        t0 = trial(cur, lo, hi);
        if (len >= n) break;
        const double full = t0 * (double)n / (double)len;
        if (full <= 30.0) {
            len = n;
            continue;
        }
        if (t0 >= 10.0 && t0 <= 40.0) break;
        const double f = std::max(0.25, std::min(8.0, 20.0 / std::max(t0, 1e-3)));
        const uint64_t next = std::max<uint64_t>(min_len, std::min<uint64_t>(n, (uint64_t)((double)len * f)));
        if (next == len) break;
        len = next;
    }
    double best = t0;
    auto consider = [&](Tune3 t) {
        const double ms = trial(t, lo, hi);
        if (ms < 0.98 * best) {
            best = ms;
            cur = t;
        }
    };
    if (n > 0) {
        // counter addressing
        for (int m : {kLut, kCube, kRank}) {
            if (m == cur.mode) continue;
            if (m == kLut && nb > kLutMaxBins) continue;
            if (m == kCube && (nb > kCubeMaxBins || weighted)) continue;
            Tune3 t = cur;
            t.mode = m;
            consider(t);
        }
        // candidates per step
        const int g0 = cur.glog;
        for (int d : {-1, 1, -2, 2}) {
            const int gl = g0 + d;
            if (gl < 0 || gl > 6) continue;
            Tune3 t = cur;
            t.glog = gl;
            consider(t);
        }
        // hubs per group
        if (cur.group > 1)
            for (int k : {1, 2}) {
                Tune3 t = cur;
                t.group = k;
                consider(t);
            }
        // hash table load
        {
            Tune3 t = cur;
            t.hload = cur.hload == 5 ? 7 : 5;
            consider(t);
        }
        // spoke-row truncation
        {
            Tune3 t = cur;
            t.trunc = cur.trunc ? 0 : 1;
            consider(t);
        }
        // step table and work-group size
        for (int f : {2, 4}) {
            Tune3 t = cur;
            t.tmax = f == 2 ? cur.tmax / 2 : cur.tmax * 2;
            if (t.tmax >= 128 && t.tmax <= 8192) consider(t);
        }
        Tune3 t = cur;
        t.block = cur.block == 512 ? 256 : 512;
        consider(t);
    }
    const uint64_t key = tune_key(nb, weighted, packed, g.max_deg, mean_row);
    bool found = false;
    for (auto &kv : ctx.tuned)
        if (kv.first == key) {
            kv.second = cur;
            found = true;
        }
    if (!found) ctx.tuned.emplace_back(key, cur);
    if (out) {
        out->block = cur.block;
        out->step_log2 = cur.glog;
        out->group = cur.group;
        out->table = cur.tmax;
        out->counters = cur.mode;
        out->hash_load = cur.hload;
        out->truncate = cur.trunc;
        out->trials = trials;
        out->sample_ms = best;
        out->default_ms = t0;
        out->sample_frac = n ? (double)(hi - lo) / (double)n : 0.0;
    }
}

}  // namespace gsn
