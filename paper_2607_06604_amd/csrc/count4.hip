// count4.hip - parity-decomposed 4-clique counts (paper Sec. 3.1.1 tetrahedra
// through the hub's list, Sec. 3.2 signed volume and degenerate rule,
// Sec. 3.5.2 per-hub local connectivity in work-group scratch).
//
// Every 4-clique {i < j < k < l} (labels) is found once, at its smallest
// label i: the clique's other vertices are a triangle of the local graph on
// N+(i). One work group per hub:
//  1. stages N+(i) (labels in an LDS hash -> local index, coordinates,
//     squared spoke lengths and bins);
//  2. streams the forward rows of its spokes as one flat coalesced sequence
//     and sets bit c of row a of an LDS bitset whenever spoke a's row holds
//     local vertex c (the paper's per-hub connectivity matrix, as bits);
//  3. lists local edges (a, b) in chunks, ANDs rows a and b into the set of
//     third vertices, and walks all (a, b, c) of the chunk as one flat index
//     space so every lane gets one clique.
// Each clique gets its six separations once (float64, minimum image); every
// one of its four vertices acts as hub with its three spokes ordered by
// squared length; the sorted spoke bins pick the configuration and the sign
// of the float64 triple product the channel: positive, negative or
// degenerate (tied lengths or |V| at most 1e-9 of the spoke-length product).
// even = pos + neg + degenerate is formed on the host.
//
// The same enumeration serves the full 6-edge 4pCF (Sec. 3.3, Sec. 5.3):
// each clique counts once into the configuration of its six edge bins up to
// relabelling of its four vertices (a table from the tuple of bins to the
// configuration's rank), and both counts optionally sum each clique's exact
// weight product (signed weights of Sec. 2.1) per counter.
#include <array>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <cstdlib>

#include "kern_util.h"

namespace gsn {
namespace {

struct C4Args {
    const uint64_t *rp;
    const uint32_t *col;
    const uint8_t *bin;
    const double *X, *Y, *Z;
    const uint32_t *perm;
    const double *thr;   // t_0 .. t_nb
    uint32_t n;
    int nb, nconf, log2h, W;
    uint32_t maxdeg;
    double L, half;
    double in_lo, in_hi;   // hubs with every coordinate in [in_lo, in_hi] see no wrapped pair
    double eb_in, eb_wrap; // margins on the shared triple product (interior hubs, the others)
    float bg_inv, bg_c;    // bin estimate of a squared separation q: sqrt(q) bg_inv - bg_c
    double t3[3];          // t_1, t_2, t_3 (t_nb past nb)
    int bguess;            // that estimate is within one bin (else a search of the thresholds)
    uint32_t anchor_lo, anchor_hi;
    uint64_t flush_limit;
    uint32_t *queue;
    unsigned long long *hist;   // parity: 3*nconf (pos | neg | degenerate); 6-edge: n6
    unsigned long long *ncl;
    const double *w;            // label-ordered weights (weighted counts)
    double wmul;                // 2^s, s the exact-sum scale of 4-weight products
    unsigned long long *wsum;   // weighted: 2 words per counter (two's complement 128-bit)
    const uint32_t *cfg6;       // 6-edge: configuration of every edge-bin tuple code
    int n6;                     // 6-edge configurations
    int lds_cnt;                // counters held in LDS (0: 6-edge counts go to global memory)
    const double *pixdir;       // pixel kind: the 256 pixel centre directions (x, y, z each)
    uint32_t h0, h1;            // hubs of this launch (a host-tiled graph: one window)
};


struct Layout4 {
    uint32_t hkey, hloc, hslot, pv, pb, pperm, R, rbnd, queue, mstart, mpref, mloc, hist, tab, lut, thr, wtot,
        misc, wlo, whi, tab6, tabp, total;
};

// A staged vertex of N+(i) in LDS, one record per local index: doubles
// x, y, z, q, sx, sy, sz, w (the parity kinds: position, squared spoke
// length, spoke from the hub, weight; then padding) or x, y, z, w (the
// 6-edge kind; then padding), so a vertex's fields share one address and
// load in pairs (w only in weighted counts).
template <int KIND, bool WEIGHTED> struct VRec {
    // 16-byte aligned records load as 128-bit pairs. The parity kind takes
    // 80 bytes (two slots of padding; the weight slot unused when
    // unweighted): the stride puts 8 consecutive records on 8 distinct
    // 4-bank groups (5 v mod 8); measured 224.5 ms against 232.9 (64 bytes)
    // and 239.8 (72) on the 2e5-point parity count. The 6-edge kind takes
    // 48 (3 v mod 8; 159.5 ms against 166.3 for 24), the pixel kind 64
    // (its LDS holds the pixel directions too: 80 bytes cost it a work
    // group per CU).
    static constexpr int ST = KIND == kSix4 ? 6 : (KIND == kPixel4 ? 8 : 10);   // doubles per record
    static constexpr int W = KIND == kSix4 ? 3 : 7;                               // the weight's slot
};
constexpr int kVx = 0, kVq = 3, kVs = 4;   // slots: position, squared length, spoke

constexpr int kLut4MaxBins = 16;   // u16 counter offsets of the ordered bin triples, up to 8 KB

// Bits per bin in the ordered-triple table's index (x << 2s | y << s | z).
__host__ __device__ inline int lut_shift(int nb) {
    int s = 0;
    while ((1 << s) < nb) ++s;
    return s;
}

constexpr int kQueue4 = 128;   // clique ring entries per wavefront

// 6-edge tuple tables of at most this many codes live in LDS (u16 ranks).
constexpr int kTab6Lds = 4096;
// 6-edge counters in LDS up to this many configurations.
constexpr int kCnt6Lds = 6144;

// kind: kParity4, kSix4 or kPixel4; ncnt: counters held in LDS; tab6: codes
// of the 6-edge table staged in LDS (0: none).
__host__ __device__ inline Layout4 layout4(int block, uint32_t H, uint32_t maxdeg, int W, int ncnt,
                                           int nb, bool anchored, int kind, bool weighted, int tab6) {
    Layout4 L{};
    uint32_t o = 0, d = maxdeg + 1;
    const bool spokes = kind != kSix4;   // hub spokes and lengths: the parity kinds
    L.pv = o;      o = lds_align(o + 8 * (kind == kSix4 ? 6 : (kind == kPixel4 ? 8 : 10)) * d, 16);
    L.wlo = o;     if (weighted) o = lds_align(o + 8 * ncnt, 16);
    L.whi = o;     if (weighted) o = lds_align(o + 8 * ncnt, 16);
    L.thr = o;     o = lds_align(o + 8 * (nb + 1), 16);
    L.mstart = o;  o = lds_align(o + 8 * block, 16);
    L.rbnd = o;    o = lds_align(o + 8 * (d + 1), 16);
    L.queue = o;   o = lds_align(o + 8 * kQueue4 * (block / 64), 16);
    L.wtot = o;    o = lds_align(o + 8 * (block / 64 + 1), 16);
    L.misc = o;    o = lds_align(o + 32, 16);
    L.hkey = o;    o = lds_align(o + 4 * H, 16);
    L.R = o;       o = lds_align(o + 4 * d * W, 16);
    L.mpref = o;   o = lds_align(o + 4 * (block + 1), 16);
    L.pperm = o;   if (anchored || kind == kPixel4) o = lds_align(o + 4 * d, 16);
    L.tabp = o;    if (kind == kPixel4) o = lds_align(o + 8 * 3 * 256, 16);
    L.hist = o;    o = lds_align(o + 4 * ncnt, 16);
    L.tab = o;     o = lds_align(o + 8 * (nb + 1), 16);
    L.lut = o;     if (spokes && nb <= kLut4MaxBins) o = lds_align(o + (2u << (3 * lut_shift(nb))), 16);
    L.tab6 = o;    o = lds_align(o + 2 * tab6, 16);
    L.hloc = o;    o = lds_align(o + 2 * H, 16);
    L.hslot = o;   o = lds_align(o + 2 * d, 16);
    L.mloc = o;    o = lds_align(o + 2 * block, 16);
    L.pb = o;      o = lds_align(o + d, 16);
    L.total = o;
    return L;
}

struct P3 {
    double x, y, z;
};

__device__ __forceinline__ P3 neg(const P3 &v) { return P3{-v.x, -v.y, -v.z}; }

// (u x v) . w, the cross product then the dot product in the definition's
// operation order.
__device__ __forceinline__ double triple(const P3 &u, const P3 &v, const P3 &w) {
    const double cx = __dsub_rn(__dmul_rn(u.y, v.z), __dmul_rn(u.z, v.y));
    const double cy = __dsub_rn(__dmul_rn(u.z, v.x), __dmul_rn(u.x, v.z));
    const double cz = __dsub_rn(__dmul_rn(u.x, v.y), __dmul_rn(u.y, v.x));
    return __dadd_rn(__dadd_rn(__dmul_rn(cx, w.x), __dmul_rn(cy, w.y)), __dmul_rn(cz, w.z));
}

// Channel (0 pos, 1 neg, 2 degenerate) and configuration of one hub with
// spokes P, Q, R (squared lengths qP, qQ, qR, bins bP, bQ, bR).
// The definition sorts the spokes by length, s0 <= s1 <= s2, and takes the
// sign of (s0 x s1) . s2. Without moving vectors: the bins are monotone in
// the length, so the sorted bins are the min, median and max of the three;
// the sorted lengths likewise. With w the longest spoke and (u, v) the other
// two in cyclic order, (s0 x s1) . s2 is (u x v) . w when u is the shorter of
// the two and its exact negation otherwise (swapping the factors of each
// product leaves it unchanged, and a rounded difference changes only its
// sign when its operands swap), so the three candidates (one per choice of
// w) are formed and one is selected. Ties in length are degenerate whatever
// the order taken among the tied spokes.
__device__ __forceinline__ int hub_channel(const P3 &P, const P3 &Q, const P3 &R, double qP, double qQ,
                                           double qR, int bP, int bQ, int bR, const int *ta, const int *tb,
                                           int *idx) {
    const int b0 = min(min(bP, bQ), bR), b2 = max(max(bP, bQ), bR);
    const int b1 = bP + bQ + bR - b0 - b2;
    *idx = ta[b0] + tb[b1] + b2;
    const bool pq = qP < qQ;
    const double lo = pq ? qP : qQ, hi = pq ? qQ : qP;
    const double q0 = lo < qR ? lo : qR, q2 = hi > qR ? hi : qR;
    const double mh = hi < qR ? hi : qR;
    const double q1 = lo > mh ? lo : mh;
    const bool selP = qP > qQ && qP > qR;
    const bool selQ = !selP && qQ > qR;
    const double vR = triple(P, Q, R), vP = triple(Q, R, P), vQ = triple(R, P, Q);
    const double V = selP ? vP : (selQ ? vQ : vR);
    const bool up = selP ? (qQ <= qR) : (selQ ? (qR <= qP) : (qP <= qQ));
    const double lim = __dmul_rn(1e-18, __dmul_rn(__dmul_rn(q0, q1), q2));
    const bool degen = (q0 == q1) | (q1 == q2) | (__dmul_rn(V, V) <= lim);
    return degen ? 2 : ((V > 0.0) == up ? 0 : 1);
}

// The part of the shared decision common to a clique's four hubs: Vc, the
// triple product (ia x ib) . ic of hub i's spokes in label order, and the
// squares of |Vc| -+ eb.
struct Shared4 {
    double Vc, x2, y2;
    bool xpos;
};

// One hub of a clique decided from Vc where that is safe. In exact
// arithmetic every hub's sorted triple product is +-T (T the signed volume
// times 6): with 4 rmax below the box size all separations are differences
// of the same four points, so (P x Q) . R of the hub's spokes in the order
// given is T for hubs i and b and -T for hubs a and c (sign0), and sorting
// the spokes multiplies it by the parity of the sorting permutation. Every
// spoke component is the exact difference rounded once (error at most u,
// the unit roundoff, times the component; where it wraps, at most u times
// the box size, the correction by L being exact), and evaluating a triple
// product rounds each of its few terms once: the definition's value for
// this hub and Vc both lie within a small multiple of u rmax^3 (plus
// u L rmax^2 near the faces) of +-T. eb is at least twice the sum of the two
// bounds, so when |Vc| - eb already squares above the hub's limit the
// definition's value does too and carries the predicted sign, and when
// |Vc| + eb squares below it the hub is degenerate. Otherwise (a clique
// within rounding of coplanar, or of the threshold, or eb infinite) *exact
// is set and the caller evaluates the hub as the definition says. Ties in
// length are decided exactly, and without a sort: the sorted lengths tie
// iff two of the three are equal, and the sorting permutation's parity is
// the parity of the inversions among (qP, qQ, qR). Returns 0 pos, 1 neg,
// 2 degenerate.
__device__ __forceinline__ int hub_fast(double qP, double qQ, double qR, const Shared4 &sh, bool sign0,
                                        bool &exact) {
    const bool tie = (qP == qQ) | (qP == qR) | (qQ == qR);
    const double lo = fmin(qP, qQ), hi = fmax(qP, qQ);
    const double q0 = fmin(lo, qR), q2 = fmax(hi, qR), q1 = fmax(lo, fmin(hi, qR));
    const double lim = __dmul_rn(1e-18, __dmul_rn(__dmul_rn(q0, q1), q2));
    const bool odd = (qP > qQ) ^ (qP > qR) ^ (qQ > qR);
    const bool sgn = !tie && sh.xpos && sh.x2 > lim;
    const bool deg = tie || (!sgn && sh.y2 <= lim);
    exact = !sgn && !deg;
    const bool pos = (sh.Vc > 0.0) ^ odd ^ !sign0;
    return deg ? 2 : (pos ? 0 : 1);
}

// A hub whose volume test is known to pass: degenerate only on an exact
// length tie, else the channel of the predicted sign (as hub_fast); returned
// as the channel's counter block offset (0, blk or 2 blk bytes).
__device__ __forceinline__ uint32_t hub_sign(double qP, double qQ, double qR, double Vc, bool sign0, uint32_t blk) {
    const bool tie = (qP == qQ) | (qP == qR) | (qQ == qR);
    const bool odd = (qP > qQ) ^ (qP > qR) ^ (qQ > qR);
    const bool pos = (Vc > 0.0) ^ odd ^ !sign0;
    return tie ? 2 * blk : (pos ? 0u : blk);
}

// Per-hub LDS state the clique evaluation reads.
struct Stage4 {
    const double *pv;             // vertex records of N+(i) (VRec)
    const uint8_t *pb;            // spoke bins
    const double *thr;            // t_0 .. t_nb
    const int *ta, *tb;           // configuration rank tables
    const uint16_t *lut;          // nb <= 16: counter byte offset of ordered bin triple x << 2s | y << s | z
    uint32_t *hist;               // pos | neg | degenerate counters (parity), 6-edge counters
    int nb, nconf;
    double L, half;
    float bg_inv, bg_c, bg_top;   // bin estimate (bin_guess); bg_top = nb - 1
    double t3[3];                 // t_1, t_2, t_3 (t_nb past nb): direct counts up to 4 bins
    int bguess;
    int lsh;                      // s of the ordered-triple table
    double limR;                  // fl(1e-18 ((t_nb t_nb) t_nb)): no hub's volume limit exceeds it
    double wmul;
    unsigned long long *wlo, *whi;  // LDS sums of the terms' low 32 bits / high parts
    unsigned long long *ghist, *gwsum;  // global counters and sums (6-edge beyond LDS)
    const uint32_t *cfg6;         // 6-edge configuration of a tuple code (global)
    const uint16_t *tab6;         // the same table in LDS (small bin counts)
    const double *pdir;           // pixel kind: centre directions in LDS (768 doubles)
    const uint32_t *pperm;        // original indices of N+(i)
};

template <int ST> __device__ __forceinline__ P3 vpos(const Stage4 &S, uint32_t v) {
    const double *r = S.pv + ST * v;
    return P3{r[kVx], r[kVx + 1], r[kVx + 2]};
}
template <int ST> __device__ __forceinline__ P3 vspoke(const Stage4 &S, uint32_t v) {
    const double *r = S.pv + ST * v;
    return P3{r[kVs], r[kVs + 1], r[kVs + 2]};
}
template <int ST> __device__ __forceinline__ double vq(const Stage4 &S, uint32_t v) { return S.pv[ST * v + kVq]; }
template <int ST> __device__ __forceinline__ double vw(const Stage4 &S, uint32_t v) {
    return S.pv[ST * v + (ST >= 8 ? 7 : 3)];   // VRec::W
}

// Bin of the squared separation q of a graph edge (t_0 <= q < t_nb): the
// number of thresholds t_1..t_{nb-1} at most q. With linear bins in r
// (e_k = rmin + k D) the float32 estimate u = sqrt(q)/D - rmin/D lies within
// (rmax/D) 1.5 2^-22 + 2^-16 of the exact (r - rmin)/D: float32 rounding of
// q (2^-25 on the root), the square root (one ulp, 2^-23), 1/D and rmin/D
// (2^-24 each) and the fused step (2^-24 of |u| <= 256). Where
// nb rmax / (rmax - rmin) <= 2^20 (bguess) that is below 0.4 bin, so floor(u)
// clamped to [0, nb) is within one bin of the answer and a single float64
// comparison with each neighbouring threshold settles it (t_0 <= q and
// q < t_nb make the ends safe). Otherwise a binary search of the thresholds
// (edge_bins).
__device__ __forceinline__ int bin_guess(const Stage4 &S, double q) {
    const float r = __builtin_amdgcn_sqrtf((float)q);
    const float u = __builtin_amdgcn_fmed3f(__builtin_fmaf(r, S.bg_inv, -S.bg_c), 0.0f, S.bg_top);
    const int g = (int)u;
    return g + (int)(q >= S.thr[g + 1]) - (int)(q < S.thr[g]);
}

// The bins of three squared separations (one branch on bguess for all).
// SMALL (the 6-edge kind): up to 4 bins the three thresholds t_1..t_3 (t_nb
// past nb) are compared directly, cheaper than the estimate.
template <bool SMALL = false>
__device__ __forceinline__ void edge_bins(const Stage4 &S, double q0, double q1, double q2, int &b0, int &b1,
                                          int &b2) {
    if (SMALL && S.nb <= 4) {
        b0 = (int)(q0 >= S.t3[0]) + (int)(q0 >= S.t3[1]) + (int)(q0 >= S.t3[2]);
        b1 = (int)(q1 >= S.t3[0]) + (int)(q1 >= S.t3[1]) + (int)(q1 >= S.t3[2]);
        b2 = (int)(q2 >= S.t3[0]) + (int)(q2 >= S.t3[1]) + (int)(q2 >= S.t3[2]);
    } else if (S.bguess) {
        b0 = bin_guess(S, q0);
        b1 = bin_guess(S, q1);
        b2 = bin_guess(S, q2);
    } else {
        b0 = bin_of(S.thr, S.nb, q0);
        b1 = bin_of(S.thr, S.nb, q1);
        b2 = bin_of(S.thr, S.nb, q2);
    }
}

// A clique's weight term in units of 2^-s: the four magnitudes in ascending
// order multiplied left to right, times 2^s (an integer); neg: the product
// of the four signs is negative.
__device__ __forceinline__ double clique_term(double w0, double w1, double w2, double w3, double wmul, bool &neg) {
    neg = (w0 < 0.0) ^ (w1 < 0.0) ^ (w2 < 0.0) ^ (w3 < 0.0);
    double a = fabs(w0), b = fabs(w1), c = fabs(w2), d = fabs(w3), t;
    if (a > b) { t = a; a = b; b = t; }
    if (c > d) { t = c; c = d; d = t; }
    if (a > c) { t = a; a = c; c = t; }
    if (b > d) { t = b; b = d; d = t; }
    if (b > c) { t = b; b = c; c = t; }
    return __dmul_rn(__dmul_rn(__dmul_rn(__dmul_rn(a, b), c), d), wmul);
}

// A term into sums k: narrow terms into the LDS sums (when LDS holds them),
// wide ones into the global 128-bit sums.
template <bool LDS_CNT>
__device__ __forceinline__ void add_term(const Stage4 &S, uint32_t k, double x, bool neg) {
    if (LDS_CNT && narrow_term(x)) {
        const long long m = (long long)big_term_u64(x);
        lds_term(&S.wlo[k], &S.whi[k], neg ? -m : m);
    } else {
        add128_words(&S.gwsum[2 * k], wide_term(x, neg));
    }
}

// The minimum-image correction of a plain difference d.
__device__ __forceinline__ double wrap1(double d, double L, double half) {
    return d > half ? __dsub_rn(d, L) : (d < -half ? __dadd_rn(d, L) : d);
}

// Separations among the clique's non-hub vertices a, b, c: plain differences,
// corrected by +-L near a face (wrap) as the definition does.
template <int ST>
__device__ __forceinline__ void local_seps(const Stage4 &S, uint32_t va, uint32_t vb, uint32_t vc, bool wrap,
                                          P3 &ab, P3 &ac, P3 &bcv) {
    const P3 A = vpos<ST>(S, va), B = vpos<ST>(S, vb), C = vpos<ST>(S, vc);
    ab = P3{__dsub_rn(B.x, A.x), __dsub_rn(B.y, A.y), __dsub_rn(B.z, A.z)};
    ac = P3{__dsub_rn(C.x, A.x), __dsub_rn(C.y, A.y), __dsub_rn(C.z, A.z)};
    bcv = P3{__dsub_rn(C.x, B.x), __dsub_rn(C.y, B.y), __dsub_rn(C.z, B.z)};
    if (wrap) {
        const double L = S.L, h = S.half;
        ab = P3{wrap1(ab.x, L, h), wrap1(ab.y, L, h), wrap1(ab.z, L, h)};
        ac = P3{wrap1(ac.x, L, h), wrap1(ac.y, L, h), wrap1(ac.z, L, h)};
        bcv = P3{wrap1(bcv.x, L, h), wrap1(bcv.y, L, h), wrap1(bcv.z, L, h)};
    }
}

// Hubs of the clique that the shared product left undecided (bit h of
// mask: 0 hub i, 1 a, 2 b, 3 c), evaluated as the definition says. The
// separations are recomputed from the staged coordinates (the same
// operations, hence the same values) so the common path holds no vectors.
template <int ST>
__device__ __forceinline__ void exact_hubs(const Stage4 &S, uint32_t va, uint32_t vb, uint32_t vc, bool wrap,
                                        uint32_t mask, int *ch) {
    const P3 ia = vspoke<ST>(S, va), ib = vspoke<ST>(S, vb), ic = vspoke<ST>(S, vc);
    const double qa = vq<ST>(S, va), qb = vq<ST>(S, vb), qc = vq<ST>(S, vc);
    P3 ab, ac, bcv;
    local_seps<ST>(S, va, vb, vc, wrap, ab, ac, bcv);
    const double qab = sq_len(ab.x, ab.y, ab.z), qac = sq_len(ac.x, ac.y, ac.z), qbc = sq_len(bcv.x, bcv.y, bcv.z);
    int idx;
    if (mask & 1u) ch[0] = hub_channel(ia, ib, ic, qa, qb, qc, 0, 0, 0, S.ta, S.tb, &idx);
    if (mask & 2u) ch[1] = hub_channel(neg(ia), ab, ac, qa, qab, qac, 0, 0, 0, S.ta, S.tb, &idx);
    if (mask & 4u) ch[2] = hub_channel(neg(ib), neg(ab), bcv, qb, qab, qbc, 0, 0, 0, S.ta, S.tb, &idx);
    if (mask & 8u) ch[3] = hub_channel(neg(ic), neg(ac), neg(bcv), qc, qac, qbc, 0, 0, 0, S.ta, S.tb, &idx);
}

// Counter address (LDS bytes) of the configuration of bins x, y, z in the
// pos block; the neg and degenerate blocks follow at 4 nconf bytes each.
template <bool LUT>
__device__ __forceinline__ uint32_t conf_addr(const Stage4 &S, uint32_t hist_addr, int x, int y, int z) {
    if (LUT)
        return hist_addr +
               (uint32_t)S.lut[((uint32_t)x << (2 * S.lsh)) | ((uint32_t)y << S.lsh) | (uint32_t)z];
    const int b0 = min(min(x, y), z), b2 = max(max(x, y), z);
    const int b1 = x + y + z - b0 - b2;
    return hist_addr + 4u * (uint32_t)(S.ta[b0] + S.tb[b1] + b2);
}

// The four hubs of the clique {i, va, vb, vc}: each hub's spokes are the
// separations to the other three; the squared lengths and bins of the
// three new separations are computed here, the hub's spokes were staged.
// wrap: the hub is near a face, so a separation may need its minimum-image
// correction (elsewhere none can apply and the plain difference is the
// value).
template <bool LUT, bool WEIGHTED>
__device__ __forceinline__ void eval_clique(const Stage4 &S, uint32_t hist_addr, uint32_t va, uint32_t vb,
                                            uint32_t vc, double eb, bool wrap, double wi) {
    constexpr int ST = VRec<kParity4, WEIGHTED>::ST;
    const double qa = vq<ST>(S, va), qb = vq<ST>(S, vb), qc = vq<ST>(S, vc);
    const int ba = S.pb[va], bb = S.pb[vb], bc = S.pb[vc];
    double qab, qac, qbc, Vc;
    {
        P3 ab, ac, bcv;
        local_seps<ST>(S, va, vb, vc, wrap, ab, ac, bcv);
        qab = sq_len(ab.x, ab.y, ab.z);
        qac = sq_len(ac.x, ac.y, ac.z);
        qbc = sq_len(bcv.x, bcv.y, bcv.z);
        Vc = triple(vspoke<ST>(S, va), vspoke<ST>(S, vb), vspoke<ST>(S, vc));
    }
    int bab, bac, bbc;
    edge_bins(S, qab, qac, qbc, bab, bac, bbc);
    Shared4 sh;
    sh.Vc = Vc;
    const double A = fabs(Vc);
    const double x = __dsub_rn(A, eb), y = __dadd_rn(A, eb);
    sh.xpos = x > 0.0;
    sh.x2 = __dmul_rn(x, x);
    sh.y2 = __dmul_rn(y, y);
    // Every hub's limit fl(1e-18 ((q0 q1) q2)) is at most limR, formed the
    // same way from t_nb (rounding is monotone, and all six pairs of a
    // clique are graph edges, so every squared length is below t_nb): when
    // (|Vc| - eb)^2 exceeds it no hub is degenerate by volume and only exact
    // length ties decide (the usual case: a clique far from coplanar);
    // otherwise each hub is decided on its own limit.
    const uint32_t blk = 4u * (uint32_t)S.nconf;
    uint32_t o0, o1, o2, o3;   // counter block offsets of the four hubs' channels
    if (sh.xpos && sh.x2 > S.limR) {
        o0 = hub_sign(qa, qb, qc, Vc, true, blk);
        o1 = hub_sign(qa, qab, qac, Vc, false, blk);
        o2 = hub_sign(qb, qab, qbc, Vc, true, blk);
        o3 = hub_sign(qc, qac, qbc, Vc, false, blk);
    } else {
        int ch[4];
        bool e0, e1, e2, e3;
        ch[0] = hub_fast(qa, qb, qc, sh, true, e0);
        ch[1] = hub_fast(qa, qab, qac, sh, false, e1);
        ch[2] = hub_fast(qb, qab, qbc, sh, true, e2);
        ch[3] = hub_fast(qc, qac, qbc, sh, false, e3);
        const uint32_t mask = (uint32_t)e0 | ((uint32_t)e1 << 1) | ((uint32_t)e2 << 2) | ((uint32_t)e3 << 3);
        if (mask) exact_hubs<ST>(S, va, vb, vc, wrap, mask, ch);
        o0 = blk * (uint32_t)ch[0];
        o1 = blk * (uint32_t)ch[1];
        o2 = blk * (uint32_t)ch[2];
        o3 = blk * (uint32_t)ch[3];
    }
    const uint32_t a0 = conf_addr<LUT>(S, hist_addr, ba, bb, bc) + o0;
    const uint32_t a1 = conf_addr<LUT>(S, hist_addr, ba, bab, bac) + o1;
    const uint32_t a2 = conf_addr<LUT>(S, hist_addr, bb, bab, bbc) + o2;
    const uint32_t a3 = conf_addr<LUT>(S, hist_addr, bc, bac, bbc) + o3;
    __hip_atomic_fetch_add((lds_u32 *)(size_t)a0, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add((lds_u32 *)(size_t)a1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add((lds_u32 *)(size_t)a2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add((lds_u32 *)(size_t)a3, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (WEIGHTED) {
        // every hub contribution carries the clique's weight product
        bool ng;
        const double x = clique_term(wi, vw<ST>(S, va), vw<ST>(S, vb), vw<ST>(S, vc), S.wmul, ng);
        add_term<true>(S, (a0 - hist_addr) >> 2, x, ng);
        add_term<true>(S, (a1 - hist_addr) >> 2, x, ng);
        add_term<true>(S, (a2 - hist_addr) >> 2, x, ng);
        add_term<true>(S, (a3 - hist_addr) >> 2, x, ng);
    }
}

// The bins of the three separations among a clique's non-hub vertices
// (the hub's spoke bins are staged): squared lengths from the staged
// coordinates, counted against the thresholds.
template <int ST>
__device__ __forceinline__ void local_bins(const Stage4 &S, uint32_t va, uint32_t vb, uint32_t vc, bool wrap,
                                           int &bab, int &bac, int &bbc) {
    P3 ab, ac, bcv;
    local_seps<ST>(S, va, vb, vc, wrap, ab, ac, bcv);
    edge_bins<true>(S, sq_len(ab.x, ab.y, ab.z), sq_len(ac.x, ac.y, ac.z), sq_len(bcv.x, bcv.y, bcv.z), bab, bac,
                    bbc);
}

// 6-edge configuration of the clique {i, a, b, c}: the code of its edge-bin
// tuple (ia, ib, ic, ab, ac, bc) looked up in the configuration table (the
// table is invariant under relabelling, so the order taken does not matter).
// LDS_CNT: counters in LDS, else 64-bit global counters.
template <bool TAB6_LDS, bool LDS_CNT, bool WEIGHTED>
__device__ __forceinline__ void eval_six(const Stage4 &S, uint32_t hist_addr, uint32_t va, uint32_t vb,
                                         uint32_t vc, bool wrap, double wi) {
    int bab, bac, bbc;
    constexpr int ST = VRec<kSix4, WEIGHTED>::ST;
    local_bins<ST>(S, va, vb, vc, wrap, bab, bac, bbc);
    const uint32_t nb = (uint32_t)S.nb;
    const uint32_t code =
        ((((((uint32_t)S.pb[va] * nb + S.pb[vb]) * nb + S.pb[vc]) * nb + (uint32_t)bab) * nb + (uint32_t)bac) * nb) +
        (uint32_t)bbc;
    const uint32_t cfg = TAB6_LDS ? (uint32_t)S.tab6[code] : S.cfg6[code];
    if (LDS_CNT)
        __hip_atomic_fetch_add((lds_u32 *)(size_t)(hist_addr + 4 * cfg), 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        atomicAdd(&S.ghist[cfg], 1ull);
    if (WEIGHTED) {
        bool ng;
        const double x = clique_term(wi, vw<ST>(S, va), vw<ST>(S, vb), vw<ST>(S, vc), S.wmul, ng);
        add_term<LDS_CNT>(S, cfg, x, ng);
    }
}

// LDS counters (and weighted sums) into the 64-bit (128-bit) results.
// ---- parity from direction pixels (Sec. 3.2 as the paper computes it) ----
// A separation's pixel: octant (bit 2: x < 0, bit 1: y < 0, bit 0: z < 0)
// times 32 plus the cell i*4 + j, i = min(7, floor(8 |x|/s)) with
// s = (|x|+|y|)+|z|, j = min(3, floor(4 |y|/(|y|+|z|))) (0 when |y|+|z| = 0);
// the zero vector is pixel 0. The reverse separation (exactly the negation)
// has the same cell and the octant of the opposite signs.
__device__ __forceinline__ void pixel_pair(const P3 &r, uint32_t &fwd, uint32_t &rev) {
    const double ax = fabs(r.x), ay = fabs(r.y), az = fabs(r.z);
    const double s = __dadd_rn(__dadd_rn(ax, ay), az);
    if (!(s > 0.0)) {
        fwd = rev = 0;
        return;
    }
    const int i = min(7, (int)floor(__dmul_rn(8.0, __ddiv_rn(ax, s))));
    const double yz = __dadd_rn(ay, az);
    const int j = yz > 0.0 ? min(3, (int)floor(__dmul_rn(4.0, __ddiv_rn(ay, yz)))) : 0;
    const uint32_t cell = (uint32_t)(i * 4 + j);
    fwd = (((r.x < 0.0) ? 4u : 0u) | ((r.y < 0.0) ? 2u : 0u) | ((r.z < 0.0) ? 1u : 0u)) * 32u + cell;
    rev = (((r.x > 0.0) ? 4u : 0u) | ((r.y > 0.0) ? 2u : 0u) | ((r.z > 0.0) ? 1u : 0u)) * 32u + cell;
}

// One hub: its three spokes' pixels (o*: the target's original index), the
// spokes taken in original-index order, V from the pixel centres in the
// definition's operation order; 2 (degenerate) iff |V| < 1e-9, else 0 pos,
// 1 neg.
__device__ __forceinline__ int hub_pixel(const double *pd, uint32_t o0, uint32_t p0, uint32_t o1, uint32_t p1,
                                         uint32_t o2, uint32_t p2) {
    uint32_t t;
    if (o0 > o1) { t = o0; o0 = o1; o1 = t; t = p0; p0 = p1; p1 = t; }
    if (o1 > o2) { t = o1; o1 = o2; o2 = t; t = p1; p1 = p2; p2 = t; }
    if (o0 > o1) { t = o0; o0 = o1; o1 = t; t = p0; p0 = p1; p1 = t; }
    const P3 u{pd[3 * p0], pd[3 * p0 + 1], pd[3 * p0 + 2]};
    const P3 v{pd[3 * p1], pd[3 * p1 + 1], pd[3 * p1 + 2]};
    const P3 w{pd[3 * p2], pd[3 * p2 + 1], pd[3 * p2 + 2]};
    const double V = triple(u, v, w);
    return fabs(V) < 1e-9 ? 2 : (V > 0.0 ? 0 : 1);
}

template <bool LUT>
__device__ __forceinline__ void eval_pixel(const Stage4 &S, uint32_t hist_addr, uint32_t va, uint32_t vb,
                                           uint32_t vc, bool wrap, uint32_t oi) {
    constexpr int ST = VRec<kPixel4, false>::ST;
    const P3 ia = vspoke<ST>(S, va), ib = vspoke<ST>(S, vb), ic = vspoke<ST>(S, vc);
    P3 ab, ac, bcv;
    local_seps<ST>(S, va, vb, vc, wrap, ab, ac, bcv);
    int bab, bac, bbc;
    edge_bins(S, sq_len(ab.x, ab.y, ab.z), sq_len(ac.x, ac.y, ac.z), sq_len(bcv.x, bcv.y, bcv.z), bab, bac, bbc);
    uint32_t fia, ria, fib, rib, fic, ric, fab, rab, fac, rac, fbc, rbc;
    pixel_pair(ia, fia, ria);
    pixel_pair(ib, fib, rib);
    pixel_pair(ic, fic, ric);
    pixel_pair(ab, fab, rab);
    pixel_pair(ac, fac, rac);
    pixel_pair(bcv, fbc, rbc);
    const uint32_t oa = S.pperm[va], ob = S.pperm[vb], oc = S.pperm[vc];
    const int ba = S.pb[va], bb = S.pb[vb], bc = S.pb[vc];
    const int ch0 = hub_pixel(S.pdir, oa, fia, ob, fib, oc, fic);
    const int ch1 = hub_pixel(S.pdir, oi, ria, ob, fab, oc, fac);
    const int ch2 = hub_pixel(S.pdir, oi, rib, oa, rab, oc, fbc);
    const int ch3 = hub_pixel(S.pdir, oi, ric, oa, rac, ob, rbc);
    const uint32_t blk = 4u * (uint32_t)S.nconf;
    const uint32_t a0 = conf_addr<LUT>(S, hist_addr, ba, bb, bc) + blk * (uint32_t)ch0;
    const uint32_t a1 = conf_addr<LUT>(S, hist_addr, ba, bab, bac) + blk * (uint32_t)ch1;
    const uint32_t a2 = conf_addr<LUT>(S, hist_addr, bb, bab, bbc) + blk * (uint32_t)ch2;
    const uint32_t a3 = conf_addr<LUT>(S, hist_addr, bc, bac, bbc) + blk * (uint32_t)ch3;
    __hip_atomic_fetch_add((lds_u32 *)(size_t)a0, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add((lds_u32 *)(size_t)a1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add((lds_u32 *)(size_t)a2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add((lds_u32 *)(size_t)a3, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int BLOCK, bool WEIGHTED>
__device__ void flush4(const C4Args &a, const Stage4 &S, uint32_t *hist) {
    for (int b = threadIdx.x; b < a.lds_cnt; b += BLOCK) {
        uint32_t v = hist[b];
        if (v) {
            atomicAdd(&a.hist[b], (unsigned long long)v);
            hist[b] = 0;
        }
        if (WEIGHTED) {
            const unsigned long long lo = S.wlo[b], hi = S.whi[b];
            if (lo | hi) {
                add128_words(&a.wsum[2 * b], lds_sum128(lo, hi));
                S.wlo[b] = 0;
                S.whi[b] = 0;
            }
        }
    }
}

// KIND kParity4: VAR 1 = configuration of an ordered bin triple from an LDS
// table (nb <= 16), 0 = rank arithmetic. KIND kSix4: VAR 0 = tuple table and
// counters in LDS, 1 = table in global memory and counters in LDS, 2 = both
// in global memory.
template <int BLOCK, int KIND, bool ANCHORED, int VAR, bool WEIGHTED>
__global__ __launch_bounds__(BLOCK) void k_count4(C4Args a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const uint32_t H = 1u << a.log2h, mask = H - 1;
    const int W = a.W;
    constexpr bool LUT = KIND != kSix4 && VAR == 1;
    constexpr bool PERM = ANCHORED || KIND == kPixel4;
    constexpr bool TAB6 = KIND == kSix4 && VAR == 0;
    constexpr bool CNT_LDS = KIND == kParity4 || VAR < 2;
    const Layout4 L = layout4(BLOCK, H, a.maxdeg, W, a.lds_cnt, a.nb, ANCHORED, KIND, WEIGHTED,
                              TAB6 ? a.nb * a.nb * a.nb * a.nb * a.nb * a.nb : 0);
    uint32_t *hkey = (uint32_t *)(sm + L.hkey);
    uint16_t *hloc = (uint16_t *)(sm + L.hloc);
    uint16_t *hslot = (uint16_t *)(sm + L.hslot);
    constexpr int ST = VRec<KIND, WEIGHTED>::ST;
    double *pv = (double *)__builtin_assume_aligned(sm + L.pv, 16);   // lds_align(.., 16)
    uint8_t *pb = (uint8_t *)(sm + L.pb);
    uint32_t *pperm = (uint32_t *)(sm + L.pperm);
    uint32_t *R = (uint32_t *)(sm + L.R);
    unsigned long long *rbnd = (unsigned long long *)(sm + L.rbnd);
    unsigned long long *mstart = (unsigned long long *)(sm + L.mstart);
    uint32_t *mpref = (uint32_t *)(sm + L.mpref);
    uint16_t *mloc = (uint16_t *)(sm + L.mloc);
    uint32_t *hist = (uint32_t *)(sm + L.hist);
    int *ta = (int *)(sm + L.tab);
    uint16_t *lut = (uint16_t *)(sm + L.lut);
    int *tb = ta + (a.nb + 1);
    double *thr = (double *)(sm + L.thr);
    uint32_t *wtot = (uint32_t *)(sm + L.wtot);
    uint64_t *wtot64 = (uint64_t *)(sm + L.wtot);
    uint32_t *s_hub = (uint32_t *)(sm + L.misc);
    uint32_t *s_row = (uint32_t *)(sm + L.misc + 4);
    unsigned long long *s_cnt = (unsigned long long *)(sm + L.misc + 8);
    unsigned long long *s_round = (unsigned long long *)(sm + L.misc + 16);
    const int tid = threadIdx.x, lane = tid & 63;
    unsigned long long *ring = (unsigned long long *)(sm + L.queue) + (tid >> 6) * kQueue4;

    unsigned long long *wlo = (unsigned long long *)(sm + L.wlo), *whi = (unsigned long long *)(sm + L.whi);
    uint16_t *tab6 = (uint16_t *)(sm + L.tab6);
    double *pdir = (double *)(sm + L.tabp);
    if (KIND == kPixel4)
        for (int t = tid; t < 3 * 256; t += BLOCK) pdir[t] = a.pixdir[t];

    for (uint32_t s = tid; s < H; s += BLOCK) hkey[s] = kEmptyKey;
    for (int b = tid; b < a.lds_cnt; b += BLOCK) {
        hist[b] = 0;
        if (WEIGHTED) {
            wlo[b] = 0;
            whi[b] = 0;
        }
    }
    if (TAB6) {
        const int n6c = a.nb * a.nb * a.nb * a.nb * a.nb * a.nb;
        for (int t = tid; t < n6c; t += BLOCK) tab6[t] = (uint16_t)a.cfg6[t];
    }
    for (int b = tid; b < a.nb; b += BLOCK) {
        ta[b] = rank_a(a.nb, b);
        tb[b] = rank_b(a.nb, b);
    }
    const int lsh = lut_shift(a.nb);
    if (LUT)
        for (int t = tid; t < (1 << (3 * lsh)); t += BLOCK) {
            const int m = (1 << lsh) - 1;
            const int x = t >> (2 * lsh), y = (t >> lsh) & m, z = t & m;
            const int b0 = min(min(x, y), z), b2 = max(max(x, y), z), b1 = x + y + z - b0 - b2;
            lut[t] = (x < a.nb && y < a.nb && z < a.nb) ? (uint16_t)(4 * (rank_a(a.nb, b0) + rank_b(a.nb, b1) + b2))
                                                       : (uint16_t)0;
        }
    for (int b = tid; b <= a.nb; b += BLOCK) thr[b] = a.thr[b];
    if (tid == 0) *s_cnt = 0;
    __syncthreads();

    unsigned long long mycl = 0;
    uint64_t acc = 0;
    HubCursor cursor;   // thread 0's claimed run of hubs
    const double Lb = a.L, half = a.half;
    const double tn = a.thr[a.nb];
    const double limR = __dmul_rn(1e-18, __dmul_rn(__dmul_rn(tn, tn), tn));
    const Stage4 S{pv, pb, thr, ta, tb, lut, hist, a.nb, a.nconf, a.L, a.half,
                   a.bg_inv, a.bg_c, (float)(a.nb - 1), {a.t3[0], a.t3[1], a.t3[2]}, a.bguess, lsh, limR,
                   a.wmul, wlo, whi, a.hist, a.wsum, a.cfg6, tab6, pdir, pperm};
    const uint32_t hist_addr = lds_addr(hist);

    while (true) {
        if (tid == 0) *s_hub = next_hub_in(a.queue, a.h0, a.h1, gridDim.x, cursor, 1);
        __syncthreads();
        const uint32_t i = *s_hub;
        if (i == kEmptyKey) break;
        const uint64_t beg = a.rp[i];
        const uint32_t d = (uint32_t)(a.rp[i + 1] - beg);
        if (d < 3) { __syncthreads(); continue; }
        const double xi = a.X[i], yi = a.Y[i], zi = a.Z[i];
        const uint32_t pi = PERM ? a.perm[i] : 0;
        // every vertex of this hub's cliques lies within rmax of the hub and
        // so, away from the faces, no separation among them wraps
        const bool inner = __builtin_amdgcn_readfirstlane((int)(xi >= a.in_lo && xi <= a.in_hi && yi >= a.in_lo &&
                                                                 yi <= a.in_hi && zi >= a.in_lo && zi <= a.in_hi)) != 0;

        // 1. stage the hub's forward row
        for (uint32_t e = tid; e < d; e += BLOCK) {
            const uint32_t k = a.col[beg + e];
            uint32_t s = label_hash(k, a.log2h);
            while (atomicCAS(&hkey[s], kEmptyKey, k) != kEmptyKey) s = (s + 1) & mask;
            hloc[s] = (uint16_t)e;
            hslot[e] = (uint16_t)s;
            const double x = a.X[k], y = a.Y[k], z = a.Z[k];
            double *rec = pv + ST * e;
            rec[kVx] = x;
            rec[kVx + 1] = y;
            rec[kVx + 2] = z;
            if (KIND != kSix4) {
                const double dx = min_image(xi, x, Lb, half), dy = min_image(yi, y, Lb, half),
                             dz = min_image(zi, z, Lb, half);
                rec[kVs] = dx;
                rec[kVs + 1] = dy;
                rec[kVs + 2] = dz;
                rec[kVq] = sq_len(dx, dy, dz);
            }
            pb[e] = a.bin[beg + e];
            if (PERM) pperm[e] = a.perm[k];
            if (WEIGHTED) rec[VRec<KIND, WEIGHTED>::W] = a.w[k];
        }
        const double wi = WEIGHTED ? a.w[i] : 0.0;
        for (uint32_t w = tid; w < d * W; w += BLOCK) R[w] = 0;
        __syncthreads();

        // 2. local adjacency bitset: bit c of row a <=> local c in N+(spoke a)
        for (uint32_t c0 = 0; c0 + 1 < d; c0 += BLOCK) {
            const uint32_t sidx = c0 + tid;
            uint32_t len = 0;
            uint64_t st = 0;
            if (sidx + 1 < d) {
                const uint32_t j = a.col[beg + sidx];
                st = a.rp[j];
                len = (uint32_t)(a.rp[j + 1] - st);
            }
            uint32_t total;
            const uint32_t pre = wg_excl_scan<BLOCK>(len, wtot, total);
            mstart[tid] = st;
            mpref[tid] = pre;
            mloc[tid] = (uint16_t)sidx;
            if (tid == 0) mpref[BLOCK] = total;
            __syncthreads();
            uint32_t sp = 0;
            for (uint32_t e0 = 0; e0 < total; e0 += BLOCK) {
                const uint32_t e = e0 + tid;
                if (e < total) {
                    while (mpref[sp + 1] <= e) ++sp;
                    const uint32_t k = a.col[mstart[sp] + (e - mpref[sp])];
                    uint32_t h = label_hash(k, a.log2h), key;
                    while ((key = hkey[h]) != k && key != kEmptyKey) h = (h + 1) & mask;
                    if (key == k) {
                        const uint32_t c = hloc[h];
                        atomicOr(&R[(uint32_t)mloc[sp] * W + (c >> 5)], 1u << (c & 31));
                    }
                }
            }
            __syncthreads();
        }

        // 3a. a bound on the counter increments of the cliques each row
        //     starts, 4 C(popcount, 2) (one increment per hub), prefix over rows
        {
            uint64_t base = 0;
            for (uint32_t r0 = 0; r0 < d; r0 += BLOCK) {
                const uint32_t r = r0 + tid;
                uint64_t bnd = 0;
                if (r < d) {
                    uint32_t cnt = 0;
                    for (int w = 0; w < W; ++w) cnt += __popc(R[r * W + w]);
                    bnd = cnt ? 2ull * cnt * (cnt - 1) : 0ull;
                }
                uint64_t total;
                const uint64_t pre = wg_excl_scan64<BLOCK>(bnd, wtot64, total);
                if (r < d) rbnd[r] = base + pre;
                base += total;
            }
            if (tid == 0) rbnd[d] = base;
            __syncthreads();
        }

        // 3b. rounds of rows whose bound fits under the counters' flush limit
        //     (normally the whole hub). In a round the wavefronts claim rows
        //     a; for every local edge (a, b) of a row they scan the common
        //     forward neighbours c (bits of row a AND row b) 64 at a time,
        //     one lane per candidate bit, and compact the cliques {i, a, b, c}
        //     into a per-wavefront ring; every 64 queued cliques are
        //     evaluated, one per lane.
        for (uint32_t r0 = 0; r0 < d;) {
            const uint64_t rest = rbnd[d] - rbnd[r0];
            if (acc > 0 && acc + rest >= a.flush_limit) {
                flush4<BLOCK, WEIGHTED>(a, S, hist);
                acc = 0;
                __syncthreads();
            }
            const uint64_t room = a.flush_limit - 1 - acc;
            uint32_t r1 = d;
            if (rest > room) {
                uint32_t lo = r0 + 1, hi = d;  // one row always fits an empty set of counters
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (rbnd[mid] - rbnd[r0] <= room) lo = mid;
                    else hi = mid;
                }
                r1 = lo;
            }
            if (tid == 0) {
                *s_row = r0;
                *s_round = 0;
            }
            __syncthreads();

            uint32_t qhead = 0, qtail = 0;   // ring positions (wavefront-uniform)
            // one clique {i, va, vb, vc} from the ring; the interior and the
            // near-face hubs take separate copies of the parity and 6-edge
            // evaluations (no wrap test per clique)
            auto evaluate = [&](unsigned long long t) {
                const uint32_t va = (uint32_t)t & 0xFFFFu, vb = (uint32_t)(t >> 16) & 0xFFFFu,
                               vc = (uint32_t)(t >> 32);
                if (KIND == kPixel4) {
                    // one copy: a second would raise the register count past
                    // four wavefronts per SIMD
                    eval_pixel<LUT>(S, hist_addr, va, vb, vc, !inner, pi);
                } else if (inner) {
                    if (KIND == kParity4)
                        eval_clique<LUT, WEIGHTED>(S, hist_addr, va, vb, vc, a.eb_in, false, wi);
                    else
                        eval_six<TAB6, CNT_LDS, WEIGHTED>(S, hist_addr, va, vb, vc, false, wi);
                } else {
                    if (KIND == kParity4)
                        eval_clique<LUT, WEIGHTED>(S, hist_addr, va, vb, vc, a.eb_wrap, true, wi);
                    else
                        eval_six<TAB6, CNT_LDS, WEIGHTED>(S, hist_addr, va, vb, vc, true, wi);
                }
            };
            unsigned long long mine_n = 0;   // cliques this lane evaluated in the round
            while (true) {
                uint32_t ra = 0;
                if (lane == 0) ra = atomicAdd(s_row, 1u);
                ra = __builtin_amdgcn_readfirstlane(ra);
                if (ra >= r1) break;
                const uint32_t *Ra = R + ra * W;
                const uint32_t pa = ANCHORED ? min(pi, pperm[ra]) : 0u;
                for (int wa = 0; wa < W; ++wa) {
                    uint32_t bits = __builtin_amdgcn_readfirstlane(Ra[wa]);
                    while (bits) {
                        const uint32_t rb = (uint32_t)(wa * 32 + __builtin_ctz(bits));
                        bits &= bits - 1;
                        const uint32_t *Rb = R + rb * W;
                        const uint32_t pab = ANCHORED ? min(pa, pperm[rb]) : 0u;
                        for (int w = (int)((rb + 1) >> 5); w < W; w += 2) {
                            const uint32_t lo = __builtin_amdgcn_readfirstlane(Ra[w] & Rb[w]);
                            const uint32_t hi =
                                w + 1 < W ? __builtin_amdgcn_readfirstlane(Ra[w + 1] & Rb[w + 1]) : 0u;
                            if ((lo | hi) == 0u) continue;
                            const uint32_t word = lane < 32 ? lo : hi;
                            const uint32_t rc = (uint32_t)(w * 32 + lane);
                            bool take = ((word >> (lane & 31)) & 1u) != 0u;
                            if (ANCHORED && take) {
                                const uint32_t mn = min(pab, pperm[rc]);
                                take = mn >= a.anchor_lo && mn < a.anchor_hi;
                            }
                            const uint64_t bal = __ballot(take);
                            if (take)
                                ring[(qtail + lanes_below(bal)) & (kQueue4 - 1)] =
                                    (unsigned long long)ra | ((unsigned long long)rb << 16) |
                                    ((unsigned long long)rc << 32);
                            qtail += (uint32_t)__popcll(bal);
                            if (qtail - qhead >= 64) {
                                wave_lds_sync();
                                const unsigned long long t = ring[(qhead + lane) & (kQueue4 - 1)];
                                qhead += 64;
                                ++mine_n;
                                evaluate(t);
                                wave_lds_sync();
                            }
                        }
                    }
                }
            }
            wave_lds_sync();
            if ((uint32_t)lane < qtail - qhead) {
                const unsigned long long t = ring[(qhead + lane) & (kQueue4 - 1)];
                ++mine_n;
                evaluate(t);
            }
            mycl += mine_n;
            if (mine_n) atomicAdd(s_round, mine_n);
            __syncthreads();
            acc += 4ull * *s_round;
            r0 = r1;
            __syncthreads();  // s_round is read before it is cleared
        }

        for (uint32_t e = tid; e < d; e += BLOCK) hkey[hslot[e]] = kEmptyKey;
        __syncthreads();
    }

    __syncthreads();
    flush4<BLOCK, WEIGHTED>(a, S, hist);
    if (mycl) atomicAdd(s_cnt, mycl);
    __syncthreads();
    if (tid == 0 && *s_cnt) atomicAdd(a.ncl, *s_cnt);
}

__global__ void k_zero4(unsigned long long *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int BLOCK, int KIND, bool A, int VAR, bool WT>
void launch4(Ctx &ctx, const C4Args &a, uint32_t lds) {
    const void *kern = reinterpret_cast<const void *>(&k_count4<BLOCK, KIND, A, VAR, WT>);
    if (lds > 65536)
        GS_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count4<BLOCK, KIND, A, VAR, WT>, BLOCK, lds));
    if (per_cu < 1) fail(GS_EUNSUPPORTED, "4-clique kernel does not fit a compute unit");
    if (getenv("GS_PLAN_LOG"))
        fprintf(stderr, "[gsn] count4 kind %d var %d block %d lds %u blocks/CU %d maxdeg %u\n", KIND, VAR, BLOCK,
                lds, per_cu, a.maxdeg);
    uint32_t grid = (uint32_t)ctx.n_cu * (uint32_t)per_cu;
    grid = (grid + kNumQueues - 1) / kNumQueues * kNumQueues;
    k_count4<BLOCK, KIND, A, VAR, WT><<<dim3(grid), dim3(BLOCK), lds, ctx.stream>>>(a);
    GS_HIP(hipGetLastError());
}

template <int VAR>
void launch4_pixel(Ctx &ctx, const C4Args &a, uint32_t lds, bool anchored) {
    if (anchored) launch4<512, kPixel4, true, VAR, false>(ctx, a, lds);
    else launch4<512, kPixel4, false, VAR, false>(ctx, a, lds);
}

template <int BLOCK, int KIND, int VAR>
void launch4_v(Ctx &ctx, const C4Args &a, uint32_t lds, bool anchored, bool wt) {
    if (anchored) wt ? launch4<BLOCK, KIND, true, VAR, true>(ctx, a, lds) : launch4<BLOCK, KIND, true, VAR, false>(ctx, a, lds);
    else wt ? launch4<BLOCK, KIND, false, VAR, true>(ctx, a, lds) : launch4<BLOCK, KIND, false, VAR, false>(ctx, a, lds);
}

// The 24 relabellings of a clique's four vertices as permutations of its six
// edges (edge order 01, 02, 03, 12, 13, 23): relabelling by p sends edge
// {x, y} to edge {p(x), p(y)}.
std::vector<std::array<int, 6>> edge_perms() {
    auto eid = [](int x, int y) {
        if (x > y) std::swap(x, y);
        static const int id[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
        return id[x][y];
    };
    static const int ex[6] = {0, 0, 0, 1, 1, 2}, ey[6] = {1, 2, 3, 2, 3, 3};
    std::array<int, 4> p{0, 1, 2, 3};
    std::vector<std::array<int, 6>> out;
    do {
        std::array<int, 6> m;
        for (int e = 0; e < 6; ++e) m[e] = eid(p[ex[e]], p[ey[e]]);
        out.push_back(m);
    } while (std::next_permutation(p.begin(), p.end()));
    return out;
}

}  // namespace

// Scratch of the allocation-free parity count: counters, the clique total,
// the hub queues and the thresholds live in this file-scope array, one copy
// per device, held until the process ends. Host code never passes the
// array's name to a kernel: it uses the device address that
// hipGetSymbolAddress gives for the current device.
constexpr size_t kStaticScratchBytes = 64u << 10;
static __device__ __align__(256) unsigned long long scratch[kStaticScratchBytes / 8];

static std::mutex g_static_mu;
static std::map<int, void *> g_static_ptr;   // device -> address of its copy of scratch

void static_scratch_init(int device) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_ptr.count(device)) return;
    int cur = 0;
    GS_HIP(hipGetDevice(&cur));
    GS_HIP(hipSetDevice(device));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) fail(GS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_static_ptr[device] = ptr;
}

void *static_scratch(int device, size_t *bytes) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    auto it = g_static_ptr.find(device);
    if (it == g_static_ptr.end()) fail(GS_EHIP, "static scratch not set up on this device");
    *bytes = kStaticScratchBytes;
    return it->second;
}

// Configuration rank of every 6-edge tuple code (code = base-nb digits of the
// bins of edges 01, 02, 03, 12, 13, 23, most significant first): the
// configurations are the orbits of tuples under the 24 relabellings, each
// represented by its smallest code, ranked by that code.
const std::vector<uint32_t> &config6_table(int nb, uint32_t *n6) {
    static std::mutex mu;
    static std::map<int, std::pair<std::vector<uint32_t>, uint32_t>> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(nb);
    if (it == cache.end()) {
        const uint32_t n = (uint32_t)nb * nb * nb * nb * nb * nb;
        std::vector<uint32_t> pw(6);
        for (int e = 0; e < 6; ++e) {
            uint32_t v = 1;
            for (int k = e + 1; k < 6; ++k) v *= (uint32_t)nb;
            pw[e] = v;
        }
        const auto perms = edge_perms();
        std::vector<uint32_t> minc(n), rank(n);
        for (uint32_t code = 0; code < n; ++code) {
            int t[6];
            uint32_t v = code;
            for (int e = 5; e >= 0; --e) { t[e] = (int)(v % nb); v /= nb; }
            uint32_t best = code;
            for (const auto &m : perms) {
                // tuple u with u[e] = t[m[e]]
                uint32_t c = 0;
                for (int e = 0; e < 6; ++e) c += (uint32_t)t[m[e]] * pw[e];
                best = std::min(best, c);
            }
            minc[code] = best;
        }
        uint32_t r = 0;
        for (uint32_t code = 0; code < n; ++code)
            if (minc[code] == code) rank[code] = r++;
        for (uint32_t code = 0; code < n; ++code) rank[code] = rank[minc[code]];
        it = cache.emplace(nb, std::make_pair(std::move(rank), r)).first;
    }
    *n6 = it->second.second;
    return it->second.first;
}

// The 256 pixel centre directions (x, y, z each): a pixel (octant o, cell
// i*4 + j) is the direction of (a, (1-a) t, (1-a)(1-t)), a = (i+0.5)/8,
// t = (j+0.5)/4, with the octant's signs (bit 2: x < 0, bit 1: y, bit 0: z),
// divided by its length sqrt((x*x + y*y) + z*z).
static const double *pixel_dirs() {
    static double dirs[3 * 256];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int p = 0; p < 256; ++p) {
            const int o = p >> 5, i = (p >> 2) & 7, j = p & 3;
            volatile double a = ((double)i + 0.5) / 8.0, t = ((double)j + 0.5) / 4.0;
            volatile double na = 1.0 - a, nt = 1.0 - t;
            volatile double x = a, y = na * t, z = na * nt;
            if (o & 4) x = -x;
            if (o & 2) y = -y;
            if (o & 1) z = -z;
            volatile double xx = x * x, yy = y * y, zz = z * z;
            volatile double s2 = xx + yy;
            s2 = s2 + zz;
            const double len = std::sqrt((double)s2);
            dirs[3 * p] = x / len;
            dirs[3 * p + 1] = y / len;
            dirs[3 * p + 2] = z / len;
        }
    });
    return dirs;
}

// The device copy of the table, kept in the context per bin count.
static const uint32_t *config6_device(Ctx &ctx, int nb, uint32_t *n6) {
    const std::vector<uint32_t> &t = config6_table(nb, n6);
    auto it = ctx.cfg6.find(nb);
    if (it == ctx.cfg6.end()) {
        DevBuf b(sizeof(uint32_t) * t.size());
        GS_HIP(hipMemcpy(b.p, t.data(), sizeof(uint32_t) * t.size(), hipMemcpyHostToDevice));
        it = ctx.cfg6.emplace(nb, std::move(b)).first;
    }
    return it->second.as<uint32_t>();
}

void count4_run(Ctx &ctx, const Graph &g, const Count4Out &o, const gs_anchor_range *anchors) {
    const int nb = g.nbins;
    const int nconf = (int)n_configs(nb);
    const bool six = o.kind == kSix4;
    const bool pixel = o.kind == kPixel4;
    const bool weighted = o.wsum[0] != nullptr;
    if (pixel && weighted) fail(GS_EUNSUPPORTED, "pixel parity counts are unweighted");
    const bool anchored = anchors != nullptr;
    if (anchored && anchors->lo > anchors->hi) fail(GS_EINVAL, "anchor range lo > hi");
    if (six && nb > kMaxBins6) fail(GS_EUNSUPPORTED, "6-edge counts take at most 12 bins");
    const uint32_t maxdeg = g.max_deg;
    if (maxdeg > 4096) fail(GS_EUNSUPPORTED, "forward degree above 4096 for 4-clique counts");
    uint32_t H = 64;
    int log2h = 6;
    while (H < 2 * maxdeg) { H <<= 1; ++log2h; }
    const int W = (int)((maxdeg + 31) / 32 > 0 ? (maxdeg + 31) / 32 : 1);

    uint32_t n6 = 0;
    const uint32_t *cfg6 = six ? config6_device(ctx, nb, &n6) : nullptr;
    const int ncnt = six ? (int)n6 : 3 * nconf;   // counters of this count
    const int var = six ? (nb * nb * nb * nb * nb * nb <= kTab6Lds ? 0 : (n6 <= (uint32_t)kCnt6Lds ? 1 : 2))
                        : (nb <= kLut4MaxBins ? 1 : 0);
    const int lds_cnt = (!six || var < 2) ? ncnt : 0;
    const int tab6 = six && var == 0 ? nb * nb * nb * nb * nb * nb : 0;
    // 512 lanes: the footprint above (set by the largest forward degree)
    // usually leaves room for two work groups per compute unit, so the
    // wider group doubles the wavefronts that hide LDS and float64 latency
    int BLOCK = 512;
    if (const char *eb = getenv("GS_BLOCK4")) BLOCK = atoi(eb) == 256 ? 256 : 512;
    if (o.kind != kParity4) BLOCK = 512;   // the other kinds are built for 512 lanes only
    Layout4 L = layout4(BLOCK, H, maxdeg, W, lds_cnt, nb, anchored, o.kind, weighted, tab6);
    if ((int)L.total > ctx.max_lds)
        fail(GS_EUNSUPPORTED, "4-clique kernel LDS footprint too large (forward degree " +
                                  std::to_string(maxdeg) + ", " + std::to_string(L.total) + " bytes)");

    // device words: counters, clique total, (weighted) 2 words per counter,
    // hub queues 256-byte aligned, then the squared thresholds
    const size_t woff = ((size_t)ncnt + 1 + 31) / 32 * 32;
    const size_t qoff = weighted ? (woff + 2 * (size_t)ncnt + 31) / 32 * 32 : woff;
    const size_t words = qoff + kQueueWords / 2;
    const size_t need = words * 8 + 256 * 8 + (pixel ? 3 * 256 * 8 : 0);
    unsigned long long *dv;
    if (o.scratch) {
        if (need > o.scratch_bytes) fail(GS_EUNSUPPORTED, "count needs " + std::to_string(need) +
                                                              " bytes of scratch, more than the static limit");
        dv = (unsigned long long *)o.scratch;
    } else {
        dv = (unsigned long long *)ctx.scratch_get(need);
    }
    double *dthr = (double *)(dv + words);
    C4Args a{};
    a.rp = g.row_ptr.as<uint64_t>();
    a.col = g.col.as<uint32_t>();
    a.bin = g.bin.as<uint8_t>();
    const double *C = g.coords.as<double>();
    a.X = C;
    a.Y = C + g.n;
    a.Z = C + 2 * g.n;
    a.perm = g.perm.as<uint32_t>();
    a.thr = dthr;
    a.n = (uint32_t)g.n;
    a.nb = nb;
    a.nconf = nconf;
    a.log2h = log2h;
    a.W = W;
    a.maxdeg = maxdeg;
    // survey geometry: no wrap anywhere (the minimum image with an infinite
    // box is the plain difference)
    a.L = g.periodic ? g.box : HUGE_VAL;
    a.half = g.periodic ? 0.5 * g.box : HUGE_VAL;
    for (int k = 0; k < 3; ++k) a.t3[k] = g.bins.t[std::min(k + 1, nb)];
    // bin estimates (bin_guess): exact after one correction while
    // nb rmax / (rmax - rmin) <= 2^20
    {
        const double span = g.rmax - g.rmin;
        a.bguess = span > 0.0 && g.rmin >= 0.0 && (double)nb * g.rmax <= 1048576.0 * span &&
                   g.rmax < 1e18 && span >= 1e-12 * nb &&   // float32 range; flushed denormals negligible
                   getenv("GS_BIN_SEARCH") == nullptr;       // tests: the search path
        a.bg_inv = a.bguess ? (float)((double)nb / span) : 0.0f;
        a.bg_c = a.bguess ? (float)(g.rmin * (double)nb / span) : 0.0f;
    }
    // Hubs at least rmax (with margin) from every face: their clique
    // vertices lie within rmax of the hub, hence unwrapped, and any two of
    // them within 2 rmax < L/2 of each other, so no separation among them
    // wraps. The window is empty unless 4 rmax is below L.
    {
        const double m = g.rmax * (1.0 + 1e-9);
        a.in_lo = m;
        a.in_hi = 4.0 * m < g.box ? g.box - m : -1.0;
        // margins: at least twice the summed error bounds of two triple
        // products of spokes no longer than rmax, each under 70 u rmax^3,
        // plus 6 u L rmax^2 where components wrap (u = 2^-53); infinite
        // (every hub evaluated exactly) unless 4 rmax is below the box size
        const bool shared = 4.0 * m < g.box;
        a.eb_in = shared ? 1e-13 * m * m * m : HUGE_VAL;
        a.eb_wrap = shared ? 1e-13 * m * m * m + 1e-14 * g.box * m * m : HUGE_VAL;
        if (!g.periodic) {
            // every separation is a plain difference of the same points:
            // every hub is interior and the shared decision always holds
            a.in_lo = -HUGE_VAL;
            a.in_hi = HUGE_VAL;
            a.eb_in = 1e-13 * m * m * m;
        }
    }
    a.anchor_lo = anchored ? (uint32_t)std::min<uint64_t>(anchors->lo, 0xFFFFFFFFull) : 0;
    a.anchor_hi = anchored ? (uint32_t)std::min<uint64_t>(anchors->hi, 0xFFFFFFFFull) : 0;
    const char *fl = getenv("GS_FLUSH_LIMIT");
    a.flush_limit = fl ? strtoull(fl, nullptr, 10) : 0xFFFFFFFFull;
    // the smallest limit a round can live with: one row's bound, 4 C(d, 2)
    const uint64_t min_limit = std::max<uint64_t>(4 * (uint64_t)BLOCK * (maxdeg + 1),
                                                  2ull * (maxdeg + 1) * (maxdeg + 1) + 4);
    if (a.flush_limit < min_limit || a.flush_limit > 0xFFFFFFFFull) a.flush_limit = 0xFFFFFFFFull;
    a.hist = dv;
    a.ncl = dv + ncnt;
    a.wsum = weighted ? dv + woff : nullptr;
    a.queue = (uint32_t *)(dv + qoff);
    a.w = weighted ? g.weights.as<double>() : nullptr;
    a.wmul = weighted ? std::ldexp(1.0, weight_scale(g, 4)) : 1.0;
    a.cfg6 = cfg6;
    a.n6 = (int)n6;
    a.lds_cnt = lds_cnt;
    a.pixdir = pixel ? dthr + 256 : nullptr;

    hipStream_t s = ctx.stream;
    GS_HIP(hipEventRecord(ctx.ev[0], s));
    k_zero4<<<64, 256, 0, s>>>(dv, words);
    GS_HIP(hipMemcpyAsync(dthr, g.bins.t, sizeof(double) * 256, hipMemcpyHostToDevice, s));
    if (pixel) GS_HIP(hipMemcpyAsync(dthr + 256, pixel_dirs(), sizeof(double) * 768, hipMemcpyHostToDevice, s));
    GS_HIP(hipEventRecord(ctx.ev[2], s));
    a.h0 = 0;
    a.h1 = (uint32_t)g.n;
    auto launch = [&]() {
        const uint32_t lds = L.total;
        if (pixel) {
            if (var == 1) launch4_pixel<1>(ctx, a, lds, anchored);
            else launch4_pixel<0>(ctx, a, lds, anchored);
        } else if (six) {
            if (var == 0) launch4_v<512, kSix4, 0>(ctx, a, lds, anchored, weighted);
            else if (var == 1) launch4_v<512, kSix4, 1>(ctx, a, lds, anchored, weighted);
            else launch4_v<512, kSix4, 2>(ctx, a, lds, anchored, weighted);
        } else if (BLOCK == 512) {
            if (var == 1) launch4_v<512, kParity4, 1>(ctx, a, lds, anchored, weighted);
            else launch4_v<512, kParity4, 0>(ctx, a, lds, anchored, weighted);
        } else {
            if (var == 1) launch4_v<256, kParity4, 1>(ctx, a, lds, anchored, weighted);
            else launch4_v<256, kParity4, 0>(ctx, a, lds, anchored, weighted);
        }
    };
    uint64_t launches = 0;
    if (g.n > 0 && g.n_windows == 1) {
        launch();
        launches = 1;
    } else if (g.n > 0) {
        // Host-tiled graph: for each hub window, the CSR entries from its
        // first row through the row of its hubs' largest spoke (every row a
        // hub or one of its spokes reads) are copied into one device
        // buffer, and the window's hubs are counted from it. Each clique is
        // counted at its smallest label, i.e. in exactly one window.
        const int W = g.n_windows;
        std::vector<uint64_t> rph((size_t)g.n + 1);
        GS_HIP(hipMemcpy(rph.data(), g.row_ptr.p, sizeof(uint64_t) * rph.size(), hipMemcpyDeviceToHost));
        const uint32_t *hc = g.hcol.as<uint32_t>();
        const uint8_t *hb = g.hbin.as<uint8_t>();
        std::vector<uint64_t> e0(W), e1(W);
        uint64_t maxspan = 1;
        for (int w = 0; w < W; ++w) {
            uint64_t jmax = g.win[w];
            for (uint64_t i = g.win[w]; i < g.win[w + 1]; ++i)
                if (rph[i + 1] > rph[i]) jmax = std::max<uint64_t>(jmax, hc[rph[i + 1] - 1]);
            e0[w] = rph[g.win[w]];
            e1[w] = rph[std::max<uint64_t>(jmax, g.win[w + 1] - 1) + 1];
            maxspan = std::max<uint64_t>(maxspan, e1[w] - e0[w]);
        }
        const uint64_t fixed = g.row_ptr.bytes + g.perm.bytes + g.coords.bytes + g.weights.bytes;
        if (fixed + 5 * (maxspan + kRowSlack) > ctx.budget)
            fail(GS_EDEVMEM, "a hub window and the rows its hubs read exceed the device budget");
        DevBuf wc((maxspan + kRowSlack) * 4, ctx.pool), wb(maxspan + kRowSlack, ctx.pool);
        for (int w = 0; w < W; ++w) {
            if (g.win[w + 1] <= g.win[w]) continue;
            const uint64_t ne = e1[w] - e0[w];
            GS_HIP(hipMemcpyAsync(wc.p, hc + e0[w], ne * 4, hipMemcpyHostToDevice, s));
            GS_HIP(hipMemcpyAsync(wb.p, hb + e0[w], ne, hipMemcpyHostToDevice, s));
            // entry e of the graph at buffer position e - e0 (only entries of
            // [e0, e1) are read)
            a.col = wc.as<uint32_t>() - e0[w];
            a.bin = wb.as<uint8_t>() - e0[w];
            a.h0 = (uint32_t)g.win[w];
            a.h1 = (uint32_t)g.win[w + 1];
            k_zero4<<<1, 256, 0, s>>>((unsigned long long *)a.queue, kQueueWords / 2);
            launch();
            ++launches;
        }
        GS_HIP(hipStreamSynchronize(s));
    }
    GS_HIP(hipEventRecord(ctx.ev[3], s));
    // results straight into the caller's arrays, one block of counters each
    const int nblk = six ? 1 : 3;
    const size_t per = six ? (size_t)n6 : (size_t)nconf;
    for (int b = 0; b < nblk; ++b) {
        GS_HIP(hipMemcpyAsync(o.cnt[b], dv + b * per, per * 8, hipMemcpyDeviceToHost, s));
        if (weighted)
            GS_HIP(hipMemcpyAsync(o.wsum[b], dv + woff + 2 * b * per, 2 * per * 8, hipMemcpyDeviceToHost, s));
    }
    GS_HIP(hipMemcpyAsync(o.ncl, dv + ncnt, 8, hipMemcpyDeviceToHost, s));
    GS_HIP(hipEventRecord(ctx.ev[1], s));
    GS_HIP(hipStreamSynchronize(s));
    if (o.wscale) *o.wscale = weighted ? weight_scale(g, 4) : 0;
    float ms = 0, kms = 0;
    GS_HIP(hipEventElapsedTime(&ms, ctx.ev[0], ctx.ev[1]));
    GS_HIP(hipEventElapsedTime(&kms, ctx.ev[2], ctx.ev[3]));
    ctx.t.count_ms = ms;
    ctx.t.kernel_ms = kms;
    ctx.t.kernel_launches = launches;
    ctx.t.alg_bytes = g.stats_ready ? (uint64_t)(2.5 * (double)g.sum_sq_deg) : 0;
}

}  // namespace gsn
