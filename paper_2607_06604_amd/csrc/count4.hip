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
#include <cstdio>
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
    uint32_t anchor_lo, anchor_hi;
    uint64_t flush_limit;
    uint32_t *queue;
    unsigned long long *hist;   // 3*nconf: pos | neg | degenerate
    unsigned long long *ncl;
};

struct Layout4 {
    uint32_t hkey, hloc, hslot, px, py, pz, sx, sy, sz, pq, pb, pperm, R, rowpref, eA, eB, epref, ecw, mstart,
        mpref, mloc, hist, tab, thr, wtot, misc, total;
};

__host__ __device__ inline Layout4 layout4(int block, uint32_t H, uint32_t maxdeg, int W, int nconf,
                                           int nb, bool anchored) {
    Layout4 L{};
    uint32_t o = 0, d = maxdeg + 1;
    L.px = o;      o = lds_align(o + 8 * d, 16);
    L.py = o;      o = lds_align(o + 8 * d, 16);
    L.pz = o;      o = lds_align(o + 8 * d, 16);
    L.sx = o;      o = lds_align(o + 8 * d, 16);
    L.sy = o;      o = lds_align(o + 8 * d, 16);
    L.sz = o;      o = lds_align(o + 8 * d, 16);
    L.pq = o;      o = lds_align(o + 8 * d, 16);
    L.thr = o;     o = lds_align(o + 8 * (nb + 1), 16);
    L.mstart = o;  o = lds_align(o + 8 * block, 16);
    L.hkey = o;    o = lds_align(o + 4 * H, 16);
    L.R = o;       o = lds_align(o + 4 * d * W, 16);
    L.ecw = o;     o = lds_align(o + 4 * block * W, 16);
    L.rowpref = o; o = lds_align(o + 4 * (d + 1), 16);
    L.epref = o;   o = lds_align(o + 4 * (block + 1), 16);
    L.mpref = o;   o = lds_align(o + 4 * (block + 1), 16);
    L.pperm = o;   if (anchored) o = lds_align(o + 4 * d, 16);
    L.hist = o;    o = lds_align(o + 4 * 3 * nconf, 16);
    L.tab = o;     o = lds_align(o + 8 * (nb + 1), 16);
    L.wtot = o;    o = lds_align(o + 4 * (block / 64 + 1), 16);
    L.misc = o;    o = lds_align(o + 16, 16);
    L.hloc = o;    o = lds_align(o + 2 * H, 16);
    L.hslot = o;   o = lds_align(o + 2 * d, 16);
    L.eA = o;      o = lds_align(o + 2 * block, 16);
    L.eB = o;      o = lds_align(o + 2 * block, 16);
    L.mloc = o;    o = lds_align(o + 2 * block, 16);
    L.pb = o;      o = lds_align(o + d, 16);
    L.total = o;
    return L;
}

struct P3 {
    double x, y, z;
};

__device__ __forceinline__ P3 neg(const P3 &v) { return P3{-v.x, -v.y, -v.z}; }

// Separation xb - xa under the minimum image. WRAP false: the caller knows
// no wrap applies (|xb - xa| <= L/2), so the plain difference is the same
// value. Branch-free: subtracting -L is adding L, and subtracting 0 leaves
// the value unchanged, so this is bitwise the definition's result.
template <bool WRAP>
__device__ __forceinline__ double sep(double xa, double xb, double L, double half) {
    const double d = __dsub_rn(xb, xa);
    if (!WRAP) return d;
    const double off = d > half ? L : (d < -half ? -L : 0.0);
    return __dsub_rn(d, off);
}

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

// Per-hub LDS state the clique evaluation reads.
struct Stage4 {
    const double *px, *py, *pz;   // absolute coordinates of N+(i)
    const double *sx, *sy, *sz;   // spokes from the hub (minimum image)
    const double *pq;             // squared spoke lengths
    const uint8_t *pb;            // spoke bins
    const double *thr;            // t_0 .. t_nb
    const int *ta, *tb;           // configuration rank tables
    uint32_t *hist;               // pos | neg | degenerate counters
    int nb, nconf;
    double L, half;
};

// The four hubs of the clique {i, va, vb, vc}: each hub's spokes are the
// separations to the other three (the hub's own spokes negated where the
// clique's edge points towards it).
template <bool WRAP>
__device__ __forceinline__ void eval_clique(const Stage4 &S, uint32_t va, uint32_t vb, uint32_t vc) {
    const P3 A{S.px[va], S.py[va], S.pz[va]};
    const P3 B{S.px[vb], S.py[vb], S.pz[vb]};
    const P3 C{S.px[vc], S.py[vc], S.pz[vc]};
    const P3 ia{S.sx[va], S.sy[va], S.sz[va]};
    const P3 ib{S.sx[vb], S.sy[vb], S.sz[vb]};
    const P3 ic{S.sx[vc], S.sy[vc], S.sz[vc]};
    const double qa = S.pq[va], qb = S.pq[vb], qc = S.pq[vc];
    const int ba = S.pb[va], bb = S.pb[vb], bc = S.pb[vc];
    const P3 ab{sep<WRAP>(A.x, B.x, S.L, S.half), sep<WRAP>(A.y, B.y, S.L, S.half), sep<WRAP>(A.z, B.z, S.L, S.half)};
    const P3 ac{sep<WRAP>(A.x, C.x, S.L, S.half), sep<WRAP>(A.y, C.y, S.L, S.half), sep<WRAP>(A.z, C.z, S.L, S.half)};
    const P3 bcv{sep<WRAP>(B.x, C.x, S.L, S.half), sep<WRAP>(B.y, C.y, S.L, S.half), sep<WRAP>(B.z, C.z, S.L, S.half)};
    const double qab = sq_len(ab.x, ab.y, ab.z), qac = sq_len(ac.x, ac.y, ac.z), qbc = sq_len(bcv.x, bcv.y, bcv.z);
    const int bab = bin_of(S.thr, S.nb, qab), bac = bin_of(S.thr, S.nb, qac), bbc = bin_of(S.thr, S.nb, qbc);
    int idx, ch;
    ch = hub_channel(ia, ib, ic, qa, qb, qc, ba, bb, bc, S.ta, S.tb, &idx);
    atomicAdd(&S.hist[ch * S.nconf + idx], 1u);
    ch = hub_channel(neg(ia), ab, ac, qa, qab, qac, ba, bab, bac, S.ta, S.tb, &idx);
    atomicAdd(&S.hist[ch * S.nconf + idx], 1u);
    ch = hub_channel(neg(ib), neg(ab), bcv, qb, qab, qbc, bb, bab, bbc, S.ta, S.tb, &idx);
    atomicAdd(&S.hist[ch * S.nconf + idx], 1u);
    ch = hub_channel(neg(ic), neg(ac), neg(bcv), qc, qac, qbc, bc, bac, bbc, S.ta, S.tb, &idx);
    atomicAdd(&S.hist[ch * S.nconf + idx], 1u);
}

template <int BLOCK>
__device__ void flush4(const C4Args &a, uint32_t *hist) {
    for (int b = threadIdx.x; b < 3 * a.nconf; b += BLOCK) {
        uint32_t v = hist[b];
        if (v) {
            atomicAdd(&a.hist[b], (unsigned long long)v);
            hist[b] = 0;
        }
    }
}

template <int BLOCK, bool ANCHORED>
__global__ __launch_bounds__(BLOCK) void k_count4(C4Args a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const uint32_t H = 1u << a.log2h, mask = H - 1;
    const int W = a.W;
    const Layout4 L = layout4(BLOCK, H, a.maxdeg, W, a.nconf, a.nb, ANCHORED);
    uint32_t *hkey = (uint32_t *)(sm + L.hkey);
    uint16_t *hloc = (uint16_t *)(sm + L.hloc);
    uint16_t *hslot = (uint16_t *)(sm + L.hslot);
    double *px = (double *)(sm + L.px), *py = (double *)(sm + L.py), *pz = (double *)(sm + L.pz);
    double *sx = (double *)(sm + L.sx), *sy = (double *)(sm + L.sy), *sz = (double *)(sm + L.sz);
    double *pq = (double *)(sm + L.pq);
    uint8_t *pb = (uint8_t *)(sm + L.pb);
    uint32_t *pperm = (uint32_t *)(sm + L.pperm);
    uint32_t *R = (uint32_t *)(sm + L.R);
    uint32_t *rowpref = (uint32_t *)(sm + L.rowpref);
    uint16_t *eA = (uint16_t *)(sm + L.eA), *eB = (uint16_t *)(sm + L.eB);
    uint32_t *epref = (uint32_t *)(sm + L.epref);
    uint32_t *ecw = (uint32_t *)(sm + L.ecw);
    unsigned long long *mstart = (unsigned long long *)(sm + L.mstart);
    uint32_t *mpref = (uint32_t *)(sm + L.mpref);
    uint16_t *mloc = (uint16_t *)(sm + L.mloc);
    uint32_t *hist = (uint32_t *)(sm + L.hist);
    int *ta = (int *)(sm + L.tab);
    int *tb = ta + (a.nb + 1);
    double *thr = (double *)(sm + L.thr);
    uint32_t *wtot = (uint32_t *)(sm + L.wtot);
    uint32_t *s_hub = (uint32_t *)(sm + L.misc);
    unsigned long long *s_cnt = (unsigned long long *)(sm + L.misc + 8);
    const int tid = threadIdx.x;

    for (uint32_t s = tid; s < H; s += BLOCK) hkey[s] = kEmptyKey;
    for (int b = tid; b < 3 * a.nconf; b += BLOCK) hist[b] = 0;
    for (int b = tid; b < a.nb; b += BLOCK) {
        ta[b] = rank_a(a.nb, b);
        tb[b] = rank_b(a.nb, b);
    }
    for (int b = tid; b <= a.nb; b += BLOCK) thr[b] = a.thr[b];
    if (tid == 0) *s_cnt = 0;
    __syncthreads();

    unsigned long long mycl = 0;
    uint64_t acc = 0;
    HubCursor cursor;   // thread 0's claimed run of hubs
    const double Lb = a.L, half = a.half;
    const Stage4 S{px, py, pz, sx, sy, sz, pq, pb, thr, ta, tb, hist, a.nb, a.nconf, a.L, a.half};

    while (true) {
        if (tid == 0) *s_hub = next_hub_in(a.queue, 0, a.n, gridDim.x, cursor, 1);
        __syncthreads();
        const uint32_t i = *s_hub;
        if (i == kEmptyKey) break;
        const uint64_t beg = a.rp[i];
        const uint32_t d = (uint32_t)(a.rp[i + 1] - beg);
        if (d < 3) { __syncthreads(); continue; }
        const double xi = a.X[i], yi = a.Y[i], zi = a.Z[i];
        const uint32_t pi = ANCHORED ? a.perm[i] : 0;
        // every vertex of this hub's cliques lies within rmax of the hub and
        // so, away from the faces, no separation among them wraps
        const bool inner = xi >= a.in_lo && xi <= a.in_hi && yi >= a.in_lo && yi <= a.in_hi &&
                           zi >= a.in_lo && zi <= a.in_hi;

        // 1. stage the hub's forward row
        for (uint32_t e = tid; e < d; e += BLOCK) {
            const uint32_t k = a.col[beg + e];
            uint32_t s = label_hash(k, a.log2h);
            while (atomicCAS(&hkey[s], kEmptyKey, k) != kEmptyKey) s = (s + 1) & mask;
            hloc[s] = (uint16_t)e;
            hslot[e] = (uint16_t)s;
            const double x = a.X[k], y = a.Y[k], z = a.Z[k];
            px[e] = x;
            py[e] = y;
            pz[e] = z;
            const double dx = min_image(xi, x, Lb, half), dy = min_image(yi, y, Lb, half),
                         dz = min_image(zi, z, Lb, half);
            sx[e] = dx;
            sy[e] = dy;
            sz[e] = dz;
            pq[e] = sq_len(dx, dy, dz);
            pb[e] = a.bin[beg + e];
            if (ANCHORED) pperm[e] = a.perm[k];
        }
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

        // 3a. local edges per row, prefix over rows
        uint32_t base = 0;
        for (uint32_t r0 = 0; r0 < d; r0 += BLOCK) {
            const uint32_t r = r0 + tid;
            uint32_t cnt = 0;
            if (r < d)
                for (int w = 0; w < W; ++w) cnt += __popc(R[r * W + w]);
            uint32_t total;
            const uint32_t pre = wg_excl_scan<BLOCK>(cnt, wtot, total);
            if (r < d) rowpref[r] = base + pre;
            base += total;
        }
        if (tid == 0) rowpref[d] = base;
        __syncthreads();
        const uint32_t nloc = base;

        // 3b. chunks of BLOCK local edges; all their cliques as one flat range
        for (uint32_t cb = 0; cb < nloc; cb += BLOCK) {
            const uint32_t x = cb + tid;
            uint32_t m = 0;
            if (x < nloc) {
                const uint32_t ra = upper_index(rowpref, d, x);
                int r = (int)(x - rowpref[ra]);
                uint32_t rb = 0;
                for (int w = 0; w < W; ++w) {
                    const uint32_t word = R[ra * W + w];
                    const int pc = __popc(word);
                    if (r < pc) { rb = (uint32_t)(w * 32 + select_bit(word, r)); break; }
                    r -= pc;
                }
                for (int w = 0; w < W; ++w) {
                    const uint32_t cw = R[ra * W + w] & R[rb * W + w];
                    ecw[tid * W + w] = cw;
                    m += __popc(cw);
                }
                eA[tid] = (uint16_t)ra;
                eB[tid] = (uint16_t)rb;
            }
            uint32_t total;
            const uint32_t pre = wg_excl_scan<BLOCK>(m, wtot, total);
            epref[tid] = pre;
            if (tid == 0) epref[BLOCK] = total;
            if (acc + 4ull * total >= a.flush_limit) {
                flush4<BLOCK>(a, hist);
                acc = 0;
            }
            acc += 4ull * total;
            __syncthreads();
            for (uint32_t e0 = 0; e0 < total; e0 += BLOCK) {
                const uint32_t e = e0 + tid;
                if (e >= total) continue;
                const uint32_t k = upper_index(epref, BLOCK, e);
                int r = (int)(e - epref[k]);
                uint32_t vc = 0;
                for (int w = 0; w < W; ++w) {
                    const uint32_t word = ecw[k * W + w];
                    const int pc = __popc(word);
                    if (r < pc) { vc = (uint32_t)(w * 32 + select_bit(word, r)); break; }
                    r -= pc;
                }
                const uint32_t va = eA[k], vb = eB[k];
                if (ANCHORED) {
                    const uint32_t mn = min(min(pi, pperm[va]), min(pperm[vb], pperm[vc]));
                    if (mn < a.anchor_lo || mn >= a.anchor_hi) continue;
                }
                ++mycl;
                if (inner) eval_clique<false>(S, va, vb, vc);
                else eval_clique<true>(S, va, vb, vc);
            }
            __syncthreads();
        }

        for (uint32_t e = tid; e < d; e += BLOCK) hkey[hslot[e]] = kEmptyKey;
        __syncthreads();
    }

    __syncthreads();
    flush4<BLOCK>(a, hist);
    if (mycl) atomicAdd(s_cnt, mycl);
    __syncthreads();
    if (tid == 0 && *s_cnt) atomicAdd(a.ncl, *s_cnt);
}

__global__ void k_zero4(unsigned long long *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int BLOCK, bool A>
void launch4(Ctx &ctx, const C4Args &a, uint32_t lds) {
    const void *kern = reinterpret_cast<const void *>(&k_count4<BLOCK, A>);
    if (lds > 65536)
        GS_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count4<BLOCK, A>, BLOCK, lds));
    if (per_cu < 1) fail(GS_EUNSUPPORTED, "parity kernel does not fit a compute unit");
    uint32_t grid = (uint32_t)ctx.n_cu * (uint32_t)per_cu;
    grid = (grid + kNumQueues - 1) / kNumQueues * kNumQueues;
    k_count4<BLOCK, A><<<dim3(grid), dim3(BLOCK), lds, ctx.stream>>>(a);
    GS_HIP(hipGetLastError());
}

}  // namespace

void count4_run(Ctx &ctx, const Graph &g, uint64_t *even, uint64_t *pos, uint64_t *neg_out,
                uint64_t *ncl, const gs_anchor_range *anchors) {
    const int nb = g.nbins;
    const int nconf = (int)n_configs(nb);
    const bool anchored = anchors != nullptr;
    if (anchored && anchors->lo > anchors->hi) fail(GS_EINVAL, "anchor range lo > hi");
    const uint32_t maxdeg = g.max_deg;
    if (maxdeg > 4096) fail(GS_EUNSUPPORTED, "forward degree above 4096 for parity counts");
    uint32_t H = 64;
    int log2h = 6;
    while (H < 2 * maxdeg) { H <<= 1; ++log2h; }
    const int W = (int)((maxdeg + 31) / 32 > 0 ? (maxdeg + 31) / 32 : 1);
    constexpr int BLOCK = 256;
    Layout4 L = layout4(BLOCK, H, maxdeg, W, nconf, nb, anchored);
    if ((int)L.total > ctx.max_lds)
        fail(GS_EUNSUPPORTED, "parity kernel LDS footprint too large (forward degree " +
                                  std::to_string(maxdeg) + ", " + std::to_string(L.total) + " bytes)");

    const size_t qoff = (3 * (size_t)nconf + 1 + 31) / 32 * 32;   // queues 256-byte aligned
    const size_t words = qoff + kQueueWords / 2;
    unsigned long long *dv = (unsigned long long *)ctx.scratch_get(words * 8 + 256 * 8);
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
    a.L = g.box;
    a.half = 0.5 * g.box;
    // Hubs at least 2 rmax (with margin) from every face: their clique
    // vertices lie within rmax of the hub, hence unwrapped, and any two of
    // them within 2 rmax < L/2 of each other, so no separation among them
    // wraps. The window is empty unless 4 rmax is below L.
    {
        const double m = 2.0 * g.rmax * (1.0 + 1e-9);
        a.in_lo = m;
        a.in_hi = m < 0.5 * g.box ? g.box - m : -1.0;
    }
    a.anchor_lo = anchored ? (uint32_t)std::min<uint64_t>(anchors->lo, 0xFFFFFFFFull) : 0;
    a.anchor_hi = anchored ? (uint32_t)std::min<uint64_t>(anchors->hi, 0xFFFFFFFFull) : 0;
    const char *fl = getenv("GS_FLUSH_LIMIT");
    a.flush_limit = fl ? strtoull(fl, nullptr, 10) : 0xFFFFFFFFull;
    if (a.flush_limit < 4 * (uint64_t)BLOCK * (maxdeg + 1) || a.flush_limit > 0xFFFFFFFFull)
        a.flush_limit = 0xFFFFFFFFull;
    a.hist = dv;
    a.ncl = dv + 3 * (size_t)nconf;
    a.queue = (uint32_t *)(dv + qoff);

    hipStream_t s = ctx.stream;
    GS_HIP(hipEventRecord(ctx.ev[0], s));
    k_zero4<<<64, 256, 0, s>>>(dv, words);
    GS_HIP(hipMemcpyAsync(dthr, g.bins.t, sizeof(double) * 256, hipMemcpyHostToDevice, s));
    GS_HIP(hipEventRecord(ctx.ev[2], s));
    if (g.n > 0) {
        if (anchored) launch4<BLOCK, true>(ctx, a, L.total);
        else launch4<BLOCK, false>(ctx, a, L.total);
    }
    GS_HIP(hipEventRecord(ctx.ev[3], s));
    std::vector<unsigned long long> h(3 * (size_t)nconf + 1);
    GS_HIP(hipMemcpyAsync(h.data(), dv, h.size() * 8, hipMemcpyDeviceToHost, s));
    GS_HIP(hipEventRecord(ctx.ev[1], s));
    GS_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < nconf; ++c) {
        pos[c] = h[c];
        neg_out[c] = h[nconf + c];
        even[c] = h[c] + h[nconf + c] + h[2 * (size_t)nconf + c];
    }
    *ncl = h[3 * (size_t)nconf];
    float ms = 0, kms = 0;
    GS_HIP(hipEventElapsedTime(&ms, ctx.ev[0], ctx.ev[1]));
    GS_HIP(hipEventElapsedTime(&kms, ctx.ev[2], ctx.ev[3]));
    ctx.t.count_ms = ms;
    ctx.t.kernel_ms = kms;
    ctx.t.kernel_launches = g.n > 0 ? 1 : 0;
    ctx.t.alg_bytes = g.stats_ready ? (uint64_t)(2.5 * (double)g.sum_sq_deg) : 0;
}

}  // namespace gsn
