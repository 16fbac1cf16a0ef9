// build.hip - GPU cell-list builder of the r < rmax graph (paper Sec. 2.1,
// CSR layout of Sec. 3.5.1).
//
// Points are relabelled in cell order (cells at least rmax wide, raster order
// x-major, original index order inside a cell). Each label's forward
// neighbours (label j > i) are written in ascending label order: its own cell
// after i, then the 13..26 periodically adjacent cells in ascending cell id,
// which is ascending label order because labels follow cell ids. Each edge
// carries the one-byte bin of its squared separation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "kern_util.h"

namespace gsn {
namespace {

constexpr int kBlock = 256;
constexpr uint32_t kChunk = 64;   // labels per build work group (at most)
constexpr uint32_t kStage = 512;  // candidates whose coordinates a work group stages in LDS

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Cell of each point; flags[0] |= 1 for a coordinate outside [0, L) or NaN.
__global__ void k_cells(const double *__restrict__ xyz, uint32_t n, double L, int nc,
                        uint32_t *__restrict__ cell_of, uint32_t *__restrict__ count,
                        uint32_t *__restrict__ flags) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c3[3];
    bool bad = false;
    for (int a = 0; a < 3; ++a) {
        double x = xyz[3 * (uint64_t)i + a];
        if (!(x >= 0.0 && x < L)) bad = true;
        double u = __ddiv_rn(__dmul_rn(x, (double)nc), L);
        int c = (u >= 0.0 && u < 1e9) ? (int)u : 0;
        c3[a] = c > nc - 1 ? nc - 1 : c;
    }
    if (bad) atomicOr(&flags[0], 1u);
    uint32_t c = ((uint32_t)c3[0] * nc + c3[1]) * nc + c3[2];
    cell_of[i] = c;
    atomicAdd(&count[c], 1u);
}

// Finite nonzero weights of either sign (signed data-minus-random weights,
// Sec. 2.1); the smallest and largest magnitude as ordered bit patterns.
__global__ void k_weights(const double *__restrict__ w, uint32_t n, uint32_t *__restrict__ flags,
                          unsigned long long *__restrict__ mm) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long lo = ~0ull, hi = 0;
    if (i < n) {
        const double v = fabs(w[i]);
        if (!(v > 0.0) || !(v <= 1.79769313486231570e308)) {
            atomicOr(&flags[0], 2u);
        } else {
            lo = hi = (unsigned long long)__double_as_longlong(v);
            if (w[i] < 0.0) atomicOr(&flags[0], 4u);
        }
    }
    // wavefront min / max first: one pair of device atomics per wavefront
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long l2 = __shfl_xor(lo, o, 64), h2 = __shfl_xor(hi, o, 64);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    if ((threadIdx.x & 63) == 0 && hi) {
        atomicMin(&mm[0], lo);
        atomicMax(&mm[1], hi);
    }
}

__global__ void k_scatter(const uint32_t *__restrict__ cell_of, uint32_t n,
                          const uint64_t *__restrict__ cstart, uint32_t *__restrict__ fill,
                          uint32_t *__restrict__ order) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c = cell_of[i];
    uint32_t r = atomicAdd(&fill[c], 1u);
    order[cstart[c] + r] = i;
}

// Stable order inside each cell: rank of a point among its cell by original index.
__global__ void k_rank(const uint32_t *__restrict__ order, const uint32_t *__restrict__ cell_of,
                       const uint64_t *__restrict__ cstart, uint32_t n, uint32_t *__restrict__ perm) {
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t me = order[p];
    uint32_t c = cell_of[me];
    uint64_t s0 = cstart[c], s1 = cstart[c + 1];
    uint32_t r = 0;
    for (uint64_t q = s0; q < s1; ++q) r += order[q] < me;
    perm[s0 + r] = me;
}

__global__ void k_gather(const uint32_t *__restrict__ perm, const double *__restrict__ xyz,
                         const double *__restrict__ w, const uint32_t *__restrict__ cell_of,
                         uint32_t n, double *__restrict__ X, double *__restrict__ Y,
                         double *__restrict__ Z, double *__restrict__ W,
                         uint32_t *__restrict__ cellL) {
    uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    uint32_t i = perm[l];
    X[l] = xyz[3 * (uint64_t)i];
    Y[l] = xyz[3 * (uint64_t)i + 1];
    Z[l] = xyz[3 * (uint64_t)i + 2];
    if (W) W[l] = w[i];
    cellL[l] = cell_of[i];
}

struct EdgeArgs {
    const double *X, *Y, *Z;
    const uint32_t *cellL;
    const uint64_t *cstart;
    const uint64_t *chpref;  // chunks before each cell; [ncell] = all chunks
    const uint32_t *gcell;   // cell of each chunk
    uint32_t ncell, chunk;   // cells; labels per chunk
    const double *thr;     // t_0 .. t_nb
    uint32_t n;
    uint32_t l0, l1;    // labels handled by this launch
    uint64_t obase;     // fill pass: rp[l] - obase indexes col / bin
    int nc, nb;
    int periodic;       // 0: neighbour cells do not wrap and no separation does
    double L, half;
    // count pass
    uint32_t *deg;
    uint32_t *maxdeg;
    // fill pass
    const uint64_t *rp;
    uint32_t *col;
    uint8_t *bin;
    unsigned long long *pair_hist;  // nb
    uint32_t *indeg;                // full-degree bookkeeping
};

// The rows of labels [i0, i1) of one cell (ce: the cell's end): a wavefront
// per label, its lanes over the label's candidates 64 at a time (the own cell
// after the label, then the forward cells' ranges rs / rq). WRAP false: the
// caller knows no candidate separation needs a minimum-image correction.
template <bool FILL, bool WRAP, bool STAGED>
__device__ __forceinline__ uint32_t edge_rows(const EdgeArgs &a, const double *t, const uint64_t *rs,
                                              const uint32_t *rq, int nr, uint32_t Mf, uint64_t i0, uint64_t i1,
                                              uint64_t cs, uint64_t ce, const double *lx, const double *ly,
                                              const double *lz, const uint32_t *lj) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double t0 = t[0], tn = t[a.nb];
    uint32_t mymax = 0;
    for (uint64_t i = i0 + wid; i < i1; i += kBlock / 64) {
        const double xi = a.X[i], yi = a.Y[i], zi = a.Z[i];
        const uint32_t own = (uint32_t)(ce - i - 1);   // own-cell labels above i
        const uint32_t M = own + Mf;
        const uint64_t out = FILL ? a.rp[i] - a.obase : 0;
        const uint32_t cap = FILL ? (uint32_t)(a.rp[i + 1] - a.rp[i]) : 0;  // the count pass's result
        uint32_t cnt = 0;
        for (uint32_t f0 = 0; f0 < M; f0 += 64) {
            const uint32_t f = f0 + lane;
            bool in = false;
            uint64_t j = 0;
            double q = 0.0;
            if (f < M) {
                double xj, yj, zj;
                if (STAGED) {
                    // the candidate's coordinates from the group's LDS copy:
                    // the own cell first, then the forward ranges in order
                    const uint32_t s = f < own ? (uint32_t)(i - cs) + 1 + f : (uint32_t)(ce - cs) + (f - own);
                    xj = lx[s];
                    yj = ly[s];
                    zj = lz[s];
                } else {
                    if (f < own) {
                        j = i + 1 + f;
                    } else {
                        const uint32_t g = f - own;
                        const uint32_t r = upper_index(rq, (uint32_t)nr, g);
                        j = rs[r] + (g - rq[r]);
                    }
                    xj = a.X[j];
                    yj = a.Y[j];
                    zj = a.Z[j];
                }
                double dx, dy, dz;
                if (WRAP) {
                    dx = min_image(xi, xj, a.L, a.half);
                    dy = min_image(yi, yj, a.L, a.half);
                    dz = min_image(zi, zj, a.L, a.half);
                } else {  // no correction can apply: the plain difference is the same double
                    dx = __dsub_rn(xj, xi);
                    dy = __dsub_rn(yj, yi);
                    dz = __dsub_rn(zj, zi);
                }
                q = sq_len(dx, dy, dz);
                in = q >= t0 && q < tn;
            }
            const uint64_t mask = __ballot(in);
            if (FILL && in) {
                const uint32_t k = cnt + lanes_below(mask);
                if (STAGED)  // the label of a hit (only the fill pass needs it)
                    j = f < own ? i + 1 + f : (uint64_t)lj[f - own];
                if (k < cap) {
                    a.col[out + k] = (uint32_t)j;
                    a.bin[out + k] = (uint8_t)bin_of(t, a.nb, q);
                }
            }
            cnt += (uint32_t)__popcll(mask);
        }
        if (!FILL && lane == 0) a.deg[i] = cnt;
        mymax = cnt > mymax ? cnt : mymax;
    }
    return mymax;
}

// Graph edges, one work group per chunk of at most 64 labels of a cell: its
// wavefronts take the chunk's labels in turn, and for a label i the 64 lanes
// sweep its candidates -- the rest of its own cell (labels above i), then
// the forward cells in ascending cell id, hence ascending labels -- one
// candidate per lane, and a ballot compacts each window's edges in label
// order. The candidates' coordinates (and, for the fill pass, labels) are
// staged in LDS when they fit. The count pass writes degrees and the largest
// degree; the fill pass writes col / bin at the offsets the count pass
// produced.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_edges(EdgeArgs a) {
    __shared__ double t[256];
    __shared__ uint64_t rs[27];   // first label of forward cell range r
    __shared__ uint32_t rq[28];   // running length before range r
    __shared__ int s_nr;
    __shared__ int s_wf;
    __shared__ double lx[kStage], ly[kStage], lz[kStage];
    __shared__ uint32_t lj[FILL ? kStage : 1];   // labels of the forward candidates (fill pass)
    // one work group per chunk of at most `chunk` labels of a cell, so that
    // a crowded cell is spread over many groups instead of forming a tail
    const uint32_t b = blockIdx.x;
    if (b >= a.chpref[a.ncell]) return;   // the grid is an upper bound
    const uint32_t c = a.gcell[b];
    const uint64_t cs = a.cstart[c], ce = a.cstart[c + 1];
    const uint64_t p0 = cs + (uint64_t)(b - a.chpref[c]) * a.chunk;
    const uint64_t p1 = p0 + a.chunk < ce ? p0 + a.chunk : ce;
    const uint64_t i0 = p0 > a.l0 ? p0 : (uint64_t)a.l0, i1 = p1 < a.l1 ? p1 : (uint64_t)a.l1;
    if (i0 >= i1) return;   // no point of this launch in the chunk (uniform)
    for (int k = threadIdx.x; k <= a.nb; k += blockDim.x) t[k] = a.thr[k];
    if (threadIdx.x == 0) {
        const int nc = a.nc;
        int ax[3], ay[3], az[3], na = 1;
        const int cx = (int)(c / (uint32_t)(nc * nc)), cy = (int)((c / nc) % nc), cz = (int)(c % nc);
        // a cell off the boundary layer with at least 5 cells per axis: its
        // candidates lie in truly adjacent cells, within 2 L / nc <= 0.4 L of
        // the label, so no minimum-image correction can apply
        s_wf = !a.periodic ||
               (nc >= 5 && cx >= 1 && cx <= nc - 2 && cy >= 1 && cy <= nc - 2 && cz >= 1 && cz <= nc - 2);
        if (!a.periodic) {
            // survey geometry: the in-range neighbours only, ascending
            auto range3 = [nc](int v, int *o, int &k) {
                k = 0;
                for (int w = v - 1; w <= v + 1; ++w)
                    if (w >= 0 && w < nc) o[k++] = w;
            };
            int kx, ky, kz;
            range3(cx, ax, kx);
            range3(cy, ay, ky);
            range3(cz, az, kz);
            int nr = 0;
            uint32_t run = 0;
            for (int u = 0; u < kx; ++u)
                for (int v = 0; v < ky; ++v)
                    for (int w = 0; w < kz; ++w) {
                        const uint32_t id = ((uint32_t)ax[u] * nc + ay[v]) * nc + az[w];
                        if (id <= c) continue;
                        const uint64_t b0 = a.cstart[id], b1 = a.cstart[id + 1];
                        if (b1 == b0) continue;
                        rs[nr] = b0;
                        rq[nr] = run;
                        run += (uint32_t)(b1 - b0);
                        ++nr;
                    }
            rq[nr] = run;
            s_nr = nr;
            na = -1;
        } else if (nc >= 3) {
            na = 3;
            auto sorted3 = [nc](int v, int *o) {
                int lo = v == 0 ? nc - 1 : v - 1, hi = v == nc - 1 ? 0 : v + 1;
                int m0 = lo < v ? lo : v, m1 = lo < v ? v : lo;  // sort {lo, v, hi}
                if (hi < m0) { o[0] = hi; o[1] = m0; o[2] = m1; }
                else if (hi < m1) { o[0] = m0; o[1] = hi; o[2] = m1; }
                else { o[0] = m0; o[1] = m1; o[2] = hi; }
            };
            sorted3(cx, ax);
            sorted3(cy, ay);
            sorted3(cz, az);
        } else {
            ax[0] = ay[0] = az[0] = 0;
        }
        int nr = 0;
        uint32_t run = 0;
        for (int u = 0; u < na; ++u)
            for (int v = 0; v < na; ++v)
                for (int w = 0; w < na; ++w) {
                    const uint32_t id = ((uint32_t)ax[u] * nc + ay[v]) * nc + az[w];
                    if (id <= c) continue;
                    const uint64_t b0 = a.cstart[id], b1 = a.cstart[id + 1];
                    if (b1 == b0) continue;
                    rs[nr] = b0;
                    rq[nr] = run;
                    run += (uint32_t)(b1 - b0);
                    ++nr;
                }
        if (na > 0) {
            rq[nr] = run;
            s_nr = nr;
        }
    }
    __syncthreads();
    const int nr = s_nr;
    const uint32_t Mf = rq[nr];
    const bool wrapfree = __builtin_amdgcn_readfirstlane((int)s_wf) != 0;
    // stage the candidates' coordinates (own cell, then the forward ranges)
    // in LDS when they fit: every label of the group sweeps the same set
    const uint32_t P = (uint32_t)(ce - cs);
    const bool staged = P + Mf <= kStage;
    if (staged) {
        for (uint32_t k = threadIdx.x; k < P + Mf; k += kBlock) {
            uint64_t l;
            if (k < P) {
                l = cs + k;
            } else {
                const uint32_t g = k - P;
                const uint32_t r = upper_index(rq, (uint32_t)nr, g);
                l = rs[r] + (g - rq[r]);
            }
            lx[k] = a.X[l];
            ly[k] = a.Y[l];
            lz[k] = a.Z[l];
            if (FILL && k >= P) lj[k - P] = (uint32_t)l;
        }
        __syncthreads();
    }
    uint32_t mymax;
    if (staged)
        mymax = wrapfree ? edge_rows<FILL, false, true>(a, t, rs, rq, nr, Mf, i0, i1, cs, ce, lx, ly, lz, lj)
                         : edge_rows<FILL, true, true>(a, t, rs, rq, nr, Mf, i0, i1, cs, ce, lx, ly, lz, lj);
    else
        mymax = wrapfree ? edge_rows<FILL, false, false>(a, t, rs, rq, nr, Mf, i0, i1, cs, ce, lx, ly, lz, lj)
                         : edge_rows<FILL, true, false>(a, t, rs, rq, nr, Mf, i0, i1, cs, ce, lx, ly, lz, lj);
    // the largest forward degree: one value per group, and a device atomic
    // only when it could raise the running maximum (one address shared by
    // every group would otherwise serialise tens of thousands of atomics)
    if (!FILL) {
        __shared__ uint32_t s_max;
        if (threadIdx.x == 0) s_max = 0;
        __syncthreads();
        if ((threadIdx.x & 63) == 0 && mymax) atomicMax(&s_max, mymax);
        __syncthreads();
        if (threadIdx.x == 0 && s_max > __atomic_load_n(a.maxdeg, __ATOMIC_RELAXED)) atomicMax(a.maxdeg, s_max);
    }
}

// Graph statistics outside the build: in-degrees (for the full degrees) and
// the undirected pair count per bin, over rows [l0, l1) whose entries start
// at obase in col / bin.
__global__ __launch_bounds__(kBlock) void k_stats(const uint64_t *__restrict__ rp,
                                                  const uint32_t *__restrict__ col,
                                                  const uint8_t *__restrict__ bin, uint32_t l0,
                                                  uint32_t l1, uint64_t obase, int nb,
                                                  uint32_t *__restrict__ indeg,
                                                  unsigned long long *__restrict__ pair_hist) {
    constexpr int kCopies = 8;
    __shared__ unsigned int ph[kCopies][256];
    for (int k = threadIdx.x; k < kCopies * 256; k += blockDim.x) (&ph[0][0])[k] = 0;
    __syncthreads();
    const uint32_t l = l0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (l < l1) {
        unsigned int *mine = ph[threadIdx.x % kCopies];
        for (uint64_t e = rp[l] - obase; e < rp[l + 1] - obase; ++e) {
            atomicAdd(&indeg[col[e]], 1u);
            atomicAdd(&mine[bin[e]], 1u);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        unsigned long long v = 0;
        for (int c = 0; c < kCopies; ++c) v += ph[c][k];
        if (v) atomicAdd(&pair_hist[k], v);
    }
}

// Pair counts and exact weighted pair sums per bin (the internal 2pCF of
// Sec. 3.3): a wavefront per row, its lanes over the row's entries; counts
// and the weighted terms' low 32 bits / arithmetic high parts summed in LDS,
// then added to the 64-bit counts and 128-bit sums. Anchored: only pairs
// whose smaller original index lies in [alo, ahi).
struct PairArgs {
    const uint64_t *rp;
    const uint32_t *col;
    const uint8_t *bin;
    const uint32_t *perm;
    const double *w;
    double wmul;
    uint32_t l0, l1;
    uint64_t obase;
    int nb;
    uint32_t alo, ahi;
    unsigned long long *cnt, *wsum;
};

template <bool WEIGHTED, bool ANCHORED>
__global__ __launch_bounds__(kBlock) void k_pairs(PairArgs a) {
    __shared__ unsigned long long sc[256], slo[256], shi[256];
    for (int k = threadIdx.x; k < 256; k += kBlock) {
        sc[k] = 0;
        if (WEIGHTED) {
            slo[k] = 0;
            shi[k] = 0;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t l = a.l0 + blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); l < a.l1; l += waves) {
        const uint64_t b0 = a.rp[l] - a.obase, b1 = a.rp[l + 1] - a.obase;
        const double wi = WEIGHTED ? a.w[l] : 0.0;
        const uint32_t pi = ANCHORED ? a.perm[l] : 0u;
        for (uint64_t e = b0 + lane; e < b1; e += 64) {
            const uint32_t j = a.col[e];
            if (ANCHORED) {
                const uint32_t m = min(pi, a.perm[j]);
                if (m < a.alo || m >= a.ahi) continue;
            }
            const uint32_t b = a.bin[e];
            atomicAdd(&sc[b], 1ull);
            if (WEIGHTED) {
                const double wj = a.w[j];
                const double x = __dmul_rn(__dmul_rn(fabs(wi), fabs(wj)), a.wmul);
                const bool ng = (wi < 0.0) ^ (wj < 0.0);
                if (narrow_term(x)) {
                    const long long m = (long long)big_term_u64(x);
                    lds_term(&slo[b], &shi[b], ng ? -m : m);
                } else {
                    add128_words(&a.wsum[2 * b], wide_term(x, ng));
                }
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < a.nb; k += kBlock) {
        if (sc[k]) atomicAdd(&a.cnt[k], sc[k]);
        if (WEIGHTED && (slo[k] | shi[k])) add128_words(&a.wsum[2 * k], lds_sum128(slo[k], shi[k]));
    }
}

// ---- exclusive scan u32 -> u64 (out has n+1 entries, out[n] = total) ----

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ uint64_t block_scan_u64(uint64_t v, uint64_t *wtot, uint64_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wtot[wid] = x;
    __syncthreads();
    uint64_t off = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        uint64_t t = wtot[k];
        if (k < wid) off += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

template <class TI>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const TI *__restrict__ in, uint64_t n,
                                                        uint64_t *__restrict__ out,
                                                        uint64_t *__restrict__ tile_sums) {
    __shared__ uint64_t wtot[kBlock / 64];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? (uint64_t)in[base + k] : 0;
        s += v[k];
    }
    uint64_t total;
    uint64_t pre = block_scan_u64(s, wtot, total);
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = pre;
        pre += v[k];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(uint64_t *__restrict__ out, uint64_t n,
                           const uint64_t *__restrict__ tile_off) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / kScanTile];
}

__global__ void k_set_total(uint64_t *out, uint64_t n, const uint64_t *tile_off, uint64_t ntiles,
                            const uint64_t *tile_sums) {
    out[n] = tile_off[ntiles - 1] + tile_sums[ntiles - 1];
}

inline unsigned grid_for(uint64_t n, int block = kBlock) { return (unsigned)((n + block - 1) / block); }

// Exclusive scan of n values into out[0..n]; out[n] = total.
// Temporaries come from the building context's cache (reused only by later
// work on the same stream) or, without one, are freed after a synchronize.
template <class TI>
void scan(const TI *in, uint64_t n, uint64_t *out, hipStream_t s, const std::shared_ptr<DevPool> &pool) {
    if (n == 0) {
        k_fill_u64<<<1, 1, 0, s>>>(out, 1, 0);
        return;
    }
    uint64_t ntiles = (n + kScanTile - 1) / kScanTile;
    DevBuf sums(sizeof(uint64_t) * ntiles, pool), offs(sizeof(uint64_t) * (ntiles + 1), pool);
    k_scan_tiles<TI><<<(unsigned)ntiles, kBlock, 0, s>>>(in, n, out, sums.as<uint64_t>());
    GS_HIP(hipGetLastError());
    if (ntiles > 1) {
        scan<uint64_t>(sums.as<uint64_t>(), ntiles, offs.as<uint64_t>(), s, pool);
        k_scan_add<<<grid_for(n), kBlock, 0, s>>>(out, n, offs.as<uint64_t>());
    } else {
        k_fill_u64<<<1, 1, 0, s>>>(offs.as<uint64_t>(), 1, 0);
    }
    k_set_total<<<1, 1, 0, s>>>(out, n, offs.as<uint64_t>(), ntiles, sums.as<uint64_t>());
    GS_HIP(hipGetLastError());
    if (!pool) GS_HIP(hipStreamSynchronize(s));  // sums/offs are freed on return
}

// Chunks of at most `chunk` labels per cell.
__global__ void k_chunk_count(const uint64_t *__restrict__ cstart, uint32_t ncell, uint32_t chunk,
                              uint32_t *__restrict__ nch) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) nch[c] = (uint32_t)((cstart[c + 1] - cstart[c] + chunk - 1) / chunk);
}

// The cell of every chunk.
__global__ void k_chunk_cells(const uint64_t *__restrict__ chpref, uint32_t ncell, uint32_t *__restrict__ gcell) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell)
        for (uint64_t k = chpref[c]; k < chpref[c + 1]; ++k) gcell[k] = c;
}

// sum of (out-degree + in-degree)^2 over labels
__global__ void k_sum_sq_deg(const uint64_t *__restrict__ rp, const uint32_t *__restrict__ indeg,
                             uint32_t n, unsigned long long *__restrict__ acc) {
    uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0;
    if (l < n) {
        uint64_t m = (rp[l + 1] - rp[l]) + indeg[l];
        v = m * m;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(acc, v);
}

// Builder arguments shared by the count and fill passes.
EdgeArgs edge_args(const Graph &g, const BuildJob &job) {
    const uint32_t n = (uint32_t)g.n;
    EdgeArgs ea{};
    ea.X = job.C;
    ea.Y = job.C + n;
    ea.Z = job.C + 2 * (size_t)n;
    ea.cellL = job.cellL.as<uint32_t>();
    ea.cstart = job.cstart.as<uint64_t>();
    ea.chpref = job.chpref.as<uint64_t>();
    ea.gcell = job.gcell.as<uint32_t>();
    ea.ncell = (uint32_t)((uint64_t)job.nc * job.nc * job.nc);
    ea.chunk = job.chunk;
    ea.thr = job.thr.as<double>();
    ea.n = n;
    ea.l0 = 0;
    ea.l1 = n;
    ea.obase = 0;
    ea.nc = job.nc;
    ea.nb = g.nbins;
    ea.periodic = g.periodic ? 1 : 0;
    ea.L = g.periodic ? g.box : HUGE_VAL;
    ea.half = g.periodic ? 0.5 * g.box : HUGE_VAL;
    return ea;
}

}  // namespace

// Phase 1: cells, relabelling, degree pass and row offsets. Afterwards the
// exact edge count (hence the CSR footprint) is known; no edge memory is held.
void build_begin(Ctx &ctx, Graph &g, const double *xyz, const double *w, BuildJob &job) {
    hipStream_t s = ctx.stream;
    const uint32_t n = (uint32_t)g.n;
    GS_HIP(hipEventRecord(ctx.ev[0], s));
    const bool on_dev = (g.flags & GS_INPUT_ON_DEVICE) != 0;
    const bool weighted = (g.flags & GS_WEIGHTED) != 0;
    const bool keep = (g.flags & GS_KEEP_COORDS) != 0;

    g.row_ptr.alloc(sizeof(uint64_t) * ((size_t)n + 1), ctx.pool);
    g.perm.alloc(sizeof(uint32_t) * (size_t)(n ? n : 1), ctx.pool);
    job.E = 0;
    job.empty = n == 0;
    if (n == 0) {
        k_fill_u64<<<1, 1, 0, s>>>(g.row_ptr.as<uint64_t>(), 1, 0);
        if (keep) g.coords.alloc(8, ctx.pool);
        if (weighted) g.weights.alloc(8, ctx.pool);
        GS_HIP(hipStreamSynchronize(s));
        return;
    }

    DevBuf in_xyz, in_w;
    const double *dxyz = xyz, *dw = w;
    if (!on_dev) {
        in_xyz.alloc(sizeof(double) * 3 * (size_t)n, ctx.pool);
        GS_HIP(hipMemcpyAsync(in_xyz.p, xyz, sizeof(double) * 3 * (size_t)n, hipMemcpyHostToDevice, s));
        dxyz = in_xyz.as<double>();
        if (weighted) {
            in_w.alloc(sizeof(double) * (size_t)n, ctx.pool);
            GS_HIP(hipMemcpyAsync(in_w.p, w, sizeof(double) * (size_t)n, hipMemcpyHostToDevice, s));
            dw = in_w.as<double>();
        }
    }

    // cells at least rmax*(1+1e-9) wide; fewer for sparse catalogues
    double ncd = std::floor(g.box / (g.rmax * (1.0 + 1e-9)));
    double cap = std::max(3.0, std::ceil(2.0 * std::cbrt((double)n)));
    ncd = std::min(ncd, std::min(cap, 256.0));
    // periodic: fewer than 3 cells per axis would make a cell its own
    // neighbour twice, so such boxes take one cell; survey geometry has no
    // wrap and takes any count
    int nc = g.periodic ? (ncd < 3 ? 1 : (int)ncd) : std::max(1, (int)ncd);
    uint64_t ncell = (uint64_t)nc * nc * nc;

    const std::shared_ptr<DevPool> &pool = ctx.pool;
    DevBuf cell_of(sizeof(uint32_t) * n, pool), count(sizeof(uint32_t) * ncell, pool),
        order(sizeof(uint32_t) * n, pool), flags(64, pool), deg(sizeof(uint32_t) * n, pool);
    job.cstart.alloc(sizeof(uint64_t) * (ncell + 1), ctx.pool);
    job.cellL.alloc(sizeof(uint32_t) * n, ctx.pool);
    DevBuf &cstart = job.cstart, &cellL = job.cellL;
    job.nc = nc;
    uint32_t *fl = flags.as<uint32_t>();
    k_fill_u32<<<1, 64, 0, s>>>(fl, 8, 0);
    k_fill_u64<<<1, 64, 0, s>>>(flags.as<uint64_t>() + 4, 1, ~0ull);  // wmin bits
    k_fill_u64<<<1, 64, 0, s>>>(flags.as<uint64_t>() + 5, 1, 0);      // wmax bits
    k_fill_u32<<<grid_for(ncell), kBlock, 0, s>>>(count.as<uint32_t>(), ncell, 0);
    k_cells<<<grid_for(n), kBlock, 0, s>>>(dxyz, n, g.box, nc, cell_of.as<uint32_t>(),
                                           count.as<uint32_t>(), fl);
    if (weighted)
        k_weights<<<grid_for(n), kBlock, 0, s>>>(dw, n, fl, (unsigned long long *)(flags.as<uint64_t>() + 4));
    GS_HIP(hipGetLastError());
    scan<uint32_t>(count.as<uint32_t>(), ncell, cstart.as<uint64_t>(), s, ctx.pool);
    {
        DevBuf nch(sizeof(uint32_t) * ncell, pool);
        job.chpref.alloc(sizeof(uint64_t) * (ncell + 1), ctx.pool);
        job.chunk = kChunk;
        if (const char *ec = getenv("GS_BUILD_CHUNK")) job.chunk = (uint32_t)std::min(1024, std::max(8, atoi(ec)));
        job.grid = (uint64_t)n / job.chunk + ncell;   // at most one partial chunk per cell
        job.gcell.alloc(sizeof(uint32_t) * job.grid, ctx.pool);
        k_chunk_count<<<grid_for(ncell), kBlock, 0, s>>>(cstart.as<uint64_t>(), (uint32_t)ncell, job.chunk,
                                                          nch.as<uint32_t>());
        scan<uint32_t>(nch.as<uint32_t>(), ncell, job.chpref.as<uint64_t>(), s, ctx.pool);
        k_chunk_cells<<<grid_for(ncell), kBlock, 0, s>>>(job.chpref.as<uint64_t>(), (uint32_t)ncell,
                                                          job.gcell.as<uint32_t>());
        GS_HIP(hipGetLastError());
    }
    k_fill_u32<<<grid_for(ncell), kBlock, 0, s>>>(count.as<uint32_t>(), ncell, 0);
    k_scatter<<<grid_for(n), kBlock, 0, s>>>(cell_of.as<uint32_t>(), n, cstart.as<uint64_t>(),
                                             count.as<uint32_t>(), order.as<uint32_t>());
    k_rank<<<grid_for(n), kBlock, 0, s>>>(order.as<uint32_t>(), cell_of.as<uint32_t>(),
                                          cstart.as<uint64_t>(), n, g.perm.as<uint32_t>());
    double *C;
    if (keep) {
        g.coords.alloc(sizeof(double) * 3 * (size_t)n, ctx.pool);
        C = g.coords.as<double>();
    } else {
        job.tmp_coords.alloc(sizeof(double) * 3 * (size_t)n, ctx.pool);
        C = job.tmp_coords.as<double>();
    }
    job.C = C;
    if (weighted) g.weights.alloc(sizeof(double) * n, ctx.pool);
    k_gather<<<grid_for(n), kBlock, 0, s>>>(g.perm.as<uint32_t>(), dxyz, dw, cell_of.as<uint32_t>(), n,
                                            C, C + n, C + 2 * (size_t)n,
                                            weighted ? g.weights.as<double>() : nullptr,
                                            cellL.as<uint32_t>());
    GS_HIP(hipGetLastError());

    job.thr.alloc(sizeof(double) * 256, ctx.pool);
    GS_HIP(hipMemcpyAsync(job.thr.p, g.bins.t, sizeof(double) * 256, hipMemcpyHostToDevice, s));

    EdgeArgs ea = edge_args(g, job);
    ea.deg = deg.as<uint32_t>();
    ea.maxdeg = fl + 1;
    k_edges<false><<<(unsigned)job.grid, kBlock, 0, s>>>(ea);
    GS_HIP(hipGetLastError());
    scan<uint32_t>(deg.as<uint32_t>(), n, g.row_ptr.as<uint64_t>(), s, ctx.pool);

    struct {
        uint32_t f[8];
        uint64_t wmin, wmax;
    } hf;
    uint64_t E = 0;
    GS_HIP(hipEventRecord(ctx.ev[1], s));
    GS_HIP(hipMemcpyAsync(&hf, fl, sizeof hf, hipMemcpyDeviceToHost, s));
    GS_HIP(hipMemcpyAsync(&E, g.row_ptr.as<uint64_t>() + n, sizeof E, hipMemcpyDeviceToHost, s));
    GS_HIP(hipStreamSynchronize(s));
    if (hf.f[0] & 1u) fail(GS_EINVAL, "coordinate outside [0, box) or NaN");
    if (hf.f[0] & 2u) fail(GS_EINVAL, "weights must be finite and nonzero");
    g.n_edges = E;
    g.max_deg = hf.f[1];
    if (weighted) {
        memcpy(&g.wmin, &hf.wmin, 8);
        memcpy(&g.wmax, &hf.wmax, 8);
        g.wneg = (hf.f[0] & 4u) != 0;
        int s3 = 0;
        g.wscale = weight_scale_ok(g, 3, &s3) ? s3 : kNoScale;
    }
    job.E = E;
    float ms = 0;
    GS_HIP(hipEventElapsedTime(&ms, ctx.ev[0], ctx.ev[1]));
    job.begin_ms = ms;
}

// CSR bytes the graph will hold once build_end runs resident.
uint64_t build_footprint(const Graph &g, const BuildJob &job) {
    return g.row_ptr.bytes + g.perm.bytes + g.coords.bytes + g.weights.bytes + 5 * (job.E + kRowSlack);
}

// Phase 2: the CSR itself, resident or in host-pinned windows (tile_ok).
void build_end(Ctx &ctx, Graph &g, BuildJob &job, bool tile_ok) {
    hipStream_t s = ctx.stream;
    const uint32_t n = (uint32_t)g.n;
    const uint64_t E = job.E;
    GS_HIP(hipEventRecord(ctx.ev[0], s));
    if (job.empty) {
        g.col.alloc(sizeof(uint32_t) * kRowSlack, ctx.pool);
        g.bin.alloc(kRowSlack, ctx.pool);
        g.device_bytes = g.row_ptr.bytes + g.perm.bytes + g.col.bytes + g.bin.bytes;
        ctx.t.build_ms = job.begin_ms;
        return;
    }
    EdgeArgs ea = edge_args(g, job);

    // resident, or host-tiled windows when the CSR would not fit the budget
    // (GS_WINDOWS forces a window count, as the paper's environment override)
    const uint64_t fixed = g.row_ptr.bytes + g.perm.bytes + g.coords.bytes + g.weights.bytes;
    const uint64_t csr = 5 * E;
    int W = 1;
    if (const char *ew = getenv("GS_WINDOWS")) W = std::max(1, atoi(ew));
    if (W == 1 && tile_ok && fixed + csr > ctx.budget) {
        if (ctx.budget <= fixed + (1u << 20)) fail(GS_EDEVMEM, "budget below the graph's per-point arrays");
        const uint64_t per_win = (ctx.budget - fixed) / 4;  // 4 window buffers while counting
        W = (int)std::min<uint64_t>((csr + per_win - 1) / per_win, 1u << 20);
    }
    if (W > 1 && (uint64_t)W > (uint64_t)n) W = (int)std::max<uint32_t>(1, n);

    ea.rp = g.row_ptr.as<uint64_t>();
    if (W == 1) {
        g.col.alloc(sizeof(uint32_t) * (E + kRowSlack), ctx.pool);
        g.bin.alloc(E + kRowSlack, ctx.pool);
        ea.col = g.col.as<uint32_t>();
        ea.bin = g.bin.as<uint8_t>();
        k_edges<true><<<(unsigned)job.grid, kBlock, 0, s>>>(ea);
    } else {
        // row-aligned windows of about E/W entries each
        std::vector<uint64_t> hrp((size_t)n + 1);
        GS_HIP(hipMemcpyAsync(hrp.data(), g.row_ptr.p, sizeof(uint64_t) * (n + 1), hipMemcpyDeviceToHost, s));
        GS_HIP(hipStreamSynchronize(s));
        g.win.assign(1, 0);
        for (int w = 1; w < W; ++w) {
            const uint64_t target = E / W * w;
            uint64_t l = (uint64_t)(std::lower_bound(hrp.begin(), hrp.end(), target) - hrp.begin());
            l = std::min<uint64_t>(l, n);
            if (l > g.win.back() && l < n) g.win.push_back(l);
        }
        g.win.push_back(n);
        W = (int)g.win.size() - 1;
        g.win_edge.resize(W + 1);
        uint64_t maxE = 1;
        for (int w = 0; w <= W; ++w) g.win_edge[w] = hrp[g.win[w]];
        for (int w = 0; w < W; ++w) maxE = std::max<uint64_t>(maxE, g.win_edge[w + 1] - g.win_edge[w]);
        g.hcol.alloc(sizeof(uint32_t) * (E ? E : 1));
        g.hbin.alloc(E ? E : 1);
        g.col.alloc(4, ctx.pool);
        g.bin.alloc(1, ctx.pool);
        DevBuf stc(sizeof(uint32_t) * maxE, ctx.pool), stb(maxE, ctx.pool);
        ea.col = stc.as<uint32_t>();
        ea.bin = stb.as<uint8_t>();
        for (int w = 0; w < W; ++w) {
            ea.l0 = (uint32_t)g.win[w];
            ea.l1 = (uint32_t)g.win[w + 1];
            ea.obase = g.win_edge[w];
            const uint64_t ne = g.win_edge[w + 1] - g.win_edge[w];
            k_edges<true><<<(unsigned)job.grid, kBlock, 0, s>>>(ea);
            GS_HIP(hipGetLastError());
            GS_HIP(hipMemcpyAsync(g.hcol.as<uint32_t>() + g.win_edge[w], stc.p, ne * 4, hipMemcpyDeviceToHost, s));
            GS_HIP(hipMemcpyAsync(g.hbin.as<uint8_t>() + g.win_edge[w], stb.p, ne, hipMemcpyDeviceToHost, s));
            GS_HIP(hipStreamSynchronize(s));
        }
    }
    g.n_windows = W;
    GS_HIP(hipGetLastError());
    GS_HIP(hipEventRecord(ctx.ev[1], s));
    GS_HIP(hipStreamSynchronize(s));
    float ms = 0;
    GS_HIP(hipEventElapsedTime(&ms, ctx.ev[0], ctx.ev[1]));
    ctx.t.build_ms = job.begin_ms + ms;
    g.device_bytes = g.row_ptr.bytes + g.col.bytes + g.bin.bytes + g.perm.bytes + g.coords.bytes +
                     g.weights.bytes;
}

// Pair histogram and sum of squared full degrees, computed once on demand
// (they are reported, not needed by the counts).
void graph_stats(Graph &g) {
    if (g.stats_ready) return;
    const uint32_t n = (uint32_t)g.n;
    std::fill(g.pair_hist, g.pair_hist + 255, 0ull);
    g.sum_sq_deg = 0;
    if (n == 0) {
        g.stats_ready = true;
        return;
    }
    hipStream_t s = nullptr;
    GS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
    } guard{s};
    DevBuf ph(sizeof(uint64_t) * 256), indeg(sizeof(uint32_t) * n), sq(8);
    k_fill_u64<<<1, 256, 0, s>>>(ph.as<uint64_t>(), 256, 0);
    k_fill_u32<<<grid_for(n), kBlock, 0, s>>>(indeg.as<uint32_t>(), n, 0);
    k_fill_u64<<<1, 1, 0, s>>>(sq.as<uint64_t>(), 1, 0);
    const uint64_t *rp = g.row_ptr.as<uint64_t>();
    unsigned long long *hp = (unsigned long long *)ph.as<uint64_t>();
    if (g.n_windows == 1) {
        k_stats<<<grid_for(n), kBlock, 0, s>>>(rp, g.col.as<uint32_t>(), g.bin.as<uint8_t>(), 0, n, 0,
                                               g.nbins, indeg.as<uint32_t>(), hp);
    } else {
        uint64_t maxE = 1;
        for (int w = 0; w < g.n_windows; ++w) maxE = std::max<uint64_t>(maxE, g.win_edge[w + 1] - g.win_edge[w]);
        DevBuf wc(maxE * 4), wb(maxE);
        for (int w = 0; w < g.n_windows; ++w) {
            const uint64_t e0 = g.win_edge[w], ne = g.win_edge[w + 1] - e0;
            GS_HIP(hipMemcpyAsync(wc.p, g.hcol.as<uint32_t>() + e0, ne * 4, hipMemcpyHostToDevice, s));
            GS_HIP(hipMemcpyAsync(wb.p, g.hbin.as<uint8_t>() + e0, ne, hipMemcpyHostToDevice, s));
            const uint32_t l0 = (uint32_t)g.win[w], l1 = (uint32_t)g.win[w + 1];
            k_stats<<<grid_for(l1 - l0), kBlock, 0, s>>>(rp, wc.as<uint32_t>(), wb.as<uint8_t>(), l0, l1, e0,
                                                         g.nbins, indeg.as<uint32_t>(), hp);
            GS_HIP(hipStreamSynchronize(s));
        }
    }
    k_sum_sq_deg<<<grid_for(n), kBlock, 0, s>>>(rp, indeg.as<uint32_t>(), n, (unsigned long long *)sq.as<uint64_t>());
    GS_HIP(hipGetLastError());
    uint64_t hph[256];
    GS_HIP(hipMemcpyAsync(hph, ph.p, sizeof hph, hipMemcpyDeviceToHost, s));
    GS_HIP(hipMemcpyAsync(&g.sum_sq_deg, sq.p, 8, hipMemcpyDeviceToHost, s));
    GS_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < 255; ++k) g.pair_hist[k] = k < g.nbins ? hph[k] : 0;
    g.stats_ready = true;
}

// Pair counts per bin and (with weights) their exact weighted sums.
void pair_sums_run(Ctx &ctx, const Graph &g, uint64_t *pairs, uint64_t *wsum, int *wscale,
                   const gs_anchor_range *anchors) {
    const int nb = g.nbins;
    const bool weighted = wsum != nullptr;
    const bool anchored = anchors != nullptr;
    if (anchored && anchors->lo > anchors->hi) fail(GS_EINVAL, "anchor range lo > hi");
    const int s2 = weighted ? weight_scale(g, 2) : 0;
    hipStream_t s = ctx.stream;
    unsigned long long *dv = (unsigned long long *)ctx.scratch_get(8 * 3 * 256);
    k_fill_u64<<<3, 256, 0, s>>>((uint64_t *)dv, 3 * 256, 0);
    PairArgs a{};
    a.rp = g.row_ptr.as<uint64_t>();
    a.perm = g.perm.as<uint32_t>();
    a.w = weighted ? g.weights.as<double>() : nullptr;
    a.wmul = std::ldexp(1.0, s2);
    a.nb = nb;
    a.alo = anchored ? (uint32_t)std::min<uint64_t>(anchors->lo, 0xFFFFFFFFull) : 0;
    a.ahi = anchored ? (uint32_t)std::min<uint64_t>(anchors->hi, 0xFFFFFFFFull) : 0;
    a.cnt = dv;
    a.wsum = dv + 256;
    auto go = [&](uint32_t l0, uint32_t l1) {
        if (l1 <= l0) return;
        a.l0 = l0;
        a.l1 = l1;
        const uint64_t waves = (uint64_t)(l1 - l0);
        const unsigned grid = (unsigned)std::min<uint64_t>((waves + 3) / 4, (uint64_t)ctx.n_cu * 16);
        if (weighted) anchored ? k_pairs<true, true><<<grid, kBlock, 0, s>>>(a) : k_pairs<true, false><<<grid, kBlock, 0, s>>>(a);
        else anchored ? k_pairs<false, true><<<grid, kBlock, 0, s>>>(a) : k_pairs<false, false><<<grid, kBlock, 0, s>>>(a);
        GS_HIP(hipGetLastError());
    };
    if (g.n_windows == 1) {
        a.col = g.col.as<uint32_t>();
        a.bin = g.bin.as<uint8_t>();
        a.obase = 0;
        go(0, (uint32_t)g.n);
    } else {
        uint64_t maxE = 1;
        for (int w = 0; w < g.n_windows; ++w) maxE = std::max<uint64_t>(maxE, g.win_edge[w + 1] - g.win_edge[w]);
        DevBuf wc(maxE * 4), wb(maxE);
        for (int w = 0; w < g.n_windows; ++w) {
            const uint64_t e0 = g.win_edge[w], ne = g.win_edge[w + 1] - e0;
            GS_HIP(hipMemcpyAsync(wc.p, g.hcol.as<uint32_t>() + e0, ne * 4, hipMemcpyHostToDevice, s));
            GS_HIP(hipMemcpyAsync(wb.p, g.hbin.as<uint8_t>() + e0, ne, hipMemcpyHostToDevice, s));
            a.col = wc.as<uint32_t>();
            a.bin = wb.as<uint8_t>();
            a.obase = e0;
            go((uint32_t)g.win[w], (uint32_t)g.win[w + 1]);
            GS_HIP(hipStreamSynchronize(s));
        }
    }
    uint64_t h[3 * 256];
    GS_HIP(hipMemcpyAsync(h, dv, sizeof h, hipMemcpyDeviceToHost, s));
    GS_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < nb; ++k) pairs[k] = h[k];
    if (weighted) {
        for (int k = 0; k < 2 * nb; ++k) wsum[k] = h[256 + k];
        if (wscale) *wscale = s2;
    }
}

void build_run(Ctx &ctx, Graph &g, const double *xyz, const double *w) {
    BuildJob job;
    build_begin(ctx, g, xyz, w, job);
    build_end(ctx, g, job, true);
}

}  // namespace gsn
