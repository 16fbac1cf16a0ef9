/*
 * oracle.c - CPU oracle for binned triangle (3pCF) and 4-clique parity (4pCF)
 * counts on the periodic r < rmax point graph.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the bench's CPU
 * baseline do. It shares no code, header or table with the GPU library.
 *
 * It is deliberately plain and slow: full symmetric neighbour rows from a
 * cell list, then for every hub the original membership test of Sec. 2.2 (a
 * binary search in the spoke's sorted row, logarithmic per candidate), not
 * the merge-walk the paper introduces in Sec. 3.1. The counts it produces are
 * the plain definitions below; the merge-walk reaches the same sets faster.
 *
 * Definitions (floating point: IEEE binary64, round to nearest, no FMA
 * contraction; compile with -ffp-contract=off and without -ffast-math):
 *
 * D1 separation a->b: per axis d = x_b - x_a; if d > L/2 then d -= L, else
 *    if d < -L/2 then d += L (periodic box of the paper's test catalogue,
 *    Sec. 4.1; the minimum-image rule is our reading). sep(b,a) = -sep(a,b)
 *    exactly. Survey geometry (Sec. 5; a negative box argument): d = x_b - x_a.
 * D2 squared length q = (dx*dx + dy*dy) + dz*dz.
 * D3 bins: equal-width radial bins from rmin to rmax (Sec. 4.1). With
 *    D = (rmax - rmin)/nb, e_0 = rmin, e_k = rmin + k*D (0<k<nb), e_nb = rmax,
 *    t_k = e_k*e_k: a pair is an edge iff t_0 <= q < t_nb, and its bin is the
 *    number of k in 1..nb-1 with q >= t_k. The bin is one byte per edge as in
 *    the paper's adjacency lists (Sec. 2.1), so nb <= 255.
 * D5 3pCF: every unordered triangle (all three pairs edges) counts once into
 *    the bin of its sorted side bins b1 <= b2 <= b3, indexed lexicographically
 *    (the sorted-side configurations r1 <= r2 <= r3 of Sec. 5; C(nb+2,3) of
 *    them). Weighted: t = +-(a1*a2)*a3 with a1 <= a2 <= a3 the three weight
 *    magnitudes in ascending order and the sign the product of the weights'
 *    signs; per bin the exact sum of t as a signed 128-bit integer multiple
 *    of 2^-s, where s = 52 - floor(log2(((m*m)*m))) and m is the smallest
 *    weight magnitude. Weights are finite and nonzero, of either sign: the
 *    signed, normalised data-minus-random weights of Sec. 2.1. (For
 *    positive weights: the product of the weights in ascending order.)
 * D4w weighted pairs (the internal 2pCF of Sec. 3.3): per bin the exact sum
 *    over edges of w_i*w_j, in units of 2^-s2, s2 = 52 - floor(log2(m*m)).
 * D6 4pCF parity (Sec. 3.2, Eq. 2 and the degenerate rule): every 4-clique
 *    contributes once per hub h (each of its four vertices): spokes r = sep(h,.)
 *    ordered by q (qa <= qb <= qc); even[idx(bins)] += 1; c = ra x rb,
 *    V = (cx*rcx + cy*rcy) + cz*rcz. Degenerate (no odd contribution) iff
 *    qa == qb or qb == qc or V*V <= 1e-18*((qa*qb)*qc) (the paper's |V| < 1e-9
 *    taken on the normalised volume); otherwise V > 0 -> pos, V < 0 -> neg.
 *
 * D8 6-edge 4pCF (the full four-point configurations of Sec. 3.3 and Sec.
 *    5.3): every 4-clique counts once into the configuration of its six
 *    edge bins. A vertex ordering (p0,p1,p2,p3) of the clique gives the tuple
 *    of the bins of edges (p0p1, p0p2, p0p3, p1p2, p1p3, p2p3); the
 *    configuration is the lexicographically smallest tuple over the 24
 *    orderings (its class under relabelling of the four vertices), and
 *    configurations are indexed by their rank in lexicographic order among
 *    all such smallest tuples.
 *
 * D9 mu-binned 3pCF (anisotropy, Sec. 6): each triangle also carries the
 *    bin of mu = |nz|/|n|, n the normal of its plane (see mu_bin below).
 * D10 parity from direction pixels (Sec. 3.2 as the paper computes it): each
 *    spoke's direction quantised to a pixel, spokes in original-index order,
 *    degenerate iff |V| < 1e-9 (see pixel_of, hub_pixel below).
 *
 * Anchors: only tuples whose smallest original point index lies in
 * [anchor_lo, anchor_hi) are counted.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-3)

typedef unsigned __int128 u128;
typedef __int128 i128;

typedef struct {
    double L, half, rmin, rmax;
    int periodic;  /* 0: survey geometry (a negative box argument), no wrap */
    int nb;
    double t[256]; /* squared bin edges t_0 .. t_nb */
} params_t;

/* box > 0: periodic cube of side box; box < 0: survey geometry (Sec. 5), the
 * points in the cube of side -box, separations without any wrap. */
static int make_params(params_t *p, double box, double rmin, double rmax, int nb) {
    p->periodic = box > 0;
    box = fabs(box);
    if (!(box > 0) || !isfinite(box)) return OR_EINVAL;
    if (nb < 1 || nb > 255) return OR_EINVAL;
    if (!(rmin >= 0) || !(rmin < rmax) || !isfinite(rmax)) return OR_EINVAL;
    if (p->periodic && !(rmax < 0.5 * box)) return OR_EINVAL;
    p->L = box;
    p->half = 0.5 * box;
    p->rmin = rmin;
    p->rmax = rmax;
    p->nb = nb;
    double D = (rmax - rmin) / (double)nb;
    for (int k = 0; k <= nb; ++k) {
        double e = (k == 0) ? rmin : (k == nb ? rmax : rmin + (double)k * D);
        p->t[k] = e * e;
    }
    return OR_OK;
}

static int check_points(const double *xyz, int64_t n, double box) {
    box = fabs(box);
    if (n < 0) return OR_EINVAL;
    if (n > 0 && !xyz) return OR_EINVAL;
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!(xyz[i] >= 0.0 && xyz[i] < box)) return OR_EINVAL; /* also rejects NaN */
    return OR_OK;
}

/* D1 */
static void separation(const params_t *p, const double *a, const double *b, double r[3]) {
    for (int c = 0; c < 3; ++c) {
        double d = b[c] - a[c];
        if (p->periodic) {
            if (d > p->half) d = d - p->L;
            else if (d < -p->half) d = d + p->L;
        }
        r[c] = d;
    }
}

/* D2 */
static double sqlen(const double r[3]) { return (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]; }

/* D3: bin of squared length q, or -1 when the pair is not an edge */
static int edge_bin(const params_t *p, double q) {
    if (!(q >= p->t[0] && q < p->t[p->nb])) return -1;
    int b = 0;
    for (int k = 1; k < p->nb; ++k)
        if (q >= p->t[k]) ++b;
    return b;
}

static int64_t binom2(int64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }
static int64_t binom3(int64_t n) { return n < 3 ? 0 : n * (n - 1) * (n - 2) / 6; }

/* lexicographic rank of the non-decreasing triple b1 <= b2 <= b3 among all
 * such triples over 0..nb-1 */
static int64_t config_index(int nb, int b1, int b2, int b3) {
    return binom3(nb + 2) - binom3(nb - b1 + 2) + binom2(nb - b1 + 1) - binom2(nb - b2 + 1) +
           (b3 - b2);
}

static void sort3i(int *a, int *b, int *c) {
    int t;
    if (*a > *b) { t = *a; *a = *b; *b = t; }
    if (*b > *c) { t = *b; *b = *c; *c = t; }
    if (*a > *b) { t = *a; *a = *b; *b = t; }
}

/* ---------------------------------------------------------------- graph -- */

typedef struct {
    int64_t n;
    int64_t *ptr;   /* n+1 */
    int32_t *col;   /* sorted ascending per row */
    uint8_t *bin;
} rows_t;

static void rows_free(rows_t *g) {
    free(g->ptr);
    free(g->col);
    free(g->bin);
    memset(g, 0, sizeof *g);
}

typedef struct { int32_t j; uint8_t b; } entry_t;

static int entry_cmp(const void *x, const void *y) {
    int32_t a = ((const entry_t *)x)->j, b = ((const entry_t *)y)->j;
    return (a > b) - (a < b);
}

/* Cell list with cells at least rmax*(1+1e-9) wide, so every pair closer than
 * rmax sits in the same or a periodically adjacent cell. If need is not NULL,
 * only rows i with need[i] != 0 are filled; the others are left empty. */
static int build_rows(const params_t *p, const double *xyz, int64_t n, int nthreads,
                      const uint8_t *need, rows_t *g) {
    memset(g, 0, sizeof *g);
    g->n = n;
    int nc = (int)floor(p->L / (p->rmax * (1.0 + 1e-9)));
    if (nc > 128) nc = 128;
    if (p->periodic && nc < 3) nc = 1;   /* fewer would list a cell twice */
    if (nc < 1) nc = 1;
    int64_t ncell = (int64_t)nc * nc * nc;
    int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *cfill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
    int64_t *cellof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int32_t *members = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    g->ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cstart || !cfill || !cellof || !members || !g->ptr) goto nomem;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c3[3];
        for (int a = 0; a < 3; ++a) {
            int64_t c = (int64_t)floor(xyz[3 * i + a] * (double)nc / p->L);
            if (c > nc - 1) c = nc - 1;
            if (c < 0) c = 0;
            c3[a] = c;
        }
        cellof[i] = (c3[0] * nc + c3[1]) * nc + c3[2];
        cstart[cellof[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
    for (int64_t i = 0; i < n; ++i) members[cstart[cellof[i]] + cfill[cellof[i]]++] = (int32_t)i;

    /* pass 1 counts, pass 2 fills */
    for (int pass = 0; pass < 2; ++pass) {
        int failed = 0;
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads)
        for (int64_t i = 0; i < n; ++i) {
            if (need && !need[i]) {
                if (pass == 0) g->ptr[i + 1] = 0;
                continue;
            }
            int64_t ci = cellof[i];
            int cx = (int)(ci / ((int64_t)nc * nc)), cy = (int)((ci / nc) % nc), cz = (int)(ci % nc);
            int64_t cells[27];
            int ncells = 0;
            if (nc == 1) {
                cells[ncells++] = 0;
            } else {
                for (int dx = -1; dx <= 1; ++dx)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dz = -1; dz <= 1; ++dz) {
                            int x = cx + dx, y = cy + dy, z = cz + dz;
                            if (p->periodic) {
                                x = (x + nc) % nc;
                                y = (y + nc) % nc;
                                z = (z + nc) % nc;
                            } else if (x < 0 || y < 0 || z < 0 || x >= nc || y >= nc || z >= nc) {
                                continue;
                            }
                            cells[ncells++] = ((int64_t)x * nc + y) * nc + z;
                        }
            }
            int64_t cnt = 0;
            entry_t *row = NULL;
            if (pass == 1) {
                int64_t m = g->ptr[i + 1] - g->ptr[i];
                row = (entry_t *)malloc(sizeof(entry_t) * (size_t)(m ? m : 1));
                if (!row) { failed = 1; continue; }
            }
            for (int u = 0; u < ncells; ++u) {
                int64_t c = cells[u];
                for (int64_t s = cstart[c]; s < cstart[c + 1]; ++s) {
                    int32_t j = members[s];
                    if (j == i) continue;
                    double r[3];
                    separation(p, &xyz[3 * i], &xyz[3 * (int64_t)j], r);
                    int b = edge_bin(p, sqlen(r));
                    if (b < 0) continue;
                    if (pass == 1) { row[cnt].j = j; row[cnt].b = (uint8_t)b; }
                    ++cnt;
                }
            }
            if (pass == 0) {
                g->ptr[i + 1] = cnt;
            } else {
                qsort(row, (size_t)cnt, sizeof(entry_t), entry_cmp);
                for (int64_t e = 0; e < cnt; ++e) {
                    g->col[g->ptr[i] + e] = row[e].j;
                    g->bin[g->ptr[i] + e] = row[e].b;
                }
                free(row);
            }
        }
        if (failed) goto nomem;
        if (pass == 0) {
            for (int64_t i = 0; i < n; ++i) g->ptr[i + 1] += g->ptr[i];
            int64_t E = g->ptr[n];
            g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E ? E : 1));
            g->bin = (uint8_t *)malloc((size_t)(E ? E : 1));
            if (!g->col || !g->bin) goto nomem;
        }
    }
    free(cstart);
    free(cfill);
    free(cellof);
    free(members);
    return OR_OK;
nomem:
    free(cstart);
    free(cfill);
    free(cellof);
    free(members);
    rows_free(g);
    return OR_ENOMEM;
}

/* position of j in row i, or -1 (binary search: the membership test of the
 * paper's original algorithm) */
static int64_t find(const rows_t *g, int64_t i, int32_t j) {
    int64_t lo = g->ptr[i], hi = g->ptr[i + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->col[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < g->ptr[i + 1] && g->col[lo] == j) ? lo : -1;
}

/* Rows for every point, or -- when only anchors [lo, hi) are counted -- for
 * the anchors and all their neighbours (every vertex of a counted tuple is an
 * anchor or a neighbour of one, and membership tests only read those rows). */
static int rows_for_anchors(const params_t *p, const double *xyz, int64_t n, int nt, int64_t lo,
                            int64_t hi, rows_t *g) {
    if (lo <= 0 && hi >= n) return build_rows(p, xyz, n, nt, NULL, g);
    uint8_t *need = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    if (!need) return OR_ENOMEM;
    for (int64_t i = lo; i < hi; ++i) need[i] = 1;
    rows_t first;
    int rc = build_rows(p, xyz, n, nt, need, &first);
    if (rc != OR_OK) { free(need); return rc; }
    for (int64_t i = lo; i < hi; ++i)
        for (int64_t e = first.ptr[i]; e < first.ptr[i + 1]; ++e) need[first.col[e]] = 1;
    rows_free(&first);
    rc = build_rows(p, xyz, n, nt, need, g);
    free(need);
    return rc;
}

static int resolve_threads(int nthreads) {
    return nthreads > 0 ? nthreads : omp_get_max_threads();
}

/* ---------------------------------------------------------------- API ---- */

int oracle_version(void) { return 1; }

int64_t oracle_config_index(int nbins, int b1, int b2, int b3) {
    return config_index(nbins, b1, b2, b3);
}

/* D3 on a given squared length (exposed for exact bin-edge tests) */
int oracle_edge_bin(double q, double box, double rmin, double rmax, int nbins) {
    params_t p;
    if (make_params(&p, box, rmin, rmax, nbins) != OR_OK) return -2;
    return edge_bin(&p, q);
}

/* D1+D2 for two points (exposed for antisymmetry tests) */
int oracle_separation(const double *a, const double *b, double box, double *r_out, double *q_out) {
    params_t p;
    if (make_params(&p, box, 0.0, 0.25 * fabs(box), 1) != OR_OK) return OR_EINVAL;
    separation(&p, a, b, r_out);
    *q_out = sqlen(r_out);
    return OR_OK;
}

/* Full symmetric neighbour rows, sorted by original index. If cap is smaller
 * than the number of entries, only *n_entries is written. */
int oracle_graph(const double *xyz, int64_t n, double box, double rmin, double rmax, int nbins,
                 int64_t *row_ptr, int32_t *col, uint8_t *bin, int64_t cap, int64_t *n_entries) {
    params_t p;
    int rc = make_params(&p, box, rmin, rmax, nbins);
    if (rc == OR_OK) rc = check_points(xyz, n, box);
    if (rc != OR_OK) return rc;
    if (n >= ((int64_t)1 << 31)) return OR_EINVAL;
    rows_t g;
    rc = build_rows(&p, xyz, n, resolve_threads(0), NULL, &g);
    if (rc != OR_OK) return rc;
    *n_entries = g.ptr[n];
    if (cap >= g.ptr[n]) {
        memcpy(row_ptr, g.ptr, sizeof(int64_t) * (size_t)(n + 1));
        memcpy(col, g.col, sizeof(int32_t) * (size_t)g.ptr[n]);
        memcpy(bin, g.bin, (size_t)g.ptr[n]);
    }
    rows_free(&g);
    return OR_OK;
}

/* scale s of the exact weighted sums of products of k weights: every product
 * of magnitude at least (((m*m)*m)...) (k factors of the smallest weight
 * magnitude m) is an integer multiple of 2^-s. Rejects zero or non-finite
 * weights and ranges whose scaled products would not leave room for 2^40
 * terms in a signed 128-bit sum. */
static int weight_scale_k(const double *w, int64_t n, int k, int *s_out) {
    double wmin = INFINITY, wmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double a = fabs(w[i]);
        if (!(a > 0.0) || !isfinite(a)) return OR_EINVAL;
        if (a < wmin) wmin = a;
        if (a > wmax) wmax = a;
    }
    if (n == 0) { *s_out = 0; return OR_OK; }
    double tlo = wmin, thi = wmax;
    for (int j = 1; j < k; ++j) { tlo = tlo * wmin; thi = thi * wmax; }
    if (!(tlo >= 0x1.0p-1022) || !isfinite(thi)) return OR_EINVAL;
    int s = 52 - ilogb(tlo);
    if (ilogb(thi) + s > 86) return OR_EINVAL;
    *s_out = s;
    return OR_OK;
}

static int weight_scale(const double *w, int64_t n, int *s_out) { return weight_scale_k(w, n, 3, s_out); }

/* +-((a1*a2)*...)*ak: the magnitudes of v[0..k) multiplied in ascending
 * order, signed by the product of their signs */
static double signed_product(const double *v, int k) {
    double a[4];
    int neg = 0;
    for (int j = 0; j < k; ++j) {
        a[j] = fabs(v[j]);
        neg ^= v[j] < 0;
    }
    for (int x = 1; x < k; ++x)
        for (int y = x; y > 0 && a[y - 1] > a[y]; --y) {
            double t = a[y];
            a[y] = a[y - 1];
            a[y - 1] = t;
        }
    double p = a[0];
    for (int j = 1; j < k; ++j) p = p * a[j];
    return neg ? -p : p;
}

static void put128(uint64_t *dst, i128 v) {
    dst[0] = (uint64_t)(u128)v;
    dst[1] = (uint64_t)((u128)v >> 64);
}

/* D4 / D4w: pairs (edges) per bin, and with weights the exact per-bin sums
 * of w_i*w_j (units of 2^-s2). Anchors: pairs whose smaller original index
 * lies in [anchor_lo, anchor_hi). */
int oracle_pair_sums(const double *xyz, int64_t n, const double *w, double box, double rmin, double rmax,
                     int nbins, int64_t anchor_lo, int64_t anchor_hi, uint64_t *pairs, uint64_t *wsum,
                     int *wscale) {
    params_t p;
    int rc = make_params(&p, box, rmin, rmax, nbins);
    if (rc == OR_OK) rc = check_points(xyz, n, box);
    if (rc != OR_OK) return rc;
    if (n >= ((int64_t)1 << 31) || !pairs) return OR_EINVAL;
    int s = 0;
    if (w) {
        if (!wsum) return OR_EINVAL;
        rc = weight_scale_k(w, n, 2, &s);
        if (rc != OR_OK) return rc;
        if (wscale) *wscale = s;
    }
    if (anchor_lo < 0) anchor_lo = 0;
    if (anchor_hi > n) anchor_hi = n;
    rows_t g;
    rc = rows_for_anchors(&p, xyz, n, resolve_threads(0), anchor_lo, anchor_hi, &g);
    if (rc != OR_OK) return rc;
    i128 *acc = (i128 *)calloc((size_t)nbins, sizeof(i128));
    if (!acc) { rows_free(&g); return OR_ENOMEM; }
    memset(pairs, 0, sizeof(uint64_t) * (size_t)nbins);
    const double scale = ldexp(1.0, s);
    for (int64_t i = anchor_lo; i < anchor_hi; ++i)
        for (int64_t e = g.ptr[i]; e < g.ptr[i + 1]; ++e) {
            const int32_t j = g.col[e];
            if (j <= i) continue;
            pairs[g.bin[e]] += 1;
            if (w) acc[g.bin[e]] += (i128)((w[i] * w[j]) * scale);
        }
    if (w)
        for (int b = 0; b < nbins; ++b) put128(&wsum[2 * b], acc[b]);
    free(acc);
    rows_free(&g);
    return OR_OK;
}

int oracle_count_3pcf(const double *xyz, int64_t n, const double *w, double box, double rmin,
                      double rmax, int nbins, int64_t anchor_lo, int64_t anchor_hi, int nthreads,
                      uint64_t *hist, uint64_t *wsum, int *wscale, uint64_t *n_tri,
                      int *threads_used) {
    params_t p;
    int rc = make_params(&p, box, rmin, rmax, nbins);
    if (rc == OR_OK) rc = check_points(xyz, n, box);
    if (rc != OR_OK) return rc;
    if (n >= ((int64_t)1 << 31) || !hist || !n_tri) return OR_EINVAL;
    int s = 0;
    if (w) {
        if (!wsum) return OR_EINVAL;
        rc = weight_scale(w, n, &s);
        if (rc != OR_OK) return rc;
        if (wscale) *wscale = s;
    }
    if (anchor_lo < 0) anchor_lo = 0;
    if (anchor_hi > n) anchor_hi = n;
    int nt = resolve_threads(nthreads);
    if (threads_used) *threads_used = nt;
    rows_t g;
    rc = rows_for_anchors(&p, xyz, n, nt, anchor_lo, anchor_hi, &g);
    if (rc != OR_OK) return rc;
    int64_t nconf = binom3(nbins + 2);
    uint64_t *th = (uint64_t *)calloc((size_t)(nt * nconf), sizeof(uint64_t));
    i128 *tw = w ? (i128 *)calloc((size_t)(nt * nconf), sizeof(i128)) : NULL;
    uint64_t *tn = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    if (!th || !tn || (w && !tw)) { free(th); free(tw); free(tn); rows_free(&g); return OR_ENOMEM; }
    double scale = ldexp(1.0, s);

#pragma omp parallel num_threads(nt)
    {
        int tid = omp_get_thread_num();
        uint64_t *H = th + (int64_t)tid * nconf;
        i128 *Wt = w ? tw + (int64_t)tid * nconf : NULL;
        uint64_t cnt = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = anchor_lo; i < anchor_hi; ++i) {
            for (int64_t a = g.ptr[i]; a < g.ptr[i + 1]; ++a) {
                int32_t j = g.col[a];
                if (j <= i) continue;
                for (int64_t b = a + 1; b < g.ptr[i + 1]; ++b) {
                    int32_t k = g.col[b];
                    int64_t f = find(&g, j, k);
                    if (f < 0) continue;
                    int b1 = g.bin[a], b2 = g.bin[b], b3 = g.bin[f];
                    sort3i(&b1, &b2, &b3);
                    int64_t idx = config_index(nbins, b1, b2, b3);
                    H[idx] += 1;
                    ++cnt;
                    if (Wt) {
                        const double v[3] = {w[i], w[j], w[k]};
                        Wt[idx] += (i128)(signed_product(v, 3) * scale);
                    }
                }
            }
        }
        tn[tid] = cnt;
    }
    memset(hist, 0, sizeof(uint64_t) * (size_t)nconf);
    *n_tri = 0;
    for (int t = 0; t < nt; ++t) {
        *n_tri += tn[t];
        for (int64_t c = 0; c < nconf; ++c) hist[c] += th[(int64_t)t * nconf + c];
    }
    if (w) {
        for (int64_t c = 0; c < nconf; ++c) {
            i128 acc = 0;
            for (int t = 0; t < nt; ++t) acc += tw[(int64_t)t * nconf + c];
            put128(&wsum[2 * c], acc);
        }
    }
    free(th);
    free(tw);
    free(tn);
    rows_free(&g);
    return OR_OK;
}

/* one hub's contribution to the parity histograms (D6): its configuration
 * in *idx; returns 0 (pos), 1 (neg) or 2 (degenerate) */
static int hub_parity(const params_t *p, const double *xyz, int64_t h, const int64_t s[3], int64_t *idx_out) {
    double r[3][3], q[3];
    int ord[3] = {0, 1, 2};
    for (int u = 0; u < 3; ++u) {
        separation(p, &xyz[3 * h], &xyz[3 * s[u]], r[u]);
        q[u] = sqlen(r[u]);
    }
    /* order spokes by squared length */
    for (int u = 1; u < 3; ++u)
        for (int v = u; v > 0 && q[ord[v - 1]] > q[ord[v]]; --v) {
            int t = ord[v];
            ord[v] = ord[v - 1];
            ord[v - 1] = t;
        }
    const double *ra = r[ord[0]], *rb = r[ord[1]], *rc = r[ord[2]];
    double qa = q[ord[0]], qb = q[ord[1]], qc = q[ord[2]];
    int b1 = edge_bin(p, qa), b2 = edge_bin(p, qb), b3 = edge_bin(p, qc);
    *idx_out = config_index(p->nb, b1, b2, b3);
    double cx = ra[1] * rb[2] - ra[2] * rb[1];
    double cy = ra[2] * rb[0] - ra[0] * rb[2];
    double cz = ra[0] * rb[1] - ra[1] * rb[0];
    double V = (cx * rc[0] + cy * rc[1]) + cz * rc[2];
    if (qa == qb || qb == qc) return 2;
    if (V * V <= 1e-18 * ((qa * qb) * qc)) return 2;
    return V > 0 ? 0 : 1;
}

/* D10 direction pixels (Sec. 3.2: each spoke direction quantised to one byte;
 * the pixelisation is not given, this is our reading): 8 octants (bit 2 for
 * x < 0, bit 1 for y < 0, bit 0 for z < 0) x 32 cells. With s = (|x|+|y|)+|z|:
 * a = |x|/s, i = min(7, floor(8a)); t = |y|/(|y|+|z|) (0 if both vanish),
 * j = min(3, floor(4t)); pixel = octant*32 + i*4 + j (a zero vector: 0). */
static int pixel_of(const double r[3]) {
    const double ax = fabs(r[0]), ay = fabs(r[1]), az = fabs(r[2]);
    const double s = (ax + ay) + az;
    if (!(s > 0.0)) return 0;
    const int oct = (r[0] < 0) * 4 + (r[1] < 0) * 2 + (r[2] < 0);
    int i = (int)floor(8.0 * (ax / s));
    if (i > 7) i = 7;
    const double yz = ay + az;
    int j = yz > 0.0 ? (int)floor(4.0 * (ay / yz)) : 0;
    if (j > 3) j = 3;
    return oct * 32 + i * 4 + j;
}

/* The unit direction of a pixel's centre: a_c = (i+0.5)/8, t_c = (j+0.5)/4,
 * v = (a_c, (1-a_c)*t_c, (1-a_c)*(1-t_c)) with the octant's signs, divided
 * by sqrt((vx*vx + vy*vy) + vz*vz). */
static void pixel_centre(int pix, double u[3]) {
    const int oct = pix >> 5, i = (pix >> 2) & 7, j = pix & 3;
    const double ac = ((double)i + 0.5) / 8.0, tc = ((double)j + 0.5) / 4.0;
    double v[3] = {ac, (1.0 - ac) * tc, (1.0 - ac) * (1.0 - tc)};
    if (oct & 4) v[0] = -v[0];
    if (oct & 2) v[1] = -v[1];
    if (oct & 1) v[2] = -v[2];
    const double len = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    for (int c = 0; c < 3; ++c) u[c] = v[c] / len;
}

/* One hub's contribution with pixel directions (Sec. 3.2 as written): the
 * spokes to s[0] < s[1] < s[2] (original indices, the paper's index order),
 * each replaced by its pixel's centre direction; V = (u1 x u2) . u3 (D6
 * operation order); degenerate iff |V| < 1e-9 (repeated pixels give V = 0
 * exactly); else pos (V > 0) or neg. The configuration: sorted spoke bins. */
static int hub_pixel(const params_t *p, const double *xyz, int64_t h, const int64_t s[3], int64_t *idx_out) {
    double r[3][3], u[3][3];
    int b[3];
    for (int k = 0; k < 3; ++k) {
        separation(p, &xyz[3 * h], &xyz[3 * s[k]], r[k]);
        b[k] = edge_bin(p, sqlen(r[k]));
        pixel_centre(pixel_of(r[k]), u[k]);
    }
    sort3i(&b[0], &b[1], &b[2]);
    *idx_out = config_index(p->nb, b[0], b[1], b[2]);
    const double cx = u[0][1] * u[1][2] - u[0][2] * u[1][1];
    const double cy = u[0][2] * u[1][0] - u[0][0] * u[1][2];
    const double cz = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    const double V = (cx * u[2][0] + cy * u[2][1]) + cz * u[2][2];
    if (fabs(V) < 1e-9) return 2;
    return V > 0 ? 0 : 1;
}

int oracle_pixel_of(const double *r) { return pixel_of(r); }

/* hub_pixel for hub h of the four points xyz4 (indices 0..3), its spokes to
 * the other three in index order: 0 pos, 1 neg, 2 degenerate, <0 error */
int oracle_hub_pixel_channel(const double *xyz4, double box, double rmin, double rmax, int nbins, int h) {
    params_t p;
    if (make_params(&p, box, rmin, rmax, nbins) != OR_OK || h < 0 || h > 3) return OR_EINVAL;
    int64_t sp[3], idx;
    int u = 0;
    for (int o = 0; o < 4; ++o)
        if (o != h) sp[u++] = o;
    return hub_pixel(&p, xyz4, h, sp, &idx);
}
void oracle_pixel_centre(int pix, double *u) { pixel_centre(pix, u); }

/* t = +-((a1*a2)*a3)*a4 of a 4-clique's weights (magnitudes ascending, the
 * sign their product's), as an integer multiple of 2^-s (scale = 2^s) */
static i128 clique_weight(const double *w, const int64_t v[4], double scale) {
    const double x[4] = {w[v[0]], w[v[1]], w[v[2]], w[v[3]]};
    return (i128)(signed_product(x, 4) * scale);
}

/* ------------------------------------------------ mu-binned triangles ---- */

/* D9 mu binning (anisotropic 3pCF, Sec. 6; our reading): a triangle with
 * vertices p0 < p1 < p2 (original indices) has normal n = sep(p0,p1) x
 * sep(p0,p2) (the D6 cross product); with s = (nx*nx + ny*ny) + nz*nz and
 * t = (nz*nz)*(nmu*nmu) its mu bin is the number of k in 1..nmu-1 with
 * t >= (k*k)*s (mu = |nz|/|n| against the z line of sight, equal bins of
 * [0, 1]); s = 0 (collinear) gives bin 0. */
static int mu_bin(const params_t *p, const double *a, const double *b, const double *c, int nmu) {
    double u[3], v[3];
    separation(p, a, b, u);
    separation(p, a, c, v);
    const double nx = u[1] * v[2] - u[2] * v[1];
    const double ny = u[2] * v[0] - u[0] * v[2];
    const double nz = u[0] * v[1] - u[1] * v[0];
    const double s = (nx * nx + ny * ny) + nz * nz;
    if (!(s > 0.0)) return 0;
    const double t = (nz * nz) * (double)(nmu * nmu);
    int m = 0;
    for (int k = 1; k < nmu; ++k)
        if (t >= (double)(k * k) * s) ++m;
    return m;
}

/* Triangles binned by sorted side bins and mu bin: counter conf*nmu + mu. */
int oracle_count_3pcf_mu(const double *xyz, int64_t n, const double *w, double box, double rmin, double rmax,
                         int nbins, int nmu, int64_t anchor_lo, int64_t anchor_hi, int nthreads, uint64_t *hist,
                         uint64_t *wsum, int *wscale, uint64_t *n_tri, int *threads_used) {
    params_t p;
    int rc = make_params(&p, box, rmin, rmax, nbins);
    if (rc == OR_OK) rc = check_points(xyz, n, box);
    if (rc != OR_OK) return rc;
    if (n >= ((int64_t)1 << 31) || !hist || !n_tri || nmu < 1 || nmu > 64) return OR_EINVAL;
    int s = 0;
    if (w) {
        if (!wsum) return OR_EINVAL;
        rc = weight_scale(w, n, &s);
        if (rc != OR_OK) return rc;
        if (wscale) *wscale = s;
    }
    if (anchor_lo < 0) anchor_lo = 0;
    if (anchor_hi > n) anchor_hi = n;
    int nt = resolve_threads(nthreads);
    if (threads_used) *threads_used = nt;
    rows_t g;
    rc = rows_for_anchors(&p, xyz, n, nt, anchor_lo, anchor_hi, &g);
    if (rc != OR_OK) return rc;
    const int64_t ncnt = binom3(nbins + 2) * nmu;
    uint64_t *th = (uint64_t *)calloc((size_t)(nt * ncnt), sizeof(uint64_t));
    i128 *tw = w ? (i128 *)calloc((size_t)(nt * ncnt), sizeof(i128)) : NULL;
    uint64_t *tn = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    if (!th || !tn || (w && !tw)) { free(th); free(tw); free(tn); rows_free(&g); return OR_ENOMEM; }
    const double scale = ldexp(1.0, s);
#pragma omp parallel num_threads(nt)
    {
        int tid = omp_get_thread_num();
        uint64_t *H = th + (int64_t)tid * ncnt;
        i128 *Wt = w ? tw + (int64_t)tid * ncnt : NULL;
        uint64_t cnt = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = anchor_lo; i < anchor_hi; ++i) {
            for (int64_t a = g.ptr[i]; a < g.ptr[i + 1]; ++a) {
                int32_t j = g.col[a];
                if (j <= i) continue;
                for (int64_t b = a + 1; b < g.ptr[i + 1]; ++b) {
                    int32_t k = g.col[b];
                    int64_t f = find(&g, j, k);
                    if (f < 0) continue;
                    /* i < j < k: the vertices in original-index order */
                    int b1 = g.bin[a], b2 = g.bin[b], b3 = g.bin[f];
                    sort3i(&b1, &b2, &b3);
                    const int64_t idx = config_index(nbins, b1, b2, b3) * nmu +
                                        mu_bin(&p, &xyz[3 * i], &xyz[3 * (int64_t)j], &xyz[3 * (int64_t)k], nmu);
                    H[idx] += 1;
                    ++cnt;
                    if (Wt) {
                        const double v[3] = {w[i], w[j], w[k]};
                        Wt[idx] += (i128)(signed_product(v, 3) * scale);
                    }
                }
            }
        }
        tn[tid] = cnt;
    }
    memset(hist, 0, sizeof(uint64_t) * (size_t)ncnt);
    *n_tri = 0;
    for (int t = 0; t < nt; ++t) {
        *n_tri += tn[t];
        for (int64_t c = 0; c < ncnt; ++c) hist[c] += th[(int64_t)t * ncnt + c];
    }
    if (w)
        for (int64_t c = 0; c < ncnt; ++c) {
            i128 acc = 0;
            for (int t = 0; t < nt; ++t) acc += tw[(int64_t)t * ncnt + c];
            put128(&wsum[2 * c], acc);
        }
    free(th);
    free(tw);
    free(tn);
    rows_free(&g);
    return OR_OK;
}

/* ------------------------------------------------ 6-edge configurations -- */

#define OR_MAX_BINS6 12

static const int k_edge[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};

/* the smallest edge-bin tuple over the 24 orderings of the four vertices */
static void canon6(const int t[6], int out[6]) {
    int first = 1;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c)
                for (int d = 0; d < 4; ++d) {
                    if (a == b || a == c || a == d || b == c || b == d || c == d) continue;
                    const int p[4] = {a, b, c, d};
                    int u[6], e = 0;
                    for (int x = 0; x < 4; ++x)
                        for (int y = x + 1; y < 4; ++y) u[e++] = t[k_edge[p[x]][p[y]]];
                    int less = first;
                    for (int k = 0; k < 6 && !first; ++k)
                        if (u[k] != out[k]) { less = u[k] < out[k]; break; }
                    if (less) memcpy(out, u, sizeof u);
                    first = 0;
                }
}

static int64_t tuple_code(int nb, const int t[6]) {
    int64_t c = 0;
    for (int k = 0; k < 6; ++k) c = c * nb + t[k];
    return c;
}

/* rank of every tuple's configuration (index nb^6 by tuple code); the
 * number of configurations in *n6 */
static int32_t *config6_table(int nb, int64_t *n6) {
    const int64_t n = (int64_t)nb * nb * nb * nb * nb * nb;
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!rank) return NULL;
    int64_t r = 0;
    /* codes in increasing order are tuples in lexicographic order */
    for (int64_t code = 0; code < n; ++code) {
        int t[6], u[6];
        int64_t v = code;
        for (int k = 5; k >= 0; --k) { t[k] = (int)(v % nb); v /= nb; }
        canon6(t, u);
        rank[code] = (tuple_code(nb, u) == code) ? (int32_t)r++ : -1;
    }
    for (int64_t code = 0; code < n; ++code) {
        if (rank[code] >= 0) continue;
        int t[6], u[6];
        int64_t v = code;
        for (int k = 5; k >= 0; --k) { t[k] = (int)(v % nb); v /= nb; }
        canon6(t, u);
        rank[code] = rank[tuple_code(nb, u)];
    }
    *n6 = r;
    return rank;
}

int64_t oracle_n_configs6(int nbins) {
    if (nbins < 1 || nbins > OR_MAX_BINS6) return -1;
    int64_t n6 = 0;
    int32_t *t = config6_table(nbins, &n6);
    if (!t) return -3;
    free(t);
    return n6;
}

/* the smallest tuple of configuration `index` */
int oracle_config6(int nbins, int64_t index, int *out) {
    if (nbins < 1 || nbins > OR_MAX_BINS6) return OR_EINVAL;
    const int64_t n = (int64_t)nbins * nbins * nbins * nbins * nbins * nbins;
    int64_t r = 0;
    for (int64_t code = 0; code < n; ++code) {
        int t[6], u[6];
        int64_t v = code;
        for (int k = 5; k >= 0; --k) { t[k] = (int)(v % nbins); v /= nbins; }
        canon6(t, u);
        if (tuple_code(nbins, u) != code) continue;
        if (r++ == index) {
            memcpy(out, t, sizeof t);
            return OR_OK;
        }
    }
    return OR_EINVAL;
}

int oracle_count_4pcf_full(const double *xyz, int64_t n, const double *w, double box, double rmin, double rmax,
                           int nbins, int64_t anchor_lo, int64_t anchor_hi, int nthreads, uint64_t *hist6,
                           uint64_t *wsum6, int *wscale, uint64_t *n_cliques, int *threads_used) {
    params_t p;
    int rc = make_params(&p, box, rmin, rmax, nbins);
    if (rc == OR_OK) rc = check_points(xyz, n, box);
    if (rc != OR_OK) return rc;
    if (n >= ((int64_t)1 << 31) || !hist6 || !n_cliques || nbins > OR_MAX_BINS6) return OR_EINVAL;
    int s = 0;
    if (w) {
        if (!wsum6) return OR_EINVAL;
        rc = weight_scale_k(w, n, 4, &s);
        if (rc != OR_OK) return rc;
        if (wscale) *wscale = s;
    }
    const double scale = ldexp(1.0, s);
    if (anchor_lo < 0) anchor_lo = 0;
    if (anchor_hi > n) anchor_hi = n;
    int64_t n6 = 0;
    int32_t *rank = config6_table(nbins, &n6);
    if (!rank) return OR_ENOMEM;
    int nt = resolve_threads(nthreads);
    if (threads_used) *threads_used = nt;
    rows_t g;
    rc = rows_for_anchors(&p, xyz, n, nt, anchor_lo, anchor_hi, &g);
    if (rc != OR_OK) { free(rank); return rc; }
    uint64_t *tH = (uint64_t *)calloc((size_t)(nt * n6), sizeof(uint64_t));
    i128 *tW = w ? (i128 *)calloc((size_t)(nt * n6), sizeof(i128)) : NULL;
    uint64_t *tn = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    if (!tH || !tn || (w && !tW)) { free(tH); free(tW); free(tn); free(rank); rows_free(&g); return OR_ENOMEM; }
#pragma omp parallel num_threads(nt)
    {
        int tid = omp_get_thread_num();
        uint64_t *H = tH + (int64_t)tid * n6;
        i128 *Wt = w ? tW + (int64_t)tid * n6 : NULL;
        uint64_t cnt = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = anchor_lo; i < anchor_hi; ++i) {
            for (int64_t a = g.ptr[i]; a < g.ptr[i + 1]; ++a) {
                int32_t j = g.col[a];
                if (j <= i) continue;
                for (int64_t b = a + 1; b < g.ptr[i + 1]; ++b) {
                    int32_t k = g.col[b];
                    int64_t fjk = find(&g, j, k);
                    if (fjk < 0) continue;
                    for (int64_t c = b + 1; c < g.ptr[i + 1]; ++c) {
                        int32_t l = g.col[c];
                        int64_t fjl = find(&g, j, l), fkl = find(&g, k, l);
                        if (fjl < 0 || fkl < 0) continue;
                        ++cnt;
                        /* vertices (i, j, k, l): edges ij, ik, il, jk, jl, kl */
                        const int t[6] = {g.bin[a], g.bin[b], g.bin[c], g.bin[fjk], g.bin[fjl], g.bin[fkl]};
                        const int32_t cfg = rank[tuple_code(nbins, t)];
                        H[cfg] += 1;
                        if (Wt) {
                            const int64_t v[4] = {i, j, k, l};
                            Wt[cfg] += clique_weight(w, v, scale);
                        }
                    }
                }
            }
        }
        tn[tid] = cnt;
    }
    memset(hist6, 0, sizeof(uint64_t) * (size_t)n6);
    *n_cliques = 0;
    for (int t = 0; t < nt; ++t) {
        *n_cliques += tn[t];
        for (int64_t c = 0; c < n6; ++c) hist6[c] += tH[(int64_t)t * n6 + c];
    }
    if (w)
        for (int64_t c = 0; c < n6; ++c) {
            i128 acc = 0;
            for (int t = 0; t < nt; ++t) acc += tW[(int64_t)t * n6 + c];
            put128(&wsum6[2 * c], acc);
        }
    free(tW);
    free(tH);
    free(tn);
    free(rank);
    rows_free(&g);
    return OR_OK;
}

/* D10 parity with direction pixels: as oracle_count_4pcf_parity, each hub
 * decided by hub_pixel. */
int oracle_count_4pcf_pixel(const double *xyz, int64_t n, double box, double rmin, double rmax, int nbins,
                            int64_t anchor_lo, int64_t anchor_hi, int nthreads, uint64_t *even, uint64_t *pos,
                            uint64_t *neg, uint64_t *n_cliques, int *threads_used) {
    params_t p;
    int rc = make_params(&p, box, rmin, rmax, nbins);
    if (rc == OR_OK) rc = check_points(xyz, n, box);
    if (rc != OR_OK) return rc;
    if (n >= ((int64_t)1 << 31) || !even || !pos || !neg || !n_cliques) return OR_EINVAL;
    if (anchor_lo < 0) anchor_lo = 0;
    if (anchor_hi > n) anchor_hi = n;
    int nt = resolve_threads(nthreads);
    if (threads_used) *threads_used = nt;
    rows_t g;
    rc = rows_for_anchors(&p, xyz, n, nt, anchor_lo, anchor_hi, &g);
    if (rc != OR_OK) return rc;
    int64_t nconf = binom3(nbins + 2);
    uint64_t *tE = (uint64_t *)calloc((size_t)(nt * nconf), sizeof(uint64_t));
    uint64_t *tP = (uint64_t *)calloc((size_t)(nt * nconf), sizeof(uint64_t));
    uint64_t *tN = (uint64_t *)calloc((size_t)(nt * nconf), sizeof(uint64_t));
    uint64_t *tn = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    if (!tE || !tP || !tN || !tn) {
        free(tE); free(tP); free(tN); free(tn); rows_free(&g);
        return OR_ENOMEM;
    }
#pragma omp parallel num_threads(nt)
    {
        int tid = omp_get_thread_num();
        uint64_t *E = tE + (int64_t)tid * nconf, *P = tP + (int64_t)tid * nconf,
                 *N = tN + (int64_t)tid * nconf;
        uint64_t cnt = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = anchor_lo; i < anchor_hi; ++i) {
            for (int64_t a = g.ptr[i]; a < g.ptr[i + 1]; ++a) {
                int32_t j = g.col[a];
                if (j <= i) continue;
                for (int64_t b = a + 1; b < g.ptr[i + 1]; ++b) {
                    int32_t k = g.col[b];
                    if (find(&g, j, k) < 0) continue;
                    for (int64_t c = b + 1; c < g.ptr[i + 1]; ++c) {
                        int32_t l = g.col[c];
                        if (find(&g, j, l) < 0 || find(&g, k, l) < 0) continue;
                        ++cnt;
                        const int64_t v[4] = {i, j, k, l};   /* ascending original indices */
                        for (int h = 0; h < 4; ++h) {
                            int64_t sp[3], idx;
                            int u = 0;
                            for (int o = 0; o < 4; ++o)
                                if (o != h) sp[u++] = v[o];
                            const int ch = hub_pixel(&p, xyz, v[h], sp, &idx);
                            E[idx] += 1;
                            if (ch == 0) P[idx] += 1;
                            if (ch == 1) N[idx] += 1;
                        }
                    }
                }
            }
        }
        tn[tid] = cnt;
    }
    memset(even, 0, sizeof(uint64_t) * (size_t)nconf);
    memset(pos, 0, sizeof(uint64_t) * (size_t)nconf);
    memset(neg, 0, sizeof(uint64_t) * (size_t)nconf);
    *n_cliques = 0;
    for (int t = 0; t < nt; ++t) {
        *n_cliques += tn[t];
        for (int64_t c = 0; c < nconf; ++c) {
            even[c] += tE[(int64_t)t * nconf + c];
            pos[c] += tP[(int64_t)t * nconf + c];
            neg[c] += tN[(int64_t)t * nconf + c];
        }
    }
    free(tE);
    free(tP);
    free(tN);
    free(tn);
    rows_free(&g);
    return OR_OK;
}

/* With weights, wsum3 (3 x 2 nconf words: even | pos | neg) receives per
 * configuration the exact sums of each hub contribution's clique weight
 * t = +-((a1*a2)*a3)*a4 (magnitudes ascending, the sign the product of the
 * weights' signs), in units of 2^-wscale. */
int oracle_count_4pcf_parity(const double *xyz, int64_t n, const double *w, double box, double rmin,
                             double rmax, int nbins, int64_t anchor_lo, int64_t anchor_hi, int nthreads,
                             uint64_t *even, uint64_t *pos, uint64_t *neg, uint64_t *wsum3, int *wscale,
                             uint64_t *n_cliques, int *threads_used) {
    params_t p;
    int rc = make_params(&p, box, rmin, rmax, nbins);
    if (rc == OR_OK) rc = check_points(xyz, n, box);
    if (rc != OR_OK) return rc;
    if (n >= ((int64_t)1 << 31) || !even || !pos || !neg || !n_cliques) return OR_EINVAL;
    int s = 0;
    if (w) {
        if (!wsum3) return OR_EINVAL;
        rc = weight_scale_k(w, n, 4, &s);
        if (rc != OR_OK) return rc;
        if (wscale) *wscale = s;
    }
    const double scale = ldexp(1.0, s);
    if (anchor_lo < 0) anchor_lo = 0;
    if (anchor_hi > n) anchor_hi = n;
    int nt = resolve_threads(nthreads);
    if (threads_used) *threads_used = nt;
    rows_t g;
    rc = rows_for_anchors(&p, xyz, n, nt, anchor_lo, anchor_hi, &g);
    if (rc != OR_OK) return rc;
    int64_t nconf = binom3(nbins + 2);
    uint64_t *tE = (uint64_t *)calloc((size_t)(nt * nconf), sizeof(uint64_t));
    uint64_t *tP = (uint64_t *)calloc((size_t)(nt * nconf), sizeof(uint64_t));
    uint64_t *tN = (uint64_t *)calloc((size_t)(nt * nconf), sizeof(uint64_t));
    i128 *tW = w ? (i128 *)calloc((size_t)(3 * nt * nconf), sizeof(i128)) : NULL;
    uint64_t *tn = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    if (!tE || !tP || !tN || !tn || (w && !tW)) {
        free(tE); free(tP); free(tN); free(tW); free(tn); rows_free(&g);
        return OR_ENOMEM;
    }
#pragma omp parallel num_threads(nt)
    {
        int tid = omp_get_thread_num();
        uint64_t *E = tE + (int64_t)tid * nconf, *P = tP + (int64_t)tid * nconf,
                 *N = tN + (int64_t)tid * nconf;
        i128 *Wt = w ? tW + 3 * (int64_t)tid * nconf : NULL;   /* even | pos | neg */
        uint64_t cnt = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = anchor_lo; i < anchor_hi; ++i) {
            for (int64_t a = g.ptr[i]; a < g.ptr[i + 1]; ++a) {
                int32_t j = g.col[a];
                if (j <= i) continue;
                for (int64_t b = a + 1; b < g.ptr[i + 1]; ++b) {
                    int32_t k = g.col[b];
                    if (find(&g, j, k) < 0) continue;
                    for (int64_t c = b + 1; c < g.ptr[i + 1]; ++c) {
                        int32_t l = g.col[c];
                        if (find(&g, j, l) < 0 || find(&g, k, l) < 0) continue;
                        ++cnt;
                        int64_t v[4] = {i, j, k, l};
                        const i128 t = Wt ? clique_weight(w, v, scale) : 0;
                        for (int h = 0; h < 4; ++h) {
                            int64_t sp[3], idx;
                            int u = 0;
                            for (int o = 0; o < 4; ++o)
                                if (o != h) sp[u++] = v[o];
                            const int ch = hub_parity(&p, xyz, v[h], sp, &idx);
                            E[idx] += 1;
                            if (ch == 0) P[idx] += 1;
                            if (ch == 1) N[idx] += 1;
                            if (Wt) {
                                Wt[idx] += t;
                                if (ch < 2) Wt[(1 + ch) * nconf + idx] += t;
                            }
                        }
                    }
                }
            }
        }
        tn[tid] = cnt;
    }
    memset(even, 0, sizeof(uint64_t) * (size_t)nconf);
    memset(pos, 0, sizeof(uint64_t) * (size_t)nconf);
    memset(neg, 0, sizeof(uint64_t) * (size_t)nconf);
    *n_cliques = 0;
    for (int t = 0; t < nt; ++t) {
        *n_cliques += tn[t];
        for (int64_t c = 0; c < nconf; ++c) {
            even[c] += tE[(int64_t)t * nconf + c];
            pos[c] += tP[(int64_t)t * nconf + c];
            neg[c] += tN[(int64_t)t * nconf + c];
        }
    }
    if (w)
        for (int64_t c = 0; c < 3 * nconf; ++c) {
            i128 acc = 0;
            for (int t = 0; t < nt; ++t) acc += tW[3 * (int64_t)t * nconf + c];
            put128(&wsum3[2 * c], acc);
        }
    free(tW);
    free(tE);
    free(tP);
    free(tN);
    free(tn);
    rows_free(&g);
    return OR_OK;
}
