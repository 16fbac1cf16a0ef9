/*
 * gsn.h - C ABI of the MI355X library for exact graph N-point counts.
 *
 * The library builds the periodic r < rmax neighbour graph of a point
 * catalogue on the GPU and counts, on that graph, triangles (3pCF) and
 * 4-cliques with their parity (4pCF), each tuple binned by its separation
 * bins into exact integer histograms (paper: graph construction Sec. 2.1,
 * hub-and-spoke enumeration Sec. 2.2, sorted-list intersection Sec. 3.1,
 * parity by signed volume Sec. 3.2 Eq. 2, CSR layout Sec. 3.5.1).
 *
 * Conventions for every function:
 *  - returns int status: GS_OK (0) or a negative GS_E* code; gs_strerror()
 *    names it and gs_last_error_detail() gives the calling thread's last
 *    message (HIP error strings included);
 *  - no function throws, aborts or exits on bad input;
 *  - pointers marked "host" are ordinary host memory; "device" pointers are
 *    HIP device memory on the context's device;
 *  - all output arrays are allocated by the caller with the stated lengths;
 *  - inputs are borrowed for the duration of the call only.
 *
 * Definitions shared by all counts (float64, round to nearest, no fused
 * multiply-add, in this order):
 *  separation a->b, per axis: d = x_b - x_a; d -= L if d > L/2; d += L if
 *    d < -L/2 (periodic box, minimum image; with GS_NONPERIODIC d = x_b - x_a);
 *  squared length q = (dx*dx + dy*dy) + dz*dz;
 *  bins: D = (rmax - rmin)/nbins, e_0 = rmin, e_k = rmin + k*D, e_nbins =
 *    rmax, t_k = e_k*e_k; a pair is an edge iff t_0 <= q < t_nbins; its bin
 *    (one byte, Sec. 2.1) is the number of k in 1..nbins-1 with q >= t_k.
 *  configuration index of sorted bins b1 <= b2 <= b3: their rank in
 *    lexicographic order among all such triples, 0 .. C(nbins+2,3)-1 (the
 *    sorted side-length configurations of Sec. 5.1).
 */
#ifndef GSN_H
#define GSN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define GS_OK 0
#define GS_EINVAL (-1)        /* bad argument or input point / parameter      */
#define GS_EOVERFLOW (-2)     /* N >= 2^32 - 1 (32-bit neighbour labels)      */
#define GS_ENOMEM (-3)        /* host allocation failed                        */
#define GS_EDEVMEM (-4)       /* device memory or budget insufficient         */
#define GS_EHIP (-5)          /* HIP runtime error (see gs_last_error_detail) */
#define GS_EAGAIN (-6)        /* submit queue full, retry later               */
#define GS_ENOTFOUND (-7)     /* unknown ticket                               */
#define GS_EUNSUPPORTED (-8)  /* valid input beyond the library's limits      */
#define GS_ENOCOORDS (-9)     /* parity count on a graph built without coords */

/* ---- graph flags (gs_graph_params.flags) ---- */
#define GS_WEIGHTED 1u         /* weights given: keep them for weighted 3pCF    */
#define GS_KEEP_COORDS 2u      /* keep label-ordered coordinates (4pCF parity)  */
#define GS_INPUT_ON_DEVICE 4u  /* xyz / weights are device pointers             */
#define GS_NONPERIODIC 8u      /* survey geometry (Sec. 5): no periodic wrap;   */
                               /* separations are plain differences x_b - x_a,  */
                               /* box is the extent of the cube holding the     */
                               /* points, and rmax may take any value > rmin     */

typedef struct gs_ctx gs_ctx;      /* device, stream, budget, tuning, scratch  */
typedef struct gs_graph gs_graph;  /* forward CSR + labels (+ coords, weights) */

typedef struct {
    double box;     /* periodic box side L > 0; points in [0, L)^3              */
    double rmin;    /* 0 <= rmin < rmax                                          */
    double rmax;    /* rmax < L/2 (periodic; any finite value with GS_NONPERIODIC) */
    int32_t nbins;  /* 1 .. 255                                                    */
    uint32_t flags; /* GS_WEIGHTED | GS_KEEP_COORDS | GS_INPUT_ON_DEVICE |
                       GS_NONPERIODIC                                              */
} gs_graph_params;

/* Count only tuples whose smallest ORIGINAL point index lies in [lo, hi).
 * The restriction does not depend on how the library labels points, so
 * disjoint ranges partition any count exactly. */
typedef struct {
    uint64_t lo, hi;
} gs_anchor_range;

typedef struct {
    int64_t n;               /* points                                            */
    uint64_t n_edges;        /* undirected edges (= forward CSR entries)          */
    uint64_t max_deg;        /* largest forward degree                             */
    uint64_t device_bytes;   /* device memory held by the graph                   */
    int32_t n_windows;       /* 1 = resident; > 1 = host-tiled (out of core)       */
    int32_t nbins;
    uint64_t pair_hist[255]; /* undirected edges per bin (the pair counts)         */
    uint64_t sum_sq_degree;  /* sum over points of (neighbour count)^2             */
} gs_graph_stats;

typedef struct {
    double build_ms;         /* last gs_build_graph, device time                  */
    double count_ms;         /* last count call, device time of its launches      */
    double kernel_ms;        /* last count call: main counting kernel(s) only      */
    uint64_t kernel_launches;/* launches of the main counting kernel in that call */
    uint64_t alg_bytes;      /* 2.5 B x sum_sq_degree of the counted graph(s), the
                                bytes a merge walk reads; 0 until gs_graph_info
                                has computed the degree statistics               */
    uint64_t probes;         /* last triangle count: candidates its hash probes
                                tested (spoke-row entries up to the hub row's
                                largest label)                                    */
    int32_t table_log2;      /* last triangle count's schedule: hub hash table of
                                2^table_log2 slots,                               */
    int32_t block;           /* threads per work group,                           */
    int32_t group;           /* hubs counted together (at most),                  */
    int32_t hash_load;       /* load bound (5: 1/2, 7: 0.7); all 0 before the first
                                triangle count                                    */
} gs_timings;

/* Create a context on HIP device `device`. hbm_budget_bytes = 0 means 90% of
 * the device memory free at creation; a smaller budget forces host-tiled
 * (out-of-core) graphs. hip_stream (hipStream_t, nullable) is borrowed: all
 * work of the context runs on it; NULL makes the context create its own. */
int gs_create(gs_ctx **out, int device, uint64_t hbm_budget_bytes, void *hip_stream);
int gs_destroy(gs_ctx *ctx);

/* Build the r < rmax graph of n points (Sec. 2.1; CSR of Sec. 3.5.1):
 *  xyz: n x 3 float64, AoS (x0,y0,z0,x1,...), host or device (flag);
 *  weights: nullable, n float64, finite and nonzero, of either sign (the
 *    signed, normalised data-minus-random weights of Sec. 2.1; required iff
 *    GS_WEIGHTED);
 *  Points are relabelled in cell order; only forward edges (label j > i) are
 *  stored: row_ptr u64[n+1], col u32[E], bin u8[E], rows strictly increasing.
 *  Errors: GS_EINVAL (NaN, coordinate outside [0, box), bad params, weights
 *  missing / zero / not finite),
 *  GS_EOVERFLOW, GS_EDEVMEM, GS_EHIP. On error *out is NULL. */
int gs_build_graph(gs_ctx *ctx, const double *xyz, int64_t n, const double *weights,
                   const gs_graph_params *p, gs_graph **out);
/* Size, degree and pair statistics of a graph. The pair histogram and the
 * squared-degree sum are computed on the first call (one pass over the CSR)
 * and cached. */
int gs_graph_info(const gs_graph *g, gs_graph_stats *out);
/* Host copies of the forward CSR in label order and the label -> original
 * index permutation: row_ptr u64[n+1], col u32[n_edges], bin u8[n_edges],
 * perm u32[n]. Any pointer may be NULL to skip it. */
int gs_graph_export(const gs_graph *g, uint64_t *row_ptr, uint32_t *col, uint8_t *bin,
                    uint32_t *perm);
int gs_graph_free(gs_graph *g);

/* Binned triangle counts (Sec. 2.2 hub-and-spoke enumeration, Sec. 3.1
 * intersection): every triangle counts once into the configuration of its
 * sorted side bins.
 *  hist: host u64[C(nbins+2,3)];
 *  wsum128: nullable, host u64[2*C(nbins+2,3)], (lo, hi) words of the exact
 *    signed 128-bit (two's complement) sum per configuration of
 *    t = +-(a1*a2)*a3, the triangle's weight magnitudes in ascending order
 *    signed by the product of the weights' signs, in units of 2^-wscale
 *    (graph must be weighted);
 *  whist: nullable, host double[C(nbins+2,3)]: those sums rounded once;
 *  wscale: nullable, out: s = 52 - floor(log2((m*m)*m)), m the smallest
 *    weight magnitude. Every term t*2^s is an integer; GS_EINVAL if the
 *    largest would reach 2^87 or the products leave the normal float64
 *    range;
 *  n_triangles: host out, counted separately from the bins;
 *  anchors: nullable (see gs_anchor_range). */
int gs_count_3pcf(gs_ctx *ctx, const gs_graph *g, uint64_t *hist, uint64_t *wsum128,
                  double *whist, int32_t *wscale, uint64_t *n_triangles,
                  const gs_anchor_range *anchors);

/* Parity-decomposed 4-clique counts (Sec. 3.2, Eq. 2 and the degenerate
 * rule): each 4-clique contributes once per hub (each of its 4 vertices):
 * spokes ordered by squared length qa <= qb <= qc; even[idx] += 1;
 * c = ra x rb, V = (cx*rcx + cy*rcy) + cz*rcz; degenerate iff qa == qb or
 * qb == qc or V*V <= 1e-18*((qa*qb)*qc); else pos[idx] (V > 0) or neg[idx]
 * (V < 0) += 1. Odd channel = pos - neg. Each array host u64[C(nbins+2,3)].
 * Needs a graph built with GS_KEEP_COORDS (else GS_ENOCOORDS). */
int gs_count_4pcf_parity(gs_ctx *ctx, const gs_graph *g, uint64_t *even, uint64_t *pos,
                         uint64_t *neg, uint64_t *n_cliques, const gs_anchor_range *anchors);

/* The parity count of gs_count_4pcf_parity, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): its counters, clique total, hub queues
 * and thresholds live in a fixed 64 KiB array of device memory that the
 * library holds per device until the process ends (its address is taken at
 * gs_create), so the call allocates nothing; results and errors are those of
 * gs_count_4pcf_parity. Limit: GS_EUNSUPPORTED when the count needs more
 * than 64 KiB of scratch (more than 23 bins). Every call on a device shares
 * that device's array: calls that overlap on one device (other contexts or
 * threads) race and must be serialised by the caller. The array is cleared
 * at the start of each call. */
int gs_count_4pcf_parity_noalloc(gs_ctx *ctx, const gs_graph *g, uint64_t *even, uint64_t *pos,
                                 uint64_t *neg, uint64_t *n_cliques, const gs_anchor_range *anchors);

/* Weighted parity counts (Sec. 3.2 with the signed weights of Sec. 2.1):
 * the counts of gs_count_4pcf_parity, and per configuration the exact sums
 * of each hub contribution's clique weight t = +-((a1*a2)*a3)*a4 (the four
 * weight magnitudes in ascending order, signed by the product of the signs):
 *  wsum128: host u64[3*2*C(nbins+2,3)]: blocks even | pos | neg, each
 *    configuration's signed 128-bit sum as (lo, hi) words, units 2^-wscale;
 *  wscale: nullable, out: s = 52 - floor(log2(((m*m)*m)*m)), m the smallest
 *    weight magnitude (GS_EINVAL if a term would reach 2^87).
 * Needs a weighted graph built with GS_KEEP_COORDS. */
int gs_count_4pcf_parity_weighted(gs_ctx *ctx, const gs_graph *g, uint64_t *even, uint64_t *pos,
                                  uint64_t *neg, uint64_t *wsum128, int32_t *wscale, uint64_t *n_cliques,
                                  const gs_anchor_range *anchors);

/* Parity counts from direction pixels (Sec. 3.2 as the paper computes
 * them): each spoke's direction is quantised to one of 256 pixels and
 * replaced by the pixel's centre direction, the spokes are taken in
 * original-index order (j1 < j2 < j3), V = (u1 x u2) . u3 in the operation
 * order above, and a hub is degenerate iff |V| < 1e-9 (repeated pixels give
 * V = 0 exactly); even / pos / neg as gs_count_4pcf_parity. Pixels: octant
 * (bit 2: x < 0, bit 1: y < 0, bit 0: z < 0) * 32 + i*4 + j with s =
 * (|x|+|y|)+|z|, i = min(7, floor(8 |x|/s)), j = min(3, floor(4 |y|/(|y|+|z|)))
 * (0 when |y|+|z| = 0), the zero vector pixel 0; centre of (o, i, j): the
 * direction of (a, (1-a) t, (1-a)(1-t)) with the octant's signs, a =
 * (i+0.5)/8, t = (j+0.5)/4, divided by sqrt((x*x + y*y) + z*z). Needs
 * GS_KEEP_COORDS (pixels are taken from the separations in the kernel). */
int gs_count_4pcf_pixel(gs_ctx *ctx, const gs_graph *g, uint64_t *even, uint64_t *pos, uint64_t *neg,
                        uint64_t *n_cliques, const gs_anchor_range *anchors);

/* Full 6-edge 4-clique counts (Sec. 3.3 and Sec. 5.3, the four-point
 * configurations): every 4-clique counts once into the configuration of its
 * six edge bins up to relabelling of its four vertices. A vertex order
 * (p0,p1,p2,p3) gives the bin tuple of edges (p0p1, p0p2, p0p3, p1p2, p1p3,
 * p2p3); the configuration is the class of tuples the 24 orders give,
 * represented by its lexicographically smallest tuple, and configurations
 * are numbered in the lexicographic order of those tuples (276 at 4 bins).
 *  hist6: host u64[n6] (gs_n_configs6);
 *  wsum128: nullable, host u64[2*n6]: exact signed 128-bit sums of the clique
 *    weights t = +-((a1*a2)*a3)*a4 (as gs_count_4pcf_parity_weighted);
 *  wscale: nullable, out (as gs_count_4pcf_parity_weighted);
 *  n_cliques: host out; anchors: nullable.
 * nbins 1..12 (GS_EUNSUPPORTED above). Needs GS_KEEP_COORDS (the three
 * separations among a hub's spokes are recomputed from the coordinates with
 * the bin rule of the graph, which gives the graph's own bins). */
int gs_count_4pcf_full(gs_ctx *ctx, const gs_graph *g, uint64_t *hist6, uint64_t *wsum128, int32_t *wscale,
                       uint64_t *n_cliques, const gs_anchor_range *anchors);
/* Number of 6-edge configurations at nbins (1..12): (k^6 + 9k^4 + 14k^2)/24. */
int gs_n_configs6(int32_t nbins, uint32_t *n6);
/* The configuration of every 6-edge bin tuple: rank: host u32[nbins^6],
 * indexed by the tuple's code sum_e bin_e * nbins^(5-e) (edges in the order
 * above). */
int gs_config6_table(int32_t nbins, uint32_t *rank);

/* Equilateral triangle counts (the restricted 3pCF kernel of Sec. 3.5):
 * triangles whose three sides lie in one bin b, per b; equal to the (b,b,b)
 * configurations of gs_count_3pcf, found without probing candidates whose
 * spoke-row bin differs from the spoke's.
 *  hist: host u64[nbins]; wsum128: nullable, host u64[2*nbins], the exact
 *    signed weighted sums (as gs_count_3pcf); wscale: nullable, out;
 *  n_triangles: host out (equilateral triangles); anchors: nullable.
 * Device-resident graphs (GS_EUNSUPPORTED for host-tiled ones). */
int gs_count_3pcf_equilateral(gs_ctx *ctx, const gs_graph *g, uint64_t *hist, uint64_t *wsum128,
                              int32_t *wscale, uint64_t *n_triangles, const gs_anchor_range *anchors);

/* mu-binned triangle counts (anisotropic 3pCF, Sec. 6): each triangle counts
 * into configuration conf * nmu + m, conf the rank of its sorted side bins
 * and m the bin of mu = |nz|/|n| of its plane's normal n against the line of
 * sight z, in nmu equal bins [k/nmu, (k+1)/nmu) of [0, 1]. With the vertices
 * in original-index order p0 < p1 < p2, n = sep(p0,p1) x sep(p0,p2) (cross
 * product as in gs_count_4pcf_parity), s = (nx*nx + ny*ny) + nz*nz, and m is
 * the number of k in 1..nmu-1 with (nz*nz)*(nmu*nmu) >= (k*k)*s; a collinear
 * triangle (s = 0) has m = 0.
 *  nmu: 1..64; hist: host u64[C(nbins+2,3)*nmu]; wsum128, wscale: nullable
 *    (as gs_count_3pcf, per counter); n_triangles: host out.
 * Needs GS_KEEP_COORDS; device-resident graphs. */
int gs_count_3pcf_mu(gs_ctx *ctx, const gs_graph *g, int32_t nmu, uint64_t *hist, uint64_t *wsum128,
                     int32_t *wscale, uint64_t *n_triangles, const gs_anchor_range *anchors);

/* Pair counts per bin and exact weighted pair sums (the internal 2pCF that
 * the connected 4pCF of Sec. 3.3 subtracts): every edge once.
 *  pairs: host u64[nbins];
 *  wsum128: nullable, host u64[2*nbins]: exact signed 128-bit sums of
 *    w_i*w_j, units 2^-wscale, s = 52 - floor(log2(m*m));
 *  anchors: nullable: pairs whose smaller original index lies in [lo, hi).
 * Works on resident and host-tiled graphs. */
int gs_pair_sums(gs_ctx *ctx, const gs_graph *g, uint64_t *pairs, uint64_t *wsum128, int32_t *wscale,
                 const gs_anchor_range *anchors);

/* Binned triangle counts of several resident graphs (same nbins) in ONE
 * persistent launch: hubs of all graphs form one queue, so small and large
 * catalogues balance across the device (paper Sec. 3.5.2 hub parallelism,
 * applied to many catalogues).
 *  graphs: host array of ng graph handles (unweighted counts);
 *  hists: host u64[ng * C(nbins+2,3)], graph g's histogram at g*C(nbins+2,3);
 *  n_triangles: host u64[ng].
 * Results are identical to ng separate gs_count_3pcf calls.
 * Errors: GS_EINVAL (differing nbins, null), GS_EUNSUPPORTED (host-tiled). */
int gs_count_3pcf_batch(gs_ctx *ctx, const gs_graph *const *graphs, int ng, uint64_t *hists,
                        uint64_t *n_triangles);

/* ---- autotuning of the triangle-count schedule ----
 * The count's schedule: threads per work group, candidates per step (the
 * lanes that walk one spoke row together, Sec. 3.5.2), hubs per group (hubs
 * counted together, their rows contiguous in the CSR of Sec. 3.5.1), step
 * table entries, how a hit finds its counter, and the hub hash table's load
 * bound. gs_tune_3pcf times
 * candidate schedules on a sample of g's hubs (counts discarded), starting
 * from the built-in choice and changing one parameter at a time while that
 * helps; the fastest is kept in the context for graphs of g's shape (bin
 * count, weighting, label width, and the scale of the largest and the mean
 * forward degree), and every later count of such a graph in this context
 * (gs_count_3pcf, gs_count_3pcf_batch, and requests served after the
 * context's first gs_submit, which takes the schedules tuned before it) uses
 * it. Not thread-safe against concurrent counts on the same context.
 *  g: a device-resident graph (GS_EUNSUPPORTED for host-tiled graphs);
 *  flags: GS_WEIGHTED tunes weighted counts (g must be weighted);
 *  out: nullable, host: the chosen schedule. Results never depend on it. */
typedef struct {
    int32_t block;       /* threads per work group (256, 512, or 768 weighted)   */
    int32_t step_log2;   /* candidates per step = 2^step_log2 (0..6)            */
    int32_t group;       /* hubs per group (1..4)                                */
    int32_t table;       /* step table entries per fill                          */
    int32_t counters;    /* 0: rank arithmetic, 1: table of counter addresses,   */
                         /* 2: per-(x,y,z) counters folded at flush              */
    int32_t hash_load;   /* hub hash table load bound: 5 (1/2) or 7 (0.7)         */
    int32_t truncate;    /* 1: spoke rows cut at the hub row's largest label     */
    int32_t trials;      /* schedules timed                                      */
    double sample_ms;    /* chosen schedule on the sample (kernel time)          */
    double default_ms;   /* built-in schedule on the same sample                 */
    double sample_frac;  /* fraction of hubs in the sample                       */
} gs_plan3;

int gs_tune_3pcf(gs_ctx *ctx, const gs_graph *g, uint32_t flags, gs_plan3 *out);

/* ---- serving: continuous batching of count requests ----
 * gs_submit copies the catalogue (and its weights) and returns a ticket at
 * once. A scheduler thread of the context admits queued requests while
 * device memory (the context budget, checked against each graph's exact
 * footprint once its edge count is known) and batch slots allow, builds
 * their graphs while the previous count step runs, and counts every graph
 * built so far in the next step: plain triangle counts of one bin count in
 * one batched launch, each weighted triangle count and each parity count as
 * a count of its own on the same stream; requests arriving meanwhile join
 * the next step. Results are identical to a lone gs_build_graph followed by
 * gs_count_3pcf (GS_3PCF) or gs_count_4pcf_parity (GS_4PCF_PARITY).
 * submit / poll / cancel are thread-safe. */
#define GS_PENDING 1      /* queued, building or counting                       */
#define GS_DONE 0         /* result available (returned once, then forgotten)   */
#define GS_FAILED 2       /* request failed: error holds the status code        */
#define GS_CANCELLED 3

/* request kinds (gs_request.kind) */
#define GS_3PCF 0          /* binned triangles (Sec. 2.2), optionally weighted   */
#define GS_4PCF_PARITY 1   /* parity-decomposed 4-cliques (Sec. 3.2)             */

typedef struct {
    const double *xyz;      /* host n x 3 float64, copied by gs_submit          */
    int64_t n;
    const double *weights;  /* host n float64, finite, nonzero; copied; non-NULL iff
                               p.flags has GS_WEIGHTED (GS_3PCF only)            */
    gs_graph_params p;      /* flags: 0 or GS_WEIGHTED (host input; parity
                               requests keep coordinates by themselves)         */
    int32_t kind;           /* GS_3PCF or GS_4PCF_PARITY                         */
    int32_t reserved;
} gs_request;

/* Outputs of a finished request; the caller sets the array pointers (any may
 * be NULL to skip) before gs_poll, which fills them on GS_DONE:
 *  hist: u64[C(nbins+2,3)]: triangle counts (GS_3PCF) or the even channel,
 *    every hub contribution (GS_4PCF_PARITY);
 *  pos, neg: u64[C(nbins+2,3)] each (GS_4PCF_PARITY), as gs_count_4pcf_parity;
 *  wsum128: u64[2*C(nbins+2,3)], whist: double[C(nbins+2,3)] and wscale
 *    (weighted GS_3PCF), as gs_count_3pcf. */
typedef struct {
    int32_t status;         /* GS_PENDING / GS_DONE / GS_FAILED / GS_CANCELLED   */
    int32_t error;          /* status code when GS_FAILED                        */
    uint64_t n_tuples;      /* triangles (GS_3PCF) or 4-cliques (GS_4PCF_PARITY) */
    uint64_t *hist;
    uint64_t *pos, *neg;
    uint64_t *wsum128;
    double *whist;
    int32_t wscale;
    uint32_t step_size;     /* requests counted in the step that held this one   */
    double t_queue_s;       /* submit -> graph build started                     */
    double t_build_s;       /* graph build                                       */
    double t_count_s;       /* the count step that held this request             */
    double t_total_s;       /* submit -> result ready                            */
} gs_result;

/* Errors: GS_EINVAL (bad request), GS_EAGAIN (queue full), GS_EUNSUPPORTED. */
int gs_submit(gs_ctx *ctx, const gs_request *req, uint64_t *ticket);
/* status GS_PENDING leaves *out's arrays untouched; DONE / FAILED / CANCELLED
 * retire the ticket. Error: GS_ENOTFOUND for an unknown or retired ticket. */
int gs_poll(gs_ctx *ctx, uint64_t ticket, gs_result *out);
/* Cancel a request not yet finished: it is dropped if still queued, its
 * result discarded if already building or counting. GS_ENOTFOUND if unknown. */
int gs_cancel(gs_ctx *ctx, uint64_t ticket);

/* ---- estimators (Sec. 2.1 signed weights, Sec. 3.3, Sec. 3.4) ----
 * A data catalogue and a random catalogue in the same periodic box give the
 * paper's compute_3pcf / compute_4pcf estimates. Data weights are divided by
 * their sum (they then sum to +1) and random weights by minus theirs (-1),
 * each sum taken left to right in index order; the combined catalogue (data,
 * then randoms) with these signed weights is counted once, and its exact
 * per-configuration weighted sum is the numerator (NN, NNN, NNNN: the
 * data-minus-random combination of Landy-Szalay / Szapudi-Szalay). The
 * denominator (RR, RRR, RRRR) is the same sum over the randoms alone with
 * their weights divided by their sum. Each exact sum is rounded once to
 * float64 and every estimate is the quotient (IEEE: 0/0 = NaN). Catalogues
 * are host arrays; the calls build and free their own graphs (two per call).
 * p: box, rmin, rmax and nbins of the graphs; of the flags only
 * GS_NONPERIODIC is used. */
typedef struct {
    const double *xyz;      /* host n x 3 float64 (AoS), in [0, box)        */
    int64_t n;
    const double *weights;  /* host n float64 (nullable: all 1); any sign  */
} gs_catalogue;

/* compute_3pcf: zeta[c] = NNN[c] / RRR[c] per sorted-side configuration.
 * Caller-set outputs (host, C(nbins+2,3) each; all but zeta nullable):
 * zeta, nnn and rrr (the rounded sums), nnn128 and rrr128 (2 words per
 * configuration, exact, units 2^-nnn_scale / 2^-rrr_scale). */
typedef struct {
    double *zeta, *nnn, *rrr;
    uint64_t *nnn128, *rrr128;
    int32_t nnn_scale, rrr_scale;   /* out */
} gs_zeta3;
int gs_compute_3pcf(gs_ctx *ctx, const gs_catalogue *data, const gs_catalogue *randoms,
                    const gs_graph_params *p, gs_zeta3 *out);

/* compute_4pcf with its parity decomposition and connected part. Caller-set
 * outputs, every one nullable (host float64):
 *  per hub configuration (C(nbins+2,3)): zeta_even = NNNN_even / RRRR_even,
 *    zeta_odd = (NNNN_pos - NNNN_neg) / RRRR_even (the difference taken
 *    exactly), nnnn_even, nnnn_odd, rrrr_even; zeta_even_disc, the
 *    disconnected part of the even channel, and zeta_even_conn =
 *    zeta_even - zeta_even_disc (the odd channel is connected as it is);
 *  per 6-edge configuration (gs_n_configs6): zeta6 = NNNN6 / RRRR6, its
 *    disconnected part zeta6_disc = xi(b01) xi(b23) + xi(b02) xi(b13) +
 *    xi(b03) xi(b12) (Eq. 4 on the configuration's smallest edge tuple,
 *    added in this order) and zeta6_conn = zeta6 - zeta6_disc (Eq. 5);
 *  xi (nbins): the internal 2pCF NN / RR on the same graph and bins.
 * The even channel's disconnected part averages Eq. 4 over the 6-edge
 * configurations whose hub contributions fall in the configuration: for
 * each 6-edge configuration c (ascending) and each of its four vertices, the
 * vertex's sorted edge bins give a hub configuration T, which gains
 * RRRR6(c) * disc(c); the total for T is divided by RRRR_even(T).
 * Any 6-edge or connected output needs nbins <= 12 (GS_EUNSUPPORTED). */
typedef struct {
    double *zeta_even, *zeta_odd, *nnnn_even, *nnnn_odd, *rrrr_even;
    double *zeta_even_disc, *zeta_even_conn;
    double *zeta6, *zeta6_disc, *zeta6_conn;
    double *xi;
} gs_zeta4;
int gs_compute_4pcf(gs_ctx *ctx, const gs_catalogue *data, const gs_catalogue *randoms,
                    const gs_graph_params *p, gs_zeta4 *out);

/* ---- attainable ceilings (measurement only; no counting) ----
 * Rates the device sustains for the work the counting kernels are made of,
 * timed with HIP events on the context's stream, so that each kernel can be
 * reported against the ceiling that binds it.
 * gs_ceiling_copy: a device-to-device copy of `bytes` (>= 1 MiB; the call
 *   allocates 2 x bytes of device memory for it): *gbs = read + written
 *   bytes per second / 1e9, best of five.
 * gs_ceiling_probe: the per-candidate work of the triangle count -- a
 *   coalesced 4-byte label and 1-byte bin load from an L2-resident array,
 *   the 24-bit hash, a linear-probe chain in an LDS table of 2^table_log2
 *   slots holding keys_in_table labels (<= 0.7 of the slots), and for the
 *   hit_rate fraction of candidates that hit, the counter address from the
 *   nbins^3 configuration table and one LDS atomic (plus, weighted != 0,
 *   the weight gather, the exact triangle integer and two u64 LDS atomics).
 *   probe == 0 skips the hash (every candidate a hit): the LDS-atomic
 *   histogram ceiling at this bin count. block: 256 or 512 threads, or 768
 *   (weighted only, as weighted counts of long rows run).
 *   *per_s = candidates per second. nbins 1..24. */
int gs_ceiling_copy(gs_ctx *ctx, uint64_t bytes, double *gbs);
int gs_ceiling_probe(gs_ctx *ctx, int32_t nbins, uint32_t table_log2, uint32_t keys_in_table,
                     double hit_rate, int32_t weighted, int32_t probe, int32_t block, double *per_s);

/* Device timings of the context's last build / count call. */
int gs_get_timings(const gs_ctx *ctx, gs_timings *out);

const char *gs_strerror(int code);
const char *gs_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* GSN_H */
