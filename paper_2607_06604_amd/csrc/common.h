// common.h - internal types and helpers of the HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gsn.h"

namespace gsn {

// ------------------------------------------------------------ errors ------

struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void set_detail(const std::string &msg);

#define GS_HIP(expr)                                                                 \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            ::gsn::fail(GS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Run body, turning library errors into status codes at the C boundary.
template <class F>
int guarded(F &&body) {
    try {
        body();
        set_detail("");
        return GS_OK;
    } catch (const Error &e) {
        set_detail(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_detail("host allocation failed");
        return GS_ENOMEM;
    } catch (...) {
        set_detail("unexpected C++ exception");
        return GS_EHIP;
    }
}

// ------------------------------------------------------- device buffers ---

// A context's cache of device blocks. Graph buffers and build temporaries
// come from it and go back to it when released, so that a build does not
// pay for hipMalloc and a graph release does not pay for hipFree (which
// waits for the whole device). Sizes are rounded up to classes (powers of two
// up to 1 MiB, then steps of an eighth of the power of two below), so a
// block serves later requests of nearly the same size. A block is handed
// back only once no kernel on another stream can still use it: graph blocks
// after the device has drained, build temporaries only to the building
// context, whose later takes are ordered after them on its one stream.
struct DevPool {
    int device = 0;
    uint64_t cap = 0;   // bytes the cache may hold
    std::mutex mu;
    std::multimap<size_t, void *> blocks;  // by block size
    uint64_t held = 0;
    static size_t round_size(size_t n);
    void *take(size_t n, size_t &got);
    void give(void *p, size_t got);
    void trim();        // free every cached block (waits for the device)
    ~DevPool();
};

// Owning device allocation, from hipMalloc or from a DevPool.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;   // size asked for
    size_t cap = 0;     // size of the block held
    std::shared_ptr<DevPool> pool;
    DevBuf() = default;
    explicit DevBuf(size_t n) { alloc(n); }
    DevBuf(size_t n, const std::shared_ptr<DevPool> &from) { alloc(n, from); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), cap(o.cap), pool(std::move(o.pool)) {
        o.p = nullptr; o.bytes = o.cap = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            reset();
            p = o.p; bytes = o.bytes; cap = o.cap; pool = std::move(o.pool);
            o.p = nullptr; o.bytes = o.cap = 0;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    void alloc(size_t n);
    void alloc(size_t n, const std::shared_ptr<DevPool> &from);
    void reset() {
        if (p) {
            if (pool) pool->give(p, cap);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = cap = 0;
        pool.reset();
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Owning pinned host allocation.
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() { reset(); }
    void alloc(size_t n);
    void reset() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ------------------------------------------------------- core objects -----

struct Timings {
    double build_ms = 0, count_ms = 0, kernel_ms = 0;
    uint64_t kernel_launches = 0, alg_bytes = 0, probes = 0;
    int32_t table_log2 = 0, block = 0, group = 0, hash_load = 0;   // last triangle count's plan
};

struct Server;

// Result staging shared by the count entry points of one context.
// A triangle-count schedule (-1: the built-in choice): work-group size,
// entries per step (log2), hubs per group, step table entries, counter mode,
// hash table load bound, spoke-row truncation.
struct Tune3 {
    int block = -1, glog = -1, group = -1, tmax = -1, mode = -1;
    int hload = 0;   // hash table load bound: 5 (1/2), 7 (0.7), 0 built-in
    int trunc = -1;  // spoke rows cut at the hub row's largest label: 0, 1, -1 built-in
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t copy_stream = nullptr;  // host<->device window copies (own)
    bool own_stream = false;
    uint64_t budget = 0;        // device bytes the context may hold in graphs + scratch
    int n_cu = 0;
    int max_lds = 0;
    Timings t;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    DevBuf scratch;             // grown on demand, reused across calls
    std::shared_ptr<DevPool> pool;  // graph buffers and build temporaries
    void *pinned = nullptr;     // small pinned host staging
    size_t pinned_bytes = 0;
    Server *server = nullptr;   // continuous-batching scheduler (gs_submit)
    std::vector<std::pair<uint64_t, Tune3>> tuned;  // autotuned schedules by graph shape
    std::map<int, DevBuf> cfg6;  // 6-edge configuration tables by bin count
    void *scratch_get(size_t bytes);
    void *pinned_get(size_t bytes);
    void use() const;
};

// Squared bin thresholds t_0..t_nb (host-computed from the definition).
struct Bins {
    int nb = 0;
    double t[256];
};

// Entries of readable slack after every device edge array (col, bin and
// their window buffers): the count kernel's lanes past the end of a row may
// load them (the values are never used), so it needs no per-lane clamp.
constexpr uint64_t kRowSlack = 64;

struct Graph {
    int device = 0;
    int64_t n = 0;
    uint64_t n_edges = 0;     // forward entries
    uint32_t max_deg = 0;     // largest forward degree
    double box = 0, rmin = 0, rmax = 0;
    bool periodic = true;     // false: GS_NONPERIODIC (plain differences, no wrap)
    int nbins = 0;
    uint32_t flags = 0;
    int wscale = 0;           // exact-sum scale of weighted triangles (kNoScale: none)
    double wmin = 0, wmax = 0;  // smallest and largest weight magnitude
    bool wneg = false;          // some weight is negative
    Bins bins;
    uint64_t pair_hist[255] = {};
    uint64_t sum_sq_deg = 0;  // sum over points of (full degree)^2
    bool stats_ready = false; // pair_hist and sum_sq_deg computed (graph_stats)
    uint64_t device_bytes = 0;
    int n_windows = 1;
    // host-tiled graphs (n_windows > 1): the forward CSR lives in pinned host
    // memory, split into row-aligned windows [win[w], win[w+1]) of labels
    // whose entries start at win_edge[w]
    std::vector<uint64_t> win, win_edge;
    HostBuf hcol;     // u32[E]
    HostBuf hbin;     // u8[E]
    // device, label order
    DevBuf row_ptr;   // u64[n+1]
    DevBuf col;       // u32[E]
    DevBuf bin;       // u8[E]
    DevBuf perm;      // u32[n]: label -> original index
    DevBuf coords;    // f64[3n] SoA x|y|z (GS_KEEP_COORDS)
    DevBuf weights;   // f64[n] (GS_WEIGHTED)
};

// State carried between the two build phases (temporaries of the degree pass).
struct BuildJob {
    DevBuf cstart;       // u64[ncell+1]
    DevBuf chpref;       // u64[ncell+1]: chunks (build work groups) before each cell
    DevBuf gcell;        // u32[grid]: cell of each chunk
    uint64_t grid = 0;   // build work groups (an upper bound on the chunks)
    uint32_t chunk = 64; // labels per build work group (at most)
    DevBuf cellL;        // u32[n]: cell of each label
    DevBuf thr;          // f64[256] squared thresholds
    DevBuf tmp_coords;   // f64[3n] when the graph does not keep coordinates
    double *C = nullptr; // label-ordered SoA coordinates
    int nc = 1;
    bool empty = false;
    uint64_t E = 0;      // forward entries, known after build_begin
    double begin_ms = 0;
};

Bins make_bins(double rmin, double rmax, int nb);

// Exact sums of products of k weights (Sec. 2.1 signed weights): every
// product +-((a1*a2)*...)*ak of magnitudes in ascending order, times 2^s, is
// an integer when s = 52 - floor(log2(wmin^k)) (the smallest possible product
// lies in [2^52, 2^53) units of 2^-s). weight_scale_ok gives s when the
// largest product then stays below 2^87 (terms below 2^63 are summed in LDS,
// wider ones straight into the 128-bit sums); weight_scale throws GS_EINVAL
// otherwise (or when the products leave the normal float64 range).
constexpr int kNoScale = -100000;
bool weight_scale_ok(const Graph &g, int k, int *s, int *why = nullptr);
int weight_scale(const Graph &g, int k);
// Whether a product of k weights may reach 2^63 at that scale (then some
// terms need the 128-bit path).
bool wide_terms(const Graph &g, int k);
// An exact signed 128-bit sum (lo, hi words, two's complement) in units of
// 2^-scale, rounded once to float64.
double sum128_to_double(const uint64_t *w, int scale);
inline int64_t n_configs(int nb) { return (int64_t)(nb + 2) * (nb + 1) * nb / 6; }

// ------------------------------------------------------- device helpers ---

// Periodic minimum-image component of x_b - x_a.
__device__ __forceinline__ double min_image(double xa, double xb, double L, double half) {
    double d = __dsub_rn(xb, xa);
    if (d > half) d = __dsub_rn(d, L);
    else if (d < -half) d = __dadd_rn(d, L);
    return d;
}

// (dx*dx + dy*dy) + dz*dz, no contraction.
__device__ __forceinline__ double sq_len(double dx, double dy, double dz) {
    return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// Number of k in 1..nb-1 with q >= t[k] (t non-decreasing): upper bound.
__device__ __forceinline__ int bin_of(const double *t, int nb, double q) {
    int lo = 1, hi = nb;  // search in t[1..nb-1]
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (q >= t[mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo - 1;
}

// Lexicographic rank tables: idx(b1<=b2<=b3) = A[b1] + B[b2] + b3.
__host__ __device__ inline int64_t c2(int64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }
__host__ __device__ inline int64_t c3(int64_t n) { return n < 3 ? 0 : n * (n - 1) * (n - 2) / 6; }
__host__ __device__ inline int rank_a(int nb, int b1) {
    return (int)(c3(nb + 2) - c3(nb - b1 + 2) + c2(nb - b1 + 1));
}
__host__ __device__ inline int rank_b(int nb, int b2) { return (int)(-c2(nb - b2 + 1) - b2); }

// ---------------------------------------------------------- launches ------

// sample_hi > sample_lo: count only hubs [sample_lo, sample_hi) of a resident
// graph (timing samples); force: a schedule to use instead of the tuned or
// built-in one.
void count3_run(Ctx &ctx, const Graph &g, uint64_t *hist, uint64_t *wsum, uint64_t *ntri,
                const gs_anchor_range *anchors, const Tune3 *force = nullptr, uint32_t sample_lo = 0,
                uint32_t sample_hi = 0);
// Time schedules on a sample of g's hubs and keep the fastest for g's shape.
void tune3(Ctx &ctx, const Graph &g, bool weighted, gs_plan3 *out);
// 4-clique counts. kind kParity4 (or kPixel4, parity from direction pixels):
// counters in three blocks of C(nb+2,3), pos | neg | degenerate (even =
// their sum); kSix4: one block of 6-edge
// configurations. Each block is copied to host cnt[b]; with wsum[0] set,
// wsum[b] receives the block's exact signed 128-bit weighted sums (2 words
// per counter, units 2^-wscale). scratch: device memory of scratch_bytes to
// use instead of the context's (nothing is allocated then).
enum { kParity4 = 0, kSix4 = 1, kPixel4 = 2 };
constexpr int kMaxBins6 = 12;
struct Count4Out {
    int kind = kParity4;
    uint64_t *cnt[3] = {nullptr, nullptr, nullptr};
    uint64_t *wsum[3] = {nullptr, nullptr, nullptr};
    int *wscale = nullptr;
    uint64_t *ncl = nullptr;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
};
void count4_run(Ctx &ctx, const Graph &g, const Count4Out &o, const gs_anchor_range *anchors);
// The allocation-free parity count's device scratch: a file-scope device
// array (one copy per device); static_scratch_init takes its address on a
// device once (at context creation), static_scratch returns it.
void static_scratch_init(int device);
void *static_scratch(int device, size_t *bytes);
// Configuration rank of every 6-edge bin-tuple code, and the number of
// configurations (host table, cached per bin count).
const std::vector<uint32_t> &config6_table(int nb, uint32_t *n6);
void build_run(Ctx &ctx, Graph &g, const double *xyz, const double *w);
void graph_stats(Graph &g);
// Pairs (edges) per bin and, with wsum (2 words per bin), the exact signed
// 128-bit sums of w_i*w_j in units of 2^-wscale (the internal 2pCF).
void pair_sums_run(Ctx &ctx, const Graph &g, uint64_t *pairs, uint64_t *wsum, int *wscale,
                   const gs_anchor_range *anchors);
void build_begin(Ctx &ctx, Graph &g, const double *xyz, const double *w, BuildJob &job);
uint64_t build_footprint(const Graph &g, const BuildJob &job);
void build_end(Ctx &ctx, Graph &g, BuildJob &job, bool tile_ok);

// Batched triangle counts over resident graphs with equal bin counts: one
// persistent launch. Results land in host memory `out` (ng x (nconf+1) u64:
// each graph's histogram then its triangle count; then one error word, 0
// when the counts are valid) once `done` has fired. One object may serve a
// launch after another once the previous one has completed; its buffers are
// kept while large enough.
struct Batch3 {
    DevBuf dv;          // device results + queues
    DevBuf gd;          // descriptors
    HostBuf hostdesc;   // staging of descriptors
    HostBuf hostcfg;    // staging of the configuration table
    HostBuf out;        // pinned results
    hipEvent_t done = nullptr;
    int ng = 0, nconf = 0;
    unsigned long long error() const { return out.as<unsigned long long>()[(size_t)ng * (nconf + 1)]; }
    ~Batch3();
};
void count3_batch_enqueue(Ctx &ctx, hipStream_t s, const Graph *const *gs, int ng, Batch3 &b);

void server_stop(Ctx &ctx);

}  // namespace gsn

struct gs_ctx : gsn::Ctx {};
struct gs_graph : gsn::Graph {};
