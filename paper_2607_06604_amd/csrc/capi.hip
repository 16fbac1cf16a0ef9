// capi.hip - C ABI entry points: contexts, graphs, errors, result marshalling.
#include <cmath>
#include <cstdio>
#include <new>

#include "common.h"

namespace gsn {

static thread_local std::string t_detail;

void set_detail(const std::string &msg) { t_detail = msg; }

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void DevBuf::alloc(size_t n) {
    reset();
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        fail(GS_EDEVMEM, "hipMalloc(" + std::to_string(n) + " bytes): " + hipGetErrorString(e));
    }
    bytes = cap = n;
}

void DevBuf::alloc(size_t n, const std::shared_ptr<DevPool> &from) {
    if (!from) {
        alloc(n);
        return;
    }
    reset();
    if (n == 0) n = 1;
    size_t got = 0;
    p = from->take(n, got);
    bytes = n;
    cap = got;
    pool = from;
}

size_t DevPool::round_size(size_t n) {
    if (n <= 256) return 256;
    size_t b = 1;
    while (b < n) b <<= 1;  // next power of two
    if (b <= (1u << 20)) return b;
    const size_t step = b >> 4;  // eighth of the power of two below
    return (n + step - 1) / step * step;
}

void *DevPool::take(size_t n, size_t &got) {
    const size_t r = round_size(n);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = blocks.lower_bound(r);
        if (it != blocks.end() && it->first <= r + r / 4) {
            void *p = it->second;
            got = it->first;
            held -= got;
            blocks.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, r);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        trim();  // cached blocks may be what the device is short of
        e = hipMalloc(&p, r);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(GS_EDEVMEM, "hipMalloc(" + std::to_string(r) + " bytes): " + hipGetErrorString(e));
        }
    }
    got = r;
    return p;
}

void DevPool::give(void *p, size_t got) {
    {
        std::lock_guard<std::mutex> lk(mu);
        if (held + got <= cap) {
            blocks.emplace(got, p);
            held += got;
            return;
        }
    }
    (void)hipDeviceSynchronize();  // the block may still be in use on the builder's stream
    (void)hipFree(p);
}

void DevPool::trim() {
    std::multimap<size_t, void *> drop;
    {
        std::lock_guard<std::mutex> lk(mu);
        drop.swap(blocks);
        held = 0;
    }
    if (drop.empty()) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    for (auto &b : drop) (void)hipFree(b.second);
    (void)hipSetDevice(cur);
}

DevPool::~DevPool() { trim(); }

void HostBuf::alloc(size_t n) {
    reset();
    if (n == 0) n = 1;
    hipError_t e = hipHostMalloc(&p, n, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        fail(GS_ENOMEM, "hipHostMalloc(" + std::to_string(n) + " bytes): " + hipGetErrorString(e));
    }
    bytes = n;
}

void Ctx::use() const { GS_HIP(hipSetDevice(device)); }

void *Ctx::scratch_get(size_t bytes) {
    if (scratch.bytes < bytes) {
        GS_HIP(hipStreamSynchronize(stream));
        scratch.alloc(bytes + bytes / 4);
    }
    return scratch.p;
}

void *Ctx::pinned_get(size_t bytes) {
    if (pinned_bytes < bytes) {
        if (pinned) (void)hipHostFree(pinned);
        pinned = nullptr;
        pinned_bytes = 0;
        GS_HIP(hipHostMalloc(&pinned, bytes, hipHostMallocDefault));
        pinned_bytes = bytes;
    }
    return pinned;
}

// Squared bin thresholds from the definition: e_0 = rmin, e_k = rmin + k*D,
// e_nb = rmax, t_k = e_k*e_k (host float64, no contraction).
Bins make_bins(double rmin, double rmax, int nb) {
    Bins b;
    b.nb = nb;
    volatile double D = (rmax - rmin) / (double)nb;
    for (int k = 0; k <= nb; ++k) {
        volatile double kd = (double)k * D;
        volatile double e = (k == 0) ? rmin : (k == nb ? rmax : rmin + kd);
        b.t[k] = e * e;
    }
    for (int k = nb + 1; k < 256; ++k) b.t[k] = b.t[nb];
    return b;
}

bool weight_scale_ok(const Graph &g, int k, int *s, int *why) {
    if (g.n == 0) {
        *s = 0;
        return true;
    }
    volatile double tlo = g.wmin, thi = g.wmax;
    for (int j = 1; j < k; ++j) {
        tlo = tlo * g.wmin;
        thi = thi * g.wmax;
    }
    if (!(tlo >= 0x1.0p-1022) || !std::isfinite((double)thi)) {
        if (why) *why = GS_EINVAL;
        return false;
    }
    const int sc = 52 - std::ilogb((double)tlo);
    if (std::ilogb((double)thi) + sc > 86) {   // every term below 2^87
        if (why) *why = GS_EINVAL;
        return false;
    }
    *s = sc;
    return true;
}

bool wide_terms(const Graph &g, int k) {
    const int s = weight_scale(g, k);
    volatile double thi = g.wmax;
    for (int j = 1; j < k; ++j) thi = thi * g.wmax;
    return std::ilogb((double)thi) + s >= 63;
}

double sum128_to_double(const uint64_t *w, int scale) {
    const __int128 v = (__int128)(((unsigned __int128)w[1] << 64) | w[0]);
    return std::ldexp((double)v, -scale);
}

int weight_scale(const Graph &g, int k) {
    int s = 0, why = GS_EINVAL;
    if (!(g.flags & GS_WEIGHTED)) fail(GS_EINVAL, "graph has no weights");
    if (!weight_scale_ok(g, k, &s, &why))
        fail(why, "weight products leave the normal float64 range or span more than 2^34 (exact sums)");
    return s;
}

}  // namespace gsn

using namespace gsn;

extern "C" {

const char *gs_strerror(int code) {
    switch (code) {
        case GS_OK: return "ok";
        case GS_EINVAL: return "invalid argument";
        case GS_EOVERFLOW: return "too many points for 32-bit labels";
        case GS_ENOMEM: return "host memory allocation failed";
        case GS_EDEVMEM: return "device memory or budget insufficient";
        case GS_EHIP: return "HIP runtime error";
        case GS_EAGAIN: return "queue full, retry";
        case GS_ENOTFOUND: return "unknown ticket";
        case GS_EUNSUPPORTED: return "input beyond the library's limits";
        case GS_ENOCOORDS: return "graph was built without coordinates";
        default: return "unknown status";
    }
}

const char *gs_last_error_detail(void) { return t_detail.c_str(); }

int gs_create(gs_ctx **out, int device, uint64_t hbm_budget_bytes, void *hip_stream) {
    if (!out) return GS_EINVAL;
    *out = nullptr;
    gs_ctx *c = nullptr;
    int rc = guarded([&] {
        int ndev = 0;
        GS_HIP(hipGetDeviceCount(&ndev));
        if (device < 0 || device >= ndev) fail(GS_EINVAL, "no such device");
        c = new gs_ctx();
        c->device = device;
        GS_HIP(hipSetDevice(device));
        hipDeviceProp_t prop;
        GS_HIP(hipGetDeviceProperties(&prop, device));
        c->n_cu = prop.multiProcessorCount;
        c->max_lds = (int)prop.sharedMemPerBlock;
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            GS_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        GS_HIP(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
        for (auto &e : c->ev) GS_HIP(hipEventCreate(&e));
        size_t fr = 0, tot = 0;
        GS_HIP(hipMemGetInfo(&fr, &tot));
        c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)fr);
        c->pool = std::make_shared<DevPool>();
        c->pool->device = device;
        c->pool->cap = c->budget / 8;
        static_scratch_init(device);
    });
    if (rc != GS_OK) {
        if (c) gs_destroy(c);
        return rc;
    }
    *out = c;
    return GS_OK;
}

int gs_destroy(gs_ctx *ctx) {
    if (!ctx) return GS_EINVAL;
    (void)hipSetDevice(ctx->device);
    server_stop(*ctx);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->copy_stream) {
        (void)hipStreamSynchronize(ctx->copy_stream);
        (void)hipStreamDestroy(ctx->copy_stream);
    }
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return GS_OK;
}

int gs_build_graph(gs_ctx *ctx, const double *xyz, int64_t n, const double *weights,
                   const gs_graph_params *p, gs_graph **out) {
    if (!out) return GS_EINVAL;
    *out = nullptr;
    gs_graph *g = nullptr;
    int rc = guarded([&] {
        if (!ctx || !p) fail(GS_EINVAL, "null context or params");
        if (n < 0) fail(GS_EINVAL, "negative n");
        if (n > 0 && !xyz) fail(GS_EINVAL, "null xyz");
        if (n >= 0xFFFFFFFFll) fail(GS_EOVERFLOW, "n must be below 2^32 - 1");
        if (!(p->box > 0) || !std::isfinite(p->box)) fail(GS_EINVAL, "box must be finite and > 0");
        if (p->nbins < 1 || p->nbins > 255) fail(GS_EINVAL, "nbins must be in 1..255");
        const bool periodic = !(p->flags & GS_NONPERIODIC);
        if (!(p->rmin >= 0) || !(p->rmin < p->rmax) || !std::isfinite(p->rmax) ||
            (periodic && !(p->rmax < 0.5 * p->box)))
            fail(GS_EINVAL, periodic ? "need 0 <= rmin < rmax < box/2" : "need 0 <= rmin < rmax, finite");
        if (p->flags & ~(GS_WEIGHTED | GS_KEEP_COORDS | GS_INPUT_ON_DEVICE | GS_NONPERIODIC))
            fail(GS_EINVAL, "unknown flags");
        bool weighted = (p->flags & GS_WEIGHTED) != 0;
        if (weighted != (weights != nullptr)) fail(GS_EINVAL, "weights given iff GS_WEIGHTED");
        ctx->use();
        g = new gs_graph();
        g->device = ctx->device;
        g->n = n;
        g->box = p->box;
        g->rmin = p->rmin;
        g->rmax = p->rmax;
        g->nbins = p->nbins;
        g->flags = p->flags;
        g->periodic = periodic;
        g->bins = make_bins(p->rmin, p->rmax, p->nbins);
        build_run(*ctx, *g, xyz, weights);
    });
    if (rc != GS_OK) {
        delete g;
        return rc;
    }
    *out = g;
    return GS_OK;
}

int gs_graph_info(const gs_graph *g, gs_graph_stats *out) {
    if (!g || !out) return GS_EINVAL;
    int rc = guarded([&] {
        GS_HIP(hipSetDevice(g->device));
        graph_stats(*const_cast<gs_graph *>(g));
    });
    if (rc != GS_OK) return rc;
    memset(out, 0, sizeof *out);
    out->sum_sq_degree = g->sum_sq_deg;
    out->n = g->n;
    out->n_edges = g->n_edges;
    out->max_deg = g->max_deg;
    out->device_bytes = g->device_bytes;
    out->n_windows = g->n_windows;
    out->nbins = g->nbins;
    memcpy(out->pair_hist, g->pair_hist, sizeof g->pair_hist);
    return GS_OK;
}

int gs_graph_export(const gs_graph *g, uint64_t *row_ptr, uint32_t *col, uint8_t *bin,
                    uint32_t *perm) {
    return guarded([&] {
        if (!g) fail(GS_EINVAL, "null graph");
        GS_HIP(hipSetDevice(g->device));
        if (row_ptr)
            GS_HIP(hipMemcpy(row_ptr, g->row_ptr.p, sizeof(uint64_t) * (g->n + 1), hipMemcpyDeviceToHost));
        if (g->n_windows > 1) {
            if (col && g->n_edges) memcpy(col, g->hcol.p, sizeof(uint32_t) * g->n_edges);
            if (bin && g->n_edges) memcpy(bin, g->hbin.p, g->n_edges);
        } else {
            if (col && g->n_edges)
                GS_HIP(hipMemcpy(col, g->col.p, sizeof(uint32_t) * g->n_edges, hipMemcpyDeviceToHost));
            if (bin && g->n_edges)
                GS_HIP(hipMemcpy(bin, g->bin.p, g->n_edges, hipMemcpyDeviceToHost));
        }
        if (perm && g->n)
            GS_HIP(hipMemcpy(perm, g->perm.p, sizeof(uint32_t) * g->n, hipMemcpyDeviceToHost));
    });
}

int gs_graph_free(gs_graph *g) {
    if (!g) return GS_EINVAL;
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    delete g;
    return GS_OK;
}

int gs_count_3pcf(gs_ctx *ctx, const gs_graph *g, uint64_t *hist, uint64_t *wsum128,
                  double *whist, int32_t *wscale, uint64_t *n_triangles,
                  const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !hist || !n_triangles) fail(GS_EINVAL, "null argument");
        bool want_w = wsum128 || whist || wscale;
        if (want_w && !(g->flags & GS_WEIGHTED)) fail(GS_EINVAL, "graph has no weights");
        if (g->device != ctx->device) fail(GS_EINVAL, "graph and context on different devices");
        ctx->use();
        int64_t nc = n_configs(g->nbins);
        std::vector<uint64_t> ws;
        uint64_t *wdst = nullptr;
        if (g->flags & GS_WEIGHTED) {
            ws.assign(2 * nc, 0);
            wdst = ws.data();
        }
        count3_run(*ctx, *g, hist, wdst, n_triangles, anchors);
        if (g->flags & GS_WEIGHTED) {
            const int sc = weight_scale(*g, 3);
            if (wsum128) memcpy(wsum128, ws.data(), sizeof(uint64_t) * 2 * nc);
            if (whist)
                for (int64_t c = 0; c < nc; ++c) whist[c] = sum128_to_double(&ws[2 * c], sc);
            if (wscale) *wscale = sc;
        }
    });
}

}  // extern "C"

static void check4(gs_ctx *ctx, const gs_graph *g) {
    if (!(g->flags & GS_KEEP_COORDS)) fail(GS_ENOCOORDS, "4-clique counts need GS_KEEP_COORDS");
    if (g->device != ctx->device) fail(GS_EINVAL, "graph and context on different devices");
}

extern "C" {

int gs_count_4pcf_parity(gs_ctx *ctx, const gs_graph *g, uint64_t *even, uint64_t *pos,
                         uint64_t *neg, uint64_t *n_cliques, const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !even || !pos || !neg || !n_cliques) fail(GS_EINVAL, "null argument");
        check4(ctx, g);
        ctx->use();
        const int64_t nc = n_configs(g->nbins);
        Count4Out o;
        o.kind = kParity4;
        o.cnt[0] = pos;
        o.cnt[1] = neg;
        o.cnt[2] = even;   // the degenerate block, then even = pos + neg + degenerate
        o.ncl = n_cliques;
        count4_run(*ctx, *g, o, anchors);
        for (int64_t c = 0; c < nc; ++c) even[c] += pos[c] + neg[c];
    });
}

int gs_count_4pcf_parity_noalloc(gs_ctx *ctx, const gs_graph *g, uint64_t *even, uint64_t *pos,
                                 uint64_t *neg, uint64_t *n_cliques, const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !even || !pos || !neg || !n_cliques) fail(GS_EINVAL, "null argument");
        if (!(g->flags & GS_KEEP_COORDS)) fail(GS_ENOCOORDS, "parity needs GS_KEEP_COORDS");
        if (g->n_windows > 1) fail(GS_EUNSUPPORTED, "parity counts need a device-resident graph");
        if (g->device != ctx->device) fail(GS_EINVAL, "graph and context on different devices");
        ctx->use();
        size_t bytes = 0;
        void *ptr = static_scratch(ctx->device, &bytes);
        const int64_t nc = n_configs(g->nbins);
        Count4Out o;
        o.kind = kParity4;
        o.cnt[0] = pos;
        o.cnt[1] = neg;
        o.cnt[2] = even;
        o.ncl = n_cliques;
        o.scratch = ptr;
        o.scratch_bytes = bytes;
        count4_run(*ctx, *g, o, anchors);
        for (int64_t c = 0; c < nc; ++c) even[c] += pos[c] + neg[c];
    });
}

// 128-bit two's complement words a + b into out (lo, hi).
static void add128w(const uint64_t *a, const uint64_t *b, uint64_t *out) {
    const unsigned __int128 x = ((unsigned __int128)a[1] << 64) | a[0], y = ((unsigned __int128)b[1] << 64) | b[0];
    const unsigned __int128 z = x + y;
    out[0] = (uint64_t)z;
    out[1] = (uint64_t)(z >> 64);
}

int gs_count_4pcf_parity_weighted(gs_ctx *ctx, const gs_graph *g, uint64_t *even, uint64_t *pos, uint64_t *neg,
                                  uint64_t *wsum128, int32_t *wscale, uint64_t *n_cliques,
                                  const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !even || !pos || !neg || !wsum128 || !n_cliques) fail(GS_EINVAL, "null argument");
        if (!(g->flags & GS_WEIGHTED)) fail(GS_EINVAL, "graph has no weights");
        check4(ctx, g);
        ctx->use();
        const int64_t nc = n_configs(g->nbins);
        std::vector<uint64_t> deg(nc), wdeg(2 * nc);
        uint64_t *we = wsum128, *wp = wsum128 + 2 * nc, *wn = wsum128 + 4 * nc;
        Count4Out o;
        o.kind = kParity4;
        o.cnt[0] = pos;
        o.cnt[1] = neg;
        o.cnt[2] = deg.data();
        o.wsum[0] = wp;
        o.wsum[1] = wn;
        o.wsum[2] = wdeg.data();
        int sc = 0;
        o.wscale = &sc;
        o.ncl = n_cliques;
        count4_run(*ctx, *g, o, anchors);
        for (int64_t c = 0; c < nc; ++c) {
            even[c] = pos[c] + neg[c] + deg[c];
            uint64_t t[2];
            add128w(&wp[2 * c], &wn[2 * c], t);
            add128w(t, &wdeg[2 * c], &we[2 * c]);
        }
        if (wscale) *wscale = sc;
    });
}

int gs_count_4pcf_pixel(gs_ctx *ctx, const gs_graph *g, uint64_t *even, uint64_t *pos, uint64_t *neg,
                        uint64_t *n_cliques, const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !even || !pos || !neg || !n_cliques) fail(GS_EINVAL, "null argument");
        check4(ctx, g);
        ctx->use();
        const int64_t nc = n_configs(g->nbins);
        Count4Out o;
        o.kind = kPixel4;
        o.cnt[0] = pos;
        o.cnt[1] = neg;
        o.cnt[2] = even;
        o.ncl = n_cliques;
        count4_run(*ctx, *g, o, anchors);
        for (int64_t c = 0; c < nc; ++c) even[c] += pos[c] + neg[c];
    });
}

int gs_count_4pcf_full(gs_ctx *ctx, const gs_graph *g, uint64_t *hist6, uint64_t *wsum128, int32_t *wscale,
                       uint64_t *n_cliques, const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !hist6 || !n_cliques) fail(GS_EINVAL, "null argument");
        if ((wsum128 || wscale) && !(g->flags & GS_WEIGHTED)) fail(GS_EINVAL, "graph has no weights");
        if (g->nbins > kMaxBins6) fail(GS_EUNSUPPORTED, "6-edge counts take at most 12 bins");
        check4(ctx, g);
        ctx->use();
        Count4Out o;
        o.kind = kSix4;
        o.cnt[0] = hist6;
        o.wsum[0] = wsum128;
        int sc = 0;
        o.wscale = &sc;
        o.ncl = n_cliques;
        count4_run(*ctx, *g, o, anchors);
        if (wscale) *wscale = sc;
    });
}

int gs_n_configs6(int32_t nbins, uint32_t *n6) {
    return guarded([&] {
        if (!n6 || nbins < 1 || nbins > kMaxBins6) fail(GS_EINVAL, "nbins must be 1..12");
        (void)config6_table(nbins, n6);
    });
}

int gs_config6_table(int32_t nbins, uint32_t *rank) {
    return guarded([&] {
        if (!rank || nbins < 1 || nbins > kMaxBins6) fail(GS_EINVAL, "nbins must be 1..12");
        uint32_t n6 = 0;
        const std::vector<uint32_t> &t = config6_table(nbins, &n6);
        memcpy(rank, t.data(), sizeof(uint32_t) * t.size());
    });
}

int gs_pair_sums(gs_ctx *ctx, const gs_graph *g, uint64_t *pairs, uint64_t *wsum128, int32_t *wscale,
                 const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !pairs) fail(GS_EINVAL, "null argument");
        if ((wsum128 || wscale) && !(g->flags & GS_WEIGHTED)) fail(GS_EINVAL, "graph has no weights");
        if (g->device != ctx->device) fail(GS_EINVAL, "graph and context on different devices");
        ctx->use();
        int sc = 0;
        pair_sums_run(*ctx, *g, pairs, wsum128, &sc, anchors);
        if (wscale) *wscale = wsum128 ? sc : 0;
    });
}

int gs_tune_3pcf(gs_ctx *ctx, const gs_graph *g, uint32_t flags, gs_plan3 *out) {
    return guarded([&] {
        if (!ctx || !g) fail(GS_EINVAL, "null argument");
        if (flags & ~GS_WEIGHTED) fail(GS_EINVAL, "unknown flags");
        if (g->device != ctx->device) fail(GS_EINVAL, "graph and context on different devices");
        ctx->use();
        tune3(*ctx, *g, (flags & GS_WEIGHTED) != 0, out);
    });
}

int gs_count_3pcf_batch(gs_ctx *ctx, const gs_graph *const *graphs, int ng, uint64_t *hists,
                        uint64_t *n_triangles) {
    return guarded([&] {
        if (!ctx || !graphs || ng < 1 || !hists || !n_triangles) fail(GS_EINVAL, "null argument");
        ctx->use();
        std::vector<const Graph *> gs(ng);
        for (int g = 0; g < ng; ++g) gs[g] = graphs[g];
        Batch3 b;
        GS_HIP(hipEventRecord(ctx->ev[0], ctx->stream));
        count3_batch_enqueue(*ctx, ctx->stream, gs.data(), ng, b);
        GS_HIP(hipEventRecord(ctx->ev[1], ctx->stream));
        GS_HIP(hipEventSynchronize(b.done));
        GS_HIP(hipStreamSynchronize(ctx->stream));
        if (b.error()) fail(GS_EUNSUPPORTED, "batched count failed on the device (LDS addressing)");
        const unsigned long long *o = b.out.as<unsigned long long>();
        const size_t per = (size_t)b.nconf + 1;
        for (int g = 0; g < ng; ++g) {
            for (int c = 0; c < b.nconf; ++c) hists[(size_t)g * b.nconf + c] = o[g * per + c];
            n_triangles[g] = o[g * per + b.nconf];
        }
        float ms = 0;
        GS_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
        ctx->t.count_ms = ms;
        ctx->t.kernel_ms = ms;
        ctx->t.kernel_launches = 1;
        uint64_t sq = 0;
        bool known = true;
        for (int g = 0; g < ng; ++g) {
            sq += gs[g]->sum_sq_deg;
            known = known && gs[g]->stats_ready;
        }
        ctx->t.alg_bytes = known ? (uint64_t)(2.5 * (double)sq) : 0;
    });
}

int gs_get_timings(const gs_ctx *ctx, gs_timings *out) {
    if (!ctx || !out) return GS_EINVAL;
    out->build_ms = ctx->t.build_ms;
    out->count_ms = ctx->t.count_ms;
    out->kernel_ms = ctx->t.kernel_ms;
    out->kernel_launches = ctx->t.kernel_launches;
    out->alg_bytes = ctx->t.alg_bytes;
    out->probes = ctx->t.probes;
    out->table_log2 = ctx->t.table_log2;
    out->block = ctx->t.block;
    out->group = ctx->t.group;
    out->hash_load = ctx->t.hash_load;
    return GS_OK;
}

}  // extern "C"
