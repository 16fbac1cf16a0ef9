// count3x.hip - restricted and anisotropic triangle counts: the equilateral
// 3pCF (paper Sec. 3.5, its restricted kernel: triangles whose three sides
// share one bin) and the mu-binned 3pCF (Sec. 6, anisotropy for redshift-
// space distortions: each triangle binned by its sorted side bins and by
// the orientation of its plane to the line of sight).
//
// One work group per hub i (hubs from the per-XCD queues). The hub's forward
// row goes into an LDS hash (label -> position) with its bins (and, for mu,
// its coordinates and original indices); the spokes' forward rows, each cut
// at the hub row's largest label, are streamed as one flat sequence so that
// every lane takes one candidate third vertex k; k closes a triangle when it
// is in the hub's row. Equilateral counts drop every candidate whose spoke-
// row bin differs from the spoke's bin before probing, and every hit whose
// hub-row bin differs. Counters are u32 in LDS, flushed to u64 before they
// could wrap; weighted terms (signed weights) are exact integers, summed in
// LDS when below 2^63 and straight into the global 128-bit sums otherwise.
//
// mu (the reading taken): with the triangle's vertices in original-index
// order p0 < p1 < p2, n = sep(p0,p1) x sep(p0,p2) (minimum image, the cross
// product in the parity kernel's operation order), s = (nx*nx + ny*ny) +
// nz*nz and t = nz*nz; the mu bin is the number of k in 1..nmu-1 with
// t*(nmu*nmu) >= (k*k)*s, i.e. mu = |nz|/|n| in equal bins [k/nmu, (k+1)/nmu)
// of [0, 1] (z is the line of sight); a collinear triangle (s = 0) is in
// bin 0. The counter of a triangle is conf(sorted side bins) * nmu + mu bin.
#include <cstdio>
#include <cstdlib>

#include "kern_util.h"

namespace gsn {
namespace {

enum { kEqui = 0, kMu = 1 };

struct XArgs {
    const uint64_t *rp;
    const uint32_t *col;
    const uint8_t *bin;
    const uint32_t *perm;
    const double *X, *Y, *Z;
    const double *w;
    double wmul, L, half;
    uint32_t n, maxdeg;
    int nb, nmu, ncnt, log2h;
    uint32_t anchor_lo, anchor_hi;
    uint32_t *queue;
    unsigned long long *hist, *wsum, *ntri;
};

struct LayoutX {
    uint32_t hkey, hloc, pb, px, py, pz, pp, pw, mstart, mpref, mloc, hist, wlo, whi, tab, wtot, misc, total;
};

__host__ __device__ inline LayoutX layoutx(int block, uint32_t H, uint32_t maxdeg, int kind, int ncnt, int nb,
                                           bool weighted, bool anchored) {
    LayoutX L{};
    uint32_t o = 0, d = maxdeg + 1;
    const bool coords = kind == kMu;
    L.px = o;     if (coords) o = lds_align(o + 8 * d, 16);
    L.py = o;     if (coords) o = lds_align(o + 8 * d, 16);
    L.pz = o;     if (coords) o = lds_align(o + 8 * d, 16);
    L.pw = o;     if (weighted) o = lds_align(o + 8 * d, 16);
    L.wlo = o;    if (weighted) o = lds_align(o + 8 * ncnt, 16);
    L.whi = o;    if (weighted) o = lds_align(o + 8 * ncnt, 16);
    L.mstart = o; o = lds_align(o + 8 * block, 16);
    L.wtot = o;   o = lds_align(o + 8 * (block / 64 + 1), 16);
    L.misc = o;   o = lds_align(o + 16, 16);
    L.hkey = o;   o = lds_align(o + 4 * H, 16);
    L.pp = o;     if (coords || anchored) o = lds_align(o + 4 * d, 16);
    L.mpref = o;  o = lds_align(o + 4 * (block + 1), 16);
    L.hist = o;   o = lds_align(o + 4 * ncnt, 16);
    L.tab = o;    o = lds_align(o + 8 * (nb + 1), 16);
    L.hloc = o;   o = lds_align(o + 2 * H, 16);
    L.mloc = o;   o = lds_align(o + 2 * block, 16);
    L.pb = o;     o = lds_align(o + d, 16);
    L.total = o;
    return L;
}

// mu bin of the triangle with (minimum-image) edge vectors u = p0->p1 and
// v = p0->p2.
__device__ __forceinline__ int mu_bin(double ux, double uy, double uz, double vx, double vy, double vz, int nmu) {
    const double nx = __dsub_rn(__dmul_rn(uy, vz), __dmul_rn(uz, vy));
    const double ny = __dsub_rn(__dmul_rn(uz, vx), __dmul_rn(ux, vz));
    const double nz = __dsub_rn(__dmul_rn(ux, vy), __dmul_rn(uy, vx));
    const double s = __dadd_rn(__dadd_rn(__dmul_rn(nx, nx), __dmul_rn(ny, ny)), __dmul_rn(nz, nz));
    const double t = __dmul_rn(__dmul_rn(nz, nz), (double)(nmu * nmu));
    int m = 0;
    if (s > 0.0)
        for (int k = 1; k < nmu; ++k) m += t >= __dmul_rn((double)(k * k), s);
    return m;
}

// A vertex: absolute coordinates and original index.
struct P3x {
    double x, y, z;
    uint32_t o;
};

__device__ __forceinline__ void swapx(P3x &a, P3x &b) {
    const P3x t = a;
    a = b;
    b = t;
}

// Sort three vertices by original index.
__device__ __forceinline__ void order3(P3x &a, P3x &b, P3x &c) {
    if (a.o > b.o) swapx(a, b);
    if (b.o > c.o) swapx(b, c);
    if (a.o > b.o) swapx(a, b);
}

template <int BLOCK, bool WEIGHTED>
__device__ void flushx(const XArgs &a, uint32_t *hist, unsigned long long *wlo, unsigned long long *whi,
                       unsigned long long &mytri) {
    for (int b = threadIdx.x; b < a.ncnt; b += BLOCK) {
        const uint32_t v = hist[b];
        if (v) {
            atomicAdd(&a.hist[b], (unsigned long long)v);
            mytri += v;
            hist[b] = 0;
        }
        if (WEIGHTED && (wlo[b] | whi[b])) {
            add128_words(&a.wsum[2 * b], lds_sum128(wlo[b], whi[b]));
            wlo[b] = 0;
            whi[b] = 0;
        }
    }
}

template <int BLOCK, int KIND, bool WEIGHTED, bool ANCHORED>
__global__ __launch_bounds__(BLOCK) void k_count3x(XArgs a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const uint32_t H = 1u << a.log2h, hmask = H - 1;
    const LayoutX L = layoutx(BLOCK, H, a.maxdeg, KIND, a.ncnt, a.nb, WEIGHTED, ANCHORED);
    uint32_t *hkey = (uint32_t *)(sm + L.hkey);
    uint16_t *hloc = (uint16_t *)(sm + L.hloc);
    uint8_t *pb = (uint8_t *)(sm + L.pb);
    double *px = (double *)(sm + L.px), *py = (double *)(sm + L.py), *pz = (double *)(sm + L.pz);
    double *pw = (double *)(sm + L.pw);
    uint32_t *pp = (uint32_t *)(sm + L.pp);
    unsigned long long *mstart = (unsigned long long *)(sm + L.mstart);
    uint32_t *mpref = (uint32_t *)(sm + L.mpref);
    uint16_t *mloc = (uint16_t *)(sm + L.mloc);
    uint32_t *hist = (uint32_t *)(sm + L.hist);
    unsigned long long *wlo = (unsigned long long *)(sm + L.wlo), *whi = (unsigned long long *)(sm + L.whi);
    int *ta = (int *)(sm + L.tab);
    int *tb = ta + (a.nb + 1);
    uint32_t *wtot = (uint32_t *)(sm + L.wtot);
    uint32_t *s_hub = (uint32_t *)(sm + L.misc);
    const int tid = threadIdx.x;

    for (uint32_t s = tid; s < H; s += BLOCK) hkey[s] = kEmptyKey;
    for (int b = tid; b < a.ncnt; b += BLOCK) {
        hist[b] = 0;
        if (WEIGHTED) {
            wlo[b] = 0;
            whi[b] = 0;
        }
    }
    for (int b = tid; b < a.nb; b += BLOCK) {
        ta[b] = rank_a(a.nb, b);
        tb[b] = rank_b(a.nb, b);
    }
    __syncthreads();

    unsigned long long mytri = 0;
    uint64_t acc = 0;   // increments since the last flush (uniform)
    HubCursor cursor;
    const double Lb = a.L, half = a.half;
    while (true) {
        if (tid == 0) *s_hub = next_hub_in(a.queue, 0, a.n, gridDim.x, cursor, 1);
        __syncthreads();
        const uint32_t i = *s_hub;
        if (i == kEmptyKey) break;
        const uint64_t beg = a.rp[i];
        const uint32_t d = (uint32_t)(a.rp[i + 1] - beg);
        if (d < 2) {
            __syncthreads();
            continue;
        }
        const uint32_t last = a.col[beg + d - 1];   // the hub row's largest label
        const double xi = KIND == kMu ? a.X[i] : 0.0, yi = KIND == kMu ? a.Y[i] : 0.0,
                     zi = KIND == kMu ? a.Z[i] : 0.0;
        const uint32_t pi = (KIND == kMu || ANCHORED) ? a.perm[i] : 0u;
        const double wi = WEIGHTED ? a.w[i] : 0.0;
        for (uint32_t e = tid; e < d; e += BLOCK) {
            const uint32_t k = a.col[beg + e];
            uint32_t s = label_hash(k, a.log2h);
            while (atomicCAS(&hkey[s], kEmptyKey, k) != kEmptyKey) s = (s + 1) & hmask;
            hloc[s] = (uint16_t)e;
            pb[e] = a.bin[beg + e];
            if (KIND == kMu) {
                px[e] = a.X[k];
                py[e] = a.Y[k];
                pz[e] = a.Z[k];
            }
            if (KIND == kMu || ANCHORED) pp[e] = a.perm[k];
            if (WEIGHTED) pw[e] = a.w[k];
        }
        __syncthreads();
        for (uint32_t c0 = 0; c0 + 1 < d; c0 += BLOCK) {
            const uint32_t sidx = c0 + tid;
            uint32_t len = 0;
            uint64_t st = 0;
            if (sidx + 1 < d) {
                const uint32_t j = a.col[beg + sidx];
                st = a.rp[j];
                uint32_t lo = 0, hi = (uint32_t)(a.rp[j + 1] - st);   // entries <= last
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (a.col[st + mid] <= last) lo = mid + 1;
                    else hi = mid;
                }
                len = lo;
            }
            uint32_t total;
            const uint32_t pre = wg_excl_scan<BLOCK>(len, wtot, total);
            mstart[tid] = st;
            mpref[tid] = pre;
            mloc[tid] = (uint16_t)sidx;
            if (tid == 0) mpref[BLOCK] = total;
            __syncthreads();
            if (acc + total >= 0xFFFFFFFFull) {
                flushx<BLOCK, WEIGHTED>(a, hist, wlo, whi, mytri);
                acc = 0;
                __syncthreads();
            }
            acc += total;
            uint32_t sp = 0;
            for (uint32_t e0 = 0; e0 < total; e0 += BLOCK) {
                const uint32_t e = e0 + tid;
                if (e >= total) continue;
                while (mpref[sp + 1] <= e) ++sp;
                const uint32_t js = mloc[sp];   // spoke position in the hub row
                const uint64_t ge = mstart[sp] + (e - mpref[sp]);
                const uint32_t z = a.bin[ge];
                const uint32_t x = pb[js];
                if (KIND == kEqui && z != x) continue;
                const uint32_t k = a.col[ge];
                uint32_t h = label_hash(k, a.log2h), key;
                while ((key = hkey[h]) != k && key != kEmptyKey) h = (h + 1) & hmask;
                if (key != k) continue;
                const uint32_t t = hloc[h];
                const uint32_t y = pb[t];
                if (KIND == kEqui && y != x) continue;
                if (ANCHORED) {
                    const uint32_t m = min(pi, min(pp[js], pp[t]));
                    if (m < a.anchor_lo || m >= a.anchor_hi) continue;
                }
                uint32_t cnt;
                if (KIND == kEqui) {
                    cnt = x;
                } else {
                    const int lo = (int)min(x, min(y, z)), hi = (int)max(x, max(y, z));
                    const int mid = (int)(x + y + z) - lo - hi;
                    // the three vertices in original-index order; u, v the
                    // separations from the first to the second and third
                    P3x v0{xi, yi, zi, pi}, v1{px[js], py[js], pz[js], pp[js]}, v2{px[t], py[t], pz[t], pp[t]};
                    order3(v0, v1, v2);
                    const double ux = min_image(v0.x, v1.x, Lb, half), uy = min_image(v0.y, v1.y, Lb, half),
                                 uz = min_image(v0.z, v1.z, Lb, half);
                    const double vx = min_image(v0.x, v2.x, Lb, half), vy = min_image(v0.y, v2.y, Lb, half),
                                 vz = min_image(v0.z, v2.z, Lb, half);
                    cnt = (uint32_t)(ta[lo] + tb[mid] + hi) * (uint32_t)a.nmu +
                          (uint32_t)mu_bin(ux, uy, uz, vx, vy, vz, a.nmu);
                }
                __hip_atomic_fetch_add((lds_u32 *)(size_t)lds_addr(&hist[cnt]), 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                if (WEIGHTED) {
                    const double w1 = pw[js], w2 = pw[t];
                    const bool ng = (wi < 0.0) ^ (w1 < 0.0) ^ (w2 < 0.0);
                    double p = fabs(wi), q = fabs(w1), r = fabs(w2), tt;
                    if (p > q) { tt = p; p = q; q = tt; }
                    if (q > r) { tt = q; q = r; r = tt; }
                    if (p > q) { tt = p; p = q; q = tt; }
                    const double xw = __dmul_rn(__dmul_rn(__dmul_rn(p, q), r), a.wmul);
                    if (narrow_term(xw)) {
                        const long long m = (long long)big_term_u64(xw);
                        lds_term(&wlo[cnt], &whi[cnt], ng ? -m : m);
                    } else {
                        add128_words(&a.wsum[2 * cnt], wide_term(xw, ng));
                    }
                }
            }
            __syncthreads();
        }
        for (uint32_t e = tid; e < d; e += BLOCK) {
            const uint32_t k = a.col[beg + e];
            uint32_t s = label_hash(k, a.log2h);
            while (hkey[s] != k) s = (s + 1) & hmask;
            hkey[s] = kEmptyKey;
        }
        __syncthreads();
    }
    __syncthreads();
    flushx<BLOCK, WEIGHTED>(a, hist, wlo, whi, mytri);
    for (int o = 32; o > 0; o >>= 1) mytri += __shfl_xor(mytri, o, 64);
    if ((tid & 63) == 0 && mytri) atomicAdd(a.ntri, mytri);
}

__global__ void k_zerox(unsigned long long *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int KIND, bool W, bool A>
void launchx(Ctx &ctx, const XArgs &a, uint32_t lds) {
    constexpr int BLOCK = 256;
    const void *kern = reinterpret_cast<const void *>(&k_count3x<BLOCK, KIND, W, A>);
    if (lds > 65536) GS_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    GS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count3x<BLOCK, KIND, W, A>, BLOCK, lds));
    if (per_cu < 1) fail(GS_EUNSUPPORTED, "restricted triangle kernel does not fit a compute unit");
    uint32_t grid = (uint32_t)ctx.n_cu * (uint32_t)per_cu;
    grid = (grid + kNumQueues - 1) / kNumQueues * kNumQueues;
    k_count3x<BLOCK, KIND, W, A><<<dim3(grid), dim3(BLOCK), lds, ctx.stream>>>(a);
    GS_HIP(hipGetLastError());
}

template <int KIND>
void launchx_k(Ctx &ctx, const XArgs &a, uint32_t lds, bool w, bool an) {
    if (w) an ? launchx<KIND, true, true>(ctx, a, lds) : launchx<KIND, true, false>(ctx, a, lds);
    else an ? launchx<KIND, false, true>(ctx, a, lds) : launchx<KIND, false, false>(ctx, a, lds);
}

}  // namespace

void count3x_run(Ctx &ctx, const Graph &g, int kind, int nmu, uint64_t *hist, uint64_t *wsum, int *wscale,
                 uint64_t *ntri, const gs_anchor_range *anchors) {
    const int nb = g.nbins;
    const bool mu = kind == kMu;
    const bool weighted = wsum != nullptr;
    const bool anchored = anchors != nullptr;
    if (anchored && anchors->lo > anchors->hi) fail(GS_EINVAL, "anchor range lo > hi");
    if (g.n_windows > 1) fail(GS_EUNSUPPORTED, "restricted triangle counts need a device-resident graph");
    if (mu && (nmu < 1 || nmu > 64)) fail(GS_EINVAL, "mu bins must be 1..64");
    if (mu && !(g.flags & GS_KEEP_COORDS)) fail(GS_ENOCOORDS, "mu binning needs GS_KEEP_COORDS");
    const int ncnt = mu ? (int)n_configs(nb) * nmu : nb;
    const uint32_t maxdeg = g.max_deg;
    if (maxdeg >= 65535) fail(GS_EUNSUPPORTED, "forward degree above 65534");
    uint32_t H = 64;
    int log2h = 6;
    while (H < 2 * maxdeg) { H <<= 1; ++log2h; }
    const LayoutX L = layoutx(256, H, maxdeg, kind, ncnt, nb, weighted, anchored);
    if ((int)L.total > ctx.max_lds)
        fail(GS_EUNSUPPORTED, "restricted triangle kernel LDS footprint too large (" + std::to_string(L.total) +
                                  " bytes)");
    const size_t woff = ((size_t)ncnt + 1 + 31) / 32 * 32;
    const size_t qoff = weighted ? (woff + 2 * (size_t)ncnt + 31) / 32 * 32 : woff;
    const size_t words = qoff + kQueueWords / 2;
    unsigned long long *dv = (unsigned long long *)ctx.scratch_get(words * 8);
    XArgs a{};
    a.rp = g.row_ptr.as<uint64_t>();
    a.col = g.col.as<uint32_t>();
    a.bin = g.bin.as<uint8_t>();
    a.perm = g.perm.as<uint32_t>();
    if (mu) {
        const double *C = g.coords.as<double>();
        a.X = C;
        a.Y = C + g.n;
        a.Z = C + 2 * g.n;
    }
    const int sc = weighted ? weight_scale(g, 3) : 0;
    a.w = weighted ? g.weights.as<double>() : nullptr;
    a.wmul = std::ldexp(1.0, sc);
    a.L = g.periodic ? g.box : HUGE_VAL;
    a.half = g.periodic ? 0.5 * g.box : HUGE_VAL;
    a.n = (uint32_t)g.n;
    a.maxdeg = maxdeg;
    a.nb = nb;
    a.nmu = mu ? nmu : 1;
    a.ncnt = ncnt;
    a.log2h = log2h;
    a.anchor_lo = anchored ? (uint32_t)std::min<uint64_t>(anchors->lo, 0xFFFFFFFFull) : 0;
    a.anchor_hi = anchored ? (uint32_t)std::min<uint64_t>(anchors->hi, 0xFFFFFFFFull) : 0;
    a.hist = dv;
    a.ntri = dv + ncnt;
    a.wsum = weighted ? dv + woff : nullptr;
    a.queue = (uint32_t *)(dv + qoff);
    hipStream_t s = ctx.stream;
    GS_HIP(hipEventRecord(ctx.ev[0], s));
    k_zerox<<<64, 256, 0, s>>>(dv, words);
    GS_HIP(hipEventRecord(ctx.ev[2], s));
    if (g.n > 0) {
        if (mu) launchx_k<kMu>(ctx, a, L.total, weighted, anchored);
        else launchx_k<kEqui>(ctx, a, L.total, weighted, anchored);
    }
    GS_HIP(hipEventRecord(ctx.ev[3], s));
    GS_HIP(hipMemcpyAsync(hist, dv, sizeof(uint64_t) * ncnt, hipMemcpyDeviceToHost, s));
    GS_HIP(hipMemcpyAsync(ntri, dv + ncnt, 8, hipMemcpyDeviceToHost, s));
    if (weighted) GS_HIP(hipMemcpyAsync(wsum, dv + woff, sizeof(uint64_t) * 2 * ncnt, hipMemcpyDeviceToHost, s));
    GS_HIP(hipEventRecord(ctx.ev[1], s));
    GS_HIP(hipStreamSynchronize(s));
    if (wscale) *wscale = sc;
    float ms = 0, kms = 0;
    GS_HIP(hipEventElapsedTime(&ms, ctx.ev[0], ctx.ev[1]));
    GS_HIP(hipEventElapsedTime(&kms, ctx.ev[2], ctx.ev[3]));
    ctx.t.count_ms = ms;
    ctx.t.kernel_ms = kms;
    ctx.t.kernel_launches = g.n > 0 ? 1 : 0;
    ctx.t.alg_bytes = g.stats_ready ? (uint64_t)(2.5 * (double)g.sum_sq_deg) : 0;
}

}  // namespace gsn

using namespace gsn;

extern "C" {

int gs_count_3pcf_equilateral(gs_ctx *ctx, const gs_graph *g, uint64_t *hist, uint64_t *wsum128, int32_t *wscale,
                              uint64_t *n_triangles, const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !hist || !n_triangles) fail(GS_EINVAL, "null argument");
        if ((wsum128 || wscale) && !(g->flags & GS_WEIGHTED)) fail(GS_EINVAL, "graph has no weights");
        if (g->device != ctx->device) fail(GS_EINVAL, "graph and context on different devices");
        ctx->use();
        int sc = 0;
        count3x_run(*ctx, *g, kEqui, 1, hist, wsum128, &sc, n_triangles, anchors);
        if (wscale) *wscale = sc;
    });
}

int gs_count_3pcf_mu(gs_ctx *ctx, const gs_graph *g, int32_t nmu, uint64_t *hist, uint64_t *wsum128,
                     int32_t *wscale, uint64_t *n_triangles, const gs_anchor_range *anchors) {
    return guarded([&] {
        if (!ctx || !g || !hist || !n_triangles) fail(GS_EINVAL, "null argument");
        if ((wsum128 || wscale) && !(g->flags & GS_WEIGHTED)) fail(GS_EINVAL, "graph has no weights");
        if (g->device != ctx->device) fail(GS_EINVAL, "graph and context on different devices");
        ctx->use();
        int sc = 0;
        count3x_run(*ctx, *g, kMu, nmu, hist, wsum128, &sc, n_triangles, anchors);
        if (wscale) *wscale = sc;
    });
}

}  // extern "C"
