// estimate.hip - estimators on top of the counts (paper Sec. 2.1 signed
// weights, Sec. 3.3 connected 4pCF, Sec. 3.4 the compute_3pcf / compute_4pcf
// interface). Host code only: every tuple is counted by the library's
// kernels through the C ABI; this file normalises weights, forms the
// combined data-minus-random catalogue and divides exact sums.
//
// Weights: data weights are divided by their sum (so they sum to +1), random
// weights by minus theirs (sum -1); sums are taken left to right in index
// order. With these weights the exact per-configuration sum over tuples of
// the combined catalogue (data then randoms) is the Landy-Szalay /
// Szapudi-Szalay numerator (NN for pairs, NNN for triangles, NNNN for
// 4-cliques). The denominators (RR, RRR, RRRR) are the same sums over the
// randoms alone with their weights divided by their (positive) sum. Every
// estimate is numerator / denominator of the two exact sums, each rounded
// once to float64 (0/0 and x/0 follow IEEE: NaN and +-inf).
//
// Connected 4pCF (Sec. 3.3 Eq. 4-5): xi(b) = NN(b) / RR(b) on the same graph
// and bins; for a 6-edge configuration with smallest tuple (b0..b5) (edges
// 01, 02, 03, 12, 13, 23) the disconnected term is
// xi(b0) xi(b5) + xi(b1) xi(b4) + xi(b2) xi(b3) (the three pairings into
// opposite edges), summed in that order. The parity channels are binned by
// a hub's sorted spoke bins; their disconnected term is the RRRR-weighted
// mean of the 6-edge term over the hub contributions that fall in the
// configuration: sum over 6-edge configurations c (ascending) and their
// hubs h (0..3) whose spoke bins sort to T of RRRR6(c) * disc(c), divided by
// the even random sum RRRR(T). It is removed from the even channel only.
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace gsn {
namespace {

// Host double arrays of a catalogue's normalised weights: w_i / S (sign +1)
// or -w_i / S (sign -1), S the left-to-right sum; unit weights if w is null.
void normalised(const gs_catalogue &c, double sign, double *out) {
    double S = 0.0;
    for (int64_t i = 0; i < c.n; ++i) S = S + (c.weights ? c.weights[i] : 1.0);
    if (!(S != 0.0) || !std::isfinite(S)) fail(GS_EINVAL, "catalogue weights must have a finite nonzero sum");
    for (int64_t i = 0; i < c.n; ++i) {
        const double w = c.weights ? c.weights[i] : 1.0;
        out[i] = sign > 0 ? w / S : -(w / S);
    }
}

void check_cat(const gs_catalogue *c, const char *what) {
    if (!c || c->n < 0 || (c->n > 0 && !c->xyz)) fail(GS_EINVAL, std::string("bad ") + what + " catalogue");
}

struct GraphGuard {
    gs_graph *g = nullptr;
    ~GraphGuard() {
        if (g) gs_graph_free(g);
    }
};

void ok(int rc, const char *where) {
    if (rc != GS_OK) fail(rc, std::string(where) + ": " + gs_last_error_detail());
}

// Build the graph of a catalogue with explicit weights.
void build_w(gs_ctx *ctx, const double *xyz, int64_t n, const double *w, const gs_graph_params &p, bool coords,
             GraphGuard &gg) {
    gs_graph_params q = p;
    q.flags = GS_WEIGHTED | (coords ? GS_KEEP_COORDS : 0u) | (p.flags & GS_NONPERIODIC);
    ok(gs_build_graph(ctx, xyz, n, w, &q, &gg.g), "gs_build_graph");
}

// Data then randoms, with the data-minus-random weights.
void combined(const gs_catalogue &d, const gs_catalogue &r, std::vector<double> &xyz, std::vector<double> &w) {
    xyz.resize(3 * (size_t)(d.n + r.n));
    w.resize((size_t)(d.n + r.n));
    if (d.n) memcpy(xyz.data(), d.xyz, sizeof(double) * 3 * d.n);
    if (r.n) memcpy(xyz.data() + 3 * d.n, r.xyz, sizeof(double) * 3 * r.n);
    normalised(d, +1.0, w.data());
    normalised(r, -1.0, w.data() + d.n);
}

double ratio(double a, double b) { return a / b; }

// Exact (lo, hi) sums rounded to float64.
void rounded(const uint64_t *w, size_t n, int scale, double *out) {
    for (size_t k = 0; k < n; ++k) out[k] = sum128_to_double(&w[2 * k], scale);
}

// The sorted spoke bins of hub h of a 6-edge tuple (edges 01,02,03,12,13,23).
void hub_triple(const int t[6], int h, int out[3]) {
    static const int at[4][3] = {{0, 1, 2}, {0, 3, 4}, {1, 3, 5}, {2, 4, 5}};
    int a = t[at[h][0]], b = t[at[h][1]], c = t[at[h][2]];
    if (a > b) std::swap(a, b);
    if (b > c) std::swap(b, c);
    if (a > b) std::swap(a, b);
    out[0] = a;
    out[1] = b;
    out[2] = c;
}

}  // namespace
}  // namespace gsn

using namespace gsn;

extern "C" {

int gs_compute_3pcf(gs_ctx *ctx, const gs_catalogue *data, const gs_catalogue *randoms, const gs_graph_params *p,
                    gs_zeta3 *out) {
    return guarded([&] {
        if (!ctx || !p || !out || !out->zeta) fail(GS_EINVAL, "null argument");
        check_cat(data, "data");
        check_cat(randoms, "random");
        const int nb = p->nbins;
        if (nb < 1 || nb > 255) fail(GS_EINVAL, "nbins must be in 1..255");
        const size_t nc = (size_t)n_configs(nb);
        std::vector<double> xyz, w, wr((size_t)randoms->n);
        combined(*data, *randoms, xyz, w);
        normalised(*randoms, +1.0, wr.data());
        std::vector<uint64_t> h(nc), sN(2 * nc), sR(2 * nc);
        std::vector<double> N(nc), R(nc);
        int32_t scN = 0, scR = 0;
        uint64_t nt = 0;
        {
            GraphGuard gg;
            build_w(ctx, xyz.data(), data->n + randoms->n, w.data(), *p, false, gg);
            ok(gs_count_3pcf(ctx, gg.g, h.data(), sN.data(), N.data(), &scN, &nt, nullptr), "gs_count_3pcf");
        }
        {
            GraphGuard gg;
            build_w(ctx, randoms->xyz, randoms->n, wr.data(), *p, false, gg);
            ok(gs_count_3pcf(ctx, gg.g, h.data(), sR.data(), R.data(), &scR, &nt, nullptr), "gs_count_3pcf");
        }
        for (size_t c = 0; c < nc; ++c) out->zeta[c] = ratio(N[c], R[c]);
        if (out->nnn) memcpy(out->nnn, N.data(), sizeof(double) * nc);
        if (out->rrr) memcpy(out->rrr, R.data(), sizeof(double) * nc);
        if (out->nnn128) memcpy(out->nnn128, sN.data(), sizeof(uint64_t) * 2 * nc);
        if (out->rrr128) memcpy(out->rrr128, sR.data(), sizeof(uint64_t) * 2 * nc);
        out->nnn_scale = scN;
        out->rrr_scale = scR;
    });
}

int gs_compute_4pcf(gs_ctx *ctx, const gs_catalogue *data, const gs_catalogue *randoms, const gs_graph_params *p,
                    gs_zeta4 *out) {
    return guarded([&] {
        if (!ctx || !p || !out) fail(GS_EINVAL, "null argument");
        check_cat(data, "data");
        check_cat(randoms, "random");
        const int nb = p->nbins;
        if (nb < 1 || nb > 255) fail(GS_EINVAL, "nbins must be in 1..255");
        const bool want6 = out->zeta6 || out->zeta6_disc || out->zeta6_conn || out->zeta_even_conn ||
                           out->zeta_even_disc;
        if (want6 && nb > kMaxBins6) fail(GS_EUNSUPPORTED, "6-edge and connected estimates take at most 12 bins");
        const size_t nc = (size_t)n_configs(nb);
        uint32_t n6 = 0;
        if (want6) ok(gs_n_configs6(nb, &n6), "gs_n_configs6");
        std::vector<double> xyz, w, wr((size_t)randoms->n);
        combined(*data, *randoms, xyz, w);
        normalised(*randoms, +1.0, wr.data());

        // numerators on the combined catalogue, denominators on the randoms
        std::vector<uint64_t> e(nc), ps(nc), ng(nc), sN(6 * nc), sR(6 * nc), pr(nb), xN(2 * nb), xR(2 * nb);
        std::vector<uint64_t> h6(n6 ? n6 : 1), s6N(2 * (size_t)n6 + 2), s6R(2 * (size_t)n6 + 2);
        int32_t scN = 0, scR = 0, sc6N = 0, sc6R = 0, scxN = 0, scxR = 0;
        uint64_t ncl = 0;
        for (int pass = 0; pass < 2; ++pass) {
            GraphGuard gg;
            if (pass == 0) build_w(ctx, xyz.data(), data->n + randoms->n, w.data(), *p, true, gg);
            else build_w(ctx, randoms->xyz, randoms->n, wr.data(), *p, true, gg);
            std::vector<uint64_t> &s = pass == 0 ? sN : sR;
            ok(gs_count_4pcf_parity_weighted(ctx, gg.g, e.data(), ps.data(), ng.data(), s.data(),
                                             pass == 0 ? &scN : &scR, &ncl, nullptr),
               "gs_count_4pcf_parity_weighted");
            if (want6) {
                ok(gs_count_4pcf_full(ctx, gg.g, h6.data(), pass == 0 ? s6N.data() : s6R.data(),
                                      pass == 0 ? &sc6N : &sc6R, &ncl, nullptr),
                   "gs_count_4pcf_full");
                ok(gs_pair_sums(ctx, gg.g, pr.data(), pass == 0 ? xN.data() : xR.data(), pass == 0 ? &scxN : &scxR,
                                nullptr),
                   "gs_pair_sums");
            }
        }
        // parity channels: even = every hub contribution, odd = pos - neg
        std::vector<double> evN(nc), evR(nc), odN(nc);
        rounded(sN.data(), nc, scN, evN.data());
        rounded(sR.data(), nc, scR, evR.data());
        for (size_t c = 0; c < nc; ++c) {
            const uint64_t *P = &sN[2 * (nc + c)], *M = &sN[2 * (2 * nc + c)];
            const unsigned __int128 a = ((unsigned __int128)P[1] << 64) | P[0];
            const unsigned __int128 b = ((unsigned __int128)M[1] << 64) | M[0];
            const unsigned __int128 d = a - b;
            const uint64_t dw[2] = {(uint64_t)d, (uint64_t)(d >> 64)};
            odN[c] = sum128_to_double(dw, scN);
        }
        for (size_t c = 0; c < nc; ++c) {
            if (out->zeta_even) out->zeta_even[c] = ratio(evN[c], evR[c]);
            if (out->zeta_odd) out->zeta_odd[c] = ratio(odN[c], evR[c]);
            if (out->nnnn_even) out->nnnn_even[c] = evN[c];
            if (out->nnnn_odd) out->nnnn_odd[c] = odN[c];
            if (out->rrrr_even) out->rrrr_even[c] = evR[c];
        }
        if (!want6) return;

        // internal 2pCF and the 6-edge estimate with its disconnected part
        std::vector<double> NN(nb), RR(nb), xi(nb), z6N(n6), z6R(n6), disc(n6);
        rounded(xN.data(), nb, scxN, NN.data());
        rounded(xR.data(), nb, scxR, RR.data());
        for (int b = 0; b < nb; ++b) xi[b] = ratio(NN[b], RR[b]);
        if (out->xi) memcpy(out->xi, xi.data(), sizeof(double) * nb);
        rounded(s6N.data(), n6, sc6N, z6N.data());
        rounded(s6R.data(), n6, sc6R, z6R.data());
        std::vector<uint32_t> rank((size_t)nb * nb * nb * nb * nb * nb);
        ok(gs_config6_table(nb, rank.data()), "gs_config6_table");
        std::vector<std::array<int, 6>> small(n6);   // smallest tuple of each configuration
        std::vector<char> seen(n6, 0);
        for (uint32_t code = 0; code < rank.size(); ++code) {
            const uint32_t c = rank[code];
            if (seen[c]) continue;   // codes ascend, so the first code of a class is its smallest
            seen[c] = 1;
            uint32_t v = code;
            for (int k = 5; k >= 0; --k) {
                small[c][k] = (int)(v % nb);
                v /= nb;
            }
        }
        for (uint32_t c = 0; c < n6; ++c) {
            const std::array<int, 6> &t = small[c];
            disc[c] = (xi[t[0]] * xi[t[5]] + xi[t[1]] * xi[t[4]]) + xi[t[2]] * xi[t[3]];
            const double z = ratio(z6N[c], z6R[c]);
            if (out->zeta6) out->zeta6[c] = z;
            if (out->zeta6_disc) out->zeta6_disc[c] = disc[c];
            if (out->zeta6_conn) out->zeta6_conn[c] = z - disc[c];
        }
        // disconnected part of the even channel: RRRR-weighted over hubs
        std::vector<double> num(nc, 0.0);
        for (uint32_t c = 0; c < n6; ++c)
            for (int hb = 0; hb < 4; ++hb) {
                int tr[3];
                hub_triple(small[c].data(), hb, tr);
                const size_t idx = (size_t)(rank_a(nb, tr[0]) + rank_b(nb, tr[1]) + tr[2]);
                num[idx] = num[idx] + z6R[c] * disc[c];
            }
        for (size_t c = 0; c < nc; ++c) {
            const double de = ratio(num[c], evR[c]);
            if (out->zeta_even_disc) out->zeta_even_disc[c] = de;
            if (out->zeta_even_conn) out->zeta_even_conn[c] = ratio(evN[c], evR[c]) - de;
        }
    });
}

}  // extern "C"
