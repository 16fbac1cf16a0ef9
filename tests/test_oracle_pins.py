"""Pins of the CPU oracle against things other than itself.

Each test ties the oracle to a fact fixed outside it: configuration counts the
paper prints, hand-derived lattice and chiral-unit closed forms
(tests/golden/), the Poisson closed form for uniform boxes, O(N^3)/O(N^4)
brute force (tests/brute.py), exact reflection/relabelling/translation
symmetries, and exact weighted-sum identities.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import brute

pytestmark = pytest.mark.filterwarnings("ignore")


def _golden(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


# ------------------------------------------------------- configuration index --

@pytest.mark.parametrize("nb", [1, 2, 3, 8, 10, 15, 20, 40])
def test_config_index_is_lexicographic_rank(nb):
    rank = brute.lex_configs(nb)
    assert len(rank) == oracle.n_configs(nb) == math.comb(nb + 2, 3)
    for (a, b, c), r in rank.items():
        assert oracle.config_index(nb, a, b, c) == r


def test_config_counts_printed_in_paper(golden_dir):
    g = _golden(golden_dir, "paper_config_counts.json")
    for nb, count in g["counts"].items():
        assert oracle.n_configs(int(nb)) == count
        assert len(brute.lex_configs(int(nb))) == count


# ------------------------------------------------------------- pair rule -----

def test_bin_rule_half_open_on_exact_edges():
    # rmin 0, rmax 1.5, 6 bins of 0.25: all edges are exact binary fractions
    L = 6.0
    eb = lambda q: oracle.edge_bin(q, L, 0.0, 1.5, 6)
    assert eb(0.0) == 0                      # rmin = 0: coincident points are edges in bin 0
    assert eb(0.0625) == 1                   # d = 0.25 exactly on e_1
    assert eb(np.nextafter(0.0625, 0)) == 0
    assert eb(1.0) == 4                      # d = 1 exactly on e_4 -> upper bin
    assert eb(np.nextafter(1.0, 0)) == 3
    assert eb(2.0) == 5
    assert eb(np.nextafter(2.25, 0)) == 5
    assert eb(2.25) == -1                    # d = rmax is not an edge (strict < rmax)
    # rmin > 0: pairs closer than rmin are not edges
    assert oracle.edge_bin(0.25, L, 0.5, 1.5, 2) == 0
    assert oracle.edge_bin(np.nextafter(0.25, 0), L, 0.5, 1.5, 2) == -1
    assert oracle.edge_bin(1.0, L, 0.5, 1.5, 2) == 1


def test_separation_minimum_image_antisymmetric():
    L = 10.0
    rng_pts = synth.uniform(400, L, 11)
    # include components exactly at +-L/2
    rng_pts[0] = [0.0, 0.0, 0.0]
    rng_pts[1] = [5.0, 5.0, 2.5]
    for a in range(0, 400, 7):
        for b in range(1, 400, 13):
            r_ab, q_ab = oracle.separation(rng_pts[a], rng_pts[b], L)
            r_ba, q_ba = oracle.separation(rng_pts[b], rng_pts[a], L)
            assert np.array_equal(r_ab, -r_ba)
            assert q_ab == q_ba
            assert np.all(np.abs(r_ab) <= 0.5 * L)
    r, _ = oracle.separation(rng_pts[0], rng_pts[1], L)
    assert list(r) == [5.0, 5.0, 2.5]
    r, _ = oracle.separation(rng_pts[1], rng_pts[0], L)
    assert list(r) == [-5.0, -5.0, -2.5]
    r, _ = oracle.separation([0.5, 9.5, 1.0], [9.5, 0.5, 1.0], L)
    assert list(r) == [-1.0, 1.0, 0.0]


def test_invalid_inputs_rejected():
    x = synth.uniform(50, 10.0, 3)
    with pytest.raises(oracle.OracleError):
        oracle.count_3pcf(x, 10.0, 0.0, 5.0, 4)        # rmax >= L/2
    with pytest.raises(oracle.OracleError):
        oracle.count_3pcf(x, 10.0, 2.0, 2.0, 4)        # rmin >= rmax
    with pytest.raises(oracle.OracleError):
        oracle.count_3pcf(x, 10.0, 0.0, 2.0, 0)        # nbins < 1
    with pytest.raises(oracle.OracleError):
        oracle.count_3pcf(x, 10.0, 0.0, 2.0, 256)      # nbins > 255
    y = x.copy()
    y[3, 1] = 10.0
    with pytest.raises(oracle.OracleError):
        oracle.count_3pcf(y, 10.0, 0.0, 2.0, 4)        # coordinate == L
    y[3, 1] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.count_3pcf(y, 10.0, 0.0, 2.0, 4)
    with pytest.raises(oracle.OracleError):
        oracle.count_3pcf(x, 10.0, 0.0, 2.0, 4, weights=np.zeros(50))


# ------------------------------------------------------------ brute force ----

TINY = [
    # (name, xyz, L, rmin, rmax, nb)
    ("uniform_dense", lambda: synth.uniform(260, 10.0, 21), 10.0, 0.0, 2.4, 5),
    ("uniform_rmin", lambda: synth.uniform(240, 10.0, 22), 10.0, 0.7, 2.6, 4),
    ("clustered", lambda: synth.neyman_scott(250, 25, 0.8, 12.0, 23), 12.0, 0.0, 2.0, 6),
    ("single_cell", lambda: synth.uniform(150, 9.0, 24), 9.0, 0.0, 3.9, 3),   # L/rmax < 3: one cell
    ("many_bins", lambda: synth.uniform(200, 8.0, 25), 8.0, 0.0, 2.2, 21),
]


@pytest.mark.parametrize("case", TINY, ids=[c[0] for c in TINY])
def test_oracle_graph_matches_brute_pairs(case):
    _, mk, L, rmin, rmax, nb = case
    x = mk()
    rp, col, b = oracle.graph(x, L, rmin, rmax, nb)
    _, _, adj, bins = brute.pair_matrix(x, L, rmin, rmax, nb)
    for i in range(len(x)):
        js = np.nonzero(adj[i])[0]
        assert np.array_equal(col[rp[i]:rp[i + 1]], js)
        assert np.array_equal(b[rp[i]:rp[i + 1]], bins[i, js])


@pytest.mark.parametrize("case", TINY, ids=[c[0] for c in TINY])
def test_oracle_3pcf_matches_brute_force(case):
    _, mk, L, rmin, rmax, nb = case
    x = mk()
    w = synth.uniform_values(len(x), 0.5, 1.0, 99)
    bh, bcount, bw, bs = brute.triangles(x, L, rmin, rmax, nb, weights=w)
    r = oracle.count_3pcf(x, L, rmin, rmax, nb, weights=w, threads=3)
    assert bcount > 50
    assert r.n_triangles == bcount
    assert np.array_equal(r.hist.astype(np.int64), bh)
    assert r.wscale == bs
    assert r.wsum_int() == bw


@pytest.mark.parametrize("case", TINY[:4], ids=[c[0] for c in TINY[:4]])
def test_oracle_3pcf_anchors_match_brute_force(case):
    _, mk, L, rmin, rmax, nb = case
    x = mk()
    n = len(x)
    parts = [(0, n // 3), (n // 3, n // 2), (n // 2, n)]
    tot = np.zeros(oracle.n_configs(nb), dtype=np.uint64)
    for lo, hi in parts:
        bh, bcount, _, _ = brute.triangles(x, L, rmin, rmax, nb, anchors=(lo, hi))
        r = oracle.count_3pcf(x, L, rmin, rmax, nb, anchors=(lo, hi))
        assert r.n_triangles == bcount
        assert np.array_equal(r.hist.astype(np.int64), bh)
        tot += r.hist
    assert np.array_equal(tot, oracle.count_3pcf(x, L, rmin, rmax, nb).hist)


TINY4 = [
    ("uniform_dense", lambda: synth.uniform(110, 8.0, 31), 8.0, 0.0, 2.6, 4),
    ("clustered", lambda: synth.neyman_scott(110, 22, 0.7, 10.0, 32), 10.0, 0.0, 2.0, 5),
    ("rmin", lambda: synth.uniform(100, 7.0, 33), 7.0, 0.5, 2.5, 3),
]


@pytest.mark.parametrize("case", TINY4, ids=[c[0] for c in TINY4])
def test_oracle_4pcf_parity_matches_brute_force(case):
    _, mk, L, rmin, rmax, nb = case
    x = mk()
    E, P, N, cnt = brute.cliques4(x, L, rmin, rmax, nb)
    r = oracle.count_4pcf_parity(x, L, rmin, rmax, nb, threads=3)
    assert cnt > 20
    assert r.n_cliques == cnt
    assert np.array_equal(r.even.astype(np.int64), E)
    assert np.array_equal(r.pos.astype(np.int64), P)
    assert np.array_equal(r.neg.astype(np.int64), N)
    assert r.pos.sum() + r.neg.sum() > 0


def test_oracle_4pcf_anchor_split():
    x = synth.uniform(110, 8.0, 31)
    full = oracle.count_4pcf_parity(x, 8.0, 0.0, 2.6, 4)
    acc = [np.zeros_like(full.even) for _ in range(3)]
    nk = 0
    for lo, hi in [(0, 20), (20, 77), (77, 110)]:
        r = oracle.count_4pcf_parity(x, 8.0, 0.0, 2.6, 4, anchors=(lo, hi))
        E, P, N, cnt = brute.cliques4(x, 8.0, 0.0, 2.6, 4, anchors=(lo, hi))
        assert r.n_cliques == cnt and np.array_equal(r.even.astype(np.int64), E)
        assert np.array_equal(r.pos.astype(np.int64), P) and np.array_equal(r.neg.astype(np.int64), N)
        for a, v in zip(acc, (r.even, r.pos, r.neg)):
            a += v
        nk += r.n_cliques
    assert nk == full.n_cliques
    assert np.array_equal(acc[0], full.even)
    assert np.array_equal(acc[1], full.pos)
    assert np.array_equal(acc[2], full.neg)


# ------------------------------------------------------------ lattice --------

def _lattice(g, shift=(0.0, 0.0, 0.0)):
    m = g["sites_per_axis"]
    a = np.arange(m, dtype=np.float64)
    X, Y, Z = np.meshgrid(a, a, a, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return np.mod(xyz + np.array(shift), g["box"])


@pytest.mark.parametrize("shift", [(0.0, 0.0, 0.0), (0.25, 0.5, 0.125), (5.5, 0.75, 3.0)])
def test_lattice_closed_forms(golden_dir, shift):
    g = _golden(golden_dir, "lattice_sc.json")
    x = _lattice(g, shift)
    nsite = len(x)
    L, rmin, rmax, nb = g["box"], g["rmin"], g["rmax"], g["nbins"]
    rp, col, b = oracle.graph(x, L, rmin, rmax, nb)
    assert np.all(np.diff(rp) == 18)
    pair = np.bincount(b, minlength=nb)
    for k, v in g["edges_per_site_by_bin"].items():
        assert pair[int(k)] == v * nsite
    assert pair.sum() == 18 * nsite
    r3 = oracle.count_3pcf(x, L, rmin, rmax, nb)
    exp3 = np.zeros(oracle.n_configs(nb), dtype=np.uint64)
    for key, v in g["triangles_per_site"].items():
        exp3[oracle.config_index(nb, *map(int, key.split(",")))] = v * nsite
    assert np.array_equal(r3.hist, exp3)
    assert r3.n_triangles == 20 * nsite
    r4 = oracle.count_4pcf_parity(x, L, rmin, rmax, nb)
    assert r4.n_cliques == g["cliques_per_site"] * nsite
    exp4 = np.zeros(oracle.n_configs(nb), dtype=np.uint64)
    for key, v in g["hub_contributions_per_site"].items():
        exp4[oracle.config_index(nb, *map(int, key.split(",")))] = v * nsite
    assert np.array_equal(r4.even, exp4)
    assert r4.pos.sum() == 0 and r4.neg.sum() == 0


# -------------------------------------------------------- chiral injection ---

def _chiral_catalogue(g, handed, spacing=8.0, origin=(2.25, 2.5, 2.75)):
    """Units on a grid `spacing` apart (> rmax + unit size); handed[u] = +1
    original, -1 mirrored (x offsets negated)."""
    L = g["box"]
    per = int(L // spacing)
    pts = []
    off = g["offsets"]
    for u, h in enumerate(handed):
        a, bb, c = u // (per * per), (u // per) % per, u % per
        O = np.array([a * spacing, bb * spacing, c * spacing]) + np.array(origin)
        pts.append(O)
        for name in ("A", "B", "C"):
            v = np.array(off[name], dtype=np.float64)
            v[0] *= h
            pts.append(O + v)
    return np.mod(np.array(pts), L)


def test_chiral_unit_hand_derived_signs(golden_dir):
    g = _golden(golden_dir, "chiral_unit.json")
    L, rmin, rmax, nb = g["box"], g["rmin"], g["rmax"], g["nbins"]
    idx = lambda t: oracle.config_index(nb, *t)
    for h in (+1, -1):
        x = _chiral_catalogue(g, [h])
        r = oracle.count_4pcf_parity(x, L, rmin, rmax, nb)
        assert r.n_cliques == 1
        exp_pos = np.zeros(oracle.n_configs(nb), dtype=np.int64)
        for t in g["pos_configs"]:
            exp_pos[idx(t)] += 1
        for t in g["neg_configs"]:
            exp_pos[idx(t)] -= 1
        assert np.array_equal(r.odd, h * exp_pos)
        assert r.even.sum() == 4
        r3 = oracle.count_3pcf(x, L, rmin, rmax, nb)
        exp3 = np.zeros(oracle.n_configs(nb), dtype=np.uint64)
        for t in g["triangle_configs"]:
            exp3[idx(t)] += 1
        assert np.array_equal(r3.hist, exp3)


@pytest.mark.parametrize("n_left,n_right", [(300, 200), (250, 250), (500, 0)])
def test_chiral_injection_count_level_prediction(golden_dir, n_left, n_right):
    """Odd channel = (N_L - N_R) x single-unit pattern (paper Sec. 4.9)."""
    g = _golden(golden_dir, "chiral_unit.json")
    L, rmin, rmax, nb = g["box"], g["rmin"], g["rmax"], g["nbins"]
    unit = oracle.count_4pcf_parity(_chiral_catalogue(g, [1]), L, rmin, rmax, nb)
    handed = [1] * n_left + [-1] * n_right
    order = synth.permutation(len(handed), 7)
    handed = [handed[i] for i in order]
    x = _chiral_catalogue(g, handed)
    r = oracle.count_4pcf_parity(x, L, rmin, rmax, nb)
    assert r.n_cliques == n_left + n_right
    assert np.array_equal(r.odd, (n_left - n_right) * unit.odd)
    assert np.array_equal(r.even, (n_left + n_right) * unit.even)


# --------------------------------------------------- exact symmetries ---------

def test_reflection_swaps_parity_channels_exactly():
    L = 16.0
    x = synth.dyadic_uniform(700, L, 41)
    y = x.copy()
    y[:, 0] = np.mod(L - y[:, 0], L)         # exact on the dyadic grid
    a = oracle.count_4pcf_parity(x, L, 0.0, 2.2, 4)
    b = oracle.count_4pcf_parity(y, L, 0.0, 2.2, 4)
    assert a.n_cliques > 100
    assert np.array_equal(a.even, b.even)
    assert np.array_equal(a.pos, b.neg)
    assert np.array_equal(a.neg, b.pos)
    assert a.pos.sum() > 0


def test_relabelling_invariance():
    L = 12.0
    x = synth.neyman_scott(900, 30, 1.0, L, 42)
    w = synth.uniform_values(900, 0.5, 1.0, 43)
    p = synth.permutation(900, 44)
    a3 = oracle.count_3pcf(x, L, 0.0, 2.0, 5, weights=w)
    b3 = oracle.count_3pcf(x[p], L, 0.0, 2.0, 5, weights=w[p])
    assert np.array_equal(a3.hist, b3.hist) and np.array_equal(a3.wsum, b3.wsum)
    a4 = oracle.count_4pcf_parity(x, L, 0.0, 1.6, 4)
    b4 = oracle.count_4pcf_parity(x[p], L, 0.0, 1.6, 4)
    assert np.array_equal(a4.even, b4.even) and np.array_equal(a4.pos, b4.pos)
    assert np.array_equal(a4.neg, b4.neg)


def test_dyadic_translation_invariance():
    L = 16.0
    x = synth.dyadic_uniform(800, L, 45)
    y = np.mod(x + np.array([3.25, 15.5, 7.125]), L)
    a3 = oracle.count_3pcf(x, L, 0.0, 2.4, 6)
    b3 = oracle.count_3pcf(y, L, 0.0, 2.4, 6)
    assert np.array_equal(a3.hist, b3.hist)
    a4 = oracle.count_4pcf_parity(x, L, 0.0, 2.2, 4)
    b4 = oracle.count_4pcf_parity(y, L, 0.0, 2.2, 4)
    assert np.array_equal(a4.even, b4.even) and np.array_equal(a4.pos, b4.pos)
    assert np.array_equal(a4.neg, b4.neg)


# --------------------------------------------------------- weighted sums -----

def test_weighted_identities():
    L = 12.0
    x = synth.uniform(1500, L, 51)
    n = len(x)
    r1 = oracle.count_3pcf(x, L, 0.0, 2.0, 6, weights=np.ones(n))
    assert r1.wscale == 52
    assert r1.wsum_int() == [int(h) << 52 for h in r1.hist]
    assert np.array_equal(r1.whist(), r1.hist.astype(np.float64))
    w = synth.uniform_values(n, 0.5, 1.0, 52)
    ra = oracle.count_3pcf(x, L, 0.0, 2.0, 6, weights=w)
    rb = oracle.count_3pcf(x, L, 0.0, 2.0, 6, weights=2.0 * w)
    assert ra.wscale == 55 and rb.wscale == 52
    assert ra.wsum_int() == rb.wsum_int()          # same integers, scale 2^3 larger
    assert np.array_equal(rb.whist(), 8.0 * ra.whist())
    # against a naive extended-precision sum of the same products
    _, _, adj, bins = brute.pair_matrix(x, L, 0.0, 2.0, 6)
    naive = np.zeros(oracle.n_configs(6), dtype=np.longdouble)
    rank = brute.lex_configs(6)
    ii, jj = np.nonzero(np.triu(adj, 1))
    for i, j in zip(ii, jj):
        for k in np.nonzero(adj[i, j + 1:] & adj[j, j + 1:])[0] + j + 1:
            s = sorted((w[i], w[j], w[k]))
            naive[rank[tuple(sorted((bins[i, j], bins[i, k], bins[j, k])))]] += np.longdouble((s[0] * s[1]) * s[2])
    got = ra.whist()
    nz = naive > 0
    assert np.all(np.abs(got[nz] - naive[nz].astype(np.float64)) <= 1e-12 * naive[nz].astype(np.float64))


# ------------------------------------------------ Poisson closed forms ------

def _expected_config_fraction(L, rmax, nb, h_steps=240):
    """For three uniform points in a periodic box with rmax <= L/4: expected
    fraction of labelled triples in each sorted-bin configuration. Side-length
    density 8 pi^2 r1 r2 r3 / L^6 on the triangle-inequality region; the r3
    integral is done in closed form, (r1, r2) by a midpoint rule."""
    D = rmax / nb
    rank = brute.lex_configs(nb)
    out = np.zeros(len(rank))
    u = (np.arange(h_steps) + 0.5) / h_steps * D
    for b1 in range(nb):
        r1 = b1 * D + u
        for b2 in range(nb):
            r2 = b2 * D + u
            R1, R2 = np.meshgrid(r1, r2, indexing="ij")
            for b3 in range(nb):
                lo = np.maximum(b3 * D, np.abs(R1 - R2))
                hi = np.minimum((b3 + 1) * D, R1 + R2)
                inner = np.where(hi > lo, 0.5 * (hi * hi - lo * lo), 0.0)
                val = 8 * math.pi ** 2 * np.sum(R1 * R2 * inner) * (D / h_steps) ** 2 / L ** 6
                out[rank[tuple(sorted((b1, b2, b3)))]] += val
    return out


def test_poisson_closed_form_total_and_bins():
    """Mean over 20 uniform seeds against E[n_T] = C(N,3) (5 pi^2/6) (R/L)^6
    and the per-configuration integrals, within 4 standard errors."""
    N, L, R, nb = 3000, 100.0, 10.0, 4
    frac = _expected_config_fraction(L, R, nb)
    ntrip = N * (N - 1) * (N - 2) / 6
    assert abs(frac.sum() - 5 * math.pi ** 2 / 6 * (R / L) ** 6) < 1e-4 * frac.sum()
    hs, ts = [], []
    for seed in range(20):
        r = oracle.count_3pcf(synth.uniform(N, L, 1000 + seed), L, 0.0, R, nb)
        hs.append(r.hist.astype(np.float64))
        ts.append(r.n_triangles)
    hs = np.array(hs)
    ts = np.array(ts, dtype=np.float64)
    exp_total = ntrip * 5 * math.pi ** 2 / 6 * (R / L) ** 6
    se = ts.std(ddof=1) / math.sqrt(len(ts))
    assert abs(ts.mean() - exp_total) < 4 * se, (ts.mean(), exp_total, se)
    m = hs.mean(axis=0)
    s = hs.std(axis=0, ddof=1) / math.sqrt(len(hs))
    e = ntrip * frac
    big = e > 50
    z = np.abs(m[big] - e[big]) / np.maximum(s[big], 1e-9)
    assert z.max() < 4.5, z


def test_sum_over_bins_invariants():
    w = synth.workload("uniform_3pcf", volume_fraction=0.125)
    r = oracle.count_3pcf(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    assert int(r.hist.sum()) == r.n_triangles
    r4 = oracle.count_4pcf_parity(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    assert int(r4.even.sum()) == 4 * r4.n_cliques
    assert np.all(r4.pos + r4.neg <= r4.even)
    # parity-symmetric field: odd channel consistent with zero
    tot = float(r4.pos.sum() + r4.neg.sum())
    assert abs(float(r4.pos.sum()) - float(r4.neg.sum())) < 4 * math.sqrt(max(tot, 1.0)) * 2


# ------------------------------------------------- degenerate-volume rule ----
# Hand-derived units (tests/golden/degenerate_units.json): a scalene coplanar
# unit (V = 0 exactly, no length ties), the same unit lifted off its plane by
# dyadic eps on both sides of each hub's 1e-9 normalised-volume limit, and a
# coincident pair (a zero-length spoke, decided by the rule's '<=').

from tests import units as _units  # noqa: E402

_COPLANAR = ["O", "A", "B", "C"]


def _degenerate_case(golden_dir, k_exp, n_units=5):
    g = _golden(golden_dir, "degenerate_units.json")
    L, rmin, rmax, nb = g["box"], g["rmin"], g["rmax"], g["nbins"]
    lifted = g["lifted"]
    if k_exp is None:
        off, signs = _units.offsets(g["coplanar"], _COPLANAR), {}
    else:
        eps = float(np.sign(k_exp)) * 2.0 ** (-abs(k_exp))
        off = _units.offsets(g["coplanar"], _COPLANAR, lift=lifted["lift_vertex"], eps=eps)
        signed = lifted["signed_hubs"][str(-abs(k_exp))]
        signs = {h: int(np.sign(k_exp)) * lifted["signs_eps_positive"][h] for h in signed}
    x = _units.place([off] * n_units, L)
    even, odd = _units.expected_parity(nb, oracle.config_index, g["coplanar"]["hub_configs"], signs)
    tri = _units.expected_triangles(nb, oracle.config_index, g["coplanar"]["triangle_configs"])
    return x, (L, rmin, rmax, nb), n_units * even, n_units * odd, n_units * tri


@pytest.mark.parametrize("k_exp", [None, -30, 30, -29, 29, -28, 28],
                         ids=["coplanar", "eps-2^-30", "eps+2^-30", "eps-2^-29", "eps+2^-29",
                              "eps-2^-28", "eps+2^-28"])
def test_degenerate_rule_coplanar_and_lifted_units(golden_dir, k_exp):
    x, (L, rmin, rmax, nb), even, odd, tri = _degenerate_case(golden_dir, k_exp)
    r = oracle.count_4pcf_parity(x, L, rmin, rmax, nb)
    assert r.n_cliques == 5
    assert np.array_equal(r.even.astype(np.int64), even)
    assert np.array_equal(r.odd, odd)
    # every non-zero odd entry is a single signed hub, never both channels
    assert int(r.pos.sum() + r.neg.sum()) == int(np.abs(odd).sum())
    r3 = oracle.count_3pcf(x, L, rmin, rmax, nb)
    assert np.array_equal(r3.hist.astype(np.int64), tri)


def test_degenerate_rule_zero_length_spoke(golden_dir):
    g = _golden(golden_dir, "degenerate_units.json")
    L, rmin, rmax, nb = g["box"], g["rmin"], g["rmax"], g["nbins"]
    c = g["coincident"]
    x = _units.place([_units.offsets(c, ["P", "Q", "X", "Y"])] * 4, L)
    even, odd = _units.expected_parity(nb, oracle.config_index, c["hub_configs"], {})
    r = oracle.count_4pcf_parity(x, L, rmin, rmax, nb)
    assert r.n_cliques == 4
    assert np.array_equal(r.even.astype(np.int64), 4 * even)
    assert r.pos.sum() == 0 and r.neg.sum() == 0
    r3 = oracle.count_3pcf(x, L, rmin, rmax, nb)
    assert np.array_equal(r3.hist.astype(np.int64),
                          4 * _units.expected_triangles(nb, oracle.config_index, c["triangle_configs"]))


# ------------------------------------------------------ 6-edge 4pCF (D8) -----

@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 6, 8])
def test_six_edge_configuration_count_is_burnside(nb):
    # edge colourings of K4 up to relabelling: (k^6 + 9 k^4 + 14 k^2) / 24
    assert oracle.n_configs6(nb) == (nb ** 6 + 9 * nb ** 4 + 14 * nb ** 2) // 24


@pytest.mark.parametrize("nb", [1, 2, 3, 4])
def test_six_edge_configuration_rank_is_lexicographic(nb):
    rank = brute.configs6(nb)
    assert len(rank) == oracle.n_configs6(nb)
    for t, r in rank.items():
        assert oracle.config6(nb, r) == t


def test_six_edge_counts_printed_in_paper(golden_dir):
    g = _golden(golden_dir, "paper_config_counts.json")["six_edge"]
    nb = g["nbins"]
    assert oracle.n_configs6(nb) == g["configurations"]
    w = (g["rmax"] - g["rmin"]) / nb
    cen = [g["rmin"] + (k + 0.5) * w for k in range(nb)]
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    realizable = 0
    for idx in range(g["configurations"]):
        t = oracle.config6(nb, idx)
        m = np.ones((5, 5))
        m[0, 0] = 0.0
        d = np.zeros((4, 4))
        for (a, b), k in zip(edges, t):
            d[a, b] = d[b, a] = cen[k] ** 2
        m[1:, 1:] = d
        realizable += np.linalg.det(m) > 0      # 288 V^2 > 0
    assert realizable == g["realizable"]


@pytest.mark.parametrize("case", TINY4, ids=[c[0] for c in TINY4])
def test_oracle_4pcf_full_matches_brute_force(case):
    _, mk, L, rmin, rmax, nb = case
    x = mk()
    H, cnt = brute.cliques4_six(x, L, rmin, rmax, nb)
    r = oracle.count_4pcf_full(x, L, rmin, rmax, nb, threads=3)
    assert cnt > 20 and r.n_cliques == cnt
    assert np.array_equal(r.hist.astype(np.int64), H)
    assert r.n_cliques == oracle.count_4pcf_parity(x, L, rmin, rmax, nb).n_cliques


def test_oracle_4pcf_full_anchor_split():
    x = synth.neyman_scott(110, 22, 0.7, 10.0, 32)
    full = oracle.count_4pcf_full(x, 10.0, 0.0, 2.0, 5)
    acc = np.zeros_like(full.hist)
    for lo, hi in [(0, 30), (30, 31), (31, 110)]:
        r = oracle.count_4pcf_full(x, 10.0, 0.0, 2.0, 5, anchors=(lo, hi))
        H, cnt = brute.cliques4_six(x, 10.0, 0.0, 2.0, 5, anchors=(lo, hi))
        assert r.n_cliques == cnt and np.array_equal(r.hist.astype(np.int64), H)
        acc += r.hist
    assert np.array_equal(acc, full.hist)


@pytest.mark.parametrize("shift", [(0.0, 0.0, 0.0), (0.25, 0.5, 0.125)])
def test_lattice_six_edge_closed_form(golden_dir, shift):
    g = _golden(golden_dir, "lattice_sc.json")
    x = _lattice(g, shift)
    nb = g["nbins"]
    r = oracle.count_4pcf_full(x, g["box"], g["rmin"], g["rmax"], nb)
    rank = brute.configs6(nb)
    exp = np.zeros(oracle.n_configs6(nb), dtype=np.int64)
    for key, v in g["six_edge_configs_per_site"].items():
        exp[rank[tuple(map(int, key.split(",")))]] = v * len(x)
    assert r.n_cliques == g["cliques_per_site"] * len(x)
    assert np.array_equal(r.hist.astype(np.int64), exp)


def test_six_edge_invariant_under_relabelling_and_reflection():
    L = 16.0
    x = synth.dyadic_uniform(700, L, 41)
    p = synth.permutation(len(x), 46)
    y = x.copy()
    y[:, 0] = np.mod(L - y[:, 0], L)
    a = oracle.count_4pcf_full(x, L, 0.0, 2.2, 4)
    assert a.n_cliques > 100
    assert np.array_equal(a.hist, oracle.count_4pcf_full(x[p], L, 0.0, 2.2, 4).hist)
    assert np.array_equal(a.hist, oracle.count_4pcf_full(y, L, 0.0, 2.2, 4).hist)


# --------------------------------------------- signed weights (Sec. 2.1) -----

def _signed_weights(n, seed, frac_neg=0.5):
    """Data weights U(0.5,1.5) and random weights -U(0.5,1.5)/2 (the signed
    data-minus-random weights of the estimator, before normalisation)."""
    w = synth.uniform_values(n, 0.5, 1.0, seed)
    neg = synth.uniform_values(n, 0.0, 1.0, seed + 1) < frac_neg
    return np.where(neg, -0.5 * w, w)


@pytest.mark.parametrize("case", TINY[:3], ids=[c[0] for c in TINY[:3]])
def test_oracle_signed_weighted_3pcf_matches_brute_force(case):
    _, mk, L, rmin, rmax, nb = case
    x = mk()
    w = _signed_weights(len(x), 201)
    bh, bcount, bw, bs = brute.triangles(x, L, rmin, rmax, nb, weights=w)
    r = oracle.count_3pcf(x, L, rmin, rmax, nb, weights=w, threads=3)
    assert r.n_triangles == bcount and r.wscale == bs
    assert r.wsum_int() == bw
    assert min(bw) < 0 < max(bw)


@pytest.mark.parametrize("case", TINY[:3], ids=[c[0] for c in TINY[:3]])
def test_oracle_weighted_pairs_match_brute_force(case):
    _, mk, L, rmin, rmax, nb = case
    x = mk()
    w = _signed_weights(len(x), 202)
    cnt, ws, s = brute.pairs_weighted(x, L, rmin, rmax, nb, w)
    r = oracle.pair_sums(x, L, rmin, rmax, nb, weights=w)
    assert np.array_equal(r.pairs.astype(np.int64), cnt)
    assert r.wscale == s and r.wsum_int() == ws
    rp, col, b = oracle.graph(x, L, rmin, rmax, nb)
    assert np.array_equal(np.bincount(b, minlength=nb), 2 * cnt)


@pytest.mark.parametrize("case", TINY4[:2], ids=[c[0] for c in TINY4[:2]])
def test_oracle_weighted_4cliques_match_brute_force(case):
    _, mk, L, rmin, rmax, nb = case
    x = mk()
    w = _signed_weights(len(x), 203)
    W6, WE, WP, WN, s = brute.cliques4_weighted(x, L, rmin, rmax, nb, w)
    r6 = oracle.count_4pcf_full(x, L, rmin, rmax, nb, weights=w)
    assert r6.wscale == s and r6.wsum_int() == W6
    r4 = oracle.count_4pcf_parity(x, L, rmin, rmax, nb, weights=w)
    assert r4.wscale == s
    assert r4.wsum_int(0) == WE and r4.wsum_int(1) == WP and r4.wsum_int(2) == WN
    assert np.array_equal(r6.hist, oracle.count_4pcf_full(x, L, rmin, rmax, nb).hist)


def test_signed_weight_identities():
    """Weights all -1: products of k weights are (-1)^k, so every sum is
    (-1)^k times the count in units of 2^52; flipping every sign negates the
    triangle sums and leaves pair and 4-clique sums unchanged."""
    L = 10.0
    x = synth.uniform(300, L, 61)
    n = len(x)
    m1 = -np.ones(n)
    r3 = oracle.count_3pcf(x, L, 0.0, 2.4, 5, weights=m1)
    assert r3.wsum_int() == [-(int(h) << 52) for h in r3.hist]
    r2 = oracle.pair_sums(x, L, 0.0, 2.4, 5, weights=m1)
    assert r2.wsum_int() == [int(c) << 52 for c in r2.pairs]
    r6 = oracle.count_4pcf_full(x, L, 0.0, 2.4, 4, weights=m1)
    assert r6.wsum_int() == [int(c) << 52 for c in r6.hist]
    w = _signed_weights(n, 62)
    a3 = oracle.count_3pcf(x, L, 0.0, 2.4, 5, weights=w)
    b3 = oracle.count_3pcf(x, L, 0.0, 2.4, 5, weights=-w)
    assert b3.wsum_int() == [-v for v in a3.wsum_int()]
    a6 = oracle.count_4pcf_full(x, L, 0.0, 2.4, 4, weights=w)
    b6 = oracle.count_4pcf_full(x, L, 0.0, 2.4, 4, weights=-w)
    assert a6.wsum_int() == b6.wsum_int()
    a4 = oracle.count_4pcf_parity(x, L, 0.0, 2.4, 4, weights=w)
    assert sum(a4.wsum_int(0)) == 4 * sum(a6.wsum_int())


# ----------------------------------------------------------- mu binning ----
# Hand-derived units: one triangle each, its normal n fixed by construction
# (edge vectors u = p1 - p0, v = p2 - p0 on a dyadic grid, so every
# separation and product below is exact).

def _mu_unit(u, v, lam=0.25, L=16.0):
    p0 = np.array([4.0, 5.0, 6.0])
    return np.array([p0, p0 + lam * np.asarray(u, float), p0 + lam * np.asarray(v, float)])


@pytest.mark.parametrize("u,v,nmu,want", [
    ((1, 0, 0), (0, 1, 0), 4, 3),     # normal along z: mu = 1, the last bin
    ((1, 0, 0), (0, 0, 1), 4, 0),     # normal along y: mu = 0
    ((1, 0, 0), (0, 1, -1), 4, 2),    # n = (0, 1, 1): mu = 0.7071, bin [0.5, 0.75)
    ((0, 1, 0), (3, 0, -4), 5, 3),    # n = (-4, 0, -3): mu = 0.6 exactly, on the edge of bin 3 (half open)
    ((0, 1, 0), (-4, 0, 3), 5, 4),    # n = (3, 0, 4): mu = 0.8 exactly, the edge of bin 4
    ((1, 1, 1), (2, 2, 2), 3, 0),     # collinear: no plane, bin 0
])
def test_mu_bin_hand_derived_units(u, v, nmu, want):
    x = _mu_unit(u, v)
    full = oracle.count_3pcf(x, 16.0, 0.0, 2.0, 4)
    got = oracle.count_3pcf_mu(x, 16.0, 0.0, 2.0, 4, nmu)
    assert got.n_triangles == full.n_triangles == 1
    h = got.hist.reshape(-1, nmu)
    c = int(np.nonzero(full.hist)[0][0])
    assert h[c, want] == 1 and int(h.sum()) == 1


def test_mu_marginal_and_symmetries():
    """Summing over mu gives the 3pCF; mu is unchanged by a reflection of z
    and by a quarter turn about the line of sight (dyadic grid: exact), and
    it is the z axis that matters (an x-y swap keeps it, an x-z swap does not)."""
    L = 16.0
    x = synth.dyadic_uniform(2500, L, 77)
    nmu = 6
    base = oracle.count_3pcf_mu(x, L, 0.0, 1.4, 5, nmu)
    full = oracle.count_3pcf(x, L, 0.0, 1.4, 5)
    assert np.array_equal(base.hist.reshape(-1, nmu).sum(axis=1), full.hist)
    zr = x.copy()
    zr[:, 2] = np.mod(L - zr[:, 2], L)
    assert np.array_equal(oracle.count_3pcf_mu(zr, L, 0.0, 1.4, 5, nmu).hist, base.hist)
    rot = np.stack([np.mod(L - x[:, 1], L), x[:, 0], x[:, 2]], axis=1)
    assert np.array_equal(oracle.count_3pcf_mu(rot, L, 0.0, 1.4, 5, nmu).hist, base.hist)
    sw = x[:, [2, 1, 0]].copy()
    assert not np.array_equal(oracle.count_3pcf_mu(sw, L, 0.0, 1.4, 5, nmu).hist, base.hist)


def test_mu_isotropic_uniform_bins():
    """Uniform points: plane normals are isotropic, so mu = |cos| of the
    normal's angle to z is uniform on [0, 1]: equal counts per mu bin within
    a few standard errors."""
    x = synth.uniform(20000, 60.0, 78)
    nmu = 5
    h = oracle.count_3pcf_mu(x, 60.0, 0.0, 3.0, 3, nmu).hist.reshape(-1, nmu).sum(axis=0).astype(float)
    tot = h.sum()
    exp = tot / nmu
    # triangles are not independent (they share points): allow 6 sigma of the
    # multinomial spread
    assert np.all(np.abs(h - exp) < 6 * math.sqrt(exp))


@pytest.mark.parametrize("case", [("uniform", 150, 6.0, 1.8, 4, 5), ("clustered", 160, 8.0, 2.0, 3, 7)])
def test_oracle_mu_matches_brute_force(case):
    name, n, L, rmax, nb, nmu = case
    x = synth.uniform(n, L, 91) if name == "uniform" else synth.neyman_scott(n, 20, 0.6, L, 92)
    got = oracle.count_3pcf_mu(x, L, 0.0, rmax, nb, nmu)
    assert np.array_equal(got.hist.astype(np.int64), brute.triangles_mu(x, L, 0.0, rmax, nb, nmu))


# ------------------------------------------------------ survey geometry ----

@pytest.mark.parametrize("case", [("uniform", 150, 6.0, 1.8, 4), ("clustered", 140, 8.0, 2.5, 3),
                                  ("rmax_beyond_half_box", 60, 4.0, 3.0, 5)])
def test_nonperiodic_matches_brute_force(case):
    """Survey geometry (no wrap): triangles, parity 4-cliques, 6-edge
    cliques and mu-binned triangles against brute force with plain
    differences; rmax may exceed half the box."""
    name, n, L, rmax, nb = case
    x = synth.uniform(n, L, 93) if name != "clustered" else synth.neyman_scott(n, 20, 0.6, L, 94)
    h, nt, _, _ = brute.triangles(x, -L, 0.0, rmax, nb)
    r = oracle.count_3pcf(x, L, 0.0, rmax, nb, periodic=False)
    assert r.n_triangles == nt and np.array_equal(r.hist.astype(np.int64), h)
    e, p, m, nk = brute.cliques4(x, -L, 0.0, rmax, nb)[:4]
    r4 = oracle.count_4pcf_parity(x, L, 0.0, rmax, nb, periodic=False)
    assert r4.n_cliques == nk
    assert np.array_equal(r4.even.astype(np.int64), e) and np.array_equal(r4.pos.astype(np.int64), p)
    assert np.array_equal(r4.neg.astype(np.int64), m)
    mu = oracle.count_3pcf_mu(x, L, 0.0, rmax, nb, 4, periodic=False)
    assert np.array_equal(mu.hist.astype(np.int64), brute.triangles_mu(x, -L, 0.0, rmax, nb, 4))


def test_nonperiodic_no_wrap_across_faces():
    """Two points 0.2 apart across a face: one edge in the periodic box, none
    without wrap; a catalogue far from every face counts the same either way."""
    L = 10.0
    x = np.array([[0.1, 5.0, 5.0], [9.9, 5.0, 5.0]])
    assert oracle.pair_sums(x, L, 0.0, 1.0, 2).pairs.sum() == 1
    assert oracle.pair_sums(x, L, 0.0, 1.0, 2, periodic=False).pairs.sum() == 0
    y = 2.5 + synth.uniform(3000, 5.0, 95)      # inside [2.5, 7.5): at least rmax from the faces
    a = oracle.count_3pcf(y, L, 0.0, 1.2, 4)
    b = oracle.count_3pcf(y, L, 0.0, 1.2, 4, periodic=False)
    assert np.array_equal(a.hist, b.hist) and a.n_triangles == b.n_triangles > 0


def test_nonperiodic_all_pairs_when_rmax_exceeds_diagonal():
    """rmax beyond the cube's diagonal: every pair is an edge, every triple a
    triangle: C(N, 3) triangles and C(N, 4) 4-cliques."""
    x = synth.uniform(40, 1.0, 96)
    r = oracle.count_3pcf(x, 1.0, 0.0, 2.0, 3, periodic=False)
    assert r.n_triangles == 40 * 39 * 38 // 6
    r4 = oracle.count_4pcf_parity(x, 1.0, 0.0, 2.0, 3, periodic=False)
    assert r4.n_cliques == 40 * 39 * 38 * 37 // 24


# ---------------------------------------------------- direction pixels ----

@pytest.mark.parametrize("r,want", [
    ((1.0, 0.0, 0.0), 28),      # octant 0; a = 1 -> i = 7 (capped); |y|+|z| = 0 -> j = 0
    ((-1.0, 0.0, 0.0), 156),    # x < 0: octant 4 -> 128 + 28
    ((0.0, 0.0, 1.0), 0),       # a = 0, t = 0
    ((1.0, 1.0, 1.0), 10),      # a = 1/3 -> i = 2; t = 1/2 -> j = 2
    ((0.0, -2.0, 0.0), 67),     # y < 0: octant 2 -> 64; a = 0; t = 1 -> j = 3 (capped)
    ((3.0, 1.0, 0.0), 27),      # a = 3/4 -> i = 6; t = 1 -> j = 3
    ((1.0, 0.0, -1.0), 48),     # z < 0: octant 1 -> 32; a = 1/2 -> i = 4; t = 0 -> j = 0
])
def test_pixel_of_hand_derived(r, want):
    assert oracle.pixel_of(r) == want


def test_pixel_centre_hand_derived():
    # pixel 10: a_c = 2.5/8 = 0.3125, t_c = 2.5/4 = 0.625 ->
    # v = (0.3125, 0.6875*0.625, 0.6875*0.375) = (0.3125, 0.4296875, 0.2578125)
    v = np.array([0.3125, 0.4296875, 0.2578125])
    u = oracle.pixel_centre(10)
    assert np.allclose(u, v / np.linalg.norm(v), rtol=0, atol=1e-15)
    # pixel 170 = octant 5 (x < 0, z < 0), i = 2, j = 2: the mirror of 10 in x and z
    w = oracle.pixel_centre(5 * 32 + 10)
    assert np.array_equal(w, u * np.array([-1.0, 1.0, -1.0]))


def test_pixel_parity_repeated_pixel_is_degenerate():
    """Hub O with spokes (1,0,0) and (1,0,0.001) in one pixel: their centre
    directions coincide, the cross product is exactly zero, the hub takes no
    odd weight; the clique's other hubs still count in even."""
    x = np.array([[2.0, 2.0, 2.0], [3.0, 2.0, 2.0], [3.0, 2.0, 2.001], [2.0, 3.0, 2.0]])
    assert oracle.pixel_of(x[1] - x[0]) == oracle.pixel_of(x[2] - x[0]) == 28
    r = oracle.count_4pcf_pixel(x, 8.0, 0.0, 2.0, 2)
    assert r.n_cliques == 1 and int(r.even.sum()) == 4
    # hub O (index 0): spokes in index order to 1, 2, 3; u1 = u2 -> V = 0
    e, p, m, _ = brute.cliques4_pixel(x, 8.0, 0.0, 2.0, 2)
    assert np.array_equal(r.pos.astype(np.int64), p) and np.array_equal(r.neg.astype(np.int64), m)
    assert int(r.pos.sum() + r.neg.sum()) <= 3


@pytest.mark.parametrize("case", [("uniform", 110, 8.0, 2.6, 4), ("clustered", 110, 10.0, 2.0, 3),
                                  ("survey", 100, 7.0, 2.6, 3)])
def test_oracle_pixel_parity_matches_brute_force(case):
    name, n, L, rmax, nb = case
    x = synth.uniform(n, L, 97) if name != "clustered" else synth.neyman_scott(n, 22, 0.7, L, 98)
    periodic = name != "survey"
    r = oracle.count_4pcf_pixel(x, L, 0.0, rmax, nb, periodic=periodic)
    e, p, m, nk = brute.cliques4_pixel(x, L if periodic else -L, 0.0, rmax, nb)
    assert r.n_cliques == nk
    assert np.array_equal(r.even.astype(np.int64), e)
    assert np.array_equal(r.pos.astype(np.int64), p) and np.array_equal(r.neg.astype(np.int64), m)


def test_pixel_parity_reflection_swaps_channels():
    """x -> L - x on a fine dyadic grid: every pixel mirrors in x (no zero
    components here), centres negate their x exactly, the index order is
    kept, so V negates exactly: pos and neg swap, even is unchanged."""
    L = 16.0
    x = synth.dyadic_uniform(3000, L, 99)
    y = x.copy()
    y[:, 0] = np.mod(L - y[:, 0], L)
    a = oracle.count_4pcf_pixel(x, L, 0.0, 1.6, 4)
    b = oracle.count_4pcf_pixel(y, L, 0.0, 1.6, 4)
    assert a.n_cliques == b.n_cliques > 0
    assert np.array_equal(a.even, b.even)
    assert np.array_equal(a.pos, b.neg) and np.array_equal(a.neg, b.pos)


def test_pixel_threshold_window():
    """Every volume of three pixel centres is either a rounding residue of an
    exactly coplanar triple (below 1e-12) or at least 2.3e-5: the 1e-9 rule
    must make the residues degenerate and keep the smallest true volumes.
    Pixels 0, 1, 3 share i = 0, so their unnormalised centres (a, (1-a)t,
    (1-a)(1-t)) all satisfy x(1-a) = a(y+z): a plane through the origin.
    Pixels 13, 93, 127 span the smallest nonzero volume, |V| = 2.9e-5."""
    import itertools
    cen = [oracle.pixel_centre(p) for p in range(256)]
    o = np.array([50.0, 50.0, 50.0])
    res = np.array([o, o + 2.0 * cen[0], o + 2.5 * cen[1], o + 3.0 * cen[3]])
    assert [oracle.pixel_of(res[k] - o) for k in (1, 2, 3)] == [0, 1, 3]
    assert oracle.hub_pixel_channel(res, 100.0, 0.0, 10.0, 2, 0) == 2
    small = np.array([o, o + 2.0 * cen[13], o + 2.5 * cen[93], o + 3.0 * cen[127]])
    assert [oracle.pixel_of(small[k] - o) for k in (1, 2, 3)] == [13, 93, 127]
    u, v, w = cen[13], cen[93], cen[127]
    V = ((u[1] * v[2] - u[2] * v[1]) * w[0] + (u[2] * v[0] - u[0] * v[2]) * w[1]) + (u[0] * v[1] - u[1] * v[0]) * w[2]
    assert 2e-5 < abs(V) < 3e-5
    assert oracle.hub_pixel_channel(small, 100.0, 0.0, 10.0, 2, 0) == (0 if V > 0 else 1)
