"""GPU 6-edge 4-clique counts, weighted parity counts, signed-weight
triangle sums and weighted pair sums against the CPU oracle, bit for bit
(counts and exact 128-bit sums), with the lattice's hand-derived 6-edge
configurations and anchor partitions."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gsn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2607_06604_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def ctx(gsn):
    c = gsn.Context(0)
    yield c
    c.close()


def signed_weights(n, seed, lo=0.5, width=1.0, neg_frac=0.4):
    """Magnitudes U(lo, lo + width), a random fraction of them negative."""
    m = synth.uniform_values(n, lo, width, seed)
    s = synth.uniform_values(n, 0.0, 1.0, seed + 1)
    return np.where(s < neg_frac, -m, m)


def estimator_weights(nd, nr, seed):
    """Data weights 1/nd (times U(0.8,1.2)), random weights -1/nr: the signed
    normalised data-minus-random weights of the paper's estimator."""
    wd = synth.uniform_values(nd, 0.8, 0.4, seed) / nd
    wr = -np.ones(nr) / nr
    return np.concatenate([wd, wr])


# (name, points, box, rmin, rmax, nbins): nbins 4 puts the 6-edge table and
# counters in LDS, 6 the table in global memory, 8 both in global memory
FULL_CASES = [
    ("uniform_nb4", lambda: synth.uniform(3000, 20.0, 501), 20.0, 0.0, 2.6, 4),
    ("clustered_nb4", lambda: synth.neyman_scott(4000, 40, 1.0, 40.0, 502), 40.0, 0.0, 2.4, 4),
    ("rmin_nb3", lambda: synth.uniform(2500, 16.0, 503), 16.0, 0.6, 2.5, 3),
    ("uniform_nb6", lambda: synth.uniform(4000, 24.0, 504), 24.0, 0.0, 2.8, 6),
    ("clustered_nb8", lambda: synth.neyman_scott(6000, 50, 1.1, 50.0, 505), 50.0, 0.0, 2.6, 8),
    ("dense_wrap_nb5", lambda: synth.uniform(300, 6.0, 506), 6.0, 0.0, 2.0, 5),
    ("dyadic_ties_nb4", lambda: synth.dyadic_uniform(2000, 16.0, 507, bits=5), 16.0, 0.0, 1.6, 4),
    ("nb1", lambda: synth.uniform(2000, 14.0, 508), 14.0, 0.0, 2.0, 1),
    ("nb12", lambda: synth.uniform(2000, 14.0, 509), 14.0, 0.0, 2.4, 12),
]


@pytest.mark.parametrize("case", FULL_CASES, ids=[c[0] for c in FULL_CASES])
def test_count4_full_matches_oracle(ctx, gsn, case):
    name, mk, L, rmin, rmax, nb = case
    x = mk()
    say("count4 full", name, len(x))
    g = ctx.build_graph(x, L, rmin, rmax, nb, keep_coords=True)
    got = ctx.count_4pcf_full(g)
    g.free()
    ref = oracle.count_4pcf_full(x, L, rmin, rmax, nb)
    assert got.n_cliques == ref.n_cliques
    assert np.array_equal(got.hist, ref.hist)
    assert int(got.hist.sum()) == got.n_cliques


@pytest.mark.parametrize("nb", [4, 8])
def test_count4_full_weighted_signed(ctx, nb):
    x = synth.neyman_scott(5000, 40, 1.0, 40.0, 511)
    w = signed_weights(len(x), 512)
    say("count4 full weighted", nb)
    g = ctx.build_graph(x, 40.0, 0.0, 2.6, nb, weights=w, keep_coords=True)
    got = ctx.count_4pcf_full(g, weighted=True)
    g.free()
    ref = oracle.count_4pcf_full(x, 40.0, 0.0, 2.6, nb, weights=w)
    assert np.array_equal(got.hist, ref.hist) and got.n_cliques == ref.n_cliques
    assert got.wscale == ref.wscale
    assert got.wsum_int() == ref.wsum_int()


def test_count4_full_lattice_closed_form(ctx):
    gl = json.load(open(os.path.join(HERE, "golden", "lattice_sc.json")))
    m = gl["sites_per_axis"]
    a = np.arange(m, dtype=np.float64)
    X, Y, Z = np.meshgrid(a, a, a, indexing="ij")
    x = np.mod(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + np.array([0.25, 0.5, 0.125]), gl["box"])
    nb = gl["nbins"]
    g = ctx.build_graph(x, gl["box"], gl["rmin"], gl["rmax"], nb, keep_coords=True)
    got = ctx.count_4pcf_full(g)
    g.free()
    exp = np.zeros(oracle.n_configs6(nb), dtype=np.uint64)
    # the configuration index of a smallest tuple: its rank among all smallest tuples
    canon = [oracle.config6(nb, k) for k in range(oracle.n_configs6(nb))]
    for key, v in gl["six_edge_configs_per_site"].items():
        exp[canon.index(tuple(map(int, key.split(","))))] = v * len(x)
    assert np.array_equal(got.hist, exp)


def test_count4_full_anchor_partition(ctx):
    x = synth.uniform(5000, 24.0, 521)
    g = ctx.build_graph(x, 24.0, 0.0, 2.8, 4, keep_coords=True)
    full = ctx.count_4pcf_full(g)
    cuts = [0, 700, 2100, 2101, 4000, 5000]
    tot = np.zeros_like(full.hist)
    n = 0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        r = ctx.count_4pcf_full(g, anchors=(lo, hi))
        tot += r.hist
        n += r.n_cliques
    g.free()
    assert np.array_equal(tot, full.hist) and n == full.n_cliques
    ref = oracle.count_4pcf_full(x, 24.0, 0.0, 2.8, 4, anchors=(700, 2100))
    g = ctx.build_graph(x, 24.0, 0.0, 2.8, 4, keep_coords=True)
    got = ctx.count_4pcf_full(g, anchors=(700, 2100))
    g.free()
    assert np.array_equal(got.hist, ref.hist)


def test_count4_full_limits(ctx, gsn):
    x = synth.uniform(500, 10.0, 531)
    g = ctx.build_graph(x, 10.0, 0.0, 2.0, 13, keep_coords=True)
    with pytest.raises(gsn.GsError) as e:
        ctx.count_4pcf_full(g)
    assert e.value.code == gsn.GS_EUNSUPPORTED
    g.free()
    g = ctx.build_graph(x, 10.0, 0.0, 2.0, 4)
    with pytest.raises(gsn.GsError) as e:
        ctx.count_4pcf_full(g)
    assert e.value.code == gsn.GS_ENOCOORDS
    g.free()


@pytest.mark.parametrize("case", ["mixed_signs", "estimator"])
def test_parity_weighted_matches_oracle(ctx, case):
    if case == "mixed_signs":
        x = synth.neyman_scott(6000, 50, 1.1, 50.0, 541)
        w = signed_weights(len(x), 542)
        L, rmax, nb = 50.0, 2.6, 8
    else:
        xd = synth.neyman_scott(3000, 30, 1.0, 40.0, 543)
        xr = synth.uniform(6000, 40.0, 544)
        x = np.concatenate([xd, xr])
        w = estimator_weights(len(xd), len(xr), 545)
        L, rmax, nb = 40.0, 2.4, 5
    say("parity weighted", case, len(x))
    g = ctx.build_graph(x, L, 0.0, rmax, nb, weights=w, keep_coords=True)
    got = ctx.count_4pcf_parity(g, weighted=True)
    plain = ctx.count_4pcf_parity(g)
    g.free()
    ref = oracle.count_4pcf_parity(x, L, 0.0, rmax, nb, weights=w)
    assert got.n_cliques == ref.n_cliques
    assert np.array_equal(got.even, ref.even) and np.array_equal(got.pos, ref.pos)
    assert np.array_equal(got.neg, ref.neg)
    assert np.array_equal(plain.even, got.even) and np.array_equal(plain.pos, got.pos)
    assert got.wscale == ref.wscale
    for ch in range(3):
        assert got.wsum_int(ch) == ref.wsum_int(ch), ch


@pytest.mark.parametrize("case", ["mixed_signs", "estimator", "all_negative"])
def test_weighted_count3_signed(ctx, case):
    if case == "estimator":
        xd = synth.neyman_scott(8000, 40, 1.5, 60.0, 551)
        xr = synth.uniform(16000, 60.0, 552)
        x = np.concatenate([xd, xr])
        w = estimator_weights(len(xd), len(xr), 553)
    else:
        x = synth.neyman_scott(20000, 40, 1.5, 80.0, 554)
        w = signed_weights(len(x), 555, neg_frac=1.0 if case == "all_negative" else 0.4)
        L = 80.0
    L = 60.0 if case == "estimator" else 80.0
    say("signed weighted count3", case, len(x))
    g = ctx.build_graph(x, L, 0.0, 3.5, 10, weights=w)
    got = ctx.count_3pcf(g, weighted=True)
    g.free()
    ref = oracle.count_3pcf(x, L, 0.0, 3.5, 10, weights=w)
    assert np.array_equal(got.hist, ref.hist) and got.n_triangles == ref.n_triangles
    assert got.wscale == ref.wscale
    assert got.wsum_int() == ref.wsum_int()
    assert np.array_equal(got.whist, ref.whist())
    if case == "all_negative":
        # every triangle's product of three negative weights is negative
        assert all(v <= 0 for v in got.wsum_int())


def test_weighted_count3_signed_tiled(ctx, monkeypatch):
    x = synth.neyman_scott(20000, 40, 1.5, 80.0, 561)
    w = signed_weights(len(x), 562)
    ref = oracle.count_3pcf(x, 80.0, 0.0, 3.5, 10, weights=w)
    monkeypatch.setenv("GS_WINDOWS", "3")
    g = ctx.build_graph(x, 80.0, 0.0, 3.5, 10, weights=w)
    assert g.info().n_windows == 3
    got = ctx.count_3pcf(g, weighted=True)
    g.free()
    assert got.wsum_int() == ref.wsum_int() and np.array_equal(got.hist, ref.hist)


@pytest.mark.parametrize("block", ["768", "512"])
def test_weighted_count3_signed_plans(ctx, monkeypatch, block):
    # signed and wide terms (the general path) in 768- and 512-thread groups
    x = synth.neyman_scott(20000, 40, 1.5, 80.0, 565)
    w = signed_weights(len(x), 566)
    w[::211] *= 300.0    # some terms beyond 2^63: straight into the 128-bit sums
    ref = oracle.count_3pcf(x, 80.0, 0.0, 3.5, 10, weights=w)
    monkeypatch.setenv("GS_BLOCK3", block)
    monkeypatch.setenv("GS_GLOG", "4")
    g = ctx.build_graph(x, 80.0, 0.0, 3.5, 10, weights=w)
    got = ctx.count_3pcf(g, weighted=True)
    g.free()
    assert got.wscale == ref.wscale and got.wsum_int() == ref.wsum_int()
    assert np.array_equal(got.hist, ref.hist)


def test_weight_range_limits(ctx, gsn):
    """Magnitudes far apart: most terms fit 64 bits, the widest do not and go
    straight into the 128-bit sums; beyond 2^87 both sides refuse."""
    x = synth.uniform(3000, 20.0, 571)
    w = signed_weights(len(x), 572)
    w[::97] *= 300.0     # a few points weigh 300 times more: triangle terms up to ~2^78
    g = ctx.build_graph(x, 20.0, 0.0, 2.6, 4, weights=w)
    got = ctx.count_3pcf(g, weighted=True)
    ref = oracle.count_3pcf(x, 20.0, 0.0, 2.6, 4, weights=w)
    assert got.wscale == ref.wscale and got.wsum_int() == ref.wsum_int()
    r = ctx.pair_sums(g, weighted=True)
    refp = oracle.pair_sums(x, 20.0, 0.0, 2.6, 4, weights=w)
    assert r.wsum_int() == refp.wsum_int()
    g.free()
    w2 = np.ones(len(x))
    w2[7] = 1e-12        # a 2^120 range: no exact 128-bit sum holds it
    g = ctx.build_graph(x, 20.0, 0.0, 2.0, 4, weights=w2)
    with pytest.raises(gsn.GsError) as e:
        ctx.count_3pcf(g, weighted=True)
    assert e.value.code == gsn.GS_EINVAL
    with pytest.raises(oracle.OracleError):
        oracle.count_3pcf(x, 20.0, 0.0, 2.0, 4, weights=w2)
    g.free()
    w2[7] = 0.0
    with pytest.raises(gsn.GsError) as e:
        ctx.build_graph(x, 20.0, 0.0, 2.0, 4, weights=w2)
    assert e.value.code == gsn.GS_EINVAL


@pytest.mark.parametrize("windows", [0, 4])
def test_pair_sums_match_oracle(ctx, monkeypatch, windows):
    x = synth.neyman_scott(30000, 50, 2.0, 100.0, 581)
    w = signed_weights(len(x), 582)
    if windows:
        monkeypatch.setenv("GS_WINDOWS", str(windows))
    g = ctx.build_graph(x, 100.0, 0.5, 6.0, 12, weights=w)
    if windows:
        assert g.info().n_windows == windows
    got = ctx.pair_sums(g, weighted=True)
    part = ctx.pair_sums(g, anchors=(1000, 17000), weighted=True)
    info = g.info()
    g.free()
    ref = oracle.pair_sums(x, 100.0, 0.5, 6.0, 12, weights=w)
    refp = oracle.pair_sums(x, 100.0, 0.5, 6.0, 12, weights=w, anchors=(1000, 17000))
    assert np.array_equal(got.pairs, ref.pairs)
    assert np.array_equal(got.pairs, np.asarray(info.pair_hist[:12], dtype=np.uint64))
    assert got.wscale == ref.wscale and got.wsum_int() == ref.wsum_int()
    assert np.array_equal(part.pairs, refp.pairs) and part.wsum_int() == refp.wsum_int()
