"""Host-tiled (out-of-core) graphs: forced window counts and budget caps give
histograms bit-identical to the resident graph and to the oracle; each spoke
is owned by exactly one (hub window, spoke window) tile (paper Sec. 3.5.3).
Includes the full-size 2e6-point weighted lognormal workload against stored
oracle values for sampled anchor ranges."""
import hashlib
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


def _ln(n, L, seed):
    x = synth.lognormal(n, L, seed, mesh=32, sigma_s=L / 40)
    w = synth.uniform_values(n, 0.5, 1.0, seed + 1)
    return x, w


@pytest.mark.parametrize("windows", [2, 3, 5, 8])
def test_forced_windows_match_resident_and_oracle(ctx, monkeypatch, windows):
    x, w = _ln(60_000, 800.0, 91)
    L, rmax, nb = 800.0, 45.0, 12
    say("ooc windows", windows)
    g = ctx.build_graph(x, L, 0.0, rmax, nb, weights=w)
    res = ctx.count_3pcf(g, weighted=True)
    rp0, col0, b0, perm0 = g.export()
    g.free()
    monkeypatch.setenv("GS_WINDOWS", str(windows))
    gt = ctx.build_graph(x, L, 0.0, rmax, nb, weights=w)
    info = gt.info()
    assert info.n_windows == windows
    rp1, col1, b1, perm1 = gt.export()
    tiled = ctx.count_3pcf(gt, weighted=True)
    part = ctx.count_3pcf(gt, anchors=(1000, 31000), weighted=True)
    gt.free()
    assert np.array_equal(rp0, rp1) and np.array_equal(col0, col1)
    assert np.array_equal(b0, b1) and np.array_equal(perm0, perm1)
    assert np.array_equal(tiled.hist, res.hist) and tiled.n_triangles == res.n_triangles
    assert tiled.wsum_int() == res.wsum_int()
    ref = oracle.count_3pcf(x, L, 0.0, rmax, nb, weights=w)
    assert np.array_equal(tiled.hist, ref.hist) and tiled.wsum_int() == ref.wsum_int()
    refp = oracle.count_3pcf(x, L, 0.0, rmax, nb, weights=w, anchors=(1000, 31000))
    assert np.array_equal(part.hist, refp.hist) and part.wsum_int() == refp.wsum_int()


def test_budget_cap_forces_tiling(gsn):
    w = synth.workload("ns_3pcf", volume_fraction=0.125)
    with gsn.Context(0) as full:
        g = full.build_graph(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
        ref = full.count_3pcf(g)
        info = g.info()
        g.free()
    fixed = 8 * (w.n + 1) + 4 * w.n
    budget = fixed + (5 * info.n_edges) // 3
    say("budget cap", budget)
    with gsn.Context(0, budget_bytes=budget) as small:
        g = small.build_graph(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
        ti = g.info()
        got = small.count_3pcf(g)
        g.free()
    assert ti.n_windows > 1
    assert np.array_equal(got.hist, ref.hist) and got.n_triangles == ref.n_triangles


@pytest.mark.parametrize("windows", [2, 3, 6])
def test_four_point_counts_on_tiled_graphs(ctx, monkeypatch, windows):
    """Parity (plain and weighted), 6-edge and pixel counts on a host-tiled
    graph: each hub window counted from the CSR range its hubs read, equal to
    the resident counts and the oracle bit for bit."""
    x = synth.neyman_scott(12000, 50, 1.2, 70.0, 93)
    w = synth.uniform_values(len(x), 0.5, 1.0, 94)
    L, rmax, nb = 70.0, 3.0, 4
    say("tiled 4-point counts", windows)
    g = ctx.build_graph(x, L, 0.0, rmax, nb, weights=w, keep_coords=True)
    res = (ctx.count_4pcf_parity(g, weighted=True), ctx.count_4pcf_full(g), ctx.count_4pcf_pixel(g))
    g.free()
    monkeypatch.setenv("GS_WINDOWS", str(windows))
    gt = ctx.build_graph(x, L, 0.0, rmax, nb, weights=w, keep_coords=True)
    assert gt.info().n_windows == windows
    til = (ctx.count_4pcf_parity(gt, weighted=True), ctx.count_4pcf_full(gt), ctx.count_4pcf_pixel(gt),
           ctx.count_4pcf_parity(gt, anchors=(2000, 7000)))
    gt.free()
    for a, b in ((res[0], til[0]), (res[2], til[2])):
        assert a.n_cliques == b.n_cliques
        assert np.array_equal(a.even, b.even) and np.array_equal(a.pos, b.pos) and np.array_equal(a.neg, b.neg)
    for ch in range(3):
        assert res[0].wsum_int(ch) == til[0].wsum_int(ch)
    assert np.array_equal(res[1].hist, til[1].hist)
    ref = oracle.count_4pcf_parity(x, L, 0.0, rmax, nb, weights=w)
    assert np.array_equal(til[0].even, ref.even) and np.array_equal(til[0].pos, ref.pos)
    assert til[0].wsum_int(1) == ref.wsum_int(1)
    refp = oracle.count_4pcf_parity(x, L, 0.0, rmax, nb, anchors=(2000, 7000))
    assert np.array_equal(til[3].even, refp.even) and np.array_equal(til[3].neg, refp.neg)


def test_noalloc_parity_refuses_tiled_graph(ctx, gsn, monkeypatch):
    monkeypatch.setenv("GS_WINDOWS", "2")
    x = synth.uniform(3000, 20.0, 95)
    g = ctx.build_graph(x, 20.0, 0.0, 2.0, 4, keep_coords=True)
    with pytest.raises(gsn.GsError) as e:
        ctx.count_4pcf_parity(g, noalloc=True)
    g.free()
    assert e.value.code == gsn.GS_EUNSUPPORTED


def test_full_size_lognormal_weighted_resident_tiled_and_sampled(ctx, monkeypatch):
    """Full-size weighted workload (2e6 lognormal points, rmax 150, 20 bins):
    the unanchored resident count (64-bit row offsets, 7.2e9 directed edges)
    and a host-tiled count over 4 windows agree bit for bit, and sampled
    anchor ranges match stored oracle values exactly (128-bit sums)."""
    gold = json.load(open(os.path.join(HERE, "golden", "lognormal_w3pcf_sampled.json")))
    w = synth.workload("lognormal_w3pcf")
    assert hashlib.sha256(np.ascontiguousarray(w.xyz).tobytes()).hexdigest() == gold["xyz_sha256"]
    assert hashlib.sha256(np.ascontiguousarray(w.weights).tobytes()).hexdigest() == gold["weights_sha256"]
    say("full lognormal resident", w.n)
    g = ctx.build_graph(w.xyz, w.box, w.rmin, w.rmax, w.nbins, weights=w.weights)
    res = ctx.count_3pcf(g, weighted=True)
    say("  resident count", res.n_triangles)
    for s in gold["samples"]:
        say("  sample", s["lo"], s["hi"])
        got = ctx.count_3pcf(g, anchors=(s["lo"], s["hi"]), weighted=True)
        assert got.n_triangles == s["n_triangles"]
        assert got.hist.tolist() == s["hist"]
        assert got.wscale == s["wscale"]
        assert got.wsum.tolist() == s["wsum"]
    g.free()
    assert int(res.hist.sum()) == res.n_triangles
    say("full lognormal tiled", 4)
    monkeypatch.setenv("GS_WINDOWS", "4")
    gt = ctx.build_graph(w.xyz, w.box, w.rmin, w.rmax, w.nbins, weights=w.weights)
    assert gt.info().n_windows == 4
    tiled = ctx.count_3pcf(gt, weighted=True)
    gt.free()
    assert np.array_equal(tiled.hist, res.hist) and tiled.wsum_int() == res.wsum_int()


def test_oversubscribed_9e9_edges(gsn):
    """A graph larger than the device budget at the paper's out-of-core scale
    (Sec. 3.5.3: 9e9 edges): 2.25e6 lognormal points in the 2000 Mpc/h box,
    rmax 150, 20 bins, weighted -- about 9.1e9 directed edges, 23 GB of
    forward CSR, counted under a 16 GB budget in host-tiled windows. The
    exact weighted sums of sampled anchor ranges equal the oracle's, and the
    whole count equals the resident count bit for bit."""
    n, L = 2_250_000, 2000.0
    x = synth.lognormal(n, L, 7)
    w = synth.uniform_values(n, 0.5, 1.0, 8)
    with gsn.Context(0, budget_bytes=16 << 30) as small:
        say("oversubscribed build", n)
        g = small.build_graph(x, L, 0.0, 150.0, 20, weights=w)
        info = g.info()
        say("  directed edges", 2 * info.n_edges, "windows", info.n_windows)
        assert 2 * info.n_edges >= 9.0e9
        assert info.n_windows > 1
        tiled = small.count_3pcf(g, weighted=True)
        samples = [(k * n // 3, k * n // 3 + 8) for k in range(3)]
        parts = [small.count_3pcf(g, anchors=s, weighted=True) for s in samples]
        g.free()
    for s, got in zip(samples, parts):
        say("  oracle sample", s)
        ref = oracle.count_3pcf(x, L, 0.0, 150.0, 20, weights=w, anchors=s)
        assert got.n_triangles == ref.n_triangles and np.array_equal(got.hist, ref.hist)
        assert got.wscale == ref.wscale and got.wsum_int() == ref.wsum_int()
    with gsn.Context(0) as big:
        say("resident count")
        g = big.build_graph(x, L, 0.0, 150.0, 20, weights=w)
        assert g.info().n_windows == 1
        res = big.count_3pcf(g, weighted=True)
        g.free()
    assert res.n_triangles == tiled.n_triangles
    assert np.array_equal(res.hist, tiled.hist) and res.wsum_int() == tiled.wsum_int()
