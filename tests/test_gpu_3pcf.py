"""GPU graph builder and triangle counts against the CPU oracle (bit-exact).

All calls go through the C ABI (ctypes binding). Sizes span several hub
tiles and ragged tails; the full-size Neyman-Scott workload is compared with
stored oracle values (tests/golden/ns_3pcf_full.json).
"""
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


def undirected_edges_gpu(rp, col, b, perm):
    n = len(rp) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp.astype(np.int64)))
    a = perm[rows].astype(np.int64)
    c = perm[col].astype(np.int64)
    lo, hi = np.minimum(a, c), np.maximum(a, c)
    key = lo * (1 << 32) + hi
    o = np.argsort(key, kind="stable")
    return key[o], b[o]


def undirected_edges_oracle(rp, col, b):
    n = len(rp) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    m = col.astype(np.int64) > rows
    key = rows[m] * (1 << 32) + col[m].astype(np.int64)
    o = np.argsort(key, kind="stable")
    return key[o], b[m][o]


CASES = [
    ("uniform_tiny", lambda: synth.uniform(300, 10.0, 21), 10.0, 0.0, 2.4, 5, None),
    ("uniform_rmin", lambda: synth.uniform(3000, 30.0, 22), 30.0, 0.7, 2.6, 4, None),
    ("clustered", lambda: synth.neyman_scott(4000, 25, 0.8, 25.0, 23), 25.0, 0.0, 2.0, 6, None),
    ("single_cell", lambda: synth.uniform(500, 9.0, 24), 9.0, 0.0, 3.9, 3, None),
    ("two_cells_per_axis", lambda: synth.uniform(700, 10.0, 26), 10.0, 0.0, 4.2, 7, None),
    ("many_bins", lambda: synth.uniform(2000, 16.0, 25), 16.0, 0.0, 2.2, 21, None),
    ("dyadic_ties", lambda: synth.dyadic_uniform(3000, 16.0, 27, bits=6), 16.0, 0.0, 1.5, 6, None),
    # crowded cells: a work group's candidates exceed its LDS stage (3 and 6
    # cells per axis: every cell wrapping, and interior cells without wraps)
    ("dense_wrap", lambda: synth.uniform(4000, 12.0, 28), 12.0, 0.0, 3.9, 5, None),
    ("dense_interior", lambda: synth.uniform(12000, 25.0, 29), 25.0, 0.0, 3.9, 5, None),
    ("uniform_c1", None, None, None, None, None, ("uniform_3pcf", 1.0)),
    ("ns_c2_eighth", None, None, None, None, None, ("ns_3pcf", 0.125)),
    ("ns_c3_full", None, None, None, None, None, ("ns_4pcf_parity", 1.0)),
]


def _case(c):
    name, mk, L, rmin, rmax, nb, wl = c
    if wl is not None:
        w = synth.workload(*wl)
        return w.xyz, w.box, w.rmin, w.rmax, w.nbins
    return mk(), L, rmin, rmax, nb


@pytest.mark.parametrize("case", CASES[:10], ids=[c[0] for c in CASES[:10]])
def test_graph_edges_and_bins_match_oracle(ctx, case):
    x, L, rmin, rmax, nb = _case(case)
    say("graph", case[0], len(x))
    g = ctx.build_graph(x, L, rmin, rmax, nb)
    rp, col, b, perm = g.export()
    info = g.info()
    g.free()
    assert sorted(perm.tolist()) == list(range(len(x)))
    # rows strictly increasing, forward only
    for i in range(len(x)):
        r = col[rp[i]:rp[i + 1]].astype(np.int64)
        assert np.all(r > i) and np.all(np.diff(r) > 0)
    orp, ocol, ob = oracle.graph(x, L, rmin, rmax, nb)
    kg, bg = undirected_edges_gpu(rp, col, b, perm)
    ko, bo = undirected_edges_oracle(orp, ocol, ob)
    assert np.array_equal(kg, ko)
    assert np.array_equal(bg, bo)
    assert info.n_edges == len(ko)
    assert list(info.pair_hist[:nb]) == np.bincount(bo, minlength=nb).tolist()
    assert info.max_deg == int(np.diff(rp.astype(np.int64)).max(initial=0))
    assert info.sum_sq_degree == int((np.diff(orp).astype(np.int64) ** 2).sum())


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_count3_matches_oracle(ctx, case):
    x, L, rmin, rmax, nb = _case(case)
    say("count3", case[0], len(x))
    g = ctx.build_graph(x, L, rmin, rmax, nb)
    got = ctx.count_3pcf(g)
    g.free()
    ref = oracle.count_3pcf(x, L, rmin, rmax, nb)
    assert got.n_triangles == ref.n_triangles
    assert np.array_equal(got.hist, ref.hist)
    assert int(got.hist.sum()) == got.n_triangles


def test_count3_full_size_ns_against_stored_oracle(ctx):
    with open(os.path.join(HERE, "golden", "ns_3pcf_full.json")) as f:
        gold = json.load(f)
    w = synth.workload("ns_3pcf")
    assert hashlib.sha256(np.ascontiguousarray(w.xyz).tobytes()).hexdigest() == gold["xyz_sha256"]
    say("count3 full ns", w.n)
    g = ctx.build_graph(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    got = ctx.count_3pcf(g)
    again = ctx.count_3pcf(g)
    g.free()
    assert got.n_triangles == gold["n_triangles"]
    assert got.hist.tolist() == gold["hist"]
    assert np.array_equal(again.hist, got.hist)


def test_count3_device_input_matches_host_input(ctx):
    import torch
    w = synth.workload("ns_3pcf", volume_fraction=0.125)
    say("count3 device input", w.n)
    gh = ctx.build_graph(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    a = ctx.count_3pcf(gh)
    gh.free()
    xd = torch.from_numpy(w.xyz).to("cuda:0")
    gd = ctx.build_graph(xd, w.box, w.rmin, w.rmax, w.nbins)
    b = ctx.count_3pcf(gd)
    gd.free()
    assert a.n_triangles == b.n_triangles and np.array_equal(a.hist, b.hist)


def test_count3_anchor_ranges_partition_and_match_oracle(ctx):
    w = synth.workload("uniform_3pcf")
    say("count3 anchors", w.n)
    g = ctx.build_graph(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    full = ctx.count_3pcf(g)
    cuts = [0, 1, 4999, 5000, 13333, 20000]
    acc = np.zeros_like(full.hist)
    tot = 0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        part = ctx.count_3pcf(g, anchors=(lo, hi))
        ref = oracle.count_3pcf(w.xyz, w.box, w.rmin, w.rmax, w.nbins, anchors=(lo, hi))
        assert part.n_triangles == ref.n_triangles and np.array_equal(part.hist, ref.hist)
        acc += part.hist
        tot += part.n_triangles
    empty = ctx.count_3pcf(g, anchors=(7, 7))
    g.free()
    assert np.array_equal(acc, full.hist) and tot == full.n_triangles
    assert empty.n_triangles == 0 and empty.hist.sum() == 0


WEIGHTED = [
    # lognormal-like field, weights 0.5 + U[0,1): (n, L, rmax, nbins, mesh)
    (30_000, 1000.0, 60.0, 20, 32),
    (60_000, 800.0, 45.0, 12, 32),
]


@pytest.mark.parametrize("case", WEIGHTED, ids=["ln30k", "ln60k"])
def test_weighted_count3_exact_sums(ctx, case):
    n, L, rmax, nb, mesh = case
    x = synth.lognormal(n, L, 81, mesh=mesh, sigma_s=L / 40)
    wt = synth.uniform_values(n, 0.5, 1.0, 82)
    say("weighted count3", n)
    g = ctx.build_graph(x, L, 0.0, rmax, nb, weights=wt)
    got = ctx.count_3pcf(g, weighted=True)
    g.free()
    ref = oracle.count_3pcf(x, L, 0.0, rmax, nb, weights=wt)
    assert got.n_triangles == ref.n_triangles and np.array_equal(got.hist, ref.hist)
    assert got.wscale == ref.wscale
    assert got.wsum_int() == ref.wsum_int()
    assert np.array_equal(got.whist, ref.whist())


def test_weighted_unit_weights_equal_counts(ctx):
    x = synth.uniform(5000, 30.0, 61)
    g = ctx.build_graph(x, 30.0, 0.0, 3.0, 6, weights=np.ones(len(x)))
    got = ctx.count_3pcf(g, weighted=True)
    g.free()
    assert got.wscale == 52
    assert np.array_equal(got.whist, got.hist.astype(np.float64))


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_tiny_and_empty_catalogues(ctx, n):
    x = synth.uniform(n, 10.0, 70 + n) if n else np.zeros((0, 3))
    g = ctx.build_graph(x, 10.0, 0.0, 4.0, 3)
    got = ctx.count_3pcf(g)
    info = g.info()
    g.free()
    ref = oracle.count_3pcf(x, 10.0, 0.0, 4.0, 3)
    assert got.n_triangles == ref.n_triangles and np.array_equal(got.hist, ref.hist)
    assert info.n == n


def test_no_edges(ctx):
    x = synth.uniform(1000, 1000.0, 71)
    g = ctx.build_graph(x, 1000.0, 0.0, 0.5, 4)
    got = ctx.count_3pcf(g)
    assert g.info().n_edges == 0
    g.free()
    assert got.n_triangles == 0 and got.hist.sum() == 0


def test_maximum_bins_uses_global_histogram(ctx):
    x = synth.uniform(3000, 20.0, 72)
    g = ctx.build_graph(x, 20.0, 0.0, 2.5, 255)
    got = ctx.count_3pcf(g)
    g.free()
    ref = oracle.count_3pcf(x, 20.0, 0.0, 2.5, 255)
    assert got.n_triangles == ref.n_triangles and np.array_equal(got.hist, ref.hist)


def test_invalid_inputs_rejected(ctx, gsn):
    x = synth.uniform(100, 10.0, 73)
    for args in [(10.0, 0.0, 5.0, 4), (10.0, 2.0, 2.0, 4), (10.0, 0.0, 2.0, 0), (10.0, 0.0, 2.0, 256)]:
        with pytest.raises(gsn.GsError) as e:
            ctx.build_graph(x, *args)
        assert e.value.code == gsn.GS_EINVAL
    y = x.copy()
    y[5, 2] = 10.0
    with pytest.raises(gsn.GsError) as e:
        ctx.build_graph(y, 10.0, 0.0, 2.0, 4)
    assert e.value.code == gsn.GS_EINVAL
    y[5, 2] = np.nan
    with pytest.raises(gsn.GsError) as e:
        ctx.build_graph(y, 10.0, 0.0, 2.0, 4)
    assert e.value.code == gsn.GS_EINVAL
    with pytest.raises(gsn.GsError) as e:
        ctx.build_graph(x, 10.0, 0.0, 2.0, 4, weights=np.zeros(100))   # weights must be nonzero
    assert e.value.code == gsn.GS_EINVAL
    g = ctx.build_graph(x, 10.0, 0.0, 2.0, 4)
    with pytest.raises(gsn.GsError) as e:
        ctx.count_3pcf(g, weighted=True)
    assert e.value.code == gsn.GS_EINVAL
    with pytest.raises(gsn.GsError) as e:
        ctx.count_4pcf_parity(g)
    assert e.value.code == gsn.GS_ENOCOORDS
    g.free()


KERNEL_PLANS = [
    {"GS_BLOCK3": "256", "GS_GLOG": "0", "GS_TRUNC": "0"},
    {"GS_BLOCK3": "256", "GS_GLOG": "2", "GS_TRUNC": "1"},
    {"GS_BLOCK3": "256", "GS_GLOG": "4", "GS_TMAX": "64", "GS_MODE3": "lut"},
    {"GS_BLOCK3": "512", "GS_GLOG": "3", "GS_PACK": "0"},
    {"GS_BLOCK3": "512", "GS_GLOG": "6", "GS_MODE3": "rank", "GS_TMAX": "100"},
    {"GS_BLOCK3": "256", "GS_GLOG": "1", "GS_PACK": "0", "GS_MODE3": "rank", "GS_TRUNC": "1"},
    {"GS_BLOCK3": "256", "GS_GLOG": "3", "GS_PACK": "0", "GS_MODE3": "lut", "GS_TRUNC": "0"},
    {"GS_BLOCK3": "256", "GS_GLOG": "3", "GS_WIDE": "1"},
    {"GS_BLOCK3": "512", "GS_GLOG": "5", "GS_WIDE": "1", "GS_PACK": "0", "GS_TRUNC": "1"},
    # 64-bit addressing with spoke-row segments of at most 3000 entries from
    # their first row: a hub's spokes go in several segments (as rows more
    # than 2^32 entries apart do at full size)
    {"GS_BLOCK3": "256", "GS_GLOG": "4", "GS_WIDE": "1", "GS_WIDE_SPAN": "3000"},
    {"GS_BLOCK3": "512", "GS_GLOG": "6", "GS_WIDE": "1", "GS_WIDE_SPAN": "1", "GS_TRUNC": "0"},
    # 768-thread groups (weighted unanchored counts take them; the anchored,
    # unweighted and batched counts of the same plan fall back to 512)
    {"GS_BLOCK3": "768", "GS_GLOG": "6"},
    {"GS_BLOCK3": "768", "GS_GLOG": "3", "GS_TMAX": "100", "GS_MODE3": "rank"},
    {"GS_BLOCK3": "768", "GS_GLOG": "5", "GS_WIDE": "1", "GS_WIDE_SPAN": "3000"},
]


@pytest.mark.parametrize("plan", KERNEL_PLANS, ids=lambda p: "-".join(f"{k[3:].lower()}{v}" for k, v in p.items()))
def test_count_kernel_plans_match_oracle(ctx, monkeypatch, plan):
    """Every kernel plan -- work-group size, entries per step, row
    truncation, step table capacity (several fills per spoke chunk), packed or
    separate hash bins, configuration table or rank arithmetic, 32-bit or
    64-bit row addressing -- on plain, weighted, anchored, tiled and batched
    counts."""
    for k, v in plan.items():
        monkeypatch.setenv(k, v)
    x = synth.neyman_scott(12_000, 40, 1.5, 60.0, 301)
    w = synth.uniform_values(len(x), 0.5, 1.0, 302)
    L, rmax, nb = 60.0, 3.5, 9
    say("plan", plan)
    ref = oracle.count_3pcf(x, L, 0.0, rmax, nb, weights=w)
    g = ctx.build_graph(x, L, 0.0, rmax, nb, weights=w)
    got = ctx.count_3pcf(g, weighted=True)
    assert np.array_equal(got.hist, ref.hist) and got.wsum_int() == ref.wsum_int()
    part = ctx.count_3pcf(g, anchors=(2000, 7000))
    refp = oracle.count_3pcf(x, L, 0.0, rmax, nb, anchors=(2000, 7000))
    assert np.array_equal(part.hist, refp.hist) and part.n_triangles == refp.n_triangles
    g.free()
    monkeypatch.setenv("GS_WINDOWS", "3")
    gt = ctx.build_graph(x, L, 0.0, rmax, nb, weights=w)
    tiled = ctx.count_3pcf(gt, weighted=True)
    gt.free()
    monkeypatch.delenv("GS_WINDOWS")
    assert np.array_equal(tiled.hist, ref.hist) and tiled.wsum_int() == ref.wsum_int()
    y = synth.uniform(9_000, L, 303)
    gs = [ctx.build_graph(c, L, 0.0, rmax, nb) for c in (x, y, x[:5000])]
    bat = ctx.count_3pcf_batch(gs)
    for gg in gs:
        gg.free()
    assert np.array_equal(bat[0].hist, ref.hist)
    assert np.array_equal(bat[1].hist, oracle.count_3pcf(y, L, 0.0, rmax, nb).hist)
    assert np.array_equal(bat[2].hist, oracle.count_3pcf(x[:5000], L, 0.0, rmax, nb).hist)
    # forced flushes of the shared / per-wave counters
    monkeypatch.setenv("GS_FLUSH_LIMIT", str(64 * 512 * 4))
    g = ctx.build_graph(x, L, 0.0, rmax, nb, weights=w)
    again = ctx.count_3pcf(g, weighted=True)
    g.free()
    assert np.array_equal(again.hist, ref.hist) and again.wsum_int() == ref.wsum_int()


def test_autotuned_schedule_counts_identical(gsn):
    """The tuner times schedules on a hub sample and keeps the fastest for the
    graph's shape; counts with the tuned schedule (plain, weighted, batched)
    equal the oracle's, and the schedule it reports is a valid one."""
    x = synth.neyman_scott(40_000, 40, 1.5, 80.0, 311)
    w = synth.uniform_values(len(x), 0.5, 1.0, 312)
    L, rmax, nb = 80.0, 3.5, 12
    ref = oracle.count_3pcf(x, L, 0.0, rmax, nb, weights=w)
    with gsn.Context(0) as c:
        g = c.build_graph(x, L, 0.0, rmax, nb)
        plan = c.tune_3pcf(g)
        say("plan", plan)
        assert plan["block"] in (256, 512) and 0 <= plan["step_log2"] <= 6
        assert 1 <= plan["group"] <= 4 and plan["counters"] in (0, 1, 2) and plan["table"] >= 64
        assert plan["hash_load"] in (5, 7) and plan["truncate"] in (0, 1)
        assert plan["trials"] >= 2 and 0 < plan["sample_ms"] <= plan["default_ms"] * 1.0001
        assert 0 < plan["sample_frac"] <= 1
        got = c.count_3pcf(g)
        assert np.array_equal(got.hist, ref.hist) and got.n_triangles == ref.n_triangles
        bat = c.count_3pcf_batch([g, g])
        assert np.array_equal(bat[0].hist, ref.hist) and np.array_equal(bat[1].hist, ref.hist)
        g.free()
        gw = c.build_graph(x, L, 0.0, rmax, nb, weights=w)
        pw = c.tune_3pcf(gw, weighted=True)
        assert pw["counters"] != 2   # no per-triple counters for weighted sums
        gotw = c.count_3pcf(gw, weighted=True)
        assert np.array_equal(gotw.hist, ref.hist) and gotw.wsum_int() == ref.wsum_int()
        with pytest.raises(gsn.GsError) as e:
            c.tune_3pcf(c.build_graph(x, L, 0.0, rmax, nb), weighted=True)
        assert e.value.code == gsn.GS_EINVAL
        gw.free()


def test_reused_device_blocks_give_exact_graphs(gsn):
    """A context hands a released graph's device blocks to later builds
    (stale contents included): a smaller catalogue built into a larger one's
    blocks, two graphs alive at once, and a graph released after its context
    all count exactly."""
    L, rmax, nb = 30.0, 2.4, 6
    big = synth.neyman_scott(12_000, 25, 0.8, L, 401)
    small = synth.uniform(5_000, L, 402)
    other = synth.uniform(7_000, L, 403)
    ref_small = oracle.count_3pcf(small, L, 0.0, rmax, nb)
    ref_other = oracle.count_3pcf(other, L, 0.0, rmax, nb)
    with gsn.Context(0) as c:
        for _ in range(2):
            g = c.build_graph(big, L, 0.0, rmax, nb)
            g.free()
            g = c.build_graph(small, L, 0.0, rmax, nb)
            h = c.build_graph(other, L, 0.0, rmax, nb)
            got_s, got_o = c.count_3pcf(g), c.count_3pcf(h)
            assert np.array_equal(got_s.hist, ref_small.hist) and got_s.n_triangles == ref_small.n_triangles
            assert np.array_equal(got_o.hist, ref_other.hist) and got_o.n_triangles == ref_other.n_triangles
            g.free()
            h.free()
        late = c.build_graph(small, L, 0.0, rmax, nb)
        assert np.array_equal(c.count_3pcf(late).hist, ref_small.hist)
    late.free()   # after the context: its blocks are released with the graph
