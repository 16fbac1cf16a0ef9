"""GPU parity-decomposed 4-clique counts against the CPU oracle (bit-exact),
the hand-derived lattice and chiral closed forms, and exact reflection."""
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


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def gpu4(ctx, x, L, rmin, rmax, nb, anchors=None):
    g = ctx.build_graph(x, L, rmin, rmax, nb, keep_coords=True)
    try:
        return ctx.count_4pcf_parity(g, anchors=anchors)
    finally:
        g.free()


def same(got, ref):
    assert got.n_cliques == ref.n_cliques
    assert np.array_equal(got.even, ref.even)
    assert np.array_equal(got.pos, ref.pos)
    assert np.array_equal(got.neg, ref.neg)


CASES = [
    ("uniform_dense", lambda: synth.uniform(110, 8.0, 31), 8.0, 0.0, 2.6, 4),
    ("clustered_small", lambda: synth.neyman_scott(110, 22, 0.7, 10.0, 32), 10.0, 0.0, 2.0, 5),
    ("rmin", lambda: synth.uniform(100, 7.0, 33), 7.0, 0.5, 2.5, 3),
    ("single_cell", lambda: synth.uniform(200, 9.0, 34), 9.0, 0.0, 3.0, 4),
    ("uniform_mid", lambda: synth.uniform(6000, 40.0, 35), 40.0, 0.0, 3.2, 8),
    ("clustered_mid", lambda: synth.neyman_scott(8000, 50, 1.2, 60.0, 36), 60.0, 0.0, 3.0, 8),
    ("dyadic_ties", lambda: synth.dyadic_uniform(2000, 16.0, 37, bits=5), 16.0, 0.0, 1.6, 4),
    ("many_bins", lambda: synth.uniform(1500, 12.0, 38), 12.0, 0.0, 2.2, 30),
    ("rmin_bins13", lambda: synth.neyman_scott(5000, 40, 1.0, 30.0, 39), 30.0, 1.1, 3.3, 13),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_count4_matches_oracle(ctx, case):
    name, mk, L, rmin, rmax, nb = case
    x = mk()
    say("count4", name, len(x))
    got = gpu4(ctx, x, L, rmin, rmax, nb)
    ref = oracle.count_4pcf_parity(x, L, rmin, rmax, nb)
    same(got, ref)
    assert int(got.even.sum()) == 4 * got.n_cliques


def test_count4_uniform_c1_full(ctx):
    w = synth.workload("uniform_3pcf")
    say("count4 C1", w.n)
    got = gpu4(ctx, w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    ref = oracle.count_4pcf_parity(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    same(got, ref)


def test_count4_ns_scaled(ctx):
    w = synth.workload("ns_4pcf_parity", volume_fraction=1.0 / 64)
    say("count4 ns 1/64", w.n)
    got = gpu4(ctx, w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    ref = oracle.count_4pcf_parity(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    same(got, ref)


def test_count4_full_size_ns_sampled_anchors(ctx):
    gold = _golden("ns_4pcf_parity_sampled.json")
    w = synth.workload("ns_4pcf_parity")
    assert hashlib.sha256(np.ascontiguousarray(w.xyz).tobytes()).hexdigest() == gold["xyz_sha256"]
    say("count4 full ns sampled", w.n)
    g = ctx.build_graph(w.xyz, w.box, w.rmin, w.rmax, w.nbins, keep_coords=True)
    full = ctx.count_4pcf_parity(g)
    for s in gold["samples"]:
        got = ctx.count_4pcf_parity(g, anchors=(s["lo"], s["hi"]))
        assert got.n_cliques == s["n_cliques"]
        assert got.even.tolist() == s["even"]
        assert got.pos.tolist() == s["pos"]
        assert got.neg.tolist() == s["neg"]
    again = ctx.count_4pcf_parity(g)
    g.free()
    assert int(full.even.sum()) == 4 * full.n_cliques
    assert np.all(full.pos + full.neg <= full.even)
    assert np.array_equal(again.even, full.even) and np.array_equal(again.pos, full.pos)


def test_count4_anchor_partition(ctx):
    x = synth.neyman_scott(8000, 50, 1.2, 60.0, 36)
    g = ctx.build_graph(x, 60.0, 0.0, 3.0, 8, keep_coords=True)
    full = ctx.count_4pcf_parity(g)
    acc = [np.zeros_like(full.even) for _ in range(3)]
    nk = 0
    for lo, hi in [(0, 1000), (1000, 1001), (1001, 5555), (5555, 8000)]:
        r = ctx.count_4pcf_parity(g, anchors=(lo, hi))
        for a_, v in zip(acc, (r.even, r.pos, r.neg)):
            a_ += v
        nk += r.n_cliques
    g.free()
    assert nk == full.n_cliques
    assert np.array_equal(acc[0], full.even)
    assert np.array_equal(acc[1], full.pos) and np.array_equal(acc[2], full.neg)


def test_count4_forced_flushes_identical(ctx, monkeypatch):
    x = synth.neyman_scott(8000, 50, 1.2, 60.0, 36)
    ref = gpu4(ctx, x, 60.0, 0.0, 3.0, 8)
    monkeypatch.setenv("GS_FLUSH_LIMIT", str(4 * 256 * 200))
    got = gpu4(ctx, x, 60.0, 0.0, 3.0, 8)
    same(got, ref)


def test_count4_bin_search_identical(ctx, monkeypatch):
    # the local separations' bins by a search of the thresholds instead of
    # the float32 estimate and its one-step correction
    x = synth.neyman_scott(8000, 50, 1.2, 60.0, 42)
    ref = gpu4(ctx, x, 60.0, 0.4, 3.0, 11)
    monkeypatch.setenv("GS_BIN_SEARCH", "1")
    got = gpu4(ctx, x, 60.0, 0.4, 3.0, 11)
    same(got, ref)
    same(got, oracle.count_4pcf_parity(x, 60.0, 0.4, 3.0, 11))


def test_count4_block256_identical(ctx, monkeypatch):
    x = synth.neyman_scott(8000, 50, 1.2, 60.0, 41)
    ref = gpu4(ctx, x, 60.0, 0.0, 3.0, 8)
    monkeypatch.setenv("GS_BLOCK4", "256")
    got = gpu4(ctx, x, 60.0, 0.0, 3.0, 8)
    same(got, ref)
    same(got, oracle.count_4pcf_parity(x, 60.0, 0.0, 3.0, 8))


def test_lattice_closed_forms_gpu(ctx):
    g = _golden("lattice_sc.json")
    m = g["sites_per_axis"]
    a = np.arange(m, dtype=np.float64)
    X, Y, Z = np.meshgrid(a, a, a, indexing="ij")
    x = np.mod(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + np.array([0.25, 0.5, 0.125]), g["box"])
    nsite = len(x)
    nb = g["nbins"]
    got = gpu4(ctx, x, g["box"], g["rmin"], g["rmax"], nb)
    assert got.n_cliques == g["cliques_per_site"] * nsite
    exp = np.zeros(oracle.n_configs(nb), dtype=np.uint64)
    for key, v in g["hub_contributions_per_site"].items():
        exp[oracle.config_index(nb, *map(int, key.split(",")))] = v * nsite
    assert np.array_equal(got.even, exp)
    assert got.pos.sum() == 0 and got.neg.sum() == 0


def test_chiral_injection_gpu(ctx):
    g = _golden("chiral_unit.json")
    L, rmin, rmax, nb = g["box"], g["rmin"], g["rmax"], g["nbins"]
    off = g["offsets"]
    handed = [1] * 320 + [-1] * 180
    order = synth.permutation(len(handed), 9)
    handed = [handed[i] for i in order]
    pts = []
    per = int(L // 8.0)
    for u, h in enumerate(handed):
        O = np.array([(u // (per * per)) * 8.0, ((u // per) % per) * 8.0, (u % per) * 8.0]) + [2.25, 2.5, 2.75]
        pts.append(O)
        for nm in ("A", "B", "C"):
            v = np.array(off[nm], dtype=np.float64)
            v[0] *= h
            pts.append(O + v)
    x = np.mod(np.array(pts), L)
    got = gpu4(ctx, x, L, rmin, rmax, nb)
    unit = np.zeros(oracle.n_configs(nb), dtype=np.int64)
    for t in g["pos_configs"]:
        unit[oracle.config_index(nb, *t)] += 1
    for t in g["neg_configs"]:
        unit[oracle.config_index(nb, *t)] -= 1
    assert got.n_cliques == 500
    assert np.array_equal(got.odd, (320 - 180) * unit)


def test_reflection_swaps_channels_gpu(ctx):
    L = 16.0
    x = synth.dyadic_uniform(3000, L, 41)
    y = x.copy()
    y[:, 0] = np.mod(L - y[:, 0], L)
    a = gpu4(ctx, x, L, 0.0, 1.6, 4)
    b = gpu4(ctx, y, L, 0.0, 1.6, 4)
    assert a.n_cliques > 1000
    assert np.array_equal(a.even, b.even)
    assert np.array_equal(a.pos, b.neg) and np.array_equal(a.neg, b.pos)


def test_count3_forced_flushes_identical(ctx, monkeypatch):
    x = synth.neyman_scott(20000, 50, 1.2, 80.0, 39)
    w = synth.uniform_values(len(x), 0.5, 1.0, 40)
    g = ctx.build_graph(x, 80.0, 0.0, 4.0, 9, weights=w)
    ref = ctx.count_3pcf(g, weighted=True)
    monkeypatch.setenv("GS_FLUSH_LIMIT", str(256 * 400))
    got = ctx.count_3pcf(g, weighted=True)
    g.free()
    assert np.array_equal(got.hist, ref.hist) and got.wsum_int() == ref.wsum_int()


# hand-derived degenerate-rule units (tests/golden/degenerate_units.json)
from tests import units as _units  # noqa: E402


@pytest.mark.parametrize("k_exp", [None, -30, 30, -29, 29, -28, 28])
def test_degenerate_rule_units_gpu(ctx, k_exp):
    g = _golden("degenerate_units.json")
    L, rmin, rmax, nb = g["box"], g["rmin"], g["rmax"], g["nbins"]
    lifted = g["lifted"]
    names = ["O", "A", "B", "C"]
    if k_exp is None:
        off, signs = _units.offsets(g["coplanar"], names), {}
    else:
        eps = float(np.sign(k_exp)) * 2.0 ** (-abs(k_exp))
        off = _units.offsets(g["coplanar"], names, lift=lifted["lift_vertex"], eps=eps)
        signs = {h: int(np.sign(k_exp)) * lifted["signs_eps_positive"][h]
                 for h in lifted["signed_hubs"][str(-abs(k_exp))]}
    n_units = 300      # interior units and units near the box faces
    x = _units.place([off] * n_units, L)
    say("degenerate units", k_exp, len(x))
    got = gpu4(ctx, x, L, rmin, rmax, nb)
    even, odd = _units.expected_parity(nb, oracle.config_index, g["coplanar"]["hub_configs"], signs)
    assert got.n_cliques == n_units
    assert np.array_equal(got.even.astype(np.int64), n_units * even)
    assert np.array_equal(got.odd, n_units * odd)
    assert int(got.pos.sum() + got.neg.sum()) == n_units * int(np.abs(odd).sum())
    same(got, oracle.count_4pcf_parity(x, L, rmin, rmax, nb))


def test_degenerate_rule_zero_length_spoke_gpu(ctx):
    g = _golden("degenerate_units.json")
    L, rmin, rmax, nb = g["box"], g["rmin"], g["rmax"], g["nbins"]
    c = g["coincident"]
    x = _units.place([_units.offsets(c, ["P", "Q", "X", "Y"])] * 200, L)
    got = gpu4(ctx, x, L, rmin, rmax, nb)
    even, _ = _units.expected_parity(nb, oracle.config_index, c["hub_configs"], {})
    assert got.n_cliques == 200
    assert np.array_equal(got.even.astype(np.int64), 200 * even)
    assert got.pos.sum() == 0 and got.neg.sum() == 0
    same(got, oracle.count_4pcf_parity(x, L, rmin, rmax, nb))
