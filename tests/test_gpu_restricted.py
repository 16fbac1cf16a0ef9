"""GPU equilateral and mu-binned triangle counts against the CPU oracle
(bit for bit, counts and exact 128-bit weighted sums)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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


def signed_weights(n, seed):
    m = synth.uniform_values(n, 0.5, 1.0, seed)
    s = synth.uniform_values(n, 0.0, 1.0, seed + 1)
    return np.where(s < 0.4, -m, m)


CASES = [
    ("uniform", lambda: synth.uniform(20000, 80.0, 701), 80.0, 0.0, 4.0, 6),
    ("clustered", lambda: synth.neyman_scott(30000, 50, 1.5, 100.0, 702), 100.0, 0.0, 4.0, 10),
    ("rmin", lambda: synth.uniform(8000, 40.0, 703), 40.0, 1.0, 3.5, 5),
    ("dense_wrap", lambda: synth.uniform(600, 8.0, 704), 8.0, 0.0, 2.5, 4),
    ("dyadic_ties", lambda: synth.dyadic_uniform(3000, 16.0, 705, bits=5), 16.0, 0.0, 1.6, 4),
    ("one_bin", lambda: synth.uniform(5000, 30.0, 706), 30.0, 0.0, 3.0, 1),
]


def diag(nb, hist):
    return np.array([hist[oracle.config_index(nb, b, b, b)] for b in range(nb)], dtype=np.uint64)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_equilateral_matches_oracle(ctx, case):
    name, mk, L, rmin, rmax, nb = case
    x = mk()
    say("equilateral", name, len(x))
    g = ctx.build_graph(x, L, rmin, rmax, nb)
    got = ctx.count_3pcf_equilateral(g)
    g.free()
    ref = oracle.count_3pcf(x, L, rmin, rmax, nb)
    assert np.array_equal(got.hist, diag(nb, ref.hist))
    assert got.n_triangles == int(diag(nb, ref.hist).sum())


def test_equilateral_weighted_and_anchored(ctx):
    x = synth.neyman_scott(30000, 50, 1.5, 100.0, 711)
    w = signed_weights(len(x), 712)
    g = ctx.build_graph(x, 100.0, 0.0, 4.0, 8, weights=w)
    got = ctx.count_3pcf_equilateral(g, weighted=True)
    part = ctx.count_3pcf_equilateral(g, anchors=(5000, 21000), weighted=True)
    g.free()
    ref = oracle.count_3pcf(x, 100.0, 0.0, 4.0, 8, weights=w)
    refp = oracle.count_3pcf(x, 100.0, 0.0, 4.0, 8, weights=w, anchors=(5000, 21000))
    idx = [oracle.config_index(8, b, b, b) for b in range(8)]
    assert np.array_equal(got.hist, ref.hist[idx]) and got.wscale == ref.wscale
    assert got.wsum_int() == [ref.wsum_int()[i] for i in idx]
    assert np.array_equal(part.hist, refp.hist[idx])
    assert part.wsum_int() == [refp.wsum_int()[i] for i in idx]


MU_CASES = [
    ("uniform", lambda: synth.uniform(20000, 80.0, 721), 80.0, 0.0, 4.0, 6, 5),
    ("clustered", lambda: synth.neyman_scott(30000, 50, 1.5, 100.0, 722), 100.0, 0.0, 4.0, 8, 8),
    ("dense_wrap", lambda: synth.uniform(600, 8.0, 723), 8.0, 0.0, 2.5, 4, 3),
    ("dyadic_ties", lambda: synth.dyadic_uniform(3000, 16.0, 724, bits=5), 16.0, 0.0, 1.6, 4, 5),
    ("one_mu_bin", lambda: synth.uniform(5000, 30.0, 725), 30.0, 0.0, 3.0, 3, 1),
]


@pytest.mark.parametrize("case", MU_CASES, ids=[c[0] for c in MU_CASES])
def test_mu_matches_oracle(ctx, case):
    name, mk, L, rmin, rmax, nb, nmu = case
    x = mk()
    say("mu", name, len(x))
    g = ctx.build_graph(x, L, rmin, rmax, nb, keep_coords=True)
    got = ctx.count_3pcf_mu(g, nmu)
    g.free()
    ref = oracle.count_3pcf_mu(x, L, rmin, rmax, nb, nmu)
    assert got.n_triangles == ref.n_triangles
    assert np.array_equal(got.hist, ref.hist)


def test_mu_weighted_anchored_and_needs_coords(ctx, gsn):
    x = synth.neyman_scott(20000, 50, 1.5, 80.0, 731)
    w = signed_weights(len(x), 732)
    g = ctx.build_graph(x, 80.0, 0.0, 4.0, 6, weights=w, keep_coords=True)
    got = ctx.count_3pcf_mu(g, 4, weighted=True, anchors=(2000, 13000))
    g.free()
    ref = oracle.count_3pcf_mu(x, 80.0, 0.0, 4.0, 6, 4, weights=w, anchors=(2000, 13000))
    assert np.array_equal(got.hist, ref.hist) and got.wsum_int() == ref.wsum_int()
    g = ctx.build_graph(x, 80.0, 0.0, 4.0, 6)
    with pytest.raises(gsn.GsError) as e:
        ctx.count_3pcf_mu(g, 4)
    g.free()
    assert e.value.code == gsn.GS_ENOCOORDS
