"""Survey geometry (no periodic wrap) on the GPU against the oracle: edges
and bins, triangles, parity and 6-edge 4-cliques, equilateral and mu counts,
the estimators and a served request, bit for bit."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from oracle import estimator as oest

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


def survey(n, L, seed):
    """Clustered points filling the cube edge to edge (Neyman-Scott children
    wrapped into the cube: the faces cut clusters, as survey edges do)."""
    return synth.neyman_scott(n, 40, 1.2, L, seed)


CASES = [("clustered", 20000, 60.0, 0.0, 3.0, 6), ("rmin", 12000, 40.0, 0.5, 3.0, 5),
         ("large_rmax", 3000, 12.0, 0.0, 7.0, 4), ("few_cells", 5000, 16.0, 0.0, 6.0, 4)]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_survey_graph_and_triangles(ctx, case):
    name, n, L, rmin, rmax, nb = case
    x = survey(n, L, 1001)
    say("survey", name, n)
    g = ctx.build_graph(x, L, rmin, rmax, nb, periodic=False)
    rp, col, b, perm = g.export()
    got = ctx.count_3pcf(g)
    g.free()
    orp, ocol, ob = oracle.graph(x, L, rmin, rmax, nb, periodic=False)
    # forward edges in original labels must be the oracle's undirected edge set
    gi = np.repeat(np.arange(len(rp) - 1), np.diff(rp.astype(np.int64)))
    a, c = perm[gi].astype(np.int64), perm[col].astype(np.int64)
    mine = set(zip(np.minimum(a, c), np.maximum(a, c), b))
    oi = np.repeat(np.arange(len(orp) - 1), np.diff(orp))
    theirs = {(int(i), int(j), int(bb)) for i, j, bb in zip(oi, ocol, ob) if i < j}
    assert {(int(i), int(j), int(bb)) for i, j, bb in mine} == theirs
    ref = oracle.count_3pcf(x, L, rmin, rmax, nb, periodic=False)
    assert got.n_triangles == ref.n_triangles and np.array_equal(got.hist, ref.hist)


def test_survey_four_point_and_restricted(ctx):
    L = 40.0
    x = survey(8000, L, 1002)
    w = synth.uniform_values(len(x), 0.5, 1.0, 1003)
    g = ctx.build_graph(x, L, 0.0, 2.8, 4, weights=w, keep_coords=True, periodic=False)
    par = ctx.count_4pcf_parity(g, weighted=True)
    six = ctx.count_4pcf_full(g, weighted=True)
    eq = ctx.count_3pcf_equilateral(g)
    mu = ctx.count_3pcf_mu(g, 5)
    g.free()
    rp = oracle.count_4pcf_parity(x, L, 0.0, 2.8, 4, weights=w, periodic=False)
    assert np.array_equal(par.even, rp.even) and np.array_equal(par.pos, rp.pos)
    assert np.array_equal(par.neg, rp.neg)
    for ch in range(3):
        assert par.wsum_int(ch) == rp.wsum_int(ch)
    r6 = oracle.count_4pcf_full(x, L, 0.0, 2.8, 4, weights=w, periodic=False)
    assert np.array_equal(six.hist, r6.hist) and six.wsum_int() == r6.wsum_int()
    r3 = oracle.count_3pcf(x, L, 0.0, 2.8, 4, periodic=False)
    assert np.array_equal(eq.hist, np.array([r3.hist[oracle.config_index(4, k, k, k)] for k in range(4)],
                                            dtype=np.uint64))
    rm = oracle.count_3pcf_mu(x, L, 0.0, 2.8, 4, 5, periodic=False)
    assert np.array_equal(mu.hist, rm.hist)


def test_survey_estimators(ctx, gsn):
    L = 40.0
    xd = survey(3000, L, 1004)
    xr = synth.uniform(9000, L, 1005)
    got3 = gsn.compute_3pcf(xd, None, xr, None, 0.0, 3.5, 5, L, ctx=ctx, periodic=False)
    ref3 = oest.compute_3pcf(xd, None, xr, None, L, 0.0, 3.5, 5, periodic=False)
    np.testing.assert_array_equal(got3.zeta, ref3.zeta)
    got4 = gsn.compute_4pcf(xd, None, xr, None, 0.0, 2.6, 3, L, ctx=ctx, periodic=False)
    ref4 = oest.compute_4pcf(xd, None, xr, None, L, 0.0, 2.6, 3, periodic=False)
    for k in ("zeta_even", "zeta_odd", "zeta6", "zeta6_conn", "zeta_even_conn", "xi"):
        np.testing.assert_array_equal(getattr(got4, k), getattr(ref4, k))


def test_survey_served_request(ctx, gsn):
    L = 50.0
    x = survey(10000, L, 1006)
    with gsn.Context(0) as s:
        t = s.submit(x, L, 0.0, 3.0, 6, periodic=False)
        r = None
        t0 = time.time()
        while r is None and time.time() - t0 < 60:
            r = s.poll(t, 6)
            time.sleep(0.002)
    assert r is not None and r["status"] == gsn.GS_DONE
    ref = oracle.count_3pcf(x, L, 0.0, 3.0, 6, periodic=False)
    assert np.array_equal(r["hist"], ref.hist)
