"""Batched counts over many catalogues and the continuous-batching server:
every catalogue's histogram is bit-identical alone and in the mix, and equal
to the oracle's."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

L, RMAX, NB = 200.0, 10.0, 10


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


def catalogues(count, seed, lo=2_000, hi=30_000):
    """Uneven sizes, alternating clustered data and uniform randoms."""
    sizes = np.floor(np.exp(np.log(lo) + synth.uniform_values(count, 0.0, 1.0, seed) *
                            (np.log(hi) - np.log(lo)))).astype(int)
    out = []
    for k, n in enumerate(sizes):
        if k % 2 == 0:
            out.append(synth.neyman_scott(int(n), 50, 2.0, L, seed * 1000 + k))
        else:
            out.append(synth.uniform(int(n), L, seed * 1000 + k))
    return out


def ref3(x, nb=NB):
    """The oracle's histogram of catalogue x."""
    return oracle.count_3pcf(x, L, 0.0, RMAX, nb).hist


def alone(ctx, x):
    g = ctx.build_graph(x, L, 0.0, RMAX, NB)
    r = ctx.count_3pcf(g)
    g.free()
    return r


def test_batch_matches_individual_and_oracle(ctx):
    cats = catalogues(14, 3)
    gs = [ctx.build_graph(x, L, 0.0, RMAX, NB) for x in cats]
    say("batch of", len(gs))
    got = ctx.count_3pcf_batch(gs)
    for g in gs:
        g.free()
    for k, x in enumerate(cats):
        a = alone(ctx, x)
        assert got[k].n_triangles == a.n_triangles and np.array_equal(got[k].hist, a.hist)
        assert np.array_equal(got[k].hist, ref3(x))


def test_batch_of_one_and_with_empty_catalogue(ctx):
    x = synth.uniform(5000, L, 5)
    g = ctx.build_graph(x, L, 0.0, RMAX, NB)
    e = ctx.build_graph(np.zeros((0, 3)), L, 0.0, RMAX, NB)
    one = ctx.count_3pcf_batch([g])
    two = ctx.count_3pcf_batch([e, g, e])
    a = ctx.count_3pcf(g)
    g.free()
    e.free()
    assert np.array_equal(one[0].hist, a.hist)
    assert np.array_equal(two[1].hist, a.hist) and two[0].n_triangles == 0 and two[2].hist.sum() == 0


def test_batch_rejects_mixed_bins(ctx, gsn):
    x = synth.uniform(1000, L, 6)
    a = ctx.build_graph(x, L, 0.0, RMAX, NB)
    b = ctx.build_graph(x, L, 0.0, RMAX, NB + 1)
    with pytest.raises(gsn.GsError) as e:
        ctx.count_3pcf_batch([a, b])
    a.free()
    b.free()
    assert e.value.code == gsn.GS_EINVAL


def drain(ctx, tickets, timeout=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        assert time.time() - t0 < timeout, "serving did not finish"
        for t in tickets:
            if t not in res:
                r = ctx.poll(t, NB)
                if r is not None:
                    res[t] = r
        time.sleep(0.002)
    return res


def test_serving_alone_vs_mix(gsn):
    cats = catalogues(24, 7)
    with gsn.Context(0) as c:
        want = [alone(c, x) for x in cats]
    with gsn.Context(0) as s:
        say("serving", len(cats))
        tickets = []
        for k, x in enumerate(cats):
            tickets.append(s.submit(x, L, 0.0, RMAX, NB))
            if k % 5 == 4:
                time.sleep(0.003)   # arrivals spread over several steps
        res = drain(s, tickets)
    steps = []
    for t, x, a in zip(tickets, cats, want):
        r = res[t]
        assert r["status"] == gsn.GS_DONE
        assert r["n_triangles"] == a.n_triangles
        assert np.array_equal(r["hist"], a.hist)
        assert np.array_equal(r["hist"], ref3(x))
        assert r["t_total_s"] >= r["t_count_s"] >= 0
        steps.append(r["step_size"])
    assert max(steps) > 1, "no request was batched with another"


def test_serving_failures_cancel_and_unknown(gsn):
    cats = catalogues(6, 9)
    bad = cats[2].copy()
    bad[10, 0] = L          # outside [0, L)
    with gsn.Context(0) as s:
        ts = [s.submit(x, L, 0.0, RMAX, NB) for x in cats[:2]]
        tb = s.submit(bad, L, 0.0, RMAX, NB)
        tc = [s.submit(x, L, 0.0, RMAX, NB) for x in cats[3:]]
        s.cancel(tc[-1])
        res = drain(s, ts + [tb] + tc)
        with pytest.raises(gsn.GsError) as e:
            s.poll(ts[0], NB)       # retired
        assert e.value.code == gsn.GS_ENOTFOUND
        with pytest.raises(gsn.GsError) as e:
            s.poll(123456789, NB)
        assert e.value.code == gsn.GS_ENOTFOUND
        with pytest.raises(gsn.GsError) as e:
            s.submit(cats[0], L, 0.0, L, NB)   # rmax >= L/2
        assert e.value.code == gsn.GS_EINVAL
    assert res[tb]["status"] == gsn.GS_FAILED and res[tb]["error"] == gsn.GS_EINVAL
    assert res[tc[-1]]["status"] in (gsn.GS_CANCELLED, gsn.GS_DONE)
    with gsn.Context(0) as c:
        for t, x in zip(ts + tc[:-1], cats[:2] + cats[3:-1]):
            assert res[t]["status"] == gsn.GS_DONE
            assert np.array_equal(res[t]["hist"], alone(c, x).hist)
            assert np.array_equal(res[t]["hist"], ref3(x))


def test_serving_small_budget_admits_one_at_a_time(gsn):
    cats = catalogues(8, 11, lo=20_000, hi=25_000)
    with gsn.Context(0) as c:
        want = [alone(c, x) for x in cats]
        g = c.build_graph(cats[0], L, 0.0, RMAX, NB)
        fp = g.info().device_bytes
        g.free()
    with gsn.Context(0, budget_bytes=int(fp * 1.3)) as s:
        ts = [s.submit(x, L, 0.0, RMAX, NB) for x in cats]
        res = drain(s, ts)
    for t, a, x in zip(ts, want, cats):
        assert res[t]["status"] == gsn.GS_DONE and np.array_equal(res[t]["hist"], a.hist)
        assert np.array_equal(res[t]["hist"], ref3(x))
        assert res[t]["step_size"] <= 2


def test_serving_mixed_bin_counts(gsn):
    """Requests with different bin counts are counted in separate steps, each
    with the histogram layout of its own bin count."""
    cats = catalogues(10, 13, lo=3_000, hi=12_000)
    nbs = [NB if k % 2 == 0 else NB + 3 for k in range(len(cats))]
    with gsn.Context(0) as c:
        want = []
        for x, nb in zip(cats, nbs):
            g = c.build_graph(x, L, 0.0, RMAX, nb)
            want.append(c.count_3pcf(g).hist)
            g.free()
    with gsn.Context(0) as s:
        ts = [s.submit(x, L, 0.0, RMAX, nb) for x, nb in zip(cats, nbs)]
        res = {}
        t0 = time.time()
        while len(res) < len(ts):
            assert time.time() - t0 < 120.0, "serving did not finish"
            for t, nb in zip(ts, nbs):
                if t not in res:
                    r = s.poll(t, nb)
                    if r is not None:
                        res[t] = r
            time.sleep(0.002)
    for t, w, x, nb in zip(ts, want, cats, nbs):
        assert res[t]["status"] == gsn.GS_DONE and np.array_equal(res[t]["hist"], w)
        assert np.array_equal(res[t]["hist"], ref3(x, nb))


def test_serving_stream_catalogues_against_stored_oracle(gsn):
    """Catalogues of the serving stream (periodic 600 Mpc/h boxes, 5e4 to
    2.5e5 points, clustered and uniform, rmax 40, 10 bins), served together
    with arrivals spread over several steps: every histogram equals the
    stored oracle count."""
    import hashlib
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "stream_served.json")))
    Ls, rmax, nb = gold["box"], gold["rmax"], gold["nbins"]
    cats = []
    for c in gold["catalogues"]:
        x = synth.stream_catalogue(c["index"], c["n"], L=Ls, seed=gold["seed"])
        assert hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest() == c["xyz_sha256"]
        cats.append(x)
    with gsn.Context(0) as s:
        say("serving stream catalogues", len(cats))
        ts = []
        for k, x in enumerate(cats):
            ts.append(s.submit(x, Ls, 0.0, rmax, nb))
            if k % 4 == 3:
                time.sleep(0.01)
        res = {}
        t0 = time.time()
        while len(res) < len(ts):
            assert time.time() - t0 < 120.0, "serving did not finish"
            for t in ts:
                if t not in res:
                    r = s.poll(t, nb)
                    if r is not None:
                        res[t] = r
            time.sleep(0.002)
    for t, c in zip(ts, gold["catalogues"]):
        assert res[t]["status"] == gsn.GS_DONE
        assert res[t]["n_triangles"] == c["n_triangles"]
        assert res[t]["hist"].tolist() == c["hist"]


def test_serving_mixed_kinds_against_oracle(gsn):
    """A stream mixing plain triangle counts, exact weighted triangle sums and
    parity-decomposed 4-clique counts, arriving over several steps: every
    result equals the oracle's (bit for bit, 128-bit weighted sums too)."""
    cats = catalogues(12, 17, lo=2_000, hi=12_000)
    kinds = []
    reqs = []
    for k, x in enumerate(cats):
        kind = ("3pcf", "w3pcf", "4pcf")[k % 3]
        w = synth.uniform_values(len(x), 0.5, 1.0, 1700 + k) if kind == "w3pcf" else None
        kinds.append(kind)
        reqs.append((x, w))
    rmax4 = 6.0
    with gsn.Context(0) as s:
        say("serving mixed kinds", len(cats))
        ts = []
        for k, ((x, w), kind) in enumerate(zip(reqs, kinds)):
            if kind == "4pcf":
                ts.append(s.submit(x, L, 0.0, rmax4, NB, kind=gsn.GS_4PCF_PARITY))
            else:
                ts.append(s.submit(x, L, 0.0, RMAX, NB, weights=w))
            if k % 4 == 3:
                time.sleep(0.005)
        res = drain(s, ts)
    for t, (x, w), kind in zip(ts, reqs, kinds):
        r = res[t]
        assert r["status"] == gsn.GS_DONE, (kind, r)
        if kind == "4pcf":
            ref = oracle.count_4pcf_parity(x, L, 0.0, rmax4, NB)
            assert r["n_tuples"] == ref.n_cliques
            assert np.array_equal(r["hist"], ref.even)
            assert np.array_equal(r["pos"], ref.pos) and np.array_equal(r["neg"], ref.neg)
        else:
            ref = oracle.count_3pcf(x, L, 0.0, RMAX, NB, weights=w)
            assert r["n_tuples"] == ref.n_triangles
            assert np.array_equal(r["hist"], ref.hist)
            if kind == "w3pcf":
                assert r["wscale"] == ref.wscale
                assert np.array_equal(r["wsum"], ref.wsum)
                assert np.array_equal(r["whist"], ref.whist())


def test_serving_rejects_bad_kinds(gsn):
    x = synth.uniform(1000, L, 19)
    with gsn.Context(0) as s:
        with pytest.raises(gsn.GsError) as e:
            s.submit(x, L, 0.0, RMAX, NB, kind=7)
        assert e.value.code == gsn.GS_EINVAL
        with pytest.raises(gsn.GsError) as e:
            s.submit(x, L, 0.0, RMAX, NB, weights=np.ones(len(x)), kind=gsn.GS_4PCF_PARITY)
        assert e.value.code == gsn.GS_EINVAL
