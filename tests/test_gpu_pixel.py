"""GPU parity counts from direction pixels (the paper's own parity
computation) against the oracle, bit for bit, with the exact reflection
swap and survey geometry."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2607_06604_amd as m
    m.load()
    c = m.Context(0)
    yield c
    c.close()


CASES = [
    ("uniform", lambda: synth.uniform(6000, 40.0, 1101), 40.0, 0.0, 3.2, 8, True),
    ("clustered", lambda: synth.neyman_scott(8000, 50, 1.2, 60.0, 1102), 60.0, 0.0, 3.0, 6, True),
    ("dense_wrap", lambda: synth.uniform(400, 8.0, 1103), 8.0, 0.0, 2.6, 4, True),
    ("dyadic_ties", lambda: synth.dyadic_uniform(2000, 16.0, 1104, bits=5), 16.0, 0.0, 1.6, 4, True),
    ("many_bins", lambda: synth.uniform(1500, 12.0, 1105), 12.0, 0.0, 2.2, 20, True),
    ("survey", lambda: synth.neyman_scott(6000, 40, 1.0, 40.0, 1106), 40.0, 0.0, 3.0, 5, False),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pixel_parity_matches_oracle(ctx, case):
    name, mk, L, rmin, rmax, nb, periodic = case
    x = mk()
    print("pixel parity", name, len(x), flush=True)
    g = ctx.build_graph(x, L, rmin, rmax, nb, keep_coords=True, periodic=periodic)
    got = ctx.count_4pcf_pixel(g)
    part = ctx.count_4pcf_pixel(g, anchors=(100, 1300))
    g.free()
    ref = oracle.count_4pcf_pixel(x, L, rmin, rmax, nb, periodic=periodic)
    refp = oracle.count_4pcf_pixel(x, L, rmin, rmax, nb, anchors=(100, 1300), periodic=periodic)
    assert got.n_cliques == ref.n_cliques
    assert np.array_equal(got.even, ref.even)
    assert np.array_equal(got.pos, ref.pos) and np.array_equal(got.neg, ref.neg)
    assert np.array_equal(part.pos, refp.pos) and np.array_equal(part.neg, refp.neg)


def test_pixel_parity_reflection_gpu(ctx):
    L = 16.0
    x = synth.dyadic_uniform(3000, L, 1107)
    y = x.copy()
    y[:, 0] = np.mod(L - y[:, 0], L)
    out = []
    for pts in (x, y):
        g = ctx.build_graph(pts, L, 0.0, 1.6, 4, keep_coords=True)
        out.append(ctx.count_4pcf_pixel(g))
        g.free()
    a, b = out
    assert a.n_cliques == b.n_cliques > 0 and np.array_equal(a.even, b.even)
    assert np.array_equal(a.pos, b.neg) and np.array_equal(a.neg, b.pos)
