"""The allocation-free parity count (gs_count_4pcf_parity_noalloc, called
through the C ABI) against gs_count_4pcf_parity: bit-identical on two calls
in a row, the second on a smaller catalogue, then once more on the first."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_parity_matches_allocating_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2607_06604_amd as gsn
    gsn.load()
    with gsn.Context(0) as ctx:
        cases = [(synth.neyman_scott(8000, 50, 1.2, 60.0, 901), 60.0, 3.0, 8),
                 (synth.uniform(1500, 14.0, 902), 14.0, 2.4, 5),
                 (synth.neyman_scott(8000, 50, 1.2, 60.0, 901), 60.0, 3.0, 8)]
        for x, L, rmax, nb in cases:
            say("noalloc parity", len(x), nb)
            g = ctx.build_graph(x, L, 0.0, rmax, nb, keep_coords=True)
            ref = ctx.count_4pcf_parity(g)
            got = ctx.count_4pcf_parity(g, noalloc=True)
            part = ctx.count_4pcf_parity(g, anchors=(100, 900), noalloc=True)
            refp = ctx.count_4pcf_parity(g, anchors=(100, 900))
            g.free()
            assert got.n_cliques == ref.n_cliques > 0
            assert np.array_equal(got.even, ref.even)
            assert np.array_equal(got.pos, ref.pos) and np.array_equal(got.neg, ref.neg)
            assert part.n_cliques == refp.n_cliques and np.array_equal(part.even, refp.even)
            assert np.array_equal(part.pos, refp.pos) and np.array_equal(part.neg, refp.neg)
        # beyond the static scratch: refused, nothing allocated
        x = synth.uniform(300, 10.0, 903)
        g = ctx.build_graph(x, 10.0, 0.0, 2.0, 30, keep_coords=True)   # 4960 configurations
        with pytest.raises(gsn.GsError) as e:
            ctx.count_4pcf_parity(g, noalloc=True)
        g.free()
        assert e.value.code == gsn.GS_EUNSUPPORTED
