"""GPU estimators (compute_3pcf / compute_4pcf) against the oracle's
estimators on the oracle's counts: every estimate bit for bit (the exact
sums are identical and every division and product is taken in the same
order), plus the estimator identities of the paper."""
import sys

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


def same(a, b):
    np.testing.assert_array_equal(np.asarray(a), np.asarray(b))


@pytest.mark.parametrize("case", ["clustered", "weighted_wide"])
def test_compute_3pcf_matches_oracle(ctx, gsn, case):
    L = 60.0
    xd = synth.neyman_scott(6000, 30, 1.5, L, 801)
    xr = synth.uniform(18000 if case == "clustered" else 60000, L, 802)
    wd = synth.uniform_values(len(xd), 0.8, 0.4, 803)
    wr = None if case == "clustered" else synth.uniform_values(len(xr), 0.9, 0.2, 804)
    say("compute_3pcf", case)
    got = gsn.compute_3pcf(xd, wd, xr, wr, 0.0, 4.0, 6, L, ctx=ctx)
    ref = oest.compute_3pcf(xd, wd, xr, wr, L, 0.0, 4.0, 6)
    same(got.NNN, ref.nnn)
    same(got.RRR, ref.rrr)
    same(got.zeta, ref.zeta)
    assert got.r1[0] == got.r2[0] == got.r3[0] == 4.0 / 12


def test_compute_3pcf_randoms_as_data_give_zero(ctx, gsn):
    """Data drawn as the randoms themselves: every data-minus-random tuple
    cancels exactly, so NNN = 0 and zeta = 0 wherever RRR > 0."""
    L = 40.0
    xr = synth.uniform(12000, L, 811)
    got = gsn.compute_3pcf(xr, None, xr, None, 0.0, 3.0, 5, L, ctx=ctx)
    assert np.all(got.NNN == 0.0)
    assert np.all(got.zeta[got.RRR > 0] == 0.0)


def test_compute_4pcf_matches_oracle(ctx, gsn):
    L = 40.0
    xd = synth.neyman_scott(3000, 30, 0.9, L, 821)
    xr = synth.uniform(9000, L, 822)
    wd = synth.uniform_values(len(xd), 0.8, 0.4, 823)
    say("compute_4pcf")
    got = gsn.compute_4pcf(xd, wd, xr, None, 0.0, 2.6, 4, L, ctx=ctx)
    ref = oest.compute_4pcf(xd, wd, xr, None, L, 0.0, 2.6, 4)
    for k in ("zeta_even", "zeta_odd", "nnnn_even", "nnnn_odd", "rrrr_even", "xi", "zeta6", "zeta6_disc",
              "zeta6_conn", "zeta_even_disc", "zeta_even_conn"):
        same(getattr(got, k), getattr(ref, k))
    # the even channel's random sum is the 6-edge random sums spread over hubs
    assert np.isfinite(got.zeta_even_disc[got.rrrr_even > 0]).all()


def test_compute_4pcf_without_connected_part_on_many_bins(ctx, gsn):
    L = 30.0
    xd = synth.neyman_scott(2000, 20, 0.8, L, 831)
    xr = synth.uniform(4000, L, 832)
    got = gsn.compute_4pcf(xd, None, xr, None, 0.0, 2.4, 14, L, connected=False, ctx=ctx)
    ref = oest.compute_4pcf(xd, None, xr, None, L, 0.0, 2.4, 14, connected=False)
    same(got.zeta_even, ref.zeta_even)
    same(got.zeta_odd, ref.zeta_odd)
    with pytest.raises(gsn.GsError) as e:
        gsn.compute_4pcf(xd, None, xr, None, 0.0, 2.4, 14, L, connected=True, ctx=ctx)
    assert e.value.code == gsn.GS_EINVAL or e.value.code == gsn.GS_EUNSUPPORTED
