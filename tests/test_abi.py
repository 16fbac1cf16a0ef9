"""The C-ABI library loads and exports every function include/gsn.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "gsn.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("gs_build_graph", "gs_count_3pcf", "gs_count_4pcf_parity", "gs_create",
                     "gs_destroy", "gs_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2607_06604_amd as gsn
    lib = ctypes.CDLL(gsn.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(gsn.EXPORTS) == _declared()


def test_strerror_without_device():
    import paper_2607_06604_amd as gsn
    lib = gsn.load()
    assert lib.gs_strerror(0) == b"ok"
    assert lib.gs_strerror(gsn.GS_EINVAL) == b"invalid argument"
    assert lib.gs_strerror(-12345) == b"unknown status"


def test_null_arguments_rejected_without_device():
    import paper_2607_06604_amd as gsn
    lib = gsn.load()
    assert lib.gs_destroy(None) == gsn.GS_EINVAL
    assert lib.gs_graph_free(None) == gsn.GS_EINVAL
    assert lib.gs_graph_info(None, None) == gsn.GS_EINVAL
    assert lib.gs_create(None, 0, 0, None) == gsn.GS_EINVAL


@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5])
def test_six_edge_table_matches_oracle(nb):
    """The library's 6-edge configuration table (host code) against the
    oracle's: the same number of configurations, each oracle configuration's
    smallest tuple ranked at its oracle index, and every tuple ranked as the
    tuples of its relabellings (checked on a sample)."""
    import itertools
    import numpy as np
    import oracle
    import paper_2607_06604_amd as gsn
    n6 = gsn.n_configs6(nb)
    assert n6 == oracle.n_configs6(nb) == (nb ** 6 + 9 * nb ** 4 + 14 * nb ** 2) // 24
    rank = gsn.config6_table(nb)
    assert rank.max() == n6 - 1
    code = lambda t: sum(v * nb ** (5 - e) for e, v in enumerate(t))
    for k in range(n6):
        assert rank[code(oracle.config6(nb, k))] == k
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    rng = np.random.default_rng(nb)
    for _ in range(200):
        t = rng.integers(0, nb, 6)
        b = {frozenset(e): int(v) for e, v in zip(edges, t)}
        for p in itertools.permutations(range(4)):
            u = [b[frozenset((p[x], p[y]))] for x, y in edges]
            assert rank[code(u)] == rank[code(t)]


def test_six_edge_table_paper_counts():
    """276 configurations at 4 bins (the paper's count)."""
    import paper_2607_06604_amd as gsn
    assert gsn.n_configs6(4) == 276
