"""CPU oracle for binned triangle and 4-clique parity counts.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the product library. The arithmetic lives
in oracle.c (plain C + OpenMP, float64 without FMA contraction); this module
compiles it with gcc and marshals numpy arrays through ctypes.

Every count here is a plain definition (see the header of oracle.c): the
periodic minimum-image separation, equal-width squared bin thresholds, sorted
side-bin triangle configurations, and per-hub signed-volume parity of
4-cliques (paper Sec. 2.1, 2.2, 3.2, Eq. 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {0: "ok", -1: "invalid argument", -3: "out of memory"}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P, d, i64, i32 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int
        lib.oracle_config_index.argtypes = [i32, i32, i32, i32]
        lib.oracle_config_index.restype = i64
        lib.oracle_edge_bin.argtypes = [d, d, d, d, i32]
        lib.oracle_edge_bin.restype = i32
        lib.oracle_separation.argtypes = [P, P, d, P, P]
        lib.oracle_separation.restype = i32
        lib.oracle_graph.argtypes = [P, i64, d, d, d, i32, P, P, P, i64, P]
        lib.oracle_graph.restype = i32
        lib.oracle_count_3pcf.argtypes = [P, i64, P, d, d, d, i32, i64, i64, i32, P, P, P, P, P]
        lib.oracle_count_3pcf.restype = i32
        lib.oracle_count_4pcf_parity.argtypes = [P, i64, P, d, d, d, i32, i64, i64, i32, P, P, P, P, P, P, P]
        lib.oracle_count_4pcf_parity.restype = i32
        lib.oracle_n_configs6.argtypes = [i32]
        lib.oracle_n_configs6.restype = i64
        lib.oracle_config6.argtypes = [i32, i64, P]
        lib.oracle_config6.restype = i32
        lib.oracle_count_4pcf_full.argtypes = [P, i64, P, d, d, d, i32, i64, i64, i32, P, P, P, P, P]
        lib.oracle_pair_sums.argtypes = [P, i64, P, d, d, d, i32, i64, i64, P, P, P]
        lib.oracle_pair_sums.restype = i32
        lib.oracle_count_4pcf_full.restype = i32
        lib.oracle_count_3pcf_mu.argtypes = [P, i64, P, d, d, d, i32, i32, i64, i64, i32, P, P, P, P, P]
        lib.oracle_count_3pcf_mu.restype = i32
        lib.oracle_count_4pcf_pixel.argtypes = [P, i64, d, d, d, i32, i64, i64, i32, P, P, P, P, P]
        lib.oracle_count_4pcf_pixel.restype = i32
        lib.oracle_pixel_of.argtypes = [P]
        lib.oracle_pixel_of.restype = i32
        lib.oracle_pixel_centre.argtypes = [i32, P]
        lib.oracle_pixel_centre.restype = None
        lib.oracle_hub_pixel_channel.argtypes = [P, d, d, d, i32, i32]
        lib.oracle_hub_pixel_channel.restype = i32
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle error %d (%s)" % (code, ERRORS.get(code, "?")))
        self.code = code


def _box(box, periodic):
    """The box argument of the C oracle: negative for survey geometry (no
    periodic wrap, the points in the cube of side box)."""
    return float(box) if periodic else -float(box)


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _xyz(xyz) -> np.ndarray:
    a = np.ascontiguousarray(xyz, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("xyz must be (N,3)")
    return a


def n_configs(nbins: int) -> int:
    """Number of sorted side-bin triples b1 <= b2 <= b3 over nbins bins: C(nb+2,3)."""
    return (nbins + 2) * (nbins + 1) * nbins // 6


def config_index(nbins: int, b1: int, b2: int, b3: int) -> int:
    return int(_load().oracle_config_index(nbins, b1, b2, b3))


def edge_bin(q: float, box: float, rmin: float, rmax: float, nbins: int) -> int:
    r = int(_load().oracle_edge_bin(q, box, rmin, rmax, nbins))
    if r == -2:
        raise OracleError(-1)
    return r


def separation(a, b, box: float, periodic=True):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.empty(3)
    q = np.empty(1)
    rc = _load().oracle_separation(_p(a), _p(b), _box(box, periodic), _p(r), _p(q))
    if rc:
        raise OracleError(rc)
    return r, float(q[0])


def graph(xyz, box, rmin, rmax, nbins, periodic=True):
    """Full symmetric rows (row_ptr int64[n+1], col int32[E], bin uint8[E]),
    each row sorted by original index."""
    x = _xyz(xyz)
    n = x.shape[0]
    lib = _load()
    ne = np.zeros(1, dtype=np.int64)
    rp = np.zeros(n + 1, dtype=np.int64)
    dummy = np.zeros(1, dtype=np.int32)
    rc = lib.oracle_graph(_p(x), n, _box(box, periodic), rmin, rmax, nbins, _p(rp), _p(dummy), _p(dummy), 0, _p(ne))
    if rc:
        raise OracleError(rc)
    E = int(ne[0])
    col = np.zeros(max(E, 1), dtype=np.int32)
    b = np.zeros(max(E, 1), dtype=np.uint8)
    rc = lib.oracle_graph(_p(x), n, _box(box, periodic), rmin, rmax, nbins, _p(rp), _p(col), _p(b), E, _p(ne))
    if rc:
        raise OracleError(rc)
    return rp, col[:E], b[:E]


def signed128(words) -> list:
    """(lo, hi) word pairs of two's-complement 128-bit sums -> Python ints."""
    out = []
    for lo, hi in np.asarray(words, dtype=np.uint64).reshape(-1, 2):
        v = int(lo) + (int(hi) << 64)
        out.append(v - (1 << 128) if v >> 127 else v)
    return out


def rounded(values, scale) -> np.ndarray:
    """Exact integers in units of 2^-scale, each rounded once to float64."""
    import math
    return np.array([math.ldexp(float(v), -scale) for v in values])


@dataclass
class Result2:
    pairs: np.ndarray           # uint64[nbins]
    wsum: np.ndarray | None     # uint64[nbins, 2]
    wscale: int | None

    def wsum_int(self):
        return signed128(self.wsum)


def pair_sums(xyz, box, rmin, rmax, nbins, weights=None, anchors=None, periodic=True) -> Result2:
    """Edges per bin and, with weights, the exact per-bin sums of w_i*w_j."""
    x = _xyz(xyz)
    n = x.shape[0]
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    lo, hi = (0, n) if anchors is None else anchors
    pairs = np.zeros(max(nbins, 1), dtype=np.uint64)
    wsum = np.zeros((max(nbins, 1), 2), dtype=np.uint64) if w is not None else None
    ws = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_pair_sums(_p(x), n, _p(w), _box(box, periodic), rmin, rmax, nbins, lo, hi, _p(pairs), _p(wsum), _p(ws))
    if rc:
        raise OracleError(rc)
    return Result2(pairs, wsum, int(ws[0]) if w is not None else None)


@dataclass
class Result3:
    hist: np.ndarray            # uint64[n_configs]
    n_triangles: int
    wsum: np.ndarray | None     # uint64[n_configs, 2] (lo, hi) exact sums in units of 2^-wscale
    wscale: int | None
    threads: int

    def wsum_int(self):
        """Exact weighted sums as Python ints (units of 2^-wscale)."""
        return signed128(self.wsum)

    def whist(self) -> np.ndarray:
        """Weighted sums rounded once to float64."""
        return rounded(self.wsum_int(), self.wscale)


def count_3pcf(xyz, box, rmin, rmax, nbins, weights=None, anchors=None, threads=0, periodic=True) -> Result3:
    x = _xyz(xyz)
    n = x.shape[0]
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if w is not None and w.shape != (n,):
        raise ValueError("weights must be (N,)")
    lo, hi = (0, n) if anchors is None else anchors
    nc = n_configs(nbins) if 1 <= nbins <= 255 else 1
    hist = np.zeros(nc, dtype=np.uint64)
    wsum = np.zeros((nc, 2), dtype=np.uint64) if w is not None else None
    ws = np.zeros(1, dtype=np.int32)
    nt = np.zeros(1, dtype=np.uint64)
    used = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_count_3pcf(_p(x), n, _p(w), _box(box, periodic), rmin, rmax, nbins, lo, hi, threads,
                                   _p(hist), _p(wsum), _p(ws), _p(nt), _p(used))
    if rc:
        raise OracleError(rc)
    return Result3(hist, int(nt[0]), wsum, int(ws[0]) if w is not None else None, int(used[0]))


@dataclass
class Result4:
    even: np.ndarray   # uint64[n_configs]: every hub contribution
    pos: np.ndarray    # uint64[n_configs]: V > 0, non-degenerate
    neg: np.ndarray    # uint64[n_configs]: V < 0, non-degenerate
    n_cliques: int
    threads: int
    wsum: np.ndarray | None = None   # uint64[3, n_configs, 2]: even | pos | neg weighted sums
    wscale: int | None = None

    @property
    def odd(self) -> np.ndarray:
        return self.pos.astype(np.int64) - self.neg.astype(np.int64)

    def wsum_int(self, channel: int):
        """Exact weighted sums of one channel (0 even, 1 pos, 2 neg)."""
        return signed128(self.wsum[channel])


def count_4pcf_parity(xyz, box, rmin, rmax, nbins, anchors=None, threads=0, weights=None, periodic=True) -> Result4:
    x = _xyz(xyz)
    n = x.shape[0]
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    lo, hi = (0, n) if anchors is None else anchors
    nc = n_configs(nbins) if 1 <= nbins <= 255 else 1
    e = np.zeros(nc, dtype=np.uint64)
    p = np.zeros(nc, dtype=np.uint64)
    m = np.zeros(nc, dtype=np.uint64)
    ws = np.zeros((3, nc, 2), dtype=np.uint64) if w is not None else None
    sc = np.zeros(1, dtype=np.int32)
    nk = np.zeros(1, dtype=np.uint64)
    used = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_count_4pcf_parity(_p(x), n, _p(w), _box(box, periodic), rmin, rmax, nbins, lo, hi, threads,
                                          _p(e), _p(p), _p(m), _p(ws), _p(sc), _p(nk), _p(used))
    if rc:
        raise OracleError(rc)
    return Result4(e, p, m, int(nk[0]), int(used[0]), ws, int(sc[0]) if w is not None else None)


def count_3pcf_mu(xyz, box, rmin, rmax, nbins, nmu, weights=None, anchors=None, threads=0, periodic=True) -> Result3:
    """Triangles binned by sorted side bins and by the mu bin of their plane's
    normal (counter conf * nmu + mu bin)."""
    x = _xyz(xyz)
    n = x.shape[0]
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    lo, hi = (0, n) if anchors is None else anchors
    nc = n_configs(nbins) * nmu if 1 <= nbins <= 255 and nmu >= 1 else 1
    hist = np.zeros(nc, dtype=np.uint64)
    wsum = np.zeros((nc, 2), dtype=np.uint64) if w is not None else None
    ws = np.zeros(1, dtype=np.int32)
    nt = np.zeros(1, dtype=np.uint64)
    used = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_count_3pcf_mu(_p(x), n, _p(w), _box(box, periodic), rmin, rmax, nbins, nmu, lo, hi, threads, _p(hist),
                                      _p(wsum), _p(ws), _p(nt), _p(used))
    if rc:
        raise OracleError(rc)
    return Result3(hist, int(nt[0]), wsum, int(ws[0]) if w is not None else None, int(used[0]))


def pixel_of(r) -> int:
    """Direction pixel (0..255) of a separation vector."""
    v = np.ascontiguousarray(r, dtype=np.float64)
    return int(_load().oracle_pixel_of(_p(v)))


def pixel_centre(pix: int) -> np.ndarray:
    u = np.zeros(3, dtype=np.float64)
    _load().oracle_pixel_centre(int(pix), _p(u))
    return u


def hub_pixel_channel(xyz4, box, rmin, rmax, nbins, h) -> int:
    """Channel of hub h (0 pos, 1 neg, 2 degenerate) of four points under the
    pixel rule, its spokes to the other three in index order."""
    x = _xyz(xyz4)
    r = int(_load().oracle_hub_pixel_channel(_p(x), box, rmin, rmax, nbins, h))
    if r < 0:
        raise OracleError(r)
    return r


def count_4pcf_pixel(xyz, box, rmin, rmax, nbins, anchors=None, threads=0, periodic=True) -> Result4:
    """Parity counts with each spoke direction quantised to a pixel and the
    spokes in original-index order (degenerate iff |V| < 1e-9)."""
    x = _xyz(xyz)
    n = x.shape[0]
    lo, hi = (0, n) if anchors is None else anchors
    nc = n_configs(nbins) if 1 <= nbins <= 255 else 1
    e, p, m = (np.zeros(nc, dtype=np.uint64) for _ in range(3))
    nk = np.zeros(1, dtype=np.uint64)
    used = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_count_4pcf_pixel(_p(x), n, _box(box, periodic), rmin, rmax, nbins, lo, hi, threads,
                                         _p(e), _p(p), _p(m), _p(nk), _p(used))
    if rc:
        raise OracleError(rc)
    return Result4(e, p, m, int(nk[0]), int(used[0]))


def n_configs6(nbins: int) -> int:
    """Number of 6-edge 4-clique configurations (edge-bin tuples up to
    relabelling of the four vertices) over nbins bins (nbins <= 12)."""
    r = int(_load().oracle_n_configs6(nbins))
    if r < 0:
        raise OracleError(r if r == -3 else -1)
    return r


def config6(nbins: int, index: int):
    """The smallest edge-bin tuple (b01, b02, b03, b12, b13, b23) of
    configuration `index`."""
    out = np.zeros(6, dtype=np.int32)
    rc = _load().oracle_config6(nbins, index, _p(out))
    if rc:
        raise OracleError(rc)
    return tuple(int(v) for v in out)


@dataclass
class Result6:
    hist: np.ndarray   # uint64[n_configs6]
    n_cliques: int
    threads: int
    wsum: np.ndarray | None = None   # uint64[n_configs6, 2]
    wscale: int | None = None

    def wsum_int(self):
        return signed128(self.wsum)


def count_4pcf_full(xyz, box, rmin, rmax, nbins, anchors=None, threads=0, weights=None, periodic=True) -> Result6:
    """Every 4-clique once, binned by the configuration of its six edge bins
    (with weights: the exact sums of ((w1*w2)*w3)*w4, ascending values)."""
    x = _xyz(xyz)
    n = x.shape[0]
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    lo, hi = (0, n) if anchors is None else anchors
    nc = n_configs6(nbins) if 1 <= nbins <= 12 else 1
    h = np.zeros(nc, dtype=np.uint64)
    ws = np.zeros((nc, 2), dtype=np.uint64) if w is not None else None
    sc = np.zeros(1, dtype=np.int32)
    nk = np.zeros(1, dtype=np.uint64)
    used = np.zeros(1, dtype=np.int32)
    rc = _load().oracle_count_4pcf_full(_p(x), n, _p(w), _box(box, periodic), rmin, rmax, nbins, lo, hi, threads, _p(h),
                                        _p(ws), _p(sc), _p(nk), _p(used))
    if rc:
        raise OracleError(rc)
    return Result6(h, int(nk[0]), int(used[0]), ws, int(sc[0]) if w is not None else None)
