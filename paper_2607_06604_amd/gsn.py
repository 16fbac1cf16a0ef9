"""ctypes binding of libgsn.so (include/gsn.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
numpy arrays (host) or torch tensors (device) into pointers and status codes
into exceptions. There is no fallback: if libgsn.so is missing or fails to
load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsn.so")

GS_OK = 0
GS_EINVAL = -1
GS_EOVERFLOW = -2
GS_ENOMEM = -3
GS_EDEVMEM = -4
GS_EHIP = -5
GS_EAGAIN = -6
GS_ENOTFOUND = -7
GS_EUNSUPPORTED = -8
GS_ENOCOORDS = -9

GS_WEIGHTED = 1
GS_KEEP_COORDS = 2
GS_INPUT_ON_DEVICE = 4
GS_NONPERIODIC = 8

GS_DONE = 0
GS_PENDING = 1
GS_FAILED = 2
GS_CANCELLED = 3

GS_3PCF = 0
GS_4PCF_PARITY = 1

# every symbol include/gsn.h declares
EXPORTS = ["gs_create", "gs_destroy", "gs_build_graph", "gs_graph_info", "gs_graph_export",
           "gs_graph_free", "gs_count_3pcf", "gs_count_4pcf_parity", "gs_count_3pcf_batch",
           "gs_tune_3pcf", "gs_submit", "gs_poll", "gs_cancel", "gs_get_timings", "gs_strerror",
           "gs_last_error_detail", "gs_ceiling_copy", "gs_ceiling_probe", "gs_count_4pcf_parity_weighted",
           "gs_count_4pcf_full", "gs_n_configs6", "gs_config6_table", "gs_pair_sums",
           "gs_count_4pcf_parity_noalloc", "gs_count_3pcf_equilateral", "gs_count_3pcf_mu",
           "gs_compute_3pcf", "gs_compute_4pcf", "gs_count_4pcf_pixel"]


class GraphParams(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double), ("rmin", ctypes.c_double), ("rmax", ctypes.c_double),
                ("nbins", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Catalogue(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("n", ctypes.c_int64), ("weights", ctypes.c_void_p)]


class Zeta3(ctypes.Structure):
    _fields_ = [("zeta", ctypes.c_void_p), ("nnn", ctypes.c_void_p), ("rrr", ctypes.c_void_p),
                ("nnn128", ctypes.c_void_p), ("rrr128", ctypes.c_void_p), ("nnn_scale", ctypes.c_int32),
                ("rrr_scale", ctypes.c_int32)]


class Zeta4(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("zeta_even", "zeta_odd", "nnnn_even", "nnnn_odd", "rrrr_even",
                                              "zeta_even_disc", "zeta_even_conn", "zeta6", "zeta6_disc",
                                              "zeta6_conn", "xi")]


class AnchorRange(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class GraphStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_edges", ctypes.c_uint64), ("max_deg", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("n_windows", ctypes.c_int32),
                ("nbins", ctypes.c_int32), ("pair_hist", ctypes.c_uint64 * 255),
                ("sum_sq_degree", ctypes.c_uint64)]


class Timings(ctypes.Structure):
    _fields_ = [("build_ms", ctypes.c_double), ("count_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("kernel_launches", ctypes.c_uint64),
                ("alg_bytes", ctypes.c_uint64), ("probes", ctypes.c_uint64),
                ("table_log2", ctypes.c_int32), ("block", ctypes.c_int32), ("group", ctypes.c_int32),
                ("hash_load", ctypes.c_int32)]


class Plan3(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("step_log2", ctypes.c_int32), ("group", ctypes.c_int32),
                ("table", ctypes.c_int32), ("counters", ctypes.c_int32), ("hash_load", ctypes.c_int32),
                ("truncate", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("sample_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("sample_frac", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("n", ctypes.c_int64), ("weights", ctypes.c_void_p),
                ("p", GraphParams), ("kind", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("error", ctypes.c_int32), ("n_tuples", ctypes.c_uint64),
                ("hist", ctypes.c_void_p), ("pos", ctypes.c_void_p), ("neg", ctypes.c_void_p),
                ("wsum128", ctypes.c_void_p), ("whist", ctypes.c_void_p), ("wscale", ctypes.c_int32),
                ("step_size", ctypes.c_uint32), ("t_queue_s", ctypes.c_double),
                ("t_build_s", ctypes.c_double), ("t_count_s", ctypes.c_double), ("t_total_s", ctypes.c_double)]


class GsError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s failed: %s (%d)%s" % (where, _strerror(code), code,
                                                   (": " + detail) if detail else ""))
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libgsn.so (raises if it is not built). If torch is importable it is
    imported first so that one HIP runtime serves both."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libgsn.so is not built (%s); run __graft_entry__.build()" % path)
    try:
        import torch  # noqa: F401  (shares its HIP runtime with the library)
    except Exception:
        pass
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "gs_create": ([ctypes.POINTER(P), i32, u64, P], i32),
        "gs_destroy": ([P], i32),
        "gs_build_graph": ([P, P, i64, P, ctypes.POINTER(GraphParams), ctypes.POINTER(P)], i32),
        "gs_graph_info": ([P, ctypes.POINTER(GraphStats)], i32),
        "gs_graph_export": ([P, P, P, P, P], i32),
        "gs_graph_free": ([P], i32),
        "gs_count_3pcf": ([P, P, P, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_count_4pcf_parity": ([P, P, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_count_4pcf_parity_weighted": ([P, P, P, P, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_count_4pcf_parity_noalloc": ([P, P, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_count_4pcf_full": ([P, P, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_count_4pcf_pixel": ([P, P, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_n_configs6": ([i32, ctypes.POINTER(ctypes.c_uint32)], i32),
        "gs_config6_table": ([i32, P], i32),
        "gs_pair_sums": ([P, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_count_3pcf_equilateral": ([P, P, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_count_3pcf_mu": ([P, P, i32, P, P, P, P, ctypes.POINTER(AnchorRange)], i32),
        "gs_compute_3pcf": ([P, ctypes.POINTER(Catalogue), ctypes.POINTER(Catalogue), ctypes.POINTER(GraphParams),
                             ctypes.POINTER(Zeta3)], i32),
        "gs_compute_4pcf": ([P, ctypes.POINTER(Catalogue), ctypes.POINTER(Catalogue), ctypes.POINTER(GraphParams),
                             ctypes.POINTER(Zeta4)], i32),
        "gs_ceiling_copy": ([P, u64, ctypes.POINTER(ctypes.c_double)], i32),
        "gs_ceiling_probe": ([P, i32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, i32, i32, i32,
                              ctypes.POINTER(ctypes.c_double)], i32),
        "gs_count_3pcf_batch": ([P, P, i32, P, P], i32),
        "gs_tune_3pcf": ([P, P, ctypes.c_uint32, ctypes.POINTER(Plan3)], i32),
        "gs_submit": ([P, ctypes.POINTER(Request), ctypes.POINTER(u64)], i32),
        "gs_poll": ([P, u64, ctypes.POINTER(Result)], i32),
        "gs_cancel": ([P, u64], i32),
        "gs_get_timings": ([P, ctypes.POINTER(Timings)], i32),
        "gs_strerror": ([i32], ctypes.c_char_p),
        "gs_last_error_detail": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _strerror(code: int) -> str:
    return load().gs_strerror(code).decode()


def _check(rc: int, where: str):
    if rc != GS_OK:
        detail = load().gs_last_error_detail().decode()
        raise GsError(rc, where, detail)


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(a.ctypes.data)


def n_configs(nbins: int) -> int:
    return (nbins + 2) * (nbins + 1) * nbins // 6


def n_configs6(nbins: int) -> int:
    """6-edge configurations at nbins (gs_n_configs6)."""
    v = ctypes.c_uint32()
    _check(load().gs_n_configs6(int(nbins), ctypes.byref(v)), "gs_n_configs6")
    return int(v.value)


def config6_table(nbins: int) -> np.ndarray:
    """Configuration of every 6-edge bin-tuple code (gs_config6_table)."""
    t = np.zeros(nbins ** 6, dtype=np.uint32)
    _check(load().gs_config6_table(int(nbins), _ptr(t)), "gs_config6_table")
    return t


def _anchors(anchors):
    return None if anchors is None else ctypes.byref(AnchorRange(int(anchors[0]), int(anchors[1])))


def _signed128(words) -> list:
    """(lo, hi) u64 word pairs as Python ints (two's complement 128-bit)."""
    out = []
    for lo, hi in np.asarray(words, dtype=np.uint64).reshape(-1, 2):
        v = int(lo) + (int(hi) << 64)
        out.append(v - (1 << 128) if v >> 127 else v)
    return out


class Context:
    """gs_ctx: one device, one stream (borrowed if given), a memory budget."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, stream=None):
        lib = load()
        self._h = ctypes.c_void_p()
        sp = None
        if stream is not None:
            sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        _check(lib.gs_create(ctypes.byref(self._h), device, budget_bytes, sp), "gs_create")

    def close(self):
        if self._h:
            load().gs_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def build_graph(self, xyz, box, rmin, rmax, nbins, weights=None, keep_coords=False, periodic=True) -> "Graph":
        """xyz: (N,3) float64 numpy array (host) or torch tensor on the GPU;
        periodic=False: survey geometry (no wrap, points in [0, box)^3)."""
        on_dev = hasattr(xyz, "is_cuda") and xyz.is_cuda
        flags = (GS_INPUT_ON_DEVICE if on_dev else 0) | (GS_KEEP_COORDS if keep_coords else 0)
        if not periodic:
            flags |= GS_NONPERIODIC
        if weights is not None:
            flags |= GS_WEIGHTED
        if on_dev:
            import torch
            if xyz.dtype != torch.float64 or not xyz.is_contiguous() or xyz.dim() != 2 or xyz.shape[1] != 3:
                raise ValueError("device xyz must be a contiguous (N,3) float64 tensor")
            if weights is not None and (weights.dtype != torch.float64 or not weights.is_cuda
                                        or not weights.is_contiguous()):
                raise ValueError("device weights must be a contiguous float64 tensor")
            n = int(xyz.shape[0])
            x, w = xyz, weights
        else:
            x = _host(xyz, np.float64)
            if x.ndim != 2 or x.shape[1] != 3:
                raise ValueError("xyz must be (N,3)")
            n = x.shape[0]
            w = None if weights is None else _host(weights, np.float64)
            if w is not None and w.shape != (n,):
                raise ValueError("weights must be (N,)")
        p = GraphParams(float(box), float(rmin), float(rmax), int(nbins), flags)
        h = ctypes.c_void_p()
        _check(load().gs_build_graph(self._h, _ptr(x), n, _ptr(w), ctypes.byref(p), ctypes.byref(h)),
               "gs_build_graph")
        return Graph(h, nbins, n)

    def count_3pcf(self, g: "Graph", anchors=None, weighted=False):
        nc = n_configs(g.nbins)
        hist = np.zeros(nc, dtype=np.uint64)
        ntri = np.zeros(1, dtype=np.uint64)
        wsum = np.zeros((nc, 2), dtype=np.uint64) if weighted else None
        whist = np.zeros(nc, dtype=np.float64) if weighted else None
        ws = np.zeros(1, dtype=np.int32) if weighted else None
        ar = None if anchors is None else ctypes.byref(AnchorRange(int(anchors[0]), int(anchors[1])))
        _check(load().gs_count_3pcf(self._h, g.handle, _ptr(hist), _ptr(wsum), _ptr(whist), _ptr(ws),
                                    _ptr(ntri), ar), "gs_count_3pcf")
        return Count3(hist, int(ntri[0]), wsum, whist, int(ws[0]) if weighted else None)

    def count_4pcf_parity(self, g: "Graph", anchors=None, weighted=False, noalloc=False):
        """Parity counts (weighted: with exact clique-weight sums; noalloc: the
        entry point that allocates no device memory)."""
        nc = n_configs(g.nbins)
        e, p, m = (np.zeros(nc, dtype=np.uint64) for _ in range(3))
        nk = np.zeros(1, dtype=np.uint64)
        if not weighted:
            f = load().gs_count_4pcf_parity_noalloc if noalloc else load().gs_count_4pcf_parity
            _check(f(self._h, g.handle, _ptr(e), _ptr(p), _ptr(m), _ptr(nk), _anchors(anchors)),
                   "gs_count_4pcf_parity_noalloc" if noalloc else "gs_count_4pcf_parity")
            return Count4(e, p, m, int(nk[0]))
        ws = np.zeros((3, nc, 2), dtype=np.uint64)
        sc = np.zeros(1, dtype=np.int32)
        _check(load().gs_count_4pcf_parity_weighted(self._h, g.handle, _ptr(e), _ptr(p), _ptr(m), _ptr(ws),
                                                    _ptr(sc), _ptr(nk), _anchors(anchors)),
               "gs_count_4pcf_parity_weighted")
        return Count4(e, p, m, int(nk[0]), ws, int(sc[0]))

    def count_4pcf_pixel(self, g: "Graph", anchors=None):
        """Parity counts from direction pixels, spokes in original-index order."""
        nc = n_configs(g.nbins)
        e, p, m = (np.zeros(nc, dtype=np.uint64) for _ in range(3))
        nk = np.zeros(1, dtype=np.uint64)
        _check(load().gs_count_4pcf_pixel(self._h, g.handle, _ptr(e), _ptr(p), _ptr(m), _ptr(nk), _anchors(anchors)),
               "gs_count_4pcf_pixel")
        return Count4(e, p, m, int(nk[0]))

    def count_4pcf_full(self, g: "Graph", anchors=None, weighted=False):
        """6-edge 4-clique counts (and exact weighted sums)."""
        n6 = n_configs6(g.nbins) if 1 <= g.nbins <= 12 else 1   # the library refuses other bin counts
        h = np.zeros(n6, dtype=np.uint64)
        nk = np.zeros(1, dtype=np.uint64)
        ws = np.zeros((n6, 2), dtype=np.uint64) if weighted else None
        sc = np.zeros(1, dtype=np.int32) if weighted else None
        _check(load().gs_count_4pcf_full(self._h, g.handle, _ptr(h), _ptr(ws), _ptr(sc), _ptr(nk),
                                         _anchors(anchors)), "gs_count_4pcf_full")
        return Count6(h, int(nk[0]), ws, int(sc[0]) if weighted else None)

    def count_3pcf_equilateral(self, g: "Graph", anchors=None, weighted=False):
        """Triangles with all three sides in one bin, per bin."""
        h = np.zeros(g.nbins, dtype=np.uint64)
        nt = np.zeros(1, dtype=np.uint64)
        ws = np.zeros((g.nbins, 2), dtype=np.uint64) if weighted else None
        sc = np.zeros(1, dtype=np.int32) if weighted else None
        _check(load().gs_count_3pcf_equilateral(self._h, g.handle, _ptr(h), _ptr(ws), _ptr(sc), _ptr(nt),
                                                _anchors(anchors)), "gs_count_3pcf_equilateral")
        return Count3(h, int(nt[0]), ws, None, int(sc[0]) if weighted else None)

    def count_3pcf_mu(self, g: "Graph", nmu: int, anchors=None, weighted=False):
        """Triangles by sorted side bins and mu bin (counter conf * nmu + mu)."""
        nc = n_configs(g.nbins) * max(1, int(nmu))
        h = np.zeros(nc, dtype=np.uint64)
        nt = np.zeros(1, dtype=np.uint64)
        ws = np.zeros((nc, 2), dtype=np.uint64) if weighted else None
        sc = np.zeros(1, dtype=np.int32) if weighted else None
        _check(load().gs_count_3pcf_mu(self._h, g.handle, int(nmu), _ptr(h), _ptr(ws), _ptr(sc), _ptr(nt),
                                       _anchors(anchors)), "gs_count_3pcf_mu")
        return Count3(h, int(nt[0]), ws, None, int(sc[0]) if weighted else None)

    def pair_sums(self, g: "Graph", anchors=None, weighted=False):
        """Pairs per bin (and exact weighted pair sums)."""
        pr = np.zeros(g.nbins, dtype=np.uint64)
        ws = np.zeros((g.nbins, 2), dtype=np.uint64) if weighted else None
        sc = np.zeros(1, dtype=np.int32) if weighted else None
        _check(load().gs_pair_sums(self._h, g.handle, _ptr(pr), _ptr(ws), _ptr(sc), _anchors(anchors)),
               "gs_pair_sums")
        return Pairs(pr, ws, int(sc[0]) if weighted else None)

    def tune_3pcf(self, g: "Graph", weighted=False) -> dict:
        """Autotune the triangle-count schedule on g's shape (kept in this
        context); returns the chosen schedule and its sample timings."""
        out = Plan3()
        _check(load().gs_tune_3pcf(self._h, g.handle, GS_WEIGHTED if weighted else 0, ctypes.byref(out)),
               "gs_tune_3pcf")
        return {k: getattr(out, k) for k, _ in Plan3._fields_}

    def count_3pcf_batch(self, graphs):
        """One persistent launch over several resident graphs (same nbins)."""
        ng = len(graphs)
        nb = graphs[0].nbins
        nc = n_configs(nb)
        hs = np.zeros((ng, nc), dtype=np.uint64)
        nt = np.zeros(ng, dtype=np.uint64)
        arr = (ctypes.c_void_p * ng)(*[g.handle.value for g in graphs])
        _check(load().gs_count_3pcf_batch(self._h, ctypes.cast(arr, ctypes.c_void_p), ng, _ptr(hs), _ptr(nt)),
               "gs_count_3pcf_batch")
        return [Count3(hs[k], int(nt[k]), None, None, None) for k in range(ng)]

    def submit(self, xyz, box, rmin, rmax, nbins, weights=None, kind=GS_3PCF, periodic=True) -> int:
        """Queue a count of host catalogue xyz (triangles, weighted triangles
        with `weights`, or parity 4-cliques with kind=GS_4PCF_PARITY);
        returns a ticket."""
        x = _host(xyz, np.float64)
        if x.ndim != 2 or x.shape[1] != 3:
            raise ValueError("xyz must be (N,3)")
        w = None if weights is None else _host(weights, np.float64)
        if w is not None and w.shape != (x.shape[0],):
            raise ValueError("weights must be (N,)")
        req = Request(ctypes.c_void_p(x.ctypes.data), x.shape[0],
                      None if w is None else ctypes.c_void_p(w.ctypes.data),
                      GraphParams(float(box), float(rmin), float(rmax), int(nbins),
                                  (GS_WEIGHTED if w is not None else 0) | (0 if periodic else GS_NONPERIODIC)),
                      int(kind), 0)
        t = ctypes.c_uint64()
        _check(load().gs_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "gs_submit")
        return int(t.value)

    def poll(self, ticket: int, nbins: int):
        """None while pending; else a dict with status, counts and timings
        (the ticket is retired). hist is the triangle histogram or the parity
        even channel; pos / neg (parity) and wsum / whist / wscale (weighted
        triangles) are filled for those kinds."""
        nc = n_configs(nbins)
        hist, pos, neg = (np.zeros(nc, dtype=np.uint64) for _ in range(3))
        wsum = np.zeros((nc, 2), dtype=np.uint64)
        whist = np.zeros(nc, dtype=np.float64)
        r = Result()
        r.hist = hist.ctypes.data
        r.pos = pos.ctypes.data
        r.neg = neg.ctypes.data
        r.wsum128 = wsum.ctypes.data
        r.whist = whist.ctypes.data
        _check(load().gs_poll(self._h, ticket, ctypes.byref(r)), "gs_poll")
        if r.status == GS_PENDING:
            return None
        done = r.status == GS_DONE
        return dict(status=int(r.status), error=int(r.error), n_tuples=int(r.n_tuples),
                    n_triangles=int(r.n_tuples), hist=hist if done else None, pos=pos if done else None,
                    neg=neg if done else None, wsum=wsum if done else None, whist=whist if done else None,
                    wscale=int(r.wscale), t_queue_s=r.t_queue_s, t_build_s=r.t_build_s,
                    t_count_s=r.t_count_s, t_total_s=r.t_total_s, step_size=int(r.step_size))

    def cancel(self, ticket: int):
        _check(load().gs_cancel(self._h, ticket), "gs_cancel")

    def ceiling_copy(self, nbytes: int) -> float:
        """Attainable device copy bandwidth, GB/s (read + written)."""
        v = ctypes.c_double()
        _check(load().gs_ceiling_copy(self._h, int(nbytes), ctypes.byref(v)), "gs_ceiling_copy")
        return v.value

    def ceiling_probe(self, nbins, table_log2, keys_in_table, hit_rate, weighted=False, probe=True,
                      block=256) -> float:
        """Attainable candidates/s of the triangle count's probe work (or of
        its LDS histogram alone with probe=False)."""
        v = ctypes.c_double()
        _check(load().gs_ceiling_probe(self._h, int(nbins), int(table_log2), int(keys_in_table),
                                       float(hit_rate), int(bool(weighted)), int(bool(probe)), int(block),
                                       ctypes.byref(v)), "gs_ceiling_probe")
        return v.value

    def timings(self) -> Timings:
        t = Timings()
        _check(load().gs_get_timings(self._h, ctypes.byref(t)), "gs_get_timings")
        return t


@dataclass
class Count3:
    hist: np.ndarray
    n_triangles: int
    wsum: np.ndarray | None
    whist: np.ndarray | None
    wscale: int | None

    def wsum_int(self):
        return _signed128(self.wsum)


@dataclass
class Count4:
    even: np.ndarray
    pos: np.ndarray
    neg: np.ndarray
    n_cliques: int
    wsum: np.ndarray | None = None   # (3, nconf, 2): even | pos | neg, 128-bit words
    wscale: int | None = None

    @property
    def odd(self):
        return self.pos.astype(np.int64) - self.neg.astype(np.int64)

    def wsum_int(self, channel: int = 0):
        return _signed128(self.wsum[channel])


@dataclass
class Count6:
    hist: np.ndarray
    n_cliques: int
    wsum: np.ndarray | None
    wscale: int | None

    def wsum_int(self):
        return _signed128(self.wsum)


@dataclass
class Pairs:
    pairs: np.ndarray
    wsum: np.ndarray | None
    wscale: int | None

    def wsum_int(self):
        return _signed128(self.wsum)


class Graph:
    """gs_graph handle (device CSR, labels, optional coords/weights)."""

    def __init__(self, handle, nbins, n):
        self._h = handle
        self.nbins = nbins
        self.n = n

    @property
    def handle(self):
        return self._h

    def info(self) -> GraphStats:
        s = GraphStats()
        _check(load().gs_graph_info(self._h, ctypes.byref(s)), "gs_graph_info")
        return s

    def export(self):
        s = self.info()
        rp = np.zeros(s.n + 1, dtype=np.uint64)
        col = np.zeros(max(s.n_edges, 1), dtype=np.uint32)
        b = np.zeros(max(s.n_edges, 1), dtype=np.uint8)
        perm = np.zeros(max(s.n, 1), dtype=np.uint32)
        _check(load().gs_graph_export(self._h, _ptr(rp), _ptr(col), _ptr(b), _ptr(perm)), "gs_graph_export")
        return rp, col[:s.n_edges], b[:s.n_edges], perm[:s.n]

    def free(self):
        if self._h:
            load().gs_graph_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------- estimators

def _catalogue(xyz, w):
    x = _host(xyz, np.float64)
    if x.ndim != 2 or x.shape[1] != 3:
        raise ValueError("positions must be (N,3)")
    wa = None if w is None else _host(w, np.float64)
    if wa is not None and wa.shape != (x.shape[0],):
        raise ValueError("weights must be (N,)")
    c = Catalogue(ctypes.c_void_p(x.ctypes.data), x.shape[0], None if wa is None else ctypes.c_void_p(wa.ctypes.data))
    return c, (x, wa)


def bin_centres(rmin, rmax, nbins):
    d = (rmax - rmin) / nbins
    return np.array([rmin + (k + 0.5) * d for k in range(nbins)])


@dataclass
class Result3pcf:
    """compute_3pcf result: zeta, NNN, RRR per sorted-side configuration,
    with the configurations' bin centres r1 <= r2 <= r3."""
    zeta: np.ndarray
    NNN: np.ndarray
    RRR: np.ndarray
    r1: np.ndarray
    r2: np.ndarray
    r3: np.ndarray
    nnn_exact: list
    nnn_scale: int


def _config_centres(rmin, rmax, nbins):
    c = bin_centres(rmin, rmax, nbins)
    t = [(a, b, d) for a in range(nbins) for b in range(a, nbins) for d in range(b, nbins)]
    return tuple(np.array([c[x[k]] for x in t]) for k in range(3))


def compute_3pcf(pos_data, w_data, pos_rand, w_rand, rmin, rmax, nbins, box, ctx=None,
                 periodic=True) -> Result3pcf:
    """The paper's compute_3pcf (Sec. 3.4) on a periodic box: zeta =
    NNN / RRR with signed, normalised data-minus-random weights."""
    own = ctx is None
    c = Context(0) if own else ctx
    try:
        d, keep_d = _catalogue(pos_data, w_data)
        r, keep_r = _catalogue(pos_rand, w_rand)
        nc = n_configs(nbins)
        zeta, nnn, rrr = (np.zeros(nc) for _ in range(3))
        n128 = np.zeros((nc, 2), dtype=np.uint64)
        out = Zeta3(zeta.ctypes.data, nnn.ctypes.data, rrr.ctypes.data, n128.ctypes.data, None, 0, 0)
        p = GraphParams(float(box), float(rmin), float(rmax), int(nbins), 0 if periodic else GS_NONPERIODIC)
        _check(load().gs_compute_3pcf(c.handle, ctypes.byref(d), ctypes.byref(r), ctypes.byref(p), ctypes.byref(out)),
               "gs_compute_3pcf")
        r1, r2, r3 = _config_centres(rmin, rmax, nbins)
        return Result3pcf(zeta, nnn, rrr, r1, r2, r3, _signed128(n128), int(out.nnn_scale))
    finally:
        if own:
            c.close()


@dataclass
class Result4pcf:
    """compute_4pcf result. Parity channels per hub configuration (sorted
    spoke bins): zeta_even, zeta_odd, their numerators and the even random
    sum, the even channel's disconnected part and connected remainder;
    6-edge configurations: zeta6, its disconnected part (Eq. 4) and
    connected remainder (Eq. 5); xi: the internal 2pCF."""
    zeta_even: np.ndarray
    zeta_odd: np.ndarray
    nnnn_even: np.ndarray
    nnnn_odd: np.ndarray
    rrrr_even: np.ndarray
    zeta_even_disc: np.ndarray | None
    zeta_even_conn: np.ndarray | None
    zeta6: np.ndarray | None
    zeta6_disc: np.ndarray | None
    zeta6_conn: np.ndarray | None
    xi: np.ndarray | None


def compute_4pcf(pos_data, w_data, pos_rand, w_rand, rmin, rmax, nbins, box, parity=True, connected=True,
                 ctx=None, periodic=True) -> Result4pcf:
    """The paper's compute_4pcf (Sec. 3.4) with its parity split (Sec. 3.2)
    and connected part (Sec. 3.3) on a periodic box."""
    own = ctx is None
    c = Context(0) if own else ctx
    try:
        d, keep_d = _catalogue(pos_data, w_data)
        r, keep_r = _catalogue(pos_rand, w_rand)
        nc = n_configs(nbins)
        ev, od, ne, no, re_ = (np.zeros(nc) for _ in range(5))
        arrs = dict(zeta_even=ev, zeta_odd=od, nnnn_even=ne, nnnn_odd=no, rrrr_even=re_)
        if connected:
            n6 = n_configs6(nbins)
            arrs.update(zeta_even_disc=np.zeros(nc), zeta_even_conn=np.zeros(nc), zeta6=np.zeros(n6),
                        zeta6_disc=np.zeros(n6), zeta6_conn=np.zeros(n6), xi=np.zeros(nbins))
        out = Zeta4(**{k: v.ctypes.data for k, v in arrs.items()})
        p = GraphParams(float(box), float(rmin), float(rmax), int(nbins), 0 if periodic else GS_NONPERIODIC)
        _check(load().gs_compute_4pcf(c.handle, ctypes.byref(d), ctypes.byref(r), ctypes.byref(p), ctypes.byref(out)),
               "gs_compute_4pcf")
        g = arrs.get
        return Result4pcf(ev, od, ne, no, re_, g("zeta_even_disc"), g("zeta_even_conn"), g("zeta6"),
                          g("zeta6_disc"), g("zeta6_conn"), g("xi"))
    finally:
        if own:
            c.close()
