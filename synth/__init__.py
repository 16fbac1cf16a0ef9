"""Seeded synthetic catalogues shared by the oracle tests, the GPU tests and the bench.

Holds no counting arithmetic: it only draws random numbers (xoshiro256** seeded
by SplitMix64, Box-Muller Gaussians) and lays out points in a periodic box.

The named workloads follow the shapes of the paper's measurements: a periodic
box of galaxies (uniform randoms, clustered data) queried for triangles and
tetrahedra below rmax in equal-width radial bins (paper, Sec. 4.1 and
Table 2). They are synthetic stand-ins; no survey data is used.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile synth.c into libsynth.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        d, i64, u64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        P = ctypes.c_void_p
        lib.synth_uniform.argtypes = [P, i64, d, u64]
        lib.synth_neyman_scott.argtypes = [P, i64, i64, d, d, u64]
        lib.synth_lognormal.argtypes = [P, i64, d, i32, d, d, u64]
        lib.synth_uniform_values.argtypes = [P, i64, d, d, u64]
        lib.synth_u64.argtypes = [P, i64, u64]
        for f in (lib.synth_uniform, lib.synth_neyman_scott, lib.synth_lognormal,
                  lib.synth_uniform_values, lib.synth_u64):
            f.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def uniform(n: int, L: float, seed: int) -> np.ndarray:
    out = np.empty((n, 3), dtype=np.float64)
    assert _load().synth_uniform(_ptr(out), n, L, seed) == 0
    return out


def neyman_scott(n: int, per_parent: int, sigma: float, L: float, seed: int) -> np.ndarray:
    out = np.empty((n, 3), dtype=np.float64)
    assert _load().synth_neyman_scott(_ptr(out), n, per_parent, sigma, L, seed) == 0
    return out


def lognormal(n: int, L: float, seed: int, mesh: int = 128, sigma_s: float = 20.0,
              sigma_g: float = 0.5) -> np.ndarray:
    out = np.empty((n, 3), dtype=np.float64)
    assert _load().synth_lognormal(_ptr(out), n, L, mesh, sigma_s, sigma_g, seed) == 0
    return out


def uniform_values(n: int, lo: float, width: float, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    assert _load().synth_uniform_values(_ptr(out), n, lo, width, seed) == 0
    return out


def raw_u64(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    assert _load().synth_u64(_ptr(out), n, seed) == 0
    return out


def permutation(n: int, seed: int) -> np.ndarray:
    """Seeded permutation of range(n) (argsort of raw draws)."""
    return np.argsort(raw_u64(n, seed), kind="stable").astype(np.int64)


def dyadic_uniform(n: int, L: float, seed: int, bits: int = 30) -> np.ndarray:
    """Points on the grid k * L * 2^-bits, so L - x and all coordinate
    differences are exact in float64 (for exact reflection/translation tests)."""
    k = (raw_u64(3 * n, seed) >> np.uint64(64 - bits)).astype(np.float64)
    return (k * (L * 2.0 ** -bits)).reshape(n, 3)


@dataclass
class Workload:
    """One synthetic catalogue plus the query parameters it is measured with."""
    name: str
    kind: str              # "3pcf" or "4pcf_parity"
    xyz: np.ndarray
    box: float
    rmin: float
    rmax: float
    nbins: int
    weights: np.ndarray | None = None
    recipe: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


def _scaled(n: int, L: float, volume_fraction: float):
    """Same number density in a box of volume_fraction of the volume."""
    if volume_fraction == 1.0:
        return n, L
    return int(round(n * volume_fraction)), L * volume_fraction ** (1.0 / 3.0)


def workload(name: str, volume_fraction: float = 1.0) -> Workload:
    """The named workloads.

    uniform_3pcf    : 20 000 uniform points, L = 250, rmax 20, 10 bins (seed 1)
    ns_3pcf         : 1 000 000 Neyman-Scott points (20 000 parents x 50,
                      sigma 3), L = 1000, rmax 30, 15 bins (seed 2)
    ns_4pcf_parity  : 200 000 Neyman-Scott points (4 000 x 50, sigma 3),
                      L = 400, rmax 20, 8 bins (seed 3)
    lognormal_w3pcf : 2 000 000 lognormal-like points, L = 2000, rmax 150,
                      20 bins, weights 0.5 + U[0,1) (seed 4)

    volume_fraction < 1 keeps density, rmax and bins and shrinks the box.
    """
    if name == "uniform_3pcf":
        n, L = _scaled(20_000, 250.0, volume_fraction)
        xyz = uniform(n, L, 1)
        return Workload(name, "3pcf", xyz, L, 0.0, 20.0, 10,
                        recipe=dict(gen="uniform", n=n, L=L, seed=1))
    if name == "ns_3pcf":
        n, L = _scaled(1_000_000, 1000.0, volume_fraction)
        xyz = neyman_scott(n, 50, 3.0, L, 2)
        return Workload(name, "3pcf", xyz, L, 0.0, 30.0, 15,
                        recipe=dict(gen="neyman_scott", n=n, per_parent=50, sigma=3.0, L=L, seed=2))
    if name == "ns_4pcf_parity":
        n, L = _scaled(200_000, 400.0, volume_fraction)
        xyz = neyman_scott(n, 50, 3.0, L, 3)
        return Workload(name, "4pcf_parity", xyz, L, 0.0, 20.0, 8,
                        recipe=dict(gen="neyman_scott", n=n, per_parent=50, sigma=3.0, L=L, seed=3))
    if name == "lognormal_w3pcf":
        n, L = _scaled(2_000_000, 2000.0, volume_fraction)
        xyz = lognormal(n, L, 4, mesh=max(8, int(round(128 * volume_fraction ** (1 / 3)))))
        w = uniform_values(n, 0.5, 1.0, 1004)
        return Workload(name, "3pcf", xyz, L, 0.0, 150.0, 20, weights=w,
                        recipe=dict(gen="lognormal", n=n, L=L, seed=4, weights="0.5+U[0,1) seed 1004"))
    raise KeyError(name)


def stream_sizes(count: int = 256, seed: int = 5, lo: float = 5e4, hi: float = 5e5) -> np.ndarray:
    """Catalogue sizes of the serving stream: floor(exp(U(ln lo, ln hi)))."""
    u = uniform_values(count, 0.0, 1.0, seed)
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def stream_catalogue(k: int, n: int, L: float = 600.0, seed: int = 5) -> np.ndarray:
    """Catalogue k of the serving stream: even k clustered data, odd k uniform randoms."""
    if k % 2 == 0:
        return neyman_scott(n, 50, 3.0, L, seed * 100_003 + k)
    return uniform(n, L, seed * 100_003 + k)
