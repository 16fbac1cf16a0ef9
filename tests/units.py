"""Catalogues of isolated small units (test helper).

Each unit is a handful of points given by offsets from a unit origin; units
sit on a grid `spacing` apart (more than rmax plus the unit's size), so no
edge joins two units and every count is a sum of per-unit counts. Origins
and offsets are dyadic, so every coordinate and every separation inside a
unit is exact in float64. Shared by the oracle pins and the GPU tests; holds
none of the method's arithmetic.
"""
from __future__ import annotations

import numpy as np


def place(units, L, spacing=8.0, origin=(2.25, 2.5, 2.75)):
    """units: list of offset arrays (k_u x 3). Returns the (N,3) catalogue."""
    per = int(L // spacing)
    pts = []
    for u, off in enumerate(units):
        a, b, c = u // (per * per), (u // per) % per, u % per
        O = np.array([a * spacing, b * spacing, c * spacing]) + np.array(origin)
        for v in np.asarray(off, dtype=np.float64):
            pts.append(O + v)
    return np.mod(np.array(pts, dtype=np.float64), L)


def offsets(g, names, lift=None, eps=0.0):
    """Offsets of a unit from its golden entry, vertex `lift` moved by eps in z."""
    out = []
    for nm in names:
        v = np.array(g["offsets"][nm], dtype=np.float64)
        if nm == lift:
            v[2] += eps
        out.append(v)
    return np.array(out)


def expected_parity(nb, config_index, hub_configs, signs):
    """even / odd arrays for one unit: hub_configs name -> sorted bins,
    signs name -> +1, -1 or 0 (degenerate)."""
    n = (nb + 2) * (nb + 1) * nb // 6
    even = np.zeros(n, dtype=np.int64)
    odd = np.zeros(n, dtype=np.int64)
    for nm, t in hub_configs.items():
        k = config_index(nb, *t)
        even[k] += 1
        odd[k] += signs.get(nm, 0)
    return even, odd


def expected_triangles(nb, config_index, configs):
    n = (nb + 2) * (nb + 1) * nb // 6
    h = np.zeros(n, dtype=np.int64)
    for t in configs:
        h[config_index(nb, *t)] += 1
    return h
