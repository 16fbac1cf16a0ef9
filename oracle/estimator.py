"""Oracle estimators: the paper's estimators written plainly over the oracle's
exact counts.

TEST INFRASTRUCTURE ONLY (imported by tests and the bench's CPU baseline).

Readings of the paper (Sec. 2.1, Sec. 3.3 Eq. 4-5, Sec. 3.4):
  * data weights are divided by their sum and random weights by minus theirs,
    each sum taken left to right in index order, so data sum to +1 and randoms
    to -1; the catalogue is the data followed by the randoms;
  * the numerator of an estimate (NN, NNN, NNNN) is the exact sum over tuples
    of that catalogue of the signed weight products; the denominator (RR, RRR,
    RRRR) the same sum over the randoms alone with their weights divided by
    their (positive) sum; each exact sum is rounded once to float64 and the
    estimate is their quotient;
  * the odd parity channel is pos - neg, subtracted exactly, then rounded;
  * xi(b) = NN(b) / RR(b); a 6-edge configuration's disconnected term is
    xi(b01) xi(b23) + xi(b02) xi(b13) + xi(b03) xi(b12) on its smallest edge
    tuple, added in that order; connected = total - disconnected;
  * the even parity channel's disconnected term: for every 6-edge
    configuration (ascending index) and each of its four vertices in turn, the
    vertex's three edge bins sorted give a hub configuration T, which gains
    RRRR6(c) * disc(c); the total for T is divided by RRRR_even(T).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle


def _unit_sum(w, sign):
    s = 0.0
    for v in w:
        s = s + float(v)
    out = np.array([float(v) / s for v in w], dtype=np.float64)
    return out if sign > 0 else -out


def _weights(n, w):
    return np.ones(n, dtype=np.float64) if w is None else np.asarray(w, dtype=np.float64)


def catalogues(xd, wd, xr, wr):
    """(combined xyz, combined weights, random weights) of the estimator."""
    wd = _unit_sum(_weights(len(xd), wd), +1)
    wrn = _weights(len(xr), wr)
    x = np.concatenate([np.asarray(xd, dtype=np.float64).reshape(-1, 3),
                        np.asarray(xr, dtype=np.float64).reshape(-1, 3)])
    return x, np.concatenate([wd, _unit_sum(wrn, -1)]), _unit_sum(wrn, +1)



@dataclass
class Zeta3:
    zeta: np.ndarray
    nnn: np.ndarray
    rrr: np.ndarray


def compute_3pcf(xd, wd, xr, wr, box, rmin, rmax, nbins, periodic=True) -> Zeta3:
    x, w, w_r = catalogues(xd, wd, xr, wr)
    n = oracle.count_3pcf(x, box, rmin, rmax, nbins, weights=w, periodic=periodic)
    r = oracle.count_3pcf(xr, box, rmin, rmax, nbins, weights=w_r, periodic=periodic)
    N = oracle.rounded(n.wsum_int(), n.wscale)
    R = oracle.rounded(r.wsum_int(), r.wscale)
    with np.errstate(divide="ignore", invalid="ignore"):
        return Zeta3(N / R, N, R)


@dataclass
class Zeta4:
    zeta_even: np.ndarray
    zeta_odd: np.ndarray
    nnnn_even: np.ndarray
    nnnn_odd: np.ndarray
    rrrr_even: np.ndarray
    xi: np.ndarray | None = None
    zeta6: np.ndarray | None = None
    zeta6_disc: np.ndarray | None = None
    zeta6_conn: np.ndarray | None = None
    zeta_even_disc: np.ndarray | None = None
    zeta_even_conn: np.ndarray | None = None


def compute_4pcf(xd, wd, xr, wr, box, rmin, rmax, nbins, connected=True, periodic=True) -> Zeta4:
    x, w, w_r = catalogues(xd, wd, xr, wr)
    pn = oracle.count_4pcf_parity(x, box, rmin, rmax, nbins, weights=w, periodic=periodic)
    pr = oracle.count_4pcf_parity(xr, box, rmin, rmax, nbins, weights=w_r, periodic=periodic)
    evN = oracle.rounded(pn.wsum_int(0), pn.wscale)
    evR = oracle.rounded(pr.wsum_int(0), pr.wscale)
    odd = [a - b for a, b in zip(pn.wsum_int(1), pn.wsum_int(2))]
    odN = oracle.rounded(odd, pn.wscale)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = Zeta4(evN / evR, odN / evR, evN, odN, evR)
    if not connected:
        return out
    # internal 2pCF on the same graphs and bins
    a = oracle.pair_sums(x, box, rmin, rmax, nbins, weights=w, periodic=periodic)
    b = oracle.pair_sums(xr, box, rmin, rmax, nbins, weights=w_r, periodic=periodic)
    NN = oracle.rounded(a.wsum_int(), a.wscale)
    RR = oracle.rounded(b.wsum_int(), b.wscale)
    with np.errstate(divide="ignore", invalid="ignore"):
        xi = NN / RR
    fn = oracle.count_4pcf_full(x, box, rmin, rmax, nbins, weights=w, periodic=periodic)
    fr = oracle.count_4pcf_full(xr, box, rmin, rmax, nbins, weights=w_r, periodic=periodic)
    N6 = oracle.rounded(fn.wsum_int(), fn.wscale)
    R6 = oracle.rounded(fr.wsum_int(), fr.wscale)
    n6 = oracle.n_configs6(nbins)
    disc = np.zeros(n6)
    num = np.zeros(oracle.n_configs(nbins))
    # vertex -> its three edges in the tuple order (01, 02, 03, 12, 13, 23)
    at = {0: (0, 1, 2), 1: (0, 3, 4), 2: (1, 3, 5), 3: (2, 4, 5)}
    for c in range(n6):
        t = oracle.config6(nbins, c)
        d = float(xi[t[0]]) * float(xi[t[5]])
        d = d + float(xi[t[1]]) * float(xi[t[4]])
        d = d + float(xi[t[2]]) * float(xi[t[3]])
        disc[c] = d
        for v in range(4):
            s = sorted(t[e] for e in at[v])
            k = oracle.config_index(nbins, *s)
            num[k] = num[k] + float(R6[c]) * d
    with np.errstate(divide="ignore", invalid="ignore"):
        z6 = N6 / R6
        de = num / evR
    out.xi = xi
    out.zeta6 = z6
    out.zeta6_disc = disc
    out.zeta6_conn = z6 - disc
    out.zeta_even_disc = de
    out.zeta_even_conn = out.zeta_even - de
    return out
