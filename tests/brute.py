"""Brute-force tuple enumeration for tiny catalogues (test helper).

Independent of oracle/ and of the GPU library: no cell list, no sorted rows,
no membership search. It forms the full N x N pair matrix with numpy and
visits every triple (O(N^3)) or quadruple (O(N^4)) of points. The pair rule
(minimum image, squared length, equal-width squared bin thresholds) and the
per-hub signed volume are restated here from the paper's definitions
(Sec. 2.1, 2.2, 3.2 Eq. 2); float64 numpy arithmetic without fused
operations, in the same evaluation order.
"""
from __future__ import annotations

import math

import numpy as np


def pair_matrix(xyz, L, rmin, rmax, nb):
    """L > 0: periodic box (minimum image); L < 0: survey geometry, no wrap."""
    x = np.asarray(xyz, dtype=np.float64)
    d = x[None, :, :] - x[:, None, :]          # d[a, b] = x_b - x_a
    if L > 0:
        half = 0.5 * L
        d = np.where(d > half, d - L, np.where(d < -half, d + L, d))
    q = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    D = (rmax - rmin) / nb
    e = [rmin] + [rmin + k * D for k in range(1, nb)] + [rmax]
    t = [v * v for v in e]
    adj = (q >= t[0]) & (q < t[nb])
    np.fill_diagonal(adj, False)
    b = np.zeros(q.shape, dtype=np.int64)
    for k in range(1, nb):
        b += (q >= t[k])
    return d, q, adj, b


def lex_configs(nb):
    """All b1 <= b2 <= b3 in lexicographic order -> {triple: rank}."""
    out = {}
    for a in range(nb):
        for bb in range(a, nb):
            for c in range(bb, nb):
                out[(a, bb, c)] = len(out)
    return out


def triangles(xyz, L, rmin, rmax, nb, weights=None, anchors=None):
    """Returns (hist by lexicographic rank, n_triangles, exact weighted sums as
    Python ints in units of 2^-s, s)."""
    n = len(xyz)
    _, _, adj, b = pair_matrix(xyz, L, rmin, rmax, nb)
    rank = lex_configs(nb)
    hist = np.zeros(len(rank), dtype=np.int64)
    wsum = [0] * len(rank)
    s = None
    if weights is not None:
        w = [float(v) for v in weights]
        wmin = min(abs(v) for v in w)
        s = 52 - math.frexp((wmin * wmin) * wmin)[1] + 1
    lo, hi = (0, n) if anchors is None else anchors
    count = 0
    for i in range(lo, hi):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            ks = np.nonzero(adj[i, j + 1:] & adj[j, j + 1:])[0] + j + 1
            for k in ks:
                key = tuple(sorted((int(b[i, j]), int(b[i, k]), int(b[j, k]))))
                hist[rank[key]] += 1
                count += 1
                if weights is not None:
                    wsum[rank[key]] += int(signed_product((w[i], w[j], w[int(k)])) * 2.0 ** s)
    return hist, count, wsum, s


def hub_volume(r_a, r_b, r_c):
    cx = r_a[1] * r_b[2] - r_a[2] * r_b[1]
    cy = r_a[2] * r_b[0] - r_a[0] * r_b[2]
    cz = r_a[0] * r_b[1] - r_a[1] * r_b[0]
    return (cx * r_c[0] + cy * r_c[1]) + cz * r_c[2]


def cliques4(xyz, L, rmin, rmax, nb, anchors=None):
    """Returns (even, pos, neg, n_cliques) for 4-cliques, one contribution per
    hub (each vertex of the clique in turn)."""
    n = len(xyz)
    d, q, adj, b = pair_matrix(xyz, L, rmin, rmax, nb)
    rank = lex_configs(nb)
    E = np.zeros(len(rank), dtype=np.int64)
    P = np.zeros(len(rank), dtype=np.int64)
    N = np.zeros(len(rank), dtype=np.int64)
    lo, hi = (0, n) if anchors is None else anchors
    count = 0
    for i in range(lo, hi):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            common = adj[i] & adj[j]
            ks = [k for k in np.nonzero(common)[0] if k > j]
            for k in ks:
                ls = [l for l in np.nonzero(common & adj[k])[0] if l > k]
                for l in ls:
                    count += 1
                    v = (i, j, int(k), int(l))
                    for h in v:
                        sp = [s for s in v if s != h]
                        sp.sort(key=lambda s: q[h, s])     # stable; ties are degenerate anyway
                        qa, qb, qc = (float(q[h, s]) for s in sp)
                        key = tuple(int(b[h, s]) for s in sp)
                        r = rank[key]
                        E[r] += 1
                        V = hub_volume(*(tuple(float(c) for c in d[h, s]) for s in sp))
                        if qa == qb or qb == qc:
                            continue
                        if V * V <= 1e-18 * ((qa * qb) * qc):
                            continue
                        if V > 0:
                            P[r] += 1
                        else:
                            N[r] += 1
    return E, P, N, count


_EDGES6 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def canonical6(t):
    """Smallest edge-bin tuple over the 24 vertex orderings (itertools)."""
    import itertools
    pos = {e: k for k, e in enumerate(_EDGES6)}
    best = None
    for p in itertools.permutations(range(4)):
        u = tuple(t[pos[tuple(sorted((p[a], p[b])))]] for a, b in _EDGES6)
        if best is None or u < best:
            best = u
    return best


def configs6(nb):
    """All 6-edge configurations in lexicographic order -> {tuple: rank}."""
    import itertools
    c = sorted({canonical6(t) for t in itertools.product(range(nb), repeat=6)})
    return {t: k for k, t in enumerate(c)}


def cliques4_six(xyz, L, rmin, rmax, nb, anchors=None):
    """Histogram of 4-cliques by their 6-edge configuration, and the count."""
    n = len(xyz)
    _, _, adj, b = pair_matrix(xyz, L, rmin, rmax, nb)
    rank = configs6(nb)
    H = np.zeros(len(rank), dtype=np.int64)
    lo, hi = (0, n) if anchors is None else anchors
    count = 0
    for i in range(lo, hi):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            common = adj[i] & adj[j]
            for k in [k for k in np.nonzero(common)[0] if k > j]:
                for l in [l for l in np.nonzero(common & adj[k])[0] if l > k]:
                    v = (i, j, int(k), int(l))
                    t = tuple(int(b[v[x], v[y]]) for x, y in _EDGES6)
                    H[rank[canonical6(t)]] += 1
                    count += 1
    return H, count


def _scale(weights, k):
    m = min(abs(float(v)) for v in weights)
    t = m
    for _ in range(k - 1):
        t = t * m
    return 52 - math.frexp(t)[1] + 1


def pairs_weighted(xyz, L, rmin, rmax, nb, weights):
    """Edges per bin and exact sums of w_i*w_j (Python ints, units 2^-s)."""
    _, _, adj, b = pair_matrix(xyz, L, rmin, rmax, nb)
    s = _scale(weights, 2)
    cnt = np.zeros(nb, dtype=np.int64)
    ws = [0] * nb
    ii, jj = np.nonzero(np.triu(adj, 1))
    for i, j in zip(ii, jj):
        cnt[b[i, j]] += 1
        ws[b[i, j]] += int((float(weights[i]) * float(weights[j])) * 2.0 ** s)
    return cnt, ws, s


def signed_product(values):
    """Magnitudes multiplied in ascending order, signed by the product of
    the signs."""
    mags = sorted(abs(float(v)) for v in values)
    p = mags[0]
    for m in mags[1:]:
        p = p * m
    neg = sum(1 for v in values if float(v) < 0) % 2
    return -p if neg else p


def _clique_t(weights, v, s):
    return int(signed_product([weights[u] for u in v]) * 2.0 ** s)


def cliques4_weighted(xyz, L, rmin, rmax, nb, weights):
    """Exact clique-weight sums: by 6-edge configuration, and per hub
    contribution for the parity channels (even, pos, neg)."""
    n = len(xyz)
    d, q, adj, b = pair_matrix(xyz, L, rmin, rmax, nb)
    s = _scale(weights, 4)
    rank6 = configs6(nb)
    rank3 = lex_configs(nb)
    W6 = [0] * len(rank6)
    WE, WP, WN = ([0] * len(rank3) for _ in range(3))
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            common = adj[i] & adj[j]
            for k in [k for k in np.nonzero(common)[0] if k > j]:
                for l in [l for l in np.nonzero(common & adj[k])[0] if l > k]:
                    v = (i, j, int(k), int(l))
                    t = _clique_t(weights, v, s)
                    W6[rank6[canonical6(tuple(int(b[v[x], v[y]]) for x, y in _EDGES6))]] += t
                    for h in v:
                        sp = sorted([u for u in v if u != h], key=lambda u: q[h, u])
                        qa, qb, qc = (float(q[h, u]) for u in sp)
                        r = rank3[tuple(int(b[h, u]) for u in sp)]
                        WE[r] += t
                        if qa == qb or qb == qc:
                            continue
                        V = hub_volume(*(tuple(float(c) for c in d[h, u]) for u in sp))
                        if V * V <= 1e-18 * ((qa * qb) * qc):
                            continue
                        (WP if V > 0 else WN)[r] += t
    return W6, WE, WP, WN, s


def triangles_mu(xyz, L, rmin, rmax, nb, nmu):
    """Triangles by (lexicographic rank of sorted side bins) * nmu + mu bin,
    mu = |n_z| / |n| for n = d(p0,p1) x d(p0,p2), p0 < p1 < p2 the vertices in
    index order, counted as the number of k in 1..nmu-1 with
    (n_z n_z)(nmu nmu) >= (k k)((n_x n_x + n_y n_y) + n_z n_z); collinear: 0."""
    n = len(xyz)
    d, _, adj, b = pair_matrix(xyz, L, rmin, rmax, nb)
    rank = lex_configs(nb)
    hist = np.zeros(len(rank) * nmu, dtype=np.int64)
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if not (adj[i, k] and adj[j, k]):
                    continue
                u, v = d[i, j], d[i, k]
                nx = u[1] * v[2] - u[2] * v[1]
                ny = u[2] * v[0] - u[0] * v[2]
                nz = u[0] * v[1] - u[1] * v[0]
                s = (nx * nx + ny * ny) + nz * nz
                m = 0
                if s > 0.0:
                    t = (nz * nz) * float(nmu * nmu)
                    m = sum(1 for kk in range(1, nmu) if t >= float(kk * kk) * s)
                c = rank[tuple(sorted((int(b[i, j]), int(b[i, k]), int(b[j, k]))))]
                hist[c * nmu + m] += 1
    return hist


def pixel(r):
    """Direction pixel: octant (x<0: 4, y<0: 2, z<0: 1) * 32 + i * 4 + j with
    i = min(7, floor(8 |x|/s)), s = (|x|+|y|)+|z|, j = min(3, floor(4 |y|/(|y|+|z|)))."""
    ax, ay, az = abs(float(r[0])), abs(float(r[1])), abs(float(r[2]))
    s = (ax + ay) + az
    if not s > 0.0:
        return 0
    o = 4 * (r[0] < 0) + 2 * (r[1] < 0) + (r[2] < 0)
    i = min(7, math.floor(8.0 * (ax / s)))
    yz = ay + az
    j = min(3, math.floor(4.0 * (ay / yz))) if yz > 0.0 else 0
    return int(o) * 32 + i * 4 + j


def pixel_dir(p):
    o, i, j = p >> 5, (p >> 2) & 7, p & 3
    ac, tc = (i + 0.5) / 8.0, (j + 0.5) / 4.0
    v = [ac, (1.0 - ac) * tc, (1.0 - ac) * (1.0 - tc)]
    for bit, c in ((4, 0), (2, 1), (1, 2)):
        if o & bit:
            v[c] = -v[c]
    n = math.sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2])
    return [c / n for c in v]


def cliques4_pixel(xyz, L, rmin, rmax, nb):
    """Parity with direction pixels: per clique and hub, spokes in index
    order, V from pixel centres, degenerate iff |V| < 1e-9."""
    n = len(xyz)
    d, q, adj, b = pair_matrix(xyz, L, rmin, rmax, nb)
    rank = lex_configs(nb)
    E = np.zeros(len(rank), dtype=np.int64)
    P = np.zeros_like(E)
    N = np.zeros_like(E)
    count = 0
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if not (adj[i, k] and adj[j, k]):
                    continue
                for l in range(k + 1, n):
                    if not (adj[i, l] and adj[j, l] and adj[k, l]):
                        continue
                    count += 1
                    v = (i, j, k, l)
                    for h in v:
                        sp = [s for s in v if s != h]
                        u = [pixel_dir(pixel(d[h, s])) for s in sp]
                        cx = u[0][1] * u[1][2] - u[0][2] * u[1][1]
                        cy = u[0][2] * u[1][0] - u[0][0] * u[1][2]
                        cz = u[0][0] * u[1][1] - u[0][1] * u[1][0]
                        V = (cx * u[2][0] + cy * u[2][1]) + cz * u[2][2]
                        c = rank[tuple(sorted(int(b[h, s]) for s in sp))]
                        E[c] += 1
                        if abs(V) >= 1e-9:
                            if V > 0:
                                P[c] += 1
                            else:
                                N[c] += 1
    return E, P, N, count
