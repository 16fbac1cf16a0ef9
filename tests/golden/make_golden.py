"""Write the stored expected values used by the full-size GPU parity tests.

Calls only oracle/ (and the seeded generators in synth/). Each file records
the workload recipe and a SHA-256 of the generated float64 coordinates, so a
test can tell a generator change from a counting mismatch.

    python tests/golden/make_golden.py [name ...]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def ns_3pcf_full():
    w = synth.workload("ns_3pcf")
    t = time.time()
    r = oracle.count_3pcf(w.xyz, w.box, w.rmin, w.rmax, w.nbins)
    return dict(workload=w.name, recipe=w.recipe, xyz_sha256=digest(w.xyz), box=w.box, rmin=w.rmin,
                rmax=w.rmax, nbins=w.nbins, n_triangles=r.n_triangles, hist=[int(v) for v in r.hist],
                oracle_seconds=round(time.time() - t, 1), oracle_threads=r.threads)


def ns_4pcf_parity_sampled():
    """Full-size parity workload; anchors (smallest original index) restricted
    to sampled ranges the oracle finishes in seconds each."""
    w = synth.workload("ns_4pcf_parity")
    ranges = [(0, 150), (99_900, 100_050), (199_850, 200_000)]
    out = []
    t = time.time()
    for lo, hi in ranges:
        r = oracle.count_4pcf_parity(w.xyz, w.box, w.rmin, w.rmax, w.nbins, anchors=(lo, hi))
        out.append(dict(lo=lo, hi=hi, n_cliques=r.n_cliques, even=[int(v) for v in r.even],
                        pos=[int(v) for v in r.pos], neg=[int(v) for v in r.neg]))
    return dict(workload=w.name, recipe=w.recipe, xyz_sha256=digest(w.xyz), box=w.box, rmin=w.rmin,
                rmax=w.rmax, nbins=w.nbins, samples=out, oracle_seconds=round(time.time() - t, 1))


def lognormal_w3pcf_sampled():
    """Full-size weighted workload; anchors restricted to sampled ranges."""
    w = synth.workload("lognormal_w3pcf")
    ranges = [(0, 40), (1_000_000, 1_000_040), (1_500_000, 1_500_030)]
    out = []
    t = time.time()
    for lo, hi in ranges:
        r = oracle.count_3pcf(w.xyz, w.box, w.rmin, w.rmax, w.nbins, weights=w.weights, anchors=(lo, hi))
        out.append(dict(lo=lo, hi=hi, n_triangles=r.n_triangles, hist=[int(v) for v in r.hist],
                        wsum=[[int(a), int(b)] for a, b in r.wsum], wscale=r.wscale))
    return dict(workload=w.name, recipe=w.recipe, xyz_sha256=digest(w.xyz),
                weights_sha256=digest(w.weights), box=w.box, rmin=w.rmin, rmax=w.rmax, nbins=w.nbins,
                samples=out, oracle_seconds=round(time.time() - t, 1))


def stream_served():
    """Serving-stream catalogues (periodic 600 Mpc/h boxes, rmax 40, 10 bins;
    even index clustered, odd index uniform), a spread of sizes from 5e4 to
    2.5e5 points, each counted in full."""
    L, rmax, nb = 600.0, 40.0, 10
    sizes = synth.stream_sizes(256, seed=5)
    picks = [1, 16, 18, 31, 80, 88, 121, 161, 162, 165, 197, 201, 212, 240]
    out = []
    t = time.time()
    for k in picks:
        x = synth.stream_catalogue(k, int(sizes[k]), L=L, seed=5)
        r = oracle.count_3pcf(x, L, 0.0, rmax, nb)
        out.append(dict(index=k, n=int(sizes[k]), xyz_sha256=digest(x), n_triangles=r.n_triangles,
                        hist=[int(v) for v in r.hist]))
    return dict(workload="stream_3pcf", box=L, rmin=0.0, rmax=rmax, nbins=nb, seed=5,
                catalogues=out, oracle_seconds=round(time.time() - t, 1))


TARGETS = {"ns_3pcf_full": ns_3pcf_full, "stream_served": stream_served, "ns_4pcf_parity_sampled": ns_4pcf_parity_sampled,
           "lognormal_w3pcf_sampled": lognormal_w3pcf_sampled}

if __name__ == "__main__":
    names = sys.argv[1:] or list(TARGETS)
    for name in names:
        d = TARGETS[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(d, f, indent=0)
        print(name, "written", d.get("oracle_seconds"))
