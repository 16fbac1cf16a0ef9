"""Benchmark of the hot path on one MI355X. Prints ONE JSON line.

The headline is the largest single-GPU workload: 2,000,000 lognormal-like
points in a periodic 2000 Mpc/h box, rmax 150 Mpc/h, 20 bins, float64
weights, exact weighted triangle sums (7.2e9 directed edges, ~2e12
triangles). One step = the whole path over the catalogue already resident
in HBM: build the r < rmax graph (cell list, sorted forward CSR, bin bytes,
label-ordered weights) and count binned triangles with their exact weighted
sums.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-extras]

value = tuples counted per second of step time (build + count). The other
workloads ride along in the same line under "configs" (fewer steps each):
the 1e6-point clustered 3pCF, the 2e5-point parity 4pCF and the serving
stream of 256 catalogues.

Rooflines. The triangle count is bound by instruction issue on its hash
probes (measured traffic is a fraction of HBM bandwidth), so its roofline is
candidates probed per second against the attainable probe rate that the
library's probe microbenchmark measures on this GPU with the same table
size, load, bin count, hit rate and weighting; the HBM share (measured
traffic against 8 TB/s and against a measured stream copy), the LDS-atomic
histogram ceiling and the merge-walk byte model are reported beside it. The
parity count is float64 work: 120 operations per 4-clique against the
published 78.6 TFLOP/s. cpu_baseline = the CPU oracle on a bounded sample
of the same catalogue (anchor ranges spread over it), on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "binned triangles/s and 4-cliques/s on 1 GPU; batched catalogues/hour + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6            # published float64 vector peak (a fused multiply-add counts two)
FP64_OPS_PER_CLIQUE = 120          # separations, squared lengths, four hub volumes and thresholds
PROFILES = os.path.join(ROOT, "profiles")

WORKLOADS = {
    "lognormal_w3pcf": dict(kind="w3pcf", unit="triangles/s",
                            desc="2,000,000 lognormal-like points in a periodic 2000 Mpc/h box, rmax 150 "
                                 "Mpc/h, 20 bins, float64 weights U(0.5,1.5), exact weighted sums"),
    "ns_3pcf": dict(kind="3pcf", unit="triangles/s",
                    desc="1,000,000 Neyman-Scott points (20,000 parents x 50, sigma 3 Mpc/h) in a periodic "
                         "1000 Mpc/h box, rmax 30 Mpc/h, 15 bins, uint64 counts"),
    "ns_4pcf_parity": dict(kind="4pcf", unit="4-cliques/s",
                           desc="200,000 Neyman-Scott points (4,000 x 50, sigma 3) in a periodic 400 Mpc/h "
                                "box, rmax 20 Mpc/h, 8 bins, even/odd uint64 counts"),
}
# oracle sample per workload: anchor ranges spread over the catalogue
# (count, anchors per range), sized to ~10-20 s of host time
CPU_SAMPLE = {"w3pcf": (8, 8), "3pcf": (4, 20000), "4pcf": (8, 50)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest(kind: str) -> str:
    name = "count4.hip" if kind == "4pcf" else "count3.hip"
    p = os.path.join(ROOT, "paper_2607_06604_amd", "csrc", name)
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic(workload: str, kind: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source (else None)."""
    p = os.path.join(PROFILES, "traffic_%s.json" % workload)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_digest(kind):
        return None
    return d.get("hbm_bytes_per_launch")


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=float), q))


def plan_table(info, t):
    """Hash table size and its typical keys for a graph under the schedule
    its last count ran with (from the library's timings): a group of up to
    `group` hubs holds about group x mean forward degree keys, at most
    min(maxdeg, block) and the table's load bound."""
    maxdeg = max(1, int(info.max_deg))
    mean = info.n_edges / max(1, info.n)
    log2h, block, group = int(t.table_log2), int(t.block), max(1, int(t.group))
    load = 0.5 if t.hash_load == 5 else 0.69
    keys = int(min(group * mean, min(maxdeg, block), load * (1 << log2h)))
    return log2h, max(1, keys), block


def cpu_baseline(w, kind):
    import oracle
    nr, per = CPU_SAMPLE[kind]
    t0 = time.perf_counter()
    cnt, threads = 0, 0
    ranges = []
    for r in range(nr):
        lo = (w.n * r) // nr
        hi = min(w.n, lo + per)
        ranges.append((lo, hi))
        if kind == "4pcf":
            rr = oracle.count_4pcf_parity(w.xyz, w.box, w.rmin, w.rmax, w.nbins, anchors=(lo, hi))
            cnt += rr.n_cliques
        else:
            rr = oracle.count_3pcf(w.xyz, w.box, w.rmin, w.rmax, w.nbins,
                                   weights=w.weights if kind == "w3pcf" else None, anchors=(lo, hi))
            cnt += rr.n_triangles
        threads = rr.threads
    dt = time.perf_counter() - t0
    return {"value": round(cnt / dt, 1), "unit": WORKLOADS_UNIT[kind], "cores": threads, "kind": "oracle",
            "sample": "tuples whose smallest original index lies in %d ranges of %d anchors spread evenly "
                      "over the %d points (%d anchors, %.2e of the catalogue; rows built for the anchors and "
                      "their neighbours), %d tuples in %.1f s" % (nr, per, w.n, nr * per, nr * per / w.n,
                                                                  cnt, dt)}


WORKLOADS_UNIT = {"w3pcf": "triangles/s", "3pcf": "triangles/s", "4pcf": "4-cliques/s"}


def run_workload(gsn, ctx, name, steps, warmup, tune=True, windows=0, with_cpu=True, ceil=None):
    """Time `steps` steps (build + count) of one named workload; returns the
    JSON fields of its line."""
    import torch
    import synth
    spec = WORKLOADS[name]
    kind = spec["kind"]
    w = synth.workload(name)
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(w.xyz).to(dev)
    wd = torch.from_numpy(w.weights).to(dev) if kind == "w3pcf" else None
    keep = kind == "4pcf"
    torch.cuda.synchronize()
    if windows:
        os.environ["GS_WINDOWS"] = str(windows)
    else:
        os.environ.pop("GS_WINDOWS", None)

    schedule = None
    if kind in ("3pcf", "w3pcf") and tune and not windows:
        g = ctx.build_graph(xd, w.box, w.rmin, w.rmax, w.nbins, weights=wd)
        tt = time.perf_counter()
        schedule = ctx.tune_3pcf(g, weighted=kind == "w3pcf")
        schedule["tune_s"] = round(time.perf_counter() - tt, 3)
        g.free()
        log("%s tuned schedule: %s" % (name, json.dumps(schedule)))

    def step():
        g = ctx.build_graph(xd, w.box, w.rmin, w.rmax, w.nbins, keep_coords=keep, weights=wd)
        t_build = ctx.timings().build_ms
        if kind == "4pcf":
            r = ctx.count_4pcf_parity(g)
            tuples = r.n_cliques
        else:
            r = ctx.count_3pcf(g, weighted=kind == "w3pcf")
            tuples = r.n_triangles
        t = ctx.timings()
        g.free()
        return tuples, t_build, t

    for k in range(warmup):
        tw = time.perf_counter()
        step()
        log("%s warmup step %d: %.1f ms" % (name, k, (time.perf_counter() - tw) * 1e3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms, launches, count_ms, build_ms, probes = 0.0, 0, 0.0, 0.0, 0
    tuples = 0
    for k in range(steps):
        tuples, tb, t = step()
        if t.count_ms > 1000 or tb > 1000 or k == steps - 1:
            log("%s step %d: build %.1f ms, count %.1f ms" % (name, k, tb, t.count_ms))
        kern_ms += t.kernel_ms
        launches += t.kernel_launches
        count_ms += t.count_ms
        build_ms += tb
        probes += t.probes
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    value = tuples / (ms_per_step / 1e3)

    # graph statistics outside the timed region: the merge-walk byte model
    g = ctx.build_graph(xd, w.box, w.rmin, w.rmax, w.nbins, keep_coords=keep, weights=wd)
    info = g.info()
    alg_bytes = int(2.5 * info.sum_sq_degree)
    g.free()
    avg_launch_ms = kern_ms / max(launches, 1)
    count_kernel_ms = kern_ms / steps          # all launches of one count
    traffic = stored_traffic(name, kind) if windows <= 1 else None

    if kind == "4pcf":
        ops = FP64_OPS_PER_CLIQUE * tuples
        tflops = ops / (count_kernel_ms / 1e3) / 1e12 if count_kernel_ms > 0 else 0.0
        roofline = {"bound": "alu", "achieved": round(tflops, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tflops / FP64_PEAK_TFLOPS, 4), "traffic": traffic, "kernel": "k_count4",
                    "fp64_ops_per_clique": FP64_OPS_PER_CLIQUE, "avg_launch_ms": round(avg_launch_ms, 4),
                    "hbm_measured_GBs": round(traffic / (avg_launch_ms / 1e3) / 1e9, 1) if traffic else None}
    else:
        probes_per_count = probes // steps
        achieved = probes_per_count / (count_kernel_ms / 1e3) / 1e9 if count_kernel_ms > 0 else 0.0
        hit = tuples / max(1, probes_per_count)
        log2h, keys, block = plan_table(info, t)
        weighted = kind == "w3pcf"
        peak = ctx.ceiling_probe(w.nbins, log2h, keys, min(1.0, max(1e-6, hit)), weighted=weighted,
                                 probe=True, block=block) / 1e9
        hist_peak = ctx.ceiling_probe(w.nbins, log2h, keys, 1.0, weighted=weighted, probe=False,
                                      block=block) / 1e9
        tri_rate = tuples / (count_kernel_ms / 1e3) / 1e9 if count_kernel_ms > 0 else 0.0
        merge_gbs = alg_bytes / (count_kernel_ms / 1e3) / 1e9 if count_kernel_ms > 0 else 0.0
        hbm = None
        if traffic:
            gbs = traffic / (avg_launch_ms / 1e3) / 1e9
            hbm = {"measured_GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                   "frac_of_copy": round(gbs / ceil["copy_GBs"], 4) if ceil else None}
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 2), "unit": "Gprobe/s",
                    "frac": round(achieved / peak, 4) if peak > 0 else None, "traffic": traffic,
                    "kernel": "k_count3", "avg_launch_ms": round(avg_launch_ms, 4),
                    "launches_per_count": launches // max(steps, 1),
                    "probes_per_count": probes_per_count, "hit_rate": round(hit, 4),
                    "peak_source": "gs_ceiling_probe: table 2^%d slots, %d keys, %d bins, hit rate %.3f, %s, "
                                   "%d threads per group" % (log2h, keys, w.nbins, hit,
                                                             "weighted" if weighted else "unweighted", block),
                    "hbm": hbm,
                    "lds_hist": {"achieved_Gtuples_s": round(tri_rate, 2), "peak_Gtuples_s": round(hist_peak, 2),
                                 "frac": round(tri_rate / hist_peak, 4) if hist_peak > 0 else None},
                    "merge_walk_model": {"alg_bytes_per_count": alg_bytes, "GBs": round(merge_gbs, 1),
                                         "note": "2.5 B x sum of squared degrees: the bytes a two-pointer merge "
                                                 "walk over both forward half lists would read; the hash probes "
                                                 "read each spoke row once per hub from L2, so this is a model, "
                                                 "not a bound"}}
    out = {
        "value": round(value, 1), "unit": spec["unit"], "steps": steps, "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "config": {"workload": name, "description": spec["desc"], "n_points": w.n, "box": w.box,
                   "rmax": w.rmax, "nbins": w.nbins, "tuples_per_step": tuples, "windows": windows or 1},
        "query_only": {"value": round(tuples / (count_ms / steps / 1e3), 1), "unit": spec["unit"],
                       "count_ms": round(count_ms / steps, 4), "build_ms": round(build_ms / steps, 4)},
        "roofline": roofline,
        "schedule": schedule,
    }
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(w, kind)
    return out


def run_stream(gsn, count, tune=True):
    """Serving workload: a stream of catalogues of uneven size (log-uniform
    5e4..5e5 points; even index clustered data, odd index uniform randoms) in
    periodic 600 Mpc/h boxes, 3pCF at rmax 40 Mpc/h in 10 bins. Measures the
    plain path (each catalogue built and counted alone, back to back), the
    server with every request arriving at once, and the server under Poisson
    arrivals at 0.8 of the measured batched capacity."""
    import numpy as np
    import torch
    import synth

    L, rmax, nb = 600.0, 40.0, 10
    sizes = synth.stream_sizes(count, seed=5)
    cats = [synth.stream_catalogue(k, int(n), L=L, seed=5) for k, n in enumerate(sizes)]
    log("stream: generated %d catalogues, %d points" % (len(cats), int(sizes.sum())))
    torch.cuda.synchronize()
    big = int(np.argmax(sizes))

    def do_tune(c):
        g = c.build_graph(cats[big], L, 0.0, rmax, nb)
        c.tune_3pcf(g)
        g.free()

    with gsn.Context(0) as c:
        if tune:
            do_tune(c)
        for x in cats[:2]:
            g = c.build_graph(x, L, 0.0, rmax, nb)
            c.count_3pcf(g)
            g.free()
        lat_seq, want, tri = [], [], 0
        t0 = time.perf_counter()
        for x in cats:
            ts = time.perf_counter()
            g = c.build_graph(x, L, 0.0, rmax, nb)
            r = c.count_3pcf(g)
            g.free()
            lat_seq.append(time.perf_counter() - ts)
            want.append(r.hist)
            tri += r.n_triangles
        t_seq = time.perf_counter() - t0
    log("stream: sequential %.3f s" % t_seq)

    def serve(arrivals):
        with gsn.Context(0) as s:
            if tune:
                do_tune(s)
            t = s.submit(cats[1][:1000], L, 0.0, rmax, nb)
            while s.poll(t, nb) is None:
                time.sleep(0.001)
            tickets = [None] * len(cats)
            res = {}
            t0 = time.perf_counter()
            k = 0
            while len(res) < len(cats):
                now = time.perf_counter() - t0
                while k < len(cats) and arrivals[k] <= now:
                    tickets[k] = s.submit(cats[k], L, 0.0, rmax, nb)
                    k += 1
                for j in range(k):
                    if j not in res:
                        r = s.poll(tickets[j], nb)
                        if r is not None:
                            res[j] = r
                time.sleep(0.0005)
            makespan = time.perf_counter() - t0
        for j in range(len(cats)):
            assert res[j]["status"] == gsn.GS_DONE and np.array_equal(res[j]["hist"], want[j]), j
        lat = [res[j]["t_total_s"] for j in range(len(cats))]
        steps = [res[j]["step_size"] for j in range(len(cats))]
        return makespan, lat, steps

    span_all, lat_all, steps_all = serve(np.zeros(len(cats)))
    log("stream: served, all at t=0: %.3f s" % span_all)
    rate = 0.8 * len(cats) / span_all
    gaps = -np.log(1.0 - synth.uniform_values(len(cats), 0.0, 1.0, 55)) / rate
    arr = np.cumsum(gaps) - gaps[0]
    span_p, lat_p, steps_p = serve(arr)
    log("stream: served, Poisson at %.1f/s: %.3f s" % (rate, span_p))
    per_hour = len(cats) / span_all * 3600.0
    return {
        "value": round(per_hour, 1), "unit": "catalogues/hour", "ms_per_step": round(span_all * 1e3, 3),
        "config": {"workload": "stream_3pcf", "catalogues": len(cats), "points": int(sizes.sum()),
                   "sizes": "log-uniform 5e4..5e5, even clustered (Neyman-Scott 50, sigma 3), odd uniform",
                   "box": L, "rmax": rmax, "nbins": nb, "triangles": int(tri)},
        "all_at_once": {"catalogues_per_hour": round(per_hour, 1), "p50_s": round(percentile(lat_all, 50), 4),
                        "p99_s": round(percentile(lat_all, 99), 4),
                        "mean_step": round(float(np.mean(steps_all)), 2),
                        "triangles_per_s": round(tri / span_all, 1)},
        "poisson": {"rate_per_s": round(rate, 2), "catalogues_per_hour": round(len(cats) / span_p * 3600, 1),
                    "p50_s": round(percentile(lat_p, 50), 4), "p99_s": round(percentile(lat_p, 99), 4),
                    "mean_step": round(float(np.mean(steps_p)), 2)},
        "sequential": {"catalogues_per_hour": round(len(cats) / t_seq * 3600, 1),
                       "p50_s": round(percentile(lat_seq, 50), 4), "p99_s": round(percentile(lat_seq, 99), 4),
                       "triangles_per_s": round(tri / t_seq, 1)},
        "speedup_vs_sequential": round(t_seq / span_all, 3),
        "results_checked": "every served histogram equals the same catalogue's lone count",
    }


def _timed(fn, steps):
    """Run fn once untimed, then `steps` times; ms per call (wall clock with
    device synchronisation) and the last result."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = None
    for _ in range(steps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, r


def run_extras(gsn, ctx):
    """The paper's further counts and estimators, each on a synthetic
    stand-in of its workload, timed as build + count per step (graphs built
    from coordinates already in device memory where the call takes them)."""
    import numpy as np
    import torch
    import synth
    out = {}
    dev = torch.device("cuda:0")

    # 6-edge 4-cliques (Sec. 3.3, Sec. 5.3): the 2e5-point clustered
    # catalogue, 4 bins (276 configurations, the paper's count)
    c3 = synth.workload("ns_4pcf_parity")
    x3 = torch.from_numpy(c3.xyz).to(dev)

    def six():
        g = ctx.build_graph(x3, c3.box, 0.0, c3.rmax, 4, keep_coords=True)
        r = ctx.count_4pcf_full(g)
        t = ctx.timings()
        g.free()
        return r, t
    ms, (r, t) = _timed(six, 2)
    out["ns_4pcf_full"] = {"value": round(r.n_cliques / (ms / 1e3), 1), "unit": "4-cliques/s",
                           "ms_per_step": round(ms, 3), "kernel_ms": round(t.kernel_ms, 3),
                           "config": {"workload": "ns_4pcf_full", "n_points": c3.n, "box": c3.box, "rmax": c3.rmax,
                                      "nbins": 4, "configurations": int(len(r.hist)),
                                      "cliques_per_step": r.n_cliques}}
    log("ns_4pcf_full: %.1f ms" % ms)

    # parity from direction pixels (Sec. 3.2 as the paper computes it)
    def pix():
        g = ctx.build_graph(x3, c3.box, 0.0, c3.rmax, c3.nbins, keep_coords=True)
        r = ctx.count_4pcf_pixel(g)
        t = ctx.timings()
        g.free()
        return r, t
    ms, (r, t) = _timed(pix, 2)
    out["ns_4pcf_pixel"] = {"value": round(r.n_cliques / (ms / 1e3), 1), "unit": "4-cliques/s",
                            "ms_per_step": round(ms, 3), "kernel_ms": round(t.kernel_ms, 3),
                            "config": {"workload": "ns_4pcf_pixel", "n_points": c3.n, "box": c3.box,
                                       "rmax": c3.rmax, "nbins": c3.nbins, "cliques_per_step": r.n_cliques}}
    log("ns_4pcf_pixel: %.1f ms" % ms)

    # restricted and anisotropic triangle counts and survey geometry on the
    # 1e6-point clustered catalogue
    c2 = synth.workload("ns_3pcf")
    x2 = torch.from_numpy(c2.xyz).to(dev)
    for name, mk in (("ns_3pcf_equilateral", lambda g: ctx.count_3pcf_equilateral(g)),
                     ("ns_3pcf_mu", lambda g: ctx.count_3pcf_mu(g, 5)),
                     ("ns_3pcf_survey", lambda g: ctx.count_3pcf(g))):
        def step(mk=mk, name=name):
            g = ctx.build_graph(x2, c2.box, 0.0, c2.rmax, c2.nbins, keep_coords=name == "ns_3pcf_mu",
                                periodic=name != "ns_3pcf_survey")
            r = mk(g)
            t = ctx.timings()
            g.free()
            return r, t
        ms, (r, t) = _timed(step, 5)
        out[name] = {"value": round(r.n_triangles / (ms / 1e3), 1), "unit": "triangles/s",
                     "ms_per_step": round(ms, 3), "kernel_ms": round(t.kernel_ms, 3),
                     "config": {"workload": name, "n_points": c2.n, "box": c2.box, "rmax": c2.rmax,
                                "nbins": c2.nbins, "mu_bins": 5 if name == "ns_3pcf_mu" else None,
                                "periodic": name != "ns_3pcf_survey", "triangles_per_step": r.n_triangles}}
        log("%s: %.2f ms" % (name, ms))

    # estimators (Sec. 2.1, 3.3, 3.4): data and randoms, signed weights
    xd = synth.neyman_scott(500_000, 50, 3.0, 1000.0, 21)
    xr = synth.uniform(500_000, 1000.0, 22)
    ms, r = _timed(lambda: gsn.compute_3pcf(xd, None, xr, None, 0.0, 30.0, 15, 1000.0, ctx=ctx), 2)
    out["estimator_3pcf"] = {"value": round(1e3 / ms * 3600.0, 1), "unit": "estimates/hour", "ms_per_step": round(ms, 3),
                             "config": {"workload": "estimator_3pcf", "data": "500,000 Neyman-Scott points",
                                        "randoms": "500,000 uniform", "box": 1000.0, "rmax": 30.0, "nbins": 15,
                                        "counts": "combined catalogue (signed weights) + randoms alone"}}
    log("estimator_3pcf: %.1f ms" % ms)
    xd4 = synth.neyman_scott(100_000, 50, 3.0, 400.0, 23)
    xr4 = synth.uniform(100_000, 400.0, 24)
    ms, r = _timed(lambda: gsn.compute_4pcf(xd4, None, xr4, None, 0.0, 20.0, 4, 400.0, ctx=ctx), 1)
    out["estimator_4pcf"] = {"value": round(1e3 / ms * 3600.0, 1), "unit": "estimates/hour", "ms_per_step": round(ms, 3),
                             "config": {"workload": "estimator_4pcf", "data": "100,000 Neyman-Scott points",
                                        "randoms": "100,000 uniform", "box": 400.0, "rmax": 20.0, "nbins": 4,
                                        "outputs": "parity even/odd, 6-edge, connected, internal 2pCF"}}
    log("estimator_4pcf: %.1f ms" % ms)
    return out


def run_oversubscribed(gsn):
    """Out of core at the paper's scale (Sec. 3.5.3): 2.25e6 lognormal points,
    L 2000, rmax 150, 20 bins, weighted, ~9.1e9 directed edges (23 GB of
    forward CSR) under a 16 GB device budget: host-tiled windows staged over
    PCIe while counting. One step; the host input is copied in the build."""
    import synth
    n, L = 2_250_000, 2000.0
    x = synth.lognormal(n, L, 7)
    w = synth.uniform_values(n, 0.5, 1.0, 8)
    with gsn.Context(0, budget_bytes=16 << 30) as c:
        t0 = time.perf_counter()
        g = c.build_graph(x, L, 0.0, 150.0, 20, weights=w)
        t1 = time.perf_counter()
        info = g.info()
        r = c.count_3pcf(g, weighted=True)
        t2 = time.perf_counter()
        tm = c.timings()
        g.free()
    log("oversubscribed: build %.2f s, count %.2f s, %d windows" % (t1 - t0, t2 - t1, info.n_windows))
    return {"value": round(r.n_triangles / (t2 - t0), 1), "unit": "triangles/s", "ms_per_step": round((t2 - t0) * 1e3, 1),
            "count_ms": round((t2 - t1) * 1e3, 1), "build_ms": round((t1 - t0) * 1e3, 1),
            "kernel_ms": round(tm.kernel_ms, 1),
            "config": {"workload": "lognormal_w3pcf_oversubscribed", "n_points": n, "box": L, "rmax": 150.0,
                       "nbins": 20, "directed_edges": 2 * int(info.n_edges), "windows": int(info.n_windows),
                       "budget_bytes": 16 << 30, "triangles": r.n_triangles,
                       "note": "host input; step time includes the host-to-device copies of every window"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal_w3pcf", choices=sorted(WORKLOADS) + ["stream_3pcf"])
    ap.add_argument("--stream-count", type=int, default=256)
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the named workload (no other configs, no ceilings)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--windows", type=int, default=0,
                    help="force a host-tiled graph with this many windows (out-of-core path)")
    ap.add_argument("--no-tune", action="store_true", help="skip the schedule autotuner (built-in schedule)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration under rocprofv3)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the counts would shard by hub ranges with one final reduction of the bins).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2607_06604_amd as gsn

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        a.fill_(1.0)
        b = a.clone()
        torch.cuda.synchronize()
        del a, b

    tune = not args.no_tune
    if args.workload == "stream_3pcf":
        r = run_stream(gsn, args.stream_count, tune=tune)
        line = {"metric": METRIC, "value": r["value"], "unit": r["unit"], "n_gpus": 1, "steps": 1, "warmup": 2,
                "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f64+int", "data": "synthetic"}
        line.update({k: v for k, v in r.items() if k not in line})
        print(json.dumps(line), flush=True)
        return

    stream = torch.cuda.current_stream(dev)
    ctx = gsn.Context(0, stream=stream)
    ceil = None
    if not args.no_extras:
        ceil = {"copy_GBs": round(ctx.ceiling_copy(2 << 30), 1)}
        log("ceiling: stream copy %.1f GB/s" % ceil["copy_GBs"])
    head = run_workload(gsn, ctx, args.workload, args.steps, args.warmup, tune=tune, windows=args.windows,
                        with_cpu=not args.no_cpu_baseline, ceil=ceil)
    line = {
        "metric": METRIC, "value": head["value"], "unit": head["unit"], "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+int",
        "data": "synthetic", "config": head["config"], "query_only": head["query_only"],
        "roofline": head["roofline"], "cpu_baseline": head.get("cpu_baseline"), "schedule": head["schedule"],
    }
    if ceil:
        line["ceilings"] = ceil
    if not args.no_extras:
        others = {}
        for name, st in (("ns_3pcf", 10), ("ns_4pcf_parity", 4)):
            if name == args.workload:
                continue
            r = run_workload(gsn, ctx, name, st, 1, tune=tune, with_cpu=not args.no_cpu_baseline, ceil=ceil)
            others[name] = r
            log("%s: %.3e %s" % (name, r["value"], r["unit"]))
        others["stream_3pcf"] = run_stream(gsn, args.stream_count, tune=tune)
        others.update(run_extras(gsn, ctx))
        others["lognormal_w3pcf_oversubscribed"] = run_oversubscribed(gsn)
        line["configs"] = others
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
