"""Serving benchmark: a seeded Poisson stream of geodesic queries over a pool of
resident meshes, served by the hg_server runtime and, on the same stream, by
plain per-query solves one at a time.

Workload (all seeded):
  * pool: `n_meshes` displaced icospheres; the first cover the levels in
    order, the rest are drawn uniformly from the level range (seed 5); mesh i
    is displaced by the harmonic sum of `meshgen.harmonic_displacement` with
    seed 5000 + i;
  * queries (seed 6): mesh uniform over the pool, k = min(64, floor(exp(U(0,
    ln 65)))) distinct uniform sources, edge form, default options;
  * arrivals: Poisson with rate `rate_frac` times the plain path's measured
    saturation rate (1 / mean service time of one query alone).

Both paths run the same solve (identical results, checked on every query),
so they are compared at the same accuracy.  Latency = completion - arrival.

With --plain-sim the plain path is not run again on each arrival clock: one
query at a time in arrival order is a single first-in-first-out server, so
its completions follow from the measured service time of every query alone
(completion_k = max(arrival_k, completion_{k-1}) + service_k).  The service
times and a hash of every reference result can be stored (--save-ref) and
reused (--load-ref) by later runs of the same pool and queries, which then
only serve the stream and compare hashes.

Run: python -m paper_1812_06060_amd.serving_bench [--levels 4-8] [--queries N] ...
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import sys
import threading
import time

import numpy as np


def build_pool(levels, n_meshes: int, seed: int = 5, workers: int = 1):
    import meshgen
    lo, hi = levels
    rng = np.random.default_rng(seed)
    lv = list(range(lo, hi + 1))
    while len(lv) < n_meshes:
        lv.append(int(rng.integers(lo, hi + 1)))
    lv = lv[:n_meshes]
    base = {}
    pool = []
    for i, L in enumerate(lv):
        if L not in base:
            base[L] = meshgen.icosphere(L)
        v, f = base[L]
        pool.append((L, meshgen.harmonic_displacement(v, seed=5000 + i, workers=workers), f))
    return pool


def make_queries(pool, n: int, seed: int = 6):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        i = int(rng.integers(len(pool)))
        k = min(64, int(math.floor(math.exp(rng.uniform(0.0, math.log(65.0))))))
        nv = pool[i][1].shape[0]
        out.append((i, rng.choice(nv, size=k, replace=False).astype(np.int32)))
    return out


def _pct(x, p):
    return float(np.percentile(np.asarray(x), p)) if len(x) else float("nan")


def _digest(t) -> str:
    return hashlib.sha256(t.cpu().numpy().tobytes()).hexdigest()


def fifo_latencies(arrivals, service):
    """Latencies of one first-in-first-out server: each query starts when it
    has arrived and the previous one has finished."""
    lat, done = [], 0.0
    for a, s in zip(arrivals, service):
        done = max(a, done) + s
        lat.append(done - a)
    return lat, done


def run(levels=(4, 8), n_meshes=32, n_queries=150, n_warm=16, rate_frac=0.9, slots=4, seed=6, log=print,
        rate_fracs=None, workers=1, plain_sim=False, save_ref=None, load_ref=None):
    """Serve the same seeded query stream at each rate in `rate_fracs`
    (default: just `rate_frac`); the pool, the queries and the references
    (one plain solve per query) are built once.  Returns one result per rate
    (a single dict when one rate is asked for)."""
    import torch

    import paper_1812_06060_amd as hg
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    pool = build_pool(levels, n_meshes, workers=workers)
    meshes = [hg.Mesh(v, f) for _, v, f in pool]
    log(f"[serve] pool of {len(meshes)} meshes (levels {levels[0]}-{levels[1]}, "
        f"{sum(m.nv for m in meshes)} vertices) ready in {time.perf_counter() - t0:.1f}s")
    opts = hg.default_opts()
    qs = make_queries(pool, n_warm + n_queries, seed)
    outs = [torch.empty(meshes[i].nv, dtype=torch.float32, device="cuda") for i, _ in qs]
    # every mesh's one-time work (its face tiles, a workspace with source
    # paths) before anything is timed
    for m in meshes:
        m.solve(np.array([0, m.nv - 1], dtype=np.int32), 0.0, opts)
    torch.cuda.synchronize()

    # service times alone, and the reference results (their hashes)
    if load_ref:
        with open(load_ref) as fh:
            stored = json.load(fh)
        if stored["queries"] != len(qs) or stored["levels"] != list(levels) or stored["meshes"] != n_meshes:
            raise SystemExit("--load-ref: stored references are for another pool or stream")
        service, ref = stored["service_s"], stored["sha256"]
    else:
        service, ref = [], []
        for j, (i, src) in enumerate(qs):
            torch.cuda.synchronize()
            a = time.perf_counter()
            meshes[i].solve(src, 0.0, opts, out=outs[j])
            torch.cuda.synchronize()
            service.append(time.perf_counter() - a)
            ref.append(_digest(outs[j]))
            if (j + 1) % 25 == 0:
                log(f"[serve] reference solves: {j + 1}/{len(qs)}")
        if save_ref:
            with open(save_ref, "w") as fh:
                json.dump({"queries": len(qs), "levels": list(levels), "meshes": n_meshes, "service_s": service,
                           "sha256": ref}, fh)
    svc = np.array(service[n_warm:])
    sat = 1.0 / svc.mean()
    log(f"[serve] plain service time mean {1e3 * svc.mean():.1f} ms (p50 {1e3 * _pct(svc, 50):.1f}, "
        f"p99 {1e3 * _pct(svc, 99):.1f}); saturation {sat:.2f} q/s")
    timed = list(range(n_warm, n_warm + n_queries))
    results = []
    for rf in (rate_fracs if rate_fracs else [rate_frac]):
        rate = rf * sat
        rng = np.random.default_rng(seed + 1)
        gaps = rng.exponential(1.0 / rate, size=n_queries)
        arrivals = np.cumsum(gaps) - gaps[0]

        if plain_sim:
            # plain: one first-in-first-out server with the measured service times
            lat_plain, span_plain = fifo_latencies(arrivals, svc)
            same_plain = True
        else:
            # plain: one query at a time, in arrival order, on the arrival clock
            lat_plain = []
            start = time.perf_counter()
            for k, j in enumerate(timed):
                now = time.perf_counter() - start
                if now < arrivals[k]:
                    time.sleep(arrivals[k] - now)
                i, src = qs[j]
                meshes[i].solve(src, 0.0, opts, out=outs[j])
                torch.cuda.synchronize()
                lat_plain.append(time.perf_counter() - start - arrivals[k])
                if (k + 1) % 25 == 0:
                    log(f"[serve] rate x{rf}: plain {k + 1}/{n_queries}")
            span_plain = time.perf_counter() - start
            same_plain = all(_digest(outs[j]) == ref[j] for j in timed)

        # served: submitted at the arrival times, completions taken by a thread
        # (the server stamps each query at submit: latency = t_end - t_submit)
        srv = hg.Server(slots)
        lat_srv = {}
        t_end = {}
        clock0 = hg.Server.clock()
        base = time.perf_counter()

        def collect():
            for c in range(len(timed)):
                r = srv.wait(-1)
                lat_srv[r["ticket"]] = r["t_end"] - r["t_submit"]
                t_end[r["ticket"]] = r["t_end"]
                if (c + 1) % 25 == 0:
                    log(f"[serve] rate x{rf}: served {c + 1}/{n_queries}")

        th = threading.Thread(target=collect)
        th.start()
        for k, j in enumerate(timed):
            now = time.perf_counter() - base
            if now < arrivals[k]:
                time.sleep(arrivals[k] - now)
            i, src = qs[j]
            srv.submit(meshes[i], src, out=outs[j], opts=opts)
        th.join()
        span_srv = max(t_end.values()) - clock0
        srv.close()
        same_srv = all(_digest(outs[j]) == ref[j] for j in timed)
        lat_s = list(lat_srv.values())
        res = {
            "queries": n_queries, "pool_levels": list(levels), "pool_meshes": len(meshes), "slots": slots,
            "rate_frac": rf, "offered_qps": rate, "plain_saturation_qps": sat,
            "served": {"qps": n_queries / span_srv, "p50_ms": 1e3 * _pct(lat_s, 50), "p99_ms": 1e3 * _pct(lat_s, 99)},
            "plain": {"qps": n_queries / span_plain, "p50_ms": 1e3 * _pct(lat_plain, 50),
                      "p99_ms": 1e3 * _pct(lat_plain, 99)},
            "results_identical": bool(same_plain and same_srv), "plain_path": "simulated" if plain_sim else "run",
        }
        log(f"[serve] rate x{rf}: served {res['served']}, plain {res['plain']}, identical {res['results_identical']}")
        results.append(res)
    for m in meshes:
        m.close()
    return results if rate_fracs else results[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", default="4-8")
    ap.add_argument("--meshes", type=int, default=32)
    ap.add_argument("--queries", type=int, default=150)
    ap.add_argument("--warm", type=int, default=16)
    ap.add_argument("--rates", default="0.9")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--workers", type=int, default=1, help="processes for the mesh displacement")
    ap.add_argument("--plain-sim", action="store_true",
                    help="plain path as a first-in-first-out server of the measured service times")
    ap.add_argument("--save-ref", default=None, help="store service times and result hashes here")
    ap.add_argument("--load-ref", default=None, help="reuse stored service times and result hashes")
    a = ap.parse_args()
    lo, hi = (int(x) for x in a.levels.split("-"))
    rates = [float(x) for x in a.rates.split(",")]
    for r in run((lo, hi), a.meshes, a.queries, a.warm, slots=a.slots, rate_fracs=rates, workers=a.workers,
                 plain_sim=a.plain_sim, save_ref=a.save_ref, load_ref=a.load_ref,
                 log=lambda s: print(s, file=sys.stderr, flush=True)):
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
