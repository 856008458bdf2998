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

Run: python -m paper_1812_06060_amd.serving_bench [--levels 4-8] [--queries N] ...
"""
from __future__ import annotations

import argparse
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


def run(levels=(4, 8), n_meshes=32, n_queries=150, n_warm=16, rate_frac=0.9, slots=4, seed=6, log=print,
        rate_fracs=None, workers=1):
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

    # service times alone (also warms every mesh's workspace once)
    service = []
    for j, (i, src) in enumerate(qs):
        torch.cuda.synchronize()
        a = time.perf_counter()
        meshes[i].solve(src, 0.0, opts, out=outs[j])
        torch.cuda.synchronize()
        service.append(time.perf_counter() - a)
        if (j + 1) % 25 == 0:
            log(f"[serve] reference solves: {j + 1}/{len(qs)}")
    ref = [o.cpu().numpy() for o in outs]
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
        same_plain = all(np.array_equal(outs[j].cpu().numpy(), ref[j]) for j in timed)

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
        same_srv = all(np.array_equal(outs[j].cpu().numpy(), ref[j]) for j in timed)
        lat_s = list(lat_srv.values())
        res = {
            "queries": n_queries, "pool_levels": list(levels), "pool_meshes": len(meshes), "slots": slots,
            "rate_frac": rf, "offered_qps": rate, "plain_saturation_qps": sat,
            "served": {"qps": n_queries / span_srv, "p50_ms": 1e3 * _pct(lat_s, 50), "p99_ms": 1e3 * _pct(lat_s, 99)},
            "plain": {"qps": n_queries / span_plain, "p50_ms": 1e3 * _pct(lat_plain, 50),
                      "p99_ms": 1e3 * _pct(lat_plain, 99)},
            "results_identical": bool(same_plain and same_srv),
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
    a = ap.parse_args()
    lo, hi = (int(x) for x in a.levels.split("-"))
    rates = [float(x) for x in a.rates.split(",")]
    for r in run((lo, hi), a.meshes, a.queries, a.warm, slots=a.slots, rate_fracs=rates, workers=a.workers,
                 log=lambda s: print(s, file=sys.stderr, flush=True)):
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
