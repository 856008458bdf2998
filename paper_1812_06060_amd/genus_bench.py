"""Genus benchmark: single-source distance on jittered tori (closed, genus 1)
with the cycle constraints of Sec. 5.1 against the same solve without them.

Workload (seeded): `meshgen.torus(nu, nv, R=1, r, jitter=0.1, seed=7)`, one
source from `meshgen.random_sources(V, 1, seed=3)`, edge form, default
options (automatic mu).  Without the loop constraints the optimised field
is locally integrable but circulates around the handles, so the integrated
distance depends on the integration paths; the reported difference between
the two answers (largest, relative to the diameter) is that error.

Run: python -m paper_1812_06060_amd.genus_bench [--shapes 2048x1024x0.4,4096x512x0.2]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def run(shapes, reps: int = 3, log=print):
    import torch

    import meshgen
    import paper_1812_06060_amd as hg
    torch.cuda.set_device(0)
    out = []
    for nu, nv, r in shapes:
        v, f = meshgen.torus(nu, nv, R=1.0, r=r, jitter=0.1, seed=7)
        src = meshgen.random_sources(v.shape[0], 1, seed=3)
        m = hg.Mesh(v, f)
        row = {"torus": f"{nu}x{nv}", "r": r, "vertices": int(v.shape[0]), "n_cycles": m.stats["n_cycles"],
               "loop_edges": m.stats["cycle_edges"]}
        res = {}
        for name, kw in (("loops", {}), ("no_loops", {"cycle_constraints": 0})):
            o = hg.default_opts(**kw)
            m.solve(src, 0.0, o)
            best = None
            for _ in range(reps):
                torch.cuda.synchronize()
                a = time.perf_counter()
                d, info = m.solve(src, 0.0, o)
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - a)
                best = ms if best is None else min(best, ms)
            res[name] = d.cpu().numpy()
            row[name] = {"ms": best, "admm_iters": info.admm_iters, "ms_admm": info.ms_admm,
                         "ms_diffusion": info.ms_diffusion, "bfs_depth": info.bfs_depth,
                         "cycle_slots": info.cycle_slots, "us_per_admm_iter": 1e3 * info.ms_admm / info.admm_iters}
        row["max_diff_no_loops_over_diam"] = float(np.abs(res["loops"] - res["no_loops"]).max() / res["loops"].max())
        log(f"[genus] torus {nu}x{nv} r={r} V={v.shape[0]}: loops {row['loops']['ms']:.1f} ms "
            f"({row['loops']['admm_iters']} ADMM iterations), without {row['no_loops']['ms']:.1f} ms "
            f"({row['no_loops']['admm_iters']}); without loops off by {row['max_diff_no_loops_over_diam']:.2e} of the diameter")
        m.close()
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shapes", default="2048x1024x0.4,4096x512x0.2")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    shapes = []
    for s in a.shapes.split(","):
        nu, nv, r = s.split("x")
        shapes.append((int(nu), int(nv), float(r)))
    for row in run(shapes, a.reps, log=lambda s: print(s, file=sys.stderr, flush=True)):
        print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
