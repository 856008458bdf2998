"""Batch benchmark: 256 independent small meshes (displaced icospheres of
levels 3-6, sizes drawn uniformly, seed 4; mesh i displaced with seed
1000 + i; one source each, seed 2000 + i), answered by one batched solve
(all meshes as components of one resident mesh: one launch per step for
all of them) against one solve per mesh.  Both are the same method; the
largest difference between the two answers is reported relative to each
mesh's diameter.

Run: python -m paper_1812_06060_amd.batch_bench [--meshes 256]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def make_meshes(n: int, levels=(3, 6), seed: int = 4):
    import meshgen
    rng = np.random.default_rng(seed)
    base = {}
    out = []
    for i in range(n):
        L = int(rng.integers(levels[0], levels[1] + 1))
        if L not in base:
            base[L] = meshgen.icosphere(L)
        v, f = base[L]
        out.append((meshgen.harmonic_displacement(v, seed=1000 + i), f))
    src = [meshgen.random_sources(v.shape[0], 1, seed=2000 + i) for i, (v, _) in enumerate(out)]
    return out, src


def run(n_meshes: int = 256, form: str = "edge", reps: int = 3, log=print):
    import torch

    import paper_1812_06060_amd as hg
    from paper_1812_06060_amd.batch import MeshBatch
    torch.cuda.set_device(0)
    meshes, src = make_meshes(n_meshes)
    nv = sum(v.shape[0] for v, _ in meshes)
    opts = hg.default_opts(formulation=form)
    b = MeshBatch(meshes)
    ds, info = b.solve(src, opts=hg.default_opts(formulation=form))
    torch.cuda.synchronize()
    tb = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ds, info = b.solve(src, opts=hg.default_opts(formulation=form))
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
    batched = [d.cpu().numpy() for d in ds]
    log(f"[batch] {n_meshes} meshes ({nv} vertices) in one solve: {1e3 * min(tb):.1f} ms "
        f"(passes {info.passes}, admm {info.admm_iters})")
    singles = [hg.Mesh(v, f) for v, f in meshes]
    for m, s in zip(singles, src):
        m.solve(s, 0.0, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = []
    for m, s in zip(singles, src):
        d, _ = m.solve(s, 0.0, opts)
        alone.append(d)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    worst = 0.0
    for a, bb in zip(alone, batched):
        a = a.cpu().numpy()
        worst = max(worst, float(np.abs(a - bb).max() / a.max()))
    log(f"[batch] one solve per mesh: {1e3 * ts:.1f} ms; largest batched-vs-alone difference {worst:.2e} of the diameter")
    for m in singles:
        m.close()
    b.close()
    return {"meshes": n_meshes, "vertices": nv, "form": form,
            "batched": {"ms": 1e3 * min(tb), "meshes_per_s": n_meshes / min(tb),
                        "passes": info.passes, "admm_iters": info.admm_iters},
            "one_per_mesh": {"ms": 1e3 * ts, "meshes_per_s": n_meshes / ts},
            "max_diff_vs_alone_over_diam": worst}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--meshes", type=int, default=256)
    ap.add_argument("--form", default="edge")
    a = ap.parse_args()
    print(json.dumps(run(a.meshes, a.form, log=lambda s: print(s, file=sys.stderr, flush=True))), flush=True)


if __name__ == "__main__":
    main()
