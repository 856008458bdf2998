"""Batch benchmark: 256 independent small meshes (displaced icospheres of
levels 3-6, sizes drawn uniformly, seed 4; mesh i displaced with seed
1000 + i; one source each, seed 2000 + i), answered by one batched solve
over the resident meshes (hg_geodesic_solve_batch: one launch per step for
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
    return meshgen.batch_meshes(n, levels, seed)


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
    singles = b.meshes   # the same resident meshes, one solve each
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
    b.close()
    return {"meshes": n_meshes, "vertices": nv, "form": form,
            "batched": {"ms": 1e3 * min(tb), "meshes_per_s": n_meshes / min(tb),
                        "passes": info.passes, "admm_iters": info.admm_iters},
            "one_per_mesh": {"ms": 1e3 * ts, "meshes_per_s": n_meshes / ts},
            "max_diff_vs_alone_over_diam": worst}


def run_fields(n_fields: int = 64, slots: int = 8, log=print, batched: bool = False):
    """64 single-source fields on the displaced level-9 icosphere (its 64
    seeded sources, one query each) on one resident mesh: served
    concurrently by an hg_server with `slots` slots (private workspaces,
    overlapping on the device) against one query at a time."""
    import torch

    import meshgen
    import paper_1812_06060_amd as hg
    torch.cuda.set_device(0)
    v, f, src = meshgen.config_mesh("bumpy9")
    src = src[:n_fields]
    mesh = hg.Mesh(v, f)
    opts = hg.default_opts()
    outs = [torch.empty(mesh.nv, dtype=torch.float32, device="cuda") for _ in src]
    mesh.solve(src[:1], 0.0, opts, out=outs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for o, s in zip(outs, src):
        mesh.solve(s, 0.0, opts, out=o)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    ref = [o.cpu().numpy() for o in outs]
    srv = hg.Server(slots)
    for o, s in zip(outs, src):           # warm the slots' workspaces
        srv.submit(mesh, [s], out=o, opts=opts)
    for _ in src:
        srv.wait(-1)
    t0 = time.perf_counter()
    for o, s in zip(outs, src):
        srv.submit(mesh, [s], out=o, opts=opts)
    for _ in src:
        srv.wait(-1)
    t_srv = time.perf_counter() - t0
    srv.close()
    same = all(np.array_equal(o.cpu().numpy(), r) for o, r in zip(outs, ref))
    log(f"[fields] {len(src)} single-source fields on L9: one at a time {t_seq:.2f} s, "
        f"{slots}-slot server {t_srv:.2f} s, identical {same}")
    out = {"fields": len(src), "vertices": int(v.shape[0]), "slots": slots,
           "one_at_a_time": {"s": t_seq, "fields_per_s": len(src) / t_seq},
           "served": {"s": t_srv, "fields_per_s": len(src) / t_srv}, "results_identical": same}
    if batched:
        # the same fields as one batched solve: one instance of the mesh per
        # field, placed side by side as the components of one resident mesh,
        # so that every step of the solve is one launch for all of them (the
        # mesh data is duplicated per field)
        from .batch import MeshBatch
        t0 = time.perf_counter()
        b = MeshBatch([mesh] * len(src))
        log(f"[fields] batch of {len(src)} instances of the resident mesh "
            f"({len(src) * mesh.mesh_bytes() / 1e9:.1f} GB joined)")
        srcs = [[int(x)] for x in src]
        ds, info = b.solve(srcs, opts=hg.default_opts())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ds, info = b.solve(srcs, opts=hg.default_opts())
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        worst = max(float(np.abs(d.cpu().numpy() - r).max() / r.max()) for d, r in zip(ds, ref))
        log(f"[fields] one batched solve: {t_b:.2f} s (passes {info.passes}, ADMM {info.admm_iters}; "
            f"bfs {info.ms_bfs:.0f} ms, diffusion {info.ms_diffusion:.0f} ms, ADMM {info.ms_admm:.0f} ms of which "
            f"kernel {info.ms_admm_kernel:.0f} ms in {info.admm_launches} launches); "
            f"largest difference from the fields alone {worst:.2e} of the diameter")
        out["batched"] = {"s": t_b, "fields_per_s": len(src) / t_b, "passes": info.passes,
                          "stage_ms": {"bfs": info.ms_bfs, "diffusion": info.ms_diffusion, "admm": info.ms_admm,
                                       "admm_kernel": info.ms_admm_kernel},
                          "admm_iters": info.admm_iters, "mesh_bytes": int(len(src) * mesh.mesh_bytes()),
                          "max_diff_vs_alone_over_diam": worst}
        b.close()
    mesh.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--meshes", type=int, default=256)
    ap.add_argument("--form", default="edge")
    ap.add_argument("--fields", action="store_true",
                    help="measure 64 single-source fields on the level-9 mesh instead")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--batched", action="store_true",
                    help="with --fields: also solve the 64 fields as one batch of 64 mesh instances")
    a = ap.parse_args()
    log = lambda s: print(s, file=sys.stderr, flush=True)
    if a.fields:
        print(json.dumps(run_fields(64, a.slots, log=log, batched=a.batched)), flush=True)
    else:
        print(json.dumps(run(a.meshes, a.form, log=log)), flush=True)


if __name__ == "__main__":
    main()
