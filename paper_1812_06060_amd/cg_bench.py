"""The comparison of Sec. 6.4 on one MI355X: accuracy against time for the
original heat method with its linear systems solved by conjugate gradients
(diagonal preconditioner), next to this library's diffusion sweeps and ADMM
gradient solver.

Workload: displaced icospheres (harmonic displacement seed 3) of the given
levels, one source (seed 104), t = hbar^2.

* Diffusion: E_1 = |(A - t L_c) u - u_0|_2 (Eq. 29) after k CG iterations
  (hg_cg_diffuse) and after k passes of the LDS-tiled sweeps (hg_diffuse
  with a sweep cap), against wall time of the call.
* Distance: from one normalised field h (the converged diffusion's), the
  exact Poisson solution d* of the form (CG run to relative residual
  1e-13), then E_2 = |d - d*|_2 / n (Eq. 30) after k CG iterations
  (hg_cg_poisson) and after k ADMM iterations plus integration
  (hg_admm_face / hg_admm_edge, then hg_integrate_*), against wall time.

Prints one JSON object per level and a markdown table.

    python -m paper_1812_06060_amd.cg_bench --levels 8,9,10 --form face
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, 1e3 * (time.perf_counter() - t0)


def run_level(level: int, form: str, log=print):
    import torch

    import meshgen
    import paper_1812_06060_amd as hg
    v, f = meshgen.icosphere(level)
    v = meshgen.harmonic_displacement(v, seed=3)
    src = meshgen.random_sources(v.shape[0], 1, seed=104)
    mesh = hg.Mesh(v, f)
    n = mesh.nv
    out = {"level": level, "vertices": n, "form": form, "diffusion": {"cg": [], "sweeps": []},
           "distance": {"cg": [], "admm": []}}
    # warm up both paths once
    mesh.cg_diffuse(src, max_iters=4, tol=0.0)
    mesh.diffuse(src, opts=hg.default_opts(max_sweeps=64), raise_on_nonconvergence=False)

    # ---- diffusion: E_1 against time
    k = 16
    while True:
        (u, info), ms = _timed(lambda: mesh.cg_diffuse(src, max_iters=k, tol=0.0))
        e1 = mesh.heat_residual(src, u)
        out["diffusion"]["cg"].append({"iters": k, "ms": ms, "E1": e1})
        log(f"[cg L{level}] CG diffusion {k:6d} it: {ms:9.1f} ms  E1={e1:.3e}")
        if e1 < 1e-14 or k >= (1 << 15):
            break
        k *= 4
    inner = 32
    p = 1
    while True:
        opts = hg.default_opts(max_sweeps=p * inner, inner_sweeps=inner, diffusion_schedule=2, tol_u=0.0)
        (res, ms) = _timed(lambda: mesh.diffuse(src, opts=opts, raise_on_nonconvergence=False))
        logu, info = res
        e1 = mesh.heat_residual(src, logu, is_log=True)
        out["diffusion"]["sweeps"].append({"passes": info.passes, "sweeps": info.sweeps, "ms": ms, "E1": e1})
        log(f"[cg L{level}] tile sweeps {info.sweeps:6d}: {ms:9.1f} ms  E1={e1:.3e}")
        if e1 < 1e-14 or p >= 4096:
            break
        p *= 4

    # ---- distance: E_2 against time, from the converged diffusion's field
    logu, dinfo = mesh.diffuse(src, opts=hg.default_opts())
    h = mesh.normalize(logu)
    dstar, sinfo = mesh.cg_poisson(h.reshape(-1), src, form=form, max_iters=1 << 20, tol=1e-13)
    dstar_h = dstar.cpu().numpy()
    log(f"[cg L{level}] d*: CG to 1e-13 in {sinfo['iters']} iterations, {sinfo['ms']:.0f} ms")
    out["distance"]["dstar_cg_iters"] = sinfo["iters"]

    def e2(d):
        return float(np.linalg.norm(d.cpu().numpy().astype(np.float64) - dstar_h) / n)

    k = 8
    while True:
        (res, ms) = _timed(lambda: mesh.cg_poisson(h.reshape(-1), src, form=form, max_iters=k, tol=0.0))
        val = e2(res[0])
        out["distance"]["cg"].append({"iters": k, "ms": ms, "E2": val})
        log(f"[cg L{level}] CG Poisson {k:6d} it: {ms:9.1f} ms  E2={val:.3e}")
        if k >= sinfo["iters"] or k >= (1 << 16):
            break
        k *= 4
    _, depth = mesh.bfs(src)[1:]
    mu = max(30.0, 0.5 * depth)
    k = 8
    while True:
        opts = hg.default_opts(formulation=form, mu=mu)
        if form == "face":
            def step():
                g, _ = mesh.admm_face(h.reshape(-1), iters=k, opts=opts)
                return mesh.integrate_face(src, g.reshape(-1))
        else:
            def step():
                x, _ = mesh.admm_edge(h.reshape(-1), iters=k, opts=opts)
                return mesh.integrate_edge(src, x)
        d, ms = _timed(step)
        val = e2(d)
        out["distance"]["admm"].append({"iters": k, "ms": ms, "E2": val})
        log(f"[cg L{level}] ADMM {form} {k:6d} it: {ms:9.1f} ms  E2={val:.3e}")
        if k >= 16384 or val < 1e-7:
            break
        k *= 4
    out["distance"]["mu"] = mu
    mesh.close()
    return out


def table(results):
    rows = ["| level | solver | iterations | ms | error |", "|---|---|---|---|---|"]
    for r in results:
        for x in r["diffusion"]["cg"]:
            rows.append(f"| L{r['level']} | CG diffusion | {x['iters']} | {x['ms']:.1f} | E1 {x['E1']:.2e} |")
        for x in r["diffusion"]["sweeps"]:
            rows.append(f"| L{r['level']} | tile sweeps | {x['sweeps']} | {x['ms']:.1f} | E1 {x['E1']:.2e} |")
        for x in r["distance"]["cg"]:
            rows.append(f"| L{r['level']} | CG Poisson ({r['form']}) | {x['iters']} | {x['ms']:.1f} | "
                        f"E2 {x['E2']:.2e} |")
        for x in r["distance"]["admm"]:
            rows.append(f"| L{r['level']} | ADMM ({r['form']}) + integration | {x['iters']} | {x['ms']:.1f} | "
                        f"E2 {x['E2']:.2e} |")
    return "\n".join(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", default="8")
    ap.add_argument("--form", default="face", choices=["face", "edge"])
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    res = []
    for lvl in (int(x) for x in a.levels.split(",")):
        r = run_level(lvl, a.form, log=log)
        print(json.dumps(r), flush=True)
        res.append(r)
    print(table(res), flush=True)


if __name__ == "__main__":
    main()
