"""Writes the full-size oracle distances used by the GPU parity tests.

Runs only the CPU oracle (oracle/) on the seeded synthetic meshes of
meshgen.  Per workload and formulation it stores, in float32, the oracle
distance d* at every vertex (``full``) or at a seeded sample of vertices
(the ones nearest to and farthest from the sources plus a uniform draw from
the rest), with the diameter max d* over ALL vertices in float64.

Where both exact diffusion routes of the oracle fit in memory (up to level
9), the diffusion is solved both ways -- whole-mesh LU of the gauge-scaled
system and the banded LU -- and the file is written only if the two agree,
max |delta log u| <= 1e-9 max |log u|; the discrepancy is stored with it
(``pin_dlogu``).

    python tests/golden/make_goldens.py sphere8 bumpy9_multi bumpy10 bumpy9_fields [--jobs 4]

Workloads:
  sphere8       level-8 jittered sphere, 1 source, edge and face form, full field
  bumpy9_multi  level-9 displaced sphere, one field of its 64 sources, full field
  bumpy10       level-10 displaced sphere, 1 source, 1,048,576 uniform + 512 extreme vertices
  bumpy9_fields the 64 single-source fields of the level-9 sources, 16,384 uniform +
                512 extreme vertices each
  batch256      the 256 small displaced spheres (levels 3-6) of the batch workload, one
                source each, 256 uniform + 128 extreme vertices each
  pin9          the two diffusion routes on the first single-source level-9 field
                (recorded in diffusion_pin_bumpy9_field0.json)
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import meshgen  # noqa: E402
from oracle import diffusion, pipeline  # noqa: E402


def sample(d, n_uniform, n_end=256, seed=7):
    """Indices of the n_end nearest and n_end farthest finite vertices plus a
    seeded uniform draw of n_uniform from the others (sorted, int32)."""
    ok = np.flatnonzero(np.isfinite(d))
    order = ok[np.argsort(d[ok], kind="stable")]
    ends = np.concatenate([order[:n_end], order[-n_end:]])
    rest = np.setdiff1d(ok, ends)
    rng = np.random.default_rng(seed)
    uni = rng.choice(rest, size=min(n_uniform, rest.size), replace=False)
    return np.sort(np.concatenate([uni, ends])).astype(np.int32)


def two_route_pin(v, f, src):
    """max |delta log u| between the gauge-scaled whole-mesh LU and the
    banded LU, and max |log u| (banded)."""
    topo, K, A, hbar = pipeline.prepare(np.asarray(v, np.float64), np.asarray(f, np.int64))
    t = hbar * hbar
    M = diffusion.heat_matrix(K, A, t)
    s = np.unique(np.asarray(src, np.int64))
    lb = diffusion.solve_log(M, s, band_rings=40, margin_rings=40) if v.shape[0] > pipeline.MG_MIN_V \
        else diffusion.solve_log(M, s)
    lg = diffusion.solve_log_gauge(M, s, diffusion.gauge_potential(M, v, topo.edges, t, s))
    dl = float(np.abs(lg - lb).max())
    mx = float(np.abs(lb[np.isfinite(lb)]).max())
    if not dl <= 1e-9 * mx:
        raise SystemExit(f"diffusion routes disagree: max |delta log u| = {dl:.3e} (max |log u| {mx:.1f})")
    return dl, mx


def solve(v, f, src, form, route="auto"):
    r = pipeline.heat_method(v, f, src, form=form, diffusion_route=route)
    fin = np.isfinite(r.d)
    return r, float(np.max(r.d[fin]))


def _save(path, payload):
    tmp = path[:-4] + ".partial.npz"
    np.savez_compressed(tmp, **payload)
    os.replace(tmp, path)


def write(name, form, v, f, src, r, diam, idx=None, **extra):
    out = os.path.join(HERE, f"{name}_{form}.npz")
    d = r.d if idx is None else r.d[idx]
    payload = dict(d=d.astype(np.float32), diam=diam, sources=np.asarray(src, dtype=np.int32), t=r.t,
                   nv=v.shape[0], full=idx is None, poisson_iters=r.poisson_iters,
                   poisson_residual=r.poisson_residual, diffusion_route=r.diffusion_route, **extra)
    if idx is not None:
        payload["idx"] = idx
    _save(out, payload)
    print(f"{out}: nv={v.shape[0]} stored={d.size} diam={diam:.6f} route={r.diffusion_route} "
          f"poisson_iters={r.poisson_iters}", flush=True)


def _field(args):
    i, s = args
    v, f, _ = meshgen.config_mesh("bumpy9")
    t0 = time.time()
    r, diam = solve(v, f, [s], "edge", route="bands")
    idx = sample(r.d, 16384, seed=1000 + i)
    print(f"  field {i} (source {s}): diam={diam:.6f} {time.time() - t0:.0f}s", flush=True)
    return i, idx, r.d[idx].astype(np.float32), diam, r.t


def main(names, jobs):
    for name in names:
        t0 = time.time()
        if name == "sphere8":
            v, f, src = meshgen.config_mesh(name)
            dl, mx = two_route_pin(v, f, src)
            for form in ("edge", "face"):
                r, diam = solve(v, f, src, form, route="bands")
                write(name, form, v, f, src, r, diam, pin_dlogu=dl, pin_max_logu=mx)
        elif name == "bumpy9_multi":
            v, f, src = meshgen.config_mesh("bumpy9")
            dl, mx = two_route_pin(v, f, src)
            r, diam = solve(v, f, src, "edge", route="bands")
            write(name, "edge", v, f, src, r, diam, pin_dlogu=dl, pin_max_logu=mx)
        elif name == "bumpy10":
            v, f, src = meshgen.config_mesh(name)
            r, diam = solve(v, f, src, "edge")
            write(name, "edge", v, f, src, r, diam, idx=sample(r.d, 1 << 20))
        elif name == "bumpy9_fields":
            v, f, src = meshgen.config_mesh("bumpy9")
            del v, f
            with mp.get_context("spawn").Pool(jobs) as pool:
                res = sorted(pool.map(_field, list(enumerate(src.tolist())), chunksize=1))
            n = max(r[1].size for r in res)
            assert all(r[1].size == n for r in res)
            out = os.path.join(HERE, "bumpy9_fields_edge.npz")
            _save(out, dict(idx=np.stack([r[1] for r in res]), d=np.stack([r[2] for r in res]),
                            diam=np.array([r[3] for r in res]), sources=np.asarray(src, dtype=np.int32),
                            t=res[0][4], nv=2621442, full=False))
            print(f"{out}: 64 fields x {n} vertices", flush=True)
        elif name == "pin9":
            # the two exact diffusion routes on a single-source level-9 field
            # (log u down to about -1,300), recorded on its own
            import json
            v, f, src = meshgen.config_mesh("bumpy9")
            dl, mx = two_route_pin(v, f, src[:1])
            out = os.path.join(HERE, "diffusion_pin_bumpy9_field0.json")
            with open(out, "w") as fh:
                json.dump({"workload": "bumpy9, single source (the first of its 64)", "source": int(src[0]),
                           "max_abs_dlogu": dl, "max_abs_logu": mx, "bar": "1e-9 * max |log u|"}, fh, indent=1)
            print(f"{out}: max |dlog u| = {dl:.3e}, max |log u| = {mx:.1f}", flush=True)
        elif name == "batch256":
            meshes, srcs = meshgen.batch_meshes(256)
            idxs, ds, diams = [], [], []
            for i, ((v, f), s) in enumerate(zip(meshes, srcs)):
                r, diam = solve(v, f, s, "edge")
                idx = sample(r.d, 256, n_end=64, seed=3000 + i)
                idxs.append(idx)
                ds.append(r.d[idx].astype(np.float32))
                diams.append(diam)
            ptr = np.concatenate([[0], np.cumsum([x.size for x in idxs])]).astype(np.int64)
            out = os.path.join(HERE, "batch256_edge.npz")
            _save(out, dict(idx=np.concatenate(idxs), d=np.concatenate(ds), ptr=ptr, diam=np.array(diams),
                            nv=np.array([v.shape[0] for v, _ in meshes])))
            print(f"{out}: 256 meshes, {ptr[-1]} stored vertices", flush=True)
        else:
            raise SystemExit(f"unknown workload {name}")
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    jobs = 4
    if "--jobs" in args:
        k = args.index("--jobs")
        jobs = int(args[k + 1])
        del args[k:k + 2]
    main(args or ["sphere8", "bumpy9_multi", "bumpy10", "bumpy9_fields"], jobs)
