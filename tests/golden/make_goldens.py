"""Writes the full-size golden samples used by the GPU parity tests.

Runs only the CPU oracle (oracle/) on the seeded synthetic meshes of
meshgen; stores, per workload and formulation, the oracle distance at a
seeded sample of vertices (uniform, plus the ones nearest to and farthest
from the sources) together with the diameter max d* over ALL vertices.

    python tests/golden/make_goldens.py sphere8 bumpy10 bumpy9_multi bumpy9_fields
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import meshgen  # noqa: E402
from oracle import pipeline  # noqa: E402


def sample(d, n_uniform=16384, n_end=256, seed=7):
    ok = np.flatnonzero(np.isfinite(d))
    rng = np.random.default_rng(seed)
    uni = rng.choice(ok, size=min(n_uniform, ok.size), replace=False)
    order = ok[np.argsort(d[ok], kind="stable")]
    idx = np.unique(np.concatenate([uni, order[:n_end], order[-n_end:]]))
    return idx.astype(np.int32)


def write(name, form, v, f, src, t0):
    r = pipeline.heat_method(v, f, src, form=form)
    idx = sample(r.d)
    out = os.path.join(HERE, f"{name}_{form}.npz")
    np.savez_compressed(out, idx=idx, d=r.d[idx], diam=np.max(r.d[np.isfinite(r.d)]),
                        sources=np.asarray(src, dtype=np.int32), t=r.t, nv=v.shape[0])
    print(f"{out}: nv={v.shape[0]} samples={idx.size} diam={r.d[np.isfinite(r.d)].max():.6f} "
          f"({time.time() - t0:.0f}s)", flush=True)


def main(names):
    for name in names:
        t0 = time.time()
        if name in ("sphere8", "bumpy10"):
            v, f, src = meshgen.config_mesh(name)
            for form in (("edge", "face") if name == "sphere8" else ("edge",)):
                write(name, form, v, f, src, t0)
        elif name == "bumpy9_multi":
            v, f, src = meshgen.config_mesh("bumpy9")
            write("bumpy9_multi", "edge", v, f, src, t0)
        elif name == "bumpy9_fields":
            v, f, src = meshgen.config_mesh("bumpy9")
            for i in range(4):
                write(f"bumpy9_field{i}", "edge", v, f, src[i:i + 1], t0)
        else:
            raise SystemExit(f"unknown workload {name}")


if __name__ == "__main__":
    main(sys.argv[1:])
