"""Parity of whole solves at full workload sizes against stored oracle
samples (tests/golden/*.npz, written by tests/golden/make_goldens.py, which
runs only the CPU oracle).  The meshes are regenerated from their seeds; the
GPU distance is compared at the stored vertices (a seeded uniform sample plus
the vertices nearest to and farthest from the sources):
mean |d - d*| <= 1e-4 and max <= 1e-3 of the diameter max d* (over all
vertices)."""
import glob
import os
import time

import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = sorted(glob.glob(os.path.join(HERE, "golden", "*.npz")))
_meshes = {}


def _mesh(hg, base):
    if base not in _meshes:
        _meshes.clear()
        v, f, _ = meshgen.config_mesh(base)
        _meshes[base] = hg.Mesh(v, f)
    return _meshes[base]


@pytest.fixture(scope="module")
def hg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06060_amd as hg
    hg.load_library()
    yield hg
    for m in _meshes.values():
        m.close()
    _meshes.clear()


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[:-4] for p in GOLDEN])
def test_full_size_parity(hg, path):
    g = np.load(path)
    name = os.path.basename(path)[:-4]
    base, form = name.rsplit("_", 1)
    base = base.split("_")[0]
    print(f"[gpu-case] golden {name} nv={int(g['nv'])} sources={g['sources'].size}", flush=True)
    mesh = _mesh(hg, base)
    assert mesh.nv == int(g["nv"])
    t0 = time.perf_counter()
    d, info = mesh.solve(g["sources"], 0.0, hg.default_opts(formulation=form))
    dt = time.perf_counter() - t0
    ds = d.cpu().numpy()[g["idx"]].astype(np.float64)
    err = np.abs(ds - g["d"]) / float(g["diam"])
    print(f"[gpu-case] {name}: {dt * 1e3:.0f} ms sweeps={info.sweeps} passes={info.passes} "
          f"admm={info.admm_iters} paths={info.n_paths} mean={err.mean():.2e} max={err.max():.2e}", flush=True)
    assert info.converged_u and info.converged_admm
    assert err.mean() <= 1e-4 and err.max() <= 1e-3
