"""Parity of whole solves at full workload sizes against stored oracle
distances (tests/golden/*.npz, written by tests/golden/make_goldens.py, which
runs only the CPU oracle).  The meshes are regenerated from their seeds.  A
file holds the oracle distance at every vertex (``full``) or at a seeded
sample (the vertices nearest to and farthest from the sources plus a uniform
draw of the rest); bumpy9_fields holds one such sample for each of the 64
single-source fields of the level-9 sources.  Bar, over the stored vertices:
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
# (batch256 holds the samples of the 256-mesh batch: tests/test_gpu_batch.py)
GOLDEN = sorted(p for p in glob.glob(os.path.join(HERE, "golden", "*.npz"))
                if not p.endswith(".partial.npz") and not os.path.basename(p).startswith("batch256"))
CASES = []
for _p in GOLDEN:
    _name = os.path.basename(_p)[:-4]
    if _name.startswith("bumpy9_fields"):
        CASES += [(_p, i) for i in range(int(np.load(_p)["sources"].size))]
    else:
        CASES.append((_p, None))
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


@pytest.mark.parametrize("path, field", CASES,
                         ids=[os.path.basename(p)[:-4] + ("" if i is None else f"[{i}]") for p, i in CASES])
def test_full_size_parity(hg, path, field):
    g = np.load(path)
    name = os.path.basename(path)[:-4]
    base, form = name.rsplit("_", 1)
    base = base.split("_")[0]
    if field is None:
        sources, diam, d_ref = g["sources"], float(g["diam"]), g["d"]
        idx = None if ("full" in g and bool(g["full"])) else g["idx"]
    else:
        sources, diam, d_ref, idx = g["sources"][field:field + 1], float(g["diam"][field]), g["d"][field], \
            g["idx"][field]
    print(f"[gpu-case] golden {name} field={field} nv={int(g['nv'])} sources={sources.size} "
          f"stored={d_ref.size}", flush=True)
    mesh = _mesh(hg, base)
    assert mesh.nv == int(g["nv"])
    t0 = time.perf_counter()
    d, info = mesh.solve(sources, 0.0, hg.default_opts(formulation=form))
    dt = time.perf_counter() - t0
    dg = d.cpu().numpy()
    ds = (dg if idx is None else dg[idx]).astype(np.float64)
    err = np.abs(ds - d_ref.astype(np.float64)) / diam
    print(f"[gpu-case] {name} field={field}: {dt * 1e3:.0f} ms sweeps={info.sweeps} passes={info.passes} "
          f"admm={info.admm_iters} paths={info.n_paths} mean={err.mean():.2e} max={err.max():.2e} "
          f"at {int(np.argmax(err)) if idx is None else int(idx[np.argmax(err)])}", flush=True)
    assert info.converged_u and info.converged_admm
    assert np.isfinite(ds).all()
    assert err.mean() <= 1e-4 and err.max() <= 1e-3


def test_batched_fields_match_their_goldens(hg):
    """Eight of the 64 single-source level-9 fields answered by one batched
    solve (hg_geodesic_solve_batch over eight instances of the resident mesh,
    each member stopping its ADMM on its own check): every member within the
    same bar of its stored oracle field."""
    from paper_1812_06060_amd.batch import MeshBatch
    path = os.path.join(HERE, "golden", "bumpy9_fields_edge.npz")
    g = np.load(path)
    pick = [0, 9, 18, 27, 36, 45, 54, 63]
    mesh = _mesh(hg, "bumpy9")
    print(f"[gpu-case] batched fields {pick}", flush=True)
    b = MeshBatch([mesh] * len(pick))
    try:
        ds, info = b.solve([[int(g["sources"][i])] for i in pick], opts=hg.default_opts())
        assert info.converged_u and info.converged_admm
        for k, i in enumerate(pick):
            d = ds[k].cpu().numpy()[g["idx"][i]].astype(np.float64)
            err = np.abs(d - g["d"][i].astype(np.float64)) / float(g["diam"][i])
            print(f"[gpu-case] batched field {i}: mean={err.mean():.2e} max={err.max():.2e}", flush=True)
            assert err.mean() <= 1e-4 and err.max() <= 1e-3, i
    finally:
        b.close()
