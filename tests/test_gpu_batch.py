"""Many meshes in one solve (components of one resident mesh, per-component
diffusion time): every mesh's distance matches the oracle run on that mesh
alone, in both forms, including a mesh with several sources; the stats see
one component per mesh."""
import numpy as np
import pytest

import meshgen
from oracle import metrics, pipeline

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _meshes():
    out = []
    for i, lvl in enumerate([3, 4, 3, 5, 4, 3, 4, 5]):
        v, f = meshgen.icosphere(lvl)
        v = meshgen.harmonic_displacement(v, seed=1000 + i)
        out.append((v, f))
    out.append(meshgen.grid(30, 0.2, seed=8))
    return out


def _sources(meshes):
    src = [meshgen.random_sources(v.shape[0], 1, seed=2000 + i) for i, (v, f) in enumerate(meshes)]
    src[3] = meshgen.random_sources(meshes[3][0].shape[0], 4, seed=77)   # several sources in one mesh
    return src


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_06060_amd.batch import MeshBatch
    meshes = _meshes()
    b = MeshBatch(meshes)
    yield meshes, b
    b.close()


def test_batch_stats(batch):
    meshes, b = batch
    assert b.mesh.stats["n_components"] == len(meshes)
    assert b.mesh.nv == sum(v.shape[0] for v, _ in meshes)


@pytest.mark.parametrize("form", ["edge", "face"])
def test_each_mesh_matches_its_oracle(batch, form):
    import paper_1812_06060_amd as hg
    meshes, b = batch
    src = _sources(meshes)
    _say("batch", len(meshes), "meshes", form)
    ds, info = b.solve(src, opts=hg.default_opts(formulation=form))
    assert info.converged_u and info.converged_admm
    for i, ((v, f), s, d) in enumerate(zip(meshes, src, ds)):
        ref = pipeline.heat_method(v, f, s, form=form)
        mean, mx = metrics.parity(d.cpu().numpy(), ref.d)
        _say("mesh", i, "V", v.shape[0], "mean", mean, "max", mx)
        assert mean <= 1e-4 and mx <= 1e-3, i


def test_shared_t_differs_from_per_mesh_t(batch):
    """Without t_per_component the whole batch diffuses with one t (the
    mean edge length of all meshes), which is not each mesh's own problem:
    the distances of some mesh differ measurably."""
    import paper_1812_06060_amd as hg
    meshes, b = batch
    src = _sources(meshes)
    ds, _ = b.solve(src, opts=hg.default_opts())
    o = hg.default_opts()
    allsrc = np.concatenate([np.asarray(s) + b.starts[i] for i, s in enumerate(src)]).astype(np.int32)
    d2, _ = b.mesh.solve(allsrc, 0.0, o)
    d2 = d2.cpu().numpy()
    diff = max(np.abs(ds[i].cpu().numpy() - d2[b.starts[i]:b.starts[i + 1]]).max() for i in range(len(b)))
    assert diff > 1e-4
