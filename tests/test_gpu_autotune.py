"""hg_mesh_autotune times the diffusion schedules and the edge form's ADMM
blocks on a probe query, stores the fastest in the mesh, and later solves
with automatic options use them and still match the oracle."""
import numpy as np
import pytest

import meshgen
from oracle import metrics, pipeline

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name", ["bumpy4", "bumpy6"])
def test_autotune_then_solve(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06060_amd as hg
    v, f, src = meshgen.config_mesh(name)
    print("[gpu-case] autotune", name, flush=True)
    mesh = hg.Mesh(v, f)
    try:
        rep = mesh.autotune(src)
        print("[gpu-case]", rep, flush=True)
        c = rep["candidates"]
        assert 0 <= rep["chosen"] < len(c)
        best = c[rep["chosen"]]["ms"]
        assert all(best <= x["ms"] + 1e-6 for x in c if x["passes"] > 0)
        if mesh.stats["n_patches"] > 16:   # global Jacobi only on meshes of a few tiles
            assert all(x["schedule"] in (2, 3) for x in c)
        assert {x["schedule"] for x in c} >= {2, 3}
        # the ADMM block: the fastest timed one, used by later solves
        a = rep["admm"]
        assert a and 0 <= rep["admm_chosen"] < len(a)
        assert all(a[rep["admm_chosen"]]["us_per_iteration"] <= x["us_per_iteration"] + 1e-6 for x in a)
        d, info = mesh.solve(src, 0.0, hg.default_opts())
        assert info.admm_block == a[rep["admm_chosen"]]["block"]
        if c[rep["chosen"]]["schedule"] in (2, 3):
            assert info.sweeps == info.passes * c[rep["chosen"]]["inner_sweeps"]
        ref = pipeline.heat_method(v, f, src, form="edge")
        mean, mx = metrics.parity(d.cpu().numpy(), ref.d)
        assert mean <= 1e-4 and mx <= 1e-3
    finally:
        mesh.close()
