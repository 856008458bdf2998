"""Several sources (Sec. 5.2): parity of the HIP path with the oracle when the
path constraints of Eqs. 24-25 are in the ADMM.

  * ADMM after k iterations with the path constraints, both forms, against
    the oracle's constrained iteration (same tolerances as single-source);
  * the whole solve against the oracle's Poisson distance with d = 0 at every
    source (mean <= 1e-4, max <= 1e-3 of the diameter);
  * meshes: a displaced icosphere with 5 sources, a jittered grid with
    sources on its boundary (boundary path edges have one face), and two
    disjoint grids with sources in both plus a duplicate (one path tree per
    component, duplicates dropped).
"""
import numpy as np
import pytest

import meshgen
from oracle import admm as oadmm
from oracle import gradient as ograd
from oracle import metrics, pipeline

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def hg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06060_amd as hg
    hg.load_library()
    return hg


def _bumpy4_5src():
    v, f, _ = meshgen.config_mesh("bumpy4")
    return v, f, meshgen.random_sources(v.shape[0], 5, seed=7)


def _grid_boundary():
    v, f = meshgen.grid(40, 0.2, seed=9)
    n = 40
    return v, f, np.array([0, n - 1, n * n - 1, n * (n // 2) + n // 2], dtype=np.int32)


def _two_components():
    v, f, st = meshgen.disjoint_union([meshgen.grid(24, 0.2, seed=4), meshgen.grid(20, 0.2, seed=5)])
    return v, f, np.array([30, st[1] + 15, 400, 30, st[1] + 300], dtype=np.int32)


CASES = {"bumpy4_5src": _bumpy4_5src, "grid40_boundary": _grid_boundary, "two_components": _two_components}
N_PATHS = {"bumpy4_5src": 4, "grid40_boundary": 3, "two_components": 2}
PARAMS = [(100.0, 1.0), (30.0, 1.8)]


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, hg):
    name = request.param
    v, f, src = CASES[name]()
    _say("mesh", name, "V", v.shape[0], "F", f.shape[0], "sources", src.tolist())
    ref_face = pipeline.heat_method(v, f, src, form="face")
    ref_edge = pipeline.heat_method(v, f, src, form="edge")
    paths = oadmm.source_paths(v, f, ref_edge.topo, src)
    assert len(paths) == N_PATHS[name]
    mesh = hg.Mesh(v, f)
    yield name, v, f, src, mesh, ref_face, ref_edge, paths
    mesh.close()


@pytest.mark.parametrize("mu, relax", PARAMS)
@pytest.mark.parametrize("k", [1, 7, 40])
def test_edge_admm_with_paths_k_iterations(case, hg, k, mu, relax):
    name, v, f, src, mesh, rf, re_, paths = case
    _say(name, "admm_edge paths", k, mu, relax)
    h32 = re_.h.astype(np.float32)
    x, info = mesh.admm_edge(torch.from_numpy(h32).cuda(), iters=k, opts=hg.default_opts(mu=mu, relax=relax),
                             sources=src)
    Z = ograd.edge_targets(v, re_.topo, h32.astype(np.float64))
    ref = oadmm.EdgeADMM(re_.topo, Z, mu, relax, paths=paths).run(k)
    assert info.n_paths == len(paths) and info.path_edges == sum(p["edge"].size for p in paths)
    assert np.abs(x.cpu().numpy() - ref.x).max() < 2e-4 * rf.hbar


@pytest.mark.parametrize("mu, relax", PARAMS)
@pytest.mark.parametrize("k", [1, 7, 40])
def test_face_admm_with_paths_k_iterations(case, hg, k, mu, relax):
    name, v, f, src, mesh, rf, re_, paths = case
    _say(name, "admm_face paths", k, mu, relax)
    h32 = rf.h.astype(np.float32)
    g, info = mesh.admm_face(torch.from_numpy(h32).cuda(), iters=k, opts=hg.default_opts(mu=mu, relax=relax),
                             sources=src)
    ref = oadmm.FaceADMM(v, f, rf.topo, h32.astype(np.float64), mu, relax, paths=paths).run(k)
    assert info.n_paths == len(paths)
    assert np.abs(g.cpu().numpy() - ref.g).max() < 2e-4


@pytest.mark.parametrize("form", ["edge", "face"])
def test_solve_several_sources_end_to_end(case, hg, form):
    name, v, f, src, mesh, rf, re_, paths = case
    _say(name, "solve paths", form)
    ref = re_ if form == "edge" else rf
    d, info = mesh.solve(src, 0.0, hg.default_opts(formulation=form))
    d = d.cpu().numpy()
    mean, mx = metrics.parity(d, ref.d)
    _say(name, form, "admm", info.admm_iters, "paths", info.n_paths, info.path_edges, "mean", mean, "max", mx)
    assert info.converged_u and info.converged_admm and info.n_paths == len(paths)
    assert np.all(d[np.unique(src)] == 0.0)
    assert mean <= 1e-4 and mx <= 1e-3


def test_source_paths_off_reports_none(case, hg):
    name, v, f, src, mesh, rf, re_, paths = case
    _say(name, "solve without paths")
    d, info = mesh.solve(src, 0.0, hg.default_opts(source_paths=0))
    assert info.n_paths == 0 and info.path_edges == 0
    assert np.all(np.isfinite(d.cpu().numpy()))


def test_seam_reported_and_required(hg):
    """The distance check's seam (largest |d_head - d_tail - x_e| / hbar,
    zero on the integration tree's edges) is reported; with tol_seam the
    ADMM runs on until it is met.  A loose distance tolerance leaves a
    visible seam on a level-7 sphere."""
    v, f = meshgen.icosphere(7)
    v = meshgen.harmonic_displacement(v, seed=3)
    src = meshgen.random_sources(v.shape[0], 1, seed=104)
    mesh = hg.Mesh(v, f)
    try:
        d0, i0 = mesh.solve(src, 0.0, hg.default_opts(tol_admm=1e-3))
        d1, i1 = mesh.solve(src, 0.0, hg.default_opts(tol_admm=1e-3, tol_seam=0.5 * i0.seam))
    finally:
        mesh.close()
    _say("seam loose", i0.seam, i0.admm_iters, "required", i1.seam, i1.admm_iters)
    assert i0.seam > 0.0 and i1.converged_admm
    assert i1.seam <= 0.5 * i0.seam and i1.admm_iters > i0.admm_iters
