"""Closed surfaces of genus g > 0 (Sec. 5.1, Eqs. 22-23): parity of the HIP
path with the oracle when the cycle constraints are in the ADMM.

  * the generator loops the library builds with the mesh equal the oracle's
    tree-cotree basis: edge ids, signs and face ids bit for bit, polyline
    segments to FP32 rounding;
  * ADMM after k iterations with the loops, both forms, against the oracle's
    constrained iteration (same tolerances as the other k-iteration tests);
  * the whole solve against the oracle's Poisson distance (mean <= 1e-4,
    max <= 1e-3 of the diameter), one source and several sources (source
    paths and loops together), and a sphere and a torus side by side;
  * without the loops the converged field misses that distance by more than
    1e-4 of the diameter (the loops are what makes it a gradient).
Meshes: jittered tori (48 x 24 and 64 x 20 vertices), two tori side by side
(four loops), a sphere next to a torus (loops on one component only).
"""
import numpy as np
import pytest

import meshgen
from oracle import admm as oadmm
from oracle import gradient as ograd
from oracle import mesh as omesh
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


CASES = {
    "torus48x24": lambda: meshgen.torus(),
    "torus64x20": lambda: meshgen.torus(64, 20, R=1.0, r=0.3, jitter=0.15, seed=11),
    "two_tori": lambda: meshgen.disjoint_union([meshgen.torus(24, 12, seed=1), meshgen.torus(20, 10, seed=2)])[:2],
    "sphere_torus": lambda: meshgen.disjoint_union([meshgen.icosphere(2), meshgen.torus(30, 14, seed=5)])[:2],
}
N_CYCLES = {"torus48x24": 2, "torus64x20": 2, "two_tori": 4, "sphere_torus": 2}


@pytest.mark.parametrize("name", sorted(CASES))
def test_loops_match_oracle_basis(hg, name):
    v, f = CASES[name]()
    _say("loops", name, "V", v.shape[0])
    topo = omesh.build_topology(f, v.shape[0])
    ec, fc = oadmm.cycle_constraints(v, f, topo)
    m = hg.Mesh(v, f)
    try:
        assert m.stats["n_cycles"] == len(ec) == N_CYCLES[name]
        assert m.stats["cycle_edges"] == sum(c["edge"].size for c in ec)
        assert m.stats["cycle_faces"] == sum(c["face"].size for c in fc)
        for (ids, sg), ref in zip(m.cycles("edge"), ec):
            assert np.array_equal(ids, ref["edge"]) and np.array_equal(sg, ref["sign"].astype(np.float32))
        for (ids, vec), ref in zip(m.cycles("face"), fc):
            assert np.array_equal(ids, ref["face"])
            assert np.abs(vec - ref["vec"]).max() <= 1e-6 * np.abs(ref["vec"]).max()
    finally:
        m.close()


@pytest.fixture(scope="module")
def torus(hg):
    v, f = CASES["torus48x24"]()
    src = [5]
    ref_face = pipeline.heat_method(v, f, src, form="face")
    ref_edge = pipeline.heat_method(v, f, src, form="edge")
    ec, fc = oadmm.cycle_constraints(v, f, ref_edge.topo)
    mesh = hg.Mesh(v, f)
    yield v, f, src, mesh, ref_face, ref_edge, ec, fc
    mesh.close()


PARAMS = [(100.0, 1.0), (30.0, 1.8)]


@pytest.mark.parametrize("mu, relax", PARAMS)
@pytest.mark.parametrize("k", [1, 7, 40])
def test_edge_admm_with_loops_k_iterations(torus, hg, k, mu, relax):
    v, f, src, mesh, rf, re_, ec, fc = torus
    _say("torus admm_edge loops", k, mu, relax)
    h32 = re_.h.astype(np.float32)
    x, info = mesh.admm_edge(torch.from_numpy(h32).cuda(), iters=k, opts=hg.default_opts(mu=mu, relax=relax))
    Z = ograd.edge_targets(v, re_.topo, h32.astype(np.float64))
    ref = oadmm.EdgeADMM(re_.topo, Z, mu, relax, paths=ec).run(k)
    assert info.n_paths == 0 and info.n_cycles == 2 and info.cycle_slots == sum(c["edge"].size for c in ec)
    assert np.abs(x.cpu().numpy() - ref.x).max() < 2e-4 * rf.hbar


@pytest.mark.parametrize("mu, relax", PARAMS)
@pytest.mark.parametrize("k", [1, 7, 40])
def test_face_admm_with_loops_k_iterations(torus, hg, k, mu, relax):
    v, f, src, mesh, rf, re_, ec, fc = torus
    _say("torus admm_face loops", k, mu, relax)
    h32 = rf.h.astype(np.float32)
    g, info = mesh.admm_face(torch.from_numpy(h32).cuda(), iters=k, opts=hg.default_opts(mu=mu, relax=relax))
    ref = oadmm.FaceADMM(v, f, rf.topo, h32.astype(np.float64), mu, relax, paths=fc).run(k)
    assert info.n_cycles == 2 and info.cycle_slots == sum(c["face"].size for c in fc)
    assert np.abs(g.cpu().numpy() - ref.g).max() < 2e-4


def test_admm_loops_off_is_plain_iteration(torus, hg):
    v, f, src, mesh, rf, re_, ec, fc = torus
    h32 = re_.h.astype(np.float32)
    x, info = mesh.admm_edge(torch.from_numpy(h32).cuda(), iters=7,
                             opts=hg.default_opts(mu=100.0, relax=1.0, cycle_constraints=0))
    Z = ograd.edge_targets(v, re_.topo, h32.astype(np.float64))
    ref = oadmm.EdgeADMM(re_.topo, Z, 100.0, 1.0).run(7)
    assert info.n_cycles == 0
    assert np.abs(x.cpu().numpy() - ref.x).max() < 2e-4 * rf.hbar


@pytest.mark.parametrize("form", ["edge", "face"])
def test_solve_torus_end_to_end(torus, hg, form):
    v, f, src, mesh, rf, re_, ec, fc = torus
    ref = re_ if form == "edge" else rf
    d, info = mesh.solve(src, 0.0, hg.default_opts(formulation=form))
    mean, mx = metrics.parity(d.cpu().numpy(), ref.d)
    _say("torus solve", form, "admm", info.admm_iters, "cycles", info.n_cycles, "mean", mean, "max", mx)
    assert info.converged_u and info.converged_admm and info.n_cycles == 2
    assert mean <= 1e-4 and mx <= 1e-3


@pytest.mark.parametrize("form", ["edge", "face"])
def test_solve_torus_without_loops_misses(torus, hg, form):
    v, f, src, mesh, rf, re_, ec, fc = torus
    ref = re_ if form == "edge" else rf
    d, info = mesh.solve(src, 0.0, hg.default_opts(formulation=form, cycle_constraints=0))
    mean, mx = metrics.parity(d.cpu().numpy(), ref.d)
    _say("torus solve without loops", form, "admm", info.admm_iters, "mean", mean, "max", mx)
    assert info.n_cycles == 0
    assert mean > 1e-4


@pytest.mark.parametrize("name, src", [("torus64x20", [3, 400, 901, 1200]), ("two_tori", [0, 100, 300, 450]),
                                       ("sphere_torus", [7, 200, 400])])
@pytest.mark.parametrize("form", ["edge", "face"])
def test_solve_loops_and_sources_end_to_end(hg, name, src, form):
    v, f = CASES[name]()
    _say("solve", name, form, "sources", src)
    ref = pipeline.heat_method(v, f, src, form=form)
    m = hg.Mesh(v, f)
    try:
        d, info = m.solve(np.array(src, dtype=np.int32), 0.0, hg.default_opts(formulation=form))
    finally:
        m.close()
    d = d.cpu().numpy()
    mean, mx = metrics.parity(d, ref.d)
    _say(name, form, "admm", info.admm_iters, "paths", info.n_paths, "cycles", info.n_cycles, "mean", mean, "max", mx)
    assert info.converged_u and info.converged_admm and info.n_cycles == N_CYCLES[name]
    assert np.all(d[np.unique(src)] == 0.0)
    assert mean <= 1e-4 and mx <= 1e-3


def test_batch_with_a_torus(hg):
    """A torus among spheres in one batched solve: each mesh matches its own
    oracle (the loops stay on the torus's component)."""
    from paper_1812_06060_amd.batch import MeshBatch
    meshes = [meshgen.icosphere(3), meshgen.torus(40, 16, seed=3), meshgen.icosphere(2)]
    meshes[0] = (meshgen.harmonic_displacement(meshes[0][0], seed=21), meshes[0][1])
    src = [[4], [17], [0]]
    b = MeshBatch(meshes)
    try:
        assert [m.stats["n_cycles"] for m in b.meshes] == [0, 2, 0]
        ds, info = b.solve(src, opts=hg.default_opts())
        assert info.converged_u and info.converged_admm and info.n_cycles == 2
        for i, ((v, f), s, d) in enumerate(zip(meshes, src, ds)):
            ref = pipeline.heat_method(v, f, s, form="edge")
            mean, mx = metrics.parity(d.cpu().numpy(), ref.d)
            _say("batch mesh", i, "mean", mean, "max", mx)
            assert mean <= 1e-4 and mx <= 1e-3, i
    finally:
        b.close()
