"""Parity of the HIP path with the CPU oracle, stage by stage and end to end.

Every GPU call goes through the C ABI (ctypes binding).  Tolerances:
  * integers (BFS levels, pairing, edge list): bit-exact;
  * log u (FP64 sweeps stopped at a relative change of 1e-12): 1e-8 absolute;
  * h (FP32 output of FP64 arithmetic): 2e-6;
  * ADMM after k iterations (FP32 vs FP64, same inputs): 2e-4 * hbar for edge
    differences, 2e-4 for face gradients (unit scale);
  * integration of given gradients (double-float sums): 1e-6 of the diameter;
  * the whole solve: mean |d - d*| <= 1e-4 and max <= 1e-3 of the diameter
    (the diameter read as max d*), d* the oracle's Poisson distance.
"""
import numpy as np
import pytest

import meshgen
from oracle import admm as oadmm
from oracle import gradient as ograd
from oracle import integrate as oint
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
    "grid64": lambda: meshgen.config_mesh("grid64"),
    "bumpy4": lambda: meshgen.config_mesh("bumpy4"),
    "sphere5": lambda: meshgen.config_mesh("sphere5"),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, hg):
    name = request.param
    v, f, src = CASES[name]()
    _say("mesh", name, "V", v.shape[0], "F", f.shape[0])
    ref_face = pipeline.heat_method(v, f, src, form="face")
    ref_edge = pipeline.heat_method(v, f, src, form="edge")
    mesh = hg.Mesh(v, f)
    yield name, v, f, src, mesh, ref_face, ref_edge
    mesh.close()


def test_mesh_stats_and_edges(case):
    name, v, f, src, mesh, rf, re_ = case
    _say(name, "edges")
    assert mesh.nv == v.shape[0] and mesh.nf == f.shape[0] and mesh.ne == rf.topo.ne
    assert abs(mesh.hbar - rf.hbar) <= 1e-14 * rf.hbar
    e = mesh.edges().cpu().numpy()
    assert np.array_equal(e, rf.topo.edges.astype(np.int32))


def test_mesh_weights(case):
    """theta_jk and A_j as the device computed them (Sec. 3.1) against the
    oracle's assembly: theta_jk = -K_jk of the cotangent stiffness matrix,
    A_j the lumped area."""
    name, v, f, src, mesh, rf, _ = case
    _say(name, "weights")
    th, ar = mesh.weights()
    th, ar = th.cpu().numpy(), ar.cpu().numpy()
    _, K, A, _ = pipeline.prepare(v, f)
    e = rf.topo.edges
    th_ref = -np.asarray(K[e[:, 0], e[:, 1]]).ravel()
    scale = np.abs(th_ref).max()
    assert np.abs(th - th_ref).max() <= 1e-12 * scale
    assert np.abs(ar - A).max() <= 1e-13 * A.max()


def test_bfs_bit_exact(case):
    name, v, f, src, mesh, rf, _ = case
    _say(name, "bfs")
    lev, par, depth = mesh.bfs(src)
    assert np.array_equal(lev.cpu().numpy(), rf.level.astype(np.int32))
    assert np.array_equal(par.cpu().numpy(), rf.parent.astype(np.int32))
    assert depth == rf.level.max()


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_diffusion_logu(case, hg, schedule):
    name, v, f, src, mesh, rf, _ = case
    _say(name, "diffuse schedule", schedule)
    o = hg.default_opts(tol_u=1e-12, diffusion_schedule=schedule)
    logu, info = mesh.diffuse(src, 0.0, o)
    assert info.converged_u and abs(info.t - rf.t) <= 1e-14 * rf.t
    lu = logu.cpu().numpy()
    assert np.abs(lu - rf.logu).max() < 1e-8


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_diffusion_beyond_fp64_range(hg, schedule):
    """t = 1e-4 hbar^2 on a displaced level-5 sphere: u reaches ~e^-800,
    far outside FP64; compared with the oracle's banded solve (pinned to an 80-bit Jacobi)."""
    from oracle import assembly, diffusion, mesh as omesh
    v, f, src = meshgen.config_mesh("bumpy5")
    _say("bumpy5 m=1e-4 diffuse schedule", schedule)
    topo = omesh.build_topology(f, v.shape[0])
    K = assembly.cotan_stiffness(v, f)
    A = assembly.lumped_areas(v, f)
    t = 1e-4 * assembly.mean_edge_length(v, topo.edges) ** 2
    ref = diffusion.solve_log(diffusion.heat_matrix(K, A, t), src)
    assert ref.min() < -760          # below the smallest FP64 subnormal, e^-744
    mesh = hg.Mesh(v, f)
    logu, info = mesh.diffuse(src, t, hg.default_opts(tol_u=1e-12, diffusion_schedule=schedule))
    lu = logu.cpu().numpy()
    assert info.converged_u and np.all(np.isfinite(lu))
    assert np.abs(lu - ref).max() < 1e-7 * np.abs(ref).max()
    mesh.close()


@pytest.mark.parametrize("rings", [1, 2, 4])
def test_overlapping_tiles_same_fixed_point_fewer_passes(hg, rings):
    """Schedule 3 (tiles that also sweep `rings` rings around themselves)
    reaches the oracle's log u on a displaced level-6 sphere, with more
    than one source, in fewer passes than the plain tiles.  At four rings
    some tiles' regions would exceed the LDS a workgroup may take: those
    tiles get fewer rings, with the same fixed point."""
    v, f = meshgen.icosphere(6)
    v = meshgen.harmonic_displacement(v, seed=3)
    src = meshgen.random_sources(v.shape[0], 3, seed=21)
    ref = pipeline.heat_method(v, f, src, form="edge")
    mesh = hg.Mesh(v, f)
    try:
        _say("bumpy6 overlap rings", rings)
        l2, i2 = mesh.diffuse(src, 0.0, hg.default_opts(tol_u=1e-12, diffusion_schedule=2, inner_sweeps=32))
        l3, i3 = mesh.diffuse(src, 0.0, hg.default_opts(tol_u=1e-12, diffusion_schedule=3, inner_sweeps=32,
                                                        overlap_rings=rings))
        _say("passes plain", i2.passes, "overlap", i3.passes, "mesh bytes", mesh.mesh_bytes())
        assert i3.converged_u
        assert np.abs(l3.cpu().numpy() - ref.logu).max() < 1e-8
        assert i3.passes < i2.passes
    finally:
        mesh.close()


def test_normalize(case):
    name, v, f, src, mesh, rf, _ = case
    _say(name, "normalize")
    h = mesh.normalize(torch.from_numpy(rf.logu).cuda()).cpu().numpy()
    assert np.abs(h - rf.h).max() < 2e-6


PARAMS = [(100.0, 1.0), (30.0, 1.8)]   # the paper's (mu, alpha) and the defaults


@pytest.mark.parametrize("mu, relax", PARAMS)
@pytest.mark.parametrize("k", [1, 7, 40])
def test_edge_admm_k_iterations(case, hg, k, mu, relax):
    name, v, f, src, mesh, rf, re_ = case
    _say(name, "admm_edge", k, mu, relax)
    h32 = re_.h.astype(np.float32)
    x, info = mesh.admm_edge(torch.from_numpy(h32).cuda(), iters=k, opts=hg.default_opts(mu=mu, relax=relax))
    Z = ograd.edge_targets(v, re_.topo, h32.astype(np.float64))
    ref = oadmm.EdgeADMM(re_.topo, Z, mu, relax).run(k)
    assert info.admm_iters == k
    assert np.abs(x.cpu().numpy() - ref.x).max() < 2e-4 * rf.hbar


@pytest.mark.parametrize("mu, relax", PARAMS)
@pytest.mark.parametrize("k", [1, 7, 40])
def test_face_admm_k_iterations(case, hg, k, mu, relax):
    name, v, f, src, mesh, rf, _ = case
    _say(name, "admm_face", k, mu, relax)
    h32 = rf.h.astype(np.float32)
    g, info = mesh.admm_face(torch.from_numpy(h32).cuda(), iters=k, opts=hg.default_opts(mu=mu, relax=relax))
    ref = oadmm.FaceADMM(v, f, rf.topo, h32.astype(np.float64), mu, relax).run(k)
    assert np.abs(g.cpu().numpy() - ref.g).max() < 2e-4


def test_integration(case):
    name, v, f, src, mesh, rf, re_ = case
    _say(name, "integrate")
    diam = rf.d[np.isfinite(rf.d)].max()
    # exact edge differences of the oracle distance, rounded to FP32
    x = (re_.d[re_.topo.edges[:, 1]] - re_.d[re_.topo.edges[:, 0]]).astype(np.float32)
    d = mesh.integrate_edge(src, torch.from_numpy(x).cuda()).cpu().numpy()
    ref = oint.integrate_edge(re_.topo, x.astype(np.float64), re_.level, re_.parent, src)
    assert np.abs(d - ref).max() < 1e-6 * diam
    g = ograd.face_gradients(v, f, rf.d).astype(np.float32)
    d = mesh.integrate_face(src, torch.from_numpy(g).cuda()).cpu().numpy()
    ref = oint.integrate_face(v, rf.topo, g.astype(np.float64), rf.level, rf.parent, src)
    assert np.abs(d - ref).max() < 1e-6 * diam


@pytest.mark.parametrize("mu, relax", PARAMS)
@pytest.mark.parametrize("form", ["edge", "face"])
def test_solve_end_to_end(case, hg, form, mu, relax):
    name, v, f, src, mesh, rf, re_ = case
    _say(name, "solve", form, mu, relax)
    ref = re_ if form == "edge" else rf
    d, info = mesh.solve(src, 0.0, hg.default_opts(formulation=form, mu=mu, relax=relax))
    mean, mx = metrics.parity(d.cpu().numpy(), ref.d)
    _say(name, form, "sweeps", info.sweeps, "admm", info.admm_iters, "mean", mean, "max", mx)
    assert info.converged_u and info.converged_admm
    assert mean <= 1e-4 and mx <= 1e-3
