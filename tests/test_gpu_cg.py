"""The Sec. 6.4 comparator on the GPU: conjugate gradients with a diagonal
preconditioner on the heat system (Eq. 4) and on both Poisson systems with
d = 0 at the sources, through the C ABI.

Bars: converged CG Poisson equals the oracle's sparse-LU Poisson solve of
the same (FP32-rounded) field h to 1e-9 of the diameter, and the oracle's
heat-method distance (FP64 h) to 1e-6 of the diameter; converged CG
diffusion equals the oracle's u to 1e-10 of max u where u stays in the FP64
range; E_1 (Eq. 29) from the library equals the residual formed on the CPU
from the oracle's matrix."""
import numpy as np
import pytest

import meshgen
from oracle import diffusion, pipeline, poisson

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


def _case(name):
    if name == "bumpy5":
        v, f = meshgen.icosphere(5)
        v = meshgen.harmonic_displacement(v, seed=3)
        return v, f, meshgen.random_sources(v.shape[0], 1, seed=5)
    if name == "bumpy4_multi":
        v, f = meshgen.icosphere(4)
        v = meshgen.harmonic_displacement(v, seed=9)
        return v, f, meshgen.random_sources(v.shape[0], 5, seed=6)
    if name == "grid40":
        v, f = meshgen.grid(40, 0.2, seed=4)
        return v, f, np.array([meshgen.grid_center_source(v)], dtype=np.int32)
    raise KeyError(name)


@pytest.mark.parametrize("form", ["face", "edge"])
@pytest.mark.parametrize("name", ["bumpy5", "bumpy4_multi", "grid40"])
def test_cg_poisson_equals_oracle_poisson(hg, name, form):
    v, f, src = _case(name)
    ref = pipeline.heat_method(v, f, src, form=form)
    h32 = ref.h.astype(np.float32)
    h64 = h32.astype(np.float64)
    d_same_h = (poisson.poisson_face(v, f, h64, src) if form == "face"
                else poisson.poisson_edge(v, f, ref.topo, h64, src))
    mesh = hg.Mesh(v, f)
    try:
        _say("cg poisson", name, form)
        d, info = mesh.cg_poisson(torch.from_numpy(h32.reshape(-1)).cuda(), src, form=form, tol=1e-13)
        d = d.cpu().numpy()
    finally:
        mesh.close()
    diam = ref.d.max()
    e_same = np.abs(d - d_same_h).max() / diam
    e_ref = np.abs(d - ref.d).max() / diam
    _say(name, form, "iters", info["iters"], "vs LU(same h)", e_same, "vs oracle", e_ref)
    assert info["converged"] and info["res_rel"] <= 1e-13
    assert np.all(d[np.asarray(src)] == 0.0)
    assert e_same <= 1e-9
    assert e_ref <= 1e-6


def test_cg_diffusion_equals_oracle_and_e1(hg):
    v, f = meshgen.icosphere(4)
    v = meshgen.harmonic_displacement(v, seed=3)
    src = meshgen.random_sources(v.shape[0], 2, seed=8)
    ref = pipeline.heat_method(v, f, src, form="edge")
    u_ref = np.exp(ref.logu)
    mesh = hg.Mesh(v, f)
    try:
        _say("cg diffusion level 4")
        u, info = mesh.cg_diffuse(src, tol=1e-14)
        e1 = mesh.heat_residual(src, u)
        ug = u.cpu().numpy()
        # E_1 of the oracle's own u, formed on the device from log u
        e1_ref_dev = mesh.heat_residual(src, torch.from_numpy(ref.logu).cuda(), is_log=True)
        # an unconverged iterate, whose residual is far above rounding
        u8, _ = mesh.cg_diffuse(src, max_iters=8, tol=0.0)
        e1_8 = mesh.heat_residual(src, u8)
        u8 = u8.cpu().numpy()
    finally:
        mesh.close()
    _say("cg diffusion iters", info["iters"], "E1", e1, "E1(oracle u)", e1_ref_dev, "E1 after 8", e1_8)
    assert info["converged"]
    assert np.abs(ug - u_ref).max() <= 1e-10 * u_ref.max()
    assert e1 <= 1e-13 and e1_ref_dev <= 1e-13
    # E_1 formed on the CPU from the oracle's matrix
    topo, K, A, hbar = pipeline.prepare(v, f)
    M = diffusion.heat_matrix(K, A, hbar * hbar)
    u0 = np.zeros(v.shape[0])
    u0[src] = 1.0
    e1_cpu = np.linalg.norm(M @ u8 - u0)
    assert e1_cpu > 1e-8
    assert abs(e1_8 - e1_cpu) <= 1e-9 * e1_cpu


def test_cg_fixed_iteration_counts_and_residual_decrease(hg):
    v, f, src = _case("bumpy5")
    ref = pipeline.heat_method(v, f, src, form="face")
    h32 = torch.from_numpy(ref.h.astype(np.float32).reshape(-1)).cuda()
    mesh = hg.Mesh(v, f)
    try:
        res = []
        for k in (5, 20, 80):
            _, info = mesh.cg_poisson(h32, src, form="face", max_iters=k, tol=0.0)
            assert info["iters"] == k and not info["converged"]
            res.append(info["res_rel"])
        u10, i10 = mesh.cg_diffuse(src, max_iters=10, tol=0.0)
        u40, i40 = mesh.cg_diffuse(src, max_iters=40, tol=0.0)
        e10, e40 = mesh.heat_residual(src, u10), mesh.heat_residual(src, u40)
        with pytest.raises(hg.NotConverged):
            mesh.cg_poisson(h32, src, form="face", max_iters=3, tol=1e-12)
    finally:
        mesh.close()
    _say("cg residuals", res, "E1", e10, e40)
    assert res[0] > res[1] > res[2]
    assert e40 < e10


def test_cg_poisson_unreached_component_is_infinite(hg):
    a = meshgen.icosphere(3)
    b = meshgen.icosphere(3)
    v, f, starts = meshgen.disjoint_union([a, b])
    src = [7]
    ref = pipeline.heat_method(v, f, src, form="edge")
    mesh = hg.Mesh(v, f)
    try:
        d, info = mesh.cg_poisson(torch.from_numpy(ref.h.astype(np.float32).reshape(-1)).cuda(), src, form="edge",
                                  tol=1e-12)
        d = d.cpu().numpy()
    finally:
        mesh.close()
    assert np.all(np.isinf(d[starts[1]:]))
    fin = np.isfinite(ref.d)
    assert np.array_equal(np.isfinite(d), fin)
    assert np.abs(d[fin] - ref.d[fin]).max() <= 1e-6 * ref.d[fin].max()
