"""Blocked edge-form ADMM launches (hg_opts.admm_block = K > 1): K
iterations per launch over LDS-resident face tiles with K-ring halos.

Every face update in a blocked launch is the arithmetic of the
single-iteration kernel, so the results must be bit-identical to
admm_block = 1 for any iteration count (remainders run as single
iterations), on meshes with boundary, several components, genus 1 without
loop constraints, and meshes with many tiles.  Solves must stop at the same
iteration with identical distances, with and without HIP graphs, also when a
run between two checks swaps the buffers' roles (an odd launch count).
Constraint groups (source paths, generator loops) fall back to single
iterations.  Parity with the oracle under the default (blocked) launches is
covered by the k-iteration and end-to-end tests of test_gpu_parity.py.
"""
import numpy as np
import pytest

import meshgen

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


def _two_parts():
    (va, fa), (vb, fb) = meshgen.grid(24, 0.2, seed=4), meshgen.icosphere(4)
    v, f, _ = meshgen.disjoint_union([(va, fa), (vb, fb)])
    return v, f, np.array([30], dtype=np.int32)


CASES = {
    "grid64": lambda: meshgen.config_mesh("grid64"),
    "bumpy6": lambda: meshgen.config_mesh("bumpy6"),
    "two_parts": _two_parts,
    "torus": lambda: (*meshgen.torus(64, 32, seed=7), np.array([5], dtype=np.int32)),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, hg):
    name = request.param
    v, f, src = CASES[name]()
    _say("mesh", name, "V", v.shape[0], "F", f.shape[0])
    mesh = hg.Mesh(v, f)
    yield name, v, f, src, mesh
    mesh.close()


def _targets(mesh, src):
    """Unit directions of a normalised heat field (the ADMM's input)."""
    logu, _ = mesh.diffuse(src)
    return mesh.normalize(logu)


@pytest.mark.parametrize("K", [2, 3, 4, 8])
@pytest.mark.parametrize("iters", [1, 5, 17, 64])
def test_blocked_iterations_bit_identical(case, hg, K, iters):
    name, v, f, src, mesh = case
    _say(name, "blocked", K, iters)
    h = _targets(mesh, src)
    o1 = hg.default_opts(admm_block=1, mu=40.0, cycle_constraints=0)
    oK = hg.default_opts(admm_block=K, mu=40.0, cycle_constraints=0)
    x1, i1 = mesh.admm_edge(h, iters=iters, opts=o1)
    xK, iK = mesh.admm_edge(h, iters=iters, opts=oK)
    assert i1.admm_block == 1 and i1.admm_launches == iters
    assert iK.admm_block == K, "tiles should fit in LDS on these meshes"
    # runs of check_every (32) iterations between residual checks, each
    # blocked launches of K and one launch of the rest
    runs = [min(32, iters - s) for s in range(0, iters, 32)]
    assert iK.admm_launches == sum(n // K + (n % K > 0) for n in runs)
    assert iK.admm_iters == iters
    a, b = x1.cpu().numpy(), xK.cpu().numpy()
    _say(name, K, iters, "max diff", float(np.abs(a - b).max()))
    assert np.array_equal(a, b)
    assert (i1.res_primal, i1.res_dual) == (iK.res_primal, iK.res_dual)


def test_blocked_to_residual_tolerance(case, hg):
    name, v, f, src, mesh = case
    h = _targets(mesh, src)
    o1 = hg.default_opts(admm_block=1, mu=40.0, cycle_constraints=0, tol_admm=1e-4)
    o4 = hg.default_opts(admm_block=4, mu=40.0, cycle_constraints=0, tol_admm=1e-4)
    x1, i1 = mesh.admm_edge(h, opts=o1)
    x4, i4 = mesh.admm_edge(h, opts=o4)
    _say(name, "to tolerance", i1.admm_iters, i4.admm_iters)
    assert i1.admm_iters == i4.admm_iters
    assert np.array_equal(x1.cpu().numpy(), x4.cpu().numpy())


@pytest.mark.parametrize("graphs", [0, 1])
@pytest.mark.parametrize("K, check", [(6, 64), (4, 64), (3, 69), (5, 66)])
def test_blocked_solve_identical(case, hg, graphs, K, check):
    """Same checks, same stop, same distances for every K; 69 / 3 = 23
    launches per run swaps the buffers' roles, so graphs are captured from
    both buffers; 64 = 10 x 6 + 4 and 66 = 13 x 5 + 1 end runs with a
    shorter blocked launch and with a single iteration."""
    name, v, f, src, mesh = case
    base = dict(use_graphs=graphs, check_every=check, cycle_constraints=0)
    d1, i1 = mesh.solve(src, 0.0, hg.default_opts(admm_block=1, **base))
    dK, iK = mesh.solve(src, 0.0, hg.default_opts(admm_block=K, **base))
    _say(name, "solve graphs", graphs, "K", K, "check", check, "iters", i1.admm_iters, iK.admm_iters,
         "launches", iK.admm_launches)
    assert iK.admm_block == K and i1.admm_block == 1
    assert i1.admm_iters == iK.admm_iters
    assert iK.admm_launches < i1.admm_launches
    a, b = d1.cpu().numpy(), dK.cpu().numpy()
    assert np.array_equal(a, b)


def test_default_is_blocked_and_paths_fall_back(hg):
    v, f = meshgen.icosphere(5)
    src = meshgen.random_sources(v.shape[0], 3, seed=11)
    mesh = hg.Mesh(v, f)
    try:
        _, i = mesh.solve(src[:1], 0.0, hg.default_opts())
        assert i.admm_block == 6
        _, i = mesh.solve(src, 0.0, hg.default_opts())         # source paths: single iterations
        assert i.admm_block == 1 and i.n_paths == 2 and i.admm_launches == i.admm_iters
        _, i = mesh.solve(src[:1], 0.0, hg.default_opts(formulation="face"))
        assert i.admm_block == 1
        for bad in (-1, 9):
            with pytest.raises(RuntimeError):
                mesh.solve(src[:1], 0.0, hg.default_opts(admm_block=bad))
    finally:
        mesh.close()
