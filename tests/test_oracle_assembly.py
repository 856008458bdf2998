"""Pins of the oracle's discrete operators (Sec. 3.1): each check uses a fact
the mathematics fixes, not the oracle's own formula."""
import numpy as np
import pytest

import meshgen
from oracle import assembly, gradient, mesh, poisson
from tests.oracle_fixtures import equilateral_patch, interior_mask


@pytest.fixture(scope="module")
def grid17():
    return meshgen.grid(17, 0.2, seed=11)


def test_stiffness_symmetric_zero_rowsum(grid17):
    v, f = grid17
    K = assembly.cotan_stiffness(v, f)
    assert abs(K - K.T).max() < 1e-13
    assert np.abs(np.asarray(K.sum(axis=1))).max() < 1e-12


def test_stiffness_psd():
    v, f = meshgen.icosphere(2)
    v = meshgen.harmonic_displacement(v, seed=5)
    K = assembly.cotan_stiffness(v, f).toarray()
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-10
    assert abs(ev[0]) < 1e-10 and ev[1] > 1e-6       # one zero mode (connected)


def test_cotan_weights_from_angles():
    """theta_jk = (cot a + cot b)/2 computed independently from arccos angles."""
    v, f = meshgen.grid(7, 0.25, seed=3)
    K = assembly.cotan_stiffness(v, f).tocsr()
    nv = v.shape[0]
    theta = {}
    for tri in f:
        for k in range(3):
            i, a, b = tri[k], tri[(k + 1) % 3], tri[(k + 2) % 3]
            u, w = v[a] - v[i], v[b] - v[i]
            ang = np.arccos(np.dot(u, w) / np.linalg.norm(u) / np.linalg.norm(w))
            key = (min(a, b), max(a, b))
            theta[key] = theta.get(key, 0.0) + 0.5 / np.tan(ang)
    for (a, b), th in theta.items():
        assert abs(-K[a, b] - th) < 1e-12 * max(1.0, abs(th))
    assert len(theta) == (K.nnz - nv) // 2


def test_laplacian_of_x_squared_is_two():
    """On an equilateral lattice, (1/A_j) sum theta_jk (u_k - u_j) = 2 for
    u = x^2 at interior vertices: pins the 1/2 in theta and the 1/3 in A_j."""
    v, f = equilateral_patch(9, h=0.37)
    K = assembly.cotan_stiffness(v, f)
    A = assembly.lumped_areas(v, f)
    u = v[:, 0] ** 2
    lap = -(K @ u) / A
    inner = interior_mask(v, f)
    assert np.allclose(lap[inner], 2.0, atol=1e-11)


def test_linear_precision(grid17):
    v, f = grid17
    K = assembly.cotan_stiffness(v, f)
    inner = interior_mask(v, f)
    for ell in (v[:, 0], v[:, 1], 0.3 * v[:, 0] - 1.7 * v[:, 1] + 2.0):
        assert np.abs((K @ ell)[inner]).max() < 1e-12


def test_lumped_area_total_and_sphere_limit():
    prev = None
    for L in (2, 3, 4, 5):
        v, f = meshgen.icosphere(L)
        A = assembly.lumped_areas(v, f)
        area, _, _ = assembly.face_geometry(v, f)
        assert abs(A.sum() - area.sum()) < 1e-12 * area.sum()
        err = abs(A.sum() - 4 * np.pi)
        if prev is not None:
            assert err < prev / 3.5                  # O(h^2) convergence to 4 pi
        prev = err
    assert prev < 5e-3


def test_mean_edge_length_equilateral():
    v, f = equilateral_patch(6, h=0.5)
    topo = mesh.build_topology(f, v.shape[0])
    assert abs(assembly.mean_edge_length(v, topo.edges) - 0.5) < 1e-14


def test_gradient_of_linear_function_exact(grid17):
    v, f = grid17
    a = np.array([0.7, -1.3, 0.0])
    g = gradient.face_gradients(v, f, v @ a + 0.4)
    assert np.abs(g - a).max() < 1e-11
    G = assembly.gradient_operator(v, f)
    assert np.abs(G @ np.ones(v.shape[0])).max() < 1e-11     # sum_i grad phi_i = 0


def test_gradient_tangent_on_sphere():
    v, f = meshgen.icosphere(3)
    v = meshgen.harmonic_displacement(v, seed=7)
    u = np.sin(3 * v[:, 0]) + v[:, 2] ** 2
    g = gradient.face_gradients(v, f, u)
    _, n, _ = assembly.face_geometry(v, f)
    assert np.abs(np.einsum("fc,fc->f", g, n)).max() < 1e-12


def test_divergence_matches_cotan_formula():
    """r = grad^T A_F h equals minus the heat method's integrated divergence
    (1/2) sum_f [cot t1 (e1.X) + cot t2 (e2.X)], written here from angles."""
    v, f = meshgen.icosphere(2)
    v = meshgen.harmonic_displacement(v, seed=9)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((f.shape[0], 3))
    _, n, _ = assembly.face_geometry(v, f)
    X -= np.einsum("fc,fc->f", X, n)[:, None] * n
    r = poisson.face_rhs(v, f, X)
    div = np.zeros(v.shape[0])
    for fi, tri in enumerate(f):
        for k in range(3):
            i, j, l = tri[k], tri[(k + 1) % 3], tri[(k + 2) % 3]
            e1, e2 = v[j] - v[i], v[l] - v[i]
            def cot(p, a, b):
                u, w = a - p, b - p
                return np.dot(u, w) / np.linalg.norm(np.cross(u, w))
            t1 = cot(v[l], v[i], v[j])       # angle opposite e1
            t2 = cot(v[j], v[i], v[l])       # angle opposite e2
            div[i] += 0.5 * (t1 * np.dot(e1, X[fi]) + t2 * np.dot(e2, X[fi]))
    assert np.abs(r + div).max() < 1e-12
    assert abs(r.sum()) < 1e-12


def test_topology_signs_exact_forms():
    """x_e = d(head) - d(tail) of any vertex function is closed on every face
    under the signs of Eq. 20 (a sign or slot mistake breaks this)."""
    v, f = meshgen.icosphere(2)
    topo = mesh.build_topology(f, v.shape[0])
    d = np.random.default_rng(1).standard_normal(v.shape[0])
    x = d[topo.edges[:, 1]] - d[topo.edges[:, 0]]
    closed = (topo.face_signs * x[topo.face_edges]).sum(axis=1)
    assert np.abs(closed).max() < 1e-12
    assert topo.ne == 30 * 4 ** 2 and np.all(topo.edge_nfaces == 2)
    # slot k of a face is the edge (tri[k], tri[k+1])
    e = topo.edges[topo.face_edges]
    a, b = f, np.roll(f, -1, axis=1)
    assert np.all(np.minimum(a, b) == e[..., 0]) and np.all(np.maximum(a, b) == e[..., 1])


def test_topology_rejects_bad_meshes():
    f = np.array([[0, 1, 2], [0, 1, 3]])        # same edge direction twice
    with pytest.raises(ValueError):
        mesh.build_topology(f, 4)
    f = np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]])
    with pytest.raises(ValueError):
        mesh.build_topology(f, 5)
