"""Pins of the oracle's diffusion, normalisation, Poisson, ADMM, BFS and
integration steps against facts the mathematics and the paper fix."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra, shortest_path

import meshgen
from tests.oracle_fixtures import equilateral_patch
from oracle import admm, assembly, bfs, diffusion, gradient, integrate, mesh, metrics, pipeline, poisson


def _setup(v, f, m=1.0):
    topo = mesh.build_topology(f, v.shape[0])
    K = assembly.cotan_stiffness(v, f)
    A = assembly.lumped_areas(v, f)
    t = m * assembly.mean_edge_length(v, topo.edges) ** 2
    return topo, K, A, t


@pytest.fixture(scope="module")
def bumpy3():
    v, f = meshgen.icosphere(3)
    v = meshgen.harmonic_displacement(v, seed=3)
    return v, f


# ------------------------------------------------------------ diffusion
def test_diffusion_dense_solve_and_bands(bumpy3):
    v, f = bumpy3
    topo, K, A, t = _setup(v, f)
    M = diffusion.heat_matrix(K, A, t)
    src = [17]
    dense = np.linalg.solve(M.toarray(), np.eye(v.shape[0])[17])
    l_one = diffusion.solve_log(M, src, band_rings=10 ** 9)     # plain FP64, one band
    l_band = diffusion.solve_log(M, src, band_rings=2, margin_rings=40)   # narrow bands
    l_auto = diffusion.solve_log(M, src)
    for l in (l_one, l_band, l_auto):
        assert np.abs(l - np.log(dense)).max() < 1e-11


@pytest.mark.parametrize("value_band", [100.0, 8.0])
def test_value_bands_repair_rings_that_misorder_u(value_band):
    """On an equilateral lattice the hop count overestimates distance by up
    to 2/sqrt(3) depending on direction, so hop rings misorder u far from
    the source: a ring-banded solve with thin margins is visibly wrong, and
    the value-ordered refinement recovers the dense solve from that same
    poor first pass (narrow value bands exercise many windows)."""
    v, f = equilateral_patch(40)
    topo, K, A, t = _setup(v, f)
    M = diffusion.heat_matrix(K, A, t)
    src = [0]
    exact = np.log(np.linalg.solve(M.toarray(), np.eye(v.shape[0])[0]))
    rough = diffusion.solve_log(M, src, band_rings=2, margin_rings=2, refine=False)
    fixed = diffusion.solve_log(M, src, band_rings=2, margin_rings=2, value_band=value_band)
    assert np.abs(rough - exact).max() > 1e-2
    assert np.abs(fixed - exact).max() < 1e-12


def test_diffusion_mass_conservation_and_symmetry(bumpy3):
    """1^T K = 0 gives sum_j A_j u_j = #sources; M symmetric gives
    u^(a)_b = u^(b)_a (Green's function symmetry)."""
    v, f = bumpy3
    topo, K, A, t = _setup(v, f, m=2.0)
    M = diffusion.heat_matrix(K, A, t)
    for src in ([5], [5, 300, 511]):
        u = np.exp(diffusion.solve_log(M, src, band_rings=3, margin_rings=40))
        assert abs((A * u).sum() - len(src)) < 1e-12 * len(src)
    a, b = 3, 600
    ua = diffusion.solve_log(M, [a], band_rings=3, margin_rings=40)
    ub = diffusion.solve_log(M, [b], band_rings=3, margin_rings=40)
    assert abs(ua[b] - ub[a]) < 1e-11


def _jacobi_longdouble(K, A, t, src, sweeps):
    """Plain Jacobi sweeps of Eq. 7 in x87 80-bit floats (exponent range
    e^-11355): an independent referee where FP64 cannot hold u."""
    import scipy.sparse as sp
    nv = A.size
    T = (-(K - sp.diags(K.diagonal()))).tocsr()
    rows = np.repeat(np.arange(nv), np.diff(T.indptr))
    data = T.data.astype(np.longdouble)
    D = (A + t * K.diagonal()).astype(np.longdouble)
    u0 = np.zeros(nv, dtype=np.longdouble)
    u0[src] = 1
    u = np.zeros(nv, dtype=np.longdouble)
    for _ in range(sweeps):
        acc = np.zeros(nv, dtype=np.longdouble)
        np.add.at(acc, rows, data * u[T.indices])
        u = (u0 + np.longdouble(t) * acc) / D
    return np.log(u).astype(np.float64)


@pytest.mark.parametrize("m", [1e-4, 0.01])
def test_diffusion_beyond_fp64_range_vs_80bit_jacobi(m):
    """Where u leaves the FP64 range the banded solve matches an 80-bit
    Jacobi iteration run to its fixed point."""
    v, f = meshgen.icosphere(5)
    v = meshgen.harmonic_displacement(v, seed=3)
    topo, K, A, t = _setup(v, f, m=m)
    M = diffusion.heat_matrix(K, A, t)
    src = [0]
    lb = diffusion.solve_log(M, src)
    lj = _jacobi_longdouble(K, A, t, src, 400 if m < 1e-3 else 1500)
    if m < 1e-3:
        assert lb.min() < -745          # below the smallest FP64 subnormal
    assert np.all(np.isfinite(lb))
    assert np.abs(lb - lj).max() < 1e-9 * np.abs(lj).max()


def test_paper_iterations_converge_to_direct(bumpy3):
    """The breadth-first Gauss-Seidel of Eqs. 6-7 and plain Jacobi sweeps
    have the exact solve as their fixed point."""
    v, f = bumpy3
    topo, K, A, t = _setup(v, f)
    M = diffusion.heat_matrix(K, A, t)
    src = [40]
    lexact = diffusion.solve_log(M, src)
    rp, col = mesh.vertex_adjacency(v.shape[0], topo.edges)
    lev, _ = bfs.bfs_levels(v.shape[0], rp, col, src)
    u_gs = diffusion.gauss_seidel_bfs(K, A, t, src, lev, 300)
    u_j = diffusion.jacobi(K, A, t, src, 600)
    assert np.abs(np.log(u_gs) - lexact).max() < 1e-10
    assert np.abs(np.log(u_j) - lexact).max() < 1e-10


# -------------------------------------------------------- normalisation
def test_normalized_field_unit_and_scale_invariant(bumpy3):
    v, f = bumpy3
    lu = -np.linalg.norm(v - v[0], axis=1) * 7.0
    h = gradient.normalized_field(v, f, lu)
    assert np.abs(np.linalg.norm(h, axis=1) - 1).max() < 1e-12
    assert np.abs(gradient.normalized_field(v, f, lu - 900.0) - h).max() < 1e-10
    # h points against grad u: for u = exp(-|p - p0|), along +grad|p - p0|
    g = gradient.face_gradients(v, f, np.linalg.norm(v - v[0], axis=1))
    assert np.all(np.einsum("fc,fc->f", h, g) > 0)


def test_normalized_field_degenerate_is_zero():
    v, f = meshgen.grid(5, 0.0)
    h = gradient.normalized_field(v, f, np.zeros(v.shape[0]))
    assert np.all(h == 0)
    lu = np.full(v.shape[0], -np.inf)
    assert np.all(gradient.normalized_field(v, f, lu) == 0)


# --------------------------------------------------------------- Poisson
def _tiny_disk():
    return meshgen.grid(6, 0.2, seed=4)


def test_face_qp_kkt_equals_poisson():
    """Dense KKT solve of the constrained problem Eqs. 9-10 gives the face
    gradients of the oracle's Poisson distance (Sec. 3.2 / 4.2 remark)."""
    v, f = _tiny_disk()
    topo = mesh.build_topology(f, v.shape[0])
    rng = np.random.default_rng(2)
    h = rng.standard_normal((f.shape[0], 3))
    h[:, 2] = 0.0
    h /= np.linalg.norm(h, axis=1, keepdims=True)
    area, _, _ = assembly.face_geometry(v, f)
    nf = f.shape[0]
    inter = np.flatnonzero(topo.edge_nfaces == 2)
    C = np.zeros((inter.size, 3 * nf))
    for r, e in enumerate(inter):
        ev = v[topo.edges[e, 1]] - v[topo.edges[e, 0]]
        ev /= np.linalg.norm(ev)
        f1, f2 = topo.edge_faces[e]
        C[r, 3 * f1:3 * f1 + 3] = ev
        C[r, 3 * f2:3 * f2 + 3] = -ev
    W = np.diag(np.repeat(area, 3))
    kkt = np.block([[2 * W, C.T], [C, np.zeros((inter.size, inter.size))]])
    rhs = np.concatenate([2 * W @ h.reshape(-1), np.zeros(inter.size)])
    sol = np.linalg.lstsq(kkt, rhs, rcond=None)[0]
    g = sol[:3 * nf].reshape(nf, 3)
    d = poisson.poisson_face(v, f, h, [7])
    gd = gradient.face_gradients(v, f, d)
    assert np.abs(g - gd).max() < 1e-9
    assert np.abs(C @ g.reshape(-1)).max() < 1e-10


def test_edge_qp_kkt_equals_edge_variant():
    """Dense KKT of the edge problem Eqs. 19-20 equals D d of the oracle's
    edge variant (closed = exact on a disk)."""
    v, f = _tiny_disk()
    topo = mesh.build_topology(f, v.shape[0])
    rng = np.random.default_rng(5)
    h = rng.standard_normal((f.shape[0], 3))
    h[:, 2] = 0.0
    Z = gradient.edge_targets(v, topo, h)
    ne, nf = topo.ne, f.shape[0]
    R = np.zeros((3 * nf, ne))
    R[np.arange(3 * nf), topo.face_edges.reshape(-1)] = 1.0
    Cn = np.zeros((nf, ne))
    for fi in range(nf):
        Cn[fi, topo.face_edges[fi]] = topo.face_signs[fi]
    kkt = np.block([[R.T @ R, Cn.T], [Cn, np.zeros((nf, nf))]])
    rhs = np.concatenate([R.T @ Z.reshape(-1), np.zeros(nf)])
    x = np.linalg.lstsq(kkt, rhs, rcond=None)[0][:ne]
    d = poisson.poisson_edge(v, f, topo, h, [9])
    assert np.abs(x - (d[topo.edges[:, 1]] - d[topo.edges[:, 0]])).max() < 1e-9


def test_integrable_target_reproduced_exactly():
    """h = grad(ell) for a linear ell gives d = ell - ell(s) in both forms."""
    v, f = meshgen.grid(9, 0.2, seed=6)
    topo = mesh.build_topology(f, v.shape[0])
    a = np.array([0.6, -0.8, 0.0])
    h = np.tile(a, (f.shape[0], 1))
    ell = v @ a
    s = 40
    for d in (poisson.poisson_face(v, f, h, [s]), poisson.poisson_edge(v, f, topo, h, [s])):
        assert np.abs(d - (ell - ell[s])).max() < 1e-12


def test_euclidean_distance_under_refinement():
    errs = []
    for n in (17, 33, 65):
        v, f = meshgen.grid(n, 0.2, seed=1)
        s = meshgen.grid_center_source(v)
        r = pipeline.heat_method(v, f, [s])
        de = np.linalg.norm(v - v[s], axis=1)
        errs.append(np.abs(r.d - de).mean())
    assert errs[1] < errs[0] and errs[2] < errs[1]
    assert errs[2] < 0.01


def test_great_circle_under_refinement():
    errs = []
    for L in (3, 4, 5):
        v, f = meshgen.icosphere(L)
        r = pipeline.heat_method(v, f, [0])
        gc = np.arccos(np.clip(v @ v[0], -1, 1))
        errs.append(np.abs(r.d - gc).mean())
    assert errs[1] < errs[0] and errs[2] < errs[1]
    assert errs[2] < 0.02


def test_distance_bounds_chord_and_dijkstra(bumpy3):
    v, f = bumpy3
    topo = mesh.build_topology(f, v.shape[0])
    s = 11
    r = pipeline.heat_method(v, f, [s], form="face")
    hbar = r.hbar
    w = np.linalg.norm(v[topo.edges[:, 0]] - v[topo.edges[:, 1]], axis=1)
    nv = v.shape[0]
    G = sp.csr_matrix((np.r_[w, w], (np.r_[topo.edges[:, 0], topo.edges[:, 1]],
                                     np.r_[topo.edges[:, 1], topo.edges[:, 0]])), shape=(nv, nv))
    dd = dijkstra(G, indices=s)
    chord = np.linalg.norm(v - v[s], axis=1)
    assert np.all(r.d >= chord - 1.5 * hbar)
    assert np.all(r.d <= dd + 1.5 * hbar)


def test_unit_sphere_near_rotational_symmetry():
    v, f = meshgen.icosphere(4)
    s = 0
    r = pipeline.heat_method(v, f, [s])
    z = np.round(v @ v[s], 6)
    spread = [np.ptp(r.d[z == zz]) for zz in np.unique(z) if (z == zz).sum() >= 5]
    assert max(spread) < 0.05


# ------------------------------------------------------------------ ADMM
def test_y_update_is_constrained_minimiser():
    rng = np.random.default_rng(3)
    for _ in range(20):
        q1, q2 = rng.standard_normal(3), rng.standard_normal(3)
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        A1, A2 = rng.uniform(0.1, 2, 2)
        y1, y2 = admm.y_update(q1, q2, e, np.float64(A1), np.float64(A2))
        # brute-force KKT of min A1|y1-q1|^2 + A2|y2-q2|^2 s.t. e.(y1-y2)=0
        H = np.diag(np.r_[np.full(3, 2 * A1), np.full(3, 2 * A2)])
        c = np.r_[e, -e]
        kkt = np.block([[H, c[:, None]], [c[None, :], np.zeros((1, 1))]])
        sol = np.linalg.solve(kkt, np.r_[2 * A1 * q1, 2 * A2 * q2, 0.0])
        assert np.abs(np.r_[y1, y2] - sol[:6]).max() < 1e-12
        assert abs(e @ (y1 - y2)) < 1e-12


def test_g_update_zero_gradient():
    rng = np.random.default_rng(4)
    mu, A = 100.0, 0.7
    al = np.sqrt(A)
    h = rng.standard_normal(3)
    ys = rng.standard_normal((3, 3))
    lams = rng.standard_normal((3, 3))
    acc = (ys + lams / (mu * al)).sum(axis=0)
    g = admm.g_update(h[None], acc[None], [3], mu)[0]
    # gradient of A|g-h|^2 + mu/2 sum |al(y_k - g) + lam_k/mu|^2 (Eq. 16)
    grad = 2 * A * (g - h) - mu * al * sum(al * (ys[k] - g) + lams[k] / mu for k in range(3))
    assert np.abs(grad).max() < 1e-10


def test_w_and_x_updates():
    rng = np.random.default_rng(6)
    mu = 100.0
    for _ in range(10):
        q = rng.choice([-1.0, 1.0], size=3)
        x, lam = rng.standard_normal(3), rng.standard_normal(3)
        w = admm.w_update(x, lam, q, mu)
        assert abs(q @ w) < 1e-13
        # brute force: minimise |w - (x - lam/mu)|^2 on the plane q.w = 0
        t = x - lam / mu
        kkt = np.block([[2 * np.eye(3), q[:, None]], [q[None, :], np.zeros((1, 1))]])
        assert np.abs(np.linalg.solve(kkt, np.r_[2 * t, 0.0])[:3] - w).max() < 1e-12
    hs, ls, ws = rng.standard_normal((3, 2))
    xe = admm.x_update(hs.sum(), ls.sum(), ws.sum(), 2.0, mu)
    # derivative of sum_h (x-h)^2/2 + lam (w - x) + mu/2 (w - x)^2 vanishes
    deriv = sum((xe - hs[k]) - ls[k] - mu * (ws[k] - xe) for k in range(2))
    assert abs(deriv) < 1e-10


def test_admm_fixed_point_on_integrable_field():
    v, f = meshgen.grid(9, 0.2, seed=2)
    topo = mesh.build_topology(f, v.shape[0])
    a = np.array([0.3, 0.9, 0.0]) / np.linalg.norm([0.3, 0.9])
    h = np.tile(a, (f.shape[0], 1))
    fs = admm.FaceADMM(v, f, topo, h).run(5)
    assert np.abs(fs.g - h).max() < 1e-14 and np.abs(fs.lam).max() < 1e-12
    es = admm.EdgeADMM(topo, gradient.edge_targets(v, topo, h)).run(5)
    ell = v @ a
    assert np.abs(es.x - (ell[topo.edges[:, 1]] - ell[topo.edges[:, 0]])).max() < 1e-13


@pytest.mark.parametrize("mu, alpha", [(100.0, 1.0), (30.0, 1.8)])
def test_converged_admm_integrates_to_poisson(bumpy3, mu, alpha):
    """Face and edge ADMM run to convergence, integrated in breadth-first
    order, reproduce the face and edge Poisson distances (with and without
    over-relaxation: same fixed point)."""
    v, f = bumpy3
    src = [23]
    for form in ("face", "edge"):
        r = pipeline.heat_method(v, f, src, form=form)
        if form == "face":
            st = admm.FaceADMM(v, f, r.topo, r.h, mu, alpha).run(6000, 1e-13, 1e-13)
            d = integrate.integrate_face(v, r.topo, st.g, r.level, r.parent, src)
        else:
            Z = gradient.edge_targets(v, r.topo, r.h)
            st = admm.EdgeADMM(r.topo, Z, mu, alpha).run(6000, 1e-13)
            d = integrate.integrate_edge(r.topo, st.x, r.level, r.parent, src)
        mean, mx = metrics.parity(d, r.d)
        assert mx < 1e-8, (form, mean, mx)


def _two_component_mesh():
    v, f, starts = meshgen.disjoint_union([meshgen.grid(6, 0.1, seed=4), meshgen.grid(5, 0.1, seed=5)])
    return v, f, starts[1]


def test_source_paths_are_tree_paths_between_sources():
    """Each path is a breadth-first shortest edge path from the component's
    first source; signs, faces and vectors follow the path direction; a
    source in another component starts its own tree; duplicates dropped."""
    v, f, n1 = _two_component_mesh()
    topo = mesh.build_topology(f, v.shape[0])
    src = [7, 30, n1 + 3, 7, 12, n1 + 20]
    paths = admm.source_paths(v, f, topo, src)
    assert len(paths) == 3
    rp, col = mesh.vertex_adjacency(v.shape[0], topo.edges)
    G = sp.csr_matrix((np.ones(col.size), col, rp), shape=(v.shape[0],) * 2)
    hops = shortest_path(G, unweighted=True, directed=False)
    for p, (root, dst) in zip(paths, [(7, 30), (7, 12), (n1 + 3, n1 + 20)]):
        assert p["edge"].size == hops[root, dst]
        cur = root
        for e, sg, fc, vec in zip(p["edge"], p["sign"], p["face"], p["vec"]):
            a, b = topo.edges[e]
            assert cur in (a, b)
            nxt = b if cur == a else a
            assert sg == (1.0 if cur < nxt else -1.0)
            assert np.allclose(vec, v[nxt] - v[cur])
            t = f[fc]
            runs = any(t[i] == cur and t[(i + 1) % 3] == nxt for i in range(3))
            assert runs or topo.edge_nfaces[e] == 1
            cur = nxt
        assert cur == dst
    assert admm.source_paths(v, f, topo, [4, 4]) == []


@pytest.mark.parametrize("mu, alpha", [(100.0, 1.0), (30.0, 1.8)])
def test_path_constraints_reach_the_dirichlet_poisson_distance(bumpy3, mu, alpha):
    """With the constraints of Eqs. 24-25 the converged ADMM field has equal
    distance at all sources, so integrated it equals the Poisson solution
    with d = 0 at every source (an independent sparse direct solve); the
    same iteration without them misses it by ~1e-2 of the diameter."""
    v, f = bumpy3
    src = [23, 300, 500, 611]
    for form in ("face", "edge"):
        r = pipeline.heat_method(v, f, src, form=form)
        paths = admm.source_paths(v, f, r.topo, src)
        errs = []
        for P in (paths, ()):
            if form == "face":
                st = admm.FaceADMM(v, f, r.topo, r.h, mu, alpha, paths=P).run(8000, 1e-13, 1e-13)
                d = integrate.integrate_face(v, r.topo, st.g, r.level, r.parent, src)
            else:
                Z = gradient.edge_targets(v, r.topo, r.h)
                st = admm.EdgeADMM(r.topo, Z, mu, alpha, paths=P).run(8000, 1e-13)
                d = integrate.integrate_edge(r.topo, st.x, r.level, r.parent, src)
            errs.append(metrics.parity(d, r.d)[1])
        assert errs[0] < 1e-8 and errs[1] > 1e-3, (form, errs)


@pytest.mark.parametrize("case, count", [("torus", 2), ("sphere", 0), ("annulus", 0), ("two_tori", 4)])
def test_cycle_basis_sizes_and_loops(case, count):
    """Tree-cotree leaves 2g generators per closed component (none for a
    component with boundary, out of the scope of the genus constraints);
    every edge cycle is a closed edge loop with signs along it, every face
    cycle a closed chain of adjacent faces whose polyline segments sum to
    zero."""
    if case == "torus":
        v, f = meshgen.torus()
    elif case == "sphere":
        v, f = meshgen.icosphere(3)
    elif case == "annulus":
        v, f = meshgen.annulus()
    else:
        v, f, _ = meshgen.disjoint_union([meshgen.torus(24, 12, seed=1), meshgen.torus(20, 10, seed=2)])
    topo = mesh.build_topology(f, v.shape[0])
    ec, fc = admm.cycle_constraints(v, f, topo)
    assert len(ec) == len(fc) == count
    for c in ec:
        cur = None
        start = None
        for e, sg in zip(c["edge"], c["sign"]):
            a, b = topo.edges[e]
            tail, head = (a, b) if sg > 0 else (b, a)
            if cur is None:
                start = tail
            else:
                assert tail == cur
            cur = head
        assert cur == start
    for c in fc:
        faces = c["face"]
        for i in range(faces.size):
            fa, fb = faces[i], faces[(i + 1) % faces.size]
            assert len(set(f[fa]) & set(f[fb])) == 2      # adjacent across an edge
        assert np.abs(c["vec"].sum(axis=0)).max() < 1e-12


def test_cycle_constraints_reach_poisson_on_torus():
    """On a torus, locally compatible fields need not be gradients: with the
    cycle constraints of Eqs. 22-23 the converged ADMM field integrates to
    the Poisson distance (an independent sparse solve, globally integrable
    by construction); without them both forms miss it by > 1e-4."""
    v, f = meshgen.torus()
    src = [5]
    for form in ("edge", "face"):
        r = pipeline.heat_method(v, f, src, form=form)
        ec, fc = admm.cycle_constraints(v, f, r.topo)
        errs = []
        for use in (True, False):
            if form == "edge":
                Z = gradient.edge_targets(v, r.topo, r.h)
                st = admm.EdgeADMM(r.topo, Z, 30, 1.8, paths=ec if use else ()).run(20000, 1e-13)
                d = integrate.integrate_edge(r.topo, st.x, r.level, r.parent, src)
            else:
                st = admm.FaceADMM(v, f, r.topo, r.h, 30, 1.8, paths=fc if use else ()).run(20000, 1e-13, 1e-13)
                d = integrate.integrate_face(v, r.topo, st.g, r.level, r.parent, src)
            errs.append(metrics.parity(d, r.d))
        assert errs[0][1] < 1e-8 and errs[1][0] > 1e-4, (form, errs)


def test_admm_residuals_decrease(bumpy3):
    v, f = bumpy3
    r = pipeline.heat_method(v, f, [0], form="edge")
    ea = admm.EdgeADMM(r.topo, gradient.edge_targets(v, r.topo, r.h))
    s10 = ea.run(10)
    s200 = ea.run(200)
    assert s200.r_primal < s10.r_primal and s200.r_dual < s10.r_dual


# ------------------------------------------------------ BFS / integration
def test_bfs_levels_match_library_and_parent_rule():
    v, f = meshgen.grid(12, 0.1, seed=8)
    topo = mesh.build_topology(f, v.shape[0])
    rp, col = mesh.vertex_adjacency(v.shape[0], topo.edges)
    src = [5, 77]
    lev, par = bfs.bfs_levels(v.shape[0], rp, col, src)
    lev2, par2 = bfs.bfs_levels_vec(v.shape[0], rp, col, src)
    G = sp.csr_matrix((np.ones(col.size), col, rp), shape=(v.shape[0],) * 2)
    hops = shortest_path(G, unweighted=True, indices=src, directed=False).min(axis=0)
    assert np.array_equal(lev, hops.astype(np.int64))
    assert np.array_equal(lev, lev2) and np.array_equal(par, par2)
    for j in range(v.shape[0]):
        if lev[j] > 0:
            nb = col[rp[j]:rp[j + 1]]
            assert par[j] == nb[lev[nb] == lev[j] - 1].min()


def test_integration_exact_for_exact_fields():
    v, f = meshgen.icosphere(3)
    topo = mesh.build_topology(f, v.shape[0])
    rp, col = mesh.vertex_adjacency(v.shape[0], topo.edges)
    src = [9]
    lev, par = bfs.bfs_levels_vec(v.shape[0], rp, col, src)
    d = np.random.default_rng(0).standard_normal(v.shape[0])
    d -= d[9]
    x = d[topo.edges[:, 1]] - d[topo.edges[:, 0]]
    assert np.abs(integrate.integrate_edge(topo, x, lev, par, src) - d).max() < 1e-12
    g = gradient.face_gradients(v, f, d)
    assert np.abs(integrate.integrate_face(v, topo, g, lev, par, src) - d).max() < 1e-12


def test_unreachable_component_is_infinite():
    v1, f1 = meshgen.icosphere(1)
    v = np.concatenate([v1, v1 + 5.0])
    f = np.concatenate([f1, f1 + v1.shape[0]])
    r = pipeline.heat_method(v, f, [0])
    assert np.all(np.isfinite(r.d[:v1.shape[0]])) and np.all(np.isinf(r.d[v1.shape[0]:]))
    assert np.all(r.level[v1.shape[0]:] == -1)


# ------------------------------------------ gauge-scaled whole-mesh diffusion
def test_gauge_route_matches_dense_and_banded(bumpy3):
    """The gauge-scaled whole-mesh LU equals a dense solve where FP64 holds
    u, and the banded solve (a different exact route) on a larger mesh."""
    v, f = bumpy3
    topo, K, A, t = _setup(v, f)
    M = diffusion.heat_matrix(K, A, t)
    dense = np.linalg.solve(M.toarray(), np.eye(v.shape[0])[17])
    psi = diffusion.gauge_potential(M, v, topo.edges, t, [17])
    lg = diffusion.solve_log_gauge(M, [17], psi)
    assert np.abs(lg - np.log(dense)).max() < 1e-11
    v6, f6 = meshgen.icosphere(6)
    v6 = meshgen.harmonic_displacement(v6, seed=3)
    topo6, K6, A6, t6 = _setup(v6, f6)
    M6 = diffusion.heat_matrix(K6, A6, t6)
    src = [5, 30001]
    lb = diffusion.solve_log(M6, src)
    lg6 = diffusion.solve_log_gauge(M6, src, diffusion.gauge_potential(M6, v6, topo6.edges, t6, src))
    assert np.abs(lg6 - lb).max() < 1e-9 * np.abs(lb).max()


@pytest.mark.parametrize("m", [1e-4, 0.01])
def test_gauge_route_beyond_fp64_range_vs_80bit_jacobi(m):
    """Where u itself leaves the FP64 range, the gauge-scaled solve matches an
    80-bit Jacobi iteration run to its fixed point."""
    v, f = meshgen.icosphere(5)
    v = meshgen.harmonic_displacement(v, seed=3)
    topo, K, A, t = _setup(v, f, m=m)
    M = diffusion.heat_matrix(K, A, t)
    lg = diffusion.solve_log_gauge(M, [0], diffusion.gauge_potential(M, v, topo.edges, t, [0]))
    lj = _jacobi_longdouble(K, A, t, [0], 400 if m < 1e-3 else 1500)
    if m < 1e-3:
        assert lg.min() < -745
    assert np.abs(lg - lj).max() < 1e-9 * np.abs(lj).max()


def test_gauge_route_mass_conservation_and_symmetry():
    """1^T K = 0 gives sum_j A_j u_j = number of sources; the Green's function
    of the symmetric M is symmetric, u^(a)_b = u^(b)_a, although the two
    solves use different potentials psi."""
    v, f = meshgen.icosphere(4)
    v = meshgen.harmonic_displacement(v, seed=9)
    topo, K, A, t = _setup(v, f)
    M = diffusion.heat_matrix(K, A, t)
    a, b = 3, 1999
    la = diffusion.solve_log_gauge(M, [a], diffusion.gauge_potential(M, v, topo.edges, t, [a]))
    lb = diffusion.solve_log_gauge(M, [b], diffusion.gauge_potential(M, v, topo.edges, t, [b]))
    lab = diffusion.solve_log_gauge(M, [a, b], diffusion.gauge_potential(M, v, topo.edges, t, [a, b]))
    assert abs(np.sum(A * np.exp(la)) - 1.0) < 1e-12
    assert abs(np.sum(A * np.exp(lab)) - 2.0) < 1e-12
    assert abs(la[b] - lb[a]) < 1e-11
    # linearity: u^(a,b) = u^(a) + u^(b)
    assert np.abs(np.log(np.exp(la - lab) + np.exp(lb - lab))).max() < 1e-12


def test_gauge_route_refuses_a_potential_that_underflows():
    """psi = 0 leaves v = u, which underflows at m = 1e-4: the solve raises
    instead of returning zeros."""
    v, f = meshgen.icosphere(5)
    topo, K, A, t = _setup(v, f, m=1e-4)
    M = diffusion.heat_matrix(K, A, t)
    with pytest.raises(RuntimeError):
        diffusion.solve_log_gauge(M, [0], np.zeros(v.shape[0]))


# ---------------------------------------------------- multigrid CG Poisson
@pytest.fixture(scope="module")
def bumpy6_field():
    v, f = meshgen.icosphere(6)
    v = meshgen.harmonic_displacement(v, seed=3)
    src = meshgen.random_sources(v.shape[0], 8, seed=11)
    r = pipeline.heat_method(v, f, src[:1], form="edge")
    return v, f, src, r


def test_subdivision_prolongations_rebuild_the_hierarchy():
    """The prolongations recovered from the finest adjacency are those of the
    generator's 1->4 subdivision: coarse vertices copy, every midpoint
    averages the two ends of the coarse edge it splits, which are the edges
    of the coarser icosphere."""
    from oracle import multigrid
    v5, f5 = meshgen.icosphere(5)
    v4, f4 = meshgen.icosphere(4)
    topo5 = mesh.build_topology(f5, v5.shape[0])
    rp, col = mesh.vertex_adjacency(v5.shape[0], topo5.edges)
    Ps = multigrid.subdivision_prolongations(v5.shape[0], rp, col)
    assert [P.shape for P in Ps] == [(10242, 2562), (2562, 642)]
    P = Ps[0]
    assert np.allclose(P.sum(axis=1), 1.0)
    # unnormalised midpoints of the level-4 positions point along the
    # level-5 midpoints (the generator projects them to the sphere)
    mid = P @ v4
    cos = np.einsum("ij,ij->i", mid, v5) / np.linalg.norm(mid, axis=1)
    assert np.all(cos > 1 - 1e-12)
    # parent pairs are exactly the level-4 edges
    topo4 = mesh.build_topology(f4, v4.shape[0])
    C = P.tocoo()
    keep = (C.row >= 2562)
    pairs = np.sort(C.col[keep].reshape(-1, 2), axis=1)
    got = np.unique(pairs[:, 0] * 2562 + pairs[:, 1])
    ref = np.unique(topo4.edges[:, 0] * 2562 + topo4.edges[:, 1])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("form", ["edge", "face"])
@pytest.mark.parametrize("nsrc", [1, 8])
def test_multigrid_cg_matches_sparse_lu(bumpy6_field, form, nsrc):
    """Both Poisson systems, Dirichlet at 1 and 8 sources: the multigrid-
    preconditioned CG of the large meshes equals the sparse LU solve."""
    from oracle import multigrid
    v, f, src, r = bumpy6_field
    s = src[:nsrc]
    topo = r.topo
    if form == "edge":
        L, b = poisson.edge_system(v, f, topo, r.h)
    else:
        L, b = assembly.cotan_stiffness(v, f), poisson.face_rhs(v, f, r.h)
    d_lu = poisson.dirichlet_solve(L, b, s)
    rp, col = mesh.vertex_adjacency(v.shape[0], topo.edges)
    Ps = multigrid.subdivision_prolongations(v.shape[0], rp, col)
    assert len(Ps) == 3
    d_mg, it, res = multigrid.dirichlet_solve_mg(L, b, s, Ps)
    assert res <= 1e-9 and it < 60
    assert np.abs(d_mg - d_lu).max() <= 1e-10 * d_lu.max()


def test_pcg_raises_when_not_converged(bumpy6_field):
    from oracle import multigrid
    v, f, src, r = bumpy6_field
    L, b = poisson.edge_system(v, f, r.topo, r.h)
    with pytest.raises(multigrid.NotConverged):
        multigrid.dirichlet_solve_mg(L, b, src[:1], [], rtol=1e-10)   # Jacobi-CG, 500 iterations


def test_pipeline_large_mesh_path_equals_small_mesh_path(monkeypatch):
    """The whole pipeline with its large-mesh routes (banded diffusion,
    multigrid CG) forced on a level-5 mesh equals the small-mesh routes
    (gauge-scaled LU, sparse LU)."""
    v, f = meshgen.icosphere(5)
    v = meshgen.harmonic_displacement(v, seed=3)
    src = meshgen.random_sources(v.shape[0], 3, seed=5)
    small = {form: pipeline.heat_method(v, f, src, form=form) for form in ("edge", "face")}
    monkeypatch.setattr(pipeline, "MG_MIN_V", 0)
    for form in ("edge", "face"):
        big = pipeline.heat_method(v, f, src, form=form, diffusion_route="bands")
        assert big.poisson_iters > 0 and small[form].poisson_iters == 0
        assert big.diffusion_route == "bands" and small[form].diffusion_route == "gauge"
        assert np.abs(big.logu - small[form].logu).max() < 1e-9 * np.abs(small[form].logu).max()
        assert np.abs(big.d - small[form].d).max() <= 1e-10 * small[form].d.max()
