"""Pins of the intrinsic Delaunay oracle (Sec. 5.3) against facts that do not
come from the oracle itself:

* a flat mesh's intrinsic Delaunay triangulation is its Euclidean Delaunay
  triangulation: no vertex lies inside any face's circumcircle (brute force
  over all vertices), every intrinsic length is the straight-line distance
  of its endpoints, and the area is unchanged;
* on a curved mesh a flipped edge is a path over the surface, never shorter
  than the chord between its endpoints; the area is unchanged;
* a mesh that is already Delaunay is left alone, and the operators built
  from lengths and local frames equal the ones built from positions
  (independent formulas: cross and dot products in 3D);
* for a linear function on a flat mesh the local-frame targets are the
  exact edge differences of -u / |grad u|;
* a flat mesh after the flips runs the extrinsic pipeline on the flipped
  connectivity to rounding;
* the quality measure is 1 for an equilateral triangle and the closed form
  for a right isosceles one;
* on a poor flat triangulation the intrinsic heat method is closer to the
  exact distance (the straight-line distance on a convex flat domain) than
  the plain one.
"""
import numpy as np
import pytest

import meshgen
from oracle import admm, assembly, gradient, integrate, intrinsic, mesh, pipeline


def _flat():
    return meshgen.affine_grid(20, shear=1.0, squash=0.3, jitter=0.1, seed=2)


def _poor_sphere(level=3, frac=0.45, seed=5):
    v, f = meshgen.icosphere(level)
    return meshgen.tangential_jitter(v, frac, seed, h=meshgen.mean_edge_length_raw(v, f)), f


def _area(v, f):
    return float(np.linalg.norm(np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]]), axis=1).sum() / 2)


def test_flat_mesh_becomes_euclidean_delaunay():
    v, f = _flat()
    im = intrinsic.intrinsic_delaunay(v, f)
    assert im.n_flips > 100 and im.n_nondelaunay == 0
    t = im.tris
    # empty circumcircles (2D, brute force)
    p = v[:, :2]
    a, b, c = p[t[:, 0]], p[t[:, 1]], p[t[:, 2]]
    d = 2.0 * (a[:, 0] * (b[:, 1] - c[:, 1]) + b[:, 0] * (c[:, 1] - a[:, 1]) + c[:, 0] * (a[:, 1] - b[:, 1]))
    sa, sb, sc = (a ** 2).sum(1), (b ** 2).sum(1), (c ** 2).sum(1)
    ux = (sa * (b[:, 1] - c[:, 1]) + sb * (c[:, 1] - a[:, 1]) + sc * (a[:, 1] - b[:, 1])) / d
    uy = (sa * (c[:, 0] - b[:, 0]) + sb * (a[:, 0] - c[:, 0]) + sc * (b[:, 0] - a[:, 0])) / d
    r2 = (a[:, 0] - ux) ** 2 + (a[:, 1] - uy) ** 2
    dist2 = (p[None, :, 0] - ux[:, None]) ** 2 + (p[None, :, 1] - uy[:, None]) ** 2
    own = np.zeros_like(dist2, dtype=bool)
    own[np.arange(t.shape[0])[:, None], t] = True
    inside = (dist2 < r2[:, None] * (1 - 1e-9)) & ~own
    assert not inside.any()
    for (x, y), L in im.length.items():
        assert L == pytest.approx(np.linalg.norm(v[x] - v[y]), rel=1e-12)
    assert _area(v, t) == pytest.approx(_area(v, f), rel=1e-12)


def test_curved_flips_are_surface_paths():
    v, f = _poor_sphere()
    im = intrinsic.intrinsic_delaunay(v, f)
    assert im.n_flips > 50 and im.n_nondelaunay == 0
    orig = {tuple(sorted(e)) for t in f for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    new = [k for k in im.length if k not in orig]
    assert new
    for x, y in new:
        assert im.length[(x, y)] >= np.linalg.norm(v[x] - v[y]) * (1 - 1e-12)
        assert im.length[(x, y)] > np.linalg.norm(v[x] - v[y]) * (1 + 1e-9)    # the sphere bends every flipped quad
    lf = intrinsic.face_lengths(im)
    assert sum(intrinsic.tri_area(*r) for r in lf) == pytest.approx(_area(v, f), rel=1e-12)


def test_delaunay_mesh_is_kept_and_operators_match():
    v, f = meshgen.icosphere(2)
    v = meshgen.harmonic_displacement(v, seed=3, amp=0.02)
    im = intrinsic.intrinsic_delaunay(v, f)
    assert im.n_flips == 0 and np.array_equal(im.tris, f)
    P = intrinsic.local_frames(intrinsic.face_lengths(im))
    area, cots = intrinsic.geometry(P)
    K, A = intrinsic.stiffness_and_areas(v.shape[0], im.tris, area, cots)
    K0 = assembly.cotan_stiffness(v, f)
    assert abs(K - K0).max() < 1e-10 * abs(K0).max()
    assert np.allclose(A, assembly.lumped_areas(v, f), rtol=1e-12, atol=0)
    r = pipeline.heat_method(v, f, [7], form="edge")
    h2 = intrinsic.normalized_field_local(P, im.tris, r.logu)
    Z = intrinsic.edge_targets_local(P, im.tris, h2)
    Z0 = gradient.edge_targets(v, r.topo, r.h)
    assert np.abs(Z - Z0).max() < 1e-10 * r.hbar
    ri = intrinsic.heat_method_intrinsic(v, f, [7])
    assert np.abs(ri.d - r.d).max() < 1e-9 * r.d.max()


def test_linear_function_targets_on_flat_mesh():
    v, f = meshgen.grid(9, 0.25, seed=4)
    a, b = 0.3, -0.2
    u = 1.0 + a * v[:, 0] + b * v[:, 1]
    im = intrinsic.intrinsic_delaunay(v, f)
    P = intrinsic.local_frames(intrinsic.face_lengths(im))
    h2 = intrinsic.normalized_field_local(P, im.tris, np.log(u))
    assert np.allclose(np.linalg.norm(h2, axis=1), 1.0, atol=1e-12)
    Z = intrinsic.edge_targets_local(P, im.tris, h2)
    topo = mesh.build_topology(im.tris, v.shape[0])
    e = topo.edges[topo.face_edges]                       # [F, 3, 2] tail, head
    du = u[e[..., 1]] - u[e[..., 0]]
    assert np.abs(Z + du / np.hypot(a, b)).max() < 1e-12


def test_flat_intrinsic_pipeline_is_extrinsic_on_flipped_mesh():
    v, f = _flat()
    src = [meshgen.grid_center_source(v, (0.8, 0.15))]
    ri = intrinsic.heat_method_intrinsic(v, f, src)
    r = pipeline.heat_method(v, ri.im.tris, src, form="edge", t=ri.t)
    assert np.abs(ri.d - r.d).max() < 1e-9 * r.d.max()
    assert np.array_equal(ri.level, r.level) and np.array_equal(ri.parent, r.parent)


def test_quality_measure_closed_forms():
    assert intrinsic.triangulation_quality(np.array([[1.0, 1.0, 1.0]])) == pytest.approx(1.0, rel=1e-14)
    s2 = np.sqrt(2.0)
    want = 2 * np.sqrt(3.0) * (1.0 / (2 + s2)) / s2      # inradius (a + b - c)/2 = 1/(2 + sqrt 2)
    assert intrinsic.triangulation_quality(np.array([[1.0, 1.0, s2]])) == pytest.approx(want, rel=1e-14)


def test_intrinsic_is_more_accurate_on_poor_flat_mesh():
    v, f = meshgen.affine_grid(24, shear=0.3, squash=0.7, jitter=0.05, seed=6)
    s = meshgen.grid_center_source(v, (0.9, 0.12))
    exact = np.linalg.norm(v - v[s], axis=1)
    plain = pipeline.heat_method(v, f, [s], form="edge")
    ri = intrinsic.heat_method_intrinsic(v, f, [s])
    assert np.isfinite(plain.d).all() and np.isfinite(ri.d).all()
    mask = exact > 0
    err_plain = np.mean(np.abs(plain.d[mask] - exact[mask]) / exact[mask])
    err_idt = np.mean(np.abs(ri.d[mask] - exact[mask]) / exact[mask])
    assert err_idt < 0.5 * err_plain, (err_idt, err_plain)


def test_intrinsic_admm_reaches_poisson():
    v, f = _poor_sphere(2, 0.4, 9)
    ri = intrinsic.heat_method_intrinsic(v, f, [3])
    st = admm.EdgeADMM(ri.topo, ri.Z, 30.0, 1.8).run(20000, 1e-13)
    d = integrate.integrate_edge(ri.topo, st.x, ri.level, ri.parent, [3])
    assert np.abs(d - ri.d).max() < 1e-7 * ri.d.max()
