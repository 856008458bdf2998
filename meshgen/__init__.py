"""Seeded synthetic triangle meshes and source sets.

This module only builds inputs: vertex positions, triangle index arrays and
source-vertex lists.  It holds none of the geodesic method's arithmetic (no
cotangent weights, areas, diffusion, gradients or integration), so both the
CPU oracle and the GPU library can consume what it produces without sharing
any computation.

Generators (all randomness from ``numpy.random.default_rng(seed)``):

* :func:`grid` -- n x n vertex grid on [0,1]^2, each square split along its
  (i,j)-(i+1,j+1) diagonal, interior vertices jittered uniformly.
* :func:`affine_grid` -- that grid sheared and squashed into a parallelogram
  (a poorly shaped, non-Delaunay planar triangulation).
* :func:`torus`, :func:`annulus` -- a jittered genus-1 torus; a grid with a
  hole (two boundary loops).
* :func:`icosphere` -- regular icosahedron refined by ``level`` rounds of
  1->4 midpoint subdivision, midpoints projected to the unit sphere each round.
* :func:`tangential_jitter` -- move each sphere vertex inside its tangent plane
  and re-project to the sphere.
* :func:`harmonic_displacement` -- radial displacement r = 1 + amp * S/max|S|
  with S a seeded sum of real spherical harmonics.
* :func:`random_sources` -- distinct uniform random vertices.

Meshes are returned as ``(verts float64[V,3], tris int32[F,3])`` with
counter-clockwise faces (outward normals on the sphere, +z on the grid).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "grid",
    "affine_grid",
    "grid_center_source",
    "icosphere",
    "mean_edge_length_raw",
    "tangential_jitter",
    "harmonic_displacement",
    "random_sources",
    "config_mesh",
    "batch_meshes",
]


# --------------------------------------------------------------------------
# flat grid
# --------------------------------------------------------------------------
def grid(n: int = 64, jitter: float = 0.2, seed: int = 1):
    """n x n grid on [0,1]^2 with vertex (i, j) at index j*n + i.

    Every square (i, j)-(i+1, j+1) is split along its diagonal into the two
    CCW triangles (a, b, d) and (a, d, c) with a=(i,j), b=(i+1,j), c=(i,j+1),
    d=(i+1,j+1).  Interior vertices move by independent U(-jitter*h, jitter*h)
    offsets in x and y, h = 1/(n-1); boundary vertices stay on the square.
    """
    h = 1.0 / (n - 1)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = ii.reshape(-1) * h
    y = jj.reshape(-1) * h
    verts = np.stack([x, y, np.zeros_like(x)], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter * h, jitter * h, size=(n * n, 2))
        interior = (ii.reshape(-1) > 0) & (ii.reshape(-1) < n - 1) & \
                   (jj.reshape(-1) > 0) & (jj.reshape(-1) < n - 1)
        verts[interior, 0] += off[interior, 0]
        verts[interior, 1] += off[interior, 1]
    i0, j0 = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    a = (j0 * n + i0).reshape(-1)
    b = a + 1
    c = a + n
    d = a + n + 1
    t1 = np.stack([a, b, d], axis=1)
    t2 = np.stack([a, d, c], axis=1)
    tris = np.empty((2 * a.size, 3), dtype=np.int32)
    tris[0::2] = t1
    tris[1::2] = t2
    return verts, tris


def torus(nu: int = 48, nv: int = 24, R: float = 1.0, r: float = 0.4, jitter: float = 0.1, seed: int = 7):
    """Closed torus of genus 1: vertex (i, j) at index j*nu + i, at angles
    u = 2 pi (i + du)/nu around the axis and v = 2 pi (j + dv)/nv around the
    tube, position ((R + r cos v) cos u, (R + r cos v) sin u, r sin v), with
    du, dv ~ U(-jitter, jitter) (seeded).  Each quad is split along its
    diagonal into two counter-clockwise (outward) triangles."""
    rng = np.random.default_rng(seed)
    jj, ii = np.meshgrid(np.arange(nv), np.arange(nu), indexing="ij")
    du = rng.uniform(-jitter, jitter, size=nu * nv) if jitter > 0 else np.zeros(nu * nv)
    dv = rng.uniform(-jitter, jitter, size=nu * nv) if jitter > 0 else np.zeros(nu * nv)
    u = 2.0 * np.pi * (ii.reshape(-1) + du) / nu
    v = 2.0 * np.pi * (jj.reshape(-1) + dv) / nv
    verts = np.stack([(R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)], axis=1)
    i0, j0 = np.meshgrid(np.arange(nu), np.arange(nv), indexing="xy")
    a = (j0 * nu + i0).reshape(-1)
    b = (j0 * nu + (i0 + 1) % nu).reshape(-1)
    c = (((j0 + 1) % nv) * nu + i0).reshape(-1)
    d = (((j0 + 1) % nv) * nu + (i0 + 1) % nu).reshape(-1)
    tris = np.concatenate([np.stack([a, b, d], axis=1), np.stack([a, d, c], axis=1)]).astype(np.int32)
    return verts.astype(np.float64), tris


def annulus(n: int = 32, hole: float = 0.2, jitter: float = 0.1, seed: int = 3):
    """The n x n grid with the faces whose centroid lies within `hole` of
    (0.5, 0.5) removed (unused vertices dropped, order kept): a disk with
    one hole, i.e. two boundary loops."""
    v, f = grid(n, jitter, seed)
    c = v[f].mean(axis=1)
    keep = (c[:, 0] - 0.5) ** 2 + (c[:, 1] - 0.5) ** 2 > hole * hole
    f = f[keep]
    used = np.unique(f)
    remap = -np.ones(v.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    return v[used], remap[f].astype(np.int32)


def affine_grid(n: int = 32, shear: float = 1.0, squash: float = 0.3, jitter: float = 0.1, seed: int = 1):
    """:func:`grid` mapped by (x, y) -> (x + shear y, squash y): a flat
    parallelogram whose cells are split along their long diagonal, so with
    shear > 0 and squash < 1 most interior edges face two obtuse angles (a
    poor, non-Delaunay triangulation of a convex planar domain)."""
    v, f = grid(n, jitter, seed)
    out = v.copy()
    out[:, 0] = v[:, 0] + shear * v[:, 1]
    out[:, 1] = squash * v[:, 1]
    return out, f


def grid_center_source(verts, target=(0.5, 0.5)) -> int:
    """Index of the vertex nearest to ``target`` (lowest index on a tie)."""
    d2 = (verts[:, 0] - target[0]) ** 2 + (verts[:, 1] - target[1]) ** 2
    return int(np.argmin(d2))


# --------------------------------------------------------------------------
# icosphere
# --------------------------------------------------------------------------
def _icosahedron():
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def icosphere(level: int, progress=None):
    """Unit icosphere after ``level`` rounds of 1->4 midpoint subdivision.

    V = 10*4^L + 2, F = 20*4^L.  Vertex order: the parent vertices first, then
    one midpoint per parent edge, edges taken in ascending (min, max) key order.
    Midpoints are projected to the unit sphere in every round.
    """
    v, f = _icosahedron()
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        key = e[:, 0] * nv + e[:, 1]
        ukey, inv = np.unique(key, return_inverse=True)
        a = ukey // nv
        b = ukey % nv
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        v = np.concatenate([v, mid], axis=0)
        nf = f.shape[0]
        m01 = nv + inv[:nf]
        m12 = nv + inv[nf:2 * nf]
        m20 = nv + inv[2 * nf:]
        f0, f1, f2 = f[:, 0], f[:, 1], f[:, 2]
        f = np.concatenate([
            np.stack([f0, m01, m20], axis=1),
            np.stack([m01, f1, m12], axis=1),
            np.stack([m20, m12, f2], axis=1),
            np.stack([m01, m12, m20], axis=1),
        ], axis=0)
        del e, key, ukey, inv, mid
        if progress is not None:
            progress(f"icosphere: subdivision round done, {v.shape[0]} vertices")
    return np.ascontiguousarray(v), np.ascontiguousarray(f.astype(np.int32))


def mean_edge_length_raw(verts, tris) -> float:
    """Mean length over unique undirected edges (used to size the jitter)."""
    nv = verts.shape[0]
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0).astype(np.int64)
    e.sort(axis=1)
    key = np.unique(e[:, 0] * nv + e[:, 1])
    a = key // nv
    b = key % nv
    return float(np.linalg.norm(verts[a] - verts[b], axis=1).mean())


def tangential_jitter(verts, frac: float, seed: int, h: float | None = None):
    """Move each vertex by U(-a,a) t1 + U(-a,a) t2 in its tangent plane and
    project back to the unit sphere, a = frac * h (h = mean edge length of
    the input mesh unless given)."""
    if h is None:
        raise ValueError("pass h (mean edge length of the unjittered mesh)")
    rng = np.random.default_rng(seed)
    a = frac * h
    n = verts / np.linalg.norm(verts, axis=1, keepdims=True)
    ref = np.zeros_like(n)
    use_x = np.abs(n[:, 2]) > 0.9
    ref[~use_x, 2] = 1.0
    ref[use_x, 0] = 1.0
    t1 = np.cross(n, ref)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(n, t1)
    off = rng.uniform(-a, a, size=(verts.shape[0], 2))
    out = n + off[:, :1] * t1 + off[:, 1:2] * t2
    out /= np.linalg.norm(out, axis=1, keepdims=True)
    return out


def _real_sph_harm(l: int, m: int, theta, phi):
    """Real orthonormal spherical harmonic; theta = polar, phi = azimuth."""
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return np.sqrt(2.0) * (-1.0) ** m * np.real(y)
    return np.sqrt(2.0) * (-1.0) ** m * np.imag(y)


def _harmonic_sum(args):
    p, ls, ms, cs = args
    theta = np.arccos(np.clip(p[:, 2], -1.0, 1.0))
    phi = np.arctan2(p[:, 1], p[:, 0])
    acc = np.zeros(p.shape[0])
    for l, m, c in zip(ls, ms, cs):
        acc += c * _real_sph_harm(int(l), int(m), theta, phi)
    return acc


def harmonic_displacement(verts, seed: int, n_terms: int = 8, lmax: int = 16,
                          amp: float = 0.05, chunk: int = 1 << 22, workers: int = 1, progress=None):
    """Radially displace unit-sphere vertices: r = 1 + amp * S / max|S| with
    S = sum_k c_k Y_{l_k}^{m_k}, l_k ~ U{1..lmax}, m_k ~ U{-l..l},
    c_k ~ U(-1, 1).  `workers` > 1 evaluates the chunks in a process pool
    (same values)."""
    rng = np.random.default_rng(seed)
    ls = rng.integers(1, lmax + 1, size=n_terms)
    ms = np.array([rng.integers(-l, l + 1) for l in ls])
    cs = rng.uniform(-1.0, 1.0, size=n_terms)
    n = verts / np.linalg.norm(verts, axis=1, keepdims=True)
    S = np.empty(n.shape[0], dtype=np.float64)
    starts = list(range(0, n.shape[0], chunk))
    jobs = ((n[s:s + chunk], ls, ms, cs) for s in starts)
    if workers > 1 and len(starts) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            for i, (s, acc) in enumerate(zip(starts, pool.imap(_harmonic_sum, jobs))):
                S[s:s + chunk] = acc
                if progress is not None and (i + 1) % 8 == 0:
                    progress(f"harmonic displacement: {i + 1}/{len(starts)} chunks")
    else:
        for s, job in zip(starts, jobs):
            S[s:s + chunk] = _harmonic_sum(job)
    r = 1.0 + amp * S / np.max(np.abs(S))
    return n * r[:, None]


def random_sources(nv: int, k: int, seed: int):
    """k distinct uniform random vertex indices (int32, in draw order)."""
    rng = np.random.default_rng(seed)
    return rng.choice(nv, size=k, replace=False).astype(np.int32)


def disjoint_union(parts, shift=3.0):
    """Several meshes side by side as one mesh with several connected
    components (each part moved by shift * index along x).  Returns
    (verts, tris, first vertex id of each part)."""
    vs, fs, starts = [], [], []
    n = 0
    for i, (v, f) in enumerate(parts):
        vs.append(np.asarray(v, dtype=np.float64) + [shift * i, 0.0, 0.0])
        fs.append(np.asarray(f, dtype=np.int32) + n)
        starts.append(n)
        n += v.shape[0]
    return np.vstack(vs), np.vstack(fs).astype(np.int32), starts


def batch_meshes(n: int = 256, levels=(3, 6), seed: int = 4):
    """The many-small-meshes workload: n displaced icospheres whose levels
    are drawn uniformly from `levels` (seed), mesh i displaced with seed
    1000 + i and given one source drawn with seed 2000 + i.  Returns
    (list of (verts, tris), list of source arrays)."""
    rng = np.random.default_rng(seed)
    base = {}
    out = []
    for i in range(n):
        L = int(rng.integers(levels[0], levels[1] + 1))
        if L not in base:
            base[L] = icosphere(L)
        v, f = base[L]
        out.append((harmonic_displacement(v, seed=1000 + i), f))
    src = [random_sources(v.shape[0], 1, seed=2000 + i) for i, (v, _) in enumerate(out)]
    return out, src


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def config_mesh(name: str):
    """Build one named workload mesh; returns (verts, tris, sources).

    * ``"grid64"``     : 64x64 grid, jitter 0.2h (seed 1), source nearest (0.5,0.5)
    * ``"sphere8"``    : L8 icosphere, tangential jitter 0.1 h (seed 2), 1 source (seed 102)
    * ``"bumpy9"``     : L9 icosphere, harmonic displacement (seed 3), 64 sources (seed 103)
    * ``"bumpy10"``    : L10 icosphere, harmonic displacement (seed 3), 1 source (seed 104)
    * ``"bumpy12"``    : L12 icosphere, harmonic displacement (seed 3), 1 source (seed 104)
    * ``"sphereL"`` / ``"bumpyL"`` for any level L (small test meshes): plain
      icosphere / harmonic displacement seed 3, 1 source seed 100+L.
    """
    if name == "grid64":
        v, f = grid(64, 0.2, seed=1)
        return v, f, np.array([grid_center_source(v)], dtype=np.int32)
    if name == "sphere8":
        v, f = icosphere(8)
        h = mean_edge_length_raw(v, f)
        v = tangential_jitter(v, 0.1, seed=2, h=h)
        return v, f, random_sources(v.shape[0], 1, seed=102)
    if name in ("bumpy9", "bumpy10", "bumpy12"):
        lvl = int(name[5:])
        v, f = icosphere(lvl)
        v = harmonic_displacement(v, seed=3)
        if lvl == 9:
            return v, f, random_sources(v.shape[0], 64, seed=103)
        return v, f, random_sources(v.shape[0], 1, seed=104)
    if name.startswith("sphere"):
        lvl = int(name[6:])
        v, f = icosphere(lvl)
        return v, f, random_sources(v.shape[0], 1, seed=100 + lvl)
    if name.startswith("bumpy"):
        lvl = int(name[5:])
        v, f = icosphere(lvl)
        v = harmonic_displacement(v, seed=3)
        return v, f, random_sources(v.shape[0], 1, seed=100 + lvl)
    raise KeyError(name)
