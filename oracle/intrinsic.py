"""The heat method on the intrinsic Delaunay triangulation (Sec. 5.3) -- test
infrastructure only.

An intrinsic triangulation keeps the mesh's vertices but describes the
surface by connectivity plus one length per edge; a triangle's angles come
from unfolding it into the plane with those lengths.  It is Delaunay when
the two angles facing every interior edge sum to at most pi, i.e.
cot a + cot b >= 0.  It is reached by flipping edges that violate this
(the edge-flip algorithm the section relies on):

* lengths start as the 3D edge lengths;
* a first-in-first-out queue holds interior edges, initially all of them in
  canonical order (sorted by (smaller id, larger id)); an edge is queued at
  most once at a time;
* a popped edge {u, v} (u < v) with the face f1 that runs u -> v and the
  face f2 that runs v -> u, c and d their third vertices: if
  cot(c) + cot(d) < -tol it is flipped to {c, d}, unless c == d or c and d
  are already joined by an edge (the flip would leave a simplicial mesh;
  such an edge stays non-Delaunay and is counted);
* the new length is the distance of c and d after unfolding the two
  triangles into the plane on either side of u v; f1 becomes (c, u, d) and
  f2 becomes (d, v, c) (the rows keep their places), and the four outer
  edges u c, c v, v d, d u are queued.

Every flip of a non-Delaunay edge lowers the Dirichlet energy of the
triangulation, so the loop ends.  Readings (the section gives no details):
the flip test uses tol = 1e-12; the diffusion time uses the mean edge length
of the input mesh (t = m hbar^2 of Eq. 27 measures the input's spacing, the
flips only change how it is discretised); the face form is not covered (the
section only outlines it), the edge form is.

Formulas (FP64), also the ones any other implementation has to use where
they decide a flip:
  area(a, b, c) = sqrt(max(0, (a + (b + c)) (c - (a - b)) (c + (a - b))
                  (a + (b - c)))) / 4 with a >= b >= c (stable Heron form),
  cot of the corner facing side a = (b^2 + c^2 - a^2) / (4 area),
  unfolding with u at the origin and v on the +x axis (length L):
    x_c = (L^2 + l_uc^2 - l_vc^2) / (2 L), y_c = 2 area(f1) / L,
    x_d = (L^2 + l_ud^2 - l_vd^2) / (2 L), y_d = -2 area(f2) / L,
    l_cd = sqrt((x_c - x_d)^2 + (y_c - y_d)^2).
Each face then gets a local frame: its first vertex at the origin, its
first edge along +x, its third vertex at y > 0; gradients (Eq. 3) and edge
targets (Eq. 18) are taken in that frame.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass
from math import sqrt

import numpy as np
import scipy.sparse as sp

from . import bfs, diffusion, mesh, poisson

FLIP_TOL = 1e-12


def tri_area(a: float, b: float, c: float) -> float:
    """Area of the triangle with side lengths a, b, c (stable Heron form)."""
    if a < b:
        a, b = b, a
    if b < c:
        b, c = c, b
    if a < b:
        a, b = b, a
    p = (a + (b + c)) * (c - (a - b)) * (c + (a - b)) * (a + (b - c))
    return 0.25 * sqrt(p) if p > 0.0 else 0.0


def corner_cot(opp: float, s1: float, s2: float, area: float) -> float:
    """Cotangent of the corner facing the side of length `opp`."""
    return (s1 * s1 + s2 * s2 - opp * opp) / (4.0 * area)


def _key(a: int, b: int):
    return (a, b) if a < b else (b, a)


@dataclass
class IntrinsicMesh:
    tris: np.ndarray        # int64[F, 3], rows in the input's order, flipped in place
    length: dict            # (min, max) -> FP64 edge length
    n_flips: int
    n_nondelaunay: int      # interior edges left with cot a + cot b < -tol

    def edge_lengths(self, edges) -> np.ndarray:
        return np.array([self.length[(int(a), int(b))] for a, b in edges], dtype=np.float64)


def intrinsic_delaunay(verts, tris, tol: float = FLIP_TOL) -> IntrinsicMesh:
    verts = np.asarray(verts, dtype=np.float64)
    T = [list(map(int, t)) for t in np.asarray(tris, dtype=np.int64)]
    length = {}
    side = {}       # key -> [face running min -> max, face running max -> min]
    for f, t in enumerate(T):
        for k in range(3):
            a, b = t[k], t[(k + 1) % 3]
            key = _key(a, b)
            if key not in length:
                p, q = verts[key[0]], verts[key[1]]
                dx, dy, dz = q[0] - p[0], q[1] - p[1], q[2] - p[2]
                length[key] = sqrt(dx * dx + dy * dy + dz * dz)
                side[key] = [-1, -1]
            side[key][0 if a < b else 1] = f

    def third(f, a, b):
        t = T[f]
        return next(x for x in t if x != a and x != b)

    def cot_sum(key):
        u, v = key
        f1, f2 = side[key]
        c, d = third(f1, u, v), third(f2, u, v)
        L = length[key]
        luc, lvc = length[_key(u, c)], length[_key(v, c)]
        lud, lvd = length[_key(u, d)], length[_key(v, d)]
        A1, A2 = tri_area(L, lvc, luc), tri_area(L, lvd, lud)
        return corner_cot(L, lvc, luc, A1) + corner_cot(L, lvd, lud, A2), (c, d, L, luc, lvc, lud, lvd, A1, A2)

    def interior(key):
        s = side[key]
        return s[0] >= 0 and s[1] >= 0

    queue = deque(sorted(k for k in side if interior(k)))
    queued = set(queue)
    flips = 0
    while queue:
        key = queue.popleft()
        queued.discard(key)
        if key not in side or not interior(key):
            continue
        s, (c, d, L, luc, lvc, lud, lvd, A1, A2) = cot_sum(key)
        if s >= -tol:
            continue
        if c == d or _key(c, d) in side:
            continue
        u, v = key
        f1, f2 = side[key]
        xc = (L * L + luc * luc - lvc * lvc) / (2.0 * L)
        yc = 2.0 * A1 / L
        xd = (L * L + lud * lud - lvd * lvd) / (2.0 * L)
        yd = -2.0 * A2 / L
        dx, dy = xc - xd, yc - yd
        del side[key], length[key]
        nk = _key(c, d)
        length[nk] = sqrt(dx * dx + dy * dy)
        side[nk] = [-1, -1]
        T[f1] = [c, u, d]
        T[f2] = [d, v, c]
        for f in (f1, f2):
            t = T[f]
            for k in range(3):
                a, b = t[k], t[(k + 1) % 3]
                side[_key(a, b)][0 if a < b else 1] = f
        flips += 1
        for a, b in ((u, c), (c, v), (v, d), (d, u)):
            k2 = _key(a, b)
            if interior(k2) and k2 not in queued:
                queue.append(k2)
                queued.add(k2)
    bad = sum(1 for k in side if interior(k) and cot_sum(k)[0] < -tol)
    return IntrinsicMesh(tris=np.array(T, dtype=np.int64).reshape(-1, 3), length=length, n_flips=flips,
                         n_nondelaunay=bad)


def face_lengths(im: IntrinsicMesh) -> np.ndarray:
    """l[f, k] = length of the edge (tri[k], tri[k+1]) of face f."""
    t = im.tris
    out = np.empty(t.shape, dtype=np.float64)
    for f in range(t.shape[0]):
        for k in range(3):
            out[f, k] = im.length[_key(int(t[f, k]), int(t[f, (k + 1) % 3]))]
    return out


def local_frames(lf: np.ndarray) -> np.ndarray:
    """Corner positions of every face in its own plane: P[f, 0] = (0, 0),
    P[f, 1] = (l_01, 0), P[f, 2] at y > 0 from the law of cosines."""
    l01, l12, l20 = lf[:, 0], lf[:, 1], lf[:, 2]
    x2 = (l01 ** 2 + l20 ** 2 - l12 ** 2) / (2.0 * l01)
    y2 = np.sqrt(np.maximum(l20 ** 2 - x2 ** 2, 0.0))
    P = np.zeros((lf.shape[0], 3, 2))
    P[:, 1, 0] = l01
    P[:, 2, 0] = x2
    P[:, 2, 1] = y2
    return P


def geometry(P: np.ndarray):
    """Per face: area and the cotangent of each corner angle, from the
    local frames (2D dot and cross products)."""
    e1 = P[:, 1] - P[:, 0]
    e2 = P[:, 2] - P[:, 0]
    dbl = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    cots = np.empty((P.shape[0], 3))
    for k in range(3):
        u = P[:, (k + 1) % 3] - P[:, k]
        w = P[:, (k + 2) % 3] - P[:, k]
        cots[:, k] = (u * w).sum(axis=1) / dbl
    return 0.5 * dbl, cots


def stiffness_and_areas(nv: int, tris: np.ndarray, area: np.ndarray, cots: np.ndarray):
    """K = -L_c with theta_jk = (cot a + cot b) / 2, and A_j = (1/3) sum of
    the incident face areas (Sec. 3.1), on the intrinsic faces."""
    i_l, j_l, w_l = [], [], []
    for k in range(3):
        a, b = tris[:, (k + 1) % 3], tris[:, (k + 2) % 3]
        w = 0.5 * cots[:, k]
        i_l += [a, b]
        j_l += [b, a]
        w_l += [w, w]
    theta = sp.csr_matrix((np.concatenate(w_l), (np.concatenate(i_l), np.concatenate(j_l))), shape=(nv, nv))
    theta.sum_duplicates()
    K = (sp.diags(np.asarray(theta.sum(axis=1)).ravel()) - theta).tocsr()
    A = np.zeros(nv)
    for k in range(3):
        np.add.at(A, tris[:, k], area / 3.0)
    return K, A


def normalized_field_local(P: np.ndarray, tris: np.ndarray, logu: np.ndarray) -> np.ndarray:
    """h_f = -grad u / |grad u| (Eq. 3) in each face's local frame, from
    log u (the face's values rescaled by exp(-max log u) first; a face with
    no finite value or a vanishing gradient gets h = 0)."""
    lf = logu[tris]
    m = lf.max(axis=1)
    ok = np.isfinite(m)
    w = np.zeros_like(lf)
    w[ok] = np.exp(lf[ok] - m[ok, None])
    area, _ = geometry(P)
    g = np.zeros((P.shape[0], 2))
    for k in range(3):
        e = P[:, (k + 2) % 3] - P[:, (k + 1) % 3]       # CCW edge opposite corner k
        g += w[:, k][:, None] * np.stack([-e[:, 1], e[:, 0]], axis=1)   # rotated by +90 degrees
    g /= (2.0 * area)[:, None]
    nrm = np.linalg.norm(g, axis=1)
    h = np.zeros_like(g)
    good = nrm > 0
    h[good] = -g[good] / nrm[good, None]
    return h


def edge_targets_local(P: np.ndarray, tris: np.ndarray, h2: np.ndarray) -> np.ndarray:
    """Z[f, k] = h_f . (P_head - P_tail) for the edge in slot k, measured
    along its orientation halfedge (smaller to larger vertex id) (Eq. 18)."""
    Z = np.empty(tris.shape, dtype=np.float64)
    for k in range(3):
        a, b = tris[:, k], tris[:, (k + 1) % 3]
        vec = P[:, (k + 1) % 3] - P[:, k]            # a -> b
        s = np.where(a < b, 1.0, -1.0)
        Z[:, k] = s * (h2 * vec).sum(axis=1)
    return Z


def poisson_edge_targets(nv: int, topo, Z: np.ndarray, sources, reach=None) -> np.ndarray:
    """Edge-form distance from edge targets: the minimiser of
    sum_f sum_k (d_head - d_tail - Z[f, k])^2 with d = 0 at the sources;
    normal equations L_E d = b_E, b_E[head] += Z, b_E[tail] -= Z."""
    w = topo.edge_nfaces.astype(np.float64)
    a, b = topo.edges[:, 0], topo.edges[:, 1]
    off = sp.csr_matrix((np.concatenate([-w, -w]), (np.concatenate([a, b]), np.concatenate([b, a]))),
                        shape=(nv, nv))
    L = (sp.diags(-np.asarray(off.sum(axis=1)).ravel()) + off).tocsr()
    bE = np.zeros(nv)
    e = topo.face_edges
    np.add.at(bE, topo.edges[e, 1].ravel(), Z.ravel())
    np.add.at(bE, topo.edges[e, 0].ravel(), -Z.ravel())
    return poisson.dirichlet_solve(L, bE, sources, reach)


def triangulation_quality(lf: np.ndarray) -> float:
    """tau of the quality measure the section uses: mean over faces of
    2 sqrt(3) r_f / l_f, r_f the inradius (2 area / perimeter) and l_f the
    longest edge; 1 for equilateral triangles."""
    area = np.array([tri_area(*row) for row in lf])
    r = 2.0 * area / lf.sum(axis=1)
    return float((2.0 * np.sqrt(3.0) * r / lf.max(axis=1)).mean())


@dataclass
class IntrinsicResult:
    im: IntrinsicMesh
    topo: mesh.Topology
    P: np.ndarray
    t: float
    hbar: float
    logu: np.ndarray
    h: np.ndarray            # [F, 2] local frames
    Z: np.ndarray            # [F, 3] edge targets
    d: np.ndarray
    level: np.ndarray
    parent: np.ndarray


def heat_method_intrinsic(verts, tris, sources, m: float = 1.0, t: float | None = None) -> IntrinsicResult:
    """Edge-form heat method on the intrinsic Delaunay triangulation: BFS
    sets on its connectivity, diffusion (Eq. 4) with its areas and
    cotangents, h in the local frames, edge targets (Eq. 18) and the
    edge-form Poisson distance (d = 0 at every source)."""
    verts = np.asarray(verts, dtype=np.float64)
    nv = verts.shape[0]
    sources = np.unique(np.asarray(sources, dtype=np.int64))
    topo0 = mesh.build_topology(np.asarray(tris, dtype=np.int64), nv)
    hbar = float(np.linalg.norm(verts[topo0.edges[:, 0]] - verts[topo0.edges[:, 1]], axis=1).mean())
    if t is None or t <= 0:
        t = m * hbar * hbar
    im = intrinsic_delaunay(verts, tris)
    topo = mesh.build_topology(im.tris, nv)
    P = local_frames(face_lengths(im))
    area, cots = geometry(P)
    K, A = stiffness_and_areas(nv, im.tris, area, cots)
    M = diffusion.heat_matrix(K, A, t)
    logu = diffusion.solve_log(M, sources)
    h = normalized_field_local(P, im.tris, logu)
    Z = edge_targets_local(P, im.tris, h)
    d = poisson_edge_targets(nv, topo, Z, sources, np.isfinite(logu))
    rp, col = mesh.vertex_adjacency(nv, topo.edges)
    level, parent = bfs.bfs_levels_vec(nv, rp, col, sources)
    return IntrinsicResult(im=im, topo=topo, P=P, t=t, hbar=hbar, logu=logu, h=h, Z=Z, d=d, level=level,
                           parent=parent)
