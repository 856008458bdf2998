"""Face gradients, the normalised field of Eq. 3 and the edge targets of
Eq. 18 (test infrastructure only)."""
from __future__ import annotations

import numpy as np

from .assembly import face_geometry


def face_gradients(verts, tris, u) -> np.ndarray:
    """grad u|_f = (1/(2 A_f)) sum_i u_i (N_f x e_i), e_i the CCW edge
    opposite corner i; float64[F, 3]."""
    area, normal, _ = face_geometry(verts, tris)
    g = np.zeros((tris.shape[0], 3))
    for k in range(3):
        e = verts[tris[:, (k + 2) % 3]] - verts[tris[:, (k + 1) % 3]]
        g += u[tris[:, k]][:, None] * np.cross(normal, e)
    return g / (2.0 * area)[:, None]


def normalized_field(verts, tris, logu) -> np.ndarray:
    """h_f = -grad u|_f / |grad u|_f| (Eq. 3) from log u.

    The three values of a face are rescaled by exp(-max log u) first; the
    direction of the gradient does not depend on that scale.  A face whose
    gradient vanishes (or whose three values all underflowed to -inf) gets
    h_f = 0: the paper does not cover this case.
    """
    lf = logu[tris]
    m = lf.max(axis=1)
    ok = np.isfinite(m)
    w = np.zeros_like(lf)
    w[ok] = np.exp(lf[ok] - m[ok, None])
    area, normal, _ = face_geometry(verts, tris)
    g = np.zeros((tris.shape[0], 3))
    for k in range(3):
        e = verts[tris[:, (k + 2) % 3]] - verts[tris[:, (k + 1) % 3]]
        g += w[:, k][:, None] * np.cross(normal, e)
    nrm = np.linalg.norm(g, axis=1)
    h = np.zeros_like(g)
    good = nrm > 0
    h[good] = -g[good] / nrm[good, None]
    return h


def edge_targets(verts, topo, h) -> np.ndarray:
    """Z[f, k] = h_f . (p_head - p_tail) for the edge in slot k of face f,
    measured along the edge's orientation halfedge (Eq. 18)."""
    e = topo.face_edges
    tail = topo.edges[e, 0]
    head = topo.edges[e, 1]
    vec = verts[head] - verts[tail]                   # [F, 3, 3]
    return np.einsum("fc,fkc->fk", h, vec)
