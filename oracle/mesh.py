"""Mesh topology for the oracle (test infrastructure only).

Edges are the unique unordered vertex pairs of the triangles.  The
orientation halfedge of edge e = {a, b} (Sec. 4.1) is taken to run from the
smaller to the larger vertex index, so x_e = d(max) - d(min).  For a face
whose CCW loop traverses e as (min -> max) the integrability sign of Eq. 20
is +1, otherwise -1 (the paper's rule: +1 iff the orientation halfedge lies
in the face).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Topology:
    nv: int
    nf: int
    ne: int
    edges: np.ndarray        # int64[E, 2] (tail=min, head=max)
    face_edges: np.ndarray   # int64[F, 3]; slot k is edge (tri[k], tri[k+1])
    face_signs: np.ndarray   # int8[F, 3]; +1 if the face runs tail->head
    edge_faces: np.ndarray   # int64[E, 2]; -1 where the edge has one face
    edge_nfaces: np.ndarray  # int64[E]; |H_e| of Eq. 19 (1 or 2)


def build_topology(tris: np.ndarray, nv: int) -> Topology:
    """Edge list, face->edge slots, Eq. 20 signs and edge->face incidence.

    Raises ValueError for an edge shared by more than two faces or for two
    faces that traverse a shared edge in the same direction (inconsistent
    orientation), since the signs of Eq. 20 need an oriented manifold.
    """
    tris = np.asarray(tris, dtype=np.int64)
    nf = tris.shape[0]
    a = np.concatenate([tris[:, 0], tris[:, 1], tris[:, 2]])
    b = np.concatenate([tris[:, 1], tris[:, 2], tris[:, 0]])
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = lo * nv + hi
    ukey, inv = np.unique(key, return_inverse=True)
    ne = ukey.size
    edges = np.stack([ukey // nv, ukey % nv], axis=1)
    face_edges = inv.reshape(3, nf).T.copy()
    face_signs = np.where(a < b, 1, -1).astype(np.int8).reshape(3, nf).T.copy()
    counts = np.bincount(inv, minlength=ne)
    if counts.max(initial=0) > 2:
        raise ValueError("non-manifold edge (more than two incident faces)")
    # consistent orientation: the two faces of an interior edge run it in
    # opposite directions, so their signs sum to zero
    ssum = np.bincount(inv, weights=np.where(a < b, 1.0, -1.0), minlength=ne)
    if np.any((counts == 2) & (ssum != 0)):
        raise ValueError("inconsistently oriented faces")
    fidx = np.tile(np.arange(nf), 3)
    order = np.argsort(inv, kind="stable")
    edge_faces = -np.ones((ne, 2), dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    first = fidx[order[starts]]
    edge_faces[:, 0] = first
    two = counts == 2
    edge_faces[two, 1] = fidx[order[starts[two] + 1]]
    return Topology(nv=nv, nf=nf, ne=ne, edges=edges, face_edges=face_edges,
                    face_signs=face_signs, edge_faces=edge_faces,
                    edge_nfaces=counts.astype(np.int64))


def vertex_adjacency(nv: int, edges: np.ndarray):
    """CSR one-ring adjacency (row_ptr, col) of the undirected edge graph."""
    import scipy.sparse as sp
    i = np.concatenate([edges[:, 0], edges[:, 1]])
    j = np.concatenate([edges[:, 1], edges[:, 0]])
    A = sp.csr_matrix((np.ones(i.size), (i, j)), shape=(nv, nv))
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int64)
