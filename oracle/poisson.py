"""The heat method's Poisson step (Sec. 3.2) -- test infrastructure only.

Face form.  The distance is the scalar field whose face gradients are
closest to the normalised field in the area-weighted least-squares sense,
min_d sum_f A_f |grad d|_f - h_f|^2.  Its normal equations are K d = r with
K the cotangent stiffness and r_i = sum_f A_f grad phi_i|_f . h_f (the
integrated divergence of h, up to sign).  On a disk or a genus-0 surface this
is also the minimiser of the constrained problem Eqs. 9-10 (compatible edge
projections make the field a gradient, Sec. 4.2 remark), so converged face
ADMM followed by integration reproduces it.

Edge form (the reading of Sec. 4.1 on a genus-0 surface): closed edge
differences are exact, x = D d, so Eqs. 19-20 become
min_d 1/2 sum_f sum_{(i,j) in f} (d_j - d_i - h_f.(p_j - p_i))^2 with normal
equations L_E d = b_E: L_E the graph Laplacian with edge weight |H_e| and
b_E,i = sum_{f ni i} sum_{j in f, j != i} h_f.(p_i - p_j).  This differs from
the face form unless the mesh is equilateral.

Sources.  One source: the paper shifts d so that it vanishes at the source.
Several sources: d = 0 at every source (the optimum of the path-constrained
problem of Eqs. 24-25, shifted so the common source value is zero).  Both are
the Dirichlet problem on the non-source vertices, solved by sparse LU.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assembly import cotan_stiffness, gradient_operator, face_geometry


def face_rhs(verts, tris, h) -> np.ndarray:
    """r = grad^T diag(A_f) h, i.e. r_i = sum_f A_f grad phi_i|_f . h_f."""
    Gop = gradient_operator(verts, tris)
    area, _, _ = face_geometry(verts, tris)
    return Gop.T @ (np.repeat(area, 3) * h.reshape(-1))


def edge_system(verts, tris, topo, h):
    """(L_E, b_E) of the edge-form variant."""
    nv = verts.shape[0]
    w = topo.edge_nfaces.astype(np.float64)
    a, b = topo.edges[:, 0], topo.edges[:, 1]
    off = sp.csr_matrix((np.concatenate([-w, -w]), (np.concatenate([a, b]), np.concatenate([b, a]))),
                        shape=(nv, nv))
    L = (sp.diags(-np.asarray(off.sum(axis=1)).ravel()) + off).tocsr()
    bE = np.zeros(nv)
    for k in range(3):
        i = tris[:, k]
        for kk in (1, 2):
            j = tris[:, (k + kk) % 3]
            np.add.at(bE, i, np.einsum("fc,fc->f", h, verts[i] - verts[j]))
    return L, bE


def dirichlet_solve(L: sp.spmatrix, rhs: np.ndarray, sources, reach=None) -> np.ndarray:
    """Solve L d = rhs with d = 0 at the sources (rows/columns eliminated).
    Vertices outside ``reach`` (a boolean mask) get +inf."""
    nv = L.shape[0]
    fixed = np.zeros(nv, dtype=bool)
    fixed[np.asarray(sources)] = True
    if reach is None:
        reach = np.ones(nv, dtype=bool)
    free = np.flatnonzero(~fixed & reach)
    d = np.full(nv, np.inf)
    d[np.asarray(sources)] = 0.0
    Lc = L.tocsr()
    Lff = Lc[free][:, free].tocsc()
    lu = spla.splu(Lff, permc_spec="COLAMD", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    d[free] = lu.solve(rhs[free])
    return d


def poisson_face(verts, tris, h, sources, reach=None) -> np.ndarray:
    """Face-form distance: K d = r, d = 0 at the sources."""
    K = cotan_stiffness(verts, tris)
    return dirichlet_solve(K, face_rhs(verts, tris, h), sources, reach)


def poisson_edge(verts, tris, topo, h, sources, reach=None) -> np.ndarray:
    """Edge-form distance: L_E d = b_E, d = 0 at the sources."""
    L, bE = edge_system(verts, tris, topo, h)
    return dirichlet_solve(L, bE, sources, reach)
