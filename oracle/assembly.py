"""Discrete operators of the heat method in FP64 (test infrastructure only).

* face areas A_f and corner cotangents;
* cotangent weights theta_jk = (cot alpha_jk + cot beta_jk)/2 (one term on a
  boundary edge) -- the coefficients of the cotangent Laplacian L_c in Eq. 4
  and the update of Eq. 7;
* the PSD stiffness K = -L_c (K_jk = -theta_jk, K_jj = sum_k theta_jk);
* lumped vertex areas A_j = (1/3) sum of incident face areas (Sec. 3.1, below
  Eq. 7);
* mean edge length h over unique edges, giving t = m h^2 (Eq. 27);
* the face gradient operator grad: R^V -> R^{3F} of piecewise-linear
  functions, grad u|_f = (1/(2 A_f)) sum_i u_i (N_f x e_i) with e_i the CCW
  edge opposite corner i (used by Eq. 3).

The factor 1/2 in theta is a reading: the paper names theta_jk "the
coefficient of v_k for the cotangent Laplacian at v_j" without a factor.  With
the 1/2, (1/A_j) sum_k theta_jk (u_k - u_j) reproduces Laplace(x^2) = 2 on an
equilateral lattice (pinned in the tests).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def face_geometry(verts: np.ndarray, tris: np.ndarray):
    """Per face: area A_f (float64[F]), unit normal (float64[F,3]) and the
    cotangent of the angle at each corner (float64[F,3])."""
    p0 = verts[tris[:, 0]]
    p1 = verts[tris[:, 1]]
    p2 = verts[tris[:, 2]]
    n = np.cross(p1 - p0, p2 - p0)
    dbl = np.linalg.norm(n, axis=1)           # 2 A_f
    area = 0.5 * dbl
    normal = n / dbl[:, None]
    cots = np.empty((tris.shape[0], 3))
    corners = ((p0, p1, p2), (p1, p2, p0), (p2, p0, p1))
    for k, (pa, pb, pc) in enumerate(corners):
        u = pb - pa
        v = pc - pa
        cots[:, k] = np.einsum("ij,ij->i", u, v) / dbl
    return area, normal, cots


def cotan_stiffness(verts: np.ndarray, tris: np.ndarray) -> sp.csr_matrix:
    """K = -L_c with off-diagonals -theta_jk, theta_jk = (cot a + cot b)/2.

    The corner cotangent at vertex k of a face weighs the opposite edge; each
    face contributes cot/2 to that edge.
    """
    nv = verts.shape[0]
    _, _, cots = face_geometry(verts, tris)
    i_list, j_list, w_list = [], [], []
    for k in range(3):
        a = tris[:, (k + 1) % 3]
        b = tris[:, (k + 2) % 3]
        w = 0.5 * cots[:, k]
        i_list += [a, b]
        j_list += [b, a]
        w_list += [w, w]
    i = np.concatenate(i_list)
    j = np.concatenate(j_list)
    w = np.concatenate(w_list)
    theta = sp.csr_matrix((w, (i, j)), shape=(nv, nv))
    theta.sum_duplicates()
    diag = np.asarray(theta.sum(axis=1)).ravel()
    K = sp.diags(diag) - theta
    return K.tocsr()


def lumped_areas(verts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """A_j = one third of the total area of the faces incident to v_j."""
    area, _, _ = face_geometry(verts, tris)
    A = np.zeros(verts.shape[0])
    for k in range(3):
        np.add.at(A, tris[:, k], area / 3.0)
    return A


def mean_edge_length(verts: np.ndarray, edges: np.ndarray) -> float:
    """Arithmetic mean of |p_a - p_b| over the unique edges (h of Eq. 27)."""
    return float(np.linalg.norm(verts[edges[:, 0]] - verts[edges[:, 1]], axis=1).mean())


def gradient_operator(verts: np.ndarray, tris: np.ndarray) -> sp.csr_matrix:
    """Sparse (3F x V) matrix mapping vertex values to face gradients, rows
    ordered (f, component): grad u|_f = (1/(2A_f)) sum_i u_i N_f x e_i."""
    nf = tris.shape[0]
    nv = verts.shape[0]
    area, normal, _ = face_geometry(verts, tris)
    rows, cols, vals = [], [], []
    for k in range(3):
        pa = verts[tris[:, (k + 1) % 3]]
        pb = verts[tris[:, (k + 2) % 3]]
        e = pb - pa                               # CCW edge opposite corner k
        gk = np.cross(normal, e) / (2.0 * area)[:, None]
        for c in range(3):
            rows.append(3 * np.arange(nf) + c)
            cols.append(tris[:, k])
            vals.append(gk[:, c])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * nf, nv))
