"""Heat diffusion of the heat method (test infrastructure only).

The backward-Euler step of Eq. 4, (A - t L_c) u = u_0 with u_0 = 1 at every
source vertex (Sec. 3.1; several sources use the generalised Dirac of
Sec. 5.2), written with the PSD stiffness K = -L_c as

        (diag(A) + t K) u = u_0 .

Exact solve (:func:`solve_log`).  For small t the solution decays by about
e^-1 per ring of vertices, so on large meshes it leaves the FP64 range.  The
paper does not say how it handles this.  The oracle solves the same linear
system in bands of the potential psi_j = (shortest edge-path length from the
sources to v_j)/sqrt(t), which bounds the decay of u from above: band b holds
the vertices with psi in [b R, (b+1) R).  Band b is solved together with a
margin of the next ``margin`` units of psi as the principal subsystem
M_UU w = u_0|_U - M_UI u_I, with the already solved inner vertices I as data
and zero beyond the margin, in plain FP64 after dividing by the largest inner
value.  Principal submatrices of the M-matrix M are M-matrices: their LU with
diagonal pivots and the right-hand side above involve no cancellation, so each
band is accurate componentwise and relatively.  Cutting the system at the
outer edge of the margin changes the band's values by a factor of order
exp(-margin) or faster; margin = 60 puts that far below FP64 rounding.  One band (the
whole mesh, no scaling) is the plain FP64 solve.  The result is log u.

Reference iteration (:func:`gauss_seidel_bfs`): the paper's breadth-first
Gauss-Seidel of Eqs. 6-7 -- the vertex sets D_i are swept in order, all
vertices of one set updated simultaneously from the latest neighbour values.
It is the paper's algorithm, kept for convergence studies; the exact solve is
the oracle's answer.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import dijkstra


def heat_matrix(K: sp.spmatrix, A: np.ndarray, t: float) -> sp.csr_matrix:
    """M = diag(A) + t K, the matrix of Eq. 4 (K = -L_c)."""
    return (sp.diags(A) + t * K).tocsr()


def edge_path_potential(verts, edges, sources, t: float) -> np.ndarray:
    """psi_j = (shortest edge-path length from the source set)/sqrt(t)."""
    nv = verts.shape[0]
    w = np.linalg.norm(verts[edges[:, 0]] - verts[edges[:, 1]], axis=1)
    G = sp.csr_matrix((np.concatenate([w, w]),
                       (np.concatenate([edges[:, 0], edges[:, 1]]),
                        np.concatenate([edges[:, 1], edges[:, 0]]))), shape=(nv, nv))
    dist = dijkstra(G, directed=False, indices=np.asarray(sources), min_only=True)
    return dist / np.sqrt(t)


def solve_log(M: sp.csr_matrix, sources, psi: np.ndarray | None = None,
              band: float = 200.0, margin: float = 60.0) -> np.ndarray:
    """log u for M u = u_0 (u_0 = 1 at each source), marching outward over
    bands of psi.  Unreachable vertices (psi = inf) get log u = -inf.  With
    psi = None the whole mesh is one band (plain FP64)."""
    nv = M.shape[0]
    sources = np.unique(np.asarray(sources, dtype=np.int64))
    if psi is None:
        psi = np.zeros(nv)
    M = M.tocsr()
    out = np.full(nv, -np.inf)
    reach = np.isfinite(psi)
    if not reach.any():
        return out
    pmax = psi[reach].max()
    nb = int(pmax // band) + 1
    u0 = np.zeros(nv)
    u0[sources] = 1.0
    solved = np.zeros(nv, dtype=bool)
    for b in range(nb):
        lo, hi = b * band, (b + 1) * band
        U = np.flatnonzero(reach & (psi >= lo) & (psi < hi + margin))
        core = reach & (psi >= lo) & (psi < hi)
        if not core.any():
            continue
        MU = M[U]
        rows = MU.tocoo()
        known = solved[rows.col]
        scale = 0.0
        if known.any():
            scale = out[rows.col[known]].max()
        rhs = np.zeros(U.size)
        src_in = u0[U] > 0
        if src_in.any():
            rhs[src_in] = np.exp(-scale)
        if known.any():
            contrib = -rows.data[known] * np.exp(out[rows.col[known]] - scale)
            rhs += np.bincount(rows.row[known], weights=contrib, minlength=U.size)
        S = MU[:, U].tocsc()
        lu = spla.splu(S, permc_spec="COLAMD", diag_pivot_thresh=0.0,
                       options=dict(SymmetricMode=True))
        w = lu.solve(rhs)
        keep = core[U]
        with np.errstate(divide="ignore"):
            out[U[keep]] = np.log(w[keep]) + scale
        solved[U[keep]] = True
    return out


def gauss_seidel_bfs(K: sp.csr_matrix, A: np.ndarray, t: float, sources,
                     levels: np.ndarray, n_outer: int, u_init=None) -> np.ndarray:
    """The paper's breadth-first Gauss-Seidel (Eqs. 6-7), n_outer outer
    iterations; plain FP64 (use on meshes where u stays in range).

    Each outer iteration visits D_0, D_1, ... in order; the vertices of one
    set are updated together by Eq. 7 from the values current before the set
    is touched.
    """
    nv = A.size
    Kc = K.tocsr()
    diag = Kc.diagonal()
    theta = -(Kc - sp.diags(diag)).tocsr()          # off-diagonal theta_jk >= ...
    u0 = np.zeros(nv)
    u0[np.asarray(sources)] = 1.0
    u = np.zeros(nv) if u_init is None else np.array(u_init, dtype=np.float64)
    denom = A + t * diag
    maxlev = int(levels.max())
    sets = [np.flatnonzero(levels == i) for i in range(maxlev + 1)]
    rows = [theta[s] for s in sets]
    for _ in range(n_outer):
        for s, Ts in zip(sets, rows):
            u[s] = (u0[s] + t * (Ts @ u)) / denom[s]
    return u


def jacobi(K: sp.csr_matrix, A: np.ndarray, t: float, sources, n_sweeps: int,
           u_init=None) -> np.ndarray:
    """Plain Jacobi sweeps of Eq. 7 (all vertices from the previous sweep)."""
    nv = A.size
    Kc = K.tocsr()
    diag = Kc.diagonal()
    theta = -(Kc - sp.diags(diag)).tocsr()
    u0 = np.zeros(nv)
    u0[np.asarray(sources)] = 1.0
    u = np.zeros(nv) if u_init is None else np.array(u_init, dtype=np.float64)
    denom = A + t * diag
    for _ in range(n_sweeps):
        u = (u0 + t * (theta @ u)) / denom
    return u
