"""Heat diffusion of the heat method (test infrastructure only).

The backward-Euler step of Eq. 4, (A - t L_c) u = u_0 with u_0 = 1 at every
source vertex (Sec. 3.1; several sources use the generalised Dirac of
Sec. 5.2), written with the PSD stiffness K = -L_c as

        (diag(A) + t K) u = u_0 .

Exact solve (:func:`solve_log`).  For small t the solution decays by about
e^-1 per ring of vertices, so on large meshes it leaves the FP64 range.  The
paper does not say how it handles this.  The oracle solves the same linear
system band by band over the breadth-first rings (hop distance to the
sources).  For an M-matrix, u_j >= c_jk u_k with c_jk = t theta_jk / M_jj,
so u falls by at most beta = max_jk ln(1/c_jk) nats per ring; bands of
B = floor(300 / beta) rings therefore span at most 300 nats.  Band b (rings
[bB, (b+1)B)) is solved together with the next B rings as the principal
subsystem M_UU w = u_0|_U - M_UI u_I, with the already solved inner rings I
as data and zero beyond, in plain FP64 after dividing by the largest inner
value.  Principal submatrices of an M-matrix are M-matrices: their LU with
diagonal pivots and the right-hand side above involve no cancellation, so
each band is accurate componentwise and relatively.  Cutting the system B
rings further out changes the band's values by a factor decaying like the
Green's function over those rings (far below FP64 rounding for the B above;
the pins check it against an independent 80-bit iteration).  One band (the
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


def heat_matrix(K: sp.spmatrix, A: np.ndarray, t: float) -> sp.csr_matrix:
    """M = diag(A) + t K, the matrix of Eq. 4 (K = -L_c)."""
    return (sp.diags(A) + t * K).tocsr()


def hop_levels(M: sp.spmatrix, sources) -> np.ndarray:
    """Breadth-first ring index of every vertex (hop distance to the source
    set over the sparsity graph of M); -1 where unreachable."""
    from scipy.sparse.csgraph import breadth_first_order
    G = M.tocsr()
    nv = G.shape[0]
    lev = np.full(nv, -1, dtype=np.int64)
    front = np.unique(np.asarray(sources, dtype=np.int64))
    lev[front] = 0
    indptr, indices = G.indptr, G.indices
    i = 0
    while front.size:
        i += 1
        nb = np.unique(np.concatenate([indices[indptr[v]:indptr[v + 1]] for v in front]))
        nb = nb[lev[nb] < 0]
        lev[nb] = i
        front = nb
    return lev


def solve_log(M: sp.csr_matrix, sources, band_rings: int | None = None,
              margin_rings: int | None = None) -> np.ndarray:
    """log u for M u = u_0 (u_0 = 1 at each source), marching outward over
    bands of breadth-first rings.  Unreachable vertices get log u = -inf.
    band_rings=None picks B = floor(300 / beta) (see the module text); the
    margin defaults to B rings.  At t = m hbar^2 the truncation error falls by
    about e^(-2 / sqrt(m)) per margin ring, so the default margin is ample for
    m up to ~30."""
    nv = M.shape[0]
    sources = np.unique(np.asarray(sources, dtype=np.int64))
    M = M.tocsr()
    lev = hop_levels(M, sources)
    out = np.full(nv, -np.inf)
    if band_rings is None:
        C = M.tocoo()
        off = C.row != C.col
        c = np.abs(C.data[off]) / M.diagonal()[C.row[off]]
        beta = float(np.log(1.0 / c[c > 0]).max()) if np.any(c > 0) else 1.0
        band_rings = max(1, int(300.0 // beta))
    B = int(band_rings)
    G = int(margin_rings) if margin_rings is not None else B
    depth = int(lev.max())
    u0 = np.zeros(nv)
    u0[sources] = 1.0
    solved = np.zeros(nv, dtype=bool)
    for lo in range(0, depth + 1, B):
        U = np.flatnonzero((lev >= lo) & (lev < lo + B + G))
        core = (lev >= lo) & (lev < lo + B)
        MU = M[U]
        rows = MU.tocoo()
        known = solved[rows.col]
        scale = out[rows.col[known]].max() if known.any() else 0.0
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
