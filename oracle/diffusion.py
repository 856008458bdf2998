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
Green's function over those rings, provided nothing beyond the cut holds a
larger u than the band -- which hop rings do not guarantee far from the
sources (the hop count overestimates distance by up to 2/sqrt(3) depending
on direction).  A refinement therefore re-solves with bands in the order of
the values themselves, taken from the previous pass, until the result
confirms its own windows (:func:`solve_log`); the pins check it against an
independent 80-bit iteration and a deliberately poor first pass.  One band
(the whole mesh, no scaling) is the plain FP64 solve.  The result is log u.

Reference iteration (:func:`gauss_seidel_bfs`): the paper's breadth-first
Gauss-Seidel of Eqs. 6-7 -- the vertex sets D_i are swept in order, all
vertices of one set updated simultaneously from the latest neighbour values.
It is the paper's algorithm, kept for convergence studies; the exact solve is
the oracle's answer.

Second exact route (:func:`solve_log_gauge`): one sparse LU of the whole
system after a diagonal similarity.  With E = diag(e^psi) for a potential psi
that grows at least as fast as log u falls, v = E u solves
(E M E^-1) v = E u_0 and stays inside the FP64 range.  A similarity by a
positive diagonal keeps an M-matrix an M-matrix and leaves the diagonal of
the inverse (hence every pivot of a diagonal-pivot LU) unchanged, so the
factorisation and both triangular solves add terms of one sign only and the
result is accurate componentwise.  It shares nothing with the banded solve
but the matrix, so the two pin each other at sizes where both run.
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


def _solve_window(M, U, core, solved, out, u0):
    """Solve the principal subsystem on the vertex set U (indices) with the
    solved vertices as data and zero beyond U; write log u on U[core]."""
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
    with np.errstate(divide="ignore"):
        out[U[core]] = np.log(w[core]) + scale
    solved[U[core]] = True


def _ring_pass(M, sources, lev, B, G):
    nv = M.shape[0]
    out = np.full(nv, -np.inf)
    u0 = np.zeros(nv)
    u0[sources] = 1.0
    solved = np.zeros(nv, dtype=bool)
    for lo in range(0, int(lev.max()) + 1, B):
        U = np.flatnonzero((lev >= lo) & (lev < lo + B + G))
        _solve_window(M, U, lev[U] < lo + B, solved, out, u0)
    return out


def _value_pass(M, sources, psi, delta, gamma, check):
    """Bands by the estimate psi of log u: band = the unsolved vertices with
    psi in [top - delta, top], window = those with psi >= top - delta - gamma.
    Returns (log u, ok) with ok = every vertex left out of a band's window
    ends at least `check` nats below that band's smallest value."""
    nv = M.shape[0]
    out = np.full(nv, -np.inf)
    u0 = np.zeros(nv)
    u0[sources] = 1.0
    solved = np.zeros(nv, dtype=bool)
    reach = np.isfinite(psi)
    order = np.flatnonzero(reach)[np.argsort(-psi[reach], kind="stable")]
    ps = psi[order]
    bands = []
    i = 0
    while i < order.size:
        top = ps[i]
        j = i + int(np.searchsorted(-ps[i:], -(top - delta), side="right"))
        k = i + int(np.searchsorted(-ps[i:], -(top - delta - gamma), side="right"))
        U = order[i:k]
        _solve_window(M, U, np.arange(U.size) < j - i, solved, out, u0)
        bands.append((i, j, k))
        i = j
    # a-posteriori: vertices beyond window k of band (i, j) are order[k:]
    tail_max = np.maximum.accumulate(out[order][::-1])[::-1] if order.size else np.zeros(0)
    ok = True
    for i, j, k in bands:
        if k < order.size and tail_max[k] > out[order[i:j]].min() - check:
            ok = False
    return out, ok


def solve_log(M: sp.csr_matrix, sources, band_rings: int | None = None,
              margin_rings: int | None = None, refine: bool = True,
              value_band: float = 100.0, value_margin: float = 60.0,
              check_nats: float = 40.0, max_refine: int = 6) -> np.ndarray:
    """log u for M u = u_0 (u_0 = 1 at each source).  Unreachable vertices
    get log u = -inf.

    First pass: bands of breadth-first rings.  band_rings=None picks
    B = floor(300 / beta) (see the module text); the margin defaults to B
    rings.  Hop rings are only a proxy for the decay of u: on a near
    equilateral lattice the hop count overestimates the distance by up to
    2/sqrt(3) depending on direction, so far from the sources a vertex
    several dozen rings out can hold a larger u than some vertices of the
    band, and cutting it off is then not negligible.

    Refinement (refine=True): bands in value order instead -- sorted by the
    previous pass's log u, each band spans value_band nats and its window
    extends value_margin nats further down, so every cut-off vertex holds a
    u e^-value_margin below the band's smallest by the previous estimate.
    Passes repeat until the result confirms its own windows: every vertex
    outside a band's window ends at least check_nats below the band's
    smallest value (the cut then changes the band relatively by less than
    e^-check_nats times the Green's function decay across the window)."""
    sources = np.unique(np.asarray(sources, dtype=np.int64))
    M = M.tocsr()
    lev = hop_levels(M, sources)
    if band_rings is None:
        C = M.tocoo()
        off = C.row != C.col
        c = np.abs(C.data[off]) / M.diagonal()[C.row[off]]
        beta = float(np.log(1.0 / c[c > 0]).max()) if np.any(c > 0) else 1.0
        band_rings = max(1, int(300.0 // beta))
    B = int(band_rings)
    G = int(margin_rings) if margin_rings is not None else B
    out = _ring_pass(M, sources, lev, B, G)
    if not refine:
        return out
    for _ in range(max_refine):
        out, ok = _value_pass(M, sources, out, value_band, value_margin, check_nats)
        if ok:
            return out
    raise RuntimeError("value-band refinement did not confirm its windows")


def gauge_potential(M: sp.csr_matrix, verts, edges, t: float, sources) -> np.ndarray:
    """psi for :func:`solve_log_gauge`: shortest-path distance from the
    sources with edge weight min(ln(1/c), l/sqrt(t)), where l is the edge's
    length and c = t theta / M_jj the smaller of its two coupling ratios.

    ln(1/c) bounds the fall of log u across the edge (u_j >= c_jk u_k for an
    M-matrix), so psi >= -log u + log u_s wherever that term is the minimum;
    l/sqrt(t) is the continuum decay rate of the 1-D heat kernel
    e^(-|x|/sqrt(t)), which the discrete solution does not exceed on
    reasonable meshes (the caller checks the range of the scaled solution,
    so a potential that falls short fails loudly instead of underflowing)."""
    from scipy.sparse.csgraph import dijkstra
    M = M.tocsr()
    a, b = np.asarray(edges[:, 0]), np.asarray(edges[:, 1])
    mab = -np.asarray(M[a, b]).ravel()          # t theta_ab (> 0 off the diagonal)
    diag = M.diagonal()
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.minimum(mab / diag[a], mab / diag[b])
        w_c = np.where(c > 0, -np.log(np.where(c > 0, c, 1.0)), np.inf)
    length = np.linalg.norm(np.asarray(verts)[a] - np.asarray(verts)[b], axis=1)
    w = np.minimum(w_c, length / np.sqrt(t))
    nv = M.shape[0]
    G = sp.csr_matrix((np.concatenate([w, w]), (np.concatenate([a, b]), np.concatenate([b, a]))),
                      shape=(nv, nv))
    return dijkstra(G, indices=np.unique(np.asarray(sources)), min_only=True)


def solve_log_gauge(M: sp.csr_matrix, sources, psi: np.ndarray) -> np.ndarray:
    """log u for M u = u_0 by one sparse LU of E M E^-1 (E = diag(e^psi)),
    diagonal pivots, then log u = log v - psi.  Vertices with psi = inf (not
    connected to a source) get -inf.  Raises if the scaled solution leaves
    [1e-280, 1e280], i.e. if psi does not keep it inside the FP64 range."""
    sources = np.unique(np.asarray(sources, dtype=np.int64))
    M = M.tocsr()
    nv = M.shape[0]
    out = np.full(nv, -np.inf)
    reach = np.flatnonzero(np.isfinite(psi))
    if reach.size == 0:
        return out
    pr = psi[reach]
    C = M[reach][:, reach].tocoo()
    S = sp.csc_matrix((C.data * np.exp(pr[C.row] - pr[C.col]), (C.row, C.col)), shape=(reach.size,) * 2)
    rhs = np.zeros(reach.size)
    pos = np.searchsorted(reach, sources)
    rhs[pos] = np.exp(pr[pos])
    lu = spla.splu(S, permc_spec="COLAMD", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    v = lu.solve(rhs)
    if not (np.all(np.isfinite(v)) and v.min() > 1e-280 and v.max() < 1e280):
        raise RuntimeError(f"gauge-scaled diffusion left the FP64 range: v in [{v.min():.3e}, {v.max():.3e}]")
    out[reach] = np.log(v) - pr
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
