"""Conjugate gradients with a multigrid preconditioner for the oracle's large
Poisson solves (test infrastructure only).

The heat method's Poisson step (Sec. 3.2) is a sparse SPD system once the
sources are fixed; sparse LU stops being practical beyond a few hundred
thousand vertices, so large meshes use preconditioned CG run to a relative
residual of 1e-10 (the answer is the linear system's solution; the
preconditioner only changes how fast CG gets there).

Hierarchy: meshes made by repeated 1->4 midpoint subdivision list their
coarse vertices first (the icosphere generator does), and every fine-only
vertex has exactly two coarse neighbours, the ends of the coarse edge it
splits.  Prolongation copies coarse values and averages the two ends at
midpoints; coarse operators are Galerkin products P^T A P; smoothing is
damped Jacobi (symmetric V-cycle, so CG stays valid); the coarsest level is
solved by sparse LU.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def subdivision_prolongations(nv: int, row_ptr, col, min_coarse: int = 700):
    """Prolongations of the icosphere hierarchy reconstructed from the
    adjacency (CSR) of the finest mesh; returns [P_L, P_{L-1}, ...] from the
    finest level down, or [] if the mesh is not of that form."""
    sizes = []
    n = nv
    while n > min_coarse and (n - 2) % 40 == 0 and n > 12:
        c = (n - 2) // 4 + 2
        sizes.append((n, c))
        n = c
    if not sizes:
        return []
    Ps = []
    rp, cl = np.asarray(row_ptr), np.asarray(col)
    for (nf_, nc_) in sizes:
        # the two parents of a fine-only vertex are its neighbours of index
        # < n_c; the parent pairs are the edges of the coarser mesh
        deg = np.diff(rp)
        src = np.repeat(np.arange(nf_), deg)
        keep = (src >= nc_) & (cl < nc_)
        pr, pc = src[keep], cl[keep]
        cnt = np.bincount(pr - nc_, minlength=nf_ - nc_)
        if not np.all(cnt == 2):
            return []
        rows = np.arange(nc_)
        P = sp.csr_matrix((np.concatenate([np.ones(nc_), np.full(pr.size, 0.5)]),
                           (np.concatenate([rows, pr]), np.concatenate([rows, pc]))), shape=(nf_, nc_))
        Ps.append(P)
        # adjacency of the coarser mesh from the parent pairs
        order = np.argsort(pr, kind="stable")
        a, b = pc[order][0::2], pc[order][1::2]
        G = sp.csr_matrix((np.ones(2 * a.size), (np.concatenate([a, b]), np.concatenate([b, a]))),
                          shape=(nc_, nc_))
        G.sum_duplicates()
        rp, cl = G.indptr, G.indices
    return Ps


class VCycle:
    def __init__(self, A: sp.csr_matrix, Ps, nu: int = 2, omega: float = 0.7):
        self.levels = [A.tocsr()]
        self.Ps = Ps
        for P in Ps:
            Ac = (P.T @ self.levels[-1] @ P).tocsr()
            self.levels.append(Ac)
        self.dinv = [1.0 / L.diagonal() for L in self.levels]
        self.coarse = spla.splu(self.levels[-1].tocsc())
        self.nu, self.omega = nu, omega

    def _cycle(self, l, b):
        A = self.levels[l]
        if l == len(self.levels) - 1:
            return self.coarse.solve(b)
        x = np.zeros_like(b)
        for _ in range(self.nu):
            x += self.omega * self.dinv[l] * (b - A @ x)
        r = b - A @ x
        xc = self._cycle(l + 1, self.Ps[l].T @ r)
        x += self.Ps[l] @ xc
        for _ in range(self.nu):
            x += self.omega * self.dinv[l] * (b - A @ x)
        return x

    def __call__(self, b):
        return self._cycle(0, b)


class NotConverged(RuntimeError):
    pass


def pcg(A, b, M, rtol: float = 1e-10, maxiter: int = 500):
    """Plain preconditioned conjugate gradients; returns (x, iterations,
    final relative residual).  Raises NotConverged if the relative residual
    is still above rtol after maxiter iterations."""
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    for it in range(1, maxiter + 1):
        Ap = A @ p
        a = rz / (p @ Ap)
        x += a * p
        r -= a * Ap
        res = np.linalg.norm(r) / nb
        if res <= rtol:
            return x, it, res
        z = M(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise NotConverged(f"pcg: relative residual {res:.3e} > {rtol:.1e} after {maxiter} iterations")


def dirichlet_solve_mg(L: sp.spmatrix, rhs: np.ndarray, sources, Ps, rtol: float = 1e-10):
    """Solve L d = rhs with d = 0 at the sources by multigrid-preconditioned
    CG; the prolongations are restricted to the free vertices.  Returns
    (d, iterations, relative residual |rhs_F - L_FF d_F| / |rhs_F| recomputed
    from d), and raises NotConverged if that residual exceeds 10 rtol."""
    nv = L.shape[0]
    fixed = np.zeros(nv, dtype=bool)
    fixed[np.asarray(sources)] = True
    free = np.flatnonzero(~fixed)
    Lc = L.tocsr()
    Aff = Lc[free][:, free].tocsr()
    Ps_f = [Ps[0][free]] + list(Ps[1:]) if Ps else []
    M = VCycle(Aff, Ps_f) if Ps_f else (lambda b: b / Aff.diagonal())
    x, it, _ = pcg(Aff, rhs[free], M, rtol=rtol)
    bf = rhs[free]
    res = float(np.linalg.norm(bf - Aff @ x) / np.linalg.norm(bf))
    if res > 10.0 * rtol:
        raise NotConverged(f"dirichlet_solve_mg: true relative residual {res:.3e}")
    d = np.zeros(nv)
    d[free] = x
    return d, it, res
