"""The plain heat method end to end in FP64 (test infrastructure only).

Steps (Algorithm 1 of the paper, with the direct solves of the original
heat method that the paper's iterations replace):

1. assembly: cotangent stiffness K, lumped areas A, t = m h^2 (Eq. 27);
2. diffusion: (diag(A) + t K) u = u_0 (Eq. 4), range-safe: one sparse LU of
   the gauge-scaled system up to GAUGE_MAX_V vertices, banded sparse LU
   above (both exact routes of :mod:`oracle.diffusion`);
3. normalisation: h_f = -grad u / |grad u| (Eq. 3);
4. Poisson: face form K d = r, or the edge-form variant L_E d = b_E, with
   d = 0 at every source: sparse LU up to 200,000 vertices, above that CG
   with a multigrid preconditioner to relative residual 1e-10 (raises if it
   does not get there).

Also returns the breadth-first sets and pairing (Eq. 6, Sec. 3.3) so that
tests can drive the integration steps.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import assembly, bfs, diffusion, gradient, mesh, multigrid, poisson


GAUGE_MAX_V = 1_000_000     # whole-mesh LU of the gauge-scaled diffusion up to here
MG_MIN_V = 200_000          # multigrid-preconditioned CG Poisson above this


@dataclass
class HeatResult:
    t: float
    hbar: float
    logu: np.ndarray
    h: np.ndarray
    d: np.ndarray
    level: np.ndarray
    parent: np.ndarray
    topo: mesh.Topology
    diffusion_route: str = ""
    poisson_iters: int = 0          # multigrid-CG iterations (0: sparse LU)
    poisson_residual: float = 0.0   # its final relative residual


def prepare(verts, tris):
    topo = mesh.build_topology(tris, verts.shape[0])
    K = assembly.cotan_stiffness(verts, tris)
    A = assembly.lumped_areas(verts, tris)
    hbar = assembly.mean_edge_length(verts, topo.edges)
    return topo, K, A, hbar


def heat_method(verts, tris, sources, m: float = 1.0, t: float | None = None,
                form: str = "face", banded: bool = True, diffusion_route: str = "auto") -> HeatResult:
    """diffusion_route: "gauge" (whole-mesh LU of the gauge-scaled system),
    "bands" (banded LU), or "auto" (gauge up to GAUGE_MAX_V vertices)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    sources = np.unique(np.asarray(sources, dtype=np.int64))
    topo, K, A, hbar = prepare(verts, tris)
    if t is None or t <= 0:
        t = m * hbar * hbar
    M = diffusion.heat_matrix(K, A, t)
    large = verts.shape[0] > MG_MIN_V
    route = diffusion_route
    if route == "auto":
        route = "gauge" if verts.shape[0] <= GAUGE_MAX_V else "bands"
    if not banded:
        route = "plain"
        logu = diffusion.solve_log(M, sources, band_rings=10 ** 9)
    elif route == "gauge":
        psi = diffusion.gauge_potential(M, verts, topo.edges, t, sources)
        logu = diffusion.solve_log_gauge(M, sources, psi)
    elif route == "bands" and large:
        logu = diffusion.solve_log(M, sources, band_rings=40, margin_rings=40)
    elif route == "bands":
        logu = diffusion.solve_log(M, sources)
    else:
        raise ValueError(diffusion_route)
    h = gradient.normalized_field(verts, tris, logu)
    reach = np.isfinite(logu)
    rp, col = mesh.vertex_adjacency(verts.shape[0], topo.edges)
    Ps = multigrid.subdivision_prolongations(verts.shape[0], rp, col) if large else []
    pit, pres = 0, 0.0
    if form == "face":
        if Ps and reach.all():
            d, pit, pres = multigrid.dirichlet_solve_mg(K, poisson.face_rhs(verts, tris, h), sources, Ps)
        else:
            d = poisson.poisson_face(verts, tris, h, sources, reach)
    elif form == "edge":
        if Ps and reach.all():
            L, bE = poisson.edge_system(verts, tris, topo, h)
            d, pit, pres = multigrid.dirichlet_solve_mg(L, bE, sources, Ps)
        else:
            d = poisson.poisson_edge(verts, tris, topo, h, sources, reach)
    else:
        raise ValueError(form)
    level, parent = bfs.bfs_levels_vec(verts.shape[0], rp, col, sources)
    return HeatResult(t=t, hbar=hbar, logu=logu, h=h, d=d, level=level,
                      parent=parent, topo=topo, diffusion_route=route, poisson_iters=pit,
                      poisson_residual=pres)
