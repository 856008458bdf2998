"""ADMM solvers of the gradient optimisation, in the paper's update order
(test infrastructure only).  FP64.

Face form (Sec. 3.2, Eqs. 9-16).  Per interior edge e with incident faces
(1, 2) there are auxiliary copies y_1, y_2 of the two face gradients and
duals lambda_1, lambda_2; M = diag(alpha), alpha = sqrt(face area of the
copy); mu = 100.  One iteration:

  Y-update  q_i = g_i - lambda_i/(mu alpha_i),
            y_1 = q_1 + A_2/(A_1+A_2) e (e.(q_2 - q_1)),
            y_2 = q_2 - A_1/(A_1+A_2) e (e.(q_2 - q_1))     (e: unit edge)
  G-update  g_i = (2 h_i + mu sum_k (y_k + lambda_k/(mu alpha_i)))
                  / (2 + mu |Y(i)|)
  l-update  lambda += mu M (Y - S G)

initialised with g = y = h, lambda = 0.  Residuals r_p = M(Y - SG) and
r_d = mu A S dG, where A is read as M^2 (face area per copy); stop when
|r_p| <= |M|_F eps1 and |r_d| <= |M|_F eps2 or after I_max iterations.

Edge form (Sec. 4.1, Eqs. 19-21).  Edge unknowns x_e, per-face copies w_f
and duals lambda_f (3 per face), targets Z, signs q_f of Eq. 20.  One
iteration:

  W-update  w_f = (I - q_f q_f^T / 3)(x_f - lambda_f/mu)
  X-update  x_e = sum_{h in H_e} (h_e + lambda_h + mu w_h) / (|H_e| (1 + mu))
  l-update  lambda += mu (W - R X)

initialised with lambda = 0, x_e = mean of its targets, w_f = Z_f.
Residuals r_p = W - RX, r_d = mu R dX.

Over-relaxation (optional, relax = alpha = 1 is the paper's iteration): the
standard over-relaxed ADMM of Boyd et al. (the ADMM survey the paper cites,
Sec. 3.4.3) replaces, in the second update and the dual update, the first
block's output by its mix with the previous second-block value:
y_hat = alpha y + (1 - alpha) S g (face form), w_hat = alpha w + (1 - alpha) R x
(edge form).  It has the same fixed points; alpha in (1, 2) typically
converges faster.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .assembly import face_geometry


# ------------------------------------------------------- closed-form steps
def y_update(q1, q2, ebar, A1, A2):
    """Face-form Y-update of one interior edge (Sec. 3.2): the minimiser of
    A_1|y_1 - q_1|^2 + A_2|y_2 - q_2|^2 subject to e.(y_1 - y_2) = 0."""
    s = np.einsum("...c,...c->...", ebar, q2 - q1)[..., None] * ebar
    w1 = (A2 / (A1 + A2))[..., None]
    w2 = (A1 / (A1 + A2))[..., None]
    return q1 + w1 * s, q2 - w2 * s


def g_update(h, acc_sum, count, mu):
    """Face-form G-update: g = (2h + mu sum_k (y_k + lambda_k/(mu alpha)))
    / (2 + mu |Y(i)|), with acc_sum the sum over the face's copies."""
    return (2.0 * h + mu * acc_sum) / (2.0 + mu * np.asarray(count, dtype=np.float64))[..., None]


def w_update(x_f, lam_f, q_f, mu):
    """Edge-form W-update: orthogonal projection of x_f - lambda_f/mu onto
    the plane q_f . w = 0, i.e. (I - q q^T/3)(x_f - lambda_f/mu)."""
    v = x_f - lam_f / mu
    return v - (np.einsum("...k,...k->...", q_f, v) / 3.0)[..., None] * q_f


def x_update(sum_h, sum_lam, sum_w, n_h, mu):
    """Edge-form X-update of Eq. 21 from the sums over the edge's copies."""
    return (sum_h + sum_lam + mu * sum_w) / (n_h * (1.0 + mu))


# ---------------------------------------------------------------- face form
@dataclass
class FaceADMMState:
    g: np.ndarray       # [F, 3]
    y: np.ndarray       # [2*Eint, 3]  rows (e,1),(e,2) interleaved
    lam: np.ndarray     # [2*Eint, 3]
    iters: int = 0
    r_primal: float = np.inf
    r_dual: float = np.inf
    kappa: list = field(default_factory=list)   # per source path (Eq. 24)


class FaceADMM:
    """Face-form ADMM.  `paths` (from :func:`source_paths`) adds the
    constraint of Eq. 24 for each path S: a group of copies y_j of the
    gradient of the face f_j chosen on each path edge, weighted by
    alpha = sqrt(A_{f_j}) like every copy, constrained to
    sum_j e_j . y_j = 0 (e_j the edge vector along the path).  Its Y-type
    update is the weighted projection
    y_j = q_j - (c / A_j) e_j,  c = sum_j e_j . q_j / sum_j |e_j|^2 / A_j,
    q_j = g_{f_j} - kappa_j / (mu alpha_j); the G-update of a face counts
    these copies among Y(i), and kappa_j += mu alpha_j (y_j - g_{f_j})."""

    def __init__(self, verts, tris, topo, h, mu: float = 100.0, relax: float = 1.0, paths=()):
        self.mu = mu
        self.relax = relax
        area, _, _ = face_geometry(verts, tris)
        interior = np.flatnonzero(topo.edge_nfaces == 2)
        self.faces = topo.edge_faces[interior].reshape(-1)          # f(k) per copy
        ev = verts[topo.edges[interior, 1]] - verts[topo.edges[interior, 0]]
        self.ebar = ev / np.linalg.norm(ev, axis=1, keepdims=True)
        self.A = area[self.faces]                                    # per copy
        self.alpha = np.sqrt(self.A)
        self.h = np.asarray(h, dtype=np.float64)
        self.nf = tris.shape[0]
        self.paths = [(p["face"], p["vec"], area[p["face"]]) for p in paths]
        pf = np.concatenate([f for f, _, _ in self.paths]) if self.paths else np.zeros(0, dtype=np.int64)
        self.count = (np.bincount(self.faces, minlength=self.nf)
                      + np.bincount(pf, minlength=self.nf)).astype(np.float64)
        self.normM = np.sqrt(self.A.sum())

    def init(self) -> FaceADMMState:
        return FaceADMMState(g=self.h.copy(), y=self.h[self.faces].copy(),
                             lam=np.zeros((self.faces.size, 3)),
                             kappa=[np.zeros((f.size, 3)) for f, _, _ in self.paths])

    def step(self, s: FaceADMMState) -> FaceADMMState:
        mu, al, A = self.mu, self.alpha, self.A
        q = s.g[self.faces] - s.lam / (mu * al)[:, None]
        y = np.empty_like(q)
        y[0::2], y[1::2] = y_update(q[0::2], q[1::2], self.ebar, A[0::2], A[1::2])
        yh = self.relax * y + (1.0 - self.relax) * s.g[self.faces]
        acc = yh + s.lam / (mu * al)[:, None]
        tot = np.zeros((self.nf, 3))
        for c in range(3):
            tot[:, c] = np.bincount(self.faces, weights=acc[:, c], minlength=self.nf)
        yhs = []
        for (f, vec, Ap), kap in zip(self.paths, s.kappa):
            ap = np.sqrt(Ap)
            qp = s.g[f] - kap / (mu * ap)[:, None]
            cc = np.sum(vec * qp) / np.sum(np.sum(vec * vec, axis=1) / Ap)
            yp = qp - (cc / Ap)[:, None] * vec
            yph = self.relax * yp + (1.0 - self.relax) * s.g[f]
            np.add.at(tot, f, yph + kap / (mu * ap)[:, None])
            yhs.append(yph)
        g = g_update(self.h, tot, self.count, mu)
        lam = s.lam + mu * al[:, None] * (yh - g[self.faces])
        kappa = [kap + mu * np.sqrt(Ap)[:, None] * (yph - g[f])
                 for (f, _, Ap), kap, yph in zip(self.paths, s.kappa, yhs)]
        r_p = np.linalg.norm(al[:, None] * (y - g[self.faces]))
        r_d = np.linalg.norm(mu * A[:, None] * (g - s.g)[self.faces])
        return FaceADMMState(g=g, y=y, lam=lam, iters=s.iters + 1, r_primal=r_p, r_dual=r_d, kappa=kappa)

    def run(self, iters: int, eps1: float = 0.0, eps2: float = 0.0, state=None):
        s = self.init() if state is None else state
        for _ in range(iters):
            s = self.step(s)
            if s.r_primal <= self.normM * eps1 and s.r_dual <= self.normM * eps2:
                break
        return s


# ---------------------------------------------------------------- edge form
@dataclass
class EdgeADMMState:
    x: np.ndarray       # [E]
    w: np.ndarray       # [F, 3]
    lam: np.ndarray     # [F, 3]
    iters: int = 0
    r_primal: float = np.inf
    r_dual: float = np.inf
    kappa: list = field(default_factory=list)   # per source path (Eq. 25)


def source_paths(verts, tris, topo, sources):
    """Edge paths between sources for the constraints of Eqs. 24-25
    (Sec. 5.2): from one source to each of the other sources, shortest in
    edge count.  Read as: a breadth-first tree grown from the first source
    alone (pairing rule of :mod:`oracle.bfs`, smallest-index neighbour one
    set closer), the path to another source is its tree path; a source the
    tree does not reach (another connected component) starts a new tree
    from itself, the first such source in the list.  Duplicates are dropped.

    Returns a list of paths, each a dict of arrays in path order (from the
    tree's root towards the source):
      edge  int64 edge ids, sign +1 where the path runs from the edge's
      smaller to its larger vertex id (the orientation halfedge) else -1,
      face  the face whose counter-clockwise boundary runs the edge in the
            path's direction (the only face of a boundary edge) -- the face
            whose gradient copy enters Eq. 24,
      vec   the edge vector in the path's direction (FP64)."""
    from .bfs import bfs_levels_vec
    from .mesh import vertex_adjacency
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    row_ptr, col = vertex_adjacency(topo.nv, topo.edges)
    key = topo.edges[:, 0] * topo.nv + topo.edges[:, 1]      # sorted: edges are unique-sorted
    src = list(dict.fromkeys(int(s) for s in np.asarray(sources).reshape(-1)))
    paths = []
    todo = src
    while len(todo) > 1:
        root = todo[0]
        level, parent = bfs_levels_vec(topo.nv, row_ptr, col, [root])
        rest = []
        for s in todo[1:]:
            if level[s] < 0:
                rest.append(s)
                continue
            steps = []
            v = s
            while parent[v] >= 0:
                steps.append((int(parent[v]), v))
                v = int(parent[v])
            steps.reverse()
            e = np.array([np.searchsorted(key, min(a, b) * topo.nv + max(a, b)) for a, b in steps], dtype=np.int64)
            sign = np.array([1.0 if a < b else -1.0 for a, b in steps])
            face = np.empty(len(steps), dtype=np.int64)
            for k, (a, b) in enumerate(steps):
                cand = [f for f in topo.edge_faces[e[k]] if f >= 0]
                face[k] = cand[0]
                for f in cand:
                    t = tris[f]
                    if any(t[i] == a and t[(i + 1) % 3] == b for i in range(3)):
                        face[k] = f
            vec = np.array([verts[b] - verts[a] for a, b in steps]).reshape(-1, 3)
            paths.append({"edge": e, "sign": sign, "face": face, "vec": vec})
        todo = rest
    return paths


def cycle_constraints(verts, tris, topo):
    """Cycle basis for global integrability on surfaces of genus g > 0 or
    with several boundary loops (Sec. 5.1, Eqs. 22-23), by tree-cotree
    (all ids are the caller's):

    * primal tree T: the breadth-first tree of :mod:`oracle.bfs` (parent =
      neighbour one level closer with the smallest id) grown from the
      smallest vertex of each connected component;
    * dual tree C: first-in-first-out breadth-first search over faces from
      the smallest face of each component, visiting a face's edges in slot
      order (tri[k], tri[k+1]) and crossing only interior edges not in T;
    * generators: interior edges in neither tree, in increasing edge id,
      of components without boundary (2g per closed component of genus g;
      loops around holes of components with boundary are not covered).

    For each generator e = (a, b), a < b:
      edge form (Eq. 23): the loop a -> b along e, then back from b to a
        through T (b up to the lowest common ancestor, down to a);
        entries {"edge", "sign"} as for source paths (sign +1 where the loop
        runs from the smaller to the larger vertex id);
      face form (Eq. 22): the dual loop f0 -> f1 across e (f0 < f1 its two
        faces), then back from f1 to f0 through C; per face of the loop the
        polyline segment from the midpoint of the edge it is entered by to
        the midpoint of the edge it is left by; entries {"face", "vec"}.
    Returns (edge_cycles, face_cycles)."""
    from collections import deque

    from .bfs import bfs_levels_vec
    from .mesh import vertex_adjacency
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    nv, nf, ne = topo.nv, tris.shape[0], topo.ne
    row_ptr, col = vertex_adjacency(nv, topo.edges)
    key = topo.edges[:, 0] * nv + topo.edges[:, 1]

    def eid(a, b):
        return int(np.searchsorted(key, min(a, b) * nv + max(a, b)))

    # components (vertex adjacency) and their smallest vertex / face
    comp = -np.ones(nv, dtype=np.int64)
    roots = []
    for v0 in range(nv):
        if comp[v0] >= 0:
            continue
        comp[v0] = len(roots)
        roots.append(v0)
        q = deque([v0])
        while q:
            u = q.popleft()
            for w in col[row_ptr[u]:row_ptr[u + 1]]:
                if comp[w] < 0:
                    comp[w] = comp[v0]
                    q.append(int(w))
    level, parent = bfs_levels_vec(nv, row_ptr, col, roots)
    in_t = np.zeros(ne, dtype=bool)
    for v in range(nv):
        if parent[v] >= 0:
            in_t[eid(v, int(parent[v]))] = True
    # dual tree
    other = topo.edge_faces
    fpar = -np.ones(nf, dtype=np.int64)
    fpar_e = -np.ones(nf, dtype=np.int64)
    seen = np.zeros(nf, dtype=bool)
    in_c = np.zeros(ne, dtype=bool)
    for f0 in range(nf):
        if seen[f0]:
            continue
        seen[f0] = True
        q = deque([f0])
        while q:
            f = q.popleft()
            for k in range(3):
                e = int(topo.face_edges[f, k])
                if topo.edge_nfaces[e] != 2 or in_t[e]:
                    continue
                g = int(other[e, 0] if other[e, 1] == f else other[e, 1])
                if seen[g]:
                    continue
                seen[g] = True
                fpar[g], fpar_e[g] = f, e
                in_c[e] = True
                q.append(g)
    # closed components only: with boundary loops the tree-cotree count
    # depends on how many boundary edges T takes (holes are not covered)
    open_comp = np.zeros(len(roots), dtype=bool)
    bnd = topo.edge_nfaces == 1
    open_comp[comp[topo.edges[bnd, 0]]] = True
    gens = [e for e in range(ne) if topo.edge_nfaces[e] == 2 and not in_t[e] and not in_c[e]
            and not open_comp[comp[topo.edges[e, 0]]]]

    def up(x, par):
        out = [x]
        while par[out[-1]] >= 0:
            out.append(int(par[out[-1]]))
        return out

    def lca_loop(a, b, par):
        pa, pb = up(a, par), up(b, par)
        sa = set(pa)
        c = next(x for x in pb if x in sa)
        return pb[:pb.index(c) + 1] + pa[:pa.index(c)][::-1]     # b ... c ... a

    mid = 0.5 * (verts[topo.edges[:, 0]] + verts[topo.edges[:, 1]])
    edge_cycles, face_cycles = [], []
    for e in gens:
        a, b = (int(x) for x in topo.edges[e])
        loop = [a] + lca_loop(a, b, parent)                     # a, b, ..., a
        es = [eid(loop[i], loop[i + 1]) for i in range(len(loop) - 1)]
        sg = [1.0 if loop[i] < loop[i + 1] else -1.0 for i in range(len(loop) - 1)]
        edge_cycles.append({"edge": np.array(es, dtype=np.int64), "sign": np.array(sg)})
        f0, f1 = sorted(int(x) for x in topo.edge_faces[e])
        floop = [f0] + lca_loop(f0, f1, fpar)                   # f0, f1, ..., f0
        cross = [e]
        for i in range(1, len(floop) - 1):
            x, y = floop[i], floop[i + 1]
            cross.append(int(fpar_e[x]) if fpar[x] == y else int(fpar_e[y]))
        faces, vecs = [], []
        for i in range(len(cross)):
            f = floop[i]
            faces.append(f)
            vecs.append(mid[cross[i]] - mid[cross[i - 1]])     # entered by cross[i-1], left by cross[i]
        face_cycles.append({"face": np.array(faces, dtype=np.int64), "vec": np.array(vecs).reshape(-1, 3)})
    return edge_cycles, face_cycles


class EdgeADMM:
    """Edge-form ADMM.  `paths` (from :func:`source_paths`) adds the
    constraint of Eq. 25 for each path S: one more group of copies
    v_S = (x_e, e in S) constrained to s . v_S = 0 (s the path signs), with
    its own duals kappa_S.  Its W-type update is the projection
    v_S = (I - s s^T / |S|)(x_S - kappa_S / mu); the X-update of an edge on
    n paths gains those copies,
    x_e = (sum_faces (h_e + lambda + mu w) + sum_paths (kappa + mu v))
          / (|H_e| (1 + mu) + mu n),
    and kappa_S += mu (v_S - x_S).  With paths the iteration converges to
    the integrable field with equal distance at every source."""

    def __init__(self, topo, Z, mu: float = 100.0, relax: float = 1.0, paths=()):
        self.mu = mu
        self.relax = relax
        self.topo = topo
        self.Z = np.asarray(Z, dtype=np.float64)                     # [F, 3]
        self.q = topo.face_signs.astype(np.float64)                  # [F, 3]
        self.fe = topo.face_edges                                    # [F, 3]
        self.ne = topo.ne
        self.nH = topo.edge_nfaces.astype(np.float64)
        self.paths = [(p["edge"], p["sign"]) for p in paths]
        self.npath = np.zeros(self.ne)
        for e, _ in self.paths:
            np.add.at(self.npath, e, 1.0)

    def _sum_to_edges(self, vals):
        return np.bincount(self.fe.reshape(-1), weights=vals.reshape(-1), minlength=self.ne)

    def init(self) -> EdgeADMMState:
        x = self._sum_to_edges(self.Z) / self.nH
        return EdgeADMMState(x=x, w=self.Z.copy(), lam=np.zeros_like(self.Z),
                             kappa=[np.zeros(e.size) for e, _ in self.paths])

    def step(self, s: EdgeADMMState) -> EdgeADMMState:
        mu, q, a = self.mu, self.q, self.relax
        w = w_update(s.x[self.fe], s.lam, q, mu)
        wh = a * w + (1.0 - a) * s.x[self.fe]
        num = self._sum_to_edges(self.Z) + self._sum_to_edges(s.lam) + mu * self._sum_to_edges(wh)
        vhs = []
        for (e, sg), kap in zip(self.paths, s.kappa):
            t = s.x[e] - kap / mu
            v = t - (sg @ t) / e.size * sg
            vh = a * v + (1.0 - a) * s.x[e]
            np.add.at(num, e, kap + mu * vh)
            vhs.append(vh)
        x = num / (self.nH * (1.0 + mu) + mu * self.npath)
        lam = s.lam + mu * (wh - x[self.fe])
        kappa = [kap + mu * (vh - x[e]) for (e, _), kap, vh in zip(self.paths, s.kappa, vhs)]
        r_p = np.linalg.norm(w - x[self.fe])
        r_d = np.linalg.norm(mu * (x - s.x)[self.fe])
        return EdgeADMMState(x=x, w=w, lam=lam, iters=s.iters + 1, r_primal=r_p, r_dual=r_d, kappa=kappa)

    def run(self, iters: int, tol: float = 0.0, state=None):
        s = self.init() if state is None else state
        for _ in range(iters):
            s = self.step(s)
            if s.r_primal <= tol and s.r_dual <= tol:
                break
        return s
