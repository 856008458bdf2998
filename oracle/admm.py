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

from dataclasses import dataclass

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


class FaceADMM:
    def __init__(self, verts, tris, topo, h, mu: float = 100.0, relax: float = 1.0):
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
        self.count = np.bincount(self.faces, minlength=self.nf).astype(np.float64)
        self.normM = np.sqrt(self.A.sum())

    def init(self) -> FaceADMMState:
        return FaceADMMState(g=self.h.copy(), y=self.h[self.faces].copy(),
                             lam=np.zeros((self.faces.size, 3)))

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
        g = g_update(self.h, tot, self.count, mu)
        lam = s.lam + mu * al[:, None] * (yh - g[self.faces])
        r_p = np.linalg.norm(al[:, None] * (y - g[self.faces]))
        r_d = np.linalg.norm(mu * A[:, None] * (g - s.g)[self.faces])
        return FaceADMMState(g=g, y=y, lam=lam, iters=s.iters + 1, r_primal=r_p, r_dual=r_d)

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


class EdgeADMM:
    def __init__(self, topo, Z, mu: float = 100.0, relax: float = 1.0):
        self.mu = mu
        self.relax = relax
        self.topo = topo
        self.Z = np.asarray(Z, dtype=np.float64)                     # [F, 3]
        self.q = topo.face_signs.astype(np.float64)                  # [F, 3]
        self.fe = topo.face_edges                                    # [F, 3]
        self.ne = topo.ne
        self.nH = topo.edge_nfaces.astype(np.float64)

    def _sum_to_edges(self, vals):
        return np.bincount(self.fe.reshape(-1), weights=vals.reshape(-1), minlength=self.ne)

    def init(self) -> EdgeADMMState:
        x = self._sum_to_edges(self.Z) / self.nH
        return EdgeADMMState(x=x, w=self.Z.copy(), lam=np.zeros_like(self.Z))

    def step(self, s: EdgeADMMState) -> EdgeADMMState:
        mu, q = self.mu, self.q
        w = w_update(s.x[self.fe], s.lam, q, mu)
        wh = self.relax * w + (1.0 - self.relax) * s.x[self.fe]
        x = x_update(self._sum_to_edges(self.Z), self._sum_to_edges(s.lam),
                     self._sum_to_edges(wh), self.nH, mu)
        lam = s.lam + mu * (wh - x[self.fe])
        r_p = np.linalg.norm(w - x[self.fe])
        r_d = np.linalg.norm(mu * (x - s.x)[self.fe])
        return EdgeADMMState(x=x, w=w, lam=lam, iters=s.iters + 1, r_primal=r_p, r_dual=r_d)

    def run(self, iters: int, tol: float = 0.0, state=None):
        s = self.init() if state is None else state
        for _ in range(iters):
            s = self.step(s)
            if s.r_primal <= tol and s.r_dual <= tol:
                break
        return s
