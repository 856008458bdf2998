"""Integration of optimised gradients into distances (Sec. 3.3 and Sec. 4),
test infrastructure only.

The distance is zero at every source and is then fixed set by set,
D_1, D_2, ... (the text's "i >= 0" should read i >= 1): a vertex v_j of D_i
takes the value of its partner v_k in D_{i-1} plus the change along the edge
(j, k).

* face form, Eq. 17: change = mean over the faces T_jk containing the edge of
  g_l . (p_j - p_k);
* edge form: change = +x_e when v_j is the head of the orientation halfedge
  of e = {j, k}, -x_e when it is the tail (the paper says the edge
  differences are integrated directly but prints no formula; this is the
  reading).

Plain FP64 accumulation in front order.  Unreached vertices get +inf.
"""
from __future__ import annotations

import numpy as np


def _edge_lookup(topo):
    nv = topo.nv
    key = topo.edges[:, 0] * nv + topo.edges[:, 1]
    order = np.argsort(key)
    return key[order], order


def _edge_ids(topo, a, b):
    skey, order = _edge_lookup(topo)
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    pos = np.searchsorted(skey, lo * topo.nv + hi)
    return order[pos]


def integrate_face(verts, topo, g, level, parent, sources) -> np.ndarray:
    """Eq. 17 front by front."""
    nv = topo.nv
    d = np.full(nv, np.inf)
    d[np.asarray(sources)] = 0.0
    has = parent >= 0
    j_all = np.flatnonzero(has)
    k_all = parent[j_all]
    e_all = _edge_ids(topo, j_all, k_all)
    f0 = topo.edge_faces[e_all, 0]
    f1 = topo.edge_faces[e_all, 1]
    dp = verts[j_all] - verts[k_all]
    s = np.einsum("ic,ic->i", g[f0], dp)
    two = f1 >= 0
    s[two] = 0.5 * (s[two] + np.einsum("ic,ic->i", g[f1[two]], dp[two]))
    step = np.zeros(nv)
    step[j_all] = s
    maxlev = int(level.max()) if level.size else 0
    for i in range(1, maxlev + 1):
        vs = np.flatnonzero(level == i)
        d[vs] = d[parent[vs]] + step[vs]
    return d


def integrate_edge(topo, x, level, parent, sources) -> np.ndarray:
    """Edge differences summed front by front: d_j = d_k +- x_e."""
    nv = topo.nv
    d = np.full(nv, np.inf)
    d[np.asarray(sources)] = 0.0
    j_all = np.flatnonzero(parent >= 0)
    k_all = parent[j_all]
    e_all = _edge_ids(topo, j_all, k_all)
    sign = np.where(topo.edges[e_all, 1] == j_all, 1.0, -1.0)
    step = np.zeros(nv)
    step[j_all] = sign * x[e_all]
    maxlev = int(level.max()) if level.size else 0
    for i in range(1, maxlev + 1):
        vs = np.flatnonzero(level == i)
        d[vs] = d[parent[vs]] + step[vs]
    return d
