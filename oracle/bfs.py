"""Breadth-first vertex sets and pairing (test infrastructure only).

D_0 is the source set (Sec. 5.2 puts every source in D_0) and
D_i = N(D_{i-1}) minus the earlier sets (Eq. 6), i.e. D_i holds the vertices
whose shortest edge path to the source set has exactly i edges (the text
after Eq. 6 says i - 1, a slip).  Each vertex of D_i (i >= 1) is paired with
a neighbour in D_{i-1} (Sec. 3.3); the paper leaves the choice open, the
oracle takes the neighbour of smallest index.  Unreached vertices get level
and parent -1.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def bfs_levels(nv: int, row_ptr, col, sources):
    """(level int64[V], parent int64[V]) by a plain FIFO traversal."""
    level = np.full(nv, -1, dtype=np.int64)
    parent = np.full(nv, -1, dtype=np.int64)
    q = deque()
    for s in np.unique(np.asarray(sources)):
        level[s] = 0
        q.append(int(s))
    while q:
        v = q.popleft()
        for k in range(row_ptr[v], row_ptr[v + 1]):
            w = int(col[k])
            if level[w] < 0:
                level[w] = level[v] + 1
                q.append(w)
    # pairing: smallest-index neighbour one level closer
    for v in range(nv):
        lv = level[v]
        if lv > 0:
            best = -1
            for k in range(row_ptr[v], row_ptr[v + 1]):
                w = int(col[k])
                if level[w] == lv - 1 and (best < 0 or w < best):
                    best = w
            parent[v] = best
    return level, parent


def bfs_levels_vec(nv: int, row_ptr, col, sources):
    """Same result as :func:`bfs_levels`, set by set with numpy (for large
    meshes)."""
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    deg = np.diff(row_ptr)
    src_of = np.repeat(np.arange(nv), deg)
    level = np.full(nv, -1, dtype=np.int64)
    front = np.unique(np.asarray(sources, dtype=np.int64))
    level[front] = 0
    i = 0
    while front.size:
        i += 1
        starts = row_ptr[front]
        cnt = deg[front]
        idx = np.repeat(starts - np.cumsum(np.concatenate([[0], cnt[:-1]])), cnt) + np.arange(cnt.sum())
        nb = np.unique(col[idx])
        nb = nb[level[nb] < 0]
        level[nb] = i
        front = nb
    parent = np.full(nv, -1, dtype=np.int64)
    lv_src = level[src_of]
    lv_dst = level[col]
    ok = (lv_src > 0) & (lv_dst == lv_src - 1)
    cand = np.full(src_of.size, np.iinfo(np.int64).max)
    cand[ok] = col[ok]
    best = np.minimum.reduceat(cand, row_ptr[:-1]) if nv else cand
    has = level > 0
    parent[has] = best[has]
    return level, parent
