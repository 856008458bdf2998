"""Small meshes for the oracle pins (pure test helpers, no method arithmetic)."""
import numpy as np


def equilateral_patch(n: int = 9, h: float = 1.0):
    """Triangular lattice: vertex (i, j) at (h(i + j/2), h j sqrt(3)/2),
    0 <= i, j < n, CCW triangles.  Interior vertices have six equilateral
    neighbours."""
    verts = []
    for j in range(n):
        for i in range(n):
            verts.append([h * (i + 0.5 * j), h * j * np.sqrt(3.0) / 2.0, 0.0])
    verts = np.array(verts)
    tris = []
    for j in range(n - 1):
        for i in range(n - 1):
            a = j * n + i
            b = a + 1
            c = a + n
            d = c + 1
            tris.append([a, b, c])
            tris.append([b, d, c])
    return verts, np.array(tris, dtype=np.int32)


def interior_mask(verts, tris):
    """Vertices not on the boundary (every incident edge has two faces)."""
    nv = verts.shape[0]
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]).astype(np.int64)
    e.sort(axis=1)
    key, cnt = np.unique(e[:, 0] * nv + e[:, 1], return_counts=True)
    bnd = key[cnt == 1]
    mask = np.ones(nv, dtype=bool)
    mask[bnd // nv] = False
    mask[bnd % nv] = False
    return mask
