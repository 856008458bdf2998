"""Many meshes in one solve: the meshes are placed side by side as the
components of one resident mesh, and one hg_geodesic_solve (one launch per
step of the path for all of them) answers a query on each.  With
opts.t_per_component every component diffuses with its own t = m hbar_c^2,
breadth-first sets, tiles and source paths never cross components, and the
integration starts from each component's own sources, so every mesh gets the
distance it has alone (to the solve's tolerances: the ADMM stopping rule and
the automatic penalty see the whole batch).
"""
from __future__ import annotations

import numpy as np

from . import _hgeo


class MeshBatch:
    """`meshes`: sequence of (verts [V_i,3], tris [F_i,3]), each connected."""

    def __init__(self, meshes, stream=None):
        vs, fs, starts = [], [], []
        n = 0
        for v, f in meshes:
            v = np.asarray(v, dtype=np.float64)
            f = np.asarray(f, dtype=np.int64)
            vs.append(v)
            fs.append(f + n)
            starts.append(n)
            n += v.shape[0]
        self.starts = np.array(starts + [n], dtype=np.int64)
        self.mesh = _hgeo.Mesh(np.vstack(vs), np.vstack(fs).astype(np.int32), stream=stream)
        if self.mesh.stats["n_components"] != len(starts):
            self.mesh.close()
            raise ValueError("every mesh of a batch must be connected")

    def __len__(self):
        return len(self.starts) - 1

    def solve(self, sources, t: float = 0.0, opts=None, stream=None, out=None):
        """`sources`: one sequence of vertex ids per mesh (its own numbering).
        Returns (list of per-mesh distance views of one device tensor, info)."""
        if len(sources) != len(self):
            raise ValueError("one source list per mesh expected")
        src = []
        for i, s in enumerate(sources):
            s = np.atleast_1d(np.asarray(s, dtype=np.int64))
            if s.size == 0:
                raise ValueError(f"mesh {i} has no source")
            if s.min() < 0 or s.max() >= self.starts[i + 1] - self.starts[i]:
                raise ValueError(f"source out of range for mesh {i}")
            src.append(s + self.starts[i])
        if opts is None:
            opts = _hgeo.default_opts()
        opts.t_per_component = 1
        d, info = self.mesh.solve(np.concatenate(src).astype(np.int32), t, opts, out=out, stream=stream)
        return [d[self.starts[i]:self.starts[i + 1]] for i in range(len(self))], info

    def close(self):
        self.mesh.close()
