"""Many resident meshes in one solve: a thin binding of
hg_geodesic_solve_batch (include/hgeo.h).  The library joins the meshes on
the device as the components of one mesh, so every step of the path is one
launch sequence for all of them; each mesh diffuses with its own
t = m hbar_i^2 and gets the distance it has alone (to the solve's
tolerances: the ADMM stopping rule and the automatic penalty see the whole
batch).
"""
from __future__ import annotations

from . import _hgeo


class MeshBatch:
    """`meshes`: resident :class:`Mesh` objects, or (verts [V_i,3], tris
    [F_i,3]) pairs, which are made resident here (and closed by close())."""

    def __init__(self, meshes, stream=None):
        self.meshes = []
        self._owned = []
        for m in meshes:
            if isinstance(m, _hgeo.Mesh):
                self.meshes.append(m)
            else:
                v, f = m
                mm = _hgeo.Mesh(v, f, stream=stream)
                self.meshes.append(mm)
                self._owned.append(mm)

    def __len__(self):
        return len(self.meshes)

    def solve(self, sources, t: float = 0.0, opts=None, stream=None, outs=None,
              raise_on_nonconvergence: bool = True):
        """`sources`: one sequence of vertex ids per mesh (its own numbering).
        Returns (list of per-mesh float32 device tensors, info of the batch)."""
        return _hgeo.solve_batch(self.meshes, sources, t, opts, outs, stream, raise_on_nonconvergence)

    def close(self):
        for m in self._owned:
            m.close()
        self._owned.clear()
        self.meshes.clear()
