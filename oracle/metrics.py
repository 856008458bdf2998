"""Error measures (test infrastructure only).

* :func:`direction_error` -- E of Eq. 8: sqrt(sum_f Abar_f |h_f - h*_f|^2)
  with Abar the face area divided by the total area.
* :func:`mean_relative_error` -- epsilon of Eq. 28: (1/|V|) sum over the
  non-source vertices of |d - d*|/|d*| (the 1/|V| is kept as printed).
* :func:`heat_residual` -- E1 of Eq. 29: |(A - t L_c) u - u_0|_2.
* :func:`distance_error_l2` -- E2 of Eq. 30: |d - d*|_2 / n.
* :func:`parity` -- mean and max of |d - d*| over reached vertices divided by
  the diameter, read as max_v d*(v) (the eccentricity of the source set).
"""
from __future__ import annotations

import numpy as np


def direction_error(h, hstar, face_area) -> float:
    w = face_area / face_area.sum()
    return float(np.sqrt((w * ((h - hstar) ** 2).sum(axis=1)).sum()))


def mean_relative_error(d, dstar, sources) -> float:
    mask = np.ones(d.size, dtype=bool)
    mask[np.asarray(sources)] = False
    mask &= np.isfinite(dstar)
    return float((np.abs(d[mask] - dstar[mask]) / np.abs(dstar[mask])).sum() / d.size)


def heat_residual(M, u, sources) -> float:
    u0 = np.zeros(u.size)
    u0[np.asarray(sources)] = 1.0
    return float(np.linalg.norm(M @ u - u0))


def distance_error_l2(d, dstar) -> float:
    return float(np.linalg.norm(d - dstar) / d.size)


def parity(d, dstar):
    """(mean, max) of |d - d*| / max(d*) over vertices where d* is finite."""
    ok = np.isfinite(dstar)
    diam = float(np.max(dstar[ok]))
    err = np.abs(np.asarray(d, dtype=np.float64)[ok] - dstar[ok]) / diam
    return float(err.mean()), float(err.max())
