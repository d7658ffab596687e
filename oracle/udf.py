"""TEST INFRASTRUCTURE ONLY: the narrow-band unsigned distance field of the
remeshing stage's mesh-to-volume step (Sec. 4.1), by its definition.

The field is sampled at the voxel centres of an R^3 grid over [0,1]^3, voxel
(i, j, k) centred at ((i + 1/2) / R, (j + 1/2) / R, (k + 1/2) / R).  Its value
is the smallest distance from the centre to any triangle of the soup (no
topology is assumed) when that distance is at most the band width, and +inf
elsewhere (the paper only needs values inside the band, 3 / R by default).
Every centre is compared with every triangle (brute force, float64 numpy,
point-triangle distances from oracle.hausdorff, edges for triangles of zero
area); meant for small grids.
"""
from __future__ import annotations

import numpy as np

from .hausdorff import _seg_dist, point_tris


def centres(res: int) -> np.ndarray:
    """voxel centres, shape (R, R, R, 3), index [i, j, k] = (x, y, z)"""
    c = (np.arange(res, dtype=np.float64) + 0.5) / res
    x, y, z = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([x, y, z], axis=-1)


def at(V, F, P, band: float) -> np.ndarray:
    """the field at arbitrary points P (n, 3).  A triangle of (nearly) zero
    area (|n|^2 <= 1e-20 |e0|^2 |e1|^2, n the cross product of two edges e0, e1)
    counts as its three edges: there the projection onto its plane is not
    defined."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F)
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    e0, e1 = B - A, C - A
    n = np.cross(e0, e1)
    flat = ~(np.einsum("ij,ij->i", n, n) > 1e-20 * np.einsum("ij,ij->i", e0, e0) * np.einsum("ij,ij->i", e1, e1))
    out = np.full(len(P), np.inf)
    for i, p in enumerate(np.asarray(P, dtype=np.float64)):
        if not len(F):
            continue
        d = point_tris(p, A, B, C)
        if flat.any():
            fa, fb, fc = A[flat], B[flat], C[flat]
            d[flat] = np.minimum(np.minimum(_seg_dist(p, fa, fb), _seg_dist(p, fb, fc)), _seg_dist(p, fc, fa))
        m = d.min()
        out[i] = m if m <= band else np.inf
    return out


def udf(V, F, res: int, band: float) -> np.ndarray:
    """shape (R, R, R): min distance to the soup where <= band, else +inf"""
    return at(V, F, centres(res).reshape(-1, 3), band).reshape(res, res, res)
