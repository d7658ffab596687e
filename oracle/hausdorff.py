"""TEST INFRASTRUCTURE ONLY: distances from points to a triangle mesh, in
float64 numpy, for checking the library's Hausdorff distance.

A point's distance to a triangle is the distance to its projection onto the
triangle's plane when that projection falls inside the triangle (barycentric
coordinates from the 2x2 normal equations), else the smallest distance to the
triangle's three edges (segments, clamped).  The one-sided Hausdorff distance
from points P to a surface is the largest of the points' distances to their
closest triangle.
"""
from __future__ import annotations

import numpy as np


def _seg_dist(p, a, b):
    ab = b - a
    t = np.einsum("ij,ij->i", p[None, :] - a, ab) / np.maximum(np.einsum("ij,ij->i", ab, ab), 1e-300)
    t = np.clip(t, 0.0, 1.0)
    q = a + t[:, None] * ab
    return np.linalg.norm(p[None, :] - q, axis=1)


def point_tris(p, A, B, C):
    """distance from point p to each triangle (A[i], B[i], C[i])"""
    e0, e1 = B - A, C - A
    d = p[None, :] - A
    a00 = np.einsum("ij,ij->i", e0, e0)
    a01 = np.einsum("ij,ij->i", e0, e1)
    a11 = np.einsum("ij,ij->i", e1, e1)
    b0 = np.einsum("ij,ij->i", d, e0)
    b1 = np.einsum("ij,ij->i", d, e1)
    det = a00 * a11 - a01 * a01
    with np.errstate(divide="ignore", invalid="ignore"):
        u = (a11 * b0 - a01 * b1) / det
        v = (a00 * b1 - a01 * b0) / det
    inside = (det > 0) & (u >= 0) & (v >= 0) & (u + v <= 1)
    n = np.cross(e0, e1)
    nn = np.linalg.norm(n, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        plane = np.abs(np.einsum("ij,ij->i", d, n)) / nn
    edge = np.minimum(np.minimum(_seg_dist(p, A, B), _seg_dist(p, B, C)), _seg_dist(p, C, A))
    return np.where(inside, plane, edge)


def distances(P, V, F):
    P = np.asarray(P, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F)
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return np.array([point_tris(p, A, B, C).min() for p in P])


def hausdorff(P, V, F):
    return float(distances(P, V, F).max()) if len(P) else 0.0
