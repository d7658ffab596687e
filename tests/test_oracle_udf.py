"""The narrow-band unsigned distance field of the mesh-to-volume step
(Sec. 4.1) in the oracle.  Pins that do not reuse its point-triangle
distance: one triangle in an axis plane against planar geometry worked out
separately (in-plane distance to the triangle, then Pythagoras), the band
cut-off, a fine sphere against the analytic distance to the sphere within
its chord error, and soup invariances (order, duplicates, added triangles)."""
import math

import numpy as np
import pytest

from oracle import udf
from paper_2509_05595_amd import meshgen as g


def _seg2(p, a, b):
    ab = (b[0] - a[0], b[1] - a[1])
    t = ((p[0] - a[0]) * ab[0] + (p[1] - a[1]) * ab[1]) / (ab[0] ** 2 + ab[1] ** 2)
    t = min(1.0, max(0.0, t))
    return math.hypot(p[0] - a[0] - t * ab[0], p[1] - a[1] - t * ab[1])


def test_one_triangle_in_an_axis_plane():
    # right triangle in z = 0.5: inside its shadow the distance is |z - 0.5|,
    # outside it is the in-plane distance to the triangle's edges combined with
    # the height
    A, B, C = (0.2, 0.2), (0.8, 0.2), (0.2, 0.8)
    V = np.array([[*A, 0.5], [*B, 0.5], [*C, 0.5]])
    F = np.array([[0, 1, 2]])
    res, band = 12, 0.4
    U = udf.udf(V, F, res, band)
    for idx, p in np.ndenumerate(udf.centres(res)[..., 0]):
        x, y, z = udf.centres(res)[idx]
        inside = x >= 0.2 and y >= 0.2 and x + y <= 1.0
        d2 = 0.0 if inside else min(_seg2((x, y), A, B), _seg2((x, y), B, C), _seg2((x, y), C, A))
        want = math.hypot(d2, z - 0.5)
        if want <= band - 1e-12:
            assert abs(U[idx] - want) <= 1e-14, (idx, U[idx], want)
        elif want > band + 1e-12:
            assert U[idx] == np.inf


def test_band_cut_off_and_empty_surroundings():
    V, F = g.tetrahedron()
    V = 0.1 * V + 0.05  # a small tetrahedron near the corner
    U = udf.udf(V, F, 10, 0.15)
    assert np.all((U <= 0.15) | (U == np.inf)) and np.isfinite(U).sum() > 0
    assert np.all(np.isinf(U[6:, 6:, 6:]))  # centres farther than the band from the corner box


def test_fine_sphere_against_the_analytic_distance():
    u, Fs = g.icosphere(4)  # unit sphere, 5,120 faces
    c, r = np.array([0.5, 0.5, 0.5]), 0.35
    V = c + r * u
    # chord error: the mesh lies between radius r cos(theta) and r, theta the
    # largest angle from a face's centre to its corners
    cen = u[Fs].mean(axis=1)
    cen /= np.linalg.norm(cen, axis=1)[:, None]
    cos_t = min(np.einsum("ij,ij->i", cen, u[Fs[:, k]]).min() for k in range(3))
    sag = r * (1 - cos_t)
    P = np.random.default_rng(3).random((400, 3))
    got = udf.at(V, Fs, P, 1.0)
    want = np.abs(np.linalg.norm(P - c, axis=1) - r)
    assert np.all(np.abs(got - want) <= sag + 1e-12) and sag < 0.01


def test_soup_invariances():
    V, F = g.bumpy_icosphere_gauss(k=2, seed=8)
    res, band = 10, 0.3
    U = udf.udf(V, F, res, band)
    perm = np.random.default_rng(1).permutation(len(F))
    assert np.array_equal(udf.udf(V, F[perm], res, band), U)  # a minimum: order-free
    Ur = udf.udf(V, F[:, [1, 2, 0]], res, band)  # corners rotated: the same up to rounding
    fin = np.isfinite(U)
    assert np.array_equal(fin, np.isfinite(Ur)) and np.abs(Ur[fin] - U[fin]).max() <= 1e-15
    assert np.array_equal(udf.udf(V, np.concatenate([F, F[:7]]), res, band), U)
    V2 = np.concatenate([V, [[0.1, 0.1, 0.1], [0.2, 0.1, 0.1], [0.1, 0.2, 0.1]]])
    F2 = np.concatenate([F, [[len(V), len(V) + 1, len(V) + 2]]])
    U2 = udf.udf(V2, F2, res, band)
    assert np.all(U2 <= U) and np.any(U2 < U)


def test_triangles_of_zero_area_count_as_their_edges():
    # a repeated corner and three collinear corners: the distance to the
    # segments they span (a point on the segment is at distance 0)
    V = np.array([[0.3, 0.3, 0.3], [0.5, 0.5, 0.5], [0.7, 0.7, 0.7], [0.2, 0.6, 0.4]])
    F = np.array([[0, 1, 2], [3, 3, 0]])
    P = np.array([[0.475, 0.475, 0.475], [0.6, 0.6, 0.6], [0.25, 0.45, 0.35], [0.9, 0.9, 0.9]])
    got = udf.at(V, F, P, 1.0)
    seg = lambda p, a, b: np.linalg.norm(p - (a + np.clip(np.dot(p - a, b - a) / np.dot(b - a, b - a), 0, 1) * (b - a)))
    for p, g_ in zip(P, got):
        want = min(seg(p, V[0], V[2]), seg(p, V[3], V[0]))
        assert abs(g_ - want) <= 1e-15
    assert got[0] <= 1e-15 and got[1] <= 1e-15
