"""Pins of the oracle's exact predicates (no GPU).

* orientation signs against exact ``Fraction`` determinants;
* the triangle-pair self-intersection test (Sec. 5.2, Appendix 3) against an
  exact-rational linear program that uses no orientation predicate at all
  (tests/lp_exact.py), on the four kinds of pairs the paper's accuracy study
  uses (coplanar, sharp, vertex-sharing, edge-sharing), plus hand-built cases
  of the paper's coplanar figure and its zero-cross-product figure.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle.oracle as orc
from lp_exact import tri_pair_exact


def _det3_exact(a, b, c, d):
    a, b, c, d = ([Fr(float(x)) for x in p] for p in (a, b, c, d))
    ad = [a[i] - d[i] for i in range(3)]
    bd = [b[i] - d[i] for i in range(3)]
    cd = [c[i] - d[i] for i in range(3)]
    det = (ad[0] * (bd[1] * cd[2] - bd[2] * cd[1]) - ad[1] * (bd[0] * cd[2] - bd[2] * cd[0])
           + ad[2] * (bd[0] * cd[1] - bd[1] * cd[0]))
    return (det > 0) - (det < 0)


def _det2_exact(a, b, c):
    a, b, c = ([Fr(float(x)) for x in p] for p in (a, b, c))
    det = (a[0] - c[0]) * (b[1] - c[1]) - (a[1] - c[1]) * (b[0] - c[0])
    return (det > 0) - (det < 0)


def _near_coplanar_points(rng):
    a, b, c = rng.random((3, 3))
    s, t = rng.random(2)
    d = a + s * (b - a) + t * (c - a)  # on the plane up to rounding
    k = rng.integers(0, 3)
    d[k] = np.nextafter(d[k], d[k] + rng.choice([-1.0, 1.0])) if rng.random() < 0.5 else d[k]
    return a, b, c, d


def test_orient3d_matches_rational_determinant():
    rng = np.random.default_rng(11)
    nz = 0
    for i in range(3000):
        if i % 3 == 0:
            pts = rng.random((4, 3))
        elif i % 3 == 1:
            pts = _near_coplanar_points(rng)
        else:
            pts = rng.integers(0, 3, (4, 3)).astype(np.float64)
        want = _det3_exact(*pts)
        nz += want == 0
        assert orc.orient3d(*pts) == want
        assert orc.orient3d(*pts, exact_only=True) == want
    assert nz > 100  # exercised the exactly-zero case


def test_orient2d_matches_rational_determinant():
    rng = np.random.default_rng(12)
    for i in range(3000):
        if i % 2:
            a, b = rng.random((2, 2))
            t = rng.random()
            c = a + t * (b - a)
            pts = (a, b, c)
        else:
            pts = rng.integers(0, 3, (3, 2)).astype(np.float64)
        want = _det2_exact(*pts)
        assert orc.orient2d(*pts) == want
        assert orc.orient2d(*pts, exact_only=True) == want


def _nondegenerate(T):
    a, b, c = ([Fr(float(x)) for x in p] for p in T)
    u = [b[i] - a[i] for i in range(3)]
    v = [c[i] - a[i] for i in range(3)]
    n = (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])
    return any(x != 0 for x in n)


def _random_pair(rng, kind):
    """Triangle pair of one of the accuracy-study kinds; ids encode sharing."""
    while True:
        if kind == "coplanar":
            P = np.c_[rng.integers(0, 5, (3, 2)), np.zeros(3)].astype(np.float64)
            Q = np.c_[rng.integers(0, 5, (3, 2)), np.zeros(3)].astype(np.float64)
        elif kind == "sharp":
            P = rng.integers(0, 6, (3, 3)).astype(np.float64)
            Q = rng.integers(0, 6, (3, 3)).astype(np.float64)
            Q[2] = Q[0] + (Q[1] - Q[0]) * 0.5 + rng.integers(-1, 2, 3) * 0.25
        else:
            P = rng.integers(0, 4, (3, 3)).astype(np.float64)
            Q = rng.integers(0, 4, (3, 3)).astype(np.float64)
        ip = np.array([0, 1, 2])
        iq = np.array([3, 4, 5])
        if kind in ("vertex", "coplanar_vertex"):
            j = rng.integers(0, 3)
            i = rng.integers(0, 3)
            Q[j] = P[i]
            iq[j] = ip[i]
        if kind in ("edge", "coplanar_edge"):
            i = rng.integers(0, 3)
            j = rng.integers(0, 3)
            Q[j], Q[(j + 1) % 3] = P[(i + 1) % 3], P[i]
            iq[j], iq[(j + 1) % 3] = ip[(i + 1) % 3], ip[i]
        if kind.startswith("coplanar_"):
            P[:, 2] = 0.0
            Q[:, 2] = 0.0
        if _nondegenerate(P) and _nondegenerate(Q):
            return P, ip, Q, iq


PAIR_KINDS = ["random", "coplanar", "sharp", "vertex", "edge", "coplanar_vertex", "coplanar_edge"]


@pytest.mark.parametrize("kind", PAIR_KINDS)
def test_tri_pair_matches_exact_lp(kind):
    # a fixed seed per kind, so a failing case replays
    rng = np.random.default_rng(7100 + PAIR_KINDS.index(kind))
    pos = neg = 0
    for _ in range(300):
        P, ip, Q, iq = _random_pair(rng, kind)
        want = tri_pair_exact(P, ip, Q, iq)
        got = orc.tri_pair(P, ip, Q, iq)
        assert got == want, (kind, P.tolist(), ip.tolist(), Q.tolist(), iq.tolist())
        # symmetric in the two triangles
        assert orc.tri_pair(Q, iq, P, ip) == want
        pos += want
        neg += not want
    assert pos > 10 and neg > 10


def _case(P, ip, Q, iq):
    P = np.array(P, dtype=np.float64)
    Q = np.array(Q, dtype=np.float64)
    return orc.tri_pair(P, ip, Q, iq), tri_pair_exact(P, ip, Q, iq)


def test_coplanar_figure_cases():
    """Coplanar cases of the paper's figure: (1)(2)(4) intersect, (3)(5) are
    legitimate vertex / edge sharing."""
    A, B, C = [0, 0, 0], [4, 0, 0], [0, 4, 0]
    # (1) no shared vertex, overlapping
    assert _case([A, B, C], [0, 1, 2], [[1, 1, 0], [5, 1, 0], [1, 5, 0]], [3, 4, 5]) == (True, True)
    # (2) shared vertex, the angles overlap
    assert _case([A, B, C], [0, 1, 2], [A, [4, 1, 0], [1, 4, 0]], [0, 4, 5]) == (True, True)
    # (3) shared vertex, angles disjoint
    assert _case([A, B, C], [0, 1, 2], [A, [-1, -4, 0], [-4, -1, 0]], [0, 4, 5]) == (False, False)
    # (4) shared edge, third corners on the same side
    assert _case([A, B, C], [0, 1, 2], [B, A, [1, 1, 0]], [1, 0, 5]) == (True, True)
    # (5) shared edge, opposite sides
    assert _case([A, B, C], [0, 1, 2], [B, A, [1, -1, 0]], [1, 0, 5]) == (False, False)


def test_zero_cross_product_cases():
    """Shared vertex with collinear edges (the paper's zero-cross-product
    figure): same direction overlaps, opposite direction only touches."""
    A, B, C = [0, 0, 0], [4, 0, 0], [0, 4, 0]
    # edge AD along AB (same direction): overlap along a segment
    assert _case([A, B, C], [0, 1, 2], [A, [2, 0, 0], [3, -3, 0]], [0, 4, 5]) == (True, True)
    # edge AD opposite to AB: they meet only at A
    assert _case([A, B, C], [0, 1, 2], [A, [-2, 0, 0], [-3, -3, 0]], [0, 4, 5]) == (False, False)


def test_3d_cases():
    A, B, C = [0, 0, 0], [4, 0, 0], [0, 4, 0]
    # shared vertex, second triangle pierces the first away from A
    assert _case([A, B, C], [0, 1, 2], [A, [1, 1, -1], [1, 1, 1]], [0, 4, 5]) == (True, True)
    # shared vertex, second triangle leaves A upwards only
    assert _case([A, B, C], [0, 1, 2], [A, [1, 1, 1], [2, 0, 1]], [0, 4, 5]) == (False, False)
    # shared edge, not coplanar: never
    assert _case([A, B, C], [0, 1, 2], [B, A, [1, 1, 1]], [1, 0, 5]) == (False, False)
    # no sharing, touching at one point counts
    assert _case([A, B, C], [0, 1, 2], [[1, 1, 0], [1, 1, 3], [3, 3, 3]], [3, 4, 5]) == (True, True)
    # identical vertex ids: always
    assert orc.tri_pair(np.array([A, B, C], float), [0, 1, 2], np.array([A, B, C], float), [2, 0, 1])


def test_degenerate_exact():
    assert orc.degenerate([0, 0, 0, 1, 1, 1, 2, 2, 2])
    assert not orc.degenerate([0, 0, 0, 1, 1, 1, 2, 2, 2 + 2 ** -40])
    a = np.array([0.1, 0.2, 0.3])
    b = np.array([0.7, 0.11, 0.9])
    # a point on segment ab up to rounding is generally not exactly collinear
    c = a + 0.5 * (b - a)
    want = all(_det2_exact(a[[i, j]], b[[i, j]], c[[i, j]]) == 0 for i, j in ((0, 1), (1, 2), (2, 0)))
    assert orc.degenerate(np.r_[a, b, c]) == want
