"""Pins of the oracle's edge cost (Eq. 1) and of its exact-target cap (no GPU).

* The skinny term of Eq. 1 sums 1 - C_ijk over the triangles a collapse
  generates: the faces around either end of the edge except the two faces
  holding both ends (they vanish), with both ends moved to the new vertex.
  It is restated here from that definition in plain Python (set of faces,
  shape factor 4 sqrt(3) A / (l1^2 + l2^2 + l3^2), quadric error as a sum of
  squared plane distances) and compared with the oracle on every edge of
  small meshes.
* On a flat patch of the regular triangular lattice the quadric error is
  zero, the new vertex is the midpoint of the edge, and the cost has a closed
  form worked out by hand: w_e l + w_s (4 (1 - 6/7) + 4 (1 - 9/10)) =
  w_e l + w_s 34/35 over the val(a) + val(b) - 4 = 8 generated triangles.
* The exact-target cap keeps, among the candidates that pass the local
  checks, exactly the `need` smallest keys.
"""
import math
from collections import defaultdict

import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g


# ---------------------------------------------------------------- helpers
def _incidence(F):
    inc = defaultdict(list)
    for f, t in enumerate(F):
        for v in t:
            inc[int(v)].append(f)
    return inc


def _edges(F):
    return sorted({(min(int(a), int(b)), max(int(a), int(b)))
                   for t in F for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))})


def _shape_defect(p0, p1, p2):
    """1 - C for one triangle, C = 4 sqrt(3) area / (sum of squared edge lengths)."""
    e = [p1 - p0, p2 - p1, p0 - p2]
    area = 0.5 * math.sqrt(sum(x * x for x in np.cross(p1 - p0, p2 - p0)))
    return 1.0 - 4.0 * math.sqrt(3.0) * area / sum(float(np.dot(x, x)) for x in e)


def _plane_dist2(p, tri):
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    return float(np.dot(p - tri[0], n)) ** 2 / float(np.dot(n, n))


def restated_cost(V, F, inc, a, b, vbar, w_e, w_s):
    """Eq. 1 from its definition: QEM error of the endpoints' quadrics at vbar,
    w_e times the edge length, w_s times the skinny defects of the generated
    triangles.  Returns (cost, number of generated triangles)."""
    q = sum(_plane_dist2(vbar, V[F[f]]) for f in inc[a]) + sum(_plane_dist2(vbar, V[F[f]]) for f in inc[b])
    gen = [f for f in set(inc[a]) | set(inc[b]) if not (a in F[f] and b in F[f])]
    skinny = 0.0
    for f in gen:
        P = [vbar if int(x) in (a, b) else V[x] for x in F[f]]
        skinny += _shape_defect(*P)
    return q + w_e * float(np.linalg.norm(V[a] - V[b])) + w_s * skinny, len(gen)


# ---------------------------------------------------------------- the skinny sum
@pytest.mark.parametrize("mesh", ["ico2", "torus", "crease"])
def test_skinny_sum_restated(mesh):
    """Every edge of the mesh: the oracle's cost equals the restatement (the
    placement is taken from the oracle; it has pins of its own).  Weights are
    large so that a wrong face set (the two vanishing faces counted, one end's
    faces missing) or positions before the collapse change the cost by far more
    than rounding."""
    if mesh == "ico2":
        V, F = g.bumpy_icosphere_gauss(k=2, seed=11)
    elif mesh == "torus":
        V, F = g.bumpy_torus(16, 8, seed=4)
    else:
        V, F = g.crease_sphere(2, 5)
    inc = _incidence(F)
    w_e, w_s = 0.25, 1.0
    for a, b in _edges(F):
        cost, vbar = orc.edge_cost(V, F, a, b, w_e=w_e, w_s=w_s)
        want, ngen = restated_cost(V, F, inc, a, b, vbar, w_e, w_s)
        assert ngen == len(inc[a]) + len(inc[b]) - 4
        assert cost == pytest.approx(want, rel=1e-12, abs=1e-14), (a, b)


def hex_prism(R=3, s=0.125, z_top=0.5, z_bot=0.25):
    """A closed mesh whose top is the regular triangular lattice of spacing s
    over a hexagon of R rings (axial coordinates (i, j), position
    (i + j/2, j sqrt(3)/2) s), its bottom a copy below, and walls between their
    boundaries.  Returns V, F and the vertex ids of lattice points (0, 0) and
    (1, 0)."""
    h = math.sqrt(3.0) / 2.0
    pts = [(i, j) for i in range(-R, R + 1) for j in range(-R, R + 1) if abs(i + j) <= R]
    idx = {p: k for k, p in enumerate(pts)}
    n = len(pts)
    V = np.array([[0.5 + s * (i + 0.5 * j), 0.5 + s * h * j, z_top] for i, j in pts] +
                 [[0.5 + s * (i + 0.5 * j), 0.5 + s * h * j, z_bot] for i, j in pts])
    top = []
    for i, j in pts:
        up = [(i, j), (i + 1, j), (i, j + 1)]
        down = [(i + 1, j), (i + 1, j + 1), (i, j + 1)]
        for t in (up, down):
            if all(p in idx for p in t):
                top.append([idx[p] for p in t])
    directed = {(t[k], t[(k + 1) % 3]) for t in top for k in range(3)}
    boundary = [(u, v) for u, v in directed if (v, u) not in directed]
    faces = list(top) + [[t[0] + n, t[2] + n, t[1] + n] for t in top]
    for u, v in boundary:  # walls: the edge v -> u on top, u' -> v' below
        faces.append([v, u, u + n])
        faces.append([v, u + n, v + n])
    return V, np.array(faces, dtype=np.int32), idx[(0, 0)], idx[(1, 0)]


@pytest.mark.parametrize("w_e,w_s", [(0.001, 0.005), (0.5, 1.0), (0.0, 1.0)])
def test_flat_patch_closed_form(w_e, w_s):
    V, F, a, b = hex_prism()
    assert orc.validate(V, F) == 0
    inc = _incidence(F)
    assert len(inc[a]) == 6 and len(inc[b]) == 6
    cost, vbar = orc.edge_cost(V, F, a, b, w_e=w_e, w_s=w_s)
    # the quadric is singular (one plane): the fallback's three options all
    # have zero error, and the midpoint comes first
    assert np.array_equal(vbar, (V[a] + V[b]) * 0.5)
    want = w_e * 0.125 + w_s * 34.0 / 35.0
    assert cost == pytest.approx(want, rel=1e-13, abs=1e-15)


# ---------------------------------------------------------------- exact-target cap
@pytest.mark.parametrize("mesh,need", [("ico3", 1), ("ico3", 9), ("ico3", 40), ("nested", 7), ("nested", 20)])
def test_cap_keeps_smallest_keys(mesh, need):
    """When more candidates pass the local checks than the round needs, the
    ones kept (committed, or undone by the intersection check) are the `need`
    passing candidates of smallest key; the rest are capped (reason 4)."""
    if mesh == "ico3":
        V, F = g.bumpy_icosphere_gauss(k=3, seed=6)
    else:
        V, F = g.nested_spheres(k=3, gap=0.004)
    target = len(F) - 2 * need
    cand, _, reason, _ = orc.check(V, F, target)
    keys = orc.keys(V, F)
    ck = keys[cand].astype(np.uint64)
    passing = np.isin(reason, (0, 3, 4))
    kept = np.isin(reason, (0, 3))
    capped = reason == 4
    assert passing.sum() > need, "the fixture must make the cap bind"
    assert kept.sum() == need
    want = np.sort(ck[passing])[:need]
    assert np.array_equal(np.sort(ck[kept]), want)
    assert ck[kept].max() < ck[capped].min()


def test_cap_absent_when_enough_faces_remain():
    V, F = g.bumpy_icosphere_gauss(k=3, seed=6)
    _, _, reason, _ = orc.check(V, F, 16)
    assert not np.any(reason == 4)
