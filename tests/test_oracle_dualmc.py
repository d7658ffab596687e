"""The volume-to-mesh step (Dual Marching Cubes, Sec. 4.2) in the oracle.
Pins that do not reuse its construction: the number of patches of every cube
configuration against the region count of the cube (positive corners joined
along edges, negative ones also across face diagonals), closed-form fields
(a plane, a sphere, a torus, two spheres) through Euler characteristics,
orientation, positions and the exact intersection-free check, and random
grids through closed edge- and vertex-manifoldness."""
from collections import Counter, defaultdict

import numpy as np
import pytest

import oracle.oracle as orc
from oracle import dualmc as dm
from oracle import udf as ou


def _components(nodes, adj):
    seen, n = set(), 0
    for x in nodes:
        if x in seen:
            continue
        n += 1
        stack = [x]
        seen.add(x)
        while stack:
            y = stack.pop()
            for z in adj(y):
                if z in nodes and z not in seen:
                    seen.add(z)
                    stack.append(z)
    return n


def test_patch_count_is_the_cube_region_count_minus_one():
    # disjoint disk patches cut the cube into patches + 1 regions: positive
    # corners joined along edges, negative corners along edges and face
    # diagonals (the ambiguous faces keep the negative region connected)
    def edge_nb(c):
        return [c ^ 1, c ^ 2, c ^ 4]

    def face_nb(c):
        return edge_nb(c) + [c ^ 3, c ^ 5, c ^ 6]

    for config in range(256):
        pos = {c for c in range(8) if (config >> c) & 1}
        neg = set(range(8)) - pos
        want = 0 if not pos or not neg else _components(pos, edge_nb) + _components(neg, face_nb) - 1
        assert len(dm.patches(config)) == want, config
        # the patches partition the valid edges
        valid = {e for e, (a, b) in enumerate(dm.EDGES) if ((config >> a) & 1) != ((config >> b) & 1)}
        got = [e for p in dm.patches(config) for e in p]
        assert sorted(got) == sorted(valid)


def _euler(V, F):
    E = {tuple(sorted((int(a), int(b)))) for t in F for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    return len(V) - len(E) + len(F)


def _manifold(F):
    de = Counter()
    for t in F:
        for x, y in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            de[(int(x), int(y))] += 1
    if not all(c == 1 and de[(y, x)] == 1 for (x, y), c in de.items()):
        return False
    star = defaultdict(dict)
    for t in F:
        for q in range(3):
            star[int(t[q])][int(t[(q + 1) % 3])] = int(t[(q + 2) % 3])
    for v, nxt in star.items():
        x0 = next(iter(nxt))
        x, n = x0, 0
        while True:
            x = nxt[x]
            n += 1
            if x == x0 or n > len(nxt):
                break
        if n != len(nxt):
            return False
    return True


def _volume(V, F):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6)


def test_sphere():
    R, r = 20, 0.3
    C = ou.centres(R)
    S = np.linalg.norm(C - 0.5, axis=-1) - r
    V, F = dm.dualmc(S)
    assert _euler(V, F) == 2 and _manifold(F) and orc.validate(V, F) == 0
    assert abs(_volume(V, F) / (4 / 3 * np.pi * r ** 3) - 1) < 0.05  # outward
    d = np.linalg.norm(V - 0.5, axis=1) - r
    assert np.abs(d).max() < 1.0 / R


def test_plane_vertices_lie_on_it():
    # a linear field is interpolated exactly: every vertex on the plane
    R, c = 10, 0.43
    S = ou.centres(R)[..., 2] - c  # an open sheet: no quads on the grid's border
    V, F = dm.dualmc(S)
    assert len(V) > 0 and np.abs(V[:, 2] - c).max() < 1e-15


def test_torus_and_two_spheres():
    R = 24
    C = ou.centres(R)
    q = np.sqrt((C[..., 0] - 0.5) ** 2 + (C[..., 1] - 0.5) ** 2) - 0.28
    S = np.sqrt(q ** 2 + (C[..., 2] - 0.5) ** 2) - 0.1
    V, F = dm.dualmc(S)
    assert _euler(V, F) == 0 and _manifold(F) and orc.validate(V, F) == 0
    S2 = np.minimum(np.linalg.norm(C - [0.3, 0.5, 0.5], axis=-1) - 0.15,
                    np.linalg.norm(C - [0.7, 0.5, 0.5], axis=-1) - 0.15)
    V2, F2 = dm.dualmc(S2)
    assert _euler(V2, F2) == 4 and _manifold(F2)


@pytest.mark.parametrize("seed", range(6))
def test_random_grids_are_closed_manifolds(seed):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((8, 8, 8)) + rng.normal() * 0.3
    S[0] = S[-1] = 1.0
    S[:, 0] = S[:, -1] = 1.0
    S[:, :, 0] = S[:, :, -1] = 1.0
    V, F = dm.dualmc(S)
    assert len(F) > 0 and _manifold(F)


def test_smoothed_crossing_on_planes():
    # Appendix 2.1: the crossing fraction t (the plane's place between two grid
    # points, known from its position) becomes 1 / (1 + exp(-beta (t - 1/2)));
    # a plane midway between grid points stays put, others move towards the middle
    R, beta = 10, 5.0
    for c, t in ((0.4, 0.5), (0.43, 0.8), (0.361, 0.11)):
        S = ou.centres(R)[..., 2] - c  # z - c: crosses between points k and k + 1, k = 3
        V, F = dm.dualmc(S, beta)
        V0, F0 = dm.dualmc(S)
        want = (3.5 + 1.0 / (1.0 + np.exp(-beta * (t - 0.5)))) / R
        assert np.abs(V[:, 2] - want).max() < 1e-12
        assert np.abs(V0[:, 2] - (3.5 + t) / R).max() < 1e-12
        assert np.array_equal(V[:, :2], V0[:, :2])


def test_smoothed_sphere_keeps_topology():
    S = np.linalg.norm(ou.centres(16) - 0.5, axis=-1) - 0.3
    V, F = dm.dualmc(S, 5.0)
    assert _euler(V, F) == 2 and _manifold(F)
    assert np.abs(np.linalg.norm(V - 0.5, axis=1) - 0.3).max() < 1.0 / 16


# ---------------------------------------------------------------- envelope quad division (Appendix 2.1)
def _reflex_2d(P, i):
    """interior angle of vertex i of the counter-clockwise polygon P (2D) above 180 degrees"""
    a, b, c = P[i - 1], P[i], P[(i + 1) % len(P)]
    return (b[0] - a[0]) * (c[1] - b[1]) - (b[1] - a[1]) * (c[0] - b[0]) < 0


def _star_quad(rng, reflex=None):
    """a planar quad at z = 0 around the z axis, counter-clockwise seen from +z,
    star-shaped from the axis (angles increasing), radius of vertex `reflex` shrunk"""
    ang = np.sort(rng.uniform(0, 2 * np.pi, 4))
    while np.max(np.diff(np.r_[ang, ang[0] + 2 * np.pi])) > 0.8 * np.pi:
        ang = np.sort(rng.uniform(0, 2 * np.pi, 4))
    rad = rng.uniform(0.5, 1.0, 4)
    if reflex is not None:
        rad[reflex] = rng.uniform(0.02, 0.15)
    return [(float(r * np.cos(t)), float(r * np.sin(t)), 0.0) for r, t in zip(rad, ang)]


def test_concavity_is_the_reflex_angle_of_planar_quads():
    """For a quad in the plane across the edge (p+ above, p- below), the
    triple-product test marks exactly the vertices whose interior angle
    exceeds 180 degrees, found here from the plane polygon alone."""
    rng = np.random.default_rng(21)
    pp, pn = (0.0, 0.0, 1.0), (0.0, 0.0, -1.0)
    seen = Counter()
    for trial in range(400):
        q = _star_quad(rng, reflex=trial % 5 if trial % 5 < 4 else None)
        for i in range(4):
            want = _reflex_2d([(x, y) for x, y, _ in q], i)
            assert dm.concave(q[i], q[i - 1], q[(i + 1) % 4], pp, pn) == want
            seen[want] += 1
    assert seen[True] > 100 and seen[False] > 100


def test_split_goes_through_the_concave_vertex():
    """A planar quad with one reflex vertex is split along the diagonal through
    it, and both triangles keep the quad's orientation (neither is inverted)."""
    rng = np.random.default_rng(22)
    pp, pn = (0.0, 0.0, 1.0), (0.0, 0.0, -1.0)
    for trial in range(200):
        i = trial % 4
        q = _star_quad(rng, reflex=i)
        if sum(_reflex_2d([(x, y) for x, y, _ in q], k) for k in range(4)) != 1:
            continue
        kind = dm.divide_quad(q, pp, pn)
        assert kind == ("A" if i % 2 == 0 else "B")
        tris = [(0, 1, 2), (0, 2, 3)] if kind == "A" else [(0, 1, 3), (1, 2, 3)]
        for a, b, c in tris:
            ux, uy = q[b][0] - q[a][0], q[b][1] - q[a][1]
            wx, wy = q[c][0] - q[a][0], q[c][1] - q[a][1]
            assert ux * wy - uy * wx > 0


def test_convex_quads_take_the_larger_smallest_angle():
    """Without concave vertices the split maximises the smallest angle of its
    two triangles (brute force with arc cosines)."""
    import math
    rng = np.random.default_rng(23)

    def min_angle(p, q, r):
        out = 10.0
        for a, b, c in ((p, q, r), (q, r, p), (r, p, q)):
            u, w = np.subtract(b, a), np.subtract(c, a)
            out = min(out, math.acos(max(-1.0, min(1.0, float(u @ w) / (np.linalg.norm(u) * np.linalg.norm(w))))))
        return out
    n = 0
    for _ in range(300):
        q = [(x, y, float(rng.uniform(-0.2, 0.2))) for x, y, _ in _star_quad(rng)]
        pp, pn = (0.0, 0.0, 1.0), (0.0, 0.0, -1.0)
        if any(dm.concave(q[i], q[i - 1], q[(i + 1) % 4], pp, pn) for i in range(4)):
            continue
        a = min(min_angle(q[0], q[1], q[2]), min_angle(q[0], q[2], q[3]))
        b = min(min_angle(q[0], q[1], q[3]), min_angle(q[1], q[2], q[3]))
        if abs(a - b) < 1e-9:
            continue
        assert dm.divide_quad(q, pp, pn) == ("A" if a > b else "B")
        n += 1
    assert n > 200


def test_both_diagonals_concave_gives_four_triangles():
    """A twisted quad going round the edge whose concave vertices (exact
    rational triple products) lie on both diagonals becomes four triangles;
    with the concave vertex on one diagonal only, that diagonal is taken."""
    from fractions import Fraction as Fr

    def triple_exact(v, l, r, p):
        a = [Fr(l[k]) - Fr(p[k]) for k in range(3)]
        b = [Fr(r[k]) - Fr(p[k]) for k in range(3)]
        c = [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]
        return sum((Fr(v[k]) - Fr(p[k])) * c[k] for k in range(3))

    pp, pn = (0.0, 0.0, 2.0), (0.0, 0.0, -2.0)
    q = [(3.0, 1.0, 1.0), (0.0, 3.0, -2.0), (-1.0, 1.0, 1.0), (-3.0, -2.0, 1.0)]
    conc = [triple_exact(q[i], q[i - 1], q[(i + 1) % 4], pp) < 0 or triple_exact(q[i], q[i - 1], q[(i + 1) % 4], pn) > 0
            for i in range(4)]
    assert conc == [False, True, True, False]
    assert [dm.concave(q[i], q[i - 1], q[(i + 1) % 4], pp, pn) for i in range(4)] == conc
    assert dm.divide_quad(q, pp, pn) == "E"
    flat = [(x, y, 0.0) for x, y, _ in q]  # planar: only the reflex vertex 2 is concave
    assert [dm.concave(flat[i], flat[i - 1], flat[(i + 1) % 4], pp, pn) for i in range(4)] == [False, False, True, False]
    assert dm.divide_quad(flat, pp, pn) == "A"


def _rough_grid(seed, n=10):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((n, n, n)) * rng.uniform(0.2, 3) + rng.normal() * 0.3
    S[0] = S[-1] = 1.0
    S[:, 0] = S[:, -1] = 1.0
    S[:, :, 0] = S[:, :, -1] = 1.0
    return S


@pytest.mark.parametrize("beta", [0.0, 5.0])
def test_extra_vertices_sit_on_their_grid_edges(beta):
    """Every vertex beyond the patch vertices belongs to a four-triangle quad:
    it lies on a crossed grid edge at that edge's (smoothed) crossing, and its
    four triangles form a closed fan around it."""
    import math
    found = 0
    for seed in range(12):
        S = _rough_grid(seed)
        info = {}
        V, F = dm.dualmc(S, beta, info)
        R = S.shape[0]
        for v in range(info["patch_vertices"], len(V)):
            p = V[v] * R - 0.5
            g = np.floor(p + 1e-12).astype(int)
            a = int(np.argmax(np.abs(p - np.round(p))))  # the edge's axis: the non-integer coordinate
            g0 = tuple(int(round(x)) if ax != a else int(g[a]) for ax, x in enumerate(p))
            g1 = list(g0)
            g1[a] += 1
            s0, s1 = S[g0], S[tuple(g1)]
            assert (s0 >= 0) != (s1 >= 0)
            t = s0 / (s0 - s1)
            if beta > 0:
                t = 1.0 / (1.0 + math.exp(-beta * (t - 0.5)))
            assert abs(p[a] - (g0[a] + t)) < 1e-12
            ring = F[np.any(F == v, axis=1)]
            others = [int(x) for t3 in ring for x in t3 if x != v]
            assert all(c == 2 for c in Counter(others).values())
            found += 1
        assert _manifold(F) and orc.validate(V, F) == 0
    assert found > 0


def test_envelope_division_is_intersection_free_on_rough_grids():
    for seed in range(8):
        for beta in (0.0, 5.0):
            V, F = dm.dualmc(_rough_grid(100 + seed), beta)
            assert orc.validate(V, F) == 0
            assert len(orc.self_intersections(V, F)) == 0
