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
