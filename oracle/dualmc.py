"""TEST INFRASTRUCTURE ONLY: the remeshing stage's volume-to-mesh step
(Sec. 4.2), Dual Marching Cubes on a grid of signed values, written from its
definition with plain loops (small grids).

Grid point (i, j, k) sits at ((i + 1/2) / R, (j + 1/2) / R, (k + 1/2) / R)
with value s[i, j, k]; a point is positive when s >= 0 (outside).  A cube is
the 2x2x2 block of points from (i, j, k); a cube edge is valid when its two
ends differ in sign, and the surface crosses it at the linear interpolation
point t = s0 / (s0 - s1) from the lower end.

Patches: on each cube face the valid edges are linked in pairs where the
surface crosses the face.  A face with two valid edges links them; a face
with four (diagonal corners of equal sign, "ambiguous") links the two edges
at each positive corner, unless the face is flipped, then the two at each
negative corner.  Every valid edge lies on two faces, so the links form
cycles: the patches of the cube, numbered by their smallest edge id.

Shared ambiguous faces (the paper's manifold fix for Dual Marching Cubes):
when both cubes of an ambiguous face have, unflipped, one patch holding all
four of its edges, the dual edge between those patches would be shared by
four quads; the face is then flipped in both cubes.  This splits both
patches, keeps the two cubes consistent, and merges no patch elsewhere, so
one pass over the faces suffices.

A patch's vertex is the mean of its edges' crossing points (each divided by
R, summed in ascending edge id, then divided by their number).  With beta > 0
the crossing uses the smoothed fraction t' = 1 / (1 + exp(-beta (t - 1/2)))
instead of t (Appendix 2.1, the paper takes beta = 5), which keeps vertices
away from the cube corners; beta = 0 is the plain linear crossing.  Quads: every
valid grid edge whose four surrounding cubes exist joins the vertices of the
patches holding it in those cubes, ordered right-handed around the edge's
axis and oriented so that the normal points from the negative end to the
positive one; a quad is split along its shorter diagonal (v0 v2 on a tie).
Vertices are numbered by (cube, patch), cubes in index order i, then j, then
k; quads by (axis, grid point) in the same order.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np


def _edge_corners(e):
    """cube edge e = 4 a + u + 2 v: axis a, the other two coordinates (u, v)
    in increasing axis order; corners c have bit 0 = x, bit 1 = y, bit 2 = z"""
    a, r = divmod(e, 4)
    u, v = r % 2, r // 2
    others = [ax for ax in range(3) if ax != a]
    c0 = (u << others[0]) | (v << others[1])
    return c0, c0 | (1 << a)


EDGES = [_edge_corners(e) for e in range(12)]
# face 2 a + w: the four edges where coordinate a equals w
FACES = [[e for e, (c0, c1) in enumerate(EDGES) if ((c0 >> a) & 1) == w and ((c1 >> a) & 1) == w]
         for a in range(3) for w in range(2)]


def patches(config: int, flips: int = 0):
    """the patches (ascending edge ids) of a cube whose corner c is positive
    iff bit c of config is set; bit f of flips flips the ambiguous face f"""
    pos = [(config >> c) & 1 for c in range(8)]
    valid = [e for e in range(12) if pos[EDGES[e][0]] != pos[EDGES[e][1]]]
    link = {e: [] for e in valid}
    for f, fe in enumerate(FACES):
        ve = [e for e in fe if e in link]
        if len(ve) == 2:
            link[ve[0]].append(ve[1])
            link[ve[1]].append(ve[0])
        elif len(ve) == 4:
            cut = 0 if (flips >> f) & 1 else 1
            for c in sorted(set(x for e in fe for x in EDGES[e])):
                if pos[c] == cut:
                    pair = [e for e in ve if c in EDGES[e]]
                    link[pair[0]].append(pair[1])
                    link[pair[1]].append(pair[0])
    seen, out = set(), []
    for e in valid:
        if e in seen:
            continue
        comp, stack = [], [e]
        seen.add(e)
        while stack:
            x = stack.pop()
            comp.append(x)
            for y in link[x]:
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
        out.append(sorted(comp))
    return out


def holds_face(config: int, f: int) -> bool:
    """one unflipped patch holds all four edges of face f"""
    return any(all(e in p for e in FACES[f]) for p in patches(config))


def dualmc(S, beta: float = 0.0):
    """S: (R, R, R) float64 grid values -> (V (n, 3) float64, F (m, 3) int32)"""
    import math
    S = np.asarray(S, dtype=np.float64)
    R = S.shape[0]
    P = S >= 0

    def cfg(i, j, k):
        c = 0
        for b in range(8):
            if P[i + (b & 1), j + ((b >> 1) & 1), k + ((b >> 2) & 1)]:
                c |= 1 << b
        return c

    flips = defaultdict(int)
    for i in range(R - 1):
        for j in range(R - 1):
            for k in range(R - 1):
                for a in range(3):
                    n = [i, j, k]
                    n[a] += 1
                    if n[a] > R - 2:
                        continue
                    if holds_face(cfg(i, j, k), 2 * a + 1) and holds_face(cfg(*n), 2 * a):
                        flips[(i, j, k)] |= 1 << (2 * a + 1)
                        flips[tuple(n)] |= 1 << (2 * a)
    vid = {}
    V = []
    for i in range(R - 1):
        for j in range(R - 1):
            for k in range(R - 1):
                for pi, pe in enumerate(patches(cfg(i, j, k), flips[(i, j, k)])):
                    sx = sy = sz = 0.0
                    for e in pe:
                        c0, c1 = EDGES[e]
                        g0 = (i + (c0 & 1), j + ((c0 >> 1) & 1), k + ((c0 >> 2) & 1))
                        g1 = (i + (c1 & 1), j + ((c1 >> 1) & 1), k + ((c1 >> 2) & 1))
                        s0, s1 = S[g0], S[g1]
                        t = s0 / (s0 - s1)
                        if beta > 0:
                            t = 1.0 / (1.0 + math.exp(-beta * (t - 0.5)))
                        q = [g0[0] + 0.5, g0[1] + 0.5, g0[2] + 0.5]
                        q[e // 4] = q[e // 4] + t
                        sx += q[0] / R
                        sy += q[1] / R
                        sz += q[2] / R
                    vid[(i, j, k, pi)] = len(V)
                    V.append((sx / len(pe), sy / len(pe), sz / len(pe)))

    def patch_of(cube, e):
        for pi, pe in enumerate(patches(cfg(*cube), flips[tuple(cube)])):
            if e in pe:
                return vid[(*cube, pi)]
        raise AssertionError("a valid edge outside every patch")

    Fo = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3  # right-handed around the axis
        for i in range(R):
            for j in range(R):
                for k in range(R):
                    g = [i, j, k]
                    if g[a] > R - 2 or g[b] < 1 or g[b] > R - 2 or g[c] < 1 or g[c] > R - 2:
                        continue
                    g1 = list(g)
                    g1[a] += 1
                    p0, p1 = P[tuple(g)], P[tuple(g1)]
                    if p0 == p1:
                        continue
                    ring = []
                    for db, dc in ((-1, -1), (0, -1), (0, 0), (-1, 0)):
                        cube = list(g)
                        cube[b] += db
                        cube[c] += dc
                        lb, lc = -db, -dc  # the grid edge in the cube's own coordinates
                        u, v = (lb, lc) if b < c else (lc, lb)
                        ring.append(patch_of(tuple(cube), 4 * a + u + 2 * v))
                    if p0:  # positive at the lower end: the normal points down the axis
                        ring = [ring[0], ring[3], ring[2], ring[1]]
                    q = [V[x] for x in ring]

                    def dist2(x, y):
                        dx, dy, dz = x[0] - y[0], x[1] - y[1], x[2] - y[2]
                        return dx * dx + dy * dy + dz * dz
                    d02, d13 = dist2(q[0], q[2]), dist2(q[1], q[3])
                    if d02 <= d13:
                        Fo += [(ring[0], ring[1], ring[2]), (ring[0], ring[2], ring[3])]
                    else:
                        Fo += [(ring[0], ring[1], ring[3]), (ring[1], ring[2], ring[3])]
    return np.array(V, dtype=np.float64).reshape(-1, 3), np.array(Fo, dtype=np.int32).reshape(-1, 3)
