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
positive one.

Quad division by the envelope of the edge (Appendix 2.1): with p+ and p- the
positive and negative ends of the grid edge and l, r the quad neighbours of
vertex v (before and after it in the quad's order), v is concave when
(v - p+) . ((l - p+) x (r - p+)) < 0 or (v - p-) . ((l - p-) x (r - p-)) > 0.
A quad whose concave vertices lie on one diagonal only is split along that
diagonal; one with concave vertices on both diagonals becomes four triangles
around an extra vertex on the grid edge, at the edge's (smoothed) crossing
point; one without concave vertices is split along the diagonal that gives
the larger smallest angle (v0 v2 on a tie).  Vertices are numbered by (cube,
patch), cubes in index order i, then j, then k, then the extra edge vertices
in quad order; quads by (axis, grid point) in the same order, two or four
triangles each.
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


def _triple(v, l, r, p):
    """(v - p) . ((l - p) x (r - p)), in this order of operations"""
    ax, ay, az = l[0] - p[0], l[1] - p[1], l[2] - p[2]
    bx, by, bz = r[0] - p[0], r[1] - p[1], r[2] - p[2]
    cx = ay * bz - az * by
    cy = az * bx - ax * bz
    cz = ax * by - ay * bx
    return (v[0] - p[0]) * cx + (v[1] - p[1]) * cy + (v[2] - p[2]) * cz


def concave(v, l, r, ppos, pneg) -> bool:
    """the concavity test of Appendix 2.1 for quad vertex v between l and r"""
    return _triple(v, l, r, ppos) < 0.0 or _triple(v, l, r, pneg) > 0.0


def _worst_cos(p, q, r):
    """the largest cosine of the three angles of triangle pqr (its smallest
    angle's cosine); 1 where an edge has zero length"""
    import math
    out = -2.0
    for a, b, c in ((p, q, r), (q, r, p), (r, p, q)):
        ux, uy, uz = b[0] - a[0], b[1] - a[1], b[2] - a[2]
        wx, wy, wz = c[0] - a[0], c[1] - a[1], c[2] - a[2]
        uu = ux * ux + uy * uy + uz * uz
        ww = wx * wx + wy * wy + wz * wz
        if uu == 0.0 or ww == 0.0:
            cs = 1.0
        else:
            cs = (ux * wx + uy * wy + uz * wz) / (math.sqrt(uu) * math.sqrt(ww))
        out = cs if cs > out else out
    return out


def divide_quad(q, ppos, pneg):
    """the division of quad q (four positions, oriented) around the grid edge
    with positive end ppos and negative end pneg: 'A' (along v0 v2), 'B' (along
    v1 v3) or 'E' (four triangles around an extra vertex on the edge)"""
    conc = [concave(q[i], q[(i + 3) % 4], q[(i + 1) % 4], ppos, pneg) for i in range(4)]
    on_a, on_b = conc[0] or conc[2], conc[1] or conc[3]
    if on_a and on_b:
        return "E"
    if on_a:
        return "A"
    if on_b:
        return "B"
    wa = max(_worst_cos(q[0], q[1], q[2]), _worst_cos(q[0], q[2], q[3]))
    wb = max(_worst_cos(q[0], q[1], q[3]), _worst_cos(q[1], q[2], q[3]))
    return "A" if wa <= wb else "B"


def crossing(S, g0, g1, axis, beta):
    """the surface's crossing point on the grid edge g0 -> g0 + axis (t from
    the lower end g0, smoothed when beta > 0)"""
    import math
    R = S.shape[0]
    s0, s1 = S[g0], S[g1]
    t = s0 / (s0 - s1)
    if beta > 0:
        t = 1.0 / (1.0 + math.exp(-beta * (t - 0.5)))
    q = [g0[0] + 0.5, g0[1] + 0.5, g0[2] + 0.5]
    q[axis] = q[axis] + t
    return (q[0] / R, q[1] / R, q[2] / R)


def dualmc(S, beta: float = 0.0, info: dict | None = None):
    """S: (R, R, R) float64 grid values -> (V (n, 3) float64, F (m, 3) int32);
    info (optional) gets "patch_vertices", the number of vertices before the
    extra edge vertices, and "kinds", the division of every quad in order
    ('A', 'B' or 'E')"""
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
    extra = []  # extra vertices on grid edges (four-triangle quads), in quad order
    kinds = []
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
                    pt0 = tuple((g[x] + 0.5) / R for x in range(3))
                    pt1 = tuple((g1[x] + 0.5) / R for x in range(3))
                    kind = divide_quad(q, pt0 if p0 else pt1, pt1 if p0 else pt0)
                    kinds.append(kind)
                    if kind == "A":
                        Fo += [(ring[0], ring[1], ring[2]), (ring[0], ring[2], ring[3])]
                    elif kind == "B":
                        Fo += [(ring[0], ring[1], ring[3]), (ring[1], ring[2], ring[3])]
                    else:
                        ve = -1 - len(extra)  # numbered after every patch vertex
                        extra.append(crossing(S, tuple(g), tuple(g1), a, beta))
                        Fo += [(ring[i], ring[(i + 1) % 4], ve) for i in range(4)]
    nv = len(V)
    if info is not None:
        info["patch_vertices"] = nv
        info["kinds"] = kinds
    V = V + extra
    Fo = [tuple(x if x >= 0 else nv + (-1 - x) for x in t) for t in Fo]
    return np.array(V, dtype=np.float64).reshape(-1, 3), np.array(Fo, dtype=np.int32).reshape(-1, 3)
