"""Seeded synthetic mesh generators.

This module only builds input meshes (vertex positions in float64, faces as
int32 triangles, counter-clockwise seen from outside).  It holds none of the
simplification arithmetic, so both the CPU oracle tests and the GPU path may
take their inputs from it.

The meshes stand in for the remeshed Thingi10K inputs the paper evaluates on
(Sec. 4 produces uniform, well-shaped, watertight, intersection-free triangle
meshes; Sec. 8 reports on 100 meshes of >300k faces, 722,472 faces on average).
Uniform icosphere and torus triangulations have that structure.  Every mesh is
scaled uniformly into [0,1]^3 (Sec. 3: inputs are normalised to the unit cube).
"""
from __future__ import annotations

import math

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


# --------------------------------------------------------------------------
# counter-based hash (SplitMix64, Steele/Lea/Flood 2014) for lattice values
# --------------------------------------------------------------------------
def _splitmix64(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _lattice_value(seed: int, octave: int, ix, iy, iz) -> np.ndarray:
    """Value in [-1, 1) for integer lattice point (ix, iy, iz) of one octave."""
    h = _splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    h = _splitmix64(h ^ np.uint64(octave))
    for c in (ix, iy, iz):
        c = np.asarray(c, dtype=np.int64).astype(np.uint64)
        h = _splitmix64(h ^ c)
    u = (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def value_noise(p: np.ndarray, freq: float, seed: int, octave: int) -> np.ndarray:
    """Smoothstep-weighted trilinear value noise at points p (n,3)."""
    q = p * freq
    i0 = np.floor(q).astype(np.int64)
    t = q - i0
    w = t * t * (3.0 - 2.0 * t)
    out = np.zeros(len(p))
    for dx in (0, 1):
        wx = w[:, 0] if dx else 1.0 - w[:, 0]
        for dy in (0, 1):
            wy = w[:, 1] if dy else 1.0 - w[:, 1]
            for dz in (0, 1):
                wz = w[:, 2] if dz else 1.0 - w[:, 2]
                val = _lattice_value(seed, octave, i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz)
                out += wx * wy * wz * val
    return out


# --------------------------------------------------------------------------
# base shapes
# --------------------------------------------------------------------------
def icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array(
        [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
         [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
         [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v, f


def icosphere(k: int):
    """Icosahedron refined k times by 4-to-1 midpoint subdivision, each round
    re-projected onto the unit sphere.  V = 10*4^k + 2, F = 20*4^k.
    Children of face i are faces 4i..4i+3; new vertices follow the old ones,
    ordered by their (min, max) parent-edge key."""
    v, f = icosahedron()
    for _ in range(k):
        nv = len(v)
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        lo = np.minimum(e[:, 0], e[:, 1])
        hi = np.maximum(e[:, 0], e[:, 1])
        key = lo * nv + hi
        uk, inv = np.unique(key, return_inverse=True)
        mids = (v[uk // nv] + v[uk % nv]) * 0.5
        mids /= np.linalg.norm(mids, axis=1, keepdims=True)
        m = inv.reshape(3, -1).T + nv  # m[:,0]=mid(f0,f1), m[:,1]=mid(f1,f2), m[:,2]=mid(f2,f0)
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        ab, bc, ca = m[:, 0], m[:, 1], m[:, 2]
        nf = np.stack([np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
                       np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)], 1)
        f = nf.reshape(-1, 3)
        v = np.concatenate([v, mids])
    return v, f


def geodesic_sphere(n: int):
    """Class-I geodesic sphere of frequency n (every icosahedron face cut by a
    barycentric lattice into n^2 triangles), projected onto the unit sphere.
    V = 10 n^2 + 2, F = 20 n^2."""
    v0, f0 = icosahedron()
    if n == 1:
        return v0.copy(), f0.copy()
    # canonical ids: corners, then edge-interior points, then face-interior points
    edges = {}
    for fi in range(20):
        for c in range(3):
            a, b = int(f0[fi, c]), int(f0[fi, (c + 1) % 3])
            edges.setdefault((min(a, b), max(a, b)), len(edges))
    ne = len(edges)
    n_edge_pts = n - 1
    n_face_pts = (n - 1) * (n - 2) // 2
    base_edge = 12
    base_face = 12 + ne * n_edge_pts
    nvert = base_face + 20 * n_face_pts
    pos = np.zeros((nvert, 3))
    pos[:12] = v0

    faces = []
    for fi in range(20):
        A, B, C = (int(x) for x in f0[fi])
        # lattice point (i, j): P = A + (B-A) i/n + (C-A) j/n, i + j <= n
        ids = {}
        interior = 0
        for i in range(n + 1):
            for j in range(n + 1 - i):
                k = n - i - j
                if i == 0 and j == 0:
                    vid = A
                elif i == n:
                    vid = B
                elif j == n:
                    vid = C
                elif j == 0:      # on edge A-B, parameter i
                    vid = _edge_pt(edges, base_edge, n, A, B, i)
                elif i == 0:      # on edge A-C, parameter j
                    vid = _edge_pt(edges, base_edge, n, A, C, j)
                elif k == 0:      # on edge B-C, parameter j (from B)
                    vid = _edge_pt(edges, base_edge, n, B, C, j)
                else:
                    vid = base_face + fi * n_face_pts + interior
                    interior += 1
                ids[(i, j)] = vid
                p = v0[A] * (k / n) + v0[B] * (i / n) + v0[C] * (j / n)
                pos[vid] = p
        for i in range(n):
            for j in range(n - i):
                faces.append((ids[(i, j)], ids[(i + 1, j)], ids[(i, j + 1)]))
                if i + j + 1 < n:
                    faces.append((ids[(i + 1, j)], ids[(i + 1, j + 1)], ids[(i, j + 1)]))
    pos /= np.linalg.norm(pos, axis=1, keepdims=True)
    return pos, np.asarray(faces, dtype=np.int64)


def _edge_pt(edges, base, n, a, b, t):
    """Id of the point at parameter t/n from a towards b on icosahedron edge ab."""
    e = edges[(min(a, b), max(a, b))]
    s = t if a < b else n - t
    return base + e * (n - 1) + (s - 1)


def torus(n: int, m: int, R: float = 1.0, r: float = 0.35):
    """Torus with n major and m minor segments; quad (i,j) is split along its
    (i,j)-(i+1,j+1) diagonal.  Returns positions, faces, unit normals."""
    i = np.arange(n)
    j = np.arange(m)
    th = 2.0 * np.pi * i / n
    ph = 2.0 * np.pi * j / m
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    x = (R + r * np.cos(PH)) * np.cos(TH)
    y = (R + r * np.cos(PH)) * np.sin(TH)
    z = r * np.sin(PH)
    nrm = np.stack([np.cos(PH) * np.cos(TH), np.cos(PH) * np.sin(TH), np.sin(PH)], -1)
    v = np.stack([x, y, z], -1).reshape(-1, 3)
    nrm = nrm.reshape(-1, 3)
    I, J = np.meshgrid(i, j, indexing="ij")
    I1 = (I + 1) % n
    J1 = (J + 1) % m
    a = (I * m + J).ravel()
    b = (I1 * m + J).ravel()
    c = (I1 * m + J1).ravel()
    d = (I * m + J1).ravel()
    f = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    # interleave so the two halves of a quad are neighbours in slot order
    f = f.reshape(2, -1, 3).transpose(1, 0, 2).reshape(-1, 3)
    # orient outward
    p0, p1, p2 = v[f[0, 0]], v[f[0, 1]], v[f[0, 2]]
    nn = np.cross(p1 - p0, p2 - p0)
    if np.dot(nn, nrm[f[0, 0]]) < 0:
        f = f[:, [0, 2, 1]]
    return v, f, nrm


def grid_cube(n: int = 6):
    """Unit cube with every side an n x n grid of squares, each split along the
    same diagonal, outward: flat sides whose collapses can make exactly
    collinear triangles (the degeneracy test's exact case)."""
    keys, verts, faces = {}, [], []

    def vid(p):
        k = tuple(int(round(c * n)) for c in p)
        if k not in keys:
            keys[k] = len(verts)
            verts.append([c / n for c in k])
        return keys[k]

    for axis in range(3):
        for side in (0, 1):
            u, w = (axis + 1) % 3, (axis + 2) % 3
            for i in range(n):
                for j in range(n):
                    q = []
                    for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0.0, 0.0, 0.0]
                        p[axis], p[u], p[w] = float(side), (i + di) / n, (j + dj) / n
                        q.append(vid(p))
                    faces += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
    v = np.asarray(verts, dtype=np.float64)
    f = np.asarray(faces)
    p0, p1, p2 = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    out = np.einsum("ij,ij->i", np.cross(p1 - p0, p2 - p0), (p0 + p1 + p2) / 3 - 0.5) < 0
    f[out] = f[out][:, [0, 2, 1]]
    return _pack(v, f)


def normalize_unit_cube(v: np.ndarray) -> np.ndarray:
    """Uniform scaling into [0,1]^3: subtract the bbox min, divide by the max extent."""
    lo = v.min(axis=0)
    ext = (v.max(axis=0) - lo).max()
    return (v - lo) / ext


def _pack(v, f):
    return np.ascontiguousarray(v, dtype=np.float64), np.ascontiguousarray(f, dtype=np.int32)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
def bumpy_icosphere_gauss(k: int = 4, seed: int = 1, sigma: float = 0.02):
    """Icosphere(k) with per-vertex radius clip(1 + sigma*N(0,1), 0.9, 1.1).
    k=4, seed=1: 2,562 vertices / 5,120 faces (the small CPU-seconds case)."""
    u, f = icosphere(k)
    z = np.random.default_rng(seed).standard_normal(len(u))
    r = np.clip(1.0 + sigma * z, 0.9, 1.1)
    return _pack(normalize_unit_cube(u * r[:, None]), f)


def noise_radius(u: np.ndarray, seed: int, octaves: int = 6, amp: float = 0.05) -> np.ndarray:
    r = np.ones(len(u))
    for k in range(octaves):
        r += (amp / 2 ** k) * value_noise(u, 4.0 * 2 ** k, seed, k)
    return r


def noisy_icosphere(k: int = 8, seed: int = 2):
    """Icosphere(k) with radius 1 + sum_{k<6} (0.05/2^k) N_k(u), N_k value noise
    at lattice frequency 4*2^k.  k=8: 655,362 vertices / 1,310,720 faces."""
    u, f = icosphere(k)
    return _pack(normalize_unit_cube(u * noise_radius(u, seed)[:, None]), f)


def noisy_geodesic_sphere(n: int, seed: int):
    u, f = geodesic_sphere(n)
    return _pack(normalize_unit_cube(u * noise_radius(u, seed)[:, None]), f)


def bumpy_torus(n: int, m: int, seed: int, R: float = 1.0, r: float = 0.35):
    """Torus with normal displacement 0.01*r*U[-1,1] per vertex."""
    v, f, nrm = torus(n, m, R, r)
    d = np.random.default_rng(seed).uniform(-1.0, 1.0, len(v))
    v = v + (0.01 * r * d)[:, None] * nrm
    return _pack(normalize_unit_cube(v), f)


def crease_sphere(k: int = 9, seed: int = 5):
    """Icosphere(k), r = 1 + 0.03|sin 12 theta||sin 9 phi| + 0.002 N(0,1)."""
    u, f = icosphere(k)
    th = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    ph = np.arctan2(u[:, 1], u[:, 0])
    z = np.random.default_rng(seed).standard_normal(len(u))
    r = 1.0 + 0.03 * np.abs(np.sin(12 * th)) * np.abs(np.sin(9 * ph)) + 0.002 * z
    return _pack(normalize_unit_cube(u * r[:, None]), f)


def batch_specs(count: int = 256, seed: int = 3, fmin: float = 5e3, fmax: float = 2e5):
    """Face counts log-uniform in [fmin, fmax]; even entries are noisy geodesic
    spheres (F = 20 n^2), odd entries bumpy tori (F = 2 n m)."""
    rng = np.random.default_rng(seed)
    fs = np.exp(rng.uniform(math.log(fmin), math.log(fmax), count))
    specs = []
    for i, fi in enumerate(fs):
        if i % 2 == 0:
            n = max(1, int(round(math.sqrt(fi / 20.0))))
            specs.append(("sphere", n, 1000 + i))
        else:
            n = int(min(512, max(64, round(math.sqrt(fi * 1.0 / (2 * 0.35))))))
            m = max(3, int(round(fi / (2 * n))))
            specs.append(("torus", (n, m), 1000 + i))
    return specs


def tori_specs(count: int = 32, seed: int = 5, fmin: float = 2e4, fmax: float = 1e5):
    """Bumpy tori of log-uniform face counts in [fmin, fmax] (the batch recipe's
    tori)."""
    rng = np.random.default_rng(seed)
    fs = np.exp(rng.uniform(math.log(fmin), math.log(fmax), count))
    out = []
    for i, fi in enumerate(fs):
        n = int(min(512, max(64, round(math.sqrt(fi * 1.0 / (2 * 0.35))))))
        m = max(3, int(round(fi / (2 * n))))
        out.append(("torus", (n, m), 2000 + i))
    return out


def make_spec(spec):
    kind, size, seed = spec
    if kind == "sphere":
        return noisy_geodesic_sphere(size, seed)
    n, m = size
    return bumpy_torus(n, m, seed)


def tetrahedron():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    f = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int32)
    return v, f


def octahedron():
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
    f = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                  [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int32)
    return _pack(normalize_unit_cube(v), f)


def csaszar_torus():
    """Seven-vertex torus (every vertex adjacent to every other, 14 faces): the
    link condition fails on every edge, so no collapse is ever legal."""
    # combinatorial 7-vertex torus: faces (i, i+1, i+3) and (i, i+3, i+2) mod 7
    faces = []
    for i in range(7):
        faces.append((i, (i + 1) % 7, (i + 3) % 7))
        faces.append((i, (i + 3) % 7, (i + 2) % 7))
    # a geometric embedding is not needed for a topology-only fixture; place the
    # vertices on a generic torus so the quadrics are finite
    th = 2 * np.pi * np.arange(7) / 7
    ph = 2 * np.pi * (3 * np.arange(7) % 7) / 7
    v = np.stack([(2 + np.cos(ph)) * np.cos(th), (2 + np.cos(ph)) * np.sin(th), np.sin(ph)], 1)
    return _pack(normalize_unit_cube(v), np.asarray(faces))


def bipyramid(n: int = 24, seed: int = 3, jitter: float = 0.05):
    """Two poles of valence n over a jittered ring of n vertices (valence 4):
    a closed mesh whose pole edges have stars beyond a small fixed bound."""
    rng = np.random.default_rng(seed)
    t = 2 * np.pi * (np.arange(n) + jitter * rng.standard_normal(n)) / n
    r = 1.0 + jitter * rng.standard_normal(n)
    ring = np.stack([r * np.cos(t), r * np.sin(t), jitter * rng.standard_normal(n)], 1)
    v = np.concatenate([ring, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]])
    i = np.arange(n)
    top = np.stack([np.full(n, n), i, (i + 1) % n], 1)
    bot = np.stack([np.full(n, n + 1), (i + 1) % n, i], 1)
    return _pack(normalize_unit_cube(v), np.concatenate([top, bot]))


def nested_spheres(k: int = 3, gap: float = 0.01, seed: int = 9, sigma: float = 0.002):
    """Two concentric bumpy icospheres (radii 1 and 1 - gap) as one closed
    two-component mesh.  Collapses on the outer sphere cut chords inward, so
    once triangles grow past the gap they hit the inner sphere: a fixture that
    forces the check/undo loop to work."""
    u, f = icosphere(k)
    rng = np.random.default_rng(seed)
    r1 = 1.0 + sigma * rng.standard_normal(len(u))
    r2 = (1.0 - gap) + sigma * rng.standard_normal(len(u))
    v = np.concatenate([u * r1[:, None], u * r2[:, None]])
    # the inner sphere faces inward (reversed orientation)
    f2 = f[:, [0, 2, 1]] + len(u)
    return _pack(normalize_unit_cube(v), np.concatenate([f, f2]))


def cube():
    """Unit cube, two triangles per side, outward."""
    v = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], dtype=np.float64)
    # vertex index = 4x + 2y + z
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    f = []
    for a, b, c, d in quads:
        f.append((a, b, c))
        f.append((a, c, d))
    f = np.asarray(f)
    p0, p1, p2 = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(p1 - p0, p2 - p0)
    out = (p0 + p1 + p2) / 3 - 0.5
    flip = np.einsum("ij,ij->i", n, out) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return _pack(v, f)
