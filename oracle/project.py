"""TEST INFRASTRUCTURE ONLY: the safe projection stage (Sec. 6) in plain float64
numpy and CPU torch, for checking the library's projection.  Only tests/, the
package's smoke check and bench.py's CPU baseline use it.

What it computes (Sec. 6.1 energies, Sec. 6.2 with Alg. 2, App. 2.2):

* the simplified mesh S0 = (X0, F) moves to X; the augmented energy is
  B(X) = k_dis (E_S2M + E_M2S) + k_elas E_elas + k_bend E_bend
         + k_bar * sum over contact pairs of b(d);
* E_S2M = sum_i s0_i |x_i - y~_i|^2, s0_i the mixed Voronoi area of vertex i on
  S0 (Meyer, Desbrun, Schroeder and Barr 2003), y~_i the point of the input
  mesh closest to x_i when the targets were last refreshed;
* E_M2S = A_in / m * sum_s d^2(y_s, triangle t_s at X), y_s uniform samples on
  the input mesh (area-weighted triangle, uniform barycentric point), t_s the
  triangle of S closest to y_s at the last refresh, d^2 the squared distance to
  the closest point of that triangle (vertex, edge or face, classified at X);
* E_elas = sum_f A0_f / 4 * |C_f - I|_F^2, C = F^T F the right Cauchy-Green
  tensor of the face's 2x2 deformation gradient against its rest shape;
* E_bend = sum_e |e0| / 2 * (theta_e - theta0_e)^2, theta the signed dihedral
  angle of the edge's two faces;
* contact pairs: a vertex and a face not holding it, two edges sharing no
  vertex, at Euclidean distance d < dhat; b(d) = -(d - dhat)^2 ln(d / dhat);
* each iteration of Alg. 2: targets refreshed every `refresh` iterations
  (starting with the first), the Hessian of every element (vertex, sample,
  face, edge stencil, contact pair) projected to positive semi-definite by
  clamping its negative eigenvalues to zero, p from H p = -grad B by conjugate
  gradients with a 3x3 block-Jacobi preconditioner, the step bounded by
  additive CCD (Li et al. 2021) over the pairs whose swept boxes overlap, then
  halved until B decreases (at most ls_max halvings, and no further once the
  step alpha |p| is shorter than LS_MIN_STEP); an iteration that finds no
  decrease leaves X as it is, and so would every later iteration until the
  targets are refreshed (the same X and targets give the same direction), so
  those are skipped.

Derivatives: every element energy is a torch function of the element's own
coordinates; gradients and Hessians come from torch's automatic differentiation
(torch.func), a library primitive.  Closest features are classified from
numpy values before the derivative is taken, so each element is one smooth
closed form at a time.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch
from torch.func import grad, hessian, vmap

torch.set_default_dtype(torch.float64)

TIE = 1e-9  # closest-triangle ties: the smallest index within this relative margin
TIE_ABS = 1e-24
PARALLEL = 1e-20  # two edges are parallel when |ea x eb|^2 <= PARALLEL |ea|^2 |eb|^2
ACCD_MAX_STEPS = 1 << 20
LS_MIN_STEP = 1e-14  # the line search stops once alpha |p| falls below this length


@dataclass
class Options:
    k_dis: float = 1e3
    k_elas: float = 1e-1
    k_bend: float = 1e-2
    k_bar: float = 1e2
    dhat: float = 1e-3
    iterations: int = 50
    refresh: int = 10
    cg_tol: float = 1e-4
    cg_max: int = 1000
    accd_s: float = 0.1
    ls_max: int = 40


# ------------------------------------------------------------------ geometry
def face_areas(V, F):
    return 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1)


def sample_surface(V, F, U):
    """m samples from uniforms U (m, 3) in [0, 1): triangle = the first index
    whose inclusive cumulative area exceeds u0 times the total, point =
    (1 - r) a + r (1 - u2) b + r u2 c with r = sqrt(u1) (uniform on the
    triangle, Osada et al. 2002)."""
    cum = np.cumsum(face_areas(V, F))
    f = np.searchsorted(cum, U[:, 0] * cum[-1], side="right")
    f = np.minimum(f, len(F) - 1)
    r = np.sqrt(U[:, 1])
    w = np.stack([1.0 - r, r * (1.0 - U[:, 2]), r * U[:, 2]], axis=1)
    T = V[F[f]]
    return np.einsum("mk,mkd->md", w, T), f


def voronoi_areas(V, F):
    """Mixed Voronoi area per vertex: in a triangle with no obtuse angle each
    corner gets the part of the triangle nearer to it than to the other
    corners, (|PR|^2 cot Q + |PQ|^2 cot R) / 8; in an obtuse triangle the
    obtuse corner gets half the area and the others a quarter each."""
    s = np.zeros(len(V))
    A = face_areas(V, F)
    for f in range(len(F)):
        idx = F[f]
        P = V[idx]
        ang = []
        for c in range(3):
            u = P[(c + 1) % 3] - P[c]
            w = P[(c + 2) % 3] - P[c]
            ang.append(math.atan2(np.linalg.norm(np.cross(u, w)), float(np.dot(u, w))))
        if max(ang) > math.pi / 2:
            for c in range(3):
                s[idx[c]] += A[f] / 2 if ang[c] > math.pi / 2 else A[f] / 4
            continue
        for c in range(3):
            q, r = (c + 1) % 3, (c + 2) % 3
            lpr = float(np.sum((P[r] - P[c]) ** 2))
            lpq = float(np.sum((P[q] - P[c]) ** 2))
            s[idx[c]] += (lpr / math.tan(ang[q]) + lpq / math.tan(ang[r])) / 8.0
    return s


def edge_stencils(F):
    """Every edge once: (i, j, k, l) with face (i, j, k) holding i -> j and face
    (j, i, l) holding j -> i (a closed, consistently oriented mesh)."""
    opp = {}
    for f in F:
        for c in range(3):
            opp[(int(f[c]), int(f[(c + 1) % 3]))] = int(f[(c + 2) % 3])
    out = []
    for (i, j), k in opp.items():
        if i < j:
            out.append((i, j, k, opp[(j, i)]))
    return np.array(out, dtype=np.int64).reshape(-1, 4)


def edges_of(F):
    st = edge_stencils(F)
    return st[:, :2].copy()


# ------------------------------------------------------- closest features
def _point_seg_d2(p, a, b):
    ab = b - a
    t = np.einsum("...d,...d->...", p - a, ab) / np.maximum(np.einsum("...d,...d->...", ab, ab), 1e-300)
    t = np.clip(t, 0.0, 1.0)
    q = a + t[..., None] * ab
    return np.einsum("...d,...d->...", p - q, p - q), t


def pt_feature(p, a, b, c):
    """Closest feature of triangle abc to p: 0 the face, 1 edge ab, 2 edge bc,
    3 edge ca, 4 vertex a, 5 vertex b, 6 vertex c.  The projection onto the
    plane when it falls inside the triangle, else the nearest of the three
    edges (segments), a vertex when the nearest point is a segment's end.
    Arrays of points and triangles (..., 3)."""
    e0, e1, d = b - a, c - a, p - a
    a00 = np.einsum("...d,...d->...", e0, e0)
    a01 = np.einsum("...d,...d->...", e0, e1)
    a11 = np.einsum("...d,...d->...", e1, e1)
    b0 = np.einsum("...d,...d->...", d, e0)
    b1 = np.einsum("...d,...d->...", d, e1)
    det = a00 * a11 - a01 * a01
    with np.errstate(divide="ignore", invalid="ignore"):
        u = (a11 * b0 - a01 * b1) / det
        v = (a00 * b1 - a01 * b0) / det
    inside = (det > 0) & (u >= 0) & (v >= 0) & (u + v <= 1)
    segs = [(a, b, 1, 4, 5), (b, c, 2, 5, 6), (c, a, 3, 6, 4)]
    best = np.full(np.shape(b0), np.inf)
    code = np.zeros(np.shape(b0), dtype=np.int64)
    for s0, s1, ecode, v0, v1 in segs:
        d2, t = _point_seg_d2(p, s0, s1)
        c_here = np.where(t <= 0.0, v0, np.where(t >= 1.0, v1, ecode))
        take = d2 < best
        best = np.where(take, d2, best)
        code = np.where(take, c_here, code)
    return np.where(inside, 0, code)


def pt_d2(p, a, b, c):
    """squared distance from p to triangle abc (arrays (..., 3))"""
    code = pt_feature(p, a, b, c)
    n = np.cross(b - a, c - a)
    nn = np.einsum("...d,...d->...", n, n)
    with np.errstate(divide="ignore", invalid="ignore"):
        face = np.einsum("...d,...d->...", p - a, n) ** 2 / nn
    out = np.where(code == 0, face, np.inf)
    for ecode, s0, s1 in ((1, a, b), (2, b, c), (3, c, a)):
        d2, _ = _point_seg_d2(p, s0, s1)
        out = np.where((code == ecode) | (code == ecode + 3), d2, out)
    return out


def closest_faces(P, V, F):
    """For each point: the triangle of (V, F) it is closest to (the smallest
    index among those within a relative margin of the smallest squared
    distance), that distance squared, and the closest point on it."""
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    out_f = np.zeros(len(P), dtype=np.int64)
    out_d = np.zeros(len(P))
    for s in range(0, len(P), 64):
        Pc = P[s:s + 64, None, :]
        d2 = pt_d2(Pc, A[None], B[None], C[None])
        dmin = d2.min(axis=1)
        ok = d2 <= dmin[:, None] * (1.0 + TIE) + TIE_ABS
        out_f[s:s + 64] = np.argmax(ok, axis=1)
        out_d[s:s + 64] = d2[np.arange(len(Pc)), out_f[s:s + 64]]
    return out_f, out_d, closest_point_on(P, V[F[out_f]])


def closest_point_on(P, T):
    """closest point of triangle T[i] (3, 3) to P[i]"""
    a, b, c = T[:, 0], T[:, 1], T[:, 2]
    code = pt_feature(P, a, b, c)
    n = np.cross(b - a, c - a)
    nn = np.einsum("id,id->i", n, n)
    with np.errstate(divide="ignore", invalid="ignore"):
        proj = P - (np.einsum("id,id->i", P - a, n) / nn)[:, None] * n
    out = proj.copy()
    for ecode, s0, s1 in ((1, a, b), (2, b, c), (3, c, a)):
        _, t = _point_seg_d2(P, s0, s1)
        q = s0 + t[:, None] * (s1 - s0)
        m = (code == ecode) | (code == ecode + 3)
        out[m] = q[m]
    return out


# ------------------------------------------------------- element energies
def _cross(u, w):
    return torch.stack([u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]])


def _d2_point_point(p, a):
    return ((p - a) ** 2).sum()


def _d2_point_line(p, a, b):
    e = b - a
    c = _cross(p - a, e)
    return (c * c).sum() / (e * e).sum()


def _d2_point_plane(p, a, b, c):
    n = _cross(b - a, c - a)
    return ((p - a) * n).sum() ** 2 / (n * n).sum()


def _d2_line_line(a0, a1, b0, b1):
    n = _cross(a1 - a0, b1 - b0)
    return ((b0 - a0) * n).sum() ** 2 / (n * n).sum()


def _pt_d2_by_code(code, p, a, b, c):
    if code == 0:
        return _d2_point_plane(p, a, b, c)
    if code in (1, 2, 3):
        s0, s1 = ((a, b), (b, c), (c, a))[code - 1]
        return _d2_point_line(p, s0, s1)
    return _d2_point_point(p, (a, b, c)[code - 4])


_OTHER = ((2, 3), (2, 3), (0, 1), (0, 1))


def ee_feature(a0, a1, b0, b1):
    """Closest features of segments a0a1 and b0b1 (arrays (..., 3)), as a code
    over the four points 0..3 = a0, a1, b0, b1: 0 when the closest points are
    inside both segments and the segments are not parallel (line against
    line); 1 + p for point p against the line of the other segment; 5 + 2 p + r
    for point p against end r of the other segment.  The interior case is the
    unconstrained minimum of the squared distance over both segment
    parameters when it lies inside (0, 1)^2; otherwise the minimum lies on the
    square's boundary: the nearest of the four point-segment distances."""
    ea, eb, w = a1 - a0, b1 - b0, a0 - b0
    n = np.cross(ea, eb)
    A = np.einsum("...d,...d->...", ea, ea)
    Bv = np.einsum("...d,...d->...", ea, eb)
    Cv = np.einsum("...d,...d->...", eb, eb)
    D = np.einsum("...d,...d->...", ea, w)
    E = np.einsum("...d,...d->...", eb, w)
    nonpar = np.einsum("...d,...d->...", n, n) > PARALLEL * A * Cv
    den = A * Cv - Bv * Bv
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (Bv * E - Cv * D) / den
        t = (A * E - Bv * D) / den
    interior = nonpar & (s > 0) & (s < 1) & (t > 0) & (t < 1)
    pts = (a0, a1, b0, b1)
    best = np.full(np.shape(A), np.inf)
    code = np.zeros(np.shape(A), dtype=np.int64)
    for p in range(4):
        u, v = _OTHER[p]
        d2, tt = _point_seg_d2(pts[p], pts[u], pts[v])
        c_here = np.where(tt <= 0.0, 5 + 2 * p, np.where(tt >= 1.0, 6 + 2 * p, 1 + p))
        take = d2 < best
        best = np.where(take, d2, best)
        code = np.where(take, c_here, code)
    return np.where(interior, 0, code)


def _ee_d2_by_code(code, a0, a1, b0, b1):
    pts = (a0, a1, b0, b1)
    if code == 0:
        return _d2_line_line(a0, a1, b0, b1)
    if code <= 4:
        p = code - 1
        u, v = _OTHER[p]
        return _d2_point_line(pts[p], pts[u], pts[v])
    p, r = divmod(code - 5, 2)
    return _d2_point_point(pts[p], pts[_OTHER[p][r]])


def ee_d2(a0, a1, b0, b1):
    """squared distance of segment pairs (arrays (..., 3))"""
    code = ee_feature(a0, a1, b0, b1)
    n = np.cross(a1 - a0, b1 - b0)
    with np.errstate(divide="ignore", invalid="ignore"):
        ll = np.einsum("...d,...d->...", b0 - a0, n) ** 2 / np.einsum("...d,...d->...", n, n)
    out = np.where(code == 0, ll, np.inf)
    pts = (a0, a1, b0, b1)
    for p in range(4):
        u, v = _OTHER[p]
        d2, _ = _point_seg_d2(pts[p], pts[u], pts[v])
        out = np.where((code == 1 + p) | (code == 5 + 2 * p) | (code == 6 + 2 * p), d2, out)
    return out


def barrier(d, dhat):
    """b(d) = -(d - dhat)^2 ln(d / dhat) below dhat, 0 at and beyond it (works
    on floats and torch scalars)"""
    if isinstance(d, torch.Tensor):
        return torch.where(d < dhat, -(d - dhat) ** 2 * torch.log(d / dhat), torch.zeros_like(d))
    if d <= 0.0:
        return math.inf
    return -(d - dhat) ** 2 * math.log(d / dhat) if d < dhat else 0.0


def _elastic(z, Binv, A0):
    x = z.reshape(3, 3)
    D = torch.stack([x[1] - x[0], x[2] - x[0]], dim=1)  # 3x2
    G = D.T @ D
    Cg = Binv.T @ G @ Binv
    Iden = torch.eye(2, dtype=z.dtype)
    return 0.25 * A0 * ((Cg - Iden) ** 2).sum()


def dihedral(xi, xj, xk, xl):
    """signed angle between the normals of faces (i, j, k) and (j, i, l) about
    the edge i -> j (torch, one stencil)"""
    e = xj - xi
    n1 = _cross(e, xk - xi)
    n2 = _cross(xi - xj, xl - xj)
    en = e / torch.sqrt((e * e).sum())
    return torch.atan2((_cross(n1, n2) * en).sum(), (n1 * n2).sum())


def _bend(z, theta0, l0):
    x = z.reshape(4, 3)
    th = dihedral(x[0], x[1], x[2], x[3])
    return 0.5 * l0 * (th - theta0) ** 2


# ---------------------------------------------------- per-element derivatives
def _derivs(fn, Z, *params):
    """values, gradients and Hessians of fn over a batch of elements"""
    Z = torch.as_tensor(Z, dtype=torch.float64)
    if Z.shape[0] == 0:
        k = Z.shape[1]
        return np.zeros(0), np.zeros((0, k)), np.zeros((0, k, k))
    params = [torch.as_tensor(p, dtype=torch.float64) for p in params]
    val = vmap(fn)(Z, *params)
    g = vmap(grad(fn))(Z, *params)
    H = vmap(hessian(fn))(Z, *params)
    return val.numpy(), g.numpy(), H.numpy()


def _grouped(keys, fn_of_key, Z, *params):
    """elements grouped by their classified feature: fn_of_key(key) is the
    element's closed form"""
    n, k = Z.shape
    val, g, H = np.zeros(n), np.zeros((n, k)), np.zeros((n, k, k))
    for key in sorted(set(keys)):
        idx = np.array([i for i, kk in enumerate(keys) if kk == key], dtype=np.int64)
        v, gg, hh = _derivs(fn_of_key(key), Z[idx], *[p[idx] for p in params])
        val[idx], g[idx], H[idx] = v, gg, hh
    return val, g, H


def _m2s_fn(code):
    def fn(z, y):
        x = z.reshape(3, 3)
        return _pt_d2_by_code(code, y, x[0], x[1], x[2])
    return fn


def _pt_barrier_fn(code, dhat):
    def fn(z):
        x = z.reshape(4, 3)
        return barrier(torch.sqrt(_pt_d2_by_code(code, x[0], x[1], x[2], x[3])), dhat)
    return fn


def _ee_barrier_fn(code, dhat):
    def fn(z):
        x = z.reshape(4, 3)
        return barrier(torch.sqrt(_ee_d2_by_code(code, x[0], x[1], x[2], x[3])), dhat)
    return fn


# ---------------------------------------------------------------- problem
@dataclass
class Problem:
    X0: np.ndarray
    F: np.ndarray
    Y: np.ndarray                 # samples on the input mesh
    area_in: float
    opt: Options
    s0: np.ndarray = None
    Binv: np.ndarray = None       # per face, inverse of the rest edge matrix in a frame of its plane
    A0: np.ndarray = None
    stencils: np.ndarray = None
    theta0: np.ndarray = None
    l0: np.ndarray = None
    edges: np.ndarray = None
    targets: np.ndarray = None    # closest input-mesh point per vertex
    tri: np.ndarray = None        # closest S triangle per sample
    log: list = field(default_factory=list)


def rest_faces(X0, F):
    """Per face: area and the inverse of its rest edge matrix [e1, e2] written
    in an orthonormal frame of the face's plane (u along e1)."""
    P0, P1, P2 = X0[F[:, 0]], X0[F[:, 1]], X0[F[:, 2]]
    e1, e2 = P1 - P0, P2 - P0
    l1 = np.linalg.norm(e1, axis=1)
    u = e1 / l1[:, None]
    n = np.cross(e1, e2)
    A0 = 0.5 * np.linalg.norm(n, axis=1)
    w = np.cross(n / np.linalg.norm(n, axis=1)[:, None], u)
    Dm = np.zeros((len(F), 2, 2))
    Dm[:, 0, 0] = l1
    Dm[:, 0, 1] = np.einsum("id,id->i", u, e2)
    Dm[:, 1, 1] = np.einsum("id,id->i", w, e2)
    return np.linalg.inv(Dm), A0


def rest_edges(X0, F):
    """Per edge stencil: the stencils, rest dihedral angles and rest lengths."""
    st = edge_stencils(F)
    X = torch.from_numpy(X0)
    th0 = np.array([float(dihedral(X[i], X[j], X[k], X[l])) for i, j, k, l in st])
    l0 = np.linalg.norm(X0[st[:, 1]] - X0[st[:, 0]], axis=1)
    return st, th0, l0


def rest_data(X0, F):
    return (*rest_faces(X0, F), *rest_edges(X0, F))


def make_problem(X0, F, Vin, Fin, U, opt=None):
    opt = opt or Options()
    X0 = np.ascontiguousarray(X0, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int64)
    Y, _ = sample_surface(np.asarray(Vin, np.float64), np.asarray(Fin, np.int64), np.asarray(U, np.float64))
    pb = Problem(X0=X0, F=F, Y=Y, area_in=float(face_areas(Vin, Fin).sum()), opt=opt)
    pb.s0 = voronoi_areas(X0, F)
    pb.Binv, pb.A0, pb.stencils, pb.theta0, pb.l0 = rest_data(X0, F)
    pb.edges = pb.stencils[:, :2].copy()
    return pb


def refresh_targets(pb, X, Vin, Fin):
    _, _, pb.targets = closest_faces(X, np.asarray(Vin, np.float64), np.asarray(Fin, np.int64))
    pb.tri, _, _ = closest_faces(pb.Y, X, pb.F)


# ---------------------------------------------------------------- contacts
def _boxes(X, idx, P=None, pad=0.0):
    """axis-aligned boxes of primitives (rows of vertex ids), over the start
    positions X and, with P, the end positions X + P"""
    pts = X[idx]
    lo, hi = pts.min(axis=1), pts.max(axis=1)
    if P is not None:
        q = (X + P)[idx]
        lo, hi = np.minimum(lo, q.min(axis=1)), np.maximum(hi, q.max(axis=1))
    return lo - pad, hi + pad


def _overlap_pairs(lo1, hi1, lo2, hi2, same=False):
    out = []
    for s in range(0, len(lo1), 256):
        ok = np.all((lo1[s:s + 256, None, :] <= hi2[None]) & (lo2[None] <= hi1[s:s + 256, None, :]), axis=2)
        i, j = np.nonzero(ok)
        out.append(np.stack([i + s, j], axis=1))
    pr = np.concatenate(out) if out else np.zeros((0, 2), np.int64)
    if same:
        pr = pr[pr[:, 0] < pr[:, 1]]
    return pr


def candidate_pairs(X, F, edges, P=None, pad=0.0):
    """vertex-face pairs (v not in f) and edge-edge pairs (no shared vertex)
    whose boxes overlap: start boxes grown by pad, or swept boxes over the
    step P"""
    nv = len(X)
    vid = np.arange(nv)[:, None]
    vlo, vhi = _boxes(X, vid, P, pad)
    flo, fhi = _boxes(X, F, P, pad)
    pt = _overlap_pairs(vlo, vhi, flo, fhi)
    pt = pt[~np.any(F[pt[:, 1]] == pt[:, 0:1], axis=1)]
    elo, ehi = _boxes(X, edges, P, pad)
    ee = _overlap_pairs(elo, ehi, elo, ehi, same=True)
    a, b = edges[ee[:, 0]], edges[ee[:, 1]]
    shared = (a[:, 0] == b[:, 0]) | (a[:, 0] == b[:, 1]) | (a[:, 1] == b[:, 0]) | (a[:, 1] == b[:, 1])
    return pt, ee[~shared]


def contacts(X, F, edges, dhat):
    """contact pairs at X: (vertex, face) and (edge, edge) pairs at distance
    below dhat, with their squared distances"""
    pt, ee = candidate_pairs(X, F, edges, pad=dhat)
    T = X[F[pt[:, 1]]]
    d2 = pt_d2(X[pt[:, 0]], T[:, 0], T[:, 1], T[:, 2]) if len(pt) else np.zeros(0)
    keep = d2 < dhat * dhat
    pt, dpt = pt[keep], d2[keep]
    a, b = edges[ee[:, 0]], edges[ee[:, 1]]
    dee = ee_d2(X[a[:, 0]], X[a[:, 1]], X[b[:, 0]], X[b[:, 1]]) if len(ee) else np.zeros(0)
    keep = dee < dhat * dhat
    return pt, dpt, ee[keep], dee[keep]


# ---------------------------------------------------------------- energy
def energy_parts(pb, X):
    """the five terms of B at X (unweighted), with the current targets"""
    o = pb.opt
    s2m = float(np.sum(pb.s0 * np.sum((X - pb.targets) ** 2, axis=1)))
    T = X[pb.F[pb.tri]]
    m2s = float(pb.area_in / len(pb.Y) * np.sum(pt_d2(pb.Y, T[:, 0], T[:, 1], T[:, 2])))
    Z = torch.from_numpy(X[pb.F].reshape(-1, 9))
    el = float(vmap(_elastic)(Z, torch.from_numpy(pb.Binv), torch.from_numpy(pb.A0)).sum())
    Zb = torch.from_numpy(X[pb.stencils].reshape(-1, 12))
    be = float(vmap(_bend)(Zb, torch.from_numpy(pb.theta0), torch.from_numpy(pb.l0)).sum())
    pt, dpt, ee, dee = contacts(X, pb.F, pb.edges, o.dhat)
    bar = float(sum(barrier(math.sqrt(d), o.dhat) for d in dpt) + sum(barrier(math.sqrt(d), o.dhat) for d in dee))
    return {"s2m": s2m, "m2s": m2s, "elastic": el, "bend": be, "barrier": bar,
            "n_pt": int(len(pt)), "n_ee": int(len(ee))}


def total(pb, parts):
    o = pb.opt
    return (o.k_dis * (parts["s2m"] + parts["m2s"]) + o.k_elas * parts["elastic"] + o.k_bend * parts["bend"]
            + o.k_bar * parts["barrier"])


def energy(pb, X):
    if not np.all(np.isfinite(X)):
        return math.inf
    return total(pb, energy_parts(pb, X))


def elements(pb, X):
    """every element of B at X: (vertex ids, weighted gradient, weighted
    Hessian) per element, Hessians not yet projected"""
    o = pb.opt
    out = []
    n = len(X)
    # E_S2M: one element per vertex
    g = 2.0 * o.k_dis * pb.s0[:, None] * (X - pb.targets)
    H = 2.0 * o.k_dis * pb.s0[:, None, None] * np.eye(3)[None]
    out.append((np.arange(n)[:, None], g, H))
    # E_M2S: one element per sample, the triangle's nine coordinates
    T = X[pb.F[pb.tri]]
    codes = [int(c) for c in pt_feature(pb.Y, T[:, 0], T[:, 1], T[:, 2])]
    _, g, H = _grouped(codes, _m2s_fn, T.reshape(-1, 9), pb.Y)
    w = o.k_dis * pb.area_in / len(pb.Y)
    out.append((pb.F[pb.tri], w * g, w * H))
    # elastic: one element per face
    _, g, H = _derivs(_elastic, X[pb.F].reshape(-1, 9), pb.Binv, pb.A0)
    out.append((pb.F, o.k_elas * g, o.k_elas * H))
    # bending: one element per edge stencil
    _, g, H = _derivs(_bend, X[pb.stencils].reshape(-1, 12), pb.theta0, pb.l0)
    out.append((pb.stencils, o.k_bend * g, o.k_bend * H))
    # barrier: one element per contact pair
    pt, _, ee, _ = contacts(X, pb.F, pb.edges, o.dhat)
    if len(pt):
        ids = np.concatenate([pt[:, :1], pb.F[pt[:, 1]]], axis=1)
        P = X[ids]
        codes = [int(c) for c in pt_feature(P[:, 0], P[:, 1], P[:, 2], P[:, 3])]
        _, g, H = _grouped(codes, lambda c: _pt_barrier_fn(c, o.dhat), P.reshape(-1, 12))
        out.append((ids, o.k_bar * g, o.k_bar * H))
    if len(ee):
        ids = np.concatenate([pb.edges[ee[:, 0]], pb.edges[ee[:, 1]]], axis=1)
        P = X[ids]
        codes = [int(c) for c in ee_feature(P[:, 0], P[:, 1], P[:, 2], P[:, 3])]
        _, g, H = _grouped(codes, lambda c: _ee_barrier_fn(c, o.dhat), P.reshape(-1, 12))
        out.append((ids, o.k_bar * g, o.k_bar * H))
    return out


def project_psd(H):
    """clamp the negative eigenvalues of each symmetric block to zero"""
    if len(H) == 0:
        return H
    w, Q = np.linalg.eigh(0.5 * (H + np.swapaxes(H, 1, 2)))
    return np.einsum("eij,ej,ekj->eik", Q, np.maximum(w, 0.0), Q)


def assemble(n, elems, project=True):
    """global gradient (3n) and sparse Hessian (3n x 3n) from element terms"""
    import scipy.sparse as sp
    g = np.zeros(3 * n)
    rows, cols, vals = [], [], []
    for ids, ge, He in elems:
        k = ids.shape[1]
        dof = (3 * ids[:, :, None] + np.arange(3)[None, None, :]).reshape(len(ids), 3 * k)
        np.add.at(g, dof, ge)
        Hp = project_psd(He) if project else He
        rows.append(np.repeat(dof, 3 * k, axis=1).ravel())
        cols.append(np.tile(dof, (1, 3 * k)).ravel())
        vals.append(Hp.reshape(len(ids), -1).ravel())
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(3 * n, 3 * n))
    return g, H.tocsr()


def pcg(H, b, tol, max_iter):
    """conjugate gradients on H x = b from x = 0 with the inverse 3x3 diagonal
    blocks of H as preconditioner; stops when |r| <= tol |b|"""
    n = len(b) // 3
    blocks = np.zeros((n, 3, 3))
    Hc = H.tocoo()
    on = (Hc.row // 3) == (Hc.col // 3)
    np.add.at(blocks, (Hc.row[on] // 3, Hc.row[on] % 3, Hc.col[on] % 3), Hc.data[on])
    Minv = np.linalg.inv(blocks)

    def prec(r):
        return np.einsum("vij,vj->vi", Minv, r.reshape(n, 3)).ravel()

    x = np.zeros_like(b)
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    bn = float(np.linalg.norm(b))
    it = 0
    while it < max_iter and float(np.linalg.norm(r)) > tol * bn:
        Ap = H @ p
        alpha = rz / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = prec(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it


# ---------------------------------------------------------------- ACCD
def accd_pairs(x, p, kind, s, t_max):
    """Additive CCD (Li, Kaufman and Jiang 2021) of a batch of pairs: x, p
    (k, 4, 3) the pairs' points and their displacements; kind 'pt' (point 0
    against triangle 1-3) or 'ee' (edge 0-1 against edge 2-3).  For each pair
    the step in [0, t_max] up to which it keeps at least the fraction s of its
    starting distance: with the common translation removed and l_p bounding
    how fast the distance can shrink, advance by 0.9 d / l_p (the first step
    (1 - s) d / l_p) until the distance falls below s times the start, or
    t_max is passed."""
    d2f = (lambda y: pt_d2(y[:, 0], y[:, 1], y[:, 2], y[:, 3])) if kind == "pt" else \
          (lambda y: ee_d2(y[:, 0], y[:, 1], y[:, 2], y[:, 3]))
    k = len(x)
    out = np.full(k, t_max)
    if k == 0:
        return out
    p = p - p.mean(axis=1, keepdims=True)
    n = np.linalg.norm(p, axis=2)
    lp = n[:, 0] + n[:, 1:].max(axis=1) if kind == "pt" else \
        np.maximum(n[:, 0], n[:, 1]) + np.maximum(n[:, 2], n[:, 3])
    x = x.copy()
    d = np.sqrt(d2f(x))
    out[(lp > 0) & (d == 0.0)] = 0.0
    live = (lp > 0) & (d > 0.0)
    g = s * d
    t = np.zeros(k)
    with np.errstate(divide="ignore", invalid="ignore"):
        tl = (1.0 - s) * d / lp
    for _ in range(ACCD_MAX_STEPS):
        idx = np.nonzero(live)[0]
        if len(idx) == 0:
            break
        x[idx] += tl[idx, None, None] * p[idx]
        dn = np.sqrt(d2f(x[idx]))
        hit = (t[idx] > 0.0) & (dn < g[idx])
        out[idx[hit]] = t[idx[hit]]
        live[idx[hit]] = False
        rest = idx[~hit]
        t[rest] += tl[rest]
        over = t[rest] > t_max
        live[rest[over]] = False
        tl[rest] = 0.9 * dn[~hit] / lp[rest]
    else:
        out[live] = t[live]
    return out


def accd(pb, X, P, t_max=1.0):
    """the largest step in [0, t_max] that additive CCD allows over every pair
    whose swept boxes overlap"""
    pt, ee = candidate_pairs(X, pb.F, pb.edges, P=P)
    step = t_max
    if len(pt):
        ids = np.concatenate([pt[:, :1], pb.F[pt[:, 1]]], axis=1)
        step = min(step, float(accd_pairs(X[ids], P[ids], "pt", pb.opt.accd_s, t_max).min()))
    if len(ee):
        ids = np.concatenate([pb.edges[ee[:, 0]], pb.edges[ee[:, 1]]], axis=1)
        step = min(step, float(accd_pairs(X[ids], P[ids], "ee", pb.opt.accd_s, t_max).min()))
    return step


# ---------------------------------------------------------------- Alg. 2
def newton_direction(pb, X):
    els = elements(pb, X)
    g, H = assemble(len(X), els)
    p, it = pcg(H, -g, pb.opt.cg_tol, pb.opt.cg_max)
    return g, H, p.reshape(-1, 3), it


def safe_project(X0, F, Vin, Fin, U, opt=None, iterations=None):
    """Alg. 2 from S0 = (X0, F) towards the input mesh (Vin, Fin) with sample
    uniforms U; returns the final positions and the problem (its log holds one
    record per iteration)."""
    pb = make_problem(X0, F, Vin, Fin, U, opt)
    o = pb.opt
    T = o.iterations if iterations is None else iterations
    X = pb.X0.copy()
    stalled, B0 = False, math.nan
    for t in range(T):
        if t % o.refresh == 0:
            refresh_targets(pb, X, Vin, Fin)
            stalled = False
        if stalled:
            pb.log.append({"B": B0, "alpha_ccd": 0.0, "alpha": 0.0, "halvings": 0, "cg_iters": 0,
                           "grad_norm": 0.0, "skipped": True})
            continue
        B0 = energy(pb, X)
        g, H, P, cg_it = newton_direction(pb, X)
        a_ccd = accd(pb, X, P)
        alpha = min(1.0, a_ccd)
        pnorm = float(np.linalg.norm(P))
        moved, halvings = False, 0
        for halvings in range(o.ls_max):
            if alpha * pnorm < LS_MIN_STEP:
                break
            Xn = X + alpha * P
            Bn = energy(pb, Xn)
            if Bn < B0:
                X, moved = Xn, True
                break
            alpha *= 0.5
        stalled = not moved
        pb.log.append({"B": B0, "alpha_ccd": a_ccd, "alpha": alpha if moved else 0.0, "halvings": halvings,
                       "cg_iters": cg_it, "grad_norm": float(np.linalg.norm(g))})
        if moved:
            B0 = Bn
    return X, pb
