"""Pins of the safe-projection oracle (Sec. 6) against facts fixed outside it
(no GPU): brute force, closed forms, finite differences and invariants.

* mixed Voronoi areas: a non-obtuse triangle's regions as polygons through
  the circumcentre; the obtuse rule; areas sum to the surface area;
* samples: on their triangles, triangle counts in proportion to area, the mean
  of a uniform triangle at its centroid;
* distances: point-triangle and segment-segment squared distances against a
  dense parameter grid, special configurations with known distance;
* energies: elastic zero under rigid motion, closed forms under scaling and
  shear; bending zero at rest, 1/2 |e| (phi - phi0)^2 for a hinge folded by
  phi; the dihedral angle against the arc cosine of the normals; the barrier's
  special values and smoothness at dhat;
* derivatives: the assembled gradient against central differences of B, the
  element Hessians against differences of the gradients;
* solver pieces: the PSD projection, the preconditioned CG against a direct
  solve, additive CCD against the exact impact time of a point falling on a
  triangle and of two crossing edges;
* one short run: B never increases within a window of fixed targets, the
  output is free of self-intersections and its distance energy is lower.
"""
import math

import numpy as np
import pytest
import torch

import oracle.oracle as orc
import oracle.project as op
from paper_2509_05595_amd import meshgen as g


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q * np.sign(np.linalg.det(q))


# ---------------------------------------------------------------- areas, samples
def _poly_area(P):
    s = np.zeros(3)
    for i in range(len(P)):
        s += np.cross(P[i], P[(i + 1) % len(P)])
    return 0.5 * np.linalg.norm(s)


def _circumcentre(a, b, c):
    ab, ac = b - a, c - a
    n = np.cross(ab, ac)
    return a + (np.dot(ac, ac) * np.cross(n, ab) + np.dot(ab, ab) * np.cross(ac, n)) / (2 * np.dot(n, n))


def test_voronoi_areas_by_polygons():
    rng = np.random.default_rng(1)
    done = 0
    while done < 40:
        P = rng.standard_normal((3, 3))
        ang = [math.acos(np.clip(np.dot(P[(c + 1) % 3] - P[c], P[(c + 2) % 3] - P[c]) /
                                 np.linalg.norm(P[(c + 1) % 3] - P[c]) / np.linalg.norm(P[(c + 2) % 3] - P[c]), -1, 1))
               for c in range(3)]
        if max(ang) >= math.pi / 2:
            continue
        o = _circumcentre(*P)
        want = [_poly_area([P[c], (P[c] + P[(c + 1) % 3]) / 2, o, (P[c] + P[(c + 2) % 3]) / 2]) for c in range(3)]
        got = op.voronoi_areas(P, np.array([[0, 1, 2]]))
        assert np.allclose(got, want, rtol=1e-12, atol=0)
        done += 1


def test_voronoi_obtuse_and_total():
    P = np.array([[0.0, 0, 0], [1, 0, 0], [0.1, 0.2, 0]])  # obtuse at vertex 2
    A = 0.5 * 0.2
    assert np.allclose(op.voronoi_areas(P, np.array([[0, 1, 2]])), [A / 4, A / 4, A / 2], rtol=1e-14)
    V, F = g.bumpy_icosphere_gauss(k=3, seed=4)
    assert op.voronoi_areas(V, F).sum() == pytest.approx(op.face_areas(V, F).sum(), rel=1e-12)


def test_samples_on_triangles_and_by_area():
    V = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [3, 0, 1], [3, 3, 1], [0, 3, 1]])
    F = np.array([[0, 1, 2], [3, 4, 5]])  # areas 1/2 and 9/2
    m = 4000
    U = np.stack([(np.arange(m) + 0.5) / m, np.random.default_rng(0).random(m), np.random.default_rng(1).random(m)], 1)
    Y, f = op.sample_surface(V, F, U)
    assert abs(int(np.sum(f == 0)) - m // 10) <= 1
    for k in (0, 1):
        T = V[F[k]]
        n = np.cross(T[1] - T[0], T[2] - T[0])
        y = Y[f == k]
        assert np.abs((y - T[0]) @ n).max() < 1e-12
        # barycentric coordinates all >= 0
        M = np.stack([T[1] - T[0], T[2] - T[0]], 1)
        uv = np.linalg.lstsq(M, (y - T[0]).T, rcond=None)[0]
        assert uv.min() > -1e-12 and (uv.sum(0)).max() < 1 + 1e-12


def test_samples_uniform_mean():
    V = np.array([[0.0, 0, 0], [2, 0, 0], [0, 1, 0]])
    U = np.random.default_rng(5).random((200000, 3))
    Y, _ = op.sample_surface(V, np.array([[0, 1, 2]]), U)
    # per coordinate, the standard deviation over a uniform triangle is below 0.5
    assert np.abs(Y.mean(0) - V.mean(0)).max() < 4 * 0.5 / math.sqrt(len(Y))


# ---------------------------------------------------------------- distances
def _tri_grid(T, n=400):
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    keep = i + j <= n
    u, v = i[keep] / n, j[keep] / n
    return T[0] + u[:, None] * (T[1] - T[0]) + v[:, None] * (T[2] - T[0])


def test_point_triangle_against_grid():
    rng = np.random.default_rng(2)
    for _ in range(30):
        T = rng.standard_normal((3, 3))
        p = rng.standard_normal(3) * 1.5
        d2 = float(op.pt_d2(p, T[0], T[1], T[2]))
        G = _tri_grid(T)
        brute = np.min(np.sum((G - p) ** 2, axis=1))
        h = max(np.linalg.norm(T[1] - T[0]), np.linalg.norm(T[2] - T[0])) / 400
        assert d2 <= brute + 1e-12
        assert math.sqrt(brute) - math.sqrt(d2) <= 2 * h
        q = op.closest_point_on(p[None], T[None])[0]
        assert np.sum((q - p) ** 2) == pytest.approx(d2, rel=1e-10, abs=1e-14)


def test_segments_against_grid_and_skew():
    rng = np.random.default_rng(3)
    n = 600
    s = np.linspace(0, 1, n + 1)
    for _ in range(30):
        a0, a1, b0, b1 = rng.standard_normal((4, 3))
        d2 = float(op.ee_d2(a0, a1, b0, b1))
        A = a0 + s[:, None] * (a1 - a0)
        B = b0 + s[:, None] * (b1 - b0)
        brute = np.min(np.sum((A[:, None] - B[None]) ** 2, axis=2))
        h = (np.linalg.norm(a1 - a0) + np.linalg.norm(b1 - b0)) / n
        assert d2 <= brute + 1e-12 and math.sqrt(brute) - math.sqrt(d2) <= h
    # skew perpendicular segments crossing above each other at height h
    R = _rot(7)
    h = 0.37
    pts = [np.array(x) @ R.T for x in ([-1, 0, 0], [1, 0, 0], [0.2, -1, h], [0.2, 1, h])]
    assert int(op.ee_feature(*pts)) == 0
    assert float(op.ee_d2(*pts)) == pytest.approx(h * h, rel=1e-13)
    # parallel segments, offset and overlapping: distance of the lines
    pts = [np.array(x) for x in ([0, 0, 0], [1, 0, 0], [0.5, 0.3, 0], [2, 0.3, 0])]
    assert float(op.ee_d2(*pts)) == pytest.approx(0.09, rel=1e-13)


# ---------------------------------------------------------------- energies
def _elastic_sum(X, X0, F):
    Binv, A0 = op.rest_faces(X0, F)
    Z = torch.from_numpy(X[F].reshape(-1, 9))
    return float(torch.vmap(op._elastic)(Z, torch.from_numpy(Binv), torch.from_numpy(A0)).sum())


def test_elastic_rigid_scaling_shear():
    V, F = g.bumpy_icosphere_gauss(k=2, seed=3)
    R = _rot(11)
    assert abs(_elastic_sum(V @ R.T + 0.3, V, F)) < 1e-24
    s = 1.07
    A = op.face_areas(V, F).sum()
    assert _elastic_sum(1.07 * V, V, F) == pytest.approx(A / 2 * (s * s - 1) ** 2, rel=1e-12)
    # a shear of one face in its own plane: x' = x + gamma y in a frame of the plane
    T = np.array([[0.0, 0, 0], [0.8, 0.1, 0], [0.3, 0.9, 0]])
    gam = 0.2
    Ts = T.copy()
    Ts[:, 0] += gam * T[:, 1]
    R = _rot(12)
    A0 = 0.5 * np.linalg.norm(np.cross(T[1] - T[0], T[2] - T[0]))
    want = A0 / 4 * (2 * gam ** 2 + gam ** 4)
    assert _elastic_sum(Ts @ R.T, T @ R.T, np.array([[0, 1, 2]])) == pytest.approx(want, rel=1e-12)


def _hinge(phi, l=0.7):
    """faces (0, 1, 2) and (1, 0, 3) about the edge 0 -> 1 on the z axis; the
    second wing rotated by phi out of the plane"""
    X = np.array([[0, 0, 0], [0, 0, l], [0.5, 0.0, 0.3], [-0.4 * math.cos(phi), -0.4 * math.sin(phi), 0.45]])
    return X, np.array([[0, 1, 2], [1, 0, 3]])


@pytest.mark.parametrize("phi0,phi1", [(0.0, 0.3), (0.0, -0.5), (0.4, 1.1), (-0.2, 0.25)])
def test_bending_hinge(phi0, phi1):
    X0, F = _hinge(phi0)
    X1, _ = _hinge(phi1)
    st = np.array([[0, 1, 2, 3]])
    T0 = torch.from_numpy(X0)
    th0 = float(op.dihedral(T0[0], T0[1], T0[2], T0[3]))
    assert abs(abs(th0) - abs(phi0)) < 1e-13
    T1 = torch.from_numpy(X1)
    z = torch.from_numpy(X1[st].reshape(-1))
    E = float(op._bend(z, th0, 0.7))
    assert E == pytest.approx(0.5 * 0.7 * (phi1 - phi0) ** 2, rel=1e-12, abs=1e-30)
    assert abs(float(op.dihedral(T1[0], T1[1], T1[2], T1[3])) - th0) == pytest.approx(abs(phi1 - phi0), abs=1e-13)


def test_dihedral_against_arccos():
    V, F = g.bumpy_icosphere_gauss(k=2, seed=8)
    st = op.edge_stencils(F)
    assert len(st) == len(F) * 3 // 2
    X = torch.from_numpy(V)
    for i, j, k, l in st[:200]:
        n1 = np.cross(V[j] - V[i], V[k] - V[i])
        n2 = np.cross(V[i] - V[j], V[l] - V[j])
        want = math.acos(np.clip(n1 @ n2 / np.linalg.norm(n1) / np.linalg.norm(n2), -1, 1))
        assert abs(abs(float(op.dihedral(X[i], X[j], X[k], X[l]))) - want) < 1e-9


def test_barrier_values():
    dh = 1e-3
    assert op.barrier(dh, dh) == 0.0 and op.barrier(2 * dh, dh) == 0.0
    assert op.barrier(dh / math.e, dh) == pytest.approx((dh - dh / math.e) ** 2, rel=1e-14)
    d = np.linspace(1e-6, dh, 50)[:-1]
    b = np.array([op.barrier(x, dh) for x in d])
    assert np.all(np.diff(b) < 0) and op.barrier(1e-12, dh) > op.barrier(1e-6, dh)
    # first and second derivatives vanish at dhat: b(dhat - e) ~ e^3 / dhat
    for e in (1e-5, 1e-6, 1e-7):
        assert op.barrier(dh - e, dh) == pytest.approx(e ** 3 / dh, rel=2 * e / dh)


# ---------------------------------------------------------------- derivatives
def _contact_problem():
    """two coarse shells 0.0008 apart (below dhat) and an input mesh between
    them: every energy term, contacts included, is active"""
    Vin, Fin = g.icosphere(2)
    Vin = g.normalize_unit_cube(Vin)
    Vs, Fs = g.nested_spheres(k=1, gap=0.0016, sigma=0.0)
    U = np.random.default_rng(4).random((256, 3))
    pb = op.make_problem(Vs, Fs, Vin, Fin, U)
    X = Vs + 1e-4 * np.random.default_rng(5).standard_normal(Vs.shape)
    op.refresh_targets(pb, X, Vin, Fin)
    return pb, X


def test_gradient_against_differences():
    pb, X = _contact_problem()
    parts = op.energy_parts(pb, X)
    assert parts["n_pt"] > 0 and parts["n_ee"] > 0 and parts["barrier"] > 0
    g_, _ = op.assemble(len(X), op.elements(pb, X))
    rng = np.random.default_rng(6)
    for _ in range(6):
        d = rng.standard_normal(X.shape)
        d /= np.linalg.norm(d)
        h = 1e-7
        fd = (op.energy(pb, X + h * d) - op.energy(pb, X - h * d)) / (2 * h)
        assert float(g_ @ d.ravel()) == pytest.approx(fd, rel=2e-5, abs=1e-9)


def test_hessians_against_differences():
    pb, X = _contact_problem()
    els = op.elements(pb, X)
    rng = np.random.default_rng(7)
    h = 1e-6
    for ids, ge, He in els[1:]:  # the vertex term's Hessian is 2 s0 I in closed form
        for e in rng.choice(len(ids), size=min(4, len(ids)), replace=False):
            # rebuild this element's gradient at shifted coordinates through the
            # whole element list (the same element is found by its vertex ids)
            k = ids.shape[1]
            for c in rng.choice(3 * k, size=3, replace=False):
                D = np.zeros_like(X)
                D[ids[e, c // 3], c % 3] = h

                def grad_at(Y):
                    for ids2, g2, _ in op.elements(pb, Y):
                        if ids2.shape == ids.shape and np.array_equal(ids2, ids):
                            return g2[e]
                    raise AssertionError("element set changed")
                col = (grad_at(X + D) - grad_at(X - D)) / (2 * h)
                scale = np.abs(He[e]).max() + 1e-12
                assert np.abs(col - He[e][:, c]).max() <= 2e-4 * scale


def test_project_psd():
    A = np.diag([-1.0, 2.0, 0.5])
    assert np.allclose(op.project_psd(A[None])[0], np.diag([0.0, 2.0, 0.5]), atol=1e-15)
    rng = np.random.default_rng(9)
    M = rng.standard_normal((5, 9, 9))
    S = M @ np.swapaxes(M, 1, 2)
    assert np.allclose(op.project_psd(S), S, atol=1e-12)
    Hs = M + np.swapaxes(M, 1, 2)
    P = op.project_psd(Hs)
    assert np.linalg.eigvalsh(P).min() > -1e-12
    # the projection is the nearest PSD matrix: H - P is negative semi-definite
    assert np.linalg.eigvalsh(Hs - P).max() < 1e-12


def test_pcg_against_direct_solve():
    import scipy.sparse.linalg as sla
    pb, X = _contact_problem()
    gr, H = op.assemble(len(X), op.elements(pb, X))
    p, it = op.pcg(H, -gr, 1e-12, 5000)
    want = sla.spsolve(H.tocsc(), -gr)
    assert it > 0
    assert np.linalg.norm(H @ p + gr) <= 1e-12 * np.linalg.norm(gr) * 1.0001
    assert np.linalg.norm(p - want) <= 1e-6 * np.linalg.norm(want)


# ---------------------------------------------------------------- ACCD
def test_accd_point_falls_on_triangle():
    R = _rot(3)
    T = np.array([[-1.0, -1, 0], [2, -1, 0], [-1, 2, 0]]) @ R.T
    for h, v in ((0.01, 0.02), (0.3, 0.5), (1e-4, 1.0)):
        x = np.vstack([np.array([0.1, 0.2, h]) @ R.T, T])[None]
        p = np.zeros((1, 4, 3))
        p[0, 0] = np.array([0, 0, -v]) @ R.T
        t = float(op.accd_pairs(x, p, "pt", 0.1, 1.0)[0])
        tstar = h / v  # impact time
        if tstar >= 1.0:
            continue
        assert t <= tstar * (1 - 0.1) + 1e-15  # stops before the distance falls below s h
        assert t >= 0.5 * tstar * (1 - 0.1)  # and is not far more cautious than that
    # moving apart: the whole step is safe
    x = np.vstack([[0.1, 0.2, 0.01], T @ R])[None]
    p = np.zeros((1, 4, 3))
    p[0, 0] = [0, 0, 0.5]
    assert float(op.accd_pairs(x, p, "pt", 0.1, 1.0)[0]) == 1.0


def test_accd_crossing_edges():
    # edge a along x at z = 0.05 moving down at speed 0.1; edge b along y at z = 0
    x = np.array([[[-1, 0, 0.05], [1, 0, 0.05], [0, -1, 0], [0, 1, 0]]], dtype=float)
    p = np.zeros_like(x)
    p[0, :2, 2] = -0.1
    t = float(op.accd_pairs(x, p, "ee", 0.1, 1.0)[0])
    assert 0.5 * 0.45 <= t <= 0.45 + 1e-15  # impact at 0.5, distance 10% of 0.05 left at 0.45


# ---------------------------------------------------------------- a short run
def test_short_run_descends_and_stays_free():
    Vin, Fin = g.noisy_icosphere(3, 2)
    r = orc.run(Vin, Fin, len(Fin) // 5)
    Vs, Fs = r["V"], r["F"]
    U = np.random.default_rng(0).random((512, 3))
    opt = op.Options(iterations=6, refresh=3)
    X, pb = op.safe_project(Vs, Fs, Vin, Fin, U, opt)
    B = [rec["B"] for rec in pb.log]
    # within a window of fixed targets B never increases; a refresh may change it
    for t in range(1, len(B)):
        if t % opt.refresh:
            assert B[t] <= B[t - 1]
    assert orc.self_intersections(X, Fs.astype(np.int32)).shape[0] == 0
    # the distance energy (both directions, targets found afresh) went down
    dis = []
    for Y in (Vs, X):
        op.refresh_targets(pb, Y, Vin, Fin)
        p = op.energy_parts(pb, Y)
        dis.append(p["s2m"] + p["m2s"])
    assert dis[1] < 0.7 * dis[0]
