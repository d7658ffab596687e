"""Pins of the learned-proposal parts of the oracle (CPU only).

Each check compares the oracle with something other than itself: features of
meshes whose values are known in closed form, overlap counts by brute force,
network logits in exact rational arithmetic, gradients by finite
differences, the Adam step in closed form, and the learned run against the
plain run when the network sets nothing aside.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle.oracle as orc
import oracle.mlp_train as mt
from paper_2509_05595_amd import meshgen as g


def plog2_ref(c):
    """piecewise-linear log2 from its definition: exact at powers of two,
    linear in between (independent of frexp)."""
    e = int(np.floor(np.log2(c)))
    while 2.0 ** e > c:
        e -= 1
    while 2.0 ** (e + 1) <= c:
        e += 1
    return e + (c - 2.0 ** e) / 2.0 ** e


def q(f, s):
    return float(np.clip(np.rint(f * 2.0 ** s), -127, 127))


def brute_ovl(V, F):
    lo = V[F].min(axis=1)
    hi = V[F].max(axis=1)
    n = len(F)
    out = np.zeros(n, dtype=np.int64)
    for t in range(n):
        meet = np.all((lo <= hi[t]) & (lo[t] <= hi), axis=1)
        share = np.isin(F, F[t]).any(axis=1)
        meet &= ~share
        meet[t] = False
        out[t] = meet.sum()
    return out


def test_octahedron_features_closed_form():
    V, F = g.octahedron()
    cand = orc.select(V, F)
    assert len(cand) > 0
    X, ovl = orc.features(V, F, cand)
    # every edge: length sqrt(1/2) after scaling to the unit cube, valence 4,
    # two common neighbours, all spokes equally long; adjacent faces meet at
    # the dihedral angle arccos(-1/3), so their outward normals at arccos(1/3)
    le = np.sqrt(0.5)
    for row, h in zip(X, cand):
        a, b = F.ravel()[h], F[h // 3][(h % 3 + 1) % 3]
        cost, _ = orc.edge_cost(V, F, a, b)
        assert row[0] == q(plog2_ref(float(np.float32(cost))), 2)
        assert row[1] == q(plog2_ref(le), 3)
        assert row[2] == 127 and row[3] == 127
        assert row[4] == q(1 / 3, 6) == 21 and row[5] == 21
        assert row[6] == row[7] == 16 and row[8] == 32
        assert np.all(row[11:] == 0)
    assert np.array_equal(ovl, brute_ovl(V, F))


def test_plog2_against_definition():
    # plog2 through feature 1 on scaled tetrahedra: edge lengths known
    for s in (0.25, 0.3, 0.5, 0.7, 1.0):
        V, F = g.tetrahedron()
        V = V * s
        X, _ = orc.features(V, F, [0])
        le = s  # edge from vertex 0 to vertex 2 has length s
        a, b = F.ravel()[0], F[0][1]
        assert np.isclose(np.linalg.norm(V[a] - V[b]), le)
        assert X[0, 1] == q(plog2_ref(le), 3)


@pytest.mark.parametrize("mesh", ["nested", "noisy"])
def test_overlap_counts_brute_force(mesh):
    V, F = g.nested_spheres(k=2, gap=0.02) if mesh == "nested" else g.bumpy_icosphere_gauss(k=2, seed=3)
    _, ovl = orc.features(V, F, [])
    assert np.array_equal(ovl, brute_ovl(V, F))
    if mesh == "nested":
        assert ovl.max() > 0


def random_model(rng, e=(9, 9, 9), a=(-3, -3), threshold=0.0):
    m = {"w1": rng.integers(-127, 128, (64, 32)) * 2.0 ** -e[0], "b1": rng.integers(-2000, 2000, 64) * 2.0 ** -e[0],
         "w2": rng.integers(-127, 128, (64, 64)) * 2.0 ** -e[1], "b2": rng.integers(-2000, 2000, 64) * 2.0 ** -e[1],
         "w3": rng.integers(-127, 128, 64) * 2.0 ** -e[2], "b3": float(rng.integers(-2000, 2000)) * 2.0 ** -e[2],
         "e1": e[0], "e2": e[1], "e3": e[2], "a1": a[0], "a2": a[1], "threshold": threshold}
    return {k: (np.asarray(v, dtype=np.float32) if isinstance(v, np.ndarray) else v) for k, v in m.items()}


def exact_logit(m, x):
    def rq(v, a):  # round half to even of v * 2^a, clamp to [0, 127]
        v = max(v, Fraction(0)) * Fraction(2) ** a
        fl = v.numerator // v.denominator
        r = v - fl
        n = fl + (1 if r > Fraction(1, 2) or (r == Fraction(1, 2) and fl % 2) else 0)
        return min(n, 127)
    F_ = Fraction
    h1 = [rq(F_(float(m["b1"][j])) + sum(F_(float(m["w1"][j][k])) * F_(float(x[k])) for k in range(32)), m["a1"])
          for j in range(64)]
    h2 = [rq(F_(float(m["b2"][j])) + sum(F_(float(m["w2"][j][k])) * h1[k] for k in range(64)), m["a2"])
          for j in range(64)]
    return F_(float(m["b3"])) + sum(F_(float(m["w3"][k])) * h2[k] for k in range(64))


def test_mlp_logits_exact():
    rng = np.random.default_rng(7)
    m = random_model(rng)
    X = rng.integers(-127, 128, (40, 32)).astype(np.float32)
    X[:, 11:] = 0
    got = orc.mlp_logits(m, X)
    for i in range(len(X)):
        assert Fraction(got[i]) == exact_logit(m, X[i])


def test_learned_run_without_set_aside_equals_plain():
    V, F = g.nested_spheres(k=2, gap=0.02)
    m = random_model(np.random.default_rng(1), threshold=-1e30)
    r = orc.run_learned(V, F, 64, m)
    p = orc.run(V, F, 64)
    assert r["demoted"] == 0 and r["fallbacks"] == 0
    assert np.array_equal(r["F"], p["F"]) and np.array_equal(r["V"].view(np.uint64), p["V"].view(np.uint64))
    assert r["stats"] == p["stats"]


def test_learned_run_valid_output():
    V, F = g.nested_spheres(k=3, gap=0.01)
    # a model that sets aside edges with many overlapping faces around them
    m = random_model(np.random.default_rng(2), e=(0, 0, 0), threshold=0.0)
    m["w1"][:] = 0
    m["b1"][:] = 0
    m["w1"][0, 9] = 1.0  # unit 0 = sum of overlap counts
    m["w2"][:] = 0
    m["b2"][:] = 0
    m["w2"][0, 0] = 1.0
    m["w3"][:] = 0
    m["w3"][0] = -1.0
    m["b3"] = 4.0  # logit = 4 - (sum of overlap counts): set aside when crowded
    m["a1"] = 0
    m["a2"] = 0
    r = orc.run_learned(V, F, 128, m)
    assert r["demoted"] > 0 and r["fallbacks"] > 0
    # the gap is too small for this target at this resolution: both forms
    # stop after the tolerance rounds; the output must still be valid
    assert r["stats"]["status"] == 1 and len(r["F"]) < len(F)
    assert orc.validate(r["V"], r["F"]) == 0
    assert len(orc.self_intersections(r["V"], r["F"])) == 0


def test_collect_rows_and_labels():
    V, F = g.nested_spheres(k=2, gap=0.02)
    X, y, r = orc.collect(V, F, 64)
    p = orc.run(V, F, 64, log_rounds=200)
    rows = sum(L["candidates"] - L["capped"] for L in p["log"])
    assert len(X) == rows and len(y) == rows
    assert y.sum() == p["stats"]["commits"]
    assert np.array_equal(r["F"], p["F"])
    assert np.all(X[:, 11:] == 0)


def meta():
    return {"e1": 9, "e2": 9, "e3": 9, "a1": -3, "a2": -3}


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    P = rng.normal(0, 0.05, mt.NPARAM)
    X = rng.normal(0, 1, (32, 32))
    y = rng.integers(0, 2, 32).astype(np.float64)
    md = meta()
    _, gr = mt.loss_and_grad(P, md, X, y, quantize=False)
    idx = rng.choice(mt.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (mt.loss_and_grad(Pp, md, X, y, False)[0] - mt.loss_and_grad(Pm, md, X, y, False)[0]) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, gr[i])


def test_quantised_forward_matches_exact_oracle():
    rng = np.random.default_rng(4)
    P = rng.normal(0, 0.05, mt.NPARAM)
    md = meta()
    X = rng.integers(-127, 128, (20, 32)).astype(np.float64)
    z, _ = mt.forward(P, md, X)
    model = mt.model_dict(P, md, 0.0)
    assert np.array_equal(z, orc.mlp_logits(model, X.astype(np.float32)))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    P = rng.normal(0, 1, 50)
    g_ = rng.normal(0, 1, 50)
    P1, m, v = mt.adam(P, np.zeros(50), np.zeros(50), g_, 1, lr=0.01)
    assert np.allclose(P1, P - 0.01 * g_ / (np.abs(g_) + 1e-8))


def test_point_triangle_distance_regions():
    import oracle.hausdorff as hd
    A, B, C = np.array([[0.0, 0, 0]]), np.array([[1.0, 0, 0]]), np.array([[0.0, 1, 0]])
    cases = [([0.25, 0.25, 0.7], 0.7),                      # above the interior: the height
             ([-1.0, -1.0, 0.0], np.sqrt(2.0)),             # beyond vertex A
             ([0.5, -2.0, 1.0], np.sqrt(5.0)),              # beside edge AB
             ([1.0, 1.0, 0.0], np.sqrt(0.5)),               # beside edge BC, in the plane
             ([3.0, 0.0, 4.0], np.sqrt(4.0 + 16.0))]        # beyond vertex B
    for p, d in cases:
        assert np.isclose(hd.point_tris(np.array(p), A, B, C)[0], d, rtol=1e-14)


def test_hausdorff_of_a_mesh_to_itself_and_a_scaled_copy():
    import oracle.hausdorff as hd
    V, F = g.icosphere(2)
    assert hd.hausdorff(V, V, F) == 0.0
    # a sphere scaled by 1.1 about its centre: every vertex of the big one is
    # at least 0.1 r from the small mesh (which lies inside the unit sphere)
    c = V.mean(axis=0)
    big = c + 1.1 * (V - c)
    r = np.linalg.norm(V - c, axis=1).max()
    d = hd.hausdorff(big, V, F)
    assert 0.1 * r - 1e-12 <= d <= 0.1 * r + 0.02 * r
