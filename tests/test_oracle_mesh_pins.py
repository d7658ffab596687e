"""Pins of the oracle's round rule (no GPU).

Each test checks the oracle against something other than itself: a closed
form, a geometric identity, an alternative formulation of the selection
rule, the literal link condition on fixtures whose answer is known, or
invariants of the whole run (Euler characteristic, manifoldness, exact face
target, no self-intersection by an exact-rational brute force).
"""
import math
import struct
from collections import defaultdict

import numpy as np
import pytest

import oracle.oracle as orc
from lp_exact import tri_pair_exact
from paper_2509_05595_amd import meshgen as g

KMAX = np.uint64(2 ** 64 - 1)


# ---------------------------------------------------------------- quadrics
def test_quadric_is_sum_of_squared_plane_distances():
    """Q_v(p) = sum over faces around v of dist(p, plane(f))^2 (the defining
    property of Garland-Heckbert quadrics)."""
    V, F = g.bumpy_icosphere_gauss(k=3, seed=4)
    Q = orc.quadrics(V, F)
    rng = np.random.default_rng(0)
    inc = defaultdict(list)
    for f, t in enumerate(F):
        for v in t:
            inc[int(v)].append(f)
    for v in rng.choice(len(V), 100, replace=False):
        p = V[v] + rng.normal(scale=0.05, size=3)
        want = 0.0
        for f in inc[int(v)]:
            a, b, c = V[F[f]]
            n = np.cross(b - a, c - a)
            want += (np.dot(p - a, n) / np.linalg.norm(n)) ** 2
        got = orc.quadric_eval(Q[v], p)
        assert got == pytest.approx(want, rel=1e-9, abs=1e-15)
        # its own vertex lies on every incident plane
        assert abs(orc.quadric_eval(Q[v], V[v])) < 1e-14


def test_quadric_symmetric_psd():
    V, F = g.bumpy_icosphere_gauss(k=2, seed=5)
    Q = orc.quadrics(V, F)
    for q in Q[:50]:
        M = np.array([[q[0], q[1], q[2], q[3]], [q[1], q[4], q[5], q[6]],
                      [q[2], q[5], q[7], q[8]], [q[3], q[6], q[8], q[9]]])
        assert np.linalg.eigvalsh(M).min() > -1e-12


# ---------------------------------------------------------------- Eq. 1 terms
def test_skinny_closed_forms():
    eq = [0, 0, 0, 1, 0, 0, 0.5, math.sqrt(3) / 2, 0]
    assert abs(orc.skinny(eq)) < 4e-16                     # equilateral: C = 1
    ri = [0, 0, 0, 1, 0, 0, 0, 1, 0]
    assert orc.skinny(ri) == pytest.approx(1 - math.sqrt(3) / 2, abs=1e-15)  # C = sqrt(3)/2
    assert orc.skinny([0, 0, 0, 1, 1, 1, 2, 2, 2]) == 1.0  # collinear: C = 0
    rng = np.random.default_rng(1)
    for _ in range(100):
        T = rng.random(9)
        s = orc.skinny(T)
        assert 0.0 <= s <= 1.0 + 1e-15
        assert orc.skinny(T * 4.0) == s  # scale invariant (power-of-two scale is exact)


def test_cube_edge_placement_and_cost():
    """Edge (0,0,0)-(1,0,0) of the two-triangles-per-side cube: the quadric
    sum is 2[x=0] + 2[x=1] + 3[y=0] + 3[z=0], minimised at (0.5, 0, 0) with
    value 2*0.25 + 2*0.25 = 1."""
    V, F = g.cube()
    cost, vbar = orc.edge_cost(V, F, 0, 4, w_e=0.0, w_s=0.0)
    assert vbar.tolist() == [0.5, 0.0, 0.0]
    assert cost == 1.0
    cost2, _ = orc.edge_cost(V, F, 0, 4, w_e=1.0, w_s=0.0)
    assert cost2 == 2.0  # + w_e * length 1


def test_fallback_placement_is_best_of_three():
    """When the quadric minimiser is rejected the new vertex is whichever of
    midpoint / endpoint / endpoint has the smallest quadric error."""
    V, F = g.bumpy_icosphere_gauss(k=2, seed=7)
    Q = orc.quadrics(V, F)
    seen = 0
    edges = {(min(a, b), max(a, b)) for t in F for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    for a, b in sorted(edges):
        _, vbar = orc.edge_cost(V, F, a, b, w_e=0.0, w_s=0.0)
        q = Q[a] + Q[b]
        mid = (V[a] + V[b]) * 0.5
        opts = [mid, V[a], V[b]]
        if any(np.array_equal(vbar, o) for o in opts):
            seen += 1
            errs = [orc.quadric_eval(q, o) for o in opts]
            assert orc.quadric_eval(q, vbar) == min(errs)
    assert seen > 0


# ---------------------------------------------------------------- keys
def _f32_total_order(x):
    b = struct.unpack("<I", struct.pack("<f", x))[0]
    return -(b & 0x7FFFFFFF) - 1 if b >> 31 else b  # -0 sorts below +0


def test_key_order_matches_float32_order():
    rng = np.random.default_rng(3)
    vals = list(rng.normal(scale=1e-3, size=300)) + list(rng.normal(scale=1e3, size=100))
    vals += [0.0, -0.0, 1e-45, -1e-45, 5e-324, -5e-324, 3.4e38, -3.4e38, 1e300, -1e300,
             float("inf"), float("-inf")]
    for i, x in enumerate(vals):
        for y in vals[i + 1: i + 40]:
            fx, fy = np.float32(x), np.float32(y)
            kx, ky = orc.make_key(x, 7), orc.make_key(y, 7)
            ox, oy = _f32_total_order(float(fx)), _f32_total_order(float(fy))
            assert (kx < ky) == (ox < oy) and (kx == ky) == (ox == oy)
    assert orc.make_key(float("nan"), 5) == 2 ** 64 - 1
    assert orc.make_key(1.0, 5) < orc.make_key(1.0, 6)  # ties broken by edge id
    assert orc.make_key(1.0, 5) & 0xFFFFFFFF == 5


# ---------------------------------------------------------------- selection
def _edges_with_keys(V, F, keys):
    out = []
    for h in np.nonzero(keys != KMAX)[0]:
        f, c = divmod(int(h), 3)
        out.append((int(h), int(F[f][c]), int(F[f][(c + 1) % 3]), int(keys[h])))
    return out


def _ring(inc, a, b):
    return set(inc[a]) | set(inc[b])


@pytest.mark.parametrize("mesh", ["ico2", "nested", "torus"])
def test_selection_pairwise_definition(mesh):
    """Candidates are exactly the edges whose key is smaller than the key of
    every other edge whose 1-ring shares a triangle with theirs; no two
    candidates share a triangle; the pull form (vertex minima over the closed
    neighbourhood) picks the same set."""
    if mesh == "ico2":
        V, F = g.bumpy_icosphere_gauss(k=2, seed=8)
    elif mesh == "nested":
        V, F = g.nested_spheres(k=2, gap=0.02)
    else:
        V, F = g.bumpy_torus(24, 10, seed=3)
    keys = orc.keys(V, F)
    cand = set(orc.select(V, F).tolist())
    inc = defaultdict(list)
    for f, t in enumerate(F):
        for v in t:
            inc[int(v)].append(f)
    E = _edges_with_keys(V, F, keys)
    by_face = defaultdict(list)
    rings = {}
    for h, a, b, k in E:
        rings[h] = _ring(inc, a, b)
        for t in rings[h]:
            by_face[t].append((k, h))
    want = set()
    for h, a, b, k in E:
        rivals = {hh for t in rings[h] for _, hh in by_face[t]} - {h}
        if all(keys[r] > k for r in rivals):
            want.add(h)
    assert cand == want and len(cand) > 0
    cl = sorted(cand)
    for i in range(len(cl)):
        for j in range(i + 1, len(cl)):
            assert not (rings[cl[i]] & rings[cl[j]])
    # pull form
    m = defaultdict(lambda: 2 ** 64 - 1)
    nbr = defaultdict(set)
    for h, a, b, k in E:
        m[a] = min(m[a], k)
        m[b] = min(m[b], k)
    for t in F:
        for x in t:
            nbr[int(x)].update(int(y) for y in t)
    pull = {h for h, a, b, k in E if k == min(m[w] for w in nbr[a] | nbr[b])}
    assert pull == cand


# ---------------------------------------------------------------- link condition
def test_link_condition_fixtures():
    V, F = g.tetrahedron()
    r = orc.run(V, F, 2)
    assert r["stats"]["status"] == 1 and len(r["F"]) == 4 and r["stats"]["rej_link"] > 0
    V, F = g.csaszar_torus()
    r = orc.run(V, F, 2)
    assert r["stats"]["status"] == 1 and len(r["F"]) == 14
    assert r["stats"]["rej_link"] > 0 and r["stats"]["rej_flip"] == 0 and r["stats"]["rej_isect"] == 0
    V, F = g.octahedron()
    r = orc.run(V, F, 6)
    assert r["stats"]["status"] == 0 and len(r["F"]) == 6 and orc.validate(r["V"], r["F"]) == 0


# ---------------------------------------------------------------- whole runs
def _euler(V, F):
    e = {(min(a, b), max(a, b)) for t in F for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    return len(np.unique(F)) - len(e) + len(F)


def _lp_self_intersections(V, F):
    lo = V[F].min(axis=1)
    hi = V[F].max(axis=1)
    n = 0
    for t in range(len(F)):
        ov = np.nonzero(np.all(lo[t + 1:] <= hi[t], axis=1) & np.all(lo[t] <= hi[t + 1:], axis=1))[0] + t + 1
        for u in ov:
            if tri_pair_exact(V[F[t]], F[t], V[F[u]], F[u]):
                n += 1
    return n


@pytest.mark.parametrize("case", ["ico2_32", "ico2_odd", "torus", "nested"])
def test_run_invariants_small(case):
    if case == "ico2_32":
        V, F = g.bumpy_icosphere_gauss(k=2, seed=1)
        target = 32
    elif case == "ico2_odd":
        V, F = g.bumpy_icosphere_gauss(k=2, seed=2)
        target = 101
    elif case == "torus":
        V, F = g.bumpy_torus(24, 10, seed=5)
        target = 48
    else:
        V, F = g.nested_spheres(k=2, gap=0.02)
        target = 40
    assert orc.validate(V, F) == 0 and _lp_self_intersections(V, F) == 0
    r = orc.run(V, F, target)
    Vo, Fo, st = r["V"], r["F"], r["stats"]
    if st["status"] == 0:
        assert len(Fo) == target - target % 2
    else:
        assert st["status"] == 1 and len(Fo) > target
    assert orc.validate(Vo, Fo) == 0
    assert _euler(Vo, Fo) == _euler(V, F)
    assert _lp_self_intersections(Vo, Fo) == 0
    assert len(Vo) == len(np.unique(Fo))  # no orphan vertex
    if case == "nested":
        assert st["rej_isect"] > 0 and sum(st["undo_hist"][1:]) > 0


def test_run_small_case_5120_to_512():
    V, F = g.bumpy_icosphere_gauss()
    assert len(F) == 5120 and len(V) == 2562
    r = orc.run(V, F, 512, log_rounds=200)
    assert r["stats"]["status"] == 0 and len(r["F"]) == 512
    assert orc.validate(r["V"], r["F"]) == 0
    assert len(orc.self_intersections(r["V"], r["F"])) == 0
    assert _euler(r["V"], r["F"]) == 2
    # faces drop by exactly two per commit, every round
    log = r["log"]
    for a, b in zip(log, log[1:]):
        assert a["faces"] - 2 * a["commits"] == b["faces"]


def test_run_resumes_bitwise():
    """Stopping after k rounds and resuming from the returned state (mesh,
    flags, streak) gives the same result as one uninterrupted run."""
    V, F = g.nested_spheres(k=2, gap=0.02)
    full = orc.run(V, F, 60)
    part = orc.run(V, F, 60, max_rounds=5)
    rest = orc.run(part["V"], part["F"], 60, flags=part["flags"], streak=part["streak"])
    assert np.array_equal(full["F"], rest["F"])
    assert np.array_equal(full["V"], rest["V"])
    assert full["stats"]["rounds"] == part["stats"]["rounds"] + rest["stats"]["rounds"]


def test_flags_retained_over_zero_commit_rounds():
    """Sec. 5.3: when a round collapses nothing, the invalid flags are kept
    (and new ones added) until something collapses or the tolerance (4) is
    reached.  On the seven-vertex torus every round rejects one edge."""
    V, F = g.csaszar_torus()
    prev = None
    for k in range(1, 5):
        r = orc.run(V, F, 2, max_rounds=k)
        fl = r["flags"].astype(bool)
        assert r["streak"] == k and fl.sum() == 2 * k
        if prev is not None:
            assert np.all(fl[prev])  # superset of the previous round's flags
        prev = fl
    assert orc.run(V, F, 2)["stats"]["rounds"] == 4


def _exact_dot_sign(o0, o1, o2, p0, p1, p2):
    from fractions import Fraction as Fr
    o0, o1, o2, p0, p1, p2 = ([Fr(float(x)) for x in p] for p in (o0, o1, o2, p0, p1, p2))

    def cross(a, b, c):
        u = [b[i] - a[i] for i in range(3)]
        v = [c[i] - a[i] for i in range(3)]
        return [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]

    a, b = cross(o0, o1, o2), cross(p0, p1, p2)
    d = sum(x * y for x, y in zip(a, b))
    return (d > 0) - (d < 0), all(x == 0 for x in b)


def test_flip_rejections_match_exact_normal_test():
    """A candidate is rejected for flipping exactly when some triangle it
    generates has a normal at 90 degrees or more from its old normal (or is
    degenerate); checked with exact rational arithmetic on every candidate of
    rounds that reject for that reason (pure-QEM weights on a creased sphere
    produce such rounds)."""
    V, F = g.crease_sphere(3, 5)
    flips_seen = 0
    state = {"V": V, "F": F, "flags": None, "streak": 0}
    for _ in range(4):
        cand, vbar, reason, _ = orc.check(state["V"], state["F"], 16, flags=state["flags"], w_e=0.0, w_s=0.0)
        Vs, Fs = state["V"], state["F"]
        for c, h in enumerate(cand):
            if reason[c] not in (0, 2, 3, 4):
                continue
            f, k = divmod(int(h), 3)
            a, b = int(Fs[f][k]), int(Fs[f][(k + 1) % 3])
            bad = False
            for t in np.nonzero(np.any(Fs == a, axis=1) | np.any(Fs == b, axis=1))[0]:
                tri = Fs[t]
                if a in tri and b in tri:
                    continue
                newp = [vbar[c] if x in (a, b) else Vs[x] for x in tri]
                sgn, degen = _exact_dot_sign(Vs[tri[0]], Vs[tri[1]], Vs[tri[2]], *newp)
                bad |= sgn <= 0 or degen
            # rounding of the float64 dot can only matter when it is ~0; the
            # fixtures stay far from that
            assert bad == (reason[c] == 2), (c, reason[c])
            flips_seen += reason[c] == 2
        r = orc.run(state["V"], state["F"], 16, flags=state["flags"], streak=state["streak"],
                    max_rounds=1, w_e=0.0, w_s=0.0)
        state = {"V": r["V"], "F": r["F"], "flags": r["flags"], "streak": r["streak"]}
    assert flips_seen > 0
