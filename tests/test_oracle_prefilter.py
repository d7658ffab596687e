"""The link/flip pre-filter in the oracle (reading: the local checks of
Sec. 5.1 run on every keyed edge before the selection instead of on the
candidates after it, and a failing edge is not selectable that round).  Pins
that do not reuse the oracle's checks: the link condition by its set
definition and the flip test with exact rational arithmetic, in Python."""
from collections import defaultdict
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g

KMAX = np.uint64(2 ** 64 - 1)


def _stars(F):
    inc = defaultdict(list)
    for f, t in enumerate(F):
        for v in t:
            inc[int(v)].append(f)
    return inc


def _link_ok(F, inc, a, b):
    """Lk(a) n Lk(b) == Lk(ab) as simplicial complexes."""
    def link(v):
        verts, edges = set(), set()
        for f in inc[v]:
            o = [int(x) for x in F[f] if x != v]
            verts.update(o)
            edges.add(frozenset(o))
        return verts, edges
    va, ea = link(a)
    vb, eb = link(b)
    apex = {int(x) for f in inc[a] if b in F[f] for x in F[f] if x not in (a, b)}
    return (va & vb) == apex and not (ea & eb)


def _cross(p, q, r):
    u = [q[i] - p[i] for i in range(3)]
    v = [r[i] - p[i] for i in range(3)]
    return [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]


def _flips(V, F, inc, a, b, vbar):
    """some surviving ring face becomes degenerate or turns by >= 90 degrees"""
    for f in set(inc[a]) | set(inc[b]):
        t = [int(x) for x in F[f]]
        if a in t and b in t:
            continue
        old = [[Fr(float(x)) for x in V[v]] for v in t]
        new = [[Fr(float(x)) for x in (vbar if v in (a, b) else V[v])] for v in t]
        n0, n1 = _cross(*old), _cross(*new)
        if all(x == 0 for x in n1) or sum(x * y for x, y in zip(n0, n1)) <= 0:
            return True
    return False


def _select(F, keys):
    """pull form of the selection over the given keys"""
    m = defaultdict(lambda: KMAX)
    nbr = defaultdict(set)
    E = []
    for h in np.nonzero(keys != KMAX)[0]:
        f, c = divmod(int(h), 3)
        a, b = int(F[f][c]), int(F[f][(c + 1) % 3])
        E.append((int(h), a, b, keys[h]))
        m[a] = min(m[a], keys[h])
        m[b] = min(m[b], keys[h])
    for t in F:
        for x in t:
            nbr[int(x)].update(int(y) for y in t)
    return {h for h, a, b, k in E if k == min(m[w] for w in nbr[a] | nbr[b])}


def test_selection_is_over_the_passing_edges():
    # pure-QEM weights on a creased sphere: some edges flip triangles; the
    # rounds of a plain run give the states
    V, F = g.crease_sphere(3, 5)
    w = dict(w_e=0.0, w_s=0.0)
    state = {"V": V, "F": F, "flags": None, "streak": 0}
    failing = changed = 0
    for _ in range(6):
        V, F, flags = state["V"], state["F"], state["flags"]
        keys = orc.keys(V, F, flags=flags, **w)
        inc = _stars(F)
        filtered = keys.copy()
        for h in np.nonzero(keys != KMAX)[0]:
            f, c = divmod(int(h), 3)
            a, b = int(F[f][c]), int(F[f][(c + 1) % 3])
            vbar = orc.edge_cost(V, F, a, b, **w)[1]
            if not _link_ok(F, inc, a, b) or _flips(V, F, inc, a, b, vbar):
                filtered[h] = KMAX
                failing += 1
        want = _select(F, filtered)
        cand, _, reason, _ = orc.check(V, F, 16, flags=flags, prefilter=1, **w)
        assert set(cand.tolist()) == want
        assert not np.any((reason == 1) | (reason == 2))
        plain = set(orc.check(V, F, 16, flags=flags, **w)[0].tolist())
        assert plain == _select(F, keys)
        changed += plain != want
        r = orc.run(V, F, 16, flags=flags, streak=state["streak"], max_rounds=1, **w)
        state = {"V": r["V"], "F": r["F"], "flags": r["flags"], "streak": r["streak"]}
    assert failing > 0 and changed > 0


def test_no_local_rejections_in_a_prefiltered_run():
    V, F = g.crease_sphere(3, 5)
    w = dict(w_e=0.0, w_s=0.0)
    plain = orc.run(V, F, 16, **w)
    pre = orc.run(V, F, 16, prefilter=1, **w)
    assert plain["stats"]["rej_flip"] > 0
    assert pre["stats"]["rej_link"] == 0 and pre["stats"]["rej_flip"] == 0
    assert pre["stats"]["status"] == 0 and len(pre["F"]) == 16
    assert orc.validate(pre["V"], pre["F"]) == 0


@pytest.mark.parametrize("make,nf", [(g.tetrahedron, 4), (g.csaszar_torus, 14)])
def test_link_fixtures_select_nothing(make, nf):
    # every edge fails the link condition, so no edge is ever a candidate
    V, F = make()
    r = orc.run(V, F, 2, prefilter=1, log_rounds=8)
    assert r["stats"]["status"] == 1 and len(r["F"]) == nf
    assert r["stats"]["candidates"] == 0 and r["stats"]["rej_link"] == 0
    assert orc.run(V, F, 2)["stats"]["rej_link"] > 0
