"""The float64 key mode in the oracle (reading: the paper converts edge costs
from floats to 32-bit codes for its atomic propagation; the other reading
orders edges by the float64 cost and then by edge id).  Pins: the selection
against a Python restatement over (float64 cost, id) pairs, the costs from the
oracle's per-edge routine; whole-run invariants on a mesh where float32
rounding merges distinct float64 costs."""
from collections import defaultdict

import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g


def _edges(F):
    """every edge once, by its half-edge of the lower id"""
    he = {(int(F[h // 3, h % 3]), int(F[h // 3, (h % 3 + 1) % 3])): h for h in range(3 * len(F))}
    return [(h, a, b) for (a, b), h in he.items() if h < he[(b, a)]]


def _select(F, keyed):
    """pull form of the selection: keyed = {h: (a, b, key)}, keys comparable"""
    INF = (float("inf"), 1 << 62)
    m = defaultdict(lambda: INF)
    nbr = defaultdict(set)
    for h, (a, b, k) in keyed.items():
        m[a] = min(m[a], k)
        m[b] = min(m[b], k)
    for t in F:
        for x in t:
            nbr[int(x)].update(int(y) for y in t)
    return {h for h, (a, b, k) in keyed.items() if k == min(m[w] for w in nbr[a] | nbr[b])}


@pytest.mark.parametrize("mesh", ["regular", "bumpy"])
def test_selection_by_float64_cost_then_id(mesh):
    V, F = (g.bumpy_icosphere_gauss(k=3, seed=3, sigma=0.0) if mesh == "regular"
            else g.bumpy_icosphere_gauss(k=2, seed=8))
    keyed = {}
    for h, a, b in _edges(F):
        c = orc.edge_cost(V, F, a, b)[0]
        keyed[h] = (a, b, (c, h))
    want = _select(F, keyed)
    got = set(orc.check(V, F, 0, key_mode=1)[0].tolist())
    assert got == want and len(got) > 0
    if mesh == "regular":
        # float32 codes tie costs that float64 tells apart: the modes differ
        assert set(orc.select(V, F).tolist()) != want


def _euler(V, F):
    E = len({tuple(sorted((int(a), int(b)))) for t in F for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))})
    return len(np.unique(F)) - E + len(F)


def test_run_invariants_and_difference():
    V, F = g.bumpy_icosphere_gauss(k=3, seed=3, sigma=0.0)
    a = orc.run(V, F, 100)
    b = orc.run(V, F, 100, key_mode=1)
    assert b["stats"]["status"] == 0 and len(b["F"]) == 100
    assert orc.validate(b["V"], b["F"]) == 0 and _euler(b["V"], b["F"]) == 2
    assert not np.array_equal(a["F"], b["F"])


def test_learned_and_logging_refuse_the_float64_key():
    V, F = g.bumpy_icosphere_gauss(k=2, seed=8)
    with pytest.raises(ValueError):
        orc.collect(V, F, 64, key_mode=1)
