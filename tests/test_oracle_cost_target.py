"""Target-cost termination in the oracle (the paper ends a run at a target
edge cost or at a target face count, Sec. 5.1 "Edge Collapse"; reading: only
edges whose Eq. 1 cost is at most the target are collapsed, and a round that
selects no edge ends the run).  Pins that do not reuse the rule's own code:
the edge costs come from the oracle's independent per-edge routine."""
import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g


def edges(F):
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    return np.unique(np.sort(e, axis=1), axis=0)


def all_costs(V, F):
    return np.array([orc.edge_cost(V, F, a, b)[0] for a, b in edges(F)])


@pytest.fixture(scope="module")
def mesh():
    return g.bumpy_icosphere_gauss(k=3, seed=1)  # 1,280 faces


def test_unreachable_cost_target_changes_nothing(mesh):
    V, F = mesh
    a = orc.run(V, F, len(F) // 10)
    b = orc.run(V, F, len(F) // 10, cost_target=1e30)
    assert np.array_equal(a["F"], b["F"]) and np.array_equal(a["V"].view(np.uint64), b["V"].view(np.uint64))
    assert a["stats"] == b["stats"]


def test_target_below_every_cost_stops_after_one_empty_round(mesh):
    V, F = mesh
    c = all_costs(V, F)
    assert c.min() > 0
    r = orc.run(V, F, 0, cost_target=0.5 * c.min())
    assert r["stats"]["rounds"] == 1 and r["stats"]["candidates"] == 0 and r["stats"]["status"] == 0
    assert np.array_equal(r["F"], F)


@pytest.mark.parametrize("q", [0.05, 0.3])
def test_at_the_end_every_unflagged_edge_costs_more_than_the_target(mesh, q):
    V, F = mesh
    target = float(np.quantile(all_costs(V, F), q))
    r = orc.run(V, F, 0, cost_target=target)
    assert r["stats"]["status"] == 0 and r["stats"]["commits"] > 0
    Vo, Fo, fl = r["V"], r["F"], r["flags"]
    flagged = set()
    for f in range(len(Fo)):
        for c in range(3):
            if fl[3 * f + c]:
                flagged.add(tuple(sorted((Fo[f, c], Fo[f, (c + 1) % 3]))))
    for a, b in edges(Fo):
        if (a, b) in flagged:
            continue
        assert orc.edge_cost(Vo, Fo, a, b)[0] > target
    # a face target reached first ends the run there
    r2 = orc.run(V, F, len(F) - 200, cost_target=target)
    assert len(r2["F"]) <= len(F) - 200 or r2["stats"]["rounds"] == r["stats"]["rounds"]
