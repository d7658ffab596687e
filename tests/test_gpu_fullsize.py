"""Full-size parity on the benchmark workload (GPU).

* The whole run of the 1,310,720-face noisy icosphere to 1% and to 0.1% is
  compared bit for bit with the CPU oracle through SHA-256 digests that
  tests/golden/make_golden.py wrote by running only the oracle.
* Round 0 at full size is compared element by element with the oracle
  (candidates, reasons, placements, the committed mesh).
* Properties that hold at any size are checked on the output: exact face
  count, Euler characteristic, manifoldness (the library's own adjacency
  build), no self-intersection (the library's whole-mesh test and the
  oracle's on the small output).
The launch configuration is the one bench.py times (default options).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_oracle.json")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_05595_amd import native
    c = native.Context("cuda:0")
    yield c
    c.close()


@pytest.fixture(scope="module")
def mesh():
    V, F = g.noisy_icosphere(8, 2)
    return V, F, torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()


def euler(F):
    e = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
    ne = len(np.unique(e[:, 0].astype(np.int64) * (1 << 32) + e[:, 1]))
    return len(np.unique(F)) - ne + len(F)


@pytest.mark.parametrize("label,frac", [("1pct", 0.01), ("0.1pct", 0.001)])
def test_full_run_matches_oracle_digest(ctx, mesh, label, frac):
    gold = json.load(open(GOLDEN))[f"noisy_icosphere_k8_seed2_{label}"]
    V, F, Vd, Fd = mesh
    assert sha(V) == gold["input_V_sha256"] and sha(F) == gold["input_F_sha256"], "generator changed"
    target = int(len(F) * frac)
    Vo, Fo, st = ctx.simplify(Vd, Fd, target)
    Vg, Fg = Vo.cpu().numpy(), Fo.cpu().numpy()
    assert len(Fg) == gold["faces_out"] == target - target % 2
    assert st["rounds"] == gold["stats"]["rounds"]
    for k in ("commits", "rej_link", "rej_flip", "rej_isect", "capped"):
        assert st[k] == gold["stats"][k], k
    assert sha(Fg) == gold["F_sha256"]
    assert sha(Vg) == gold["V_sha256"]
    # properties at any size
    assert euler(Fg) == 2
    ctx.quadrics(Vo.contiguous(), Fo.contiguous())  # raises unless closed and manifold
    _, n = ctx.self_intersections(Vo.contiguous(), Fo.contiguous())
    assert n == 0
    assert len(orc.self_intersections(Vg, Fg)) == 0


def test_round0_full_size_elementwise(ctx, mesh):
    V, F, Vd, Fd = mesh
    target = len(F) // 100
    cand, _, n = ctx.select(Vd, Fd)
    vbar, reason, iters = ctx.check(Vd, Fd, target, cand, n)
    co, vo, ro, it_o = orc.check(V, F, target)
    assert np.array_equal(cand.cpu().numpy(), co)
    assert np.array_equal(reason.cpu().numpy(), ro)
    assert np.array_equal(vbar.cpu().numpy().view(np.uint64), vo.view(np.uint64))
    assert iters == it_o
    V1, F1, fl1 = ctx.collapse(Vd, Fd, cand, n, vbar, reason)
    r = orc.run(V, F, target, max_rounds=1)
    assert np.array_equal(F1.cpu().numpy(), r["F"])
    assert np.array_equal(V1.cpu().numpy().view(np.uint64), r["V"].view(np.uint64))
    assert np.array_equal(fl1.cpu().numpy(), r["flags"])


@pytest.mark.parametrize("opt", [{"prefilter": 1}, {"key_mode": 1}, {"prefilter": 1, "key_mode": 1}])
def test_rule_variants_full_size(ctx, mesh, opt):
    """The pre-filter and the float64 key mode on the 1,310,720-face mesh: the
    round-0 selection element by element against the oracle, and the whole run
    to 1% checked by properties that hold at any size."""
    from paper_2509_05595_amd import native
    V, F, Vd, Fd = mesh
    target = len(F) // 100
    ctx.set_options(native.default_options(**opt))
    try:
        cand, _, _ = ctx.select(Vd, Fd)
        Vo, Fo, st = ctx.simplify(Vd, Fd, target)
    finally:
        ctx.set_options(native.default_options())
    co = orc.check(V, F, target, **opt)[0]
    assert np.array_equal(np.sort(cand.cpu().numpy()), np.sort(co))
    Fg = Fo.cpu().numpy()
    assert st["status"] == 0 and len(Fg) == target - target % 2
    assert euler(Fg) == 2
    ctx.quadrics(Vo.contiguous(), Fo.contiguous())  # raises unless closed and manifold
    _, n = ctx.self_intersections(Vo.contiguous(), Fo.contiguous())
    assert n == 0
    if opt.get("prefilter"):
        assert st["rej_link"] == 0 and st["rej_flip"] == 0


def test_round0_beyond_two_pass_scan(ctx):
    """Round 0 of a 1,568,000-face noisy geodesic sphere (4,704,000 half-edges,
    more than 1,024 scan tiles of 4,096: the compactions take their three-pass
    form) element by element against the oracle: candidates, reasons,
    placements and the collapsed mesh."""
    V, F = g.noisy_geodesic_sphere(280, 7)
    assert 3 * len(F) > 1024 * 4096
    Vd, Fd = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    target = len(F) // 100
    cand, _, n = ctx.select(Vd, Fd)
    vbar, reason, iters = ctx.check(Vd, Fd, target, cand, n)
    co, vo, ro, it_o = orc.check(V, F, target)
    assert np.array_equal(cand.cpu().numpy(), co)
    assert np.array_equal(reason.cpu().numpy(), ro)
    assert np.array_equal(vbar.cpu().numpy().view(np.uint64), vo.view(np.uint64))
    assert iters == it_o
    V1, F1, fl1 = ctx.collapse(Vd, Fd, cand, n, vbar, reason)
    r = orc.run(V, F, target, max_rounds=1)
    assert np.array_equal(F1.cpu().numpy(), r["F"])
    assert np.array_equal(V1.cpu().numpy().view(np.uint64), r["V"].view(np.uint64))
    assert np.array_equal(fl1.cpu().numpy(), r["flags"])


def test_whole_mesh_check_on_interpenetrating_spheres(ctx):
    """The whole-mesh exact check (the benchmark's pamo_self_intersections) on
    two noisy geodesic spheres of 124,820 faces each, the second shifted by 0.6
    of a radius so the two surfaces cross along a closed curve: the pair set
    equals the oracle's (grid-based, exact predicate) element by element, and
    each sphere alone reports none."""
    V1, F1 = g.noisy_geodesic_sphere(79, 3)
    V2, F2 = g.noisy_geodesic_sphere(79, 4)
    V2 = V2 + np.array([0.3, 0.0, 0.0])
    V = np.ascontiguousarray(np.concatenate([V1, V2]))
    F = np.ascontiguousarray(np.concatenate([F1, F2 + len(V1)]).astype(np.int32))
    want = orc.self_intersections(V, F, cap=1 << 20)
    assert len(want) > 1000
    pairs, n = ctx.self_intersections(torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda(), cap=1 << 20)
    assert n == len(want)
    got = pairs.cpu().numpy()
    key = lambda p: np.sort(np.minimum(p[:, 0], p[:, 1]).astype(np.int64) * (1 << 32) + np.maximum(p[:, 0], p[:, 1]))
    assert np.array_equal(key(got), key(np.asarray(want)))
    for Vs, Fs in ((V1, F1), (V2, F2)):
        _, n1 = ctx.self_intersections(torch.from_numpy(np.ascontiguousarray(Vs)).cuda(), torch.from_numpy(Fs).cuda())
        assert n1 == 0
