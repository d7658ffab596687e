"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Connectivity and integer results are compared bit-exactly; vertex positions
too (the tolerance the method allows is 1e-9 relative; both sides evaluate
the same float64 operation sequence, so the expected difference is zero and
the test asserts the looser bound only as a diagnostic).
"""
import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_05595_amd import native
    c = native.Context("cuda:0")
    yield c
    c.close()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    return t.cpu().numpy()


def meshes():
    return {
        "ico2": g.bumpy_icosphere_gauss(k=2, seed=1),
        "small5120": g.bumpy_icosphere_gauss(),
        "torus": g.bumpy_torus(24, 10, seed=5),
        "nested": g.nested_spheres(k=3, gap=0.01),
        "crease": g.crease_sphere(3, 5),
        # flat sides: with pure-QEM weights many collapses make exactly
        # collinear triangles, which only the exact degeneracy test decides
        "cube4": g.grid_cube(4),
        # two poles of valence 24: stars beyond the stored slots
        "bipyr": g.bipyramid(24),
    }


MESHES = meshes()


@pytest.mark.parametrize("name", list(MESHES))
def test_quadrics_bitwise(ctx, name):
    V, F = MESHES[name]
    Q = host(ctx.quadrics(dev(V, torch.float64), dev(F, torch.int32)))
    Qo = orc.quadrics(V, F)
    assert np.array_equal(Q.view(np.uint64), Qo.view(np.uint64)), np.abs(Q - Qo).max()


@pytest.mark.parametrize("name", list(MESHES))
def test_keys_and_selection(ctx, name):
    V, F = MESHES[name]
    cand, keys, _ = ctx.select(dev(V, torch.float64), dev(F, torch.int32))
    ko = orc.keys(V, F)
    rep = ko != np.uint64(2 ** 64 - 1)
    kg = host(keys).view(np.uint64)
    assert np.array_equal(kg[rep], ko[rep])
    assert np.array_equal(np.sort(host(cand)), orc.select(V, F))


@pytest.mark.parametrize("name,target,we,ws", [("small5120", 512, 0.001, 0.005), ("nested", 128, 0.001, 0.005),
                                                 ("crease", 16, 0.0, 0.0), ("ico2", 33, 0.001, 0.005)])
def test_check_round(ctx, name, target, we, ws):
    from paper_2509_05595_amd import native
    V, F = MESHES[name]
    ctx.set_options(native.default_options(w_e=we, w_s=ws))
    try:
        Vd, Fd = dev(V, torch.float64), dev(F, torch.int32)
        cand, _, n = ctx.select(Vd, Fd)
        vbar, reason, iters = ctx.check(Vd, Fd, target, cand, n)
        co, vo, ro, it_o = orc.check(V, F, target, w_e=we, w_s=ws)
        assert np.array_equal(host(cand), co)
        assert np.array_equal(host(reason), ro)
        ok = ro != 1
        assert np.array_equal(host(vbar)[ok].view(np.uint64), vo[ok].view(np.uint64))
        assert iters == it_o
        # one committed round equals the oracle's round
        V1, F1, fl1 = ctx.collapse(Vd, Fd, cand, n, vbar, reason)
        r = orc.run(V, F, target, max_rounds=1, w_e=we, w_s=ws)
        assert np.array_equal(host(F1), r["F"])
        assert np.array_equal(host(V1).view(np.uint64), r["V"].view(np.uint64))
        assert np.array_equal(host(fl1), r["flags"])
    finally:
        ctx.set_options(native.default_options())


@pytest.mark.parametrize("name,target,we,ws", [
    ("ico2", 32, 0.001, 0.005), ("ico2", 101, 0.001, 0.005), ("small5120", 512, 0.001, 0.005),
    ("torus", 48, 0.001, 0.005), ("nested", 128, 0.001, 0.005), ("crease", 16, 0.0, 0.0),
    ("cube4", 12, 0.0, 0.0), ("bipyr", 8, 0.001, 0.005)])
def test_simplify_bitwise(ctx, name, target, we, ws):
    from paper_2509_05595_amd import native
    V, F = MESHES[name]
    ctx.set_options(native.default_options(w_e=we, w_s=ws))
    try:
        Vo, Fo, st = ctx.simplify(dev(V, torch.float64), dev(F, torch.int32), target)
    finally:
        ctx.set_options(native.default_options())
    r = orc.run(V, F, target, w_e=we, w_s=ws)
    Fg, Vg = host(Fo), host(Vo)
    assert st["status"] == r["stats"]["status"]
    assert st["rounds"] == r["stats"]["rounds"]
    assert np.array_equal(Fg, r["F"])
    rel = np.abs(Vg - r["V"]).max() / max(1e-300, np.abs(r["V"]).max())
    assert rel <= 1e-9
    assert np.array_equal(Vg.view(np.uint64), r["V"].view(np.uint64))
    for k in ("commits", "rej_link", "rej_flip", "rej_isect", "capped"):
        assert st[k] == r["stats"][k], k
    assert st["undo_hist"] == r["stats"]["undo_hist"]


@pytest.mark.parametrize("target", [0, 1, 5, 318, 319, 320, 321, 10 ** 9])
def test_targets_at_the_ends(ctx, target):
    # 320 faces: down to a tetrahedron (the target unreachable below 4 faces),
    # odd targets (T - T mod 2), one collapse, none, a target above the count
    V, F = MESHES["ico2"]
    Vo, Fo, st = ctx.simplify(dev(V, torch.float64), dev(F, torch.int32), target)
    r = orc.run(V, F, target)
    assert np.array_equal(host(Fo), r["F"])
    assert np.array_equal(host(Vo).view(np.uint64), r["V"].view(np.uint64))
    assert st["status"] == r["stats"]["status"] and st["rounds"] == r["stats"]["rounds"]
    if target >= len(F):
        assert st["rounds"] == 0 and np.array_equal(host(Fo), F)


def test_batch_targets_at_the_ends(ctx):
    V, F = MESHES["ico2"]
    targets = [0, 319, 320, 10 ** 9, 5]
    out = ctx.simplify_batch([(dev(V, torch.float64), dev(F, torch.int32))] * len(targets), targets)
    for t, (Vo, Fo, st) in zip(targets, out):
        r = orc.run(V, F, t)
        assert np.array_equal(host(Fo), r["F"])
        assert np.array_equal(host(Vo).view(np.uint64), r["V"].view(np.uint64))
        assert st["status"] == r["stats"]["status"] and st["rounds"] == r["stats"]["rounds"]


def test_tri_pairs_match_oracle(ctx):
    from test_oracle_predicates import _random_pair
    rng = np.random.default_rng(77)
    P, IP, Q, IQ, want = [], [], [], [], []
    for kind in ["random", "coplanar", "sharp", "vertex", "edge", "coplanar_vertex", "coplanar_edge"]:
        for _ in range(400):
            p, ip, q, iq = _random_pair(rng, kind)
            P.append(p.ravel()); IP.append(ip); Q.append(q.ravel()); IQ.append(iq)
            want.append(orc.tri_pair(p, ip, q, iq))
    # float triangles whose corners lie on the other's plane up to rounding
    while len(want) < 4800:
        p = rng.random((3, 3))
        st = rng.random((3, 2))
        q = p[0] + st[:, :1] * (p[1] - p[0]) + st[:, 1:] * (p[2] - p[0])
        q[rng.integers(0, 3)] += rng.choice([-1, 0, 1], size=3) * np.spacing(q[0])
        if orc.degenerate(q):
            continue
        ids = rng.permutation(6)
        P.append(p.ravel()); IP.append(ids[:3]); Q.append(q.ravel()); IQ.append(ids[3:])
        want.append(orc.tri_pair(p, ids[:3], q, ids[3:]))
    out = host(ctx.tri_pairs(dev(np.array(P), torch.float64), dev(np.array(IP), torch.int32),
                             dev(np.array(Q), torch.float64), dev(np.array(IQ), torch.int32)))
    assert np.array_equal(out.astype(bool), np.array(want))


def test_self_intersections_match_oracle(ctx):
    V, F = g.nested_spheres(k=4, gap=0.005)  # the inner sphere pokes through
    want = orc.self_intersections(V, F)
    pairs, n = ctx.self_intersections(dev(V, torch.float64), dev(F, torch.int32), cap=1 << 16)
    got = host(pairs)
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    want = want[np.lexsort((want[:, 1], want[:, 0]))]
    assert n == len(want) and n > 0
    assert np.array_equal(got, want)
    V, F = MESHES["small5120"]
    _, n = ctx.self_intersections(dev(V, torch.float64), dev(F, torch.int32))
    assert n == 0


def test_invalid_inputs(ctx):
    from paper_2509_05595_amd import native
    V, F = MESHES["ico2"]
    Fo = F[:-1]  # an open mesh
    with pytest.raises(native.PamoError) as e:
        ctx.simplify(dev(V, torch.float64), dev(Fo, torch.int32), 10)
    assert e.value.code == -2
    Fb = F.copy()
    Fb[0, 0] = len(V) + 5
    with pytest.raises(native.PamoError) as e:
        ctx.simplify(dev(V, torch.float64), dev(Fb, torch.int32), 10)
    assert e.value.code == -1
    Fd = F.copy()
    Fd[0, 1] = Fd[0, 0]
    with pytest.raises(native.PamoError):
        ctx.simplify(dev(V, torch.float64), dev(Fd, torch.int32), 10)
    # link condition everywhere fails: the seven-vertex torus stays as it is
    V7, F7 = g.csaszar_torus()
    Vo, Fo7, st = ctx.simplify(dev(V7, torch.float64), dev(F7, torch.int32), 2)
    assert st["status"] == 1 and Fo7.shape[0] == 14
