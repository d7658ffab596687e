"""GPU parity of the link/flip pre-filter (pamo_options.prefilter: the local
checks run on every keyed edge before the selection): the library and the
oracle end with the same mesh bit for bit and the same statistics, alone and
in a batch."""
import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("rounds", "candidates", "commits", "rej_link", "rej_flip", "rej_isect", "capped", "status")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_05595_amd import native
    c = native.Context("cuda:0")
    yield c
    c.close()


def dev(V, F):
    return (torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(F, dtype=np.int32)).cuda())


# (name, mesh, target, Eq. 1 weights): pure-QEM weights on a creased sphere
# flip triangles; the noisy sphere rejects a few collapses for flips; the thin
# shell undoes collapses for intersections; every edge of the seven-vertex
# torus fails the link condition
CASES = [("crease_pure_qem", lambda: g.crease_sphere(3, 5), 16, (0.0, 0.0)),
         ("noisy_k4", lambda: g.bumpy_icosphere_gauss(k=4, seed=4), 51, None),
         ("thin_shell", lambda: g.nested_spheres(k=3, gap=0.01), 51, None),
         ("crease_k5", lambda: g.crease_sphere(5, 5), 20, None),
         ("csaszar", g.csaszar_torus, 2, None),
         # flat sides under pure-QEM weights (exactly collinear triangles
         # for the exact degeneracy test); poles of valence 24
         ("grid_cube_pure_qem", lambda: g.grid_cube(4), 12, (0.0, 0.0)),
         ("bipyramid_24", lambda: g.bipyramid(24), 8, None)]


def run_both(ctx, V, F, target, w):
    from paper_2509_05595_amd import native
    kw = {} if w is None else {"w_e": w[0], "w_s": w[1]}
    want = orc.run(V, F, target, prefilter=1, **kw)
    ctx.set_options(native.default_options(prefilter=1, **kw))
    try:
        got = ctx.simplify(*dev(V, F), target)
    finally:
        ctx.set_options(native.default_options())
    return got, want


@pytest.mark.parametrize("name,make,target,w", CASES)
def test_prefilter_matches_oracle(ctx, name, make, target, w):
    V, F = make()
    (Vo, Fo, st), want = run_both(ctx, V, F, target, w)
    assert np.array_equal(Fo.cpu().numpy(), want["F"])
    assert np.array_equal(Vo.cpu().numpy().view(np.uint64), want["V"].view(np.uint64))
    for k in KEYS:
        assert st[k] == want["stats"][k], (k, st[k], want["stats"][k])
    assert st["rej_link"] == 0 and st["rej_flip"] == 0


def test_prefilter_in_a_batch_matches_oracle(ctx):
    from paper_2509_05595_amd import native
    meshes = [g.bumpy_icosphere_gauss(k=4, seed=4), g.nested_spheres(k=3, gap=0.01), g.csaszar_torus(),
              g.bumpy_torus(32, 16, seed=4)]
    targets = [51, 51, 2, 10]
    ctx.set_options(native.default_options(prefilter=1))
    try:
        out = ctx.simplify_batch([dev(V, F) for V, F in meshes], targets)
    finally:
        ctx.set_options(native.default_options())
    for (V, F), t, (Vo, Fo, st) in zip(meshes, targets, out):
        want = orc.run(V, F, t, prefilter=1)
        assert np.array_equal(Fo.cpu().numpy(), want["F"])
        assert np.array_equal(Vo.cpu().numpy().view(np.uint64), want["V"].view(np.uint64))
        for k in KEYS:
            assert st[k] == want["stats"][k], (k, st[k], want["stats"][k])
