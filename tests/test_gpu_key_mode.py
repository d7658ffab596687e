"""GPU parity of the float64 key mode (pamo_options.key_mode = 1: edges ordered
by the float64 cost, then the edge id): selections, whole runs alone and in a
batch equal the oracle's bit for bit; the learned proposal and the logging
entry points refuse the mode."""
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


def options(**kw):
    from paper_2509_05595_amd import native
    return native.default_options(key_mode=1, **kw)


# a noise-free icosphere (float32 codes tie costs that float64 tells apart),
# a bumpy sphere, a thin shell (undo loop), pure-QEM weights on a creased
# sphere (flip rejections), a torus
CASES = [("regular", lambda: g.bumpy_icosphere_gauss(k=3, seed=3, sigma=0.0), 100, None),
         ("bumpy_k4", lambda: g.bumpy_icosphere_gauss(k=4, seed=4), 51, None),
         ("thin_shell", lambda: g.nested_spheres(k=3, gap=0.01), 51, None),
         ("crease_pure_qem", lambda: g.crease_sphere(3, 5), 16, (0.0, 0.0)),
         ("torus", lambda: g.bumpy_torus(32, 16, seed=4), 20, None)]


@pytest.mark.parametrize("name,make,target,w", CASES)
def test_key_mode_run_matches_oracle(ctx, name, make, target, w):
    from paper_2509_05595_amd import native
    V, F = make()
    kw = {} if w is None else {"w_e": w[0], "w_s": w[1]}
    want = orc.run(V, F, target, key_mode=1, **kw)
    ctx.set_options(options(**kw))
    try:
        Vo, Fo, st = ctx.simplify(*dev(V, F), target)
        cand, _, _ = ctx.select(*dev(V, F))
    finally:
        ctx.set_options(native.default_options())
    assert np.array_equal(Fo.cpu().numpy(), want["F"])
    assert np.array_equal(Vo.cpu().numpy().view(np.uint64), want["V"].view(np.uint64))
    for k in KEYS:
        assert st[k] == want["stats"][k], (k, st[k], want["stats"][k])
    assert np.array_equal(np.sort(cand.cpu().numpy()), np.sort(orc.check(V, F, 0, key_mode=1, **kw)[0]))


def test_key_mode_in_a_batch_matches_oracle(ctx):
    from paper_2509_05595_amd import native
    meshes = [g.bumpy_icosphere_gauss(k=3, seed=3, sigma=0.0), g.nested_spheres(k=3, gap=0.01),
              g.bumpy_torus(32, 16, seed=4), g.bumpy_icosphere_gauss(k=4, seed=4)]
    targets = [100, 51, 20, 51]
    ctx.set_options(options())
    try:
        out = ctx.simplify_batch([dev(V, F) for V, F in meshes], targets)
    finally:
        ctx.set_options(native.default_options())
    for (V, F), t, (Vo, Fo, st) in zip(meshes, targets, out):
        want = orc.run(V, F, t, key_mode=1)
        assert np.array_equal(Fo.cpu().numpy(), want["F"])
        assert np.array_equal(Vo.cpu().numpy().view(np.uint64), want["V"].view(np.uint64))
        for k in KEYS:
            assert st[k] == want["stats"][k], (k, st[k], want["stats"][k])


def test_learned_and_logging_refuse_the_float64_key(ctx):
    from paper_2509_05595_amd import native
    V, F = g.bumpy_icosphere_gauss(k=2, seed=8)
    Vd, Fd = dev(V, F)
    ctx.set_options(options())
    try:
        with pytest.raises(native.PamoError) as e:
            ctx.collect(Vd, Fd, 64, 1024)
        assert e.value.code == -1
        with pytest.raises(native.PamoError) as e:
            ctx.features(Vd, Fd, torch.arange(6, dtype=torch.int32))
        assert e.value.code == -1
        from paper_2509_05595_amd import learn
        ctx.set_mlp(learn.load_model())  # a network is set: the refusal is for the key mode
        ctx.set_options(options(learned=1))
        with pytest.raises(native.PamoError) as e:
            ctx.simplify(Vd, Fd, 64)
        assert e.value.code == -1 and "key_mode" in str(e.value)
    finally:
        ctx.set_mlp(None)
        ctx.set_options(native.default_options())
