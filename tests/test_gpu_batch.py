"""GPU parity of the batched form (pamo_simplify_batch).

Every mesh of a batch must come out exactly as pamo_simplify makes it alone,
and therefore exactly as the CPU oracle makes it: connectivity and vertex bits,
rounds, status and the per-round statistics.
"""
import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STAT_KEYS = ("rounds", "faces_out", "verts_out", "candidates", "commits", "rej_link", "rej_flip", "rej_isect",
             "capped", "undo_hist", "status")


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


def same(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64)) if a.dtype == np.float64 else np.array_equal(a, b)


def check_against_single(ctx, meshes, targets, oracle=True):
    dm = [dev(V, F) for V, F in meshes]
    out = ctx.simplify_batch(dm, targets)
    assert len(out) == len(meshes)
    for i, ((V, F), (Vd, Fd), t, (Vb, Fb, sb)) in enumerate(zip(meshes, dm, targets, out)):
        Vs, Fs, ss = ctx.simplify(Vd, Fd, t)
        Vb, Fb, Vs, Fs = (x.cpu().numpy() for x in (Vb, Fb, Vs, Fs))
        assert same(Fb, Fs), f"mesh {i}: faces differ from the single-mesh run"
        assert same(Vb, Vs), f"mesh {i}: vertices differ from the single-mesh run"
        for k in STAT_KEYS:
            assert sb[k] == ss[k], (i, k, sb[k], ss[k])
        if oracle:
            r = orc.run(V, F, t)
            assert same(Fb, r["F"]) and same(Vb, r["V"]), f"mesh {i}: differs from the oracle"
            assert sb["rounds"] == r["stats"]["rounds"] and sb["status"] == r["stats"]["status"]
            assert sb["undo_hist"] == r["stats"]["undo_hist"]
    return out


def test_batch_mixed_meshes(ctx):
    """Different kinds and targets, one already at its target, one that cannot
    reach it (a tetrahedron: every collapse breaks the link condition)."""
    meshes = [g.bumpy_icosphere_gauss(k=2, seed=1), g.bumpy_icosphere_gauss(), g.bumpy_torus(24, 10, seed=5),
              g.nested_spheres(k=3, gap=0.01), g.tetrahedron(), g.bumpy_icosphere_gauss(k=2, seed=7),
              g.octahedron()]
    targets = [32, 512, 48, 128, 0, 10_000, 4]
    out = check_against_single(ctx, meshes, targets)
    assert out[4][2]["status"] == 1 and out[4][2]["rounds"] == 4  # unreachable: tolerance rounds
    assert out[5][2]["rounds"] == 0 and out[5][1].shape[0] == 320  # at its target from the start


def test_batch_uneven_sizes(ctx):
    """Spheres and tori of log-uniform face counts, each to 1% (the batched
    workload's recipe at small sizes)."""
    specs = g.batch_specs(count=16, seed=11, fmin=300, fmax=6000)
    meshes = [g.make_spec(s) for s in specs]
    targets = [len(F) // 100 for _, F in meshes]
    check_against_single(ctx, meshes, targets)


def test_batch_of_one_and_repeat(ctx):
    V, F = g.bumpy_icosphere_gauss()
    a = check_against_single(ctx, [(V, F)], [512], oracle=False)
    b = check_against_single(ctx, [(V, F)] * 3, [512, 300, 1000], oracle=False)
    assert same(a[0][1].cpu().numpy(), b[0][1].cpu().numpy())


def test_batch_meshes_share_space(ctx):
    """Copies of one mesh scaled beyond the unit cube overlap the cells the BVH
    gives other meshes; pairs across meshes must still never be tested."""
    V, F = g.bumpy_icosphere_gauss(k=3, seed=3)
    Vb = V * 5.0 - 2.0
    check_against_single(ctx, [(Vb, F), (Vb.copy(), F), (Vb + 0.25, F)], [64, 128, 64], oracle=False)


def test_batch_max_rounds_and_weights(ctx):
    from paper_2509_05595_amd import native
    meshes = [g.crease_sphere(3, 5), g.bumpy_icosphere_gauss(k=3, seed=2)]
    for opt in (native.default_options(max_rounds=3), native.default_options(w_e=0.0, w_s=0.0)):
        ctx.set_options(opt)
        try:
            dm = [dev(V, F) for V, F in meshes]
            out = ctx.simplify_batch(dm, [16, 40])
            for (Vd, Fd), t, (Vb, Fb, sb) in zip(dm, [16, 40], out):
                Vs, Fs, ss = ctx.simplify(Vd, Fd, t)
                assert same(Fb.cpu().numpy(), Fs.cpu().numpy()) and same(Vb.cpu().numpy(), Vs.cpu().numpy())
                assert sb["rounds"] == ss["rounds"]
        finally:
            ctx.set_options(native.default_options())


def test_batch_invalid_inputs(ctx):
    import ctypes as C
    from paper_2509_05595_amd import native
    V, F = g.bumpy_icosphere_gauss(k=2, seed=1)
    good = dev(V, F)
    # a local vertex id beyond its own mesh (valid only as a global id)
    Fbad = F.copy()
    Fbad[0, 0] = len(V)
    with pytest.raises(native.PamoError) as e:
        ctx.simplify_batch([good, dev(V, Fbad)], [32, 32])
    assert e.value.code == -1
    # an open mesh in the batch
    with pytest.raises(native.PamoError) as e:
        ctx.simplify_batch([good, dev(V, F[:-2])], [32, 32])
    assert e.value.code == -2
    # bad offsets / counts through the raw ABI
    L = native.lib()
    z = np.zeros(2, dtype=np.int64)
    h = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    st = (native.Stats * 1)()
    p = C.c_void_p(good[0].data_ptr())
    Vo, Fo = torch.empty_like(good[0]), torch.empty_like(good[1])
    for nm, voff, foff in ((0, z, z), (1, np.array([0, 2]), np.array([0, 320])), (1, np.array([1, 162]), np.array([0, 320]))):
        voff = np.ascontiguousarray(voff, dtype=np.int64)
        foff = np.ascontiguousarray(foff, dtype=np.int64)
        rc = L.pamo_simplify_batch(ctx._h, nm, p, h(voff), C.c_void_p(good[1].data_ptr()), h(foff),
                                   h(np.zeros(1, dtype=np.int64)), C.c_void_p(Vo.data_ptr()), h(z.copy()),
                                   C.c_void_p(Fo.data_ptr()), h(z.copy()), st)
        assert rc == -1
    # the context still works afterwards
    check_against_single(ctx, [(V, F)], [32], oracle=False)
