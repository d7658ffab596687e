"""The safe projection at the benchmark's size, as bench.py runs it: the
1,310,720-face noisy icosphere simplified to 1% on the GPU (13,106 faces),
then projected back towards the input with 16,384 samples and the paper's
settings (T = 50, targets every 10 iterations).  The oracle cannot run the
whole projection at this size in seconds, so parity is checked on what it can
compute: every sample, the closest-feature targets of sampled vertices and
samples (exact brute force over the faces that can hold them), and the
energy terms and the gradient at the projected positions with those targets.
Properties that hold at any size cover the rest: B never increases between
two refreshes, the result is free of self-intersections, and the distance
energy went down.
"""
import numpy as np
import pytest

import oracle.project as op
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


def _closest_checked(P, V, F, bound2):
    """the oracle's closest triangles of points P, brute force over the faces
    whose boxes lie within the squared distance bound2[i] (an upper bound of
    the smallest distance: no face outside can be closer or tie)"""
    lo = np.minimum(np.minimum(V[F[:, 0]], V[F[:, 1]]), V[F[:, 2]])
    hi = np.maximum(np.maximum(V[F[:, 0]], V[F[:, 1]]), V[F[:, 2]])
    out_f, out_p = [], []
    for i, p in enumerate(P):
        d = np.maximum(np.maximum(lo - p, p - hi), 0.0)
        near = np.nonzero(np.sum(d * d, axis=1) <= bound2[i] * (1 + 1e-6) + 1e-20)[0]
        f, _, q = op.closest_faces(p[None], V, F[near])
        out_f.append(near[f[0]])
        out_p.append(q[0])
    return np.array(out_f), np.array(out_p)


def test_projection_at_benchmark_size(ctx):
    V, F = g.noisy_icosphere(8, 2)
    Vd = torch.from_numpy(V).cuda()
    Fd = torch.from_numpy(F).cuda()
    Vs, Fs, _ = ctx.simplify(Vd, Fd, len(F) // 100)
    Vs, Fs = Vs.contiguous(), Fs.contiguous()
    U = np.random.default_rng(7).random((16384, 3))
    Y, area = ctx.sample_surface(Vd, Fd, torch.from_numpy(U).cuda())
    Yo, _ = op.sample_surface(V, F.astype(np.int64), U)
    Yh = Y.cpu().numpy()
    assert np.abs(Yh - Yo).max() < 1e-14
    assert area == pytest.approx(op.face_areas(V, F).sum(), rel=1e-12)

    from paper_2509_05595_amd import native
    opt = native.project_options()
    X, log, st = ctx.safe_project(Vs, Fs, Vd, Fd, Y, options=opt)
    assert st["iterations"] == 50
    B = log[:, 0]
    for t in range(1, 50):
        if t % opt.refresh:
            assert B[t] <= B[t - 1], t
    _, npairs = ctx.self_intersections(X, Fs)
    assert npairs == 0

    # targets at the result, sampled, against the oracle's brute force
    tg, tri = ctx.project_targets(X, Fs, Vd, Fd, Y)
    Xh, Fh = X.cpu().numpy(), Fs.cpu().numpy().astype(np.int64)
    tgh, trih = tg.cpu().numpy(), tri.cpu().numpy()
    rng = np.random.default_rng(1)
    iv = rng.choice(len(Xh), 24, replace=False)
    _, q = _closest_checked(Xh[iv], V, F.astype(np.int64), np.sum((Xh[iv] - tgh[iv]) ** 2, axis=1))
    assert np.abs(q - tgh[iv]).max() < 1e-13
    isamp = rng.choice(len(Yh), 64, replace=False)
    Tg = Xh[Fh[trih[isamp]]]
    bound = op.pt_d2(Yh[isamp], Tg[:, 0], Tg[:, 1], Tg[:, 2])
    f, _ = _closest_checked(Yh[isamp], Xh, Fh, bound)
    assert np.array_equal(f, trih[isamp])

    # the energy terms and the gradient at the result with those targets
    out = ctx.project_eval(Vs, X, Fs, tg, Y, tri, area, options=opt, grad=True)
    pb = op.make_problem(Vs.cpu().numpy(), Fh, V, F.astype(np.int64), U)
    pb.Y, pb.targets, pb.tri = Yh, tgh, trih.astype(np.int64)
    parts = op.energy_parts(pb, Xh)
    assert out["contacts"] == (parts["n_pt"], parts["n_ee"])
    for k, name in enumerate(("s2m", "m2s", "elastic", "bend", "barrier")):
        assert out["parts"][k] == pytest.approx(parts[name], rel=1e-10, abs=1e-300), name
    gr, _ = op.assemble(len(Xh), op.elements(pb, Xh))
    assert np.abs(out["grad"].cpu().numpy().ravel() - gr).max() <= 1e-10 * np.abs(gr).max()

    # the distance energy (targets found afresh) went down
    tg0, tri0 = ctx.project_targets(Vs, Fs, Vd, Fd, Y)
    p0 = ctx.project_eval(Vs, Vs, Fs, tg0, Y, tri0, area, options=opt)["parts"]
    assert out["parts"][0] + out["parts"][1] < p0[0] + p0[1]
