"""GPU parity of the safe projection (Sec. 6, Alg. 2, App. 2.2) against the
oracle (oracle/project.py), through the C-ABI.

Both sides compute in float64 from the same definitions but by different
formulas and summation orders (hyper-dual numbers against automatic
differentiation, Jacobi against LAPACK eigen-decompositions, atomic against
sequential sums), so values agree to rounding: relative 1e-10 on energies
and gradients (sums of a few thousand terms of relative error ~1e-15), 1e-9
on Hessian products, and the CG directions within the solver tolerance (on
ill-conditioned contact systems the iteration at which the residual crosses
the tolerance may move by one or two).  Discrete decisions (closest
triangles, contact sets, line-search halvings) must match exactly.  Whole
runs of a few iterations then agree to 1e-8 in positions.
"""
import numpy as np
import pytest

import oracle.oracle as orc
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


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def gpu_opts(o):
    from paper_2509_05595_amd import native
    return native.project_options(k_dis=o.k_dis, k_elas=o.k_elas, k_bend=o.k_bend, k_bar=o.k_bar, dhat=o.dhat,
                                  cg_tol=o.cg_tol, accd_s=o.accd_s, iterations=o.iterations, refresh=o.refresh,
                                  cg_max=o.cg_max, ls_max=o.ls_max)


def simplified_case(k=3, frac=5, m=512):
    Vin, Fin = g.noisy_icosphere(k, 2)
    r = orc.run(Vin, Fin, len(Fin) // frac)
    U = np.random.default_rng(0).random((m, 3))
    return r["V"], r["F"].astype(np.int32), Vin, Fin.astype(np.int32), U


def contact_case(k_s=1, k_in=2, gap=0.0016, m=256):
    """two shells closer than dhat and one input sphere between them: every
    energy term, contacts included, is active.  The shells carry a little
    radial noise: exactly scaled copies would start with exactly parallel
    edges, where the edge-edge distance has no unique gradient."""
    Vin, Fin = g.icosphere(k_in)
    Vin = g.normalize_unit_cube(Vin)
    Vs, Fs = g.nested_spheres(k=k_s, gap=gap, sigma=1e-4)
    U = np.random.default_rng(4).random((m, 3))
    return Vs, Fs.astype(np.int32), Vin, Fin.astype(np.int32), U


def test_samples(ctx):
    _, _, Vin, Fin, U = simplified_case(m=4096)
    Y, area = ctx.sample_surface(dev(Vin), dev(Fin, torch.int32), dev(U))
    Yo, _ = op.sample_surface(Vin, Fin.astype(np.int64), U)
    assert area == pytest.approx(op.face_areas(Vin, Fin).sum(), rel=1e-13)
    assert np.abs(Y.cpu().numpy() - Yo).max() < 1e-14


@pytest.mark.parametrize("case", ["simplified", "contact"])
def test_targets(ctx, case):
    Vs, Fs, Vin, Fin, U = simplified_case() if case == "simplified" else contact_case()
    X = Vs + 2e-3 * np.random.default_rng(1).standard_normal(Vs.shape)
    pb = op.make_problem(Vs, Fs, Vin, Fin, U)
    op.refresh_targets(pb, X, Vin, Fin)
    Y = dev(pb.Y)
    tg, tri = ctx.project_targets(dev(X), dev(Fs, torch.int32), dev(Vin), dev(Fin, torch.int32), Y)
    assert np.array_equal(tri.cpu().numpy(), pb.tri)
    assert np.abs(tg.cpu().numpy() - pb.targets).max() < 1e-13


def _eval_pair(ctx, Vs, Fs, Vin, Fin, U, X, opt):
    pb = op.make_problem(Vs, Fs, Vin, Fin, U, opt)
    op.refresh_targets(pb, X, Vin, Fin)
    args = (dev(Vs), dev(X), dev(Fs, torch.int32), dev(pb.targets), dev(pb.Y), dev(pb.tri, torch.int32),
            pb.area_in)
    return pb, args


@pytest.mark.parametrize("case", ["simplified", "contact"])
def test_energy_gradient_hessian(ctx, case):
    Vs, Fs, Vin, Fin, U = simplified_case() if case == "simplified" else contact_case()
    rng = np.random.default_rng(2)
    X = Vs + (1e-4 if case == "contact" else 2e-3) * rng.standard_normal(Vs.shape)
    opt = op.Options()
    pb, args = _eval_pair(ctx, Vs, Fs, Vin, Fin, U, X, opt)
    v = rng.standard_normal(X.shape)
    out = ctx.project_eval(*args, options=gpu_opts(opt), grad=True, v=dev(v))
    parts = op.energy_parts(pb, X)
    if case == "contact":
        assert parts["n_pt"] > 0 and parts["n_ee"] > 0
    assert out["contacts"] == (parts["n_pt"], parts["n_ee"])
    for k, name in enumerate(("s2m", "m2s", "elastic", "bend", "barrier")):
        assert out["parts"][k] == pytest.approx(parts[name], rel=1e-10, abs=1e-300), name
    assert out["parts"][5] == pytest.approx(op.total(pb, parts), rel=1e-10)
    gr, H = op.assemble(len(X), op.elements(pb, X))
    got = out["grad"].cpu().numpy().ravel()
    assert np.abs(got - gr).max() <= 1e-10 * np.abs(gr).max()
    Hv = out["Hv"].cpu().numpy().ravel()
    want = H @ v.ravel()
    assert np.abs(Hv - want).max() <= 1e-9 * np.abs(want).max()


@pytest.mark.parametrize("case", ["simplified", "contact"])
def test_direction_and_ccd_step(ctx, case):
    Vs, Fs, Vin, Fin, U = simplified_case() if case == "simplified" else contact_case()
    X = Vs + (1e-4 if case == "contact" else 2e-3) * np.random.default_rng(3).standard_normal(Vs.shape)
    opt = op.Options(cg_tol=1e-10)
    pb, args = _eval_pair(ctx, Vs, Fs, Vin, Fin, U, X, opt)
    out = ctx.project_eval(*args, options=gpu_opts(opt), direction=True, step=True)
    gr, H, P, it = op.newton_direction(pb, X)
    d = out["direction"].cpu().numpy()
    # on the ill-conditioned contact system rounding moves the step at which
    # the residual crosses the tolerance by an iteration or so
    assert abs(out["cg_iters"] - it) <= max(2, it // 50)
    assert np.linalg.norm(H @ d.ravel() + gr) <= 2 * opt.cg_tol * np.linalg.norm(gr)
    assert np.linalg.norm(d - P) <= 1e-6 * np.linalg.norm(P)
    # the CCD bound of the GPU's own direction, by the oracle
    assert out["step"] == pytest.approx(op.accd(pb, X, d), rel=1e-9)


@pytest.mark.parametrize("case,iters,refresh", [("simplified", 6, 3), ("contact", 4, 2)])
def test_run_matches_oracle(ctx, case, iters, refresh):
    Vs, Fs, Vin, Fin, U = simplified_case() if case == "simplified" else contact_case()
    opt = op.Options(iterations=iters, refresh=refresh, cg_tol=1e-10)
    Xo, pb = op.safe_project(Vs, Fs, Vin, Fin, U, opt)
    Y, _ = ctx.sample_surface(dev(Vin), dev(Fin, torch.int32), dev(U))
    V, log, st = ctx.safe_project(dev(Vs), dev(Fs, torch.int32), dev(Vin), dev(Fin, torch.int32), Y,
                                  options=gpu_opts(opt))
    assert st["iterations"] == iters
    for t, rec in enumerate(pb.log):
        assert log[t, 0] == pytest.approx(rec["B"], rel=1e-8), t
        assert int(log[t, 3]) == rec["halvings"], t
        assert abs(int(log[t, 4]) - rec["cg_iters"]) <= max(2, rec["cg_iters"] // 50), t
        assert log[t, 1] == pytest.approx(rec["alpha_ccd"], rel=1e-6), t
    assert np.abs(V.cpu().numpy() - Xo).max() < 1e-8
    assert len(orc.self_intersections(V.cpu().numpy(), Fs)) == 0


def test_bad_mesh_and_arguments(ctx):
    from paper_2509_05595_amd import native
    Vs, Fs, Vin, Fin, U = contact_case()
    Y, _ = ctx.sample_surface(dev(Vin), dev(Fin, torch.int32), dev(U))
    with pytest.raises(native.PamoError) as e:  # an open mesh: one face removed
        ctx.safe_project(dev(Vs), dev(Fs[1:], torch.int32), dev(Vin), dev(Fin, torch.int32), Y)
    assert e.value.code == -2
    with pytest.raises(native.PamoError) as e:
        ctx.safe_project(dev(Vs), dev(Fs, torch.int32), dev(Vin), dev(Fin, torch.int32), Y,
                         options=native.project_options(dhat=-1.0))
    assert e.value.code == -1


def test_whole_pipeline_matches_oracle_chain(ctx):
    """The three stages of Sec. 3 on the GPU (distance field and surface
    extraction, simplification, safe projection back towards the input)
    against the same chain in the oracle: the extraction and the
    simplification agree as their own tests require (faces equal, vertices to
    rounding), and the projection, started from meshes that differ by
    rounding, ends within 1e-8, free of self-intersections and with a lower
    distance energy."""
    from oracle import dualmc as dm
    from oracle import udf as ou
    V, F = g.bumpy_icosphere_gauss(k=3, seed=2)
    V = 0.5 + (V - 0.5) * 0.7
    F = F.astype(np.int32)
    R = 24
    Ug = ctx.udf(dev(V), dev(F, torch.int32), R)
    Ve, Fe = ctx.dualmc(Ug, 0.9 / R)
    Vo, Fo = dm.dualmc(ou.udf(V, F, R, 3.0 / R) - 0.9 / R)
    assert np.array_equal(Fe.cpu().numpy(), Fo)
    target = len(Fo) // 10
    Vs, Fs, _ = ctx.simplify(Ve.contiguous(), Fe.contiguous(), target)
    r = orc.run(Vo, Fo, target)
    assert np.array_equal(Fs.cpu().numpy(), r["F"])
    U = np.random.default_rng(3).random((512, 3))
    opt = op.Options(iterations=6, refresh=3, cg_tol=1e-10)
    Xo, pb = op.safe_project(r["V"], r["F"].astype(np.int64), V, F.astype(np.int64), U, opt)
    Y, _ = ctx.sample_surface(dev(V), dev(F, torch.int32), dev(U))
    X, log, _ = ctx.safe_project(Vs.contiguous(), Fs.contiguous(), dev(V), dev(F, torch.int32), Y,
                                 options=gpu_opts(opt))
    Xg = X.cpu().numpy()
    assert np.abs(Xg - Xo).max() < 1e-8
    assert len(orc.self_intersections(Xg, Fs.cpu().numpy())) == 0
    dis = []
    for Z in (r["V"], Xo):
        op.refresh_targets(pb, Z, V, F.astype(np.int64))
        p = op.energy_parts(pb, Z)
        dis.append(p["s2m"] + p["m2s"])
    assert dis[1] < dis[0]
