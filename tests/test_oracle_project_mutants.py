"""The safe-projection oracle's pins catch plausible mistakes (no GPU).

Each case plants one mistake in the oracle (a patched function, restored
afterwards) and checks that the named pin of tests/test_oracle_project.py
fails; the unpatched oracle passes the same pins (that file's own run)."""
import math

import numpy as np
import pytest
import torch

import oracle.project as op
import test_oracle_project as pins


def _barrier_of_d2(d, dhat):
    """the barrier taken of the squared distance"""
    if isinstance(d, torch.Tensor):
        return torch.where(d < dhat, -(d * d - dhat) ** 2 * torch.log(d * d / dhat), torch.zeros_like(d))
    return -(d * d - dhat) ** 2 * math.log(d * d / dhat) if d < dhat else 0.0


def _barycentric_areas(V, F):
    """a third of each face's area per corner instead of the Voronoi areas"""
    s = np.zeros(len(V))
    A = op.face_areas(V, F)
    for f in range(len(F)):
        for v in F[f]:
            s[v] += A[f] / 3
    return s


def _elastic_half(z, Binv, A0):
    return 0.5 * op._ORIG["_elastic"](z, Binv, A0)


def _bend_no_rest(z, theta0, l0):
    x = z.reshape(4, 3)
    th = op.dihedral(x[0], x[1], x[2], x[3])
    return 0.5 * l0 * th ** 2


def _samples_linear(V, F, U):
    """u1 used directly instead of its square root: not uniform on the triangle"""
    cum = np.cumsum(op.face_areas(V, F))
    f = np.minimum(np.searchsorted(cum, U[:, 0] * cum[-1], side="right"), len(F) - 1)
    r = U[:, 1]
    w = np.stack([1.0 - r, r * (1.0 - U[:, 2]), r * U[:, 2]], axis=1)
    return np.einsum("mk,mkd->md", w, V[F[f]]), f


def _accd_no_shrink(x, p, kind, s, t_max):
    """stops at the impact itself: ignores the fraction s of the distance kept"""
    return op._ORIG["accd_pairs"](x, p, kind, 1e-12, t_max)


def _pcg_one_step(H, b, tol, max_iter):
    return op._ORIG["pcg"](H, b, tol, 1)


def _dihedral_unsigned(xi, xj, xk, xl):
    e = xj - xi
    n1 = op._cross(e, xk - xi)
    n2 = op._cross(xi - xj, xl - xj)
    c = (n1 * n2).sum() / torch.sqrt((n1 * n1).sum() * (n2 * n2).sum())
    return torch.arccos(torch.clamp(c, -1.0, 1.0))


MUTANTS = [
    ("barrier of d^2", "barrier", _barrier_of_d2, [pins.test_barrier_values]),
    ("barycentric vertex areas", "voronoi_areas", _barycentric_areas, [pins.test_voronoi_areas_by_polygons]),
    ("membrane energy halved", "_elastic", _elastic_half, [pins.test_elastic_rigid_scaling_shear]),
    ("bending without the rest angle", "_bend", _bend_no_rest,
     [lambda: pins.test_bending_hinge(0.4, 1.1)]),
    ("unsigned dihedral angle", "dihedral", _dihedral_unsigned, [lambda: pins.test_bending_hinge(-0.2, 0.25)]),
    ("non-uniform samples", "sample_surface", _samples_linear, [pins.test_samples_uniform_mean]),
    ("CCD without the kept fraction", "accd_pairs", _accd_no_shrink, [pins.test_accd_point_falls_on_triangle]),
    ("CG stopped after one step", "pcg", _pcg_one_step, [pins.test_pcg_against_direct_solve]),
]


@pytest.mark.parametrize("name,attr,fn,tests", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, attr, fn, tests, monkeypatch):
    monkeypatch.setattr(op, "_ORIG", {k: getattr(op, k) for k in ("_elastic", "accd_pairs", "pcg")}, raising=False)
    monkeypatch.setattr(op, attr, fn)
    for t in tests:
        with pytest.raises(AssertionError):
            t()
