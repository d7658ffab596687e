"""The caller's workspace and the pair-buffer regrowth (GPU, through the C ABI).

* A run in a torch-owned workspace (pamo_set_workspace, sized by
  pamo_workspace_bytes) equals a run in the library's own workspace bit for
  bit, and the context holds no device scratch of its own meanwhile.
* A workspace that is too small fails with PAMO_ERR_CAPACITY, naming the
  buffer, and leaves the context usable.
* A tiny first capacity of the candidate-pair buffer forces every query pass
  of a heavy-undo run to overflow, grow the buffer and run again; the result
  still equals the oracle's (F, V bits, rejections, undo iterations).
"""
import ctypes as C

import numpy as np
import pytest

import oracle.oracle as orc
from paper_2509_05595_amd import meshgen as g

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def native():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_05595_amd import native as n
    return n


def dev(V, F):
    return (torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(F, dtype=np.int32)).cuda())


def bits(t):
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.float64 else a


def test_torch_workspace_equals_library_workspace(native):
    V, F = g.bumpy_icosphere_gauss(k=5, seed=3)  # 20,480 faces
    Vd, Fd = dev(V, F)
    a = native.Context("cuda:0", workspace="torch")
    b = native.Context("cuda:0", workspace="library")
    try:
        ra = a.simplify(Vd, Fd, 200)
        rb = b.simplify(Vd, Fd, 200)
        assert np.array_equal(bits(ra[0]), bits(rb[0])) and np.array_equal(bits(ra[1]), bits(rb[1]))
        assert ra[2] == rb[2]
        assert a.workspace_held() == 0 and b.workspace_held() > 0
        assert a.workspace_tensor().numel() == native.workspace_bytes(len(V), len(F))
        # a smaller mesh in the same (larger) workspace, then the larger again
        V2, F2 = g.bumpy_icosphere_gauss(k=3, seed=4)
        r2 = a.simplify(*dev(V2, F2), 100)
        o2 = orc.run(V2, F2, 100)
        assert np.array_equal(bits(r2[1]), o2["F"]) and np.array_equal(bits(r2[0]), o2["V"].view(np.uint64))
        ra2 = a.simplify(Vd, Fd, 200)
        assert np.array_equal(bits(ra2[1]), bits(ra[1]))
        assert a.workspace_held() == 0
    finally:
        a.close()
        b.close()


def test_torch_workspace_batch_and_check(native):
    meshes = [g.bumpy_icosphere_gauss(k=3, seed=s) for s in (1, 2)] + [g.bumpy_torus(24, 10, seed=5)]
    dm = [dev(V, F) for V, F in meshes]
    targets = [len(F) // 10 for _, F in meshes]
    a = native.Context("cuda:0", workspace="torch")
    b = native.Context("cuda:0", workspace="library")
    try:
        ra = a.simplify_batch(dm, targets)
        rb = b.simplify_batch(dm, targets)
        for x, y in zip(ra, rb):
            assert np.array_equal(bits(x[0]), bits(y[0])) and np.array_equal(bits(x[1]), bits(y[1]))
        V, F = g.nested_spheres(k=3, gap=0.01)
        Vd, Fd = dev(V, F)
        cand, _, n = a.select(Vd, Fd)
        vbar, reason, it = a.check(Vd, Fd, 128, cand, n)
        co, vo, ro, ito = orc.check(V, F, 128)
        assert np.array_equal(bits(cand), co) and np.array_equal(bits(reason), ro) and it == ito
        assert a.workspace_held() == 0
    finally:
        a.close()
        b.close()


def test_workspace_too_small_fails_cleanly(native):
    V, F = g.bumpy_icosphere_gauss(k=3, seed=1)
    Vd, Fd = dev(V, F)
    c = native.Context("cuda:0", workspace="library")
    try:
        L = native.lib()
        small = torch.empty(1 << 16, dtype=torch.uint8, device="cuda:0")
        assert L.pamo_set_workspace(c._h, C.c_void_p(small.data_ptr()), small.numel()) == 0
        Vo, Fo = torch.empty_like(Vd), torch.empty_like(Fd)
        nv, nf, st = C.c_int64(0), C.c_int64(0), native.Stats()
        rc = L.pamo_simplify(c._h, C.c_void_p(Vd.data_ptr()), len(V), C.c_void_p(Fd.data_ptr()), len(F), 100,
                             C.c_void_p(Vo.data_ptr()), C.byref(nv), C.c_void_p(Fo.data_ptr()), C.byref(nf),
                             C.byref(st))
        assert rc == native.PAMO_ERR_CAPACITY
        assert L.pamo_last_error(c._h).decode().startswith("workspace of")
        # misaligned workspace is refused
        assert L.pamo_set_workspace(c._h, C.c_void_p(small.data_ptr() + 8), 4096) == -1
        # enough workspace: the same call succeeds and equals the oracle
        need = native.workspace_bytes(len(V), len(F))
        big = torch.empty(need, dtype=torch.uint8, device="cuda:0")
        assert L.pamo_set_workspace(c._h, C.c_void_p(big.data_ptr()), need) == 0
        rc = L.pamo_simplify(c._h, C.c_void_p(Vd.data_ptr()), len(V), C.c_void_p(Fd.data_ptr()), len(F), 100,
                             C.c_void_p(Vo.data_ptr()), C.byref(nv), C.c_void_p(Fo.data_ptr()), C.byref(nf),
                             C.byref(st))
        assert rc == 0
        o = orc.run(V, F, 100)
        assert np.array_equal(bits(Fo[: nf.value]), o["F"])
        assert L.pamo_set_workspace(c._h, None, 0) == 0  # back to the library's own
        del small, big
    finally:
        c.close()


@pytest.mark.parametrize("workspace", ["library", "torch"])
def test_pair_buffer_regrowth_matches_oracle(native, workspace):
    """pair_capacity 64: every query pass of this nested-sphere run collects
    more candidate pairs than that, so it grows the buffer and repeats."""
    V, F = g.nested_spheres(k=4, gap=0.004)  # 10,240 faces, many undone collapses
    target = len(F) // 20
    c = native.Context("cuda:0", options=native.default_options(pair_capacity=64), workspace=workspace)
    try:
        Vo, Fo, st = c.simplify(*dev(V, F), target)
    finally:
        c.close()
    o = orc.run(V, F, target)
    assert o["stats"]["rej_isect"] > 0 and sum(o["stats"]["undo_hist"][1:]) > 0
    assert np.array_equal(bits(Fo), o["F"]) and np.array_equal(bits(Vo), o["V"].view(np.uint64))
    for k in ("rounds", "commits", "rej_link", "rej_flip", "rej_isect", "capped", "status"):
        assert st[k] == o["stats"][k], k
    assert st["undo_hist"] == o["stats"]["undo_hist"]

