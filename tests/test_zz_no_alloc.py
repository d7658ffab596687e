"""pamo_simplify_noalloc against pamo_simplify, through the C ABI (GPU).

The no-allocation entry point runs the method in the library's static
per-device scratch.  Two calls in a row, the second on a smaller mesh, must
each equal pamo_simplify on the same input bit for bit (faces, vertex bits,
statistics); the context's own workspace is left as it was; a mesh too large
for the scratch is refused before any work.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2509_05595_amd import meshgen as g

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def native():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_05595_amd import native as n
    return n


def run(native, ctx, entry, V, F, target):
    L = native.lib()
    Vd = torch.from_numpy(np.ascontiguousarray(V)).cuda()
    Fd = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    Vo, Fo = torch.empty_like(Vd), torch.empty_like(Fd)
    nv, nf, st = C.c_int64(0), C.c_int64(0), native.Stats()
    fn = getattr(L, entry)
    rc = fn(ctx, C.c_void_p(Vd.data_ptr()), len(V), C.c_void_p(Fd.data_ptr()), len(F), int(target),
            C.c_void_p(Vo.data_ptr()), C.byref(nv), C.c_void_p(Fo.data_ptr()), C.byref(nf), C.byref(st))
    msg = L.pamo_last_error(ctx).decode()
    torch.cuda.synchronize()
    return rc, msg, Vo[: nv.value].cpu().numpy(), Fo[: nf.value].cpu().numpy(), st.as_dict()


def test_noalloc_equals_simplify_twice_then_smaller(native):
    L = native.lib()
    h = C.c_void_p()
    opt = native.default_options()
    assert L.pamo_create(C.byref(h), 0, C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(opt)) == 0
    try:
        cases = [(g.bumpy_icosphere_gauss(k=5, seed=3), 400),  # 20,480 faces
                 (g.nested_spheres(k=3, gap=0.004), 128),       # 2,560 faces, undone collapses
                 (g.bumpy_icosphere_gauss(k=3, seed=8), 64)]    # 1,280 faces
        for (V, F), target in cases:
            held = L.pamo_workspace_held(h)
            rc1, m1, V1, F1, s1 = run(native, h, "pamo_simplify_noalloc", V, F, target)
            assert L.pamo_workspace_held(h) == held  # the context's own workspace is untouched
            rc0, m0, V0, F0, s0 = run(native, h, "pamo_simplify", V, F, target)
            assert rc1 == rc0 and rc0 in (0, 1), (m1, m0)
            assert np.array_equal(F1, F0)
            assert np.array_equal(V1.view(np.uint64), V0.view(np.uint64))
            assert s1 == s0
        # a mesh too large for the scratch is refused before any work
        V, F = g.noisy_icosphere(7, 2)  # 327,680 faces
        rc, msg, _, _, _ = run(native, h, "pamo_simplify_noalloc", V, F, len(F) // 100)
        print(msg)
        assert rc == native.PAMO_ERR_CAPACITY and "static scratch" in msg
        # ... and the context still works afterwards, both ways
        (V, F), target = cases[2]
        rc1, _, V1, F1, _ = run(native, h, "pamo_simplify_noalloc", V, F, target)
        rc0, _, V0, F0, _ = run(native, h, "pamo_simplify", V, F, target)
        assert rc1 == rc0 == 0 and np.array_equal(F1, F0) and np.array_equal(V1.view(np.uint64), V0.view(np.uint64))
    finally:
        L.pamo_destroy(h)
