"""Thin Python binding of libpamo.so (include/pamo.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory and the current stream.  Importing this module
raises if the built library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpamo.so")

PAMO_OK = 0
PAMO_ERR_CAPACITY = -7
PAMO_TARGET_UNREACHED = 1
ERRORS = {-1: "ARG", -2: "NONMANIFOLD", -3: "SELF_INTERSECTING", -4: "DEGENERATE", -6: "HIP", -7: "CAPACITY"}

EXPORTS = ["pamo_default_options", "pamo_create", "pamo_destroy", "pamo_set_options", "pamo_last_error",
           "pamo_workspace_bytes", "pamo_set_workspace", "pamo_workspace_held", "pamo_quadrics", "pamo_select", "pamo_check", "pamo_collapse",
           "pamo_simplify", "pamo_simplify_noalloc", "pamo_simplify_batch", "pamo_set_mlp", "pamo_features", "pamo_mlp_logits",
           "pamo_collect", "pamo_mlp_grad", "pamo_mlp_train", "pamo_hausdorff", "pamo_self_intersections", "pamo_tri_pairs",
           "pamo_udf", "pamo_dualmc", "pamo_project_defaults", "pamo_sample_surface", "pamo_project_targets",
           "pamo_project_eval", "pamo_safe_project", "pamo_profile_enable",
           "pamo_profile_phases", "pamo_profile_name", "pamo_profile_read", "pamo_profile_reset"]


class Options(C.Structure):
    _fields_ = [("w_e", C.c_double), ("w_s", C.c_double), ("tolerance", C.c_int32),
                ("max_rounds", C.c_int32), ("validate_input", C.c_int32), ("query_packet", C.c_int32),
                ("resort_every", C.c_int32), ("query_coop", C.c_int32), ("coop_below", C.c_int32),
                ("learned", C.c_int32), ("cost_target", C.c_double), ("prefilter", C.c_int32),
                ("key_mode", C.c_int32), ("pair_capacity", C.c_int32)]


class ProjectOptions(C.Structure):
    _fields_ = [("k_dis", C.c_double), ("k_elas", C.c_double), ("k_bend", C.c_double), ("k_bar", C.c_double),
                ("dhat", C.c_double), ("cg_tol", C.c_double), ("accd_s", C.c_double), ("iterations", C.c_int32),
                ("refresh", C.c_int32), ("cg_max", C.c_int32), ("ls_max", C.c_int32)]


class ProjectStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("cg_iters", C.c_int32), ("halvings", C.c_int32), ("stalled", C.c_int32),
                ("max_pt", C.c_int64), ("max_ee", C.c_int64), ("B_first", C.c_double), ("B_last", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PROJECT_LOG = ("B", "alpha_ccd", "alpha", "halvings", "cg_iters", "n_pt", "n_ee", "grad_norm")


class Stats(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("faces_out", C.c_int64), ("verts_out", C.c_int64),
                ("candidates", C.c_int64), ("commits", C.c_int64), ("rej_link", C.c_int64),
                ("rej_flip", C.c_int64), ("rej_isect", C.c_int64), ("capped", C.c_int64),
                ("undo_hist", C.c_int64 * 5), ("deferred_pairs", C.c_int64), ("status", C.c_int64),
                ("demoted", C.c_int64), ("fallbacks", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "undo_hist"}
        d["undo_hist"] = list(self.undo_hist)
        return d


NFEAT = 32
NPARAM = 6337


class MLP(C.Structure):
    """pamo_mlp: the learned proposal's network (include/pamo.h)."""
    _fields_ = [("w1", (C.c_float * 32) * 64), ("b1", C.c_float * 64), ("w2", (C.c_float * 64) * 64),
                ("b2", C.c_float * 64), ("w3", C.c_float * 64), ("b3", C.c_float),
                ("e1", C.c_int32), ("e2", C.c_int32), ("e3", C.c_int32), ("a1", C.c_int32), ("a2", C.c_int32),
                ("threshold", C.c_float)]


def mlp_struct(model: dict) -> MLP:
    import numpy as np
    m = MLP()
    for k in ("w1", "b1", "w2", "b2", "w3"):
        a = np.ascontiguousarray(model[k], dtype=np.float32)
        C.memmove(C.addressof(getattr(m, k)), a.ctypes.data, a.nbytes)
    m.b3 = float(model["b3"])
    for k in ("e1", "e2", "e3", "a1", "a2"):
        setattr(m, k, int(model[k]))
    m.threshold = float(model["threshold"])
    return m


class PamoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pamo error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_2509_05595_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
        L.pamo_default_options.argtypes = [C.POINTER(Options)]
        L.pamo_default_options.restype = None
        L.pamo_create.argtypes = [C.POINTER(P), C.c_int, P, C.POINTER(Options)]
        L.pamo_destroy.argtypes = [P]
        L.pamo_destroy.restype = None
        L.pamo_set_options.argtypes = [P, C.POINTER(Options)]
        L.pamo_last_error.argtypes = [P]
        L.pamo_last_error.restype = C.c_char_p
        L.pamo_workspace_bytes.argtypes = [I64, I64, C.POINTER(Options)]
        L.pamo_workspace_bytes.restype = C.c_size_t
        L.pamo_set_workspace.argtypes = [P, P, C.c_size_t]
        L.pamo_workspace_held.argtypes = [P]
        L.pamo_workspace_held.restype = I64
        L.pamo_quadrics.argtypes = [P, P, I64, P, I64, P]
        L.pamo_select.argtypes = [P, P, I64, P, I64, P, P, P, P, P]
        L.pamo_check.argtypes = [P, P, I64, P, I64, P, I64, P, P, P, P, C.POINTER(I64)]
        L.pamo_collapse.argtypes = [P, P, C.POINTER(I64), P, C.POINTER(I64), P, P, P, P, P]
        L.pamo_simplify.argtypes = [P, P, I64, P, I64, I64, P, C.POINTER(I64), P, C.POINTER(I64),
                                    C.POINTER(Stats)]
        L.pamo_simplify_noalloc.argtypes = [P, P, I64, P, I64, I64, P, C.POINTER(I64), P, C.POINTER(I64),
                                            C.POINTER(Stats)]
        L.pamo_simplify_batch.argtypes = [P, I32, P, P, P, P, P, P, P, P, P, P]
        L.pamo_set_mlp.argtypes = [P, P]
        L.pamo_features.argtypes = [P, P, I64, P, I64, P, I64, P, P]
        L.pamo_mlp_logits.argtypes = [P, P, I64, P]
        L.pamo_collect.argtypes = [P, P, I64, P, I64, I64, P, P, I64, C.POINTER(I64), C.POINTER(Stats)]
        L.pamo_mlp_grad.argtypes = [P, P, P, P, P, I64, P, C.POINTER(C.c_float)]
        L.pamo_mlp_train.argtypes = [P, P, P, P, P, P, P, I64, P, I64, I64, C.c_float, I64, P]
        L.pamo_hausdorff.argtypes = [P, P, I64, P, I64, P, I64, P, C.POINTER(C.c_double)]
        L.pamo_self_intersections.argtypes = [P, P, I64, P, I64, P, I64, C.POINTER(I64)]
        L.pamo_udf.argtypes = [P, P, I64, P, I64, C.c_int32, C.c_double, P]
        L.pamo_dualmc.argtypes = [P, P, C.c_int32, C.c_double, C.c_double, P, I64, P, I64, C.POINTER(I64),
                                  C.POINTER(I64)]
        L.pamo_tri_pairs.argtypes = [P, P, P, P, P, I64, P]
        L.pamo_project_defaults.argtypes = [C.POINTER(ProjectOptions)]
        L.pamo_project_defaults.restype = None
        L.pamo_sample_surface.argtypes = [P, P, I64, P, I64, P, I64, P, C.POINTER(C.c_double)]
        L.pamo_project_targets.argtypes = [P, P, I64, P, I64, P, I64, P, I64, P, I64, P, P]
        L.pamo_project_eval.argtypes = [P, P, P, I64, P, I64, P, P, P, I64, C.c_double, C.POINTER(ProjectOptions),
                                        P, P, P, P, P, P, C.POINTER(I32), C.POINTER(C.c_double)]
        L.pamo_safe_project.argtypes = [P, P, I64, P, I64, P, I64, P, I64, P, I64, C.POINTER(ProjectOptions), P, P,
                                        C.POINTER(ProjectStats)]
        L.pamo_profile_enable.argtypes = [P, C.c_uint32]
        L.pamo_profile_phases.argtypes = []
        L.pamo_profile_name.argtypes = [I32]
        L.pamo_profile_name.restype = C.c_char_p
        L.pamo_profile_read.argtypes = [P, I32, C.POINTER(I64), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.pamo_profile_reset.argtypes = [P]
        for n in EXPORTS:
            if n not in ("pamo_default_options", "pamo_destroy", "pamo_last_error", "pamo_workspace_bytes",
                         "pamo_workspace_held", "pamo_profile_name", "pamo_project_defaults"):
                getattr(L, n).restype = I32
        _lib = L
    return _lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def default_options(**kw) -> Options:
    o = Options()
    lib().pamo_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def project_options(**kw) -> ProjectOptions:
    """pamo_project_options with the paper's defaults, fields overridden by kw"""
    o = ProjectOptions()
    lib().pamo_project_defaults(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def workspace_bytes(nv: int, nf: int, options: Options | None = None) -> int:
    """Device workspace that suffices for every mesh entry point on a mesh (or
    batch) of nv vertices and nf faces (pamo_workspace_bytes)."""
    opt = options if options is not None else default_options()
    return int(lib().pamo_workspace_bytes(int(nv), int(nf), C.byref(opt)))


class Context:
    """A library context bound to one device and the current torch stream.

    workspace="torch" (default): the library's device scratch is a torch uint8
    tensor the context allocates (pamo_set_workspace), sized by
    pamo_workspace_bytes before each mesh call and grown when a larger mesh
    comes; "library": the library allocates its own scratch."""

    def __init__(self, device=None, options: Options | None = None, stream=None, workspace: str = "torch"):
        if workspace not in ("torch", "library"):
            raise ValueError("workspace must be 'torch' or 'library'")
        dev = torch.device(device if device is not None else "cuda")
        self.device = torch.device("cuda", dev.index if dev.index is not None else torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        self._h = C.c_void_p()
        self._ws_mode = workspace
        self._ws = None
        opt = options if options is not None else default_options()
        self.options = Options.from_buffer_copy(opt)
        rc = lib().pamo_create(C.byref(self._h), self.device.index, C.c_void_p(s.cuda_stream), C.byref(opt))
        if rc != 0:
            raise PamoError(rc, "pamo_create failed")

    # ---- workspace
    def _set_workspace(self, nbytes):
        t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self._check(lib().pamo_set_workspace(self._h, _ptr(t), int(nbytes)))  # synchronises the stream
        self._ws = t

    def _ensure_workspace(self, nv, nf):
        """Before a mesh entry point: a torch workspace of at least the bytes
        pamo_workspace_bytes asks for this size."""
        if self._ws_mode != "torch":
            return
        need = int(lib().pamo_workspace_bytes(int(nv), int(nf), C.byref(self.options)))
        if need and (self._ws is None or self._ws.numel() < need):
            self._set_workspace(need)

    def _call_growing(self, fn, allow=(PAMO_OK,)):
        """Entry points that carve their workspace as they go (remeshing,
        training, utilities): a call that finds the torch workspace too small
        runs again with a larger one."""
        if self._ws_mode == "torch" and self._ws is None:
            self._set_workspace(64 << 20)
        for _ in range(12):
            rc = fn()
            if (rc == PAMO_ERR_CAPACITY and self._ws_mode == "torch"
                    and lib().pamo_last_error(self._h).decode().startswith("workspace of")):
                self._set_workspace(2 * self._ws.numel())
                continue
            break
        return self._check(rc, allow)

    def workspace_held(self) -> int:
        """Device bytes the library itself holds for this context (0 while it
        works in the torch workspace)."""
        return int(lib().pamo_workspace_held(self._h))

    def workspace_tensor(self):
        return self._ws

    def close(self):
        if self._h:
            lib().pamo_destroy(self._h)  # synchronises the stream first
            self._h = C.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(PAMO_OK,)):
        if rc not in allow:
            raise PamoError(rc, lib().pamo_last_error(self._h).decode())
        return rc

    def set_options(self, options: Options):
        self._check(lib().pamo_set_options(self._h, C.byref(options)))
        self.options = Options.from_buffer_copy(options)

    def _mesh(self, V, F):
        assert V.is_cuda and F.is_cuda and V.device == self.device and F.device == self.device
        assert V.dtype == torch.float64 and F.dtype == torch.int32
        assert V.is_contiguous() and F.is_contiguous() and V.shape[-1] == 3 and F.shape[-1] == 3
        return V, F

    def quadrics(self, V, F):
        V, F = self._mesh(V, F)
        self._ensure_workspace(V.shape[0], F.shape[0])
        Q = torch.empty((V.shape[0], 10), dtype=torch.float64, device=self.device)
        self._check(lib().pamo_quadrics(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(Q)))
        return Q

    def select(self, V, F, flags=None, demote=None):
        """Returns (cand int32 [ncand], keys uint64-as-int64 [3 nf])."""
        V, F = self._mesh(V, F)
        self._ensure_workspace(V.shape[0], F.shape[0])
        nh = 3 * F.shape[0]
        keys = torch.empty(nh, dtype=torch.int64, device=self.device)
        cand = torch.empty(nh, dtype=torch.int32, device=self.device)
        n = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._check(lib().pamo_select(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(flags),
                                      _ptr(demote), _ptr(keys), _ptr(cand), _ptr(n)))
        k = int(n.item())
        return cand[:k].clone(), keys, n

    def check(self, V, F, target, cand, ncand_dev, flags=None):
        """Returns (vbar [n,3], reason uint8 [n], undo iterations)."""
        V, F = self._mesh(V, F)
        self._ensure_workspace(V.shape[0], F.shape[0])
        n = max(1, cand.shape[0])
        vbar = torch.zeros((n, 3), dtype=torch.float64, device=self.device)
        reason = torch.zeros(n, dtype=torch.uint8, device=self.device)
        it = C.c_int64(0)
        self._call_growing(lambda: lib().pamo_check(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(flags), int(target),
                                     _ptr(cand), _ptr(ncand_dev), _ptr(vbar), _ptr(reason), C.byref(it)))
        k = cand.shape[0]
        return vbar[:k], reason[:k], it.value

    def collapse(self, V, F, cand, ncand_dev, vbar, reason, flags=None):
        """Commit reason-0 collapses; returns (V, F, flags) (new tensors)."""
        V, F = self._mesh(V, F)
        self._ensure_workspace(V.shape[0], F.shape[0])
        V = V.clone()
        F = F.clone()
        fl = flags.clone() if flags is not None else torch.zeros(3 * F.shape[0], dtype=torch.uint8,
                                                                   device=self.device)
        nv = C.c_int64(V.shape[0])
        nf = C.c_int64(F.shape[0])
        self._check(lib().pamo_collapse(self._h, _ptr(V), C.byref(nv), _ptr(F), C.byref(nf), _ptr(cand),
                                        _ptr(ncand_dev), _ptr(vbar), _ptr(reason), _ptr(fl)))
        return V[: nv.value].clone(), F[: nf.value].clone(), fl[: 3 * nf.value].clone()

    def simplify(self, V, F, target):
        """Returns (V_out, F_out, stats dict)."""
        V, F = self._mesh(V, F)
        self._ensure_workspace(V.shape[0], F.shape[0])
        Vo = torch.empty_like(V)
        Fo = torch.empty_like(F)
        nv, nf, st = C.c_int64(0), C.c_int64(0), Stats()
        self._call_growing(lambda: lib().pamo_simplify(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], int(target), _ptr(Vo),
                                        C.byref(nv), _ptr(Fo), C.byref(nf), C.byref(st)),
                    allow=(PAMO_OK, PAMO_TARGET_UNREACHED))
        return Vo[: nv.value], Fo[: nf.value], st.as_dict()

    def simplify_batch(self, meshes, targets):
        """Simplify a list of (V, F) device meshes together.

        Returns a list of (V_out, F_out, stats dict), one per mesh."""
        import numpy as np
        n = len(meshes)
        for V, F in meshes:
            self._mesh(V, F)
        V = torch.cat([m[0] for m in meshes]).contiguous()
        F = torch.cat([m[1] for m in meshes]).contiguous()
        self._ensure_workspace(V.shape[0], F.shape[0])
        v_off = np.zeros(n + 1, dtype=np.int64)
        f_off = np.zeros(n + 1, dtype=np.int64)
        v_off[1:] = np.cumsum([m[0].shape[0] for m in meshes])
        f_off[1:] = np.cumsum([m[1].shape[0] for m in meshes])
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        assert tg.shape == (n,)
        Vo = torch.empty_like(V)
        Fo = torch.empty_like(F)
        vo = np.zeros(n + 1, dtype=np.int64)
        fo = np.zeros(n + 1, dtype=np.int64)
        st = (Stats * max(n, 1))()
        h = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
        self._call_growing(lambda: lib().pamo_simplify_batch(self._h, n, _ptr(V), h(v_off), _ptr(F), h(f_off), h(tg), _ptr(Vo),
                                              h(vo), _ptr(Fo), h(fo), st),
                    allow=(PAMO_OK, PAMO_TARGET_UNREACHED))
        return [(Vo[vo[m]:vo[m + 1]], Fo[fo[m]:fo[m + 1]], st[m].as_dict()) for m in range(n)]

    # ---- learned proposal
    def set_mlp(self, model):
        """model: dict (w1, b1, w2, b2, w3, b3, e1, e2, e3, a1, a2, threshold) or None."""
        if model is None:
            self._check(lib().pamo_set_mlp(self._h, None))
            return
        m = mlp_struct(model)
        self._check(lib().pamo_set_mlp(self._h, C.byref(m)))

    def features(self, V, F, edges):
        """(features float32 [n, 32], overlap counts int32 [nf]) of the given half-edges."""
        V, F = self._mesh(V, F)
        self._ensure_workspace(V.shape[0], F.shape[0])
        e = edges.to(self.device, torch.int32).contiguous()
        X = torch.zeros((max(1, e.shape[0]), NFEAT), dtype=torch.float32, device=self.device)
        ovl = torch.zeros(F.shape[0], dtype=torch.int32, device=self.device)
        self._call_growing(lambda: lib().pamo_features(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(e), e.shape[0],
                                        _ptr(X), _ptr(ovl)))
        return X[: e.shape[0]], ovl

    def mlp_logits(self, X):
        X = X.to(self.device, torch.float32).contiguous()
        out = torch.empty(max(1, X.shape[0]), dtype=torch.float32, device=self.device)
        self._call_growing(lambda: lib().pamo_mlp_logits(self._h, _ptr(X), X.shape[0], _ptr(out)))
        return out[: X.shape[0]]

    def collect(self, V, F, target, cap):
        """Plain run logging training rows: (X [n, 32], y [n], stats)."""
        V, F = self._mesh(V, F)
        self._ensure_workspace(V.shape[0], F.shape[0])
        X = torch.empty((max(1, cap), NFEAT), dtype=torch.float32, device=self.device)
        y = torch.empty(max(1, cap), dtype=torch.uint8, device=self.device)
        n, st = C.c_int64(0), Stats()
        self._call_growing(lambda: lib().pamo_collect(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], int(target), _ptr(X),
                                       _ptr(y), int(cap), C.byref(n), C.byref(st)),
                    allow=(PAMO_OK, PAMO_TARGET_UNREACHED))
        return X[: n.value], y[: n.value], st.as_dict()

    def mlp_grad(self, params, meta, X, y):
        import numpy as np
        md = np.ascontiguousarray(meta, dtype=np.int32)
        g = torch.empty(NPARAM, dtype=torch.float32, device=self.device)
        loss = C.c_float(0)
        self._call_growing(lambda: lib().pamo_mlp_grad(self._h, _ptr(params), md.ctypes.data_as(C.c_void_p), _ptr(X),
                                                       _ptr(y), X.shape[0], _ptr(g), C.byref(loss)))
        return g, loss.value

    def mlp_train(self, params, m, v, meta, X, y, order, steps, batch, lr, t0):
        """Adam steps in place on params (and moments m, v); returns per-step losses."""
        import numpy as np
        md = np.ascontiguousarray(meta, dtype=np.int32)
        loss = torch.empty(max(1, steps), dtype=torch.float32, device=self.device)
        self._call_growing(lambda: lib().pamo_mlp_train(self._h, _ptr(params), _ptr(m), _ptr(v),
                                                        md.ctypes.data_as(C.c_void_p), _ptr(X), _ptr(y),
                                                        int(X.shape[0]), _ptr(order), int(steps), int(batch),
                                                        float(lr), int(t0), _ptr(loss)))
        return loss[:steps]

    def hausdorff(self, P, V, F, per_point=False):
        """Largest distance from the points P to the surface (V, F) (and each point's)."""
        V, F = self._mesh(V, F)
        P = P.contiguous()
        d = torch.empty(max(1, P.shape[0]), dtype=torch.float64, device=self.device) if per_point else None
        dm = C.c_double(0)
        self._call_growing(lambda: lib().pamo_hausdorff(self._h, _ptr(P), P.shape[0], _ptr(V), V.shape[0], _ptr(F),
                                                        F.shape[0], _ptr(d), C.byref(dm)))
        return (dm.value, d[: P.shape[0]]) if per_point else dm.value

    def self_intersections(self, V, F, cap=1 << 16):
        V, F = self._mesh(V, F)
        self._ensure_workspace(V.shape[0], F.shape[0])
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=self.device)
        n = C.c_int64(0)
        self._call_growing(lambda: lib().pamo_self_intersections(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(pairs),
                                                  cap, C.byref(n)))
        return pairs[: min(cap, n.value)], n.value

    def udf(self, V, F, res, band=None):
        """Narrow-band unsigned distance field (res, res, res) float64 at the voxel
        centres of [0,1]^3 (+inf beyond the band, default 3 / res)."""
        V, F = self._mesh(V, F)
        band = 3.0 / res if band is None else float(band)
        out = torch.empty((res, res, res), dtype=torch.float64, device=self.device)
        self._call_growing(lambda: lib().pamo_udf(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], int(res), band,
                                                  _ptr(out)))
        return out

    def dualmc(self, S, iso=0.0, vcap=None, fcap=None, beta=0.0):
        """Dual Marching Cubes of the (res, res, res) float64 grid S at level iso
        -> (V (nv, 3) float64, F (nf, 3) int32) on the device; beta > 0 smooths
        the crossing fractions (the paper uses 5)."""
        assert S.dtype == torch.float64 and S.is_contiguous() and S.dim() == 3
        res = S.shape[0]
        nv, nf = C.c_int64(0), C.c_int64(0)
        if vcap is None or fcap is None:  # sizes first: a call with no room writes only them
            self._call_growing(lambda: lib().pamo_dualmc(self._h, _ptr(S), int(res), float(iso), float(beta), None, 0,
                                                         None, 0, C.byref(nv), C.byref(nf)),
                               allow=(PAMO_OK, PAMO_ERR_CAPACITY))
            vcap = nv.value if vcap is None else int(vcap)
            fcap = nf.value if fcap is None else int(fcap)
        V = torch.empty((max(vcap, 1), 3), dtype=torch.float64, device=self.device)
        F = torch.empty((max(fcap, 1), 3), dtype=torch.int32, device=self.device)
        self._call_growing(lambda: lib().pamo_dualmc(self._h, _ptr(S), int(res), float(iso), float(beta), _ptr(V), vcap,
                                                     _ptr(F), fcap, C.byref(nv), C.byref(nf)))
        return V[:nv.value], F[:nf.value]

    # ---- safe projection
    def sample_surface(self, V, F, U):
        """samples on (V, F) from uniforms U (m, 3) -> (Y (m, 3), total area)"""
        V, F = self._mesh(V, F)
        assert U.dtype == torch.float64 and U.is_contiguous() and U.device == self.device
        Y = torch.empty((U.shape[0], 3), dtype=torch.float64, device=self.device)
        area = C.c_double(0.0)
        self._call_growing(lambda: lib().pamo_sample_surface(self._h, _ptr(V), V.shape[0], _ptr(F), F.shape[0],
                                                             _ptr(U), U.shape[0], _ptr(Y), C.byref(area)))
        return Y, area.value

    def project_targets(self, X, F, Vin, Fin, Y):
        """closest input-mesh point per vertex, closest triangle of (X, F) per sample"""
        X, F = self._mesh(X, F)
        Vin, Fin = self._mesh(Vin, Fin)
        targets = torch.empty_like(X)
        tri = torch.empty((Y.shape[0],), dtype=torch.int32, device=self.device)
        self._call_growing(lambda: lib().pamo_project_targets(
            self._h, _ptr(X), X.shape[0], _ptr(F), F.shape[0], _ptr(Vin), Vin.shape[0], _ptr(Fin), Fin.shape[0],
            _ptr(Y), Y.shape[0], _ptr(targets), _ptr(tri)))
        return targets, tri

    def project_eval(self, X0, X, F, targets, Y, tri, area_in, options=None, grad=False, v=None, direction=False,
                     step=False):
        """the pieces of one iteration at X: dict with parts (s2m, m2s, elastic,
        bend, barrier, B), contacts (pt, ee) and, when asked, grad, Hv,
        direction, cg_iters, step"""
        X, F = self._mesh(X, F)
        opt = options if options is not None else project_options()
        parts = (C.c_double * 6)()
        cont = (C.c_int64 * 2)()
        g = torch.empty_like(X) if grad else None
        Hv = torch.empty_like(X) if v is not None else None
        d = torch.empty_like(X) if (direction or step) else None
        it = C.c_int32(0)
        st = C.c_double(0.0)
        self._call_growing(lambda: lib().pamo_project_eval(
            self._h, _ptr(X0), _ptr(X), X.shape[0], _ptr(F), F.shape[0], _ptr(targets), _ptr(Y), _ptr(tri),
            Y.shape[0], float(area_in), C.byref(opt), parts, cont, _ptr(g), _ptr(v), _ptr(Hv), _ptr(d),
            C.byref(it), C.byref(st) if step else None))
        out = {"parts": list(parts), "contacts": (cont[0], cont[1])}
        if grad:
            out["grad"] = g
        if Hv is not None:
            out["Hv"] = Hv
        if d is not None:
            out["direction"] = d
            out["cg_iters"] = it.value
        if step:
            out["step"] = st.value
        return out

    def safe_project(self, Vs, Fs, Vin, Fin, Y, options=None, out=None):
        """Alg. 2: -> (V_out, per-iteration log (iterations, 8) float64 on the
        host, stats dict)"""
        import numpy as np
        Vs, Fs = self._mesh(Vs, Fs)
        Vin, Fin = self._mesh(Vin, Fin)
        opt = options if options is not None else project_options()
        V_out = out if out is not None else torch.empty_like(Vs)
        log = np.zeros((max(opt.iterations, 1), 8))
        st = ProjectStats()
        self._call_growing(lambda: lib().pamo_safe_project(
            self._h, _ptr(Vs), Vs.shape[0], _ptr(Fs), Fs.shape[0], _ptr(Vin), Vin.shape[0], _ptr(Fin), Fin.shape[0],
            _ptr(Y), Y.shape[0], C.byref(opt), _ptr(V_out), C.c_void_p(log.ctypes.data), C.byref(st)))
        return V_out, log[:opt.iterations], st.as_dict()

    # ---- measurement
    @staticmethod
    def phase_names():
        L = lib()
        return [L.pamo_profile_name(i).decode() for i in range(L.pamo_profile_phases())]

    def profile(self, phases=None):
        """Enable HIP-event timing for the named phases (None: all, []: off)."""
        names = self.phase_names()
        if phases is None:
            mask = (1 << len(names)) - 1
        else:
            mask = 0
            for p in phases:
                mask |= 1 << names.index(p)
        self._check(lib().pamo_profile_enable(self._h, mask))
        self._check(lib().pamo_profile_reset(self._h))

    def profile_read(self):
        """{phase: (launches, ms, algorithmic bytes)} for phases with launches."""
        out = {}
        for i, n in enumerate(self.phase_names()):
            k, ms, b = C.c_int64(0), C.c_double(0), C.c_double(0)
            self._check(lib().pamo_profile_read(self._h, i, C.byref(k), C.byref(ms), C.byref(b)))
            if k.value:
                out[n] = (k.value, ms.value, b.value)
        return out

    def tri_pairs(self, P, ip, Q, iq):
        n = P.shape[0]
        out = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._call_growing(lambda: lib().pamo_tri_pairs(self._h, _ptr(P), _ptr(ip), _ptr(Q), _ptr(iq), n, _ptr(out)))
        return out
