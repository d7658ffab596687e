"""ctypes binding of the C oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain serial C implementation of one round of the method
(Sec. 5 of the paper) and of the whole round loop.  ``build()`` compiles it
with gcc; float contraction is off so the float64 arithmetic is exactly the
sequence the source spells out.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = ["oracle_exact.c", "oracle_tri.c", "oracle_mesh.c"]
LIB_PATH = os.environ.get("PAMO_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

W_E = 0.001  # Eq. 1 default weights (Sec. 5.1)
W_S = 0.005
TOLERANCE = 4  # Sec. 5.3


SOURCES = tuple(_SRC)


def build(force: bool = True, src_dir: str = _HERE, out: str = None) -> str:
    """Compile liboracle.so with gcc (no GPU involved).  src_dir / out: build
    the sources of another directory into another file (the mutation tests
    build planted variants this way)."""
    out = out or LIB_PATH
    if not force and os.path.exists(out):
        return out
    srcs = [os.path.join(src_dir, s) for s in _SRC]
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class Opts(C.Structure):
    _fields_ = [("w_e", C.c_double), ("w_s", C.c_double), ("tolerance", C.c_int32),
                ("max_rounds", C.c_int32), ("cost_target", C.c_double), ("prefilter", C.c_int32),
                ("key_mode", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("commits", C.c_int64), ("candidates", C.c_int64),
                ("rej_link", C.c_int64), ("rej_flip", C.c_int64), ("rej_isect", C.c_int64),
                ("capped", C.c_int64), ("undo_hist", C.c_int64 * 5), ("status", C.c_int64)]


NFEAT = 32  # features per edge (11 used, the rest zero)


class MLP(C.Structure):
    """The learned proposal's network: 32 -> 64 -> 64 -> 1 (see oracle_mesh.c)."""
    _fields_ = [("w1", (C.c_float * 32) * 64), ("b1", C.c_float * 64),
                ("w2", (C.c_float * 64) * 64), ("b2", C.c_float * 64),
                ("w3", C.c_float * 64), ("b3", C.c_float),
                ("e1", C.c_int32), ("e2", C.c_int32), ("e3", C.c_int32),
                ("a1", C.c_int32), ("a2", C.c_int32), ("threshold", C.c_float)]


def mlp_struct(model: dict) -> MLP:
    """model: w1 (64,32), b1 (64), w2 (64,64), b2 (64), w3 (64), b3, a1, a2, threshold."""
    m = MLP()
    for k in ("w1", "b1", "w2", "b2", "w3"):
        a = np.ascontiguousarray(model[k], dtype=np.float32)
        C.memmove(C.addressof(getattr(m, k)), a.ctypes.data, a.nbytes)
    m.b3 = float(model["b3"])
    m.e1, m.e2, m.e3 = (int(model[k]) for k in ("e1", "e2", "e3"))
    m.a1 = int(model["a1"])
    m.a2 = int(model["a2"])
    m.threshold = float(model["threshold"])
    return m


class RoundLog(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "faces", "verts", "edges", "candidates", "passing", "chosen", "changed_faces",
        "undo_iters", "commits", "rej_link", "rej_flip", "rej_isect", "capped")]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        I64 = C.c_int64
        L.oracle_quadrics.argtypes = [P, I64, P, I64, P]
        L.oracle_keys.argtypes = [P, I64, P, I64, P, C.c_double, C.c_double, P]
        L.oracle_select.argtypes = [P, I64, P, I64, P, C.c_double, C.c_double, P, P]
        L.oracle_check.argtypes = [P, I64, P, I64, P, C.c_double, C.c_double, I64, C.c_int32, C.c_int32, P, P, P, P, P]
        L.oracle_run.argtypes = [P, I64, P, I64, P, C.c_int32, I64, P, P, P, P, P, P, P, P, P, I64]
        L.oracle_tri_pair.argtypes = [P, P, P, P]
        L.oracle_degenerate.argtypes = [P]
        L.oracle_self_intersections.argtypes = [P, I64, P, I64, P, I64, P]
        L.oracle_validate.argtypes = [P, I64, P, I64]
        for n in ("oracle_orient2d", "oracle_orient2d_exact"):
            getattr(L, n).argtypes = [P, P, P]
        for n in ("oracle_orient3d", "oracle_orient3d_exact"):
            getattr(L, n).argtypes = [P, P, P, P]
        L.oracle_skinny.argtypes = [P]
        L.oracle_skinny.restype = C.c_double
        L.oracle_make_key.argtypes = [C.c_double, C.c_uint32]
        L.oracle_make_key.restype = C.c_uint64
        L.oracle_quadric_eval.argtypes = [P, P]
        L.oracle_quadric_eval.restype = C.c_double
        L.oracle_edge_cost.argtypes = [P, I64, P, I64, C.c_int32, C.c_int32, C.c_double, C.c_double, P, P]
        L.oracle_run_learned.argtypes = [P, I64, P, I64, I64, P, P, P, P, P, P, P, P]
        L.oracle_collect.argtypes = [P, I64, P, I64, I64, P, P, P, I64, P, P, P, P, P, P]
        L.oracle_features.argtypes = [P, I64, P, I64, P, I64, C.c_double, C.c_double, P, P]
        L.oracle_mlp_logits.argtypes = [P, P, I64, P]
        for n in ("oracle_sizeof_opts", "oracle_sizeof_stats", "oracle_sizeof_round_log", "oracle_sizeof_mlp"):
            getattr(L, n).restype = C.c_int64
        assert L.oracle_sizeof_opts() == C.sizeof(Opts)
        assert L.oracle_sizeof_stats() == C.sizeof(Stats)
        assert L.oracle_sizeof_round_log() == C.sizeof(RoundLog)
        assert L.oracle_sizeof_mlp() == C.sizeof(MLP)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _mesh(V, F):
    V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, 3)
    F = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
    return V, F


def _flags(flags, nf):
    if flags is None:
        return None
    f = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)
    assert f.size == 3 * nf
    return f


def quadrics(V, F):
    V, F = _mesh(V, F)
    Q = np.zeros((len(V), 10))
    rc = lib().oracle_quadrics(_p(V), len(V), _p(F), len(F), _p(Q))
    if rc:
        raise ValueError(f"oracle_quadrics: {rc}")
    return Q


def keys(V, F, flags=None, w_e=W_E, w_s=W_S):
    """64-bit keys at every representative half-edge (h < twin(h)), else 2^64-1."""
    V, F = _mesh(V, F)
    K = np.zeros(3 * len(F), dtype=np.uint64)
    rc = lib().oracle_keys(_p(V), len(V), _p(F), len(F), _p(_flags(flags, len(F))), w_e, w_s, _p(K))
    if rc:
        raise ValueError(f"oracle_keys: {rc}")
    return K


def select(V, F, flags=None, w_e=W_E, w_s=W_S):
    """Candidate edges (representative half-edge ids, ascending)."""
    V, F = _mesh(V, F)
    cand = np.zeros(3 * len(F) + 1, dtype=np.int32)
    n = np.zeros(1, dtype=np.int64)
    rc = lib().oracle_select(_p(V), len(V), _p(F), len(F), _p(_flags(flags, len(F))), w_e, w_s,
                             _p(cand), _p(n))
    if rc:
        raise ValueError(f"oracle_select: {rc}")
    return cand[: n[0]].copy()


def check(V, F, target, flags=None, w_e=W_E, w_s=W_S, prefilter=0, key_mode=0):
    """One round up to the end of the check/undo loop (prefilter, key_mode: as in run).
    Returns (cand, vbar (n,3), reason (n,), undo_iterations)."""
    V, F = _mesh(V, F)
    cap = 3 * len(F) + 1
    cand = np.zeros(cap, dtype=np.int32)
    vbar = np.zeros((cap, 3))
    reason = np.zeros(cap, dtype=np.uint8)
    n = np.zeros(1, dtype=np.int64)
    it = np.zeros(1, dtype=np.int64)
    rc = lib().oracle_check(_p(V), len(V), _p(F), len(F), _p(_flags(flags, len(F))), w_e, w_s,
                            int(target), int(prefilter), int(key_mode), _p(cand), _p(n), _p(vbar), _p(reason), _p(it))
    if rc:
        raise ValueError(f"oracle_check: {rc}")
    k = n[0]
    return cand[:k].copy(), vbar[:k].copy(), reason[:k].copy(), int(it[0])


def run(V, F, target, flags=None, streak=0, max_rounds=-1, w_e=W_E, w_s=W_S,
        tolerance=TOLERANCE, log_rounds=0, cost_target=0.0, prefilter=0, key_mode=0):
    """Whole method.  Returns dict with V, F, flags, streak, stats, log.
    cost_target > 0: only edges costing at most this collapse, and a round that
    selects nothing ends the run (the paper's target-cost termination).
    prefilter: the link and flip checks run on every keyed edge before the
    selection, and failing edges are not selectable that round.
    key_mode 1: keys ordered by the float64 cost, then the edge id."""
    V, F = _mesh(V, F)
    Vo = np.zeros_like(V)
    Fo = np.zeros_like(F)
    fo = np.zeros(3 * len(F), dtype=np.uint8)
    nvo = np.zeros(1, dtype=np.int64)
    nfo = np.zeros(1, dtype=np.int64)
    so = np.zeros(1, dtype=np.int32)
    st = Stats()
    opt = Opts(w_e, w_s, tolerance, max_rounds, cost_target, int(prefilter), int(key_mode))
    LogArr = RoundLog * max(1, log_rounds)
    log = LogArr()
    rc = lib().oracle_run(_p(V), len(V), _p(F), len(F), _p(_flags(flags, len(F))), int(streak),
                          int(target), C.byref(opt), _p(Vo), _p(nvo), _p(Fo), _p(nfo), _p(fo),
                          _p(so), C.byref(st), C.byref(log), log_rounds)
    if rc:
        raise ValueError(f"oracle_run: {rc}")
    nv, nf = int(nvo[0]), int(nfo[0])
    stats = {k: getattr(st, k) for k, _ in Stats._fields_ if k != "undo_hist"}
    stats["undo_hist"] = list(st.undo_hist)
    rows = [{k: getattr(log[i], k) for k, _ in RoundLog._fields_}
            for i in range(min(log_rounds, stats["rounds"]))]
    return {"V": Vo[:nv].copy(), "F": Fo[:nf].copy(), "flags": fo[: 3 * nf].copy(),
            "streak": int(so[0]), "stats": stats, "log": rows}


def tri_pair(P, ip, Q, iq) -> bool:
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(9)
    Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(9)
    ip = np.ascontiguousarray(ip, dtype=np.int32)
    iq = np.ascontiguousarray(iq, dtype=np.int32)
    return bool(lib().oracle_tri_pair(_p(P), _p(ip), _p(Q), _p(iq)))


def degenerate(P) -> bool:
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(9)
    return bool(lib().oracle_degenerate(_p(P)))


def orient2d(a, b, c, exact_only=False):
    a, b, c = (np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, c))
    f = lib().oracle_orient2d_exact if exact_only else lib().oracle_orient2d
    return f(_p(a), _p(b), _p(c))


def orient3d(a, b, c, d, exact_only=False):
    a, b, c, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, c, d))
    f = lib().oracle_orient3d_exact if exact_only else lib().oracle_orient3d
    return f(_p(a), _p(b), _p(c), _p(d))


def skinny(P) -> float:
    """1 - C_ijk of one triangle (Eq. 1)."""
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(9)
    return float(lib().oracle_skinny(_p(P)))


def make_key(cost: float, edge_id: int) -> int:
    return int(lib().oracle_make_key(float(cost), int(edge_id)))


def quadric_eval(q10, v) -> float:
    q = np.ascontiguousarray(q10, dtype=np.float64).reshape(10)
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(3)
    return float(lib().oracle_quadric_eval(_p(q), _p(v)))


def edge_cost(V, F, a, b, w_e=W_E, w_s=W_S):
    """(cost, placement) of collapsing edge (a, b)."""
    V, F = _mesh(V, F)
    cost = np.zeros(1)
    vbar = np.zeros(3)
    rc = lib().oracle_edge_cost(_p(V), len(V), _p(F), len(F), int(a), int(b), w_e, w_s, _p(cost), _p(vbar))
    if rc:
        raise ValueError(f"oracle_edge_cost: {rc}")
    return float(cost[0]), vbar


def self_intersections(V, F, cap=1 << 20):
    V, F = _mesh(V, F)
    pairs = np.zeros((cap, 2), dtype=np.int32)
    n = np.zeros(1, dtype=np.int64)
    rc = lib().oracle_self_intersections(_p(V), len(V), _p(F), len(F), _p(pairs), cap, _p(n))
    if rc:
        raise ValueError(f"oracle_self_intersections: {rc}")
    k = int(n[0])
    if k > cap:
        raise ValueError("pair buffer too small")
    return pairs[:k].copy()


def validate(V, F) -> int:
    V, F = _mesh(V, F)
    return int(lib().oracle_validate(_p(V), len(V), _p(F), len(F)))


def _stats_dict(st):
    d = {k: getattr(st, k) for k, _ in Stats._fields_ if k != "undo_hist"}
    d["undo_hist"] = list(st.undo_hist)
    return d


def features(V, F, edges, w_e=W_E, w_s=W_S):
    """Quantised features (n, 32) of the given edges (half-edge ids) and the
    per-face overlap counts of the mesh."""
    V, F = _mesh(V, F)
    e = np.ascontiguousarray(edges, dtype=np.int32)
    X = np.zeros((len(e), NFEAT), dtype=np.float32)
    ovl = np.zeros(len(F), dtype=np.int32)
    rc = lib().oracle_features(_p(V), len(V), _p(F), len(F), _p(e), len(e), w_e, w_s, _p(X), _p(ovl))
    if rc:
        raise ValueError(f"oracle_features: {rc}")
    return X, ovl


def mlp_logits(model, X):
    X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, NFEAT)
    out = np.zeros(len(X))
    m = mlp_struct(model)
    lib().oracle_mlp_logits(C.byref(m), _p(X), len(X), _p(out))
    return out


def run_learned(V, F, target, model, max_rounds=-1, w_e=W_E, w_s=W_S, tolerance=TOLERANCE, prefilter=0,
                key_mode=0):
    """The method with the learned proposal.  Returns dict with V, F, stats,
    demoted (candidates set aside) and fallbacks (rounds run again plain)."""
    V, F = _mesh(V, F)
    Vo, Fo = np.zeros_like(V), np.zeros_like(F)
    nvo, nfo = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
    info = np.zeros(2, dtype=np.int64)
    st = Stats()
    opt = Opts(w_e, w_s, tolerance, max_rounds, 0.0, int(prefilter), int(key_mode))
    m = mlp_struct(model)
    rc = lib().oracle_run_learned(_p(V), len(V), _p(F), len(F), int(target), C.byref(opt), C.byref(m), _p(Vo),
                                  _p(nvo), _p(Fo), _p(nfo), C.byref(st), _p(info))
    if rc:
        raise ValueError(f"oracle_run_learned: {rc}")
    nv, nf = int(nvo[0]), int(nfo[0])
    return {"V": Vo[:nv].copy(), "F": Fo[:nf].copy(), "stats": _stats_dict(st), "demoted": int(info[0]),
            "fallbacks": int(info[1])}


def collect(V, F, target, cap=1 << 20, w_e=W_E, w_s=W_S, tolerance=TOLERANCE, key_mode=0):
    """The plain method, logging (features, committed?) of every candidate the
    checks decided.  Returns (X (n, 32) float32, y (n,) uint8, run dict)."""
    V, F = _mesh(V, F)
    X = np.zeros((cap, NFEAT), dtype=np.float32)
    y = np.zeros(cap, dtype=np.uint8)
    n = np.zeros(1, dtype=np.int64)
    Vo, Fo = np.zeros_like(V), np.zeros_like(F)
    nvo, nfo = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
    st = Stats()
    opt = Opts(w_e, w_s, tolerance, -1, 0.0, 0, int(key_mode))
    rc = lib().oracle_collect(_p(V), len(V), _p(F), len(F), int(target), C.byref(opt), _p(X), _p(y), cap, _p(n),
                              _p(Vo), _p(nvo), _p(Fo), _p(nfo), C.byref(st))
    if rc:
        raise ValueError(f"oracle_collect: {rc}")
    k = int(n[0])
    return X[:k].copy(), y[:k].copy(), {"V": Vo[: int(nvo[0])].copy(), "F": Fo[: int(nfo[0])].copy(),
                                        "stats": _stats_dict(st)}
