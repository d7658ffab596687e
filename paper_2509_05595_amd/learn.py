"""Training of the learned proposal's network on the GPU.

Rows come from plain runs of the library (pamo_collect: the features of each
round's candidates and whether the checks let them through); the network is
trained by the library's own kernels (pamo_mlp_train: forward, backward and
Adam on float32 master weights, straight-through roundings); the trained
weights are rounded to their grids and handed to pamo_set_mlp.

    python -m paper_2509_05595_amd.learn out.json     # collect, train, write a model
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "models", "mlp_v2.json")
NPARAM = 6337
O_W1, O_B1, O_W2, O_B2, O_W3, O_B3 = 0, 2048, 2112, 6208, 6272, 6336


def training_meshes():
    """The meshes whose plain runs provide the rows: thin shells (two nested
    spheres close to each other, the case where collapses get undone for
    intersections), crease spheres simplified far (flipped triangles in the
    late rounds), and the noisy spheres and tori of the benchmark recipes,
    where nearly every candidate passes.  Pairs (mesh, face target)."""
    from . import meshgen as g
    out = []
    for k, gap in ((3, 0.03), (3, 0.015), (4, 0.01), (4, 0.006), (4, 0.004), (5, 0.003), (5, 0.002)):
        V, F = g.nested_spheres(k=k, gap=gap)
        out.append(((V, F), len(F) // 50))
    for seed in (100, 101, 102):
        V, F = g.noisy_icosphere(6, seed)
        out.append(((V, F), len(F) // 100))
    for seed in (11, 12):
        V, F = g.bumpy_torus(128, 48, seed=seed)
        out.append(((V, F), len(F) // 100))
    for seed in (11, 12):  # crease spheres: late, coarse rounds reject many collapses for flips
        V, F = g.crease_sphere(8, seed)
        out.append(((V, F), len(F) // 1000))
    return out


def held_out_meshes():
    """Meshes not used for training: a finer crease sphere, thin shells of
    other resolution / gap."""
    from . import meshgen as g
    return [(g.crease_sphere(9, 5), 0.001), (g.nested_spheres(k=5, gap=0.005), 0.02),
            (g.nested_spheres(k=6, gap=0.002), 0.02)]


def collect(ctx, meshes, cap_per_mesh=1 << 21):
    import torch
    Xs, ys = [], []
    for (V, F), target in meshes:
        Vd = torch.from_numpy(np.ascontiguousarray(V)).to(ctx.device)
        Fd = torch.from_numpy(np.ascontiguousarray(F)).to(ctx.device)
        X, y, _ = ctx.collect(Vd, Fd, target, cap=cap_per_mesh)
        Xs.append(X)
        ys.append(y)
    return torch.cat(Xs), torch.cat(ys)


def init_params(seed):
    """He-initialised float master weights in the library's flat layout."""
    rng = np.random.default_rng(seed)
    P = np.zeros(NPARAM, dtype=np.float32)
    P[O_W1:O_B1] = rng.normal(0, math.sqrt(2.0 / 11.0), 2048) * (np.arange(2048) % 32 < 11)
    P[O_W2:O_B2] = rng.normal(0, math.sqrt(2.0 / 64.0), 4096)
    P[O_W3:O_B3] = rng.normal(0, math.sqrt(1.0 / 64.0), 64)
    return P


def calibrate(P, X, e=(8, 8, 8)):
    """Activation shifts that map the 99th percentile of each hidden layer's
    positive pre-activations to about 100 (computed on the host from a sample,
    with the grid-rounded weights)."""
    Xs = X[: min(len(X), 20000)].astype(np.float64)
    W1 = np.clip(np.rint(np.ldexp(P[O_W1:O_B1].reshape(64, 32), e[0])), -127, 127) * 2.0 ** -e[0]
    z1 = np.maximum(Xs @ W1.T, 0)
    q1 = np.quantile(z1[z1 > 0], 0.99) if np.any(z1 > 0) else 1.0
    a1 = int(np.floor(np.log2(100.0 / q1)))
    h1 = np.minimum(np.rint(np.ldexp(z1, a1)), 127)
    W2 = np.clip(np.rint(np.ldexp(P[O_W2:O_B2].reshape(64, 64), e[1])), -127, 127) * 2.0 ** -e[1]
    z2 = np.maximum(h1 @ W2.T, 0)
    q2 = np.quantile(z2[z2 > 0], 0.99) if np.any(z2 > 0) else 1.0
    a2 = int(np.floor(np.log2(100.0 / q2)))
    return {"e1": e[0], "e2": e[1], "e3": e[2], "a1": a1, "a2": a2}


def train(ctx, X, y, steps=4000, batch=4096, lr=1e-3, seed=4, log=None):
    """Train on device rows (X float32 [n, 32], y uint8 [n]); returns (params, meta, losses)."""
    import torch
    P0 = init_params(seed)
    meta = calibrate(P0, X.cpu().numpy())
    md = [meta[k] for k in ("e1", "e2", "e3", "a1", "a2")]
    P = torch.from_numpy(P0).to(ctx.device)
    m = torch.zeros(NPARAM, device=ctx.device)
    v = torch.zeros(NPARAM, device=ctx.device)
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    losses = []
    chunk = 250
    t = 0
    while t < steps:
        k = min(chunk, steps - t)
        need = k * batch
        order = np.concatenate([rng.permutation(n) for _ in range(need // n + 1)])[:need].astype(np.int32)
        L = ctx.mlp_train(P, m, v, md, X, y, torch.from_numpy(order).to(ctx.device), k, batch, lr, t)
        t += k
        losses.extend(L.cpu().numpy().tolist())
        if log:
            log(f"step {t}: loss {np.mean(losses[-k:]):.4f}")
    return P.cpu().numpy(), meta, losses


def model_dict(P, meta, threshold):
    """Grid-rounded weights as pamo_set_mlp takes them."""
    def qw(w, e):
        return (np.clip(np.rint(np.ldexp(w, e)), -127, 127) * 2.0 ** -e).astype(np.float32)

    def qb(b, e):
        return (np.clip(np.rint(np.ldexp(b, e)), -2 ** 22, 2 ** 22) * 2.0 ** -e).astype(np.float32)
    e1, e2, e3 = meta["e1"], meta["e2"], meta["e3"]
    P = np.asarray(P, dtype=np.float64)
    return {"w1": qw(P[O_W1:O_B1].reshape(64, 32), e1), "b1": qb(P[O_B1:O_W2], e1),
            "w2": qw(P[O_W2:O_B2].reshape(64, 64), e2), "b2": qb(P[O_B2:O_W3], e2),
            "w3": qw(P[O_W3:O_B3], e3), "b3": float(qb(P[O_B3:], e3)[0]),
            "e1": e1, "e2": e2, "e3": e3, "a1": meta["a1"], "a2": meta["a2"], "threshold": float(threshold)}


def save_model(model, path, info=None):
    """Weights as integers on their grids (exact), with the exponents."""
    out = {"format": "pamo_mlp grid integers: value = k * 2^-e of its layer", "info": info or {}}
    for k, e in (("w1", "e1"), ("b1", "e1"), ("w2", "e2"), ("b2", "e2"), ("w3", "e3")):
        out[k] = np.rint(np.ldexp(np.asarray(model[k], dtype=np.float64), model[e])).astype(np.int64).tolist()
    out["b3"] = int(np.rint(np.ldexp(model["b3"], model["e3"])))
    for k in ("e1", "e2", "e3", "a1", "a2"):
        out[k] = int(model[k])
    out["threshold"] = float(model["threshold"])
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(out, f)


def load_model(path=MODEL_PATH):
    with open(path) as f:
        d = json.load(f)
    m = {}
    for k, e in (("w1", "e1"), ("b1", "e1"), ("w2", "e2"), ("b2", "e2"), ("w3", "e3")):
        m[k] = np.ldexp(np.asarray(d[k], dtype=np.float64), -d[e]).astype(np.float32)
    m["b3"] = float(np.ldexp(float(d["b3"]), -d["e3"]))
    for k in ("e1", "e2", "e3", "a1", "a2"):
        m[k] = int(d[k])
    m["threshold"] = float(d["threshold"])
    return m


def compare(ctx, model, meshes, reps=2):
    """Plain against learned on (mesh, target fraction) pairs: time, rounds,
    one-sided Hausdorff distance (input vertices to output surface)."""
    import torch
    from . import native
    rows = []
    for (V, F), frac in meshes:
        Vd = torch.from_numpy(np.ascontiguousarray(V)).to(ctx.device)
        Fd = torch.from_numpy(np.ascontiguousarray(F)).to(ctx.device)
        target = int(len(F) * frac)
        res = {}
        for name, learned in (("plain", 0), ("learned", 1)):
            ctx.set_mlp(model if learned else None)
            ctx.set_options(native.default_options(learned=learned))
            out = ctx.simplify(Vd, Fd, target)
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(reps):
                t0 = time.perf_counter()
                out = ctx.simplify(Vd, Fd, target)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            Vo, Fo, st = out
            res[name] = {"ms": best * 1e3, "faces_per_s": len(F) / best, "rounds": st["rounds"],
                         "faces_out": int(Fo.shape[0]), "status": st["status"], "demoted": st["demoted"],
                         "fallbacks": st["fallbacks"], "rej_isect": st["rej_isect"],
                         "hausdorff": ctx.hausdorff(Vd, Vo.contiguous(), Fo.contiguous())}
        ctx.set_options(native.default_options())
        ctx.set_mlp(None)
        rows.append({"faces": int(len(F)), "target": target, **res})
    return rows


def main(argv):
    import torch
    from . import native
    out = argv[0] if argv else MODEL_PATH
    ctx = native.Context(torch.device("cuda:0"))
    log = lambda s: print(f"[learn] {s}", file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.time()
    X, y = collect(ctx, training_meshes())
    log(f"collected {X.shape[0]} rows ({int(y.sum())} committed) in {time.time() - t0:.1f} s")
    P, meta, losses = train(ctx, X, y, log=log)
    model = model_dict(P, meta, threshold=0.0)
    rows = compare(ctx, model, held_out_meshes())
    for r in rows:
        log(json.dumps(r))
    save_model(model, out, {"rows": int(X.shape[0]), "committed": int(y.sum()), "final_loss": float(np.mean(losses[-100:])),
                            "held_out": rows})
    log(f"wrote {out}")


if __name__ == "__main__":
    main(sys.argv[1:])
