"""Autotuner of the traversal and BVH-order knobs.

The knobs (pamo_options.query_packet, query_coop, coop_below, resort_every)
change how the check/undo loop walks the BVH, never what it finds, so any
setting gives the same meshes; only the time differs.  The tuner times
candidate settings on a workload, keeps the fastest, and records it per
workload class (single mesh or batch, by size) in tuned.json next to this
file; ``options_for`` looks a setting up for a given face count.

    python -m paper_2509_05595_amd.autotune            # tune and write tuned.json
"""
from __future__ import annotations

import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned.json")

# the search space: packet sizes of the one-lane-per-query walk, lanes per
# query of the cooperative walk, the query count below which it is used, and
# the leaf re-sort interval (0 = never)
SPACE = {
    "query_packet": [1, 2, 8],
    "query_coop": [1, 4, 8, 16],
    "coop_below": [32768, 65536, 131072, 524288],
    "resort_every": [0, 8],
}
KNOBS = list(SPACE)


def candidates(full: bool = False):
    """Settings to time: the full grid, or a coordinate search seed list."""
    grid = [dict(zip(KNOBS, v)) for v in itertools.product(*(SPACE[k] for k in KNOBS))]
    if full:
        return grid
    # query_coop = 1 makes coop_below irrelevant: keep one of those
    out, seen = [], set()
    for g in grid:
        key = tuple(g[k] for k in KNOBS if not (g["query_coop"] == 1 and k == "coop_below"))
        if key not in seen:
            seen.add(key)
            out.append(g)
    return out


def _time(run, reps: int) -> float:
    import torch
    run()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def coordinate_search(measure, start: dict, rounds: int = 2):
    """Minimise measure(setting) one knob at a time (a few passes)."""
    cur = dict(start)
    best = measure(cur)
    log = [(dict(cur), best)]
    for _ in range(rounds):
        improved = False
        for k in KNOBS:
            for v in SPACE[k]:
                if v == cur[k]:
                    continue
                trial = dict(cur, **{k: v})
                t = measure(trial)
                log.append((trial, t))
                if t < best * 0.995:
                    best, cur, improved = t, trial, True
        if not improved:
            break
    return cur, best, log


def tune_single(ctx_factory, V, F, target, reps=2):
    def measure(setting):
        ctx = ctx_factory(setting)
        t = _time(lambda: ctx.simplify(V, F, target), reps)
        ctx.close()
        return t
    start = {"query_packet": 1, "query_coop": 8, "coop_below": 65536, "resort_every": 0}
    return coordinate_search(measure, start)


def tune_batch(ctx_factory, meshes, targets, reps=1):
    def measure(setting):
        ctx = ctx_factory(setting)
        t = _time(lambda: ctx.simplify_batch(meshes, targets), reps)
        ctx.close()
        return t
    start = {"query_packet": 1, "query_coop": 8, "coop_below": 65536, "resort_every": 0}
    return coordinate_search(measure, start)


def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def options_for(faces: int, batch: bool = False, path: str = TABLE) -> dict:
    """The tuned knobs for the workload class nearest to `faces` total faces
    (empty dict: library defaults)."""
    table = load_table(path).get("batch" if batch else "single", [])
    if not table:
        return {}
    best = min(table, key=lambda e: abs(_log2(e["faces"]) - _log2(faces)))
    return dict(best["setting"])


def _log2(x):
    import math
    return math.log2(max(1, x))


def main(argv=None):
    import torch
    from . import meshgen, native

    dev = torch.device("cuda:0")

    def factory(setting):
        return native.Context(dev, options=native.default_options(**setting))

    out = {"single": [], "batch": [], "device": torch.cuda.get_device_name(0)}
    for refine in (6, 7, 8):
        V, F = meshgen.noisy_icosphere(refine, 2)
        Vd, Fd = torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)
        best, t, log = tune_single(factory, Vd, Fd, len(F) // 100)
        out["single"].append({"faces": int(len(F)), "setting": best, "seconds": t,
                              "tried": [[s, round(x, 6)] for s, x in log]})
        print(f"single {len(F)} faces: {best} {t * 1e3:.2f} ms", file=sys.stderr, flush=True)
    for count in (64, 256):
        specs = meshgen.batch_specs(count=count)
        ms = [meshgen.make_spec(s) for s in specs]
        dm = [(torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)) for V, F in ms]
        tg = [len(F) // 100 for _, F in ms]
        best, t, log = tune_batch(factory, dm, tg)
        nf = sum(len(F) for _, F in ms)
        out["batch"].append({"faces": int(nf), "meshes": count, "setting": best, "seconds": t,
                             "tried": [[s, round(x, 6)] for s, x in log]})
        print(f"batch {count} meshes {nf} faces: {best} {t * 1e3:.2f} ms", file=sys.stderr, flush=True)
    path = argv[0] if argv else TABLE
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, file=sys.stderr)


if __name__ == "__main__":
    main(sys.argv[1:])
