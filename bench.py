"""Benchmark: input faces simplified per second on one MI355X.

Workload: icosphere refined 8 times (1,310,720 faces, 655,362 vertices) with
6-octave value-noise radial displacement, float64 positions, int32 faces,
simplified to 1% of its faces (13,106) by the full parallel intersection-free
QEM method.  A step is one complete ``pamo_simplify`` call (every round:
quadrics, costs, selection, local checks, LBVH check/undo loop, commit,
compaction) with input and output resident in HBM.

Besides the throughput line the JSON carries
  roofline      the dominant kernel: algorithmic bytes of its launches in the
                timed steps divided by their HIP-event duration, against the
                8 TB/s HBM peak;
  cpu_baseline  the serial C oracle (the same round rule, one thread) on the
                headline workload itself (about 100 s);
  batched       the batched form: 256 meshes (noisy geodesic spheres and
                bumpy tori, face counts log-uniform in [5k, 200k]) each to 1%
                in one pamo_simplify_batch call, beside the same meshes run
                one pamo_simplify call at a time (a 32-mesh sample);
  learned_vs_plain, sharp_feature_batch
                the learned proposal against the plain method (headline mesh,
                a thin shell; a 5.24M-face crease sphere batched with 32 tori).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
# single-kernel phases eligible as "the dominant kernel" of the roofline
SINGLE_KERNEL = ["quadrics", "cost_keys", "face_boxes", "apply", "query", "pairs", "resolve", "undo", "commit"]


def host_cpu():
    """Logical CPUs of this host and their model name (from /proc/cpuinfo)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(V, F, target):
    """The serial C oracle (one thread) on the headline workload itself: the
    same mesh and target as the timed GPU steps, one run."""
    import oracle.oracle as orc
    t0 = time.perf_counter()
    r = orc.run(V, F, target)
    dt = time.perf_counter() - t0
    ncpu, model = host_cpu()
    return {"value": len(F) / dt, "unit": "input faces/s", "cores": 1, "kind": "oracle",
            "sample": f"the headline workload itself: noisy icosphere k=8 ({len(F)} faces) to 1% "
                      f"({len(r['F'])} faces, {r['stats']['rounds']} rounds), serial C oracle (one thread), "
                      f"one run of {dt:.1f} s",
            "seconds": dt, "host_logical_cpus": ncpu, "host_cpu_model": model}


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "simplify__noisy-icosphere-1310720f-to-1pct.md")


def measured_traffic():
    """HBM bytes per launch of each phase from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE of the phase's own kernels, scaled by a
    plain copy's counts); empty when there is none or a kernel source changed
    since it was taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_PROFILE):
        return {}
    vals, ok = {}, True
    for line in open(TRAFFIC_PROFILE):
        f = line.split()
        if len(f) == 3 and f[0] == "traffic_bytes_per_launch":
            vals[f[1]] = float(f[2])
        if len(f) == 3 and f[0] == "source_sha256":
            path = os.path.join(HERE, f[1])
            ok = ok and os.path.exists(path) and hashlib.sha256(open(path, "rb").read()).hexdigest() == f[2]
    return vals if ok else {}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batched(native, torch, dev, steps, warmup, count, seq_sample):
    """The batched form on the 256-mesh recipe: spheres and tori of log-uniform
    face counts in [5k, 200k], each to 1%, all in one pamo_simplify_batch call
    per step; beside it the same meshes one pamo_simplify call each (a sample)."""
    from paper_2509_05595_amd import meshgen
    specs = meshgen.batch_specs(count=count)
    meshes = [meshgen.make_spec(sp) for sp in specs]
    log(f"batch generated: {count} meshes")
    dm = [(torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)) for V, F in meshes]
    targets = [len(F) // 100 for _, F in meshes]
    nf_total = sum(len(F) for _, F in meshes)
    from paper_2509_05595_amd import autotune
    tuned = autotune.options_for(nf_total, batch=True)
    ctx = native.Context(dev, options=native.default_options(**tuned))
    for _ in range(max(1, warmup)):
        out = ctx.simplify_batch(dm, targets)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.simplify_batch(dm, targets)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    log(f"batch timed: {dt * 1e3:.1f} ms per call")
    rounds = max(o[2]["rounds"] for o in out)
    # one mesh at a time, on the first seq_sample meshes
    sub = list(range(min(seq_sample, count)))
    for i in sub[:2]:
        ctx.simplify(dm[i][0], dm[i][1], targets[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in sub:
        ctx.simplify(dm[i][0], dm[i][1], targets[i])
    torch.cuda.synchronize()
    dts = time.perf_counter() - t0
    nf_sub = sum(len(meshes[i][1]) for i in sub)
    ctx.close()
    return {
        "value": nf_total / dt, "unit": "input faces/s", "ms_per_step": dt * 1e3, "steps": steps,
        "workload": f"{count} meshes (spheres and tori, log-uniform 5k-200k faces, {nf_total} faces in total) "
                    f"-> 1% each, one pamo_simplify_batch call",
        "rounds": rounds, "faces_out": int(sum(o[1].shape[0] for o in out)), "tuned_options": tuned,
        "one_at_a_time": {"value": nf_sub / dts, "unit": "input faces/s", "meshes": len(sub),
                          "faces": nf_sub, "ms": dts * 1e3},
    }


def learned_vs_plain(native, torch, dev, Vd, Fd, target, steps):
    """The learned proposal (the committed trained network) against the plain
    method on the same mesh: throughput, rounds, one-sided Hausdorff distance
    from the input vertices to the output surface; also on a thin-shell mesh
    (two nested spheres), where the plain method's candidates get undone for
    intersections."""
    from paper_2509_05595_amd import learn, meshgen
    if not os.path.exists(learn.MODEL_PATH):
        return None
    model = learn.load_model()
    ctx = native.Context(dev)
    out = {"model": os.path.relpath(learn.MODEL_PATH, os.path.dirname(os.path.abspath(__file__)))}
    Vs, Fs = meshgen.nested_spheres(k=6, gap=0.002)
    cases = {"headline": (Vd, Fd, target),
             "thin_shell": (torch.from_numpy(Vs).to(dev), torch.from_numpy(Fs).to(dev), len(Fs) // 50)}
    for name, (V, F, t) in cases.items():
        row = {"faces": int(F.shape[0]), "target": int(t)}
        for mode in ("plain", "learned"):
            ctx.set_mlp(model if mode == "learned" else None)
            ctx.set_options(native.default_options(learned=int(mode == "learned")))
            res = ctx.simplify(V, F, t)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                res = ctx.simplify(V, F, t)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            Vo, Fo, st = res
            row[mode] = {"faces_per_s": F.shape[0] / dt, "ms": dt * 1e3, "rounds": st["rounds"],
                         "faces_out": int(Fo.shape[0]), "demoted": st["demoted"], "fallbacks": st["fallbacks"],
                         "rej_isect": st["rej_isect"],
                         "hausdorff": ctx.hausdorff(V, Vo.contiguous(), Fo.contiguous())}
        row["speedup"] = row["learned"]["faces_per_s"] / row["plain"]["faces_per_s"]
        row["hausdorff_ratio"] = row["learned"]["hausdorff"] / max(row["plain"]["hausdorff"], 1e-300)
        out[name] = row
        log(f"learned vs plain on {name}: {row['speedup']:.3f}x")
    ctx.set_options(native.default_options())
    ctx.close()
    return out


def whole_mesh_check(native, torch, dev, reps=5):
    """The whole-mesh exact self-intersection check (pamo_self_intersections:
    face boxes, Morton sort, BVH build, all-pairs query, pair predicate, exact
    resolve) on noisy geodesic spheres of about the three sizes the paper times
    its check at (Tab. 6); the inputs are intersection-free, so every pair is
    tested and none reported.  The paper's figures are for another GPU
    (context, not the target)."""
    from paper_2509_05595_amd import meshgen
    paper_ms = {2500000: 48.3, 1100000: 26.1, 250000: 6.7}
    freq = {2500000: 354, 1100000: 235, 250000: 112}  # F = 20 n^2
    ctx = native.Context(dev)
    rows = []
    for size in (250000, 1100000, 2500000):
        V, F = meshgen.noisy_geodesic_sphere(freq[size], 11)
        Vd, Fd = torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)
        ctx.self_intersections(Vd, Fd)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            _, npairs = ctx.self_intersections(Vd, Fd)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        ms = sorted(times)[len(times) // 2] * 1e3
        rows.append({"faces": int(len(F)), "ms": ms, "faces_per_s": len(F) / ms * 1e3, "pairs": int(npairs),
                     "paper_size": size, "paper_ms": paper_ms[size], "paper_ms_over_ours": paper_ms[size] / ms})
        log(f"whole-mesh check {len(F)} faces: {ms:.2f} ms")
    ctx.close()
    return {"workload": "noisy geodesic spheres (seed 11), whole-mesh exact self-intersection check, median of "
                        f"{reps} calls including the count read-back", "rows": rows}


def remesh_udf(native, torch, dev, reps=5):
    """The remeshing stage's mesh-to-volume step (pamo_udf, Sec. 4.1): the
    narrow-band unsigned distance field (band 3 / R) of noisy icospheres at the
    voxel centres of R^3 grids.  The paper remeshes meshes of over 100k
    vertices in about 3 ms on another GPU, this step and the surface
    extraction together (context, not the target)."""
    import numpy as np
    from paper_2509_05595_amd import meshgen
    ctx = native.Context(dev)
    rows = []
    for k, res in ((7, 256), (7, 512), (8, 512)):
        V, F = meshgen.noisy_icosphere(k, 2)
        V = np.ascontiguousarray(0.5 + (V - 0.5) * 0.9)  # the band stays inside the grid: a closed extraction
        Vd, Fd = torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)
        U = ctx.udf(Vd, Fd, res)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            U = ctx.udf(Vd, Fd, res)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        ms = sorted(times)[len(times) // 2] * 1e3
        row = {"faces": int(len(F)), "vertices": int(len(V)), "res": res, "ms": ms,
               "voxels_in_band": int(torch.isfinite(U).sum())}
        log(f"distance field {len(F)} faces at {res}^3: {ms:.2f} ms")
        if True:  # the surface extraction (pamo_dualmc)
            Vo, Fo = ctx.dualmc(U, 0.9 / res, beta=5.0)
            nv, nf = len(Vo), len(Fo)
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                Vo, Fo = ctx.dualmc(U, 0.9 / res, vcap=nv, fcap=nf, beta=5.0)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            row.update({"dualmc_ms": sorted(times)[len(times) // 2] * 1e3, "out_vertices": nv, "out_faces": nf})
            log(f"dual marching cubes at {res}^3 -> {nf} faces: {row['dualmc_ms']:.2f} ms")
        rows.append(row)
    ctx.close()
    return {"workload": "noisy icospheres (seed 2, scaled by 0.9 about the centre), narrow-band unsigned distance "
                        "field at voxel centres, band 3/R, "
                        "then Dual Marching Cubes of the field less 0.9/R (smoothed crossings, beta 5), "
                        f"median of {reps} calls each", "rows": rows}


def safe_projection(native, torch, dev, Vd, Fd, Vs, Fs, reps=2, m=16384):
    """The stage after the path (Sec. 6, Alg. 2): the headline's simplified
    mesh projected back towards its input mesh with the paper's settings (m
    samples, T = 50 iterations, targets refreshed every 10), median of reps
    calls after one warm-up; the distance energy (both directions, targets
    found afresh) before and after."""
    import numpy as np
    ctx = native.Context(dev)
    U = torch.from_numpy(np.random.default_rng(7).random((m, 3))).to(dev)
    Y, area = ctx.sample_surface(Vd, Fd, U)
    opt = native.project_options()

    def distance_energy(X):
        tg, tri = ctx.project_targets(X, Fs, Vd, Fd, Y)
        p = ctx.project_eval(Vs, X, Fs, tg, Y, tri, area, options=opt)["parts"]
        return p[0] + p[1], p

    before, parts0 = distance_energy(Vs)
    Xo, lg, st = ctx.safe_project(Vs, Fs, Vd, Fd, Y, options=opt)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        Xo, lg, st = ctx.safe_project(Vs, Fs, Vd, Fd, Y, options=opt)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = sorted(times)[len(times) // 2] * 1e3
    after, parts1 = distance_energy(Xo)
    _, npairs = ctx.self_intersections(Xo, Fs)
    ctx.close()
    log(f"safe projection {int(Fs.shape[0])} faces towards {int(Fd.shape[0])}: {ms:.1f} ms, "
        f"{st['cg_iters']} CG iterations, distance energy {before:.4g} -> {after:.4g}")
    return {"workload": f"the headline's simplified mesh ({int(Fs.shape[0])} faces) projected towards its input "
                        f"({int(Fd.shape[0])} faces), {m} samples, T = {opt.iterations}, refresh every "
                        f"{opt.refresh}, paper weights; median of {reps} calls",
            "ms": ms, "iterations_per_s": opt.iterations / (ms / 1e3), "stats": st,
            "distance_energy_before": before, "distance_energy_after": after,
            "parts_before": parts0, "parts_after": parts1, "intersecting_pairs_after": int(npairs),
            "log_first": lg[0].tolist(), "log_last": lg[-1].tolist()}


def sharp_feature(native, torch, dev, steps):
    """Crease sphere (icosphere refined 9x, 5,242,880 faces, radius
    1 + 0.03|sin 12 theta||sin 9 phi| + 0.002 N(0,1)) to 0.1%, in one batch with 32
    bumpy tori of 20k-100k faces to 1%: plain and learned batched forms, the
    plain form with the link/flip checks run on every edge before the selection
    (the part of the learned form's gain that needs no network), and the
    network on top of that pre-filter."""
    from paper_2509_05595_amd import learn, meshgen
    meshes = [meshgen.crease_sphere(9, 5)] + [meshgen.make_spec(sp) for sp in meshgen.tori_specs()]
    targets = [len(meshes[0][1]) // 1000] + [len(F) // 100 for _, F in meshes[1:]]
    dm = [(torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)) for V, F in meshes]
    nf_total = sum(len(F) for _, F in meshes)
    log("sharp-feature batch generated")
    ctx = native.Context(dev)
    model = learn.load_model() if os.path.exists(learn.MODEL_PATH) else None
    out = {"workload": f"crease sphere 5,242,880 faces -> 0.1% with 32 tori ({nf_total} faces in total), "
                       f"one pamo_simplify_batch call"}
    for mode in ("plain", "learned", "prefilter", "learned_prefilter"):
        learned = mode in ("learned", "learned_prefilter")
        if learned and model is None:
            continue
        ctx.set_mlp(model if learned else None)
        ctx.set_options(native.default_options(learned=int(learned), prefilter=int("prefilter" in mode)))
        res = ctx.simplify_batch(dm, targets)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = ctx.simplify_batch(dm, targets)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        Vo, Fo, st = res[0]
        out[mode] = {"faces_per_s": nf_total / dt, "ms": dt * 1e3, "rounds": max(r[2]["rounds"] for r in res),
                     "sphere_faces_out": int(Fo.shape[0]), "sphere_rejected": st["rej_link"] + st["rej_flip"] +
                     st["rej_isect"], "demoted": sum(r[2]["demoted"] for r in res),
                     "sphere_hausdorff": ctx.hausdorff(dm[0][0], Vo.contiguous(), Fo.contiguous())}
        log(f"sharp-feature batch {mode}: {dt * 1e3:.1f} ms")
    ctx.set_options(native.default_options())
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--refine", type=int, default=8, help="icosphere refinement level (8: 1,310,720 faces)")
    ap.add_argument("--target-frac", type=float, default=0.01)
    ap.add_argument("--packet", type=int, default=0, help="BVH query packet size (0: library default)")
    ap.add_argument("--resort", type=int, default=0, help="re-sort BVH leaves every n rounds (0: library default)")
    ap.add_argument("--coop", type=int, default=0, help="lanes per query when few remain (0: library default, 1: off)")
    ap.add_argument("--coop-below", type=int, default=0, help="query count below which lanes share a query")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-versus-plain comparison")
    ap.add_argument("--no-sharp", action="store_true", help="skip the sharp-feature batch")
    ap.add_argument("--no-check", action="store_true", help="skip the whole-mesh self-intersection check")
    ap.add_argument("--no-udf", action="store_true", help="skip the remeshing distance-field measurement")
    ap.add_argument("--no-project", action="store_true", help="skip the safe-projection measurement")
    ap.add_argument("--only", choices=["check", "udf", "project"], default=None,
                    help="run only that section (whole-mesh check or distance field) and print its JSON")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB on the device three times (scale of the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); the method shards by mesh "
              "across GPUs, which is not built here", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        # a plain device copy of known size: FETCH_SIZE / WRITE_SIZE of this
        # kernel against the 1 GiB it moves give the counters' scale
        a = torch.ones(1 << 28, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {4 << 28} bytes three times")
        return
    from paper_2509_05595_amd import meshgen, native

    if args.only in ("check", "udf"):  # one section alone (for kernel profiles of its workload)
        dev = torch.device("cuda:0")
        res = whole_mesh_check(native, torch, dev) if args.only == "check" else remesh_udf(native, torch, dev)
        print(json.dumps(res), flush=True)
        return
    if args.only == "project":
        dev = torch.device("cuda:0")
        V, F = meshgen.noisy_icosphere(args.refine, 2)
        Vd, Fd = torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)
        c = native.Context(dev)
        Vs, Fs, _ = c.simplify(Vd, Fd, int(len(F) * args.target_frac))
        c.close()
        print(json.dumps(safe_projection(native, torch, dev, Vd, Fd, Vs.contiguous(), Fs.contiguous(), reps=1)),
              flush=True)
        return

    V, F = meshgen.noisy_icosphere(args.refine, 2)
    log("mesh generated")
    nf0 = len(F)
    target = int(nf0 * args.target_frac)
    dev = torch.device("cuda:0")
    Vd = torch.from_numpy(V).to(dev)
    Fd = torch.from_numpy(F).to(dev)
    ctx = native.Context(dev, options=native.default_options(query_packet=args.packet, resort_every=args.resort,
                                                             query_coop=args.coop, coop_below=args.coop_below))

    # warm-up; the last warm-up step times every phase (diagnostic breakdown)
    for i in range(max(1, args.warmup)):
        if i == max(1, args.warmup) - 1:
            ctx.profile(None)
        Vo, Fo, st = ctx.simplify(Vd, Fd, target)
    torch.cuda.synchronize()
    breakdown = ctx.profile_read()
    dominant = max((p for p in breakdown if p in SINGLE_KERNEL), key=lambda p: breakdown[p][1])

    # timed steps: only the dominant kernel carries HIP events
    ctx.profile([dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Vo, Fo, st = ctx.simplify(Vd, Fd, target)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile([])
    log(f"single mesh timed: {dt / args.steps * 1e3:.2f} ms per step")
    ms_per_step = dt / args.steps * 1e3
    value = nf0 / (ms_per_step / 1e3)
    launches, kms, kbytes = prof[dominant]
    traffic = measured_traffic()
    achieved = kbytes / (kms / 1e3) / 1e9

    out = {
        "metric": "input faces simplified/s at 1% target; learned vs plain at equal Hausdorff",
        "value": value,
        "unit": "input faces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"noisy icosphere refined {args.refine}x ({nf0} faces, {len(V)} vertices) -> "
                        f"{args.target_frac:.1%} target ({int(Fo.shape[0])} faces), plain method, single mesh",
            "rounds": st["rounds"], "faces_out": int(Fo.shape[0]), "commits": st["commits"],
            "rej_isect": st["rej_isect"], "undo_hist": st["undo_hist"],
        },
        "roofline": {
            "bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic.get(dominant),
            "launches": launches, "avg_launch_us": kms / launches * 1e3,
            "bytes_per_launch": kbytes / launches,
        },
        "phases_ms_per_step": {k: v[1] for k, v in sorted(breakdown.items(), key=lambda kv: -kv[1][1])},
        # every phase of one profiled step: launches, HIP-event milliseconds, the
        # algorithmic bytes of its launches and their rate against the HBM peak
        "phases": {k: {"launches": v[0], "ms": v[1], "bytes": v[2],
                       "GBs": v[2] / (v[1] / 1e3) / 1e9 if v[1] > 0 else None,
                       "frac": v[2] / (v[1] / 1e3) / 1e9 / HBM_PEAK_GBS if v[1] > 0 else None,
                       # counted HBM bytes per launch (rocprofv3 summary) and their rate
                       "traffic": traffic.get(k),
                       "traffic_frac": (traffic[k] * v[0] / (v[1] / 1e3) / 1e9 / HBM_PEAK_GBS
                                        if k in traffic and v[1] > 0 else None)}
                   for k, v in sorted(breakdown.items(), key=lambda kv: -kv[1][1])},
    }
    tot_bytes = sum(v[2] for v in breakdown.values())
    out["path_roofline"] = {"algorithmic_bytes_per_step": tot_bytes,
                            "achieved_GBs": tot_bytes / (ms_per_step / 1e3) / 1e9,
                            "frac": tot_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS}
    if not args.no_learned:
        lv = learned_vs_plain(native, torch, dev, Vd, Fd, target, 2)
        if lv is not None:
            out["learned_vs_plain"] = lv
    if not args.no_batch:
        ctx.close()
        out["batched"] = batched(native, torch, dev, args.batch_steps, 1, args.batch_count, 32)
    if not args.no_sharp:
        out["sharp_feature_batch"] = sharp_feature(native, torch, dev, 1)
    if not args.no_check:
        out["whole_mesh_check"] = whole_mesh_check(native, torch, dev)
    if not args.no_udf:
        out["remesh_udf"] = remesh_udf(native, torch, dev)
    if not args.no_project:
        out["safe_projection"] = safe_projection(native, torch, dev, Vd, Fd, Vo.contiguous(), Fo.contiguous())
    if not args.no_cpu_baseline and args.gpus == 1:
        out["cpu_baseline"] = cpu_baseline(V, F, target)
        log("cpu baseline timed")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
