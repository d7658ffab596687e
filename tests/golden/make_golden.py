"""Write the stored expected values of the full-size parity tests.

Runs only the CPU oracle (oracle/) on seeded generator inputs and records
SHA-256 digests of its outputs, so a GPU test can compare a full-size run bit
for bit without re-running the oracle.

    python tests/golden/make_golden.py [group ...]

Groups (each writes its own file next to this script):
  headline    full_size_oracle.json: the 1,310,720-face noisy icosphere to 1%
              and to 0.1%
  batch       batch256_oracle.json: the 256 meshes of the batched workload
              (spheres and tori, log-uniform 5k-200k faces), each to 1%, each
              run alone (a batch must give every mesh its lone result)
  shell       thin_shell_oracle.json: two nested spheres of 81,920 faces each
              (gap 0.002) to 2%, where most collapses are undone for
              intersections, plain and with the committed network
  sharp       sharp_tori_oracle.json: the 32 tori of the sharp-feature batch,
              each to 1%
With no argument every group is written.
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.oracle as orc  # noqa: E402
from paper_2509_05595_amd import meshgen  # noqa: E402


def digest(a):
    return hashlib.sha256(a.tobytes()).hexdigest()


def record(V, F, target, r, seconds):
    st = r["stats"]
    out = {
        "input_V_sha256": digest(V), "input_F_sha256": digest(F), "faces_in": int(len(F)), "target": int(target),
        "faces_out": int(len(r["F"])), "verts_out": int(len(r["V"])),
        "V_sha256": digest(r["V"]), "F_sha256": digest(r["F"]),
        "stats": {k: (list(v) if isinstance(v, list) else int(v)) for k, v in st.items()},
        "oracle_seconds": round(seconds, 1),
    }
    for k in ("demoted", "fallbacks"):
        if k in r:
            out[k] = int(r[k])
    return out


def case(V, F, target, **kw):
    t0 = time.time()
    r = orc.run(V, F, target, **kw)
    return record(V, F, target, r, time.time() - t0)


def _spec_case(args):
    i, spec = args
    V, F = meshgen.make_spec(spec)
    return i, case(V, F, len(F) // 100)


def _write(name, out):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote", path, flush=True)


def headline():
    out = {}
    V, F = meshgen.noisy_icosphere(8, 2)
    for frac, label in ((0.01, "1pct"), (0.001, "0.1pct")):
        k = f"noisy_icosphere_k8_seed2_{label}"
        out[k] = case(V, F, int(len(F) * frac))
        print(k, out[k]["faces_out"], out[k]["oracle_seconds"], flush=True)
    _write("full_size_oracle.json", out)


def _faces(spec):
    kind, size, _ = spec
    return 20 * size * size if kind == "sphere" else 2 * size[0] * size[1]


def _spec_group(specs, workers):
    res = [None] * len(specs)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        # largest first, so the pool drains evenly
        order = sorted(range(len(specs)), key=lambda i: -_faces(specs[i]))
        for i, rec in ex.map(_spec_case, [(i, specs[i]) for i in order]):
            res[i] = rec
            print("mesh", i, rec["faces_in"], "->", rec["faces_out"], rec["oracle_seconds"], "s", flush=True)
    return res


def batch(workers):
    specs = meshgen.batch_specs(count=256)
    res = _spec_group(specs, workers)
    _write("batch256_oracle.json", {"recipe": "meshgen.batch_specs(count=256), each to len(F) // 100",
                                    "meshes": res})


def sharp(workers):
    specs = meshgen.tori_specs()
    res = _spec_group(specs, workers)
    _write("sharp_tori_oracle.json", {"recipe": "meshgen.tori_specs(), each to len(F) // 100", "meshes": res})


def shell():
    from paper_2509_05595_amd import learn
    V, F = meshgen.nested_spheres(k=6, gap=0.002)
    target = len(F) // 50
    out = {"plain": case(V, F, target)}
    print("shell plain", out["plain"]["stats"], flush=True)
    t0 = time.time()
    r = orc.run_learned(V, F, target, learn.load_model())
    out["learned"] = record(V, F, target, r, time.time() - t0)
    out["model_sha256"] = hashlib.sha256(open(learn.MODEL_PATH, "rb").read()).hexdigest()
    print("shell learned", out["learned"]["stats"], flush=True)
    _write("thin_shell_oracle.json", out)


def main():
    groups = sys.argv[1:] or ["headline", "batch", "shell", "sharp"]
    workers = int(os.environ.get("GOLDEN_WORKERS", "6"))
    for g in groups:
        if g == "headline":
            headline()
        elif g == "batch":
            batch(workers)
        elif g == "shell":
            shell()
        elif g == "sharp":
            sharp(workers)
        else:
            raise SystemExit(f"unknown group {g}")


if __name__ == "__main__":
    main()
