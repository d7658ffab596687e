"""Write the stored expected values of the full-size parity tests.

Runs only the CPU oracle (oracle/) on seeded generator inputs and records
SHA-256 digests of its outputs, so a GPU test can compare a full-size run bit
for bit without re-running the ~100 s oracle.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.oracle as orc  # noqa: E402
from paper_2509_05595_amd import meshgen  # noqa: E402


def digest(a):
    return hashlib.sha256(a.tobytes()).hexdigest()


def case(name, V, F, target, **kw):
    t0 = time.time()
    r = orc.run(V, F, target, **kw)
    st = r["stats"]
    return name, {
        "input_V_sha256": digest(V), "input_F_sha256": digest(F), "faces_in": int(len(F)), "target": int(target),
        "faces_out": int(len(r["F"])), "verts_out": int(len(r["V"])),
        "V_sha256": digest(r["V"]), "F_sha256": digest(r["F"]),
        "stats": {k: (list(v) if isinstance(v, list) else int(v)) for k, v in st.items()},
        "oracle_seconds": round(time.time() - t0, 1),
    }


def main():
    out = {}
    V, F = meshgen.noisy_icosphere(8, 2)
    for frac, label in ((0.01, "1pct"), (0.001, "0.1pct")):
        k, v = case(f"noisy_icosphere_k8_seed2_{label}", V, F, int(len(F) * frac))
        out[k] = v
        print(k, v["faces_out"], v["oracle_seconds"], flush=True)
    path = os.path.join(HERE, "full_size_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
