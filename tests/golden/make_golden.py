"""Writes the stored expected values under tests/golden/ by calling only the
oracle. Run from the repository root: python tests/golden/make_golden.py"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from synth import workload  # noqa: E402


def small_l64_summary():
    p = workload("small_l64")
    u0, v0 = O.init_cube(L=p["L"], side=p["cube_side"], cu=p["cube_u"], cv=p["cube_v"])
    u, v = O.run(u0, v0, p["steps"], **p)
    d = O.diagnostics(u, v)
    L = p["L"]
    samples = {}
    for (z, y, x) in [(32, 32, 32), (26, 26, 26), (37, 37, 37), (20, 32, 40), (0, 0, 0), (31, 40, 25)]:
        samples[f"{z},{y},{x}"] = [u[z, y, x].hex(), v[z, y, x].hex()]
    return dict(
        workload="small_l64", params={k: p[k] for k in ("L", "steps", "Du", "Dv", "F", "k", "dt", "noise")},
        sha256_u=hashlib.sha256(u.tobytes()).hexdigest(), sha256_v=hashlib.sha256(v.tobytes()).hexdigest(),
        diagnostics={k: (float(x).hex() if isinstance(x, float) else x) for k, x in d.items()},
        samples_zyx_hex=samples)


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_l64_oracle.json")
    with open(out, "w") as f:
        json.dump(small_l64_summary(), f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", out)
