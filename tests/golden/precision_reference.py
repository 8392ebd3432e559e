"""Writes the FP64 oracle's reference for the storage-precision report.

The report compares the GPU path in FP64, FP32 and FP16 storage with the FP64 CPU oracle on
two workloads, after the full step count of each:

- ``grf512``: the 512x512 cavity with a Gaussian-random-field porosity (seed 1), 50000 steps;
- ``band2048``: the 2048x2048 cavity with 8 porosity bands (seed 2), 20000 steps.

This script calls the oracle only (plus the seeded input generators) and stores, per
workload, the observables (Nu and Sh at every side, sums, largest velocities), the band means
of T and C, the largest |T|, |C| and speed over the lattice (the denominators of the relative
field errors), and the fields rho, ux, uy, T, C at 2048 seeded sample nodes.  The 2048x2048
case is 8.4e10 node updates: about half an hour on 8 host cores.

    python tests/golden/precision_reference.py grf512 [--threads N]
    python tests/golden/precision_reference.py band2048
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

CASES = {
    "grf512": lambda: workloads.grf_cavity(seed=1, n=512),
    "band2048": lambda: workloads.band_cavity(seed=2, n=2048),
}
SAMPLE_COUNT = 2048
SAMPLE_SEED = 12345


def path_of(name: str) -> str:
    return os.path.join(HERE, f"precision_{name}.json")


def run(name: str, steps=None, chunk: int = 1000) -> dict:
    case = CASES[name]()
    p = case["params"]
    nx, ny = p["nx"], p["ny"]
    steps = steps or case["steps"]
    o = oracle.Oracle(p, phi=case["phi"], T=case["T"], C=case["C"])
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        o.step(k)
        done += k
        print(f"{name}: {done}/{steps} steps, {time.perf_counter() - t0:.0f} s", flush=True)
    wall = time.perf_counter() - t0
    ob = o.observables()
    F = o.fields()
    xs, ys = workloads.sample_nodes(nx, ny, SAMPLE_COUNT, SAMPLE_SEED)
    bands = workloads.band_rows(ny, 8)
    out = {
        "what": "FP64 CPU oracle after the full step count; fields at seeded sample nodes",
        "case": case["name"], "nx": nx, "ny": ny, "steps": steps,
        "params": {k: (list(v) if isinstance(v, tuple) else v) for k, v in p.items()},
        "porosity": "grf seed 1" if name == "grf512" else "8 bands seed 2",
        "noise_seed": 1 if name == "grf512" else 2,
        "oracle_threads": oracle.threads(), "oracle_wall_s": round(wall, 1),
        "observables": {k: ob[k] for k in ("Nu", "Sh", "mass", "heat", "solute", "max_ux", "max_uy")},
        "field_max": {"T": float(np.abs(F["T"]).max()), "C": float(np.abs(F["C"]).max()),
                      "speed": float(np.hypot(F["ux"], F["uy"]).max())},
        "band_rows": bands,
        "band_mean": {k: [float(F[k][a:b].mean()) for a, b in bands] for k in ("T", "C")},
        "sample_seed": SAMPLE_SEED,
        "samples": {"x": xs.tolist(), "y": ys.tolist(),
                    **{k: F[k][ys, xs].tolist() for k in ("rho", "ux", "uy", "T", "C")}},
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=sorted(CASES))
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--steps", type=int, default=0, help="override the step count (tests only)")
    a = ap.parse_args()
    if a.threads:
        oracle.set_threads(a.threads)
    out = run(a.case, a.steps or None)
    dst = path_of(a.case) if not a.steps else path_of(a.case) + f".{a.steps}"
    with open(dst, "w") as f:
        json.dump(out, f)
    print(f"wrote {dst}", flush=True)


if __name__ == "__main__":
    main()
