"""Throughput of the fused D2Q9 + 2 x D2Q5 MRT lattice Boltzmann step on one MI355X.

Workload: the 2048 x 2048 layered porous cavity (8 horizontal porosity bands drawn from
U[0.35, 0.9], Ra = 1e7, Da = 1e-4, Pr = 0.7, Le = 10, N = 2), FP32 population storage.
A step is one time step of f, g and h over every node.  Inputs are resident in HBM before
the timed region.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# algorithmic bytes per lattice update: 19 population loads + 19 stores, 4 + 4 previous-step
# field accesses, 1 porosity load (the porosity is a field here)
BYTES_PER_LU = {"fp64": 19 * 8 * 2 + 4 * 8 * 2 + 8, "fp32": 19 * 4 * 2 + 4 * 4 * 2 + 4,
                "fp16s": 19 * 2 * 2 + 4 * 4 * 2 + 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="fp32", choices=("fp64", "fp32", "fp16s"))
    ap.add_argument("--n", type=int, default=2048, help="lattice side")
    ap.add_argument("--variant-steps", type=int, default=2000,
                    help="steps for the FP64 and FP16-storage side measurements (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", default="", help="tile_x,tile_y (default: library default)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="instead of the solver, run 10 plain device-to-device copies of MIB MiB "
                         "(reference kernel for scaling the HBM byte counters)")
    return ap.parse_args()


def copy_probe(mib):
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    print(json.dumps({"copy_probe_MiB": mib, "ms_per_copy": ms,
                      "GB_s_read_plus_write": 2 * mib * 1048576 / (ms * 1e-3) / 1e9}), flush=True)


def timed_run(case, prec, steps, warmup, tile=None):
    import torch
    from paper_1708_07525_amd import Solver

    s = Solver(case["params"], phi=case["phi"], T=case["T"], C=case["C"], precision=prec, tile=tile)
    stream = torch.cuda.current_stream()
    s.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ob = s.observables()
    tile_used = s.get_tile()
    s.close()
    return ms, wall, ob, tile_used


def cpu_baseline(case, target_s):
    """The FP64 oracle (plain, untuned) on the host cores, on a bounded sample of the same
    workload: the full lattice for as many steps as fit in about target_s seconds."""
    import oracle
    o = oracle.Oracle(case["params"], phi=case["phi"], T=case["T"], C=case["C"])
    nodes = case["params"]["nx"] * case["params"]["ny"]
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    steps = max(1, int(target_s / max(one, 1e-6)) - 1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return dict(value=round(nodes * steps / dt / 1e6, 3), unit="MLUPS", cores=oracle.threads(), kind="oracle",
                sample=f"{case['params']['nx']}x{case['params']['ny']} lattice, {steps} steps (after 1 untimed), "
                       f"FP64 oracle, OpenMP over rows")


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU design is in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads

    torch.cuda.set_device(0)
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    case = workloads.band_cavity(seed=2, n=a.n)
    nodes = a.n * a.n
    tile = tuple(int(v) for v in a.tile.split(",")) if a.tile else None
    ms, wall, ob, tile_used = timed_run(case, a.precision, a.steps, a.warmup, tile)
    mlups = nodes * a.steps / (ms * 1e-3) / 1e6
    achieved = BYTES_PER_LU[a.precision] * nodes / (ms * 1e-3 / a.steps) / 1e9
    out = {
        "metric": "MLUPS (D2Q9+2xD2Q5) & % HBM roofline; batched p50/p99 solve latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": f"porous cavity {a.n}x{a.n}, 8 porosity bands U[0.35,0.9] (seed 2), Ra=1e7, "
                               f"Da=1e-4, Pr=0.7, Le=10, N=2, D2Q9+2xD2Q5 MRT, {a.precision} population storage",
                   "nx": a.n, "ny": a.n, "precision": a.precision, "tile": list(tile_used)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "bytes_per_lu": BYTES_PER_LU[a.precision], "kernel": "step_kernel"},
        "wall_s": round(wall, 3),
        "Nu_hot": ob["Nu"][0], "Sh_hot": ob["Sh"][0],
    }
    if a.variant_steps > 0:
        var = {}
        for prec in ("fp64", "fp32", "fp16s"):
            if prec == a.precision:
                continue
            vms, _, vob, vt = timed_run(case, prec, a.variant_steps, a.warmup)
            v = nodes * a.variant_steps / (vms * 1e-3) / 1e6
            ach = BYTES_PER_LU[prec] * nodes / (vms * 1e-3 / a.variant_steps) / 1e9
            var[prec] = {"MLUPS": round(v, 1), "GB_s": round(ach, 1), "frac": round(ach / PEAK_HBM_GBS, 4),
                         "steps": a.variant_steps, "tile": list(vt)}
        out["precisions"] = var
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
