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
# algorithmic bytes of one node of one launch: the populations and fields of the level the
# launch starts from are read once (19 populations, 4 previous-step fields, 1 porosity) and
# those of the level it ends on are written once (19 + 4); a launch that advances k steps keeps
# the k - 1 levels in between on chip, so the bytes it must move do not grow with k.  For one
# step per launch this is the per-lattice-update figure (188 B in FP32).
BYTES_PER_LU = {"fp64": 19 * 8 * 2 + 4 * 8 * 2 + 8, "fp32": 19 * 4 * 2 + 4 * 4 * 2 + 4,
                "fp16s": 19 * 2 * 2 + 4 * 4 * 2 + 4}


def roofline_fields(prec, nodes, ms_per_step, spl):
    """Bandwidth of a launch against the HBM peak: ``achieved`` is the bytes a launch must move
    (BYTES_PER_LU per node) over the average launch time (ms_per_step x steps per launch), so
    frac <= 1 whatever the steps per launch; ``effective_per_step`` counts BYTES_PER_LU per
    node and step instead (the bandwidth a one-step kernel would need for the same rate, above
    the peak when a launch advances several steps)."""
    launch_s = ms_per_step * 1e-3 * spl
    ach = BYTES_PER_LU[prec] * nodes / launch_s / 1e9
    return {"achieved": round(ach, 1), "frac": round(ach / PEAK_HBM_GBS, 4),
            "effective_per_step_GB_s": round(ach * spl, 1),
            "effective_per_step_frac": round(ach * spl / PEAK_HBM_GBS, 4), "launch_us": round(launch_s * 1e6, 2)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="fp32", choices=("fp64", "fp32", "fp16s"))
    ap.add_argument("--n", type=int, default=2048, help="lattice side")
    ap.add_argument("--variant-steps", type=int, default=2000,
                    help="steps for the side measurements: FP64 and FP16 storage, walls through the "
                         "nodes, and (4x the steps) the 512^2 porosity-field cavity (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", default="auto",
                    help="tile_x,tile_y, 'default' (library rule) or 'auto' (time every tile shape, cache "
                         "policy and steps per launch on the workload before the timed region; default)")
    ap.add_argument("--policy", type=int, default=-1, help="cache policy 0/1/2 with an explicit --tile (-1: rule)")
    ap.add_argument("--spl", type=int, default=0, help="steps per launch 1/2/3 with an explicit --tile (0: rule)")
    ap.add_argument("--strip", type=int, default=-1,
                    help="tile order of the multi-step launches with an explicit --tile: 0 row by row, k strips "
                         "of k tiles (-1: rule)")
    ap.add_argument("--rows", type=int, default=0,
                    help="rows of the FP32 three-step / FP16 two-step tile with an explicit --tile: 8 or 12 "
                         "(0: rule)")
    ap.add_argument("--workload", default="cavity", choices=("cavity", "sweep", "serve", "precision"),
                    help="cavity: the 2048^2 throughput line (default); sweep: 256 independent cavities, "
                         "batched launch vs one by one; serve: continuous-batching request stream; "
                         "precision: FP64/FP32/FP16-storage errors against the FP64 oracle on the 512^2 and "
                         "2048^2 cavities")
    ap.add_argument("--precision-case", default="all", choices=("all", "grf512", "band2048"),
                    help="precision: which workload")
    ap.add_argument("--cavities", type=int, default=256, help="sweep: number of cavities")
    ap.add_argument("--chunk", type=int, default=120,
                    help="sweep and serve: steps per batched graph replay (a multiple of 12 lets FP32 and "
                         "FP64 groups take three steps per launch)")
    ap.add_argument("--until-converged", action="store_true",
                    help="sweep: run every cavity to steady state (residual 1e-8) or --max-steps, "
                         "batched through the serving loop and one by one with plain launches")
    ap.add_argument("--requests", type=int, default=256, help="serve: number of requests")
    ap.add_argument("--max-steps", type=int, default=0,
                    help="step cap per solve (serve and sweep --until-converged: default 100000)")
    ap.add_argument("--oracle-samples", type=int, default=4,
                    help="serve: requests re-run on the oracle (the smallest of each precision, alternating)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="instead of the solver, run 10 plain device-to-device copies of MIB MiB "
                         "(reference kernel for scaling the HBM byte counters)")
    return ap.parse_args()


def copy_rate(mib):
    """A plain device-to-device copy of `mib` MiB, 10 times after one untimed copy: ms per copy and
    GB/s counting the bytes read and written (the ceiling a streaming kernel reaches on this GPU)."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    return ms, 2 * mib * 1048576 / (ms * 1e-3) / 1e9


def copy_probe(mib):
    ms, gbs = copy_rate(mib)
    print(json.dumps({"copy_probe_MiB": mib, "ms_per_copy": ms, "GB_s_read_plus_write": gbs}), flush=True)


KERNEL_SOURCE = os.path.join(ROOT, "paper_1708_07525_amd", "csrc", "lbm_kernels.hip")
KERNEL_HEADER = os.path.join(ROOT, "paper_1708_07525_amd", "csrc", "lbm_internal.h")


def profiled_traffic(prec, n, launch):
    """HBM bytes per launch of the step kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size), or None when there is no
    summary for this workload, the kernel code has changed since the counters were taken, or
    the launch [tile_x, tile_y, policy, steps per launch, strip width, tile rows] differs from
    the profiled one."""
    import re
    kernel = {2: "step2_kernel", 3: "step3_kernel"}.get(launch[3], "step_kernel")
    path = os.path.join(ROOT, "profiles", f"{kernel}_{prec}_cavity{n}.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    same = d.get("kernel_code_sha256_16") == kernel_code_hash() and d.get("launch") == list(launch)
    return d["traffic_bytes_per_launch"] if same else None


def kernel_code_hash():
    """sha256 (first 16 hex digits) of the kernel source and its header with comments and
    whitespace removed: changes with the code, not with its comments."""
    import hashlib
    import re
    src = "".join(open(f).read() for f in (KERNEL_SOURCE, KERNEL_HEADER))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return hashlib.sha256("".join(src.split()).encode()).hexdigest()[:16]


def timed_run(case, prec, steps, warmup, tile="auto", policy=None, spl=0, strip=-1, rows=0):
    import torch
    from paper_1708_07525_amd import Solver

    s = Solver(case["params"], phi=case["phi"], T=case["T"], C=case["C"], precision=prec,
               tile=None if tile in ("auto", "default") else tile)
    if tile == "auto":
        s.autotune(120)                # restores the state it started from
    else:
        if policy is not None:
            s.set_cache_policy(policy)
        s.set_steps_per_launch(spl)
        s.set_strip_width(strip)
        s.set_tile_rows(rows if prec != "fp64" else 0)   # FP64 has 8-row tiles only
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
    tile_used = list(s.get_tile()) + [s.get_cache_policy(), s.get_steps_per_launch(), s.get_strip_width(),
                                      s.get_tile_rows()]
    s.close()
    return ms, wall, ob, tile_used


def cpu_baseline(case, target_s):
    """The FP64 oracle (plain, untuned) on the host cores, on a bounded sample of the same
    workload: the full lattice for as many steps as fit in about target_s seconds.  Also the
    same lattice on one thread (a few steps), and the 64^2 and 512^2 cavities of the parity
    tests, all threads."""
    import oracle
    import workloads

    def rate(params, phi, T, C, seconds, threads=None):
        o = oracle.Oracle(params, phi=phi, T=T, C=C)
        nodes = params["nx"] * params["ny"]
        if threads:
            oracle.set_threads(threads)
        try:
            t0 = time.perf_counter()
            o.step(1)
            one = time.perf_counter() - t0
            steps = max(1, int(seconds / max(one, 1e-6)) - 1)
            t0 = time.perf_counter()
            o.step(steps)
            dt = time.perf_counter() - t0
        finally:
            if threads:
                oracle.set_threads(0)
        return nodes * steps / dt / 1e6, steps

    p = case["params"]
    ml, steps = rate(p, case["phi"], case["T"], case["C"], target_s)
    out = dict(value=round(ml, 3), unit="MLUPS", cores=oracle.threads(), kind="oracle",
               sample=f"{p['nx']}x{p['ny']} lattice, {steps} steps (after 1 untimed), FP64 oracle, OpenMP over rows")
    ml1, steps1 = rate(p, case["phi"], case["T"], case["C"], max(2.0, target_s / 4), threads=1)
    out["one_thread"] = {"MLUPS": round(ml1, 3), "steps": steps1}
    small = workloads.small_cavity(seed=0)
    grf = workloads.grf_cavity(seed=1, n=512)
    out["other_samples"] = {
        name: {"MLUPS": round(m, 3), "steps": k}
        for name, (m, k) in (("cavity64", rate(small["params"], None, small["T"], small["C"], 1.0)),
                             ("grf512", rate(grf["params"], grf["phi"], grf["T"], grf["C"], 2.0)))}
    try:
        with open("/proc/cpuinfo") as f:
            out["cpu_model"] = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    out["nproc"] = os.cpu_count()
    return out


def sweep(a):
    """Independent cavities of uneven size and parameters (sides 64..512, aspect 1 or 2,
    Ra, Da, porosity, Le, N drawn per cavity), FP32: aggregate MLUPS of the batch (cache-sized
    groups, two or three steps per batched launch as the batch autotuner chooses, replayed
    from a HIP graph), against the same
    cavities stepped one by one with one plain launch per step (the one-step kernel, no
    graph), and one by one with the library defaults (three steps per launch, graph replay)."""
    import torch
    import workloads
    from paper_1708_07525_amd import Batch, Solver

    cav = workloads.sweep_cavities(a.cavities, seed=3)
    if a.until_converged:
        sweep_until_converged(a, cav)
        return
    solvers = []
    for e in cav:
        T, C = workloads.cavity_fields(e)
        solvers.append(Solver(e["params"], T=T, C=C, precision="fp32"))
    nodes = sum(s.nx * s.ny for s in solvers)
    steps = a.steps
    out = {"metric": "aggregate MLUPS, batched sweep vs one-by-one", "unit": "MLUPS", "cavities": len(solvers),
           "nodes": nodes, "steps": steps, "data": "synthetic"}
    # one by one, plain launches
    for mode, chunk, spl in (("one_by_one_plain", 0, 1), ("one_by_one_graph", 64, 0)):
        for s in solvers:
            s.set_graph_chunk(chunk)
            s.set_steps_per_launch(spl)
            s.step(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in solvers:
            s.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[mode] = round(nodes * steps / dt / 1e6, 1)
    b = Batch(len(solvers), chunk=a.chunk)
    for s in solvers:
        b.attach(s)
    t0 = time.perf_counter()
    chosen = b.autotune(24)
    out["batch_autotune"] = {"seconds": round(time.perf_counter() - t0, 2),
                             "choices": {f"{p}|{c}": {"shape": v[0], "policy": v[1]} for (p, c), v in chosen.items()}}
    b.step(200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["batched"] = round(nodes * steps / dt / 1e6, 1)
    out["value"] = out["batched"]
    out["speedup_vs_one_by_one_plain"] = round(out["batched"] / out["one_by_one_plain"], 3)
    out["speedup_vs_one_by_one_graph"] = round(out["batched"] / out["one_by_one_graph"], 3)
    b.close()
    print(json.dumps(out), flush=True)


def precision_report(a):
    """The 512^2 Gaussian-random-field cavity (50000 steps) and the 2048^2 banded cavity (20000
    steps), run on the GPU with FP64, FP32 and FP16 storage and compared with the FP64 CPU
    oracle's result after the same steps (tests/golden/precision_<case>.json, written by
    tests/golden/precision_reference.py from the oracle alone): Nu and Sh at both held sides,
    the fields at the 2048 seeded sample nodes the reference keeps (relative to the largest
    |T|, |C| and speed over the lattice; rho absolute), and the band means of T and C.  Also
    MLUPS and the HBM roofline fraction of each run."""
    import torch
    import workloads
    from paper_1708_07525_amd import Solver

    golden = os.path.join(ROOT, "tests", "golden")
    cases = [("grf512", workloads.grf_cavity(seed=1, n=512)), ("band2048", workloads.band_cavity(seed=2, n=2048))]
    if a.precision_case != "all":
        cases = [c for c in cases if c[0] == a.precision_case]
    out = {"metric": "field and Nu/Sh error by storage precision against the FP64 CPU oracle", "data": "synthetic",
           "cases": []}
    for name, case in cases:
        path = os.path.join(golden, f"precision_{name}.json")
        if not os.path.exists(path):
            raise SystemExit(f"{path} is missing: write it with tests/golden/precision_reference.py {name}")
        ref = json.load(open(path))
        steps = ref["steps"]
        n = case["params"]["nx"]
        xs, ys = np.array(ref["samples"]["x"]), np.array(ref["samples"]["y"])
        rob = ref["observables"]
        c = {"case": case["name"], "steps": steps, "reference": f"FP64 oracle ({os.path.basename(path)})",
             "oracle_Nu": rob["Nu"][:2], "oracle_Sh": rob["Sh"][:2]}
        for prec in ("fp64", "fp32", "fp16s"):
            s = Solver(case["params"], phi=case["phi"], T=case["T"], C=case["C"], precision=prec)
            s.step(2)                               # first launches and graph capture
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(steps - 2)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ob = s.observables()
            F = s.fields()
            spl = s.get_steps_per_launch()
            s.close()
            ml = n * n * (steps - 2) / dt / 1e6
            rf = roofline_fields(prec, n * n, dt * 1e3 / (steps - 2), spl)
            fm = ref["field_max"]
            err = {k: float(np.abs(F[k][ys, xs] - np.array(ref["samples"][k])).max() / fm[k]) for k in ("T", "C")}
            err.update({k: float(np.abs(F[k][ys, xs] - np.array(ref["samples"][k])).max() / fm["speed"])
                        for k in ("ux", "uy")})
            err["rho"] = float(np.abs(F["rho"][ys, xs] - np.array(ref["samples"]["rho"])).max())
            band = {k: float(max(abs(F[k][lo:hi].mean() - m) for (lo, hi), m in zip(ref["band_rows"], ref["band_mean"][k])))
                    for k in ("T", "C")}
            row = {"MLUPS": round(ml, 1), "frac": rf["frac"], "effective_per_step_frac": rf["effective_per_step_frac"],
                   "steps_per_launch": spl, "Nu": ob["Nu"][:2], "Sh": ob["Sh"][:2],
                   "Nu_rel_err": [abs(ob["Nu"][i] - rob["Nu"][i]) / abs(rob["Nu"][i]) for i in (0, 1)],
                   "Sh_rel_err": [abs(ob["Sh"][i] - rob["Sh"][i]) / abs(rob["Sh"][i]) for i in (0, 1)],
                   "sample_field_err": err, "band_mean_abs_err": band}
            c[prec] = row
            print(json.dumps({"case": name, prec: row}), flush=True)
        out["cases"].append(c)
    print(json.dumps(out), flush=True)


def sweep_until_converged(a, cav):
    """Every cavity of the sweep to steady state (K-step velocity residual below 1e-8, checked
    every 10 replay chunks) or the step cap: all together through the continuous-batching loop,
    then the same solves one by one with one plain launch per step (one-step kernel, no graph),
    checked at the same steps."""
    import torch
    import workloads
    from paper_1708_07525_amd import Solver
    from paper_1708_07525_amd.serving import Request, Server, converged

    cap = a.max_steps or 100000
    reqs = []
    for i, e in enumerate(cav):
        T, C = workloads.cavity_fields(e)
        reqs.append(Request(i, 0.0, e["params"], "fp32", None, T, C))
    srv = Server(200 * 10 ** 9, max_slots=len(reqs), chunk=a.chunk, check_every=10 * a.chunk, tol=1e-8, max_steps=cap,
                 autotune_steps=20)

    def note(d):
        print("progress", json.dumps(d), file=sys.stderr, flush=True)
    res, summ = srv.run(reqs, progress=note)
    srv.close()
    steps_batched = {r.id: r.steps for r in res}
    node_steps = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_alone = {}
    for r in reqs:
        s = Solver(r.params, T=r.T, C=r.C, precision="fp32")
        s.set_graph_chunk(0)
        s.set_steps_per_launch(1)
        n = 0
        while True:
            s.step(10 * a.chunk)
            n += 10 * a.chunk
            ob = s.observables()
            if converged(ob, 1e-8, 1e-12 * max(s.derived()["U"], 1e-30)) or ob["nonfinite"] or n >= cap:
                break
        steps_alone[r.id] = n
        node_steps += s.nx * s.ny * n
        s.close()
        print("one-by-one", r.id, n, round(time.perf_counter() - t0, 1), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"metric": "aggregate MLUPS to steady state, batched vs one-by-one", "unit": "MLUPS",
           "cavities": len(reqs), "step_cap": cap, "tol": 1e-8, "data": "synthetic",
           "batched": round(summ["aggregate_MLUPS"], 1), "batched_wall_s": round(summ["wall_s"], 2),
           "one_by_one_plain": round(node_steps / dt / 1e6, 1), "one_by_one_wall_s": round(dt, 2),
           "converged": summ["converged"], "same_stopping_step": steps_alone == steps_batched}
    out["value"] = out["batched"]
    out["speedup"] = round(out["batched"] / out["one_by_one_plain"], 3)
    print(json.dumps(out), flush=True)


def serve(a):
    """Poisson stream of solve requests (square sides 128/256/512/1024 with p = 0.4/0.3/0.2/0.1,
    parameters drawn as in the sweep, FP32 or FP16 storage 50/50), admitted by device
    footprint under a 200 GB budget, advanced together until the K-step velocity residual
    falls below 1e-8 or the step cap; p50/p99 time-to-solution, aggregate MLUPS, and the
    Nu/Sh error of sampled requests against the FP64 oracle."""
    import torch
    import workloads
    from paper_1708_07525_amd.serving import Request, Server

    def build(stream):
        out = []
        for r in stream:
            T, C = workloads.cavity_fields(r)
            out.append(Request(r["id"], r["arrival"], r["params"], r["precision"], None, T, C))
        return out

    budget = 200 * 10 ** 9
    # closed-loop capacity with everything arriving at once, to set the arrival rate
    cal = build(workloads.request_stream(count=max(8, a.requests // 4), seed=40, rate=1e9))
    cap = a.max_steps or 100000
    def note(d):
        print("progress", json.dumps(d), file=sys.stderr, flush=True)

    srv = Server(budget, max_slots=256, chunk=a.chunk, check_every=10 * a.chunk, tol=1e-8, max_steps=cap,
                 autotune_steps=24)
    _, cs = srv.run(cal, progress=note)
    srv.close()
    capacity = cs["requests"] / cs["wall_s"]
    rate = 0.8 * capacity
    reqs = build(workloads.request_stream(count=a.requests, seed=4, rate=rate))
    srv = Server(budget, max_slots=256, chunk=a.chunk, check_every=10 * a.chunk, tol=1e-8, max_steps=cap,
                 autotune_steps=24)
    results, summ = srv.run(reqs, progress=note)
    srv.close()
    torch.cuda.synchronize()
    out = {"metric": "batched p50/p99 solve latency and aggregate MLUPS (continuous batching)",
           "unit": "s", "value": round(summ["p50_s"], 4), "p50_s": round(summ["p50_s"], 4),
           "p99_s": round(summ["p99_s"], 4), "aggregate_MLUPS": round(summ["aggregate_MLUPS"], 1),
           "requests": summ["requests"], "converged": summ["converged"], "rate_per_s": round(rate, 3),
           "closed_loop_capacity_per_s": round(capacity, 3), "step_cap": cap, "tol": 1e-8,
           "higher_is_better": False, "data": "synthetic"}
    # per precision: converged count, time-to-solution of the converged requests, the residual
    # reached by the others, and the slowest diffusive time L^2 max(sigma/alpha_e, phi/D_e) of
    # the scalars (in steps), which sets how long a request needs to settle
    from paper_1708_07525_amd import lbm as _l
    by_id = {r.id: r for r in reqs}

    def pct(v, q):
        return float(f"{np.percentile(v, q):.4g}") if len(v) else None

    def t_slow(req):
        d = _l.derive(req.params, req.precision)
        return d["L"] ** 2 * max(req.params.get("sigma", 1.0) / d["alpha_e"], req.params.get("phi", 1.0) / d["D_e"])

    out["by_precision"] = {}
    for prec in ("fp32", "fp16s"):
        rs = [r for r in results if r.precision == prec]
        conv = [r for r in rs if r.converged]
        rest = [r for r in rs if not r.converged]
        out["by_precision"][prec] = dict(
            requests=len(rs), converged=len(conv),
            converged_p50_s=pct([r.latency for r in conv], 50), converged_p99_s=pct([r.latency for r in conv], 99),
            converged_steps_p50=pct([r.steps for r in conv], 50),
            unconverged_r_u_p10_p50_p90=[pct([r.obs["r_u"] for r in rest], q) for q in (10, 50, 90)],
            t_slow_steps_p50_converged=pct([t_slow(by_id[r.id]) for r in conv], 50),
            t_slow_steps_p50_unconverged=pct([t_slow(by_id[r.id]) for r in rest], 50))
    if a.oracle_samples > 0:
        import oracle
        errs = []
        small = sorted((r for r in results if r.nodes <= 256 * 256), key=lambda r: (r.nodes, r.id))
        # the smallest requests of each storage precision, alternating
        by_prec = [[r for r in small if r.precision == q] for q in ("fp32", "fp16s")]
        picks = [r for pair in zip(*by_prec) for r in pair]
        for res in picks[:a.oracle_samples]:
            req = by_id[res.id]
            o = oracle.Oracle(req.params, T=req.T, C=req.C)
            o.step(res.steps)
            ob = o.observables()
            errs.append({"id": res.id, "precision": res.precision, "steps": res.steps, "nodes": res.nodes,
                         "Nu_rel_err": abs(res.obs["Nu"][0] - ob["Nu"][0]) / abs(ob["Nu"][0]),
                         "Sh_rel_err": abs(res.obs["Sh"][0] - ob["Sh"][0]) / abs(ob["Sh"][0])})
        out["oracle_samples"] = errs
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}): the library has no sharded lattice; "
              "independent cavities would be placed on GPUs by footprint, one process per GPU",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads

    torch.cuda.set_device(0)
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    if a.workload == "sweep":
        sweep(a)
        return
    if a.workload == "serve":
        serve(a)
        return
    if a.workload == "precision":
        precision_report(a)
        return
    case = workloads.band_cavity(seed=2, n=a.n)
    nodes = a.n * a.n
    tile = a.tile if a.tile in ("auto", "default") else tuple(int(v) for v in a.tile.split(","))
    ms, wall, ob, tile_used = timed_run(case, a.precision, a.steps, a.warmup, tile,
                                        a.policy if a.policy >= 0 else None, a.spl, a.strip, a.rows)
    mlups = nodes * a.steps / (ms * 1e-3) / 1e6
    spl = tile_used[3]
    rf = roofline_fields(a.precision, nodes, ms / a.steps, spl)
    kernel = {2: "step2_kernel", 3: "step3_kernel"}.get(spl, "step_kernel")
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
                   "nx": a.n, "ny": a.n, "precision": a.precision, "tile": tile_used[:2],
                   "cache_policy": tile_used[2], "steps_per_launch": tile_used[3], "strip_width": tile_used[4],
                   "tile_rows": tile_used[5],
                   "launch_shape": "autotuned" if tile == "auto" else str(a.tile)},
        "roofline": {"bound": "hbm", "achieved": rf["achieved"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": rf["frac"],
                     "traffic": profiled_traffic(a.precision, a.n, tile_used), "traffic_unit": "bytes/launch",
                     "kernel": kernel, "steps_per_launch": spl, "launch_us": rf["launch_us"],
                     "algorithmic_bytes_per_launch": BYTES_PER_LU[a.precision] * nodes,
                     "bytes_per_node_and_launch": BYTES_PER_LU[a.precision],
                     "effective_per_step_GB_s": rf["effective_per_step_GB_s"],
                     "effective_per_step_frac": rf["effective_per_step_frac"]},
        "wall_s": round(wall, 3),
        "Nu_hot": ob["Nu"][0], "Sh_hot": ob["Sh"][0],
    }
    # the measured HBM traffic of a launch (rocprofv3 counters, when they match this kernel and
    # launch) over the launch's time from the timed region: the real bandwidth the kernel draws
    # the same launch against what a plain copy reaches on this GPU (1 GiB, read + write)
    _, copy_gbs = copy_rate(1024)
    out["roofline"]["copy_ceiling_GB_s"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_copy_ceiling"] = round(rf["achieved"] / copy_gbs, 4)
    tr = out["roofline"]["traffic"]
    if tr is not None:
        launch_s = rf["launch_us"] * 1e-6
        out["roofline"]["traffic_GB_s"] = round(tr / launch_s / 1e9, 1)
        out["roofline"]["traffic_frac"] = round(tr / launch_s / 1e9 / PEAK_HBM_GBS, 4)
    if a.variant_steps > 0:
        var = {}
        for prec in ("fp64", "fp32", "fp16s"):
            if prec == a.precision:
                continue
            vms, _, vob, vt = timed_run(case, prec, a.variant_steps, a.warmup, tile)
            v = nodes * a.variant_steps / (vms * 1e-3) / 1e6
            vr = roofline_fields(prec, nodes, vms / a.variant_steps, vt[3])
            var[prec] = {"MLUPS": round(v, 1), "GB_s": vr["achieved"], "frac": vr["frac"],
                         "effective_per_step_frac": vr["effective_per_step_frac"], "steps": a.variant_steps,
                         "tile": vt[:2], "cache_policy": vt[2], "steps_per_launch": vt[3], "strip_width": vt[4],
                         "tile_rows": vt[5]}
        out["precisions"] = var
        # the same cavity with the walls through the boundary nodes (Eqs. 33-37): the boundary
        # rule inside the tiles (two steps per launch) or perimeter work-groups (one step);
        # per-node bytes as above (the rule's second pull is 0.2% of the nodes)
        nee = dict(case, params=dict(case["params"], sides=("nee_hot", "nee_cold", "nee_adiabatic", "nee_adiabatic")))
        vms, _, vob, vt = timed_run(nee, a.precision, a.variant_steps, a.warmup, tile)
        v = nodes * a.variant_steps / (vms * 1e-3) / 1e6
        vr = roofline_fields(a.precision, nodes, vms / a.variant_steps, vt[3])
        out["node_walls"] = {"MLUPS": round(v, 1), "GB_s": vr["achieved"], "frac": vr["frac"],
                             "effective_per_step_frac": vr["effective_per_step_frac"], "steps": a.variant_steps,
                             "tile": vt[:2], "cache_policy": vt[2], "steps_per_launch": vt[3], "strip_width": vt[4],
                             "precision": a.precision, "Nu_hot": vob["Nu"][0]}
        # the 512^2 Gaussian-random-field cavity (FP32): its 53 MB stay in the 256 MB Infinity
        # Cache, so its bytes per second are not HBM bandwidth; the HBM roofline is quoted at
        # 2048^2 only
        grf = workloads.grf_cavity(seed=1, n=512)
        gn = 512 * 512
        vms, _, vob, vt = timed_run(grf, "fp32", 4 * a.variant_steps, a.warmup, tile)
        v = gn * 4 * a.variant_steps / (vms * 1e-3) / 1e6
        out["grf512"] = {"MLUPS": round(v, 1), "precision": "fp32", "steps": 4 * a.variant_steps, "tile": vt[:2],
                         "cache_policy": vt[2], "steps_per_launch": vt[3], "Nu_hot": vob["Nu"][0],
                         "note": "cache-resident lattice (53 MB): rate is not HBM-bound"}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
