#!/usr/bin/env python3
"""Benchmark of the PERKS hot path on one MI355X.

One bench step = one pass of the stencil sweep: 2D 5-point and 9-point box on
3072^2 and 3D 7-point on 256^3, each in FP64 and FP32, 1000 Jacobi steps per
case, every case ONE persistent kernel launch.  The per-step-launch baseline
(one launch per Jacobi step) is timed on the same inputs, outside the timed
region.  Conjugate gradient (7-point Poisson 128^3, FP64, to 1e-10 relative
residual) is timed the same way, persistent vs host-looped, when the library
exports it.  Inputs are seeded synthetic grids / matrices already resident in
HBM when timing starts.

Prints ONE JSON line on stdout (details go to stderr).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

STENCIL_STEPS = 1000
CASES = [
    ("2d5pt", (3072, 3072), "float64"),
    ("2d5pt", (3072, 3072), "float32"),
    ("2d9pt", (3072, 3072), "float64"),
    ("2d9pt", (3072, 3072), "float32"),
    ("3d7pt", (256, 256, 256), "float64"),
    ("3d7pt", (256, 256, 256), "float32"),
]
FLOPS_PER_CELL = {"2d5pt": 10, "2d9pt": 18, "3d7pt": 14}
PEAK_TFLOPS = {"float64": 78.6, "float32": 157.3}   # MI355X vector FP64 / FP32
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def interior(shape):
    return math.prod(s - 2 for s in shape)


def cpu_baseline(target_s=10.0):
    """The oracle (single thread) on a bounded sample of the 2d5pt 3072^2 FP64 case."""
    import numpy as np

    import oracle
    import workloads
    g = workloads.stencil_grid((3072, 3072), seed=0)
    w = workloads.stencil_weights("2d5pt")
    t0 = time.perf_counter()
    g = oracle.stencil(g, w, 1)
    one = time.perf_counter() - t0
    k = max(1, min(40, int(target_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    oracle.stencil(g, w, k)
    dt = time.perf_counter() - t0
    cells = interior((3072, 3072)) * k
    return {"value": cells / dt / 1e9, "unit": "GCells/s", "cores": 1, "kind": "oracle",
            "sample": f"2d5pt 3072^2 FP64, {k} Jacobi steps ({dt:.1f} s), single thread"}


def bench_cg(pk, torch, args):
    """CG time-to-tolerance, persistent vs host-looped, FP64, x0 = 0."""
    import numpy as np

    import workloads
    systems = [("poisson3d 128^3", lambda: workloads.poisson_csr(128, 3))]
    if args.cg_random:
        systems.append(("random SPD n=1M lognormal(12,1)", lambda: workloads.random_spd_csr(1 << 20, seed=0)))
    out = []
    for name, make in systems:
        rp, ci, v = make()
        n = rp.size - 1
        A = pk.CsrMatrix(rp, ci, v)
        b = torch.from_numpy(workloads.rhs_uniform(n, seed=0)).cuda()
        for tol in (1e-10, 1e-8):
            rec = {"system": name, "n": int(n), "nnz": int(ci.size), "tol": tol}
            for label, fn in (("persistent", pk.cg_solve), ("baseline", pk.cg_solve_baseline)):
                x = torch.zeros(n, dtype=torch.float64, device="cuda")
                fn(A, b, x, tol=tol, maxit=5000)               # warm-up (allocations, caches)
                times = []
                for _ in range(max(1, min(args.steps, 3))):
                    x.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    info = fn(A, b, x, tol=tol, maxit=5000)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                t = float(np.median(times))
                rec[label] = {"seconds": t, "iters": info["iters"], "us_per_iter": t / max(1, info["iters"]) * 1e6,
                              "relres_true": info["relres_true"], "status": info["status"]}
            rec["speedup"] = rec["baseline"]["seconds"] / rec["persistent"]["seconds"]
            log(f"CG {name} tol {tol:.0e}: persistent {rec['persistent']['seconds']*1e3:.2f} ms "
                f"({rec['persistent']['iters']} it, {rec['persistent']['us_per_iter']:.1f} us/it)  baseline "
                f"{rec['baseline']['seconds']*1e3:.2f} ms ({rec['baseline']['iters']} it)  x{rec['speedup']:.2f}")
            out.append(rec)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-baseline", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cases", default="all")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--cg-random", action="store_true", help="also the n=1M random SPD system")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the method and this "
              "library are single-GPU; see DESIGN.md for how the path would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2204_02064_amd as pk
    import workloads

    pk.lib()
    dev = torch.device("cuda:0")
    cases = CASES if args.cases == "all" else [c for c in CASES if c[0] in args.cases.split(",")]
    grids = []
    for kind, shape, dt in cases:
        g = workloads.stencil_grid(shape, seed=0).astype(np.float64 if dt == "float64" else np.float32)
        grids.append(torch.from_numpy(g).to(dev))
    weights = {k: workloads.stencil_weights(k) for k in FLOPS_PER_CELL}
    stream = torch.cuda.current_stream()

    def run_case(i, baseline=False):
        kind, shape, dt = cases[i]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if baseline:
            pk.stencil_run_baseline(grids[i], weights[kind], STENCIL_STEPS)
        else:
            pk.stencil_run(grids[i], weights[kind], STENCIL_STEPS)
        e1.record(stream)
        return e0, e1

    for _ in range(args.warmup):
        for i in range(len(cases)):
            run_case(i)
    torch.cuda.synchronize()

    per_case = [[] for _ in cases]
    t_start = time.perf_counter()
    for _ in range(args.steps):
        evs = [run_case(i) for i in range(len(cases))]
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(evs):
            per_case[i].append(a.elapsed_time(b) / 1e3)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    results = []
    total_cells, total_time = 0, 0.0
    for i, (kind, shape, dt) in enumerate(cases):
        t = float(np.median(per_case[i]))
        cells = interior(shape) * STENCIL_STEPS
        total_cells += cells * args.steps
        total_time += sum(per_case[i])
        plan = pk.stencil_plan(shape, weights[kind], dt)
        results.append({"case": f"{kind} {'x'.join(map(str, shape))} {dt}", "kind": kind, "dtype": dt,
                        "persistent_ms": t * 1e3, "persistent_gcells": cells / t / 1e9,
                        "launch_us": None, "plan": plan})

    if not args.no_baseline:
        for i, r in enumerate(results):
            a, b = run_case(i, baseline=True)
            torch.cuda.synchronize()
            tb = a.elapsed_time(b) / 1e3
            cells = interior(cases[i][1]) * STENCIL_STEPS
            r["baseline_ms"] = tb * 1e3
            r["baseline_gcells"] = cells / tb / 1e9
            r["speedup"] = r["persistent_gcells"] / r["baseline_gcells"]

    for r in results:
        log(f"{r['case']:28s} persistent {r['persistent_gcells']:8.1f} GCells/s"
            + (f"  baseline {r['baseline_gcells']:8.1f} GCells/s  x{r['speedup']:.2f}" if "speedup" in r else "")
            + f"  plan R={r['plan']['rows_per_lane']} cached {r['plan']['cached_tiles']}/{r['plan']['tiles']}")

    # dominant kernel (largest share of the timed region) -> roofline entry
    dom = max(range(len(results)), key=lambda i: results[i]["persistent_ms"])
    kind, shape, dt = cases[dom]
    t_dom = results[dom]["persistent_ms"] / 1e3
    flops = FLOPS_PER_CELL[kind] * interior(shape) * STENCIL_STEPS
    achieved = flops / t_dom / 1e12
    roofline = {"bound": "alu", "kernel": f"stencil{len(shape)}d_persistent {results[dom]['case']}",
                "achieved": achieved, "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS[dt], "traffic": None}

    value = total_cells / total_time / 1e9
    out = {
        "metric": "stencil GCells/s + CG s-to-1e-8 resid: persistent vs per-step launch, 1 GPU",
        "value": value,
        "unit": "GCells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_time / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic (seeded U[0,1) grids, zero Dirichlet ring)",
        "config": {"workload": "stencil sweep: 2d5pt + 2d9pt-box 3072^2, 3d7pt 256^3; FP64 and FP32; "
                               "1000 Jacobi steps per case, one persistent launch each",
                   "stencil_steps": STENCIL_STEPS, "parallelism": "1 GPU"},
        "cases": results,
        "roofline": roofline,
        "wall_s": wall,
    }
    if not args.no_baseline:
        base_time = sum(r["baseline_ms"] for r in results) / 1e3
        out["baseline_value"] = sum(interior(c[1]) * STENCIL_STEPS for c in cases) / base_time / 1e9
        out["speedup_vs_per_step_launch"] = value / out["baseline_value"]
    if not args.no_cg:
        out["cg"] = bench_cg(pk, torch, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
