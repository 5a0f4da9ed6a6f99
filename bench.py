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

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0: the factors a 1 GiB device
# copy reads back), with one SHA-256 over the source files the kernel is built
# from: a changed source reports null until measured again.
MEASURED_TRAFFIC = {
    ("3d7pt", (256, 256, 256), "float64"): {
        "bytes": 190.31e9,   # profiles/stencil3d_column_f64_256cubed.md
        "sources": ["paper_2204_02064_amd/csrc/stencil3d.hpp", "paper_2204_02064_amd/csrc/barrier.hpp",
                    "paper_2204_02064_amd/csrc/common.hpp", "paper_2204_02064_amd/csrc/stencil3d_f64.hip"],
        "sha256": "57bf5d50dba114748affa16306a451bdd0efd4c69033d4b4bf424a55a1a3c591",
    },
}


# Fabric bytes per Jacobi step (FETCH_SIZE x2 + WRITE_SIZE x1, rocprofv3
# --pmc) of the persistent launch and of the per-step baseline, default plans
# (profiles/stencil_hbm_traffic_persistent_vs_per_step.md); reported while the
# kernels' sources are unchanged (null otherwise).
_CSRC = "paper_2204_02064_amd/csrc/"
_SRC2 = [_CSRC + "stencil2d_wide.hpp", _CSRC + "barrier.hpp", _CSRC + "common.hpp"]
_SRC3 = [_CSRC + "stencil3d.hpp", _CSRC + "barrier.hpp", _CSRC + "common.hpp"]
STEP_TRAFFIC = {
    ("2d5pt", "float64"): {"persistent": 20.0e6, "per_step": 174.4e6,
                           "sources": [_CSRC + "stencil2d_tb.hip"] + _SRC2 + [_CSRC + "stencil2d_wide_f64.hip"],
                           "sha256": "91f7ef17091b0d3c5aee6f93a7e84c2da4fb0787205164a6c13dbde7369d6aa8"},
    ("2d5pt", "float32"): {"persistent": 14.7e6, "per_step": 92.8e6,
                           "sources": [_CSRC + "stencil2d_tb.hip"] + _SRC2 + [_CSRC + "stencil2d_wide_f32.hip"],
                           "sha256": "4a9cc640085b58e073036b3431295137e76da1cb4781bfea188170d613ad0e36"},
    ("3d7pt", "float64"): {"persistent": 190.3e6, "per_step": 407.5e6, "sources": _SRC3 + [_CSRC + "stencil3d_f64.hip"],
                           "sha256": "57bf5d50dba114748affa16306a451bdd0efd4c69033d4b4bf424a55a1a3c591"},
    ("3d7pt", "float32"): {"persistent": 29.0e6, "per_step": 215.6e6, "sources": _SRC3 + [_CSRC + "stencil3d_f32.hip"],
                           "sha256": "0710262a0734a41ba516abc125917221919a59ce7295c236d3155cb1b456f833"},
}


def sources_digest(paths):
    """SHA-256 over the named files (repository-relative), in order."""
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for rel in paths:
        with open(os.path.join(root, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(case):
    m = MEASURED_TRAFFIC.get(case)
    if not m or m["bytes"] is None:
        return None
    try:
        digest = sources_digest(m["sources"])
    except OSError:
        return None
    return m["bytes"] if digest == m["sha256"] else None


def step_traffic():
    """Measured fabric bytes per Jacobi step, persistent vs per-step launch
    (STEP_TRAFFIC), for the cases whose kernel sources are unchanged."""
    out = {}
    for (kind, dt), m in STEP_TRAFFIC.items():
        try:
            ok = sources_digest(m["sources"]) == m["sha256"]
        except OSError:
            ok = False
        key = f"{kind} {dt}"
        out[key] = ({"persistent_bytes": m["persistent"], "per_step_bytes": m["per_step"],
                     "reduction": m["per_step"] / m["persistent"]} if ok else None)
    return {"unit": "fabric bytes per Jacobi step (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1)", "cases": out,
            "source": "profiles/stencil_hbm_traffic_persistent_vs_per_step.md"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def interior(shape):
    return math.prod(s - 2 for s in shape)


def _host_cpu():
    """(threads this process may run on, CPU model string)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def cpu_baseline(target_s=10.0):
    """The oracle on a bounded sample of the 2d5pt 3072^2 FP64 case, run twice:
    single-threaded and with its rows shared by every host core this process
    may use (same arithmetic).  Each leg runs as many Jacobi steps as take
    about target_s (per-step time from a 2-step run).  The reported value is
    the all-core leg."""
    import oracle
    import workloads
    cores, model = _host_cpu()
    g = workloads.stencil_grid((3072, 3072), seed=0)
    w = workloads.stencil_weights("2d5pt")
    legs = {}
    for threads in (1, cores):
        t0 = time.perf_counter()
        oracle.stencil(g, w, 2, threads=threads)
        one = (time.perf_counter() - t0) / 2
        k = max(1, min(1000, int(target_s / max(one, 1e-4))))
        t0 = time.perf_counter()
        oracle.stencil(g, w, k, threads=threads)
        dt = time.perf_counter() - t0
        legs[threads] = (interior((3072, 3072)) * k / dt / 1e9, k, dt)
    v, k, dt = legs[cores]
    v1, k1, dt1 = legs[1]
    return {"value": v, "unit": "GCells/s", "cores": cores, "kind": "oracle",
            "sample": f"2d5pt 3072^2 FP64, {k} Jacobi steps ({dt:.1f} s) on {cores} threads; "
                      f"single thread {v1:.3f} GCells/s ({k1} steps, {dt1:.1f} s)",
            "single_thread_value": v1, "cpu_model": model}


def _time(fn, torch, reps):
    """Median wall time of fn() over reps runs (each bracketed by device syncs)."""
    import numpy as np
    ts = []
    out = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), out


def bench_cg(pk, torch, args):
    """CG time-to-tolerance, persistent vs host-looped, x0 = 0.

    FP64 to 1e-10 and 1e-8, and mixed precision (one FP32 recurrence with
    FP64 residual replacement) to 1e-8, on the 7-point Poisson 128^3 system
    and (unless --no-cg-random) the n=1M random SPD system, the latter
    Jacobi-preconditioned; and the random system as configured, FP64
    unpreconditioned to 1e-10 with maxit 5000, which does not converge: its
    record gives the residual reached and the time of the 5000 iterations.
    """
    import workloads
    systems = [("poisson3d 128^3", lambda: workloads.poisson_csr(128, 3), None)]
    if not args.no_cg_random:
        systems.append(("random SPD n=1M lognormal(12,1)", lambda: workloads.random_spd_csr(1 << 20, seed=0),
                        "jacobi"))
    out = []
    reps = max(1, min(args.steps, 3))
    for name, make, precond in systems:
        rp, ci, v = make()
        n = rp.size - 1
        A = pk.CsrMatrix(rp, ci, v)
        b = torch.from_numpy(workloads.rhs_uniform(n, seed=0)).cuda()
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        runs = [(1e-10, None, precond, reps), (1e-8, None, precond, reps), (1e-8, "mixed", precond, reps)]
        if precond is not None:
            runs.append((1e-10, None, None, 1))   # as configured: unpreconditioned, maxit 5000
        for tol, precision, pc, nrep in runs:
            rec = {"system": name, "n": int(n), "nnz": int(ci.size), "tol": tol, "precond": pc,
                   "precision": precision or "f64"}
            for label, fn in (("persistent", pk.cg_solve), ("baseline", pk.cg_solve_baseline)):
                def run():
                    x.zero_()
                    return fn(A, b, x, tol=tol, maxit=5000, precond=pc, precision=precision)
                run()                                          # warm-up (allocations, caches)
                t, info = _time(run, torch, nrep)
                rec[label] = {"seconds": t, "iters": info["iters"], "us_per_iter": t / max(1, info["iters"]) * 1e6,
                              "relres_true": info["relres_true"], "status": info["status"],
                              "outer": info.get("outer")}
                if label == "persistent":
                    bs = pk.barrier_stats()
                    rec[label]["barrier"] = {"wait_share": bs["wait_share"],
                                             "barriers_per_workgroup": bs["barriers"],
                                             "wait_cycles_per_barrier": bs["wait_cycles"] / max(1, bs["barriers"])}
            rec["speedup"] = rec["baseline"]["seconds"] / rec["persistent"]["seconds"]
            log(f"CG {name} {rec['precision']} precond {pc} tol {tol:.0e}: persistent "
                f"{rec['persistent']['seconds']*1e3:.2f} ms [{rec['persistent']['status']}, relres "
                f"{rec['persistent']['relres_true']:.1e}] "
                f"({rec['persistent']['iters']} it, {rec['persistent']['us_per_iter']:.1f} us/it)  baseline "
                f"{rec['baseline']['seconds']*1e3:.2f} ms ({rec['baseline']['iters']} it)  x{rec['speedup']:.2f}")
            out.append(rec)
    return out


def bench_small(pk, torch, args):
    """The 256^2 FP64 2d5pt case, 100 Jacobi steps (zero ring, U[0,1) seed 0):
    latency-bound, so microseconds per step: the persistent kernel (untuned
    plan: the temporally blocked kernel, a grid barrier every 8 steps; also
    the radius-1 kernel with point-to-point halo words every step and the
    radius-2..4 family with a device barrier every step) vs one launch per
    step.  HIP events on the launch stream, median of repeated runs."""
    import numpy as np
    import workloads
    steps, shape = 100, (256, 256)
    w = workloads.stencil_weights("2d5pt")
    g = torch.from_numpy(workloads.stencil_grid(shape, seed=0)).cuda()
    stream = torch.cuda.current_stream()
    reps = max(5, min(args.steps, 20))

    def timed(fn):
        fn()
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1) * 1e3 / steps)
        return float(np.median(out))

    rec = {"workload": "2d5pt 256x256 FP64, 100 steps", "steps": steps,
           "persistent_us_per_step": timed(lambda: pk.stencil_run(g, w, steps)),
           "persistent_point_to_point_kernel_us_per_step": timed(lambda: pk.stencil_run(g, w, steps,
                                                                                         tuning={"kernel": 1})),
           "persistent_barrier_kernel_us_per_step": timed(lambda: pk.stencil_run(g, w, steps, tuning={"kernel": 2})),
           "baseline_us_per_step": timed(lambda: pk.stencil_run_baseline(g, w, steps)),
           "plan": pk.stencil_plan(shape, w, "float64")}
    rec["speedup"] = rec["baseline_us_per_step"] / rec["persistent_us_per_step"]
    log(f"2d5pt 256^2 FP64 100 steps: persistent {rec['persistent_us_per_step']:.2f} us/step "
        f"(point-to-point kernel {rec['persistent_point_to_point_kernel_us_per_step']:.2f}, device-barrier kernel "
        f"{rec['persistent_barrier_kernel_us_per_step']:.2f}), per-step launches "
        f"{rec['baseline_us_per_step']:.2f} us/step  x{rec['speedup']:.2f}")
    return rec


WIDE_FLOPS = {"2ds9pt": 18, "2d13pt": 26, "2d17pt": 34, "2d25pt": 50,
              "3d13pt": 26, "3d17pt": 34, "3d27pt": 54, "poisson": 38}


def bench_wide(pk, torch, args):
    """The rest of tab:domain's suite: the 2D stars of radius 2, 3, 4 and the
    radius-2 box at 3072^2, the 3D radius-2 star, 17-, 27- and 19-point
    stencils at 256^3; FP64 and FP32, 1000 steps: persistent (default plan)
    vs one launch per step."""
    import numpy as np
    import workloads
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = []
    # (the radius-1 3D box patterns are disabled in the library)
    for kind in workloads.WIDE_KINDS + tuple(k for k in workloads.WIDE3_KINDS if workloads.stencil_radius(k) == 2):
        r = workloads.stencil_radius(kind)
        w = workloads.stencil_weights(kind)
        shape = (3072, 3072) if kind.startswith("2d") else (256, 256, 256)
        cells = math.prod(s - 2 * r for s in shape) * STENCIL_STEPS
        label = "x".join(map(str, shape))
        for dt in ("float64", "float32"):
            g = torch.from_numpy(workloads.stencil_grid(shape, seed=0, r=r).astype(dt)).to(dev)

            def timed(fn):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / 1e3

            pk.stencil_run(g, w, 100)
            tp = float(np.median([timed(lambda: pk.stencil_run(g, w, STENCIL_STEPS)) for _ in range(max(1, args.steps))]))
            tb = timed(lambda: pk.stencil_run_baseline(g, w, STENCIL_STEPS))
            plan = pk.stencil_plan(shape, w, dt)
            flops = WIDE_FLOPS[kind] * cells / tp / 1e12
            peak = PEAK_TFLOPS[dt]
            out.append({"case": f"{kind} {label} {dt}", "persistent_ms": tp * 1e3,
                        "persistent_gcells": cells / tp / 1e9, "baseline_ms": tb * 1e3,
                        "baseline_gcells": cells / tb / 1e9, "speedup": tb / tp, "tflops": flops,
                        "alu_frac": flops / peak, "plan": plan})
            log(f"{kind} {label} {dt:8s} persistent {cells / tp / 1e9:8.1f} GCells/s ({flops:5.1f} TFLOP/s, "
                f"{flops / peak:.2f} of vector peak)  baseline {cells / tb / 1e9:8.1f} GCells/s  x{tb / tp:.2f}  "
                f"plan R={plan['rows_per_lane']} cached {plan['cached_tiles']}/{plan['tiles']}")
            del g
    return out


def bench_batched_stencil(pk, torch, args):
    """512 2D 5-point FP64 grids, sides round(exp(U[ln 64, ln 1024])), 100 Jacobi
    steps each: one batched persistent launch (the one-shot call, and the same
    launch as a reusable plan) vs one persistent launch per grid vs one launch
    per step per grid (HIP events on the current stream)."""
    import numpy as np

    import workloads
    count, steps = args.batch_count, 100
    sides = workloads.lognormal_sides(count, seed=0)
    w = workloads.stencil_weights("2d5pt")
    grids = [torch.from_numpy(workloads.stencil_grid((int(n), int(n)), seed=j)).cuda() for j, n in enumerate(sides)]
    cells = sum(interior((int(n), int(n))) for n in sides) * steps
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()                                   # warm-up (plans, scratch)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    t_batch = timed(lambda: pk.stencil_run_batched(grids, w, steps))
    plan = pk.StencilBatch(grids, w, steps)    # the same launch as a reusable plan (graph launch)
    t_plan = timed(plan.run)
    graph = plan.has_graph()
    plan.close()
    t_seq = timed(lambda: [pk.stencil_run(g, w, steps) for g in grids])
    t_base = timed(lambda: [pk.stencil_run_baseline(g, w, steps) for g in grids])
    log(f"batched stencil: {count} 2d5pt FP64 grids ({cells / steps / 1e6:.1f}M cells), {steps} steps: one launch "
        f"{t_batch * 1e3:.2f} ms ({cells / t_batch / 1e9:.1f} GCells/s; as a plan {t_plan * 1e3:.2f} ms, graph "
        f"{graph}) | per-grid persistent {t_seq * 1e3:.2f} ms "
        f"(x{t_seq / t_batch:.2f}) | per-step launches {t_base * 1e3:.2f} ms (x{t_base / t_batch:.2f})")
    return {"grids": count, "steps": steps, "cells": int(cells // steps), "batched_ms": t_batch * 1e3,
            "batched_gcells": cells / t_batch / 1e9, "plan_run_ms": t_plan * 1e3, "plan_graph": graph,
            "per_grid_persistent_ms": t_seq * 1e3,
            "per_step_launch_ms": t_base * 1e3, "speedup_vs_per_grid": t_seq / t_batch,
            "speedup_vs_per_step": t_base / t_batch}


def bench_batched(pk, torch, args):
    """512 independent 2D 5-point Poisson systems, sides round(exp(U[ln 64, ln 1024])),
    rhs N(0,1), mixed precision to 1e-8 each: one batched persistent launch vs the
    same systems solved one after another by the single-system persistent solver
    (and, with --batched-baseline, by the host-looped baseline)."""
    import numpy as np

    import workloads
    count = args.batch_count
    sides = workloads.lognormal_sides(count, seed=0)
    As, bs, xs = [], [], []
    cache = {}
    for j, s in enumerate(sides):
        s = int(s)
        if s not in cache:
            cache[s] = pk.CsrMatrix(*workloads.poisson2d_csr_torch(s, device="cuda"))
        As.append(cache[s])
        g = torch.Generator(device="cuda").manual_seed(j)
        bs.append(torch.randn(s * s, generator=g, device="cuda", dtype=torch.float64))
        xs.append(torch.zeros(s * s, device="cuda", dtype=torch.float64))
    n_total = int(sum(int(s) ** 2 for s in sides))
    nnz_total = int(sum(A.nnz for A in As))
    tol, maxit = 1e-8, 20000
    plan = pk.CgBatch(As, bs, xs, tol=tol, maxit=maxit, precision="mixed")

    def run_batch():
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run()
        infos = plan.results()
        return time.perf_counter() - t0, infos

    run_batch()
    t_batch, infos = run_batch()
    ok = sum(1 for i in infos if i["status"] == "converged")
    worst = max(i["relres_true"] for i in infos)
    rec = {"workload": f"{count} x 2D 5-point Poisson, sides log-uniform [64,1024] (seed 0), rhs N(0,1), "
                       f"mixed precision to {tol:.0e}", "n_total": n_total, "nnz_total": nnz_total,
           "batched_s": t_batch, "converged": ok, "worst_relres_true": worst,
           "max_iters": max(i["iters"] for i in infos), "graph": plan.has_graph()}
    # sequential single-system persistent solves of the same systems
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_ok = 0
    for A, b, x in zip(As, bs, xs):
        info = pk.cg_solve(A, b, x, tol=tol, maxit=maxit, precision="mixed")
        seq_ok += info["status"] == "converged"
    torch.cuda.synchronize()
    rec["sequential_persistent_s"] = time.perf_counter() - t0
    rec["speedup_vs_sequential"] = rec["sequential_persistent_s"] / t_batch
    if args.batched_baseline:
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for A, b, x in zip(As, bs, xs):
            pk.cg_solve_baseline(A, b, x, tol=tol, maxit=maxit, precision="mixed")
        torch.cuda.synchronize()
        rec["sequential_baseline_s"] = time.perf_counter() - t0
        rec["speedup_vs_baseline"] = rec["sequential_baseline_s"] / t_batch
    plan.close()
    log(f"batched: {count} systems ({n_total/1e6:.1f}M unknowns) in {t_batch:.3f} s ({ok}/{count} converged, "
        f"worst relres {worst:.2e}); sequential persistent {rec['sequential_persistent_s']:.3f} s "
        f"(x{rec['speedup_vs_sequential']:.2f})"
        + (f"; sequential baseline {rec['sequential_baseline_s']:.3f} s" if "sequential_baseline_s" in rec else ""))
    return rec


def bench_learned(pk, torch, args):
    """Learned preconditioner: train on pairs harvested from the persistent PCG
    on seeded 256^2 diffusion problems (log k a Gaussian random field, sigma 1,
    correlation length 16 cells), then solve held-out problems at 256^2, 512^2
    and 1024^2 to 1e-8 with FCG + network vs persistent Jacobi-PCG."""
    import numpy as np

    import workloads
    from paper_2204_02064_amd import learned
    n_train = args.nn_fields
    t0 = time.perf_counter()
    probs = [workloads.diffusion_problem_torch(256, seed=s) for s in range(n_train)]
    planes = torch.stack([workloads.diffusion_planes_torch(torch.exp(workloads.grf_log_k_torch(256, seed=s)))
                          for s in range(n_train)]).to(torch.float32)
    X, T, field = learned.harvest_pairs(probs, with_field=True)
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    del probs
    t0 = time.perf_counter()
    params, losses = learned.train(X, T, epochs=args.nn_epochs, batch=16, lr=1e-3, seed=0, planes=planes,
                                   field=field)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    rec = {"train_fields": n_train, "pairs": int(X.shape[0]), "harvest_s": t_harvest, "train_s": t_train,
           "loss": "energy norm of the output error (||z - e||_A^2 up to a constant)",
           "epochs": args.nn_epochs, "loss_per_epoch": [float(l) for l in losses], "eval": []}
    del X, T, planes
    log(f"learned: {rec['pairs']} pairs from {n_train} fields in {t_harvest:.1f} s; trained {len(losses)} epochs "
        f"in {t_train:.1f} s, loss per epoch {losses[0]:.3e} -> {losses[-1]:.3e}")
    for n in (256, 512, 1024):
        for s in range(10000, 10000 + args.nn_test):
            rp, ci, v, lk, f = workloads.diffusion_problem_torch(n, seed=s)
            A = pk.CsrMatrix(rp, ci, v)
            x = torch.zeros_like(f)
            e = {"n": n, "seed": s}
            for label, fn in (("jacobi_pcg", lambda: pk.cg_solve(A, f, x, tol=1e-8, maxit=20000, precond="jacobi")),
                              ("fcg_net", lambda: pk.fcg_solve(A, f, x, n, n, params=params, logk=lk, tol=1e-8,
                                                               maxit=20000, stall=args.nn_stall))):
                x.zero_()
                fn()
                t, info = _time(lambda: (x.zero_(), fn())[1], torch, 2)
                e[label] = {"seconds": t, "iters": info["iters"], "status": info["status"],
                            "relres_true": info["relres_true"], "fallbacks": info.get("fallbacks"),
                            "switched_at": info.get("switched_at")}
            e["speedup"] = e["jacobi_pcg"]["seconds"] / e["fcg_net"]["seconds"]
            log(f"learned {n}^2 seed {s}: Jacobi-PCG {e['jacobi_pcg']['iters']} it {e['jacobi_pcg']['seconds']*1e3:.2f} ms"
                f" | FCG+net {e['fcg_net']['iters']} it {e['fcg_net']['seconds']*1e3:.2f} ms "
                f"(fallbacks {e['fcg_net']['fallbacks']}, switched {e['fcg_net']['switched_at']})  x{e['speedup']:.2f}")
            rec["eval"].append(e)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-baseline", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="use the planner's default plans")
    ap.add_argument("--cases", default="all")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the 256^2 100-step latency case")
    ap.add_argument("--no-wide", action="store_true", help="skip the radius-2..4 2D stencils")
    ap.add_argument("--no-cg-random", action="store_true", help="skip the n=1M random SPD system")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched mixed-precision CG")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned preconditioner")
    ap.add_argument("--nn-fields", type=int, default=2000, help="training fields (256^2) for the network")
    ap.add_argument("--nn-epochs", type=int, default=3)
    ap.add_argument("--nn-stall", type=int, default=20,
                    help="FCG iterations without a new residual minimum before it continues as Jacobi-PCG")
    ap.add_argument("--nn-test", type=int, default=2, help="held-out problems per size")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batched-baseline", action="store_true",
                    help="also time the host-looped baseline on every batched system (slow)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device (a plain copy kernel of known traffic, the "
                         "reference for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the library runs each "
              "solve on one GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2204_02064_amd as pk
    import workloads

    pk.lib()
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 1 GiB read + 1 GiB written in {(time.perf_counter() - t0) * 1e3:.3f} ms")
        del src, dst
    cases = CASES if args.cases == "all" else [c for c in CASES if c[0] in args.cases.split(",")]
    grids = []
    for kind, shape, dt in cases:
        g = workloads.stencil_grid(shape, seed=0).astype(np.float64 if dt == "float64" else np.float32)
        grids.append(torch.from_numpy(g).to(dev))
    weights = {k: workloads.stencil_weights(k) for k in FLOPS_PER_CELL}
    stream = torch.cuda.current_stream()
    # autotune each case (outside the timed region); untuned runs then use the winner
    tuned = {}
    if not args.no_autotune:
        for kind, shape, dt in cases:
            t0 = time.perf_counter()
            tuned[(kind, shape, dt)], rate = pk.stencil_autotune(shape, weights[kind], dt, probe_steps=100)
            log(f"autotune {kind} {shape} {dt}: {tuned[(kind, shape, dt)]} ({rate:.1f} GCells/s probe, "
                f"{time.perf_counter() - t0:.1f} s)")

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
    total_cells = {"float64": 0, "float32": 0}
    total_time = {"float64": 0.0, "float32": 0.0}
    for i, (kind, shape, dt) in enumerate(cases):
        t = float(np.median(per_case[i]))
        cells = interior(shape) * STENCIL_STEPS
        total_cells[dt] += cells * args.steps
        total_time[dt] += sum(per_case[i])
        plan = pk.stencil_plan(shape, weights[kind], dt, tuning=tuned.get((kind, shape, dt)))
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

    # barrier clock of each persistent launch (one more untimed run per case)
    for i, r in enumerate(results):
        run_case(i)
        bs = pk.barrier_stats()
        r["barrier"] = {"wait_share": bs["wait_share"], "barriers_per_workgroup": bs["barriers"],
                        "wait_cycles_per_barrier": bs["wait_cycles"] / max(1, bs["barriers"])}

    for r in results:
        log(f"{r['case']:28s} persistent {r['persistent_gcells']:8.1f} GCells/s"
            + (f"  baseline {r['baseline_gcells']:8.1f} GCells/s  x{r['speedup']:.2f}" if "speedup" in r else "")
            + f"  plan R={r['plan']['rows_per_lane']} cached {r['plan']['cached_tiles']}/{r['plan']['tiles']}")

    # dominant kernel (largest share of the timed region) -> roofline entry.
    # A launch whose tiles are all on chip touches HBM only for halos: bound
    # by vector ALU, algorithmic FLOPs per cell update (tab:domain).  With
    # streamed tiles the algorithmic bytes follow Eq. 5: cached cells loaded
    # and stored once, streamed cells read and written every step, plus the
    # halo faces of every step; bound by HBM.
    roofline = None
    if results:
        dom = max(range(len(results)), key=lambda i: results[i]["persistent_ms"])
        kind, shape, dt = cases[dom]
        pl = results[dom]["plan"]
        t_dom = results[dom]["persistent_ms"] / 1e3
        esz = 8 if dt == "float64" else 4
        cells = interior(shape)
        streamed = cells - pl["cached_cells"]
        name = f"{'stencil3d_column' if len(shape) == 3 else 'stencil2d_persistent'} {results[dom]['case']}"
        if streamed == 0:
            flops = FLOPS_PER_CELL[kind] * cells * STENCIL_STEPS
            achieved = flops / t_dom / 1e12
            roofline = {"bound": "alu", "kernel": name, "achieved": achieved, "peak": PEAK_TFLOPS[dt],
                        "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[dt], "traffic": None,
                        "algorithmic": f"{FLOPS_PER_CELL[kind]} FLOP per cell update x {cells} cells x "
                                       f"{STENCIL_STEPS} steps"}
        else:
            nbytes = (2 * pl["cached_cells"] * esz + 2 * STENCIL_STEPS * streamed * esz
                      + STENCIL_STEPS * pl["halo_bytes_per_step"])
            achieved = nbytes / t_dom / 1e9
            traffic = measured_traffic(cases[dom])
            roofline = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "traffic_unit": "bytes per launch",
                        "algorithmic": f"Eq. 5: 2*{pl['cached_cells']} cached + 2*{STENCIL_STEPS}*{streamed} streamed "
                                       f"cells x {esz} B + {STENCIL_STEPS} x {pl['halo_bytes_per_step']} halo B"}

    def rate(dt):
        return total_cells[dt] / total_time[dt] / 1e9 if total_time[dt] > 0 else None

    value = rate("float64")
    out = {
        "metric": "stencil GCells/s + CG s-to-1e-8 resid: persistent vs per-step launch, 1 GPU",
        "value": value,
        "unit": "GCells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_time["float64"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded U[0,1) grids, zero Dirichlet ring)",
        "config": {"workload": "FP64 stencil sweep: 2d5pt + 2d9pt-box 3072^2, 3d7pt 256^3; 1000 Jacobi steps "
                               "per case, one persistent launch each (autotuned plans)",
                   "stencil_steps": STENCIL_STEPS, "parallelism": "1 GPU"},
        "fp32": {"value": rate("float32"), "unit": "GCells/s",
                 "ms_per_step": total_time["float32"] / args.steps * 1e3,
                 "workload": "the same sweep in FP32 (storage and arithmetic), timed in the same loop"},
        "cases": results,
        "roofline": roofline,
        "wall_s": wall,
    }
    if not args.no_baseline and results:
        for dt, key in (("float64", "baseline_value"), ("float32", None)):
            sel = [(r, c) for r, c in zip(results, cases) if c[2] == dt]
            if not sel:
                continue
            base = sum(interior(c[1]) * STENCIL_STEPS for _, c in sel) / (sum(r["baseline_ms"] for r, _ in sel) / 1e3) / 1e9
            if key:
                out[key] = base
                out["speedup_vs_per_step_launch"] = value / base if value else None
            else:
                out["fp32"]["baseline_value"] = base
                out["fp32"]["speedup_vs_per_step_launch"] = out["fp32"]["value"] / base if out["fp32"]["value"] else None
    out["traffic_per_step"] = step_traffic()
    if not args.no_small:
        out["config_256"] = bench_small(pk, torch, args)
    if not args.no_wide:
        out["wide_stencils"] = bench_wide(pk, torch, args)
    if not args.no_cg:
        out["cg"] = bench_cg(pk, torch, args)
    if not args.no_batched:
        out["batched_stencil"] = bench_batched_stencil(pk, torch, args)
        out["batched_cg"] = bench_batched(pk, torch, args)
    if not args.no_learned:
        out["learned_preconditioner"] = bench_learned(pk, torch, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
