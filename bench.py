#!/usr/bin/env python3
"""Throughput of the strongly coupled IB step on one MI355X.

Workload: 1024^2 cells per level, 4 nested levels, one deformable clamped flag
(101 points, mass ratio 0.2, bending stiffness 1e-3), Re 500, sub-domain operator
B' built offline (excluded from the timing, reported as prepare_s).  Metric: grid-cell
steps per second = n^2 * levels * steps / wall time, for the FP32-flow form (value) and
the plain FP64 form (value_fp64), inputs resident in HBM before the timed region.

One JSON line on stdout.  ``--gpus`` above 1 is not supported (one GPU per run).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-cell steps/s (1024², 4 levels) fp32 vs fp64; served p50/p99 latency"
PEAK_HBM = 8.0e12
# HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter passes (each scaled by what the
# counter reads for a 256 MiB reference copy; profiles/flow_1024x4_fp32_hbm_traffic.md), by kernel
# class and configuration (variant), at n = 1024 in FP32, for the kernels as measured there; a
# configuration without a measurement reports no traffic
TRAFFIC_PER_LAUNCH = {
    ("col_solve", 0): 12.35e6, ("col_solve", 1): 13.41e6, ("col_solve", 2): 13.13e6,
    ("col_solve", 3): 13.78e6, ("col_solve", 4): 13.08e6, ("col_solve", 5): 13.02e6,
    ("col_solve", 6): 41.88e6, ("col_solve", 7): 49.80e6, ("rhs_rowdst", 0): 21.75e6,
    ("rhs_rowdst", 1): 21.75e6, ("rhs_rowdst", 2): 21.64e6, ("rhs_rowdst", 3): 21.63e6,
    ("rhs_rowdst", 4): 21.61e6, ("rhs_rowdst", 5): 21.71e6, ("rhs_rowdst", 6): 21.68e6,
    ("rhs_rowdst", 7): 21.65e6, ("row_idst", 0): 17.12e6, ("row_idst", 1): 17.15e6,
    ("row_idst", 2): 17.05e6, ("row_idst", 3): 17.04e6, ("row_idst", 4): 17.05e6,
    ("row_idst", 5): 17.11e6, ("row_idst", 6): 17.05e6, ("row_idst", 7): 17.07e6,
}


def survey_bytes_per_launch(cls, n, es):
    """Algorithmic bytes of one launch in the fused three-pass Poisson model: words per
    interior vertex for the pass times the (n-1)^2 vertices a launch covers.  Pass 1
    (right-hand side + row transform) reads s and the AB2 history and writes the history and
    the rows, 4 words; pass 2 (column transform, spectral divide, inverse column transform)
    reads and writes the array once, 2 words; pass 3 (inverse row transform) 2 words."""
    words = {"rhs_rowdst": 4, "col_solve": 2, "row_idst": 2}[cls]
    return words * (n - 1) ** 2 * es


def step_bytes(n, levels, es):
    """Algorithmic bytes of one step: w n^2 (8 G + 4 + 6 (G - 1)) -- 8 words per level for the
    predictor, 4 for the corrector on level 0 (its source is sparse), 6 per coarse level for
    the re-solve after coarsification (counted although the reading used here coarsifies on
    read and spends no extra solve)."""
    return es * n * n * (8 * levels + 4 + 6 * (levels - 1))


def algorithmic_bytes(cls, n, levels, steps, es, body_rows):
    """Bytes a launch class of this design moves per timed region: it carries the
    circulation as state beside s, so a level's passes move 12 words per vertex (5 + 3 + 4)
    where the three-pass model counts 8."""
    m = (n - 1) ** 2
    full = (n + 1) ** 2
    if cls == "col_solve":
        # predictor per level: read spectral rows, write s and gamma rows;
        # corrector: read the source rows, read + write both arrays
        return steps * (levels * 3 * m + 4 * m + body_rows * (n - 1)) * es
    if cls == "rhs_rowdst":
        # read s (with ring), gamma, the history; write the history and the rows
        coarsify = (levels - 1) * (n // 2) ** 2
        return steps * (levels * (full + 4 * m) + coarsify) * es
    if cls == "row_idst":
        # read two spectral arrays, write s (with ring) and gamma; plus s* rows on level 0
        return steps * (levels * (3 * m + full) + 2 * (body_rows + 6) * (n - 1)) * es
    return 0


def run(problem, precision, steps, warmup, timing=True, graphs=False):
    import torch
    from paper_2103_06415_amd import binding
    # a stream of its own (which graph recording needs)
    s = binding.Solver(problem, precision=precision, stream=torch.cuda.Stream())
    s.set_option(binding.IB_OPT_GRAPHS, 1 if graphs else 0)
    t0 = time.perf_counter()
    s.prepare()
    s.sync()
    prep = time.perf_counter() - t0
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = {}
    if timing:
        # a second, instrumented pass gives the per-kernel durations (events add a few
        # microseconds per launch, so it is kept out of the wall-clock region above)
        s.set_kernel_timing(True)
        s.step(steps)
        s.sync()
        names = ["rhs_rowdst", "col_solve", "row_idst", "fsi", "correct", "ring"]
        for k, name in enumerate(names):
            kt[name] = s.kernel_timing(k)
        s.set_kernel_timing(False)
    st = s.stats()
    st["flow_tuning"] = s.flow_tuning()
    s.close()
    return wall, prep, kt, st


def concurrent(problem, count, steps, warmup=3):
    """`count` copies of the workload, each on its own stream driven by its own host thread
    (steps recorded as graphs); aggregate grid-cell steps/s over the timed steps."""
    import threading
    import torch
    from paper_2103_06415_amd import binding
    sol = []
    for _ in range(count):
        s = binding.Solver(problem, precision=binding.IB_FP32_FLOW, stream=torch.cuda.Stream())
        s.prepare()
        sol.append(s)
    torch.cuda.synchronize()
    bar = threading.Barrier(count + 1)

    def work(s):
        s.step(warmup)
        s.sync()
        bar.wait()
        s.step(steps)
        s.sync()
        bar.wait()

    th = [threading.Thread(target=work, args=(s,)) for s in sol]
    for t in th:
        t.start()
    bar.wait()
    t0 = time.perf_counter()
    bar.wait()
    wall = time.perf_counter() - t0
    for t in th:
        t.join()
    for s in sol:
        s.close()
    fl = problem.flow
    return {"instances": count, "steps_each": steps, "wall_s": wall,
            "throughput": count * fl.n * fl.n * fl.levels * steps / wall,
            "throughput_unit": "grid-cell steps/s", "ms_per_step_each": 1e3 * wall / steps}


def batch_run(problems, steps, warmup, alone_steps=None):
    """The problems as one batch (ib_batch_*): every launch of a step covers all members.
    Reports the aggregate grid-cell steps/s and, for comparison, the same members stepped
    one after another on their own (alone_steps each, after the batched steps)."""
    import torch
    from paper_2103_06415_amd import binding
    st = torch.cuda.Stream()
    t0 = time.perf_counter()
    sol = []
    for p in problems:
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW, stream=st)
        s.prepare()
        sol.append(s)
    torch.cuda.synchronize()
    prep = time.perf_counter() - t0
    b = binding.Batch(sol, stream=st)
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = b.stats()
    b.close()
    cells = sum(p.flow.n ** 2 * p.flow.levels for p in problems)
    out = {"instances": len(problems), "steps": steps, "wall_s": wall,
           "throughput": cells * steps / wall, "throughput_unit": "grid-cell steps/s",
           "ms_per_step": 1e3 * wall / steps, "prepare_s": prep,
           "launches_per_step": stats["launches"] / max(1, stats["member_steps_batched"] / len(problems)),
           "member_steps_alone": stats["member_steps_alone"], "fsi_resumes": stats["fsi_resumes"]}
    if alone_steps:
        t0 = time.perf_counter()
        for s in sol:
            s.step(alone_steps)
        torch.cuda.synchronize()
        wall_a = time.perf_counter() - t0
        out["throughput_alone_sequential"] = cells * alone_steps / wall_a
        out["batched_over_alone"] = out["throughput"] / out["throughput_alone_sequential"]
    for s in sol:
        s.close()
    return out


def serve(problems, max_active=8, budget=200 << 30, precision=None, per_request=False,
          progress=False):
    """Run (arrival, Problem) requests through the continuous-batching server."""
    from paper_2103_06415_amd import binding
    prec = binding.IB_FP32_FLOW if precision is None else precision
    server = binding.Server(max_active=max_active, hbm_budget_bytes=budget, chunk_steps=50)
    solvers, tickets, cells = [], [], 0
    for arrival, p in problems:
        s = binding.Solver(p, precision=prec, torch_alloc=False, stream=False)
        solvers.append(s)
        tickets.append(server.submit(s, p.steps, arrival=arrival))
        cells += p.flow.n * p.flow.n * p.flow.levels * p.steps
    t0 = time.perf_counter()
    if progress:
        # the server runs in a thread of its own; a line for every few requests that finish
        import threading
        err = []

        def go():
            try:
                server.run()
            except Exception as e:  # noqa: BLE001 (re-raised below)
                err.append(e)
        th = threading.Thread(target=go)
        th.start()
        shown = 0
        while th.is_alive():
            th.join(0.5)
            done = sum(1 for t in tickets if server.info(t)["status"] <= 0)
            if done - shown >= max(1, len(tickets) // 20) or (done == len(tickets) > shown):
                shown = done
                print(f"  served {shown}/{len(tickets)} requests, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
        if err:
            raise err[0]
    else:
        server.run()
    wall = time.perf_counter() - t0
    infos = [server.info(t) for t in tickets]
    stats = [s.stats() for s in solvers]
    sources = [st["operator_source"] for st in stats]
    prep = [st["prepare_seconds"] for st in stats]
    failures = [{"request": k, "status": i["status"], "steps_done": i["steps_done"],
                 "n": p.flow.n, "levels": p.flow.levels,
                 "bodies": [type(b).__name__ for b in p.bodies], "error": s.last_error()}
                for k, ((_, p), i, s) in enumerate(zip(problems, infos, solvers)) if i["status"] != 0]
    for s in solvers:
        s.close()
    server.close()
    ok = [i for i in infos if i["status"] == 0]
    lat = sorted(i["finished"] - i["arrival"] for i in ok)
    done_cells = sum(p.flow.n ** 2 * p.flow.levels * p.steps
                     for (_, p), i in zip(problems, infos) if i["status"] == 0)
    makespan = max(i["finished"] for i in infos) if infos else 0.0

    def pct(q):
        return lat[min(len(lat) - 1, int(math.ceil(q * len(lat))) - 1)] if lat else None
    return {"requests": len(infos), "failed": len(infos) - len(ok), "failures": failures,
            "p50_latency_s": pct(0.50), "p99_latency_s": pct(0.99),
            "makespan_s": makespan, "wall_s": wall,
            "throughput": done_cells / makespan if makespan > 0 else None,
            "throughput_unit": "grid-cell steps/s", "requests_per_s": len(ok) / makespan if makespan else None,
            "max_active": max_active,
            "operators_built": sources.count(0), "operators_from_cache": sources.count(1),
            "cache_hit_share": sources.count(1) / max(1, sources.count(0) + sources.count(1)),
            "offline_seconds_total": sum(prep), "offline_seconds_max": max(prep) if prep else None,
            "per_request": [{"n": p.flow.n, "levels": p.flow.levels, "bodies": len(p.bodies),
                             "steps": p.steps, "offline_s": round(pr, 4), "source": src,
                             "latency_s": (round(i["finished"] - i["arrival"], 4)
                                           if i["status"] == 0 else None)}
                            for (_, p), pr, src, i in zip(problems, prep, sources, infos)]
            if per_request else None}


def trace_gaps(path, step_kernel="k_spread_multi", pattern="_multi", split_us=1000.0):
    """Busy and idle time of the batched step from a rocprofv3 kernel trace (CSV): the region
    runs from the first to the last dispatch whose name contains `pattern`; busy is the union
    of the dispatches' [start, end] intervals in it, idle the rest (launch gaps and host
    waits); steps are counted by the dispatches of `step_kernel` (one per batched step).  Idle
    stretches longer than split_us are the caller's own pauses between calls (warm-up, timing)
    and are left out of the span; the per-step host round trip is the largest gap of each step."""
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"],
                         int(r.get("Grid_Size") or r.get("Grid_Size_X") or 0),
                         int(r.get("Workgroup_Size") or r.get("Workgroup_Size_X") or 1)))
    rows.sort()
    sel = [r for r in rows if pattern in r[2]]
    if not sel:
        return {"error": f"no dispatch named *{pattern}* in {path}"}
    t0, t1 = sel[0][0], max(r[1] for r in sel)
    inside = [r for r in rows if r[0] >= t0 and r[1] <= t1]
    steps = sum(1 for r in inside if step_kernel in r[2])
    busy, cs, ce = 0, None, None
    gaps = []
    for s0, e0, *_ in inside:
        if ce is None:
            cs, ce = s0, e0
        elif s0 > ce:
            busy += ce - cs
            gaps.append(s0 - ce)
            cs, ce = s0, e0
        else:
            ce = max(ce, e0)
    busy += ce - cs
    pauses = [g for g in gaps if g > split_us * 1e3]
    gaps = [g for g in gaps if g <= split_us * 1e3]
    span = t1 - t0 - sum(pauses)
    # the largest gap between consecutive step-kernel dispatches: the host's per-step wait
    marks = [r[1] for r in inside if step_kernel in r[2]]
    step_max = []
    for a, b in zip(marks, marks[1:]):
        seg = [r for r in inside if a <= r[0] < b]
        m, ce2 = 0, a
        for s0, e0, *_ in seg:
            if s0 - ce2 <= split_us * 1e3:
                m = max(m, s0 - ce2)
            ce2 = max(ce2, e0)
        step_max.append(m)
    by = {}
    for s0, e0, name, grid, wg in inside:
        key = name.split("(")[0]
        d = by.setdefault(key, [0, 0.0, 0])
        d[0] += 1
        d[1] += (e0 - s0) * 1e-3
        d[2] = max(d[2], grid // max(wg, 1))
    top = sorted(by.items(), key=lambda kv: -kv[1][1])[:12]
    per = max(steps, 1)
    return {"trace": os.path.basename(path), "steps": steps, "dispatches": len(inside),
            "dispatches_per_step": len(inside) / per, "span_ms_per_step": span * 1e-6 / per,
            "busy_ms_per_step": busy * 1e-6 / per, "idle_ms_per_step": (span - busy) * 1e-6 / per,
            "idle_share": (span - busy) / span, "gaps_per_step": len(gaps) / per,
            "mean_gap_us": (sum(gaps) / len(gaps) * 1e-3) if gaps else 0.0,
            "pauses_left_out_ms": [round(g * 1e-6, 3) for g in pauses],
            "largest_gap_per_step_us_mean": (sum(step_max) / len(step_max) * 1e-3) if step_max else 0.0,
            "other_idle_ms_per_step": ((span - busy) - sum(step_max)) * 1e-6 / per,
            "top_kernels_us_per_step": [(k, round(v[1] / per, 1), v[0] // per, v[2]) for k, v in top]}


def paper_grid(steps, warmup):
    """Flow steps on levels of the size of the paper's largest run (Sec. 5.3: 4000 x 2000 cells,
    5 levels), without bodies: a seeded vortex pair with noise on level 0, h = 0.002, Re 500,
    free stream (1, 0), FP32 flow."""
    import numpy as np
    import workloads as W
    from paper_2103_06415_amd import binding
    nx, ny, levels, h = 4000, 2000, 5, 0.002
    flow = W.Flow(n=nx, ny=ny, levels=levels, h=h, dt=0.2 * h, re=500.0)
    rng = np.random.default_rng(9)
    x = -0.5 * nx * h + h * np.arange(1, nx)
    y = -0.5 * ny * h + h * np.arange(1, ny)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    w = (5.0 * np.exp(-((xx + 1.0) ** 2 + (yy - 0.3) ** 2) / 0.05)
         - 5.0 * np.exp(-((xx + 1.0) ** 2 + (yy + 0.3) ** 2) / 0.05)
         + 1e-3 * rng.normal(size=xx.shape))
    p = W.Problem("paper_grid", flow, [], vorticity0=[w] + [None] * (levels - 1))
    wall, prep, _, st = run(p, binding.IB_FP32_FLOW, steps, warmup, timing=False)
    cells = nx * ny * levels
    return {"value": cells * steps / wall, "unit": "grid-cell steps/s",
            "ms_per_step": 1e3 * wall / steps, "prepare_s": prep, "steps": steps,
            "workload": "flow without bodies on 5 levels of 4000 x 2000 cells (Sec. 5.3's grid), "
                        "FP32 flow, default transform configurations"}


def library_gemm():
    """Matrix-core library products (torch's matmul, hipBLASLt on this platform) at the shapes of
    one sine transform as a dense product: BF16 inputs with FP32 accumulation, the split form's
    k = 3 (n - 1) padded and unpadded, and a large square product for the library's own best
    rate.  Times are averages over 200 back-to-back products between two events."""
    import torch
    out = {}
    for m, k, n, dt in ((1024, 1024, 1024, torch.bfloat16), (1024, 3072, 1024, torch.bfloat16),
                        (1023, 3069, 1023, torch.bfloat16), (4096, 4096, 4096, torch.bfloat16),
                        (1024, 1024, 1024, torch.float32)):
        a = torch.randn(m, k, device="cuda", dtype=dt)
        b = torch.randn(k, n, device="cuda", dtype=dt)
        for _ in range(5):
            c = a @ b
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(200):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 200
        tf = 2.0 * m * n * k / (us * 1e-6) / 1e12
        peak = 2500.0 if dt == torch.bfloat16 else 157.3
        out[f"{m}x{k}x{n}_{str(dt).split('.')[-1]}"] = {"us": round(us, 2), "tflops": round(tf, 1),
                                                         "frac_of_dense_peak": round(tf / peak, 3)}
        del a, b, c
    return out


def serve_legs(args, W):
    """The serving traces: continuous batching of seeded Poisson arrivals (latency = finish -
    arrival).  The family trace repeats six geometries, so most requests reuse an offline
    operator; the drawn trace draws every request's grid, levels, Re and bodies, so nearly every
    request builds its own."""
    out = {"served": serve(W.serve_trace())}
    out["served"]["workload"] = ("48 requests, Poisson arrivals 40/s, 6 families of "
                                 "256^2x1 .. 1024^2x4 grids with 1-3 rigid/torsional/"
                                 "deformable bodies, 200-2000 steps, FP32 flow")
    if args.serve_drawn > 0:
        r = serve(W.drawn_trace(count=args.serve_drawn), per_request=True, progress=True)
        per = r.pop("per_request")
        big = [q for q in per if q["n"] == 1024 and q["source"] == 0]
        r["offline_s_median_1024"] = (sorted(q["offline_s"] for q in big)[len(big) // 2]
                                      if big else None)
        r["workload"] = (f"{args.serve_drawn} requests, Poisson arrivals 40/s, each drawing N in "
                         "{256,384,512,768,1024}, 1-4 levels, Re in [50, 400], 1-3 circles, "
                         "plates or flags (a sub-domain rectangle per plate or flag), 200-2000 "
                         "steps, FP32 flow")
        out["served_drawn"] = r
    return out


def exact_compare(make, tors_body, force_bodies, steps, workload):
    """Sub-domain operator against the exact one rebuilt at every FSI iterate (the paper's
    "true E"): time per step and the difference in a hinge angle and in the lift over the
    run.  make(subdomain) builds the problem; tors_body is the torsional body whose angle is
    compared, force_bodies those whose vertical force is summed into the lift."""
    import numpy as np
    from paper_2103_06415_amd import binding
    out = {}
    hist = {}
    for mode, sd in (("subdomain", True), ("exact", False)):
        p = make(sd)
        s = binding.Solver(p, precision=binding.IB_FP32_FLOW)
        s.prepare()
        s.sync()
        th, fy = [], []
        for _ in range(steps):
            s.step(1)
            th.append(s.deflection(tors_body)[0])
            lift = 0.0
            for b in force_bodies:
                f = s.stresses(b)
                lift += float(f[f.size // 2:].sum() * p.bodies[b].ds)
            fy.append(lift)
        # timing pass without host reads
        t0 = time.perf_counter()
        s.step(20)
        s.sync()
        out[f"ms_per_step_{mode}"] = 1e3 * (time.perf_counter() - t0) / 20
        hist[mode] = (np.array(th), np.array(fy))
        s.close()
    th_sd, fy_sd = hist["subdomain"]
    th_ex, fy_ex = hist["exact"]
    out["speedup_subdomain_over_exact"] = out["ms_per_step_exact"] / out["ms_per_step_subdomain"]
    # after the start-up transient (first quarter of the run): largest difference relative
    # to the largest value, and the difference of the means
    k0 = steps // 4
    out["theta_rel_diff"] = float(np.max(np.abs(th_sd[k0:] - th_ex[k0:])) /
                                  max(np.max(np.abs(th_ex[k0:])), 1e-30))
    out["lift_rel_diff"] = float(np.max(np.abs(fy_sd[k0:] - fy_ex[k0:])) /
                                 max(np.max(np.abs(fy_ex[k0:])), 1e-30))
    out["mean_lift_rel_diff"] = float(abs(fy_sd[k0:].mean() - fy_ex[k0:].mean()) /
                                      max(abs(fy_ex[k0:].mean()), 1e-30))
    out["lift_rel_diff_incl_start"] = float(np.max(np.abs(fy_sd - fy_ex)) /
                                            max(np.max(np.abs(fy_ex)), 1e-30))
    # the paper's error measure (Sec. 5): ||eta - eta_ref||_2 / ||eta_ref||_2 over the run
    out["theta_l2_err"] = float(np.linalg.norm(th_sd - th_ex) / max(np.linalg.norm(th_ex), 1e-30))
    out["lift_l2_err"] = float(np.linalg.norm(fy_sd - fy_ex) / max(np.linalg.norm(fy_ex), 1e-30))
    out["workload"] = workload
    return out


def refinement_study():
    """Sub-domain against exact operator on successively finer grids, the physical time of
    each run fixed: the torsional plate (3 levels, 200 steps at 512^2 scaled with n) and Sec.
    5.1's two plates (case 2, 3 levels, one flapping period: 2000 steps at 256^2 scaled with
    n).  The sub-domain method's hat interpolation P is second order in h, so the differences
    should shrink about fourfold per halving of h once the flow is resolved."""
    import workloads as W
    out = {"plate": {}, "two_plates": {}}
    for n in (256, 512, 1024):
        steps = 200 * n // 512
        print(f"  refinement: plate n={n}, {steps} steps", file=sys.stderr, flush=True)
        r = exact_compare(lambda sd, n=n, steps=steps: W.plate_problem(n=n, levels=3, steps=steps,
                                                                       subdomain=sd),
                          0, [0], steps, f"torsional plate {n}^2 x 3, {steps} steps")
        out["plate"][n] = {k: r[k] for k in ("theta_l2_err", "lift_l2_err", "theta_rel_diff",
                                             "lift_rel_diff", "mean_lift_rel_diff",
                                             "ms_per_step_subdomain", "ms_per_step_exact")}
    for n in (128, 256, 512):
        steps = 2000 * n // 256
        print(f"  refinement: two plates n={n}, {steps} steps", file=sys.stderr, flush=True)
        r = exact_compare(lambda sd, n=n, steps=steps: W.two_plate_problem(n=n, levels=3, steps=steps,
                                                                           case=2, subdomain=sd),
                          1, [0, 1], steps, f"two plates {n}^2 x 3, {steps} steps")
        out["two_plates"][n] = {k: r[k] for k in ("theta_l2_err", "lift_l2_err", "theta_rel_diff",
                                                  "lift_rel_diff", "mean_lift_rel_diff",
                                                  "ms_per_step_subdomain", "ms_per_step_exact")}
    return out


# ---- CPU leg: the FP64 oracle on the host cores (run as a child process of this script,
# with the BLAS thread variables set in its environment before numpy is imported; the child
# touches no GPU) ----

def _host_info():
    import platform
    model = platform.processor()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        import threadpoolctl
        blas = [{"library": d.get("internal_api"), "threads": d.get("num_threads")}
                for d in threadpoolctl.threadpool_info() if d.get("user_api") == "blas"]
    except Exception:
        blas = []
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "blas": blas}


def _oracle_coupled(n, levels, seconds, max_steps=400):
    """The full step of the flag workload (predictor on every level, FSI iterations on the
    sub-domain Schur system with the beam's Newton update, corrector); B' built first and
    reported apart, as the paper excludes the offline stage."""
    import workloads as W
    from oracle.step import Oracle
    o = Oracle(W.flag_problem(n=n, levels=levels))
    t0 = time.perf_counter()
    o.prepare()
    prep = time.perf_counter() - t0
    o.step()  # warm-up (the first step has no history)
    k = 0
    t0 = time.perf_counter()
    while k < max_steps:
        o.step()
        k += 1
        if time.perf_counter() - t0 > seconds:
            break
    wall = time.perf_counter() - t0
    return {"value": n * n * levels * k / wall, "steps": k, "wall_s": wall,
            "ms_per_step": 1e3 * wall / k, "offline_s": prep,
            "subdomain_rows": int(o.b_filtered.shape[0]), "newton_iters_last": o.last_iters}


def _oracle_flow(n, levels, seconds, max_steps=50):
    """Flow steps of the headline grid without body coupling (B' at 1024^2 is out of the
    oracle's reach: about 100,000 dense point-source solves)."""
    import numpy as np

    import workloads as W
    from oracle.step import Oracle
    p = W.flag_problem(n=n, levels=levels)
    o = Oracle(W.Problem("flow", p.flow, [], vorticity0=None))
    rng = np.random.default_rng(0)
    o.s[0][1:-1, 1:-1] = 1e-3 * rng.normal(size=(n - 1, n - 1))
    o.step()
    k = 0
    t0 = time.perf_counter()
    while k < max_steps:
        o.step()
        k += 1
        if time.perf_counter() - t0 > seconds:
            break
    wall = time.perf_counter() - t0
    return {"value": n * n * levels * k / wall, "steps": k, "wall_s": wall,
            "ms_per_step": 1e3 * wall / k}


def cpu_leg(args):
    out = {"coupled": _oracle_coupled(args.cpu_n, args.levels, args.cpu_seconds)}
    if args.cpu_flow_n > 0:
        out["flow"] = _oracle_flow(args.cpu_flow_n, args.levels, args.cpu_seconds)
    out["host"] = _host_info()  # after numpy has loaded its BLAS
    print(json.dumps(out))


def cpu_baseline(n_coupled, n_flow, levels, gpu_coupled, seconds=10.0):
    """The oracle in two child processes, one BLAS thread and the default count; the
    coupled-step figure at n_coupled x levels is the baseline (the GPU's throughput on the
    same workload beside it), the flow-only figure on the headline grid comes second."""
    import subprocess
    runs = {}
    for label, threads in (("one_thread", "1"), ("all_threads", None)):
        env = dict(os.environ)
        if threads is not None:
            for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
                env[var] = threads
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", "--cpu-n", str(n_coupled),
               "--cpu-flow-n", str(n_flow if threads is None else 0), "--levels", str(levels),
               "--cpu-seconds", str(seconds)]
        r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
        if r.returncode != 0:
            runs[label] = {"error": r.stderr[-400:]}
            continue
        runs[label] = json.loads(r.stdout.strip().splitlines()[-1])
    allc = runs.get("all_threads", {})
    one = runs.get("one_thread", {})
    host = allc.get("host", {})
    threads = max([b.get("threads") or 0 for b in host.get("blas", [])] or [0]) or host.get("nproc")
    coupled = allc.get("coupled", {})
    out = {"value": coupled.get("value"), "unit": "grid-cell steps/s", "cores": threads,
           "kind": "oracle",
           "sample": (f"{coupled.get('steps')} full coupled oracle steps of the flag workload at "
                      f"{n_coupled}^2 x {levels} levels (dense FP64 sine-matrix solves on every "
                      f"level, sub-domain Schur system and beam Newton update by numpy.linalg, "
                      f"corrector), {coupled.get('wall_s', 0):.1f} s after B' was built in "
                      f"{coupled.get('offline_s', 0):.1f} s"),
           "one_thread_value": one.get("coupled", {}).get("value"),
           "host": host,
           "gpu_same_workload": gpu_coupled,
           "flow_1024x4": allc.get("flow")}
    if out["value"] and gpu_coupled and gpu_coupled.get("value_fp32"):
        out["gpu_fp32_over_oracle"] = gpu_coupled["value_fp32"] / out["value"]
    return out


def tuning_summary(t):
    """Chosen transform-kernel configurations and the measured launch times (us)."""
    from paper_2103_06415_amd import binding
    out = {"n": t["n"]}
    for kind, k in (("rhs_rowdst", "rhs"), ("col_solve", "col"), ("row_idst", "idst")):
        v = t[k + "_variant"]
        w, th, r = binding.flow_variant_info(1 if k == "col" else 0, v)
        out[kind] = {"variant": v, ("columns" if k == "col" else "rows") + "_per_wg": w,
                     "threads": th, "max_radix": r,
                     "us_by_variant": [round(u, 2) for u in t[k + "_us"]]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the run with the predictor's sine transforms on the BF16 matrix cores")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving trace (48 Poisson arrivals at 40/s, 256^2..1024^2)")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the sub-domain vs exact-operator comparison (plate, 512^2 x 3)")
    ap.add_argument("--concurrent", type=int, default=4,
                    help="also run this many copies of the workload concurrently (0: skip)")
    ap.add_argument("--batch", action="store_true",
                    help="also run the 64 instances through the scheduler")
    ap.add_argument("--no-batch64", action="store_true",
                    help="skip the 64-instance batch (sizes 128^2..768^2) as one ib_batch")
    ap.add_argument("--no-paper-grid", action="store_true",
                    help="skip the flow on levels of 4000 x 2000 cells (5 levels, FP32)")
    ap.add_argument("--no-plate", action="store_true",
                    help="skip the plate workload (512^2 x 3, FP32 and FP64)")
    ap.add_argument("--batch-copies", type=int, default=4,
                    help="also step this many copies of the workload as one ib_batch (0: skip)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batch legs (--batch-copies, --batch); for profiling them")
    ap.add_argument("--cpu-leg", action="store_true",
                    help="(internal) the oracle's CPU timing, run as a child process")
    ap.add_argument("--cpu-n", type=int, default=128)
    ap.add_argument("--cpu-flow-n", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--serve-drawn", type=int, default=48,
                    help="requests in the drawn serving trace (grid, levels, Re and 1-3 bodies "
                         "drawn per request, Poisson arrivals 40/s); 0: skip")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the two serving traces (--serve-drawn sets the drawn one's "
                         "length)")
    ap.add_argument("--refinement", action="store_true",
                    help="only run the sub-domain vs exact comparison on three grid sizes")
    ap.add_argument("--library-gemm", action="store_true",
                    help="only time the matrix-core library's products at the sine-transform shapes")
    ap.add_argument("--trace-gaps", default=None, metavar="CSV",
                    help="only analyse a rocprofv3 kernel trace (kernel_trace.csv) of a "
                         "--batch-only run: busy and idle time of the batched step")
    ap.add_argument("--copy-ref-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a reference "
                         "dispatch of known traffic for hardware counter calibration)")
    args = ap.parse_args()
    if args.trace_gaps:
        print(json.dumps(trace_gaps(args.trace_gaps), indent=1))
        return
    if args.cpu_leg:
        cpu_leg(args)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: each MI355X box here has one, and the "
              "single-instance step does not shard across GPUs (see DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2103_06415_amd import binding
    torch.cuda.set_device(0)
    if args.copy_ref_mb > 0:
        src = torch.ones(args.copy_ref_mb * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n, levels = args.n, args.levels
    prob = W.flag_problem(n=n, levels=levels)
    cells = n * n * levels
    if args.library_gemm:
        print(json.dumps({"library_gemm": library_gemm()}))
        return
    if args.refinement:
        print(json.dumps({"refinement": refinement_study()}))
        return
    if args.serve_only:
        out = {"metric": METRIC, "unit": "grid-cell steps/s", "n_gpus": 1, "data": "synthetic",
               "legs": "serving only"}
        out.update(serve_legs(args, W))
        print(json.dumps(out))
        return
    if args.batch_only:
        out = {"metric": METRIC, "unit": "grid-cell steps/s", "n_gpus": 1, "steps": args.steps,
               "data": "synthetic", "legs": "batch only"}
        if args.batch_copies > 0:
            out["batch_copies"] = batch_run([prob] * args.batch_copies, args.steps, 3)
        if not args.no_batch64:
            out["batch64"] = batch_run(W.batch_problems(), args.steps, 3)
        print(json.dumps(out))
        return
    wall32, prep32, kt, st32 = run(prob, binding.IB_FP32_FLOW, args.steps, args.warmup)
    value = cells * args.steps / wall32
    value64 = None
    if not args.no_fp64:
        wall64, prep64, _, _ = run(prob, binding.IB_FP64, args.steps, args.warmup, timing=False)
        value64 = cells * args.steps / wall64
    # the same step replayed from recorded HIP graphs
    wall_g, _, _, st_g = run(prob, binding.IB_FP32_FLOW, args.steps, args.warmup, timing=False,
                             graphs=True)
    value_graph = cells * args.steps / wall_g
    value_bf16 = None
    if not args.no_bf16:
        wall_b, _, kt_b, _ = run(prob, binding.IB_FP32_FLOW_BF16_DST, args.steps, args.warmup)
        value_bf16 = cells * args.steps / wall_b
    # roofline of the dominant flow kernel class
    body_rows = 0
    sd = prob.subdomain
    if sd is not None:
        body_rows = int((sd[3] - sd[2]) / prob.flow.h) + 9
    flow_classes = ["rhs_rowdst", "col_solve", "row_idst"]
    dom = max(flow_classes, key=lambda c: kt[c][1])
    launches, ms = kt[dom]
    dom_variant = st32["flow_tuning"][{"rhs_rowdst": "rhs", "col_solve": "col",
                                       "row_idst": "idst"}[dom] + "_variant"]
    tot_bytes = algorithmic_bytes(dom, n, levels, args.steps, 4, body_rows)
    avg_launch_s = ms * 1e-3 / max(launches, 1)
    alg_launch = survey_bytes_per_launch(dom, n, 4)
    achieved = alg_launch / avg_launch_s if ms > 0 else 0.0
    sbytes = step_bytes(n, levels, 4)
    times_ms = {k: round(v[1] / args.steps, 5) for k, v in kt.items()}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-cell steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"deformable flag, {n}^2 cells x {levels} levels, 101 body points, "
                               "Re 500, sub-domain B' (eps 0.007), FSI tol 1e-7; FP32 flow + "
                               "FP64 Schur/LU/structure",
                   "n": n, "levels": levels, "subdomain_nnz": st32["subdomain_nnz"],
                   "newton_iters_max": st32["newton_iters_max"],
                   "schur_refine_sweeps_last": st32["refine_iters"],
                   "schur_inverse_rebuilds": st32["inverse_rebuilds"],
                   "fsi_host_resumes": st32["fsi_resumes"]},
        "value_fp64": value64,
        "value_graph_replay": value_graph,
        "graph_launches": st_g["graph_launches"],
        "value_bf16_dst_gemm": value_bf16,
        "kernel_ms_per_step_bf16_dst_gemm": ({k: round(v[1] / args.steps, 5) for k, v in kt_b.items()}
                                             if value_bf16 else None),
        "fp32_over_fp64": (value / value64) if value64 else None,
        "prepare_s": prep32,
        "kernel_ms_per_step": times_ms,
        "flow_tuning": tuning_summary(st32["flow_tuning"]),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM,
                     "traffic": (TRAFFIC_PER_LAUNCH.get((dom, dom_variant)) if n == 1024 else None),
                     "variant": dom_variant,
                     "algorithmic_bytes_per_launch": alg_launch,
                     "design_bytes_per_launch": tot_bytes / max(launches, 1),
                     "design_over_algorithmic": (tot_bytes / max(launches, 1)) / alg_launch,
                     "avg_launch_us": 1e6 * avg_launch_s,
                     "step_bytes": sbytes,
                     "step_achieved": sbytes / (wall32 / args.steps) / 1e9,
                     "step_frac": sbytes / (wall32 / args.steps) / PEAK_HBM},
    }
    if args.concurrent > 1:
        out["concurrent"] = concurrent(prob, args.concurrent, args.steps)
        out["concurrent"]["workload"] = (f"{args.concurrent} copies of the flag workload, one stream "
                                         "and host thread each, FP32 flow")
    if not args.no_serve:
        out.update(serve_legs(args, W))
    if not args.no_exact:
        out["subdomain_vs_exact"] = exact_compare(
            lambda sd: W.plate_problem(n=512, levels=3, steps=200, subdomain=sd), 0, [0], 200,
            "torsional plate, 512^2 x 3 levels, 200 steps from an impulsive start, FP32 flow; "
            "exact mode rebuilds E C K C^T E^T by point-source solves at every FSI iterate")
        out["two_plates_subdomain_vs_exact"] = exact_compare(
            lambda sd: W.two_plate_problem(n=256, levels=3, steps=2000, case=2, subdomain=sd), 1,
            [0, 1], 2000,
            "two torsionally connected plates (driven plate in the case-2 flapping motion, passive "
            "plate on its hinge), 256^2 x 3 levels, 2000 steps (one flapping period), FP32 flow; "
            "lift of both plates, angle of the passive plate")
    if args.batch_copies > 0:
        out["batch_copies"] = batch_run([prob] * args.batch_copies, args.steps, 3,
                                        alone_steps=max(1, args.steps // 4))
        out["batch_copies"]["workload"] = (f"{args.batch_copies} copies of the flag workload as "
                                           "one batch (one launch per kernel for all), FP32 flow")
    if args.batch:
        out["batched"] = serve([(0.0, p) for p in W.batch_problems()], max_active=16)
        out["batched"]["workload"] = ("the same 64 instances (200 steps) through the scheduler, "
                                      "16 slots")
    # the plate workload: 512^2 x 3 levels, FP32 flow next to the plain FP64 form
    if not args.no_plate:
        pl = W.plate_problem(n=512, levels=3)
        pc = 512 * 512 * 3
        w32, p32, _, s32 = run(pl, binding.IB_FP32_FLOW, args.steps, args.warmup, timing=False)
        w64p, _, _, _ = run(pl, binding.IB_FP64, args.steps, args.warmup, timing=False)
        out["plate_512x3"] = {"value_fp32": pc * args.steps / w32, "value_fp64": pc * args.steps / w64p,
                              "ms_per_step_fp32": 1e3 * w32 / args.steps,
                              "ms_per_step_fp64": 1e3 * w64p / args.steps, "prepare_s": p32,
                              "newton_iters_max": s32["newton_iters_max"],
                              "workload": "torsional plate (51 points, I 5, k 1, c 0.1, 20 deg), "
                                          "512^2 x 3 levels, Re 200, sub-domain B', FSI tol 1e-7"}
    if not args.no_paper_grid:
        out["paper_grid_4000x2000x5"] = paper_grid(args.steps, args.warmup)
    if not args.no_batch64:
        out["batch64"] = batch_run(W.batch_problems(), 20, 3, alone_steps=5)
        out["batch64"]["workload"] = ("64 instances, 128^2..768^2 x 1-3 levels, 1-3 rigid or "
                                      "torsional bodies, one batch, FP32 flow")
    if not args.no_cpu:
        # the GPU on the oracle's coupled sample (the flag at 128^2 x 4)
        small = W.flag_problem(n=args.cpu_n, levels=levels)
        sc = args.cpu_n ** 2 * levels
        k = max(args.steps, 200)
        w32s, _, _, _ = run(small, binding.IB_FP32_FLOW, k, args.warmup, timing=False)
        w64s, _, _, _ = run(small, binding.IB_FP64, k, args.warmup, timing=False)
        gpu_small = {"value_fp32": sc * k / w32s, "value_fp64": sc * k / w64s,
                     "ms_per_step_fp32": 1e3 * w32s / k, "ms_per_step_fp64": 1e3 * w64s / k,
                     "steps": k}
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, n, levels, gpu_small, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
