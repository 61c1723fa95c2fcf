#!/usr/bin/env python3
"""Throughput benchmark of the 1D electrostatic PIC engine on one MI355X.

Metric: particle-steps/s on one GPU, batched vs plain (one particle-step = one
particle through gather, kick, drift, wrap and deposit, with its run's field
solve amortised in).  Default workload: the batched ensemble of 256
independent runs (Np log-uniform in [1e4, 4e6], Ng in {64, ..., 2048},
L = 0.032 Ng, two warm beams, dt = 0.1), stepped by one persistent particle
launch plus one solve launch per step from a captured HIP graph.  The same
runs are also stepped one after another on the plain per-run path (ordinary
launches sized to each run), and a single large warm two-stream run
(Np = 2^26, Ng = 4096) is timed for reference.  Then the serving load:
Poisson arrivals at 50 runs/s of runs drawn as the ensemble with 100..2000
steps, admitted by HBM footprint under a 200 GB budget (and again under
40 MiB), reporting p50/p99 completion latency and aggregate particle-steps/s.

Prints ONE JSON line.  Inputs are seeded and synthetic; particle state is
resident in HBM before the timed region starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0          # MI355X HBM3E peak
BYTES_PER_PSTEP = 16            # FP32 state: read x, v; write x, v


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nruns", type=int, default=256)
    ap.add_argument("--np-scale", type=float, default=1.0, help="shrink every ensemble run (smoke use)")
    ap.add_argument("--graph-steps", type=int, default=20)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving load")
    ap.add_argument("--serving-runs", type=int, default=1000)
    ap.add_argument("--serving-rate", type=float, default=50.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run plain 1 GiB device copies (the reference for rocprofv3 byte counters)")
    ap.add_argument("--serving-tight-runs", type=int, default=300,
                    help="requests replayed under a 40 MiB budget (0: skip)")
    ap.add_argument("--workload", default="full", choices=("full", "paper", "small", "probe"),
                    help="full: the benchmark line (default).  For profiling one kernel at a time: "
                         "paper (the paper's workload, exact solve), small (the first --small-runs runs of "
                         "the serving load in one batch), probe (the bandwidth reference)")
    ap.add_argument("--small-runs", type=int, default=8)
    return ap.parse_args()


def kernel_source_hash() -> str:
    """Hash of the particle pass's code (its two source files without
    comments and blank space, and the compiler flags other than include
    paths), so that the counter figures in profiles/traffic.json are used
    only for the code they were taken on."""
    from paper_1108_1954_amd import build as B
    h = hashlib.sha256()
    for f in ("pic_kernels.hip", "pic_internal.h"):
        with open(os.path.join(ROOT, "paper_1108_1954_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    h.update(" ".join(f for f in B.FLAGS if not f.startswith("-I")).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per particle-pass launch from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def generate(specs):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda s: s.particles(), specs))


def host_threads() -> int:
    """Host cores this process may use, at most 16 (one GPU's share of the
    box's cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(specs, parts, budget_s=15.0):
    """The FP64 oracle as it stands (plain FP64 deposit), timed on a bounded
    sample of the ensemble workload: every run of the ensemble stepped the
    same number of steps, the runs spread over all host threads (independent
    runs, one per thread at a time, largest first; the oracle's C code runs
    outside the GIL), and, for the single-core figure, one thread stepping
    every run.  Each run's time includes its initial deposit and solve, which
    are not counted as particle-steps."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    total = sum(s.np_ for s in specs)
    order = sorted(range(len(specs)), key=lambda k: -specs[k].np_)

    def one(k, n):
        s = specs[k]
        x, v = parts[k]
        O.run(O.params(s.L, s.ng, s.np_, dt=s.dt), x, v, n, mode=O.DEPOSIT_PLAIN)

    # single core: every run, a few steps (about budget_s / 2)
    t = time.perf_counter()
    for k in order:
        one(k, 1)
    per_step = time.perf_counter() - t
    n1 = max(1, int(0.5 * budget_s / max(per_step, 1e-6)))
    t = time.perf_counter()
    for k in order:
        one(k, n1)
    t1 = time.perf_counter() - t
    # all host threads: every run, steps chosen for about budget_s of wall time
    threads = host_threads()
    nall = max(2, int(budget_s * threads / max(per_step, 1e-6)))
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda k: one(k, nall), order))
    tall = time.perf_counter() - t
    return {"value": total * nall / tall, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, plain FP64 deposit, all {len(specs)} ensemble runs ({total} particles) "
                      f"x {nall} steps each, {threads} threads (independent runs in parallel), {tall:.1f} s",
            "single_core": {"value": total * n1 / t1, "cores": 1,
                            "sample": f"the same runs x {n1} steps each on one thread, {t1:.1f} s"},
            "cpu": cpu_model(), "host_cores": os.cpu_count()}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


COPY_BYTES = 1 << 30


def calibrate_copy(reps=4):
    """Plain device-to-device copies of COPY_BYTES bytes: what FETCH_SIZE and
    WRITE_SIZE read for one dispatch of these calibrates the counters."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": COPY_BYTES, "dispatches": reps}), flush=True)


def workload_paper(args, P, I, torch):
    """The paper's weak-scaling workload at its 128-thread size, exact solve,
    K graph-replayed steps and K profiled ones."""
    sp = I.paper_weak_scaling(cores=128)
    pp = P.make_params(sp.L, sp.ng, sp.np_, sp.dt)
    with P.Run(pp, loader=P.make_loader(**sp.loader)) as rp:
        rp.step(args.warmup + args.graph_steps, graph_steps=args.graph_steps)    # incl. graph capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rp.step(args.steps, graph_steps=args.graph_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mp, ms = P.pic_step_profiled(rp.handle, args.steps)
    return {"workload": f"paper weak-scaling run, ng={sp.ng}, np={sp.np_}", "ms_per_step": 1e3 * wall / args.steps,
            "particle_pass_ms": mp, "solve_ms": ms,
            "particle_pass_GBps": BYTES_PER_PSTEP * sp.np_ / (mp * 1e6)}


def workload_small(args, P, I, torch):
    """The serving regime: the first --small-runs runs of the serving load
    (drawn as the ensemble, seed 4) in one batch sized like the server's
    (256 slots, ng up to 2048), stepped from a captured graph."""
    from paper_1108_1954_amd import serve
    n = args.small_runs
    specs = I.ensemble(nruns=n, seed=4, steps_range=(100, 2000))
    parts = generate(specs)
    total = sum(s.np_ for s in specs)
    steps = args.warmup + 2 * args.steps + 2
    b = P.pic_batch_create(2 << 30, 2048, max_runs=256, graph_steps=10, stream=P.current_stream())
    try:
        for s, (x, v) in zip(specs, parts):
            P.pic_batch_admit(b, P.make_params(s.L, s.ng, s.np_, s.dt), x, v, steps)
        P.pic_batch_step(b, args.warmup)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        P.pic_batch_step(b, args.steps)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        mp, msv = P.pic_batch_step_profiled(b, args.steps)
    finally:
        P.pic_batch_destroy(b)
    return {"workload": f"first {n} runs of the serving load in one batch, {total} particles, "
                        f"ng {sorted(set(s.ng for s in specs))}", "ms_per_step": ms,
            "particle_pass_ms": mp, "solve_ms": msv, "particle_pass_GBps": BYTES_PER_PSTEP * total / (mp * 1e6)}


def workload_probe(args, P, torch, nbytes=2 << 30):
    """The bandwidth reference: two FP32 arrays of 1 GiB each swapped in
    place (16 bytes per element pair, the particle pass's pattern), and a
    plain torch device copy of 1 GiB for comparison."""
    n = nbytes // 8
    a = torch.zeros(n, dtype=torch.float32, device="cuda")
    b = torch.ones(n, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ms = P.pic_bandwidth_probe(a.data_ptr(), b.data_ptr(), n, reps=args.steps, stream=P.current_stream())
    # The same swap over exactly the state of each workload's particle pass
    # (one launch per swap, as one pass is one launch): the achievable rate
    # for that many bytes, launch ramp and tail included, with non-temporal
    # and with cached accesses (the pass's two cache policies; a state that
    # fits the last-level cache stays there between launches).
    sized = {}
    for name, npart in (("serving batch of 8 runs", 1_804_773), ("paper workload", 8_192_000),
                        ("single run 2^26", 1 << 26), ("ensemble", 145_439_881)):
        m = npart // 4 * 4
        row = {"particles": m, "bytes": 16 * m}
        for key, cached in (("", False), ("cached_", True)):
            t = P.pic_bandwidth_probe(a.data_ptr(), b.data_ptr(), m, reps=max(args.steps, 50),
                                      stream=P.current_stream(), cached=cached)
            row[key + "swap_us"] = 1e3 * t
            row[key + "GBps"] = 16 * m / (t * 1e6)
        sized[name] = row
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    mc = ev0.elapsed_time(ev1) / args.steps
    return {"workload": "bandwidth reference", "swap_bytes": 16 * n, "swap_ms": ms,
            "swap_GBps": 16 * n / (ms * 1e6), "swap_frac_of_peak": 16 * n / (ms * 1e6) / PEAK_HBM_GBPS,
            "torch_copy_bytes": 2 * COPY_BYTES, "torch_copy_ms": mc,
            "torch_copy_GBps": 2 * COPY_BYTES / (mc * 1e6), "swap_at_workload_sizes": sized}


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): there is no multi-GPU path "
              "to run; how runs and particles would shard across GPUs is a design note only.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1108_1954_amd import inputs as I
    from paper_1108_1954_amd import pic as P
    P.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.cuda.get_device_properties(0)
    stream = P.current_stream()
    K, W = args.steps, args.warmup
    if args.workload != "full":
        fn = {"paper": lambda: workload_paper(args, P, I, torch), "small": lambda: workload_small(args, P, I, torch),
              "probe": lambda: workload_probe(args, P, torch)}[args.workload]
        print(json.dumps(fn()), flush=True)
        return

    # ------------------------------------------------------------ ensemble
    t0 = time.perf_counter()
    specs = I.ensemble(nruns=args.nruns, seed=3, nsteps=500, np_scale=args.np_scale)
    parts = generate(specs)
    total_np = sum(s.np_ for s in specs)
    log(f"ensemble: {len(specs)} runs, {total_np} particles, generated in {time.perf_counter() - t0:.1f} s")
    prof_steps = 5
    run_steps = W + K + prof_steps + 1
    params = [P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=run_steps) for s in specs]
    budget = int(sum(P.pic_footprint(p) for p in params) * 1.05) + (64 << 20)
    ng_max = max(s.ng for s in specs)
    b = P.pic_batch_create(budget, ng_max, max_runs=len(specs), graph_steps=args.graph_steps, stream=stream)
    t0 = time.perf_counter()
    for p, (x, v) in zip(params, parts):
        P.pic_batch_admit(b, p, x, v, run_steps)
    torch.cuda.synchronize()
    log(f"admitted in {time.perf_counter() - t0:.1f} s")
    P.pic_batch_step(b, W)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    P.pic_batch_step(b, K)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / K
    batched_rate = total_np * K / wall
    ms_particle, ms_solve = P.pic_batch_step_profiled(b, prof_steps)
    torch.cuda.synchronize()
    d0, _, _ = P.pic_diagnostics(P.pic_batch_run(b, 1))
    assert d0["charge_fixed_sum"] == specs[0].np_ << 32
    P.pic_batch_destroy(b)
    log(f"batched: {ms_step:.3f} ms/step (events), {batched_rate:.4g} particle-steps/s (wall), "
        f"particle pass {ms_particle:.3f} ms, solve {ms_solve:.3f} ms")
    # The measured bandwidth reference for these bytes: a plain swap of two
    # FP32 arrays of total_np elements with the pass's byte pattern
    # (non-temporal 16-byte loads and stores, one launch per swap).
    nswap = total_np // 4 * 4
    sa = torch.zeros(nswap, dtype=torch.float32, device="cuda")
    sb = torch.ones(nswap, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ms_swap = P.pic_bandwidth_probe(sa.data_ptr(), sb.data_ptr(), nswap, reps=20, stream=stream)
    del sa, sb
    swap = {"bytes": BYTES_PER_PSTEP * nswap, "ms": ms_swap, "GBps": BYTES_PER_PSTEP * nswap / (ms_swap * 1e6),
            "pass_fraction_of_swap": ms_swap / ms_particle,
            "note": "pic_bandwidth_probe: in-place swap of the same bytes, non-temporal 16-byte accesses, "
                    "mean of 20 back-to-back launches; its rate depends on where the two arrays land in "
                    "physical memory (398-479 us for these bytes across placements measured)"}

    # ---------------------------------------------------- plain per-run path
    plain = None
    if not args.no_plain:
        runs = [P.Run(p, x, v) for p, (x, v) in zip(params, parts)]
        for r in runs:
            r.step(W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in runs:                        # runs one after another, plain launches
            r.step(K)
        torch.cuda.synchronize()
        wall_p = time.perf_counter() - t0
        plain = {"value": total_np * K / wall_p, "ms_per_step": 1e3 * wall_p / K,
                 "path": "same kernels, one plain launch pair per run per step, runs in sequence"}
        for r in runs:
            r.close()
        log(f"plain: {plain['ms_per_step']:.3f} ms/step, {plain['value']:.4g} particle-steps/s")

    # ------------------------------------------------- single large run (c2)
    single = None
    if not args.no_single:
        s2 = I.warm_two_stream_large(np_=1 << 26, ng=4096, nsteps=1000)
        x, v = s2.particles()
        p2 = P.make_params(s2.L, s2.ng, s2.np_, s2.dt)
        r2 = P.Run(p2, x, v)
        del x, v
        r2.step(W + args.graph_steps, graph_steps=args.graph_steps)      # warm, incl. graph capture
        torch.cuda.synchronize()
        ev0.record()
        r2.step(K, graph_steps=args.graph_steps)
        ev1.record()
        torch.cuda.synchronize()
        ms2 = ev0.elapsed_time(ev1) / K
        mp2, msv2 = P.pic_step_profiled(r2.handle, prof_steps)
        r2.close()
        # cell sort (a7) on the same run, which is created with room for it
        p2s = P.make_params(s2.L, s2.ng, s2.np_, s2.dt, sort_every=1 << 30)
        x, v = s2.particles()
        r3 = P.Run(p2s, x, v)
        del x, v
        r3.step(2)

        def timed_sort():
            torch.cuda.synchronize()
            ev0.record()
            r3.sort()
            ev1.record()
            torch.cuda.synchronize()
            return ev0.elapsed_time(ev1)
        sort_random = timed_sort()                         # from the loaded (random) order
        sort_sorted = min(timed_sort() for _ in range(3))  # already in cell order
        mp_sorted, _ = P.pic_step_profiled(r3.handle, prof_steps)
        r3.close()
        # the period the engine chooses for this run by itself (PIC_SORT_AUTO)
        x, v = s2.particles()
        with P.Run(P.make_params(s2.L, s2.ng, s2.np_, s2.dt, sort_every=P.PIC_SORT_AUTO), x, v) as r4:
            auto_k = r4.sort_period()
        del x, v
        single = {"workload": "warm two-stream, np=2^26, ng=4096, L=131.39, dt=0.1",
                  "value": s2.np_ / (ms2 * 1e-3), "ms_per_step": ms2,
                  "particle_pass_ms": mp2, "solve_ms": msv2,
                  "particle_pass_GBps": BYTES_PER_PSTEP * s2.np_ / (mp2 * 1e6),
                  "cell_sort": {"ms_from_random_order": sort_random, "ms_when_sorted": sort_sorted,
                                "particle_pass_ms_after_sort": mp_sorted,
                                "auto_period": auto_k,
                                "note": "reported overhead; sort_every = PIC_SORT_AUTO chooses the period "
                                        "shown (0: never)"}}
        log(f"single run: {ms2:.3f} ms/step, particle pass {mp2:.3f} ms, solve {msv2:.3f} ms; cell sort "
            f"{sort_random:.3f} ms (random order), {sort_sorted:.3f} ms (sorted), pass after sort {mp_sorted:.3f} ms; "
            f"auto period {auto_k}")

    # ----------------------------- the paper's weak-scaling workload, one GPU
    paper = None
    if not args.no_single:
        sp = I.paper_weak_scaling(cores=128)
        paper = {"workload": f"the paper's weak-scaling run at its 128-thread size on one GPU: ng={sp.ng}, "
                             f"np={sp.np_}, L={sp.L:.1f}, Maxwellian vth=0.2, dt=0.1, {sp.nsteps} cycles; "
                             "lattice start, particles drawn on the device (pic_create_loaded)"}
        for label, solver in (("exact_solve", P.PIC_SOLVE_EXACT), ("paper_cg_150", P.PIC_SOLVE_CG_PAPER)):
            pp = P.make_params(sp.L, sp.ng, sp.np_, sp.dt, solver=solver, cg_iters=150)
            rp = P.Run(pp, loader=P.make_loader(**sp.loader))
            rp.step(args.graph_steps, graph_steps=args.graph_steps)   # warm, incl. graph capture
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rp.step(sp.nsteps, graph_steps=args.graph_steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            mp, ms = P.pic_step_profiled(rp.handle, prof_steps)
            rp.close()
            paper[label] = {"seconds_per_1000_cycles": wall * 1000 / sp.nsteps,
                            "ms_per_cycle": 1e3 * wall / sp.nsteps, "particle_pass_ms": mp, "solve_ms": ms,
                            "particle_steps_per_s": sp.np_ * sp.nsteps / wall}
        log(f"paper workload: {paper}")

    # ------------------ the precision workload: FP32 and FP64 particle state
    precision = None
    if not args.no_single:
        s5 = I.warm_maxwellian_large()
        precision = {"workload": f"warm Maxwellian, np=2^28, ng={s5.ng}, L={s5.L:.2f}, dt={s5.dt}; "
                                 "particles drawn on the device (pic_create_loaded)"}
        for label, prec, bpp in (("fp32_state", P.PIC_FP32, 16), ("fp64_state", P.PIC_FP64, 32)):
            p5 = P.make_params(s5.L, s5.ng, s5.np_, s5.dt, precision=prec)
            r5 = P.Run(p5, loader=P.make_loader(**s5.loader))
            r5.step(args.graph_steps, graph_steps=args.graph_steps)   # warm, incl. graph capture
            torch.cuda.synchronize()
            ev0.record()
            r5.step(K, graph_steps=args.graph_steps)
            ev1.record()
            torch.cuda.synchronize()
            ms5 = ev0.elapsed_time(ev1) / K
            mp5, msv5 = P.pic_step_profiled(r5.handle, prof_steps)
            r5.close()
            precision[label] = {"ms_per_step": ms5, "particle_steps_per_s": s5.np_ / (ms5 * 1e-3),
                                "particle_pass_ms": mp5, "solve_ms": msv5,
                                "particle_pass_GBps": bpp * s5.np_ / (mp5 * 1e6),
                                "bytes_per_particle_step": bpp}
        log(f"precision workload: {precision}")

    # ------------------------------------------------------------- serving
    serving = None
    if not args.no_serving:
        from paper_1108_1954_amd import serve
        t0 = time.perf_counter()
        reqs = serve.make_requests(args.serving_runs, rate=args.serving_rate, np_scale=args.np_scale)
        log(f"serving: {len(reqs)} requests generated in {time.perf_counter() - t0:.1f} s")
        serving = serve.serve_load(rate=args.serving_rate, budget=200 << 30, requests=reqs)
        serving["workload"] = (f"Poisson arrivals {args.serving_rate:g}/s, {len(reqs)} runs drawn as the "
                               "ensemble with steps U{100..2000}, 200 GB budget")
        log(f"serving: {serving}")
        if args.serving_tight_runs > 0:
            tight = serve.serve_load(rate=args.serving_rate, budget=40 << 20,
                                     requests=reqs[:args.serving_tight_runs])
            tight["workload"] = (f"first {args.serving_tight_runs} requests of the same load, 40 MiB budget "
                                 "(the largest run is ~31 MiB)")
            serving["tight_budget"] = tight
            log(f"serving (40 MiB): {tight}")
        del reqs

    # --------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(specs, parts)
        log(f"cpu baseline: {cpu}")

    achieved = BYTES_PER_PSTEP * total_np / (ms_particle * 1e6)   # GB/s of the particle pass
    out = {
        "metric": "particle-steps/s on 1 GPU, batched vs plain; p50/p99 run latency under load",
        "value": batched_rate,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "numerics": "f32 particle state and push, int64 fixed-point deposit, f64 solve and diagnostics",
        "data": "synthetic (seeded SplitMix64 inputs)",
        "config": {"workload": f"batched ensemble: {len(specs)} runs, Np log-uniform [1e4,4e6]"
                               f"{'' if args.np_scale == 1.0 else f' x{args.np_scale}'}, Ng 64..2048, "
                               "L=0.032 Ng, dt=0.1, one graph-captured persistent launch pair per step; "
                               f"every run admitted for {run_steps} steps (none finishes inside a measured "
                               f"launch): steps {W + 1}..{W + K} timed after {W} warm-up steps, then "
                               f"{prof_steps} more with per-launch HIP events",
                   "total_particles": total_np, "runs": len(specs), "ng_max": ng_max,
                   "graph_steps": args.graph_steps, "device": dev.name, "cus": dev.multi_processor_count},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBPS, "traffic": measured_traffic("ensemble"),
                     "kernel": "step_kernel (particle pass)", "kernel_ms": ms_particle,
                     "bytes_per_launch": BYTES_PER_PSTEP * total_np, "solve_ms": ms_solve,
                     "same_size_swap": swap},
        "plain": plain,
        "batched_vs_plain": (batched_rate / plain["value"]) if plain else None,
        "single_run": single,
        "paper_weak_scaling_one_gpu": paper,
        "precision_state": precision,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
