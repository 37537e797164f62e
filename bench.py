#!/usr/bin/env python3
"""Benchmark: walk-steps/s of parallel flatPERM on one MI355X.

One benchmark step is one whole job of the parallel square-lattice workload:
4096 interacting flatPERM sequences (Algorithm 2), n_max = 500, a merge every
64 tours, 38 epochs = 9,961,472 tours, followed by the read-out of log c_n.
Every step runs a fresh job with its own seed; the workspaces are allocated
and initialised before the timed region, so the timed region holds exactly the
hot path: growth with a_+ scans, weight updates, prune/enrich, accumulation,
merges and the estimate read-out.

Printed: one JSON line with the metric, a roofline object for the dominant
kernel (the growth kernel, timed with HIP events on its stream) and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# Algorithmic work per walk-step of the growth kernel (32-bit VALU lane operations
# of the minimal single-walk step: Philox4x32-10 block 100, occupancy scan
# 7 per neighbour query with 2d - 1 queries, control 15, growth 15, record 6).
ALG_OPS_PER_STEP = {2: 100 + 7 * 3 + 15 + 15 + 6, 3: 100 + 7 * 5 + 15 + 15 + 6}
# MI355X 32-bit VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one lane-op per lane per clock).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2002_03000_amd", "csrc", "pperm_kernels.hip")


def measured_traffic(name):
    """HBM bytes per launch of the growth kernel from a committed counter
    summary, or None when the kernel source has changed since it was taken."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_code_sha256") != kernel_code_digest() or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def kernel_code_digest():
    """sha256 of the kernel source with comments and blank lines removed: the
    key under which counter summaries stay valid."""
    import hashlib
    import re
    src = open(KERNEL_SOURCE).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in src.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln.strip()).encode()).hexdigest()


WORKLOADS = {
    "parallel2d": workloads.PARALLEL_2D,
    "parallel3d": workloads.PARALLEL_3D,
    "long2d": workloads.LONG_2D,       # n_max = 10^4: sums in global memory
    "plain2d": workloads.PLAIN_2D,
    "batched": None,          # the 256-problem mix, see run_batched()
    "served": None,           # the Poisson job stream, see run_served()
    "compare": None,          # Algorithm 1 vs Algorithm 2, see run_compare()
}


def describe(p):
    sched = p.schedule()
    return (f"parallel flatPERM (Algorithm 2), Z^{p.dim}, N={p.n_sequences} sequences, "
            f"n_max={p.n_max}, {len(sched)} epochs: warm-up {sched[:len(sched) - p.epochs + 1]} "
            f"then {p.epochs - 1} x {p.tours_per_epoch} tours/sequence ({p.total_tours} tours)")


def cpu_baseline(p, budget_s=15.0):
    """The oracle, as it stands, on a bounded sample of the same job: its epochs
    in order (run + merge, all sequences, all host cores) until the time budget
    is spent, stopping at an epoch boundary."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    o = oracle.Oracle(p.dim, p.n_max, p.n_sequences, p.seed, threads=threads)
    done, t0 = 0, time.perf_counter()
    for T in p.schedule():
        o.run_tours(T)
        o.merge_epoch()
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    steps = o.walk_steps()
    return {"value": steps / dt, "unit": "walk-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {done} epochs of the same job ({steps} walk-steps, "
                      f"{o.N * int(o.MG[0]) // max(o.N, 1)} tours) in {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="default 3 (long2d: 1)")
    ap.add_argument("--warmup", type=int, default=None, help="default 1 (long2d: 0)")
    ap.add_argument("--workload", default="parallel2d", choices=sorted(WORKLOADS))
    ap.add_argument("--epochs", type=int, default=0, help="override the epoch count (profiling)")
    ap.add_argument("--walks-per-wave", type=int, default=0)
    ap.add_argument("--hash-slots", type=int, default=0)
    ap.add_argument("--sums-global", choices=("auto", "on", "off"), default="auto",
                    help="launch tuning: per-length sums in global memory, more walks per CU "
                         "(auto: on for parallel3d, whose in-LDS sums allow only four walks per CU)")
    ap.add_argument("--autotune", action="store_true", help="pick the launch shape by short trial runs first")
    ap.add_argument("--problems", type=int, default=0, help="batched: use the first P problems of the mix")
    ap.add_argument("--lockstep", action="store_true",
                    help="batched: lock-step rounds of batched calls instead of device-chained epochs")
    ap.add_argument("--compare-n", default="1,2,12,64", help="compare: sequence counts")
    ap.add_argument("--compare-s", default="1,10,100,1000,10000", help="compare: tours per sequence")
    ap.add_argument("--compare-replicas", type=int, default=8, help="compare: independent runs per cell")
    ap.add_argument("--serve-duration", type=float, default=60.0, help="served: arrival window (s)")
    ap.add_argument("--serve-rate", type=float, default=50.0, help="served: arrivals per second")
    ap.add_argument("--serve-cap", type=int, default=4096, help="served: tour cap per job")
    ap.add_argument("--serve-target", type=float, default=1e-3, help="served: relative-error target")
    ap.add_argument("--serve-pool-gib", type=float, default=64.0)
    ap.add_argument("--serve-max-sequences", type=int, default=262144)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency-bound", action="store_true",
                    help="skip the critical-path replay that follows the timed region")
    ap.add_argument("--kernel-digest", action="store_true",
                    help="print the digest that keys the committed counter summaries")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to calibrate the HBM byte counters)")
    args = ap.parse_args()
    if args.sums_global == "auto":
        args.sums_global = (args.workload == "parallel3d")
    else:
        args.sums_global = (args.sums_global == "on")
    # a long2d job runs for about a minute and a half
    if args.steps is None:
        args.steps = 1 if args.workload == "long2d" else 3
    if args.warmup is None:
        args.warmup = 0 if args.workload == "long2d" else 1

    if args.kernel_digest:
        print(kernel_code_digest())
        return
    if args.copy_calibration:
        copy_calibration()
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding "
              "of the method is described in the design notes, not run.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        run_batched(args)
        return
    if args.workload == "served":
        run_served(args)
        return
    if args.workload == "compare":
        run_compare(args)
        return

    import numpy as np
    import torch
    from paper_2002_03000_amd import ParallelFlatPERM

    p = WORKLOADS[args.workload]
    if args.epochs:
        p = p.scaled(epochs=args.epochs)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    tuning = None
    if args.autotune:
        # launch shape from short trial runs, before and outside the timed region
        from paper_2002_03000_amd import autotune
        best, tuning = autotune(p.dim, p.n_max, p.n_sequences, mode=p.mode, trial=tuple(p.schedule()[:5]))
        args.walks_per_wave, args.hash_slots = best["walks_per_wave"], best["hash_slots"]
        args.sums_global = best["sums_global"]

    def make(seed):
        return ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, seed, mode=p.mode,
                                walks_per_wave=args.walks_per_wave, hash_slots=args.hash_slots,
                                sums_global=args.sums_global)

    sched = p.schedule()

    def job(g, ev=None):
        for T in sched:
            if ev is not None:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                g.run_tours(T)
                b.record(stream)
                ev.append((a, b))
            else:
                g.run_tours(T)
            g.merge_epoch()
        return g.estimates()

    # warmup (its own seeds)
    for i in range(args.warmup):
        g = make(p.seed + 1000 + i)
        job(g)
        g.close()
        del g
    torch.cuda.synchronize()

    ctxs = [make(p.seed + i) for i in range(args.steps)]
    torch.cuda.synchronize()
    events = []
    results = []
    t0 = time.perf_counter()
    for g in ctxs:
        results.append(job(g, events))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    steps_total = 0
    scans_total = 0                    # a_+ evaluations: one per growth event or trapped walk
    for g in ctxs:
        st = g.stats()
        steps_total += st["steps"]
        scans_total += st["events"] + st["traps"]
    run_ms = sum(a.elapsed_time(b) for a, b in events)
    launches = len(events)
    shape = ctxs[0].launch_shape()

    value = steps_total / elapsed
    kernel_rate = steps_total / (run_ms / 1e3)
    ops = ALG_OPS_PER_STEP[p.dim]
    achieved = kernel_rate * ops / 1e12
    est_top = np.array([r[0][p.n_max] for r in results])
    rel_err = float(np.std(np.exp(est_top - est_top.mean()), ddof=1)) if len(results) > 1 else None

    kernel = "batch_long_kernel" if (args.workload == "long2d" or args.sums_global) else "batch_kernel"
    line = {
        "metric": "walk-steps/s (parallel flatPERM, 1 GPU)",
        "value": value,
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (walks grown from parameters; seeds per job)",
        "config": {"workload": describe(p), "dim": p.dim, "n_max": p.n_max,
                   "n_sequences": p.n_sequences, "tours_per_epoch": p.tours_per_epoch,
                   "epochs": len(sched), "schedule": sched[:len(sched) - p.epochs + 2],
                   "walk_steps_per_job": steps_total // args.steps,
                   "launch": dict(shape, sums_global=bool(args.sums_global)), "autotune": tuning},
        "cn_rel_err_nmax": rel_err,
        "log_cn_nmax": float(est_top[0]),
        "a_plus_evaluations_per_step": scans_total / steps_total,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / ALU_PEAK_TOPS,
                     "traffic": measured_traffic(f"{kernel}_{args.workload}_traffic.md")
                     if not args.epochs else None,
                     "kernel": kernel, "avg_launch_ms": run_ms / launches,
                     "alg_ops_per_step": ops},
        "cpu_baseline": None,
    }
    if not args.no_latency_bound:
        line["latency_bound"] = latency_bound(p, make, sched, elapsed / args.steps, args.sums_global)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(line), flush=True)


def latency_bound(p, make, sched, seconds_per_job, sums_global=False):
    """The floor an epoch-synchronous job cannot go below on any number of
    waves: each epoch lasts at least as long as its heaviest sequence takes,
    one step after another on one wave.  Measured outside the timed region:
    the first timed job is replayed (same seed, same bits) with every
    sequence's step count read after each epoch, and the latency of one step
    of a wave running alone comes from a one-sequence problem of the same
    dimension and length."""
    import numpy as np
    import torch
    from paper_2002_03000_amd import ParallelFlatPERM
    g = make(p.seed)
    prev = np.zeros(p.n_sequences, dtype=np.uint64)
    crit = 0
    for T in sched:
        g.run_tours(T)
        g.merge_epoch()
        st = g.sequence_stats()["steps"]
        crit += int((st - prev).max())
        prev = st
    g.close()
    # one wave alone: a single sequence through the same schedule (the first
    # epochs warm its own estimates), timed over the full-length epochs
    lone = ParallelFlatPERM(p.dim, p.n_max, 1, p.seed + 77, sums_global=sums_global)
    head = len(sched) - p.epochs + 1
    for T in sched[:head]:
        lone.run_tours(T)
        lone.merge_epoch()
    torch.cuda.synchronize()
    s0 = lone.stats()["steps"]
    t0 = time.perf_counter()
    for T in sched[head:head + 8]:
        lone.run_tours(T)
        lone.merge_epoch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lone_steps = lone.stats()["steps"] - s0
    lone.close()
    t_step = dt / max(lone_steps, 1)
    bound = crit * t_step
    return {"critical_path_steps": crit, "lone_step_us": t_step * 1e6, "lone_sample_steps": int(lone_steps),
            "bound_ms_per_step": bound * 1e3, "frac": bound / seconds_per_job}


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of a known size: under `rocprofv3 --pmc FETCH_SIZE`
    (then WRITE_SIZE) the copy reads and writes exactly nbytes, so counter /
    nbytes converts another kernel's counter into bytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}), flush=True)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_batched(args, plain_budget_s=40.0):
    """The 256-problem mix as one batched job: in each round every problem that
    still has an epoch runs it, all of them in one batched launch, then each
    merges.  Beside it: the same problems on the single-problem path one at a
    time (a time-bounded prefix of the mix), and the oracle on a sample."""
    import numpy as np
    import torch
    from paper_2002_03000_amd import Batch, ParallelFlatPERM

    mix = workloads.batched_mix()
    if args.problems:
        mix = mix[:args.problems]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    scheds = [p.schedule() for p in mix]
    rounds = max(len(s) for s in scheds)

    def make(p, offset):
        return ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, p.seed + offset, mode=p.mode,
                                stream_id=p.stream)

    from paper_2002_03000_amd import run_job
    batch = Batch(len(mix))
    # warm-up: the first two epochs of a few problems, their own seeds
    warm = [make(p, 7_000_000) for p in mix[:8]]
    if args.lockstep:
        for r in range(2):
            batch.run_tours(warm, [s[r] for s in scheds[:8]])
            for g in warm:
                g.merge_epoch()
    else:
        run_job(warm, [s[:2] for s in scheds[:8]], stream=stream)
    torch.cuda.synchronize()
    for g in warm:
        g.close()
    del warm

    steps_total, elapsed_total, events = 0, 0.0, []
    results = []
    for k in range(args.steps):
        probs = [make(p, k) for p in mix]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if args.lockstep:
            # every problem's epoch of a round in one batched call, then the merges
            last = t0
            for r in range(rounds):
                tours = [s[r] if r < len(s) else 0 for s in scheds]
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                batch.run_tours(probs, tours)
                b.record(stream)
                events.append((a, b))
                for g, t in zip(probs, tours):
                    if t:
                        g.merge_epoch()
                torch.cuda.synchronize()
                if time.perf_counter() - last > 10:
                    last = time.perf_counter()
                    _log(f"batched job {k}: round {r + 1}/{rounds}, {last - t0:.1f} s")
        else:
            # the whole job in persistent launches that chain epochs on the device
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ws = run_job(probs, scheds, stream=stream)
            b.record(stream)
            events.append((a, b))
            last = t0
            while not b.query():
                time.sleep(0.5)
                if time.perf_counter() - last > 10:
                    last = time.perf_counter()
                    _log(f"batched job {k}: running, {last - t0:.0f} s")
            del ws
        ests = [g.estimates() for g in probs]
        torch.cuda.synchronize()
        elapsed_total += time.perf_counter() - t0
        by_dim = {2: 0, 3: 0}
        for p, g in zip(mix, probs):
            by_dim[p.dim] += g.stats()["steps"]
        steps_total += sum(by_dim.values())
        results.append(ests)
        for g in probs:
            g.close()
        del probs
        _log(f"batched job {k} done: {elapsed_total:.1f} s so far")

    run_ms = sum(a.elapsed_time(b) for a, b in events)
    value = steps_total / elapsed_total
    ops = (ALG_OPS_PER_STEP[2] * by_dim[2] + ALG_OPS_PER_STEP[3] * by_dim[3]) / max(1, sum(by_dim.values()))
    achieved = steps_total / (run_ms / 1e3) * ops / 1e12

    # plain path, one problem at a time, same problems and seeds (offset 0)
    t0 = time.perf_counter()
    plain_steps, plain_problems, plain_epochs = 0, 0, 0
    for p, sch in zip(mix, scheds):
        g = make(p, 0)
        for T in sch:
            g.run_tours(T)
            g.merge_epoch()
            torch.cuda.synchronize()
            plain_epochs += 1
            if time.perf_counter() - t0 > plain_budget_s:
                break
        g.estimates()
        plain_steps += g.stats()["steps"]
        g.close()
        plain_problems += 1
        if time.perf_counter() - t0 > plain_budget_s:
            break
    plain_dt = time.perf_counter() - t0
    _log(f"plain path: {plain_problems} problems, {plain_epochs} epochs in {plain_dt:.1f} s")

    total_tours = sum(p.total_tours for p in mix)
    line = {
        "metric": "walk-steps/s (parallel flatPERM, 1 GPU)",
        "value": value,
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": elapsed_total * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (walks grown from parameters; seeds per problem)",
        "config": {"workload": f"batched mix of {len(mix)} independent problems (seed 4): d in {{2,3}}, "
                               f"n_max in [64,2048], N in 64..1024, {total_tours} tours in total, "
                               + (f"{rounds} lock-step batched rounds" if args.lockstep else
                                  "epochs chained on the device in one persistent launch per LDS class"),
                   "problems": len(mix), "rounds": rounds, "lockstep": bool(args.lockstep),
                   "walk_steps_per_job": steps_total // args.steps},
        "plain_path": {"value": plain_steps / plain_dt, "unit": "walk-steps/s",
                       "sample": f"the first {plain_problems} problems of the mix one at a time "
                                 f"({plain_epochs} epochs, {plain_steps} walk-steps) in {plain_dt:.2f} s"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / ALU_PEAK_TOPS, "traffic": None,
                     "kernel": "batch_kernel" if args.lockstep else "job_kernel",
                     "avg_launch_ms": run_ms / len(events),
                     "alg_ops_per_step": ops},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_mix(mix)
    print(json.dumps(line), flush=True)


def run_served(args, plain_budget_s=30.0):
    """A Poisson stream of sampling jobs served with continuous batching: jobs
    arrive in real time, are admitted by workspace footprint and active
    sequences, advance their epochs at their own pace in each server step (one
    time-sliced chained launch over every active job), and retire at the first
    merge that meets their stop rule."""
    import numpy as np
    import torch
    from paper_2002_03000_amd import Server

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    jobs = workloads.served_arrivals(rate_per_s=args.serve_rate, duration_s=args.serve_duration,
                                     target_rel_err=args.serve_target, tour_cap=args.serve_cap)
    pool = int(args.serve_pool_gib * (1 << 30))

    # warm-up: a few small jobs through their own server
    warm = Server(64 << 20, 4096)
    for j in jobs[:4]:
        warm.submit(j.problem.dim, min(j.problem.n_max, 100), j.problem.n_sequences, j.problem.seed + 99,
                    j.problem.tours_per_epoch, 4096, 0.0, stream_id=j.problem.stream)
    while warm.counts()[:2] != (0, 0):
        warm.step()
    warm.close()
    torch.cuda.synchronize()

    srv = Server(pool, args.serve_max_sequences)
    arrival, index = {}, {}
    lat = np.full(len(jobs), np.nan)
    steps_done, step_events, active_sum, n_steps = 0, [], 0, 0
    stops = {1: 0, 2: 0}
    nxt = 0
    t0 = time.perf_counter()
    last = t0
    while True:
        now = time.perf_counter() - t0
        while nxt < len(jobs) and jobs[nxt].arrival_s <= now:
            j = jobs[nxt]
            jid = srv.submit_problem(j.problem, j.tour_cap, j.target_rel_err)
            arrival[jid], index[jid] = j.arrival_s, nxt
            nxt += 1
        q, a, _ = srv.counts()
        if q == 0 and a == 0:
            if nxt >= len(jobs):
                break
            time.sleep(max(0.0, jobs[nxt].arrival_s - now))
            continue
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        fin = srv.step()
        ev1.record(stream)
        step_events.append((ev0, ev1))
        active_sum += a
        n_steps += 1
        tnow = time.perf_counter() - t0
        for jid in fin:
            info = srv.info(jid)
            if info["state"] != "done":
                raise RuntimeError(f"served job {index[jid]} failed: {info}")
            lat[index[jid]] = tnow - arrival[jid]
            steps_done += info["steps"]
            stops[info["stop"]] = stops.get(info["stop"], 0) + 1
            srv.release(jid)
        if time.perf_counter() - last > 10:
            last = time.perf_counter()
            _log(f"served: t={tnow:.1f} s, {nxt}/{len(jobs)} arrived, {int(np.sum(~np.isnan(lat)))} done, "
                 f"{q} queued, {a} active")
    elapsed = time.perf_counter() - t0
    srv.close()
    gpu_ms = sum(a.elapsed_time(b) for a, b in step_events)
    value = steps_done / elapsed

    # the plain path on the same jobs, one at a time (same results by construction)
    t1 = time.perf_counter()
    plain_steps, plain_jobs = 0, 0
    for j in jobs:
        one = Server(256 << 20, 4096)
        jid = one.submit_problem(j.problem, j.tour_cap, j.target_rel_err)
        while one.info(jid)["state"] not in ("done", "failed"):
            one.step()
        plain_steps += one.info(jid)["steps"]
        one.close()
        plain_jobs += 1
        if time.perf_counter() - t1 > plain_budget_s:
            break
    plain_dt = time.perf_counter() - t1

    ops = (ALG_OPS_PER_STEP[2] + ALG_OPS_PER_STEP[3]) / 2
    achieved = steps_done / (gpu_ms / 1e3) * ops / 1e12
    line = {
        "metric": "walk-steps/s (parallel flatPERM, 1 GPU)",
        "value": value,
        "unit": "walk-steps/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": elapsed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Poisson arrivals, seed 5; walks grown from parameters)",
        "config": {"workload": f"served: Poisson {args.serve_rate}/s for {args.serve_duration} s "
                               f"({len(jobs)} jobs), d in {{2,3}}, n_max in [50,2000], N=256, T=16, "
                               f"stop at rel. err <= {args.serve_target} or {args.serve_cap} tours",
                   "jobs": len(jobs), "tour_cap": args.serve_cap, "target_rel_err": args.serve_target,
                   "pool_bytes": pool, "max_active_sequences": args.serve_max_sequences},
        "latency_s": {"p50": float(np.nanpercentile(lat, 50)), "p99": float(np.nanpercentile(lat, 99)),
                      "max": float(np.nanmax(lat))},
        "server": {"steps": n_steps, "mean_active_jobs": active_sum / max(1, n_steps),
                   "stopped_by_target": stops.get(1, 0), "stopped_by_cap": stops.get(2, 0),
                   "gpu_busy_frac": gpu_ms / 1e3 / elapsed},
        "plain_path": {"value": plain_steps / plain_dt, "unit": "walk-steps/s",
                       "sample": f"the first {plain_jobs} jobs one at a time ({plain_steps} walk-steps) "
                                 f"in {plain_dt:.2f} s"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / ALU_PEAK_TOPS, "traffic": None,
                     "kernel": "server step (job_kernel, time-sliced)", "avg_launch_ms": gpu_ms / max(1, n_steps),
                     "alg_ops_per_step": ops},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_mix([j.problem for j in jobs])
    print(json.dumps(line), flush=True)


def tour_schedule(S, T=64):
    """S tours per sequence as epochs: 1, 1, 2, 4, ... doubling up to T, then T,
    the last epoch cut so that the total is exactly S."""
    out, head = [], [1]
    while 2 * sum(head) <= T:
        head.append(sum(head))
    for t in head + [T] * (S // T + 1):
        if sum(out) >= S:
            break
        out.append(min(t, S - sum(out)))
    return out


def run_compare(args):
    """Algorithm 1 (independent sequences, estimates combined by the arithmetic
    mean of eqn (7) and by the geometric mean) against Algorithm 2 (shared
    running averages) on the square lattice at n_max = 500: T_M of eqn (9)
    against a reference run 15x longer than the longest compared run, and the
    band width E of the eqn-(15) fit, for N sequences and S tours per
    sequence (the layout of the paper's Tables 3 and 4)."""
    import numpy as np
    import torch
    from paper_2002_03000_amd import ParallelFlatPERM, analysis, run_schedules

    torch.cuda.set_device(0)
    n_max = 500
    ref_p = workloads.PARALLEL_2D
    ref = ParallelFlatPERM(2, n_max, ref_p.n_sequences, 900_001, mode="shared")
    for T in ref_p.schedule():
        ref.run_tours(T)
        ref.merge_epoch()
    log_best, _, ref_tours = ref.estimates()
    ref.close()
    ref_fit = analysis.ratio_fit(log_best)
    _log(f"reference: {ref_tours} tours, mu {ref_fit['mu']:.6f}, gamma {ref_fit['gamma']:.4f}")

    Ns = [int(x) for x in args.compare_n.split(",")]
    Ss = [int(x) for x in args.compare_s.split(",")]
    R = args.compare_replicas
    # every (algorithm, N, S, replica) is one problem; all of them run together
    # as lock-step batched rounds (each problem's epochs exactly as alone)
    cells, probs, scheds = [], [], []
    seed = 910_000
    for N in Ns:
        for S in Ss:
            for mode in ("independent", "shared"):
                if mode == "shared" and N == 1:
                    continue                      # one sequence: the two algorithms coincide
                for r in range(R):
                    seed += 1
                    cells.append((mode, N, S, r))
                    probs.append(ParallelFlatPERM(2, n_max, N, seed, mode=mode, stream_id=len(probs)))
                    scheds.append(tour_schedule(S))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_schedules(probs, scheds)
    done = torch.cuda.Event()
    done.record()
    last = t0
    while not done.query():
        time.sleep(0.5)
        if time.perf_counter() - last > 10:
            last = time.perf_counter()
            _log(f"compare: {len(probs)} problems running, {last - t0:.0f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps = {"independent": 0, "shared": 0}
    results = {}
    for (mode, N, S, r), g in zip(cells, probs):
        steps[mode] += g.stats()["steps"]
        lc, _, _ = g.estimates()
        if mode == "independent":
            per = g.sequence_log_estimates()
            ests = {"alg1_mean": lc, "alg1_geometric": analysis.combine_geometric(per)}
        else:
            ests = {"alg2": lc}
        for kind, est in ests.items():
            fin = np.isfinite(est)
            top = int(np.max(np.nonzero(fin)[0])) if fin.any() else 0
            tm = analysis.total_abs_error(log_best, est, M=top) if top > 0 else float("nan")
            e = analysis.ratio_fit(est, n_max=top)["E"] if top > 3 else float("nan")
            results.setdefault((kind, N, S), []).append((tm, e, top))
        g.close()
    table = {"T_M": {}, "T_M_se": {}, "E": {}, "E_se": {}, "sampled_lengths_min": {}}
    for (kind, N, S), vals in sorted(results.items()):
        v = np.array(vals, dtype=np.float64)
        for name, col in (("T_M", 0), ("E", 1)):
            x = v[:, col]
            table[name].setdefault(kind, {}).setdefault(f"N={N}", {})[f"S={S}"] = float(np.nanmean(x))
            table[name + "_se"].setdefault(kind, {}).setdefault(f"N={N}", {})[f"S={S}"] = \
                float(np.nanstd(x, ddof=1) / np.sqrt(np.sum(np.isfinite(x)))) if len(x) > 1 else None
        table["sampled_lengths_min"].setdefault(kind, {}).setdefault(f"N={N}", {})[f"S={S}"] = int(v[:, 2].min())
    line = {
        "metric": "T_M (eqn 9) and band width E (eqn 15 fit): Algorithm 1 vs Algorithm 2, 1 GPU",
        "unit": "log units",
        "n_gpus": 1,
        "data": "synthetic (walks grown from parameters)",
        "config": {"workload": f"square lattice, n_max={n_max}, N in {Ns}, S tours per sequence in {Ss}, "
                               f"{R} replicas per cell (all cells in one set of batched rounds); "
                               f"reference: Algorithm 2, N=4096, {ref_tours} tours",
                   "reference_fit": ref_fit, "replicas": R},
        "tables": table,
        "walk_steps": {"alg1": steps["independent"], "alg2": steps["shared"]},
        "walk_steps_per_s_all": (steps["independent"] + steps["shared"]) / elapsed,
        "seconds": elapsed,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_mix(mix, budget_s=15.0):
    """The oracle on the mix's problems one at a time, epoch by epoch, until the
    time budget is spent."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    t0 = time.perf_counter()
    steps, done = 0, 0
    for p in mix:
        o = oracle.Oracle(p.dim, p.n_max, p.n_sequences, p.seed, stream=p.stream, threads=threads)
        for T in p.schedule():
            o.run_tours(T)
            o.merge_epoch()
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        steps += o.walk_steps()
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "walk-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the mix's problems in order, {done} epochs ({steps} walk-steps) in {dt:.2f} s"}


if __name__ == "__main__":
    main()
