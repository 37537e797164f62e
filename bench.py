#!/usr/bin/env python3
"""Benchmark: walk-steps/s of parallel flatPERM on one MI355X.

One benchmark step is one whole job of the default workload, the cubic-lattice
configuration: 16384 interacting flatPERM sequences (Algorithm 2), n_max = 1000,
a merge every 32 tours after the warm-up epochs, 8,388,608 tours in all,
followed by the read-out of log c_n.  Every step runs a fresh job with its own
seed; the workspaces are allocated and initialised before the timed region, so
the timed region holds exactly the hot path: growth with a_+ scans, weight
updates, prune/enrich, accumulation, merges and the estimate read-out.

Printed: one JSON line with the metric, a roofline object for the dominant
kernel (the growth kernel, timed with HIP events on its stream) with the
VALU, LDS and L2 fractions against ceilings probed on the device, the
critical-path bound, and the CPU oracle timed on bounded samples of the same
workload (single core and all cores, median of three each).
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


def lds_bytes_per_step(dim, n_max):
    """Algorithmic LDS bytes per walk-step: 2d - 1 occupancy-key reads and one
    insert of the packed key (4 bytes on the square lattice and, up to
    n_max = 1023, on the cubic one; 8 bytes for longer cubic walks)."""
    key = 4 if (dim == 2 or n_max <= 1023) else 8
    return 2 * dim * key
# Algorithmic L2 bytes per walk-step: the pooled sum of the length read (8),
# and where the sequence's sums live in global memory also its sum read and
# written (16) and its count read and written (8).
def l2_bytes_per_step(sums_global):
    return 32 if sums_global else 8
# MI355X 32-bit VALU peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6 T lane-op/s, the
# published FP32 vector rate (157.3 TFLOP/s) with one operation per FMA.  (FP64 operations,
# most of the prune/enrich arithmetic, issue at half that rate.)
ALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12

# the headline metric: walk-steps/s (with the relative error of c_{n_max} at
# the run's fixed budget beside it) of plain, batched and served flatPERM
METRIC = "walk-steps/s and c_n rel. error at fixed budget, batched/served vs plain, 1 GPU"

PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2002_03000_amd", "csrc", "pperm_kernels.hip")


def profile_field(name, field):
    """One figure of a committed counter summary, or None when the summary is
    missing or the kernel source has changed since it was taken."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_code_sha256") != kernel_code_digest() or field not in fields:
        return None
    return fields[field]


def measured_traffic(name):
    """HBM bytes per launch of the growth kernel (FETCH_SIZE + WRITE_SIZE,
    calibrated), from a committed counter summary of the current kernel."""
    v = profile_field(name, "traffic_bytes_per_launch")
    return None if v is None else int(v)


def issue_fraction(steps_per_s, kernel, workload, probes):
    """The kernel's instruction issue against the SIMD issue ceilings the
    probes measure: instructions per walk-step (the SQ_INSTS counters of a
    committed summary of the current kernel) times the walk-step rate, against
    the rates of independent mixed vector/scalar streams, of vector and scalar
    instructions that feed each other (at eight and at four waves per SIMD),
    and of scalar-only streams."""
    v = profile_field(f"{kernel}_{workload}_sq_counters.md", "instructions_per_step")
    if v is None or not probes:
        return None
    per_step = float(v)
    ach = steps_per_s * per_step
    hz = probes["simds"] * probes["clock_khz"] * 1e3
    return {"instructions_per_step": per_step, "achieved": ach, "unit": "wave-instr/s",
            "peak_mixed": probes["mixed_instr_per_s"], "frac_mixed": ach / probes["mixed_instr_per_s"],
            "peak_dependent": probes["dependent_instr_per_s"],
            "frac_dependent": ach / probes["dependent_instr_per_s"],
            "peak_dependent_4_waves": probes["dependent4_instr_per_s"],
            "peak_scalar_only": probes["salu_instr_per_s"],
            "per_simd_cycle": ach / hz, "peak_mixed_per_simd_cycle": probes["mixed_instr_per_s"] / hz}


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_rate(p, threads, budget_s):
    """The oracle, as it stands, on the job's epochs in order (run + merge,
    every sequence) until budget_s is spent, stopping at an epoch boundary.
    Returns (walk-steps/s, walk-steps, epochs, seconds)."""
    import oracle
    o = oracle.Oracle(p.dim, p.n_max, p.n_sequences, p.seed, stream=p.stream, threads=threads)
    done, t0 = 0, time.perf_counter()
    for T in p.schedule():
        o.run_tours(T)
        o.merge_epoch()
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    steps = o.walk_steps()
    return steps / dt, steps, done, dt


def cpu_baseline(p, budget_s=4.0, runs=3):
    """The oracle on bounded samples of the same job: single core and all host
    cores, each the median of `runs` runs of about budget_s seconds."""
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    single = [oracle_rate(p, 1, budget_s) for _ in range(runs)]
    allc = [oracle_rate(p, threads, budget_s) for _ in range(runs)]
    med = lambda xs: float(sorted(x[0] for x in xs)[len(xs) // 2])
    a = sorted(allc, key=lambda x: x[0])[len(allc) // 2]
    return {"value": med(allc), "unit": "walk-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the job's first epochs in order, about {budget_s:.0f} s per run, median of {runs} "
                      f"runs (all cores: {a[2]} epochs, {a[1]} walk-steps in {a[3]:.2f} s)",
            "single_core": {"value": med(single), "runs": [x[0] for x in single],
                            "epochs": [x[2] for x in single]},
            "all_cores": {"value": med(allc), "runs": [x[0] for x in allc], "epochs": [x[2] for x in allc]},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def probed_roofline(steps_per_s, ops_per_step, lds_per_step, l2_per_step, probes):
    """Achieved fractions of the probed VALU, LDS and L2 ceilings at the growth
    kernel's walk-step rate (algorithmic work per step)."""
    out = {}
    for name, per_step, peak, unit in (
            ("valu", ops_per_step, probes["valu_lane_ops_per_s"], "lane-op/s"),
            ("lds", lds_per_step, probes["lds_bytes_per_s"], "B/s"),
            ("l2", l2_per_step, probes["l2_bytes_per_s"], "B/s")):
        ach = steps_per_s * per_step
        out[name] = {"achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak, "per_step": per_step}
    out["binding_of_three"] = max(("valu", "lds", "l2"), key=lambda k: out[k]["frac"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="default 3 (long2d: 1)")
    ap.add_argument("--warmup", type=int, default=None, help="default 1 (long2d: 0)")
    ap.add_argument("--workload", default="parallel3d", choices=sorted(WORKLOADS))
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
    ap.add_argument("--compare-t", default="64,1", help="compare: Algorithm 2 tours per epoch")
    ap.add_argument("--compare-nmax", type=int, default=500, help="compare: maximum walk length")
    ap.add_argument("--compare-step-cap", type=int, default=0,
                    help="compare: walk-steps one sequence may take per call (0: that of a 64-tour epoch)")
    ap.add_argument("--compare-short-t-max-s", type=int, default=1000,
                    help="compare: Algorithm 2 with T < 64 only up to this many tours per sequence")
    ap.add_argument("--serve-duration", type=float, default=60.0, help="served: arrival window (s)")
    ap.add_argument("--serve-rate", type=float, default=50.0, help="served: arrivals per second")
    ap.add_argument("--serve-cap", type=int, default=1_000_000, help="served: tour cap per job")
    ap.add_argument("--serve-target", type=float, default=1e-3, help="served: relative-error target")
    ap.add_argument("--serve-pool-gib", type=float, default=64.0)
    ap.add_argument("--serve-max-sequences", type=int, default=262144)
    ap.add_argument("--plain-full", action="store_true",
                    help="batched / served: time the plain path on every problem, not a stratified subset")
    ap.add_argument("--accuracy-runs", type=int, default=None,
                    help="independent runs for the c_n accuracy report (default 8; long2d 0; 0: none)")
    ap.add_argument("--reference-factor", type=int, default=16,
                    help="accuracy report: the reference run has this many times the steady tours")
    ap.add_argument("--plain-strata", type=int, default=32,
                    help="batched / served: strata (by walk-steps) of the plain-path subset")
    ap.add_argument("--no-probe", action="store_true", help="skip the VALU / LDS / L2 ceiling probes")
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

    if args.accuracy_runs is None:
        args.accuracy_runs = 0 if args.workload == "long2d" else 8
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
        # timed on the first steady-state epoch, after the warm-up epochs
        head = len(p.schedule()) - p.epochs + 1
        best, tuning = autotune(p.dim, p.n_max, p.n_sequences, mode=p.mode,
                                trial=tuple(p.schedule()[:head + 1]), untimed=head)
        args.walks_per_wave, args.hash_slots = best["walks_per_wave"], best["hash_slots"]
        args.sums_global = best["sums_global"]

    def make(seed):
        return ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, seed, mode=p.mode,
                                walks_per_wave=args.walks_per_wave, hash_slots=args.hash_slots,
                                sums_global=args.sums_global)

    sched = p.schedule()

    last_note = [time.perf_counter()]

    def note(msg):
        # a progress line at most every 20 s (long jobs: one epoch can take seconds)
        if time.perf_counter() - last_note[0] > 20:
            last_note[0] = time.perf_counter()
            _log(msg)

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
        out = g.estimates()
        note(f"{args.workload}: a job done")
        return out

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
    probes = None if args.no_probe else probe_ceilings()
    line = {
        "metric": METRIC,
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
                     "alg_ops_per_step": ops,
                     "probed": probed_roofline(kernel_rate, ops, lds_bytes_per_step(p.dim, p.n_max),
                                               l2_bytes_per_step(args.sums_global or args.workload == "long2d"),
                                               probes) if probes else None,
                     "issue": issue_fraction(kernel_rate, kernel, args.workload, probes)},
        "probes": probes,
        "cpu_baseline": None,
    }
    if args.workload == "long2d":
        line["gamma_nmin"] = gamma_extrapolation(results[0][0], p.n_max)
    if not args.no_latency_bound:
        line["latency_bound"] = latency_bound(p, make, sched, elapsed / args.steps, args.sums_global)
    if args.accuracy_runs > 1 and not args.epochs:
        line["accuracy"] = accuracy(p, make, job, results, args.accuracy_runs, args.reference_factor)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(line), flush=True)


def probe_ceilings():
    """VALU, LDS and L2 ceilings of this device, measured by the library's probes."""
    from paper_2002_03000_amd import probe
    return probe()


def gamma_extrapolation(log_c, n_max):
    """gamma from eqn-(16) fits over n >= n_min, extrapolated against n_min
    (three parameters, and two with the literature mu of the square lattice)."""
    from paper_2002_03000_amd import analysis
    n_mins = [m for m in (50, 100, 200, 400, 800, 1600) if m < n_max // 4]
    if len(n_mins) < 3:
        return None
    free = analysis.gamma_nmin_extrapolation(log_c, n_mins, n_max=n_max)
    fixed = analysis.gamma_nmin_extrapolation(log_c, n_mins, n_max=n_max, log_mu=0.970081147258)
    return {"three_parameter": free, "two_parameter_mu_fixed": fixed}


def accuracy(p, make, job, results, runs, factor):
    """The c_n relative error at this fixed budget: ĉ_{n_max} over `runs`
    independent runs of the job (the timed ones and more with the next seeds),
    their relative standard deviation, their bias against a reference run of
    the same configuration with `factor` times the steady-state tours, and
    T_M of eqn (9) over n <= n_max against that reference, per run.  Outside
    the timed region."""
    import numpy as np
    from paper_2002_03000_amd import analysis
    logs = [r[0] for r in results]
    for i in range(len(results), runs):
        g = make(p.seed + i)
        logs.append(job(g)[0])
        g.close()
    head = p.schedule()[:len(p.schedule()) - p.epochs + 1]
    ref_sched = head + [p.tours_per_epoch] * ((p.epochs - 1) * factor)
    g = make(p.seed + 5000)
    t0 = time.perf_counter()
    for k, T in enumerate(ref_sched):
        g.run_tours(T)
        g.merge_epoch()
        if k % 50 == 49:
            g.sync()
            _log(f"accuracy: reference epoch {k + 1}/{len(ref_sched)}, {time.perf_counter() - t0:.0f} s")
    ref, _, ref_tours = g.estimates()
    g.close()
    top = np.array([lc[p.n_max] for lc in logs])
    ratio = np.exp(top - ref[p.n_max])                     # ĉ / ĉ_ref at n_max
    tm = [analysis.total_abs_error(ref, lc, M=p.n_max) for lc in logs]
    return {"runs": len(logs), "reference_tours": int(ref_tours), "job_tours": int(p.total_tours),
            "c_nmax_rel_std": float(np.std(ratio, ddof=1) / np.mean(ratio)),
            "c_nmax_bias_vs_reference": float(np.mean(ratio) - 1.0),
            "c_nmax_bias_se": float(np.std(ratio, ddof=1) / np.sqrt(len(ratio))),
            "T_M_mean": float(np.mean(tm)), "T_M_max": float(np.max(tm)),
            "reference_log_c_nmax": float(ref[p.n_max])}


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
    t_note = time.perf_counter()
    for e, T in enumerate(sched):
        g.run_tours(T)
        g.merge_epoch()
        st = g.sequence_stats()["steps"]
        crit += int((st - prev).max())
        prev = st
        if time.perf_counter() - t_note > 20:
            t_note = time.perf_counter()
            _log(f"latency bound: replay epoch {e + 1}/{len(sched)}")
    g.close()
    # one wave alone: a single sequence through the same schedule (the first
    # epochs warm its own estimates), timed over the full-length epochs
    lone = ParallelFlatPERM(p.dim, p.n_max, 1, p.seed + 77, sums_global=sums_global)
    head = len(sched) - p.epochs + 1
    for T in sched[:head]:
        lone.run_tours(T)
        lone.merge_epoch()
        torch.cuda.synchronize()
        if time.perf_counter() - t_note > 20:
            t_note = time.perf_counter()
            _log("latency bound: one sequence alone, warm-up epochs")
    torch.cuda.synchronize()
    s0 = lone.stats()["steps"]
    t0 = time.perf_counter()
    for k, T in enumerate(sched[head:head + 8]):
        lone.run_tours(T)
        lone.merge_epoch()
        # (a wait per epoch, tens of microseconds against epochs of milliseconds
        # or more, so that a long run can say how far it is; a stream wait, not
        # pperm_sync: a lone long walk may stop on its step cap, and its steps up
        # to there still time the step)
        torch.cuda.synchronize()
        if time.perf_counter() - t_note > 20:
            t_note = time.perf_counter()
            _log(f"latency bound: one sequence alone, timed epoch {k + 1}/8")
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


def stratified_plain(steps_each, run_one, strata, full):
    """The plain path's time for a whole problem set, at equal work.  Every
    problem's walk-steps are known exactly from the batched or served run
    (both paths give the same bits, hence the same steps).  With `full` every
    problem is timed alone; otherwise the problems are sorted by walk-steps
    into `strata` groups, the middle problem of each group is timed alone, and
    its time scaled by its group's walk-steps over its own stands for the
    group.  run_one(i) returns (seconds, walk-steps) of problem i alone."""
    import numpy as np
    steps_each = np.asarray(steps_each, dtype=np.int64)
    order = np.argsort(steps_each, kind="stable")
    groups = [[int(i)] for i in order] if full else \
        [list(map(int, g)) for g in np.array_split(order, min(strata, len(order))) if len(g)]
    est, timed_s, timed_steps, last = 0.0, 0.0, 0, time.perf_counter()
    for k, grp in enumerate(groups):
        rep = grp[len(grp) // 2]
        dt, st = run_one(rep)
        if st != int(steps_each[rep]):
            raise RuntimeError(f"problem {rep}: {st} walk-steps alone, {int(steps_each[rep])} in the mix")
        est += dt * float(steps_each[grp].sum()) / max(st, 1)
        timed_s += dt
        timed_steps += st
        if time.perf_counter() - last > 10:
            last = time.perf_counter()
            _log(f"plain path: {k + 1}/{len(groups)} timed, {timed_s:.1f} s")
    total = int(steps_each.sum())
    return {"value": total / est, "unit": "walk-steps/s", "seconds_for_the_set": est,
            "walk_steps": total, "timed_problems": len(groups), "timed_seconds": timed_s,
            "timed_walk_steps": timed_steps,
            "method": "every problem alone" if full else
            f"one problem per stratum of {len(groups)} strata by walk-steps, scaled by the stratum's walk-steps"}


def run_batched(args):
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

    from paper_2002_03000_amd import job_report, run_job
    batch = Batch(len(mix))
    report = None
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
            report = job_report(ws)
            del ws
        ests = [g.estimates() for g in probs]
        torch.cuda.synchronize()
        elapsed_total += time.perf_counter() - t0
        by_dim = {2: 0, 3: 0}
        per = [g.stats()["steps"] for g in probs]
        if k == 0:
            steps_first = per
        for p, st in zip(mix, per):
            by_dim[p.dim] += st
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
    # algorithmic LDS and L2 bytes per step, weighted by each problem's steps
    # (the mix's sums stay in LDS: n_max <= 2048)
    w_steps = max(1, sum(per))
    lds_avg = sum(int(st) * lds_bytes_per_step(p.dim, p.n_max) for p, st in zip(mix, per)) / w_steps
    probes = None if args.no_probe else probe_ceilings()

    # the plain path on the same problems and seeds (those of the first timed
    # job), one problem at a time through pperm_run_tours / pperm_merge_epoch
    def plain_one(i):
        g = make(mix[i], 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for T in scheds[i]:
            g.run_tours(T)
            g.merge_epoch()
        g.estimates()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = g.stats()["steps"]
        g.close()
        return dt, st

    plain = stratified_plain(steps_first, plain_one, args.plain_strata, args.plain_full)
    _log(f"plain path: {plain['timed_problems']} problems timed in {plain['timed_seconds']:.1f} s, "
         f"{plain['value']:.3e} walk-steps/s")

    total_tours = sum(p.total_tours for p in mix)
    line = {
        "metric": METRIC,
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
        "plain_path": plain,
        "batched_vs_plain": value / plain["value"],
        "job_report": report,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / ALU_PEAK_TOPS, "traffic": None,
                     "kernel": "batch_kernel" if args.lockstep else "job_kernel",
                     "avg_launch_ms": run_ms / len(events),
                     "alg_ops_per_step": ops,
                     "probed": probed_roofline(steps_total / (run_ms / 1e3), ops, lds_avg, l2_bytes_per_step(False),
                                               probes) if probes else None},
        "probes": probes,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_mix(mix)
    print(json.dumps(line), flush=True)


def run_served(args):
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
    job_steps = [0] * len(jobs)
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
            job_steps[index[jid]] = info["steps"]
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
    _log(f"served: {len(jobs)} jobs, {steps_done} walk-steps in {elapsed:.1f} s = {value:.3e} walk-steps/s, "
         f"latency p50 {np.nanpercentile(lat, 50):.1f} s p99 {np.nanpercentile(lat, 99):.1f} s, "
         f"{n_steps} server steps, {active_sum / max(1, n_steps):.1f} jobs active on average, "
         f"stops {stops}, GPU busy {gpu_ms / 1e3 / elapsed:.3f}")

    # the plain path on the same jobs: each job alone through pperm_run_tours /
    # pperm_merge_epoch, its stop rule checked on the host after every merge
    # (the same rule, the same bits, hence the same walk-steps)
    from paper_2002_03000_amd import ParallelFlatPERM

    def plain_one(i):
        j = jobs[i]
        p = j.problem
        g = ParallelFlatPERM(p.dim, p.n_max, p.n_sequences, p.seed, mode=p.mode, stream_id=p.stream,
                             group_stats=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = 0
        epochs = j.tour_cap // (p.n_sequences * p.tours_per_epoch) + 8
        for T in workloads.Problem(p.dim, p.n_max, p.n_sequences, p.tours_per_epoch, epochs, p.seed,
                                   stream=p.stream).schedule():
            g.run_tours(T)
            g.merge_epoch()
            M += p.n_sequences * T
            rel, _ = g.error_estimate()
            if (j.target_rel_err > 0 and rel <= j.target_rel_err) or M >= j.tour_cap:
                break
        g.estimates()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = g.stats()["steps"]
        g.close()
        return dt, st

    done_idx = [i for i in range(len(jobs)) if job_steps[i] > 0]
    plain = stratified_plain([job_steps[i] for i in done_idx], lambda k: plain_one(done_idx[k]),
                             min(args.plain_strata, 16), args.plain_full)
    _log(f"plain path: {plain['timed_problems']} jobs timed in {plain['timed_seconds']:.1f} s, "
         f"{plain['value']:.3e} walk-steps/s")

    # algorithmic work per step, weighted by each job's steps
    w_steps = max(1, sum(job_steps))
    ops = sum(st * ALG_OPS_PER_STEP[j.problem.dim] for j, st in zip(jobs, job_steps)) / w_steps
    lds_avg = sum(st * lds_bytes_per_step(j.problem.dim, j.problem.n_max) for j, st in zip(jobs, job_steps)) / w_steps
    achieved = steps_done / (gpu_ms / 1e3) * ops / 1e12
    probes = None if args.no_probe else probe_ceilings()
    line = {
        "metric": METRIC,
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
        "plain_path": plain,
        "served_vs_plain": value / plain["value"],
        "offered_walk_steps_per_s": steps_done / args.serve_duration,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / ALU_PEAK_TOPS, "traffic": None,
                     "kernel": "server step (job_kernel, time-sliced)", "avg_launch_ms": gpu_ms / max(1, n_steps),
                     "alg_ops_per_step": ops,
                     "probed": probed_roofline(steps_done / (gpu_ms / 1e3), ops, lds_avg, l2_bytes_per_step(False),
                                               probes) if probes else None},
        "probes": probes,
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
    running averages, merged every T tours for each T of --compare-t; T = 1 is
    closest to the paper's continuous sharing) on the square lattice: T_M of
    eqn (9) against a longer reference run of Algorithm 2, the band width E of
    the eqn-(16) fit, and log c_{n_max}, for N sequences and S tours per
    sequence (the layout of the paper's Tables 1-4 at --compare-nmax 10000).
    Every cell is --compare-replicas independent runs; all of them chain their
    epochs on the device in one launch, each at its own pace (each problem's
    epochs exactly as alone)."""
    import numpy as np
    import torch
    from paper_2002_03000_amd import ParallelFlatPERM, analysis

    torch.cuda.set_device(0)
    n_max = args.compare_nmax
    # the reference: Algorithm 2 with many sequences, many more tours than any
    # compared run (the square-lattice job at n_max <= 500, the long-walk job
    # at longer lengths)
    ref_p = workloads.PARALLEL_2D if n_max <= 500 else workloads.LONG_2D
    ref = ParallelFlatPERM(2, n_max, ref_p.n_sequences, 900_001, mode="shared")
    t0 = time.perf_counter()
    for T in ref_p.schedule():
        ref.run_tours(T)
        ref.merge_epoch()
    log_best, _, ref_tours = ref.estimates()
    ref.close()
    ref_fit = analysis.ratio_fit(log_best)
    _log(f"reference: {ref_tours} tours in {time.perf_counter() - t0:.0f} s, mu {ref_fit['mu']:.6f}, "
         f"gamma {ref_fit['gamma']:.4f}, log c_n_max {log_best[n_max]:.3f}")

    Ns = [int(x) for x in args.compare_n.split(",")]
    Ss = [int(x) for x in args.compare_s.split(",")]
    Ts = [int(x) for x in args.compare_t.split(",")]
    R = args.compare_replicas
    # the same step watchdog per call for every epoch length: the default one
    # of a 64-tour epoch (a one-tour epoch's default would stop the enrichment
    # cascades short epochs meet at rarely reached lengths), or a smaller one
    # that bounds the run's time at long n_max
    cap = args.compare_step_cap or min(2 ** 31 - 1, 4096 * 64 * (n_max + 1))
    # cells: (mode, T, N, S, replica, indices of its problems).  Algorithm 1's N
    # independent sequences are N one-sequence problems (a flatPERM sequence
    # alone; with one sequence the epoch length changes nothing but rounding
    # order), Algorithm 2 is one problem of N sequences
    cells, probs, scheds = [], [], []
    seed = 910_000
    for N in Ns:
        for S in Ss:
            kinds = [("independent", 64)] + [("shared", T) for T in Ts]
            for mode, T in kinds:
                if mode == "shared" and N == 1 and T != Ts[0]:
                    continue                      # one sequence: T changes nothing
                if mode == "shared" and T < 64 and S > args.compare_short_t_max_s:
                    continue                      # short epochs only up to this many tours
                for r in range(R):
                    seed += 1
                    members = N if mode == "independent" else 1
                    idx = []
                    for _ in range(members):
                        idx.append(len(probs))
                        probs.append(ParallelFlatPERM(2, n_max, 1 if mode == "independent" else N, seed,
                                                      mode="shared", stream_id=len(probs), step_cap=cap))
                        scheds.append(tour_schedule(S, T))
                    cells.append((mode, T, N, S, r, idx))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    from paper_2002_03000_amd import run_job, job_report
    last_log = [time.perf_counter()]

    def wait(label):
        # wait for the stream, saying what runs at least every 10 s
        ev = torch.cuda.Event()
        ev.record()
        while not ev.query():
            time.sleep(0.05)
            if time.perf_counter() - last_log[0] > 10:
                last_log[0] = time.perf_counter()
                _log(f"compare: {label}, {last_log[0] - t0:.0f} s")

    # every problem chains its epochs on the device, each at its own pace
    job_ws = run_job(probs, scheds)
    wait(f"{len(probs)} problems chained on the device")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    report = job_report(job_ws)
    del job_ws
    from paper_2002_03000_amd import PPermError
    steps = {}
    results = {}
    capped = {}
    for (mode, T, N, S, r, idx) in cells:
        key = f"{mode} T={T} N={N} S={S}"
        try:
            lcs = [probs[i].estimates()[0] for i in idx]
        except PPermError as exc:
            # a sequence hit the step cap (an enrichment cascade at lengths
            # no sequence had reached): counted, left out of the tables
            capped[key] = capped.get(key, 0) + 1
            _log(f"compare: {key} replica {r}: {exc}")
            continue
        st = sum(probs[i].stats()["steps"] for i in idx)
        if mode == "independent":
            ests = {"alg1_mean": analysis.combine_mean(lcs), "alg1_geometric": analysis.combine_geometric(lcs)}
            steps["alg1"] = steps.get("alg1", 0) + st
        else:
            ests = {f"alg2_T{T}": lcs[0]}
            steps[f"alg2_T{T}"] = steps.get(f"alg2_T{T}", 0) + st
        for kind, est in ests.items():
            fin = np.isfinite(est)
            top = int(np.max(np.nonzero(fin)[0])) if fin.any() else 0
            tm = analysis.total_abs_error(log_best, est, M=top) if top > 0 else float("nan")
            e = analysis.ratio_fit(est, n_max=top)["E"] if top > 3 else float("nan")
            results.setdefault((kind, N, S), []).append((tm, e, top, est[n_max]))
    for g in probs:
        g.close()
    table = {"T_M": {}, "T_M_se": {}, "E": {}, "E_se": {}, "log_c_nmax": {}, "log_c_nmax_se": {},
             "sampled_lengths_min": {}}
    for (kind, N, S), vals in sorted(results.items()):
        v = np.array(vals, dtype=np.float64)
        for name, col in (("T_M", 0), ("E", 1), ("log_c_nmax", 3)):
            x = v[:, col]
            ok = np.isfinite(x)
            table[name].setdefault(kind, {}).setdefault(f"N={N}", {})[f"S={S}"] = \
                float(np.mean(x[ok])) if ok.any() else None
            table[name + "_se"].setdefault(kind, {}).setdefault(f"N={N}", {})[f"S={S}"] = \
                float(np.std(x[ok], ddof=1) / np.sqrt(ok.sum())) if ok.sum() > 1 else None
        table["sampled_lengths_min"].setdefault(kind, {}).setdefault(f"N={N}", {})[f"S={S}"] = int(v[:, 2].min())
    line = {
        "metric": "T_M (eqn 9), band width E (eqn 16 fit) and log c_n_max: Algorithm 1 vs Algorithm 2, 1 GPU",
        "unit": "log units",
        "n_gpus": 1,
        "data": "synthetic (walks grown from parameters)",
        "config": {"workload": f"square lattice, n_max={n_max}, N in {Ns}, S tours per sequence in {Ss}, "
                               f"Algorithm 2 merged every T in {Ts} tours (after warm-up epochs 1, 1, 2, ... "
                               f"up to T), {R} replicas per cell; reference: Algorithm 2, "
                               f"N={ref_p.n_sequences}, {ref_tours} tours",
                   "reference_fit": ref_fit, "reference_log_c_nmax": float(log_best[n_max]), "replicas": R},
        "tables": table,
        "walk_steps": steps,
        "stopped_by_step_cap": capped,
        "step_cap_per_call": cap,
        "job_report": report,
        "walk_steps_per_s_all": sum(steps.values()) / elapsed,
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
