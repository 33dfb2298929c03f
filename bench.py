#!/usr/bin/env python3
"""Throughput of the bosonic PIMD step on one MI355X.

Workload: N=1600 Gaussian-interacting bosons in a 2-D harmonic trap, P=32 beads, beta=3,
xi=1, A=0.5, s=0.5 (hbar = m = omega = 1), seeded positions N(0, 2^2), Maxwell-Boltzmann
momenta, massive Nose-Hoover chains of length 4, dt=0.01.  A step is one full MD step:
thermostat and integrator halves, all-pairs forces of every slice, springs and trap, the
forward and backward exchange recursions, connection probabilities and end-bead forces.

Reported: aggregate replica-steps/s of the mixed-precision batched path (R replicas of the
workload, seeds 303+r, in one context), the plain FP64 single-replica path beside it, the
bead-updates/s (= steps/s * sum_r N P), the roofline of the dominant kernel (per-launch HIP
events on the stream it runs on), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2404_02628_amd.workloads import WORKLOADS, initial_state  # noqa: E402

PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector (published)
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (published)
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E (published)


def progress(msg):
    """One line per finished phase on stderr (the JSON result is the only line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_systems(R):
    base = WORKLOADS["large_gauss"]
    return [base.with_(seed=base.seed + r) for r in range(R)]


def make_ctx(precision, R, nhc_len=4, knobs=None):
    from paper_2404_02628_amd.pimd import Context
    systems = bench_systems(R)
    kw = knobs.as_kwargs() if knobs is not None else {}
    ctx = Context(systems, precision=precision, nhc_len=nhc_len, density_bins=64, density_rmax=8.0,
                  trace_capacity=0, **kw)
    for r, s in enumerate(systems):
        x, p = initial_state(s)
        ctx.set_state(r, x, p)
    return ctx, systems


def timed_steps(ctx, steps):
    import torch
    ctx.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps, 0)
    ctx.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_path(precision, R, steps, warmup, profile=False, knobs=None):
    """Times `steps` MD steps after `warmup`; with profile, every kernel launch of the timed region
    is bracketed by HIP events on the stream it runs on, and the per-kind times are returned."""
    ctx, systems = make_ctx(precision, R, knobs=knobs)
    times = None
    try:
        ctx.step(warmup, 0)
        if profile:
            ctx.profile(True)
        dt = timed_steps(ctx, steps)
        if profile:
            times = ctx.kernel_times()
            ctx.profile(False)
    finally:
        ctx.close()
    return dt, systems, times


def algorithmic_work(kind, systems, P, D, precision="mixed"):
    """(bound, units per launch, work per unit, unit name, peak) for one kernel kind."""
    npairs = sum(P * s.n * (s.n - 1) // 2 for s in systems if s.pair_amp > 0)  # unordered pairs
    tri = sum(s.n * (s.n + 1) // 2 for s in systems)
    dofs = sum(D * P * s.n for s in systems)
    parts = sum(s.n for s in systems)
    if kind == "pair":
        # per unordered pair (Eq. 20 counts each once): D subtractions, D FMAs (|dr|^2), one exp,
        # D FMAs for the force on each of the two particles = 7D + 1 flops (FMA = 2)
        return "alu", npairs, 7 * D + 1, "TFLOP/s", PEAK_FP32_TFLOPS
    if kind == "recursion":
        # two recursions, each N(N+1)/2 terms; per term (FP64, FMA = 2): distance D + 2D, exponent 4,
        # table exp 17, sum 1, payload sums 2(D+1)  ->  5D + 24 flops
        return "alu", 2 * tri, 5 * D + 24, "TFLOP/s", PEAK_FP64_TFLOPS
    if kind == "springs":
        # per dof: read x, write f (8 B each), FP32 shadow (4 B, mixed); per particle: end beads,
        # link and internal energy ((2D + 2) x 8 B), spread over its D P dofs
        per = 16 + (4 if precision == "mixed" else 0) + (2 * D + 2) * 8 / (D * P)
        return "hbm", dofs, per, "GB/s", PEAK_HBM_GBS
    # the chain positions are kept as per-wavefront sums (a few bytes per 64 dofs, not counted)
    if kind == "integrate_first":
        # read x, p, f, v_eta[4]; write x, p, v_eta[4]
        return "hbm", dofs, 8 * (7 + 6), "GB/s", PEAK_HBM_GBS
    if kind == "integrate_second":
        # read p, f, f_pair, v_eta[4]; write p, f, v_eta[4]
        return "hbm", dofs, 8 * (7 + 6), "GB/s", PEAK_HBM_GBS
    if kind == "integrate_fused":
        # read x, p, f, f_pair, v_eta[4]; write x, p, v_eta[4]
        return "hbm", dofs, 8 * (8 + 6), "GB/s", PEAK_HBM_GBS
    if kind == "exchange_forces":
        # per particle: potentials and links (7), row averages (2D + 1), end beads and their
        # neighbours (6D) read, bead 1 and bead P forces read and written (4D)  ->  (8 + 12D) x 8 B
        return "hbm", parts, 8 * (8 + 12 * D), "GB/s", PEAK_HBM_GBS
    return "hbm", dofs, 8, "GB/s", PEAK_HBM_GBS


KERNEL_OF_KIND = {("pair", "mixed"): "k_pair_sym_f32", ("pair", "fp64"): "k_pair_sym_f64",
                  ("recursion", "mixed"): "k_recursion", ("recursion", "fp64"): "k_recursion"}


def traffic_bytes(kind, precision, R):
    """HBM bytes per launch of the kernel from its committed counter record (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, each scaled by what the counter reads for a plain device copy of known size), or None
    when there is no record for this batch size or the kernel's sources changed since it was taken."""
    import hashlib
    import re
    name = KERNEL_OF_KIND.get((kind, precision))
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", f"{name}_large_gauss_counters.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json traffic-record\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("replicas") != R or rec.get("precision") != precision:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(src.encode() + b"\0" + f.read() + b"\0")
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0


def _oracle_worker(args):
    """One oracle replica of the workload: `steps` MD steps after its initial force evaluation,
    started together with the other workers (barrier); returns (steps, t_start, t_end)."""
    r, steps, barrier = args
    import oracle
    s = WORKLOADS["large_gauss"].with_(seed=WORKLOADS["large_gauss"].seed + r)
    par = oracle.OracleParams(n=s.n, p=s.p, dim=s.dim, beta=s.beta, xi=s.xi, pair_amp=s.pair_amp,
                              pair_width=s.pair_width)
    md = oracle.OracleMD(dt=s.dt, nhc_len=4)
    x, p = initial_state(s)
    f, _ = oracle.compute_forces(par, x)
    eta = np.zeros((4,) + x.shape)
    veta = np.zeros_like(eta)
    if barrier is not None:
        barrier.wait()
    t0 = time.perf_counter()
    oracle.step(par, md, x, p, eta, veta, f, steps)
    return steps, t0, time.perf_counter()


_BARRIER = None


def _pool_init(barrier):
    global _BARRIER
    _BARRIER = barrier


def _oracle_worker_in_pool(args):
    return _oracle_worker(args + (_BARRIER,))


def cpu_baseline(single_steps=16, worker_steps=6):
    """The CPU oracle as it stands (plain sequential FP64 C, one thread per replica) on bounded
    samples of the workload: one replica on one core, then one independent replica per host core
    (the replicas of a batch are independent, so this is how the oracle uses a multi-core host).
    Runs before anything touches the GPU, so that the worker processes can be forked."""
    import multiprocessing as mp
    import platform
    import oracle
    if not os.path.exists(oracle.lib_path()):
        oracle.build()
    steps1, a, b = _oracle_worker((0, single_steps, None))
    one = steps1 / (b - a)
    # the host's CPU share: the affinity mask, capped at the 16 cores a one-GPU machine grants
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    ctx = mp.get_context("fork")
    barrier = ctx.Barrier(cores)
    with ctx.Pool(cores, initializer=_pool_init, initargs=(barrier,)) as pool:
        res = pool.map(_oracle_worker_in_pool, [(r, worker_steps) for r in range(cores)])
    t0 = min(r[1] for r in res)
    t1 = max(r[2] for r in res)
    agg = sum(r[0] for r in res) / (t1 - t0)
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": agg, "unit": "replica-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} independent N=1600, P=32 replicas (seeds 303+r), {worker_steps} full MD steps "
                      f"each, one process per core, started together; plain sequential FP64 C oracle",
            "single_core_steps_per_s": one,
            "single_core_sample": f"{single_steps} full MD steps of one replica on one core",
            "cpu_model": model, "host_logical_cpus": os.cpu_count()}


def energy_precision_error(R, knobs_mixed, knobs_fp64):
    """Mixed vs FP64 estimators of the same R replicas at their seeded configurations, each in the
    launch configuration that is timed (batched symmetric pair kernel in mixed precision): the
    largest relative difference over the replicas, per estimator."""
    out = {}
    for prec, kn in (("fp64", knobs_fp64), ("mixed", knobs_mixed)):
        ctx, _ = make_ctx(prec, R, knobs=kn)
        try:
            ctx.compute_forces()
            out[prec] = [ctx.energies(r) for r in range(R)]
        finally:
            ctx.close()
    rel = {}
    for k in ("e_prim", "e_vir", "u_pair", "v_exch"):
        rel[k] = max(abs(m[k] - f[k]) / max(abs(f[k]), 1e-300) for m, f in zip(out["mixed"], out["fp64"]))
    return rel


def lse2_latency_ns():
    """ns of one dependent two-term log-sum-exp (the library's FP64 exp and log, one wavefront),
    from the committed issue-rate record, or None."""
    import re
    path = os.path.join(ROOT, "profiles", "valu_mfma_issue_rates.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"^lse2\s+\S+ ms\s+([0-9.]+) ns", open(path).read(), re.M)
    return float(m.group(1)) if m else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--replicas", type=int, default=0, help="0 = choose by a short sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path (independent "
              "replicas, or the imaginary-time slices of one replica, would shard over GPUs); use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    # the CPU baseline forks its worker processes, so it runs before anything touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    if cpu is not None:
        progress(f"cpu baseline: {cpu['value']:.2f} replica-steps/s on {cpu['cores']} cores")
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    base = WORKLOADS["large_gauss"]
    P, D = base.p, base.dim

    from paper_2404_02628_amd import autotune

    # plain FP64 path: one replica, with its own best launch choices.  Graph replay is not among
    # the candidates: once a process has replayed a captured graph, the runtime slows every later
    # kernel dispatch of the process, which would distort all measurements below.
    tune64 = autotune.tune(bench_systems(1), "fp64", steps=20, warmup=5)
    t64, _, _ = run_path("fp64", 1, args.steps, args.warmup, knobs=tune64.best)
    fp64_sps = args.steps / t64
    progress(f"fp64 single replica: {fp64_sps:.1f} steps/s")
    # its recursion per chain row: both directions run concurrently, each a chain of N rows
    _, _, times64 = run_path("fp64", 1, max(20, args.steps // 5), args.warmup, profile=True,
                             knobs=dataclasses.replace(tune64.best, graphs=False))
    rec_ms, rec_n = times64.get("recursion", (0.0, 0))
    rec_ns_per_row = rec_ms / max(rec_n, 1) * 1e6 / base.n
    progress(f"fp64 single replica recursion: {rec_ns_per_row:.1f} ns per chain row")

    # mixed batched: choose R by a short sweep unless given
    curve = {}
    if args.replicas > 0:
        R = args.replicas
    else:
        for r in (1, 4, 16, 64, 128, 256):
            n = max(20, args.steps // 10)
            t, _, _ = run_path("mixed", r, n, 5)
            curve[r] = r * n / t
            progress(f"mixed R={r}: {curve[r]:.1f} replica-steps/s")
        # the smallest batch within 2% of the best rate: short sweep runs differ by a few percent
        # from run to run, and a larger batch only costs memory once the device is full
        best = max(curve.values())
        R = min(r for r, v in curve.items() if v >= 0.98 * best)
    # launch choices for that batch; then the timed region without instrumentation (the value),
    # and the same run again with HIP events around every launch on the stream it runs on (the
    # per-kernel times of the roofline: the events cost the two-stream step a few percent of its
    # overlap, so they stay out of the run that gives the throughput)
    tunemix = autotune.tune(bench_systems(R), "mixed", steps=10, warmup=3)
    best = tunemix.best
    tmix, systems, _ = run_path("mixed", R, args.steps, args.warmup, knobs=best)
    _, _, times = run_path("mixed", R, args.steps, args.warmup, profile=True,
                           knobs=dataclasses.replace(best, graphs=False))
    sps = R * args.steps / tmix
    beads = sum(s.n * s.p for s in systems)
    progress(f"mixed R={R} timed: {sps:.1f} replica-steps/s")

    # FP64 at the same batch size: the precision gain apart from the batching gain
    tune64b = autotune.tune(bench_systems(R), "fp64", steps=5, warmup=2)
    steps64b = max(20, args.steps // 5)
    t64b, _, _ = run_path("fp64", R, steps64b, args.warmup, knobs=tune64b.best)
    fp64_batched_sps = R * steps64b / t64b
    progress(f"fp64 R={R}: {fp64_batched_sps:.1f} replica-steps/s")
    mixed_single_sps = curve.get(1)
    if mixed_single_sps is None:
        t1, _, _ = run_path("mixed", 1, max(20, args.steps // 10), 5)
        mixed_single_sps = max(20, args.steps // 10) / t1

    # roofline of the dominant kernel of the mixed batched step
    dom = max(times.items(), key=lambda kv: kv[1][0])
    kind, (ms_total, launches) = dom[0], dom[1]
    avg_s = ms_total / max(launches, 1) / 1e3
    bound, units, per_unit, unit, peak = algorithmic_work(kind, systems, P, D)
    achieved = units * per_unit / avg_s / (1e12 if unit == "TFLOP/s" else 1e9)
    kernels = {}
    for k, v in times.items():
        if v[1] == 0:
            continue
        b, u, pu, un, pk = algorithmic_work(k, systems, P, D)
        avg = v[0] / v[1] / 1e3
        ach = u * pu / avg / (1e12 if un == "TFLOP/s" else 1e9)
        kernels[k] = {"avg_us": avg * 1e6, "launches": v[1], "total_ms": v[0], "bound": b,
                      "achieved": ach, "unit": un, "frac": ach / pk}

    rel = energy_precision_error(R, best, tune64b.best)
    progress(f"mixed vs fp64 estimators over {R} replicas: {rel}")
    lse2 = lse2_latency_ns()
    rec = {
        "metric": "PIMD steps/s & bead-updates/s at N=1600,P=32: mixed vs FP64 at <=0.2% energy error",
        "value": sps,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tmix / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "large_gauss: N=1600 bosons, 2-D trap, P=32, beta=3, A=0.5, s=0.5, mixed precision",
                   "replicas": R, "global_batch": R, "beads": P, "particles": base.n,
                   "parallelism": "replica batching on 1 GPU"},
        "bead_updates_per_s": sps * beads / R,
        "fp64_single_steps_per_s": fp64_sps,
        "fp64_single_bead_updates_per_s": fp64_sps * base.n * base.p,
        "fp64_batched_steps_per_s": fp64_batched_sps,
        "mixed_single_steps_per_s": mixed_single_sps,
        "speedup_mixed_batched_vs_fp64": sps / fp64_sps,
        "gain_precision_at_R": sps / fp64_batched_sps,
        "gain_batching_fp64": fp64_batched_sps / fp64_sps,
        "gain_precision_single": mixed_single_sps / fp64_sps,
        "energy_rel_err_mixed_vs_fp64_same_config": rel,
        "recursion_fp64_single": {"ns_per_chain_row": rec_ns_per_row, "rows": base.n,
                                  "schedule_workgroups": tune64.best.recursion_workgroups,
                                  "lse2_latency_model_ns": lse2,
                                  "ratio_to_model": (rec_ns_per_row / lse2) if lse2 else None},
        "replica_curve_steps_per_s": curve,
        "autotune": {"mixed": {"best": best.as_kwargs(),
                               "s_per_step": {str(k.as_kwargs()): v for k, v in tunemix.seconds_per_step.items()}},
                     "fp64": {"best": tune64.best.as_kwargs(),
                              "s_per_step": {str(k.as_kwargs()): v for k, v in tune64.seconds_per_step.items()}}},
        "roofline": {"kernel": kind, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": traffic_bytes(kind, "mixed", R)},
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
