"""Workload driver for rocprofv3 runs (kernel traces and hardware counters).

    python -m paper_2404_02628_amd.profile_run --path mixed --replicas 64 --steps 20

runs, in order: a plain device-to-device copy of --copy-mib MiB (torch, known traffic: that
many bytes read and written), used to scale the FETCH_SIZE / WRITE_SIZE counters to bytes;
then --steps MD steps of a workload on the chosen path (mixed or fp64, recursion schedule
--workgroups), after --warmup untimed steps: --replicas copies (seeds base+r) of a named
workload (default the N=1600, P=32 Gaussian system), or with --workload batched the 64
uneven replicas (N ~ U{64..512}, xi = 0.2 (1 + r mod 5)).  It prints one line per phase so a
profiled run can be matched to its dispatches, and the workspace size.
"""
from __future__ import annotations

import argparse
import sys
import time


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--path", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--workload", default="large_gauss")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--graphs", action="store_true", help="replay steady steps from a HIP graph")
    ap.add_argument("--n2", type=int, default=0, help="particles of a second species in every replica")
    ap.add_argument("--no-persistent", action="store_true",
                    help="one launch per kernel and step even for replicas small enough for the persistent kernel")
    ap.add_argument("--tune", action="store_true",
                    help="choose the launch knobs with the autotuner first (printed) and run with them")
    ap.add_argument("--kernel-times", action="store_true",
                    help="also time the steps with the library's HIP-event profiler and print per-kernel averages")
    args = ap.parse_args(argv)

    import torch

    from .pimd import Context
    from .workloads import WORKLOADS, batched_systems, initial_state

    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy {args.copy_mib} MiB done", flush=True)
    del src, dst

    if args.workload == "batched":
        systems = batched_systems(64, 505)
    else:
        base = WORKLOADS[args.workload]
        systems = [base.with_(seed=base.seed + r, n2=args.n2) for r in range(args.replicas)]
    if args.tune:
        from . import autotune
        res = autotune.tune(systems, args.path, steps=10, warmup=3)
        print("autotuned: " + ", ".join(f"{k}={v}" for k, v in res.best.as_kwargs().items()), flush=True)
        for k, v in sorted(res.seconds_per_step.items(), key=lambda kv: kv[1])[:6]:
            print(f"  {v * 1e6:8.1f} us/step  {k.as_kwargs()}", flush=True)
        ctx = Context(systems, precision=args.path, **res.best.as_kwargs())
    else:
        ctx = Context(systems, precision=args.path, recursion_workgroups=args.workgroups, graphs=args.graphs,
                      persistent=not args.no_persistent)
    for r, sy in enumerate(systems):
        x, p = initial_state(sy)
        ctx.set_state(r, x, p)
    print(f"workspace {ctx.nbytes / 2**20:.1f} MiB for {len(systems)} replicas", flush=True)
    ctx.step(args.warmup, 0)
    ctx.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps, 0)
    ctx.synchronize()
    dt = time.perf_counter() - t0
    beads = sum(sy.n * sy.p for sy in systems)
    print(f"{args.workload} {args.path}{' graphs' if args.graphs else ''} R={len(systems)} {args.steps} steps {dt * 1e3:.2f} ms "
          f"({len(systems) * args.steps / dt:.1f} replica-steps/s, {beads * args.steps / dt:.3e} bead-updates/s)",
          flush=True)
    if args.kernel_times:
        ctx.profile(True)
        ctx.step(args.steps, 0)
        kt = ctx.kernel_times()
        ctx.profile(False)
        print("  " + ", ".join(f"{k} {v[0] / v[1] * 1e3:.1f} us" for k, v in kt.items() if v[1] > 0), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
