"""Workload driver for rocprofv3 runs (kernel traces and hardware counters).

    python -m paper_2404_02628_amd.profile_run --path mixed --replicas 64 --steps 20

runs, in order: a plain device-to-device copy of --copy-mib MiB (torch, known traffic: that
many bytes read and written), used to scale the FETCH_SIZE / WRITE_SIZE counters to bytes;
then --steps MD steps of the N=1600, P=32 Gaussian workload on the chosen path (mixed or
fp64, R replicas, recursion schedule --workgroups), after --warmup untimed steps.  It prints
one line per phase so a profiled run can be matched to its dispatches.
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
    args = ap.parse_args(argv)

    import torch

    from .pimd import Context
    from .workloads import WORKLOADS, initial_state

    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy {args.copy_mib} MiB done", flush=True)
    del src, dst

    base = WORKLOADS[args.workload]
    systems = [base.with_(seed=base.seed + r) for r in range(args.replicas)]
    ctx = Context(systems, precision=args.path, recursion_workgroups=args.workgroups)
    for r, s in enumerate(systems):
        x, p = initial_state(s)
        ctx.set_state(r, x, p)
    ctx.step(args.warmup, 0)
    ctx.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps, 0)
    ctx.synchronize()
    dt = time.perf_counter() - t0
    print(f"{args.path} R={args.replicas} {args.steps} steps {dt * 1e3:.2f} ms "
          f"({args.replicas * args.steps / dt:.1f} replica-steps/s)", flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
