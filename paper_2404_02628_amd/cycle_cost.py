"""Cost of the original O(N^3 P) cycle-energy table against the exchange path that replaces it.

    python -m paper_2404_02628_amd.cycle_cost [--n 100 400 1600 3200 6400] [--p 32] [--dim 2]

For each N (one FP64 replica, thermal rings, beta = 3, no pair term) it prints the device time of
the direct table (every E^{[u,v]} from its definition, Eq. 7) and, from HIP events of the
library's own profiler, the time per force evaluation of the recursions (both directions of
Eqs. 6 and 11 with the probability sums) and of the whole evaluation.  The direct table is only
the first of the original algorithm's steps: its recursions and probabilities would come on top.
"""
from __future__ import annotations

import argparse


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[100, 400, 1600, 3200, 6400])
    ap.add_argument("--p", type=int, default=32)
    ap.add_argument("--dim", type=int, default=2)
    ap.add_argument("--evals", type=int, default=10)
    args = ap.parse_args(argv)

    from .pimd import Context
    from .workloads import System, thermal_rings

    print(f"{'N':>6} {'direct table ms':>16} {'recursion ms':>13} {'evaluation ms':>14} {'table/recursion':>16}",
          flush=True)
    for n in args.n:
        s = System(n=n, p=args.p, dim=args.dim, beta=3.0, sigma=2.0, seed=303)
        ctx = Context([s], precision="fp64")
        try:
            ctx.set_state(0, thermal_rings(n, args.p, args.dim, s.beta, s.sigma, s.seed))
            ctx.cycle_energies(0)
            _, ms_table = ctx.cycle_energies(0)
            ctx.compute_forces()
            ctx.synchronize()
            ctx.profile(True)
            for _ in range(args.evals):
                ctx.compute_forces()
            kt = ctx.kernel_times()
            ctx.profile(False)
        finally:
            ctx.close()
        rec = kt["recursion"][0] / max(kt["recursion"][1], 1)
        ev = sum(v[0] for v in kt.values()) / args.evals
        print(f"{n:>6} {ms_table:>16.3f} {rec:>13.3f} {ev:>14.3f} {ms_table / rec:>16.1f}", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
