"""Long thermostatted runs on the GPU against exact energies and across precisions.

Three checks of what the dynamics samples (Sec. IV.A compares PIMD energies with exact ones):

* ``ideal_small``  N = 8 ideal bosons, d = 2, beta = 3, P = 12 (positions N(0, 0.5^2)), FP64, many
  independent replicas in the persistent kernel: <E_prim> and <E_vir> against the exact finite-P
  canonical energy of the oracle (8.0597243...).
* ``ideal_10k``    N = 10^4 ideal bosons, d = 3, beta = 2, P = 16, FP64, replicas started from
  thermal ring shapes: <E_vir> and <E_prim> against the exact finite-P energy (14971.58...).
* ``mixed_vs_fp64`` the benchmark system (N = 1600, P = 32, d = 2, beta = 3, A = 0.5, s = 0.5):
  replicas in mixed precision and in FP64 from independent seeds, equilibrated, then sampled;
  per observable (E_prim, E_vir, U_trap, U_pair, the normalised radial density) the two means,
  their errors and the relative difference (the mixed path is to stay within 0.2% in energy).

Per replica the time series gets a Flyvbjerg-Petersen blocking error; replicas are independent,
so their means combine with the larger of the propagated error and the replica spread.

``python tests/long_runs.py --check all --out <dir>/long_runs.md`` runs the full protocol
(10^5 steps for the benchmark system) and writes a summary; the GPU tests run shortened versions.
This is test infrastructure: it calls the CPU oracle for the exact energies.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2404_02628_amd.workloads import WORKLOADS, initial_state, thermal_rings  # noqa: E402
from paper_2404_02628_amd.xi_extrapolation import blocking_error, combine_replicas  # noqa: E402

OBS = ("e_prim", "e_vir", "u_trap", "u_pair")


def log(msg):
    print(msg, flush=True)


def sample_run(systems, precision, equil, steps, every, starts, bins=40, rmax=6.0, chunks=10, **ctx_kw):
    """Runs the replicas from the given (x, p) starts: `equil` steps, then `steps` more sampled every
    `every` steps (in `chunks` calls, each logged).  Returns {obs: [(mean, err) per replica]}, the
    density counts (bins + 1) and sample count per replica, and the wall time."""
    from paper_2404_02628_amd.pimd import Context
    cap = steps // every
    ctx = Context(systems, precision=precision, trace_capacity=cap, density_bins=bins, density_rmax=rmax, **ctx_kw)
    t0 = time.perf_counter()
    try:
        for r, (x, p) in enumerate(starts):
            ctx.set_state(r, x, p)
        ctx.step(equil, 0)
        ctx.synchronize()
        log(f"    {precision}: equilibrated ({equil} steps, {time.perf_counter() - t0:.1f} s)")
        ctx.reset_accumulators()
        per_chunk = (steps // every + chunks - 1) // chunks * every
        done = 0
        while done < steps:
            k = min(per_chunk, steps - done)
            ctx.step(k, every)
            ctx.synchronize()
            done += k
            log(f"    {precision}: {done}/{steps} sampled steps ({time.perf_counter() - t0:.1f} s)")
        per = {k: [] for k in OBS}
        dens = []
        for r in range(len(systems)):
            tr = ctx.trace(r, cap)
            assert len(tr) == cap, (len(tr), cap)
            for k in OBS:
                per[k].append(blocking_error([t[k] for t in tr]))
            counts, ns = ctx.density(r)
            dens.append((counts.astype(np.float64), ns))
    finally:
        ctx.close()
    return per, dens, time.perf_counter() - t0


def exact_energy(orc, s):
    return orc.exact_energy(s.n, s.dim, s.beta, s.p, s.xi)


def primitive_dt2_shift(s):
    """Time-step shift of <E_prim> for ideal trapped rings (d N copies of one P-bead ring).

    Velocity Verlet with a thermostat on the momenta samples a harmonic mode of frequency w with
    the shadow potential (1/2) m w^2 (1 - w^2 dt^2 / 4) q^2, so <(1/2) m w^2 q^2> is kT/2 divided by
    (1 - w^2 dt^2/4).  A ring of P beads of mass m' with springs m omega_P^2 in the trap has modes
    w_k^2 = (4 m omega_P^2 sin^2(pi k/P) + m omega^2/P) / m'; the spring share of each mode's
    potential enters S (the expected spring energy), so S rises and E_prim = d N P/(2 beta) - S +
    U/P falls by the spring part of the excess.  Exchange joins rings into longer rings whose mode
    sums per particle are the same to this order.  Returns the predicted <E_prim> - E_exact."""
    kT = 1.0 / s.beta
    mp = s.bead_mass if s.bead_mass > 0 else s.mass
    wp2 = s.p / (s.beta * s.hbar) ** 2
    shift = 0.0
    for k in range(s.p):
        spring = 4.0 * s.mass * wp2 * math.sin(math.pi * k / s.p) ** 2
        w2 = (spring + s.mass * s.omega ** 2 / s.p) / mp
        excess = 0.5 * kT * (1.0 / (1.0 - w2 * s.dt ** 2 / 4.0) - 1.0)      # per mode, potential energy
        trap_share = s.mass * s.omega ** 2 / s.p / (spring + s.mass * s.omega ** 2 / s.p)
        # the spring part lowers E_prim through S; the trap part raises U/P (U carries 1/P already)
        shift += -excess * (1.0 - trap_share) + excess * trap_share
    return shift * s.dim * s.n


def check_ideal(orc, which, replicas, equil, steps, every, sigma=None, seed0=None):
    """Ideal bosons against the exact finite-P energy; returns a result dict."""
    base = WORKLOADS["small_ideal" if which == "ideal_small" else "huge_ideal_10k"]
    seed0 = base.seed if seed0 is None else seed0
    systems = [base.with_(seed=seed0 + r) for r in range(replicas)]
    if which == "ideal_small":
        starts = [initial_state(s) for s in systems]
    else:
        # centroids with the classical variance 1/(beta m omega^2) of the trap, thermal ring shapes
        sig = math.sqrt(1.0 / (base.beta * base.mass * base.omega ** 2)) if sigma is None else sigma
        starts = []
        for s in systems:
            x = thermal_rings(s.n, s.p, s.dim, s.beta, sig, s.seed)
            p = initial_state(s)[1]
            starts.append((x, p))
    per, _, wall = sample_run(systems, "fp64", equil, steps, every, starts)
    exact = exact_energy(orc, base)
    out = {"check": which, "n": base.n, "p": base.p, "dim": base.dim, "beta": base.beta, "replicas": replicas,
           "equil_steps": equil, "sampled_steps": steps, "sample_every": every, "exact": exact, "wall_s": wall}
    for k in ("e_prim", "e_vir"):
        m, e = combine_replicas(per[k])
        out[k] = {"mean": m, "err": e, "z": (m - exact) / e, "rel": (m - exact) / exact}
    shift = primitive_dt2_shift(base)
    out["e_prim"]["dt2_shift_predicted"] = shift
    out["e_prim"]["z_after_dt2_shift"] = (out["e_prim"]["mean"] - exact - shift) / out["e_prim"]["err"]
    return out


def check_mixed_vs_fp64(replicas, equil, steps, every, bins=40, rmax=6.0):
    """The benchmark system in both precisions from independent seeds."""
    base = WORKLOADS["large_gauss"]
    res = {"check": "mixed_vs_fp64", "n": base.n, "p": base.p, "dim": base.dim, "beta": base.beta,
           "pair_amp": base.pair_amp, "pair_width": base.pair_width, "replicas_per_precision": replicas,
           "equil_steps": equil, "sampled_steps": steps, "sample_every": every}
    runs = {}
    for prec, seed0 in (("mixed", base.seed), ("fp64", base.seed + 1000)):
        systems = [base.with_(seed=seed0 + r) for r in range(replicas)]
        starts = [initial_state(s) for s in systems]
        per, dens, wall = sample_run(systems, prec, equil, steps, every, starts, bins=bins, rmax=rmax)
        runs[prec] = (per, dens)
        res[f"wall_s_{prec}"] = wall
        log(f"  {prec}: {replicas} replicas x {equil + steps} steps in {wall:.1f} s")
    for k in OBS:
        ma, ea = combine_replicas(runs["mixed"][0][k])
        mb, eb = combine_replicas(runs["fp64"][0][k])
        err = math.hypot(ea, eb)
        res[k] = {"mixed": ma, "mixed_err": ea, "fp64": mb, "fp64_err": eb, "diff": ma - mb, "err": err,
                  "z": (ma - mb) / err, "rel": (ma - mb) / abs(mb)}
    # normalised radial density per replica: counts / (samples N P shell area), 2-D shells
    edges = np.linspace(0.0, rmax, bins + 1)
    shell = math.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    rho = {}
    for prec in ("mixed", "fp64"):
        per_rep = np.array([c[:bins] / (ns * base.n * base.p * shell) for c, ns in runs[prec][1]])
        rho[prec] = (per_rep.mean(axis=0), per_rep.std(axis=0, ddof=1) / math.sqrt(per_rep.shape[0]))
    dm, em = rho["mixed"]
    df, ef = rho["fp64"]
    err = np.sqrt(em ** 2 + ef ** 2)
    ok = err > 0
    zb = np.zeros_like(dm)
    zb[ok] = (dm[ok] - df[ok]) / err[ok]
    res["density"] = {"bins": bins, "rmax": rmax, "max_abs_z": float(np.max(np.abs(zb))),
                      "chi2_per_bin": float(np.mean(zb[ok] ** 2)), "bins_compared": int(ok.sum()),
                      "rho_mixed": dm.tolist(), "rho_fp64": df.tolist(), "rho_err": err.tolist()}
    return res


def summary_md(results, cmd):
    lines = ["# Long runs: exact energies and mixed precision against FP64 — one MI355X", "",
             "```", cmd, "```", ""]
    for r in results:
        if r["check"] in ("ideal_small", "ideal_10k"):
            lines.append(f"## {r['check']}: N={r['n']}, P={r['p']}, d={r['dim']}, beta={r['beta']}, ideal bosons, FP64")
            lines.append("")
            lines.append(f"{r['replicas']} independent replicas, {r['equil_steps']} equilibration steps, "
                         f"{r['sampled_steps']} sampled steps (every {r['sample_every']}), {r['wall_s']:.1f} s.  "
                         f"Exact finite-P energy (oracle): {r['exact']:.6f}.")
            lines.append("")
            lines.append("| estimator | mean | error | (mean - exact)/error | relative |")
            lines.append("|---|---:|---:|---:|---:|")
            for k in ("e_prim", "e_vir"):
                v = r[k]
                lines.append(f"| {k} | {v['mean']:.5f} | {v['err']:.5f} | {v['z']:+.2f} | {v['rel']:+.2e} |")
            lines.append("")
            v = r["e_prim"]
            lines.append(f"Velocity Verlet at dt = {WORKLOADS['small_ideal' if r['check'] == 'ideal_small' else 'huge_ideal_10k'].dt} "
                         f"samples each ring mode of frequency w with <q^2> larger by 1/(1 - w^2 dt^2/4), which "
                         f"moves <E_prim> by {v['dt2_shift_predicted']:+.4f} (primitive_dt2_shift; <E_vir> moves by "
                         f"less than 1e-4 relative); (mean - exact - shift)/error = {v['z_after_dt2_shift']:+.2f}.")
            lines.append("")
        else:
            lines.append(f"## mixed vs FP64: N={r['n']}, P={r['p']}, d={r['dim']}, beta={r['beta']}, "
                         f"A={r['pair_amp']}, s={r['pair_width']}")
            lines.append("")
            lines.append(f"{r['replicas_per_precision']} replicas per precision from independent seeds (mixed "
                         f"303+r, FP64 1303+r), {r['equil_steps']} equilibration steps, {r['sampled_steps']} "
                         f"sampled steps (every {r['sample_every']}); wall {r['wall_s_mixed']:.0f} s mixed, "
                         f"{r['wall_s_fp64']:.0f} s FP64.")
            lines.append("")
            lines.append("| observable | mixed | FP64 | difference | error of difference | z | relative |")
            lines.append("|---|---:|---:|---:|---:|---:|---:|")
            for k in OBS:
                v = r[k]
                lines.append(f"| {k} | {v['mixed']:.4f} ± {v['mixed_err']:.4f} | {v['fp64']:.4f} ± {v['fp64_err']:.4f} "
                             f"| {v['diff']:+.4f} | {v['err']:.4f} | {v['z']:+.2f} | {v['rel']:+.2e} |")
            dd = r["density"]
            lines.append("")
            lines.append(f"Normalised radial density ({dd['bins']} bins to r = {dd['rmax']}): largest |z| over "
                         f"{dd['bins_compared']} bins {dd['max_abs_z']:.2f}, mean z^2 {dd['chi2_per_bin']:.2f}.")
            lines.append("")
    lines.append("```json long-runs")
    slim = [{k: v for k, v in r.items() if k != "density"} | ({"density": {k: v for k, v in r["density"].items()
                                                                             if not k.startswith("rho")}}
                                                            if "density" in r else {}) for r in results]
    lines.append(json.dumps(slim, indent=1))
    lines.append("```")
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--check", choices=["ideal_small", "ideal_10k", "mixed_vs_fp64", "all"], default="all")
    ap.add_argument("--out", default="")
    ap.add_argument("--mixed-replicas", type=int, default=16)
    ap.add_argument("--mixed-steps", type=int, default=80000)
    ap.add_argument("--mixed-equil", type=int, default=20000)
    ap.add_argument("--from-summary", default="",
                    help="re-render a summary written by this script from its json block (adds the derived "
                         "time-step predictions; no GPU)")
    args = ap.parse_args(argv)
    if args.from_summary:
        import re
        text = open(args.from_summary).read()
        results = json.loads(re.search(r"```json long-runs\n(.*?)\n```", text, re.S).group(1))
        first_cmd = re.search(r"```\n(.*?)\n```", text, re.S).group(1).splitlines()[0]
        for r in results:
            if r["check"] in ("ideal_small", "ideal_10k"):
                base = WORKLOADS["small_ideal" if r["check"] == "ideal_small" else "huge_ideal_10k"]
                shift = primitive_dt2_shift(base)
                r["e_prim"]["dt2_shift_predicted"] = shift
                r["e_prim"]["z_after_dt2_shift"] = (r["e_prim"]["mean"] - r["exact"] - shift) / r["e_prim"]["err"]
        md = summary_md(results, first_cmd + "\n(rendered again by: python tests/long_runs.py --from-summary <that file>)")
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(md)
        print(md)
        return
    import oracle
    if not os.path.exists(oracle.lib_path()):
        oracle.build()
    results = []
    if args.check in ("ideal_small", "all"):
        log("ideal_small ...")
        results.append(check_ideal(oracle, "ideal_small", replicas=1024, equil=5000, steps=50000, every=50))
        log(json.dumps({k: results[-1][k] for k in ("e_prim", "e_vir")}))
    if args.check in ("ideal_10k", "all"):
        log("ideal_10k ...")
        results.append(check_ideal(oracle, "ideal_10k", replicas=4, equil=4000, steps=40000, every=20))
        log(json.dumps({k: results[-1][k] for k in ("e_prim", "e_vir")}))
    if args.check in ("mixed_vs_fp64", "all"):
        log("mixed_vs_fp64 ...")
        results.append(check_mixed_vs_fp64(args.mixed_replicas, args.mixed_equil, args.mixed_steps, every=10))
        log(json.dumps({k: results[-1][k] for k in OBS}))
    cmd = "python tests/long_runs.py " + " ".join(argv if argv is not None else sys.argv[1:])
    md = summary_md(results, cmd)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(md)
    print(md)


if __name__ == "__main__":
    main()
