"""The persistent small-replica kernel (whole MD steps of every replica in one launch, one
workgroup per replica) against the oracle and against the multi-kernel path.

* Trajectories: 40 thermostatted steps from the same state stay within 1e-9 of the oracle's
  integrator (the bar of the multi-kernel trajectory test) for N = 1 to 64, P = 2 to 16,
  d = 1, 2, 3, xi = 0, 0.5, 1, with and without pair term and with two species; the forces,
  potentials and probabilities left behind equal the oracle's at the final state within the
  parity bars (1e-10 relative; c_X for probabilities).
* Against the multi-kernel path (FP64, which also evaluates the pair term in FP64): a batch of
  uneven replicas sampled every 10 steps for 60 steps gives the same states within 1e-10 and the
  same trace records (energies within 1e-9 relative, equal step numbers); density counts agree
  except for beads within rounding of a bin edge.
* A call longer than one launch chunk (4096 steps) equals the same steps split over two calls
  bit for bit, and its trace holds consecutive sample steps."""
import numpy as np
import pytest

from paper_2404_02628_amd.workloads import System, initial_state
from test_gpu_parity import oracle_params, rel_max

pytestmark = pytest.mark.gpu

CASES = [  # n, n2, p, d, xi, A, s, sigma, seed
    (1, 0, 2, 1, 1.0, 0.0, 0.5, 0.7, 11),
    (2, 0, 4, 2, 1.0, 1.0, 0.6, 0.8, 12),
    (3, 0, 12, 2, 0.5, 0.0, 0.5, 0.5, 13),
    (8, 0, 12, 2, 1.0, 0.0, 0.5, 0.5, 101),
    (8, 3, 8, 3, 0.6, 1.0, 0.5, 0.5, 14),
    (33, 0, 4, 2, 0.0, 2.0, 0.5, 1.0, 15),
    (40, 15, 4, 3, 1.0, 1.0, 0.5, 1.0, 16),
    (64, 0, 8, 1, 1.0, 1.0, 0.5, 1.0, 17),
]


def _run_trajectory(s, x, p, steps, **kw):
    from paper_2404_02628_amd.pimd import Context
    ctx = Context([s], precision="fp64", nhc_len=4, **kw)
    try:
        ctx.set_state(0, x, p)
        ctx.step(steps, 0)
        xg, pg, _ = ctx.get_state(0)
        f = ctx.forces(0)
        X, Y = ctx.potentials(0)
        G = ctx.probabilities(0)
    finally:
        ctx.close()
    return xg, pg, f, X, Y, G


@pytest.mark.parametrize("case", CASES, ids=[f"N{c[0]}n2_{c[1]}P{c[2]}d{c[3]}xi{c[4]}A{c[5]}" for c in CASES])
def test_persistent_trajectory_matches_oracle(orc, case):
    n, n2, p, d, xi, A, s_, sigma, seed = case
    s = System(n=n, n2=n2, p=p, dim=d, beta=3.0, xi=xi, pair_amp=A, pair_width=s_, sigma=sigma, seed=seed)
    x, pm = initial_state(s)
    print(f"persistent trajectory N={n} n2={n2} P={p} d={d}", flush=True)
    xg, pg, f, X, Y, G = _run_trajectory(s, x, pm, 40)
    par = oracle_params(orc, s)
    md = orc.OracleMD(dt=s.dt, nhc_len=4)
    xo, po = x.copy(), pm.copy()
    fo, _ = orc.compute_forces(par, xo)
    eta = np.zeros((4,) + x.shape)
    veta = np.zeros_like(eta)
    orc.step(par, md, xo, po, eta, veta, fo, 40)
    assert rel_max(xg, xo) <= 1e-9, rel_max(xg, xo)
    assert rel_max(pg, po) <= 1e-9, rel_max(pg, po)
    # what the call leaves behind is the evaluation at its final state
    f_or, _, X_or, Y_or, G_or = orc.compute_forces(par, xg, want_tables=True)
    kappa = s.mass * s.p / (s.beta * s.hbar) ** 2
    scale = max(float(np.max(np.abs(f_or))), 4.0 * kappa * float(np.max(np.abs(xg))))
    c_x = 1e-10 + 32 * np.finfo(float).eps * float(np.max(np.abs(X_or)))
    assert float(np.max(np.abs(f - f_or))) / scale <= c_x
    assert rel_max(X, X_or) <= 1e-10 and rel_max(Y[1:], Y_or[1:]) <= 1e-10
    assert float(np.max(np.abs(G - G_or))) <= c_x


def _batch():
    specs = [(1, 0, 1.0, 0.0), (3, 0, 0.2, 1.0), (8, 2, 0.6, 1.0), (13, 0, 1.0, 2.0), (32, 16, 0.8, 0.5)]
    return [System(n=n, n2=n2, p=8, dim=2, beta=2.0, xi=xi, pair_amp=A, pair_width=0.5, sigma=0.8, seed=70 + k)
            for k, (n, n2, xi, A) in enumerate(specs)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_persistent_matches_multikernel_path(prec):
    from paper_2404_02628_amd.pimd import Context
    systems = _batch()
    states = [initial_state(s) for s in systems]
    out = {}
    for mode, kw in (("persistent", dict(precision=prec)), ("multi", dict(precision="fp64", persistent=False))):
        print(f"{mode} path ({kw['precision']}), 60 steps sampled every 10", flush=True)
        ctx = Context(systems, nhc_len=4, trace_capacity=8, density_bins=32, density_rmax=4.0, **kw)
        try:
            for r, (x, p) in enumerate(states):
                ctx.set_state(r, x, p)
            ctx.profile(True)
            ctx.step(60, 10)
            out[mode] = dict(state=[ctx.get_state(r) for r in range(len(systems))],
                             trace=[ctx.trace(r, 8) for r in range(len(systems))],
                             dens=[ctx.density(r) for r in range(len(systems))],
                             kt=ctx.kernel_times())
        finally:
            ctx.close()
    assert out["persistent"]["kt"]["persistent_steps"][1] >= 1
    assert out["multi"]["kt"]["persistent_steps"][1] == 0
    for r in range(len(systems)):
        (x1, p1, n1), (x2, p2, n2) = out["persistent"]["state"][r], out["multi"]["state"][r]
        assert rel_max(x1, x2) <= 1e-10 and rel_max(p1, p2) <= 1e-10 and rel_max(n1, n2) <= 1e-10, r
        t1, t2 = out["persistent"]["trace"][r], out["multi"]["trace"][r]
        assert [t["step"] for t in t1] == [t["step"] for t in t2] == [10, 20, 30, 40, 50, 60]
        for a, b in zip(t1, t2):
            for k in ("v_exch", "u_trap", "u_pair", "spring_expect", "virial", "e_prim", "e_vir", "kinetic",
                      "nhc_energy", "h_conserved"):
                assert abs(a[k] - b[k]) <= 1e-9 * max(abs(b[k]), 1.0), (r, k, a[k], b[k])
        (c1, s1), (c2, s2) = out["persistent"]["dens"][r], out["multi"]["dens"][r]
        assert s1 == s2 == 6 and c1.sum() == c2.sum()
        assert np.abs(c1.astype(np.int64) - c2.astype(np.int64)).sum() <= 2, r


def test_persistent_chunks_repeat_bitwise():
    from paper_2404_02628_amd.pimd import Context
    s = System(n=4, p=6, dim=2, beta=2.0, xi=0.8, pair_amp=1.0, pair_width=0.5, sigma=0.6, seed=5)
    x, p = initial_state(s)
    res = []
    for split in ((5000,), (2500, 2500)):
        ctx = Context([s], precision="fp64", trace_capacity=64)
        try:
            ctx.set_state(0, x, p)
            for k in split:
                ctx.step(k, 100)
            res.append((ctx.get_state(0), ctx.trace(0, 64)))
        finally:
            ctx.close()
    (a, ta), (b, tb) = res
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert [t["step"] for t in ta] == [t["step"] for t in tb] == list(range(100, 5001, 100))
    assert all(np.isfinite(t["h_conserved"]) for t in ta)
