"""Two species (spin mixtures) on the GPU against the two-species oracle.

The last n2 particles form a second species: exchange cycles stay within a species, each
species counts its own 1/n factors, and the trap and pair terms act on all particles.  The
boundary na = N - n2 is placed on and around the 64-row blocks of the recursions (na = 1, 63,
64, 80, 265, 299 and n2 = 1), so that both directions see the boundary inside a block, on a
block edge, and with whole blocks of the second species after it, under all three recursion
schedules (one workgroup per chain, automatic, chain plus four helpers).  Bars: those of the
single-species parity tests (FP64 within 1e-10 and c_X, mixed pair terms within 1e-5).
Replicas of different n2 (including 0) share one batched context; a short thermostatted
trajectory follows the oracle's integrator; and an ideal two-species ensemble samples the exact
finite-P energy, which is the sum of the two species' canonical energies."""
import numpy as np
import pytest

from paper_2404_02628_amd.workloads import System, initial_state, random_positions
from test_gpu_parity import _check_against_oracle, oracle_params, rel_max

pytestmark = pytest.mark.gpu

CASES = [
    # n, n2, p, d, beta, xi, A, s, sigma, seed
    (2, 1, 4, 2, 2.0, 1.0, 1.0, 0.6, 0.8, 21),
    (10, 4, 6, 2, 3.0, 1.0, 0.0, 0.5, 0.6, 22),
    (128, 64, 5, 2, 2.0, 0.8, 1.0, 0.5, 1.0, 23),
    (150, 70, 8, 3, 2.0, 1.0, 0.5, 0.6, 1.2, 24),
    (200, 137, 6, 1, 2.5, 0.5, 1.0, 0.5, 1.0, 25),
    (300, 1, 4, 2, 3.0, 1.0, 0.0, 0.5, 1.0, 26),
    (300, 299, 4, 2, 3.0, 0.3, 1.0, 0.5, 1.0, 27),
    (400, 135, 4, 2, 3.0, 1.0, 1.0, 0.5, 1.5, 28),
    (700, 300, 4, 2, 2.0, 0.0, 0.5, 0.5, 2.0, 29),
]
SCHEDULES = [1, 0, 5]


@pytest.mark.parametrize("sched", SCHEDULES, ids=[f"wg{k}" for k in SCHEDULES])
@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=[f"N{c[0]}n2_{c[1]}d{c[3]}xi{c[5]}" for c in CASES])
def test_two_species_match_oracle(orc, case, mixed, sched):
    from paper_2404_02628_amd.pimd import Context
    n, n2, p, d, beta, xi, A, s_, sigma, seed = case
    s = System(n=n, n2=n2, p=p, dim=d, beta=beta, xi=xi, pair_amp=A, pair_width=s_, sigma=sigma, seed=seed)
    x = random_positions(n, p, d, sigma, seed)
    print(f"two species N={n} n2={n2} {'mixed' if mixed else 'fp64'} schedule {sched}", flush=True)
    ctx = Context([s], precision="mixed" if mixed else "fp64", recursion_workgroups=sched)
    try:
        ctx.set_state(0, x)
        ctx.compute_forces()
        _check_against_oracle(orc, ctx, 0, s, x, mixed)
        G = ctx.probabilities(0)
        na = n - n2
        assert np.all(G[:na, na:] == 0.0) and np.all(G[na:, :na] == 0.0)
    finally:
        ctx.close()


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_batched_species_mix(orc, mixed):
    """Replicas with n2 = 0 and n2 > 0 in one context; in FP64 with one workgroup per chain a
    replica equals the same replica run alone bit for bit."""
    from paper_2404_02628_amd.pimd import Context
    specs = [(5, 2, 0.5), (64, 0, 1.0), (65, 1, 1.0), (130, 65, 0.7), (200, 0, 1.0), (257, 128, 1.0)]
    systems = [System(n=n, n2=n2, p=8, dim=2, beta=3.0, xi=xi, pair_amp=1.0, pair_width=0.5, sigma=1.0,
                      seed=60 + k) for k, (n, n2, xi) in enumerate(specs)]
    xs = [random_positions(s.n, s.p, s.dim, s.sigma, s.seed) for s in systems]
    print(f"batched species mix, {'mixed' if mixed else 'fp64'}", flush=True)
    ctx = Context(systems, precision="mixed" if mixed else "fp64", recursion_workgroups=1)
    try:
        for r, x in enumerate(xs):
            ctx.set_state(r, x)
        ctx.compute_forces()
        for r, (s, x) in enumerate(zip(systems, xs)):
            _check_against_oracle(orc, ctx, r, s, x, mixed)
        if not mixed:
            for r in (3, 5):
                solo = Context([systems[r]], precision="fp64", recursion_workgroups=1)
                try:
                    solo.set_state(0, xs[r])
                    solo.compute_forces()
                    assert np.array_equal(solo.forces(0), ctx.forces(r))
                finally:
                    solo.close()
    finally:
        ctx.close()


def test_two_species_trajectory_matches_oracle(orc):
    from paper_2404_02628_amd.pimd import Context
    s = System(n=9, n2=4, p=12, dim=2, beta=3.0, xi=0.6, pair_amp=1.0, pair_width=0.5, sigma=0.5, seed=78)
    x, p = initial_state(s)
    print("two species trajectory, 40 steps", flush=True)
    ctx = Context([s], precision="fp64", nhc_len=4)
    try:
        ctx.set_state(0, x, p)
        ctx.step(40, 0)
        xg, pg, _ = ctx.get_state(0)
    finally:
        ctx.close()
    par = oracle_params(orc, s)
    md = orc.OracleMD(dt=s.dt, nhc_len=4)
    xo, po = x.copy(), p.copy()
    f, _ = orc.compute_forces(par, xo)
    eta = np.zeros((4,) + x.shape)
    veta = np.zeros_like(eta)
    orc.step(par, md, xo, po, eta, veta, f, 40)
    assert rel_max(xg, xo) <= 1e-9
    assert rel_max(pg, po) <= 1e-9


def test_ideal_mixture_samples_exact_energy(orc):
    """Ideal trapped bosons, 3 + 2 particles in d = 2 at beta = 1, P = 12: the sampled virial
    energy matches E_3 + E_2 (exact finite-P canonical energies of each species) within 4
    standard errors plus 0.2%."""
    from paper_2404_02628_amd.xi_extrapolation import run_ensemble
    base = System(n=5, n2=2, p=12, dim=2, beta=1.0, xi=1.0, pair_amp=0.0, sigma=1.0, seed=0)
    print("ideal mixture: 64 replicas, 20000 warm-up steps, 40000 sampled", flush=True)
    res = run_ensemble(base, [1.0], replicas_per_xi=64, steps=40000, sample_every=10, warmup=20000, seed0=9100)
    exact = orc.exact_energy(3, 2, 1.0, 12, 1.0) + orc.exact_energy(2, 2, 1.0, 12, 1.0)
    m, e = res.means[0], res.errors[0]
    print(f"mixture: {m:.4f} +- {e:.4f}, exact {exact:.4f} (one species of 5: "
          f"{orc.exact_energy(5, 2, 1.0, 12, 1.0):.4f})", flush=True)
    assert abs(m - exact) <= 4.0 * e + 2e-3 * exact
