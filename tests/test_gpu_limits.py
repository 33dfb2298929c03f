"""The size limits the API accepts, against the oracle.

* P = 4096 (the largest bead count) with N = 3 and N = 70 in d = 1 and 3: the spring kernel's
  bead chunks, the widest slice loops of the pair kernels and the largest per-replica shadow.
* One particle (no exchange partner: V_xi = E_int, Pr[1->1] = 1) and two particles, in many
  replicas at once, in both precisions and through the persistent and multi-kernel paths.
* xi = 0 (distinguishable particles: only the identity permutation, 0^0 = 1) at N = 200 across
  several recursion blocks, where only the j = i-1 term of every row survives.
Bars: those of the parity tests (FP64 1e-10 and c_X; mixed 1e-5 for pair terms)."""
import numpy as np
import pytest

from paper_2404_02628_amd.workloads import System, initial_state, random_positions
from test_gpu_parity import _check_against_oracle, oracle_params, rel_max

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,d,A", [(3, 1, 1.0), (70, 3, 0.5)])
@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_largest_bead_count(orc, n, d, A, mixed):
    from paper_2404_02628_amd.pimd import Context
    s = System(n=n, p=4096, dim=d, beta=4.0, xi=0.8, pair_amp=A, pair_width=0.5, sigma=0.7, seed=41 + n)
    x = random_positions(n, 4096, d, 0.7, 41 + n)
    print(f"P=4096 N={n} d={d} {'mixed' if mixed else 'fp64'}", flush=True)
    ctx = Context([s], precision="mixed" if mixed else "fp64")
    try:
        ctx.set_state(0, x)
        ctx.compute_forces()
        _check_against_oracle(orc, ctx, 0, s, x, mixed)
    finally:
        ctx.close()


@pytest.mark.parametrize("persistent", [True, False], ids=["persistent", "multikernel"])
@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_one_and_two_particles_in_many_replicas(orc, mixed, persistent):
    from paper_2404_02628_amd.pimd import Context
    systems = [System(n=1 + (r % 2), p=8, dim=2, beta=2.0, xi=0.5 + 0.01 * r, pair_amp=1.0, pair_width=0.5,
                      sigma=0.8, seed=300 + r) for r in range(50)]
    states = [initial_state(s) for s in systems]
    print(f"50 replicas of N=1,2 ({'mixed' if mixed else 'fp64'}, persistent={persistent})", flush=True)
    ctx = Context(systems, precision="mixed" if mixed else "fp64", persistent=persistent, nhc_len=4)
    try:
        for r, (x, p) in enumerate(states):
            ctx.set_state(r, x, p)
        ctx.compute_forces()
        for r in (0, 1, 48, 49):
            _check_against_oracle(orc, ctx, r, systems[r], states[r][0], mixed)
        # one particle: the exchange potential is its own ring energy
        en = ctx.energies(0)
        s0, x0 = systems[0], states[0][0]
        e_ring = orc.ring_energy(oracle_params(orc, s0), x0, 1, 1)
        assert abs(en["v_exch"] - e_ring) <= 1e-12 * abs(e_ring)
        ctx.step(20, 0)
        for r in (0, 49):
            s, (x, p) = systems[r], states[r]
            md = orc.OracleMD(dt=s.dt, nhc_len=4)
            xo, po = x.copy(), p.copy()
            fo, _ = orc.compute_forces(oracle_params(orc, s), xo)
            eta = np.zeros((4,) + x.shape)
            veta = np.zeros_like(eta)
            orc.step(oracle_params(orc, s), md, xo, po, eta, veta, fo, 20)
            xg = ctx.get_state(r)[0]
            assert rel_max(xg, xo) <= (1e-6 if mixed else 1e-9), (r, rel_max(xg, xo))
    finally:
        ctx.close()


@pytest.mark.parametrize("sched", [1, 0], ids=["wg1", "auto"])
def test_distinguishable_particles_across_blocks(orc, sched):
    from paper_2404_02628_amd.pimd import Context
    s = System(n=200, p=8, dim=2, beta=2.0, xi=0.0, pair_amp=1.0, pair_width=0.5, sigma=1.5, seed=77)
    x = random_positions(200, 8, 2, 1.5, 77)
    ctx = Context([s], precision="fp64", recursion_workgroups=sched)
    try:
        ctx.set_state(0, x)
        ctx.compute_forces()
        _check_against_oracle(orc, ctx, 0, s, x, False)
        G = ctx.probabilities(0)
        # xi = 0: every particle closes its own ring, Pr[l -> l] = 1
        assert np.allclose(np.diag(G), 1.0, atol=1e-12) and abs(G.sum() - 200) <= 1e-9
    finally:
        ctx.close()
