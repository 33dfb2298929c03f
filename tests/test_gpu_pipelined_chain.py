"""The cooperative recursion schedule in its pipelined form (used from 64 row blocks on, N >=
4032: the previous block's in-block payloads and row averages are formed by the waves that
would otherwise wait while wave 0 runs the serial passes, with two alternating coefficient
buffers) against the oracle, and against the one-workgroup schedule.

Cases chosen to cross the parts of the chain that the pipelining touches: a pair term with
0 < xi < 1 in d = 2, and two species in d = 3 (the species boundary masks in-block terms), both
with N = 4100 (65 row blocks, a ragged last block).  Bars as for the large configurations:
potentials within 1e-10, forces within c_X = 1e-10 + sqrt(N) eps max|X| of their scale."""
import numpy as np
import pytest

from paper_2404_02628_amd.workloads import System, random_positions

pytestmark = pytest.mark.gpu

CASES = [  # n, n2, dim, xi, A
    (4100, 0, 2, 0.6, 1.0),
    (4100, 1500, 3, 1.0, 0.0),
]


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", CASES, ids=[f"N{c[0]}n2_{c[1]}d{c[2]}xi{c[3]}A{c[4]}" for c in CASES])
def test_pipelined_chain_matches_oracle(orc, case):
    from paper_2404_02628_amd.pimd import Context
    n, n2, dim, xi, A = case
    s = System(n=n, p=4, dim=dim, beta=2.0, xi=xi, pair_amp=A, pair_width=0.5, sigma=3.0, seed=71 + n2, n2=n2)
    x = random_positions(s.n, s.p, s.dim, s.sigma, s.seed)
    par = orc.OracleParams(n=s.n, p=s.p, dim=s.dim, beta=s.beta, xi=s.xi, pair_amp=s.pair_amp,
                           pair_width=s.pair_width, hbar=s.hbar, mass=s.mass, omega=s.omega, n2=s.n2)
    f_or, en_or, X_or, Y_or = orc.compute_forces(par, x, want_tables=True)[:4]
    c_x = 1e-10 + np.sqrt(n) * np.finfo(float).eps * float(np.max(np.abs(X_or)))
    kappa = s.mass * s.p / (s.beta * s.hbar) ** 2
    fscale = max(float(np.max(np.abs(f_or))), 4 * kappa * float(np.max(np.abs(x))))
    out = {}
    for sched in (0, 1):   # 0: cooperative chain + helpers (pipelined at this N); 1: one workgroup
        print(f"pipelined chain: N={n} n2={n2} d={dim} xi={xi} A={A} schedule {sched}", flush=True)
        ctx = Context([s], precision="fp64", recursion_workgroups=sched)
        try:
            ctx.set_state(0, x)
            ctx.compute_forces()
            f = ctx.forces(0)
            X, Y = ctx.potentials(0)
            en = ctx.energies(0)
        finally:
            ctx.close()
        assert float(np.max(np.abs(f - f_or))) <= c_x * fscale, (sched, float(np.max(np.abs(f - f_or))) / fscale)
        assert _rel(X, X_or) <= 1e-10, (sched, "X", _rel(X, X_or))
        assert _rel(Y[1:], Y_or[1:]) <= 1e-10, (sched, "Y", _rel(Y[1:], Y_or[1:]))
        assert abs(en["v_exch"] - en_or["v_exch"]) <= 1e-10 * abs(en_or["v_exch"])
        assert abs(en["spring_expect"] - en_or["spring_expect"]) <= c_x * abs(en_or["spring_expect"])
        out[sched] = f
    assert float(np.max(np.abs(out[0] - out[1]))) <= c_x * fscale
