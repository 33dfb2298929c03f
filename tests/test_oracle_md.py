"""Pins of the oracle's integrator: second-order energy conservation (velocity Verlet and
the massive Nose-Hoover-chain extension), equipartition, and long-run estimator means
against the exact canonical energy of trapped non-interacting bosons."""
import math

import numpy as np
import pytest

from paper_2404_02628_amd.workloads import System, initial_state


def blocking_error(a):
    """Flyvbjerg-Petersen blocking: the plateau (max over levels) of the standard error."""
    a = np.asarray(a, dtype=float)
    best = a.std(ddof=1) / math.sqrt(len(a))
    while len(a) >= 32:
        a = 0.5 * (a[0:len(a) // 2 * 2:2] + a[1:len(a) // 2 * 2:2])
        best = max(best, a.std(ddof=1) / math.sqrt(len(a)))
    return best


def _setup(orc, sysm, nhc_len, dt):
    par = orc.OracleParams(n=sysm.n, p=sysm.p, dim=sysm.dim, beta=sysm.beta, xi=sysm.xi,
                           pair_amp=sysm.pair_amp, pair_width=sysm.pair_width)
    md = orc.OracleMD(dt=dt, nhc_len=nhc_len)
    x, p = initial_state(sysm)
    f, _ = orc.compute_forces(par, x)
    eta = np.zeros((max(nhc_len, 1),) + x.shape)
    veta = np.zeros_like(eta)
    return par, md, x, p, f, eta, veta


def _max_dev(orc, sysm, nhc_len, dt, t_total):
    par, md, x, p, f, eta, veta = _setup(orc, sysm, nhc_len, dt)
    h0 = orc.conserved(par, md, x, p, eta, veta)
    n = int(round(t_total / dt))
    dev = 0.0
    for _ in range(20):
        orc.step(par, md, x, p, eta, veta, f, n // 20)
        dev = max(dev, abs(orc.conserved(par, md, x, p, eta, veta) - h0))
    return dev, h0


@pytest.mark.parametrize("nhc_len", [0, 4])
def test_conserved_quantity_is_second_order(orc, nhc_len):
    """|H'(t) - H'(0)| shrinks ~4x when dt halves (second-order splitting)."""
    sysm = System(n=4, p=6, dim=2, beta=2.0, xi=0.8, pair_amp=1.0, pair_width=0.6, sigma=0.4, seed=31)
    d1, h0 = _max_dev(orc, sysm, nhc_len, 0.004, 2.0)
    d2, _ = _max_dev(orc, sysm, nhc_len, 0.002, 2.0)
    assert d1 < 1e-4 * abs(h0)
    assert 2.8 < d1 / d2 < 5.5, (d1, d2)


@pytest.mark.slow
@pytest.mark.parametrize("xi", [1.0, 0.5])
def test_long_run_energy_matches_exact(orc, xi):
    """Massive-NHC sampling of 3 ideal particles in a 2-D trap: <E_prim>, <E_vir> agree with
    the exact finite-P canonical energy, and <p^2/m'> = 1/beta per degree of freedom."""
    sysm = System(n=3, p=6, dim=2, beta=2.0, xi=xi, sigma=0.7, seed=41 + int(10 * xi))
    par, md, x, p, f, eta, veta = _setup(orc, sysm, 4, 0.05)
    orc.step(par, md, x, p, eta, veta, f, 4000)
    ep, ev, kin = [], [], []
    for _ in range(9000):
        orc.step(par, md, x, p, eta, veta, f, 20)
        _, en = orc.compute_forces(par, x)
        ep.append(en["e_prim"])
        ev.append(en["e_vir"])
        kin.append(float(np.mean(p * p)))
    exact = orc.exact_energy(3, 2, 2.0, 6, xi)
    for series in (ep, ev):
        m, err = float(np.mean(series)), blocking_error(series)
        assert abs(m - exact) < 4.5 * err + 1e-3 * exact, (m, err, exact)
        assert err < 0.015 * exact
    mk, ek = float(np.mean(kin)), blocking_error(kin)
    assert abs(mk - 1.0 / 2.0) < 4.5 * ek + 2e-3, (mk, ek)
