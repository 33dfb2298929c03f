"""What the thermostatted dynamics samples, on the GPU (shortened versions of tests/long_runs.py).

* N = 8 ideal bosons (d = 2, beta = 3, P = 12): <E_prim> and <E_vir> over many independent
  replicas match the exact finite-P canonical energy within 4 standard errors.
* N = 10^4 ideal bosons (d = 3, beta = 2, P = 16): <E_vir> of replicas started from thermal ring
  shapes matches the exact energy within 4 standard errors, and <E_prim> does after the predicted
  time-step shift of the velocity-Verlet ring modes (long_runs.primitive_dt2_shift).
* The N = 1600 benchmark system in mixed precision and in FP64, from independent seeds: the mean
  energies (and trap, pair energies) agree within 4 standard errors of the difference and within
  0.2%.
The full-length protocol and its summary are produced by tests/long_runs.py."""
import pytest

import long_runs

pytestmark = pytest.mark.gpu


def test_small_ideal_bosons_sample_the_exact_energy(orc):
    r = long_runs.check_ideal(orc, "ideal_small", replicas=512, equil=3000, steps=20000, every=50)
    print({k: r[k] for k in ("exact", "e_prim", "e_vir")}, flush=True)
    for k in ("e_prim", "e_vir"):
        assert abs(r[k]["z"]) <= 4.0, (k, r[k])


def test_large_ideal_bosons_sample_the_exact_energy(orc):
    # eight replicas: with four, the blocking error of E_vir (22-32 over realizations, ~15% scatter)
    # straddled the 0.2% bound below (29.9), so whether a run resolved the metric depended on the
    # realization rather than on the sampling
    r = long_runs.check_ideal(orc, "ideal_10k", replicas=8, equil=1500, steps=6000, every=20)
    print({k: r[k] for k in ("exact", "e_prim", "e_vir")}, flush=True)
    # E_prim carries the velocity-Verlet shift of the ring modes (-24 here, 1.6e-3 relative), which
    # the full-length run resolves; E_vir's shift is below 1e-4 relative
    assert abs(r["e_prim"]["z_after_dt2_shift"]) <= 4.0, r["e_prim"]
    assert abs(r["e_vir"]["z"]) <= 4.0, r["e_vir"]
    for k in ("e_prim", "e_vir"):
        # the run resolves the energy to the metric's 0.2% (a bias of 0.8% would be seen at 4
        # sigma); the blocking estimate of the error itself scatters by ~15% between trajectories
        assert r[k]["err"] <= 2e-3 * r["exact"], (k, r[k])


def test_mixed_precision_samples_the_fp64_energies():
    r = long_runs.check_mixed_vs_fp64(replicas=4, equil=2000, steps=4000, every=10)
    print({k: r[k] for k in long_runs.OBS}, flush=True)
    for k in long_runs.OBS:
        assert abs(r[k]["z"]) <= 4.0, (k, r[k])
    for k in ("e_prim", "e_vir"):
        assert abs(r[k]["rel"]) <= 2e-3, (k, r[k])
