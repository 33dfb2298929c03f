"""Host logic of the xi-extrapolation: blocking error bars and the weighted polynomial fit."""
import numpy as np
import pytest

from paper_2404_02628_amd.xi_extrapolation import blocking_error, combine_replicas, fit_extrapolate


def test_blocking_recovers_the_error_of_a_correlated_mean():
    # AR(1): x_t = phi x_{t-1} + e_t, var(e) = 1; the variance of the mean of n samples is
    # 1 / ((1 - phi)^2 n) for n >> 1/(1 - phi).  Checked over independent series.
    rng = np.random.default_rng(1)
    phi, n = 0.9, 1 << 15
    target = 1.0 / ((1.0 - phi) * np.sqrt(n))
    ests = []
    for _ in range(20):
        e = rng.normal(size=n)
        x = np.empty(n)
        x[0] = e[0] / np.sqrt(1 - phi * phi)
        for t in range(1, n):
            x[t] = phi * x[t - 1] + e[t]
        ests.append(blocking_error(x)[1])
    assert 0.8 * target <= np.median(ests) <= 1.25 * target
    # white noise: blocking leaves the naive error
    w = rng.normal(size=n)
    assert abs(blocking_error(w)[1] / (1 / np.sqrt(n)) - 1) < 0.25


def test_fit_reproduces_exact_polynomials_and_matches_numpy():
    xis = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    coef = np.array([0.7, -1.3, 2.0])
    y = np.polyval(coef, xis)
    err = np.array([0.01, 0.02, 0.015, 0.02, 0.01])
    ex = fit_extrapolate(xis, y, err, degree=2, target=-1.0)
    assert abs(ex.value - np.polyval(coef, -1.0)) < 1e-12
    assert ex.chi2_per_dof < 1e-20
    # weighted fit and its covariance against numpy.polyfit (independent implementation)
    rng = np.random.default_rng(2)
    ynoisy = y + rng.normal(scale=err)
    ex = fit_extrapolate(xis, ynoisy, err, degree=2)
    c_np, cov_np = np.polyfit(xis, ynoisy, 2, w=1.0 / err, cov="unscaled")
    assert np.allclose(ex.coefficients, c_np, rtol=1e-10, atol=1e-12)
    assert np.allclose(ex.covariance, cov_np, rtol=1e-8)
    v = np.array([1.0, -1.0, 1.0])
    assert abs(ex.error - np.sqrt(v @ cov_np @ v)) < 1e-10


def test_combine_and_argument_checks():
    m, e = combine_replicas([(1.0, 0.1), (3.0, 0.1)])
    assert m == 2.0 and abs(e - 1.0) < 1e-15          # the replica spread dominates
    m, e = combine_replicas([(1.0, 0.1), (1.0, 0.1)])
    assert m == 1.0 and abs(e - np.sqrt(0.02) / 2) < 1e-15
    with pytest.raises(ValueError):
        fit_extrapolate([0.0, 1.0], [1.0, 2.0], [0.1, 0.1], degree=2)
    with pytest.raises(ValueError):
        fit_extrapolate([0.0, 0.5, 1.0], [1.0, 2.0, 3.0], [0.1, 0.0, 0.1], degree=1)
