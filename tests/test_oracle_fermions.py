"""Pins of the oracle's signed exact energy (any real xi, fermions included), the reference of
the xi-extrapolation.  Each pin is independent of the routine's own formula:

* for 0 <= xi <= 1 it equals the log-domain cycle recursion (a separate implementation);
* one-dimensional harmonic-trap fermions are bosons shifted by N(N-1)/2 quanta: the fermionic
  single-particle levels are the bosonic ones with the ground-state Fermi sea removed, so
  Z_F(B) = e^{-B N(N-1)/2} Z_B(B) and E_F - E_B = N(N-1)/2 dB/dbeta (finite P: B = P arccosh
  (1 + beta^2/2P^2); continuum: B = beta);
* two particles: Z_2 = (z(B)^2 + xi z(2B))/2 with z(B) = (2 sinh(B/2))^{-d}, differentiated
  numerically.
"""
import math

import numpy as np
import pytest


def _dB(beta, p):
    if p == 0:
        return 1.0
    a = 1.0 + beta * beta / (2.0 * p * p)
    return (beta / p) / math.sqrt(a * a - 1.0)


def _B(beta, p):
    return beta if p == 0 else p * math.acosh(1.0 + beta * beta / (2.0 * p * p))


@pytest.mark.parametrize("p", [0, 12])
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_signed_equals_log_domain_for_nonnegative_xi(orc, dim, p):
    for n in (1, 2, 5, 10):
        for xi in (0.0, 0.2, 0.5, 1.0):
            a = orc.exact_energy(n, dim, 1.7, p, xi)
            b = orc.exact_energy_signed(n, dim, 1.7, p, xi)
            assert abs(a - b) <= 1e-12 * abs(a), (n, xi, a, b)


@pytest.mark.parametrize("p", [0, 8, 32])
def test_one_dimensional_fermions_are_shifted_bosons(orc, p):
    """The signed sums cancel down to |Z_F| = e^{-B N(N-1)/2} Z_B, so the routine loses that
    factor of precision: the bar is 16 eps e^{B N(N-1)/2} relative to the energy."""
    beta = 1.3
    for n in (2, 3, 4, 5, 6):
        shift = orc.exact_energy_signed(n, 1, beta, p, -1.0) - orc.exact_energy(n, 1, beta, p, 1.0)
        cond = math.exp(_B(beta, p) * n * (n - 1) / 2.0)
        bar = 1e-12 + 16 * np.finfo(float).eps * cond * orc.exact_energy(n, 1, beta, p, 1.0)
        assert abs(shift - 0.5 * n * (n - 1) * _dB(beta, p)) <= bar, (n, shift, bar)


@pytest.mark.parametrize("xi", [-1.0, -0.5, 0.3])
@pytest.mark.parametrize("dim", [2, 3])
def test_two_particles_closed_form(orc, xi, dim):
    beta, p = 2.0, 16

    def lnZ(b):
        B = _B(b, p)
        z = lambda t: (2.0 * math.sinh(t / 2.0)) ** (-dim)
        return math.log(0.5 * (z(B) ** 2 + xi * z(2 * B)))

    h = 1e-5
    e_fd = -(lnZ(beta + h) - lnZ(beta - h)) / (2 * h)
    e = orc.exact_energy_signed(2, dim, beta, p, xi)
    assert abs(e - e_fd) <= 1e-7 * abs(e), (e, e_fd)
