"""Independent pin of the oracle's exact finite-P energy of ideal trapped particles.

The oracle evaluates the canonical partition function with the cycle recursion and a closed
form for one k-cycle at finite P.  Here nothing of that closed form is used:

* one k-cycle of the permutation sum (Eq. 2) joins k rings end to start, so its beads form a
  single ring of k*P beads with imaginary-time step beta/P (Eqs. 4, 7).  Its Gaussian integral is
  taken from the explicit (k P) x (k P) matrix of the discretised action:
      ln z_k = d [ (kP/2) ln(P/beta) - (1/2) ln det K_k ],  K_k = (P/beta) L_{kP} + (beta/P) I,
  L the periodic second-difference matrix (hbar = m = omega = 1), so that z_1 is the P-bead
  ring and the free-particle normalisation of every link is included;
* Z_N is the plain sum over all N! permutations, each weighted xi^(N - #cycles) (every k-cycle
  carries xi^(k-1), Sec. II) times the product of its cycles' z_k, divided by N!;
* the energy -d ln Z/d beta uses the exact derivative of each log-determinant,
      d ln det K_k / d beta = tr(K_k^{-1} dK_k/d beta),  dK_k/d beta = -(P/beta^2) L + I/P.

A mistake in the finite-P mapping of a k-cycle (for example the continuum factor z(k beta)
for k >= 2, or a wrong effective inverse temperature) changes Z_N for N >= 2 at any xi > 0.
"""
import itertools
import math

import numpy as np
import pytest


def _ring_logz_and_derivative(k, p, dim, beta):
    """(ln z_k, d ln z_k / d beta) of one ring of k*p beads at step beta/p, from its matrix."""
    m = k * p
    eye = np.eye(m)
    lap = 2.0 * eye - np.roll(eye, 1, axis=1) - np.roll(eye, -1, axis=1)
    kmat = (p / beta) * lap + (beta / p) * eye
    sign, logdet = np.linalg.slogdet(kmat)
    assert sign > 0
    dk = -(p / beta ** 2) * lap + eye / p
    dlogdet = float(np.trace(np.linalg.solve(kmat, dk)))
    lnz = dim * (0.5 * m * math.log(p / beta) - 0.5 * logdet)
    dlnz = dim * (-0.5 * m / beta - 0.5 * dlogdet)
    return lnz, dlnz


def _cycle_lengths(perm):
    seen = [False] * len(perm)
    out = []
    for s in range(len(perm)):
        if seen[s]:
            continue
        k, t = 0, s
        while not seen[t]:
            seen[t] = True
            t = perm[t]
            k += 1
        out.append(k)
    return out


def exact_energy_by_permutations(n, dim, beta, p, xi):
    """-d ln Z_N / d beta from the explicit permutation sum and the ring determinants."""
    ring = {k: _ring_logz_and_derivative(k, p, dim, beta) for k in range(1, n + 1)}
    # scale every term by the identity permutation's weight so that the sums stay O(1)
    ref = n * ring[1][0]
    z = 0.0
    dz = 0.0
    for perm in itertools.permutations(range(n)):
        ks = _cycle_lengths(perm)
        w = xi ** (n - len(ks)) if n - len(ks) > 0 else 1.0
        lnw = sum(ring[k][0] for k in ks) - ref
        term = w * math.exp(lnw)
        z += term
        dz += term * sum(ring[k][1] for k in ks)
    return -dz / z


CASES = [(n, d, beta, p) for n in (2, 3, 4) for d in (1, 2, 3) for (beta, p) in ((1.3, 4), (3.0, 12))]


@pytest.mark.parametrize("n,d,beta,p", CASES)
@pytest.mark.parametrize("xi", [1.0, 0.6, 0.2, 0.0])
def test_finite_p_exact_energy_against_ring_determinants(orc, n, d, beta, p, xi):
    ref = exact_energy_by_permutations(n, d, beta, p, xi)
    got = orc.exact_energy(n, d, beta, p, xi)
    assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)


@pytest.mark.parametrize("n,d,beta,p", [(2, 1, 1.3, 4), (2, 2, 3.0, 12), (3, 2, 1.3, 4), (3, 3, 2.0, 16),
                                        (4, 2, 1.0, 6)])
@pytest.mark.parametrize("xi", [-1.0, -0.5, 0.7])
def test_finite_p_signed_exact_energy_against_ring_determinants(orc, n, d, beta, p, xi):
    """Negative xi (fermions at xi = -1): the permutation sum alternates in sign; at these sizes
    the cancellation costs a few digits at most, far inside the bar."""
    ref = exact_energy_by_permutations(n, d, beta, p, xi)
    got = orc.exact_energy_signed(n, d, beta, p, xi)
    assert abs(got - ref) <= 1e-9 * abs(ref), (got, ref)


def test_one_ring_of_kp_beads_is_not_k_rings_at_k_beta():
    """The finite-P cycle factor differs measurably from the continuum one at the configurations'
    bead counts, so the pin above can tell the two apart (about 0.3% at N = 3, P = 6, beta = 3)."""
    lnz2, _ = _ring_logz_and_derivative(2, 12, 2, 3.0)
    cont = -2 * math.log(2 * math.sinh(2 * 3.0 / 2))
    assert abs(lnz2 - cont) > 1e-3
