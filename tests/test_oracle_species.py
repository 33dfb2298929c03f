"""Pins of the two-species oracle (spin mixtures): exchange cycles stay within a species and
each species' exchange sum is its own Eq. 6, so without a pair term the composite system is
two independent systems, a fact that the single-species oracle (pinned on its own) checks:
potentials add, forces, probability blocks and the expected spring energy equal those of the
species run separately, and no probability connects the species.  The pair term acts on all
particles of a slice, so it couples the species: switching it on changes the forces by exactly
the pair forces of the full system."""
import numpy as np
import pytest

from paper_2404_02628_amd.workloads import random_positions


def _par(orc, n, n2=0, **kw):
    base = dict(p=5, dim=2, beta=1.3, xi=0.7)
    base.update(kw)
    return orc.OracleParams(n=n, n2=n2, **base)


@pytest.mark.parametrize("n,n2,xi,dim", [(7, 3, 0.7, 2), (5, 1, 1.0, 3), (6, 5, 0.3, 1), (8, 4, 0.0, 2), (2, 1, 1.0, 2)])
def test_two_species_factorise_without_pair_term(orc, n, n2, xi, dim):
    x = random_positions(n, 5, dim, 0.8, n + 10 * n2)
    na = n - n2
    f, en, X, Y, G = orc.compute_forces(_par(orc, n, n2, xi=xi, dim=dim), x, want_tables=True)
    fa, ea, Xa, Ya, Ga = orc.compute_forces(_par(orc, na, xi=xi, dim=dim), x[:, :, :na].copy(), want_tables=True)
    fb, eb, Xb, Yb, Gb = orc.compute_forces(_par(orc, n2, xi=xi, dim=dim), x[:, :, na:].copy(), want_tables=True)
    tol = 1e-12 * max(1.0, abs(X[n]))
    assert abs(X[n] - (Xa[na] + Xb[n2])) <= tol
    assert abs(X[n] - Y[1]) <= tol
    assert np.allclose(X[:na + 1], Xa, rtol=1e-13, atol=tol)
    assert np.allclose(Y[na + 1:n + 1], Yb[1:n2 + 1], rtol=1e-13, atol=tol)
    assert abs(en["v_exch"] - (ea["v_exch"] + eb["v_exch"])) <= 1e-12 * abs(en["v_exch"])
    scale = max(np.abs(f).max(), 1.0)
    assert np.abs(f[:, :, :na] - fa).max() <= 1e-11 * scale
    assert np.abs(f[:, :, na:] - fb).max() <= 1e-11 * scale
    assert np.abs(G[:na, :na] - Ga).max() <= 1e-12 and np.abs(G[na:, na:] - Gb).max() <= 1e-12
    assert np.abs(G[:na, na:]).max() == 0.0 and np.abs(G[na:, :na]).max() == 0.0
    assert np.allclose(G.sum(axis=1), 1.0, atol=1e-12) and np.allclose(G.sum(axis=0), 1.0, atol=1e-12)
    S = ea["spring_expect"] + eb["spring_expect"]
    assert abs(en["spring_expect"] - S) <= 1e-12 * abs(S)


def test_pair_term_couples_the_species(orc):
    n, n2 = 6, 2
    x = random_positions(n, 5, 2, 0.5, 77)
    on = dict(pair_amp=1.5, pair_width=0.6)
    f0, _ = orc.compute_forces(_par(orc, n, n2), x)
    f1, _ = orc.compute_forces(_par(orc, n, n2, **on), x)
    fu_on = orc.interaction(_par(orc, n, n2, **on), x)[0]
    fu_off = orc.interaction(_par(orc, n, n2), x)[0]
    assert np.abs((f1 - f0) - (fu_on - fu_off)).max() <= 1e-12 * np.abs(f1).max()
    # moving species B changes the pair forces on species A: cross-species pairs contribute
    xb = x.copy()
    xb[:, :, n - n2:] += 0.3
    fu_b = orc.interaction(_par(orc, n, n2, **on), xb)[0]
    assert np.abs(fu_b[:, :, :n - n2] - fu_on[:, :, :n - n2]).max() > 1e-6


def test_species_count_is_validated(orc):
    x = random_positions(4, 5, 2, 0.8, 1)
    for bad in (-1, 4, 5):
        with pytest.raises(Exception):
            orc.compute_forces(_par(orc, 4, bad), x)
