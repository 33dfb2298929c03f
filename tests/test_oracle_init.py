"""Pins of the oracle's seeded initial state (Philox4x32-10 + Box-Muller).

* Philox4x32-10 reproduces the generator authors' published known-answer vectors (zero counter
  and key, all-ones counter and key, and the counter/key taken from the hexadecimal digits of
  pi), which fixes every multiplier, Weyl constant, word order and the round count.
* The Box-Muller deviates are N(0, 1): mean, variance and fourth moment within 5 standard
  errors over 10^6 deviates, and a Kolmogorov-Smirnov test against the normal distribution.
* Positions scale with sigma, momenta have variance m'/beta (bead mass honoured), the two
  arrays are uncorrelated, a seed repeats bit for bit and another seed does not."""
import numpy as np
import pytest

KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT, ids=["zero", "ones", "pi"])
def test_philox_known_answers(orc, ctr, key, out):
    assert orc.philox4x32_10(ctr, key) == out


def _state(orc, n=500, p=1000, dim=2, sigma=1.0, seed=12345, beta=1.0, bead_mass=0.0):
    par = orc.OracleParams(n=n, p=p, dim=dim, beta=beta)
    md = orc.OracleMD(dt=0.01, nhc_len=4, bead_mass=bead_mass)
    return orc.init_state(par, md, sigma, seed)


def test_deviates_are_standard_normal(orc):
    from scipy import stats
    x, p = _state(orc)
    for z in (x.ravel(), p.ravel()):
        n = z.size
        assert abs(z.mean()) <= 5.0 / np.sqrt(n)
        assert abs(z.var() - 1.0) <= 5.0 * np.sqrt(2.0 / n)
        assert abs(np.mean(z ** 4) - 3.0) <= 5.0 * np.sqrt(96.0 / n)
        assert stats.kstest(z, "norm").pvalue > 1e-4
    # consecutive deviates (the cosine and sine of one pair) are uncorrelated
    zz = x.ravel()
    assert abs(np.mean(zz[0::2] * zz[1::2])) <= 5.0 / np.sqrt(zz.size / 2)


def test_scales_seeds_and_independence(orc):
    x, p = _state(orc, n=300, p=200, dim=3, sigma=2.5, seed=7, beta=3.0, bead_mass=2.0)
    n = x.size
    assert abs(x.var() / 2.5 ** 2 - 1.0) <= 5.0 * np.sqrt(2.0 / n)
    assert abs(p.var() / (2.0 / 3.0) - 1.0) <= 5.0 * np.sqrt(2.0 / n)
    assert abs(np.mean(x.ravel() * p.ravel())) / (2.5 * np.sqrt(2.0 / 3.0)) <= 5.0 / np.sqrt(n)
    x2, p2 = _state(orc, n=300, p=200, dim=3, sigma=2.5, seed=7, beta=3.0, bead_mass=2.0)
    assert np.array_equal(x, x2) and np.array_equal(p, p2)
    x3, _ = _state(orc, n=300, p=200, dim=3, sigma=2.5, seed=8, beta=3.0, bead_mass=2.0)
    assert np.mean(x3 == x) < 1e-4
    # seeds differing only in the high word give different streams
    x4, _ = _state(orc, n=300, p=200, dim=3, sigma=2.5, seed=7 + (1 << 32), beta=3.0, bead_mass=2.0)
    assert np.mean(x4 == x) < 1e-4
