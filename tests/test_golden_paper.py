"""Checks against the values the paper prints (tests/golden/paper_printed_values.json)."""
import json
import math
import os

import numpy as np

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))


def test_ground_state_energy_is_N(orc):
    """Sec. IV.A: at beta = 6 the 2-D ideal Bose gas is in its ground state, E = N; the
    exact finite-P canonical energy lies well inside the paper's 0.3% band."""
    g = GOLD["ground_state_energy_2d_ideal"]
    for n in g["n_values"]:
        for p in (g["beads"], 0):
            e = orc.exact_energy(n, 2, g["beta"], p, 1.0)
            assert abs(e - n * g["energy_per_particle"]) < g["stated_deviation"] * n


def test_normalised_density_convention_reproduces_ground_state(orc):
    """Sec. IV.A: rho(r) = exp(-r^2)/pi with int rho d^2r = 1.  Beads of one free ring at
    beta = 6 are Gaussian and very close to the ground state; the histogram normalised by
    counts / (samples N P pi (r_{b+1}^2 - r_b^2)) must reproduce the paper's curve."""
    g = GOLD["ground_state_density_2d"]
    P, beta, bins, rmax = 24, g["beta"], 16, 2.4
    L = 2 * np.eye(P) - np.roll(np.eye(P), 1, axis=1) - np.roll(np.eye(P), -1, axis=1)
    cov = np.linalg.inv((P / beta) * L + (beta / P) * np.eye(P))
    rng = np.random.default_rng(1)
    par = orc.OracleParams(n=1, p=P, dim=2, beta=beta)
    counts = np.zeros(bins + 1, dtype=np.uint64)
    samp = rng.multivariate_normal(np.zeros(P), cov, size=(3000, 2))
    for k in range(samp.shape[0]):
        orc.density(par, np.ascontiguousarray(samp[k][:, :, None]), bins, rmax, counts)
    edges = np.linspace(0, rmax, bins + 1)
    rho = counts[:bins] / (counts.sum() * math.pi * (edges[1:] ** 2 - edges[:-1] ** 2))
    rc = 0.5 * (edges[1:] + edges[:-1])
    ref = np.exp(-rc ** 2) / math.pi
    assert np.max(np.abs(rho[:10] - ref[:10])) < 0.05 * ref[0]
