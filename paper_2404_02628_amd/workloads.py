"""Seeded synthetic inputs for the trapped-particle PIMD workloads.

This module only draws random numbers; it holds none of the method's
arithmetic, so both the GPU path and the CPU oracle can be fed from it.
Every array uses the layout [dim][P][N] (numpy shape ``(dim, P, N)``).

Workloads (Sec. IV of the paper studies ideal and Gaussian-interacting bosons
in 2-D and 3-D isotropic harmonic traps, hbar = m = omega = k_B = 1):

* ``small_ideal``   N=8,     P=12, d=2, beta=3, xi=1, no pair term, positions N(0, 0.5^2), seed 101
* ``medium_gauss``  N=100,   P=32, d=2, beta=3, xi=1, A=2,   s=0.5, positions N(0, 1),     seed 202
* ``large_gauss``   N=1600,  P=32, d=2, beta=3, xi=1, A=0.5, s=0.5, positions N(0, 2^2),   seed 303
* ``huge_ideal``    N=10000 (seed 404) / 40000 (seed 405), P=16, d=3, beta=2, xi=1, positions N(0, 3^2)
* ``batched``       64 replicas, N ~ U{64..512}, xi = 0.2 (1 + r mod 5), P=32, d=2, beta=3, A=1, s=0.5,
                    positions N(0, 1), seed 505 (+ r for replica r)

Momenta are Maxwell-Boltzmann at beta for bead mass m' (variance m'/beta),
thermostat chains start at zero.  Random numbers come from numpy's PCG64
(``numpy.random.default_rng``).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List

import numpy as np


@dataclass
class System:
    n: int
    p: int
    dim: int
    beta: float
    xi: float = 1.0
    pair_amp: float = 0.0
    pair_width: float = 0.5
    hbar: float = 1.0
    mass: float = 1.0
    omega: float = 1.0
    sigma: float = 1.0       # std of the initial bead positions
    seed: int = 0
    dt: float = 0.01
    nhc_len: int = 4
    bead_mass: float = 0.0   # <= 0: the particle mass
    n2: int = 0              # particles of a second species (the last n2); exchange stays within a species

    def with_(self, **kw) -> "System":
        return replace(self, **kw)


WORKLOADS = {
    "small_ideal": System(n=8, p=12, dim=2, beta=3.0, xi=1.0, pair_amp=0.0, sigma=0.5, seed=101),
    "medium_gauss": System(n=100, p=32, dim=2, beta=3.0, xi=1.0, pair_amp=2.0, pair_width=0.5, sigma=1.0,
                           seed=202),
    "large_gauss": System(n=1600, p=32, dim=2, beta=3.0, xi=1.0, pair_amp=0.5, pair_width=0.5, sigma=2.0,
                          seed=303),
    "huge_ideal_10k": System(n=10000, p=16, dim=3, beta=2.0, xi=1.0, pair_amp=0.0, sigma=3.0, seed=404),
    "huge_ideal_40k": System(n=40000, p=16, dim=3, beta=2.0, xi=1.0, pair_amp=0.0, sigma=3.0, seed=405),
    # one replica of the xi-extrapolation ensembles (N = 3 ideal particles, d = 2, beta = 1, P = 12)
    "xi_ensemble_n3": System(n=3, p=12, dim=2, beta=1.0, xi=1.0, pair_amp=0.0, sigma=1.0, seed=0),
}


def batched_systems(count: int = 64, seed: int = 505) -> List[System]:
    """Uneven replicas: N_r ~ U{64..512}, xi_r = 0.2 (1 + r mod 5)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(64, 513, size=count)
    return [System(n=int(ns[r]), p=32, dim=2, beta=3.0, xi=0.2 * (1 + r % 5), pair_amp=1.0, pair_width=0.5,
                   sigma=1.0, seed=seed + r) for r in range(count)]


def initial_state(sysm: System, seed: int | None = None):
    """Positions N(0, sigma^2) and Maxwell-Boltzmann momenta, shape (dim, P, N) each."""
    rng = np.random.default_rng(sysm.seed if seed is None else seed)
    shape = (sysm.dim, sysm.p, sysm.n)
    x = rng.normal(0.0, sysm.sigma, size=shape)
    mp = sysm.bead_mass if sysm.bead_mass > 0 else sysm.mass
    p = rng.normal(0.0, np.sqrt(mp / sysm.beta), size=shape)
    return np.ascontiguousarray(x), np.ascontiguousarray(p)


def thermal_rings(n: int, p: int, dim: int, beta: float, sigma: float, seed: int, mass: float = 1.0,
                  hbar: float = 1.0) -> np.ndarray:
    """Ring polymers with centroids N(0, sigma^2) and internal shapes drawn from the free-ring
    Boltzmann weight exp(-(beta m P / (2 (beta hbar)^2)) sum_j |r^{j+1} - r^j|^2): the bead
    statistics of an equilibrated run, so test configurations have realistic spring energies."""
    rng = np.random.default_rng(seed)
    lap = 2.0 * np.eye(p) - np.roll(np.eye(p), 1, axis=1) - np.roll(np.eye(p), -1, axis=1)
    lam, vec = np.linalg.eigh(lap)                       # lam[0] = 0 is the centroid mode
    stiff = beta * mass * p / (beta * hbar) ** 2         # beta * m omega_P^2
    shape_map = vec[:, 1:] / np.sqrt(stiff * lam[1:])    # (p, p-1)
    out = np.empty((dim, p, n))
    for a in range(dim):
        out[a] = shape_map @ rng.normal(size=(p - 1, n))
        out[a] += rng.normal(0.0, sigma, size=n)[None, :]
    return np.ascontiguousarray(out)


def random_positions(n: int, p: int, dim: int, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.normal(0.0, sigma, size=(dim, p, n)))
