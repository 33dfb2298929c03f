"""xi-extrapolation for fictitious identical particles (post-processing of batched runs).

The exchange parameter xi interpolates between distinguishable particles (0) and bosons (1);
fermions are xi = -1 (Sec. II), where the weight exp(-beta V_xi) is no longer positive and
PIMD cannot sample directly.  The method the paper builds on (its fictitious-particle section)
samples 0 <= xi <= 1, where the weight is positive, fits the energy as a function of xi, and
evaluates the fit at xi = -1.  Here every xi of the ensemble runs as replicas of one batched
context; each replica records its energy estimator every `sample_every` steps; per xi the
mean and an error bar are formed (blocking within a replica, and the spread of the independent
replicas, whichever is larger); a weighted least-squares polynomial in xi gives the
extrapolated value and its propagated statistical error.  The fit's own model bias is not part
of that error: for strongly degenerate systems a low-order polynomial is a poor model.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .workloads import System, initial_state


def blocking_error(series: Sequence[float], min_blocks: int = 16) -> Tuple[float, float]:
    """Mean of a correlated series and its standard error by blocking (Flyvbjerg and Petersen,
    J. Chem. Phys. 91, 461 (1989)): pairs are averaged repeatedly, and the error estimate of a
    level is sqrt(var / (n - 1)); the first level whose next level does not raise the estimate
    beyond its own uncertainty is taken (else the last level with min_blocks blocks)."""
    x = np.asarray(series, dtype=float)
    if x.size < 2:
        raise ValueError("need at least two samples")
    mean = float(x.mean())
    levels = []
    while x.size >= min_blocks:
        n = x.size
        s = float(np.sqrt(x.var() / (n - 1)))
        levels.append((s, s / np.sqrt(2.0 * (n - 1))))
        x = 0.5 * (x[: n // 2 * 2 : 2] + x[1 : n // 2 * 2 : 2])
    if not levels:
        n = len(series)
        return mean, float(np.std(series) / np.sqrt(n - 1))
    for k in range(len(levels) - 1):
        s, ds = levels[k]
        if levels[k + 1][0] - s <= ds:
            return mean, max(s, levels[k + 1][0])
    return mean, levels[-1][0]


def combine_replicas(estimates: Sequence[Tuple[float, float]]) -> Tuple[float, float]:
    """Mean over independent replicas (equal weight).  Its error is the larger of the value
    propagated from the per-replica blocking errors and the standard error of the replica
    means: when a run is short against the correlation time, blocking underestimates, while
    the spread of independent replicas does not."""
    m = np.array([e[0] for e in estimates])
    s = np.array([e[1] for e in estimates])
    err = float(np.sqrt(np.sum(s * s)) / len(estimates))
    if len(estimates) >= 2:
        err = max(err, float(m.std(ddof=1) / np.sqrt(len(estimates))))
    return float(m.mean()), err


@dataclass
class Extrapolation:
    value: float           # fit evaluated at the target xi
    error: float           # propagated statistical error of that value
    coefficients: np.ndarray  # polynomial coefficients, highest power first (numpy.polyval order)
    covariance: np.ndarray
    chi2_per_dof: float


def fit_extrapolate(xis: Sequence[float], means: Sequence[float], errors: Sequence[float], degree: int = 2,
                    target: float = -1.0) -> Extrapolation:
    """Weighted least-squares polynomial of the given degree through (xi, mean +- error),
    evaluated at `target` with the error propagated through the fit's covariance."""
    x = np.asarray(xis, dtype=float)
    y = np.asarray(means, dtype=float)
    e = np.asarray(errors, dtype=float)
    if x.size <= degree:
        raise ValueError("need more xi values than the polynomial degree")
    if np.any(e <= 0):
        raise ValueError("errors must be positive")
    V = np.vander(x, degree + 1)                 # columns x^degree .. x^0
    w = 1.0 / (e * e)
    A = V.T @ (w[:, None] * V)
    cov = np.linalg.inv(A)
    coef = cov @ (V.T @ (w * y))
    v = np.vander(np.array([target], dtype=float), degree + 1)[0]
    val = float(v @ coef)
    err = float(np.sqrt(v @ cov @ v))
    resid = (y - V @ coef) / e
    dof = max(x.size - degree - 1, 1)
    return Extrapolation(val, err, coef, cov, float(resid @ resid / dof))


@dataclass
class EnsembleResult:
    xis: List[float]
    means: List[float]
    errors: List[float]
    replicas: Dict[float, List[Tuple[float, float]]]


def run_ensemble(base: System, xis: Sequence[float], replicas_per_xi: int, steps: int, sample_every: int,
                 warmup: int, precision: str = "fp64", estimator: str = "e_vir", seed0: int = 7000,
                 **ctx_kw) -> EnsembleResult:
    """Runs replicas of `base` at every xi in one batched context and returns the per-xi mean
    estimator with its error (replica seeds seed0, seed0+1, ...)."""
    from .pimd import Context
    systems = [base.with_(xi=float(xi), seed=seed0 + k) for k, xi in
               enumerate(x for x in xis for _ in range(replicas_per_xi))]
    cap = steps // sample_every
    ctx = Context(systems, precision=precision, trace_capacity=cap, **ctx_kw)
    try:
        for r, s in enumerate(systems):
            x, p = initial_state(s)
            ctx.set_state(r, x, p)
        ctx.step(warmup, 0)
        ctx.reset_accumulators()
        ctx.step(steps, sample_every)
        per_xi: Dict[float, List[Tuple[float, float]]] = {float(x): [] for x in xis}
        for r, s in enumerate(systems):
            series = [t[estimator] for t in ctx.trace(r, cap)]
            per_xi[float(s.xi)].append(blocking_error(series))
    finally:
        ctx.close()
    means, errors = [], []
    for x in xis:
        m, e = combine_replicas(per_xi[float(x)])
        means.append(m)
        errors.append(e)
    return EnsembleResult([float(x) for x in xis], means, errors, per_xi)
