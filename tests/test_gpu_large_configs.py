"""The large single-replica configurations (N = 10^4 and 4 10^4 ideal bosons, d = 3, P = 16,
beta = 2, FP64) and the batched uneven-xi configuration (64 replicas, N ~ U{64..512},
xi = 0.2 (1 + r mod 5), A = 1, s = 0.5, P = 32, d = 2).

N = 10^4 is compared with the oracle directly, potentials within 1e-10 and forces within c_X of
their scale as in the parity tests, with c_X = 1e-10 + max(32, sqrt(N)) eps max|X|: every one of
the N sequential steps of Eqs. 6 and 11 rounds at eps |X| and passes earlier errors on with gain
at most one, so the error of X grows like sqrt(N) eps max|X| (a random walk), and the
probabilities of Eq. 12 inherit it as relative error through X_N - X_{l'-1} - Y_{l+1}.  The GPU
keeps its potentials in the normalised form G^f_n = beta sum_{l<=n} (E_int + link) - X_n (and the
mirror G^b), whose size max|G| can exceed max|X| when neighbouring rings are far apart, so its
probabilities carry c_G = 1e-10 + max(32, sqrt(N)) eps max|G| in the same way.  The expected
spring energy S = sum_{l'<=l} Pr[l->l'] E^{[l',l]} is the internal energies (exact on both
sides) plus a sum of non-negative terms, each a probability whose exponent carries three
potentials, times the closing term and links of its cycle; so its exchange part S - sum E_int
is compared within 4 (c_X + c_G) of itself.  It is also tied to the GPU's own forces by the
homogeneity identity below at 1e-10.
At N = 4 10^4 the oracle's O(N^2) tables do not fit a test, so the check uses identities that
hold at any size:
  * X_N = Y_1: the forward (Eq. 6) and backward (Eq. 11) recursions give the same V_xi^{[1,N]};
  * translation invariance: the spring and exchange forces sum to zero, so the total force
    plus the trap force (m omega^2 / P) r sums to zero;
  * homogeneity: every E^{[u,v]} is homogeneous of degree 2 in the positions, so
    sum r . (spring and exchange forces) = -2 S with S the expected spring energy.  The GPU's S
    is a sum of non-negative terms, but its end-bead forces take Pr[l -> l+1] from Eq. 13 as
    1 - exp(...) of a difference of normalised potentials, with an absolute error of up to c_G
    (the rounding of potentials of size max|G|); each link l then moves the sum by at most
    c_G (2 link_l + kappa (|b_l| |b_l - r_l^{P-1}| + |a_{l+1}| |a_{l+1} - r_{l+1}^2|)), which
    bounds the residual (homogeneity_bound below), with max|G| bounded from the positions alone
    (gpu_potential_bound);
  * the estimator identity E_prim = d N P / (2 beta) - S + U/P;
  * a second evaluation of the same state repeats the first bit for bit.
The batched configuration is checked replica by replica against the oracle."""
import numpy as np
import pytest

from paper_2404_02628_amd.workloads import WORKLOADS, batched_systems, initial_state, thermal_rings

pytestmark = pytest.mark.gpu


def _par(orc, s):
    return orc.OracleParams(n=s.n, p=s.p, dim=s.dim, beta=s.beta, xi=s.xi, pair_amp=s.pair_amp,
                            pair_width=s.pair_width, hbar=s.hbar, mass=s.mass, omega=s.omega)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _springs(s, x):
    """Internal energies, links and self-closing terms of Eqs. 7-9 from the positions."""
    c = 0.5 * s.mass * s.p / (s.beta * s.hbar) ** 2
    eint = c * np.sum((x[:, 1:, :] - x[:, :-1, :]) ** 2, axis=(0, 1))
    link = np.zeros(s.n)
    link[:-1] = c * np.sum((x[:, s.p - 1, :-1] - x[:, 0, 1:]) ** 2, axis=0)
    close = c * np.sum((x[:, s.p - 1, :] - x[:, 0, :]) ** 2, axis=0)
    return eint, link, close


def gpu_potential_bound(s, x):
    """Upper bound of max|G| for the GPU's normalised potentials G^f_n = beta sum_{l<=n} (E_int + link)
    - X_n (and the mirror G^b), from the positions alone: every E is non-negative and the weights
    prod 1/max(I) of the compositions of 1..n sum to one, so 0 <= X_n; the all-singletons
    composition alone gives X_n <= beta sum_{l<=n} E^{[l,l]} + log n!."""
    import math
    eint, link, close = _springs(s, x)
    tot = s.beta * (float(np.sum(eint)) + float(np.sum(link)) + float(np.sum(eint + close)))
    return tot + math.lgamma(s.n + 1)


def homogeneity_bound(s, x, c_g):
    """Largest change of sum r . F that an absolute error c_g in every Pr[l -> l+1] can cause."""
    eint, link, _ = _springs(s, x)
    kappa = s.mass * s.p / (s.beta * s.hbar) ** 2
    a, b = x[:, 0, :], x[:, s.p - 1, :]
    ra = np.linalg.norm(a, axis=0)
    rb = np.linalg.norm(b, axis=0)
    tb = np.linalg.norm(b - x[:, s.p - 2, :], axis=0)   # |b_l - r_l^{P-1}|
    ta = np.linalg.norm(a - x[:, 1, :], axis=0)         # |a_l - r_l^2|
    w = 2.0 * link[:-1] + kappa * (rb[:-1] * tb[:-1] + ra[1:] * ta[1:])
    return c_g * float(np.sum(w))


def test_ideal_10k_matches_oracle(orc):
    from paper_2404_02628_amd.pimd import Context
    s = WORKLOADS["huge_ideal_10k"]
    x = thermal_rings(s.n, s.p, s.dim, s.beta, s.sigma, s.seed)
    print(f"N={s.n} P={s.p} d={s.dim}: GPU evaluation", flush=True)
    ctx = Context([s], precision="fp64")
    try:
        ctx.set_state(0, x)
        ctx.compute_forces()
        f = ctx.forces(0)
        en = ctx.energies(0)
        X, Y = ctx.potentials(0)
    finally:
        ctx.close()
    print("oracle evaluation", flush=True)
    f_or, en_or, X_or, Y_or = orc.compute_forces(_par(orc, s), x, want_tables=True)[:4]
    eps = np.finfo(float).eps
    c_x = 1e-10 + max(32.0, np.sqrt(s.n)) * eps * float(np.max(np.abs(X_or)))
    # size of the GPU's normalised forward potentials: beta sum_{l<=n} (E_int + link) - X_n
    eint = orc.internal_energies(_par(orc, s), x)
    _, link, _ = _springs(s, x)
    g_f = s.beta * np.concatenate([[0.0], np.cumsum(eint + link)]) - X_or
    c_g = 1e-10 + max(32.0, np.sqrt(s.n)) * eps * max(float(np.max(np.abs(g_f))), float(np.max(np.abs(X_or))))
    s_exch = abs(en_or["spring_expect"] - float(np.sum(eint)))
    kappa = s.mass * s.p / (s.beta * s.hbar) ** 2
    scale = max(float(np.max(np.abs(f_or))), 4.0 * kappa * float(np.max(np.abs(x))))
    errs = {"forces": float(np.max(np.abs(f - f_or))) / scale, "X": _rel(X, X_or), "Y": _rel(Y[1:], Y_or[1:]),
            "v_exch": abs(en["v_exch"] - en_or["v_exch"]) / abs(en_or["v_exch"]),
            "spring_expect": abs(en["spring_expect"] - en_or["spring_expect"]) / abs(en_or["spring_expect"]),
            "e_vir": abs(en["e_vir"] - en_or["e_vir"]) / abs(en_or["e_vir"])}
    # homogeneity residual |sum r . (spring + exchange forces) + 2 S| of each side
    trap = s.mass * s.omega ** 2 / s.p
    res = {name: abs(float(np.sum(x * (ff + trap * x))) + 2.0 * e["spring_expect"])
           for name, ff, e in (("gpu", f, en), ("oracle", f_or, en_or))}
    hom = homogeneity_bound(s, x, c_g) + 1e-10 * abs(2.0 * en["spring_expect"])
    print(f"c_X = {c_x:.3e}, max|X| = {np.max(np.abs(X_or)):.3e}, c_G = {c_g:.3e}, S - sum E_int = {s_exch:.6e}, "
          f"errors {errs}, identity residuals {res} (bound {hom:.3e})", flush=True)
    assert errs["forces"] <= c_x
    assert errs["X"] <= 1e-10 and errs["Y"] <= 1e-10 and errs["v_exch"] <= 1e-10
    assert errs["e_vir"] <= 1e-10
    # S - sum E_int = sum_{l'<=l} Pr[l->l'] (E^{[l',l]} - sum_{m=l'}^{l} E_int^{(m)}) is a sum of
    # non-negative terms, so its relative error is at most the largest relative error of a term.
    # A probability of Eq. 12 is the exponential of X_N - X_{l'-1} - Y_{l+1} - beta E + log
    # weights, so its relative error is the absolute error of that exponent: at most c_X (oracle)
    # or c_G (GPU) for each of the three potentials and for the beta E term, 4 (c_X + c_G) for the
    # difference of the two sides.  The GPU's S is also tied to its own forces by the homogeneity
    # identity, within the error its end-bead forces take from Eq. 13.
    assert res["gpu"] <= hom, (res["gpu"], hom)
    d_s = abs(en["spring_expect"] - en_or["spring_expect"])
    assert d_s <= 4.0 * (c_x + c_g) * s_exch + 1e-14 * abs(en_or["spring_expect"]), (d_s, s_exch, c_x, c_g)


@pytest.mark.parametrize("start", ["thermal", "seeded"])
def test_ideal_40k_identities(start):
    from paper_2404_02628_amd.pimd import Context
    s = WORKLOADS["huge_ideal_40k"]
    x = thermal_rings(s.n, s.p, s.dim, s.beta, s.sigma, s.seed) if start == "thermal" else initial_state(s)[0]
    print(f"N={s.n} P={s.p} d={s.dim} ({start}): GPU evaluations", flush=True)
    ctx = Context([s], precision="fp64")
    try:
        ctx.set_state(0, x)
        ctx.compute_forces()
        f = ctx.forces(0)
        en = ctx.energies(0)
        X, Y = ctx.potentials(0)
        ctx.compute_forces()
        f2 = ctx.forces(0)
    finally:
        ctx.close()
    assert np.array_equal(f, f2)
    assert abs(X[s.n] - Y[1]) <= 1e-12 * abs(X[s.n])
    trap = s.mass * s.omega ** 2 / s.p
    g = f + trap * x                      # spring + exchange forces
    for a in range(s.dim):
        assert abs(g[a].sum()) <= 1e-11 * float(np.abs(g[a]).sum())
    S = en["spring_expect"]
    c_g = 1e-10 + max(32.0, np.sqrt(s.n)) * np.finfo(float).eps * gpu_potential_bound(s, x)
    hom = homogeneity_bound(s, x, c_g) + 1e-10 * abs(2.0 * S)
    print(f"homogeneity residual {abs(float(np.sum(x * g)) + 2.0 * S):.3e}, bound {hom:.3e} (c_G {c_g:.3e})", flush=True)
    assert abs(float(np.sum(x * g)) + 2.0 * S) <= hom
    e_prim = s.dim * s.n * s.p / (2.0 * s.beta) - S + en["u_trap"] / s.p
    assert abs(en["e_prim"] - e_prim) <= 1e-12 * abs(e_prim)


@pytest.mark.parametrize("mixed,wide,order", [(False, False, "index"), (True, False, "index"),
                                              (True, True, "longest"), (False, True, "index")],
                         ids=["fp64", "mixed", "mixed-wide-longest", "fp64-wide"])
def test_batched_uneven_xi_matches_oracle(orc, mixed, wide, order):
    from paper_2404_02628_amd.pimd import Context
    systems = batched_systems(64, 505)
    xs = [initial_state(s)[0] for s in systems]
    print(f"64 uneven replicas, {'mixed' if mixed else 'fp64'}, wide={wide}, order={order}", flush=True)
    ctx = Context(systems, precision="mixed" if mixed else "fp64", wide_recursion=wide, order=order,
                  recursion_workgroups=1)
    try:
        for r, x in enumerate(xs):
            ctx.set_state(r, x)
        ctx.compute_forces()
        for r in range(0, 64, 3):
            s, x = systems[r], xs[r]
            f_or, en_or, X_or = orc.compute_forces(_par(orc, s), x, want_tables=True)[:3]
            f = ctx.forces(r)
            en = ctx.energies(r)
            X, _ = ctx.potentials(r)
            c_x = 1e-10 + 32 * np.finfo(float).eps * float(np.max(np.abs(X_or)))
            if mixed:
                assert _rel(f, f_or) <= 1e-5, (r, _rel(f, f_or))
            else:
                kappa = s.mass * s.p / (s.beta * s.hbar) ** 2
                scale = max(float(np.max(np.abs(f_or))), 4.0 * kappa * float(np.max(np.abs(x))))
                assert float(np.max(np.abs(f - f_or))) / scale <= c_x, r
            assert _rel(X, X_or) <= 1e-10, r
            tol = 1e-5 if mixed else 1e-10
            U = abs(en_or["u_trap"]) + abs(en_or["u_pair"])
            assert abs(en["u_pair"] - en_or["u_pair"]) <= tol * U, r
            assert abs(en["e_vir"] - en_or["e_vir"]) <= tol * abs(en_or["e_vir"]), r
    finally:
        ctx.close()
