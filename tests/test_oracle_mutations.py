"""The oracle's pins catch plausible mistakes: each mutation below is planted in a temporary
copy of oracle/pimd_oracle.c (CPU only), compiled, and the pin suite must fail on it."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "drop 1/l in Eq. 12": ("double lw = log_xi_pow(s->xi, l - lp) - log(local_index(s, l));",
                           "double lw = log_xi_pow(s->xi, l - lp);"),
    "transposed Pr in Eq. 15": ("double g_in = G[(size_t)(lp - 1) * N + (l - 1)];",
                                "double g_in = G[(size_t)(l - 1) * N + (lp - 1)];"),
    "local index in Eq. 11": ("- log(local_index(s, l)) - (s->beta * e + Y[l + 1]);",
                              "- log((double)(l - u + 1)) - (s->beta * e + Y[l + 1]);"),
    "sign in Eq. 10": ("+ c * sqdist_beads(s, x, P, u, 1, u + 1)", "- c * sqdist_beads(s, x, P, u, 1, u + 1)"),
    "xi power in Eq. 6": (": log_xi_pow(s->xi, k - 1) - (s->beta * e + X[n - k]);",
                          ": log_xi_pow(s->xi, k) - (s->beta * e + X[n - k]);"),
    "pair force sign": ("g[(size_t)(l - 1) * D + a] += -2.0 * u * d * inv_s2;",
                        "g[(size_t)(l - 1) * D + a] += 2.0 * u * d * inv_s2;"),
    "bead index in Eq. 17": ("R(x, a, j + 1, l) - R(x, a, j - 1, l));", "R(x, a, j + 1, l) - R(x, a, j, l));"),
    "primitive sign": ("- e->spring_expect + (ut + up)", "+ e->spring_expect + (ut + up)"),
    "cycle energy factor k": ("double eps = 0.5 * (double)dim * (double)k / tanh(0.5 * kb);",
                              "double eps = 0.5 * (double)dim / tanh(0.5 * kb);"),
    "sign in Eq. 13": ("pr = 1.0 - exp(-(X[l] + Y[l + 1]) + XN);", "pr = 1.0 - exp(-(X[l] + Y[l + 1]) - XN);"),
    "virial half": ("ks_add(&vir, 0.5 * R(x, a, j, l) * gr);", "ks_add(&vir, R(x, a, j, l) * gr);"),
    "density binning": ("int b = (r >= rmax) ? bins : (int)(r / rmax * bins);",
                        "int b = (r >= rmax) ? bins : (int)(r * r / rmax * bins);"),
    "signed recursion: xi power": ("            xk *= xi;\n", "            xk *= -xi;\n"),
    "signed recursion: product rule": ("ds += xk * (dzt * Z[m - k] + zt * dZ[m - k]);",
                                       "ds += xk * (dzt * Z[m - k]);"),
    "signed recursion: ground-state shift": ("double EB = 0.5 * (double)dim * (double)n - dZ[n] / Z[n];",
                                             "double EB = 0.5 * (double)dim - dZ[n] / Z[n];"),
    "species: global 1/n": ("return (double)(v > species_a(s) ? v - species_a(s) : v);", "return (double)v;"),
    "species: cycles across species": ("return s->n2 > 0 && u <= species_a(s) && v > species_a(s);",
                                       "return s->n2 > 0 && u < species_a(s) && v > species_a(s) + 1;"),
    "species: Pr across the boundary in Eq. 12": ("if (!crosses(s, lp, l)) {", "if (1) {"),
    "species: boundary in Eq. 6": ("t[k - 1] = crosses(s, n - k + 1, n) ? -INFINITY",
                                   "t[k - 1] = crosses(s, n - k, n) ? -INFINITY"),
    "philox round count": ("for (int round = 0; round < 10; ++round) {", "for (int round = 0; round < 9; ++round) {"),
    "philox word order": ("uint32_t n1 = (uint32_t)p1;", "uint32_t n1 = (uint32_t)p0;"),
    "Box-Muller radius": ("double rad = sqrt(-2.0 * log(u1));", "double rad = sqrt(-log(u1));"),
    # the continuum factor z(k beta) for every cycle longer than one ring, planted alike in the
    # log-domain and the signed routine so that they still agree with each other
    "finite-P cycle factor z(k beta) for k >= 2": [
        ("            double kb = (double)k * B;\n            /* ln z(kB)",
         "            double kb = k == 1 ? B : (double)k * beta;\n            /* ln z(kB)"),
        ("double q = exp(-(double)k * B);", "double q = exp(-(double)k * (k == 1 ? B : beta));"),
    ],
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_fail_on_planted_mistake(name):
    src = open(os.path.join(ROOT, "oracle", "pimd_oracle.c")).read()
    edits = MUTATIONS[name]
    for old, new in ([edits] if isinstance(edits, tuple) else edits):
        assert src.count(old) == 1, f"mutation anchor not found: {name}"
        src = src.replace(old, new)
    with tempfile.TemporaryDirectory() as d:
        csrc = os.path.join(d, "pimd_oracle.c")
        with open(csrc, "w") as fh:
            fh.write(src)
        with open(os.path.join(d, "pimd_oracle.h"), "w") as fh:
            fh.write(open(os.path.join(ROOT, "oracle", "pimd_oracle.h")).read())
        lib = os.path.join(d, "liboracle.so")
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", lib, csrc, "-lm"])
        env = dict(os.environ, PIMD_ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "tests/test_oracle_pins.py", "tests/test_golden_paper.py",
                            "tests/test_oracle_fermions.py", "tests/test_oracle_species.py",
                            "tests/test_oracle_init.py", "tests/test_oracle_finite_p_exact.py"],
                           cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode != 0, f"pins did not catch: {name}\n{r.stdout[-2000:]}"
