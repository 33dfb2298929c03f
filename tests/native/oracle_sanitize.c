/* Drives every entry point of the CPU oracle over small systems, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: one, two, five and nine particles, two to
 * seven beads, d = 1..3, xi in {0, 0.5, 1}, two species, with and without the pair term, a
 * few thermostatted steps, the exact energies, the generator, and invalid arguments (which must
 * be refused with a negative status).  Every buffer is allocated at exactly the documented
 * size, so a read or write past it is reported by the sanitizer.  Prints "ok" and the number of
 * configurations on success; any sanitizer report ends the process with a non-zero status. */
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/pimd_oracle.h"

static int fails = 0;

static void check(int cond, const char* what, int n, int p, int d) {
    if (!cond) {
        fprintf(stderr, "FAILED %s (n=%d p=%d d=%d)\n", what, n, p, d);
        ++fails;
    }
}

static double* alloc(size_t count) {
    double* a = (double*)malloc((count ? count : 1) * sizeof(double));
    for (size_t i = 0; i < count; ++i) a[i] = 0.0;
    return a;
}

static int run_case(int n, int n2, int p, int d, double xi, double amp) {
    oracle_params s;
    memset(&s, 0, sizeof(s));
    s.n = n; s.p = p; s.dim = d; s.beta = 2.0; s.hbar = 1.0; s.mass = 1.0; s.omega = 1.0;
    s.xi = xi; s.pair_amp = amp; s.pair_width = 0.6; s.n2 = n2;
    oracle_md md;
    memset(&md, 0, sizeof(md));
    md.dt = 0.01; md.nhc_len = 3; md.nhc_q = 0.0; md.sy_order = 3; md.bead_mass = 0.0;
    const size_t dof = (size_t)d * p * n;
    double *x = alloc(dof), *pm = alloc(dof), *f = alloc(dof), *f2 = alloc(dof);
    double *eta = alloc(dof * md.nhc_len), *veta = alloc(dof * md.nhc_len);
    double *eint = alloc(n), *E = alloc((size_t)n * n), *X = alloc(n + 1), *Y = alloc(n + 2);
    double *G = alloc((size_t)n * n), *X2 = alloc(n + 1), *Y2 = alloc(n + 2), *G2 = alloc((size_t)n * n);
    check(oracle_init_state(&s, &md, 1.0, 1234u + (uint64_t)n, x, pm) == 0, "init_state", n, p, d);
    for (size_t i = 0; i < dof; ++i) check(isfinite(x[i]) && isfinite(pm[i]), "finite state", n, p, d);
    for (int v = 1; v <= n; ++v)
        for (int u = 1; u <= v; ++u) check(isfinite(oracle_ring_energy(&s, x, u, v)), "ring_energy", n, p, d);
    check(oracle_internal_energies(&s, x, eint) == 0, "internal_energies", n, p, d);
    check(oracle_cycle_energies(&s, x, E) == 0, "cycle_energies", n, p, d);
    check(oracle_forward_potentials(&s, E, X) == 0, "forward_potentials", n, p, d);
    check(oracle_backward_potentials(&s, E, Y) == 0, "backward_potentials", n, p, d);
    check(oracle_connection_probabilities(&s, E, X, Y, G) == 0, "probabilities", n, p, d);
    check(oracle_exchange_forces(&s, x, G, f) == 0, "exchange_forces", n, p, d);
    double ut = 0.0, up = 0.0, vir = 0.0;
    check(oracle_interaction(&s, x, f2, &ut, &up, &vir) == 0, "interaction", n, p, d);
    oracle_energies en;
    check(oracle_compute_forces(&s, x, f, &en, X2, Y2, G2) == 0, "compute_forces", n, p, d);
    check(oracle_compute_forces(&s, x, f, &en, NULL, NULL, NULL) == 0, "compute_forces (no tables)", n, p, d);
    check(isfinite(en.v_exch) && isfinite(en.e_prim) && isfinite(en.e_vir), "finite energies", n, p, d);
    check(oracle_step(&s, &md, x, pm, eta, veta, f, 3) == 0, "step", n, p, d);
    check(isfinite(oracle_conserved(&s, &md, x, pm, eta, veta)), "conserved", n, p, d);
    uint64_t* counts = (uint64_t*)calloc(17, sizeof(uint64_t));
    check(oracle_density(&s, x, 16, 4.0, counts) == 0, "density", n, p, d);
    uint64_t total = 0;
    for (int b = 0; b <= 16; ++b) total += counts[b];
    check(total == (uint64_t)n * p, "density counts", n, p, d);
    /* NVE (no thermostat arrays) and the first-order splitting */
    oracle_md nve = md;
    nve.nhc_len = 0; nve.sy_order = 1;
    check(oracle_step(&s, &nve, x, pm, NULL, NULL, f, 2) == 0, "step (NVE)", n, p, d);
    /* invalid arguments are refused */
    oracle_params bad = s;
    bad.n = 0;
    check(oracle_compute_forces(&bad, x, f, &en, NULL, NULL, NULL) < 0, "refuses n = 0", n, p, d);
    bad = s; bad.p = 1;
    check(oracle_compute_forces(&bad, x, f, &en, NULL, NULL, NULL) < 0, "refuses p = 1", n, p, d);
    bad = s; bad.dim = 4;
    check(oracle_compute_forces(&bad, x, f, &en, NULL, NULL, NULL) < 0, "refuses dim = 4", n, p, d);
    bad = s; bad.n2 = n;
    check(oracle_compute_forces(&bad, x, f, &en, NULL, NULL, NULL) < 0, "refuses n2 = n", n, p, d);
    free(counts);
    free(x); free(pm); free(f); free(f2); free(eta); free(veta); free(eint); free(E); free(X); free(Y);
    free(G); free(X2); free(Y2); free(G2);
    return 1;
}

int main(void) {
    const int ns[] = {1, 2, 5, 9}, ps[] = {2, 3, 7};
    const double xis[] = {0.0, 0.5, 1.0};
    int cases = 0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 3; ++b)
            for (int d = 1; d <= 3; ++d)
                for (int k = 0; k < 3; ++k) {
                    const int n = ns[a];
                    cases += run_case(n, 0, ps[b], d, xis[k], (a + k) % 2 ? 1.0 : 0.0);
                    if (n >= 2) cases += run_case(n, n / 2, ps[b], d, xis[k], 0.5);
                }
    for (int m = 1; m <= 6; ++m)
        for (int pp = 0; pp <= 8; pp += 4) {
            check(isfinite(oracle_exact_energy(m, 2, 1.5, pp, 1.0)), "exact_energy", m, pp, 2);
            check(isfinite(oracle_exact_energy_signed(m, 2, 1.5, pp, -1.0)), "exact_energy_signed", m, pp, 2);
        }
    uint32_t ctr[4] = {1u, 2u, 3u, 4u}, key[2] = {5u, 6u}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("ok %d\n", cases);
    return 0;
}
