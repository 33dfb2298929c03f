/*
 * pimd_oracle.c -- plain CPU FP64 oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Reference: Y. Xiong, "GPU acceleration of ab initio simulations of
 * large-scale identical particles based on path integral molecular dynamics",
 * arXiv:2404.02628.  Sec. II (Eqs. 2-5) defines the sampled weight
 * exp(-beta (V_xi^{[1,N]} + U/P)); Sec. III (Eqs. 6-17) gives the quadratic
 * algorithm for V_xi and its gradient; Sec. IV (Eqs. 19, 20) the trapped
 * systems.  The thermostat is the massive Nose-Hoover chain the paper names
 * in Sec. IV.A, integrated with the Suzuki-Yoshida factorisation of Martyna,
 * Tuckerman, Tobias and Klein (Mol. Phys. 87, 1117 (1996)).
 *
 * Everything is sequential double precision in the order the paper states
 * it.  Sums of exponentials are evaluated as max + log(sum exp(t - max)),
 * which is the same sum written so that it neither overflows nor underflows.
 * Large global sums use Neumaier (compensated) summation.
 *
 * Only the tests, the smoke entry point and the benchmark's CPU-baseline leg
 * may call this library.
 */
#include "pimd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ helpers */

/* 1-based access to bead j of particle l, component a, layout [dim][P][N]. */
#define R(x, a, j, l) ((x)[((size_t)(a) * (size_t)P + (size_t)((j) - 1)) * (size_t)N + (size_t)((l) - 1)])

typedef struct { double s, c; } ksum; /* Neumaier compensated sum */
static void ks_add(ksum* k, double v) {
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static double ks_val(const ksum* k) { return k->s + k->c; }

static int check_params(const oracle_params* s) {
    if (!s) return -1;
    if (s->n < 1 || s->p < 2 || s->dim < 1 || s->dim > 3) return -1;
    if (!(s->beta > 0) || !(s->hbar > 0) || !(s->mass > 0) || !(s->omega >= 0)) return -1;
    if (!(s->xi >= 0 && s->xi <= 1)) return -1;
    if (!(s->pair_amp >= 0)) return -1;
    if (s->pair_amp > 0 && !(s->pair_width > 0)) return -1;
    if (s->n2 < 0 || s->n2 >= s->n) return -1;
    return 0;
}

/* Two species: particles 1..nA and nA+1..N (nA = N - n2).  A cycle [u,v] is allowed only
 * within one species, and the 1/n factor of a block ending at particle v counts v within
 * its species (the exchange sum of each species is its own Eq. 6).                    */
static int species_a(const oracle_params* s) { return s->n - s->n2; }
static int crosses(const oracle_params* s, int u, int v) {
    return s->n2 > 0 && u <= species_a(s) && v > species_a(s);
}
static double local_index(const oracle_params* s, int v) {
    return (double)(v > species_a(s) ? v - species_a(s) : v);
}

/* omega_P^2 = P / (beta hbar)^2  (Sec. III, after Eq. 7). */
static double omega_p2(const oracle_params* s) {
    return (double)s->p / (s->beta * s->beta * s->hbar * s->hbar);
}

/* log of xi^k with the convention 0^0 = 1 (Sec. II, after Eq. 2). */
static double log_xi_pow(double xi, int k) {
    if (k == 0) return 0.0;
    if (xi == 0.0) return -INFINITY;
    return (double)k * log(xi);
}

/* log(sum_k exp(t[k])) over k = 0..n-1, with -inf terms allowed. */
static double log_sum_exp(const double* t, int n) {
    double m = -INFINITY;
    for (int k = 0; k < n; ++k) if (t[k] > m) m = t[k];
    if (m == -INFINITY) return -INFINITY;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += exp(t[k] - m);
    return m + log(acc);
}

static double sqdist_beads(const oracle_params* s, const double* x, int j1, int l1, int j2, int l2) {
    const int N = s->n, P = s->p;
    double d2 = 0.0;
    for (int a = 0; a < s->dim; ++a) {
        double d = R(x, a, j1, l1) - R(x, a, j2, l2);
        d2 += d * d;
    }
    return d2;
}

/* --------------------------------------------------------- cycle energies */

/* Eq. 7 for the ring u..v: (1/2) m omega_P^2 sum_l sum_j (r_l^{j+1} - r_l^j)^2
 * with r_l^{P+1} = r_{l+1}^1 for l < v and r_v^{P+1} = r_u^1.              */
double oracle_ring_energy(const oracle_params* s, const double* x, int u, int v) {
    if (check_params(s) || !x || u < 1 || v > s->n || u > v) return NAN;
    const int P = s->p;
    double acc = 0.0;
    for (int l = u; l <= v; ++l) {
        for (int j = 1; j <= P; ++j) {
            int jn = j + 1, ln = l;
            if (j == P) { jn = 1; ln = (l < v) ? l + 1 : u; }
            acc += sqdist_beads(s, x, jn, ln, j, l);
        }
    }
    return 0.5 * s->mass * omega_p2(s) * acc;
}

/* Eq. 9: E_int^{(v)} = (1/2) m omega_P^2 sum_{j=1}^{P-1} (r_v^{j+1} - r_v^j)^2. */
int oracle_internal_energies(const oracle_params* s, const double* x, double* eint) {
    if (check_params(s) || !x || !eint) return -1;
    const int N = s->n, P = s->p;
    const double c = 0.5 * s->mass * omega_p2(s);
    for (int v = 1; v <= N; ++v) {
        double acc = 0.0;
        for (int j = 1; j <= P - 1; ++j) acc += sqdist_beads(s, x, j + 1, v, j, v);
        eint[v - 1] = c * acc;
    }
    return 0;
}

/* Eqs. 8-10.  The diagonal E^{[v,v]} = E_int^{(v)} + c |r_v^P - r_v^1|^2 (Eq. 8);
 * then, for each v, E^{[u,v]} for u = v-1 down to 1 by the update of Eq. 10:
 * E^{[u,v]} = E^{[u+1,v]} - c|r_v^P - r_{u+1}^1|^2 + c|r_u^P - r_{u+1}^1|^2
 *           + c|r_v^P - r_u^1|^2 + E_int^{(u)}.                              */
int oracle_cycle_energies(const oracle_params* s, const double* x, double* E) {
    if (check_params(s) || !x || !E) return -1;
    const int N = s->n, P = s->p;
    const double c = 0.5 * s->mass * omega_p2(s);
    double* eint = (double*)malloc(sizeof(double) * (size_t)N);
    if (!eint) return -2;
    oracle_internal_energies(s, x, eint);
    memset(E, 0, sizeof(double) * (size_t)N * (size_t)N);
    for (int v = 1; v <= N; ++v) {
        E[(size_t)(v - 1) * N + (v - 1)] = eint[v - 1] + c * sqdist_beads(s, x, P, v, 1, v);
        for (int u = v - 1; u >= 1; --u) {
            double prev = E[(size_t)u * N + (v - 1)]; /* E^{[u+1,v]} */
            E[(size_t)(u - 1) * N + (v - 1)] = prev
                - c * sqdist_beads(s, x, P, v, 1, u + 1)
                + c * sqdist_beads(s, x, P, u, 1, u + 1)
                + c * sqdist_beads(s, x, P, v, 1, u)
                + eint[u - 1];
        }
    }
    free(eint);
    return 0;
}

/* ------------------------------------------------------ exchange potentials */

/* Eq. 6 for every n (V^{[1,0]} = 0):
 * exp(-beta V^{[1,n]}) = (1/n) sum_{k=1}^{n} xi^{k-1} exp(-beta (E^{[n-k+1,n]} + V^{[1,n-k]})).
 * Returns X[n] = beta V^{[1,n]}.                                            */
int oracle_forward_potentials(const oracle_params* s, const double* E, double* X) {
    if (check_params(s) || !E || !X) return -1;
    const int N = s->n;
    double* t = (double*)malloc(sizeof(double) * (size_t)N);
    if (!t) return -2;
    X[0] = 0.0;
    for (int n = 1; n <= N; ++n) {
        for (int k = 1; k <= n; ++k) {
            double e = E[(size_t)(n - k) * N + (n - 1)]; /* E^{[n-k+1,n]} */
            t[k - 1] = crosses(s, n - k + 1, n) ? -INFINITY
                                                : log_xi_pow(s->xi, k - 1) - (s->beta * e + X[n - k]);
        }
        X[n] = log(local_index(s, n)) - log_sum_exp(t, n);
    }
    free(t);
    return 0;
}

/* Eq. 11, with the empty suffix V^{[N+1,N]} = 0:
 * exp(-beta V^{[u,N]}) = sum_{l=u}^{N} xi^{l-u} (1/l) exp(-beta (E^{[u,l]} + V^{[l+1,N]})).
 * Returns Y[u] = beta V^{[u,N]} for u = 1..N and Y[N+1] = 0.                 */
int oracle_backward_potentials(const oracle_params* s, const double* E, double* Y) {
    if (check_params(s) || !E || !Y) return -1;
    const int N = s->n;
    double* t = (double*)malloc(sizeof(double) * (size_t)N);
    if (!t) return -2;
    Y[0] = 0.0;
    Y[N + 1] = 0.0;
    for (int u = N; u >= 1; --u) {
        int cnt = 0;
        for (int l = u; l <= N; ++l) {
            double e = E[(size_t)(u - 1) * N + (l - 1)]; /* E^{[u,l]} */
            t[cnt++] = crosses(s, u, l) ? -INFINITY
                                        : log_xi_pow(s->xi, l - u) - log(local_index(s, l)) - (s->beta * e + Y[l + 1]);
        }
        Y[u] = -log_sum_exp(t, cnt);
    }
    free(t);
    return 0;
}

/* Eqs. 12-14 for xi >= 0:
 *   l' <= l :  Pr = xi^{l-l'} (1/l) exp(-beta (V^{[1,l'-1]} + E^{[l',l]} + V^{[l+1,N]})) / exp(-beta V^{[1,N]})
 *   l' = l+1:  Pr = 1 - exp(-beta (V^{[1,l]} + V^{[l+1,N]})) / exp(-beta V^{[1,N]})
 *   otherwise: Pr = 0.                                                       */
int oracle_connection_probabilities(const oracle_params* s, const double* E,
                                    const double* X, const double* Y, double* G) {
    if (check_params(s) || !E || !X || !Y || !G) return -1;
    const int N = s->n;
    const double XN = X[N];
    for (int l = 1; l <= N; ++l) {
        for (int lp = 1; lp <= N; ++lp) {
            double pr = 0.0;
            if (lp <= l) {
                if (!crosses(s, lp, l)) {
                    double e = E[(size_t)(lp - 1) * N + (l - 1)]; /* E^{[l',l]} */
                    double lw = log_xi_pow(s->xi, l - lp) - log(local_index(s, l));
                    pr = exp(lw - (X[lp - 1] + s->beta * e + Y[l + 1]) + XN);
                }
            } else if (lp == l + 1 && !crosses(s, l, l + 1)) {
                pr = 1.0 - exp(-(X[l] + Y[l + 1]) + XN);
            }
            G[(size_t)(l - 1) * N + (lp - 1)] = pr;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ forces */

/* Eqs. 15-17 with m omega_P^2 = kappa:
 *   bead 1 : -sum_{l'} Pr[G(l')=l] kappa (2 r_l^1 - r_l^2 - r_{l'}^P)
 *   bead P : -sum_{l'} Pr[G(l)=l'] kappa (2 r_l^P - r_l^{P-1} - r_{l'}^1)
 *   bead j : -kappa (2 r_l^j - r_l^{j+1} - r_l^{j-1}),  j = 2..P-1          */
int oracle_exchange_forces(const oracle_params* s, const double* x, const double* G, double* f) {
    if (check_params(s) || !x || !G || !f) return -1;
    const int N = s->n, P = s->p;
    const double kappa = s->mass * omega_p2(s);
    for (int a = 0; a < s->dim; ++a) {
        for (int l = 1; l <= N; ++l) {
            double f1 = 0.0, fP = 0.0;
            for (int lp = 1; lp <= N; ++lp) {
                double g_in = G[(size_t)(lp - 1) * N + (l - 1)];  /* Pr[G(l')=l] */
                double g_out = G[(size_t)(l - 1) * N + (lp - 1)]; /* Pr[G(l)=l'] */
                f1 -= g_in * kappa * (2.0 * R(x, a, 1, l) - R(x, a, 2, l) - R(x, a, P, lp));
                fP -= g_out * kappa * (2.0 * R(x, a, P, l) - R(x, a, P - 1, l) - R(x, a, 1, lp));
            }
            R(f, a, 1, l) = f1;
            R(f, a, P, l) = fP;
            for (int j = 2; j <= P - 1; ++j)
                R(f, a, j, l) = -kappa * (2.0 * R(x, a, j, l) - R(x, a, j + 1, l) - R(x, a, j - 1, l));
        }
    }
    return 0;
}

/* Eq. 5 with the slice potential of Eqs. 19-20:
 * V(r_1..r_N) = sum_l (1/2) m omega^2 |r_l|^2 + sum_{l<l'} A exp(-|r_l - r_l'|^2 / s^2)
 * (each unordered pair once, i.e. (1/2) sum_{i != j}).  The weight carries U/P
 * (Eq. 4), so the force is -(1/P) grad U.                                     */
int oracle_interaction(const oracle_params* s, const double* x, double* f,
                       double* u_trap, double* u_pair, double* virial) {
    if (check_params(s) || !x || !f) return -1;
    const int N = s->n, P = s->p, D = s->dim;
    const double mw2 = s->mass * s->omega * s->omega;
    const double A = s->pair_amp;
    const double inv_s2 = (A > 0) ? 1.0 / (s->pair_width * s->pair_width) : 0.0;
    ksum ut = {0, 0}, up = {0, 0}, vir = {0, 0};
    double* g = (double*)malloc(sizeof(double) * (size_t)N * (size_t)D); /* grad U_j for one slice */
    if (!g) return -2;
    for (int j = 1; j <= P; ++j) {
        memset(g, 0, sizeof(double) * (size_t)N * (size_t)D);
        for (int l = 1; l <= N; ++l) {
            double r2 = 0.0;
            for (int a = 0; a < D; ++a) {
                double r = R(x, a, j, l);
                r2 += r * r;
                g[(size_t)(l - 1) * D + a] += mw2 * r;
            }
            ks_add(&ut, 0.5 * mw2 * r2);
        }
        if (A > 0) {
            for (int l = 1; l <= N; ++l) {
                for (int lp = l + 1; lp <= N; ++lp) {
                    double d2 = sqdist_beads(s, x, j, l, j, lp);
                    double u = A * exp(-d2 * inv_s2);
                    ks_add(&up, u);
                    for (int a = 0; a < D; ++a) {
                        double d = R(x, a, j, l) - R(x, a, j, lp);
                        /* d/dr_l of A exp(-|r_l - r_l'|^2/s^2) = -2 u (r_l - r_l')/s^2 */
                        g[(size_t)(l - 1) * D + a] += -2.0 * u * d * inv_s2;
                        g[(size_t)(lp - 1) * D + a] -= -2.0 * u * d * inv_s2;
                    }
                }
            }
        }
        /* virial part of this slice: 1/2 sum_l r_l . grad_l U_j */
        for (int l = 1; l <= N; ++l)
            for (int a = 0; a < D; ++a) {
                double gr = g[(size_t)(l - 1) * D + a];
                ks_add(&vir, 0.5 * R(x, a, j, l) * gr);
                R(f, a, j, l) = -gr / (double)P;
            }
    }
    free(g);
    double UT = ks_val(&ut), UP = ks_val(&up);
    if (u_trap) *u_trap = UT;
    if (u_pair) *u_pair = UP;
    if (virial) *virial = UT + UP + ks_val(&vir);
    return 0;
}

int oracle_compute_forces(const oracle_params* s, const double* x, double* f,
                          oracle_energies* e, double* X_out, double* Y_out, double* G_out) {
    if (check_params(s) || !x || !f) return -1;
    const int N = s->n, P = s->p, D = s->dim;
    const size_t nd = (size_t)D * P * N;
    double* E = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* X = (double*)malloc(sizeof(double) * (size_t)(N + 1));
    double* Y = (double*)malloc(sizeof(double) * (size_t)(N + 2));
    double* G = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* fu = (double*)malloc(sizeof(double) * nd);
    int rc = -2;
    if (!E || !X || !Y || !G || !fu) goto done;
    /* Sec. III in order: cycle energies, forward and backward potentials,
     * connection probabilities, exchange forces; then the interaction U.     */
    if ((rc = oracle_cycle_energies(s, x, E))) goto done;
    if ((rc = oracle_forward_potentials(s, E, X))) goto done;
    if ((rc = oracle_backward_potentials(s, E, Y))) goto done;
    if ((rc = oracle_connection_probabilities(s, E, X, Y, G))) goto done;
    if ((rc = oracle_exchange_forces(s, x, G, f))) goto done;
    double ut, up, vir;
    if ((rc = oracle_interaction(s, x, fu, &ut, &up, &vir))) goto done;
    for (size_t i = 0; i < nd; ++i) f[i] += fu[i];
    if (e) {
        ksum S = {0, 0};
        for (int l = 1; l <= N; ++l)
            for (int lp = 1; lp <= l; ++lp)
                ks_add(&S, G[(size_t)(l - 1) * N + (lp - 1)] * E[(size_t)(lp - 1) * N + (l - 1)]);
        e->v_exch = X[N] / s->beta;
        e->u_trap = ut;
        e->u_pair = up;
        e->spring_expect = ks_val(&S);
        e->virial = vir;
        /* primitive: -d ln Z / d beta with beta V_xi differentiated at fixed R
         * (beta E^{[u,v]} scales as 1/beta) and the prefactor of Eq. 4.      */
        e->e_prim = (double)D * N * P / (2.0 * s->beta) - e->spring_expect + (ut + up) / (double)P;
        /* origin virial: beta V_xi(sqrt(beta) X) is beta-independent, so
         * -d ln Z/d beta = < U/P + (1/2P) R . grad U >.                        */
        e->e_vir = vir / (double)P;
    }
    if (X_out) memcpy(X_out, X, sizeof(double) * (size_t)(N + 1));
    if (Y_out) memcpy(Y_out, Y, sizeof(double) * (size_t)(N + 2));
    if (G_out) memcpy(G_out, G, sizeof(double) * (size_t)N * N);
    rc = 0;
done:
    free(E); free(X); free(Y); free(G); free(fu);
    return rc;
}

/* -------------------------------------------------------------- integrator */

static int check_md(const oracle_md* md) {
    if (!md || !(md->dt > 0) || md->nhc_len < 0 || md->nhc_len > 16) return -1;
    if (md->sy_order != 1 && md->sy_order != 3 && md->sy_order != 5) return -1;
    return 0;
}
static double bead_mass(const oracle_params* s, const oracle_md* md) {
    return md->bead_mass > 0 ? md->bead_mass : s->mass;
}
static double nhc_mass(const oracle_params* s, const oracle_md* md) {
    return md->nhc_q > 0 ? md->nhc_q : 1.0 / (s->beta * omega_p2(s));
}
/* Suzuki-Yoshida weights of order 1, 3, 5. */
static int sy_weights(int order, double* w) {
    if (order == 1) { w[0] = 1.0; return 1; }
    if (order == 3) {
        double a = 1.0 / (2.0 - cbrt(2.0));
        w[0] = a; w[1] = 1.0 - 2.0 * a; w[2] = a;
        return 3;
    }
    double a = 1.0 / (4.0 - pow(4.0, 1.0 / 3.0));
    w[0] = a; w[1] = a; w[2] = 1.0 - 4.0 * a; w[3] = a; w[4] = a;
    return 5;
}

/* Propagate one degree of freedom's chain for a time tau (= dt/2) under the
 * chain Liouvillian, Trotter-split with Suzuki-Yoshida weights (one
 * multiple-time-step cycle).  Chain variables: positions eta[k], velocities
 * v[k] = p_eta_k / Q, thermostat masses Q, target kT = 1/beta.
 * Forces on the chain:  G_1 = (p^2/m' - kT)/Q,  G_k = (Q v_{k-1}^2 - kT)/Q.   */
static void nhc_propagate(double* p, double mp, double* eta, double* v, int M,
                          double Q, double kT, double tau, const double* w, int nw) {
    for (int iw = 0; iw < nw; ++iw) {
        const double h = w[iw] * tau;
        /* inward sweep: last chain element first */
        {
            double Gm = (M == 1) ? ((*p) * (*p) / mp - kT) / Q : (Q * v[M - 2] * v[M - 2] - kT) / Q;
            v[M - 1] += 0.5 * h * Gm;
        }
        for (int k = M - 2; k >= 0; --k) {
            double sc = exp(-0.25 * h * v[k + 1]);
            double Gk = (k == 0) ? ((*p) * (*p) / mp - kT) / Q : (Q * v[k - 1] * v[k - 1] - kT) / Q;
            v[k] = (v[k] * sc + 0.5 * h * Gk) * sc;
        }
        /* scale the particle momentum and advance the chain positions */
        *p *= exp(-h * v[0]);
        for (int k = 0; k < M; ++k) eta[k] += h * v[k];
        /* outward sweep */
        for (int k = 0; k <= M - 2; ++k) {
            double sc = exp(-0.25 * h * v[k + 1]);
            double Gk = (k == 0) ? ((*p) * (*p) / mp - kT) / Q : (Q * v[k - 1] * v[k - 1] - kT) / Q;
            v[k] = (v[k] * sc + 0.5 * h * Gk) * sc;
        }
        {
            double Gm = (M == 1) ? ((*p) * (*p) / mp - kT) / Q : (Q * v[M - 2] * v[M - 2] - kT) / Q;
            v[M - 1] += 0.5 * h * Gm;
        }
    }
}

static void nhc_half_step(const oracle_params* s, const oracle_md* md, double* p,
                          double* eta, double* veta, size_t nd) {
    const int M = md->nhc_len;
    if (M == 0) return;
    double w[5];
    int nw = sy_weights(md->sy_order, w);
    const double mp = bead_mass(s, md), Q = nhc_mass(s, md), kT = 1.0 / s->beta;
    double e[16], v[16];
    for (size_t i = 0; i < nd; ++i) {
        for (int k = 0; k < M; ++k) { e[k] = eta[(size_t)k * nd + i]; v[k] = veta[(size_t)k * nd + i]; }
        nhc_propagate(&p[i], mp, e, v, M, Q, kT, 0.5 * md->dt, w, nw);
        for (int k = 0; k < M; ++k) { eta[(size_t)k * nd + i] = e[k]; veta[(size_t)k * nd + i] = v[k]; }
    }
}

/* Velocity Verlet with the thermostat half-steps outside the force update:
 * NHC(dt/2), p += f dt/2, x += p dt/m', f = F(x), p += f dt/2, NHC(dt/2).   */
int oracle_step(const oracle_params* s, const oracle_md* md, double* x, double* p,
                double* eta, double* veta, double* f, int64_t n_steps) {
    if (check_params(s) || check_md(md) || !x || !p || !f) return -1;
    if (md->nhc_len > 0 && (!eta || !veta)) return -1;
    const size_t nd = (size_t)s->dim * s->p * s->n;
    const double mp = bead_mass(s, md), dt = md->dt;
    for (int64_t it = 0; it < n_steps; ++it) {
        nhc_half_step(s, md, p, eta, veta, nd);
        for (size_t i = 0; i < nd; ++i) p[i] += 0.5 * dt * f[i];
        for (size_t i = 0; i < nd; ++i) x[i] += dt * p[i] / mp;
        int rc = oracle_compute_forces(s, x, f, NULL, NULL, NULL, NULL);
        if (rc) return rc;
        for (size_t i = 0; i < nd; ++i) p[i] += 0.5 * dt * f[i];
        nhc_half_step(s, md, p, eta, veta, nd);
    }
    return 0;
}

double oracle_conserved(const oracle_params* s, const oracle_md* md, const double* x,
                        const double* p, const double* eta, const double* veta) {
    if (check_params(s) || check_md(md) || !x || !p) return NAN;
    const size_t nd = (size_t)s->dim * s->p * s->n;
    const double mp = bead_mass(s, md), Q = nhc_mass(s, md), kT = 1.0 / s->beta;
    oracle_energies e;
    double* f = (double*)malloc(sizeof(double) * nd);
    if (!f) return NAN;
    int rc = oracle_compute_forces(s, x, f, &e, NULL, NULL, NULL);
    free(f);
    if (rc) return NAN;
    ksum h = {0, 0};
    for (size_t i = 0; i < nd; ++i) ks_add(&h, 0.5 * p[i] * p[i] / mp);
    ks_add(&h, e.v_exch);
    ks_add(&h, (e.u_trap + e.u_pair) / (double)s->p);
    for (int k = 0; k < md->nhc_len; ++k)
        for (size_t i = 0; i < nd; ++i) {
            double v = veta[(size_t)k * nd + i];
            ks_add(&h, 0.5 * Q * v * v + kT * eta[(size_t)k * nd + i]);
        }
    return ks_val(&h);
}

int oracle_density(const oracle_params* s, const double* x, int bins, double rmax, uint64_t* counts) {
    if (check_params(s) || !x || !counts || bins < 1 || !(rmax > 0)) return -1;
    const int N = s->n, P = s->p;
    for (int j = 1; j <= P; ++j)
        for (int l = 1; l <= N; ++l) {
            double r2 = 0.0;
            for (int a = 0; a < s->dim; ++a) r2 += R(x, a, j, l) * R(x, a, j, l);
            double r = sqrt(r2);
            int b = (r >= rmax) ? bins : (int)(r / rmax * bins);
            if (b > bins) b = bins;
            counts[b] += 1;
        }
    return 0;
}

/* ------------------------------------------------------------ exact energy */

/* Non-interacting particles in an isotropic trap, hbar = m = omega = 1.
 * A k-cycle of the permutation sum of Eq. 2 is one harmonic ring of k*P beads
 * at imaginary-time step beta/P; its partition function is z(k B) with
 * z(B) = (2 sinh(B/2))^{-d} and B = P arccosh(1 + beta^2/(2 P^2)) (the
 * continuum has B = beta).  The canonical sum over permutations obeys
 * Z_n = (1/n) sum_k xi^{k-1} z(k B) Z_{n-k}, Z_0 = 1, and the energy is
 * E = -d ln Z_N/d beta = E_B(B) dB/dbeta with E_B = -d ln Z_N/dB.         */
double oracle_exact_energy(int n, int dim, double beta, int p, double xi) {
    if (n < 1 || dim < 1 || !(beta > 0) || p < 0 || !(xi >= 0)) return NAN;
    double B = beta, dB = 1.0;
    if (p > 0) {
        double a = 1.0 + beta * beta / (2.0 * (double)p * p);
        B = (double)p * acosh(a);
        dB = (beta / (double)p) / sqrt(a * a - 1.0);
    }
    /* lnZ[m] and EB[m] = -d lnZ_m/dB for m = 0..n. */
    double* lnZ = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* EB = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    if (!lnZ || !EB || !t) { free(lnZ); free(EB); free(t); return NAN; }
    lnZ[0] = 0.0; EB[0] = 0.0;
    for (int m = 1; m <= n; ++m) {
        for (int k = 1; k <= m; ++k) {
            double kb = (double)k * B;
            /* ln z(kB) = -d ln(2 sinh(kB/2)) = -d (kB/2 + ln(1 - e^{-kB})) */
            double lnz = -(double)dim * (0.5 * kb + log1p(-exp(-kb)));
            t[k - 1] = log_xi_pow(xi, k - 1) + lnz + lnZ[m - k];
        }
        double lse = log_sum_exp(t, m);
        lnZ[m] = lse - log((double)m);
        double e = 0.0;
        for (int k = 1; k <= m; ++k) {
            if (t[k - 1] == -INFINITY) continue;
            double kb = (double)k * B;
            /* -d ln z(kB)/dB = (d k/2) coth(kB/2) */
            double eps = 0.5 * (double)dim * (double)k / tanh(0.5 * kb);
            e += exp(t[k - 1] - lse) * (eps + EB[m - k]);
        }
        EB[m] = e;
    }
    double out = EB[n] * dB;
    free(lnZ); free(EB); free(t);
    return out;
}

/* Linear-domain form of the same recursion for any real xi.  With
 * zt(k) = z(kB) e^{d k B/2} = (1 - e^{-kB})^{-d} and Z_m = e^{-d m B/2} Zt_m:
 *   Zt_m  = (1/m) sum_k xi^{k-1} zt(k) Zt_{m-k},            Zt_0 = 1,
 *   Zt'_m = (1/m) sum_k xi^{k-1} (zt'(k) Zt_{m-k} + zt(k) Zt'_{m-k}),
 *   zt'(k) = d zt/dB = -d k e^{-kB} (1 - e^{-kB})^{-d-1},
 * and -d ln Z_n/dB = d n/2 - Zt'_n/Zt_n; E = (-d ln Z_n/dB) dB/dbeta.          */
double oracle_exact_energy_signed(int n, int dim, double beta, int p, double xi) {
    if (n < 1 || dim < 1 || !(beta > 0) || p < 0 || !isfinite(xi)) return NAN;
    double B = beta, dB = 1.0;
    if (p > 0) {
        double a = 1.0 + beta * beta / (2.0 * (double)p * p);
        B = (double)p * acosh(a);
        dB = (beta / (double)p) / sqrt(a * a - 1.0);
    }
    double* Z = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* dZ = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    if (!Z || !dZ) { free(Z); free(dZ); return NAN; }
    Z[0] = 1.0; dZ[0] = 0.0;
    for (int m = 1; m <= n; ++m) {
        double s = 0.0, ds = 0.0, xk = 1.0;   /* xk = xi^{k-1} */
        for (int k = 1; k <= m; ++k) {
            double q = exp(-(double)k * B);
            double zt = pow(1.0 - q, -(double)dim);
            double dzt = -(double)dim * (double)k * q * pow(1.0 - q, -(double)dim - 1.0);
            s += xk * zt * Z[m - k];
            ds += xk * (dzt * Z[m - k] + zt * dZ[m - k]);
            xk *= xi;
        }
        Z[m] = s / (double)m;
        dZ[m] = ds / (double)m;
    }
    double EB = 0.5 * (double)dim * (double)n - dZ[n] / Z[n];
    free(Z); free(dZ);
    return EB * dB;
}

/* ------------------------------------------------------------------ seeded initial state */

/* One Philox round on (c0, c1, c2, c3) with round key (k0, k1): the products
 * M0 c0 and M1 c2 are split into high and low words, and
 * (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53 random bits from two words, centred in (0, 1). */
static double unit_open(uint32_t hi, uint32_t lo) {
    uint64_t m = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
    return ((double)m + 0.5) * 0x1p-53;
}

/* Deviate e of array a (Box and Muller, Ann. Math. Stat. 29, 610 (1958)). */
static double normal_deviate(uint64_t seed, uint32_t a, uint64_t e) {
    uint64_t k = e >> 1;
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), a, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    double u1 = unit_open(w[1], w[0]);
    double u2 = unit_open(w[3], w[2]);
    double rad = sqrt(-2.0 * log(u1));
    double th = 6.283185307179586476925286766559 * u2;   /* 2 pi u2 */
    return (e & 1) ? rad * sin(th) : rad * cos(th);
}

int oracle_init_state(const oracle_params* s, const oracle_md* md, double sigma, uint64_t seed,
                      double* x, double* p) {
    if (check_params(s) || !md || !(sigma >= 0) || !x || !p) return -1;
    const double mp = md->bead_mass > 0 ? md->bead_mass : s->mass;
    const double sp = sqrt(mp / s->beta);
    const uint64_t n = (uint64_t)s->dim * (uint64_t)s->p * (uint64_t)s->n;
    for (uint64_t e = 0; e < n; ++e) {
        x[e] = sigma * normal_deviate(seed, 0u, e);
        p[e] = sp * normal_deviate(seed, 1u, e);
    }
    return 0;
}
