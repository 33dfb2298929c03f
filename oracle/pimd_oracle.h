/*
 * pimd_oracle.h -- plain CPU FP64 oracle for one force-and-energy step of
 * bosonic / fictitious-particle path integral molecular dynamics.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the method as the paper states it (Y. Xiong, "GPU acceleration of
 * ab initio simulations of large-scale identical particles based on path
 * integral molecular dynamics", arXiv:2404.02628).  Only the test-suite, the
 * smoke entry point and the CPU-baseline leg of the benchmark may load it.
 * It shares no source, header, table or helper with the GPU library.
 *
 * Every routine is plain double precision, sequential, and follows the
 * paper's equations in their order (Sec. II and III, Eqs. 4-17), so that it
 * can be checked against the paper by eye.
 *
 * Coordinates are stored "[dim][P][N]":  x[(a*P + j)*N + l] is component a of
 * bead j (0-based, the paper's j+1) of particle l (0-based, the paper's l+1).
 * Forces and momenta use the same layout.
 *
 * All functions return 0 on success and a negative value on invalid input.
 */
#ifndef PIMD_ORACLE_H
#define PIMD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n;          /* number of particles N >= 1                              */
    int32_t p;          /* beads per ring polymer P >= 2                           */
    int32_t dim;        /* spatial dimensions d in 1..3                            */
    double beta;        /* 1/(k_B T) > 0                                           */
    double hbar;        /* > 0                                                     */
    double mass;        /* particle mass m > 0                                     */
    double omega;       /* harmonic trap frequency (>= 0)                          */
    double xi;          /* exchange parameter, 0 <= xi <= 1 (Sec. II, Eq. 2)       */
    double pair_amp;    /* Gaussian pair amplitude A >= 0 (Eq. 20 with A = g/(pi s^2) or A = g) */
    double pair_width;  /* Gaussian width s > 0                                    */
    int32_t n2;         /* particles of a second species (the last n2; 0 = one species,
                           0 <= n2 < n): exchange cycles stay within a species, the
                           1/n factors of Eqs. 6, 11, 12 count within the species, and the
                           pair and trap terms act on all particles                 */
} oracle_params;

typedef struct {
    double v_exch;        /* V_xi^{[1,N]}  (Eq. 6 at n = N)                                   */
    double u_trap;        /* sum over slices of the trap energy  (part of U, Eq. 5)             */
    double u_pair;        /* sum over slices of the pair energy  (part of U, Eq. 5)             */
    double spring_expect; /* S = sum_{l'<=l} Pr[l->l'] E^{[l',l]}                                */
    double virial;        /* sum_j [ U_j + 1/2 sum_l r_l^j . grad U_j ]                          */
    double e_prim;        /* primitive estimator  d N P/(2 beta) - S + U/P                       */
    double e_vir;         /* virial estimator     virial / P                                     */
} oracle_energies;

typedef struct {
    double dt;          /* MD time step                                              */
    int32_t nhc_len;    /* Nose-Hoover chain length M (0 = plain velocity Verlet)    */
    double nhc_q;       /* thermostat mass Q; <= 0 selects 1/(beta omega_P^2)        */
    int32_t sy_order;   /* Suzuki-Yoshida order: 1, 3 or 5                           */
    double bead_mass;   /* fictitious bead mass m'; <= 0 selects the particle mass  */
} oracle_md;

/* Eq. 7, written for the ring formed by particles u..v (1-based, u <= v):
 * bead P of particle l joins bead 1 of l+1, bead P of v joins bead 1 of u.   */
double oracle_ring_energy(const oracle_params* s, const double* x, int u, int v);

/* Eq. 9: E_int^{(v)} for v = 1..N, written to eint[v-1].                       */
int oracle_internal_energies(const oracle_params* s, const double* x, double* eint);

/* Eqs. 8-10: E^{[u,v]} for 1 <= u <= v <= N, written to E[(u-1)*N + (v-1)]
 * (entries with u > v are set to 0).                                          */
int oracle_cycle_energies(const oracle_params* s, const double* x, double* E);

/* Eq. 6 applied for every n = 1..N:  X[n] = beta V^{[1,n]},  X[0] = 0.          */
int oracle_forward_potentials(const oracle_params* s, const double* E, double* X);

/* Eq. 11:  Y[u] = beta V^{[u,N]} for u = 1..N,  Y[N+1] = 0  (array of N+2;
 * Y[0] is unused and set to 0).                                                */
int oracle_backward_potentials(const oracle_params* s, const double* E, double* Y);

/* Eqs. 12-14: G[(l-1)*N + (l'-1)] = Pr[G(l) = l'] for l, l' = 1..N.           */
int oracle_connection_probabilities(const oracle_params* s, const double* E,
                                    const double* X, const double* Y, double* G);

/* Eqs. 15-17: f = -grad V_xi^{[1,N]} on every bead (overwrites f).            */
int oracle_exchange_forces(const oracle_params* s, const double* x, const double* G, double* f);

/* Eqs. 5, 19, 20: f = -(1/P) grad U (overwrites f); the trap and pair parts of
 * U summed over slices; virial = sum_j [U_j + 1/2 sum_l r.grad U_j].            */
int oracle_interaction(const oracle_params* s, const double* x, double* f,
                       double* u_trap, double* u_pair, double* virial);

/* Whole force-and-energy evaluation: f = -grad (V_xi + U/P), energies.  The
 * optional out-arrays (may be NULL) receive X (N+1), Y (N+2) and G (N*N).     */
int oracle_compute_forces(const oracle_params* s, const double* x, double* f,
                          oracle_energies* e, double* X_out, double* Y_out, double* G_out);

/* n_steps of velocity Verlet with massive Nose-Hoover chains.  x, p, f have
 * d*P*N entries; eta and veta have nhc_len*d*P*N entries ([k][dof]); f must hold
 * the forces at the incoming x and holds the forces at the outgoing x.       */
int oracle_step(const oracle_params* s, const oracle_md* md, double* x, double* p,
                double* eta, double* veta, double* f, int64_t n_steps);

/* Conserved quantity of the thermostatted dynamics:
 * sum p^2/(2m') + V_xi + U/P + sum_dof sum_k (Q veta_k^2/2 + eta_k/beta).     */
double oracle_conserved(const oracle_params* s, const oracle_md* md, const double* x,
                        const double* p, const double* eta, const double* veta);

/* Radial histogram of |r_l^j| over all N*P beads: bins of width rmax/bins,
 * counts[bins] collects r >= rmax.  Counts are added to (not overwritten).   */
int oracle_density(const oracle_params* s, const double* x, int bins, double rmax, uint64_t* counts);

/* Exact canonical energy of N non-interacting particles with exchange
 * parameter xi in a d-dimensional isotropic harmonic trap (hbar = m = omega = 1),
 * for the P-bead discretisation (p >= 1) or the continuum (p = 0).           */
double oracle_exact_energy(int n, int dim, double beta, int p, double xi);

/* The same energy for any real xi, fermions (xi = -1) included, from the cycle
 * recursion of the partition function written in the linear domain with signed
 * terms: Z_m = (1/m) sum_k xi^{k-1} z(kB) Z_{m-k}.  The factors z(kB) are scaled
 * by e^{d k B / 2} so that every term is O(1); intended for small n (the
 * alternating sums of xi < 0 cancel increasingly with n).                    */
double oracle_exact_energy_signed(int n, int dim, double beta, int p, double xi);

/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC11): ten rounds of two 32x32->64
 * multiplications (multipliers 0xD2511F53, 0xCD9E8D57) on the counter, with the
 * key bumped by the Weyl constants 0x9E3779B9, 0xBB67AE85 between rounds.      */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Seeded initial state: x iid N(0, sigma^2) and p iid N(0, m'/beta) per coordinate
 * (Maxwell-Boltzmann at beta for the bead mass m' of md).  Element e of array a
 * (a = 0 positions, a = 1 momenta; e in the [dim][P][N] order) is deviate e mod 2
 * of the Box-Muller pair k = e/2: Philox4x32-10 with counter {k mod 2^32,
 * k / 2^32, a, 0} and key {seed mod 2^32, seed / 2^32} gives words w0..w3;
 * u1 = ((w1 * 2^21 + w0 / 2^11) + 1/2) 2^-53, u2 likewise from w3, w2;
 * deviates sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2).          */
int oracle_init_state(const oracle_params* s, const oracle_md* md, double sigma, uint64_t seed,
                      double* x, double* p);

#ifdef __cplusplus
}
#endif
#endif
