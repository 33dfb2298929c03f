/*
 * pimd.h -- C ABI of libpimd, an MI355X (gfx950) library for bosonic and
 * fictitious-particle path integral molecular dynamics (PIMD).
 *
 * Method: Y. Xiong, "GPU acceleration of ab initio simulations of large-scale
 * identical particles based on path integral molecular dynamics",
 * arXiv:2404.02628.  N identical particles, each a ring polymer of P beads in
 * d dimensions, sampled with weight exp(-beta (V_xi^{[1,N]} + U/P)) (Sec. II,
 * Eq. 4).  U is the trap plus Gaussian pair energy of every imaginary-time
 * slice (Eqs. 5, 19, 20); V_xi^{[1,N]} is the exchange potential of Eq. 6,
 * built from the cycle spring energies of Eqs. 7-10; its gradient comes from
 * the backward potentials and connection probabilities of Eqs. 11-17.  The
 * exchange parameter xi is 1 for bosons, 0 for distinguishable particles and
 * in (0,1) for fictitious identical particles (Sec. II).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a pimd_status; nothing throws across the ABI.  On
 *   failure pimd_last_error() returns a thread-local, library-owned message
 *   that stays valid until the next call on the same thread.
 * - Coordinates, momenta and forces of one replica are double arrays in the
 *   layout [dim][P][N]: element ((a*P + j)*N + l) is component a of bead j
 *   (0-based) of particle l (0-based).
 * - Device memory: the caller allocates ONE device workspace of
 *   pimd_workspace_bytes() bytes (for example a torch uint8 CUDA tensor) and
 *   passes it to pimd_create; the library never allocates device memory.
 *   The workspace and the stream are borrowed: they must outlive the context.
 * - Streams: work is enqueued on the caller's HIP stream (hipStream_t passed
 *   as void*; NULL selects the default stream).  pimd_compute_forces and
 *   pimd_step only enqueue; getters that return data synchronise the stream.
 * - A context is not thread-safe.  Contexts are independent of each other.
 * - Arguments that are invalid (bad sizes, NULL where not allowed, replica
 *   index out of range, parameters outside their domain) give
 *   PIMD_ERR_INVALID and leave the context unchanged.  HIP runtime failures
 *   give PIMD_ERR_DEVICE.
 * - Failures inside enqueued work are recorded on the device and reported by
 *   the next call that synchronises (pimd_synchronize, pimd_get_state,
 *   pimd_get_forces, pimd_energies, pimd_trace, pimd_density), after that call
 *   has written its outputs:
 *     PIMD_ERR_NONFINITE  a force, momentum or position of some replica became
 *                         non-finite; pimd_last_error() names the lowest such
 *                         replica;
 *     PIMD_ERR_DEVICE     a wait of the cooperative recursion schedule timed
 *                         out (pimd_config.recursion_workgroups).
 *   Either halts the run on the device from the pass that detected it on: the
 *   integrator, the estimators, the trace and the density histogram stop
 *   writing, so the state stays at the step where the failure appeared.  Once
 *   a call has reported it, pimd_step and pimd_compute_forces return
 *   PIMD_ERR_STATE until pimd_set_state or pimd_init_system restarts the run.
 */
#ifndef PIMD_H
#define PIMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIMD_ABI_VERSION 8

typedef enum {
    PIMD_OK = 0,
    PIMD_ERR_INVALID = -1,    /* invalid argument; nothing changed                         */
    PIMD_ERR_DEVICE = -2,     /* HIP runtime error (message in pimd_last_error)            */
    PIMD_ERR_NONFINITE = -3,  /* a force or energy of some replica is not finite           */
    PIMD_ERR_WORKSPACE = -4,  /* workspace NULL, misaligned (256 B) or smaller than needed */
    PIMD_ERR_STATE = -5       /* call out of order (e.g. energies before any evaluation)   */
} pimd_status;

typedef enum {
    PIMD_FP64 = 0,   /* every quantity in double precision                                   */
    PIMD_MIXED = 1   /* pair distances, Gaussian terms and pair forces in FP32 (a particle's
                        pair force summed in FP32 up to its slice total, then scaled in FP64);
                        springs, recursions, probabilities, thermostat and all other
                        reductions in FP64                                                   */
} pimd_precision;

typedef enum { PIMD_HOST = 0, PIMD_DEVICE = 1 } pimd_mem;

/* pimd_config.flags */
#define PIMD_FLAG_GRAPH 1      /* replay steady MD steps from a captured HIP graph (default: direct launches).
                                  Note: on ROCm 7, once a process has captured and replayed a graph,
                                  every later kernel dispatch of the process costs ~35 us more
                                  (measured on MI355X), contexts without this flag included. */
#define PIMD_FLAG_PAIR_ORDERED 2  /* use the ordered pair kernel even where the symmetric
                                     per-slice kernel would be chosen (at least 256 interacting
                                     slices whose largest one fits the LDS of a compute unit:
                                     N up to 9,024 in 2-D in mixed precision, 4,416 in FP64);
                                     for tuning and testing */
#define PIMD_FLAG_NO_PERSISTENT 4 /* run pimd_step with one launch per kernel and step even when
                                     every replica is small enough (N <= 64 and dim*P*N <= 512)
                                     for the persistent kernel, which otherwise runs whole steps
                                     of every replica (one workgroup each, state on chip) in one
                                     launch per 4096 steps; its pair term is FP64 in both
                                     precision modes; for tuning and testing                 */
#define PIMD_FLAG_LONGEST_FIRST 8 /* dispatch the per-replica work of the pair kernel and of the batched
                                     recursion longest replica first (descending N) instead of in
                                     replica order; a packing choice for batches of uneven N      */
#define PIMD_FLAG_PAIR_SPLIT_1 16 /* waves per 64-particle tile of the ordered pair kernel: the value
                                     (flags & PIMD_FLAG_PAIR_SPLIT_MASK) / PIMD_FLAG_PAIR_SPLIT_1 is
                                     0 (chosen from the work size), 1, 2 or 3 (1, 2 or 4 waves)    */
#define PIMD_FLAG_PAIR_SPLIT_MASK 48
#define PIMD_FLAG_RECURSION_WIDE 64 /* eight wavefronts per workgroup of the one-workgroup-per-replica
                                     recursion schedule instead of four: more parallel work per row
                                     block of the chain, but the whole register file of a compute
                                     unit, so the pair kernel cannot run beside it there; pays when
                                     the chains are the critical path and the pair work is small
                                     (measured: 64 replicas of N ~ U{64..512} +7%, 128 replicas of
                                     N = 1600 -11%); for the autotuner                            */

/* One independent system (replica).  Units are free; the paper uses
 * hbar = m = omega = k_B = 1 (Sec. IV.A). */
typedef struct {
    int32_t n;            /* particles, N >= 1                                               */
    int32_t n2;           /* particles of a second species, 0 <= n2 < n (0: one species).  The
                             last n2 particles form it.  Sec. II treats one spin-polarised
                             species and notes that coexisting spins follow directly: the
                             exchange sum factorises over species, so exchange cycles (Eqs. 6-14)
                             never join particles of different species, each species counts its
                             own 1/n factors, and Pr[n - n2 -> n - n2 + 1] = 0.  The trap and the
                             pair term act on all particles alike.                           */
    double beta;          /* inverse temperature > 0                                         */
    double hbar;          /* > 0                                                             */
    double mass;          /* particle mass m > 0; spring constant m omega_P^2, omega_P = sqrt(P)/(beta hbar) (Sec. III) */
    double omega;         /* trap frequency >= 0: U_trap = (1/2) m omega^2 r^2 per bead (Eq. 19) */
    double xi;            /* exchange parameter, 0 <= xi <= 1 (the probabilities of Eqs. 12-14 need xi >= 0) */
    double pair_amp;      /* Gaussian amplitude A >= 0: A exp(-|r_i - r_j|^2 / s^2) per unordered pair (Eq. 20) */
    double pair_width;    /* s > 0 (ignored when A == 0)                                     */
    double dt;            /* MD time step > 0                                                */
    double nhc_q;         /* thermostat mass Q; <= 0 selects 1/(beta omega_P^2)              */
    double bead_mass;     /* fictitious bead mass m'; <= 0 selects the particle mass         */
} pimd_replica;

typedef struct {
    int32_t n_replicas;      /* >= 1                                                         */
    int32_t p;               /* beads per ring, P >= 2 (Eqs. 15-16 need distinct end beads)  */
    int32_t dim;             /* 1, 2 or 3                                                    */
    int32_t precision;       /* pimd_precision                                               */
    int32_t nhc_len;         /* Nose-Hoover chain length per degree of freedom, 0..8 (0 = NVE) */
    int32_t sy_order;        /* Suzuki-Yoshida order of the thermostat step: 1, 3 or 5       */
    int32_t density_bins;    /* radial density bins >= 1 (one extra overflow bin is kept)    */
    int32_t trace_capacity;  /* energy samples kept per replica (ring buffer), >= 0          */
    int32_t recursion_workgroups; /* schedule of the exchange recursions (Eqs. 6, 11): 0 = chosen
                                from the batch size and the device; 1 = one workgroup per replica
                                and direction; k > 1 = one chain workgroup plus k-1 helpers that
                                pre-sum finished column panels (cooperative launch; reduced to fit
                                the device, or 1 if cooperative launch is unavailable)        */
    int32_t flags;           /* PIMD_FLAG_* bits; all other bits must be 0                   */
    double density_rmax;     /* radius covered by the bins > 0                               */
    const pimd_replica* replicas; /* n_replicas entries, copied by pimd_create              */
} pimd_config;

/* Estimators of one evaluation (Sec. IV reports energies and densities). */
typedef struct {
    double v_exch;         /* V_xi^{[1,N]} (Eq. 6 at n = N)                                     */
    double u_trap;         /* trap part of U = sum_j V(slice j) (Eqs. 5, 19)                    */
    double u_pair;         /* pair part of U (Eq. 20, each unordered pair once)                 */
    double spring_expect;  /* S = sum_{l'<=l} Pr[l->l'] E^{[l',l]}: expected spring energy      */
    double virial;         /* sum_j [U_j + (1/2) sum_l r_l^j . grad U_j]                        */
    double e_prim;         /* primitive estimator d N P/(2 beta) - S + U/P                       */
    double e_vir;          /* origin-virial estimator virial / P                                 */
    double kinetic;        /* sum p^2/(2 m') over all bead coordinates                           */
    double nhc_energy;     /* sum over chains of Q v^2/2 + eta/beta                              */
    double h_conserved;    /* kinetic + V_xi + U/P + nhc_energy: conserved by the dynamics       */
    int64_t step;          /* MD step count at which the values were taken                       */
} pimd_estimates;

typedef struct pimd_ctx pimd_ctx;

/* ABI version of the loaded library (PIMD_ABI_VERSION at build time). */
int pimd_abi_version(void);

/* Message of the last failing call on this thread ("" if none). Library-owned. */
const char* pimd_last_error(void);

/* Bytes of device workspace that pimd_create needs for `cfg` (written to *bytes).
 * Validates cfg like pimd_create.  Errors: PIMD_ERR_INVALID. */
pimd_status pimd_workspace_bytes(const pimd_config* cfg, size_t* bytes);

/* Creates a context on the current HIP device.  d_workspace: device pointer,
 * 256-byte aligned, at least pimd_workspace_bytes(cfg) bytes, owned by the
 * caller.  hip_stream: hipStream_t (or NULL).  Copies cfg and its replicas.
 * All replicas start at x = p = 0 with zeroed thermostats and accumulators.
 * Errors: PIMD_ERR_INVALID, PIMD_ERR_WORKSPACE, PIMD_ERR_DEVICE. */
pimd_status pimd_create(const pimd_config* cfg, void* d_workspace, size_t bytes,
                        void* hip_stream, pimd_ctx** out);

/* Destroys the host-side context (synchronises its stream first).  NULL is a no-op. */
pimd_status pimd_destroy(pimd_ctx* ctx);

/* Seeded initial state of every replica on the device: positions iid
 * N(0, pos_sigma[r]^2) and momenta iid N(0, m'/beta) per coordinate (Maxwell-
 * Boltzmann at beta for the bead mass m'), thermostat chains at rest.  Every
 * element is a pure function of (seeds[r], array, element index): element e of
 * array a (a = 0 positions, a = 1 momenta; [dim][P][N] order) is deviate e mod 2
 * of the Box-Muller pair k = e/2, drawn with the counter-based generator
 * Philox4x32-10 (Salmon et al., SC11) at counter {k mod 2^32, k / 2^32, a, 0}
 * and key {seed mod 2^32, seed / 2^32}: with words w0..w3,
 * u1 = (w1 2^21 + floor(w0 / 2^11) + 1/2) 2^-53, u2 likewise from w3, w2, and the
 * deviates are sqrt(-2 ln u1) cos(2 pi u2), sqrt(-2 ln u1) sin(2 pi u2).
 * pos_sigma and seeds are host arrays of n_replicas entries; pos_sigma[r]
 * must be finite and >= 0.  Invalidates the forces.  Synchronises. */
pimd_status pimd_init_system(pimd_ctx* ctx, const double* pos_sigma, const uint64_t* seeds);

/* Sets positions x and (optionally) momenta p of replica r, layout [dim][P][N].
 * nhc (optional) holds the thermostat state: the chain velocities v_eta as
 * [nhc_len][dim][P][N], followed by ONE double, the sum of all chain positions eta
 * of the replica (over its coordinates and chain elements).  The chain positions
 * never act on the dynamics; they enter only the conserved quantity, through
 * kT times that sum, so the library keeps the sum instead of every eta.  NULL
 * zeroes the thermostat state (p NULL zeroes p).
 * `where` says whether the pointers are host or device memory.  Invalidates the
 * forces of replica r until the next evaluation, and restarts a halted run
 * (a replica that is still non-finite halts it again at the next evaluation).
 * Together with pimd_get_state this is a checkpoint: a context of the same
 * configuration given every replica's x, p and nhc continues the trajectory
 * bit for bit.  Synchronous. */
pimd_status pimd_set_state(pimd_ctx* ctx, int32_t r, const double* x, const double* p,
                           const double* nhc, pimd_mem where);

/* Copies the state of replica r out (any pointer may be NULL; nhc in the layout of
 * pimd_set_state, nhc_len*dim*P*N + 1 doubles).  Synchronous.  The library holds the
 * chain positions' sum as partial sums; reading nhc folds them into the one value
 * returned, so the context and any context restarted from the returned state
 * continue bit for bit alike.
 * Reports a halted run (PIMD_ERR_NONFINITE, PIMD_ERR_DEVICE) after copying. */
pimd_status pimd_get_state(pimd_ctx* ctx, int32_t r, double* x, double* p, double* nhc,
                           pimd_mem where);

/* One force-and-energy evaluation of every replica at its current positions:
 * pair and trap forces (Eqs. 5, 20), cycle energies (Eqs. 7-10), forward and
 * backward exchange potentials (Eqs. 6, 11), connection probabilities (Eqs.
 * 12-14), exchange forces (Eqs. 15-17) and all estimators.  Enqueued only. */
pimd_status pimd_compute_forces(pimd_ctx* ctx);

/* Bytes of the device scratch that pimd_compute_forces_noalloc holds per GPU. */
#define PIMD_NOALLOC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the evaluation of pimd_compute_forces for ONE replica
 * (cfg->n_replicas must be 1), with no context, no workspace and no allocation of any kind.
 *   x    device array, layout [dim][P][N]: the positions (read only);
 *   f    device array, layout [dim][P][N]: receives the total force -grad(V_xi + U/P);
 *   est  device pointer to one pimd_estimates, or NULL: receives the estimators of this
 *        evaluation (kinetic and nhc_energy are 0, h_conserved is V_xi + U/P, step is 0); all
 *        NaN if the device found a non-finite force or a cooperative wait gave up;
 *   hip_stream  hipStream_t (or NULL): every kernel is enqueued on it, nothing synchronises.
 * Everything else lives in a static device array of PIMD_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends (32 MiB: every single-replica workload up
 * to N = 4*10^4 at P = 16, d = 3 fits).  All calls on one GPU share it and it keeps the last
 * call's contents (the call clears what must start at zero): calls that overlap on one GPU race,
 * so serialise them (one stream, or the caller's own ordering).  pimd_config fields that concern
 * dynamics or sampling (nhc_len, sy_order, density, trace) are validated and otherwise ignored;
 * flags and recursion_workgroups choose kernels as for pimd_create.  Errors (returned before
 * anything is enqueued): PIMD_ERR_INVALID (bad cfg, n_replicas != 1, NULL x or f),
 * PIMD_ERR_WORKSPACE (the replica needs more scratch than PIMD_NOALLOC_SCRATCH_BYTES; use
 * pimd_create), PIMD_ERR_DEVICE (HIP launch failure). */
pimd_status pimd_compute_forces_noalloc(const pimd_config* cfg, const double* x, double* f,
                                        pimd_estimates* est, void* hip_stream);

/* Total force -grad(V_xi + U/P) of replica r from the last evaluation, layout
 * [dim][P][N].  Synchronises.  Errors: PIMD_ERR_STATE if never evaluated. */
pimd_status pimd_get_forces(pimd_ctx* ctx, int32_t r, double* f, pimd_mem where);

/* Advances every replica by n_steps velocity-Verlet steps with massive
 * Nose-Hoover chains at k_B T = 1/beta (Sec. IV.A): NHC(dt/2), p += F dt/2,
 * x += p dt/m', F = force(x), p += F dt/2, NHC(dt/2).  The estimators, the
 * density histogram and the trace are taken every `sample_every` steps
 * (0 = never).  The first call evaluates the forces of the initial state.
 * Enqueued only.  Errors: PIMD_ERR_INVALID (n_steps < 0, sample_every < 0),
 * PIMD_ERR_STATE (the run is halted, see the conventions above).
 * When every replica has N <= 64 and dim*P*N <= 512 (and PIMD_FLAG_NO_PERSISTENT
 * is not set) the steps run in the persistent kernel: one launch per 4096 steps,
 * one workgroup per replica with its state on chip, FP64 pair term in both
 * precision modes; PIMD_FLAG_GRAPH has no effect then.  Otherwise:
 * steps that are neither sampled nor the first or last of the call are all the
 * same launch sequence (evaluation plus the fused second/first integrator
 * halves); with PIMD_FLAG_GRAPH (and profiling off) that sequence is captured
 * once into a HIP graph and replayed on the stream.  If the device cannot
 * capture it, the steps run by direct launches (pimd_graph_info).  Replay cuts
 * host launch cost but runs the pair kernel and the recursions one after the
 * other instead of on two streams, so it pays only for small systems. */
pimd_status pimd_step(pimd_ctx* ctx, int64_t n_steps, int32_t sample_every);

/* State of the step graph: *state = 0 not built yet (and stays 0 while the
 * steps run in the persistent kernel), 1 built and replayed,
 * 2 not requested (no PIMD_FLAG_GRAPH), 3 capture failed (direct launches);
 * *replays = steps run by graph replay so far.  Either pointer may be NULL. */
pimd_status pimd_graph_info(pimd_ctx* ctx, int32_t* state, int64_t* replays);

/* Estimators of replica r from its most recent sampled evaluation (every
 * pimd_compute_forces samples).  Synchronises.  Errors: PIMD_ERR_STATE if none
 * yet; PIMD_ERR_NONFINITE if a value is not finite (values still written). */
pimd_status pimd_energies(pimd_ctx* ctx, int32_t r, pimd_estimates* out);

/* Copies up to max_samples most recent trace records of replica r (oldest
 * first) into out (host, pimd_estimates array); *n_samples receives the count
 * written.  Synchronises. */
pimd_status pimd_trace(pimd_ctx* ctx, int32_t r, pimd_estimates* out, int64_t max_samples,
                       int64_t* n_samples);

/* Radial density histogram of replica r over all N*P beads of every sample:
 * counts[b] for |r| in [b, b+1) * rmax/bins, counts[bins] for |r| >= rmax
 * (host array of bins+1).  *n_samples receives the number of samples.  The
 * normalised density of Sec. IV.A is counts / (n_samples N P shell_b).
 * Synchronises. */
pimd_status pimd_density(pimd_ctx* ctx, int32_t r, uint64_t* counts, int64_t* n_samples);

/* Clears the trace and density accumulators of every replica. Enqueued. */
pimd_status pimd_reset_accumulators(pimd_ctx* ctx);

/* Exchange potentials of replica r from the last evaluation (host arrays):
 * X[n] = beta V^{[1,n]} for n = 0..N (Eq. 6, X[0] = 0) and Y[u] = beta V^{[u,N]}
 * for u = 1..N+1 (Eq. 11, Y[N+1] = 0; Y[0] is set to 0).  Synchronises. */
pimd_status pimd_debug_potentials(pimd_ctx* ctx, int32_t r, double* X, double* Y);

/* Dense connection probabilities of replica r (Eqs. 12-14) from the last
 * evaluation: G[(l-1)*N + (l'-1)] = Pr[G(l) = l'] (host array of N*N doubles).
 * Intended for tests at small N; recomputes the entries.  Synchronises. */
pimd_status pimd_debug_probs(pimd_ctx* ctx, int32_t r, double* G);

/* Cycle energies of replica r by their definition (Eq. 7), every entry evaluated
 * on its own from the current positions: E[(u-1)*N + (v-1)] = E^{[u,v]} for
 * u <= v and 0 for u > v (host array of N*N doubles).  This is the O(N^3 P)
 * original algorithm of Sec. III; the force path never forms this table (its
 * recursions regroup E into per-particle terms), so it serves as an
 * independent cross-check and as a cost reference.  If ms is not NULL it
 * receives the summed device time of the kernel launches (HIP events on the
 * context's stream), copies excluded.  PIMD_ERR_STATE before any
 * pimd_set_state or pimd_init_system.  Synchronises. */
pimd_status pimd_cycle_energies(pimd_ctx* ctx, int32_t r, double* E, double* ms);

/* Not an operation of the method: a test hook for the failure path of the cooperative
 * recursion schedule (one chain workgroup plus helper workgroups that hand each other work
 * through device flags).  It raises the device error word, so that every wait of the next
 * evaluation that finds its flag not yet set gives up at once, as a wait that ran out of polls
 * would.  The kernels still run to their end, with invalid results.  The next call that
 * synchronises returns PIMD_ERR_DEVICE, whatever the schedule; the run is then halted (see the conventions above) until pimd_set_state or
 * pimd_init_system lowers the word, after which evaluations are valid again.  Enqueued. */
pimd_status pimd_debug_fail_waits(pimd_ctx* ctx);

/* Per-kernel timing with HIP events on the stream each kernel is launched
 * on.  pimd_profile(ctx, 1) clears and enables, 0 disables.  pimd_kernel_times
 * synchronises and writes, for up to max_kinds kernel kinds, the summed
 * milliseconds and the launch counts; *n_kinds receives the number of kinds.
 * pimd_kernel_name(k) names kind k. */
pimd_status pimd_profile(pimd_ctx* ctx, int enable);
pimd_status pimd_kernel_times(pimd_ctx* ctx, double* ms, int64_t* launches, int32_t max_kinds,
                              int32_t* n_kinds);
const char* pimd_kernel_name(int32_t kind);

/* Waits for all work enqueued by the context; reports a halted run (PIMD_ERR_NONFINITE,
 * PIMD_ERR_DEVICE). */
pimd_status pimd_synchronize(pimd_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PIMD_H */
