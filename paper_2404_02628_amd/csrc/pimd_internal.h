// pimd_internal.h -- device data layout shared by the libpimd translation units.
//
// One context holds R independent replicas that share P (beads), d (dim) and the
// precision mode.  All device arrays live in the caller's workspace; this header
// fixes how that workspace is carved up and what each kernel reads and writes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pimd {

constexpr int kTile = 64;          // rows/columns of one exchange tile (= wavefront size)
constexpr int kMaxNhc = 8;         // longest thermostat chain
constexpr int kRec = 16;           // doubles per energy record
constexpr int kSpringBlock = 256;  // particles per spring-kernel workgroup
constexpr int kIntBlock = 256;     // degrees of freedom per integrator workgroup
constexpr int kEtaSlots = kIntBlock / 64;   // chain-position sums per integrator work item (one per wave)

// Integrator work item: replica r, the `count` degrees of freedom from global index g0 on.  The
// global index is stored directly so that the integrator issues its loads after reading the work
// item alone, not after the replica's record as well.
__host__ __device__ inline int4 int_work_item(int r, long long g0, long long count) {
  return make_int4(r, (int)count, (int)(unsigned)(g0 & 0xffffffffLL), (int)(g0 >> 32));
}
__host__ __device__ inline long long int_work_first(const int4& wk) {
  return ((long long)wk.w << 32) | (long long)(unsigned)wk.z;
}

// Energy record slots (per replica, and per trace sample).
enum RecSlot {
  kVExch = 0, kUTrap, kUPair, kSpring, kVirial, kEPrim, kEVir, kKinetic, kNhcE, kHCons, kStep,
  kEintSum, kLinkSum, kPairW, kValid, kRecPad
};

// Per-replica constants and offsets, resident in device memory.
struct RepDev {
  int n;            // particles N
  int npad;         // N rounded up to kTile
  int npp;          // per-replica stride of particle arrays (npad + kTile, holds N+1 entries)
  int nblk;         // ceil(N / kTile)
  int na;           // particles of the first species (N - n2): cycles never join l <= na and l > na
  long long dof;    // offset of this replica's x, p, f, fpair block ([dim][P][N], contiguous)
  long long ndof;   // dim * P * N
  long long part;   // offset unit for particle arrays (sum of npp of earlier replicas)
  long long shadow; // offset of the FP32 shadow ([P][npad][dp] floats)
  long long spw0, spw1;    // spring workgroups [spw0, spw1)
  long long pw0, pw1;      // pair work items [pw0, pw1)
  long long rw0, rw1;      // probability-reduce workgroups [rw0, rw1)
  long long iw0, iw1;      // integrator work items [iw0, iw1)
  long long es0, es1;      // this replica's chain-position sums etasum[es0, es1): kEtaSlots per integrator
                           // work item, or one per dof when steps run in the persistent kernel
  double beta, hbar, mass, omega, xi, amp, width, dt, q, mp;
  double c;         // (1/2) m omega_P^2, omega_P = sqrt(P)/(beta hbar)
  double kappa;     // m omega_P^2
  double lnxi;      // log(xi), -inf for xi = 0
  double mw2;       // m omega^2 (trap)
  double inv_s2;    // 1/s^2 (0 if no pair term)
  double inv_mp;    // 1/m' (bead mass)
  double inv_q;     // 1/Q (thermostat mass)
  double kT;        // 1/beta
  double dt_mp;     // dt/m'
  double trap_p;    // m omega^2 / P (trap force constant per bead)
  float pair_k;     // sqrt(log2 e)/s, scale of the FP32 pair shadow (1 without pair term)
};

// Device pointers into the workspace (all replicas concatenated).
struct DevPtrs {
  RepDev* reps;
  double* x; double* p; double* f; double* fpair;
  float* xs;                   // FP32 shadow of x for the pair kernel, layout per replica [P][npad][dp]
  double* etasum;              // sums of the chain positions eta over dofs and chain elements: per
                               // integrator work item and wavefront ([nintwg][kEtaSlots]), or per dof
                               // ([G]) for the persistent kernel
  double* veta;                // [M][G] chain velocities
  double* ends;                // per replica: [2*dim][npp]  (a = first beads, then b = last beads)
  double* link;                // [npp]: c |b_l - a_{l+1}|^2, 0 for the last particle of each species
  double* eint;                // [npp]: internal spring energy of each ring
  double* gf; double* gb;      // [npp]: forward / backward normalised log-potentials, rows 0..N
  double4* colrec;             // [2][npp] per replica: recursion column records {q_j, colc_j + G_j}
  double* avg;                 // [2][dim+1][npp] per replica: weighted row averages of the recursions
  double* lam;                 // [2][npp] per replica: link prefixes lam_j = (1/c) sum_{m<j} link_m of the
                               // forward recursion's columns (zeros for the backward one)
  int* flags;                  // [4][npp] per replica: panel / partial ready flags (epochs), per direction
  double* partial;             // [2][dim+3][npp] per replica: helper partial sums (m, s, payloads)
  int* err;                    // status words: [0] raised by a timed-out wait of the cooperative
                               // recursion, [1] evaluation stamp (advanced by the spring kernel),
                               // [2] non-finite word: kNonfiniteBase - r of the lowest replica r
                               // whose force, momentum or position was found non-finite (0: none)
  double* springpart;          // [nspringwg][4]
  double* pairpart;            // [npairwork][2]
  double* reducepart;          // [nreducewg][2]
  double* rec;                 // [R][kRec] last estimators
  double* trace;               // [R][cap][kRec]
  long long* tracecount;       // [R]
  unsigned long long* dens;    // [R][bins+1]
  long long* denssamples;      // [R]
  int4* springwork;            // {rep, l0, 0, 0}
  int4* pairwork;              // {rep, slice, i0, 0}
  int4* reducework;            // {rep, l0, 0, 0}
  int4* intwork;               // {rep, dofs, first global dof (low word, high word)}: see int_work_item
  int* reporder;               // [R] replica of the k-th recursion workgroup pair (launch order)
  double* dbg;                 // debug scratch (N+2 doubles of the largest replica, x2)
};

struct Dims {
  int R, P, D, M, precision, sy_order, bins, cap;
  double rmax;
  long long G;                 // total dof (padded)
  long long NPtot;             // sum of npp
  long long XStot;             // floats in the shadow
  long long nspringwg, npairwork, nreducewg, nintwg;
  int maxn;                    // largest N of any replica
  int pair_maxn;               // largest N of a replica with pair interactions
};

__host__ __device__ inline int shadow_dp(int D) { return D == 3 ? 4 : D; }

constexpr int kNonfiniteBase = 0x7fffffff;

// A raised status word halts the dynamics: the integrator, the estimators and the density stop
// writing, so the state and the accumulators stay as they were when the failure was detected.
// Both words are read together (one memory round trip, not two).
__device__ inline bool status_halted(const int* err) {
  const int a = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int b = __hip_atomic_load(err + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (a | b) != 0;
}

// Records that replica r produced a non-finite value (the lowest such replica wins).
__device__ inline void status_nonfinite(int* err, int r) { atomicMax(err + 2, kNonfiniteBase - r); }

// Launchers (one per translation unit).
hipError_t launch_springs(const Dims& d, const DevPtrs& w, hipStream_t s);
hipError_t launch_pair(const Dims& d, const DevPtrs& w, bool estimators, int jsplit, hipStream_t s);
int pair_sym_lds_bytes(int D, int maxn, int precision);   // dynamic LDS of the symmetric pair kernel
// sp: also average the cycles' spring payload (the expected spring energy of the estimators)
// wide: eight waves per batched recursion workgroup instead of four
hipError_t launch_recursion(const Dims& d, const DevPtrs& w, bool sp, bool wide, hipStream_t s);
hipError_t launch_recursion_coop(const Dims& d, const DevPtrs& w, int helpers, bool sp, hipStream_t s);
int recursion_coop_max_blocks_per_cu(int D, int maxn);   // for the variant launched at this largest N
hipError_t launch_probs_reduce(const Dims& d, const DevPtrs& w, hipStream_t s);
hipError_t launch_integrate_first(const Dims& d, const DevPtrs& w, hipStream_t s);
hipError_t launch_integrate_second(const Dims& d, const DevPtrs& w, bool kick, hipStream_t s);
hipError_t launch_integrate_fused(const Dims& d, const DevPtrs& w, hipStream_t s);
hipError_t launch_estimators(const Dims& d, const DevPtrs& w, long long step, bool record, hipStream_t s);
hipError_t launch_density(const Dims& d, const DevPtrs& w, hipStream_t s);
hipError_t launch_debug_potentials(const Dims& d, const DevPtrs& w, int r, double* X, double* Y, hipStream_t s);
hipError_t launch_debug_probs(const Dims& d, const DevPtrs& w, int r, int n, int row0, int nrows, double* G,
                              hipStream_t s);
bool persistent_fits(int D, int P, int n);   // one workgroup can hold the replica's state
hipError_t launch_persistent(const Dims& d, const DevPtrs& w, int maxdof, long long step0, long long nsteps,
                             int sample_every, bool need_forces, hipStream_t s);
hipError_t launch_init_state(const Dims& d, const DevPtrs& w, const double* params, hipStream_t s);
hipError_t launch_cycle_direct(const Dims& d, const DevPtrs& w, int r, int n, int row0, int nrows, double* out,
                               hipStream_t s);

}  // namespace pimd
