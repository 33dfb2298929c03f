// capi.hip -- C ABI of libpimd: validation, workspace plan, per-step launch order.
//
// A force evaluation of all replicas is, in order on the caller's stream:
//   springs (interior/trap forces, end beads, links, E_int, FP32 shadow)
//   -> [pair kernel on a second stream, joined before the integrator]
//   -> forward+backward exchange recursions (potentials and the weighted row averages that
//      stand in for the probability matrix) -> per-particle end-bead forces and spring energy
// and an MD step wraps it in the two halves of the thermostatted velocity-Verlet step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pimd.h"
#include "pimd_internal.h"

using namespace pimd;

namespace {

thread_local std::string g_err;

pimd_status fail(pimd_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(PIMD_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

enum Kind { K_SPRINGS = 0, K_PAIR, K_RECURSION, K_REDUCE, K_INT1, K_INT2, K_INTF, K_EST, K_DENS, K_PERSIST, K_COUNT };
const char* kKindNames[K_COUNT] = {"springs", "pair", "recursion", "exchange_forces", "integrate_first",
                                   "integrate_second", "integrate_fused", "estimators", "density",
                                   "persistent_steps"};

// LDS one workgroup may hold on gfx950 (160 KiB per compute unit): the symmetric pair kernel keeps a
// whole slice there, which bounds the N it serves (mixed: 9,024 particles in 2-D, 5,184 in 3-D,
// 18,112 in 1-D; FP64: 4,416 in 2-D, 2,944 in 3-D, 8,896 in 1-D).
constexpr int kMaxLdsBytes = 160 * 1024;

// Steps per launch of the persistent kernel (a call with more steps is split).
constexpr long long kPersistChunk = 4096;

long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

struct Plan {
  Dims d{};
  int jsplit = 1;
  int ipw = 0;               // particles per pair work item (1 << 30: the whole slice)
  RepDev rep0{};             // constants of replica 0 (also when the lists are not stored)
  bool persistent = false;   // every replica fits one workgroup: steps run in the persistent kernel
  int persist_maxdof = 0;
  std::vector<RepDev> reps;
  std::vector<int4> springwork, pairwork, intwork;
  std::vector<int> reporder;  // replica of each recursion workgroup pair, in launch order
  size_t off[40]{};
  size_t total = 0;
};

enum Seg { S_REPS = 0, S_X, S_P, S_F, S_FPAIR, S_XS, S_ETA, S_VETA, S_ENDS, S_LINK, S_EINT, S_GF, S_GB, S_COLREC, S_AVG, S_LAM,
           S_FLAGS, S_PARTIAL, S_ERR,
           S_SPRINGP, S_PAIRP, S_REDP, S_REC, S_TRACE, S_TRACECNT, S_DENS, S_DENSN, S_SPRINGW, S_PAIRW, S_INTW, S_DBG,
           S_REPORD, S_COUNT };

// Doubles of the debug scratch: two potential arrays, up to 2^20 entries of a dense N x N table
// (filled in row chunks), or two parameters per replica for the seeded initial state.
long long dbg_doubles(int maxn, int R) {
  return std::max<long long>(std::max<long long>(2LL * (maxn + 2), 2LL * R),
                             std::min<long long>((long long)maxn * maxn, 1LL << 20));
}

// Checks one replica's parameters (the message is only built on failure).
pimd_status validate_replica(const pimd_replica& q, int r) {
  auto bad = [r](const char* what) { return fail(PIMD_ERR_INVALID, "replica " + std::to_string(r) + ": " + what); };
  if (q.n < 1 || q.n > (1 << 20)) return bad("n must be in 1..2^20");
  if (q.n2 < 0 || q.n2 >= q.n) return bad("n2 must be in 0..n-1");
  if (!(q.beta > 0) || !std::isfinite(q.beta)) return bad("beta must be > 0");
  if (!(q.hbar > 0) || !std::isfinite(q.hbar)) return bad("hbar must be > 0");
  if (!(q.mass > 0) || !std::isfinite(q.mass)) return bad("mass must be > 0");
  if (!(q.omega >= 0) || !std::isfinite(q.omega)) return bad("omega must be >= 0");
  if (!(q.xi >= 0 && q.xi <= 1)) return bad("xi must be in [0, 1]");
  if (!(q.pair_amp >= 0) || !std::isfinite(q.pair_amp)) return bad("pair_amp must be >= 0");
  if (q.pair_amp > 0 && (!(q.pair_width > 0) || !std::isfinite(q.pair_width))) return bad("pair_width must be > 0");
  if (!(q.dt > 0) || !std::isfinite(q.dt)) return bad("dt must be > 0");
  if (!std::isfinite(q.nhc_q) || !std::isfinite(q.bead_mass)) return bad("non-finite nhc_q/bead_mass");
  return PIMD_OK;
}

pimd_status validate(const pimd_config* c) {
  if (!c) return fail(PIMD_ERR_INVALID, "config is NULL");
  if (c->n_replicas < 1) return fail(PIMD_ERR_INVALID, "n_replicas must be >= 1");
  if (!c->replicas) return fail(PIMD_ERR_INVALID, "replicas is NULL");
  if (c->p < 2) return fail(PIMD_ERR_INVALID, "P must be >= 2");
  if (c->p > 4096) return fail(PIMD_ERR_INVALID, "P must be <= 4096");
  if (c->dim < 1 || c->dim > 3) return fail(PIMD_ERR_INVALID, "dim must be 1, 2 or 3");
  if (c->precision != PIMD_FP64 && c->precision != PIMD_MIXED) return fail(PIMD_ERR_INVALID, "bad precision");
  if (c->nhc_len < 0 || c->nhc_len > kMaxNhc) return fail(PIMD_ERR_INVALID, "nhc_len must be in 0..8");
  if (c->sy_order != 1 && c->sy_order != 3 && c->sy_order != 5) return fail(PIMD_ERR_INVALID, "sy_order must be 1, 3 or 5");
  if (c->density_bins < 1 || c->density_bins > 4096) return fail(PIMD_ERR_INVALID, "density_bins must be in 1..4096");
  if (!(c->density_rmax > 0)) return fail(PIMD_ERR_INVALID, "density_rmax must be > 0");
  if (c->trace_capacity < 0) return fail(PIMD_ERR_INVALID, "trace_capacity must be >= 0");
  if (c->recursion_workgroups < 0 || c->recursion_workgroups > 4096)
    return fail(PIMD_ERR_INVALID, "recursion_workgroups must be in 0..4096");
  if ((c->flags & ~(PIMD_FLAG_GRAPH | PIMD_FLAG_PAIR_ORDERED | PIMD_FLAG_NO_PERSISTENT | PIMD_FLAG_LONGEST_FIRST |
                    PIMD_FLAG_PAIR_SPLIT_MASK | PIMD_FLAG_RECURSION_WIDE)) != 0)
    return fail(PIMD_ERR_INVALID, "unknown bits in flags");
  for (int r = 0; r < c->n_replicas; ++r) {
    const pimd_status st = validate_replica(c->replicas[r], r);
    if (st != PIMD_OK) return st;
  }
  return PIMD_OK;
}

// Plans the workspace of a configuration: per-replica constants, work lists and segment offsets.
// With lists = false (the no-allocation entry point) nothing is stored on the heap: the work
// lists are only counted (their entries follow from the counts, see the prepare kernel), the
// first replica's constants go to pl.rep0, and the segments that the evaluation of one replica
// does not need (state it takes from the caller, thermostat, trace, density, debug) are empty.
void make_plan(const pimd_config* c, Plan& pl, bool lists = true) {
  Dims& d = pl.d;
  d.R = c->n_replicas; d.P = c->p; d.D = c->dim; d.M = c->nhc_len; d.precision = c->precision;
  d.sy_order = c->sy_order; d.bins = c->density_bins; d.cap = c->trace_capacity; d.rmax = c->density_rmax;
  const int dp = shadow_dp(d.D);
  // Pair kernel: with many interacting slices, one workgroup per slice that evaluates each
  // unordered pair once (either precision); otherwise the ordered kernel, split so that there are
  // enough waves to cover the machine (256 CUs x 4 SIMDs x ~2).
  long long tiles64 = 0, pair_slices = 0;
  int pair_maxn = 0;
  for (int r = 0; r < d.R; ++r)
    if (c->replicas[r].pair_amp > 0) {
      tiles64 += (long long)d.P * ((c->replicas[r].n + 63) / 64);
      pair_slices += d.P;
      pair_maxn = std::max(pair_maxn, c->replicas[r].n);
    }
  const bool sym = pair_slices >= 256 && pair_sym_lds_bytes(d.D, pair_maxn, d.precision) <= kMaxLdsBytes &&
                   (c->flags & PIMD_FLAG_PAIR_ORDERED) == 0;
  const int split_code = (c->flags & PIMD_FLAG_PAIR_SPLIT_MASK) / PIMD_FLAG_PAIR_SPLIT_1;   // 0, 1, 2, 3
  const int forced_split = split_code == 0 ? 0 : (1 << (split_code - 1));                   // 0, 1, 2, 4
  pl.jsplit = sym ? 0 : (forced_split ? forced_split : (tiles64 < 1024 ? 4 : (tiles64 < 2048 ? 2 : 1)));
  const int ipw = sym ? (1 << 30) : 64 * (4 / pl.jsplit);  // particles per pair workgroup
  pl.ipw = ipw;
  long long G = 0, NP = 0, XS = 0;
  long long nspring = 0, npair = 0, nint = 0;
  int maxn = 0;
  if (lists) pl.reps.resize(d.R);
  for (int r = 0; r < d.R; ++r) {
    const pimd_replica& q = c->replicas[r];
    RepDev R;
    std::memset(&R, 0, sizeof(R));
    R.n = q.n;
    R.npad = (int)round_up(q.n, kTile);
    R.npp = R.npad + kTile;
    R.nblk = (q.n + kTile - 1) / kTile;
    R.na = q.n - q.n2;
    R.ndof = (long long)d.D * d.P * q.n;
    R.dof = G;
    G += round_up(R.ndof, 64);
    R.part = NP;
    NP += R.npp;
    R.shadow = XS;
    if (d.precision == PIMD_MIXED) XS += (long long)d.P * R.npad * dp;
    maxn = std::max(maxn, q.n);
    R.beta = q.beta; R.hbar = q.hbar; R.mass = q.mass; R.omega = q.omega; R.xi = q.xi;
    R.amp = q.pair_amp; R.width = q.pair_amp > 0 ? q.pair_width : 1.0; R.dt = q.dt;
    const double wp2 = (double)d.P / (q.beta * q.beta * q.hbar * q.hbar);
    R.c = 0.5 * q.mass * wp2;
    R.kappa = q.mass * wp2;
    R.q = q.nhc_q > 0 ? q.nhc_q : 1.0 / (q.beta * wp2);
    R.mp = q.bead_mass > 0 ? q.bead_mass : q.mass;
    R.lnxi = q.xi > 0 ? std::log(q.xi) : -INFINITY;
    R.mw2 = q.mass * q.omega * q.omega;
    R.inv_s2 = q.pair_amp > 0 ? 1.0 / (q.pair_width * q.pair_width) : 0.0;
    R.inv_mp = 1.0 / R.mp;
    R.inv_q = 1.0 / R.q;
    R.kT = 1.0 / q.beta;
    R.dt_mp = q.dt / R.mp;
    R.trap_p = R.mw2 / (double)d.P;
    R.pair_k = (float)(q.pair_amp > 0 ? std::sqrt(1.4426950408889634) / q.pair_width : 1.0);
    R.spw0 = nspring;
    for (int l0 = 0; l0 < q.n; l0 += kSpringBlock, ++nspring)
      if (lists) pl.springwork.push_back(make_int4(r, l0, 0, 0));
    R.spw1 = nspring;
    R.rw0 = R.spw0; R.rw1 = R.spw1;
    R.iw0 = nint;
    for (long long d0 = 0; d0 < R.ndof; d0 += kIntBlock, ++nint)
      if (lists) pl.intwork.push_back(int_work_item(r, R.dof + d0, std::min<long long>(kIntBlock, R.ndof - d0)));
    R.iw1 = nint;
    if (lists) pl.reps[r] = R;
    if (r == 0) pl.rep0 = R;
  }
  // Launch order of the per-replica work of the pair kernel and the batched recursion: replica
  // index order, or longest first (descending N, ties by index) so that the most expensive
  // workgroups are dispatched first and the short ones fill in behind them.
  const bool longest = (c->flags & PIMD_FLAG_LONGEST_FIRST) != 0;
  if (lists) {
    pl.reporder.resize(d.R);
    for (int r = 0; r < d.R; ++r) pl.reporder[r] = r;
    if (longest)
      std::stable_sort(pl.reporder.begin(), pl.reporder.end(),
                       [c](int a, int b) { return c->replicas[a].n > c->replicas[b].n; });
  }
  // pair work items, one contiguous range per replica
  for (int k = 0; k < d.R; ++k) {
    const int r = lists ? pl.reporder[k] : k;
    const pimd_replica& q = c->replicas[r];
    long long pw0 = npair;
    if (q.pair_amp > 0)
      for (int j = 0; j < d.P; ++j)
        for (int i0 = 0; i0 < q.n; i0 += ipw, ++npair)
          if (lists) pl.pairwork.push_back(make_int4(r, j, i0, 0));
    if (lists) { pl.reps[r].pw0 = pw0; pl.reps[r].pw1 = npair; }
    if (r == 0) { pl.rep0.pw0 = pw0; pl.rep0.pw1 = npair; }
  }
  d.G = G; d.NPtot = NP; d.XStot = XS; d.maxn = maxn; d.pair_maxn = pair_maxn;
  // small replicas: whole steps in one persistent launch (unless the caller asks otherwise)
  pl.persistent = (c->flags & PIMD_FLAG_NO_PERSISTENT) == 0;
  pl.persist_maxdof = 0;
  for (int r = 0; r < d.R; ++r) {
    pl.persistent = pl.persistent && persistent_fits(d.D, d.P, c->replicas[r].n);
    pl.persist_maxdof = std::max(pl.persist_maxdof, d.D * d.P * c->replicas[r].n);
  }
  for (int r = 0; r < (lists ? d.R : 0); ++r) {
    RepDev& R = pl.reps[r];
    R.es0 = pl.persistent ? R.dof : R.iw0 * kEtaSlots;
    R.es1 = pl.persistent ? R.dof + R.ndof : R.iw1 * kEtaSlots;
  }
  pl.rep0.es0 = pl.persistent ? pl.rep0.dof : pl.rep0.iw0 * kEtaSlots;
  pl.rep0.es1 = pl.persistent ? pl.rep0.dof + pl.rep0.ndof : pl.rep0.iw1 * kEtaSlots;
  d.nspringwg = nspring;
  d.npairwork = npair;
  d.nreducewg = d.nspringwg;
  d.nintwg = nint;
  // segment sizes in bytes
  size_t sz[S_COUNT];
  sz[S_REPS] = sizeof(RepDev) * d.R;
  sz[S_X] = sz[S_P] = sz[S_F] = sz[S_FPAIR] = 8ull * G;
  sz[S_XS] = 4ull * XS;
  // chain-position sums: per dof on the persistent path (the sums of a coordinate stay with its
  // thread across launches), per integrator wavefront on the streaming path
  sz[S_ETA] = d.M == 0 ? 0 : (pl.persistent ? 8ull * G : 8ull * kEtaSlots * nint);
  sz[S_VETA] = 8ull * G * d.M;
  sz[S_ENDS] = 8ull * 2 * d.D * NP;
  sz[S_LINK] = sz[S_EINT] = sz[S_GF] = sz[S_GB] = 8ull * NP;
  sz[S_COLREC] = 32ull * 2 * NP;
  sz[S_AVG] = 8ull * 2 * (d.D + 1) * NP;
  sz[S_LAM] = 8ull * 2 * NP;
  sz[S_FLAGS] = 4ull * 4 * NP;
  sz[S_PARTIAL] = 8ull * 2 * (d.D + 3) * NP;
  sz[S_ERR] = 256;
  sz[S_SPRINGP] = 8ull * 4 * d.nspringwg;
  sz[S_PAIRP] = 8ull * 2 * std::max<long long>(d.npairwork, 1);
  sz[S_REDP] = 8ull * 2 * d.nreducewg;
  sz[S_REC] = 8ull * kRec * d.R;
  sz[S_TRACE] = 8ull * kRec * d.R * (size_t)d.cap;
  sz[S_TRACECNT] = 8ull * d.R;
  sz[S_DENS] = 8ull * d.R * (d.bins + 1);
  sz[S_DENSN] = 8ull * d.R;
  sz[S_SPRINGW] = sizeof(int4) * d.nspringwg;
  sz[S_PAIRW] = sizeof(int4) * std::max<long long>(d.npairwork, 1);
  sz[S_INTW] = sizeof(int4) * d.nintwg;
  sz[S_DBG] = 8ull * dbg_doubles(maxn, d.R);
  sz[S_REPORD] = sizeof(int) * d.R;
  if (!lists)
    for (int k : {S_X, S_P, S_F, S_ETA, S_VETA, S_TRACE, S_TRACECNT, S_DENS, S_DENSN, S_DBG}) sz[k] = 0;
  size_t o = 0;
  for (int s = 0; s < S_COUNT; ++s) {
    pl.off[s] = o;
    o += (size_t)round_up((long long)sz[s], 256);
  }
  pl.total = o;
}

// Device pointers of the workspace segments laid out by make_plan, from the workspace base.
void carve(char* ws, const size_t* off, DevPtrs& w) {
  w.reps = (RepDev*)(ws + off[S_REPS]);
  w.x = (double*)(ws + off[S_X]);
  w.p = (double*)(ws + off[S_P]);
  w.f = (double*)(ws + off[S_F]);
  w.fpair = (double*)(ws + off[S_FPAIR]);
  w.xs = (float*)(ws + off[S_XS]);
  w.etasum = (double*)(ws + off[S_ETA]);
  w.veta = (double*)(ws + off[S_VETA]);
  w.ends = (double*)(ws + off[S_ENDS]);
  w.link = (double*)(ws + off[S_LINK]);
  w.eint = (double*)(ws + off[S_EINT]);
  w.gf = (double*)(ws + off[S_GF]);
  w.gb = (double*)(ws + off[S_GB]);
  w.colrec = (double4*)(ws + off[S_COLREC]);
  w.avg = (double*)(ws + off[S_AVG]);
  w.lam = (double*)(ws + off[S_LAM]);
  w.flags = (int*)(ws + off[S_FLAGS]);
  w.partial = (double*)(ws + off[S_PARTIAL]);
  w.err = (int*)(ws + off[S_ERR]);
  w.springpart = (double*)(ws + off[S_SPRINGP]);
  w.pairpart = (double*)(ws + off[S_PAIRP]);
  w.reducepart = (double*)(ws + off[S_REDP]);
  w.rec = (double*)(ws + off[S_REC]);
  w.trace = (double*)(ws + off[S_TRACE]);
  w.tracecount = (long long*)(ws + off[S_TRACECNT]);
  w.dens = (unsigned long long*)(ws + off[S_DENS]);
  w.denssamples = (long long*)(ws + off[S_DENSN]);
  w.springwork = (int4*)(ws + off[S_SPRINGW]);
  w.pairwork = (int4*)(ws + off[S_PAIRW]);
  w.reducework = w.springwork;
  w.intwork = (int4*)(ws + off[S_INTW]);
  w.dbg = (double*)(ws + off[S_DBG]);
  w.reporder = (int*)(ws + off[S_REPORD]);
}

// Schedule of the exchange recursions: helper workgroups per cooperative chain (0: one workgroup
// per replica and direction).  Helpers pay when a few replicas would otherwise leave most of the
// device idle.  `req` is pimd_config.recursion_workgroups.
int choose_helpers(int req, const Dims& d) {
  int dev = 0, cus = 0, coop = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
    return 0;
  const int per_cu = recursion_coop_max_blocks_per_cu(d.D, d.maxn);
  const long long nchains = 2LL * d.R;
  const long long capacity = (long long)per_cu * cus;
  const int max_nblk = (d.maxn + 1 + kTile - 1) / kTile;
  const long long useful = std::max(0, max_nblk - 2);
  long long H = 0;
  if (req > 1) H = req - 1;
  else if (req == 0 && nchains * 4 <= cus && useful > 0) {
    // as many as fit, but about one helper per three row blocks: more only add polling
    // (one replica, FP64: N = 10^4 runs 7% faster with 52 helpers than with 127, while
    // N = 4 10^4 still gains up to the device's capacity)
    H = std::min<long long>(capacity / nchains - 1, std::max<long long>(24, max_nblk / 3));
  }
  H = std::min(H, useful);
  if (nchains * (1 + H) > capacity) H = capacity / nchains - 1;
  return (int)std::max(0LL, H);
}

}  // namespace

struct pimd_ctx {
  Plan pl;
  DevPtrs w{};
  char* ws = nullptr;
  hipStream_t s = nullptr, s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool forces_valid = false;
  bool evaluated = false;
  bool has_state = false;   // some replica's positions were set
  bool halted = false;      // a status word was seen raised: no steps until set_state / init_system
  long long step = 0;
  bool has_pair = false;
  int helpers = 0;       // helper workgroups per recursion chain (0: one workgroup per chain)
  bool wide = false;     // eight waves per workgroup of the one-workgroup schedule
  hipStream_t sc = nullptr;          // stream the step graph is captured on
  hipGraphExec_t gexec = nullptr;    // one steady MD step (evaluation + fused integrator halves)
  int graph_state = 0;               // 0 not built, 1 built, 2 not requested, 3 capture failed
  long long graph_replays = 0;
  bool profiling = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[K_COUNT] = {};
  long long prof_n[K_COUNT] = {};
};

namespace {

hipEvent_t take_event(pimd_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs `launch` on stream st, bracketed by events when profiling.
template <class F>
pimd_status timed(pimd_ctx* c, int kind, hipStream_t st, F&& launch) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profiling) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (!e0 || !e1) return fail(PIMD_ERR_DEVICE, "hipEventCreate failed");
    HIPCHK(hipEventRecord(e0, st));
  }
  hipError_t e = launch();
  if (e != hipSuccess) return fail(PIMD_ERR_DEVICE, std::string("kernel launch (") + kKindNames[kind] + "): " + hipGetErrorString(e));
  if (c->profiling) {
    HIPCHK(hipEventRecord(e1, st));
    c->prof.push_back({kind, {e0, e1}});
    if (c->prof.size() > 4096) {  // fold finished records to bound the pool
      HIPCHK(hipEventSynchronize(e1));
      for (auto& pr : c->prof) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, pr.second.first, pr.second.second));
        c->prof_ms[pr.first] += ms;
        c->prof_n[pr.first] += 1;
        c->ev_pool.push_back(pr.second.first);
        c->ev_pool.push_back(pr.second.second);
      }
      c->prof.clear();
    }
  }
  return PIMD_OK;
}

#define RUN(kind, st, expr)                                      \
  do {                                                           \
    pimd_status r_ = timed(c, kind, st, [&]() { return (expr); }); \
    if (r_ != PIMD_OK) return r_;                                \
  } while (0)

// One force evaluation of every replica at the current positions, enqueued on stream ms.  The
// exchange recursions are launched before the pair kernel (which runs on the second stream), so
// their few long-lived workgroups are placed first and the pair workgroups fill the rest.
pimd_status evaluate(pimd_ctx* c, bool est, hipStream_t ms) {
  const Dims& d = c->pl.d;
  const DevPtrs& w = c->w;
  RUN(K_SPRINGS, ms, launch_springs(d, w, ms));
  const bool fork = c->has_pair;
  if (fork) HIPCHK(hipEventRecord(c->ev_fork, ms));
  if (c->helpers > 0) RUN(K_RECURSION, ms, launch_recursion_coop(d, w, c->helpers, est, ms));
  else RUN(K_RECURSION, ms, launch_recursion(d, w, est, c->wide, ms));
  RUN(K_REDUCE, ms, launch_probs_reduce(d, w, ms));
  if (c->has_pair) {
    hipStream_t ps = fork ? c->s2 : ms;
    if (fork) HIPCHK(hipStreamWaitEvent(c->s2, c->ev_fork, 0));
    RUN(K_PAIR, ps, launch_pair(d, w, est, c->pl.jsplit, ps));
    if (fork) {
      HIPCHK(hipEventRecord(c->ev_join, c->s2));
      HIPCHK(hipStreamWaitEvent(ms, c->ev_join, 0));
    }
  }
  return PIMD_OK;
}

// Captures one steady MD step (evaluation, then the fused second half of this step and first
// half of the next) into c->gexec.  On any failure the graph stays absent and graph_state = 3.
void build_step_graph(pimd_ctx* c) {
  hipGraph_t g = nullptr;
  pimd_status st = PIMD_ERR_DEVICE;
  hipError_t e = hipStreamBeginCapture(c->sc, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = evaluate(c, false, c->sc);
    if (st == PIMD_OK) {
      e = launch_integrate_fused(c->pl.d, c->w, c->sc);
      if (e != hipSuccess) st = PIMD_ERR_DEVICE;
    }
    const hipError_t e2 = hipStreamEndCapture(c->sc, &g);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess && st == PIMD_OK && g != nullptr) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  if (g != nullptr) (void)hipGraphDestroy(g);
  if (e != hipSuccess || st != PIMD_OK || c->gexec == nullptr) {
    c->gexec = nullptr;
    c->graph_state = 3;
    (void)hipGetLastError();
  } else {
    c->graph_state = 1;
  }
}

pimd_status sample(pimd_ctx* c, bool record) {
  const Dims& d = c->pl.d;
  RUN(K_EST, c->s, launch_estimators(d, c->w, c->step, record, c->s));
  if (record) RUN(K_DENS, c->s, launch_density(d, c->w, c->s));
  return PIMD_OK;
}

pimd_status check_ctx_r(pimd_ctx* c, int32_t r) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  if (r < 0 || r >= c->pl.d.R) return fail(PIMD_ERR_INVALID, "replica index out of range");
  return PIMD_OK;
}

hipMemcpyKind kind_in(pimd_mem m) { return m == PIMD_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind kind_out(pimd_mem m) { return m == PIMD_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

}  // namespace

// Reads the device status words (after the work enqueued so far).  A timed-out wait of the
// cooperative recursion gives PIMD_ERR_DEVICE, a non-finite force, momentum or position
// PIMD_ERR_NONFINITE naming the lowest such replica.  Either halts the context: the kernels have
// stopped advancing the state, and pimd_step / pimd_compute_forces refuse to run until
// pimd_set_state or pimd_init_system lowers the words.
static pimd_status check_status(pimd_ctx* c) {
  int st[3] = {0, 0, 0};
  HIPCHK(hipMemcpyAsync(st, c->w.err, sizeof(st), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  if (st[0] != 0) {
    c->halted = true;
    c->forces_valid = false;
    return fail(PIMD_ERR_DEVICE, "a wait of the cooperative exchange recursion timed out; results are invalid "
                                 "and the run is halted until pimd_set_state or pimd_init_system");
  }
  if (st[2] != 0) {
    c->halted = true;
    return fail(PIMD_ERR_NONFINITE, "replica " + std::to_string(kNonfiniteBase - st[2]) +
                                        ": non-finite force, momentum or position; the run is halted at the step "
                                        "where it appeared until pimd_set_state or pimd_init_system");
  }
  return PIMD_OK;
}

// Lowers the wait-failure and non-finite words (the evaluation stamp between them is kept).
static pimd_status clear_status(pimd_ctx* c) {
  HIPCHK(hipMemsetAsync(c->w.err, 0, sizeof(int), c->s));
  HIPCHK(hipMemsetAsync(c->w.err + 2, 0, sizeof(int), c->s));
  c->halted = false;
  return PIMD_OK;
}

static pimd_status check_not_halted(pimd_ctx* c) {
  if (c->halted)
    return fail(PIMD_ERR_STATE, "the run is halted after a failure; call pimd_set_state or pimd_init_system");
  return PIMD_OK;
}


// ------------------------------------------------------------------ no-allocation entry point
//
// pimd_compute_forces_noalloc keeps everything an evaluation of one replica needs beyond the
// caller's positions and forces (per-replica constants, work lists, end beads, links, potentials,
// recursion records, row averages, partial sums, FP32 shadow, pair forces, estimator record and
// status words) in `scratch`, a static device array: every GPU the library runs on holds its own
// copy until the process ends.  Host code never passes the array's name to a kernel (on the host
// it only stands in for the symbol): its device address on each GPU is looked up once, with that
// GPU current, and that address is what the kernels receive.

static __device__ __align__(256) unsigned char scratch[PIMD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current GPU (looked up on the first call on that GPU).
pimd_status noalloc_scratch(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(PIMD_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return fail(PIMD_ERR_DEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PIMD_OK;
}

// The per-replica constants and the work lists of a one-replica plan, whose entries follow from
// their counts (the lists make_plan builds on the host for pimd_create), and the status words
// lowered.  The cooperative recursion's progress flags are cleared as well: the scratch keeps
// whatever the previous call left there, and a call of another size lays its arrays out
// differently, so a stale word could otherwise equal this evaluation's stamp.
__global__ void k_noalloc_prepare(RepDev rep0, DevPtrs w, long long nspring, long long npair, long long per_slice,
                                  int ipw, long long nint, long long nflags) {
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (t0 == 0) {
    *w.reps = rep0;
    w.reporder[0] = 0;
    w.err[0] = 0;
    w.err[2] = 0;
  }
  for (long long k = t0; k < nspring; k += stride) w.springwork[k] = make_int4(0, (int)(k * kSpringBlock), 0, 0);
  for (long long k = t0; k < npair; k += stride)
    w.pairwork[k] = make_int4(0, (int)(k / per_slice), (int)(k % per_slice) * ipw, 0);
  for (long long k = t0; k < nint; k += stride)
    w.intwork[k] = int_work_item(0, rep0.dof + k * kIntBlock, min((long long)kIntBlock, rep0.ndof - k * kIntBlock));
  for (long long k = t0; k < nflags; k += stride) w.flags[k] = 0;
}

// The estimator record as pimd_estimates (NaN everywhere if a status word was raised).
__global__ void k_noalloc_estimates(const double* rec, const int* err, pimd_estimates* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const bool bad = status_halted(err);
  const double nan = __builtin_nan("");
  out->v_exch = bad ? nan : rec[kVExch];
  out->u_trap = bad ? nan : rec[kUTrap];
  out->u_pair = bad ? nan : rec[kUPair];
  out->spring_expect = bad ? nan : rec[kSpring];
  out->virial = bad ? nan : rec[kVirial];
  out->e_prim = bad ? nan : rec[kEPrim];
  out->e_vir = bad ? nan : rec[kEVir];
  out->kinetic = 0.0;
  out->nhc_energy = 0.0;
  out->h_conserved = bad ? nan : rec[kHCons];
  out->step = 0;
}

}  // namespace

extern "C" {

int pimd_abi_version(void) { return PIMD_ABI_VERSION; }

const char* pimd_last_error(void) { return g_err.c_str(); }

pimd_status pimd_workspace_bytes(const pimd_config* cfg, size_t* bytes) {
  pimd_status st = validate(cfg);
  if (st != PIMD_OK) return st;
  if (!bytes) return fail(PIMD_ERR_INVALID, "bytes is NULL");
  Plan pl;
  make_plan(cfg, pl);
  *bytes = pl.total;
  return PIMD_OK;
}

pimd_status pimd_create(const pimd_config* cfg, void* d_workspace, size_t bytes, void* hip_stream, pimd_ctx** out) {
  pimd_status st = validate(cfg);
  if (st != PIMD_OK) return st;
  if (!out) return fail(PIMD_ERR_INVALID, "out is NULL");
  *out = nullptr;
  pimd_ctx* c = new pimd_ctx();
  make_plan(cfg, c->pl);
  if (!d_workspace || ((uintptr_t)d_workspace & 255u) || bytes < c->pl.total) {
    size_t need = c->pl.total;
    delete c;
    return fail(PIMD_ERR_WORKSPACE, "workspace must be 256-byte aligned and at least " + std::to_string(need) + " bytes");
  }
  c->ws = (char*)d_workspace;
  c->s = (hipStream_t)hip_stream;
  carve(c->ws, c->pl.off, c->w);
  DevPtrs& w = c->w;
  for (auto& r : c->pl.reps) c->has_pair = c->has_pair || r.amp > 0;
  c->graph_state = (cfg->flags & PIMD_FLAG_GRAPH) ? 0 : 2;
  auto cleanup = [&](pimd_status s2) {
    if (c->s2) (void)hipStreamDestroy(c->s2);
    if (c->sc) (void)hipStreamDestroy(c->sc);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    delete c;
    return s2;
  };
  hipError_t e = hipMemsetAsync(c->ws, 0, c->pl.total, c->s);
  if (e == hipSuccess) e = hipMemcpyAsync(w.reps, c->pl.reps.data(), sizeof(RepDev) * c->pl.reps.size(), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess && !c->pl.springwork.empty())
    e = hipMemcpyAsync(w.springwork, c->pl.springwork.data(), sizeof(int4) * c->pl.springwork.size(), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess && !c->pl.pairwork.empty())
    e = hipMemcpyAsync(w.pairwork, c->pl.pairwork.data(), sizeof(int4) * c->pl.pairwork.size(), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess && !c->pl.intwork.empty())
    e = hipMemcpyAsync(w.intwork, c->pl.intwork.data(), sizeof(int4) * c->pl.intwork.size(), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(w.reporder, c->pl.reporder.data(), sizeof(int) * c->pl.reporder.size(), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->sc, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  if (e != hipSuccess) return cleanup(fail(PIMD_ERR_DEVICE, std::string("pimd_create: ") + hipGetErrorString(e)));
  c->helpers = choose_helpers(cfg->recursion_workgroups, c->pl.d);
  c->wide = (cfg->flags & PIMD_FLAG_RECURSION_WIDE) != 0;
  *out = c;
  return PIMD_OK;
}

pimd_status pimd_destroy(pimd_ctx* c) {
  if (!c) return PIMD_OK;
  (void)hipStreamSynchronize(c->s);
  if (c->s2) (void)hipStreamSynchronize(c->s2);
  for (auto& pr : c->prof) { (void)hipEventDestroy(pr.second.first); (void)hipEventDestroy(pr.second.second); }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->s2) (void)hipStreamDestroy(c->s2);
  if (c->sc) (void)hipStreamDestroy(c->sc);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  delete c;
  return PIMD_OK;
}

pimd_status pimd_set_state(pimd_ctx* c, int32_t r, const double* x, const double* p, const double* nhc, pimd_mem where) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (!x) return fail(PIMD_ERR_INVALID, "x is NULL");
  if (where != PIMD_HOST && where != PIMD_DEVICE) return fail(PIMD_ERR_INVALID, "bad memory kind");
  const RepDev& R = c->pl.reps[r];
  const Dims& d = c->pl.d;
  const size_t nb = sizeof(double) * (size_t)R.ndof;
  HIPCHK(hipStreamSynchronize(c->s));
  if ((st = clear_status(c)) != PIMD_OK) return st;
  HIPCHK(hipMemcpyAsync(c->w.x + R.dof, x, nb, kind_in(where), c->s));
  if (p) HIPCHK(hipMemcpyAsync(c->w.p + R.dof, p, nb, kind_in(where), c->s));
  else HIPCHK(hipMemsetAsync(c->w.p + R.dof, 0, nb, c->s));
  // thermostat: chain velocities, then the chain positions' sum into the replica's first slot
  for (int k = 0; k < d.M; ++k) {
    if (nhc) HIPCHK(hipMemcpyAsync(c->w.veta + (long long)k * d.G + R.dof, nhc + (size_t)k * R.ndof, nb, kind_in(where), c->s));
    else HIPCHK(hipMemsetAsync(c->w.veta + (long long)k * d.G + R.dof, 0, nb, c->s));
  }
  if (d.M > 0) {
    double* slots = c->w.etasum + R.es0;
    const size_t nslots = (size_t)(R.es1 - R.es0);
    HIPCHK(hipMemsetAsync(slots, 0, sizeof(double) * nslots, c->s));
    if (nhc) HIPCHK(hipMemcpyAsync(slots, nhc + (size_t)d.M * R.ndof, sizeof(double), kind_in(where), c->s));
  }
  HIPCHK(hipStreamSynchronize(c->s));
  c->forces_valid = false;
  c->has_state = true;
  return PIMD_OK;
}

pimd_status pimd_get_state(pimd_ctx* c, int32_t r, double* x, double* p, double* nhc, pimd_mem where) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (where != PIMD_HOST && where != PIMD_DEVICE) return fail(PIMD_ERR_INVALID, "bad memory kind");
  const RepDev& R = c->pl.reps[r];
  const Dims& d = c->pl.d;
  const size_t nb = sizeof(double) * (size_t)R.ndof;
  if (x) HIPCHK(hipMemcpyAsync(x, c->w.x + R.dof, nb, kind_out(where), c->s));
  if (p) HIPCHK(hipMemcpyAsync(p, c->w.p + R.dof, nb, kind_out(where), c->s));
  if (nhc && d.M > 0) {
    for (int k = 0; k < d.M; ++k)
      HIPCHK(hipMemcpyAsync(nhc + (size_t)k * R.ndof, c->w.veta + (long long)k * d.G + R.dof, nb, kind_out(where), c->s));
    // the sum of the chain positions, from the replica's slots in a fixed order
    std::vector<double> slots((size_t)(R.es1 - R.es0));
    HIPCHK(hipMemcpyAsync(slots.data(), c->w.etasum + R.es0, sizeof(double) * slots.size(), hipMemcpyDeviceToHost,
                          c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    double total = 0.0;
    for (double v : slots) total += v;
    HIPCHK(hipMemcpy(nhc + (size_t)d.M * R.ndof, &total, sizeof(double),
                     where == PIMD_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    // fold the slots into the value returned, as pimd_set_state stores it: a context started
    // from this state then adds the same increments to the same slots, bit for bit
    std::fill(slots.begin(), slots.end(), 0.0);
    slots[0] = total;
    HIPCHK(hipMemcpy(c->w.etasum + R.es0, slots.data(), sizeof(double) * slots.size(), hipMemcpyHostToDevice));
  }
  HIPCHK(hipStreamSynchronize(c->s));
  return check_status(c);
}

pimd_status pimd_compute_forces_noalloc(const pimd_config* cfg, const double* x, double* f, pimd_estimates* est,
                                        void* hip_stream) {
  pimd_status st = validate(cfg);
  if (st != PIMD_OK) return st;
  if (cfg->n_replicas != 1) return fail(PIMD_ERR_INVALID, "pimd_compute_forces_noalloc evaluates one replica (n_replicas = 1)");
  if (!x || !f) return fail(PIMD_ERR_INVALID, "x and f must be device arrays");
  Plan pl;   // the plan without lists stores nothing on the heap
  make_plan(cfg, pl, false);
  if (pl.total > (size_t)PIMD_NOALLOC_SCRATCH_BYTES)
    return fail(PIMD_ERR_WORKSPACE, "this replica needs " + std::to_string(pl.total) +
                                        " bytes of scratch; pimd_compute_forces_noalloc holds " +
                                        std::to_string((size_t)PIMD_NOALLOC_SCRATCH_BYTES));
  void* base = nullptr;
  if ((st = noalloc_scratch(&base)) != PIMD_OK) return st;
  DevPtrs w{};
  carve((char*)base, pl.off, w);
  // the caller's arrays; no momenta, thermostats, trace, density or debug output
  w.x = const_cast<double*>(x);
  w.f = f;
  w.p = nullptr; w.etasum = nullptr; w.veta = nullptr; w.trace = nullptr; w.tracecount = nullptr;
  w.dens = nullptr; w.denssamples = nullptr; w.dbg = nullptr;
  Dims d = pl.d;
  d.M = 0;
  d.cap = 0;
  const RepDev& R = pl.rep0;
  hipStream_t s = (hipStream_t)hip_stream;
  const int helpers = choose_helpers(cfg->recursion_workgroups, d);
  const long long per_slice = pl.ipw >= (1 << 30) ? 1 : (R.n + pl.ipw - 1) / pl.ipw;
  const long long nflags = 4LL * d.NPtot;
  const long long most = std::max({d.nspringwg, d.npairwork, d.nintwg, nflags});
  const unsigned grid = (unsigned)std::min<long long>(1024, std::max<long long>(1, (most + 255) / 256));
  hipLaunchKernelGGL(k_noalloc_prepare, dim3(grid), dim3(256), 0, s, R, w, d.nspringwg, d.npairwork, per_slice, pl.ipw,
                     d.nintwg, nflags);
  HIPCHK(hipGetLastError());
  // the evaluation of pimd_compute_forces, every kernel on the caller's stream
  HIPCHK(launch_springs(d, w, s));
  const bool want_est = est != nullptr;
  const bool wide = (cfg->flags & PIMD_FLAG_RECURSION_WIDE) != 0;
  HIPCHK(helpers > 0 ? launch_recursion_coop(d, w, helpers, want_est, s) : launch_recursion(d, w, want_est, wide, s));
  HIPCHK(launch_probs_reduce(d, w, s));
  HIPCHK(launch_pair(d, w, est != nullptr, pl.jsplit, s));
  HIPCHK(launch_integrate_second(d, w, false, s));   // f += pair forces; non-finite check
  if (est != nullptr) {
    HIPCHK(launch_estimators(d, w, 0, false, s));
    hipLaunchKernelGGL(k_noalloc_estimates, dim3(1), dim3(64), 0, s, w.rec, w.err, est);
    HIPCHK(hipGetLastError());
  }
  return PIMD_OK;
}

pimd_status pimd_compute_forces(pimd_ctx* c) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  pimd_status st = check_not_halted(c);
  if (st != PIMD_OK) return st;
  st = evaluate(c, true, c->s);
  if (st != PIMD_OK) return st;
  RUN(K_INT2, c->s, launch_integrate_second(c->pl.d, c->w, false, c->s));
  st = sample(c, false);
  if (st != PIMD_OK) return st;
  c->forces_valid = true;
  c->evaluated = true;
  return PIMD_OK;
}

pimd_status pimd_get_forces(pimd_ctx* c, int32_t r, double* f, pimd_mem where) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (!f) return fail(PIMD_ERR_INVALID, "f is NULL");
  if (!c->forces_valid) return fail(PIMD_ERR_STATE, "no force evaluation since the last set_state");
  const RepDev& R = c->pl.reps[r];
  HIPCHK(hipMemcpyAsync(f, c->w.f + R.dof, sizeof(double) * (size_t)R.ndof, kind_out(where), c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return check_status(c);
}

pimd_status pimd_step(pimd_ctx* c, int64_t n_steps, int32_t sample_every) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  if (n_steps < 0 || sample_every < 0) return fail(PIMD_ERR_INVALID, "n_steps and sample_every must be >= 0");
  const Dims& d = c->pl.d;
  pimd_status st = check_not_halted(c);
  if (st != PIMD_OK) return st;
  if (c->pl.persistent) {
    bool need = !c->forces_valid;
    for (long long done = 0; done < n_steps; done += kPersistChunk) {
      const long long k = std::min<long long>(kPersistChunk, n_steps - done);
      RUN(K_PERSIST, c->s, launch_persistent(d, c->w, c->pl.persist_maxdof, c->step, k, sample_every, need, c->s));
      if (sample_every > 0 && (c->step + k) / sample_every > c->step / sample_every) c->evaluated = true;
      c->step += k;
      need = false;
      c->forces_valid = true;
    }
    return PIMD_OK;
  }
  if (!c->forces_valid && n_steps > 0) {
    if ((st = evaluate(c, false, c->s)) != PIMD_OK) return st;
    RUN(K_INT2, c->s, launch_integrate_second(d, c->w, false, c->s));
    c->forces_valid = true;
  }
  // Step k: [first half] evaluate [second half].  The second half of step k and the first
  // half of step k+1 run as one fused pass unless step k is sampled (the estimators need the
  // state between the halves) or k is the last step of this call.
  // A steady step (first half already fused into the previous step, not sampled, not last) is
  // replayed from the captured step graph when one is available.
  bool pending_first = true;
  for (int64_t it = 0; it < n_steps; ++it) {
    const bool smp = sample_every > 0 && ((c->step + 1) % sample_every == 0);
    const bool last = (it + 1 == n_steps);
    if (!pending_first && !smp && !last && !c->profiling && (c->graph_state == 0 || c->graph_state == 1)) {
      if (c->graph_state == 0) build_step_graph(c);
      if (c->gexec != nullptr) {
        HIPCHK(hipGraphLaunch(c->gexec, c->s));
        c->step += 1;
        c->graph_replays += 1;
        continue;
      }
    }
    if (pending_first) RUN(K_INT1, c->s, launch_integrate_first(d, c->w, c->s));
    if ((st = evaluate(c, smp, c->s)) != PIMD_OK) return st;
    c->step += 1;
    if (smp || last) {
      RUN(K_INT2, c->s, launch_integrate_second(d, c->w, true, c->s));
      if (smp) {
        if ((st = sample(c, true)) != PIMD_OK) return st;
        c->evaluated = true;
      }
      pending_first = true;
    } else {
      RUN(K_INTF, c->s, launch_integrate_fused(d, c->w, c->s));
      pending_first = false;
    }
  }
  return PIMD_OK;
}

static void rec_to_struct(const double* o, pimd_estimates* e) {
  e->v_exch = o[kVExch]; e->u_trap = o[kUTrap]; e->u_pair = o[kUPair]; e->spring_expect = o[kSpring];
  e->virial = o[kVirial]; e->e_prim = o[kEPrim]; e->e_vir = o[kEVir]; e->kinetic = o[kKinetic];
  e->nhc_energy = o[kNhcE]; e->h_conserved = o[kHCons]; e->step = (int64_t)o[kStep];
}

pimd_status pimd_energies(pimd_ctx* c, int32_t r, pimd_estimates* out) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (!out) return fail(PIMD_ERR_INVALID, "out is NULL");
  double o[kRec];
  HIPCHK(hipMemcpyAsync(o, c->w.rec + (long long)kRec * r, sizeof(o), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  if (o[kValid] == 1.0) rec_to_struct(o, out);
  if ((st = check_status(c)) != PIMD_OK) return st;
  if (o[kValid] != 1.0) return fail(PIMD_ERR_STATE, "no sampled evaluation yet");
  for (int k = 0; k < kStep; ++k)
    if (!std::isfinite(o[k])) return fail(PIMD_ERR_NONFINITE, "replica " + std::to_string(r) + ": non-finite estimator");
  return PIMD_OK;
}

pimd_status pimd_trace(pimd_ctx* c, int32_t r, pimd_estimates* out, int64_t max_samples, int64_t* n_samples) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (!n_samples || max_samples < 0 || (max_samples > 0 && !out)) return fail(PIMD_ERR_INVALID, "bad output arguments");
  const Dims& d = c->pl.d;
  long long cnt = 0;
  HIPCHK(hipMemcpyAsync(&cnt, c->w.tracecount + r, sizeof(cnt), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  long long avail = std::min<long long>(cnt, d.cap);
  long long take = std::min<long long>(avail, max_samples);
  std::vector<double> buf((size_t)d.cap * kRec);
  if (take > 0) {
    HIPCHK(hipMemcpyAsync(buf.data(), c->w.trace + (long long)r * d.cap * kRec, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    for (long long k = 0; k < take; ++k) {
      long long idx = (cnt - take + k) % d.cap;
      rec_to_struct(&buf[(size_t)idx * kRec], &out[k]);
    }
  }
  *n_samples = take;
  return check_status(c);
}

pimd_status pimd_density(pimd_ctx* c, int32_t r, uint64_t* counts, int64_t* n_samples) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (!counts || !n_samples) return fail(PIMD_ERR_INVALID, "NULL output");
  const Dims& d = c->pl.d;
  long long ns = 0;
  HIPCHK(hipMemcpyAsync(counts, c->w.dens + (long long)r * (d.bins + 1), 8ull * (d.bins + 1), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipMemcpyAsync(&ns, c->w.denssamples + r, sizeof(ns), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  *n_samples = ns;
  return check_status(c);
}

pimd_status pimd_reset_accumulators(pimd_ctx* c) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  const size_t* off = c->pl.off;
  const Dims& d = c->pl.d;
  HIPCHK(hipMemsetAsync(c->ws + off[S_TRACECNT], 0, 8ull * d.R, c->s));
  HIPCHK(hipMemsetAsync(c->ws + off[S_DENS], 0, 8ull * d.R * (d.bins + 1), c->s));
  HIPCHK(hipMemsetAsync(c->ws + off[S_DENSN], 0, 8ull * d.R, c->s));
  return PIMD_OK;
}

pimd_status pimd_debug_potentials(pimd_ctx* c, int32_t r, double* X, double* Y) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (!X || !Y) return fail(PIMD_ERR_INVALID, "NULL output");
  if (!c->forces_valid) return fail(PIMD_ERR_STATE, "no force evaluation since the last set_state");
  const int N = c->pl.reps[r].n;
  double* dX = c->w.dbg;
  double* dY = c->w.dbg + (N + 2);
  HIPCHK(launch_debug_potentials(c->pl.d, c->w, r, dX, dY, c->s));
  HIPCHK(hipMemcpyAsync(X, dX, sizeof(double) * (N + 1), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipMemcpyAsync(Y, dY, sizeof(double) * (N + 2), hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return PIMD_OK;
}

pimd_status pimd_debug_probs(pimd_ctx* c, int32_t r, double* G) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (!G) return fail(PIMD_ERR_INVALID, "NULL output");
  if (!c->forces_valid) return fail(PIMD_ERR_STATE, "no force evaluation since the last set_state");
  const long long N = c->pl.reps[r].n;
  const long long rows = std::max<long long>(1, dbg_doubles(c->pl.d.maxn, c->pl.d.R) / N);
  for (long long r0 = 0; r0 < N; r0 += rows) {
    const long long nr = std::min(rows, N - r0);
    HIPCHK(launch_debug_probs(c->pl.d, c->w, r, (int)N, (int)r0, (int)nr, c->w.dbg, c->s));
    HIPCHK(hipMemcpyAsync(G + r0 * N, c->w.dbg, sizeof(double) * nr * N, hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
  }
  return PIMD_OK;
}

pimd_status pimd_init_system(pimd_ctx* c, const double* pos_sigma, const uint64_t* seeds) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  if (!pos_sigma || !seeds) return fail(PIMD_ERR_INVALID, "NULL pos_sigma or seeds");
  const int R = c->pl.d.R;
  std::vector<double> prm(2 * (size_t)R);
  for (int r = 0; r < R; ++r) {
    if (!(pos_sigma[r] >= 0) || !std::isfinite(pos_sigma[r]))
      return fail(PIMD_ERR_INVALID, "replica " + std::to_string(r) + ": pos_sigma must be finite and >= 0");
    prm[2 * r] = pos_sigma[r];
    std::memcpy(&prm[2 * r + 1], &seeds[r], sizeof(double));
  }
  HIPCHK(hipStreamSynchronize(c->s));
  pimd_status st = clear_status(c);
  if (st != PIMD_OK) return st;
  HIPCHK(hipMemcpyAsync(c->w.dbg, prm.data(), sizeof(double) * prm.size(), hipMemcpyHostToDevice, c->s));
  HIPCHK(launch_init_state(c->pl.d, c->w, c->w.dbg, c->s));
  if (c->pl.d.M > 0)   // chains at rest: every chain-position sum to zero
    HIPCHK(hipMemsetAsync(c->w.etasum, 0, c->pl.off[S_ETA + 1] - c->pl.off[S_ETA], c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  c->forces_valid = false;
  c->has_state = true;
  return PIMD_OK;
}

pimd_status pimd_cycle_energies(pimd_ctx* c, int32_t r, double* E, double* ms) {
  pimd_status st = check_ctx_r(c, r);
  if (st != PIMD_OK) return st;
  if (!E) return fail(PIMD_ERR_INVALID, "NULL output");
  if (!c->has_state) return fail(PIMD_ERR_STATE, "no state set");
  const long long N = c->pl.reps[r].n;
  const long long rows = std::max<long long>(1, dbg_doubles(c->pl.d.maxn, c->pl.d.R) / N);
  hipEvent_t e0 = take_event(c), e1 = take_event(c);
  if (!e0 || !e1) return fail(PIMD_ERR_DEVICE, "hipEventCreate failed");
  auto run = [&]() -> pimd_status {
    double total = 0.0;
    for (long long r0 = 0; r0 < N; r0 += rows) {
      const long long nr = std::min(rows, N - r0);
      HIPCHK(hipEventRecord(e0, c->s));
      HIPCHK(launch_cycle_direct(c->pl.d, c->w, r, (int)N, (int)r0, (int)nr, c->w.dbg, c->s));
      HIPCHK(hipEventRecord(e1, c->s));
      HIPCHK(hipMemcpyAsync(E + r0 * N, c->w.dbg, sizeof(double) * nr * N, hipMemcpyDeviceToHost, c->s));
      HIPCHK(hipStreamSynchronize(c->s));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, e0, e1));
      total += t;
    }
    if (ms) *ms = total;
    return PIMD_OK;
  };
  st = run();
  c->ev_pool.push_back(e0);
  c->ev_pool.push_back(e1);
  return st;
}

pimd_status pimd_profile(pimd_ctx* c, int enable) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  HIPCHK(hipStreamSynchronize(c->s));
  for (auto& pr : c->prof) { c->ev_pool.push_back(pr.second.first); c->ev_pool.push_back(pr.second.second); }
  c->prof.clear();
  for (int k = 0; k < K_COUNT; ++k) { c->prof_ms[k] = 0.0; c->prof_n[k] = 0; }
  c->profiling = enable != 0;
  return PIMD_OK;
}

pimd_status pimd_kernel_times(pimd_ctx* c, double* ms, int64_t* launches, int32_t max_kinds, int32_t* n_kinds) {
  if (!c || !n_kinds || max_kinds < 0 || (max_kinds > 0 && (!ms || !launches))) return fail(PIMD_ERR_INVALID, "bad arguments");
  HIPCHK(hipStreamSynchronize(c->s));
  for (auto& pr : c->prof) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, pr.second.first, pr.second.second));
    c->prof_ms[pr.first] += t;
    c->prof_n[pr.first] += 1;
    c->ev_pool.push_back(pr.second.first);
    c->ev_pool.push_back(pr.second.second);
  }
  c->prof.clear();
  for (int k = 0; k < K_COUNT && k < max_kinds; ++k) { ms[k] = c->prof_ms[k]; launches[k] = c->prof_n[k]; }
  *n_kinds = K_COUNT;
  return PIMD_OK;
}

const char* pimd_kernel_name(int32_t kind) {
  if (kind < 0 || kind >= K_COUNT) return "";
  return kKindNames[kind];
}

pimd_status pimd_synchronize(pimd_ctx* c) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  HIPCHK(hipStreamSynchronize(c->s));
  return check_status(c);
}

pimd_status pimd_debug_fail_waits(pimd_ctx* c) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  static const int one = 1;   // pageable source: the copy is staged before the call returns
  HIPCHK(hipMemcpyAsync(c->w.err, &one, sizeof(int), hipMemcpyHostToDevice, c->s));
  return PIMD_OK;
}

pimd_status pimd_graph_info(pimd_ctx* c, int32_t* state, int64_t* replays) {
  if (!c) return fail(PIMD_ERR_INVALID, "context is NULL");
  if (state) *state = c->graph_state;
  if (replays) *replays = c->graph_replays;
  return PIMD_OK;
}

}  // extern "C"
