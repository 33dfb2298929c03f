// k_persistent.hip -- whole MD steps of small replicas in one launch.
//
// A replica with N <= 64 particles and d P N <= 512 coordinates fits one workgroup: each thread
// owns one coordinate (x, p, the force and its thermostat chain stay in registers), the positions
// are mirrored in LDS for the terms that couple coordinates, and the workgroup runs many MD steps
// without returning to the host.  Every replica of the batch is one workgroup of the same launch.
// Per step (velocity Verlet with massive Nose-Hoover chains, as the streaming integrator):
//   NHC(dt/2); p += F dt/2; x += p dt/m';  F = force(x);  p += F dt/2; NHC(dt/2)
// and force(x) is the whole evaluation of the multi-kernel path:
//   * per particle: end beads, E_int (Eq. 9), links, trap energy;
//   * per coordinate: interior springs (Eq. 17), trap force, Gaussian pair force of its slice
//     (Eq. 20, FP64 in both precision modes);
//   * the forward (Eq. 6) and backward (Eq. 11) recursions, one wavefront each, in the normalised
//     form of the exchange kernels (lane = row i; the columns j are added in order as they
//     complete: lane i keeps a running log-sum-exp (m_i, s_i) and the weighted sums of its
//     column points, and G_j = m_j + log s_j is only formed at the end, the term of column j
//     entering row i as exp(alpha_{i,j} + m_j - m_i) s_j);
//   * per particle: the probabilities and end-bead forces of Eqs. 12-16 from the row sums, and the
//     expected spring energy from the averaged cycle energies (closing term plus the links inside
//     the cycle: lam is the prefix of link / c, as in the exchange kernels).
// Sampled steps add the estimators (trace record) and the density histogram.  At the end the
// state and the last evaluation's end beads, links, internal energies and potentials go back to
// the workspace, so every getter of the library sees what the multi-kernel path would leave.
#include "pimd_internal.h"
#include "device_util.h"
#include "fast_exp.h"
#include "nhc.h"

namespace pimd {

constexpr int kPMaxN = kTile;       // particles per replica
constexpr int kPMaxDof = 512;       // coordinates per replica (one per thread)
constexpr int kPMaxWaves = kPMaxDof / 64;

template <int D>
struct PersistShared {
  double tab[kExpTable];
  double xs[kPMaxDof];                     // positions [D][P][N]
  double a[D][kPMaxN], b[D][kPMaxN];       // first and last beads
  double lk[kPMaxN], ei[kPMaxN];           // links (0 at the end of a species), E_int
  double g[2][kPMaxN + 1];                 // G^f, G^b, rows 0..N
  double av[2][D + 1][kPMaxN + 1];         // row averages of q_j and |p_i - q_j|^2 + lam_{i-1} - lam_j
  double fe[2][D][kPMaxN];                 // end-bead exchange forces: bead 1, bead P
  double part[kPMaxN][4];                  // per-particle trap, S and pair partial sums
  double red[8 * kPMaxWaves];
  int halt;                                // a status word was raised before the launch
};

struct PersistArgs {
  const RepDev* reps;
  double* x; double* p; double* f; double* etasum; double* veta;
  double* ends; double* link; double* eint; double* gf; double* gb;
  double* rec; double* trace; long long* tracecount;
  unsigned long long* dens; long long* denssamples;
  int* status;
  long long G;
  int P, cap, bins, sample_every, need_forces;
  double rmax;
  long long step0, nsteps;
  SyW sy;
};

// One evaluation: returns the total force on this thread's coordinate; with `est`, thread 0 ends
// with the energies {E_int sum, link sum, U_trap, U_pair, pair virial part, S - E_int sum}.
template <int D>
__device__ double persist_evaluate(PersistShared<D>& sh, const RepDev& R, int P, int t, bool own, int ca, int cj,
                                   int cl, double xv, bool est, double (&en)[6]) {
  const int N = R.n;
  const int lane = t & 63, wave = t >> 6;
  if (own) sh.xs[t] = xv;
  __syncthreads();
  // per particle: end beads, E_int, link, trap energy
  if (t < N) {
    const int l = t;
    double e_int = 0.0, lkv = 0.0, ut = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double* xa = sh.xs + c * P * N;
      double prev = xa[l];
      sh.a[c][l] = prev;
      ut += prev * prev;
      for (int j = 1; j < P; ++j) {
        const double cur = xa[j * N + l];
        const double dd = cur - prev;
        e_int += dd * dd;
        ut += cur * cur;
        prev = cur;
      }
      sh.b[c][l] = prev;
      if (l + 1 < N && l + 1 != R.na) {
        const double dl = prev - xa[l + 1];
        lkv += dl * dl;
      }
    }
    sh.ei[l] = e_int * R.c;
    sh.lk[l] = lkv * R.c;
    sh.part[l][0] = ut * 0.5 * R.mw2;
  }
  // per coordinate: interior springs, trap, pair term of the slice
  double fs = 0.0, fp = 0.0, U = 0.0, W = 0.0;
  if (own) {
    const double* xa = sh.xs + ca * P * N;
    if (cj >= 1 && cj <= P - 2) fs = -R.kappa * (2.0 * xv - xa[(cj + 1) * N + cl] - xa[(cj - 1) * N + cl]);
    fs -= R.trap_p * xv;
    if (R.amp > 0.0) {
      const double inv_s = 1.0 / R.width;
      double xi[D];
#pragma unroll
      for (int c = 0; c < D; ++c) xi[c] = sh.xs[(c * P + cj) * N + cl] * inv_s;
      double F = 0.0;
      for (int m = 0; m < N; ++m) {
        double dv[D], r2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          dv[c] = xi[c] - sh.xs[(c * P + cj) * N + m] * inv_s;
          r2 = fma(dv[c], dv[c], r2);
        }
        const double u = fast_exp(-r2, sh.tab);
        F = fma(u, dv[ca], F);
        if (m != cl) {
          U += u;
          W = fma(u, r2, W);
        }
      }
      fp = 2.0 * R.amp / ((double)P * R.width) * F;
    }
  }
  __syncthreads();
  // recursions: wave 0 forward, wave 1 backward; lane = row i = lane + 1
  if (wave < 2) {
    const int dir = wave, i = lane + 1;
    const int bnd = dir == 0 ? R.na : N - R.na;
    const double bc = R.beta * R.c;
    double pi[D], rho = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) pi[c] = 0.0;
    if (i <= N) {
      if (dir == 0) {
#pragma unroll
        for (int c = 0; c < D; ++c) pi[c] = sh.b[c][i - 1];
        rho = R.beta * sh.lk[i - 1] - log((double)(i > bnd ? i - bnd : i));
      } else {
#pragma unroll
        for (int c = 0; c < D; ++c) pi[c] = sh.a[c][N - i];
        rho = i < N ? R.beta * sh.lk[N - i - 1] : 0.0;
      }
    }
    // lam of column `lane` (forward: prefix of link / c; backward: zero); row i = lane + 1 takes
    // lam_{i-1} = its own lane's value
    double lrow = (dir == 0 && lane >= 1 && lane < N) ? sh.lk[lane - 1] / R.c : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double tl = __shfl_up(lrow, off, 64);
      if (lane >= off) lrow += tl;
    }
    double m = -INFINITY, s = 0.0, Pq[D + 1];
#pragma unroll
    for (int q = 0; q <= D; ++q) Pq[q] = 0.0;
    double mj = 0.0, sj = 1.0;   // column 0: G_0 = 0
    for (int j = 0; j < N; ++j) {
      if (j > 0) {
        mj = read_lane(m, j - 1);
        sj = read_lane(s, j - 1);
      }
      double q[D], gam;
      if (dir == 0) {
#pragma unroll
        for (int c = 0; c < D; ++c) q[c] = sh.a[c][j];
        gam = 0.0;
      } else {
#pragma unroll
        for (int c = 0; c < D; ++c) q[c] = sh.b[c][N - j - 1];
        gam = -log((double)(j < bnd ? bnd - j : N - j));
      }
      const double lamj = read_lane(lrow, j);
      if (lane >= j && i <= N && (i <= bnd || j >= bnd)) {
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) { const double tq = pi[c] - q[c]; d2 = fma(tq, tq, d2); }
        const double cterm = fma(-bc, d2, rho + gam + mj) + xi_pow_log(i - 1 - j, R.lnxi);
        if (cterm > -INFINITY) {
          const double dl = cterm - m;
          const double ex = fast_exp(-fabs(dl), sh.tab);
          const double pv = d2 + (lrow - lamj);
          if (dl > 0.0) {
            s = fma(s, ex, sj);
#pragma unroll
            for (int c = 0; c < D; ++c) Pq[c] = fma(Pq[c], ex, sj * q[c]);
            Pq[D] = fma(Pq[D], ex, sj * pv);
            m = cterm;
          } else {
            const double w = ex * sj;
            s += w;
#pragma unroll
            for (int c = 0; c < D; ++c) Pq[c] = fma(w, q[c], Pq[c]);
            Pq[D] = fma(w, pv, Pq[D]);
          }
        }
      }
    }
    if (i <= N) {
      sh.g[dir][i] = m + log(s);
      const double inv = 1.0 / s;
#pragma unroll
      for (int q = 0; q <= D; ++q) sh.av[dir][q][i] = Pq[q] * inv;
    }
    if (lane == 0) sh.g[dir][0] = 0.0;
  }
  __syncthreads();
  // per particle: row factors, Eq. 13 links, end-bead forces (as the probability reduction)
  if (t < N) {
    const int l = t;
    const double* g0 = sh.g[0];
    const double* g1 = sh.g[1];
    const double GN = g0[N];
    const double w_end = exp(g0[l + 1] + g1[N - 1 - l] - GN - R.beta * sh.lk[l]);
    const double w_start = exp(g1[N - l] + g0[l] - GN - (l > 0 ? R.beta * sh.lk[l - 1] : 0.0));
    const double pn = (l >= N - 1 || l == R.na - 1) ? 0.0 : -expm1(g0[l + 1] + g1[N - 1 - l] - GN - R.beta * sh.lk[l]);
    const double pp = (l == 0 || l - 1 == R.na - 1) ? 0.0 : -expm1(g0[l] + g1[N - l] - GN - R.beta * sh.lk[l - 1]);
    const double rs = w_end + pn, cs = w_start + pp;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double ra = w_end * sh.av[0][c][l + 1];
      double cb = w_start * sh.av[1][c][N - l];
      if (pn != 0.0) ra = fma(pn, sh.a[c][l + 1], ra);
      if (pp != 0.0) cb = fma(pp, sh.b[c][l - 1], cb);
      const double rP1 = sh.xs[(c * P + (P - 2)) * N + l];
      const double r2 = sh.xs[(c * P + 1) * N + l];
      sh.fe[1][c][l] = -R.kappa * (rs * (2.0 * sh.b[c][l] - rP1) - ra);
      sh.fe[0][c][l] = -R.kappa * (cs * (2.0 * sh.a[c][l] - r2) - cb);
    }
    sh.part[l][1] = w_end * R.c * sh.av[0][D][l + 1];
  }
  __syncthreads();
  if (own) {
    if (cj == P - 1) fs += sh.fe[1][ca][cl];
    if (cj == 0) fs += sh.fe[0][ca][cl];
  }
  if (est) {
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (t < N) { v[0] = sh.ei[t]; v[1] = sh.lk[t]; v[2] = sh.part[t][0]; v[5] = sh.part[t][1]; }
    if (own && ca == 0) { v[3] = U; v[4] = U - W; }
    block_sum<6>(v, sh.red);
    if (t == 0) {
      en[0] = v[0]; en[1] = v[1]; en[2] = v[2];
      en[3] = 0.5 * R.amp * v[3];
      en[4] = 0.5 * R.amp * v[4];
      en[5] = v[5];
    }
  }
  return fs + fp;
}

template <int D, int M>
__global__ __launch_bounds__(kPMaxDof) void k_persistent(PersistArgs A) {
  __shared__ PersistShared<D> sh;
  const int r = blockIdx.x;
  const RepDev& R = A.reps[r];
  const int N = R.n, P = A.P, PN = P * N;
  const int t = threadIdx.x;
  const int ndof = D * PN;
  const bool own = t < ndof;
  const int ca = own ? t / PN : 0, cj = own ? (t / N) % P : 0, cl = own ? t % N : 0;
  const long long gi = R.dof + t;
  const long long G = A.G;
  fill_exp_table(sh.tab);
  if (t == 0) sh.halt = status_halted(A.status) ? 1 : 0;
  // es: the sum of this coordinate's chain positions (they only enter H', so one number per
  // coordinate is kept instead of one per chain element; it stays with the thread across launches)
  double xv = 0.0, pv = 0.0, fv = 0.0, es = 0.0, v[M > 0 ? M : 1];
#pragma unroll
  for (int k = 0; k < (M > 0 ? M : 1); ++k) v[k] = 0.0;
  if (own) {
    xv = A.x[gi];
    pv = A.p[gi];
    fv = A.f[gi];
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = A.veta[k * G + gi];
    if (M > 0) es = A.etasum[R.es0 + t];
  }
  __syncthreads();
  if (sh.halt) return;   // a halted run advances no further (uniform over the workgroup)
  double en[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (A.need_forces) fv = persist_evaluate<D>(sh, R, P, t, own, ca, cj, cl, xv, false, en);
  const double hdt = 0.5 * R.dt;
  for (long long it = 0; it < A.nsteps; ++it) {
    const long long stp = A.step0 + it + 1;
    const bool smp = A.sample_every > 0 && (stp % A.sample_every == 0);
    if (own) {
      if (M > 0) nhc_propagate<false>(pv, R.inv_mp, es, v, M, R.inv_q, R.kT, hdt, A.sy);
      pv += hdt * fv;
      xv += R.dt_mp * pv;
    }
    fv = persist_evaluate<D>(sh, R, P, t, own, ca, cj, cl, xv, smp, en);
    if (own) {
      pv += hdt * fv;
      if (M > 0) nhc_propagate<false>(pv, R.inv_mp, es, v, M, R.inv_q, R.kT, hdt, A.sy);
    }
    if (smp) {
      double kv[2] = {0.0, 0.0};
      if (own) {
        kv[0] = 0.5 * pv * pv / R.mp;
#pragma unroll
        for (int k = 0; k < M; ++k) kv[1] += 0.5 * R.q * v[k] * v[k];
        kv[1] += R.kT * es;
      }
      block_sum<2>(kv, sh.red);
      if (t == 0) {
        const double eint = en[0], lkv = en[1], ut = en[2], up = en[3], wp = en[4];
        const double S = eint + en[5];
        const double V = eint + lkv - sh.g[0][N] / R.beta;
        const double U = ut + up;
        double o[kRec];
        o[kVExch] = V;
        o[kUTrap] = ut;
        o[kUPair] = up;
        o[kSpring] = S;
        o[kVirial] = 2.0 * ut + wp;
        o[kEPrim] = (double)D * N * P / (2.0 * R.beta) - S + U / (double)P;
        o[kEVir] = (2.0 * ut + wp) / (double)P;
        o[kKinetic] = kv[0];
        o[kNhcE] = kv[1];
        o[kHCons] = kv[0] + V + U / (double)P + kv[1];
        o[kStep] = (double)stp;
        o[kEintSum] = eint;
        o[kLinkSum] = lkv;
        o[kPairW] = wp;
        o[kValid] = 1.0;
        o[kRecPad] = 0.0;
        double* orec = A.rec + (long long)kRec * r;
        for (int k = 0; k < kRec; ++k) orec[k] = o[k];
        if (A.cap > 0) {
          const long long c = A.tracecount[r];
          double* tr = A.trace + ((long long)r * A.cap + (c % A.cap)) * kRec;
          for (int k = 0; k < kRec; ++k) tr[k] = o[k];
          A.tracecount[r] = c + 1;
        }
        A.denssamples[r] += 1;
      }
      // density: every bead once (the thread of its first coordinate), |r| as the density kernel
      if (own && ca == 0) {
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const double xc = sh.xs[(c * P + cj) * N + cl];
          r2 = __dadd_rn(r2, __dmul_rn(xc, xc));
        }
        const double rr = __dsqrt_rn(r2);
        int bin = (rr < A.rmax) ? (int)__dmul_rn(__ddiv_rn(rr, A.rmax), (double)A.bins) : A.bins;
        if (bin < 0) bin = 0;
        if (bin > A.bins) bin = A.bins;
        atomicAdd(A.dens + (long long)r * (A.bins + 1) + bin, 1ull);
      }
      __syncthreads();   // the next evaluation rewrites the positions in LDS
    }
  }
  // state and the last evaluation back to the workspace; a non-finite value raises the status word
  if (own) {
    if (!isfinite(xv) || !isfinite(pv) || !isfinite(fv)) status_nonfinite(A.status, r);
    A.x[gi] = xv;
    A.p[gi] = pv;
    A.f[gi] = fv;
#pragma unroll
    for (int k = 0; k < M; ++k) A.veta[k * G + gi] = v[k];
    if (M > 0) A.etasum[R.es0 + t] = es;
  }
  if (!A.need_forces && A.nsteps == 0) return;   // no evaluation ran: nothing more to store
  if (t < N) {
    double* a_out = A.ends + 2LL * D * R.part;
    double* b_out = a_out + (long long)D * R.npp;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      a_out[(long long)c * R.npp + t] = sh.a[c][t];
      b_out[(long long)c * R.npp + t] = sh.b[c][t];
    }
    A.link[R.part + t] = sh.lk[t];
    A.eint[R.part + t] = sh.ei[t];
  }
  if (t <= N) {
    A.gf[R.part + t] = sh.g[0][t];
    A.gb[R.part + t] = sh.g[1][t];
  }
}

bool persistent_fits(int D, int P, int n) { return n >= 1 && n <= kPMaxN && D * P * n <= kPMaxDof; }

hipError_t launch_persistent(const Dims& d, const DevPtrs& w, int maxdof, long long step0, long long nsteps,
                             int sample_every, bool need_forces, hipStream_t s) {
  PersistArgs A;
  A.reps = w.reps;
  A.x = w.x; A.p = w.p; A.f = w.f; A.etasum = w.etasum; A.veta = w.veta;
  A.ends = w.ends; A.link = w.link; A.eint = w.eint; A.gf = w.gf; A.gb = w.gb;
  A.rec = w.rec; A.trace = w.trace; A.tracecount = w.tracecount;
  A.dens = w.dens; A.denssamples = w.denssamples;
  A.status = w.err;
  A.G = d.G;
  A.P = d.P; A.cap = d.cap; A.bins = d.bins; A.sample_every = sample_every; A.need_forces = need_forces ? 1 : 0;
  A.rmax = d.rmax;
  A.step0 = step0; A.nsteps = nsteps;
  A.sy = sy_weights(d.sy_order);
  const int threads = std::max(128, (maxdof + 63) / 64 * 64);
  dim3 grid((unsigned)d.R), block((unsigned)threads);
#define L(DD, MM) hipLaunchKernelGGL((k_persistent<DD, MM>), grid, block, 0, s, A)
#define LM(DD)                                                                            \
  switch (d.M) {                                                                          \
    case 0: L(DD, 0); break; case 1: L(DD, 1); break; case 2: L(DD, 2); break;            \
    case 3: L(DD, 3); break; case 4: L(DD, 4); break; case 5: L(DD, 5); break;            \
    case 6: L(DD, 6); break; case 7: L(DD, 7); break; case 8: L(DD, 8); break;            \
    default: return hipErrorInvalidValue;                                                 \
  }
  switch (d.D) {
    case 1: LM(1); break;
    case 2: LM(2); break;
    case 3: LM(3); break;
    default: return hipErrorInvalidValue;
  }
#undef LM
#undef L
  return hipGetLastError();
}

}  // namespace pimd
