// Density optimisation of libskx: reductions that close each evaluation,
// and a preconditioned compact limited-memory BFGS on sqrt(n) with the
// electron-count constraint, driven by a per-solve state machine so that a
// batch of solves advances with one fixed kernel sequence (no host decision
// per step).
//
// The paper minimises the free energy at fixed electron number ("SCF
// iterations", Methods, Table A caption) without naming the algorithm.
// Reading used here: L-BFGS on the sphere int phi^2 = N_e,
//   r = dE/dphi - 2 mu phi,  mu = int phi dE/dphi / (2 N_e),
//   d = -H r, H the L-BFGS inverse Hessian of the last m pairs with initial
//       matrix H0 = gamma P, P(G) = 1/(G^2 + kappa) (kinetic preconditioner,
//       kappa the Thomas-Fermi curvature 4 n0 dmu0/dn of the uniform gas)
//       and gamma = s.y / y.P y of the newest pair,
//   d <- d + kappa' phi, kappa' making d tangent to the sphere,
//   phi(t) = cos(t) phi + sin(t) sqrt(N_e) d/|d|,
//   t0 = min(|d|/sqrt(N_e), t_max), backtracking Armijo with quadratic
//   interpolation, rounding-level energy changes accepted.
// Compact form (same operator as the two-loop recursion with H0 = gamma P):
//   H r = gamma P r + S a - gamma (P Y) p,  p = R^-1 S^T r,
//   a = R^-T ((D + gamma Y^T P Y) p - gamma (P Y)^T r),
//   R = upper(S^T Y), D = diag(S^T Y).
// Only S and P Y are stored; y = r_t - r and P y = P r_t - P r are formed
// on the fly from the residual pair and its preconditioned pair.
#include "skx_device.hpp"
#include <math.h>

namespace skx {


// The control state of one solve is staged in LDS for the serial part of
// each finalize kernel, so that thread 0 works at LDS latency instead of a
// chain of dependent global-memory round trips; every thread copies one
// slice in and out (the state is at most 256 doubles), its load in flight
// together with the kernel's partial-sum loads.
static_assert(sizeof(OptState) % 8 == 0, "OptState is copied as doubles");
constexpr int NSTATE = (int)(sizeof(OptState) / 8);
static_assert(NSTATE <= 256, "one state slice per thread");
__device__ __forceinline__ double state_slice(const OptState *src, int tid) {
  return tid < NSTATE ? reinterpret_cast<const double *>(src)[tid] : 0.0;
}
__device__ __forceinline__ void put_slice(OptState *dst, int tid, double v) {
  if (tid < NSTATE) reinterpret_cast<double *>(dst)[tid] = v;
}

// Per-thread sums of the partial rows r = tid, tid + 256, ... (N values per
// row); the workgroup sum follows in block_reduce.
template <int N, int OFF, int TOT>
__device__ __forceinline__ void row_sums(const double *part, int nrow, int tid, double (&v)[TOT]) {
#pragma unroll
  for (int q = 0; q < N; ++q) v[OFF + q] = 0.0;
  for (int r = tid; r < nrow; r += 256)
#pragma unroll
    for (int q = 0; q < N; ++q) v[OFF + q] += part[r * N + q];
}

// Direction d = -P r + kappa' phi (history dropped).
__device__ void set_steepest(OptState *st, double ne) {
  st->k = 0;
  st->head = 0;
  st->gamma = 1.0;
  st->cr = -1.0;
  for (int i = 0; i < MMAX; ++i) { st->cS[i] = 0.0; st->cY[i] = 0.0; }
  st->cphi = st->phiPr / ne;
}

// ---------------------------------------------------------------------------
// Close an evaluation: energies, mu, and the line-search decision.
// ---------------------------------------------------------------------------
__device__ void finalize_eval_body(OptState *st, const SKX_C SolveDev &S, const double *tA,
                                   const double *tB, const double *tC, int ph) {
  const double PI = 3.14159265358979323846;
  double e[12];
  e[E_TF] = S.dV * tA[0];
  e[E_XC] = S.dV * tA[1];
  e[E_NELEC] = S.dV * tA[2];
  e[E_VW] = 0.5 * S.V * tB[0];
  e[E_H] = 0.5 * S.V * 4.0 * PI * tB[1];
  e[E_NL0] = S.V * tB[2];
  e[E_NL1] = S.beta * S.V / 3.0 * tB[3];
  e[E_LOC] = S.V * tB[4];
  e[E_FREE] = e[E_TF] + e[E_VW] + e[E_NL0] + e[E_NL1] + e[E_H] + e[E_LOC] + e[E_XC];
  e[E_MU] = S.dV * tC[0] / (2.0 * S.ne);
  const double bad = tA[3] + tB[5] + tC[1];
  const bool finite = (bad == 0.0) && (e[E_FREE] == e[E_FREE]) && fabs(e[E_FREE]) < 1e300;
  e[E_NONFINITE] = finite ? 0.0 : 1.0;
  e[E_SPARE] = 0.0;
  for (int q = 0; q < 12; ++q) st->e_trial[q] = e[q];
  st->evals += 1;
  if (ph == PH_EVAL_ONLY) { st->phase = PH_IDLE; return; }
  if (ph == PH_EVAL_INIT) {
    if (!finite) { st->phase = PH_FAILED; st->status = -5; return; }
    st->Et = e[E_FREE];
    st->mut = e[E_MU];
    st->phase = PH_UPDATE;
    return;
  }
  // trial point of the line search
  const double Et = e[E_FREE];
  const double tolE = st->tolE_rel * fmax(1.0, fabs(st->E));
  if (finite && Et <= st->E + st->c1 * st->theta * st->g0 + tolE) {
    st->Et = Et;
    st->mut = e[E_MU];
    st->phase = PH_UPDATE;
    return;
  }
  st->trials += 1;
  if (!finite) {
    st->theta *= 0.1;
  } else {
    const double den = 2.0 * (Et - st->E - st->g0 * st->theta);
    double tn = (den > 0.0) ? -st->g0 * st->theta * st->theta / den : 0.5 * st->theta;
    tn = fmin(fmax(tn, 0.1 * st->theta), 0.5 * st->theta);
    st->theta = tn;
  }
  if (st->trials >= st->max_trials) {
    if (st->k > 0) {
      set_steepest(st, S.ne);
      st->resets += 1;
      st->trials = 0;
      st->phase = PH_NEED_DIR;
    } else {
      st->phase = PH_FAILED;
      st->status = finite ? 1 : -5;
    }
  }
}

__global__ __launch_bounds__(256) void k_finalize_eval(SolveDev *dev, int nsolve) {
  constexpr int NP = PART_A + PART_B + PART_C;
  __shared__ double sh[4 * NP];
  __shared__ double t[NP];
  __shared__ OptState lst;
  const int s = blockIdx.x;
  if (s >= nsolve) return;
  const SKX_C SolveDev &S = *cptr<SolveDev>(dev + s);
  OptState *st = S.st;
  const int ph = cptr<OptState>(st)->phase;
  if (!(ph == PH_EVAL_INIT || ph == PH_TRIAL || ph == PH_EVAL_ONLY)) return;
  const int tid = threadIdx.x;
  const double sv = state_slice(st, tid);
  double v[NP];
  row_sums<PART_A, 0>(S.partA, S.nwg_vec, tid, v);
  row_sums<PART_B, PART_A>(S.partB, S.n2 * S.nkb, tid, v);
  row_sums<PART_C, PART_A + PART_B>(S.partC, S.rowsC, tid, v);
  put_slice(&lst, tid, sv);
  block_reduce<NP>(v, sh, tid, 256, t);
  if (tid == 0) finalize_eval_body(&lst, S, t, t + PART_A, t + PART_A + PART_B, ph);
  __syncthreads();
  put_slice(st, tid, tid < NSTATE ? reinterpret_cast<const double *>(&lst)[tid] : 0.0);
}

// ---------------------------------------------------------------------------
// Update pass: the new pair (s, P y) and every inner product the compact
// L-BFGS needs, in one sweep over the history. Reads the current point
// (buffers par) and the accepted trial point (buffers 1 - par).
// ---------------------------------------------------------------------------
// H is the storage type of the history S, P Y: the field type, or FP32
// for FP64 fields of a mixed-precision solve. Every inner product that
// involves a history vector is taken with the stored (rounded) values, the
// new pair's included, so the compact matrices describe exactly the pairs
// the direction pass reads back.
template <typename R, typename H, int NT, int MM>
__device__ __forceinline__ void update_body(const SolveDev &S, const SKX_C OptState *st, int wl,
                                            int tid, double *sh, double *tot) {
  const long long g0 = (long long)wl * S.uchunk;
  const long long g1 = min((long long)S.M, g0 + S.uchunk);
  const int par = st->par;
  const SKX_G R *phi = gptr<R>(S.phi2[par]);
  const SKX_G R *phit = gptr<R>(S.phi2[1 - par]);
  const SKX_G R *r = gptr<R>(S.r2[par]);
  const SKX_G R *rt = gptr<R>(S.r2[1 - par]);
  const SKX_G R *pr = gptr<R>(S.pr2[par]);
  const SKX_G R *prt = gptr<R>(S.pr2[1 - par]);
  SKX_G H *Sv = gptr<H>(S.S);
  SKX_G H *Yv = gptr<H>(S.Y);
  // MM = largest history length of the batch: at most KO = MM - 1 old pairs
  // take part, so only NA sums are carried (laid out in blocks of KO, then
  // the ten new-pair sums) and scattered to the MMAX layout at the end
  constexpr int KO = MM - 1, NA = 6 * KO + 10;
  double acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = 0.0;
  // acc layout: [i] s_i.y, [M+i] Py_i.y, [2M+i] s_i.r_t, [3M+i] Py_i.r_t,
  // [4M+i] s_i.phi_t, [5M+i] Py_i.phi_t (old pairs), then at B = 6M:
  // s.y, y.Py, s.r_t, Py.r_t, s.phi_t, Py.phi_t, r_t.r_t, r_t.Pr_t,
  // phi_t.Pr_t, r_t.phi_t
  const int B = 6 * KO;
  if (st->reset_pending == 1) {
    // first accepted point: residual inner products only
    for (long long g = g0 + tid; g < g1; g += NT) {
      const double a = rt[g], b = prt[g], f = phit[g];
      acc[B + 6] += a * a;
      acc[B + 7] += a * b;
      acc[B + 8] += f * b;
      acc[B + 9] += a * f;
    }
  } else {
    const int m = st->m, k = st->k, head = st->head;
    const int kold = (k == m) ? m - 1 : k;
    int slot[KO > 0 ? KO : 1];
#pragma unroll
    for (int i = 0; i < KO; ++i) slot[i] = (i < kold) ? ((head - kold + i + 2 * m) % m) : 0;
    SKX_G H *Snew = Sv + (size_t)head * S.M;
    SKX_G H *Ynew = Yv + (size_t)head * S.M;
    for (long long g = g0 + tid; g < g1; g += NT) {
      const R pt = phit[g], rtg = rt[g], prtg = prt[g];
      const H svh = (H)(pt - phi[g]);
      const R yv = rtg - r[g];
      const H pyh = (H)(prtg - pr[g]);
      const double sv = (double)svh, pyv = (double)pyh;
#pragma unroll
      for (int i = 0; i < KO; ++i) {
        if (i < kold) {
          const double Si = (double)Sv[(size_t)slot[i] * S.M + g];
          const double Yi = (double)Yv[(size_t)slot[i] * S.M + g];
          acc[i] += Si * yv;
          acc[KO + i] += Yi * yv;
          acc[2 * KO + i] += Si * rtg;
          acc[3 * KO + i] += Yi * rtg;
          acc[4 * KO + i] += Si * pt;
          acc[5 * KO + i] += Yi * pt;
        }
      }
      acc[B + 0] += sv * yv;
      acc[B + 1] += (double)yv * pyv;
      acc[B + 2] += sv * rtg;
      acc[B + 3] += pyv * rtg;
      acc[B + 4] += sv * pt;
      acc[B + 5] += pyv * pt;
      acc[B + 6] += (double)rtg * rtg;
      acc[B + 7] += (double)rtg * prtg;
      acc[B + 8] += (double)pt * prtg;
      acc[B + 9] += (double)rtg * pt;
      Snew[g] = svh;
      Ynew[g] = pyh;
    }
  }
  block_reduce_many<NA>(acc, sh, tid, NT, tot);
  if (tid < NDOT) {
    double v;
    if (tid < 6 * MMAX) {
      const int blk = tid / MMAX, i = tid - blk * MMAX;
      v = (i < KO) ? tot[blk * KO + i] : 0.0;
    } else {
      v = tot[6 * KO + tid - 6 * MMAX];
    }
    S.partU[wl * NDOT + tid] = v;
  }
}

template <typename R, int NT, int MM>
__global__ __launch_bounds__(NT) void k_update(SolveDev *dev, const int *first, int nsolve,
                                               int grid) {
  __shared__ double sh[64 * (NT / 64)];
  __shared__ double tot[NDOT];
  const int item = blockIdx.x;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (st->phase != PH_UPDATE) return;
  const int wl = item - first_of(first, s);
  if (sizeof(R) == 8 && S.hist32)
    update_body<R, float, NT, MM>(S, st, wl, threadIdx.x, sh, tot);
  else
    update_body<R, R, NT, MM>(S, st, wl, threadIdx.x, sh, tot);
}

// t holds the NDOT sums of the update pass, already scaled by dV; the
// caller has copied e_trial to e_acc. The history blocks and vectors are
// worked on as register copies whose every index is fixed at compile time
// (loops to MM, the batch's largest history length, with guards), so no
// step waits on a chain of LDS loads.
template <int MM>
__device__ void finalize_update_body(OptState *st, const SKX_C SolveDev &S, const double *t) {
  const int B = 6 * MMAX;
  const int m = st->m;
  st->E = st->Et;
  st->mu = st->mut;
  st->par = 1 - st->par;            // the trial point becomes the current point
  st->rr = t[B + 6];
  st->rPr = t[B + 7];
  st->phiPr = t[B + 8];
  st->rphi = t[B + 9];
  // upper triangles only (SY is used there, YPY is symmetric); the
  // vectors are refilled from t below the history length
  double SY[MM][MM], YPY[MM][MM], Sr[MM], YPr[MM], Sphi[MM], PYphi[MM];
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    Sr[i] = 0.0;
    YPr[i] = 0.0;
    Sphi[i] = 0.0;
    PYphi[i] = 0.0;
#pragma unroll
    for (int j = i; j < MM; ++j) {
      SY[i][j] = st->SY[i][j];
      YPY[i][j] = st->YPY[i][j];
    }
  }
  int k = st->k;
  if (st->reset_pending == 1) {
    st->reset_pending = 0;
    set_steepest(st, S.ne);
    k = 0;
  } else {
    st->iters += 1;
    if (k == m) {
      // the oldest pair's memory now holds the new pair: drop it
#pragma unroll
      for (int i = 0; i + 1 < MM; ++i)
#pragma unroll
        for (int j = i; j + 1 < MM; ++j) {
          SY[i][j] = SY[i + 1][j + 1];
          YPY[i][j] = YPY[i + 1][j + 1];
        }
      k = m - 1;
    }
#pragma unroll
    for (int i = 0; i < MM; ++i)
      if (i < k) {
        Sr[i] = t[2 * MMAX + i];
        YPr[i] = t[3 * MMAX + i];
        Sphi[i] = t[4 * MMAX + i];
        PYphi[i] = t[5 * MMAX + i];
      }
    const double sy = t[B + 0], ypy = t[B + 1];
    const bool ok = (sy > 0.0) && (ypy > 0.0) && (sy == sy) && (ypy == ypy);
    if (ok) {
#pragma unroll
      for (int c = 0; c < MM; ++c)
        if (c == k) {
#pragma unroll
          for (int i = 0; i < MM; ++i)
            if (i < c) {
              SY[i][c] = t[i];
              YPY[i][c] = t[MMAX + i];
            }
          SY[c][c] = sy;
          YPY[c][c] = ypy;
          Sr[c] = t[B + 2];
          YPr[c] = t[B + 3];
          Sphi[c] = t[B + 4];
          PYphi[c] = t[B + 5];
        }
      k += 1;
      st->head = (st->head + 1) % m;
    }
    st->k = k;
    st->pair_ok = ok ? 1 : 0;
  }
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    st->Sr[i] = Sr[i];
    st->YPr[i] = YPr[i];
    st->Sphi[i] = Sphi[i];
    st->PYphi[i] = PYphi[i];
#pragma unroll
    for (int j = i; j < MM; ++j) {
      st->SY[i][j] = SY[i][j];
      st->YPY[i][j] = YPY[i][j];
    }
  }
  st->rnorm = sqrt(fmax(st->rr, 0.0));
  if (!(st->rnorm == st->rnorm)) { st->phase = PH_FAILED; st->status = -5; return; }
  if (st->rnorm < st->gtol) { st->phase = PH_DONE; st->status = 0; return; }
  if (st->iters >= st->max_iter) { st->phase = PH_DONE; st->status = 1; return; }
  if (st->stall_limit > 0) {
    // low-precision phase: stop once the residual no longer improves
    if (st->rnorm < st->stall_factor * st->best_r) { st->best_r = st->rnorm; st->stall = 0; }
    else if (++st->stall >= st->stall_limit) { st->phase = PH_DONE; st->status = 2; return; }
  }
  // compact L-BFGS coefficients, H0 = gamma P
  if (k == 0) {
    set_steepest(st, S.ne);
    st->phase = PH_NEED_DIR;
    return;
  }
  double gamma = 1.0;
#pragma unroll
  for (int c = 0; c < MM; ++c)
    if (c == k - 1) gamma = SY[c][c] / YPY[c][c];
  double p[MM], z[MM], a[MM];
#pragma unroll
  for (int i = MM - 1; i >= 0; --i) {
    double v = Sr[i];
#pragma unroll
    for (int j = i + 1; j < MM; ++j)
      if (j < k) v -= SY[i][j] * p[j];
    p[i] = i < k ? v / SY[i][i] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    double v = SY[i][i] * p[i] - gamma * YPr[i];
#pragma unroll
    for (int j = 0; j < MM; ++j)
      if (j < k) v += gamma * (i <= j ? YPY[i][j] : YPY[j][i]) * p[j];
    z[i] = v;
  }
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    double v = z[i];
#pragma unroll
    for (int j = 0; j < i; ++j) v -= SY[j][i] * a[j];
    a[i] = i < k ? v / SY[i][i] : 0.0;
  }
  double dphi = -gamma * st->phiPr;
  double rd = -gamma * st->rPr;
#pragma unroll
  for (int i = 0; i < MM; ++i)
    if (i < k) {
      dphi += -a[i] * Sphi[i] + gamma * p[i] * PYphi[i];
      rd += -a[i] * Sr[i] + gamma * p[i] * YPr[i];
    }
  const double kap = -dphi / S.ne;
  rd += kap * st->rphi;
  if (!(rd < 0.0)) {
    set_steepest(st, S.ne);
    st->resets += 1;
  } else {
    st->gamma = gamma;
    st->cr = -gamma;
#pragma unroll
    for (int i = 0; i < MMAX; ++i) {
      st->cS[i] = (i < k && i < MM) ? -a[i < MM ? i : 0] : 0.0;
      st->cY[i] = (i < k && i < MM) ? gamma * p[i < MM ? i : 0] : 0.0;
    }
    st->cphi = kap;
  }
  st->phase = PH_NEED_DIR;
}

template <int MM>
__global__ __launch_bounds__(256) void k_finalize_update(SolveDev *dev, int nsolve) {
  __shared__ double sh[64 * 4];
  __shared__ double t[NDOT];
  __shared__ OptState lst;
  const int s = blockIdx.x;
  if (s >= nsolve) return;
  const SKX_C SolveDev &S = *cptr<SolveDev>(dev + s);
  OptState *st = S.st;
  if (cptr<OptState>(st)->phase != PH_UPDATE) return;
  const int tid = threadIdx.x;
  const double sv = state_slice(st, tid);
  {
    double v[NDOT];
    row_sums<NDOT, 0>(S.partU, S.nwg_upd, tid, v);
    put_slice(&lst, tid, sv);
    block_reduce_many<NDOT>(v, sh, tid, 256, t);
  }
  if (tid < NDOT) t[tid] *= S.dV;
  if (tid < 12) lst.e_acc[tid] = lst.e_trial[tid];
  __syncthreads();
  if (tid == 0) finalize_update_body<MM>(&lst, S, t);
  __syncthreads();
  put_slice(st, tid, tid < NSTATE ? reinterpret_cast<const double *>(&lst)[tid] : 0.0);
}

// ---------------------------------------------------------------------------
// Direction pass: d = cr P r + sum cS_i s_i + sum cY_i P y_i + cphi phi,
// with |d|^2 and r.d.
// ---------------------------------------------------------------------------
template <typename R, typename H, int NT, int MM>
__device__ __forceinline__ void dir_body(const SolveDev &S, const SKX_C OptState *st, int wl,
                                         int tid, double *sh, double *tot) {
  const long long g0 = (long long)wl * CHUNK;
  const long long g1 = min((long long)S.M, g0 + CHUNK);
  const int par = st->par;
  const SKX_G R *phi = gptr<R>(S.phi2[par]);
  const SKX_G R *r = gptr<R>(S.r2[par]);
  const SKX_G R *pr = gptr<R>(S.pr2[par]);
  const SKX_G H *Sv = gptr<H>(S.S);
  const SKX_G H *Yv = gptr<H>(S.Y);
  SKX_G R *d = gptr<R>(S.d);
  const int m = st->m, k = st->k, head = st->head;
  int slot[MM];
  R cS[MM], cY[MM];
#pragma unroll
  for (int i = 0; i < MM; ++i) {
    slot[i] = (i < k) ? ((head - k + i + 2 * m) % m) : 0;
    cS[i] = (R)st->cS[i];
    cY[i] = (R)st->cY[i];
  }
  const R cr = (R)st->cr, cphi = (R)st->cphi;
  double dd = 0.0, rd = 0.0;
  for (long long g = g0 + tid; g < g1; g += NT) {
    R v = cr * pr[g] + cphi * phi[g];
#pragma unroll
    for (int i = 0; i < MM; ++i) {
      if (i < k)
        v += cS[i] * (R)Sv[(size_t)slot[i] * S.M + g] + cY[i] * (R)Yv[(size_t)slot[i] * S.M + g];
    }
    d[g] = v;
    dd += (double)v * v;
    rd += (double)r[g] * v;
  }
  double acc[2] = {dd, rd};
  block_reduce<2>(acc, sh, tid, NT, tot);
  if (tid == 0) { S.partD[wl * 2] = tot[0]; S.partD[wl * 2 + 1] = tot[1]; }
}

template <typename R, int NT, int MM>
__global__ __launch_bounds__(NT) void k_dir(SolveDev *dev, const int *first, int nsolve, int grid) {
  __shared__ double sh[2 * (NT / 64)];
  __shared__ double tot[2];
  const int item = blockIdx.x;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (st->phase != PH_NEED_DIR) return;
  const int wl = item - first_of(first, s);
  if (sizeof(R) == 8 && S.hist32)
    dir_body<R, float, NT, MM>(S, st, wl, threadIdx.x, sh, tot);
  else
    dir_body<R, R, NT, MM>(S, st, wl, threadIdx.x, sh, tot);
}

__device__ void finalize_dir_body(OptState *st, const SKX_C SolveDev &S, const double *t) {
  const double dd = S.dV * t[0], rd = S.dV * t[1];
  const double dn = sqrt(fmax(dd, 0.0));
  if (!(rd < 0.0) || !(dn > 0.0)) {
    if (st->k > 0) {
      set_steepest(st, S.ne);
      st->resets += 1;
      return;                       // stays in NEED_DIR: preconditioned steepest descent next
    }
    st->phase = PH_FAILED;
    st->status = 1;
    return;
  }
  st->dnorm = dn;
  st->rd = rd;
  st->theta = fmin(dn * S.inv_sqrt_ne, st->theta_max);
  st->g0 = rd / dn * S.sqrt_ne;
  st->trials = 0;
  st->phase = PH_TRIAL;
}

__global__ __launch_bounds__(256) void k_finalize_dir(SolveDev *dev, int nsolve) {
  __shared__ double sh[2 * 4];
  __shared__ double t[2];
  __shared__ OptState lst;
  const int s = blockIdx.x;
  if (s >= nsolve) return;
  const SKX_C SolveDev &S = *cptr<SolveDev>(dev + s);
  OptState *st = S.st;
  if (cptr<OptState>(st)->phase != PH_NEED_DIR) return;
  const int tid = threadIdx.x;
  const double sv = state_slice(st, tid);
  double v[2];
  row_sums<2, 0>(S.partD, S.nwg_vec, tid, v);
  put_slice(&lst, tid, sv);
  block_reduce<2>(v, sh, tid, 256, t);
  if (tid == 0) finalize_dir_body(&lst, S, t);
  __syncthreads();
  put_slice(st, tid, tid < NSTATE ? reinterpret_cast<const double *>(&lst)[tid] : 0.0);
}

// ---------------------------------------------------------------------------
// Normalisation of the starting point: phi <- phi sqrt(N_e / int phi^2).
// With reset_pending == 2 the buffer holds a density and phi = sqrt(max(rho,0)).
// ---------------------------------------------------------------------------
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_norm(SolveDev *dev, const int *first, int nsolve, int grid) {
  __shared__ double sh[2 * (NT / 64)];
  __shared__ double tot[2];
  const int item = blockIdx.x;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (st->phase != PH_EVAL_INIT) return;
  const int tid = threadIdx.x;
  const int wl = item - first_of(first, s);
  const long long g0 = (long long)wl * CHUNK;
  const long long g1 = min((long long)S.M, g0 + CHUNK);
  SKX_G R *phi = gptr<R>(S.phi2[st->par]);
  const bool from_rho = st->reset_pending == 2;
  double ss = 0.0, bad = 0.0;
  for (long long g = g0 + tid; g < g1; g += NT) {
    R v = phi[g];
    if (from_rho) {
      v = v > (R)0 ? sqrt(v) : (R)0;
      phi[g] = v;
    }
    if (!(v == v)) bad += 1.0;
    ss += (double)v * v;
  }
  double acc[2] = {ss, bad};
  block_reduce<2>(acc, sh, tid, NT, tot);
  if (tid == 0) { S.partD[wl * 2] = tot[0]; S.partD[wl * 2 + 1] = tot[1]; }
}

__device__ void finalize_norm_body(OptState *st, const SKX_C SolveDev &S, const double *t) {
  const double nrm = S.dV * t[0];
  if (t[1] != 0.0 || !(nrm > 0.0) || !(nrm < 1e300)) {
    st->phase = PH_FAILED;
    st->status = -5;
    return;
  }
  st->theta = sqrt(S.ne / nrm);
  st->reset_pending = 1;             // the first update only forms the residual
}

__global__ __launch_bounds__(256) void k_finalize_norm(SolveDev *dev, int nsolve) {
  __shared__ double sh[2 * 4];
  __shared__ double t[2];
  __shared__ OptState lst;
  const int s = blockIdx.x;
  if (s >= nsolve) return;
  const SKX_C SolveDev &S = *cptr<SolveDev>(dev + s);
  OptState *st = S.st;
  if (cptr<OptState>(st)->phase != PH_EVAL_INIT) return;
  const int tid = threadIdx.x;
  const double sv = state_slice(st, tid);
  double v[2];
  row_sums<2, 0>(S.partD, S.nwg_vec, tid, v);
  put_slice(&lst, tid, sv);
  block_reduce<2>(v, sh, tid, 256, t);
  if (tid == 0) finalize_norm_body(&lst, S, t);
  __syncthreads();
  put_slice(st, tid, tid < NSTATE ? reinterpret_cast<const double *>(&lst)[tid] : 0.0);
}

// ---------------------------------------------------------------------------
template <typename R>
static hipError_t launch_update_t(const BatchLaunch &b, hipStream_t s) {
  switch (b.mh) {
#define SKX_UPD(MM)                                                                         \
  case MM:                                                                                  \
    SKX_TIMED_LAUNCH((k_update<R, 256, MM>), dim3(b.gridU), dim3(256), 0, s, b.dev,        \
                       b.firstU, b.nsolve, b.gridU);                                        \
    SKX_TIMED_LAUNCH((k_finalize_update<MM>), dim3(b.nsolve), dim3(256), 0, s, b.dev,       \
                       b.nsolve);                                                           \
    break;
    SKX_UPD(1) SKX_UPD(2) SKX_UPD(3) SKX_UPD(4) SKX_UPD(5) SKX_UPD(6) SKX_UPD(7)
    default: SKX_UPD(8)
#undef SKX_UPD
  }
  return hipGetLastError();
}

template <typename R>
static hipError_t launch_dir_t(const BatchLaunch &b, hipStream_t s) {
  switch (b.mh) {
#define SKX_DIR(MM)                                                                         \
  case MM:                                                                                  \
    SKX_TIMED_LAUNCH((k_dir<R, 256, MM>), dim3(b.gridV), dim3(256), 0, s, b.dev, b.firstV, \
                       b.nsolve, b.gridV);                                                  \
    break;
    SKX_DIR(1) SKX_DIR(2) SKX_DIR(3) SKX_DIR(4) SKX_DIR(5) SKX_DIR(6) SKX_DIR(7)
    default: SKX_DIR(8)
#undef SKX_DIR
  }
  SKX_TIMED_LAUNCH(k_finalize_dir, dim3(b.nsolve), dim3(256), 0, s, b.dev, b.nsolve);
  return hipGetLastError();
}

template <typename R>
static hipError_t launch_norm_t(const BatchLaunch &b, hipStream_t s) {
  hipLaunchKernelGGL((k_norm<R, 256>), dim3(b.gridV), dim3(256), 0, s, b.dev, b.firstV, b.nsolve,
                     b.gridV);
  hipLaunchKernelGGL(k_finalize_norm, dim3(b.nsolve), dim3(256), 0, s, b.dev, b.nsolve);
  return hipGetLastError();
}

hipError_t launch_finalize_eval(const BatchLaunch &b, hipStream_t s) {
  SKX_TIMED_LAUNCH(k_finalize_eval, dim3(b.nsolve), dim3(256), 0, s, b.dev, b.nsolve);
  return hipGetLastError();
}

hipError_t launch_opt_update(const BatchLaunch &b, hipStream_t s) {
  return b.prec == 0 ? launch_update_t<double>(b, s) : launch_update_t<float>(b, s);
}
hipError_t launch_opt_dir(const BatchLaunch &b, hipStream_t s) {
  return b.prec == 0 ? launch_dir_t<double>(b, s) : launch_dir_t<float>(b, s);
}
hipError_t launch_normalize(const BatchLaunch &b, hipStream_t s) {
  return b.prec == 0 ? launch_norm_t<double>(b, s) : launch_norm_t<float>(b, s);
}

}  // namespace skx
