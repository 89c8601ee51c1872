// Host runtime and C ABI of libskx: contexts, device buffers, plans, the
// batched step sequence and the optimisation driver.
#include "skx_internal.hpp"
#include "skx_device.hpp"
#include "../../include/skx.h"
#include "skx_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace skx;

namespace skx {
namespace host {

// ---------------------------------------------------------------------------
// Per-device resources shared by all contexts: FFT twiddle bank and the
// universal Fermi-Dirac Chebyshev table.
// ---------------------------------------------------------------------------
constexpr double FD_Y0 = -46.0, FD_H = 1.0 / 64.0;
constexpr int FD_N = 62 * 64;                 // covers ln(n/n_T) in [-46, 16)

struct DeviceRes {
  bool ready = false;
  double *twbank = nullptr;
  int tw_off[514];
  double *fdcoef = nullptr;
  FDTable fd{};
};
DeviceRes g_res[64];
std::mutex g_mu;

bool five_smooth_even(int n) {
  if (n < 8 || n > 512 || (n & 1)) return false;
  int m = n;
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  return m == 1;
}

hipError_t init_device(int dev, std::string &err) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev < 0 || dev >= 64) { err = "device index out of range"; return hipErrorInvalidDevice; }
  DeviceRes &r = g_res[dev];
  if (r.ready) return hipSuccess;
  hipError_t e = hipSetDevice(dev);
  if (e != hipSuccess) { err = "hipSetDevice failed"; return e; }
  std::vector<int> sizes, offs;
  int off = 0;
  for (int n = 2; n <= 512; ++n) {
    r.tw_off[n] = -1;
    int m = n;
    for (int p : {2, 3, 5})
      while (m % p == 0) m /= p;
    if (m != 1) continue;
    r.tw_off[n] = off;
    sizes.push_back(n);
    offs.push_back(off);
    off += n;
  }
  e = hipMalloc((void **)&r.twbank, sizeof(double) * 2 * off);
  if (e != hipSuccess) { err = "twiddle bank allocation failed"; return e; }
  int *dsz = nullptr, *doff = nullptr;
  e = hipMalloc((void **)&dsz, sizeof(int) * sizes.size());
  if (e == hipSuccess) e = hipMalloc((void **)&doff, sizeof(int) * offs.size());
  if (e == hipSuccess) e = hipMemcpy(dsz, sizes.data(), sizeof(int) * sizes.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(doff, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = build_twiddles(r.twbank, dsz, doff, (int)sizes.size(), 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(dsz);
  (void)hipFree(doff);
  if (e != hipSuccess) { err = "twiddle kernel failed"; return e; }
  e = hipMalloc((void **)&r.fdcoef, sizeof(double) * 4 * (FD_N + 1));
  if (e != hipSuccess) { err = "FD table allocation failed"; return e; }
  e = build_fd_table(r.fdcoef, FD_Y0, FD_H, FD_N, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) { err = "FD table kernel failed"; return e; }
  r.fd.y0 = FD_Y0;
  r.fd.h = FD_H;
  r.fd.inv_h = 1.0 / FD_H;
  r.fd.n = FD_N;
  r.fd.node = r.fdcoef;
  e = init_noalloc_scratch(dev);
  if (e != hipSuccess) { err = "fixed scratch symbol lookup failed"; return e; }
  r.ready = true;
  return hipSuccess;
}

// Radix orders for a transform length: the default (radix 8 first, then 4,
// 2, 3, 5) and the alternatives the autotuner times against it.
std::vector<std::vector<int>> radix_candidates(int n) {
  auto greedy = [n](std::initializer_list<int> order) {
    std::vector<int> r;
    int m = n;
    for (int x : order)
      while (m % x == 0 && (int)r.size() < MAX_STAGES) { r.push_back(x); m /= x; }
    return r;
  };
  std::vector<std::vector<int>> c;
  c.push_back(greedy({8, 4, 2, 3, 5}));
  c.push_back(greedy({4, 2, 3, 5}));
  c.push_back(greedy({5, 3, 8, 4, 2}));
  std::vector<int> rev = c[0];
  std::reverse(rev.begin(), rev.end());
  c.push_back(rev);
  std::vector<std::vector<int>> out;
  for (auto &x : c)
    if (std::find(out.begin(), out.end(), x) == out.end()) out.push_back(x);
  return out;
}

// Radix order chosen by the autotuner per precision and length (empty: default).
std::vector<int> g_tuned[2][513];
bool g_autotune = false;
int g_shape_kernels = 7;
bool g_chunk_planes = false;

Plan make_plan_from(int n, int twoff, const std::vector<int> &rads) {
  Plan p{};
  p.n = n;
  p.tw = twoff;
  for (int r : rads) { p.rad |= (unsigned)r << (4 * p.nst); p.nst++; }
  int Ns = 1;
  for (int st = 0; st < p.nst; ++st) {
    const int r = (p.rad >> (4 * st)) & 15u;
    const unsigned nb = (unsigned)(n / r);
    p.m_nb[st] = (0xFFFFFFFFull / nb) + 1ull;
    p.m_ns[st] = (0xFFFFFFFFull / (unsigned)Ns) + 1ull;
    p.twstep[st] = n / (Ns * r);
    Ns *= r;
  }
  return p;
}

Plan make_plan(int n, int twoff, int prec) {
  const std::vector<int> &t = g_tuned[prec][n];
  return make_plan_from(n, twoff, t.empty() ? radix_candidates(n)[0] : t);
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace host
}  // namespace skx

namespace skx {
namespace host {

int fail(skx_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(skx_ctx *c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(c, SKX_E_NOMEM, m);
  return fail(c, SKX_E_DEVICE, m);
}

void free_instance(Instance &I) {
  if (I.mem) hipFree(I.mem);
  if (I.dptr) hipFree(I.dptr);
  if (I.st) hipFree(I.st);
  if (I.first) hipFree(I.first);
  I = Instance{};
}

int fields_mask(unsigned terms, double beta) {
  int f = F_N;
  if (terms & SKX_TERM_VW) f |= F_PHI;
  if (terms & (SKX_TERM_NL0 | SKX_TERM_NL1)) f |= F_F;
  if ((terms & SKX_TERM_NL1) && beta != 0.0) f |= F_H;
  return f;
}

// LDS bytes of the three passes for one solve
void lds_sizes(const SolveDev &h, int prec, size_t &a, size_t &b, size_t &c) {
  size_t v = prec == 0 ? 16 : 8;
  a = v * ((size_t)h.n2 * h.nh + h.n2 + h.n3);
  b = v * ((size_t)h.n1 * (h.nf * h.tk + 1) + h.n1);
  c = a;
  a = std::max(a, (size_t)1024);
  b = std::max(b, (size_t)1024);
  c = std::max(c, (size_t)1024);
}

constexpr size_t LDS_MAX = 160 * 1024;

// LDS bytes of the split plane kernels for one solve: a row-pair chunk of
// every field (rows of pitch 2 nh, z twiddles) and a column chunk (pitch split_cc + 1,
// y twiddles)
void split_lds(const SolveDev &h, int prec, size_t &row, size_t &col) {
  const size_t v = prec == 0 ? 16 : 8;
  row = v * ((size_t)NFIELD * h.rp * 2 * h.nh + h.n3);
  col = v * ((size_t)h.n2 * (split_cc(prec) + 1) + h.n2);
  row = std::max(row, (size_t)1024);
}

// Allocate (or reuse) the buffers of one precision instance and fill the
// descriptor's grid and buffer fields.
// Points per workgroup of the optimiser update: larger on large grids,
// where the single-block finaliser would otherwise read thousands of rows of
// partial sums.
int update_chunk(long long M) { return M >= (1LL << 20) ? UCHUNK : CHUNK; }

// Width (complex columns) of pass B's column blocks, which also aligns the
// spectrum pitch: 8 in FP64 and 16 in FP32, narrower on long x axes; for
// the cubic lengths with
// compile-time-shaped kernels 16 in FP32 only where it divides n/2, else 8.
// Where 8 does not divide n/2 either (36, 40, 50, 54, 60, 72) the shaped
// pass B takes ragged blocks over all n/2 + 1 columns.
int block_width(int n1, int n2, int n3, int prec) {
  // Pass B's workgroup holds an x tile of n1 x (NFIELD tk) complex values;
  // on long x axes narrower blocks keep it small enough for several
  // workgroups per CU (measured on MI355X, runtime-shaped pass B: FP64
  // blocks of 4 from 78 points on, 128^3 179 -> 138 us and 192^3 667 ->
  // 589 us for two solves, neutral at 96^3; FP32 blocks of 8 from 158 points
  // on, 192^3 444 -> 315 us, while at 96^3-144^3 blocks of 16 stay faster).
  const int tk = passb_width(n1, prec);
  if (n1 != n2 || n2 != n3) return tk;
  switch (n1) {
    case 36: case 40: case 48: case 50: case 54: case 60: case 64: case 72: case 80: break;
    default: return tk;
  }
  return (prec == 1 && (n1 / 2) % 16 == 0) ? 16 : 8;
}

struct ArenaLayout {
  size_t o_phi, o_phit, o_grad, o_r, o_rt, o_pr, o_prt, o_d, o_vpt, o_fpt, o_qpt, o_npa, o_S, o_Y;
  size_t o_spec, o_vloc, o_pA, o_pB, o_pC, o_pU, o_pD, total;
};

// own_hist false: no history arrays (the FP64 instance of a mixed solve
// keeps its S, P Y in the FP32 instance's arrays, stored as FP32).
ArenaLayout arena_layout(int n1, int n2, int n3, int prec, int m, bool own_hist) {
  const size_t rsz = prec == 0 ? 8 : 4;
  const int tk = block_width(n1, n2, n3, prec);
  const int nh = n3 / 2 + 1;
  const int pitch = (int)align_up(nh, tk);
  const long long M = (long long)n1 * n2 * n3;
  const long long H = (long long)n1 * n2 * pitch;
  const int nkb = (nh + tk - 1) / tk;
  const int nwg = (int)((M + CHUNK - 1) / CHUNK);
  const int nwu = (int)((M + update_chunk(M) - 1) / update_chunk(M));
  ArenaLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  L.o_phi = take(rsz * M); L.o_phit = take(rsz * M); L.o_grad = take(rsz * M);
  L.o_r = take(rsz * M); L.o_rt = take(rsz * M); L.o_pr = take(rsz * M); L.o_prt = take(rsz * M);
  L.o_d = take(rsz * M); L.o_vpt = take(rsz * M); L.o_fpt = take(rsz * M);
  L.o_qpt = take(rsz * M); L.o_npa = take(rsz * M);
  const size_t hist = own_hist ? rsz * M * m : 0;
  L.o_S = take(hist); L.o_Y = take(hist);
  L.o_spec = take(2 * rsz * H * NFIELD); L.o_vloc = take(2 * rsz * H);
  L.o_pA = take(8 * (size_t)nwg * PART_A); L.o_pB = take(8 * (size_t)n2 * nkb * PART_B);
  const int nrc = (n2 / 2 + split_rp(n3) - 1) / split_rp(n3);
  L.o_pC = take(8 * (size_t)n1 * nrc * PART_C); L.o_pU = take(8 * (size_t)nwu * NDOT);
  L.o_pD = take(8 * (size_t)nwg * 2);
  L.total = off;
  return L;
}

size_t instance_bytes(int n1, int n2, int n3, int prec, int m, bool own_hist) {
  return arena_layout(n1, n2, n3, prec, std::max(m, 1), own_hist).total +
         sizeof(SolveDev) * batch_desc_count(1) + sizeof(OptState) +
         batch_first_count(1) * sizeof(int);
}

int ensure_instance(skx_ctx *c, int prec, int m) {
  Instance &I = c->inst[prec];
  const int n1 = c->n1, n2 = c->n2, n3 = c->n3;
  const size_t rsz = prec == 0 ? 8 : 4;
  const int tk = block_width(n1, n2, n3, prec);
  const int nh = n3 / 2 + 1;
  const int pitch = (int)align_up(nh, tk);
  const long long M = (long long)n1 * n2 * n3;
  const long long H = (long long)n1 * n2 * pitch;
  const int nkb = (nh + tk - 1) / tk;
  const int nwg = (int)((M + CHUNK - 1) / CHUNK);
  if (m < 1) m = 1;
  const bool own_hist = !(prec == 0 && c->fn.precision == SKX_MIXED);
  if (I.mem && I.prec == prec && I.m_alloc >= m && I.h.n1 == n1 && I.h.n2 == n2 &&
      I.h.n3 == n3 && I.own_hist == own_hist)
    return SKX_OK;
  free_instance(I);
  (void)hipSetDevice(c->device);
  const ArenaLayout A = arena_layout(n1, n2, n3, prec, m, own_hist);
  const size_t off = A.total;
  const size_t o_phi = A.o_phi, o_phit = A.o_phit, o_grad = A.o_grad, o_r = A.o_r, o_rt = A.o_rt;
  const size_t o_pr = A.o_pr, o_prt = A.o_prt, o_d = A.o_d, o_vpt = A.o_vpt, o_fpt = A.o_fpt;
  const size_t o_qpt = A.o_qpt, o_npa = A.o_npa;
  const size_t o_S = A.o_S, o_Y = A.o_Y, o_spec = A.o_spec, o_vloc = A.o_vloc;
  const size_t o_pA = A.o_pA, o_pB = A.o_pB, o_pC = A.o_pC, o_pU = A.o_pU, o_pD = A.o_pD;
  hipError_t e = hipMalloc(&I.mem, off);
  if (e != hipSuccess) { I.mem = nullptr; return hip_fail(c, e, "device arena allocation"); }
  hipMemsetAsync(I.mem, 0, off, c->stream);
  e = hipMalloc((void **)&I.dptr, sizeof(SolveDev) * batch_desc_count(1));
  if (e == hipSuccess) e = hipMalloc((void **)&I.st, sizeof(OptState));
  if (e == hipSuccess) e = hipMalloc((void **)&I.first, sizeof(int) * batch_first_count(1));
  if (e != hipSuccess) { free_instance(I); return hip_fail(c, e, "descriptor allocation"); }
  hipMemsetAsync(I.st, 0, sizeof(OptState), c->stream);
  I.prec = prec;
  I.rsz = rsz;
  I.bytes = off;
  I.m_alloc = m;
  I.own_hist = own_hist;
  char *base = (char *)I.mem;
  SolveDev &h = I.h;
  h = SolveDev{};
  h.n1 = n1; h.n2 = n2; h.n3 = n3; h.nh = nh; h.pitch = pitch;
  h.nkb = nkb; h.tk = tk; h.nwg_vec = nwg; h.mh = m;
  h.rp = split_rp(n3);
  h.nrc = (n2 / 2 + h.rp - 1) / h.rp;
  h.nrcp = (n2 / 2 + NFIELD * h.rp - 1) / (NFIELD * h.rp);
  h.rowsC = n1;
  h.uchunk = update_chunk(M);
  h.nwg_upd = (int)((M + h.uchunk - 1) / h.uchunk);
  h.M = M; h.H = H;
  h.phi2[0] = base + o_phi; h.phi2[1] = base + o_phit; h.grad = base + o_grad;
  h.r2[0] = base + o_r; h.r2[1] = base + o_rt; h.pr2[0] = base + o_pr; h.pr2[1] = base + o_prt;
  h.d = base + o_d;
  h.S = own_hist ? base + o_S : nullptr;
  h.Y = own_hist ? base + o_Y : nullptr;
  h.vpt = base + o_vpt; h.fpt = base + o_fpt; h.qpt = base + o_qpt;
  h.npa = base + o_npa;
  h.spec = base + o_spec; h.vloc = base + o_vloc;
  h.partA = (double *)(base + o_pA); h.partB = (double *)(base + o_pB);
  h.partC = (double *)(base + o_pC); h.partU = (double *)(base + o_pU);
  h.partD = (double *)(base + o_pD);
  h.st = I.st;
  const DeviceRes &R = g_res[c->device];
  h.p1 = make_plan(n1, R.tw_off[n1], prec);
  h.p2 = make_plan(n2, R.tw_off[n2], prec);
  h.p3 = make_plan(n3, R.tw_off[n3], prec);
  I.vloc_ok = false;
  return SKX_OK;
}

// Fill the physics fields of the descriptor from the context.
void fill_physics(skx_ctx *c, SolveDev &h) {
  const double PI = 3.14159265358979323846;
  h.L = c->L;
  h.V = c->L * c->L * c->L;
  h.dV = h.V / (double)h.M;
  h.ne = c->ne;
  h.n0 = c->ne / h.V;
  h.a = c->fn.alpha;
  h.n0a = std::pow(h.n0, h.a);
  h.T = c->fn.T;
  h.beta = c->fn.beta;
  h.kscale = (2.0 * PI / c->L) * (2.0 * PI / c->L);
  h.lnnT = std::log(std::sqrt(2.0) / (PI * PI) * c->fn.T * std::sqrt(c->fn.T));
  h.sqrt_ne = std::sqrt(c->ne);
  h.inv_sqrt_ne = 1.0 / h.sqrt_ne;
  h.terms = c->fn.terms;
  h.xc = c->fn.xc;
  h.fields = fields_mask(h.terms, h.beta);
  int nf = 0;
  for (int b = 0; b < NFIELD; ++b) h.slot[b] = (h.fields & (1 << b)) ? nf++ : -1;
  h.nf = nf;
  h.w = c->w;
  h.wp = c->wp;
  h.kappa = c->kappa;
}

// Length of the compile-time-shaped kernels a solve runs on (0: the
// runtime-shaped ones): cubic grids of the lengths with such kernels, unless
// they are switched off, every plane is forced onto the split kernels, or
// the solve is an FFT check.
// Large cubic length whose pass B alone runs on the compile-time-shaped
// kernel (0: none), unless shaped pass B is switched off or the solve is an
// FFT check.
int shaped_b_length(const SolveDev &h) {
  if (!(g_shape_kernels & 2) || h.debug) return 0;
  if (h.n1 != h.n2 || h.n2 != h.n3 || !shaped_b_only(h.n1)) return 0;
  return h.n1;
}

int shaped_length(const SolveDev &h) {
  if (!g_shape_kernels || g_chunk_planes || h.debug) return 0;
  if (h.n1 != h.n2 || h.n2 != h.n3) return 0;
  switch (h.n1) {
    case 36: case 40: case 48: case 50: case 54: case 60: case 64: case 72: case 80: return h.n1;
    default: return 0;
  }
}

// Prefix sums of passes A, B, C of one group, its runtime-shaped LDS sizes
// and kernel choices.
int fill_group(skx_ctx *c, const std::vector<SolveDev> &hs, int prec, PassGroup &g,
               std::vector<int> &fa, std::vector<int> &fb, std::vector<int> &fc) {
  const int n = (int)hs.size();
  fa.assign(n + 1, 0); fb.assign(n + 1, 0); fc.assign(n + 1, 0);
  size_t la = 0, lb = 0, lc = 0, lbp = 1024;
  for (int i = 0; i < n; ++i) {
    const SolveDev &h = hs[i];
    fa[i + 1] = fa[i] + h.n1 * h.nf;
    fb[i + 1] = fb[i] + h.n2 * h.nkb;
    fc[i + 1] = fc[i] + h.n1;
    size_t a, b, cc;
    lds_sizes(h, prec, a, b, cc);
    lb = std::max(lb, b);
    // the preconditioner's pass B holds one field's tile
    lbp = std::max(lbp, (size_t)(prec == 0 ? 16 : 8) * ((size_t)h.n1 * (h.tk + 1) + h.n1));
    if (!(h.big & 1)) la = std::max(la, a);
    // the forward-only check (debug 1) launches no pass C
    if (!(h.big & 2) && h.debug != 1) lc = std::max(lc, cc);
  }
  if ((!(g.shape & 1) && la > LDS_MAX) || (!(g.shape & 2) && lb > LDS_MAX) ||
      (!(g.shape & 4) && lc > LDS_MAX))
    return fail(c, SKX_E_INVALID, "grid too large for the fused plane kernels at this precision");
  g.nsolve = n;
  g.gridA = fa[n]; g.gridB = fb[n]; g.gridC = fc[n];
  // pass C keeps dE/dphi beside the plane in LDS when every solve fits
  // (FP64: the dE/dphi plane; FP32: that plane and a copy of phi_t), only
  // while that leaves room for two workgroups per CU: beyond 80 KB the
  // accumulation in the output buffer was measured faster, e.g. FP64 96^3
  // pass C 216 -> 167 us
  size_t lc_acc = 0;
  for (const SolveDev &h : hs)
    if (!(h.big & 2))
      lc_acc = std::max(lc_acc, (prec == 0 ? 16 : 8) * ((size_t)h.n2 * h.nh + h.n2 + h.n3) +
                                    8 * (size_t)h.n2 * h.n3);
  g.accC_lds = lc_acc <= 80 * 1024 ? 1 : 0;
  if (g.accC_lds) lc = std::max(lc, lc_acc);
  g.ldsA = la; g.ldsB = lb; g.ldsC = lc; g.ldsBp = std::min(lbp, lb);
  g.bigA = g.smallA = g.bigC = g.smallC = 0;
  g.krow = g.kcol = g.krowp = 0;
  g.ldsRow = g.ldsCol = 0;
  for (const SolveDev &h : hs) {
    ((h.big & 1) ? g.bigA : g.smallA) = 1;
    ((h.big & 2) ? g.bigC : g.smallC) = 1;
    if (h.big) {
      size_t lr, lcol;
      split_lds(h, prec, lr, lcol);
      g.krow = std::max(g.krow, h.nrc);
      g.krowp = std::max(g.krowp, h.nrcp);
      g.kcol = std::max(g.kcol, (h.nh + split_cc(prec) - 1) / split_cc(prec));
      g.ldsRow = std::max(g.ldsRow, lr);
      g.ldsCol = std::max(g.ldsCol, lcol);
    }
  }
  if (g.ldsRow > LDS_MAX || g.ldsCol > LDS_MAX)
    return fail(c, SKX_E_INVALID, "grid too large for the split plane kernels at this precision");
  return SKX_OK;
}

// Descriptors, prefix sums and pass groups of a batch. ddev holds
// batch_desc_count(n) descriptors (the batch, then the groups' copies),
// dfirst batch_first_count(n) ints.
int build_batch(skx_ctx *c, const std::vector<SolveDev> &hs_in, int prec, SolveDev *ddev,
                int *dfirst, BatchLaunch &bl, hipStream_t s) {
  const int n = (int)hs_in.size();
  // Passes A and C of planes beyond LDS take the split kernels, and so do
  // those where the split kernels were measured faster on MI355X: pass C
  // from 24 KB planes (80^2) on in FP32 and from 80 KB (108^2) in FP64
  // (108^3 FP64 275 -> 188 us for three solves, 128^3 200 -> 177 us), FP32
  // pass A from 80 KB (144^2); FP64 pass A is faster in LDS wherever it
  // fits. Solves on the compile-time-shaped kernels take none.
  std::vector<SolveDev> hs(hs_in);
  for (SolveDev &h : hs) {
    size_t a, b, cc;
    lds_sizes(h, prec, a, b, cc);
    const size_t plane = (prec == 0 ? 16 : 8) * (size_t)h.n2 * h.nh;
    const bool forced = g_chunk_planes && !h.debug;
    const bool bigA = forced || a > LDS_MAX || (prec == 1 && plane > 80 * 1024);
    const bool bigC = forced || cc > LDS_MAX || plane > (size_t)(prec == 1 ? 24 : 80) * 1024;
    h.big = (bigA ? 1 : 0) | (bigC ? 2 : 0);
    // the forward-only check (debug 1) keeps the split pass A; the split
    // pass C has no check mode
    if (h.debug) h.big &= h.debug == 1 ? 1 : 0;
    if (shaped_length(h)) h.big = 0;
    h.rowsC = (h.big & 2) ? h.n1 * h.nrc : h.n1;
  }
  std::vector<int> fv(n + 1), fu(n + 1);
  fv[0] = fu[0] = 0;
  for (int i = 0; i < n; ++i) {
    fv[i + 1] = fv[i] + hs[i].nwg_vec;
    fu[i + 1] = fu[i] + hs[i].nwg_upd;
  }
  // pass groups: the runtime-shaped solves (one group per column-block
  // width), then one group per compile-time length
  auto key_of = [](const SolveDev &h) {
    const int k = shaped_length(h) ? shaped_length(h) : shaped_b_length(h);
    return k ? k : -h.tk;
  };
  std::vector<int> keys;
  for (const SolveDev &h : hs) {
    const int k = key_of(h);
    if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
  }
  std::sort(keys.begin(), keys.end());
  if ((int)keys.size() > MAX_GROUPS) return fail(c, SKX_E_DEVICE, "too many pass groups");
  std::vector<SolveDev> part;
  std::vector<int> all;
  all.insert(all.end(), fv.begin(), fv.end());
  all.insert(all.end(), fu.begin(), fu.end());
  bl.ngroup = (int)keys.size();
  struct Off { size_t desc, a, b, cc; };
  std::vector<Off> offs;
  for (int gi = 0; gi < bl.ngroup; ++gi) {
    PassGroup &g = bl.grp[gi];
    g = PassGroup{};
    g.shapeN = std::max(keys[gi], 0);
    std::vector<SolveDev> sub;
    for (const SolveDev &h : hs)
      if (key_of(h) == keys[gi]) sub.push_back(h);
    g.tk = sub[0].tk;
    std::vector<int> fa, fb, fc;
    // passes on compile-time-shaped kernels: all three for the lengths that
    // have them, pass B alone for the large lengths (at the width the
    // kernel is built for)
    if (g.shapeN && shaped_b_only(g.shapeN))
      g.shape = (g.tk == passb_width(g.shapeN, prec)) ? (g_shape_kernels & 2) : 0;
    else if (g.shapeN)
      g.shape = g_shape_kernels & 7;
    int rc = fill_group(c, sub, prec, g, fa, fb, fc);
    if (rc) return rc;
    Off o;
    o.desc = part.size();
    part.insert(part.end(), sub.begin(), sub.end());
    o.a = all.size(); all.insert(all.end(), fa.begin(), fa.end());
    o.b = all.size(); all.insert(all.end(), fb.begin(), fb.end());
    o.cc = all.size(); all.insert(all.end(), fc.begin(), fc.end());
    offs.push_back(o);
  }
  if (all.size() > batch_first_count(n) || part.size() != (size_t)n)
    return fail(c, SKX_E_DEVICE, "batch layout exceeds its buffers");
  hipError_t e = hipMemcpyAsync(dfirst, all.data(), sizeof(int) * all.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ddev, hs.data(), sizeof(SolveDev) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ddev + n, part.data(), sizeof(SolveDev) * n, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "descriptor upload");
  for (int gi = 0; gi < bl.ngroup; ++gi) {
    PassGroup &g = bl.grp[gi];
    g.dev = ddev + n + offs[gi].desc;
    g.firstA = dfirst + offs[gi].a;
    g.firstB = dfirst + offs[gi].b;
    g.firstC = dfirst + offs[gi].cc;
  }
  const DeviceRes &R = g_res[c->device];
  bl.dev = ddev;
  bl.nsolve = n;
  bl.prec = prec;
  bl.twbank = R.twbank;
  bl.fd = R.fd;
  bl.gridV = fv[n]; bl.gridU = fu[n];
  bl.firstV = dfirst;
  bl.firstU = dfirst + (n + 1);
  bl.mh = 1;
  for (const SolveDev &h : hs) bl.mh = std::max(bl.mh, std::min(h.mh, MMAX));
  return SKX_OK;
}

int check_grid(skx_ctx *c, int prec) {
  const int n1 = c->n1, n2 = c->n2, n3 = c->n3;
  SolveDev h{};
  h.n1 = n1; h.n2 = n2; h.n3 = n3; h.nh = n3 / 2 + 1; h.nf = NFIELD; h.tk = prec == 0 ? 8 : 16;
  size_t a, b, cc;
  lds_sizes(h, prec, a, b, cc);
  // planes beyond LDS run the split kernels (a chunk of row pairs, a chunk
  // of columns); pass B's x tile must fit as it is
  h.rp = split_rp(n3);
  size_t lr, lcol;
  split_lds(h, prec, lr, lcol);
  if (b > LDS_MAX || lr > LDS_MAX || lcol > LDS_MAX)
    return fail(c, SKX_E_INVALID, "grid too large for the fused plane kernels at this precision");
  (void)a;
  return SKX_OK;
}

int ensure_tables(skx_ctx *c) {
  if (c->tables_ok) return SKX_OK;
  const int smax = (c->n1 / 2) * (c->n1 / 2) + (c->n2 / 2) * (c->n2 / 2) + (c->n3 / 2) * (c->n3 / 2);
  // the buffers are kept while the shell count does not grow (a free
  // synchronises the whole device; engine admissions reuse contexts)
  hipError_t e = hipSuccess;
  if (!c->w || !c->wp || smax + 1 > c->w_cap) {
    if (c->w) { (void)hipFree(c->w); c->w = nullptr; }
    if (c->wp) { (void)hipFree(c->wp); c->wp = nullptr; }
    c->w_cap = 0;
    e = hipMalloc((void **)&c->w, sizeof(double) * (smax + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&c->wp, sizeof(double) * (smax + 1));
    if (e != hipSuccess) return hip_fail(c, e, "kernel table allocation");
    c->w_cap = smax + 1;
  }
  c->smax = smax;
  const double V = c->L * c->L * c->L;
  double gas[3] = {0, 1, 0};
  const double n0 = c->ne / V;
  e = build_kernel_tables(c->w, c->wp, smax, c->L, n0, c->fn.T, c->fn.alpha,
                          g_res[c->device].fd, gas, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kernel table build");
  // preconditioner shift: 4 n0 dmu0/dn, the curvature of the TF term in phi
  const double dmudn = std::sqrt(2.0) * M_PI * M_PI / (std::sqrt(c->fn.T) * gas[1]);
  c->kappa = std::isfinite(dmudn) && dmudn > 0 ? std::max(4.0 * n0 * dmudn, 1e-3) : 1.0;
  c->tables_ok = true;
  return SKX_OK;
}

// FP32 V_loc(G) from the FP64 instance's: k_vloc computes every entry in
// FP64 and rounds it to the field type, so the rounded copy is the same
// array (the two instances may differ in spectrum pitch).
__global__ void k_vloc_d2f(const double2 *src, int spitch, float2 *dst, int dpitch, int rows,
                           int nh) {
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= (long long)rows * nh) return;
  const long long row = idx / nh;
  const int k = (int)(idx - row * nh);
  const double2 v = src[row * spitch + k];
  dst[row * dpitch + k] = make_float2((float)v.x, (float)v.y);
}

int ensure_vloc(skx_ctx *c, Instance &I) {
  if (I.vloc_ok) return SKX_OK;
  const Instance &I64 = c->inst[0];
  if (I.prec == 1 && I64.mem && I64.vloc_ok && I64.h.n1 == I.h.n1 && I64.h.n2 == I.h.n2 &&
      I64.h.n3 == I.h.n3) {
    const int rows = I.h.n1 * I.h.n2, nh = I.h.nh;
    hipLaunchKernelGGL(k_vloc_d2f, dim3((unsigned)(((long long)rows * nh + 255) / 256)), dim3(256), 0,
                       c->stream, (const double2 *)I64.h.vloc, I64.h.pitch, (float2 *)I.h.vloc,
                       I.h.pitch, rows, nh);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "V_loc conversion");
    I.vloc_ok = true;
    return SKX_OK;
  }
  const int nions = (int)c->species.size();
  const int nh = c->n3 / 2 + 1;
  double2 *scr = nullptr;
  size_t ns = (size_t)std::max(1, nions) * (c->n1 + c->n2 + nh);
  hipError_t e = hipMallocAsync((void **)&scr, sizeof(double2) * ns, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "phase table allocation");
  e = build_vloc(I.h.vloc, I.prec, c->n1, c->n2, c->n3, I.h.pitch, c->L, nions, c->ion_pos,
                 c->ion_sp, c->nspecies, c->sp_z, c->sp_rc, scr, c->stream);
  (void)hipFreeAsync(scr, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "structure factor kernel");
  I.vloc_ok = true;
  return SKX_OK;
}

// Time one evaluation (passes A, B, C) of instance I as a batch of one, in
// milliseconds (mean of `reps` after a warm-up). Leaves phi uniform and the
// state idle.
double time_eval(skx_ctx *c, Instance &I, int reps) {
  hipStream_t s = c->stream;
  if (start_uniform(c, I, s) != hipSuccess) return -1.0;
  OptState st{};
  st.phase = PH_EVAL_ONLY;
  BatchLaunch bl{};
  std::vector<SolveDev> hs(1, I.h);
  if (build_batch(c, hs, I.prec, I.dptr, I.first, bl, s)) return -1.0;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  double best = -1.0;
  hipError_t e = hipSuccess;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    e = hipMemcpyAsync(I.st, &st, sizeof(OptState), hipMemcpyHostToDevice, s);
    (void)hipEventRecord(a, s);
    if (e == hipSuccess) e = launch_eval(bl, s, 7);
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, a, b);
    if (r > 0 && (best < 0 || t < best)) best = t;
  }
  hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamSynchronize(s);
  return e == hipSuccess ? best : -1.0;
}

// Pick, per transform length of this instance not tuned yet in this
// precision, the fastest radix order among radix_candidates by timing whole
// evaluations; the choice holds for the rest of the process.
int autotune(skx_ctx *c, Instance &I) {
  const int prec = I.prec;
  const DeviceRes &R = g_res[c->device];
  const int ns[3] = {I.h.n1, I.h.n2, I.h.n3};
  for (int ax = 0; ax < 3; ++ax) {
    const int n = ns[ax];
    if (!g_tuned[prec][n].empty()) continue;
    const auto cands = radix_candidates(n);
    std::vector<int> best = cands[0];
    double tbest = -1.0;
    for (const auto &cand : cands) {
      g_tuned[prec][n] = cand;
      I.h.p1 = make_plan(I.h.n1, R.tw_off[I.h.n1], prec);
      I.h.p2 = make_plan(I.h.n2, R.tw_off[I.h.n2], prec);
      I.h.p3 = make_plan(I.h.n3, R.tw_off[I.h.n3], prec);
      const double t = time_eval(c, I, 3);
      if (t < 0) return fail(c, SKX_E_DEVICE, "autotune timing failed");
      if (tbest < 0 || t < tbest) { tbest = t; best = cand; }
    }
    g_tuned[prec][n] = best;
  }
  I.h.p1 = make_plan(I.h.n1, R.tw_off[I.h.n1], prec);
  I.h.p2 = make_plan(I.h.n2, R.tw_off[I.h.n2], prec);
  I.h.p3 = make_plan(I.h.n3, R.tw_off[I.h.n3], prec);
  return SKX_OK;
}

// Prepare instance `prec` of a context for a run: buffers, tables, V_loc,
// descriptor upload for the batch of one.
// The FP64 instance of a mixed solve takes the FP32 instance's history
// arrays (the pairs stay FP32 through the refinement, and the pairs of the
// FP32 phase are there when it starts).
void link_history(skx_ctx *c) {
  Instance &I64 = c->inst[0];
  if (!I64.mem) return;
  if (I64.own_hist) { I64.h.hist32 = 0; return; }
  const Instance &I32 = c->inst[1];
  const bool ok = I32.mem && I32.h.n1 == I64.h.n1 && I32.h.n2 == I64.h.n2 && I32.h.n3 == I64.h.n3;
  I64.h.S = ok ? I32.h.S : nullptr;
  I64.h.Y = ok ? I32.h.Y : nullptr;
  I64.h.mh = ok ? std::min(I64.m_alloc, I32.m_alloc) : 0;
  I64.h.hist32 = 1;
}

int prepare(skx_ctx *c, int prec, int m) {
  if (!c->has_cell || !c->has_ions || !c->has_fn)
    return fail(c, SKX_E_STATE, "set_cell, set_ions and set_functional must precede this call");
  int rc = check_grid(c, prec);
  if (rc) return rc;
  rc = ensure_instance(c, prec, m);
  if (rc) return rc;
  rc = ensure_tables(c);
  if (rc) return rc;
  Instance &I = c->inst[prec];
  fill_physics(c, I.h);
  rc = ensure_vloc(c, I);
  if (rc) return rc;
  if (g_autotune) rc = autotune(c, I);
  link_history(c);
  return rc;
}


__global__ void k_sqrt_field(const double *in, double *out, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) { double v = in[i]; out[i] = v > 0 ? sqrt(v) : 0.0; }
}
// MD start density: n <- max(2 n - n_prev, n / 10) (second-order extrapolation
// in time, kept positive), n_prev <- the old n.
__global__ void k_md_extrapolate(double *n, double *n_prev, long long m) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < m) {
    const double v = n[i];
    n[i] = fmax(2.0 * v - n_prev[i], 0.1 * v);
    n_prev[i] = v;
  }
}
__global__ void k_sqrt_field_f(const float *in, float *out, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) { float v = in[i]; out[i] = v > 0 ? sqrtf(v) : 0.0f; }
}
template <typename R>
__global__ void k_fill(R *p, R v, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
template <typename R>
__global__ void k_square_out(const R *phi, double *rho, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) { double v = (double)phi[i]; rho[i] = v * v; }
}
template <typename R>
__global__ void k_from_rho(const double *rho, R *phi, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) phi[i] = (R)rho[i];
}
__global__ void k_f2d(const float *a, double *b, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

unsigned blocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t start_uniform(skx_ctx *c, Instance &I, hipStream_t s) {
  const long long M = I.h.M;
  const double v = std::sqrt(c->ne / (c->L * c->L * c->L));
  if (I.prec == 0)
    hipLaunchKernelGGL(k_fill<double>, dim3(blocks(M, 256)), dim3(256), 0, s,
                       (double *)I.h.phi2[0], v, M);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(blocks(M, 256)), dim3(256), 0, s,
                       (float *)I.h.phi2[0], (float)v, M);
  return hipGetLastError();
}

hipError_t promote_phi(const Instance &I32, int par, Instance &I64, hipStream_t s) {
  hipLaunchKernelGGL(k_f2d, dim3(blocks(I64.h.M, 256)), dim3(256), 0, s,
                     (const float *)I32.h.phi2[par], (double *)I64.h.phi2[0], I64.h.M);
  return hipGetLastError();
}

hipError_t square_out(const Instance &I, int par, double *rho, hipStream_t s) {
  if (I.prec == 0)
    hipLaunchKernelGGL(k_square_out<double>, dim3(blocks(I.h.M, 256)), dim3(256), 0, s,
                       (const double *)I.h.phi2[par], rho, I.h.M);
  else
    hipLaunchKernelGGL(k_square_out<float>, dim3(blocks(I.h.M, 256)), dim3(256), 0, s,
                       (const float *)I.h.phi2[par], rho, I.h.M);
  return hipGetLastError();
}

__global__ void k_gather_phases(const SolveDev *dev, int n, int *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = dev[i].st->phase;
}

// Optimiser states between one packed array and the per-solve state
// buffers (their addresses in a device array): one workgroup per state,
// 4-byte words.
__global__ void k_put_states(const OptState *src, OptState *const *dst, int n) {
  constexpr int W = (int)(sizeof(OptState) / 4);
  const int *a = reinterpret_cast<const int *>(src + blockIdx.x);
  int *b = reinterpret_cast<int *>(dst[blockIdx.x]);
  for (int w = threadIdx.x; w < W; w += blockDim.x) b[w] = a[w];
}

__global__ void k_get_states(OptState *const *src, OptState *dst, int n) {
  constexpr int W = (int)(sizeof(OptState) / 4);
  const int *a = reinterpret_cast<const int *>(src[blockIdx.x]);
  int *b = reinterpret_cast<int *>(dst + blockIdx.x);
  for (int w = threadIdx.x; w < W; w += blockDim.x) b[w] = a[w];
}

hipError_t gather_phases(const SolveDev *dev, int n, int *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_phases, dim3(blocks(n, 256)), dim3(256), 0, s, dev, n, out);
  return hipGetLastError();
}

void energy_from(const double *e, double e_ii, skx_energy *out) {
  out->f_tf = e[E_TF]; out->e_vw = e[E_VW]; out->f_nl0 = e[E_NL0]; out->f_nl1 = e[E_NL1];
  out->e_h = e[E_H]; out->e_loc = e[E_LOC]; out->e_xc = e[E_XC]; out->e_ii = e_ii;
  out->free_energy = e[E_FREE]; out->total = e[E_FREE] + e_ii; out->mu = e[E_MU];
  out->nelec = e[E_NELEC];
}

// Initialise the optimiser state of one instance (host -> device).
#ifndef SKX_FP32_STALL_LIMIT
#define SKX_FP32_STALL_LIMIT 3
#endif
#ifndef SKX_FP32_STALL_FACTOR
#define SKX_FP32_STALL_FACTOR 0.5
#endif
void init_state(OptState &st, const skx_opt_params &p, double gtol, int from_rho, int prec) {
  st = OptState{};
  st.phase = PH_EVAL_INIT;
  st.m = std::min(std::max(p.lbfgs_m, 1), MMAX);
  st.max_iter = p.max_iter;
  st.max_trials = 20;
  st.gtol = gtol;
  st.c1 = 1e-4;
  st.theta_max = 0.5;
  // energies carry the rounding of the field precision
  st.tolE_rel = prec == 0 ? 1e-12 : 2e-6;
  // A solve stops when its best ||r|| has not dropped below stall_factor
  // of itself for stall_limit iterations. FP64: 10% in 150 iterations
  // (SKX_NOT_CONVERGED; a density straddling the PZ81 branch point rs = 1
  // floors ||r|| near 1e-4, the potential jumps there). FP32: the rounding
  // of the large, nearly cancelling potential terms floors ||r|| at
  // 1e-5..1e-3 (growing with the cell volume), where L-BFGS stops
  // converging fast; the FP32 phase ends (and the FP64 refinement starts)
  // once ||r|| fails to halve within 3 iterations.
  st.stall_limit = prec == 0 ? 150 : SKX_FP32_STALL_LIMIT;
  st.stall_factor = prec == 0 ? 0.9 : SKX_FP32_STALL_FACTOR;
  st.best_r = 1e300;
  st.par = 0;
  st.reset_pending = from_rho ? 2 : 0;
}

// ---------------------------------------------------------------------------
// Optional per-pass timing with HIP events on the launch stream.
// ---------------------------------------------------------------------------
enum { PP_A = 0, PP_B, PP_C, PP_FIN, PP_UPD, PP_DIR, PP_PREC, PP_POINT, PP_FLOC, PP_FII, PP_SF, PP_N };
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  struct Pair { int which, launches; hipEvent_t a, b; };
  std::vector<Pair> pending;
  double ms[PP_N] = {0};
  long long count[PP_N] = {0};
  int kernel_tag = -1;               // pass whose kernels take their own events
  int kernel_pairs = 0;              // pairs taken by the current pass launch
  unsigned mask = ~0u;               // passes timed while profiling is on
  std::mutex mu;
} g_prof;

// Step sequences of the optimisation driver may be captured into a HIP
// graph and replayed (process-wide switch). Off by default: on MI355X the
// eager launches of the 64^3 scan ran 8.6 ms per batched solve against 9.9
// ms replayed (the ensemble and the serving engine ran the same either way).
bool g_graphs = false;

bool graphs_enabled() { return g_graphs && !g_prof.on; }

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  (void)hipEventCreate(&e);
  return e;
}

}  // namespace host

// Events for the next kernel launch of the pass being timed per kernel: the
// kernel is launched with them as its start and stop events, so the time
// covers the kernel's execution only (not the dispatch of an event between
// launches).
bool kernel_events(hipEvent_t *start, hipEvent_t *stop) {
  using namespace host;
  if (!g_prof.on || g_prof.kernel_tag < 0) return false;
  *start = prof_event();
  *stop = prof_event();
  g_prof.pending.push_back({g_prof.kernel_tag, g_prof.kernel_pairs == 0 ? 1 : 0, *start, *stop});
  ++g_prof.kernel_pairs;
  return true;
}

namespace host {

// Time the kernels `fn` launches when profiling is on (the driver launches
// eagerly then): every kernel launch of the pass carries its own start/stop
// events (SKX_TIMED_LAUNCH), so no event packet sits between launches.
template <typename F>
hipError_t timed(int which, hipStream_t, F fn) {
  if (!g_prof.on || !((g_prof.mask >> which) & 1u)) return fn();
  g_prof.kernel_tag = which;
  g_prof.kernel_pairs = 0;
  hipError_t e = fn();
  g_prof.kernel_tag = -1;
  return e;
}

// Fold finished event pairs into the totals (call after a stream sync).
void prof_fold() {
  for (auto &p : g_prof.pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      g_prof.ms[p.which] += t;
      g_prof.count[p.which] += p.launches;
    }
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.clear();
}

// The fixed step sequence: direction, trial evaluation, update.
hipError_t step_sequence(const BatchLaunch &bl, hipStream_t s) {
  hipError_t e = timed(PP_DIR, s, [&] { return launch_opt_dir(bl, s); });
  if (e == hipSuccess) e = timed(PP_POINT, s, [&] { return launch_eval(bl, s, 8); });
  if (e == hipSuccess) e = timed(PP_A, s, [&] { return launch_eval(bl, s, 16); });
  if (e == hipSuccess) e = timed(PP_B, s, [&] { return launch_eval(bl, s, 2); });
  if (e == hipSuccess) e = timed(PP_C, s, [&] { return launch_eval(bl, s, 4); });
  if (e == hipSuccess) e = timed(PP_FIN, s, [&] { return launch_finalize_eval(bl, s); });
  if (e == hipSuccess) e = timed(PP_PREC, s, [&] { return launch_prec(bl, s); });
  if (e == hipSuccess) e = timed(PP_UPD, s, [&] { return launch_opt_update(bl, s); });
  return e;
}

// Drive a batch until every solve is DONE or FAILED. States are polled
// every `chunk` steps; the step sequence itself makes every decision, so a
// chunk is the same work every time: launched eagerly (the default), or,
// with graphs on, captured once into a HIP graph and replayed (eager again
// while per-pass events are on or when capture is refused). When half of
// the solves have finished, the batch is
// rebuilt from the unfinished ones (into the same descriptor buffers) so that
// the launches stop covering finished solves; a solve's arithmetic does not
// depend on the batch it is in.
int drive(skx_ctx *c, std::vector<SolveDev> hs, int prec, SolveDev *ddev, int *dfirst,
          int max_steps, hipStream_t s) {
  for (const SolveDev &h : hs)
    if (!h.S || !h.Y) return fail(c, SKX_E_STATE, "history arrays missing (mixed solve without its FP32 instance)");
  BatchLaunch bl{};
  int rc = build_batch(c, hs, prec, ddev, dfirst, bl, s);
  if (rc) return rc;
  hipError_t e = launch_normalize(bl, s);
  if (e != hipSuccess) return hip_fail(c, e, "normalisation kernels");
  const int chunk = 8;
  int n = bl.nsolve;
  int *dph = nullptr;
  e = hipMallocAsync((void **)&dph, sizeof(int) * n, s);
  if (e != hipSuccess) return hip_fail(c, e, "phase buffer");
  // the phases are read back into pinned host memory (kept per thread for
  // the life of the process), which avoids a staged copy at every poll
  static thread_local int *ph = nullptr;
  static thread_local int ph_cap = 0;
  if (ph_cap < n) {
    if (ph) (void)hipHostFree(ph);
    ph = nullptr;
    ph_cap = 0;
    e = hipHostMalloc((void **)&ph, sizeof(int) * n, hipHostMallocDefault);
    if (e != hipSuccess) { (void)hipFreeAsync(dph, s); return hip_fail(c, e, "pinned phase buffer"); }
    ph_cap = n;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto drop_graph = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  };
  auto capture = [&]() {
    // per-launch HIP-event timing needs the eager launches
    if (!g_graphs || g_prof.on) return;
    hipError_t ec = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (ec != hipSuccess) { (void)hipGetLastError(); return; }
    for (int k = 0; k < chunk && ec == hipSuccess; ++k) ec = step_sequence(bl, s);
    if (ec == hipSuccess) ec = gather_phases(bl.dev, n, dph, s);
    hipError_t ee = hipStreamEndCapture(s, &graph);
    if (ec == hipSuccess && ee == hipSuccess) ee = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ec != hipSuccess || ee != hipSuccess) {
      drop_graph();
      (void)hipGetLastError();
    }
  };
  capture();
  int steps = 0;
  while (steps < max_steps) {
    if (exec) {
      e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) { rc = hip_fail(c, e, "step graph"); break; }
    } else {
      for (int k = 0; k < chunk && e == hipSuccess; ++k) e = step_sequence(bl, s);
      if (e == hipSuccess) e = gather_phases(bl.dev, n, dph, s);
      if (e != hipSuccess) { rc = hip_fail(c, e, "step kernels"); break; }
    }
    steps += chunk;
    e = hipMemcpyAsync(ph, dph, sizeof(int) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { rc = hip_fail(c, e, "step execution"); break; }
    prof_fold();
    int active = 0;
    for (int i = 0; i < n; ++i)
      if (ph[i] != PH_DONE && ph[i] != PH_FAILED) ++active;
    if (active == 0) break;
    if (n > 1 && 2 * active <= n) {
      std::vector<SolveDev> keep;
      for (int i = 0; i < n; ++i)
        if (ph[i] != PH_DONE && ph[i] != PH_FAILED) keep.push_back(hs[i]);
      hs.swap(keep);
      drop_graph();
      rc = build_batch(c, hs, prec, ddev, dfirst, bl, s);
      if (rc) break;
      e = hipStreamSynchronize(s);          // hs is read from pageable memory
      if (e != hipSuccess) { rc = hip_fail(c, e, "batch rebuild"); break; }
      n = bl.nsolve;
      capture();
    }
  }
  drop_graph();
  (void)hipFreeAsync(dph, s);
  return rc;
}

int run_optimize(skx_ctx *c, Instance &I, void *rho_dev, const skx_opt_params &p, double gtol,
                 int start_mode /* 0 uniform, 1 rho_dev (FP64 density), 2 keep I.phi */,
                 OptState &out) {
  const long long M = I.h.M;
  hipStream_t s = c->stream;
  if (start_mode == 0) {
    const double v = std::sqrt(c->ne / (c->L * c->L * c->L));
    if (I.prec == 0)
      hipLaunchKernelGGL(k_fill<double>, dim3(blocks(M, 256)), dim3(256), 0, s,
                         (double *)I.h.phi2[0], v, M);
    else
      hipLaunchKernelGGL(k_fill<float>, dim3(blocks(M, 256)), dim3(256), 0, s,
                         (float *)I.h.phi2[0], (float)v, M);
  } else if (start_mode == 1) {
    if (I.prec == 0)
      hipLaunchKernelGGL(k_from_rho<double>, dim3(blocks(M, 256)), dim3(256), 0, s,
                         (const double *)rho_dev, (double *)I.h.phi2[0], M);
    else
      hipLaunchKernelGGL(k_from_rho<float>, dim3(blocks(M, 256)), dim3(256), 0, s,
                         (const double *)rho_dev, (float *)I.h.phi2[0], M);
  }
  OptState st;
  init_state(st, p, gtol, start_mode == 1 ? 1 : 0, I.prec);
  hipError_t e = hipMemcpyAsync(I.st, &st, sizeof(OptState), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "state upload");
  const int max_steps = (p.max_iter + 2) * 24 + 64;
  int rc = drive(c, std::vector<SolveDev>(1, I.h), I.prec, I.dptr, I.first, max_steps, s);
  if (rc) return rc;
  e = hipMemcpyAsync(&out, I.st, sizeof(OptState), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "state readback");
  return SKX_OK;
}

}  // namespace host
}  // namespace skx

using namespace skx::host;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int skx_create(skx_ctx **out, int device, void *hip_stream) {
  if (!out) return SKX_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return SKX_E_DEVICE;
  skx_ctx *c = new skx_ctx();
  c->device = device;
  std::string err;
  if (init_device(device, err) != hipSuccess) { delete c; return SKX_E_DEVICE; }
  hipSetDevice(device);
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return SKX_E_DEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return SKX_OK;
}

void skx_destroy(skx_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto &I : c->inst) free_instance(I);
  (void)hipFree(c->w); (void)hipFree(c->wp);
  (void)hipFree(c->ion_pos); (void)hipFree(c->ion_z); (void)hipFree(c->sp_z); (void)hipFree(c->sp_rc); (void)hipFree(c->ion_sp);
  (void)hipFree(c->sf_off); (void)hipFree(c->sf_idx);
  (void)hipFree(c->md_prev);
  if (c->own_stream) hipStreamDestroy(c->stream);
  delete c;
}

const char *skx_last_error(const skx_ctx *c) { return c ? c->err.c_str() : "null context"; }

int skx_set_cell(skx_ctx *c, const double lattice[9], int n1, int n2, int n3) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!lattice) return fail(c, SKX_E_INVALID, "lattice is NULL");
  const double L = lattice[0];
  for (int i = 0; i < 9; ++i) {
    const double want = (i % 4 == 0) ? L : 0.0;
    if (!(std::isfinite(lattice[i])) || std::fabs(lattice[i] - want) > 1e-12 * std::fabs(L))
      return fail(c, SKX_E_INVALID, "only cubic cells (L on the diagonal) are supported");
  }
  if (!(L > 0)) return fail(c, SKX_E_INVALID, "cell side must be positive");
  if (!five_smooth_even(n1) || !five_smooth_even(n2) || !five_smooth_even(n3))
    return fail(c, SKX_E_INVALID, "grid sizes must be even, 5-smooth and in [8, 512]");
  c->L = L;
  c->n1 = n1; c->n2 = n2; c->n3 = n3;
  c->has_cell = true;
  c->has_ions = false;
  c->tables_ok = false;
  for (auto &I : c->inst) I.vloc_ok = false;
  return SKX_OK;
}

int skx_set_ions(skx_ctx *c, int nions, const double *pos, const int *species, int nspecies,
                 const double *zval, const double *rc) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!c->has_cell) return fail(c, SKX_E_STATE, "set_cell first");
  if (nions < 1 || nspecies < 1 || !pos || !species || !zval || !rc)
    return fail(c, SKX_E_INVALID, "need at least one ion and one species");
  double ne = 0;
  for (int i = 0; i < nions; ++i) {
    if (species[i] < 0 || species[i] >= nspecies)
      return fail(c, SKX_E_INVALID, "species index out of range");
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(pos[3 * i + a])) return fail(c, SKX_E_INVALID, "non-finite position");
    ne += zval[species[i]];
  }
  for (int s = 0; s < nspecies; ++s)
    if (!(zval[s] > 0) || !(rc[s] > 0)) return fail(c, SKX_E_INVALID, "zval and rc must be > 0");
  (void)hipSetDevice(c->device);
  c->pos.assign(pos, pos + 3 * nions);
  // wrap positions into the cell
  for (auto &x : c->pos) x -= c->L * std::floor(x / c->L);
  c->species.assign(species, species + nions);
  c->zsp.assign(zval, zval + nspecies);
  c->rcsp.assign(rc, rc + nspecies);
  c->nspecies = nspecies;
  const double ne_old = c->ne;
  c->ne = ne;
  std::vector<double> zi(nions);
  for (int i = 0; i < nions; ++i) zi[i] = zval[species[i]];
  // the device ion arrays are reallocated only when they must grow (a free
  // synchronises the whole device; MD steps and engine reuse call this often)
  hipError_t e = hipSuccess;
  if (nions > c->ion_cap || nspecies > c->sp_cap || !c->ion_pos) {
    (void)hipFree(c->ion_pos); (void)hipFree(c->ion_z); (void)hipFree(c->sp_z); (void)hipFree(c->sp_rc); (void)hipFree(c->ion_sp);
    c->ion_pos = c->ion_z = c->sp_z = c->sp_rc = nullptr;
    c->ion_sp = nullptr;
    c->ion_cap = c->sp_cap = 0;
    e = hipMalloc((void **)&c->ion_pos, sizeof(double) * 3 * nions);
    if (e == hipSuccess) e = hipMalloc((void **)&c->ion_z, sizeof(double) * nions);
    if (e == hipSuccess) e = hipMalloc((void **)&c->sp_z, sizeof(double) * nspecies);
    if (e == hipSuccess) e = hipMalloc((void **)&c->sp_rc, sizeof(double) * nspecies);
    if (e == hipSuccess) e = hipMalloc((void **)&c->ion_sp, sizeof(int) * nions);
    if (e != hipSuccess) return hip_fail(c, e, "ion arrays");
    c->ion_cap = nions;
    c->sp_cap = nspecies;
  }
  hipStream_t s = c->stream;
  e = hipMemcpyAsync(c->ion_pos, c->pos.data(), sizeof(double) * 3 * nions, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ion_z, zi.data(), sizeof(double) * nions, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->sp_z, zval, sizeof(double) * nspecies, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->sp_rc, rc, sizeof(double) * nspecies, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ion_sp, species, sizeof(int) * nions, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "ion upload");
  // Ewald energy on the device
  {
    const double L = c->L;
    const double alpha = 3.2 / L;
    const double gcut = 2.0 * alpha * std::sqrt(44.0);
    const int mmax = (int)std::ceil(gcut * L / (2.0 * M_PI));
    const long long side = 2 * mmax + 1;
    const long long ng = side * side * side;
    const long long npair = (long long)nions * (nions + 1) / 2;
    const long long len = std::max(ng, npair);
    double *scr = nullptr, *out = nullptr;
    e = hipMallocAsync((void **)&scr, sizeof(double) * len, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&out, sizeof(double) * 2, s);
    if (e != hipSuccess) return hip_fail(c, e, "Ewald scratch");
    e = ewald_energy(L, nions, c->ion_pos, c->ion_z, scr, (int)len, out, s);
    double parts[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(parts, out, sizeof(parts), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(scr, s);
    (void)hipFreeAsync(out, s);
    if (e != hipSuccess) return hip_fail(c, e, "Ewald kernels");
    double z2 = 0;
    for (double z : zi) z2 += z * z;
    const double V = L * L * L;
    c->e_ii = parts[0] + parts[1] - alpha / std::sqrt(M_PI) * z2 - M_PI * ne * ne / (2.0 * V * alpha * alpha);
  }
  // the kernel tables depend on n0 = N_e / V only
  if (!c->has_ions || ne != ne_old) c->tables_ok = false;
  c->has_ions = true;
  for (auto &I : c->inst) I.vloc_ok = false;
  return SKX_OK;
}

int skx_set_functional(skx_ctx *c, const skx_functional *fn) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!fn) return fail(c, SKX_E_INVALID, "functional is NULL");
  if (!(fn->T > 0) || !std::isfinite(fn->T)) return fail(c, SKX_E_INVALID, "T must be > 0");
  if (!(fn->alpha > 0.5 && fn->alpha <= 1.5)) return fail(c, SKX_E_INVALID, "alpha must be in (0.5, 1.5]");
  if (!std::isfinite(fn->beta)) return fail(c, SKX_E_INVALID, "beta must be finite");
  if (fn->precision < SKX_FP64 || fn->precision > SKX_MIXED)
    return fail(c, SKX_E_INVALID, "unknown precision");
  if (fn->xc != SKX_XC_NONE && fn->xc != SKX_XC_PZ81 && fn->xc != SKX_XC_PZ81_C1)
    return fail(c, SKX_E_INVALID, "unknown xc");
  if (fn->terms & ~127u) return fail(c, SKX_E_INVALID, "unknown term bits");
  const bool tables_change = !c->has_fn || fn->T != c->fn.T || fn->alpha != c->fn.alpha;
  c->fn = *fn;
  if (fn->xc == SKX_XC_NONE) c->fn.terms &= ~(unsigned)SKX_TERM_XC;
  c->has_fn = true;
  if (tables_change) c->tables_ok = false;
  return SKX_OK;
}

int skx_evaluate_energy_potential(skx_ctx *c, const void *in_dev, int in_kind, void *out_dev,
                                  skx_energy *e) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!in_dev || !e) return fail(c, SKX_E_INVALID, "input field and energy struct are required");
  if (in_kind != SKX_RHO && in_kind != SKX_SQRT_RHO) return fail(c, SKX_E_INVALID, "bad in_kind");
  (void)hipSetDevice(c->device);
  const int prec = c->has_fn && c->fn.precision == SKX_FP32 ? 1 : 0;
  int rc = prepare(c, prec, 1);
  if (rc) return rc;
  Instance &I = c->inst[prec];
  SolveDev h = I.h;
  const long long M = h.M;
  if (in_kind == SKX_SQRT_RHO) {
    h.phi2[0] = const_cast<void *>(in_dev);
  } else {
    if (prec == 0)
      hipLaunchKernelGGL(k_sqrt_field, dim3(blocks(M, 256)), dim3(256), 0, c->stream,
                         (const double *)in_dev, (double *)I.h.phi2[0], M);
    else
      hipLaunchKernelGGL(k_sqrt_field_f, dim3(blocks(M, 256)), dim3(256), 0, c->stream,
                         (const float *)in_dev, (float *)I.h.phi2[0], M);
  }
  if (out_dev) h.grad = out_dev;
  OptState st{};
  st.phase = PH_EVAL_ONLY;
  hipError_t he = hipMemcpyAsync(I.st, &st, sizeof(OptState), hipMemcpyHostToDevice, c->stream);
  if (he != hipSuccess) return hip_fail(c, he, "state upload");
  std::vector<SolveDev> hs(1, h);
  rc = build_batch(c, hs, prec, I.dptr, I.first, I.bl, c->stream);
  if (rc) return rc;
  {
    hipStream_t s = c->stream;
    const BatchLaunch &bl = I.bl;
    he = timed(PP_POINT, s, [&] { return launch_eval(bl, s, 8); });
    if (he == hipSuccess) he = timed(PP_A, s, [&] { return launch_eval(bl, s, 16); });
    if (he == hipSuccess) he = timed(PP_B, s, [&] { return launch_eval(bl, s, 2); });
    if (he == hipSuccess) he = timed(PP_C, s, [&] { return launch_eval(bl, s, 4); });
    if (he == hipSuccess) he = timed(PP_FIN, s, [&] { return launch_finalize_eval(bl, s); });
  }
  if (he != hipSuccess) return hip_fail(c, he, "evaluation kernels");
  double ev[12];
  he = hipMemcpyAsync(ev, I.st->e_trial, sizeof(ev), hipMemcpyDeviceToHost, c->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  if (he != hipSuccess) return hip_fail(c, he, "evaluation");
  prof_fold();
  energy_from(ev, c->e_ii, e);
  if (ev[E_NONFINITE] != 0.0)
    return fail(c, SKX_E_NUMERIC, "non-finite field or density outside the Fermi-Dirac table");
  return SKX_OK;
}

int skx_optimize_density(skx_ctx *c, void *rho_dev, const skx_opt_params *p, skx_opt_result *res) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!rho_dev || !p || !res) return fail(c, SKX_E_INVALID, "rho_dev, params and result are required");
  if (p->lbfgs_m < 1 || p->lbfgs_m > MMAX) return fail(c, SKX_E_INVALID, "lbfgs_m must be in 1..8");
  if (!(p->gtol > 0) || p->max_iter < 1) return fail(c, SKX_E_INVALID, "gtol > 0 and max_iter >= 1 required");
  (void)hipSetDevice(c->device);
  std::memset(res, 0, sizeof(*res));
  const int mode = c->has_fn ? c->fn.precision : SKX_FP64;
  int rc;
  OptState out{};
  if (mode == SKX_FP64 || mode == SKX_FP32) {
    const int prec = mode == SKX_FP64 ? 0 : 1;
    rc = prepare(c, prec, p->lbfgs_m);
    if (rc) return rc;
    Instance &I = c->inst[prec];
    rc = run_optimize(c, I, rho_dev, *p, p->gtol, p->warm_start ? 1 : 0, out);
    if (rc) return rc;
    if (prec == 0)
      hipLaunchKernelGGL(k_square_out<double>, dim3(blocks(I.h.M, 256)), dim3(256), 0, c->stream,
                         (const double *)I.h.phi2[out.par], (double *)rho_dev, I.h.M);
    else
      hipLaunchKernelGGL(k_square_out<float>, dim3(blocks(I.h.M, 256)), dim3(256), 0, c->stream,
                         (const float *)I.h.phi2[out.par], (double *)rho_dev, I.h.M);
    res->iters = out.iters;
    res->evals = out.evals;
    if (prec == 1) { res->fp32_iters = out.iters; res->fp32_evals = out.evals; }
  } else {
    // mixed: FP32 phase to fp32_switch_gtol, then FP64 refinement from there
    // FP64 first: the FP32 instance then copies its V_loc(G) (ensure_vloc)
    rc = prepare(c, 0, p->lbfgs_m);
    if (rc) return rc;
    rc = prepare(c, 1, p->lbfgs_m);
    if (rc) return rc;
    Instance &I32 = c->inst[1];
    Instance &I64 = c->inst[0];
    const double sw = p->fp32_switch_gtol > 0 ? p->fp32_switch_gtol : 1e-5;
    OptState o32{};
    rc = run_optimize(c, I32, rho_dev, *p, std::max(sw, p->gtol), p->warm_start ? 1 : 0, o32);
    if (rc) return rc;
    res->fp32_iters = o32.iters;
    res->fp32_evals = o32.evals;
    if (o32.phase == PH_FAILED && o32.status < 0) {
      // a numerical failure of the FP32 phase ends the solve (the same rule
      // as skx_run_batch and the serving engine): no refinement from it
      out = o32;
      res->iters = o32.iters;
      res->evals = o32.evals;
      hipLaunchKernelGGL(k_square_out<float>, dim3(blocks(I32.h.M, 256)), dim3(256), 0, c->stream,
                         (const float *)I32.h.phi2[o32.par], (double *)rho_dev, I32.h.M);
    } else {
      hipLaunchKernelGGL(k_f2d, dim3(blocks(I64.h.M, 256)), dim3(256), 0, c->stream,
                         (const float *)I32.h.phi2[o32.par], (double *)I64.h.phi2[0], I64.h.M);
      rc = run_optimize(c, I64, rho_dev, *p, p->gtol, 2, out);
      if (rc) return rc;
      hipLaunchKernelGGL(k_square_out<double>, dim3(blocks(I64.h.M, 256)), dim3(256), 0,
                         c->stream, (const double *)I64.h.phi2[out.par], (double *)rho_dev,
                         I64.h.M);
      res->iters = o32.iters + out.iters;
      res->evals = o32.evals + out.evals;
    }
  }
  hipError_t he = hipStreamSynchronize(c->stream);
  if (he != hipSuccess) return hip_fail(c, he, "optimisation");
  energy_from(out.e_acc, c->e_ii, &res->e);
  res->gnorm = out.rnorm;
  res->resets = out.resets;
  if (out.phase == PH_FAILED && out.status < 0) {
    res->status = out.status;
    return fail(c, out.status, "numerical failure in the optimisation");
  }
  res->status = (out.phase == PH_DONE && out.status == 0) ? SKX_OK : SKX_NOT_CONVERGED;
  return res->status;
}

int skx_get_kernel_tables(skx_ctx *c, double *w_host, double *wp_host, int len) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!c->has_cell || !c->has_ions || !c->has_fn) return fail(c, SKX_E_STATE, "incomplete setup");
  (void)hipSetDevice(c->device);
  int rc = ensure_tables(c);
  if (rc) return rc;
  if (len > c->smax + 1 || len < 0) return fail(c, SKX_E_INVALID, "len exceeds the shell count");
  hipError_t e = hipSuccess;
  if (w_host) e = hipMemcpyAsync(w_host, c->w, sizeof(double) * len, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && wp_host)
    e = hipMemcpyAsync(wp_host, c->wp, sizeof(double) * len, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "table copy");
  return SKX_OK;
}

int skx_num_shells(const skx_ctx *c) {
  if (!c || !c->has_cell) return 0;
  return (c->n1 / 2) * (c->n1 / 2) + (c->n2 / 2) * (c->n2 / 2) + (c->n3 / 2) * (c->n3 / 2) + 1;
}

int skx_get_vloc(skx_ctx *c, double *host) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!host) return fail(c, SKX_E_INVALID, "host buffer is NULL");
  (void)hipSetDevice(c->device);
  int rc = prepare(c, 0, 1);
  if (rc) return rc;
  Instance &I = c->inst[0];
  const int nh = c->n3 / 2 + 1;
  hipError_t e = hipMemcpy2DAsync(host, sizeof(double) * 2 * nh, I.h.vloc,
                                  sizeof(double) * 2 * I.h.pitch, sizeof(double) * 2 * nh,
                                  (size_t)c->n1 * c->n2, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "V_loc copy");
  return SKX_OK;
}

int skx_fd_eval(int device, const double *u_host, double *eta_host, double *psi_host, long long n) {
  if (n < 0 || (n > 0 && (!u_host || !eta_host || !psi_host))) return SKX_E_INVALID;
  for (long long i = 0; i < n; ++i)
    if (!(u_host[i] > 0) || !std::isfinite(u_host[i])) return SKX_E_INVALID;
  std::string err;
  if (init_device(device, err) != hipSuccess) return SKX_E_DEVICE;
  (void)hipSetDevice(device);
  if (n == 0) return SKX_OK;
  double *d = nullptr;
  if (hipMalloc((void **)&d, sizeof(double) * 3 * n) != hipSuccess) return SKX_E_NOMEM;
  hipError_t e = hipMemcpy(d, u_host, sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = debug_fd_eval(d, d + n, d + 2 * n, n, g_res[device].fd, 0);
  if (e == hipSuccess) e = hipMemcpy(eta_host, d + n, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(psi_host, d + 2 * n, sizeof(double) * n, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return e == hipSuccess ? SKX_OK : SKX_E_DEVICE;
}

}  // extern "C"

// ===========================================================================
// FFT check and batched solves
// ===========================================================================
extern "C" {

int skx_fft_check(skx_ctx *c, const double *in_host, double *out_host, double *spec_host) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!c->has_cell) return fail(c, SKX_E_STATE, "set_cell first");
  if (!in_host || !out_host) return fail(c, SKX_E_INVALID, "host buffers are required");
  (void)hipSetDevice(c->device);
  int rc = check_grid(c, 0);
  if (rc) return rc;
  rc = ensure_instance(c, 0, 1);
  if (rc) return rc;
  Instance &I = c->inst[0];
  SolveDev h = I.h;
  {
    // the inverse check runs the in-LDS pass C
    size_t a, b, cc;
    lds_sizes(h, 0, a, b, cc);
    if (cc > LDS_MAX) return fail(c, SKX_E_INVALID, "the FFT check needs FP64 planes that fit LDS");
  }
  h.fields = F_PHI | F_N;
  h.nf = 2;
  h.slot[0] = 0; h.slot[1] = 1; h.slot[2] = -1; h.slot[3] = -1;
  h.terms = 0;
  h.L = c->L; h.V = c->L * c->L * c->L; h.dV = h.V / (double)h.M;
  h.ne = 1.0; h.n0 = 1.0; h.a = 1.0; h.n0a = 1.0; h.T = 1.0; h.beta = 0.0;
  h.debug = 1;
  hipStream_t s = c->stream;
  const long long M = h.M;
  hipError_t e = hipMemcpyAsync(h.phi2[0], in_host, sizeof(double) * M, hipMemcpyHostToDevice, s);
  OptState st{};
  st.phase = PH_EVAL_ONLY;
  if (e == hipSuccess) e = hipMemcpyAsync(I.st, &st, sizeof(OptState), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "upload");
  std::vector<SolveDev> hs(1, h);
  rc = build_batch(c, hs, 0, I.dptr, I.first, I.bl, s);
  if (rc) return rc;
  e = launch_eval(I.bl, s, 3);
  if (e != hipSuccess) return hip_fail(c, e, "forward passes");
  const int nh = c->n3 / 2 + 1;
  if (spec_host) {
    e = hipMemcpy2DAsync(spec_host, sizeof(double) * 2 * nh, h.spec, sizeof(double) * 2 * h.pitch,
                         sizeof(double) * 2 * nh, (size_t)c->n1 * c->n2, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(c, e, "spectrum copy");
  }
  hs[0].debug = 2;
  rc = build_batch(c, hs, 0, I.dptr, I.first, I.bl, s);
  if (rc) return rc;
  e = launch_eval(I.bl, s, 6);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_host, h.grad, sizeof(double) * M, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "inverse passes");
  return SKX_OK;
}

// The density's half spectrum (1/M normalised, FP64, [n1][n2][pitch] in
// slot 1 of the FP64 instance's spectrum buffer): pass A and pass B's
// forward x transform of the fields (phi, n), as in the FFT check. Enqueued
// on the ctx stream; *spec_out receives the slot's address.
static int density_spectrum(skx_ctx *c, const void *in_dev, int in_kind, const double2 **spec_out,
                            int *pitch_out) {
  int rc = check_grid(c, 0);
  if (rc == SKX_OK) rc = ensure_instance(c, 0, 1);
  if (rc != SKX_OK) return rc;
  hipStream_t s = c->stream;
  Instance &I = c->inst[0];
  SolveDev h = I.h;
  h.fields = F_PHI | F_N;
  h.nf = 2;
  h.slot[0] = 0; h.slot[1] = 1; h.slot[2] = -1; h.slot[3] = -1;
  h.terms = 0;
  h.L = c->L; h.V = c->L * c->L * c->L; h.dV = h.V / (double)h.M;
  h.ne = 1.0; h.n0 = 1.0; h.a = 1.0; h.n0a = 1.0; h.T = 1.0; h.beta = 0.0;
  h.debug = 1;
  if (in_kind == SKX_SQRT_RHO)
    h.phi2[0] = const_cast<void *>(in_dev);
  else
    hipLaunchKernelGGL(k_sqrt_field, dim3(blocks(h.M, 256)), dim3(256), 0, s,
                       (const double *)in_dev, (double *)h.phi2[0], h.M);
  OptState st{};
  st.phase = PH_EVAL_ONLY;
  hipError_t e = hipMemcpyAsync(I.st, &st, sizeof(OptState), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "state upload");
  std::vector<SolveDev> hs(1, h);
  rc = build_batch(c, hs, 0, I.dptr, I.first, I.bl, s);
  if (rc != SKX_OK) return rc;
  e = launch_eval(I.bl, s, 3);
  if (e != hipSuccess) return hip_fail(c, e, "forward transform");
  *spec_out = reinterpret_cast<const double2 *>(h.spec) + h.H;
  *pitch_out = h.pitch;
  return SKX_OK;
}

int skx_ion_forces(skx_ctx *c, const void *in_dev, int in_kind, double *f_loc, double *f_ii) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!f_loc && !f_ii) return fail(c, SKX_E_INVALID, "no force output requested");
  if (f_loc && !in_dev) return fail(c, SKX_E_INVALID, "the local force needs the density");
  if (f_loc && in_kind != SKX_RHO && in_kind != SKX_SQRT_RHO) return fail(c, SKX_E_INVALID, "bad in_kind");
  if (!c->has_cell || !c->has_ions) return fail(c, SKX_E_STATE, "set_cell and set_ions must precede this call");
  (void)hipSetDevice(c->device);
  hipStream_t s = c->stream;
  const int nions = (int)c->species.size();
  const int n1 = c->n1, n2 = c->n2, n3 = c->n3, nh = n3 / 2 + 1;
  const int nblk = force_row_blocks(n1, n2, n3);
  const int ng = ewald_force_terms(c->L);
  // one scratch allocation: [f_loc | f_ii] (2 nions x 3), ordered sums,
  // phase tables, structure factor, species order
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t n_out = 6 * (size_t)nions, n_part = (size_t)nions * nblk * 3;
  const size_t n_ph = (size_t)nions * (n1 + n2 + nh);
  const size_t o_part = al(sizeof(double) * n_out), o_ph = o_part + al(sizeof(double) * n_part);
  const size_t o_sf = o_ph + al(sizeof(double2) * n_ph), o_ord = o_sf + al(sizeof(double2) * ng);
  const size_t bytes = o_ord + al(sizeof(int) * nions);
  char *scr = nullptr;
  hipError_t e = hipMallocAsync((void **)&scr, bytes, s);
  if (e != hipSuccess) return hip_fail(c, e, "force scratch allocation");
  double *out = reinterpret_cast<double *>(scr);
  double *part = reinterpret_cast<double *>(scr + o_part);
  double2 *ph = reinterpret_cast<double2 *>(scr + o_ph);
  double2 *sf = reinterpret_cast<double2 *>(scr + o_sf);
  int *order = reinterpret_cast<int *>(scr + o_ord);
  int rc = SKX_OK;
  if (f_loc) {
    const double2 *spec = nullptr;
    int pitch = 0;
    rc = density_spectrum(c, in_dev, in_kind, &spec, &pitch);
    if (rc != SKX_OK) { (void)hipStreamSynchronize(s); (void)hipFreeAsync(scr, s); return rc; }
    // ions sorted by species: the form factor is computed once per run
    std::vector<int> ord(nions);
    for (int i = 0; i < nions; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int x, int y) { return c->species[x] < c->species[y]; });
    if (e == hipSuccess && rc == SKX_OK)
      e = hipMemcpyAsync(order, ord.data(), sizeof(int) * nions, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && rc == SKX_OK) e = ion_phase_tables(ph, nions, c->ion_pos, n1, n2, n3, c->L, s);
    if (e == hipSuccess && rc == SKX_OK)
      e = timed(PP_FLOC, s, [&] {
        return local_forces(spec, n1, n2, n3, pitch, c->L, ph, order, nions, c->ion_sp, c->sp_z,
                            c->sp_rc, part, out, s);
      });
    if (e == hipSuccess && rc == SKX_OK) e = hipStreamSynchronize(s);
  }
  if (e == hipSuccess && rc == SKX_OK && f_ii)
    e = timed(PP_FII, s, [&] {
      return ewald_forces(c->L, nions, c->ion_pos, c->ion_z, sf, part, out + 3 * (size_t)nions, s);
    });
  if (e == hipSuccess && rc == SKX_OK && f_loc)
    e = hipMemcpyAsync(f_loc, out, sizeof(double) * 3 * nions, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && rc == SKX_OK && f_ii)
    e = hipMemcpyAsync(f_ii, out + 3 * (size_t)nions, sizeof(double) * 3 * nions,
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFreeAsync(scr, s);
  if (rc != SKX_OK) return rc;
  if (e != hipSuccess) return hip_fail(c, e, "force kernels");
  prof_fold();
  return SKX_OK;
}

int skx_structure_factors(skx_ctx *c, const void *in_dev, int in_kind, double *s_ei,
                          double *s_ee, double *s_ii, int *count, int len) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!in_dev) return fail(c, SKX_E_INVALID, "the density is required");
  if (in_kind != SKX_RHO && in_kind != SKX_SQRT_RHO) return fail(c, SKX_E_INVALID, "bad in_kind");
  if (!c->has_cell || !c->has_ions) return fail(c, SKX_E_STATE, "set_cell and set_ions must precede this call");
  const int nshell = skx_num_shells(c);
  if (len < nshell) return fail(c, SKX_E_INVALID, "len must be at least skx_num_shells(ctx)");
  if (!s_ei && !s_ee && !s_ii && !count) return fail(c, SKX_E_INVALID, "no output requested");
  (void)hipSetDevice(c->device);
  hipStream_t s = c->stream;
  const int nions = (int)c->species.size();
  const int n1 = c->n1, n2 = c->n2, n3 = c->n3, nh = n3 / 2 + 1;
  const long long items = (long long)n1 * n2 * nh;
  hipError_t e = hipSuccess;
  if (c->sf_n[0] != n1 || c->sf_n[1] != n2 || c->sf_n[2] != n3) {
    // items of the half spectrum listed by shell (counting sort, fixed
    // order), kept on the device while the grid stays the same
    std::vector<int> off(nshell + 1, 0), idx(items);
    auto shell = [&](long long it) {
      const int k3 = (int)(it % nh), row = (int)(it / nh);
      const int k1 = row / n2, k2 = row % n2;
      const int g1 = 2 * k1 < n1 ? k1 : k1 - n1, g2 = 2 * k2 < n2 ? k2 : k2 - n2;
      return g1 * g1 + g2 * g2 + k3 * k3;
    };
    for (long long it = 0; it < items; ++it) ++off[shell(it) + 1];
    for (int k = 0; k < nshell; ++k) off[k + 1] += off[k];
    {
      std::vector<int> fill(off.begin(), off.end() - 1);
      for (long long it = 0; it < items; ++it) idx[fill[shell(it)]++] = (int)it;
    }
    hipFree(c->sf_off); (void)hipFree(c->sf_idx);
    c->sf_off = c->sf_idx = nullptr;
    c->sf_n[0] = c->sf_n[1] = c->sf_n[2] = 0;
    e = hipMalloc((void **)&c->sf_off, sizeof(int) * (nshell + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&c->sf_idx, sizeof(int) * items);
    if (e == hipSuccess) e = hipMemcpy(c->sf_off, off.data(), sizeof(int) * (nshell + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->sf_idx, idx.data(), sizeof(int) * items, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "shell lists");
    c->sf_n[0] = n1; c->sf_n[1] = n2; c->sf_n[2] = n3;
  }
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t n_ph = (size_t)nions * (n1 + n2 + nh);
  const size_t o_val = al(sizeof(double2) * n_ph), o_out = o_val + al(sizeof(double) * 3 * items);
  const size_t bytes = o_out + al(sizeof(double) * 4 * nshell);
  char *scr = nullptr;
  e = hipMallocAsync((void **)&scr, bytes, s);
  if (e != hipSuccess) return hip_fail(c, e, "structure factor scratch allocation");
  double2 *ph = reinterpret_cast<double2 *>(scr);
  double *val = reinterpret_cast<double *>(scr + o_val);
  double *out = reinterpret_cast<double *>(scr + o_out);
  const int *doff = c->sf_off, *didx = c->sf_idx;
  const double2 *spec = nullptr;
  int pitch = 0;
  int rc = density_spectrum(c, in_dev, in_kind, &spec, &pitch);
  if (rc == SKX_OK) {
    const double V = c->L * c->L * c->L;
    e = ion_phase_tables(ph, nions, c->ion_pos, n1, n2, n3, c->L, s);
    if (e == hipSuccess)
      e = timed(PP_SF, s, [&] { return structure_items(spec, n1, n2, n3, pitch, V, ph, nions, val, s); });
    if (e == hipSuccess)
      e = structure_shells(val, doff, didx, nshell, n3, 1.0 / std::sqrt(c->ne * nions), 1.0 / c->ne,
                           1.0 / nions, out, s);
  }
  std::vector<double> host(4 * (size_t)nshell);
  if (rc == SKX_OK && e == hipSuccess)
    e = hipMemcpyAsync(host.data(), out, sizeof(double) * 4 * nshell, hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  (void)hipFreeAsync(scr, s);
  if (rc != SKX_OK) return rc;
  if (e != hipSuccess) return hip_fail(c, e, "structure factor kernels");
  prof_fold();
  for (int k = 0; k < nshell; ++k) {
    if (s_ei) s_ei[k] = host[4 * k];
    if (s_ee) s_ee[k] = host[4 * k + 1];
    if (s_ii) s_ii[k] = host[4 * k + 2];
    if (count) count[k] = (int)host[4 * k + 3];
  }
  return SKX_OK;
}

int skx_density_deviation(skx_ctx *c, const void *a_dev, const void *b_dev, double *out) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!a_dev || !b_dev || !out) return fail(c, SKX_E_INVALID, "null argument");
  if (!c->has_cell) return fail(c, SKX_E_STATE, "set_cell first");
  (void)hipSetDevice(c->device);
  hipStream_t s = c->stream;
  const long long M = (long long)c->n1 * c->n2 * c->n3;
  const int nb = deviation_blocks(M);
  double *scr = nullptr;
  hipError_t e = hipMallocAsync((void **)&scr, sizeof(double) * (nb + 1), s);
  if (e != hipSuccess) return hip_fail(c, e, "deviation scratch");
  const double dV = c->L * c->L * c->L / (double)M;
  e = density_deviation((const double *)a_dev, (const double *)b_dev, M, dV, scr, scr + nb, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, scr + nb, sizeof(double), hipMemcpyDeviceToHost, s);
  const hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  (void)hipFreeAsync(scr, s);
  if (e != hipSuccess) return hip_fail(c, e, "deviation kernels");
  return SKX_OK;
}

int skx_fit_beta(skx_ctx *c, const void *rho_ref_dev, void *rho_dev, double beta_lo,
                 double beta_hi, double xtol, const skx_opt_params *p, double *beta_out,
                 double *dev_out, int *nsolves) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!rho_ref_dev || !rho_dev || !p || !beta_out) return fail(c, SKX_E_INVALID, "null argument");
  if (!(beta_lo < beta_hi) || !std::isfinite(beta_lo) || !std::isfinite(beta_hi))
    return fail(c, SKX_E_INVALID, "need a finite interval beta_lo < beta_hi");
  if (!(xtol > 0)) return fail(c, SKX_E_INVALID, "xtol must be positive");
  if (!c->has_cell || !c->has_ions || !c->has_fn)
    return fail(c, SKX_E_STATE, "set_cell, set_ions and set_functional must precede this call");
  const skx_functional fn0 = c->fn;
  int solves = 0, err = SKX_OK;
  double last = 0.0;
  // D(beta): minimise at beta (warm-started from rho_dev after the first
  // solve), then the integrated absolute deviation from the reference
  auto D = [&](double beta) {
    skx_functional fn = fn0;
    fn.beta = beta;
    int rc = skx_set_functional(c, &fn);
    skx_opt_params q = *p;
    q.warm_start = (solves > 0 || p->warm_start) ? 1 : 0;
    skx_opt_result res;
    if (rc == SKX_OK) rc = skx_optimize_density(c, rho_dev, &q, &res);
    ++solves;
    last = beta;
    double d = 0.0;
    if (rc >= 0) rc = skx_density_deviation(c, rho_dev, rho_ref_dev, &d);
    if (rc < 0) { err = rc; return HUGE_VAL; }
    return d;
  };
  // Brent's minimisation on [beta_lo, beta_hi]: golden-section steps with
  // parabolic interpolation through the three best points when it stays
  // inside the bracket and shrinks the step (Brent 1973, ch. 5)
  const double gold = 0.5 * (3.0 - std::sqrt(5.0));
  double a = beta_lo, b = beta_hi;
  double x = a + gold * (b - a), w = x, v = x;
  double fx = D(x), fw = fx, fv = fx;
  double d = 0.0, e = 0.0;
  for (int it = 0; it < 200 && err == SKX_OK; ++it) {
    const double m = 0.5 * (a + b);
    const double tol1 = 1e-10 * std::fabs(x) + xtol / 3.0, tol2 = 2.0 * tol1;
    if (std::fabs(x - m) <= tol2 - 0.5 * (b - a)) break;
    bool golden = true;
    if (std::fabs(e) > tol1) {
      double r = (x - w) * (fx - fv), q = (x - v) * (fx - fw);
      double pp = (x - v) * q - (x - w) * r;
      q = 2.0 * (q - r);
      if (q > 0.0) pp = -pp; else q = -q;
      const double e_prev = e;
      e = d;
      if (std::fabs(pp) < std::fabs(0.5 * q * e_prev) && pp > q * (a - x) && pp < q * (b - x)) {
        d = pp / q;
        const double u = x + d;
        if (u - a < tol2 || b - u < tol2) d = x < m ? tol1 : -tol1;
        golden = false;
      }
    }
    if (golden) {
      e = (x < m ? b : a) - x;
      d = gold * e;
    }
    const double u = std::fabs(d) >= tol1 ? x + d : x + (d > 0.0 ? tol1 : -tol1);
    const double fu = D(u);
    if (err != SKX_OK) break;
    if (fu <= fx) {
      if (u < x) b = x; else a = x;
      v = w; fv = fw; w = x; fw = fx; x = u; fx = fu;
    } else {
      if (u < x) a = u; else b = u;
      if (fu <= fw || w == x) { v = w; fv = fw; w = u; fw = fu; }
      else if (fu <= fv || v == x || v == w) { v = u; fv = fu; }
    }
  }
  // leave rho_dev at the minimum of the returned beta
  if (err == SKX_OK && last != x) fx = D(x);
  skx_set_functional(c, &fn0);
  if (err != SKX_OK) return err;
  *beta_out = x;
  if (dev_out) *dev_out = fx;
  if (nsolves) *nsolves = solves;
  return SKX_OK;
}

}  // extern "C"

namespace {

// Half a step (h = dt/2) of the Nose-Hoover thermostat, symmetric in
// itself: xi += (h/2) G, v *= exp(-xi h), eta += xi h, xi += (h/2) G with
// G = (2 K - g T_ion) / Q, K the ionic kinetic energy, g = 3 N_ion.
void nose_hoover_half(skx_nose_hoover *nh, double h, double *vel, const double *mass,
                      const std::vector<int> &species, int nions) {
  auto kinetic = [&] {
    double k = 0.0;
    for (int i = 0; i < nions; ++i)
      for (int a = 0; a < 3; ++a) k += 0.5 * mass[species[i]] * vel[3 * i + a] * vel[3 * i + a];
    return k;
  };
  const double g = 3.0 * nions;
  nh->xi += 0.5 * h * (2.0 * kinetic() - g * nh->T_ion) / nh->Q;
  const double sc = std::exp(-nh->xi * h);
  for (int i = 0; i < 3 * nions; ++i) vel[i] *= sc;
  nh->eta += nh->xi * h;
  nh->xi += 0.5 * h * (2.0 * kinetic() - g * nh->T_ion) / nh->Q;
}

// Velocity Verlet with a warm-started density minimisation and forces at
// the new positions; with nh, wrapped in two Nose-Hoover half steps.
int md_step_impl(skx_ctx *c, void *rho_dev, double *pos, double *vel, double *force,
                 const double *mass, double dt, skx_nose_hoover *nh, const skx_opt_params *p,
                 skx_opt_result *res) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!rho_dev || !pos || !vel || !force || !mass || !p || !res)
    return fail(c, SKX_E_INVALID, "null argument");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(c, SKX_E_INVALID, "dt must be positive");
  if (nh && (!(nh->Q > 0) || !std::isfinite(nh->Q) || !(nh->T_ion >= 0) || !std::isfinite(nh->xi)))
    return fail(c, SKX_E_INVALID, "thermostat needs Q > 0, T_ion >= 0 and a finite xi");
  if (!c->has_cell || !c->has_ions || !c->has_fn)
    return fail(c, SKX_E_STATE, "set_cell, set_ions and set_functional must precede this call");
  const int nions = (int)c->species.size();
  for (int k = 0; k < c->nspecies; ++k)
    if (!(mass[k] > 0) || !std::isfinite(mass[k])) return fail(c, SKX_E_INVALID, "masses must be positive");
  const std::vector<int> sp(c->species);
  if (nh) nose_hoover_half(nh, 0.5 * dt, vel, mass, sp, nions);
  // half kick and drift (positions are wrapped into the cell by set_ions)
  for (int i = 0; i < nions; ++i) {
    const double m = mass[sp[i]];
    for (int a = 0; a < 3; ++a) {
      vel[3 * i + a] += 0.5 * dt * force[3 * i + a] / m;
      pos[3 * i + a] += dt * vel[3 * i + a];
    }
  }
  const std::vector<double> z(c->zsp), r(c->rcsp);
  int rc = skx_set_ions(c, nions, pos, sp.data(), (int)z.size(), z.data(), r.data());
  if (rc != SKX_OK) return rc;
  for (int i = 0; i < 3 * nions; ++i) pos[i] = c->pos[i];
  // start density: extrapolated from this and the previous step's minimum
  // (the ctx keeps the previous one; the first step starts from rho_dev)
  {
    const long long M = (long long)c->n1 * c->n2 * c->n3;
    hipError_t e = hipSuccess;
    if (c->md_prev && c->md_prev_n == M) {
      hipLaunchKernelGGL(k_md_extrapolate, dim3(blocks(M, 256)), dim3(256), 0, c->stream,
                         (double *)rho_dev, c->md_prev, M);
      e = hipGetLastError();
    } else {
      (void)hipFree(c->md_prev);
      c->md_prev = nullptr;
      c->md_prev_n = 0;
      e = hipMalloc((void **)&c->md_prev, sizeof(double) * M);
      if (e == hipSuccess)
        e = hipMemcpyAsync(c->md_prev, rho_dev, sizeof(double) * M, hipMemcpyDeviceToDevice, c->stream);
      if (e == hipSuccess) c->md_prev_n = M;
    }
    if (e != hipSuccess) return hip_fail(c, e, "MD start density");
  }
  skx_opt_params q = *p;
  q.warm_start = 1;
  rc = skx_optimize_density(c, rho_dev, &q, res);
  if (rc < 0) return rc;
  const int status = rc;
  std::vector<double> fl(3 * (size_t)nions), fi(3 * (size_t)nions);
  rc = skx_ion_forces(c, rho_dev, SKX_RHO, fl.data(), fi.data());
  if (rc != SKX_OK) return rc;
  for (int i = 0; i < nions; ++i) {
    const double m = mass[sp[i]];
    for (int a = 0; a < 3; ++a) {
      force[3 * i + a] = fl[3 * i + a] + fi[3 * i + a];
      vel[3 * i + a] += 0.5 * dt * force[3 * i + a] / m;
    }
  }
  if (nh) nose_hoover_half(nh, 0.5 * dt, vel, mass, sp, nions);
  return status;
}

}  // namespace

extern "C" {

int skx_pressure(skx_ctx *c, const void *rho_dev, double eps, const skx_opt_params *p, double *P,
                 double *F_lo, double *F_hi) {
  if (!c) return SKX_E_INVALID;
  c->err.clear();
  if (!rho_dev || !p || !P) return fail(c, SKX_E_INVALID, "null argument");
  if (!(eps > 0.0 && eps < 0.1)) return fail(c, SKX_E_INVALID, "eps must be in (0, 0.1)");
  if (!c->has_cell || !c->has_ions || !c->has_fn)
    return fail(c, SKX_E_STATE, "set_cell, set_ions and set_functional must precede this call");
  (void)hipSetDevice(c->device);
  hipStream_t s = c->stream;
  const double L0 = c->L, V0 = L0 * L0 * L0;
  const int n1 = c->n1, n2 = c->n2, n3 = c->n3;
  const int nions = (int)c->species.size();
  const std::vector<double> pos0(c->pos), z(c->zsp), r(c->rcsp);
  const std::vector<int> sp(c->species);
  const size_t M = (size_t)n1 * n2 * n3;
  void *work = nullptr;
  hipError_t e = hipMalloc(&work, sizeof(double) * M);
  if (e != hipSuccess) return hip_fail(c, e, "pressure work density");
  double F[2] = {0.0, 0.0}, V[2] = {0.0, 0.0};
  int rc = SKX_OK;
  int worst = SKX_OK;                // SKX_NOT_CONVERGED of either solve is kept
  for (int k = 0; k < 2 && rc >= 0; ++k) {
    // the cell scaled to V0 (1 -+ eps), ions at fixed fractional positions
    V[k] = V0 * (k == 0 ? 1.0 - eps : 1.0 + eps);
    const double L = std::cbrt(V[k]);
    const double lat[9] = {L, 0, 0, 0, L, 0, 0, 0, L};
    std::vector<double> pos(pos0);
    for (double &x : pos) x *= L / L0;
    rc = skx_set_cell(c, lat, n1, n2, n3);
    if (rc == SKX_OK) rc = skx_set_ions(c, nions, pos.data(), sp.data(), (int)z.size(), z.data(), r.data());
    if (rc == SKX_OK) {
      e = hipMemcpyAsync(work, rho_dev, sizeof(double) * M, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) rc = hip_fail(c, e, "density copy");
    }
    skx_opt_params q = *p;
    q.warm_start = 1;
    skx_opt_result res;
    if (rc == SKX_OK) rc = skx_optimize_density(c, work, &q, &res);
    if (rc >= 0) F[k] = res.e.total;
    if (rc > worst) worst = rc;
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(work);
  // restore the configuration (the error text of a failed solve is kept)
  const std::string err = c->err;
  const double lat0[9] = {L0, 0, 0, 0, L0, 0, 0, 0, L0};
  int rc2 = skx_set_cell(c, lat0, n1, n2, n3);
  if (rc2 == SKX_OK) rc2 = skx_set_ions(c, nions, pos0.data(), sp.data(), (int)z.size(), z.data(), r.data());
  if (rc < 0) { c->err = err; return rc; }
  if (rc2 != SKX_OK) return rc2;
  *P = -(F[1] - F[0]) / (V[1] - V[0]);
  if (F_lo) *F_lo = F[0];
  if (F_hi) *F_hi = F[1];
  return worst;
}

int skx_md_step(skx_ctx *c, void *rho_dev, double *pos, double *vel, double *force,
                const double *mass, double dt, const skx_opt_params *p, skx_opt_result *res) {
  return md_step_impl(c, rho_dev, pos, vel, force, mass, dt, nullptr, p, res);
}

int skx_md_step_nvt(skx_ctx *c, void *rho_dev, double *pos, double *vel, double *force,
                    const double *mass, double dt, skx_nose_hoover *nh, const skx_opt_params *p,
                    skx_opt_result *res) {
  if (!nh) return c ? fail(c, SKX_E_INVALID, "thermostat state is NULL") : SKX_E_INVALID;
  return md_step_impl(c, rho_dev, pos, vel, force, mass, dt, nh, p, res);
}

int skx_run_batch(skx_ctx **ctxs, int nctx, void **rho_devs, const skx_opt_params *p,
                  skx_opt_result *res) {
  if (!ctxs || nctx < 1 || !rho_devs || !p || !res) return SKX_E_INVALID;
  skx_ctx *c0 = ctxs[0];
  if (!c0) return SKX_E_INVALID;
  c0->err.clear();
  if (p->lbfgs_m < 1 || p->lbfgs_m > MMAX) return fail(c0, SKX_E_INVALID, "lbfgs_m must be in 1..8");
  if (!(p->gtol > 0) || p->max_iter < 1) return fail(c0, SKX_E_INVALID, "gtol > 0 and max_iter >= 1 required");
  for (int i = 0; i < nctx; ++i) {
    if (!ctxs[i] || !rho_devs[i]) return fail(c0, SKX_E_INVALID, "null context or density");
    if (ctxs[i]->device != c0->device) return fail(c0, SKX_E_INVALID, "all contexts must share a device");
    if (!ctxs[i]->has_fn || ctxs[i]->fn.precision != c0->fn.precision)
      return fail(c0, SKX_E_INVALID, "all contexts must use the same precision mode");
  }
  hipSetDevice(c0->device);
  const int mode = c0->fn.precision;
  std::vector<int> precs;
  if (mode == SKX_FP64) precs = {0};
  else if (mode == SKX_FP32) precs = {1};
  else precs = {1, 0};
  for (int i = 0; i < nctx; ++i) {
    std::memset(&res[i], 0, sizeof(skx_opt_result));
    // FP64 first: the FP32 instance then copies its V_loc(G) (ensure_vloc)
    for (int pr : {0, 1}) {
      if (std::find(precs.begin(), precs.end(), pr) == precs.end()) continue;
      int rc = prepare(ctxs[i], pr, p->lbfgs_m);
      if (rc) { c0->err = "solve " + std::to_string(i) + ": " + ctxs[i]->err; return rc; }
    }
    (void)hipStreamSynchronize(ctxs[i]->stream);
  }
  hipStream_t s = c0->stream;
  SolveDev *ddev = nullptr;
  int *dfirst = nullptr;
  OptState *dstage = nullptr;           // packed states (upload and readback)
  OptState **dsptr = nullptr;           // each solve's state buffer
  hipError_t e = hipMallocAsync((void **)&ddev, sizeof(SolveDev) * batch_desc_count(nctx), s);
  if (e == hipSuccess)
    e = hipMallocAsync((void **)&dfirst, sizeof(int) * batch_first_count(nctx), s);
  if (e == hipSuccess) e = hipMallocAsync((void **)&dstage, sizeof(OptState) * nctx, s);
  if (e == hipSuccess) e = hipMallocAsync((void **)&dsptr, sizeof(OptState *) * nctx, s);
  if (e != hipSuccess) return hip_fail(c0, e, "batch descriptors");
  std::vector<OptState> outs(nctx), o32(nctx);
  int rc = SKX_OK;
  for (size_t ph = 0; ph < precs.size() && rc == SKX_OK; ++ph) {
    const int pr = precs[ph];
    const bool last = ph + 1 == precs.size();
    const double gtol = last ? p->gtol
                             : std::max(p->gtol, p->fp32_switch_gtol > 0 ? p->fp32_switch_gtol : 1e-5);
    std::vector<SolveDev> hs;
    std::vector<OptState *> states;
    std::vector<OptState> init;
    std::vector<int> members;                 // solves of this phase
    for (int i = 0; i < nctx; ++i) {
      // a numerical failure of the FP32 phase ends that solve (no refinement)
      if (ph > 0 && o32[i].phase == PH_FAILED && o32[i].status < 0) continue;
      members.push_back(i);
      Instance &I = ctxs[i]->inst[pr];
      const long long M = I.h.M;
      int start = 0;
      if (ph > 0) {
        hipLaunchKernelGGL(k_f2d, dim3(blocks(M, 256)), dim3(256), 0, s,
                           (const float *)ctxs[i]->inst[1].h.phi2[o32[i].par], (double *)I.h.phi2[0],
                           M);
        start = 2;
      } else if (p->warm_start) {
        start = 1;
        if (pr == 0)
          hipLaunchKernelGGL(k_from_rho<double>, dim3(blocks(M, 256)), dim3(256), 0, s,
                             (const double *)rho_devs[i], (double *)I.h.phi2[0], M);
        else
          hipLaunchKernelGGL(k_from_rho<float>, dim3(blocks(M, 256)), dim3(256), 0, s,
                             (const double *)rho_devs[i], (float *)I.h.phi2[0], M);
      } else {
        const double v = std::sqrt(ctxs[i]->ne / (ctxs[i]->L * ctxs[i]->L * ctxs[i]->L));
        if (pr == 0)
          hipLaunchKernelGGL(k_fill<double>, dim3(blocks(M, 256)), dim3(256), 0, s,
                             (double *)I.h.phi2[0], v, M);
        else
          hipLaunchKernelGGL(k_fill<float>, dim3(blocks(M, 256)), dim3(256), 0, s,
                             (float *)I.h.phi2[0], (float)v, M);
      }
      init.emplace_back();
      init_state(init.back(), *p, gtol, start == 1 ? 1 : 0, pr);
      hs.push_back(I.h);
      states.push_back(I.st);
    }
    const int nm = (int)members.size();
    if (nm == 0) continue;
    // every state in one copy, scattered to the solves' buffers on the device
    e = hipMemcpyAsync(dstage, init.data(), sizeof(OptState) * nm, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dsptr, states.data(), sizeof(OptState *) * nm, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_put_states, dim3(nm), dim3(64), 0, s, dstage, dsptr, nm);
      e = hipGetLastError();
    }
    if (e != hipSuccess) { rc = hip_fail(c0, e, "state upload"); break; }
    rc = drive(c0, hs, pr, ddev, dfirst, (p->max_iter + 2) * 24 + 64, s);
    if (rc) break;
    hipLaunchKernelGGL(k_get_states, dim3(nm), dim3(64), 0, s, dsptr, dstage, nm);
    e = hipGetLastError();
    std::vector<OptState> got(nm);
    if (e == hipSuccess)
      e = hipMemcpyAsync(got.data(), dstage, sizeof(OptState) * nm, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) { rc = hip_fail(c0, e, "state readback"); break; }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) { rc = hip_fail(c0, e, "batch"); break; }
    for (int k = 0; k < nm; ++k) (last ? outs : o32)[members[k]] = got[k];
  }
  if (rc == SKX_OK) {
    for (int i = 0; i < nctx; ++i) {
      // a solve whose FP32 phase failed numerically reports that phase
      const bool failed32 = precs.size() > 1 && o32[i].phase == PH_FAILED && o32[i].status < 0;
      if (failed32) outs[i] = o32[i];
      const int pr = failed32 ? 1 : precs.back();
      Instance &I = ctxs[i]->inst[pr];
      const OptState &o = outs[i];
      if (pr == 0)
        hipLaunchKernelGGL(k_square_out<double>, dim3(blocks(I.h.M, 256)), dim3(256), 0, s,
                           (const double *)I.h.phi2[o.par], (double *)rho_devs[i], I.h.M);
      else
        hipLaunchKernelGGL(k_square_out<float>, dim3(blocks(I.h.M, 256)), dim3(256), 0, s,
                           (const float *)I.h.phi2[o.par], (double *)rho_devs[i], I.h.M);
      energy_from(o.e_acc, ctxs[i]->e_ii, &res[i].e);
      res[i].gnorm = o.rnorm;
      res[i].resets = o.resets;
      if (failed32) {
        res[i].fp32_iters = res[i].iters = o32[i].iters;
        res[i].fp32_evals = res[i].evals = o32[i].evals;
      } else if (precs.size() > 1) {
        res[i].fp32_iters = o32[i].iters;
        res[i].fp32_evals = o32[i].evals;
        res[i].iters = o.iters + o32[i].iters;
        res[i].evals = o.evals + o32[i].evals;
      } else {
        res[i].iters = o.iters;
        res[i].evals = o.evals;
        if (pr == 1) { res[i].fp32_iters = o.iters; res[i].fp32_evals = o.evals; }
      }
      if (o.phase == PH_FAILED && o.status < 0) res[i].status = o.status;
      else res[i].status = (o.phase == PH_DONE && o.status == 0) ? SKX_OK : SKX_NOT_CONVERGED;
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(c0, e, "batch output");
  }
  hipFreeAsync(ddev, s);
  (void)hipFreeAsync(dfirst, s);
  (void)hipFreeAsync(dstage, s);
  (void)hipFreeAsync(dsptr, s);
  (void)hipStreamSynchronize(s);
  if (rc) return rc;
  int worst = SKX_OK;
  for (int i = 0; i < nctx; ++i)
    if (res[i].status != SKX_OK) worst = (res[i].status < 0) ? res[i].status : (worst < 0 ? worst : SKX_NOT_CONVERGED);
  return worst;
}

}  // extern "C"

// ===========================================================================
// Instrumentation
// ===========================================================================
extern "C" {

int skx_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
  return SKX_OK;
}

unsigned skx_profile_mask(unsigned mask) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  const unsigned old = g_prof.mask;
  g_prof.mask = mask;
  return old;
}

int skx_set_autotune(int on) {
  const int old = g_autotune ? 1 : 0;
  g_autotune = on != 0;
  return old;
}

int skx_set_plane_chunking(int force) {
  const int old = g_chunk_planes ? 1 : 0;
  g_chunk_planes = force != 0;
  return old;
}

int skx_set_shape_kernels(int mask) {
  const int old = g_shape_kernels;
  g_shape_kernels = mask & 7;
  return old;
}

int skx_get_radix_order(int n, int precision, int *radices, int max) {
  if (n < 2 || n > 512 || !radices || max < 1) return SKX_E_INVALID;
  const int prec = precision == SKX_FP32 ? 1 : 0;
  const std::vector<int> r = g_tuned[prec][n].empty() ? radix_candidates(n)[0] : g_tuned[prec][n];
  const int k = std::min((int)r.size(), max);
  for (int i = 0; i < k; ++i) radices[i] = r[i];
  return (int)r.size();
}

int skx_set_graphs(int on) {
  const int old = g_graphs ? 1 : 0;
  g_graphs = on != 0;
  return old;
}

int skx_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (int i = 0; i < PP_N; ++i) { g_prof.ms[i] = 0; g_prof.count[i] = 0; }
  return SKX_OK;
}

int skx_profile_read(double *ms, long long *launches, int n) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (n < 0) return SKX_E_INVALID;
  prof_fold();
  for (int i = 0; i < n && i < PP_N; ++i) {
    if (ms) ms[i] = g_prof.ms[i];
    if (launches) launches[i] = g_prof.count[i];
  }
  return PP_N;
}

}  // extern "C"

// ===========================================================================
// Pass timing over a batch (used by the tile/launch autotuner and tools)
// ===========================================================================
extern "C" int skx_bench_eval(skx_ctx **ctxs, int nctx, int reps, double *ms_out) {
  if (!ctxs || nctx < 1 || reps < 1 || !ms_out) return SKX_E_INVALID;
  skx_ctx *c0 = ctxs[0];
  c0->err.clear();
  (void)hipSetDevice(c0->device);
  const int prec = c0->fn.precision == SKX_FP32 ? 1 : 0;
  for (int i = 0; i < nctx; ++i) {
    if (!ctxs[i] || ctxs[i]->device != c0->device) return fail(c0, SKX_E_INVALID, "bad context");
    int rc = prepare(ctxs[i], prec, 1);
    if (rc) { c0->err = ctxs[i]->err; return rc; }
    (void)hipStreamSynchronize(ctxs[i]->stream);
  }
  hipStream_t s = c0->stream;
  std::vector<SolveDev> hs;
  for (int i = 0; i < nctx; ++i) {
    Instance &I = ctxs[i]->inst[prec];
    const double v = std::sqrt(ctxs[i]->ne / (ctxs[i]->L * ctxs[i]->L * ctxs[i]->L));
    if (prec == 0)
      hipLaunchKernelGGL(k_fill<double>, dim3(blocks(I.h.M, 256)), dim3(256), 0, s,
                         (double *)I.h.phi2[0], v, I.h.M);
    else
      hipLaunchKernelGGL(k_fill<float>, dim3(blocks(I.h.M, 256)), dim3(256), 0, s,
                         (float *)I.h.phi2[0], (float)v, I.h.M);
    OptState st{};
    st.phase = PH_EVAL_ONLY;
    (void)hipMemcpyAsync(I.st, &st, sizeof(OptState), hipMemcpyHostToDevice, s);
    hs.push_back(I.h);
  }
  SolveDev *ddev = nullptr;
  int *dfirst = nullptr;
  hipError_t e = hipMallocAsync((void **)&ddev, sizeof(SolveDev) * batch_desc_count(nctx), s);
  if (e == hipSuccess)
    e = hipMallocAsync((void **)&dfirst, sizeof(int) * batch_first_count(nctx), s);
  if (e != hipSuccess) return hip_fail(c0, e, "bench descriptors");
  BatchLaunch bl{};
  int rc = build_batch(c0, hs, prec, ddev, dfirst, bl, s);
  if (rc == SKX_OK) {
    hipEvent_t ev[4];
    for (auto &x : ev) hipEventCreate(&x);
    double tot[3] = {0, 0, 0};
    for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {
      (void)hipEventRecord(ev[0], s);
      e = launch_eval(bl, s, 1);
      (void)hipEventRecord(ev[1], s);
      if (e == hipSuccess) e = launch_eval(bl, s, 2);
      (void)hipEventRecord(ev[2], s);
      if (e == hipSuccess) e = launch_eval(bl, s, 4);
      (void)hipEventRecord(ev[3], s);
      (void)hipEventSynchronize(ev[3]);
      if (r == 0) continue;            // first repetition warms caches
      for (int q = 0; q < 3; ++q) {
        float t = 0.f;
        (void)hipEventElapsedTime(&t, ev[q], ev[q + 1]);
        tot[q] += t;
      }
    }
    for (auto &x : ev) hipEventDestroy(x);
    for (int q = 0; q < 3; ++q) ms_out[q] = tot[q] / reps;
    if (e != hipSuccess) rc = hip_fail(c0, e, "bench passes");
  }
  hipFreeAsync(ddev, s);
  (void)hipFreeAsync(dfirst, s);
  (void)hipStreamSynchronize(s);
  return rc;
}
