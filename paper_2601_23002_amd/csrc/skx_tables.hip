// Set-up kernels of libskx: FFT twiddle bank, the universal Fermi-Dirac
// table, the nonlocal kernel tables w(q), w'(q), the local pseudopotential
// through the ionic structure factor, and the Ewald ion-ion energy.
//
// All of these run once per solve (or once per device) on the GPU; the hot
// loop only reads their results.
#include "skx_internal.hpp"
#include "skx_device.hpp"
#include <math.h>
#include <type_traits>

namespace skx {

// ---------------------------------------------------------------------------
// FFT twiddle bank: for every planned length n, exp(-2 pi i k / n), k < n.
// ---------------------------------------------------------------------------
__global__ void k_twiddles(double2 *bank, const int *sizes, const int *offsets, int nsizes) {
  int s = blockIdx.x;
  if (s >= nsizes) return;
  int n = sizes[s];
  double2 *out = bank + offsets[s];
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)k / (double)n, &sn, &cs);
    out[k] = make_double2(cs, -sn);
  }
}

hipError_t build_twiddles(double *bank_dev, const int *sizes, const int *offsets, int nsizes,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_twiddles, dim3(nsizes), dim3(256), 0, s,
                     reinterpret_cast<double2 *>(bank_dev), sizes, offsets, nsizes);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fermi-Dirac integrals by the trapezoidal rule on the whole real line.
//
// With x = t^2, I_nu(eta) = int_0^inf 2 t^(2nu+1) F(t^2 - eta) dt and the
// integrand is even and analytic in a strip whose half-width is the
// imaginary part of sqrt(eta + i pi) (the nearest pole of the Fermi
// function). The trapezoidal rule then converges like exp(-2 pi d / h);
// h = d / 7 gives about 1e-19 relative. This route is independent of the
// panel Gauss-Legendre quadrature a CPU reference may use.
// ---------------------------------------------------------------------------
struct FDSums { double i_m12, i_12, i_32, di_m12; };

// Degenerate limit: the Sommerfeld expansion
//   I_nu(eta) = eta^(nu+1)/(nu+1) + sum_k 2 (1 - 2^(1-2k)) zeta(2k)
//               nu (nu-1) ... (nu-2k+2) eta^(nu-2k+1),
// whose neglected terms are below 1e-17 relative for eta > 300, with
// exponentially small (exp(-eta)) corrections.
__device__ void sommerfeld(double nu, double eta, double &val, double &deriv) {
  const double PI2 = 9.8696044010893586188;
  const double c[4] = {PI2 / 6.0, 7.0 * PI2 * PI2 / 360.0, 31.0 * PI2 * PI2 * PI2 / 15120.0,
                       127.0 * PI2 * PI2 * PI2 * PI2 / 604800.0};
  val = pow(eta, nu + 1.0) / (nu + 1.0);
  deriv = pow(eta, nu);
  double fall = nu;                  // nu (nu-1) ... (nu-2k+2)
  double pw = pow(eta, nu - 1.0);    // eta^(nu-2k+1)
  for (int k = 1; k <= 4; ++k) {
    const double ex = nu - 2.0 * k + 1.0;
    val += c[k - 1] * fall * pw;
    deriv += c[k - 1] * fall * ex * pw / eta;
    fall *= (nu - 2.0 * k + 1.0) * (nu - 2.0 * k);
    pw /= eta * eta;
  }
}

__device__ FDSums fd_trapezoid(double eta) {
  const double PI = 3.14159265358979323846;
  if (eta > 300.0) {
    FDSums r;
    double dd;
    sommerfeld(-0.5, eta, r.i_m12, r.di_m12);
    sommerfeld(0.5, eta, r.i_12, dd);
    sommerfeld(1.5, eta, r.i_32, dd);
    return r;
  }
  double mod = sqrt(eta * eta + PI * PI);
  double d = sqrt(0.5 * (mod - eta));
  double h = d / 7.0;
  if (h > 0.1) h = 0.1;
  double tmax = sqrt(fmax(eta, 0.0) + 62.0);
  int nk = (int)ceil(tmax / h);
  FDSums r{0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k <= nk; ++k) {
    double t = k * h;
    double x = t * t - eta;
    double F, dF;
    if (x > 0) { double e = exp(-x); F = e / (1.0 + e); dF = F * (1.0 / (1.0 + e)); }
    else       { double e = exp(x);  F = 1.0 / (1.0 + e); dF = F * (e / (1.0 + e)); }
    double wgt = (k == 0) ? 0.5 : 1.0;
    double t2 = t * t;
    r.i_m12 += wgt * 2.0 * F;
    r.i_12 += wgt * 2.0 * t2 * F;
    r.i_32 += wgt * 2.0 * t2 * t2 * F;
    r.di_m12 += wgt * 2.0 * dF;
  }
  r.i_m12 *= h; r.i_12 *= h; r.i_32 *= h; r.di_m12 *= h;
  return r;
}

// eta with I_1/2(eta) = exp(y): Newton on ln I_1/2, which is concave and
// increasing in eta, so the iteration converges from any start.
__device__ double fd_invert(double y, FDSums *out) {
  const double LN_G32 = -0.12078223763524522;   // ln Gamma(3/2)
  double u = exp(y);
  double eta = (y < 1.0) ? (y - LN_G32) : pow(1.5 * u, 2.0 / 3.0);
  FDSums s{};
  for (int it = 0; it < 100; ++it) {
    s = fd_trapezoid(eta);
    double g = log(s.i_12) - y;
    double step = g / (0.5 * s.i_m12 / s.i_12);
    eta -= step;
    if (fabs(step) <= 1e-15 * fmax(1.0, fabs(eta))) break;
  }
  s = fd_trapezoid(eta);
  if (out) *out = s;
  return eta;
}

// One thread per node y_k = y0 + k h: eta(y_k), its first two derivatives
// and psi = eta - (2/3) I_3/2(eta) / u, u = exp(y). With dI_1/2/deta =
// I_-1/2 / 2:  eta' = 2u / I_-1/2,  eta'' = eta' (1 - eta' I_-1/2' / I_-1/2).
__global__ void k_fd_nodes(double *node, double y0, double h, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > n) return;
  double y = y0 + h * k;
  FDSums s;
  double eta = fd_invert(y, &s);
  double u = exp(y);
  double d1 = 2.0 * u / s.i_m12;
  double d2 = d1 * (1.0 - d1 * s.di_m12 / s.i_m12);
  node[4 * k + 0] = eta;
  node[4 * k + 1] = d1;
  node[4 * k + 2] = d2;
  node[4 * k + 3] = eta - (2.0 / 3.0) * s.i_32 / u;
}

hipError_t build_fd_table(double *node_dev, double y0, double h, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fd_nodes, dim3((n + 1 + 63) / 64), dim3(64), 0, s, node_dev, y0, h, n);
  return hipGetLastError();
}

__global__ void k_debug_fd(const double *u, double *eta, double *psi, long long n, FDTable fd) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double e, p;
  fd_lookup(log(u[i]), fd, e, p);
  eta[i] = e;
  psi[i] = p;
}

hipError_t debug_fd_eval(const double *u_dev, double *eta_dev, double *psi_dev, long long n,
                         const FDTable &fd, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_fd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, u_dev,
                     eta_dev, psi_dev, n, fd);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Nonlocal kernel tables on integer shells s = g1^2 + g2^2 + g3^2.
//
// The kernel makes TF + vW + F0 reproduce the free-gas static response at
// the mean density (the F0 kernel is the second functional derivative at
// the mean valence density, Results around Eq. (2)):
//   K(q) = -1/chi0(q) - dmu0/dn - q^2/(4 n0),  w = K n0^(2-2a) / (2 a^2)
// chi0 is computed in the integrated-by-parts form
//   chi0(q) = -(1/(pi^2 q T)) int_0^inf g(k) k f(1-f) dk,
//   g(k) = (k^2/2 - q^2/8) ln|(2k+q)/(2k-q)| + q k / 2,
// which is continuous at k = q/2, and w' = dw/dn0 analytically through
// d f / d eta0 = f(1-f) and d eta0 / d n0 = 2 / (n_T I_{-1/2}(eta0)).
// Quadrature: tanh-sinh on intervals split at q/2 and around the Fermi edge.
// ---------------------------------------------------------------------------
struct Chi { double chi, dchi; };

// One wavefront per shell: lane l takes the nodes k = -K + l, -K + l + 64,
// ... of every interval, the lane sums are added across the wavefront.
__device__ Chi chi0_byparts(double q, double T, double eta0, int lane) {
  const double PI = 3.14159265358979323846;
  double kmax = sqrt(2.0 * T * (fmax(eta0, 0.0) + 55.0));
  double pts[6];
  int np = 0;
  pts[np++] = 0.0;
  double half = fmin(0.5 * q, kmax);
  double extra[3];
  int ne = 0;
  if (eta0 > 0) {
    double kf = sqrt(2.0 * T * eta0), wid = 3.0 * T / kf;
    extra[ne++] = fmax(kf - wid, 0.0);
    extra[ne++] = kf;
    extra[ne++] = fmin(kf + wid, kmax);
  }
  // insertion sort of {half, extra...} into pts
  double cand[4];
  int nc = 0;
  cand[nc++] = half;
  for (int i = 0; i < ne; ++i) cand[nc++] = extra[i];
  for (int i = 1; i < nc; ++i) {
    double v = cand[i]; int j = i - 1;
    while (j >= 0 && cand[j] > v) { cand[j + 1] = cand[j]; --j; }
    cand[j + 1] = v;
  }
  for (int i = 0; i < nc; ++i) pts[np++] = cand[i];
  pts[np++] = kmax;
  const double h = 1.0 / 40.0;
  const int K = 150;                       // |t| <= 3.75
  double acc = 0.0, dacc = 0.0;
  for (int c = 0; c + 1 < np; ++c) {
    double a = pts[c], b = pts[c + 1], L = b - a;
    if (!(L > 0)) continue;
    bool lsing = (a == half) && (half == 0.5 * q);
    bool rsing = (b == half) && (half == 0.5 * q);
    double sum = 0.0, dsum = 0.0;
    for (int k = -K + lane; k <= K; k += 64) {
      double t = k * h;
      double u = 0.5 * PI * sinh(t);
      double ch = cosh(u);
      double wgt = 0.5 * PI * cosh(t) / (ch * ch);
      double fl = 1.0 / (1.0 + exp(-2.0 * u));   // (k - a) / L
      double fr = 1.0 / (1.0 + exp(2.0 * u));    // (b - k) / L
      double kk = a + L * fl;
      double dist;                               // |k - q/2|
      if (lsing) dist = L * fl;
      else if (rsing) dist = L * fr;
      else dist = fabs(kk - 0.5 * q);
      double g;
      if (dist > 0.0) {
        double lg = log(2.0 * kk + q) - log(2.0 * dist);
        g = 0.5 * (kk - 0.5 * q) * (kk + 0.5 * q) * lg + 0.5 * q * kk;
      } else {
        g = 0.5 * q * kk;
      }
      double x = kk * kk / (2.0 * T) - eta0;
      double f = (x > 0) ? exp(-x) / (1.0 + exp(-x)) : 1.0 / (1.0 + exp(x));
      double ff = f * (1.0 - f);
      sum += wgt * g * kk * ff;
      dsum += wgt * g * kk * ff * (1.0 - 2.0 * f);
    }
    acc += 0.5 * L * h * sum;
    dacc += 0.5 * L * h * dsum;
  }
  for (int off = 32; off > 0; off >>= 1) {
    acc += __shfl_down(acc, off, 64);
    dacc += __shfl_down(dacc, off, 64);
  }
  Chi r;
  r.chi = -acc / (PI * PI * q * T);
  r.dchi = -dacc / (PI * PI * q * T);
  return r;
}

__device__ double fd_table_eta(double y, const FDTable &fd) {
  double e, p;
  fd_lookup(y, fd, e, p);
  return e;
}

__global__ __launch_bounds__(256) void k_kernel_tables(double *w, double *wp, int smax, double L,
                                                       double n0, double T, double a, double eta0,
                                                       double im12, double dim12) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (s > smax) return;
  if (s == 0) {
    if (lane == 0) { w[0] = 0.0; wp[0] = 0.0; }
    return;
  }
  const double PI = 3.14159265358979323846;
  const double SQ2 = 1.41421356237309504880;
  double q = (2.0 * PI / L) * sqrt((double)s);
  Chi c = chi0_byparts(q, T, eta0, lane);
  if (lane != 0) return;
  double dmudn = SQ2 * PI * PI / (sqrt(T) * im12);
  double K = -1.0 / c.chi - dmudn - q * q / (4.0 * n0);
  double pref = pow(n0, 2.0 - 2.0 * a) / (2.0 * a * a);
  double nT = SQ2 / (PI * PI) * T * sqrt(T);
  double deta_dn0 = 2.0 / (nT * im12);
  double ddmudn_deta = -SQ2 * PI * PI / (sqrt(T) * im12 * im12) * dim12;
  double dK_deta = c.dchi / (c.chi * c.chi) - ddmudn_deta;
  double dK_dn0 = dK_deta * deta_dn0 + q * q / (4.0 * n0 * n0);
  w[s] = K * pref;
  wp[s] = dK_dn0 * pref + K * (2.0 - 2.0 * a) * pow(n0, 1.0 - 2.0 * a) / (2.0 * a * a);
}

__global__ void k_uniform_gas(double *out, double n0, double T, FDTable fd) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double PI = 3.14159265358979323846;
  double nT = 1.41421356237309504880 / (PI * PI) * T * sqrt(T);
  double eta0 = fd_table_eta(log(n0 / nT), fd);
  FDSums s = fd_trapezoid(eta0);
  out[0] = eta0;
  out[1] = s.i_m12;
  out[2] = s.di_m12;
}

hipError_t build_kernel_tables(double *w, double *wp, int smax, double L, double n0, double T,
                               double a, const FDTable &fd, double *gas_out, hipStream_t s) {
  double *tmp = nullptr;
  hipError_t e = hipMallocAsync((void **)&tmp, 4 * sizeof(double), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_uniform_gas, dim3(1), dim3(64), 0, s, tmp, n0, T, fd);
  double host[3];
  e = hipMemcpyAsync(host, tmp, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFreeAsync(tmp, s);
  if (e != hipSuccess) return e;
  if (gas_out) { gas_out[0] = host[0]; gas_out[1] = host[1]; gas_out[2] = host[2]; }
  hipLaunchKernelGGL(k_kernel_tables, dim3((smax + 1 + 3) / 4), dim3(256), 0, s, w, wp, smax, L,
                     n0, T, a, host[0], host[1], host[2]);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Local pseudopotential through the ionic structure factor.
//
// V(G) = (1/V) sum_I v_I(G) exp(-i G.R_I),  v(G) = -4 pi Z exp(-G^2 rc^2/4)/G^2,
// V(0) = (1/V) sum_I pi Z_I rc_I^2. On an even grid the potential is the
// real part of the plane-wave sum, so the spectrum is replaced by its
// Hermitian part (V(m) + conj V(-m))/2. With the phase factorised per axis,
// exp(-i G.R) = Q P where P collects the Nyquist axes of m and Q the others;
// flipping the sign of every Nyquist component conjugates P only, so the
// Hermitian part is Q Re(P).
// ---------------------------------------------------------------------------
__global__ void k_phase_tables(double2 *ph, int nions, const double *pos, int n1, int n2, int nh3,
                               int n3, double L) {
  // layout per ion: [n1 | n2 | nh3]
  int stride = n1 + n2 + nh3;
  long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= (long long)nions * stride) return;
  int I = (int)(idx / stride), m = (int)(idx % stride);
  int ax, mm, n;
  if (m < n1) { ax = 0; mm = m; n = n1; }
  else if (m < n1 + n2) { ax = 1; mm = m - n1; n = n2; }
  else { ax = 2; mm = m - n1 - n2; n = n3; }
  double x = pos[3 * I + ax] / L;               // fractional coordinate
  int g = (2 * mm < n) ? mm : mm - n;           // Nyquist maps to -n/2
  // exp(-2 pi i g x), argument reduced exactly in fractional units
  double arg = 2.0 * g * x;
  arg -= 2.0 * floor(0.5 * arg);
  double sn, cs;
  sincospi(arg, &sn, &cs);
  ph[idx] = make_double2(cs, -sn);
}

template <typename R>
__global__ void k_vloc(void *vloc_v, int n1, int n2, int n3, int nh, int pitch, double L,
                       int nions, const double2 *ph, const int *species, int nspecies,
                       const double *zval, const double *rc) {
  typedef typename std::conditional<sizeof(R) == 8, double2, float2>::type V2;
  V2 *vloc = reinterpret_cast<V2 *>(vloc_v);
  long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  long long tot = (long long)n1 * n2 * nh;
  if (idx >= tot) return;
  int k3 = (int)(idx % nh);
  long long t = idx / nh;
  int k2 = (int)(t % n2), k1 = (int)(t / n2);
  const double PI = 3.14159265358979323846;
  double V = L * L * L;
  int g1 = (2 * k1 < n1) ? k1 : k1 - n1;
  int g2 = (2 * k2 < n2) ? k2 : k2 - n2;
  int g3 = k3;
  double G2 = (2.0 * PI / L) * (2.0 * PI / L) * (double)(g1 * g1 + g2 * g2 + g3 * g3);
  int stride = n1 + n2 + nh;
  const bool ny1 = (2 * k1 == n1), ny2 = (2 * k2 == n2), ny3 = (2 * k3 == n3);
  double re = 0.0, im = 0.0;
  if (g1 == 0 && g2 == 0 && g3 == 0) {
    for (int I = 0; I < nions; ++I) {
      int sp = species[I];
      re += PI * zval[sp] * rc[sp] * rc[sp];
    }
  } else {
    // accumulate the structure factor per species, then weight by v_s(G)
    for (int sp = 0; sp < nspecies; ++sp) {
      double sr = 0.0, si = 0.0;
      for (int I = 0; I < nions; ++I) {
        if (species[I] != sp) continue;
        const double2 *p = ph + (size_t)I * stride;
        const double2 f[3] = {p[k1], p[n1 + k2], p[n1 + n2 + k3]};
        double qr = 1.0, qi = 0.0, pr = 1.0, pi = 0.0;
        for (int a = 0; a < 3; ++a) {
          const bool nyq = (a == 0) ? ny1 : (a == 1) ? ny2 : ny3;
          double &xr = nyq ? pr : qr;
          double &xi = nyq ? pi : qi;
          const double tr = xr * f[a].x - xi * f[a].y;
          xi = xr * f[a].y + xi * f[a].x;
          xr = tr;
        }
        sr += qr * pr;
        si += qi * pr;
      }
      double vG = -4.0 * PI * zval[sp] * exp(-G2 * rc[sp] * rc[sp] / 4.0) / G2;
      re += vG * sr;
      im += vG * si;
    }
  }
  V2 out;
  out.x = (R)(re / V);
  out.y = (R)(im / V);
  vloc[((size_t)k1 * n2 + k2) * pitch + k3] = out;
}

hipError_t ion_phase_tables(double2 *ph, int nions, const double *pos_dev, int n1, int n2, int n3,
                            double L, hipStream_t s) {
  const int nh = n3 / 2 + 1;
  const long long ntab = (long long)nions * (n1 + n2 + nh);
  if (ntab > 0)
    hipLaunchKernelGGL(k_phase_tables, dim3((unsigned)((ntab + 255) / 256)), dim3(256), 0, s, ph,
                       nions, pos_dev, n1, n2, nh, n3, L);
  return hipGetLastError();
}

hipError_t build_vloc(void *vloc, int prec, int n1, int n2, int n3, int pitch, double L,
                      int nions, const double *pos_dev, const int *species_dev, int nspecies,
                      const double *zval_dev, const double *rc_dev, double2 *phase_scratch,
                      hipStream_t s) {
  int nh = n3 / 2 + 1;
  long long ntab = (long long)nions * (n1 + n2 + nh);
  if (ntab > 0)
    hipLaunchKernelGGL(k_phase_tables, dim3((unsigned)((ntab + 255) / 256)), dim3(256), 0, s,
                       phase_scratch, nions, pos_dev, n1, n2, nh, n3, L);
  long long tot = (long long)n1 * n2 * nh;
  if (prec == 0)
    hipLaunchKernelGGL(k_vloc<double>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, vloc,
                       n1, n2, n3, nh, pitch, L, nions, phase_scratch, species_dev, nspecies,
                       zval_dev, rc_dev);
  else
    hipLaunchKernelGGL(k_vloc<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, vloc,
                       n1, n2, n3, nh, pitch, L, nions, phase_scratch, species_dev, nspecies,
                       zval_dev, rc_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ewald energy of the point ions in a neutralising background.
// Real-space part: one thread per ion pair (i <= j) summing periodic images;
// reciprocal part: one thread per G vector. Partial sums are reduced in a
// fixed order by a single workgroup (deterministic).
// ---------------------------------------------------------------------------
// One wavefront per ion pair i <= j: the lanes share the periodic images.
__global__ __launch_bounds__(256) void k_ewald_real(double *part, int nions, const double *pos,
                                                    const double *Z, double L, double alpha,
                                                    int nimg, double rcut) {
  const long long npair = (long long)nions * (nions + 1) / 2;
  const long long idx = blockIdx.x * 4LL + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= npair) return;
  // decode (i, j) with i <= j: row i starts at S(i) = i n - i (i - 1) / 2;
  // the root of S(i) = idx, then exact integer fix-ups
  auto row_start = [&](long long r) { return r * nions - r * (r - 1) / 2; };
  const double b = 2.0 * nions + 1.0;
  long long i = (long long)floor(0.5 * (b - sqrt(fmax(0.0, b * b - 8.0 * (double)idx))));
  if (i < 0) i = 0;
  if (i > nions - 1) i = nions - 1;
  while (i > 0 && row_start(i) > idx) --i;
  while (i < nions - 1 && row_start(i + 1) <= idx) ++i;
  const int j = (int)(i + (idx - row_start(i)));
  const double dx = pos[3 * i] - pos[3 * j], dy = pos[3 * i + 1] - pos[3 * j + 1],
               dz = pos[3 * i + 2] - pos[3 * j + 2];
  const int side = 2 * nimg + 1, nimgs = side * side * side;
  double acc = 0.0;
  for (int m = lane; m < nimgs; m += 64) {
    const int a = m / (side * side) - nimg, b = (m / side) % side - nimg, c = m % side - nimg;
    const double x = dx + a * L, y = dy + b * L, z = dz + c * L;
    const double r = sqrt(x * x + y * y + z * z);
    if (r > 0.0 && r < rcut) acc += erfc(alpha * r) / r;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) part[idx] = acc * ((i == j) ? 0.5 : 1.0) * Z[i] * Z[j];
}

__global__ void k_ewald_recip(double *part, int nions, const double *pos, const double *Z, double L,
                              double alpha, int mmax, double gcut2) {
  int side = 2 * mmax + 1;
  long long ng = (long long)side * side * side;
  long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (idx < ng) {
    int a = (int)(idx / (side * side)) - mmax;
    int b = (int)((idx / side) % side) - mmax;
    int c = (int)(idx % side) - mmax;
    const double PI = 3.14159265358979323846;
    double k = 2.0 * PI / L;
    double G2 = k * k * (double)(a * a + b * b + c * c);
    if ((a | b | c) != 0 && G2 < gcut2) {
      double sr = 0.0, si = 0.0;
      for (int I = 0; I < nions; ++I) {
        double arg = 2.0 * (a * pos[3 * I] + b * pos[3 * I + 1] + c * pos[3 * I + 2]) / L;
        arg -= 2.0 * floor(0.5 * arg);
        double sn, cs;
        sincospi(arg, &sn, &cs);
        sr += Z[I] * cs;
        si += Z[I] * sn;
      }
      double V = L * L * L;
      acc = (2.0 * PI / V) * (sr * sr + si * si) * exp(-G2 / (4.0 * alpha * alpha)) / G2;
    }
    part[idx] = acc;
  }
}

__global__ void k_sum_fixed(const double *part, long long n, double *out, int slot) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[slot] = sh[0];
}

hipError_t ewald_energy(double L, int nions, const double *pos_dev, const double *charge_dev,
                        double *scratch_dev, int scratch_len, double *out_dev, hipStream_t s) {
  // out_dev[0] = real, [1] = reciprocal (host adds self and background)
  double alpha = 3.2 / L;
  double rcut = 6.5 / alpha;
  int nimg = (int)ceil(rcut / L) + 1;
  long long npair = (long long)nions * (nions + 1) / 2;
  double gcut = 2.0 * alpha * sqrt(44.0);
  int mmax = (int)ceil(gcut * L / (2.0 * 3.14159265358979323846));
  long long side = 2 * mmax + 1;
  long long ng = side * side * side;
  if (npair > scratch_len || ng > scratch_len) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ewald_real, dim3((unsigned)((npair + 3) / 4)), dim3(256), 0, s,
                     scratch_dev, nions, pos_dev, charge_dev, L, alpha, nimg, rcut);
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, scratch_dev, npair, out_dev, 0);
  hipLaunchKernelGGL(k_ewald_recip, dim3((unsigned)((ng + 127) / 128)), dim3(128), 0, s,
                     scratch_dev, nions, pos_dev, charge_dev, L, alpha, mmax, gcut * gcut);
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, scratch_dev, ng, out_dev, 1);
  return hipGetLastError();
}

}  // namespace skx
