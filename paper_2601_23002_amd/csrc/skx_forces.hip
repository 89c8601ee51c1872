// Forces on the ions at a given density, for molecular dynamics in the NVT
// ensemble (Methods, molecular dynamics and static structure factors). At
// the minimising density only the position-dependent energy terms move the
// ions (Hellmann-Feynman): the local pseudopotential energy and the Ewald
// ion-ion energy.
//
// Local part, from the density's half spectrum n~ (plane-wave coefficients,
// 1/M normalised) and the per-axis ion phase tables exp(-2 pi i g x):
//   F_I = sum_m G_m v_I(G_m) Im[exp(i G_m.R_I) n~(m)],
//   v(G) = -4 pi Z exp(-G^2 rc^2 / 4) / G^2,
// summed over every index m of the full grid with G_m from the index map
// (Nyquist -> -n/2). The half spectrum holds k3 in [0, n3/2]; an index with
// 0 < k3 < n3/2 stands for itself and its conjugate partner
// ((-k1) mod n1, (-k2) mod n2, n3 - k3), whose term equals its own except on
// the Nyquist rows of x or y, where the partner's G is not -G and its term
// is added explicitly.
//
// Ewald part: real-space sum over ion pairs and images, reciprocal sum over
// G with the structure factor S(G) = sum_J Z_J exp(i G.R_J), the same split
// (alpha = 3.2 / L, real cutoff 6.5 / alpha, |G| < 2 alpha sqrt(44)) as the
// Ewald energy.
//
// Every reduction runs in a fixed order (per-workgroup partials, then one
// ordered sum per ion), so results are deterministic.
#include "skx_internal.hpp"

#include <algorithm>

namespace skx {

namespace {

constexpr double PI_D = 3.14159265358979323846;

// Sum of NV doubles over a 256-thread workgroup; the totals land in tot on
// every thread. red holds 4 * NV doubles.
template <int NV>
__device__ __forceinline__ void group_sum(double (&v)[NV], double *red, double (&tot)[NV]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wave * NV + q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) tot[q] = ((red[q] + red[NV + q]) + red[2 * NV + q]) + red[3 * NV + q];
  __syncthreads();
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }

// One thread per segment of KS consecutive k3 of a (k1, k2) row of the half
// spectrum, one workgroup row per tile of IT ions (ions sorted by species,
// so the form factor is computed once per G point and species run).
// part[(I * gridDim.x + blockIdx.x) * 3 + c] receives this workgroup's share
// of F_I.
template <int IT, int KS>
__global__ __launch_bounds__(256) void k_force_loc(const double2 *spec, int n1, int n2, int n3,
                                                   int nh, int pitch, double L, const double2 *ph,
                                                   const int *order, int nions, const int *species,
                                                   const double *zval, const double *rc,
                                                   double *part) {
  __shared__ double red[4 * 3];
  const int nseg = (nh + KS - 1) / KS;
  const long long item = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool live = item < (long long)n1 * n2 * nseg;
  const int row = live ? (int)(item / nseg) : 0;
  const int seg = live ? (int)(item - (long long)row * nseg) : 0;
  const int k1 = row / n2, k2 = row - (row / n2) * n2;
  const int g1 = 2 * k1 < n1 ? k1 : k1 - n1, g2 = 2 * k2 < n2 ? k2 : k2 - n2;
  // partner row and its G components (differ from -g only on Nyquist rows)
  const int q1 = (n1 - k1) % n1, q2 = (n2 - k2) % n2;
  const int h1 = 2 * q1 < n1 ? q1 : q1 - n1, h2 = 2 * q2 < n2 ? q2 : q2 - n2;
  const bool nyq = 2 * k1 == n1 || 2 * k2 == n2;
  const int stride = n1 + n2 + nh;
  const double kk = 2.0 * PI_D / L;
  int ion[IT];
  double2 pxy[IT];
  double f[IT][3];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int idx = blockIdx.y * IT + i;
    ion[i] = idx < nions ? order[idx] : -1;
    f[i][0] = f[i][1] = f[i][2] = 0.0;
    pxy[i] = make_double2(0.0, 0.0);
    if (ion[i] >= 0) {
      const double2 *p = ph + (size_t)ion[i] * stride;
      // the tables hold exp(-2 pi i g x); conjugate for exp(+i G.R)
      pxy[i] = conjd(cmul(p[k1], p[n1 + k2]));
    }
  }
  if (live) {
    const double2 *srow = spec + (size_t)row * pitch;
    const int kend = min(nh, (seg + 1) * KS);
    for (int k3 = seg * KS; k3 < kend; ++k3) {
      const int g3 = 2 * k3 < n3 ? k3 : k3 - n3;
      const double G2 = kk * kk * (double)(g1 * g1 + g2 * g2 + g3 * g3);
      if (G2 == 0.0) continue;
      const bool pair = k3 > 0 && 2 * k3 < n3;
      const double2 nt = srow[k3];
      int csp = -1;
      double vf = 0.0;
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        if (ion[i] < 0) continue;
        const int sp = species[ion[i]];
        if (sp != csp) {
          csp = sp;
          const double r = rc[sp];
          vf = -4.0 * PI_D * zval[sp] * exp(-G2 * r * r * 0.25) / G2;
        }
        const double2 pz = ph[(size_t)ion[i] * stride + n1 + n2 + k3];   // exp(-i G3 x3)
        const double2 e = cmul(pxy[i], conjd(pz));                       // exp(+i G.R)
        double t = vf * (e.x * nt.y + e.y * nt.x);                       // v Im[e n~]
        if (pair && !nyq) t *= 2.0;
        f[i][0] += t * g1;
        f[i][1] += t * g2;
        f[i][2] += t * g3;
        if (pair && nyq) {
          const double2 *p = ph + (size_t)ion[i] * stride;
          const double2 qxy = conjd(cmul(p[q1], p[n1 + q2]));
          const double2 ep = cmul(qxy, pz);                              // partner phase
          const double tp = vf * (ep.y * nt.x - ep.x * nt.y);            // v Im[e' conj(n~)]
          f[i][0] += tp * h1;
          f[i][1] += tp * h2;
          f[i][2] -= tp * g3;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    double v[3] = {f[i][0], f[i][1], f[i][2]}, tot[3];
    group_sum<3>(v, red, tot);
    if (threadIdx.x < 3 && ion[i] >= 0)
      part[((size_t)ion[i] * gridDim.x + blockIdx.x) * 3 + threadIdx.x] = kk * tot[threadIdx.x];
  }
}

// out[I][c] = sum over the row blocks of part, in order.
__global__ void k_force_sum(const double *part, int nblk, int nions, double *out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * nions) return;
  const int I = idx / 3, c = idx - 3 * I;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += part[((size_t)I * nblk + b) * 3 + c];
  out[idx] = acc;
}

// Real-space Ewald force on ion i, split over gridDim.y workgroups: lanes
// run over (J, image) pairs, d = R_i - R_J + L t, r = |d| in (0, rcut):
//   F_i += Z_i Z_J [erfc(a r)/r^2 + 2a/sqrt(pi) exp(-a^2 r^2)/r] d/r;
// part[(i * gridDim.y + blockIdx.y) * 3 + c] receives each share.
__global__ __launch_bounds__(256) void k_ewald_force_real(double *part, int nions, const double *pos,
                                                          const double *Z, double L, double alpha,
                                                          int nimg, double rcut) {
  __shared__ double red[4 * 3];
  const int i = blockIdx.x;
  const int side = 2 * nimg + 1, nimgs = side * side * side;
  const long long tot = (long long)nions * nimgs;
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  const double c2 = 2.0 * alpha / sqrt(PI_D);
  double v[3] = {0.0, 0.0, 0.0};
  for (long long m = (long long)blockIdx.y * 256 + threadIdx.x; m < tot; m += 256LL * gridDim.y) {
    const int j = (int)(m / nimgs), t = (int)(m - (long long)j * nimgs);
    const int a = t / (side * side) - nimg, b = (t / side) % side - nimg, c = t % side - nimg;
    const double x = xi - pos[3 * j] + a * L, y = yi - pos[3 * j + 1] + b * L,
                 z = zi - pos[3 * j + 2] + c * L;
    const double r = sqrt(x * x + y * y + z * z);
    if (r > 0.0 && r < rcut) {
      const double s = Z[j] * (erfc(alpha * r) / (r * r) + c2 * exp(-alpha * alpha * r * r) / r) / r;
      v[0] += s * x;
      v[1] += s * y;
      v[2] += s * z;
    }
  }
  double sum[3];
  group_sum<3>(v, red, sum);
  if (threadIdx.x < 3) part[((size_t)i * gridDim.y + blockIdx.y) * 3 + threadIdx.x] = Z[i] * sum[threadIdx.x];
}

// S(G) = sum_J Z_J exp(i G.R_J) on the cube of integer vectors |m_c| <= mmax;
// zero at G = 0 and outside the cutoff sphere.
__global__ void k_ewald_sf(double2 *S, int nions, const double *pos, const double *Z, double L,
                           int mmax, double gcut2) {
  const int side = 2 * mmax + 1;
  const long long ng = (long long)side * side * side;
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= ng) return;
  const int a = (int)(idx / (side * side)) - mmax, b = (int)((idx / side) % side) - mmax,
            c = (int)(idx % side) - mmax;
  const double k = 2.0 * PI_D / L;
  const double G2 = k * k * (double)(a * a + b * b + c * c);
  double sr = 0.0, si = 0.0;
  if ((a | b | c) != 0 && G2 < gcut2) {
    for (int J = 0; J < nions; ++J) {
      double arg = 2.0 * (a * pos[3 * J] + b * pos[3 * J + 1] + c * pos[3 * J + 2]) / L;
      arg -= 2.0 * floor(0.5 * arg);
      double sn, cs;
      sincospi(arg, &sn, &cs);
      sr += Z[J] * cs;
      si += Z[J] * sn;
    }
  }
  S[idx] = make_double2(sr, si);
}

// Reciprocal-space Ewald force on ion i (one workgroup per ion), added to
// the real-space part already in out:
//   F_i += (4 pi Z_i / V) sum_G G exp(-G^2/4a^2)/G^2 Im[exp(i G.R_i) conj(S(G))].
__global__ __launch_bounds__(256) void k_ewald_force_recip(double *out, const double2 *S,
                                                           const double *pos, const double *Z,
                                                           double L, double alpha, int mmax) {
  __shared__ double red[4 * 3];
  const int i = blockIdx.x;
  const int side = 2 * mmax + 1;
  const int ng = side * side * side;
  const double k = 2.0 * PI_D / L;
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  double v[3] = {0.0, 0.0, 0.0};
  for (int m = threadIdx.x; m < ng; m += 256) {
    const double2 s = S[m];
    if (s.x == 0.0 && s.y == 0.0) continue;
    const int a = m / (side * side) - mmax, b = (m / side) % side - mmax, c = m % side - mmax;
    const double G2 = k * k * (double)(a * a + b * b + c * c);
    double arg = 2.0 * (a * xi + b * yi + c * zi) / L;
    arg -= 2.0 * floor(0.5 * arg);
    double sn, cs;
    sincospi(arg, &sn, &cs);
    const double w = exp(-G2 / (4.0 * alpha * alpha)) / G2 * (sn * s.x - cs * s.y);
    v[0] += w * a;
    v[1] += w * b;
    v[2] += w * c;
  }
  double sum[3];
  group_sum<3>(v, red, sum);
  if (threadIdx.x < 3)
    out[3 * i + threadIdx.x] += 4.0 * PI_D * Z[i] / (L * L * L) * k * sum[threadIdx.x];
}

}  // namespace

constexpr int FORCE_IT = 4, FORCE_KS = 16, EWALD_SPLIT = 16;

int force_row_blocks(int n1, int n2, int n3) {
  const long long items = (long long)n1 * n2 * ((n3 / 2 + 1 + FORCE_KS - 1) / FORCE_KS);
  return std::max((int)((items + 255) / 256), EWALD_SPLIT);
}

hipError_t local_forces(const double2 *spec, int n1, int n2, int n3, int pitch, double L,
                        const double2 *ph, const int *order_dev, int nions, const int *species_dev,
                        const double *zval_dev, const double *rc_dev, double *part_dev,
                        double *out_dev, hipStream_t s) {
  constexpr int IT = FORCE_IT;
  const long long items = (long long)n1 * n2 * ((n3 / 2 + 1 + FORCE_KS - 1) / FORCE_KS);
  const int nblk = (int)((items + 255) / 256);
  SKX_TIMED_LAUNCH((k_force_loc<IT, FORCE_KS>), dim3(nblk, (nions + IT - 1) / IT), dim3(256), 0, s, spec,
                   n1, n2, n3, n3 / 2 + 1, pitch, L, ph, order_dev, nions, species_dev, zval_dev,
                   rc_dev, part_dev);
  hipLaunchKernelGGL(k_force_sum, dim3((3 * nions + 255) / 256), dim3(256), 0, s, part_dev, nblk,
                     nions, out_dev);
  return hipGetLastError();
}

int ewald_force_terms(double L) {
  const double alpha = 3.2 / L;
  const int mmax = (int)ceil(2.0 * alpha * sqrt(44.0) * L / (2.0 * PI_D));
  return (2 * mmax + 1) * (2 * mmax + 1) * (2 * mmax + 1);
}

hipError_t ewald_forces(double L, int nions, const double *pos_dev, const double *charge_dev,
                        double2 *sf_dev, double *part_dev, double *out_dev, hipStream_t s) {
  const double alpha = 3.2 / L;
  const double rcut = 6.5 / alpha;
  const int nimg = (int)ceil(rcut / L) + 1;
  const double gcut = 2.0 * alpha * sqrt(44.0);
  const int mmax = (int)ceil(gcut * L / (2.0 * PI_D));
  const int ng = (2 * mmax + 1) * (2 * mmax + 1) * (2 * mmax + 1);
  SKX_TIMED_LAUNCH(k_ewald_force_real, dim3(nions, EWALD_SPLIT), dim3(256), 0, s, part_dev, nions,
                   pos_dev, charge_dev, L, alpha, nimg, rcut);
  hipLaunchKernelGGL(k_force_sum, dim3((3 * nions + 255) / 256), dim3(256), 0, s, part_dev,
                     EWALD_SPLIT, nions, out_dev);
  SKX_TIMED_LAUNCH(k_ewald_sf, dim3((ng + 255) / 256), dim3(256), 0, s, sf_dev, nions, pos_dev,
                     charge_dev, L, mmax, gcut * gcut);
  SKX_TIMED_LAUNCH(k_ewald_force_recip, dim3(nions), dim3(256), 0, s, out_dev, sf_dev, pos_dev,
                     charge_dev, L, alpha, mmax);
  return hipGetLastError();
}

}  // namespace skx
