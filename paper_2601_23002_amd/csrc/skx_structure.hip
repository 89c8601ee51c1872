// Static structure factors of one snapshot (Methods, static structure
// factors): S_ab(q) = <n_a(q) n_b*(q)> / sqrt(N_a N_b), averaged over the
// grid's wave vectors of equal |q|, with
//   n_e(q) = V n~(q)                  (n~ the 1/M-normalised spectrum),
//   n_i(q) = sum_I exp(-i q.R_I)      (all ions as one species),
// shells s = g1^2 + g2^2 + g3^2 of the index map (Nyquist -> -n/2), every
// grid index counted once, real parts of the products.
//
// k_sf_items: one thread per half-spectrum index; n_i from the per-axis
// phase tables exp(-2 pi i g x) summed over the ions. An index with
// 0 < k3 < n3/2 also stands for its conjugate partner, whose products equal
// its own except on the Nyquist rows of x or y (there the partner's G is not
// -G and its ion sum is formed separately). k_shell_sum then adds the items
// of each shell in a fixed order (host-built list sorted by shell, a fixed
// lane assignment and shuffle tree), so the result is deterministic.
#include "skx_internal.hpp"

namespace skx {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(256) void k_sf_items(const double2 *spec, int n1, int n2, int n3,
                                                  int nh, int pitch, double V, const double2 *ph,
                                                  int nions, double *val) {
  const long long item = (long long)blockIdx.x * 256 + threadIdx.x;
  if (item >= (long long)n1 * n2 * nh) return;
  const int row = (int)(item / nh), k3 = (int)(item - (long long)row * nh);
  const int k1 = row / n2, k2 = row - (row / n2) * n2;
  const int q1 = (n1 - k1) % n1, q2 = (n2 - k2) % n2;
  const bool pair = k3 > 0 && 2 * k3 < n3;
  const bool nyq = 2 * k1 == n1 || 2 * k2 == n2;
  const int stride = n1 + n2 + nh;
  const double2 t = spec[(size_t)row * pitch + k3];
  const double ex = V * t.x, ey = V * t.y;                  // n_e(G)
  double2 ni = make_double2(0.0, 0.0), np = make_double2(0.0, 0.0);
  for (int I = 0; I < nions; ++I) {
    const double2 *p = ph + (size_t)I * stride;
    const double2 pz = p[n1 + n2 + k3];
    const double2 e = cmul(cmul(p[k1], p[n1 + k2]), pz);    // exp(-i G.R_I)
    ni.x += e.x;
    ni.y += e.y;
    if (pair && nyq) {
      // partner G' = (h1, h2, -g3): exp(-i G'.R) with the z factor conjugated
      const double2 e2 = cmul(cmul(p[q1], p[n1 + q2]), make_double2(pz.x, -pz.y));
      np.x += e2.x;
      np.y += e2.y;
    }
  }
  const double ee = ex * ex + ey * ey;
  double a = ex * ni.x + ey * ni.y;                          // Re[n_e conj(n_i)]
  double b = ee;
  double c = ni.x * ni.x + ni.y * ni.y;
  if (pair && !nyq) {
    a *= 2.0; b *= 2.0; c *= 2.0;
  } else if (pair) {
    // the partner's electron coefficient is conj(n_e(G))
    a += ex * np.x - ey * np.y;
    b += ee;
    c += np.x * np.x + np.y * np.y;
  }
  val[3 * item] = a;
  val[3 * item + 1] = b;
  val[3 * item + 2] = c;
}

// out[4 s + (0..3)] = S_ei, S_ee, S_ii, count of shell s, from the items of
// the shell (list idx[off[s] .. off[s+1])): one wavefront per shell, lane l
// adding list entries l, l + 64, ... in order, then a fixed shuffle tree.
__global__ __launch_bounds__(256) void k_shell_sum(const double *val, const int *off,
                                                   const int *idx, int nshell, int n3, int nh,
                                                   double norm_ei, double norm_ee,
                                                   double norm_ii, double *out) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (s >= nshell) return;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = off[s] + lane; j < off[s + 1]; j += 64) {
    const int it = idx[j];
    const int k3 = it % nh;
    v[0] += val[3 * (size_t)it];
    v[1] += val[3 * (size_t)it + 1];
    v[2] += val[3 * (size_t)it + 2];
    v[3] += (k3 > 0 && 2 * k3 < n3) ? 2.0 : 1.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
  if (lane == 0) {
    const double inv = v[3] > 0.0 ? 1.0 / v[3] : 0.0;
    out[4 * s] = v[0] * inv * norm_ei;
    out[4 * s + 1] = v[1] * inv * norm_ee;
    out[4 * s + 2] = v[2] * inv * norm_ii;
    out[4 * s + 3] = v[3];
  }
}

}  // namespace

hipError_t structure_items(const double2 *spec, int n1, int n2, int n3, int pitch, double V,
                           const double2 *ph, int nions, double *val, hipStream_t s) {
  const long long items = (long long)n1 * n2 * (n3 / 2 + 1);
  SKX_TIMED_LAUNCH(k_sf_items, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, spec, n1,
                   n2, n3, n3 / 2 + 1, pitch, V, ph, nions, val);
  return hipGetLastError();
}

hipError_t structure_shells(const double *val, const int *off, const int *idx, int nshell, int n3,
                            double norm_ei, double norm_ee, double norm_ii, double *out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_shell_sum, dim3((nshell + 3) / 4), dim3(256), 0, s, val, off, idx,
                     nshell, n3, n3 / 2 + 1, norm_ei, norm_ee, norm_ii, out);
  return hipGetLastError();
}

}  // namespace skx
