// The functional evaluation of libskx as three fused passes over a batch of
// solves, and the same three passes reused to apply the optimiser's
// preconditioner.
//
// Evaluation (MODE_EVAL):
//   pass A  real space, one workgroup per (solve, x-plane, field):
//           trial point phi_t = cos(t) phi + sqrt(N_e) sin(t) d/|d|, the
//           pointwise fields phi, n = phi^2, f = n^a, h = (f - n0^a)(n - n0),
//           the local energy densities (finite-T TF through the Fermi-Dirac
//           table, PZ LDA), then the real-to-complex z transform and the y
//           transform of the plane in LDS.
//   pass B  reciprocal space, one workgroup per (solve, y index, z block):
//           x transform of the column block, every G-space energy term and
//           the four reciprocal multipliers, inverse x transform.
//   pass C  real space, one workgroup per (solve, x-plane): inverse y and
//           complex-to-real z transforms of the four outputs, assembled with
//           their pointwise coefficients into dE/dphi.
//
// Energy terms (paper Eq. (1), Eq. (2); readings as stated in include/skx.h):
//   F_TF = dV sum f_TF(n),   F_vW = (V/2) sum G^2 |phi~|^2,
//   F0 = V sum w |f~|^2,     F1 = (V/3) sum w' Re(f~ h~*),
//   E_H = (V/2) sum' 4 pi |n~|^2 / G^2,  E_loc = V sum Re(n~ V_loc*),
//   E_xc = dV sum n eps_xc(n).
// dE/dphi = A + 2 phi [B + T eta + v_xc] + c_P P + c_Q Q with
//   A = G^2 phi~, B = 4 pi n~/G^2 + V_loc, P = 2 w f~ + (beta/3) w' h~,
//   Q = (beta/3) w' f~, c_P = 2 a sign(phi)|phi|^(2a-1),
//   c_Q = c_P (n - n0) + 2 phi (f - n0^a).
//
// Preconditioner (MODE_PREC), for solves whose trial point was accepted:
//   pass A  r_t = dE/dphi - 2 mu_t phi_t (stored), transformed like phi;
//   pass B  multiplied by 1 / (G^2 + kappa);
//   pass C  transformed back into P r_t.
#include "skx_device.hpp"
#include <math.h>

namespace skx {

constexpr int MAXB_A = 2;
constexpr int MAXB_C = 2;
constexpr int MAXB_B = 2;
// vector loads (pairs of grid values or complex values) each thread issues
// before using any of them
constexpr int LU_A = 4;
constexpr int LU_C = 2;
constexpr int LU_L = 8;
constexpr int LU_B = 4;
constexpr int MODE_EVAL = 0, MODE_PREC = 1;

// x^a for x >= 0 through exp(a ln x): in FP64 the error stays ~1e-15
// relative; in FP32 the hardware log2/exp2 keep it ~1e-6, the rounding level
// of the FP32 fields (a correctly rounded powf costs ~160 instructions).
template <typename R> __device__ __forceinline__ R rpow(R x, R a);
template <> __device__ __forceinline__ double rpow(double x, double a) {
  return x > 0.0 ? exp(a * log(x)) : 0.0;
}
template <> __device__ __forceinline__ float rpow(float x, float a) {
  return x > 1e-30f ? __builtin_amdgcn_exp2f(a * __builtin_amdgcn_logf(x)) : 0.0f;
}

// n^a for pass A is derived again from phi_t instead of being handed over
// by the pointwise kernel, and in FP32 so are pass C's assembly coefficients
// c_P, c_Q, which saves their round trips through HBM. FP32 takes n^a
// through the hardware log2/exp2; FP64 with a = 5/6 takes n^a = |phi|
// n^(1/3) with the cube root from an FP32 estimate and two Newton steps on
// n^(-1/3) (about 15 FP64 operations instead of a logarithm and an
// exponential), other a through exp(a ln n). FP64 pass C keeps the handed
// c_P, c_Q: deriving them there pushed it past its register budget.
template <typename R> constexpr bool derive_na() { return true; }
template <typename R> constexpr bool derive_coefs() { return sizeof(R) == 4; }

template <typename R> struct NaCfg {
  R a, a2, n0, n0a;
  bool a56;
};
template <typename R> __device__ __forceinline__ NaCfg<R> na_cfg(const SolveDev &S) {
  NaCfg<R> c;
  c.a = (R)S.a;
  c.a2 = (R)(2.0 * S.a);
  c.n0 = (R)S.n0;
  c.n0a = (R)S.n0a;
  c.a56 = S.a == 5.0 / 6.0;
  return c;
}

// x^(-1/3) for x > 0 in FP64: an FP32 estimate and two Newton steps on
// z^-3 = x (quadratic convergence from ~1e-7 to the FP64 rounding)
__device__ __forceinline__ double rcbrt_pos(double x) {
  if (x < 1e-30 || x > 1e30) return exp(log(x) * (-1.0 / 3.0));
  double z = (double)__builtin_amdgcn_exp2f(-0.333333343f * __builtin_amdgcn_logf((float)x));
  z = fma(z * (1.0 / 3.0), fma(-x * z, z * z, 1.0), z);
  z = fma(z * (1.0 / 3.0), fma(-x * z, z * z, 1.0), z);
  return z;
}
// x^(1/3) for x > 0 in FP64
__device__ __forceinline__ double cbrt_pos(double x) {
  const double z = rcbrt_pos(x);
  return x * z * z;
}

template <typename R> __device__ __forceinline__ R derived_na(R p, const NaCfg<R> &c);
// FP32: with L = log2 |phi|, n^a = 2^(2a L) and c_P = 2a sign(phi) 2^((2a-1) L)
// (no division); |phi| below 1e-15 gives 0 for both.
template <> __device__ __forceinline__ float derived_na(float p, const NaCfg<float> &c) {
  const float ap = fabsf(p);
  return ap > 1e-15f ? __builtin_amdgcn_exp2f(2.0f * c.a * __builtin_amdgcn_logf(ap)) : 0.0f;
}
template <> __device__ __forceinline__ double derived_na(double p, const NaCfg<double> &c) {
  const double n = p * p;
  if (!(n > 0.0)) return 0.0;
  return c.a56 ? fabs(p) * cbrt_pos(n) : exp(c.a * log(n));
}
// c_P (fb = 2) or c_Q (fb = 3) of one point
template <typename R> __device__ __forceinline__ R derived_coef(R p, int fb, const NaCfg<R> &c);
template <> __device__ __forceinline__ float derived_coef(float p, int fb, const NaCfg<float> &c) {
  const float n = p * p, ap = fabsf(p);
  float f = 0.0f, cP = 0.0f;
  if (ap > 1e-15f) {
    const float L = __builtin_amdgcn_logf(ap);
    f = __builtin_amdgcn_exp2f(2.0f * c.a * L);
    cP = copysignf(c.a2 * __builtin_amdgcn_exp2f((2.0f * c.a - 1.0f) * L), p);
  }
  return fb == 2 ? cP : cP * (n - c.n0) + 2.0f * p * (f - c.n0a);
}
template <> __device__ __forceinline__ double derived_coef(double p, int fb, const NaCfg<double> &c) {
  const double n = p * p;
  double f = 0.0, cP = 0.0;
  if (n > 0.0) {
    if (c.a56) {
      const double e3 = cbrt_pos(n);
      f = fabs(p) * e3;
      cP = copysign(c.a2 * e3, p);
    } else {
      f = exp(c.a * log(n));
      cP = c.a2 * f / p;
    }
  }
  return fb == 2 ? cP : cP * (n - c.n0) + 2.0 * p * (f - c.n0a);
}

__device__ __forceinline__ int nth_field(int mask, int c) {
  // bit index of the c-th set bit of mask (slot order phi, n, f, h)
  for (int b = 0; b < NFIELD; ++b)
    if (mask & (1 << b)) { if (c == 0) return b; --c; }
  return -1;
}

template <typename V>
__device__ __forceinline__ void load_twiddles(V *dst, const double *bank, int off, int n, int tid,
                                              int nthr) {
  const double2 *src = reinterpret_cast<const double2 *>(bank) + off;
  for (int k = tid; k < n; k += nthr) {
    double2 t = src[k];
    V v; v.x = t.x; v.y = t.y;
    dst[k] = v;
  }
}

// Trial-point coefficients: phi_t = ca phi + cb d.
__device__ __forceinline__ void trial_coef(const SKX_C OptState *st, const SolveDev &S, double &ca,
                                           double &cb, bool &use_d) {
  int ph = st->phase;
  if (ph == PH_TRIAL) {
    double sn, cs;
    sincos(st->theta, &sn, &cs);
    ca = cs;
    cb = S.sqrt_ne * sn / st->dnorm;
    use_d = true;
  } else {
    ca = (ph == PH_EVAL_INIT) ? st->theta : 1.0;   // theta holds the normalising scale
    cb = 0.0;
    use_d = false;
  }
}

template <int MODE> __device__ __forceinline__ bool active_phase(int ph) {
  if (MODE == MODE_PREC) return ph == PH_UPDATE;
  return ph == PH_EVAL_INIT || ph == PH_TRIAL || ph == PH_EVAL_ONLY;
}

// Complex values per lane the wavefront-owned transforms may stage.
#ifndef SKX_WAVEV_F32
#define SKX_WAVEV_F32 16
#endif
#ifndef SKX_WAVEV_F64
#define SKX_WAVEV_F64 8
#endif
template <typename R> struct WaveV {
  static constexpr int value = sizeof(R) == 4 ? SKX_WAVEV_F32 : SKX_WAVEV_F64;
};

// Real-to-complex split of the row pairs [lo, hi) after their z transform,
// by the wavefront that owns them (X_k of the pair 2p + i 2p+1 becomes the
// half spectra A_k of row 2p and B_k of row 2p+1, in place).
template <typename V, typename R, int U>
__device__ __forceinline__ void split_rows_w(V *buf, int lo, int hi, int n3, int nk, int pl,
                                             int lane) {
  const int tot = (hi - lo) * nk;
  const UDiv dnk = make_udiv((unsigned)nk);
  V A[U], B[U];
  int ia[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = lane + 64 * u;
    ia[u] = -1;
    if (e < tot) {
      const int q = (int)udiv((unsigned)e, dnk);
      const int p = lo + q, k = e - q * nk;
      const V X = buf[p * 2 * pl + k];
      const V Xm = buf[p * 2 * pl + (k == 0 ? 0 : n3 - k)];
      A[u].x = (R)0.5 * (X.x + Xm.x); A[u].y = (R)0.5 * (X.y - Xm.y);
      B[u].x = (R)0.5 * (X.y + Xm.y); B[u].y = (R)-0.5 * (X.x - Xm.x);
      ia[u] = 2 * p * pl + k;
    }
  }
  SKX_WAVE_SYNC();
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (ia[u] >= 0) { buf[ia[u]] = A[u]; buf[ia[u] + pl] = B[u]; }
  SKX_WAVE_SYNC();
}

// Complex-to-real merge of the row pairs [lo, hi) before their inverse z
// transform (X = A + i B over the full row, Hermitian-extended; the columns
// k = 0 and k = n3/2 keep only their real parts), by the owning wavefront.
template <typename V, typename R, int U>
__device__ __forceinline__ void merge_rows_w(V *buf, int lo, int hi, int n3, int pl, int lane) {
  const int tot = (hi - lo) * n3;
  const UDiv dn3 = make_udiv((unsigned)n3);
  V X[U];
  int ix[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = lane + 64 * u;
    ix[u] = -1;
    if (e < tot) {
      const int q = (int)udiv((unsigned)e, dn3);
      const int p = lo + q, k = e - q * n3;
      V Av, Bv;
      if (2 * k <= n3) {
        Av = buf[(2 * p) * pl + k];
        Bv = buf[(2 * p + 1) * pl + k];
        if (k == 0 || 2 * k == n3) { Av.y = 0; Bv.y = 0; }
      } else {
        Av = buf[(2 * p) * pl + n3 - k];
        Bv = buf[(2 * p + 1) * pl + n3 - k];
        Av.y = -Av.y; Bv.y = -Bv.y;
      }
      X[u].x = Av.x - Bv.y;
      X[u].y = Av.y + Bv.x;
      ix[u] = p * 2 * pl + k;
    }
  }
  SKX_WAVE_SYNC();
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (ix[u] >= 0) buf[ix[u]] = X[u];
  SKX_WAVE_SYNC();
}

// Real-to-complex z transform of the rows held pairwise in LDS (pair p at
// buf[2p pl ...] as x_{2p} + i x_{2p+1}), then the y transform of every
// z column. On exit (after a workgroup barrier) row j of the plane holds
// the half spectrum in [0, nh). Each step runs on wavefront-owned
// transforms when they fit in registers, else on the workgroup-wide stages.
template <typename V, typename R, int NT>
__device__ __forceinline__ void plane_forward(V *buf, const SolveDev &S, const V *tw2,
                                              const V *tw3, int tid) {
  constexpr int NW = NT / 64, MAXV = WaveV<R>::value;
  const int lane = tid & 63, wave = tid >> 6;
  const int n2 = S.n2, n3 = S.n3, nh = S.nh, pl = nh;
  const int nk = n3 / 2 + 1, cz = n2 / 2;
  const int zmax = (cz + NW - 1) / NW;
  if (wave_fits<MAXV>(S.p3, zmax) && zmax * nk <= 64 * (MAXV / 2)) {
    int lo, hi;
    wave_share(cz, wave, NW, lo, hi);
    fft_lds_w<V, MAXV, false>(buf, S.p3, lo, hi - lo, 1, 2 * pl, tw3, lane);
    split_rows_w<V, R, MAXV / 2>(buf, lo, hi, n3, nk, pl, lane);
    __syncthreads();
  } else {
    fft_lds<V, MAXB_A, false>(buf, S.p3, cz, 1, 2 * pl, tw3, tid, NT);
    int per = (MAXB_A * NT) / nk;
    if (per < 1) per = 1;
    const UDiv dnk = make_udiv((unsigned)nk);
    for (int p0 = 0; p0 < cz; p0 += per) {
      const int p1 = min(cz, p0 + per);
      const int tot = (p1 - p0) * nk;
      V A[MAXB_A], B[MAXB_A];
#pragma unroll
      for (int i = 0; i < MAXB_A; ++i) {
        const int e = tid + i * NT;
        if (e < tot) {
          const int q = (int)udiv((unsigned)e, dnk);
          const int p = p0 + q, k = e - q * nk;
          const V X = buf[p * 2 * pl + k];
          const V Xm = buf[p * 2 * pl + (k == 0 ? 0 : n3 - k)];
          A[i].x = (R)0.5 * (X.x + Xm.x); A[i].y = (R)0.5 * (X.y - Xm.y);
          B[i].x = (R)0.5 * (X.y + Xm.y); B[i].y = (R)-0.5 * (X.x - Xm.x);
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < MAXB_A; ++i) {
        const int e = tid + i * NT;
        if (e < tot) {
          const int q = (int)udiv((unsigned)e, dnk);
          const int p = p0 + q, k = e - q * nk;
          buf[(2 * p) * pl + k] = A[i];
          buf[(2 * p + 1) * pl + k] = B[i];
        }
      }
      __syncthreads();
    }
  }
  const int ymax = (nh + NW - 1) / NW;
  if (wave_fits<MAXV>(S.p2, ymax)) {
    int lo, hi;
    wave_share(nh, wave, NW, lo, hi);
    fft_lds_w<V, MAXV, false>(buf, S.p2, lo, hi - lo, pl, 1, tw2, lane);
    __syncthreads();
  } else {
    fft_lds<V, MAXB_A, false>(buf, S.p2, nh, pl, 1, tw2, tid, NT);
  }
}

// Inverse of plane_forward for one field loaded as a half spectrum in LDS:
// inverse y transform, then complex-to-real along z, two rows at a time
// (X = A + i B over the full row, A and B Hermitian-extended; the columns
// k = 0 and k = n3/2 keep only their real parts, i.e. the real part of the
// plane-wave sum). On exit (after a workgroup barrier) row j's real values
// sit in component j&1 of buf[(j>>1) 2 pl + k].
template <typename V, typename R, int NT>
__device__ __forceinline__ void plane_inverse(V *buf, const SolveDev &S, const V *tw2,
                                              const V *tw3, int tid) {
  SKX_OPAQUE(tid);
  constexpr int NW = NT / 64, MAXV = WaveV<R>::value;
  const int lane = tid & 63, wave = tid >> 6;
  const int n2 = S.n2, n3 = S.n3, nh = S.nh, pl = nh;
  const int cz = n2 / 2;
  const int ymax = (nh + NW - 1) / NW;
  if (wave_fits<MAXV>(S.p2, ymax)) {
    int lo, hi;
    wave_share(nh, wave, NW, lo, hi);
    fft_lds_w<V, MAXV, true>(buf, S.p2, lo, hi - lo, pl, 1, tw2, lane);
    __syncthreads();
  } else {
    fft_lds<V, MAXB_C, true>(buf, S.p2, nh, pl, 1, tw2, tid, NT);
  }
  const int zmax = (cz + NW - 1) / NW;
  if (wave_fits<MAXV>(S.p3, zmax) && zmax * n3 <= 64 * MAXV) {
    int lo, hi;
    wave_share(cz, wave, NW, lo, hi);
    merge_rows_w<V, R, MAXV>(buf, lo, hi, n3, pl, lane);
    fft_lds_w<V, MAXV, true>(buf, S.p3, lo, hi - lo, 1, 2 * pl, tw3, lane);
    __syncthreads();
    return;
  }
  int per = (MAXB_C * 2 * NT) / n3;
  if (per < 1) per = 1;
  const UDiv dn3 = make_udiv((unsigned)n3);
  for (int p0 = 0; p0 < cz; p0 += per) {
    const int p1 = min(cz, p0 + per);
    const int tot = (p1 - p0) * n3;
    V X[MAXB_C * 2];
#pragma unroll
    for (int i = 0; i < MAXB_C * 2; ++i) {
      const int e = tid + i * NT;
      if (e < tot) {
        const int q = (int)udiv((unsigned)e, dn3);
        const int p = p0 + q, k = e - q * n3;
        V Av, Bv;
        if (2 * k <= n3) {
          Av = buf[(2 * p) * pl + k];
          Bv = buf[(2 * p + 1) * pl + k];
          if (k == 0 || 2 * k == n3) { Av.y = 0; Bv.y = 0; }
        } else {
          Av = buf[(2 * p) * pl + n3 - k];
          Bv = buf[(2 * p + 1) * pl + n3 - k];
          Av.y = -Av.y; Bv.y = -Bv.y;
        }
        X[i].x = Av.x - Bv.y;
        X[i].y = Av.y + Bv.x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB_C * 2; ++i) {
      const int e = tid + i * NT;
      if (e < tot) {
        const int q = (int)udiv((unsigned)e, dn3);
        const int p = p0 + q, k = e - q * n3;
        buf[p * 2 * pl + k] = X[i];
      }
    }
    __syncthreads();
  }
  fft_lds<V, MAXB_C, true>(buf, S.p3, cz, 1, 2 * pl, tw3, tid, NT);
}

// Copy one x-plane of a half spectrum ([n2][pitch] complex in HBM) into the
// LDS plane [n2][pl], LU_L loads in flight per thread.
template <typename V, int NT>
__device__ __forceinline__ void load_plane(V *buf, const SKX_G V *src, int n2, int nh, int pitch,
                                           int pl, int tid) {
  SKX_OPAQUE(tid);
  const UDiv dnh = make_udiv((unsigned)nh);
  const int tot = n2 * nh;
  for (int e0 = tid; e0 < tot; e0 += LU_L * NT) {
    V t[LU_L];
    int li[LU_L];
#pragma unroll
    for (int u = 0; u < LU_L; ++u) {
      const int e = e0 + u * NT;
      li[u] = -1;
      if (e < tot) {
        const int j = (int)udiv((unsigned)e, dnh), k = e - j * nh;
        li[u] = j * pl + k;
        t[u] = ldg(src + (size_t)j * pitch + k);
      }
    }
#pragma unroll
    for (int u = 0; u < LU_L; ++u)
      if (li[u] >= 0) buf[li[u]] = t[u];
  }
}

// load_plane for a compile-time plane shape: N2 rows of NH values, stored
// at LDS row pitch PL.
template <typename V, int N2, int NH, int PL, int NT>
__device__ __forceinline__ void load_plane_f(V *buf, const SKX_G V *src, int pitch, int tid) {
  constexpr int TOT = N2 * NH;
  constexpr int NU = (TOT + NT - 1) / NT;
  V t[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = tid + u * NT;
    if (TOT % NT == 0 || e < TOT) t[u] = ldg(src + (size_t)(e / NH) * pitch + e % NH);
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = tid + u * NT;
    if (TOT % NT == 0 || e < TOT) buf[(e / NH) * PL + e % NH] = t[u];
  }
}

// ---------------------------------------------------------------------------
// The pointwise terms of one grid point at the trial point phi_t: the local
// energy densities (finite-T TF through the Fermi-Dirac table, PZ LDA) added
// to the running sums, the local potential v0 = T eta + v_xc, f = n^a and
// the assembly coefficients c_P = 2 a f / phi_t (-> 0 as phi_t -> 0) and
// c_Q = c_P (n - n0) + 2 phi_t (f - n0^a). Shared by the pointwise kernel
// and the compile-time-shaped pass A, so both compute the same values.
// ---------------------------------------------------------------------------
struct PointCfg {
  double T, lnnT;
  bool do_tf, do_xc, xcj, a56, need_f, need_h;
};

__device__ __forceinline__ PointCfg point_cfg(const SolveDev &S) {
  PointCfg c;
  c.T = S.T;
  c.lnnT = S.lnnT;
  c.do_tf = (S.terms & 1u) != 0;
  c.do_xc = (S.terms & 64u) != 0;
  c.xcj = S.xc == 2;       // C1-joined PZ81 branches
  c.a56 = S.a == 5.0 / 6.0;
  c.need_f = (S.fields & F_F) != 0;
  c.need_h = (S.fields & F_H) != 0;
  return c;
}

template <typename R>
__device__ __forceinline__ void point_terms(R ph, const PointCfg &c, R a, R a2, R n0, R n0a,
                                            const FDTable &fd, double &e_tf, double &e_xc,
                                            double &nel, double &bad, R &v0, R &f, R &cP, R &cQ) {
  const R n = ph * ph;
  const double nd = (double)n;
  double v = 0.0, lx = 0.0, e3 = 0.0, ie3 = 0.0;
  if (!(nd == nd) || nd > 1e300) bad += 1.0;
  if (nd > 0.0) {
    nel += nd;
    // FP32 evaluations take the logarithm in FP32 (its error is below the
    // FP32 rounding of the potential it feeds)
    lx = sizeof(R) == 4 ? (double)(0.69314718055994531f * __builtin_amdgcn_logf((float)n))
                        : log(nd);
    // FP64: n^(1/3), shared by PZ81 and, for a = 5/6, by n^a
    if (sizeof(R) == 8 && (c.do_xc || c.a56)) {
      ie3 = rcbrt_pos(nd);
      e3 = nd * ie3 * ie3;
    }
    if (c.do_tf) {
      double eta, psi;
      bad += fd_lookup(lx - c.lnnT, fd, eta, psi);
      e_tf += c.T * nd * psi;
      v += c.T * eta;
    }
    if (c.do_xc) {
      double eps, vx;
      if (sizeof(R) == 4) {
        float ef, vf;
        pz81_lnf(0.69314718055994531f * __builtin_amdgcn_logf((float)n), c.xcj, ef, vf);
        eps = ef;
        vx = vf;
      } else {
        pz81_ln_e3(lx, e3, ie3, c.xcj, eps, vx);
      }
      e_xc += nd * eps;
      v += vx;
    }
  }
  v0 = (R)v;
  f = (R)0;
  cP = (R)0;
  cQ = (R)0;
  if (c.need_f) {
    // FP64: n^a = exp(a ln n) with the logarithm taken above; for a = 5/6,
    // n^a = |phi| n^(1/3) and c_P = 2 a sign(phi) n^(1/3)
    if (sizeof(R) == 8 && c.a56) {
      f = (R)(fabs((double)ph) * e3);
      cP = (ph != (R)0) ? (R)copysign((double)a2 * e3, (double)ph) : (R)0;
    } else {
      f = sizeof(R) == 8 ? (nd > 0.0 ? (R)exp((double)a * lx) : (R)0) : rpow(n, a);
      // c_P = 2 a sign(phi) |phi|^(2a-1) = 2 a f / phi (-> 0 as phi -> 0)
      cP = (ph != (R)0) ? a2 * f / ph : (R)0;
    }
    if (c.need_h) cQ = cP * (n - n0) + (R)2 * ph * (f - n0a);
  }
}

// ---------------------------------------------------------------------------
// Pointwise pass (first kernel of pass A), one workgroup per CHUNK points of
// a solve: the trial point phi_t = ca phi + cb d and point_terms; writes
// phi_t and w0 = 2 phi_t v0, and in FP64 also n^a for the transform kernel
// and c_P, c_Q for pass C.
// ---------------------------------------------------------------------------
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_point(SolveDev *dev, const int *first, int nsolve,
                                              int grid, FDTable fd) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (!active_phase<MODE_EVAL>(st->phase)) return;
  const int par = st->par;
  const int tid = threadIdx.x;
  const int wl = item - first_of(first, s);
  const long long g0 = (long long)wl * CHUNK;
  const int cnt = (int)min((long long)CHUNK, S.M - g0);
  double ca, cb;
  bool use_d;
  trial_coef(st, S, ca, cb, use_d);
  const SKX_G R *phi = gptr<R>(S.phi2[par]) + g0;
  const SKX_G R *dd = gptr<R>(S.d) + g0;
  SKX_G R *phit = gptr<R>(S.phi2[1 - par]) + g0;
  SKX_G R *v0s = gptr<R>(S.vpt) + g0;
  SKX_G R *fps = gptr<R>(S.fpt) + g0;
  SKX_G R *qps = gptr<R>(S.qpt) + g0;
  SKX_G R *nas = gptr<R>(S.npa) + g0;
  const R a = (R)S.a, a2 = (R)(2.0 * S.a), n0 = (R)S.n0, n0a = (R)S.n0a;
  const PointCfg pc = point_cfg(S);
  constexpr int PER = CHUNK / NT;
  R pv[PER], dv[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + u * NT;
    if (e < cnt) {
      pv[u] = phi[e];
      if (use_d) dv[u] = dd[e];
    }
  }
  double e_tf = 0.0, e_xc = 0.0, nel = 0.0, bad = 0.0;
  // the points of a thread unrolled, so that their table lookups and
  // arithmetic interleave (measured against one point at a time: FP64
  // pointwise + pass A 80^3 146.5 -> 138.8 us per batch of eight, 64^3
  // 117 -> 111 us, 80 instead of 128 VGPRs)
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + u * NT;
    if (e >= cnt) break;
    const R p0 = pv[u], d0 = use_d ? dv[u] : (R)0;
    const R ph = use_d ? (R)(ca * (double)p0 + cb * (double)d0) : (R)(ca * (double)p0);
    phit[e] = ph;
    R v0, f, cP, cQ;
    point_terms<R>(ph, pc, a, a2, n0, n0a, fd, e_tf, e_xc, nel, bad, v0, f, cP, cQ);
    v0s[e] = (R)2 * ph * v0;
    if (pc.need_f) {
      if (!derive_na<R>()) nas[e] = f;
      if (!derive_coefs<R>()) {
        fps[e] = cP;
        if (pc.need_h) qps[e] = cQ;
      }
    }
  }
  double vsum[PART_A] = {e_tf, e_xc, nel, bad};
  double tot[PART_A];
  block_reduce<PART_A>(vsum, reinterpret_cast<double *>(smem), tid, NT, tot);
  if (tid == 0)
    for (int q = 0; q < PART_A; ++q) S.partA[wl * PART_A + q] = tot[q];
}

// ---------------------------------------------------------------------------
// Pass A
// ---------------------------------------------------------------------------
template <typename R, int NT, int MODE>
__global__ __launch_bounds__(NT, sizeof(R) == 4 ? 5 : 4) void k_passA(SolveDev *dev, const int *first, int nsolve,
                                              int grid, const double *twbank, FDTable fd) {
  typedef typename Vec2<R>::T V;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  if (S.big & 1) return;
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (!active_phase<MODE>(st->phase)) return;
  const int par = st->par;
  const int tid = threadIdx.x;
  const int local = item - first_of(first, s);
  const int nf = MODE == MODE_EVAL ? S.nf : 1;
  const int plane = local / nf, c = local % nf;
  const int fb = MODE == MODE_EVAL ? nth_field(S.fields, c) : 0;
  const int n2 = S.n2, n3 = S.n3, nh = S.nh;
  const int pl = nh;                         // LDS row pitch (complex)
  V *buf = reinterpret_cast<V *>(smem);
  V *tw2 = buf + n2 * pl;
  V *tw3 = tw2 + n2;
  load_twiddles(tw2, twbank, S.p2.tw, n2, tid, NT);
  load_twiddles(tw3, twbank, S.p3.tw, n3, tid, NT);

  const R invM = (R)(1.0 / (double)S.M);
  const size_t pbase = (size_t)plane * n2 * n3;
  const int np = n2 * n3;
  if (MODE == MODE_EVAL) {
    // the field of this workgroup from phi_t and f = n^a of the pointwise
    // kernel, read as pairs of neighbours along z (n3 is even, so a pair
    // never straddles a row), LU_A pairs per thread in flight
    const size_t qbase = pbase >> 1;
    const SKX_G V *pt = gptr<V>(S.phi2[1 - par]) + qbase;
    const SKX_G V *fa = gptr<V>(S.npa) + qbase;
    constexpr bool DER = derive_na<R>();
    const bool need_p = fb != 2 || DER, need_fa = fb >= 2 && !DER;
    const R n0 = (R)S.n0, n0a = (R)S.n0a;
    const NaCfg<R> nc = na_cfg<R>(S);
    const int npair = np >> 1, h3 = n3 >> 1;
    const UDiv dh3 = make_udiv((unsigned)h3);
    for (int q0 = tid; q0 < npair; q0 += LU_A * NT) {
      V pv[LU_A], fv[LU_A];
#pragma unroll
      for (int u = 0; u < LU_A; ++u) {
        const int q = q0 + u * NT;
        if (q < npair) {
          if (need_p) pv[u] = ldg(pt + q);
          if (need_fa) fv[u] = ldg(fa + q);
        }
      }
#pragma unroll
      for (int u = 0; u < LU_A; ++u) {
        const int q = q0 + u * NT;
        if (q < npair) {
          const int j = (int)udiv((unsigned)q, dh3), k = 2 * (q - j * h3);
          R xv[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const R p = need_p ? (h ? pv[u].y : pv[u].x) : (R)0;
            const R f = DER ? (fb >= 2 ? derived_na(p, nc) : (R)0)
                            : (need_fa ? (h ? fv[u].y : fv[u].x) : (R)0);
            xv[h] = fb == 0 ? p : fb == 1 ? p * p : fb == 2 ? f : (f - n0a) * (p * p - n0);
          }
          R *slot = reinterpret_cast<R *>(&buf[(j >> 1) * 2 * pl + k]);
          slot[j & 1] = xv[0] * invM;
          slot[2 + (j & 1)] = xv[1] * invM;
        }
      }
    }
  } else {
    // residual of the accepted trial point, stored for the update pass
    const size_t qbase = pbase >> 1;
    const SKX_G V *g = gptr<V>(S.grad) + qbase;
    const SKX_G V *phit = gptr<V>(S.phi2[1 - par]) + qbase;
    SKX_G V *rt = gptr<V>(S.r2[1 - par]) + qbase;
    const R mu2 = (R)(2.0 * st->mut);
    const int npair = np >> 1, h3 = n3 >> 1;
    const UDiv dh3 = make_udiv((unsigned)h3);
    for (int q0 = tid; q0 < npair; q0 += LU_A * NT) {
      V gv[LU_A], pv[LU_A];
#pragma unroll
      for (int u = 0; u < LU_A; ++u) {
        const int q = q0 + u * NT;
        if (q < npair) { gv[u] = ldg(g + q); pv[u] = ldg(phit + q); }
      }
#pragma unroll
      for (int u = 0; u < LU_A; ++u) {
        const int q = q0 + u * NT;
        if (q < npair) {
          const int j = (int)udiv((unsigned)q, dh3), k = 2 * (q - j * h3);
          V x;
          x.x = gv[u].x - mu2 * pv[u].x;
          x.y = gv[u].y - mu2 * pv[u].y;
          stg(rt + q, x);
          R *slot = reinterpret_cast<R *>(&buf[(j >> 1) * 2 * pl + k]);
          slot[j & 1] = x.x * invM;
          slot[2 + (j & 1)] = x.y * invM;
        }
      }
    }
  }
  __syncthreads();
  plane_forward<V, R, NT>(buf, S, tw2, tw3, tid);
  SKX_G V *spec = gptr<V>(S.spec) +
            (size_t)(MODE == MODE_EVAL ? S.slot[fb] : 0) * S.H;
  const size_t obase = (size_t)plane * n2 * S.pitch;
  const UDiv dnh = make_udiv((unsigned)nh);
  for (int e = tid; e < n2 * nh; e += NT) {
    const int j = (int)udiv((unsigned)e, dnh), k = e - j * nh;
    stg(spec + obase + (size_t)j * S.pitch + k, buf[j * pl + k]);
  }
}

// ---------------------------------------------------------------------------
// Pass B
// ---------------------------------------------------------------------------
template <typename R, int NT, int TK, int MODE>
__global__ __launch_bounds__(NT) void k_passB(SolveDev *dev, const int *first, int nsolve,
                                              int grid, const double *twbank) {
  typedef typename Vec2<R>::T V;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (!active_phase<MODE>(st->phase)) return;
  const int tid = threadIdx.x;
  const int local = item - first_of(first, s);
  const int j = local / S.nkb, kb = local % S.nkb;
  const int k0 = kb * TK;
  // columns of this block: TK, or fewer in the last block (the Nyquist
  // column alone when n3/2 is a multiple of TK)
  const int tkv = min(TK, S.nh - k0);
  const UDiv dtk = make_udiv((unsigned)tkv);
  const int n1 = S.n1, nf = MODE == MODE_EVAL ? S.nf : 1, W = nf * tkv;
  // one padding element per tile row keeps the x transform (stride Wp)
  // off a single LDS bank
  const int Wp = W + 1;
  V *tile = reinterpret_cast<V *>(smem);
  V *tw1 = tile + n1 * Wp;
  load_twiddles(tw1, twbank, S.p1.tw, n1, tid, NT);
  SKX_G V *spec = gptr<V>(S.spec);
  const size_t rowstride = (size_t)S.n2 * S.pitch;
  const UDiv dW = make_udiv((unsigned)W);
  for (int e0 = tid; e0 < n1 * W; e0 += LU_L * NT) {
    V t[LU_L];
    int li[LU_L];
#pragma unroll
    for (int u = 0; u < LU_L; ++u) {
      const int e = e0 + u * NT;
      li[u] = -1;
      if (e < n1 * W) {
        const int i = (int)udiv((unsigned)e, dW), r = e - i * W;
        const int cc = (int)udiv((unsigned)r, dtk), kk = r - cc * tkv;
        li[u] = i * Wp + r;
        t[u] = ldg(spec + (size_t)cc * S.H + (size_t)i * rowstride + (size_t)j * S.pitch + k0 + kk);
      }
    }
#pragma unroll
    for (int u = 0; u < LU_L; ++u)
      if (li[u] >= 0) tile[li[u]] = t[u];
  }
  __syncthreads();
  // x transforms of the tile columns, wavefront-owned when they fit
  constexpr int NW = NT / 64, MAXV = WaveV<R>::value;
  const int lane = tid & 63, wave = tid >> 6;
  const bool xw = wave_fits<MAXV>(S.p1, (W + NW - 1) / NW);
  int xlo, xhi;
  wave_share(W, wave, NW, xlo, xhi);
  if (S.debug != 2) {
    if (xw) {
      fft_lds_w<V, MAXV, false>(tile, S.p1, xlo, xhi - xlo, Wp, 1, tw1, lane);
      __syncthreads();
    } else {
      fft_lds<V, MAXB_B, false>(tile, S.p1, W, Wp, 1, tw1, tid, NT);
    }
  }
  if (S.debug == 1) {
    for (int e = tid; e < n1 * W; e += NT) {
      const int i = (int)udiv((unsigned)e, dW), r = e - i * W;
      const int cc = (int)udiv((unsigned)r, dtk), kk = r - cc * tkv;
      stg(spec + (size_t)cc * S.H + (size_t)i * rowstride + (size_t)j * S.pitch + k0 + kk,
          tile[i * Wp + r]);
    }
    return;
  }
  const double kscale = S.kscale;
  const int g2 = gidx(j, S.n2);
  double evw = 0, eh = 0, ef0 = 0, ef1 = 0, eloc = 0, bad = 0;
  if (MODE == MODE_PREC) {
    for (int e = tid; e < n1 * tkv; e += NT) {
      const int i = (int)udiv((unsigned)e, dtk), kk = e - i * tkv;
      const int k3 = k0 + kk;
      const int g1 = gidx(i, n1);
      const double G2 = kscale * (double)(g1 * g1 + g2 * g2 + k3 * k3);
      const R pg = (R)(1.0 / (G2 + S.kappa));
      V x = tile[i * Wp + kk];
      x.x *= pg; x.y *= pg;
      tile[i * Wp + kk] = x;
    }
  } else {
    const unsigned terms = S.terms;
    const bool do_vw = terms & 2u, do_nl0 = terms & 4u;
    const bool do_h = terms & 16u, do_loc = terms & 32u;
    const int sphi = S.slot[0], sn = S.slot[1], sf = S.slot[2], sh = S.slot[3];
    const SKX_G V *vloc = gptr<V>(S.vloc);
    const R b3 = (R)(S.beta / 3.0);
    const double FOURPI = 12.566370614359172954;
    const SKX_G double *wt = gptr<double>(S.w);
    const SKX_G double *wpt = gptr<double>(S.wp);
    for (int e0 = tid; e0 < n1 * tkv; e0 += LU_B * NT) {
      // gathers of this batch first: V_loc(G) and the kernel tables
      V vlb[LU_B];
      double wb[LU_B], wpb[LU_B];
#pragma unroll
      for (int u = 0; u < LU_B; ++u) {
        const int e = e0 + u * NT;
        const int i = (int)udiv((unsigned)e, dtk), kk = e - i * tkv;
        const int k3 = k0 + kk;
        if (e < n1 * tkv) {
          const int g1 = gidx(i, n1);
          const int sidx = g1 * g1 + g2 * g2 + k3 * k3;
          if (do_loc) vlb[u] = ldg(vloc + ((size_t)i * S.n2 + j) * S.pitch + k3);
          if (sf >= 0) { wb[u] = wt[sidx]; wpb[u] = wpt[sidx]; }
        }
      }
#pragma unroll
    for (int u = 0; u < LU_B; ++u) {
      const int e = e0 + u * NT;
      const int i = (int)udiv((unsigned)e, dtk), kk = e - i * tkv;
      const int k3 = k0 + kk;
      if (e >= n1 * tkv || S.debug) continue;
      const int g1 = gidx(i, n1);
      const int sidx = g1 * g1 + g2 * g2 + k3 * k3;
      const double G2 = kscale * (double)sidx;
      const double wgt = (k3 == 0 || 2 * k3 == S.n3) ? 1.0 : 2.0;
      V *row = tile + i * Wp;
      if (sphi >= 0) {
        V x = row[sphi * tkv + kk];
        if (do_vw) evw += wgt * G2 * ((double)x.x * x.x + (double)x.y * x.y);
        const R g2r = (R)G2;
        x.x *= g2r; x.y *= g2r;
        row[sphi * tkv + kk] = x;
      }
      {
        const V x = row[sn * tkv + kk];
        double bx = 0.0, by = 0.0;
        if (do_h && sidx > 0) {
          const double m2 = (double)x.x * x.x + (double)x.y * x.y;
          const double ig = 1.0 / G2;
          eh += wgt * m2 * ig;
          bx = FOURPI * ig * x.x;
          by = FOURPI * ig * x.y;
        }
        if (do_loc) {
          const V vl = vlb[u];
          eloc += wgt * ((double)x.x * vl.x + (double)x.y * vl.y);
          bx += vl.x;
          by += vl.y;
        }
        if (!(x.x == x.x) || !(x.y == x.y)) bad += 1.0;
        V o; o.x = (R)bx; o.y = (R)by;
        row[sn * tkv + kk] = o;
      }
      if (sf >= 0) {
        const V f = row[sf * tkv + kk];
        const R w = (R)wb[u];
        const R wp = (R)wpb[u];
        V P; P.x = 0; P.y = 0;
        if (do_nl0) {
          ef0 += wgt * (double)w * ((double)f.x * f.x + (double)f.y * f.y);
          P.x = (R)2 * w * f.x; P.y = (R)2 * w * f.y;
        }
        if (sh >= 0) {
          const V h = row[sh * tkv + kk];
          ef1 += wgt * (double)wp * ((double)f.x * h.x + (double)f.y * h.y);
          P.x += b3 * wp * h.x; P.y += b3 * wp * h.y;
          V Q; Q.x = b3 * wp * f.x; Q.y = b3 * wp * f.y;
          row[sh * tkv + kk] = Q;
        }
        row[sf * tkv + kk] = P;
      }
    }
    }
  }
  __syncthreads();
  if (xw) {
    fft_lds_w<V, MAXV, true>(tile, S.p1, xlo, xhi - xlo, Wp, 1, tw1, lane);
    __syncthreads();
  } else {
    fft_lds<V, MAXB_B, true>(tile, S.p1, W, Wp, 1, tw1, tid, NT);
  }
  for (int e = tid; e < n1 * W; e += NT) {
    const int i = (int)udiv((unsigned)e, dW), r = e - i * W;
    const int cc = (int)udiv((unsigned)r, dtk), kk = r - cc * tkv;
    stg(spec + (size_t)cc * S.H + (size_t)i * rowstride + (size_t)j * S.pitch + k0 + kk,
        tile[i * Wp + r]);
  }
  if (MODE == MODE_EVAL) {
    double v[PART_B] = {evw, eh, ef0, ef1, eloc, bad};
    double tot[PART_B];
    __syncthreads();
    block_reduce<PART_B>(v, reinterpret_cast<double *>(smem), tid, NT, tot);
    if (tid == 0)
      for (int q = 0; q < PART_B; ++q) S.partB[local * PART_B + q] = tot[q];
  }
}

// ---------------------------------------------------------------------------
// Pass C
//
// dE/dphi is accumulated field by field, either in LDS beside the plane
// (ACC_LDS, when both fit) or in the output buffer itself, whose plane the
// workgroup revisits while it is still in L2.
// ---------------------------------------------------------------------------
template <typename R, int NT, bool ACC_LDS, int MODE>
__global__ __launch_bounds__(NT, 4) void k_passC(SolveDev *dev, const int *first, int nsolve,
                                              int grid, const double *twbank, FDTable fd) {
  typedef typename Vec2<R>::T V;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  if (S.big & 2) return;
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (!active_phase<MODE>(st->phase)) return;
  const int par = st->par;
  const int tid = threadIdx.x;
  const int plane = item - first_of(first, s);
  const int n2 = S.n2, n3 = S.n3, nh = S.nh;
  const int pl = nh;
  V *buf = reinterpret_cast<V *>(smem);
  V *tw2 = buf + n2 * pl;
  V *tw3 = tw2 + n2;
  load_twiddles(tw2, twbank, S.p2.tw, n2, tid, NT);
  load_twiddles(tw3, twbank, S.p3.tw, n3, tid, NT);
  const size_t pbase = (size_t)plane * n2 * n3;
  const int np = n2 * n3;
  const SKX_G V *spec = gptr<V>(S.spec);
  const size_t ibase = (size_t)plane * n2 * S.pitch;

  if (MODE == MODE_PREC) {
    SKX_G R *out = gptr<R>(S.pr2[1 - par]);
    const UDiv dn3 = make_udiv((unsigned)n3);
    load_plane<V, NT>(buf, spec + ibase, n2, nh, S.pitch, pl, tid);
    __syncthreads();
    plane_inverse<V, R, NT>(buf, S, tw2, tw3, tid);
    for (int e = tid; e < np; e += NT) {
      const int j = (int)udiv((unsigned)e, dn3), k = e - j * n3;
      const R *cv = reinterpret_cast<const R *>(&buf[(j >> 1) * 2 * pl + k]);
      out[pbase + e] = cv[j & 1];
    }
    return;
  }

  // dE/dphi starts from w0 = 2 phi_t v0; the fields enter with the
  // coefficients 1 (phi), 2 phi_t (n), c_P (f) and c_Q (h), stored by the
  // pointwise pass; read as pairs along z, LU_C pairs per thread in flight.
  // In FP32 phi_t is also kept in LDS beside dE/dphi, so that every array
  // is read from HBM once.
  constexpr bool PCACHE = ACC_LDS && sizeof(R) == 4;
  constexpr bool DER = derive_coefs<R>();         // c_P, c_Q from phi_t
  const NaCfg<R> nc = na_cfg<R>(S);
  const size_t qbase = pbase >> 1;
  const SKX_G V *phit = gptr<V>(S.phi2[1 - par]) + qbase;
  const SKX_G V *v0 = gptr<V>(S.vpt) + qbase;
  const SKX_G V *cpw = gptr<V>(S.fpt) + qbase;
  const SKX_G V *cqw = gptr<V>(S.qpt) + qbase;
  SKX_G R *grad = gptr<R>(S.grad);
  R *acc = ACC_LDS ? reinterpret_cast<R *>(tw3 + n3) : (R *)(grad + pbase);
  V *pc = reinterpret_cast<V *>(acc + np);        // phi_t pairs (PCACHE)
  const int npair = np >> 1;
  for (int q0 = tid; q0 < npair; q0 += LU_C * NT) {
    V pv[LU_C], vv[LU_C];
#pragma unroll
    for (int u = 0; u < LU_C; ++u) {
      const int q = q0 + u * NT;
      if (q < npair) {
        if (PCACHE) pv[u] = ldg(phit + q);
        vv[u] = ldg(v0 + q);
      }
    }
#pragma unroll
    for (int u = 0; u < LU_C; ++u) {
      const int q = q0 + u * NT;
      if (q < npair) {
        acc[2 * q] = S.debug ? (R)0 : vv[u].x;
        acc[2 * q + 1] = S.debug ? (R)0 : vv[u].y;
        if (PCACHE) pc[q] = pv[u];
      }
    }
  }
  const int h3 = n3 >> 1;
  const UDiv dh3 = make_udiv((unsigned)h3);
  for (int fb = 0; fb < NFIELD; ++fb) {
    const int sl = S.slot[fb];
    if (sl < 0 || (S.debug && fb != 0)) continue;
    __syncthreads();
    load_plane<V, NT>(buf, spec + (size_t)sl * S.H + ibase, n2, nh, S.pitch, pl, tid);
    __syncthreads();
    plane_inverse<V, R, NT>(buf, S, tw2, tw3, tid);
    int tq = tid;
    SKX_OPAQUE(tq);
    for (int q0 = tq; q0 < npair; q0 += LU_C * NT) {
      V cv2[LU_C];
#pragma unroll
      for (int u = 0; u < LU_C; ++u) {
        const int q = q0 + u * NT;
        if (q < npair) {
          if (fb == 1 || (fb >= 2 && DER)) cv2[u] = PCACHE ? pc[q] : ldg(phit + q);
          else if (fb == 2) cv2[u] = ldg(cpw + q);
          else if (fb == 3) cv2[u] = ldg(cqw + q);
        }
      }
#pragma unroll
      for (int u = 0; u < LU_C; ++u) {
        const int q = q0 + u * NT;
        if (q < npair) {
          const int j = (int)udiv((unsigned)q, dh3), k = 2 * (q - j * h3);
          const R *cv = reinterpret_cast<const R *>(&buf[(j >> 1) * 2 * pl + k]);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const R val = cv[2 * h + (j & 1)];
            const R c = h ? cv2[u].y : cv2[u].x;
            const R coef = fb == 0 ? (R)1
                         : fb == 1 ? (R)2 * c
                                   : (DER ? derived_coef(c, fb, nc) : c);
            acc[2 * q + h] += coef * val;
          }
        }
      }
    }
  }
  __syncthreads();
  double sphig = 0.0, bad = 0.0;
  SKX_G V *grad2 = gptr<V>(S.grad) + qbase;
  for (int q0 = tid; q0 < npair; q0 += LU_C * NT) {
    V pv[LU_C];
#pragma unroll
    for (int u = 0; u < LU_C; ++u) {
      const int q = q0 + u * NT;
      if (q < npair) pv[u] = PCACHE ? pc[q] : ldg(phit + q);
    }
#pragma unroll
    for (int u = 0; u < LU_C; ++u) {
      const int q = q0 + u * NT;
      if (q < npair) {
        V g;
        g.x = acc[2 * q];
        g.y = acc[2 * q + 1];
        if (ACC_LDS) stg(grad2 + q, g);
        sphig += (double)pv[u].x * (double)g.x + (double)pv[u].y * (double)g.y;
        if (!(g.x == g.x)) bad += 1.0;
        if (!(g.y == g.y)) bad += 1.0;
      }
    }
  }
  double v[PART_C] = {sphig, bad};
  double tot[PART_C];
  __syncthreads();
  block_reduce<PART_C>(v, reinterpret_cast<double *>(smem), tid, NT, tot);
  if (tid == 0)
    for (int q = 0; q < PART_C; ++q) S.partC[plane * PART_C + q] = tot[q];
}

// ---------------------------------------------------------------------------
// Passes A and C for planes whose half spectrum does not fit in LDS (FP64
// beyond 128 x 128, FP32 beyond 192 x 192) and where these kernels were
// measured faster (pass C from 80 KB planes in FP64 and 24 KB in FP32, FP32
// pass A from 80 KB): each pass runs as two launches over many small
// workgroups, so that many of them share a CU and hide each other's load
// latency. Pass A: z transforms over chunks of rp row pairs (one workgroup
// per chunk reads phi_t once and transforms every field's rows together),
// then y transforms over chunks of split_cc columns of one field. Pass C:
// the inverse y transforms over column chunks, then the inverse z
// transforms over row-pair chunks (every field together), dE/dphi assembled
// from LDS. The half spectrum sits in its HBM slot between the two launches
// of a pass.
// ---------------------------------------------------------------------------
// Loop over the elements e = tid, tid + NT, ... < tot with U iterations' loads
// in flight: load(e) for U elements first, then use(e, loaded) for each.
template <int U, int NT, typename T, typename FL, typename FU>
__device__ __forceinline__ void batched(int tot, int tid, FL load, FU use) {
  for (int e0 = tid; e0 < tot; e0 += U * NT) {
    T t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT;
      if (e < tot) t[u] = load(e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT;
      if (e < tot) use(e, t[u]);
    }
  }
}

template <typename R> struct Quad { R a, b, c, d; };

// Row-pair chunk `j` of an x-plane: work item -> (solve, plane, chunk), or
// false for items past the solve's chunks or phase.
struct SplitItem { int s, plane, j; };
template <int MODE>
__device__ __forceinline__ bool split_item(const SolveDev *dev, const int *first, int nsolve,
                                           int item, int per, int bigbit, SplitItem &it) {
  const int pi = item / per;
  it.j = item - pi * per;
  it.s = find_solve(first, nsolve, pi);
  const SolveDev &S = dev[it.s];
  if (!(S.big & bigbit)) return false;
  if (!active_phase<MODE>(cptr<OptState>(S.st)->phase)) return false;
  it.plane = pi - first_of(first, it.s);
  return true;
}

// Pass A, z transforms of one chunk of row pairs: every field of the chunk
// built from phi_t (MODE_PREC: r_t = dE/dphi - 2 mu_t phi_t, also stored),
// rows 2p and 2p+1 packed as one complex row, all fields' rows transformed
// together, then split into the two rows' half spectra straight to HBM.
template <typename R, int MODE>
__global__ __launch_bounds__(SPLIT_NT) void k_passA_rows(SolveDev *dev, const int *first,
                                                         int nsolve, int grid, int krow,
                                                         const double *twbank) {
  typedef typename Vec2<R>::T V;
  static_assert(derive_na<R>(), "the split kernels derive n^a from phi_t");
  constexpr int NT = SPLIT_NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  SplitItem it;
  if (!split_item<MODE>(dev, first, nsolve, item, krow, 1, it)) return;
  const SolveDev &S = dev[it.s];
  // the preconditioner's single field takes NFIELD times the row pairs
  const int rpm = MODE == MODE_PREC ? NFIELD * S.rp : S.rp;
  if (it.j >= (MODE == MODE_PREC ? S.nrcp : S.nrc)) return;
  const SKX_C OptState *st = cptr<OptState>(S.st);
  const int par = st->par;
  const int tid = threadIdx.x;
  const int n2 = S.n2, n3 = S.n3, nh = S.nh, pitch = S.pitch, pl2 = 2 * nh;
  const int p0 = it.j * rpm, np = min(rpm, n2 / 2 - p0), tot = np * n3;
  const int nf = MODE == MODE_EVAL ? S.nf : 1;
  const int fs = np * pl2;                      // LDS stride between the fields' rows
  V *tw3 = reinterpret_cast<V *>(smem);
  V *buf = tw3 + n3;
  load_twiddles(tw3, twbank, S.p3.tw, n3, tid, NT);
  const size_t pbase = (size_t)it.plane * n2 * n3 + (size_t)2 * p0 * n3;
  const UDiv dn3 = make_udiv((unsigned)n3);
  const SKX_G R *pt = gptr<R>(S.phi2[1 - par]) + pbase;
  const SKX_G R *gr = gptr<R>(S.grad) + pbase;
  SKX_G R *rt = gptr<R>(S.r2[1 - par]) + pbase;
  const R mu2 = MODE == MODE_PREC ? (R)(2.0 * st->mut) : (R)0;
  const R invM = (R)(1.0 / (double)S.M);
  const R n0 = (R)S.n0, n0a = (R)S.n0a;
  const int fields = S.fields;
  batched<4, NT, Quad<R>>(
      tot, tid,
      [&](int e) {
        const int q = (int)udiv((unsigned)e, dn3), o = 2 * q * n3 + (e - q * n3);
        Quad<R> w{pt[o], pt[o + n3], (R)0, (R)0};
        if (MODE == MODE_PREC) { w.c = gr[o]; w.d = gr[o + n3]; }
        return w;
      },
      [&](int e, const Quad<R> &w) {
        const int q = (int)udiv((unsigned)e, dn3), z = e - q * n3;
        V *dst = buf + q * pl2 + z;
        if (MODE == MODE_PREC) {
          const R x0 = w.c - mu2 * w.a, x1 = w.d - mu2 * w.b;    // r_t
          rt[2 * q * n3 + z] = x0;
          rt[2 * q * n3 + z + n3] = x1;
          V v;
          v.x = x0 * invM;
          v.y = x1 * invM;
          dst[0] = v;
        } else {
          // n^a of both rows once for the f and h fields
          R f0 = (R)0, f1 = (R)0;
          if (fields & (F_F | F_H)) {
            f0 = derived_na(w.a, na_cfg<R>(S));
            f1 = derived_na(w.b, na_cfg<R>(S));
          }
          int c = 0;
#pragma unroll
          for (int fb = 0; fb < NFIELD; ++fb) {
            if (!(fields & (1 << fb))) continue;
            R x0, x1;
            if (fb == 0) { x0 = w.a; x1 = w.b; }
            else if (fb == 1) { x0 = w.a * w.a; x1 = w.b * w.b; }
            else if (fb == 2) { x0 = f0; x1 = f1; }
            else { x0 = (f0 - n0a) * (w.a * w.a - n0); x1 = (f1 - n0a) * (w.b * w.b - n0); }
            V v;
            v.x = x0 * invM;
            v.y = x1 * invM;
            dst[c * fs] = v;
            ++c;
          }
        }
      });
  __syncthreads();
  fft_lds<V, MAXB_A, false>(buf, S.p3, nf * np, 1, pl2, tw3, tid, NT);
  const int nk = n3 / 2 + 1, per = np * nk;
  const UDiv dnk = make_udiv((unsigned)nk), dper = make_udiv((unsigned)per);
  SKX_G V *spec0 = gptr<V>(S.spec) + ((size_t)it.plane * n2 + 2 * p0) * pitch;
  for (int e = tid; e < nf * per; e += NT) {
    const int c = (int)udiv((unsigned)e, dper), r = e - c * per;
    const int q = (int)udiv((unsigned)r, dnk), k = r - q * nk;
    const V *row = buf + c * fs + q * pl2;
    const V X = row[k];
    const V Xm = row[k == 0 ? 0 : n3 - k];
    V A, B;
    A.x = (R)0.5 * (X.x + Xm.x); A.y = (R)0.5 * (X.y - Xm.y);
    B.x = (R)0.5 * (X.y + Xm.y); B.y = (R)-0.5 * (X.x - Xm.x);
    SKX_G V *spec = spec0 + (size_t)c * S.H;
    stg(spec + (size_t)(2 * q) * pitch + k, A);
    stg(spec + (size_t)(2 * q + 1) * pitch + k, B);
  }
}

// y transforms (forward in pass A, inverse in pass C) of one chunk of
// split_cc columns of one field's half-spectrum plane, in place in HBM.
template <typename R, int MODE, bool INV>
__global__ __launch_bounds__(SPLIT_NT, 4) void k_plane_cols(SolveDev *dev, const int *first,
                                                         int nsolve, int grid, int kcol,
                                                         const double *twbank) {
  typedef typename Vec2<R>::T V;
  constexpr int NT = SPLIT_NT, NFC = MODE == MODE_EVAL ? NFIELD : 1;
  constexpr int CC = split_cc(sizeof(R) == 8 ? 0 : 1), CCP = CC + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  SplitItem it;
  if (!split_item<MODE>(dev, first, nsolve, item, NFC * kcol, INV ? 2 : 1, it)) return;
  const SolveDev &S = dev[it.s];
  const int c = it.j / kcol, k0 = (it.j - c * kcol) * CC;
  if (MODE == MODE_EVAL && c >= S.nf) return;
  if (k0 >= S.nh) return;
  const int tid = threadIdx.x;
  const int n2 = S.n2, pitch = S.pitch, kc = min(CC, S.nh - k0);
  V *tw2 = reinterpret_cast<V *>(smem);
  V *buf = tw2 + n2;
  load_twiddles(tw2, twbank, S.p2.tw, n2, tid, NT);
  SKX_G V *spec = gptr<V>(S.spec) + (size_t)c * S.H + (size_t)it.plane * n2 * pitch + k0;
  const UDiv dkc = make_udiv((unsigned)kc);
  batched<8, NT, V>(
      n2 * kc, tid,
      [&](int e) {
        const int y = (int)udiv((unsigned)e, dkc), kk = e - y * kc;
        return ldg(spec + (size_t)y * pitch + kk);
      },
      [&](int e, const V &v) {
        const int y = (int)udiv((unsigned)e, dkc), kk = e - y * kc;
        buf[y * CCP + kk] = v;
      });
  __syncthreads();
  fft_lds<V, MAXB_A, INV>(buf, S.p2, kc, CCP, 1, tw2, tid, NT);
  for (int e = tid; e < n2 * kc; e += NT) {
    const int y = (int)udiv((unsigned)e, dkc), kk = e - y * kc;
    stg(spec + (size_t)y * pitch + kk, buf[y * CCP + kk]);
  }
}

// Pass C, inverse z transforms of one chunk of row pairs: every field's two
// half-spectrum rows as one complex row, all fields' rows transformed
// together in LDS, then dE/dphi = w0 + A + 2 phi_t B + c_P P + c_Q Q
// (MODE_PREC: the single field is P r_t) and the chunk's partials of
// int phi_t dE/dphi.
template <typename R, int MODE>
__global__ __launch_bounds__(SPLIT_NT) void k_passC_rows(SolveDev *dev, const int *first,
                                                         int nsolve, int grid, int krow,
                                                         const double *twbank) {
  typedef typename Vec2<R>::T V;
  constexpr int NT = SPLIT_NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  SplitItem it;
  if (!split_item<MODE>(dev, first, nsolve, item, krow, 2, it)) return;
  const SolveDev &S = dev[it.s];
  // the preconditioner's single field takes NFIELD times the row pairs
  const int rpm = MODE == MODE_PREC ? NFIELD * S.rp : S.rp;
  if (it.j >= (MODE == MODE_PREC ? S.nrcp : S.nrc)) return;
  const SKX_C OptState *st = cptr<OptState>(S.st);
  const int par = st->par;
  const int tid = threadIdx.x;
  const int n2 = S.n2, n3 = S.n3, pitch = S.pitch, pl2 = 2 * S.nh;
  const int p0 = it.j * rpm, np = min(rpm, n2 / 2 - p0), tot = np * n3;
  const int nf = MODE == MODE_EVAL ? S.nf : 1;
  const int fs = np * pl2;
  V *tw3 = reinterpret_cast<V *>(smem);
  V *buf = tw3 + n3;
  load_twiddles(tw3, twbank, S.p3.tw, n3, tid, NT);
  const UDiv dn3 = make_udiv((unsigned)n3), dtot = make_udiv((unsigned)tot);
  const SKX_G V *spec0 = gptr<V>(S.spec) + ((size_t)it.plane * n2 + 2 * p0) * pitch;
  // x_{2p} + i x_{2p+1} over the full row from the two half spectra, every
  // field (spectrum slot c)
  batched<4, NT, Quad<R>>(
      nf * tot, tid,
      [&](int e) {
        const int c = (int)udiv((unsigned)e, dtot), r = e - c * tot;
        const int q = (int)udiv((unsigned)r, dn3), k = r - q * n3;
        const int kk = 2 * k <= n3 ? k : n3 - k;
        const SKX_G V *spec = spec0 + (size_t)c * S.H;
        const V Av = ldg(spec + (size_t)(2 * q) * pitch + kk);
        const V Bv = ldg(spec + (size_t)(2 * q + 1) * pitch + kk);
        return Quad<R>{Av.x, Av.y, Bv.x, Bv.y};
      },
      [&](int e, const Quad<R> &w) {
        const int c = (int)udiv((unsigned)e, dtot), r = e - c * tot;
        const int q = (int)udiv((unsigned)r, dn3), k = r - q * n3;
        R ay = w.b, by = w.d;
        if (k == 0 || 2 * k == n3) { ay = 0; by = 0; }
        else if (2 * k > n3) { ay = -ay; by = -by; }
        V X;
        X.x = w.a - by;
        X.y = ay + w.c;
        buf[c * fs + q * pl2 + k] = X;
      });
  __syncthreads();
  fft_lds<V, MAXB_C, true>(buf, S.p3, nf * np, 1, pl2, tw3, tid, NT);
  const size_t pbase = (size_t)it.plane * n2 * n3 + (size_t)2 * p0 * n3;
  SKX_G R *out = MODE == MODE_EVAL ? gptr<R>(S.grad) + pbase : gptr<R>(S.pr2[1 - par]) + pbase;
  double sphig = 0.0, bad = 0.0;
  if (MODE == MODE_PREC) {
    for (int e = tid; e < tot; e += NT) {
      const int q = (int)udiv((unsigned)e, dn3), z = e - q * n3;
      const V X = buf[q * pl2 + z];
      out[2 * q * n3 + z] = X.x;
      out[2 * q * n3 + z + n3] = X.y;
    }
  } else {
    // w0 (= 2 phi_t v0) and phi_t of both rows; the FP64 c_P, c_Q arrays
    struct Pt { R w0a, w0b, pa, pb, fa, fb, qa, qb; };
    const SKX_G R *v0 = gptr<R>(S.vpt) + pbase;
    const SKX_G R *phit = gptr<R>(S.phi2[1 - par]) + pbase;
    const SKX_G R *cfP = gptr<R>(S.fpt) + pbase, *cfQ = gptr<R>(S.qpt) + pbase;
    const int sphi = S.slot[0], sn = S.slot[1], sf = S.slot[2], sh = S.slot[3];
    const NaCfg<R> nc = na_cfg<R>(S);
    batched<2, NT, Pt>(
        tot, tid,
        [&](int e) {
          const int q = (int)udiv((unsigned)e, dn3), o = 2 * q * n3 + (e - q * n3);
          Pt p{v0[o], v0[o + n3], phit[o], phit[o + n3], (R)0, (R)0, (R)0, (R)0};
          if (!derive_coefs<R>()) {
            if (sf >= 0) { p.fa = cfP[o]; p.fb = cfP[o + n3]; }
            if (sh >= 0) { p.qa = cfQ[o]; p.qb = cfQ[o + n3]; }
          }
          return p;
        },
        [&](int e, const Pt &p) {
          const int q = (int)udiv((unsigned)e, dn3), z = e - q * n3;
          const V *x = buf + q * pl2 + z;
          R a0 = p.w0a, a1 = p.w0b;
          if (sphi >= 0) { const V X = x[sphi * fs]; a0 += X.x; a1 += X.y; }
          { const V X = x[sn * fs]; a0 += (R)2 * p.pa * X.x; a1 += (R)2 * p.pb * X.y; }
          if (sf >= 0) {
            const R k0 = derive_coefs<R>() ? derived_coef(p.pa, 2, nc) : p.fa;
            const R k1 = derive_coefs<R>() ? derived_coef(p.pb, 2, nc) : p.fb;
            const V X = x[sf * fs];
            a0 += k0 * X.x;
            a1 += k1 * X.y;
          }
          if (sh >= 0) {
            const R k0 = derive_coefs<R>() ? derived_coef(p.pa, 3, nc) : p.qa;
            const R k1 = derive_coefs<R>() ? derived_coef(p.pb, 3, nc) : p.qb;
            const V X = x[sh * fs];
            a0 += k0 * X.x;
            a1 += k1 * X.y;
          }
          out[2 * q * n3 + z] = a0;
          out[2 * q * n3 + z + n3] = a1;
          sphig += (double)p.pa * (double)a0 + (double)p.pb * (double)a1;
          if (!(a0 == a0)) bad += 1.0;
          if (!(a1 == a1)) bad += 1.0;
        });
    double v[PART_C] = {sphig, bad};
    double tot2[PART_C];
    __syncthreads();
    block_reduce<PART_C>(v, reinterpret_cast<double *>(smem), tid, NT, tot2);
    if (tid == 0)
      for (int q = 0; q < PART_C; ++q)
        S.partC[((size_t)it.plane * S.nrc + it.j) * PART_C + q] = tot2[q];
  }
}

// ---------------------------------------------------------------------------
// Pass A on cubic grids of a length N fixed at compile time (radix order,
// wavefront count and LDS pitch from CShape<N>), one workgroup of NW
// wavefronts per (x-plane, field) (MODE_PREC: per x-plane, the residual
// field). Every wavefront takes N/(2 NW) row pairs: its first z stage reads
// x_{2p} + i x_{2p+1} straight from the pointwise arrays, the remaining
// stages run in LDS and leave the row pair's spectrum there, which is then
// split into the two half spectra with the real DC and Nyquist values of
// each row folded into its column 0. After a barrier every wavefront takes
// N/(2 NW) of the N/2 columns for the y transform, whose last stage goes
// from registers to HBM; the folded column is unfolded into the DC and
// Nyquist columns on the way.
// ---------------------------------------------------------------------------
template <typename R, int N, int MODE>
__global__ __launch_bounds__(CS<N>::NT) void k_passAf(SolveDev *dev, const int *first, int nsolve,
                                                      int grid, const double *twbank) {
  typedef typename Vec2<R>::T V;
  typedef CS<N> K;
  constexpr int NT = K::NT, C = K::C, PL = K::PL, YC = K::YC, ZP = K::ZP;
  constexpr int R0 = K::R0, YL = K::RL, NSL = K::NSL;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (!active_phase<MODE>(st->phase)) return;
  const int par = st->par;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int local = item - first_of(first, s);
  const int nf = MODE == MODE_EVAL ? S.nf : 1;
  const int plane = local / nf;
  const int fb = MODE == MODE_EVAL ? nth_field(S.fields, local - plane * nf) : 0;
  V *buf = reinterpret_cast<V *>(smem);
  V *tw2 = buf + N * PL;
  V *tw3 = tw2 + N;
  // both twiddle tables (tw3 follows tw2) are fetched into registers here
  // and written to LDS after the first z stage, so their latency overlaps
  // that of the stage's HBM loads
  static_assert(2 * N <= NT, "one twiddle per thread");
  const bool has_tw = tid < 2 * N;
  double2 twv = make_double2(0.0, 0.0);
  if (has_tw) twv = ldg(gptr<double2>(twbank) + (tid < N ? S.p2.tw + tid : S.p3.tw + tid - N));
  const R invM = (R)(1.0 / (double)S.M);
  const size_t pbase = (size_t)plane * N * N;
  V *zb = buf + wave * ZP * 2 * PL;
  {
    // first z stage, inputs from HBM: element e = j + NB r of pair p
    typedef CMap<N, R0, ZP, false> M;
    V v[M::MB][R0];
    const SKX_G R *pt = gptr<R>(S.phi2[1 - par]) + pbase;
    const SKX_G R *fa = gptr<R>(S.npa) + pbase;
    const SKX_G R *gr = gptr<R>(S.grad) + pbase;
    SKX_G R *rt = gptr<R>(S.r2[1 - par]) + pbase;
    const R n0 = (R)S.n0, n0a = (R)S.n0a;
    const NaCfg<R> nc = na_cfg<R>(S);
    const R mu2 = MODE == MODE_PREC ? (R)(2.0 * st->mut) : (R)0;
    constexpr bool DER = derive_na<R>();
    const bool need_p = fb != 2 || DER, need_fa = fb >= 2 && !DER;
#pragma unroll
    for (int i = 0; i < M::MB; ++i) {
      const int b = lane + 64 * i;
      if (M::ok(b)) {
        const int o = 2 * (wave * ZP + M::t(b)) * N + M::j(b);
        R x[2][R0];
        if (MODE == MODE_EVAL) {
          R pv[2][R0], fv[2][R0];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              const int q = o + h * N + M::NB * r;
              if (need_p) pv[h][r] = pt[q];
              if (need_fa) fv[h][r] = fa[q];
            }
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              const R p = need_p ? pv[h][r] : (R)0;
              const R f = DER ? (fb >= 2 ? derived_na(p, nc) : (R)0) : (need_fa ? fv[h][r] : (R)0);
              x[h][r] = fb == 0 ? p : fb == 1 ? p * p : fb == 2 ? f : (f - n0a) * (p * p - n0);
            }
        } else {
          R gv[2][R0], pv[2][R0];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              const int q = o + h * N + M::NB * r;
              gv[h][r] = gr[q];
              pv[h][r] = pt[q];
            }
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < R0; ++r) {
              x[h][r] = gv[h][r] - mu2 * pv[h][r];
              rt[o + h * N + M::NB * r] = x[h][r];
            }
        }
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          v[i][r].x = x[0][r] * invM;
          v[i][r].y = x[1][r] * invM;
        }
        Bfly<R0, false, V>::run(v[i]);
        V *out = zb + 2 * M::t(b) * PL + M::j(b) * R0;
#pragma unroll
        for (int r = 0; r < R0; ++r) out[r] = v[i][r];
      }
    }
    if (has_tw) { V t; t.x = twv.x; t.y = twv.y; tw2[tid] = t; }
    __syncthreads();
  }
  CStages<typename K::Rest>::template run<V, N, R0, 1, 2 * PL, ZP, false, false>(zb, tw3, lane);
  {
    // split X_k of the pair into the rows' half spectra; column 0 of each
    // row takes (DC, Nyquist), both real
    constexpr int TOT = ZP * C, NU = (TOT + 63) / 64;
    V A[NU], B[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = lane + 64 * u;
      if (TOT % 64 == 0 || e < TOT) {
        const int p = e / C, k = e % C;
        const V *row = zb + 2 * p * PL;
        const V X = row[k];
        const V Xm = row[k == 0 ? C : N - k];
        if (k == 0) {
          A[u].x = X.x; A[u].y = Xm.x;
          B[u].x = X.y; B[u].y = Xm.y;
        } else {
          A[u].x = (R)0.5 * (X.x + Xm.x); A[u].y = (R)0.5 * (X.y - Xm.y);
          B[u].x = (R)0.5 * (X.y + Xm.y); B[u].y = (R)-0.5 * (X.x - Xm.x);
        }
      }
    }
    SKX_WAVE_SYNC();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = lane + 64 * u;
      if (TOT % 64 == 0 || e < TOT) {
        const int p = e / C, k = e % C;
        zb[2 * p * PL + k] = A[u];
        zb[(2 * p + 1) * PL + k] = B[u];
      }
    }
  }
  __syncthreads();
  SKX_G V *spec = gptr<V>(S.spec) + (size_t)(MODE == MODE_EVAL ? S.slot[fb] : 0) * S.H +
                  (size_t)plane * N * S.pitch;
  const int pitch = S.pitch;
  V *cb = buf + wave * YC;
  CStages<typename K::Init>::template run<V, N, 1, PL, 1, YC, true, false>(cb, tw2, lane);
  {
    typedef CMap<N, YL, YC, true> M;
#pragma unroll
    for (int i = 0; i < M::MB; ++i) {
      const int b = lane + 64 * i;
      if (M::ok(b)) {
        const int t = M::t(b), j = M::j(b);
        V v[YL];
#pragma unroll
        for (int r = 0; r < YL; ++r) v[r] = cb[t + (j + M::NB * r) * PL];
        cbfly<V, N, YL, NSL, false>(v, j, tw2);
        const int col = wave * YC + t;
        if (col != 0) {
#pragma unroll
          for (int r = 0; r < YL; ++r) stg(spec + (size_t)(j + NSL * r) * pitch + col, v[r]);
        } else {
#pragma unroll
          for (int r = 0; r < YL; ++r) buf[(j + NSL * r) * PL] = v[r];
        }
      }
    }
  }
  if (wave == 0) {
    // unfold column 0: Z = F_DC + i F_Nyq of two real columns
    SKX_WAVE_SYNC();
    constexpr int NY = (N + 63) / 64;
#pragma unroll
    for (int u = 0; u < NY; ++u) {
      const int y = lane + 64 * u;
      if (y < N) {
        const V Z = buf[y * PL], Zm = buf[((N - y) % N) * PL];
        V F0, Fn;
        F0.x = (R)0.5 * (Z.x + Zm.x); F0.y = (R)0.5 * (Z.y - Zm.y);
        Fn.x = (R)0.5 * (Z.y + Zm.y); Fn.y = (R)-0.5 * (Z.x - Zm.x);
        stg(spec + (size_t)y * pitch, F0);
        stg(spec + (size_t)y * pitch + C, Fn);
      }
    }
  }
}

// The Nyquist column (k3 = N/2) of pass B on k_passBf, one wavefront per y
// index: the x transform of that column of every field (the first stage
// one butterfly per lane, from HBM), the multipliers and energy terms of
// its G points, and the energy row k_passB's last column block would
// write. tile holds NFIELD (N + 1) values of this wavefront.
template <typename R, int N, int MODE>
__device__ __forceinline__ void passB_nyquist(const SolveDev &S, int jy, typename Vec2<R>::T *tile,
                                              const typename Vec2<R>::T *tw1, int lane) {
  typedef typename Vec2<R>::T V;
  typedef CS<N> K;
  constexpr int X0 = K::R0, XL = K::RL, NSL = K::NSL;
  constexpr int TP = N + 1;                           // LDS pitch between fields
  const int kc = S.nh - 1;                            // the Nyquist column
  const int nf = MODE == MODE_EVAL ? S.nf : 1;
  const size_t rowstride = (size_t)S.n2 * S.pitch;
  SKX_G V *spec = gptr<V>(S.spec) + (size_t)jy * S.pitch + kc;
  typedef CMap<N, X0, NFIELD, false> M;               // lane -> (field slot, butterfly)
  static_assert(M::MB == 1, "one first-stage butterfly per lane");
  {
    const int b = lane;
    if (M::ok(b)) {
      const int t = M::t(b), jj = M::j(b);
      V v[X0];
#pragma unroll
      for (int r = 0; r < X0; ++r) {
        if (t < nf) v[r] = ldg(spec + (size_t)t * S.H + (size_t)(jj + M::NB * r) * rowstride);
        else { v[r].x = 0; v[r].y = 0; }
      }
      Bfly<X0, false, V>::run(v);
#pragma unroll
      for (int r = 0; r < X0; ++r) tile[t * TP + jj * X0 + r] = v[r];
    }
  }
  SKX_WAVE_SYNC();
  CStages<typename K::Rest>::template run<V, N, X0, 1, TP, NFIELD, false, false>(tile, tw1, lane);
  double evw = 0, eh = 0, ef0 = 0, ef1 = 0, eloc = 0, bad = 0;
  const int k3 = kc, g2 = gidx(jy, S.n2);
  const unsigned terms = S.terms;
  const bool do_vw = terms & 2u, do_nl0 = terms & 4u;
  const bool do_h = terms & 16u, do_loc = terms & 32u;
  const int sphi = S.slot[0], sn = S.slot[1], sfl = S.slot[2], sh = S.slot[3];
  const R b3 = (R)(S.beta / 3.0);
  const double FOURPI = 12.566370614359172954;
  // G points kx = lane, lane + 64, ... of the column
  for (int kx = lane; kx < N; kx += 64) {
    const int g1 = gidx(kx, N);
    const int sidx = g1 * g1 + g2 * g2 + k3 * k3;
    const double G2 = S.kscale * (double)sidx;
    if (MODE == MODE_PREC) {
      const R pg = (R)(1.0 / (G2 + S.kappa));
      V x = tile[kx];
      x.x *= pg; x.y *= pg;
      tile[kx] = x;
      continue;
    }
    V vl;
    vl.x = 0; vl.y = 0;
    if (do_loc) vl = ldg(gptr<V>(S.vloc) + ((size_t)kx * S.n2 + jy) * S.pitch + k3);
    double wv = 0.0, wpv = 0.0;
    if (sfl >= 0) { wv = gptr<double>(S.w)[sidx]; wpv = gptr<double>(S.wp)[sidx]; }
    // the Nyquist column has weight 1 in the Hermitian sums
    if (sphi >= 0) {
      V x = tile[sphi * TP + kx];
      if (do_vw) evw += G2 * ((double)x.x * x.x + (double)x.y * x.y);
      const R g2r = (R)G2;
      x.x *= g2r; x.y *= g2r;
      tile[sphi * TP + kx] = x;
    }
    {
      const V x = tile[sn * TP + kx];
      double bx = 0.0, by = 0.0;
      if (do_h && sidx > 0) {
        eh += ((double)x.x * x.x + (double)x.y * x.y) / G2;
        bx = FOURPI * x.x / G2;
        by = FOURPI * x.y / G2;
      }
      if (do_loc) {
        eloc += (double)x.x * vl.x + (double)x.y * vl.y;
        bx += vl.x;
        by += vl.y;
      }
      if (!(x.x == x.x) || !(x.y == x.y)) bad += 1.0;
      V o; o.x = (R)bx; o.y = (R)by;
      tile[sn * TP + kx] = o;
    }
    if (sfl >= 0) {
      const V f = tile[sfl * TP + kx];
      const R w = (R)wv, wp = (R)wpv;
      V P; P.x = 0; P.y = 0;
      if (do_nl0) {
        ef0 += (double)w * ((double)f.x * f.x + (double)f.y * f.y);
        P.x = (R)2 * w * f.x; P.y = (R)2 * w * f.y;
      }
      if (sh >= 0) {
        const V h = tile[sh * TP + kx];
        ef1 += (double)wp * ((double)f.x * h.x + (double)f.y * h.y);
        P.x += b3 * wp * h.x; P.y += b3 * wp * h.y;
        V Q; Q.x = b3 * wp * f.x; Q.y = b3 * wp * f.y;
        tile[sh * TP + kx] = Q;
      }
      tile[sfl * TP + kx] = P;
    }
  }
  SKX_WAVE_SYNC();
  CStages<typename K::Init>::template run<V, N, 1, 1, TP, NFIELD, false, true>(tile, tw1, lane);
  {
    typedef CMap<N, XL, NFIELD, false> ML;
#pragma unroll
    for (int i = 0; i < ML::MB; ++i) {
      const int b = lane + 64 * i;
      if (ML::ok(b)) {
        const int t = ML::t(b), jj = ML::j(b);
        V v[XL];
#pragma unroll
        for (int r = 0; r < XL; ++r) v[r] = tile[t * TP + jj + ML::NB * r];
        cbfly<V, N, XL, NSL, true>(v, jj, tw1);
        if (t < nf) {
#pragma unroll
          for (int r = 0; r < XL; ++r)
            stg(spec + (size_t)t * S.H + (size_t)(jj + NSL * r) * rowstride, v[r]);
        }
      }
    }
  }
  if (MODE == MODE_EVAL) {
    double vals[PART_B] = {evw, eh, ef0, ef1, eloc, bad};
#pragma unroll
    for (int q = 0; q < PART_B; ++q)
      for (int off = 32; off > 0; off >>= 1) vals[q] += __shfl_down(vals[q], off, 64);
    if (lane == 0)
      for (int q = 0; q < PART_B; ++q) S.partB[(jy * S.nkb + S.nkb - 1) * PART_B + q] = vals[q];
  }
}

// ---------------------------------------------------------------------------
// Pass B for cubic grids of a length N fixed at compile time, one workgroup
// of four wavefronts per (y index, block of TK z columns). In MODE_EVAL
// wavefront w owns the x transforms of field slot w (all TK columns); in
// MODE_PREC the one field's columns are split over the four. The first
// forward stage reads its inputs from HBM, the last inverse stage writes its
// outputs there from registers; between the two directions the multipliers
// and energy terms of every G point run over the LDS tiles. Needs
// (N/2) % TK == 0: the column blocks stop below the Nyquist column, which
// extra workgroups take for four y rows each, one per wavefront.
// ---------------------------------------------------------------------------
// LDS of the shaped pass B in complex elements before its twiddle table:
// the four field tiles in MODE_EVAL; in MODE_PREC (one field) one tile, or
// the Nyquist workgroups' per-wavefront tiles where those exist, so the
// preconditioner's launches take a quarter of the LDS and fit more
// workgroups per CU.
// Ragged column blocks over all N/2 + 1 columns (the last one holding the
// Nyquist column) where TK does not divide N/2, or where the Nyquist
// column's first transform stage would not fit one butterfly per lane.
template <int N, int TK> constexpr bool passb_ragged() {
  return (N / 2) % TK != 0 || NFIELD * N / CS<N>::R0 > 64;
}
template <int N, int TK, int MODE> constexpr int passb_tw_off() {
  constexpr int TP = TK + 1;
  constexpr bool RAG = passb_ragged<N, TK>();
  constexpr int NY = RAG ? 0 : 4 * NFIELD * (N + 1);
  return MODE == MODE_EVAL ? NFIELD * N * TP : (N * TP > NY ? N * TP : NY);
}

template <typename R, int N, int TK, int MODE>
__global__ __launch_bounds__(256) void k_passBf(SolveDev *dev, const int *first, int nsolve,
                                                int grid, const double *twbank) {
  typedef typename Vec2<R>::T V;
  typedef CS<N> K;
  constexpr int NT = 256, NW = 4;
  constexpr int X0 = K::R0, XL = K::RL, NSL = K::NSL;
  constexpr int TP = TK + 1;                       // LDS row pitch of a field tile
  constexpr int SL = MODE == MODE_EVAL ? TK : TK / NW;   // columns per wavefront
  static_assert(MODE == MODE_EVAL || TK % NW == 0, "preconditioner columns split evenly");
  extern __shared__ __align__(16) unsigned char smem[];
  // Whole blocks below the Nyquist column when TK divides N/2, the Nyquist
  // column then on passB_nyquist; otherwise (ragged) blocks over all N/2 + 1
  // columns, the last one partial and holding the Nyquist column.
  constexpr bool RAG = passb_ragged<N, TK>();
  constexpr int NB = RAG ? (N / 2 + TK) / TK : (N / 2) / TK;
  constexpr int PER = N * NB + (RAG ? 0 : N / NW);  // workgroups per solve
  static_assert(RAG || N % NW == 0, "Nyquist rows split evenly");
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  const int s = __builtin_amdgcn_readfirstlane(item / PER);
  const SolveDev &S = dev[s];
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (!active_phase<MODE>(st->phase)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rem = item - s * PER;
  if constexpr (!RAG) {
    if (rem >= N * NB) {
      V *tw = reinterpret_cast<V *>(smem) + passb_tw_off<N, TK, MODE>();
      load_twiddles(tw, twbank, S.p1.tw, N, tid, NT);
      __syncthreads();
      passB_nyquist<R, N, MODE>(S, (rem - N * NB) * NW + wave,
                                reinterpret_cast<V *>(smem) + wave * NFIELD * (N + 1), tw, lane);
      return;
    }
  }
  const int jy = rem / NB, kb = rem - (rem / NB) * NB;
  const int local = jy * S.nkb + kb;                 // energy row, as in k_passB
  const int k0 = kb * TK;
  const int tkv = RAG ? min(TK, N / 2 + 1 - k0) : TK;
  const int nf = MODE == MODE_EVAL ? S.nf : 1;
  V *tile = reinterpret_cast<V *>(smem);             // [NFIELD][N][TP] (MODE_PREC: [1][N][TP])
  V *tw1 = tile + passb_tw_off<N, TK, MODE>();
  SKX_G V *spec = gptr<V>(S.spec) + (size_t)jy * S.pitch + k0;
  const size_t rowstride = (size_t)S.n2 * S.pitch;
  const int cc = MODE == MODE_EVAL ? wave : 0;       // field slot of this wavefront
  const int c0 = MODE == MODE_EVAL ? 0 : wave * SL;  // its first column
  const bool active = cc < nf;
  V *tf = tile + cc * N * TP + c0;
  SKX_G V *sf = spec + (size_t)cc * S.H + c0;
  const int cv = tkv - c0;                           // valid columns from c0
  typedef CMap<N, X0, SL, true> M0;
  V v[M0::MB][X0];
  if (active) {
    typedef M0 M;
#pragma unroll
    for (int i = 0; i < M::MB; ++i) {
      const int b = lane + 64 * i;
      if (M::ok(b)) {
        const int t = M::t(b), jj = M::j(b);
#pragma unroll
        for (int r = 0; r < X0; ++r) {
          if (t < cv) v[i][r] = ldg(sf + (size_t)(jj + M::NB * r) * rowstride + t);
          else { v[i][r].x = 0; v[i][r].y = 0; }
        }
      }
    }
  }
  // the twiddle table is loaded while the spectrum loads are in flight
  load_twiddles(tw1, twbank, S.p1.tw, N, tid, NT);
  __syncthreads();
  if (active) {
    typedef M0 M;
#pragma unroll
    for (int i = 0; i < M::MB; ++i) {
      const int b = lane + 64 * i;
      if (M::ok(b)) {
        const int t = M::t(b), jj = M::j(b);
        Bfly<X0, false, V>::run(v[i]);
#pragma unroll
        for (int r = 0; r < X0; ++r) tf[(jj * X0 + r) * TP + t] = v[i][r];
      }
    }
    SKX_WAVE_SYNC();
    CStages<typename K::Rest>::template run<V, N, X0, TP, 1, SL, true, false>(tf, tw1, lane);
  }
  __syncthreads();
  const double kscale = S.kscale;
  const int g2 = gidx(jy, S.n2);
  double evw = 0, eh = 0, ef0 = 0, ef1 = 0, eloc = 0, bad = 0;
  constexpr int NP = (N * TK + NT - 1) / NT;
  if (MODE == MODE_PREC) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = tid + u * NT;
      const int kx = e / TK, col = e % TK;
      if ((N * TK % NT == 0 || e < N * TK) && col < tkv) {
        const int k3 = k0 + col, g1 = gidx(kx, N);
        const double G2 = kscale * (double)(g1 * g1 + g2 * g2 + k3 * k3);
        const R pg = (R)(1.0 / (G2 + S.kappa));
        V x = tile[kx * TP + col];
        x.x *= pg; x.y *= pg;
        tile[kx * TP + col] = x;
      }
    }
  } else {
    const unsigned terms = S.terms;
    const bool do_vw = terms & 2u, do_nl0 = terms & 4u;
    const bool do_h = terms & 16u, do_loc = terms & 32u;
    const int sphi = S.slot[0], sn = S.slot[1], sfl = S.slot[2], sh = S.slot[3];
    const SKX_G V *vloc = gptr<V>(S.vloc);
    const R b3 = (R)(S.beta / 3.0);
    const double FOURPI = 12.566370614359172954;
    const SKX_G double *wt = gptr<double>(S.w);
    const SKX_G double *wpt = gptr<double>(S.wp);
    V vlb[NP];
    double wb[NP], wpb[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = tid + u * NT;
      const int kx = e / TK, col = e % TK;
      if ((N * TK % NT == 0 || e < N * TK) && col < tkv) {
        const int k3 = k0 + col, g1 = gidx(kx, N);
        const int sidx = g1 * g1 + g2 * g2 + k3 * k3;
        if (do_loc) vlb[u] = ldg(vloc + ((size_t)kx * S.n2 + jy) * S.pitch + k3);
        if (sfl >= 0) { wb[u] = wt[sidx]; wpb[u] = wpt[sidx]; }
      }
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = tid + u * NT;
      const int kx = e / TK, col = e % TK;
      if (!((N * TK % NT == 0 || e < N * TK) && col < tkv)) continue;
      const int k3 = k0 + col, g1 = gidx(kx, N);
      const int sidx = g1 * g1 + g2 * g2 + k3 * k3;
      const double G2 = kscale * (double)sidx;
      const double wgt = (k3 == 0 || 2 * k3 == S.n3) ? 1.0 : 2.0;
      V *pt = tile + kx * TP + col;                  // field slot c at pt[c N TP]
      if (sphi >= 0) {
        V x = pt[sphi * N * TP];
        if (do_vw) evw += wgt * G2 * ((double)x.x * x.x + (double)x.y * x.y);
        const R g2r = (R)G2;
        x.x *= g2r; x.y *= g2r;
        pt[sphi * N * TP] = x;
      }
      {
        const V x = pt[sn * N * TP];
        double bx = 0.0, by = 0.0;
        if (do_h && sidx > 0) {
          const double m2 = (double)x.x * x.x + (double)x.y * x.y;
          const double ig = 1.0 / G2;
          eh += wgt * m2 * ig;
          bx = FOURPI * ig * x.x;
          by = FOURPI * ig * x.y;
        }
        if (do_loc) {
          const V vl = vlb[u];
          eloc += wgt * ((double)x.x * vl.x + (double)x.y * vl.y);
          bx += vl.x;
          by += vl.y;
        }
        if (!(x.x == x.x) || !(x.y == x.y)) bad += 1.0;
        V o; o.x = (R)bx; o.y = (R)by;
        pt[sn * N * TP] = o;
      }
      if (sfl >= 0) {
        const V f = pt[sfl * N * TP];
        const R w = (R)wb[u];
        const R wp = (R)wpb[u];
        V P; P.x = 0; P.y = 0;
        if (do_nl0) {
          ef0 += wgt * (double)w * ((double)f.x * f.x + (double)f.y * f.y);
          P.x = (R)2 * w * f.x; P.y = (R)2 * w * f.y;
        }
        if (sh >= 0) {
          const V h = pt[sh * N * TP];
          ef1 += wgt * (double)wp * ((double)f.x * h.x + (double)f.y * h.y);
          P.x += b3 * wp * h.x; P.y += b3 * wp * h.y;
          V Q; Q.x = b3 * wp * f.x; Q.y = b3 * wp * f.y;
          pt[sh * N * TP] = Q;
        }
        pt[sfl * N * TP] = P;
      }
    }
  }
  __syncthreads();
  if (active) {
    CStages<typename K::Init>::template run<V, N, 1, TP, 1, SL, true, true>(tf, tw1, lane);
    typedef CMap<N, XL, SL, true> M;
#pragma unroll
    for (int i = 0; i < M::MB; ++i) {
      const int b = lane + 64 * i;
      if (M::ok(b)) {
        const int t = M::t(b), jj = M::j(b);
        V w[XL];
#pragma unroll
        for (int r = 0; r < XL; ++r) w[r] = tf[(jj + M::NB * r) * TP + t];
        cbfly<V, N, XL, NSL, true>(w, jj, tw1);
        if (t < cv) {
#pragma unroll
          for (int r = 0; r < XL; ++r) stg(sf + (size_t)(jj + NSL * r) * rowstride + t, w[r]);
        }
      }
    }
  }
  if (MODE == MODE_EVAL) {
    double vals[PART_B] = {evw, eh, ef0, ef1, eloc, bad};
    double tot[PART_B];
    __syncthreads();
    block_reduce<PART_B>(vals, reinterpret_cast<double *>(smem), tid, NT, tot);
    if (tid == 0)
      for (int q = 0; q < PART_B; ++q) S.partB[local * PART_B + q] = tot[q];
  }
}

// ---------------------------------------------------------------------------
// Pass C on cubic grids of a length N fixed at compile time, one workgroup
// of NW wavefronts per x-plane, every index a constant. Per field:
//  * the half spectrum of the plane is copied into LDS;
//  * the DC and Nyquist columns, whose inverse y transforms are real, are
//    each reduced to their Hermitian part (whose inverse is the real part of
//    the plain inverse) and folded into one complex column, so the N/2
//    columns split evenly over the wavefronts;
//  * after a barrier every wavefront takes N/(2 NW) row pairs: its first z
//    stage builds x_{2p} + i x_{2p+1} over the full row from the two half
//    spectra, its last stage keeps the outputs in registers, where they are
//    assembled with their pointwise coefficients into dE/dphi of the points
//    of the butterflies the lane owns (the same points for every field).
// MODE_PREC transforms the one preconditioner field back to real space.
// ---------------------------------------------------------------------------
template <typename V, int N, int RAD, int ZP>
__device__ __forceinline__ void zfirst_merge(V *buf, int lane) {
  constexpr int C = N / 2, PL = CS<N>::PL;
  typedef CMap<N, RAD, ZP, false> M;
  static_assert(RAD % 2 == 0, "even first radix");
  V v[M::MB][RAD];
#pragma unroll
  for (int i = 0; i < M::MB; ++i) {
    const int b = lane + 64 * i;
    if (M::ok(b)) {
      const int p = M::t(b), j = M::j(b);
      const V *ra = buf + 2 * p * PL, *rb = ra + PL;
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        const int e = j + M::NB * r;
        V a, c;
        if (r < RAD / 2) {                   // 0 <= e < C
          a = ra[e]; c = rb[e];
          if (r == 0 && j == 0) { a.y = 0; c.y = 0; }        // DC: real part of column 0
        } else {                             // C <= e < N: Hermitian mirror
          const bool nyq = (r == RAD / 2) && (j == 0);
          const int m = nyq ? 0 : N - e;
          a = ra[m]; c = rb[m];
          if (nyq) { a.x = a.y; a.y = 0; c.x = c.y; c.y = 0; }  // Nyquist: imaginary part of column 0
          else { a.y = -a.y; c.y = -c.y; }
        }
        v[i][r].x = a.x - c.y;
        v[i][r].y = a.y + c.x;
      }
    }
  }
  SKX_WAVE_SYNC();
#pragma unroll
  for (int i = 0; i < M::MB; ++i) {
    const int b = lane + 64 * i;
    if (M::ok(b)) {
      const int p = M::t(b), j = M::j(b);
      Bfly<RAD, true, V>::run(v[i]);
      V *out = buf + 2 * p * PL + j * RAD;
#pragma unroll
      for (int r = 0; r < RAD; ++r) out[r] = v[i][r];
    }
  }
  SKX_WAVE_SYNC();
}

// Columns 0 and C of the plane (rows [0, N)) folded into column 0 as
// herm(X_0) + i herm(X_C), by one wavefront.
template <typename V, int N>
__device__ __forceinline__ void fold_dc_nyquist(V *buf, int lane) {
  typedef decltype(buf[0].x) R;
  constexpr int C = N / 2, PL = CS<N>::PL, NY = (N + 63) / 64;
  V z[NY];
#pragma unroll
  for (int u = 0; u < NY; ++u) {
    const int y = lane + 64 * u;
    if (y < N) {
      const int ym = (N - y) % N;
      const V a = buf[y * PL], am = buf[ym * PL], b = buf[y * PL + C], bm = buf[ym * PL + C];
      const R h0x = (R)0.5 * (a.x + am.x), h0y = (R)0.5 * (a.y - am.y);
      const R hnx = (R)0.5 * (b.x + bm.x), hny = (R)0.5 * (b.y - bm.y);
      z[u].x = h0x - hny;
      z[u].y = h0y + hnx;
    }
  }
  SKX_WAVE_SYNC();
#pragma unroll
  for (int u = 0; u < NY; ++u) {
    const int y = lane + 64 * u;
    if (y < N) buf[y * PL] = z[u];
  }
  SKX_WAVE_SYNC();
}

// Inverse y transform and the z stages but the last of the plane in buf; on
// return the lane's last-stage butterflies are in v (outputs at
// z = j + NSL r of the row pair p, real parts row 2p, imaginary parts row
// 2p+1).
template <typename V, int N, int MB>
__device__ __forceinline__ void plane_inverse_f(V *buf, const V *tw2, const V *tw3, int lane,
                                                int wave, V (&v)[MB][CS<N>::RL]) {
  typedef CS<N> K;
  constexpr int PL = K::PL, YC = K::YC, ZP = K::ZP, R0 = K::R0, RL = K::RL, NSL = K::NSL;
  if (wave == 0) fold_dc_nyquist<V, N>(buf, lane);
  CStages<typename K::L>::template run<V, N, 1, PL, 1, YC, true, true>(buf + wave * YC, tw2, lane);
  __syncthreads();
  V *zb = buf + wave * ZP * 2 * PL;
  zfirst_merge<V, N, R0, ZP>(zb, lane);
  CStages<typename K::Mid>::template run<V, N, R0, 1, 2 * PL, ZP, false, true>(zb, tw3, lane);
  typedef CMap<N, RL, ZP, false> ZM;
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = lane + 64 * i;
    if (ZM::ok(b)) {
      const int p = ZM::t(b), j = ZM::j(b);
      const V *base = zb + 2 * p * PL + j;
#pragma unroll
      for (int r = 0; r < RL; ++r) v[i][r] = base[r * ZM::NB];
      cbfly<V, N, RL, NSL, true>(v[i], j, tw3);
    }
  }
}

// (the launch bound asks for CShape's CW waves per SIMD: FP64 at 64^3 fits
// 168 VGPRs with three 256-thread groups)
// Pass C prefetches the next field's plane at the lengths where it measured
// faster (60, 72, 80: 5-7% per launch); at 48 and 64 the extra registers
// spill.
template <typename R, int N> constexpr bool passc_prefetch() { return N == 60 || N >= 72; }

template <typename R, int N, int MODE>
__global__ __launch_bounds__(CS<N>::NT, CS<N>::CW)
void k_passCf(SolveDev *dev, const int *first, int nsolve, int grid, const double *twbank) {
  typedef typename Vec2<R>::T V;
  typedef CS<N> K;
  constexpr int NT = K::NT, C = K::C, PL = K::PL, ZP = K::ZP, RL = K::RL, NSL = K::NSL;
  typedef CMap<N, RL, ZP, false> ZM;
  constexpr int MB = ZM::MB;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = xcd_item(blockIdx.x, grid);
  if (item >= grid) return;
  const int s = find_solve(first, nsolve, item);
  const SolveDev &S = dev[s];
  const SKX_C OptState *st = cptr<OptState>(S.st);
  if (!active_phase<MODE>(st->phase)) return;
  const int par = st->par;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int plane = item - first_of(first, s);
  V *buf = reinterpret_cast<V *>(smem);
  V *tw2 = buf + N * PL;
  V *tw3 = tw2 + N;
  load_twiddles(tw2, twbank, S.p2.tw, N, tid, NT);
  load_twiddles(tw3, twbank, S.p3.tw, N, tid, NT);
  const size_t pbase = (size_t)plane * N * N;
  const SKX_G V *spec = gptr<V>(S.spec) + (size_t)plane * N * S.pitch;
  const int pitch = S.pitch;
  // the lane's points: row 2p + h, z = j + NSL r of butterfly slot i
  int pt[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = lane + 64 * i;
    pt[i] = ZM::ok(b) ? 2 * (wave * ZP + ZM::t(b)) * N + ZM::j(b) : -1;
  }
  V v[MB][RL];

  if (MODE == MODE_PREC) {
    load_plane_f<V, N, C + 1, PL, NT>(buf, spec, pitch, tid);
    __syncthreads();
    plane_inverse_f<V, N, MB>(buf, tw2, tw3, lane, wave, v);
    SKX_G R *out = gptr<R>(S.pr2[1 - par]) + pbase;
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (pt[i] >= 0) {
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          out[pt[i] + NSL * r] = v[i][r].x;
          out[pt[i] + N + NSL * r] = v[i][r].y;
        }
      }
    return;
  }

  // dE/dphi = w0 + A + 2 phi_t B + c_P P + c_Q Q with w0 = 2 phi_t v0 from
  // the pointwise pass, the fields in slot order; phi_t is kept in
  // registers in FP32, and read again for B and the closing sums in FP64.
  constexpr bool KEEP_PHI = sizeof(R) == 4;
  constexpr bool DER = derive_coefs<R>();         // c_P, c_Q from phi_t
  const NaCfg<R> nc = na_cfg<R>(S);
  const SKX_G R *phit = gptr<R>(S.phi2[1 - par]) + pbase;
  const SKX_G R *cfp[NFIELD] = {nullptr, phit, gptr<R>(S.fpt) + pbase, gptr<R>(S.qpt) + pbase};
  SKX_G R *grad = gptr<R>(S.grad) + pbase;
  R acc[MB][2][RL];
  R ph[KEEP_PHI ? MB : 1][2][RL];
  {
    const SKX_G R *w0 = gptr<R>(S.vpt) + pbase;
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (pt[i] >= 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < RL; ++r) {
            const int o = pt[i] + h * N + NSL * r;
            acc[i][h][r] = w0[o];
            if (KEEP_PHI) ph[KEEP_PHI ? i : 0][h][r] = phit[o];
          }
      }
  }
  double sphig = 0.0, bad = 0.0;
  // With PF the next field's plane is loaded into registers while the
  // current one is transformed (the lengths whose pass C holds one
  // workgroup per CU, where nothing else would hide the load latency).
  constexpr bool PF = passc_prefetch<R, N>();
  constexpr int TOTP = N * (C + 1), NUP = (TOTP + NT - 1) / NT;
  V pre[PF ? NUP : 1];
  auto fetch = [&](int f) {
    const SKX_G V *src = spec + (size_t)S.slot[f] * S.H;
#pragma unroll
    for (int u = 0; u < NUP; ++u) {
      const int e = tid + u * NT;
      if (TOTP % NT == 0 || e < TOTP) pre[PF ? u : 0] = ldg(src + (size_t)(e / (C + 1)) * pitch + e % (C + 1));
    }
  };
  auto next_field = [&](int f) {
    for (int q = f + 1; q < NFIELD; ++q)
      if (S.slot[q] >= 0) return q;
    return NFIELD;
  };
  if (PF) {
    const int f0 = next_field(-1);
    if (f0 < NFIELD) fetch(f0);
  }
  for (int fb = 0; fb < NFIELD; ++fb) {
    const int sl = S.slot[fb];
    if (sl < 0) continue;
    __syncthreads();
    if (PF) {
#pragma unroll
      for (int u = 0; u < NUP; ++u) {
        const int e = tid + u * NT;
        if (TOTP % NT == 0 || e < TOTP) buf[(e / (C + 1)) * PL + e % (C + 1)] = pre[PF ? u : 0];
      }
    } else {
      load_plane_f<V, N, C + 1, PL, NT>(buf, spec + (size_t)sl * S.H, pitch, tid);
    }
    __syncthreads();
    if (PF) {
      const int fn = next_field(fb);
      if (fn < NFIELD) fetch(fn);
    }
    plane_inverse_f<V, N, MB>(buf, tw2, tw3, lane, wave, v);
    R cf[MB][2][RL];
    if (fb >= 2 ? !(DER && KEEP_PHI) : (fb == 1 && !KEEP_PHI)) {
      const SKX_G R *src = (fb >= 2 && DER) ? phit : cfp[fb];
#pragma unroll
      for (int i = 0; i < MB; ++i)
        if (pt[i] >= 0) {
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < RL; ++r) cf[i][h][r] = src[pt[i] + h * N + NSL * r];
        }
    }
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (pt[i] >= 0) {
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const R g0 = v[i][r].x, g1 = v[i][r].y;
          if (fb == 0) {
            acc[i][0][r] += g0;
            acc[i][1][r] += g1;
          } else if (fb == 1) {
            const R p0 = KEEP_PHI ? ph[KEEP_PHI ? i : 0][0][r] : cf[i][0][r];
            const R p1 = KEEP_PHI ? ph[KEEP_PHI ? i : 0][1][r] : cf[i][1][r];
            acc[i][0][r] += (R)2 * p0 * g0;
            acc[i][1][r] += (R)2 * p1 * g1;
          } else if (DER) {
            const R p0 = KEEP_PHI ? ph[KEEP_PHI ? i : 0][0][r] : cf[i][0][r];
            const R p1 = KEEP_PHI ? ph[KEEP_PHI ? i : 0][1][r] : cf[i][1][r];
            acc[i][0][r] += derived_coef(p0, fb, nc) * g0;
            acc[i][1][r] += derived_coef(p1, fb, nc) * g1;
          } else {
            acc[i][0][r] += cf[i][0][r] * g0;
            acc[i][1][r] += cf[i][1][r] * g1;
          }
        }
      }
  }
#pragma unroll
  for (int i = 0; i < MB; ++i)
    if (pt[i] >= 0) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int o = pt[i] + h * N + NSL * r;
          const R g = acc[i][h][r];
          const R p = KEEP_PHI ? ph[KEEP_PHI ? i : 0][h][r] : phit[o];
          grad[o] = g;
          sphig += (double)p * (double)g;
          if (!(g == g)) bad += 1.0;
        }
    }
  double vals[PART_C] = {sphig, bad};
  double tot[PART_C];
  __syncthreads();
  block_reduce<PART_C>(vals, reinterpret_cast<double *>(smem), tid, NT, tot);
  if (tid == 0)
    for (int q = 0; q < PART_C; ++q) S.partC[plane * PART_C + q] = tot[q];
}

// ---------------------------------------------------------------------------
// Launch
// ---------------------------------------------------------------------------

// Runtime-shaped pass B with 512 threads: measured faster in FP32 at every
// size, and in FP64 once the x tile takes more than half of a CU's LDS (one
// workgroup per CU).
template <typename R> static bool wide_b(const PassGroup &g) {
  return sizeof(R) == 4 || g.ldsB > 80 * 1024;
}
// Runtime-shaped pass A with 512 threads once its plane takes more than
// 45 KB of LDS (measured: FP64 96^3 177 -> 161 us, 128^3 540 -> 442 us;
// FP32 108^3 157 -> 144 us; smaller planes are faster with 256).
static bool wide_a(const PassGroup &g) { return g.ldsA > 45 * 1024; }

// Compile-time-shaped pass kernels of one length N over one group.
// Pass B column-block width of a compile-time length (the host's
// block_width): 16 in FP32 where it divides N/2, else 8, in ragged blocks
// where 8 does not divide N/2 (measured: ragged blocks of 8 beat whole
// blocks of 4 at 40 and 72).
template <int N, typename R> constexpr int shaped_tk() {
  return (sizeof(R) == 4 && (N / 2) % 16 == 0) ? 16 : 8;
}

template <typename R, int N>
static void launch_shaped(const PassGroup &g, const double *twbank, hipStream_t s, int mask,
                          int mode) {
  typedef typename Vec2<R>::T V;
  constexpr int TK = shaped_tk<N, R>();
  constexpr int NT = CS<N>::NT;
  const size_t lds_plane = CS<N>::lds_plane(sizeof(V));
  if (mode == MODE_EVAL) {
    if (g.gridA > 0 && (mask & 16) && (g.shape & 1))
      SKX_TIMED_LAUNCH((k_passAf<R, N, MODE_EVAL>), dim3(g.gridA), dim3(NT), lds_plane, s, g.dev,
                       g.firstA, g.nsolve, g.gridA, twbank);
  } else if (g.gridC > 0 && (mask & 1) && (g.shape & 1)) {
    // one field per solve: pass A has one workgroup per plane, like pass C
    SKX_TIMED_LAUNCH((k_passAf<R, N, MODE_PREC>), dim3(g.gridC), dim3(NT), lds_plane, s, g.dev,
                     g.firstC, g.nsolve, g.gridC, twbank);
  }
  {
    if (g.gridB > 0 && (mask & 2) && (g.shape & 2) && g.tk == TK) {
      constexpr bool RAG = passb_ragged<N, TK>();
      const int gb = g.nsolve * (RAG ? N * ((N / 2 + TK) / TK) : N * (N / 2 / TK) + N / 4);
      if (mode == MODE_EVAL) {
        const size_t lb = (passb_tw_off<N, TK, MODE_EVAL>() + N) * sizeof(V);
        SKX_TIMED_LAUNCH((k_passBf<R, N, TK, MODE_EVAL>), dim3(gb), dim3(256), lb, s, g.dev,
                         g.firstB, g.nsolve, gb, twbank);
      } else {
        const size_t lb = (passb_tw_off<N, TK, MODE_PREC>() + N) * sizeof(V);
        SKX_TIMED_LAUNCH((k_passBf<R, N, TK, MODE_PREC>), dim3(gb), dim3(256), lb, s, g.dev,
                         g.firstB, g.nsolve, gb, twbank);
      }
    }
  }
  if (g.gridC > 0 && (mask & 4) && (g.shape & 4)) {
    if (mode == MODE_EVAL)
      SKX_TIMED_LAUNCH((k_passCf<R, N, MODE_EVAL>), dim3(g.gridC), dim3(NT), lds_plane, s, g.dev,
                       g.firstC, g.nsolve, g.gridC, twbank);
    else
      SKX_TIMED_LAUNCH((k_passCf<R, N, MODE_PREC>), dim3(g.gridC), dim3(NT), lds_plane, s, g.dev,
                       g.firstC, g.nsolve, g.gridC, twbank);
  }
}

// Pass B alone on the compile-time-shaped kernel, for the larger lengths
// (the group's width equals passb_width, which the host checks).
template <typename R, int N>
static void launch_shaped_b(const PassGroup &g, const double *twbank, hipStream_t s, int mask,
                            int mode) {
  typedef typename Vec2<R>::T V;
  constexpr int TK = passb_width(N, sizeof(R) == 8 ? 0 : 1);
  if (g.gridB <= 0 || !(mask & 2) || !(g.shape & 2) || g.tk != TK) return;
  constexpr bool RAG = passb_ragged<N, TK>();
  const int gb = g.nsolve * (RAG ? N * ((N / 2 + TK) / TK) : N * (N / 2 / TK) + N / 4);
  if (mode == MODE_EVAL) {
    const size_t lb = (passb_tw_off<N, TK, MODE_EVAL>() + N) * sizeof(V);
    SKX_TIMED_LAUNCH((k_passBf<R, N, TK, MODE_EVAL>), dim3(gb), dim3(256), lb, s, g.dev,
                     g.firstB, g.nsolve, gb, twbank);
  } else {
    const size_t lb = (passb_tw_off<N, TK, MODE_PREC>() + N) * sizeof(V);
    SKX_TIMED_LAUNCH((k_passBf<R, N, TK, MODE_PREC>), dim3(gb), dim3(256), lb, s, g.dev,
                     g.firstB, g.nsolve, gb, twbank);
  }
}

template <typename R>
static void launch_shaped_n(const PassGroup &g, const double *twbank, hipStream_t s, int mask,
                            int mode) {
  switch (g.shapeN) {
    case 90: launch_shaped_b<R, 90>(g, twbank, s, mask, mode); break;
    case 96: launch_shaped_b<R, 96>(g, twbank, s, mask, mode); break;
    case 100: launch_shaped_b<R, 100>(g, twbank, s, mask, mode); break;
    case 108: launch_shaped_b<R, 108>(g, twbank, s, mask, mode); break;
    case 120: launch_shaped_b<R, 120>(g, twbank, s, mask, mode); break;
    case 128: launch_shaped_b<R, 128>(g, twbank, s, mask, mode); break;
    case 144: launch_shaped_b<R, 144>(g, twbank, s, mask, mode); break;
    case 150: launch_shaped_b<R, 150>(g, twbank, s, mask, mode); break;
    case 160: launch_shaped_b<R, 160>(g, twbank, s, mask, mode); break;
    case 162: launch_shaped_b<R, 162>(g, twbank, s, mask, mode); break;
    case 180: launch_shaped_b<R, 180>(g, twbank, s, mask, mode); break;
    case 192: launch_shaped_b<R, 192>(g, twbank, s, mask, mode); break;
    case 36: launch_shaped<R, 36>(g, twbank, s, mask, mode); break;
    case 40: launch_shaped<R, 40>(g, twbank, s, mask, mode); break;
    case 48: launch_shaped<R, 48>(g, twbank, s, mask, mode); break;
    case 50: launch_shaped<R, 50>(g, twbank, s, mask, mode); break;
    case 54: launch_shaped<R, 54>(g, twbank, s, mask, mode); break;
    case 60: launch_shaped<R, 60>(g, twbank, s, mask, mode); break;
    case 64: launch_shaped<R, 64>(g, twbank, s, mask, mode); break;
    case 72: launch_shaped<R, 72>(g, twbank, s, mask, mode); break;
    case 80: launch_shaped<R, 80>(g, twbank, s, mask, mode); break;
    default: break;
  }
}

// Runtime-shaped pass B of one group (column blocks of TK, the group's
// width; every solve of a group has the same).
template <typename R, int TK, int MODE>
static void launch_passB_runtime(const PassGroup &g, const double *twbank, hipStream_t s) {
  const size_t lds = MODE == MODE_EVAL ? g.ldsB : g.ldsBp;
  if (wide_b<R>(g))
    SKX_TIMED_LAUNCH((k_passB<R, 512, TK, MODE>), dim3(g.gridB), dim3(512), lds, s, g.dev,
                     g.firstB, g.nsolve, g.gridB, twbank);
  else
    SKX_TIMED_LAUNCH((k_passB<R, 256, TK, MODE>), dim3(g.gridB), dim3(256), lds, s, g.dev,
                     g.firstB, g.nsolve, g.gridB, twbank);
}

// The split plane kernels of one group: pass A's z transforms over row-pair
// chunks then its y transforms over column chunks; pass C in the opposite
// order. Both launches of a pass are timed as that pass.
template <typename R, int MODE>
static void launch_split_a(const PassGroup &g, const double *twbank, hipStream_t s) {
  const int kr = MODE == MODE_EVAL ? g.krow : g.krowp;
  const int gr = g.gridC * kr;
  const int gc = g.gridC * (MODE == MODE_EVAL ? NFIELD : 1) * g.kcol;
  SKX_TIMED_LAUNCH((k_passA_rows<R, MODE>), dim3(gr), dim3(SPLIT_NT), g.ldsRow, s, g.dev,
                   g.firstC, g.nsolve, gr, kr, twbank);
  SKX_TIMED_LAUNCH((k_plane_cols<R, MODE, false>), dim3(gc), dim3(SPLIT_NT), g.ldsCol, s, g.dev,
                   g.firstC, g.nsolve, gc, g.kcol, twbank);
}
template <typename R, int MODE>
static void launch_split_c(const PassGroup &g, const double *twbank, hipStream_t s) {
  const int kr = MODE == MODE_EVAL ? g.krow : g.krowp;
  const int gr = g.gridC * kr;
  const int gc = g.gridC * (MODE == MODE_EVAL ? NFIELD : 1) * g.kcol;
  SKX_TIMED_LAUNCH((k_plane_cols<R, MODE, true>), dim3(gc), dim3(SPLIT_NT), g.ldsCol, s, g.dev,
                   g.firstC, g.nsolve, gc, g.kcol, twbank);
  SKX_TIMED_LAUNCH((k_passC_rows<R, MODE>), dim3(gr), dim3(SPLIT_NT), g.ldsRow, s, g.dev,
                   g.firstC, g.nsolve, gr, kr, twbank);
}

// Runtime-shaped (and split) pass kernels over one group, for the passes
// in `mask` (1|16 pass A's transform, 2 pass B, 4 pass C) that the group
// does not run on compile-time-shaped kernels.
template <typename R>
static void launch_eval_runtime(const PassGroup &g, const BatchLaunch &b, hipStream_t s, int mask) {
  constexpr int NTC = 512;
  if (g.gridA > 0 && (mask & 16) && !(g.shape & 1)) {
    if (g.smallA && wide_a(g))
      SKX_TIMED_LAUNCH((k_passA<R, 512, MODE_EVAL>), dim3(g.gridA), dim3(512), g.ldsA, s, g.dev,
                       g.firstA, g.nsolve, g.gridA, b.twbank, b.fd);
    else if (g.smallA)
      SKX_TIMED_LAUNCH((k_passA<R, 256, MODE_EVAL>), dim3(g.gridA), dim3(256), g.ldsA, s, g.dev,
                       g.firstA, g.nsolve, g.gridA, b.twbank, b.fd);
    if (g.bigA) launch_split_a<R, MODE_EVAL>(g, b.twbank, s);
  }
  if (g.gridB > 0 && (mask & 2) && !(g.shape & 2)) {
    switch (g.tk) {
      case 4: launch_passB_runtime<R, 4, MODE_EVAL>(g, b.twbank, s); break;
      case 8: launch_passB_runtime<R, 8, MODE_EVAL>(g, b.twbank, s); break;
      default: launch_passB_runtime<R, 16, MODE_EVAL>(g, b.twbank, s); break;
    }
  }
  if (g.gridC > 0 && (mask & 4) && !(g.shape & 4) && g.smallC) {
    // In FP32 two 512-thread groups share a CU; when the last round of
    // those would be less than half full (e.g. 576 planes), 256-thread
    // groups spread the planes more evenly over the CUs.
    const int fill = g.gridC % (2 * 256);
    if (sizeof(R) == 4 && fill > 0 && fill <= 256) {
      if (g.accC_lds)
        SKX_TIMED_LAUNCH((k_passC<R, 256, true, MODE_EVAL>), dim3(g.gridC), dim3(256), g.ldsC,
                         s, g.dev, g.firstC, g.nsolve, g.gridC, b.twbank, b.fd);
      else
        SKX_TIMED_LAUNCH((k_passC<R, 256, false, MODE_EVAL>), dim3(g.gridC), dim3(256), g.ldsC,
                         s, g.dev, g.firstC, g.nsolve, g.gridC, b.twbank, b.fd);
    } else if (g.accC_lds) {
      SKX_TIMED_LAUNCH((k_passC<R, NTC, true, MODE_EVAL>), dim3(g.gridC), dim3(NTC), g.ldsC, s,
                       g.dev, g.firstC, g.nsolve, g.gridC, b.twbank, b.fd);
    } else {
      SKX_TIMED_LAUNCH((k_passC<R, NTC, false, MODE_EVAL>), dim3(g.gridC), dim3(NTC), g.ldsC,
                       s, g.dev, g.firstC, g.nsolve, g.gridC, b.twbank, b.fd);
    }
  }
  if (g.gridC > 0 && (mask & 4) && !(g.shape & 4) && g.bigC)
    launch_split_c<R, MODE_EVAL>(g, b.twbank, s);
}

template <typename R>
static hipError_t launch_eval_t(const BatchLaunch &b, hipStream_t s, int mask) {
  // mask: 1 pass A (pointwise kernel and transform), 2 pass B, 4 pass C,
  // 8 the pointwise kernel alone, 16 pass A's transform alone
  if (mask & 1) mask |= 8 | 16;
  if (b.gridV > 0 && (mask & 8))
    SKX_TIMED_LAUNCH((k_point<R, 256>), dim3(b.gridV), dim3(256), 256 * sizeof(double), s, b.dev,
                     b.firstV, b.nsolve, b.gridV, b.fd);
  // pass by pass over the groups (each pass of every group before the next
  // pass starts)
  for (const int pm : {16, 2, 4}) {
    if (!(mask & pm)) continue;
    for (int gi = 0; gi < b.ngroup; ++gi) {
      const PassGroup &g = b.grp[gi];
      if (g.shapeN) launch_shaped_n<R>(g, b.twbank, s, pm, MODE_EVAL);
      launch_eval_runtime<R>(g, b, s, pm);
    }
  }
  return hipGetLastError();
}

template <typename R>
static hipError_t launch_prec_t(const BatchLaunch &b, hipStream_t s, int mask) {
  for (const int pm : {1, 2, 4}) {
    if (!(mask & pm)) continue;
    for (int gi = 0; gi < b.ngroup; ++gi) {
      const PassGroup &g = b.grp[gi];
      if (g.shapeN) launch_shaped_n<R>(g, b.twbank, s, pm, MODE_PREC);
      // one field per solve: pass A has one workgroup per plane, like pass C
      if (g.gridC > 0 && (pm & 1) && !(g.shape & 1)) {
        if (g.smallA && wide_a(g))
          SKX_TIMED_LAUNCH((k_passA<R, 512, MODE_PREC>), dim3(g.gridC), dim3(512), g.ldsA, s,
                           g.dev, g.firstC, g.nsolve, g.gridC, b.twbank, b.fd);
        else if (g.smallA)
          SKX_TIMED_LAUNCH((k_passA<R, 256, MODE_PREC>), dim3(g.gridC), dim3(256), g.ldsA, s,
                           g.dev, g.firstC, g.nsolve, g.gridC, b.twbank, b.fd);
        if (g.bigA) launch_split_a<R, MODE_PREC>(g, b.twbank, s);
      }
      if (g.gridB > 0 && (pm & 2) && !(g.shape & 2)) {
        switch (g.tk) {
          case 4: launch_passB_runtime<R, 4, MODE_PREC>(g, b.twbank, s); break;
          case 8: launch_passB_runtime<R, 8, MODE_PREC>(g, b.twbank, s); break;
          default: launch_passB_runtime<R, 16, MODE_PREC>(g, b.twbank, s); break;
        }
      }
      if (g.gridC > 0 && (pm & 4) && !(g.shape & 4) && g.smallC)
        SKX_TIMED_LAUNCH((k_passC<R, 512, false, MODE_PREC>), dim3(g.gridC), dim3(512), g.ldsC, s,
                         g.dev, g.firstC, g.nsolve, g.gridC, b.twbank, b.fd);
      if (g.gridC > 0 && (pm & 4) && !(g.shape & 4) && g.bigC)
        launch_split_c<R, MODE_PREC>(g, b.twbank, s);
    }
  }
  return hipGetLastError();
}

hipError_t launch_eval(const BatchLaunch &b, hipStream_t s, int mask) {
  return b.prec == 0 ? launch_eval_t<double>(b, s, mask) : launch_eval_t<float>(b, s, mask);
}

hipError_t launch_prec(const BatchLaunch &b, hipStream_t s, int mask) {
  return b.prec == 0 ? launch_prec_t<double>(b, s, mask) : launch_prec_t<float>(b, s, mask);
}

}  // namespace skx
