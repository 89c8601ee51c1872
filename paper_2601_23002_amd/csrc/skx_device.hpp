// Device-side building blocks of libskx: complex arithmetic, the LDS
// Stockham FFT, the Fermi-Dirac table lookup, Perdew-Zunger LDA, workgroup
// reductions and the workgroup-to-work-item mapping.
#pragma once

#include "skx_internal.hpp"
#include <type_traits>

namespace skx {

// Pointers read from descriptors are generic (flat) pointers; the fields
// they name live in global memory. Qualifying them lets the compiler issue
// global loads that do not alias LDS, so loads can be batched ahead of LDS
// stores.
#define SKX_G __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ SKX_G T *gptr(const void *p) {
  return (SKX_G T *)(void *)(p);
}

// Per-solve control state is read-only in the grid-wide kernels; reading it
// through the constant address space turns every field into a scalar load,
// and the branches on it into uniform branches.
#define SKX_C __attribute__((address_space(4)))
template <typename T> __device__ __forceinline__ const SKX_C T *cptr(const void *p) {
  return (const SKX_C T *)(p);
}

// HIP's vector structs cannot be copied through address-space-qualified
// pointers; move them as clang native vectors instead.
template <typename V> struct NativeOf;
template <> struct NativeOf<double2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct NativeOf<float2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct NativeOf<double4> { typedef double T __attribute__((ext_vector_type(4))); };
template <typename V> __device__ __forceinline__ V ldg(const SKX_G V *p) {
  typedef typename NativeOf<V>::T N;
  const N v = *reinterpret_cast<const SKX_G N *>(p);
  V r;
  __builtin_memcpy(&r, &v, sizeof(V));
  return r;
}
template <typename V> __device__ __forceinline__ void stg(SKX_G V *p, const V &v) {
  typedef typename NativeOf<V>::T N;
  N w;
  __builtin_memcpy(&w, &v, sizeof(V));
  *reinterpret_cast<SKX_G N *>(p) = w;
}

// An empty asm that "redefines" a lane index: index arithmetic after it
// cannot be hoisted out of enclosing loops, where it would stay live in
// registers for the whole kernel and cut the occupancy.
#define SKX_OPAQUE(x) asm volatile("" : "+v"(x))

template <typename R> struct Vec2;
template <> struct Vec2<double> { typedef double2 T; };
template <> struct Vec2<float> { typedef float2 T; };

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
  V r; r.x = a.x * b.x + a.y * b.y; r.y = a.y * b.x - a.x * b.y; return r;
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) {
  V r; r.x = a.x * s; r.y = a.y * s; return r;
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V> __device__ __forceinline__ V cmul_mi(V a) {
  V r;
  if (INV) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
  return r;
}

// ---------------------------------------------------------------------------
// Small DFTs in registers. Forward kernel exp(-2 pi i jk/R), inverse +.
// ---------------------------------------------------------------------------
template <int RAD, bool INV, typename V> struct Bfly;

template <bool INV, typename V> struct Bfly<2, INV, V> {
  __device__ __forceinline__ static void run(V *v) {
    V a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  }
};

template <bool INV, typename V> struct Bfly<3, INV, V> {
  __device__ __forceinline__ static void run(V *v) {
    typedef decltype(v[0].x) R;
    const R S3 = (R)0.86602540378443864676;   // sin(2 pi / 3)
    V a = v[0], b = v[1], c = v[2];
    V t1 = cadd(b, c);
    V t2; t2.x = a.x - (R)0.5 * t1.x; t2.y = a.y - (R)0.5 * t1.y;
    V d = csub(b, c);
    // forward: X1 = t2 - i s d, X2 = t2 + i s d
    V sd = cmul_mi<INV>(cscale(d, S3));
    v[0] = cadd(a, t1);
    v[1] = cadd(t2, sd);
    v[2] = csub(t2, sd);
  }
};

template <bool INV, typename V> struct Bfly<4, INV, V> {
  __device__ __forceinline__ static void run(V *v) {
    V a = v[0], b = v[1], c = v[2], d = v[3];
    V s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d);
    V s3 = cmul_mi<INV>(csub(b, d));
    v[0] = cadd(s0, s2);
    v[1] = cadd(s1, s3);
    v[2] = csub(s0, s2);
    v[3] = csub(s1, s3);
  }
};

// Radix 8 as two radix-4 DFTs of the even and odd points combined with the
// eighth roots of unity (forward w = (1 - i)/sqrt2, inverse its conjugate).
template <bool INV, typename V> struct Bfly<8, INV, V> {
  __device__ __forceinline__ static void run(V *v) {
    typedef decltype(v[0].x) R;
    const R H = (R)0.70710678118654752440;     // 1/sqrt(2)
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<4, INV, V>::run(e);
    Bfly<4, INV, V>::run(o);
    V t1, t2, t3;
    if (!INV) {
      t1.x = H * (o[1].x + o[1].y); t1.y = H * (o[1].y - o[1].x);
      t3.x = H * (o[3].y - o[3].x); t3.y = -H * (o[3].x + o[3].y);
    } else {
      t1.x = H * (o[1].x - o[1].y); t1.y = H * (o[1].x + o[1].y);
      t3.x = -H * (o[3].x + o[3].y); t3.y = H * (o[3].x - o[3].y);
    }
    t2 = cmul_mi<INV>(o[2]);
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], t1);   v[5] = csub(e[1], t1);
    v[2] = cadd(e[2], t2);   v[6] = csub(e[2], t2);
    v[3] = cadd(e[3], t3);   v[7] = csub(e[3], t3);
  }
};

template <bool INV, typename V> struct Bfly<5, INV, V> {
  __device__ __forceinline__ static void run(V *v) {
    typedef decltype(v[0].x) R;
    const R C1 = (R)0.30901699437494742410;    // cos(2 pi/5)
    const R C2 = (R)-0.80901699437494742410;   // cos(4 pi/5)
    const R S1 = (R)0.95105651629515357212;    // sin(2 pi/5)
    const R S2 = (R)0.58778525229247312917;    // sin(4 pi/5)
    V x0 = v[0];
    V t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    V t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    V a1; a1.x = x0.x + C1 * t1.x + C2 * t2.x; a1.y = x0.y + C1 * t1.y + C2 * t2.y;
    V a2; a2.x = x0.x + C2 * t1.x + C1 * t2.x; a2.y = x0.y + C2 * t1.y + C1 * t2.y;
    V b1; b1.x = S1 * t3.x + S2 * t4.x; b1.y = S1 * t3.y + S2 * t4.y;
    V b2; b2.x = S2 * t3.x - S1 * t4.x; b2.y = S2 * t3.y - S1 * t4.y;
    V m1 = cmul_mi<INV>(b1), m2 = cmul_mi<INV>(b2);
    v[0] = cadd(x0, cadd(t1, t2));
    v[1] = cadd(a1, m1);
    v[4] = csub(a1, m1);
    v[2] = cadd(a2, m2);
    v[3] = csub(a2, m2);
  }
};

// ---------------------------------------------------------------------------
// Division by a workgroup-uniform divisor d <= 2^16 for x < 2^16:
// q = floor(x * ceil(2^32/d) / 2^32) is exact in that range (the rounding
// term is below 2^-16 <= 1/d), and costs one 32x64 multiply.
// ---------------------------------------------------------------------------
struct UDiv {
  unsigned d;
  unsigned long long m;
};
// ceil(2^32/d) = floor((2^32 - 1)/d) + 1 for d >= 1: one 32-bit division
// (a 64-bit integer division would cost ~100 scalar instructions per call).
__device__ __forceinline__ UDiv make_udiv(unsigned d) {
  UDiv r;
  r.d = d;
  r.m = (unsigned long long)(0xFFFFFFFFu / d) + 1ull;
  return r;
}
__device__ __forceinline__ unsigned udiv(unsigned x, const UDiv &v) {
  return (unsigned)(((unsigned long long)x * v.m) >> 32);
}

// ---------------------------------------------------------------------------
// One Stockham stage over `count` transforms of length N held in LDS.
// Element e of transform t sits at buf[t*ts + e*es]. Butterflies are staged
// in registers: every thread first reads all of its butterflies of a group
// of whole transforms, the workgroup synchronises, then every thread writes
// its results, so the stage runs in place. tw[k] = exp(-2 pi i k / N).
// ---------------------------------------------------------------------------
template <typename V, int RAD, int MAXB, bool INV>
__device__ __forceinline__ void fft_stage(V *buf, int N, int Ns, int twstep,
                                          unsigned long long m_nb, unsigned long long m_ns,
                                          int count, int es, int ts, const V *tw, int tid,
                                          int nthr) {
  const int nb = N / RAD;
  const UDiv dnb{(unsigned)nb, m_nb}, dns{(unsigned)Ns, m_ns};
  SKX_OPAQUE(tid);
  int per = (int)udiv((unsigned)(MAXB * nthr), dnb);
  if (per < 1) per = 1;
#pragma unroll 1
  for (int t0 = 0; t0 < count; t0 += per) {
    const int t1 = (t0 + per < count) ? t0 + per : count;
    const int gtot = (t1 - t0) * nb;
    V v[MAXB][RAD];
    int tq[MAXB], jq[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int b = tid + i * nthr;
      const int q = (int)udiv((unsigned)b, dnb);
      tq[i] = t0 + q;
      jq[i] = b - q * nb;
      if (b < gtot) {
        const V *base = buf + tq[i] * ts + jq[i] * es;
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[i][r] = base[r * nb * es];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int b = tid + i * nthr;
      if (b < gtot) {
        const int j = jq[i];
        const int k = j - (int)udiv((unsigned)j, dns) * Ns;
        if (Ns > 1) {
#pragma unroll
          for (int r = 1; r < RAD; ++r) {
            const V w = tw[k * r * twstep];
            v[i][r] = INV ? cmulc(v[i][r], w) : cmul(v[i][r], w);
          }
        }
        Bfly<RAD, INV, V>::run(v[i]);
        V *out = buf + tq[i] * ts + ((j - k) * RAD + k) * es;
#pragma unroll
        for (int r = 0; r < RAD; ++r) out[r * Ns * es] = v[i][r];
      }
    }
    __syncthreads();
  }
}

// Full transform of `count` sequences of length pl.n (plan radices in
// order; the per-stage division constants come precomputed in the plan).
template <typename V, int MAXB, bool INV>
__device__ __forceinline__ void fft_lds(V *buf, const Plan &pl, int count, int es, int ts,
                                        const V *tw, int tid, int nthr) {
  SKX_OPAQUE(tid);
  const int n = pl.n, nst = pl.nst;
  const unsigned code = pl.rad;
  int Ns = 1;
#pragma unroll 1
  for (int s = 0; s < nst; ++s) {
    const int rad = (code >> (4 * s)) & 15u;
    const int tws = pl.twstep[s];
    const unsigned long long mb = pl.m_nb[s], ms = pl.m_ns[s];
    switch (rad) {
      case 8: fft_stage<V, 8, (MAXB + 1) / 2, INV>(buf, n, Ns, tws, mb, ms, count, es, ts, tw, tid, nthr); break;
      case 4: fft_stage<V, 4, MAXB, INV>(buf, n, Ns, tws, mb, ms, count, es, ts, tw, tid, nthr); break;
      case 2: fft_stage<V, 2, MAXB, INV>(buf, n, Ns, tws, mb, ms, count, es, ts, tw, tid, nthr); break;
      case 3: fft_stage<V, 3, MAXB, INV>(buf, n, Ns, tws, mb, ms, count, es, ts, tw, tid, nthr); break;
      default: fft_stage<V, 5, MAXB, INV>(buf, n, Ns, tws, mb, ms, count, es, ts, tw, tid, nthr); break;
    }
    Ns *= rad;
  }
}

// ---------------------------------------------------------------------------
// Wavefront-owned transforms. When every transform of a call is read and
// written by one wavefront only, a stage needs no workgroup barrier: the LDS
// operations of a wavefront execute in order, so each lane's reads of a
// stage precede every write of that stage (all butterflies of the stage are
// held in registers first), and the next stage's reads follow them. The
// compiler keeps that order through a wavefront-scope fence between the
// halves (no instruction: a wavefront's LDS operations are already ordered).
// ---------------------------------------------------------------------------
#define SKX_WAVE_SYNC()                                   \
  do {                                                    \
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                      \
  } while (0)

// tfast: consecutive lanes take consecutive transforms (for transforms that
// are adjacent in memory, ts = 1: their elements then sit in consecutive
// LDS words instead of one row pitch apart, which avoids bank conflicts);
// otherwise consecutive butterflies of one transform.
template <typename V, int RAD, int MB, bool INV>
__device__ __forceinline__ void fft_stage_w(V *buf, int N, int Ns, int twstep,
                                            unsigned long long m_nb, unsigned long long m_ns,
                                            int t0, int ntr, const UDiv &dntr, bool tfast,
                                            int es, int ts, const V *tw, int lane) {
  const int nb = N / RAD;
  const UDiv dnb{(unsigned)nb, m_nb}, dns{(unsigned)Ns, m_ns};
  const int tot = ntr * nb;
  V v[MB][RAD];
  int tq[MB], jq[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = lane + 64 * i;
    if (tfast) {
      const int q = (int)udiv((unsigned)b, dntr);
      tq[i] = t0 + (b - q * ntr);
      jq[i] = q;
    } else {
      const int q = (int)udiv((unsigned)b, dnb);
      tq[i] = t0 + q;
      jq[i] = b - q * nb;
    }
    if (b < tot) {
      const V *base = buf + tq[i] * ts + jq[i] * es;
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[i][r] = base[r * nb * es];
    }
  }
  SKX_WAVE_SYNC();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = lane + 64 * i;
    if (b < tot) {
      const int j = jq[i];
      const int k = j - (int)udiv((unsigned)j, dns) * Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          const V w = tw[k * r * twstep];
          v[i][r] = INV ? cmulc(v[i][r], w) : cmul(v[i][r], w);
        }
      }
      Bfly<RAD, INV, V>::run(v[i]);
      V *out = buf + tq[i] * ts + ((j - k) * RAD + k) * es;
#pragma unroll
      for (int r = 0; r < RAD; ++r) out[r * Ns * es] = v[i][r];
    }
  }
  SKX_WAVE_SYNC();
}

// Can a wavefront hold ntr transforms of this plan in registers, at most
// MAXV complex values per lane in every stage? (Workgroup-uniform.)
template <int MAXV>
__device__ __forceinline__ bool wave_fits(const Plan &pl, int ntr) {
  for (int s = 0; s < pl.nst; ++s) {
    const int rad = (pl.rad >> (4 * s)) & 15u;
    if (ntr * (pl.n / rad) > 64 * (MAXV / rad)) return false;
  }
  return true;
}

// The transforms [t0, t0 + ntr) of this wavefront, every stage in place.
template <typename V, int MAXV, bool INV>
__device__ __forceinline__ void fft_lds_w(V *buf, const Plan &pl, int t0, int ntr, int es, int ts,
                                          const V *tw, int lane) {
  SKX_OPAQUE(lane);
  const int n = pl.n, nst = pl.nst;
  const unsigned code = pl.rad;
  if (ntr <= 0) return;
  const UDiv dntr = make_udiv((unsigned)ntr);
  const bool tf = ts == 1 && es != 1;
  int Ns = 1;
#pragma unroll 1
  for (int s = 0; s < nst; ++s) {
    const int rad = (code >> (4 * s)) & 15u;
    const int tws = pl.twstep[s];
    const unsigned long long mb = pl.m_nb[s], ms = pl.m_ns[s];
    switch (rad) {
      case 8: fft_stage_w<V, 8, MAXV / 8, INV>(buf, n, Ns, tws, mb, ms, t0, ntr, dntr, tf, es, ts, tw, lane); break;
      case 4: fft_stage_w<V, 4, MAXV / 4, INV>(buf, n, Ns, tws, mb, ms, t0, ntr, dntr, tf, es, ts, tw, lane); break;
      case 2: fft_stage_w<V, 2, MAXV / 2, INV>(buf, n, Ns, tws, mb, ms, t0, ntr, dntr, tf, es, ts, tw, lane); break;
      case 3: fft_stage_w<V, 3, MAXV / 3, INV>(buf, n, Ns, tws, mb, ms, t0, ntr, dntr, tf, es, ts, tw, lane); break;
      default: fft_stage_w<V, 5, MAXV / 5, INV>(buf, n, Ns, tws, mb, ms, t0, ntr, dntr, tf, es, ts, tw, lane); break;
    }
    Ns *= rad;
  }
}

// Transforms [lo, hi) of `count` owned by wavefront w of nw.
__device__ __forceinline__ void wave_share(int count, int w, int nw, int &lo, int &hi) {
  lo = (count * w) / nw;
  hi = (count * (w + 1)) / nw;
}

// ---------------------------------------------------------------------------
// Wavefront-owned transforms whose length, radix order and storage are fixed
// at compile time, so every index is a constant or a shift. The wavefront
// owns SLOTS transforms starting at buf (element e of transform t at
// buf[t*TS + e*ES]); lanes take consecutive transforms (TFAST) or
// consecutive butterflies of one transform, one or more butterflies each.
// Same Stockham stage as fft_stage_w: all reads of the stage before any
// write, tw[k] = exp(-2 pi i k / N).
// ---------------------------------------------------------------------------
template <int N, int RAD, int SLOTS, bool TFAST> struct CMap {
  static constexpr int NB = N / RAD;               // butterflies per transform
  static constexpr int TOT = SLOTS * NB;
  static constexpr int MB = (TOT + 63) / 64;       // butterflies per lane
  __device__ __forceinline__ static int t(int b) { return TFAST ? b % SLOTS : b / NB; }
  __device__ __forceinline__ static int j(int b) { return TFAST ? b / SLOTS : b % NB; }
  __device__ __forceinline__ static bool ok(int b) { return TOT % 64 == 0 || b < TOT; }
};

// Twiddle and butterfly of one radix-RAD group whose inputs are in v.
template <typename V, int N, int RAD, int NS, bool INV>
__device__ __forceinline__ void cbfly(V (&v)[RAD], int k, const V *tw) {
  if (NS > 1) {
    constexpr int TWS = N / (NS * RAD);
#pragma unroll
    for (int r = 1; r < RAD; ++r) {
      const V w = tw[k * r * TWS];
      v[r] = INV ? cmulc(v[r], w) : cmul(v[r], w);
    }
  }
  Bfly<RAD, INV, V>::run(v);
}

template <typename V, int N, int RAD, int NS, int ES, int TS, int SLOTS, bool TFAST, bool INV>
__device__ __forceinline__ void cstage(V *buf, const V *tw, int lane) {
  typedef CMap<N, RAD, SLOTS, TFAST> M;
  V v[M::MB][RAD];
#pragma unroll
  for (int i = 0; i < M::MB; ++i) {
    const int b = lane + 64 * i;
    if (M::ok(b)) {
      const V *base = buf + M::t(b) * TS + M::j(b) * ES;
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[i][r] = base[r * M::NB * ES];
    }
  }
  SKX_WAVE_SYNC();
#pragma unroll
  for (int i = 0; i < M::MB; ++i) {
    const int b = lane + 64 * i;
    if (M::ok(b)) {
      const int j = M::j(b), k = j % NS;
      cbfly<V, N, RAD, NS, INV>(v[i], k, tw);
      V *out = buf + M::t(b) * TS + ((j - k) * RAD + k) * ES;
#pragma unroll
      for (int r = 0; r < RAD; ++r) out[r * NS * ES] = v[i][r];
    }
  }
  SKX_WAVE_SYNC();
}

// Stages of the radix list RS... starting at span NS.
template <typename V, int N, int NS, int ES, int TS, int SLOTS, bool TFAST, bool INV>
__device__ __forceinline__ void cstages(V *, const V *, int) {}
template <typename V, int N, int NS, int ES, int TS, int SLOTS, bool TFAST, bool INV, int R0,
          int... RS>
__device__ __forceinline__ void cstages(V *buf, const V *tw, int lane) {
  cstage<V, N, R0, NS, ES, TS, SLOTS, TFAST, INV>(buf, tw, lane);
  cstages<V, N, NS * R0, ES, TS, SLOTS, TFAST, INV, RS...>(buf, tw, lane);
}

// Compile-time radix lists and the operations the shaped kernels need on
// them: first, last, all but the first, all but the last, and running the
// stages of a list from a given span.
template <int... Rs> struct RList {};
template <typename L> struct RFirst;
template <int R0, int... Rs> struct RFirst<RList<R0, Rs...>> { static constexpr int value = R0; };
template <typename L> struct RLast;
template <int R0> struct RLast<RList<R0>> { static constexpr int value = R0; };
template <int R0, int R1, int... Rs>
struct RLast<RList<R0, R1, Rs...>> { static constexpr int value = RLast<RList<R1, Rs...>>::value; };
template <typename L> struct RRest;
template <int R0, int... Rs> struct RRest<RList<R0, Rs...>> { typedef RList<Rs...> T; };
template <int R, typename L> struct RPrepend;
template <int R, int... Rs> struct RPrepend<R, RList<Rs...>> { typedef RList<R, Rs...> T; };
template <typename L> struct RInit;
template <int R0> struct RInit<RList<R0>> { typedef RList<> T; };
template <int R0, int R1, int... Rs> struct RInit<RList<R0, R1, Rs...>> {
  typedef typename RPrepend<R0, typename RInit<RList<R1, Rs...>>::T>::T T;
};
template <typename L> struct RProd;
template <> struct RProd<RList<>> { static constexpr int value = 1; };
template <int R0, int... Rs> struct RProd<RList<R0, Rs...>> {
  static constexpr int value = R0 * RProd<RList<Rs...>>::value;
};
template <typename L> struct CStages;
template <int... Rs> struct CStages<RList<Rs...>> {
  template <typename V, int N, int NS, int ES, int TS, int SLOTS, bool TFAST, bool INV>
  __device__ __forceinline__ static void run(V *buf, const V *tw, int lane) {
    cstages<V, N, NS, ES, TS, SLOTS, TFAST, INV, Rs...>(buf, tw, lane);
  }
};

// Cubic grids with compile-time-shaped kernels. Per length N:
//   L   radix order (the same along x, y and z). The first radix is even:
//       the real transforms fold their Nyquist terms into the first stage.
//   NW  wavefronts per workgroup of passes A and C; they split the N/2 row
//       pairs (z transforms) and the N/2 columns (y transforms) evenly.
//   PL  LDS row pitch (complex values) of a half-spectrum plane,
//       >= N/2 + 1; N/2 + 4 spreads the column transforms (adjacent
//       columns of rows one pitch apart) and the row-pair transforms over
//       the LDS banks.
//   CW  waves per SIMD pass C's launch bound asks for: as many as its
//       register-resident dE/dphi (N^2 / (64 NW) points per lane) allows
//       without spilling.
// 64 holds the scan workload; 36-80 are the grids of the thermal
// ensemble (h = 0.25 bohr) and of the smaller serving requests.
template <int N> struct CShape;
template <> struct CShape<36> { typedef RList<4, 3, 3> L; static constexpr int NW = 3, PL = 22, CW = 3; };
template <> struct CShape<40> { typedef RList<8, 5> L; static constexpr int NW = 4, PL = 24, CW = 3; };
template <> struct CShape<48> { typedef RList<8, 3, 2> L; static constexpr int NW = 4, PL = 28, CW = 3; };
template <> struct CShape<50> { typedef RList<2, 5, 5> L; static constexpr int NW = 5, PL = 29, CW = 3; };
template <> struct CShape<54> { typedef RList<2, 3, 3, 3> L; static constexpr int NW = 3, PL = 31, CW = 2; };
template <> struct CShape<60> { typedef RList<4, 3, 5> L; static constexpr int NW = 6, PL = 34, CW = 2; };
template <> struct CShape<64> { typedef RList<8, 8> L; static constexpr int NW = 4, PL = 36, CW = 3; };
template <> struct CShape<72> { typedef RList<8, 3, 3> L; static constexpr int NW = 6, PL = 40, CW = 2; };
template <> struct CShape<80> { typedef RList<8, 5, 2> L; static constexpr int NW = 8, PL = 44, CW = 1; };
// Larger serving lengths: pass B only (passes A and C run on the in-LDS
// runtime-shaped or the split kernels); NW, PL and CW only satisfy the
// checks below.
template <> struct CShape<90> { typedef RList<2, 5, 3, 3> L; static constexpr int NW = 3, PL = 49, CW = 1; };
template <> struct CShape<96> { typedef RList<8, 4, 3> L; static constexpr int NW = 4, PL = 52, CW = 1; };
template <> struct CShape<100> { typedef RList<4, 5, 5> L; static constexpr int NW = 5, PL = 54, CW = 1; };
template <> struct CShape<108> { typedef RList<4, 3, 3, 3> L; static constexpr int NW = 3, PL = 58, CW = 1; };
template <> struct CShape<120> { typedef RList<8, 5, 3> L; static constexpr int NW = 4, PL = 64, CW = 1; };
template <> struct CShape<128> { typedef RList<8, 4, 4> L; static constexpr int NW = 4, PL = 68, CW = 1; };
template <> struct CShape<144> { typedef RList<4, 4, 3, 3> L; static constexpr int NW = 4, PL = 76, CW = 1; };
template <> struct CShape<150> { typedef RList<2, 5, 5, 3> L; static constexpr int NW = 5, PL = 79, CW = 1; };
template <> struct CShape<160> { typedef RList<8, 4, 5> L; static constexpr int NW = 4, PL = 84, CW = 1; };
template <> struct CShape<162> { typedef RList<2, 3, 3, 3, 3> L; static constexpr int NW = 3, PL = 85, CW = 1; };
template <> struct CShape<180> { typedef RList<4, 5, 3, 3> L; static constexpr int NW = 6, PL = 94, CW = 1; };
template <> struct CShape<192> { typedef RList<8, 8, 3> L; static constexpr int NW = 4, PL = 100, CW = 1; };
// derived per-length constants
template <int N> struct CS {
  typedef typename CShape<N>::L L;
  static constexpr int NW = CShape<N>::NW, NT = 64 * NW, PL = CShape<N>::PL, C = N / 2;
  static constexpr int CW = CShape<N>::CW;
  static constexpr int R0 = RFirst<L>::value;      // first stage
  static constexpr int RL = RLast<L>::value;       // last stage
  static constexpr int NSL = N / RL;               // span of the last stage
  typedef typename RRest<L>::T Rest;               // stages after the first
  typedef typename RInit<L>::T Init;               // stages before the last
  typedef typename RInit<Rest>::T Mid;             // stages between first and last
  static constexpr int ZP = N / 2 / NW;            // row pairs per wavefront
  static constexpr int YC = C / NW;                // y columns per wavefront
  static_assert(RProd<L>::value == N, "radix order must multiply to N");
  static_assert(R0 % 2 == 0, "even first radix");
  static_assert(ZP * NW * 2 == N && YC * NW == C, "even split over the wavefronts");
  static_assert(PL >= C + 1 && 2 * PL >= N, "LDS row pitch");
  // LDS of passes A and C: the plane and both twiddle tables
  static constexpr size_t lds_plane(size_t v) { return v * (size_t)(N * PL + 2 * N); }
};

// ---------------------------------------------------------------------------
// Universal Fermi-Dirac table: eta and psi = f_TF / (n T) as functions of
// y = ln(n / n_T), by quintic Hermite interpolation between nodes that store
// eta, eta', eta'' and psi (psi' = eta - psi and psi'' = eta' - eta + psi
// follow from d(u psi)/du = eta). One lookup reads 64 contiguous bytes.
// Below the table the non-degenerate limit is exact to double precision;
// above it the value is clamped and flagged.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fd_lookup(double y, const FDTable &fd, double &eta, double &psi) {
  const double LN_G32 = -0.12078223763524522;    // ln Gamma(3/2)
  double t = (y - fd.y0) * fd.inv_h;
  if (t < 0.0) { eta = y - LN_G32; psi = eta - 1.0; return 0; }
  int k = (int)t;
  int bad = 0;
  if (k >= fd.n) { k = fd.n - 1; bad = 1; }
  const double s = t - k;
  const double4 a = ldg(gptr<double4>(fd.node) + k);
  const double4 b = ldg(gptr<double4>(fd.node) + k + 1);
  const double h = fd.h;
  const double s2 = s * s, s3 = s2 * s, s4 = s3 * s, s5 = s4 * s;
  const double h0 = 1.0 - 10.0 * s3 + 15.0 * s4 - 6.0 * s5;
  const double h1 = s - 6.0 * s3 + 8.0 * s4 - 3.0 * s5;
  const double h2 = 0.5 * s2 - 1.5 * s3 + 1.5 * s4 - 0.5 * s5;
  const double h3 = 10.0 * s3 - 15.0 * s4 + 6.0 * s5;
  const double h4 = -4.0 * s3 + 7.0 * s4 - 3.0 * s5;
  const double h5 = 0.5 * s3 - s4 + 0.5 * s5;
  eta = a.x * h0 + h * (a.y * h1 + h * a.z * h2) + b.x * h3 + h * (b.y * h4 + h * b.z * h5);
  const double pa1 = a.x - a.w, pa2 = a.y - a.x + a.w;
  const double pb1 = b.x - b.w, pb2 = b.y - b.x + b.w;
  psi = a.w * h0 + h * (pa1 * h1 + h * pa2 * h2) + b.w * h3 + h * (pb1 * h4 + h * pb2 * h5);
  return bad;
}

// Perdew-Zunger 1981 LDA (spin-unpolarised): energy per electron and
// potential, from x = ln n (rs = (3/(4 pi))^(1/3) exp(-x/3)). The paper uses
// PZ LDA in the adiabatic approximation. Two variants (uniform per solve):
//   join = false  the published fit: dilute branch for rs >= 1, dense branch
//                 below; the branches jump by ~3e-5 Ha at rs = 1;
//   join = true   the branches joined C1 over 0.99 <= rs <= 1.01 with
//                 w = 3t^2 - 2t^3, t = (rs - 0.99)/0.02,
//                 e_c = (1 - w) e_dense + w e_dilute, v_c the exact potential
//                 of that e_c: v_c = e_c - (rs/3) de_c/drs.
template <typename T> struct PZ {
  static constexpr T G = (T)-0.1423, B1 = (T)1.0529, B2 = (T)0.3334;
  static constexpr T A = (T)0.0311, B = (T)-0.048, C = (T)0.0020, D = (T)-0.0116;
  static constexpr T LO = (T)0.99, HI = (T)1.01;
};

// dilute branch: e_c and de_c/drs from rs and sqrt(rs) and 1/den
template <typename T>
__device__ __forceinline__ void pz_dilute(T rs, T sq, T iden, T &e, T &de) {
  e = PZ<T>::G * iden;
  de = -PZ<T>::G * ((T)0.5 * PZ<T>::B1 / sq + PZ<T>::B2) * iden * iden;
}
// dense branch: e_c and de_c/drs from rs and ln rs
template <typename T>
__device__ __forceinline__ void pz_dense(T rs, T lr, T irs, T &e, T &de) {
  e = PZ<T>::A * lr + PZ<T>::B + PZ<T>::C * rs * lr + PZ<T>::D * rs;
  de = PZ<T>::A * irs + PZ<T>::C * lr + PZ<T>::C + PZ<T>::D;
}

// (e3 = n^(1/3) = exp(x/3) and ie3 = 1/e3, computed by the caller)
__device__ __forceinline__ void pz81_ln_e3(double x, double e3, double ie3, bool join,
                                           double &eps, double &v) {
  const double RS1 = 0.62035049089940001667;   // (3/(4 pi))^(1/3)
  const double LNRS1 = -0.47747065276706024;  // ln RS1
  const double CX = 0.45816529328314287;      // (3/(4 pi)) (9 pi / 4)^(1/3)
  const double rs = RS1 * ie3;
  const double ex = -CX / RS1 * e3;
  const double hi = join ? PZ<double>::HI : 1.0;
  const double lo = join ? PZ<double>::LO : 1.0;
  double ec, dec;
  if (rs >= hi) {
    const double sq = sqrt(rs);
    pz_dilute(rs, sq, 1.0 / (1.0 + PZ<double>::B1 * sq + PZ<double>::B2 * rs), ec, dec);
  } else if (rs <= lo) {
    pz_dense(rs, LNRS1 - x * (1.0 / 3.0), e3 * (1.0 / RS1), ec, dec);
  } else {
    double e1, d1, e2, d2;
    pz_dense(rs, LNRS1 - x * (1.0 / 3.0), e3 * (1.0 / RS1), e1, d1);
    const double sq = sqrt(rs);
    pz_dilute(rs, sq, 1.0 / (1.0 + PZ<double>::B1 * sq + PZ<double>::B2 * rs), e2, d2);
    const double t = (rs - PZ<double>::LO) / (PZ<double>::HI - PZ<double>::LO);
    const double w = t * t * (3.0 - 2.0 * t);
    const double dw = 6.0 * t * (1.0 - t) / (PZ<double>::HI - PZ<double>::LO);
    ec = (1.0 - w) * e1 + w * e2;
    dec = (1.0 - w) * d1 + w * d2 + dw * (e2 - e1);
  }
  eps = ex + ec;
  v = (4.0 / 3.0) * ex + ec - rs * (1.0 / 3.0) * dec;
}

__device__ __forceinline__ void pz81_ln(double x, bool join, double &eps, double &v) {
  const double e3 = exp(x * (1.0 / 3.0));
  pz81_ln_e3(x, e3, 1.0 / e3, join, eps, v);
}

// Single-precision PZ81 for the FP32 evaluations (the exchange-correlation
// potential then carries FP32 rounding like every other FP32 field; the
// FP64 refinement uses pz81_ln). Hardware exp2 / reciprocal / square root.
__device__ __forceinline__ void pz81_lnf(float x, bool join, float &eps, float &v) {
  const float RS1 = 0.62035049089940001667f;   // (3/(4 pi))^(1/3)
  const float LNRS1 = -0.47747065276706024f;  // ln RS1
  const float CX = 0.45816529328314287f;       // (3/(4 pi)) (9 pi / 4)^(1/3)
  const float L2E3 = 0.48089834696298783f;     // log2(e) / 3
  const float e3 = __builtin_amdgcn_exp2f(x * L2E3);
  const float rs = RS1 * __builtin_amdgcn_rcpf(e3);
  const float ex = -(CX / RS1) * e3;
  const float hi = join ? PZ<float>::HI : 1.0f;
  const float lo = join ? PZ<float>::LO : 1.0f;
  float ec, dec;
  if (rs >= hi) {
    const float sq = __builtin_amdgcn_sqrtf(rs);
    pz_dilute(rs, sq, __builtin_amdgcn_rcpf(1.0f + PZ<float>::B1 * sq + PZ<float>::B2 * rs), ec,
              dec);
  } else if (rs <= lo) {
    pz_dense(rs, LNRS1 - x * (1.0f / 3.0f), e3 * (1.0f / RS1), ec, dec);
  } else {
    float e1, d1, e2, d2;
    pz_dense(rs, LNRS1 - x * (1.0f / 3.0f), e3 * (1.0f / RS1), e1, d1);
    const float sq = __builtin_amdgcn_sqrtf(rs);
    pz_dilute(rs, sq, __builtin_amdgcn_rcpf(1.0f + PZ<float>::B1 * sq + PZ<float>::B2 * rs), e2,
              d2);
    const float t = (rs - PZ<float>::LO) * (1.0f / (PZ<float>::HI - PZ<float>::LO));
    const float w = t * t * (3.0f - 2.0f * t);
    const float dw = 6.0f * t * (1.0f - t) * (1.0f / (PZ<float>::HI - PZ<float>::LO));
    ec = (1.0f - w) * e1 + w * e2;
    dec = (1.0f - w) * d1 + w * d2 + dw * (e2 - e1);
  }
  eps = ex + ec;
  v = (4.0f / 3.0f) * ex + ec - rs * (1.0f / 3.0f) * dec;
}

// ---------------------------------------------------------------------------
// Reductions and work mapping
// ---------------------------------------------------------------------------
// Workgroup sum of N values per thread: wavefront shuffles, then one lane
// per wavefront through LDS, summed in a fixed order (deterministic).
// sh must hold N * (nthr / 64) doubles. The totals land in out[0..N) of
// thread 0 only.
template <int N>
__device__ __forceinline__ void block_reduce(double (&vals)[N], double *sh, int tid, int nthr,
                                             double *out) {
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double v = vals[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    vals[q] = v;
  }
  const int lane = tid & 63, wid = tid >> 6, nw = nthr >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) sh[wid * N + q] = vals[q];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double acc = 0.0;
      for (int w = 0; w < nw; ++w) acc += sh[w * N + q];
      out[q] = acc;
    }
  }
  __syncthreads();
}

// Workgroup sums of up to 64 values per thread (N <= 64). Within a
// wavefront a reduce-scatter butterfly halves the values per lane at every
// exchange (63 shuffles in all instead of 6 N), after which lane q holds
// the wavefront total of value q; the wavefront totals are then summed in a
// fixed order (deterministic). sh must hold 64 * (nthr / 64) doubles; the
// totals land in out[0..N) (written by threads 0..N-1).
template <int N>
__device__ __forceinline__ void block_reduce_many(const double (&vals)[N], double *sh, int tid,
                                                  int nthr, double *out) {
  static_assert(N <= 64, "at most 64 values");
  double w[64];
#pragma unroll
  for (int q = 0; q < 64; ++q) w[q] = (q < N) ? vals[q] : 0.0;
  const int lane = tid & 63, wid = tid >> 6, nw = nthr >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int i = 0; i < off; ++i) {
      const double send = up ? w[i] : w[off + i];
      const double keep = up ? w[off + i] : w[i];
      w[i] = keep + __shfl_xor(send, off, 64);
    }
  }
  sh[wid * 64 + lane] = w[0];
  __syncthreads();
  if (tid < N) {
    double acc = 0.0;
    for (int v = 0; v < nw; ++v) acc += sh[v * 64 + tid];
    out[tid] = acc;
  }
  __syncthreads();
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Give every XCD one contiguous range of work items so neighbouring
// items (the fields of one plane, adjacent planes) share an L2. Blocks
// b = x, x+8, x+16, ... land on XCD x; there are q + (x < r) of them for
// grid = 8q + r, and they take the items [x q + min(x, r), ...): a bijection
// of [0, grid).
__device__ __forceinline__ int xcd_item(int b, int grid) {
  const int NX = 8;
  const int q = grid / NX, r = grid - q * NX;
  const int x = b % NX;
  return x * q + (x < r ? x : r) + b / NX;
}

// Solve index of a work item (binary search of the batch prefix sums). The
// result is workgroup-uniform; saying so lets every descriptor field live in
// scalar registers instead of being loaded per lane.
__device__ __forceinline__ int find_solve(const int *first, int nsolve, int item) {
  int lo = 0, hi = nsolve;     // first[lo] <= item < first[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (__builtin_amdgcn_readfirstlane(first[mid]) <= item) lo = mid; else hi = mid;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// first[s] of the batch prefix sums as a workgroup-uniform value.
__device__ __forceinline__ int first_of(const int *first, int s) {
  return __builtin_amdgcn_readfirstlane(first[s]);
}

__device__ __forceinline__ int gidx(int m, int n) { return (2 * m < n) ? m : m - n; }

}  // namespace skx
