// Compile-time FFT machinery for the transform passes (gfx950).
//
// Every supported lattice size N (even, 8..256, factors 2, 3, 5) gets its own
// instantiation: the radix plan, the thread map of every stage and the LDS
// index arithmetic are compile-time constants, so stages fully unroll, index
// division becomes multiply-shift, and LDS addresses stay in the LDS address
// space (ds_read/ds_write rather than flat accesses).
//
// 1D transforms are Stockham autosort FFTs: stage s with radix R and
// Ns = product of the earlier radices reads x[j + r N/R], multiplies by the
// twiddle w^{r (j mod Ns) N/(Ns R)} (w = e^{-2 pi i/N}, conjugated for the
// inverse), applies a radix-R DFT and writes y[(j - j mod Ns) R + j mod Ns + r Ns].
// Each stage reads its inputs into registers, synchronises and writes, so a
// single LDS buffer holds the lines.
#pragma once

#include "common.h"

namespace qf {

// Radix plans: RPlan and make_rplan in common.h (the host's row-tile rule uses them too).

constexpr bool fft_size_ok(int N) {
  int m = N;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  while (m % 5 == 0) m /= 5;
  return m == 1 && N % 2 == 0 && N >= 8 && N <= 256;
}

// ------------------------------------------------------------- butterflies

template <int R, bool INV, typename V> struct Dft;

template <bool INV, typename V> struct Dft<2, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV, typename V> struct Dft<4, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    V t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    V t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

// x * e^{-+ 2 pi i m / 16} for a compile-time m (forward sign -, inverse +)
template <int M, bool INV, typename V>
__device__ __forceinline__ V rot16(V a) {
  using T = decltype(a.x);
  constexpr int m = M & 15;
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, r2 = 0.70710678118654752440;
  constexpr double cs[16] = {1, c1, r2, s1, 0, -s1, -r2, -c1, -1, -c1, -r2, -s1, 0, s1, r2, c1};
  constexpr double sn[16] = {0, s1, r2, c1, 1, c1, r2, s1, 0, -s1, -r2, -c1, -1, -c1, -r2, -s1};
  if constexpr (m == 0) return a;
  else if constexpr (m == 4) return mul_mi<INV>(a);
  else if constexpr (m == 8) { V r; r.x = -a.x; r.y = -a.y; return r; }
  else if constexpr (m == 12) return mul_mi<!INV>(a);
  else {
    const T c = (T)cs[m];
    const T s = INV ? (T)sn[m] : (T)-sn[m];
    V r;
    r.x = fmaT(a.x, c, -(a.y * s));
    r.y = fmaT(a.x, s, a.y * c);
    return r;
  }
}

template <bool INV, typename V> struct Dft<8, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV, V>::run(e);
    Dft<4, INV, V>::run(o);
    const V o1 = rot16<2, INV>(o[1]), o2 = rot16<4, INV>(o[2]), o3 = rot16<6, INV>(o[3]);
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
  }
};

// 16 = 4 x 4: DFT4 over n1 of x[4 n1 + n2], twiddle w16^{n2 k1}, DFT4 over n2 -> X[k1 + 4 k2]
template <bool INV, typename V> struct Dft<16, INV, V> {
  template <int N2>
  static __device__ __forceinline__ void col(V *v, V (&y)[4][4]) {
    V t[4] = {v[N2], v[4 + N2], v[8 + N2], v[12 + N2]};
    Dft<4, INV, V>::run(t);
    y[0][N2] = t[0];
    y[1][N2] = rot16<N2, INV>(t[1]);
    y[2][N2] = rot16<2 * N2, INV>(t[2]);
    y[3][N2] = rot16<3 * N2, INV>(t[3]);
  }
  static __device__ __forceinline__ void run(V *v) {
    V y[4][4];
    col<0>(v, y);
    col<1>(v, y);
    col<2>(v, y);
    col<3>(v, y);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      Dft<4, INV, V>::run(y[k1]);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = y[k1][k2];
    }
  }
};

template <bool INV, typename V> struct Dft<3, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    using T = decltype(v[0].x);
    const T s = (T)0.86602540378443864676;
    V t = cadd(v[1], v[2]);
    V u = cscale(csub(v[1], v[2]), s);
    V a;
    a.x = fmaT((T)-0.5, t.x, v[0].x);
    a.y = fmaT((T)-0.5, t.y, v[0].y);
    V iu = mul_mi<INV>(u);
    v[0] = cadd(v[0], t);
    v[1] = cadd(a, iu);
    v[2] = csub(a, iu);
  }
};

template <bool INV, typename V> struct Dft<5, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    using T = decltype(v[0].x);
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    V t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    V u1 = csub(v[1], v[4]), u2 = csub(v[2], v[3]);
    V a1, a2, p1, p2;
    a1.x = fmaT(c2, t2.x, fmaT(c1, t1.x, v[0].x));
    a1.y = fmaT(c2, t2.y, fmaT(c1, t1.y, v[0].y));
    a2.x = fmaT(c1, t2.x, fmaT(c2, t1.x, v[0].x));
    a2.y = fmaT(c1, t2.y, fmaT(c2, t1.y, v[0].y));
    p1.x = fmaT(s2, u2.x, s1 * u1.x);
    p1.y = fmaT(s2, u2.y, s1 * u1.y);
    p2.x = fmaT(-s1, u2.x, s2 * u1.x);
    p2.y = fmaT(-s1, u2.y, s2 * u1.y);
    V b1 = mul_mi<INV>(p1);
    V b2 = mul_mi<INV>(p2);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// x * e^{-+ 2 pi i m / NN} for NN = 6, 9, 10, 12, 15, 18, 20, 25 or 32 and a compile-time m
// (forward sign -, inverse +).
// The tables hold cos and sin of 2 pi m / NN to 21 digits, with the symmetries
// cos(2 pi (NN - m)/NN) = cos(2 pi m/NN), sin(2 pi (NN - m)/NN) = -sin(2 pi m/NN) exact.
template <int M, int NN, bool INV, typename V>
__device__ __forceinline__ V rot_root(V a) {
  using T = decltype(a.x);
  constexpr int m = M % NN;
  if constexpr (m == 0) {
    return a;
  } else {
    double cm, sm;
    if constexpr (NN == 6) {
      constexpr double cs[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
      constexpr double sn[6] = {0.0, 0.866025403784438646764, 0.866025403784438646764, 0.0,
                                -0.866025403784438646764, -0.866025403784438646764};
      cm = cs[m];
      sm = sn[m];
    } else if constexpr (NN == 10) {
      constexpr double cs[10] = {1.0, 0.809016994374947424102, 0.309016994374947424102, -0.309016994374947424102,
                                 -0.809016994374947424102, -1.0, -0.809016994374947424102,
                                 -0.309016994374947424102, 0.309016994374947424102, 0.809016994374947424102};
      constexpr double sn[10] = {0.0, 0.587785252292473129169, 0.951056516295153572116, 0.951056516295153572116,
                                 0.587785252292473129169, 0.0, -0.587785252292473129169,
                                 -0.951056516295153572116, -0.951056516295153572116, -0.587785252292473129169};
      cm = cs[m];
      sm = sn[m];
    } else if constexpr (NN == 18) {
      constexpr double cs[18] = {1.0, 0.939692620785908384054, 0.766044443118978035202, 0.5,
                                 0.173648177666930348852, -0.173648177666930348852, -0.5,
                                 -0.766044443118978035202, -0.939692620785908384054, -1.0,
                                 -0.939692620785908384054, -0.766044443118978035202, -0.5,
                                 -0.173648177666930348852, 0.173648177666930348852, 0.5,
                                 0.766044443118978035202, 0.939692620785908384054};
      constexpr double sn[18] = {0.0, 0.342020143325668733044, 0.642787609686539326323, 0.866025403784438646764,
                                 0.984807753012208059367, 0.984807753012208059367, 0.866025403784438646764,
                                 0.642787609686539326323, 0.342020143325668733044, 0.0,
                                 -0.342020143325668733044, -0.642787609686539326323, -0.866025403784438646764,
                                 -0.984807753012208059367, -0.984807753012208059367, -0.866025403784438646764,
                                 -0.642787609686539326323, -0.342020143325668733044};
      cm = cs[m];
      sm = sn[m];
    } else if constexpr (NN == 12) {
      constexpr double cs[12] = {1.0, 0.866025403784438646764, 0.5, 0.0, -0.5, -0.866025403784438646764, -1.0, -0.866025403784438646764, -0.5, 0.0, 0.5, 0.866025403784438646764};
      constexpr double sn[12] = {0.0, 0.5, 0.866025403784438646764, 1.0, 0.866025403784438646764, 0.5, 0.0, -0.5, -0.866025403784438646764, -1.0, -0.866025403784438646764, -0.5};
      cm = cs[m];
      sm = sn[m];
    } else if constexpr (NN == 15) {
      constexpr double cs[15] = {1.0, 0.913545457642600895502, 0.669130606358858213826, 0.309016994374947424102, -0.1045284632676534714, -0.5, -0.809016994374947424102, -0.978147600733805637929, -0.978147600733805637929, -0.809016994374947424102, -0.5, -0.1045284632676534714, 0.309016994374947424102, 0.669130606358858213826, 0.913545457642600895502};
      constexpr double sn[15] = {0.0, 0.406736643075800207754, 0.743144825477394235015, 0.951056516295153572116, 0.994521895368273336923, 0.866025403784438646764, 0.587785252292473129169, 0.207911690817759337102, -0.207911690817759337102, -0.587785252292473129169, -0.866025403784438646764, -0.994521895368273336923, -0.951056516295153572116, -0.743144825477394235015, -0.406736643075800207754};
      cm = cs[m];
      sm = sn[m];
    } else if constexpr (NN == 9) {
      constexpr double cs[9] = {1.0, 0.766044443118978035202, 0.173648177666930348852, -0.5,
                                -0.939692620785908384054, -0.939692620785908384054, -0.5,
                                0.173648177666930348852, 0.766044443118978035202};
      constexpr double sn[9] = {0.0, 0.642787609686539326323, 0.984807753012208059367, 0.866025403784438646764,
                                0.342020143325668733044, -0.342020143325668733044, -0.866025403784438646764,
                                -0.984807753012208059367, -0.642787609686539326323};
      cm = cs[m];
      sm = sn[m];
    } else if constexpr (NN == 20) {
      // the first quadrant; cos and sin of 2 pi m / 20 follow by the quarter-turn symmetries
      constexpr double q[6] = {0.0, 0.309016994374947424102, 0.587785252292473129169, 0.809016994374947424102,
                               0.951056516295153572116, 1.0};
      constexpr int oc = m / 5, r = m % 5;       // 2 pi m / 20 = oc pi/2 + 2 pi r / 20
      constexpr double c0 = q[5 - r], s0 = q[r];
      cm = oc == 0 ? c0 : oc == 1 ? -s0 : oc == 2 ? -c0 : s0;
      sm = oc == 0 ? s0 : oc == 1 ? c0 : oc == 2 ? -s0 : -c0;
    } else if constexpr (NN == 32) {
      // the first octant; cos and sin of 2 pi m / 32 follow by the quarter-turn symmetries
      constexpr double q[9] = {0.0, 0.195090322016128267848, 0.382683432365089771728, 0.555570233019602224743,
                               0.707106781186547524401, 0.831469612302545237079, 0.923879532511286756128,
                               0.980785280403230449126, 1.0};
      constexpr int oc = m / 8, r = m % 8;       // 2 pi m / 32 = oc pi/2 + 2 pi r / 32
      constexpr double c0 = q[8 - r], s0 = q[r];
      cm = oc == 0 ? c0 : oc == 1 ? -s0 : oc == 2 ? -c0 : s0;
      sm = oc == 0 ? s0 : oc == 1 ? c0 : oc == 2 ? -s0 : -c0;
    } else {
      static_assert(NN == 25, "roots of unity of order 6, 9, 10, 12, 15, 18, 20, 25 or 32");
      constexpr double cs[25] = {
          1.0, 0.968583161128631119490, 0.876306680043863587308, 0.728968627421411523147,
          0.535826794978996618271, 0.309016994374947424102, 0.062790519529313376076, -0.187381314585724630543,
          -0.425779291565072648863, -0.637423989748689710177, -0.809016994374947424102, -0.929776485888251403661,
          -0.992114701314477831050, -0.992114701314477831050, -0.929776485888251403661, -0.809016994374947424102,
          -0.637423989748689710177, -0.425779291565072648863, -0.187381314585724630543, 0.062790519529313376076,
          0.309016994374947424102, 0.535826794978996618271, 0.728968627421411523147, 0.876306680043863587308,
          0.968583161128631119490};
      constexpr double sn[25] = {
          0.0, 0.248689887164854788242, 0.481753674101715274987, 0.684547105928688673732,
          0.844327925502015078549, 0.951056516295153572116, 0.998026728428271561952, 0.982287250728688681086,
          0.904827052466019527714, 0.770513242775789230803, 0.587785252292473129169, 0.368124552684677959157,
          0.125333233564304245373, -0.125333233564304245373, -0.368124552684677959157, -0.587785252292473129169,
          -0.770513242775789230803, -0.904827052466019527714, -0.982287250728688681086, -0.998026728428271561952,
          -0.951056516295153572116, -0.844327925502015078549, -0.684547105928688673732, -0.481753674101715274987,
          -0.248689887164854788242};
      cm = cs[m];
      sm = sn[m];
    }
    const T c = (T)cm;
    const T s = INV ? (T)sm : (T)-sm;
    V r;
    r.x = fmaT(a.x, c, -(a.y * s));
    r.y = fmaT(a.x, s, a.y * c);
    return r;
  }
}

// 9 = 3 x 3: DFT3 over n1 of x[3 n1 + n2], twiddle w9^{n2 k1}, DFT3 over n2 -> X[k1 + 3 k2]
template <bool INV, typename V> struct Dft<9, INV, V> {
  template <int N2>
  static __device__ __forceinline__ void col(V *v, V (&y)[3][3]) {
    V t[3] = {v[N2], v[3 + N2], v[6 + N2]};
    Dft<3, INV, V>::run(t);
    y[0][N2] = t[0];
    y[1][N2] = rot_root<N2, 9, INV>(t[1]);
    y[2][N2] = rot_root<2 * N2, 9, INV>(t[2]);
  }
  static __device__ __forceinline__ void run(V *v) {
    V y[3][3];
    col<0>(v, y);
    col<1>(v, y);
    col<2>(v, y);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      Dft<3, INV, V>::run(y[k1]);
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) v[k1 + 3 * k2] = y[k1][k2];
    }
  }
};

// 25 = 5 x 5: DFT5 over n1 of x[5 n1 + n2], twiddle w25^{n2 k1}, DFT5 over n2 -> X[k1 + 5 k2]
template <bool INV, typename V> struct Dft<25, INV, V> {
  template <int N2>
  static __device__ __forceinline__ void col(V *v, V (&y)[5][5]) {
    V t[5] = {v[N2], v[5 + N2], v[10 + N2], v[15 + N2], v[20 + N2]};
    Dft<5, INV, V>::run(t);
    y[0][N2] = t[0];
    y[1][N2] = rot_root<N2, 25, INV>(t[1]);
    y[2][N2] = rot_root<2 * N2, 25, INV>(t[2]);
    y[3][N2] = rot_root<3 * N2, 25, INV>(t[3]);
    y[4][N2] = rot_root<4 * N2, 25, INV>(t[4]);
  }
  static __device__ __forceinline__ void run(V *v) {
    V y[5][5];
    col<0>(v, y);
    col<1>(v, y);
    col<2>(v, y);
    col<3>(v, y);
    col<4>(v, y);
#pragma unroll
    for (int k1 = 0; k1 < 5; ++k1) {
      Dft<5, INV, V>::run(y[k1]);
#pragma unroll
      for (int k2 = 0; k2 < 5; ++k2) v[k1 + 5 * k2] = y[k1][k2];
    }
  }
};

// Radix 2R = 2 x R (R = 3, 5; R = 9 is available but unused): DFT2 over n1 of x[R n1 + n2],
// twiddle w_{2R}^{n2 k1}, DFT_R over n2 -> X[k1 + 2 k2].  A plan with a single factor 2 merges
// it into a radix-3 or radix-5 stage, so that the two-point stage does not cost an LDS exchange
// of its own.
template <int R, bool INV, typename V, int N2 = 0>
__device__ __forceinline__ void split2_cols(V *v, V (&y)[2][R]) {
  if constexpr (N2 < R) {
    V t[2] = {v[N2], v[R + N2]};
    Dft<2, INV, V>::run(t);
    y[0][N2] = t[0];
    y[1][N2] = rot_root<N2, 2 * R, INV>(t[1]);
    split2_cols<R, INV, V, N2 + 1>(v, y);
  }
}
template <int R, bool INV, typename V>
__device__ __forceinline__ void dft_split2(V *v) {
  V y[2][R];
  split2_cols<R, INV, V>(v, y);
#pragma unroll
  for (int k1 = 0; k1 < 2; ++k1) {
    Dft<R, INV, V>::run(y[k1]);
#pragma unroll
    for (int k2 = 0; k2 < R; ++k2) v[k1 + 2 * k2] = y[k1][k2];
  }
}
template <bool INV, typename V> struct Dft<6, INV, V> {
  static __device__ __forceinline__ void run(V *v) { dft_split2<3, INV, V>(v); }
};
template <bool INV, typename V> struct Dft<10, INV, V> {
  static __device__ __forceinline__ void run(V *v) { dft_split2<5, INV, V>(v); }
};
template <bool INV, typename V> struct Dft<18, INV, V> {
  static __device__ __forceinline__ void run(V *v) { dft_split2<9, INV, V>(v); }
};

// Radix A B (A, B small): DFT_A over n1 of x[B n1 + n2], twiddle w_{AB}^{n2 k1}, DFT_B over
// n2 -> X[k1 + A k2].  Used for the two-stage complex64 plans of sizes with several small
// factors (radices 12 = 4 x 3 and 15 = 3 x 5) and for radices 20 = 4 x 5 and 32 = 4 x 8.
template <int A, int B, bool INV, typename V, int N2, int K1>
__device__ __forceinline__ void splitab_twiddle(V (&t)[A], V (&y)[A][B]) {
  if constexpr (K1 < A) {
    y[K1][N2] = rot_root<N2 * K1, A * B, INV>(t[K1]);
    splitab_twiddle<A, B, INV, V, N2, K1 + 1>(t, y);
  }
}
template <int A, int B, bool INV, typename V, int N2 = 0>
__device__ __forceinline__ void splitab_cols(V *v, V (&y)[A][B]) {
  if constexpr (N2 < B) {
    V t[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) t[n1] = v[B * n1 + N2];
    Dft<A, INV, V>::run(t);
    splitab_twiddle<A, B, INV, V, N2, 0>(t, y);
    splitab_cols<A, B, INV, V, N2 + 1>(v, y);
  }
}
template <int A, int B, bool INV, typename V>
__device__ __forceinline__ void dft_splitab(V *v) {
  V y[A][B];
  splitab_cols<A, B, INV, V>(v, y);
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    Dft<B, INV, V>::run(y[k1]);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = y[k1][k2];
  }
}
template <bool INV, typename V> struct Dft<12, INV, V> {
  static __device__ __forceinline__ void run(V *v) { dft_splitab<4, 3, INV, V>(v); }
};
template <bool INV, typename V> struct Dft<15, INV, V> {
  static __device__ __forceinline__ void run(V *v) { dft_splitab<3, 5, INV, V>(v); }
};
// 20 = 4 x 5 and 32 = 4 x 8 (x2 parts of split-x2 tiles)
template <bool INV, typename V> struct Dft<20, INV, V> {
  static __device__ __forceinline__ void run(V *v) { dft_splitab<4, 5, INV, V>(v); }
};
template <bool INV, typename V> struct Dft<32, INV, V> {
  static __device__ __forceinline__ void run(V *v) { dft_splitab<4, 8, INV, V>(v); }
};

// ---------------------------------------------------------- line geometry

// Padded index inside a contiguous line: one spare slot every 16 elements,
// so that the stride-R writes of the early Stockham stages spread over banks.
__host__ __device__ constexpr int padn(int n) { return n + (n >> 4); }
__host__ __device__ constexpr int padded_len(int N) { return padn(N - 1) + 1; }

// Lines of a plane / row tile stored row-major: element n of line b at b*P + padn(n).
template <int NL, int P> struct RowsGeo {
  static constexpr int nlines = NL;
  static constexpr bool linefast = false;
  static __device__ __forceinline__ int at(int b, int n) { return b * P + padn(n); }
};
// Columns of a row-major plane: element n of line b (column b) at n*P + padn(b).
template <int NL, int P> struct ColsGeo {
  static constexpr int nlines = NL;
  static constexpr bool linefast = true;
  static __device__ __forceinline__ int at(int b, int n) { return n * P + padn(b); }
};

// ------------------------------------------------------- twiddle tables
//
// Each stage with Ns > 1 gets its own LDS table laid out [r-1][j mod Ns]
// holding w^{r (j mod Ns) N/(Ns R)}, so that lanes with consecutive j read
// consecutive entries (a single table indexed r (j mod Ns) N/(Ns R) makes
// lanes stride through it and collide on LDS banks).  Tables of the radix
// plan come first, then those of the reversed plan.

template <typename T, int N, bool REV> __host__ __device__ constexpr RPlan plan_of() {
  RPlan p = make_rplan(N, sizeof(T) == 8);
  if (REV) {
    RPlan q = p;
    for (int i = 0; i < p.n; ++i) q.r[i] = p.r[p.n - 1 - i];
    return q;
  }
  return p;
}
template <typename T, int N, bool REV, int S> __host__ __device__ constexpr int ns_before() {
  int ns = 1;
  for (int i = 0; i < S; ++i) ns *= plan_of<T, N, REV>().r[i];
  return ns;
}
template <typename T, int N, bool REV> __host__ __device__ constexpr int tw_plan_size() {
  constexpr RPlan p = plan_of<T, N, REV>();
  int sz = 0, ns = 1;
  for (int i = 0; i < p.n; ++i) {
    if (ns > 1) sz += (p.r[i] - 1) * ns;
    ns *= p.r[i];
  }
  return sz;
}
template <typename T, int N> __host__ __device__ constexpr int tw_total() { return tw_plan_size<T, N, false>() + tw_plan_size<T, N, true>(); }
template <typename T, int N, bool REV, int S> __host__ __device__ constexpr int tw_off() {
  constexpr RPlan p = plan_of<T, N, REV>();
  int off = REV ? tw_plan_size<T, N, false>() : 0, ns = 1;
  for (int i = 0; i < S; ++i) {
    if (ns > 1) off += (p.r[i] - 1) * ns;
    ns *= p.r[i];
  }
  return off;
}

template <typename T, int N, bool REV, int NT, int S>
__device__ __forceinline__ void fill_tw_plan(C<T> *lt, const C<T> *gtw) {
  constexpr RPlan p = plan_of<T, N, REV>();
  if constexpr (S < p.n) {
    constexpr int R = p.r[S];
    constexpr int NS = ns_before<T, N, REV, S>();
    if constexpr (NS > 1) {
      constexpr int off = tw_off<T, N, REV, S>();
      constexpr int twstep = N / (NS * R);
      for (int i = threadIdx.x; i < (R - 1) * NS; i += NT) {
        const int r = i / NS + 1, kk = i - (r - 1) * NS;
        lt[off + i] = gtw[r * kk * twstep];
      }
    }
    fill_tw_plan<T, N, REV, NT, S + 1>(lt, gtw);
  }
}

// stage twiddle tables of both plans from the roots of unity w^m, m < N (global)
template <typename T, int N, int NT>
__device__ __forceinline__ void fill_twiddles(C<T> *lt, const C<T> *gtw) {
  fill_tw_plan<T, N, false, NT, 0>(lt, gtw);
  fill_tw_plan<T, N, true, NT, 0>(lt, gtw);
}

// ----------------------------------------------------------------- stages

template <typename T, int N, int R, int NS, bool INV, class G, int NT, int TWOFF>
__device__ __forceinline__ void tstage(C<T> *buf, const C<T> *tw) {
  constexpr int NR = N / R;
  constexpr int total = G::nlines * NR;
  constexpr int CAPQ = (total + NT - 1) / NT;
  const int tid = threadIdx.x;
  C<T> v[CAPQ][R];
  int jq[CAPQ], bq[CAPQ];
#pragma unroll
  for (int q = 0; q < CAPQ; ++q) {
    const int f = tid + q * NT;
    if (total % NT == 0 || f < total) {
      int j, b;
      if constexpr (G::linefast) { b = f % G::nlines; j = f / G::nlines; }
      else { j = f % NR; b = f / NR; }
      jq[q] = j;
      bq[q] = b;
      const int kk = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C<T> x = buf[G::at(b, j + r * NR)];
        if constexpr (NS > 1) {
          if (r > 0) {
            C<T> w = tw[TWOFF + (r - 1) * NS + kk];
            if (INV) w.y = -w.y;
            x = cmul(x, w);
          }
        }
        v[q][r] = x;
      }
      Dft<R, INV, C<T>>::run(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < CAPQ; ++q) {
    if (total % NT == 0 || tid + q * NT < total) {
      const int j = jq[q], b = bq[q];
      const int kk = j % NS;
      const int base = (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[G::at(b, base + r * NS)] = v[q][r];
    }
  }
  __syncthreads();
}

template <typename T, int N, bool INV, class G, int NT, int S, int NS>
__device__ __forceinline__ void run_stages(C<T> *buf, const C<T> *tw) {
  constexpr RPlan P = make_rplan(N, sizeof(T) == 8);
  if constexpr (S < P.n) {
    constexpr int R = P.r[S];
    tstage<T, N, R, NS, INV, G, NT, tw_off<T, N, false, S>()>(buf, tw);
    run_stages<T, N, INV, G, NT, S + 1, NS * R>(buf, tw);
  }
}

template <typename T, int N, bool INV, class G, int NT>
__device__ __forceinline__ void fft_lines_t(C<T> *buf, const C<T> *tw) {
  run_stages<T, N, INV, G, NT, 0, 1>(buf, tw);
}

// ------------------------------------------- stages with explicit data paths
//
// The steady-state passes fuse the first and last radix stages with global
// memory (inputs loaded straight into registers, outputs stored straight from
// registers) and fuse an inverse transform's last stage with the next forward
// transform's first stage (same radix, same thread map) around a pointwise
// multiply, skipping LDS round trips.  A transform run with the reversed radix
// plan consumes the natural-order output of the forward plan's last stage.

template <class G, int N, int R, int NT> struct SG {
  static constexpr int NR = N / R;
  static constexpr int total = G::nlines * NR;
  static constexpr int CAPQ = (total + NT - 1) / NT;
  static __device__ __forceinline__ bool active(int q) { return total % NT == 0 || (int)threadIdx.x + q * NT < total; }
  static __device__ __forceinline__ void jb(int q, int &j, int &b) {
    const int f = (int)threadIdx.x + q * NT;
    if constexpr (G::linefast) { b = f % G::nlines; j = f / G::nlines; }
    else { j = f % NR; b = f / NR; }
  }
};

// inputs x[b][j + r N/R] from src(b, n), twiddles of a stage with NS, radix-R DFT
template <typename T, int N, int R, int NS, bool INV, class G, int NT, int TWOFF, int CQ, class Src>
__device__ __forceinline__ void st_read(C<T> (&v)[CQ][R], const C<T> *tw, Src src) {
  using S = SG<G, N, R, NT>;
#pragma unroll
  for (int q = 0; q < S::CAPQ; ++q) {
    if (S::active(q)) {
      int j, b;
      S::jb(q, j, b);
      const int kk = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C<T> x = src(b, j + r * S::NR);
        if constexpr (NS > 1) {
          if (r > 0) {
            C<T> w = tw[TWOFF + (r - 1) * NS + kk];
            if (INV) w.y = -w.y;
            x = cmul(x, w);
          }
        }
        v[q][r] = x;
      }
      Dft<R, INV, C<T>>::run(v[q]);
    }
  }
}

// outputs y[b][(j - j mod NS) R + j mod NS + r NS] to dst(b, n, value)
template <typename T, int N, int R, int NS, class G, int NT, int CQ, class Dst>
__device__ __forceinline__ void st_write(C<T> (&v)[CQ][R], Dst dst) {
  using S = SG<G, N, R, NT>;
#pragma unroll
  for (int q = 0; q < S::CAPQ; ++q) {
    if (S::active(q)) {
      int j, b;
      S::jb(q, j, b);
      const int kk = j % NS;
      const int base = (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) dst(b, base + r * NS, v[q][r]);
    }
  }
}

// stages [S0, S1) of plan (N, REV), LDS -> LDS
template <typename T, int N, bool REV, bool INV, class G, int NT, int S0, int S1>
__device__ __forceinline__ void lds_stages(C<T> *buf, const C<T> *tw) {
  if constexpr (S0 < S1) {
    constexpr int R = plan_of<T, N, REV>().r[S0];
    constexpr int NS = ns_before<T, N, REV, S0>();
    C<T> v[SG<G, N, R, NT>::CAPQ][R];
    st_read<T, N, R, NS, INV, G, NT, tw_off<T, N, REV, S0>()>(v, tw, [&](int b, int n) { return buf[G::at(b, n)]; });
    __syncthreads();
    st_write<T, N, R, NS, G, NT>(v, [&](int b, int n, C<T> x) { buf[G::at(b, n)] = x; });
    __syncthreads();
    lds_stages<T, N, REV, INV, G, NT, S0 + 1, S1>(buf, tw);
  }
}

}  // namespace qf
