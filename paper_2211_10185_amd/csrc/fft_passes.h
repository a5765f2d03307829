// Transform passes of the split-operator step (templates; instantiated per N).
//
// One step of an FFT kinetic term (Sec. 2, eqs. HK1-HK3, with the symmetric
// split h F^-1[e^{-dt T} F[h psi]]) is carried out as passes over HBM, each
// reading and writing the state once:
//
//   plane pass  (x2-x3 plane in LDS): inverse x2,x3 -> x h^2 -> forward x3,x2
//   row pass    (x3 rows in LDS):     inverse x3 -> x h^2 -> forward x3
//   column pass (TC contiguous x3 columns along x1 or x2 in LDS):
//               forward -> x e^{-dt T(k)}/N^3 -> inverse
//
// Mode bits (common.h) select which of these pieces a launch performs, so
// the same kernels also start and end a chunk (x h instead of x h^2) and run
// plain forward/inverse transforms.
#pragma once

#include "fft_core.h"

namespace qf {

template <int N> __host__ __device__ constexpr int plane_threads() {
  int t = (N * N / 16 + 63) / 64 * 64;
  return t < 64 ? 64 : (t > 1024 ? 1024 : t);
}
// Row pitch of the plane in LDS (elements).  LDS serves a wave's 64 accesses
// in 128-byte passes (16 lanes of 8-byte or 8 lanes of 16-byte elements);
// distinct elements of one pass that share (index mod 128/element size)
// serialise.  The pitches below minimise those repeats over every access of
// the steady plane pass (both row-stage lane maps, the stride-R Stockham
// writes) for the sizes where the padded length alone leaves them; found with
// a model of that access pattern and checked against the LDS bank-conflict
// counter at N = 128 (7x fewer conflict cycles).
template <typename T, int N> __host__ __device__ constexpr int plane_pitch() {
  if constexpr (sizeof(T) == 4) {
    switch (N) {
      case 18: return 25; case 24: return 35; case 32: return 36; case 40: return 44; case 48: return 51;
      case 50: return 56; case 64: return 72; case 80: return 85; case 96: return 108; case 128: return 136;
      default: return padded_len(N);
    }
  } else {
    switch (N) {
      case 12: return 19; case 24: return 27; case 32: return 36; case 40: return 45; case 48: return 51;
      case 80: return 85;
      default: return padded_len(N);
    }
  }
}
template <typename T, int N> __host__ __device__ constexpr size_t plane_lds_t() {
  return (size_t)(N * plane_pitch<T, N>() + tw_total<T, N>()) * sizeof(C<T>);
}
template <typename T, int N> __host__ __device__ constexpr bool plane_fits() {
  return plane_lds_t<T, N>() <= 160 * 1024 && N * N <= 16 * 1024;
}
template <typename T, int N> __host__ __device__ constexpr int row_block_t() { return row_block(N, sizeof(T) == 8); }
template <typename T, int N> __host__ __device__ constexpr size_t row_lds_t() {
  return (size_t)(row_block_t<T, N>() * padded_len(N) + tw_total<T, N>()) * sizeof(C<T>);
}
template <typename T> __host__ __device__ constexpr int col_tile_t() { return col_tile(sizeof(T) == 8); }
template <typename T, int N> __host__ __device__ constexpr size_t col_lds_t() {
  return (size_t)(N * (col_tile_t<T>() + 1) + tw_total<T, N>()) * sizeof(C<T>);
}

// psi * f where f is real (T) or complex (C<T>) at site `off`.
template <typename T>
__device__ __forceinline__ C<T> vmul_t(C<T> v, const void *f, int vcomplex, size_t off) {
  if (vcomplex) return cmul(v, ((const C<T> *)f)[off]);
  return cscale(v, ((const T *)f)[off]);
}

// k-space factor at FFT indices (i1, i2, i3): e^{-dt T(k)} / N^3 for the split
// step, dt T(k) / N^3 for the A/B update (the column pass then yields dt H_K psi).
template <typename T>
__device__ __forceinline__ T kin_factor_t(const PassDesc &d, int i1, int i2, int i3) {
  const T *kt = (const T *)d.ktab;
  if (d.kin == KIN_REL) {
    const T p2 = kt[i1] + kt[i2] + kt[i3];
    const T m = (T)d.m;
    if constexpr (sizeof(T) == 4) {
      // single-instruction sqrt, reciprocal and 2^x (about 1 ulp each).  The A/B factor is
      // dt T itself, so T = p^2 / (sqrt(p^2 + m^2) + m) avoids the cancellation; in the split
      // factor T only enters the exponent, where sqrt(p^2 + m^2) - m is off by at most
      // dt sqrt(p^2 + m^2) 2^-24 in absolute terms, and the reciprocal is saved
      const float r = __builtin_amdgcn_sqrtf(p2 + m * m);
      if (d.scheme == SCHEME_AB) return p2 * __builtin_amdgcn_rcpf(r + m) * (float)(d.dt * d.inv_n3);
      return __builtin_amdgcn_exp2f(-(float)d.dt * 1.4426950408889634f * (r - m)) * (float)d.inv_n3;
    } else {
      const T tk = p2 / (sqrt(p2 + m * m) + m);   // sqrt(p^2 + m^2) - m without cancellation
      if (d.scheme == SCHEME_AB) return tk * (T)(d.dt * d.inv_n3);
      return exp(-(T)d.dt * tk) * (T)d.inv_n3;
    }
  }
  // separable terms: the table holds t(k_j) (A/B) or e^{-dt t(k_j)} (split)
  if (d.scheme == SCHEME_AB) return (kt[i1] + kt[i2] + kt[i3]) * (T)(d.dt * d.inv_n3);
  return kt[i1] * kt[i2] * kt[i3] * (T)d.inv_n3;
}

// A/B update at one site: psi' = A psi - B x with x = dt H_K psi,
// A = (1 - dt V/2)/(1 + dt V/2), B = 1/(1 + dt V/2) (complex when V is).
template <typename T>
__device__ __forceinline__ C<T> ab_combine(C<T> p, C<T> x, const PassDesc &d, size_t off) {
  const T hdt = (T)(0.5 * d.dt);
  if (d.vcomplex) {
    const C<T> V = ((const C<T> *)d.vtab)[off];
    const T dr = fmaT(hdt, V.x, (T)1), di = hdt * V.y;
    const T den = (T)1 / fmaT(dr, dr, di * di);
    const C<T> B = mkc<T>(dr * den, -di * den);
    const C<T> A = cmul(mkc<T>(fmaT(-hdt, V.x, (T)1), -hdt * V.y), B);
    return csub(cmul(A, p), cmul(B, x));
  }
  const T V = ((const T *)d.vtab)[off];
  const T B = (T)1 / fmaT(hdt, V, (T)1);
  const T A = fmaT(-hdt, V, (T)1) * B;
  return mkc<T>(fmaT(A, p.x, -(B * x.x)), fmaT(A, p.y, -(B * x.y)));
}

template <typename T, int N, int NT>
__device__ __forceinline__ void load_tw(C<T> *tw, const PassDesc &d) {
  fill_twiddles<T, N, NT>(tw, (const C<T> *)d.tw);
}

// ------------------------------------------------------------- plane pass

// Steady-state plane pass (inverse x2,x3 -> x h^2 -> forward x3,x2) with the
// first stage read from HBM, the last stage written to HBM, and the inverse-x3
// last stage, the potential factor and the forward-x3 first stage fused in
// registers.  The inverse uses the radix plan, the forward its reverse.
template <typename T, bool VC> struct FacT { using type = T; };
template <typename T> struct FacT<T, true> { using type = C<T>; };

//
// AB: the steady pass of the A/B update instead: g is alt (holding the
// transformed dt H_K psi), and the fused middle stage replaces the h^2
// multiply by psi' = A psi - B (dt H_K psi), reading psi and writing psi' at
// gp; the forward transform of psi' goes back to alt.
template <typename T, int N, int NT, int P, bool VC, bool AB = false>
__device__ __forceinline__ void plane_steady(C<T> *pl, const C<T> *tw, C<T> *g, const PassDesc &d, size_t voff,
                                             C<T> *gp = nullptr) {
  using Rows = RowsGeo<N, P>;
  using Cols = ColsGeo<N, P>;
  constexpr RPlan PL = plan_of<T, N, false>();
  constexpr int M = PL.n - 1;
  // potential factors of the fused middle stage, fetched before any transform
  // work so their latency overlaps the inverse transforms
  constexpr int RMID = PL.r[M];
  using SMID = SG<Rows, N, RMID, NT>;
  using F = typename FacT<T, VC>::type;
  F hq[AB ? 1 : SMID::CAPQ][AB ? 1 : RMID];
  if constexpr (!AB) {
#pragma unroll
    for (int q = 0; q < SMID::CAPQ; ++q) {
      if (SMID::active(q)) {
        int j, b;
        SMID::jb(q, j, b);
#pragma unroll
        for (int r = 0; r < RMID; ++r) hq[q][r] = ((const F *)d.h2fac)[voff + (size_t)b * N + j + r * SMID::NR];
      }
    }
  }
  {
    constexpr int R = PL.r[0];
    C<T> v[SG<Cols, N, R, NT>::CAPQ][R];
    st_read<T, N, R, 1, true, Cols, NT, 0>(v, tw, [&](int b, int n) { return g[n * N + b]; });
    st_write<T, N, R, 1, Cols, NT>(v, [&](int b, int n, C<T> x) { pl[Cols::at(b, n)] = x; });
    __syncthreads();
  }
  lds_stages<T, N, false, true, Cols, NT, 1, PL.n>(pl, tw);
  lds_stages<T, N, false, true, Rows, NT, 0, M>(pl, tw);
  {
    constexpr int R = PL.r[M];
    constexpr int NSL = ns_before<T, N, false, M>();
    using S = SG<Rows, N, R, NT>;
    C<T> v[S::CAPQ][R];
    st_read<T, N, R, NSL, true, Rows, NT, tw_off<T, N, false, M>()>(v, tw, [&](int b, int n) { return pl[Rows::at(b, n)]; });
    __syncthreads();
#pragma unroll
    for (int q = 0; q < S::CAPQ; ++q) {
      if (S::active(q)) {
        int j, b;
        S::jb(q, j, b);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if constexpr (AB) {
            // the last inverse stage leaves element n = j + r N/R of line b in v[q][r]
            const size_t o = (size_t)b * N + j + r * S::NR;
            const C<T> y = ab_combine<T>(gp[o], v[q][r], d, voff + o);
            gp[o] = y;
            v[q][r] = y;
          } else if constexpr (VC) {
            v[q][r] = cmul(v[q][r], hq[q][r]);
          } else {
            v[q][r] = cscale(v[q][r], hq[q][r]);
          }
        }
        Dft<R, false, C<T>>::run(v[q]);
      }
    }
    st_write<T, N, R, 1, Rows, NT>(v, [&](int b, int n, C<T> x) { pl[Rows::at(b, n)] = x; });
    __syncthreads();
  }
  lds_stages<T, N, true, false, Rows, NT, 1, PL.n>(pl, tw);
  lds_stages<T, N, true, false, Cols, NT, 0, M>(pl, tw);
  {
    constexpr int R = plan_of<T, N, true>().r[M];
    constexpr int NSL = ns_before<T, N, true, M>();
    C<T> v[SG<Cols, N, R, NT>::CAPQ][R];
    st_read<T, N, R, NSL, false, Cols, NT, tw_off<T, N, true, M>()>(v, tw, [&](int b, int n) { return pl[Cols::at(b, n)]; });
    st_write<T, N, R, NSL, Cols, NT>(v, [&](int b, int n, C<T> x) { g[n * N + b] = x; });
  }
}

// A/B update on one plane.  Chunk start (M_FWD | M_ALT): psi -> F3 F2 -> alt.
// Steady (M_INV | M_COMB | M_FWD | M_ALT): alt -> F2^-1 F3^-1 gives dt H_K psi,
// combined with psi into psi' (written to psi), then F3 F2 psi' -> alt.
// Chunk end (M_INV | M_COMB): the same without the forward transform.
template <typename T, int N, int NT, int P>
__device__ __forceinline__ void plane_ab(C<T> *pl, const C<T> *tw, const PassDesc &d, uint32_t mode, int s, int i1) {
  constexpr size_t N2 = (size_t)N * N;
  const size_t base = ((size_t)s * N + i1) * N2;
  C<T> *gp = (C<T> *)d.psi + base;
  C<T> *ga = (C<T> *)d.alt + base;
  const size_t voff = (size_t)i1 * N2;
  const bool comb = (mode & M_COMB) != 0;
  const C<T> *src = comb ? ga : gp;
  for (int idx = threadIdx.x; idx < N * N; idx += NT) {
    const int r = idx / N, c = idx - r * N;
    pl[r * P + padn(c)] = src[idx];
  }
  __syncthreads();
  using Rows = RowsGeo<N, P>;
  using Cols = ColsGeo<N, P>;
  if (mode & M_INV) {
    fft_lines_t<T, N, true, Cols, NT>(pl, tw);
    fft_lines_t<T, N, true, Rows, NT>(pl, tw);
  }
  if (comb) {
    for (int idx = threadIdx.x; idx < N * N; idx += NT) {
      const int r = idx / N, c = idx - r * N;
      const int a = r * P + padn(c);
      const C<T> o = ab_combine<T>(gp[idx], pl[a], d, voff + idx);
      gp[idx] = o;
      pl[a] = o;
    }
    __syncthreads();
  }
  if (mode & M_FWD) {
    fft_lines_t<T, N, false, Rows, NT>(pl, tw);
    fft_lines_t<T, N, false, Cols, NT>(pl, tw);
    C<T> *dst = (mode & M_ALT) ? ga : gp;
    for (int idx = threadIdx.x; idx < N * N; idx += NT) {
      const int r = idx / N, c = idx - r * N;
      dst[idx] = pl[r * P + padn(c)];
    }
  }
}

// Tile = one x2-x3 plane (state s, i1).  NT = threads of the block (the
// plane kernel of a single size uses plane_threads<N>(); a multi-size kernel
// runs every size with its own, larger, block).
template <typename T, int N, int NT>
__device__ __forceinline__ void plane_body(const LaunchList &L, int e, int t, unsigned char *smem) {
  constexpr int P = plane_pitch<T, N>();
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const int s = t / N, i1 = t - s * N;
  C<T> *pl = (C<T> *)smem;
  C<T> *tw = pl + N * P;
  load_tw<T, N, NT>(tw, d);
  constexpr size_t N2 = (size_t)N * N;
  C<T> *g = (C<T> *)d.psi + ((size_t)s * N + i1) * N2;
  const size_t voff = (size_t)i1 * N2;
  if (mode & (M_COMB | M_ALT)) {
    if constexpr (plan_of<T, N, false>().n >= 2) {
      if (mode == (M_INV | M_COMB | M_FWD | M_ALT)) {
        __syncthreads();
        C<T> *ga = (C<T> *)d.alt + ((size_t)s * N + i1) * N2;
        plane_steady<T, N, NT, P, false, true>(pl, tw, ga, d, voff, g);
        return;
      }
    }
    plane_ab<T, N, NT, P>(pl, tw, d, mode, s, i1);
    return;
  }
  if constexpr (plan_of<T, N, false>().n >= 2) {
    if (mode == (M_INV | M_MID | M_FWD)) {
      __syncthreads();
      if (d.vcomplex) plane_steady<T, N, NT, P, true>(pl, tw, g, d, voff);
      else plane_steady<T, N, NT, P, false>(pl, tw, g, d, voff);
      return;
    }
  }
  for (int idx = threadIdx.x; idx < N * N; idx += NT) {
    const int r = idx / N, c = idx - r * N;
    C<T> v = g[idx];
    if (mode & M_PRE) v = vmul_t<T>(v, d.hfac, d.vcomplex, voff + idx);
    pl[r * P + padn(c)] = v;
  }
  __syncthreads();
  using Rows = RowsGeo<N, P>;
  using Cols = ColsGeo<N, P>;
  if (mode & M_INV) {
    fft_lines_t<T, N, true, Cols, NT>(pl, tw);
    fft_lines_t<T, N, true, Rows, NT>(pl, tw);
  }
  if (mode & M_MID) {
    for (int idx = threadIdx.x; idx < N * N; idx += NT) {
      const int r = idx / N, c = idx - r * N;
      const int a = r * P + padn(c);
      pl[a] = vmul_t<T>(pl[a], d.h2fac, d.vcomplex, voff + idx);
    }
    __syncthreads();
  }
  if (mode & M_FWD) {
    fft_lines_t<T, N, false, Rows, NT>(pl, tw);
    fft_lines_t<T, N, false, Cols, NT>(pl, tw);
  }
  for (int idx = threadIdx.x; idx < N * N; idx += NT) {
    const int r = idx / N, c = idx - r * N;
    C<T> v = pl[r * P + padn(c)];
    if (mode & M_POST) v = vmul_t<T>(v, d.hfac, d.vcomplex, voff + idx);
    g[idx] = v;
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(plane_threads<N>()) k_plane_t(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int e = find_entry(L, blockIdx.x);
  plane_body<T, N, plane_threads<N>()>(L, e, blockIdx.x - L.tile_start[e], smem);
}

// --------------------------------------------------------------- row pass

// Site offset within its state of element x (< RB N) of a row tile whose first row starts at
// offset voff0 (< N^3) of its state.  Where a tile spans at most two states (RB N <= N^3, all
// N >= 16) the offset wraps at most once and one compare replaces a 64-bit remainder per
// element.
template <typename T, int N>
__device__ __forceinline__ size_t row_site(size_t voff0, size_t x) {
  constexpr size_t N3 = (size_t)N * N * N;
  const size_t o = voff0 + x;
  if constexpr ((size_t)row_block_t<T, N>() * N <= N3) return o >= N3 ? o - N3 : o;
  else return o % N3;
}

// Steady-state row pass (inverse x3 -> x h^2 -> forward x3): first stage from
// HBM, last stage to HBM, middle stages fused around the potential factor.
template <typename T, int N, int NT, int RB, int P, bool AB = false>
__device__ __forceinline__ void row_steady(C<T> *buf, const C<T> *tw, C<T> *g, const PassDesc &d, size_t voff0,
                                           int nrows, C<T> *gp = nullptr) {
  using Rows = RowsGeo<RB, P>;
  constexpr RPlan PL = plan_of<T, N, false>();
  constexpr int M = PL.n - 1;
  constexpr size_t N3 = (size_t)N * N * N;
  const C<T> zero = mkc<T>(0, 0);
  // complex64: the potential factors of the fused middle stage are fetched before the first
  // stage, so that their latency overlaps the inverse transform (at most one largest-radix
  // butterfly's worth of values per lane; complex128 keeps its registers for the transform)
  constexpr bool PRE = !AB && sizeof(T) == 4;
  using SMID = SG<Rows, N, PL.r[M], NT>;
  C<T> hq[PRE ? SMID::CAPQ : 1][PRE ? PL.r[M] : 1];
  if constexpr (PRE) {
    const bool vc = d.vcomplex != 0;
#pragma unroll
    for (int q = 0; q < SMID::CAPQ; ++q) {
      if (SMID::active(q)) {
        int j, b;
        SMID::jb(q, j, b);
#pragma unroll
        for (int r = 0; r < PL.r[M]; ++r) {
          hq[q][r] = zero;
          if (b < nrows) {
            const size_t s = row_site<T, N>(voff0, (size_t)b * N + j + r * SMID::NR);
            hq[q][r] = vc ? ((const C<T> *)d.h2fac)[s] : mkc<T>(((const T *)d.h2fac)[s], 0);
          }
        }
      }
    }
  }
  {
    constexpr int R = PL.r[0];
    C<T> v[SG<Rows, N, R, NT>::CAPQ][R];
    st_read<T, N, R, 1, true, Rows, NT, 0>(v, tw, [&](int b, int n) { return b < nrows ? g[b * N + n] : zero; });
    st_write<T, N, R, 1, Rows, NT>(v, [&](int b, int n, C<T> x) { buf[Rows::at(b, n)] = x; });
    __syncthreads();
  }
  lds_stages<T, N, false, true, Rows, NT, 1, M>(buf, tw);
  {
    constexpr int R = PL.r[M];
    constexpr int NSL = ns_before<T, N, false, M>();
    using SS = SG<Rows, N, R, NT>;
    C<T> v[SS::CAPQ][R];
    st_read<T, N, R, NSL, true, Rows, NT, tw_off<T, N, false, M>()>(v, tw, [&](int b, int n) { return buf[Rows::at(b, n)]; });
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SS::CAPQ; ++q) {
      if (SS::active(q)) {
        int j, b;
        SS::jb(q, j, b);
        if (b < nrows) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if constexpr (AB) {
              // A/B update (g is alt): psi' = A psi - B (dt H_K psi), psi read and written at gp
              const size_t o = (size_t)b * N + j + r * SS::NR;
              const C<T> y = ab_combine<T>(gp[o], v[q][r], d, row_site<T, N>(voff0, o));
              gp[o] = y;
              v[q][r] = y;
            } else if constexpr (PRE) {
              v[q][r] = d.vcomplex ? cmul(v[q][r], hq[q][r]) : cscale(v[q][r], hq[q][r].x);
            } else {
              v[q][r] = vmul_t<T>(v[q][r], d.h2fac, d.vcomplex, row_site<T, N>(voff0, (size_t)b * N + j + r * SS::NR));
            }
          }
        }
        Dft<R, false, C<T>>::run(v[q]);
      }
    }
    st_write<T, N, R, 1, Rows, NT>(v, [&](int b, int n, C<T> x) { buf[Rows::at(b, n)] = x; });
    __syncthreads();
  }
  lds_stages<T, N, true, false, Rows, NT, 1, M>(buf, tw);
  {
    constexpr int R = plan_of<T, N, true>().r[M];
    constexpr int NSL = ns_before<T, N, true, M>();
    C<T> v[SG<Rows, N, R, NT>::CAPQ][R];
    st_read<T, N, R, NSL, false, Rows, NT, tw_off<T, N, true, M>()>(v, tw, [&](int b, int n) { return buf[Rows::at(b, n)]; });
    st_write<T, N, R, NSL, Rows, NT>(v, [&](int b, int n, C<T> x) {
      if (b < nrows) g[b * N + n] = x;
    });
  }
}

// A/B update on a row tile (modes as for plane_ab, transforms along x3 only).
template <typename T, int N, int NT, int RB, int P>
__device__ __forceinline__ void row_ab(C<T> *buf, const C<T> *tw, const PassDesc &d, uint32_t mode, long long row0,
                                       int nrows, size_t voff0) {
  constexpr size_t N3 = (size_t)N * N * N;
  C<T> *gp = (C<T> *)d.psi + (size_t)row0 * N;
  C<T> *ga = (C<T> *)d.alt + (size_t)row0 * N;
  const bool comb = (mode & M_COMB) != 0;
  const C<T> *src = comb ? ga : gp;
  for (int idx = threadIdx.x; idx < RB * N; idx += NT) {
    const int r = idx / N, c = idx - r * N;
    buf[r * P + padn(c)] = r < nrows ? src[idx] : mkc<T>(0, 0);
  }
  __syncthreads();
  using Rows = RowsGeo<RB, P>;
  if (mode & M_INV) fft_lines_t<T, N, true, Rows, NT>(buf, tw);
  if (comb) {
    for (int idx = threadIdx.x; idx < nrows * N; idx += NT) {
      const int r = idx / N, c = idx - r * N;
      const int a = r * P + padn(c);
      const C<T> o = ab_combine<T>(gp[idx], buf[a], d, row_site<T, N>(voff0, idx));
      gp[idx] = o;
      buf[a] = o;
    }
    __syncthreads();
  }
  if (mode & M_FWD) {
    fft_lines_t<T, N, false, Rows, NT>(buf, tw);
    C<T> *dst = (mode & M_ALT) ? ga : gp;
    for (int idx = threadIdx.x; idx < nrows * N; idx += NT) {
      const int r = idx / N, c = idx - r * N;
      dst[idx] = buf[r * P + padn(c)];
    }
  }
}

// Tile = RB consecutive x3 rows over all states (the last tile may be short).
template <typename T, int N, int NT>
__device__ __forceinline__ void row_body(const LaunchList &L, int e, int t, unsigned char *smem) {
  constexpr int P = padded_len(N);
  constexpr int RB = row_block_t<T, N>();
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const long long rows_total = (long long)d.k * N * N;
  // Where whole tiles tile each state, consecutive blocks take the same rows of successive
  // states: the k reads of the potential factor for those rows then fall close together in
  // time and all but the first are served by the shared last-level cache instead of HBM.
  // A bijection on [0, k N^2 / RB); the arithmetic of every tile is unchanged.
  long long tile = t;
  if constexpr (((long long)N * N) % RB == 0) {
    if (d.k > 1) tile = (long long)(t % d.k) * ((long long)N * N / RB) + t / d.k;
  }
  const long long row0 = tile * RB;
  const int nrows = (int)((rows_total - row0) < RB ? (rows_total - row0) : RB);
  C<T> *buf = (C<T> *)smem;
  C<T> *tw = buf + RB * P;
  load_tw<T, N, NT>(tw, d);
  constexpr size_t N3 = (size_t)N * N * N;
  C<T> *g = (C<T> *)d.psi + (size_t)row0 * N;
  // site offset of the tile's first row within its state; (voff0 + idx) % N^3 wraps at state boundaries
  const size_t voff0 = (size_t)(row0 % (long long)(N * N)) * N;
  if (mode & (M_COMB | M_ALT)) {
    if constexpr (plan_of<T, N, false>().n >= 2) {
      if (mode == (M_INV | M_COMB | M_FWD | M_ALT)) {
        __syncthreads();
        row_steady<T, N, NT, RB, P, true>(buf, tw, (C<T> *)d.alt + (size_t)row0 * N, d, voff0, nrows, g);
        return;
      }
    }
    row_ab<T, N, NT, RB, P>(buf, tw, d, mode, row0, nrows, voff0);
    return;
  }
  if constexpr (plan_of<T, N, false>().n >= 2) {
    if (mode == (M_INV | M_MID | M_FWD)) {
      __syncthreads();
      row_steady<T, N, NT, RB, P>(buf, tw, g, d, voff0, nrows);
      return;
    }
  }
  for (int idx = threadIdx.x; idx < RB * N; idx += NT) {
    const int r = idx / N, c = idx - r * N;
    C<T> v = mkc<T>(0, 0);
    if (r < nrows) {
      v = g[idx];
      if (mode & M_PRE) v = vmul_t<T>(v, d.hfac, d.vcomplex, row_site<T, N>(voff0, idx));
    }
    buf[r * P + padn(c)] = v;
  }
  __syncthreads();
  using Rows = RowsGeo<RB, P>;
  if (mode & M_INV) fft_lines_t<T, N, true, Rows, NT>(buf, tw);
  if (mode & M_MID) {
    for (int idx = threadIdx.x; idx < nrows * N; idx += NT) {
      const int r = idx / N, c = idx - r * N;
      const int a = r * P + padn(c);
      buf[a] = vmul_t<T>(buf[a], d.h2fac, d.vcomplex, row_site<T, N>(voff0, idx));
    }
    __syncthreads();
  }
  if (mode & M_FWD) fft_lines_t<T, N, false, Rows, NT>(buf, tw);
  for (int idx = threadIdx.x; idx < nrows * N; idx += NT) {
    const int r = idx / N, c = idx - r * N;
    C<T> v = buf[r * P + padn(c)];
    if (mode & M_POST) v = vmul_t<T>(v, d.hfac, d.vcomplex, row_site<T, N>(voff0, idx));
    g[idx] = v;
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(LINE_THREADS) k_row_t(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int e = find_entry(L, blockIdx.x);
  row_body<T, N, LINE_THREADS>(L, e, blockIdx.x - L.tile_start[e], smem);
}

// ------------------------------------------------------------ column pass

template <int NL, int PC> struct TileGeo {
  static constexpr int nlines = NL;
  static constexpr bool linefast = true;
  static __device__ __forceinline__ int at(int b, int n) { return n * PC + b; }
};

// Steady-state column pass (forward -> x e^{-dt T}/N^3 -> inverse) with the
// first stage read from HBM, the last written to HBM, and the forward last
// stage, the kinetic factor and the inverse first stage fused in registers.
template <typename T, int N, int NT, class Geo>
__device__ __forceinline__ void col_steady(C<T> *buf, const C<T> *tw, C<T> *g, size_t S, const PassDesc &d, bool ax1,
                                           int o, int c0, int nc) {
  constexpr RPlan PL = plan_of<T, N, false>();
  constexpr int M = PL.n - 1;
  constexpr int TC = Geo::nlines;
  const C<T> zero = mkc<T>(0, 0);
  {
    constexpr int R = PL.r[0];
    C<T> v[SG<Geo, N, R, NT>::CAPQ][R];
    st_read<T, N, R, 1, false, Geo, NT, 0>(
        v, tw, [&](int b, int n) { return (N % TC == 0 || b < nc) ? g[(size_t)n * S + b] : zero; });
    st_write<T, N, R, 1, Geo, NT>(v, [&](int b, int n, C<T> x) { buf[Geo::at(b, n)] = x; });
    __syncthreads();
  }
  lds_stages<T, N, false, false, Geo, NT, 1, M>(buf, tw);
  {
    constexpr int R = PL.r[M];
    constexpr int NSL = ns_before<T, N, false, M>();
    using SS = SG<Geo, N, R, NT>;
    C<T> v[SS::CAPQ][R];
    st_read<T, N, R, NSL, false, Geo, NT, tw_off<T, N, false, M>()>(v, tw, [&](int b, int n) { return buf[Geo::at(b, n)]; });
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SS::CAPQ; ++q) {
      if (SS::active(q)) {
        int j, b;
        SS::jb(q, j, b);
        const int i3 = (N % TC == 0 || b < nc) ? c0 + b : c0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int n = j + r * SS::NR;
          v[q][r] = cscale(v[q][r], kin_factor_t<T>(d, ax1 ? n : o, ax1 ? o : n, i3));
        }
        Dft<R, true, C<T>>::run(v[q]);
      }
    }
    st_write<T, N, R, 1, Geo, NT>(v, [&](int b, int n, C<T> x) { buf[Geo::at(b, n)] = x; });
    __syncthreads();
  }
  lds_stages<T, N, true, true, Geo, NT, 1, M>(buf, tw);
  {
    constexpr int R = plan_of<T, N, true>().r[M];
    constexpr int NSL = ns_before<T, N, true, M>();
    C<T> v[SG<Geo, N, R, NT>::CAPQ][R];
    st_read<T, N, R, NSL, true, Geo, NT, tw_off<T, N, true, M>()>(v, tw, [&](int b, int n) { return buf[Geo::at(b, n)]; });
    st_write<T, N, R, NSL, Geo, NT>(v, [&](int b, int n, C<T> x) {
      if (N % TC == 0 || b < nc) g[(size_t)n * S + b] = x;
    });
  }
}

// Column pass in one direction only (forward, or inverse with optional 1/N^3):
// first stage from HBM, last stage to HBM.
template <typename T, int N, int NT, class Geo, bool INV>
__device__ __forceinline__ void col_single(C<T> *buf, const C<T> *tw, C<T> *g, size_t S, int nc, T post) {
  constexpr RPlan PL = plan_of<T, N, false>();
  constexpr int M = PL.n - 1;
  constexpr int TC = Geo::nlines;
  const C<T> zero = mkc<T>(0, 0);
  {
    constexpr int R = PL.r[0];
    C<T> v[SG<Geo, N, R, NT>::CAPQ][R];
    st_read<T, N, R, 1, INV, Geo, NT, 0>(
        v, tw, [&](int b, int n) { return (N % TC == 0 || b < nc) ? g[(size_t)n * S + b] : zero; });
    st_write<T, N, R, 1, Geo, NT>(v, [&](int b, int n, C<T> x) { buf[Geo::at(b, n)] = x; });
    __syncthreads();
  }
  lds_stages<T, N, false, INV, Geo, NT, 1, M>(buf, tw);
  {
    constexpr int R = PL.r[M];
    constexpr int NSL = ns_before<T, N, false, M>();
    C<T> v[SG<Geo, N, R, NT>::CAPQ][R];
    st_read<T, N, R, NSL, INV, Geo, NT, tw_off<T, N, false, M>()>(v, tw, [&](int b, int n) { return buf[Geo::at(b, n)]; });
    st_write<T, N, R, NSL, Geo, NT>(v, [&](int b, int n, C<T> x) {
      if (N % TC == 0 || b < nc) g[(size_t)n * S + b] = cscale(x, post);
    });
  }
}

// Tile = TC contiguous x3 columns at one position of the other transverse
// axis; all N elements along the transform axis (x1 if M_AXIS1, else x2).
template <typename T, int N, int NT>
__device__ __forceinline__ void col_body(const LaunchList &L, int e, int t, unsigned char *smem) {
  constexpr int TC = col_tile_t<T>();
  constexpr int PC = TC + 1;
  constexpr int NCB = (N + TC - 1) / TC;
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  constexpr int per_state = N * NCB;
  const int s = t / per_state;
  const int rem = t - s * per_state;
  const int o = rem / NCB, cb = rem - o * NCB;
  const bool ax1 = (mode & M_AXIS1) != 0;
  const size_t S = ax1 ? (size_t)N * N : (size_t)N;
  const size_t OS = ax1 ? (size_t)N : (size_t)N * N;
  const int c0 = cb * TC;
  C<T> *buf = (C<T> *)smem;
  C<T> *tw = buf + N * PC;
  load_tw<T, N, NT>(tw, d);
  C<T> *g = (C<T> *)((mode & M_ALT) ? d.alt : d.psi) + (size_t)s * N * N * N + (size_t)o * OS + c0;
  using Geo = TileGeo<TC, PC>;
  if constexpr (plan_of<T, N, false>().n >= 2) {
    const int nc = (N - c0) < TC ? (N - c0) : TC;
    const uint32_t m3 = mode & (M_FWD | M_KIN | M_INV);
    if (m3 == (M_FWD | M_KIN | M_INV) && !(mode & M_SCALE)) {
      col_steady<T, N, NT, Geo>(buf, tw, g, S, d, ax1, o, c0, nc);
      return;
    }
    if (m3 == M_FWD || m3 == M_INV) {
      const T post = (mode & M_SCALE) ? (T)d.inv_n3 : (T)1;
      if (m3 == M_FWD) col_single<T, N, NT, Geo, false>(buf, tw, g, S, nc, post);
      else col_single<T, N, NT, Geo, true>(buf, tw, g, S, nc, post);
      return;
    }
  }
  for (int idx = threadIdx.x; idx < N * TC; idx += NT) {
    const int n = idx / TC, c = idx - n * TC;
    C<T> v = mkc<T>(0, 0);
    if (N % TC == 0 || c0 + c < N) v = g[(size_t)n * S + c];
    buf[n * PC + c] = v;
  }
  __syncthreads();
  if (mode & M_FWD) fft_lines_t<T, N, false, Geo, NT>(buf, tw);
  if (mode & M_KIN) {
    for (int idx = threadIdx.x; idx < N * TC; idx += NT) {
      const int n = idx / TC, c = idx - n * TC;
      const int i1 = ax1 ? n : o, i2 = ax1 ? o : n;
      const int i3 = (N % TC == 0 || c0 + c < N) ? c0 + c : c0;
      const int a = n * PC + c;
      buf[a] = cscale(buf[a], kin_factor_t<T>(d, i1, i2, i3));
    }
    __syncthreads();
  }
  if (mode & M_INV) fft_lines_t<T, N, true, Geo, NT>(buf, tw);
  const T post = (mode & M_SCALE) ? (T)d.inv_n3 : (T)1;
  for (int idx = threadIdx.x; idx < N * TC; idx += NT) {
    const int n = idx / TC, c = idx - n * TC;
    if (N % TC == 0 || c0 + c < N) g[(size_t)n * S + c] = cscale(buf[n * PC + c], post);
  }
}

// Block order of the column passes.  From N = 192 up the states no longer fit the 256 MB
// on-package cache, and runs of 64 consecutive tiles per XCD (the x3 tiles of neighbouring x2
// rows) turn a row's scattered 128-byte segments into longer runs per XCD: 153 against 168 us
// per launch at 256^3 x 3 states.  Below that size the plain order is as fast or faster.
constexpr int COL_XCD_MIN_N = 192, COL_XCD_RUN = 64;
__device__ __forceinline__ int col_block(int N) {
  return N >= COL_XCD_MIN_N ? xcd_block_chunked(blockIdx.x, gridDim.x, COL_XCD_RUN) : (int)blockIdx.x;
}

template <typename T, int N>
__global__ void __launch_bounds__(LINE_THREADS) k_col_t(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int blk = col_block(N);
  const int e = find_entry(L, blk);
  col_body<T, N, LINE_THREADS>(L, e, blk - L.tile_start[e], smem);
}

// ------------------------------------------------- slab and pencil passes (split x2)
//
// For large N the x2 transform is split four-step style, N = N1 N2 with i2 = N2 a + b
// (a < N1, b < N2):
//   forward  A (slab pass):   Y[k1][b] = W_N^{b k1} sum_a x[N2 a + b] W_N1^{a k1}, stored at row N2 k1 + b;
//            B (pencil pass): X[k1 + N1 k2] = sum_b Y[k1][b] W_N2^{b k2},        stored at row N2 k1 + k2;
//   inverse  B^-1 then A^-1 with conjugate roots, on the same rows.
// The slab pass holds the N1 rows {N2 a + b} of one x1 plane (b fixed): A^-1, the x3
// transforms around the potential factor, A.  The pencil pass holds the N2 consecutive rows
// N2 k1 .. N2 k1 + N2 - 1 of TT consecutive x3 columns over all x1: B, the x1 transforms
// around the kinetic factor (x2 frequency k1 + N1 k2 at row N2 k1 + k2), B^-1.  One step is
// then two passes over the state (a pencil pass and a slab pass) instead of a row pass and
// three column passes.  Between the passes of a chunk the state is held in this split x2
// order; the chunk's first and last slab passes take it from and return it to real space
// in natural order.
//
// Plane groups.  Between the passes the XI x1 planes XI p .. XI p + XI - 1 of a group are also
// interleaved: the memory of row r of plane XI p + j (its "row slot" j) holds columns
// j N/XI .. (j + 1) N/XI - 1 of all XI planes of the group, column j N/XI + w / XI of plane
// XI p + w mod XI at element w.  A pencil tile's (x1, row) piece then spans XI times the bytes of
// its TT columns, and a slab tile, which holds the N1 rows of all planes of a group, reads and
// writes exactly the memory of those rows in either order (the in-place chunk-edge passes that
// convert from and to natural order touch no other tile's memory).

template <typename T, int N, int N1, int XI> __host__ __device__ constexpr size_t slab_lds_t() {
  return (size_t)(XI * N1 * padded_len(N) + 8 * (XI - 1) + tw_total<T, N>() + N1) * sizeof(C<T>);
}
// Lines of a slab tile: row a of the group's plane j is line j N1 + a, and the lines of plane j start
// 8 j elements (64 bytes) further, so that the A stages' lanes, which alternate between the planes
// of one column, fall on distinct LDS banks (N1 P elements is a multiple of 128 bytes at N1 = 16).
template <int NL, int P, int N1, int XI> struct SlabGeo {
  static constexpr int nlines = NL;
  static constexpr bool linefast = false;
  static __device__ __forceinline__ int at(int b, int n) {
    if constexpr (XI == 1) return b * P + padn(n);
    else return b * P + (b / N1) * 8 + padn(n);
  }
};
// Pencil tile in LDS: element n (x1) of line l = k2 TT + c at n PC + l.  PC = lines + 4 (+ 4 more
// where that is a multiple of 32) puts the 16 lanes of one 128-byte LDS pass (4 x1 positions x 4
// columns, or 8 x 2) on distinct banks when the B stage writes its outputs.
template <int N2, int TT> __host__ __device__ constexpr int pencil_pitch() {
  return N2 * TT + 4 + ((N2 * TT + 4) % 32 == 0 ? 4 : 0);
}
template <typename T, int N, int N2, int TT> __host__ __device__ constexpr size_t pencil_lds_t() {
  return (size_t)(N * pencil_pitch<N2, TT>() + tw_total<T, N>()) * sizeof(C<T>) + N * sizeof(T);
}

// Loads and stores of one state with a block-uniform base and a 32-bit per-lane byte offset.
// The base goes through readfirstlane, so the compiler holds it (plus any uniform offset) in
// scalar registers and each access needs one 32-bit offset register instead of a 64-bit address:
// a lane keeps one access per x2 row of a split-x2 stage in flight.
// With G the pointer is taken in the global address space and each row's uniform offset is kept in a
// scalar register (the empty asm stops the compiler from folding it into a 64-bit vector address),
// so the accesses can use the global forms; without G they are flat accesses.  The slab pass
// measured faster with the global forms, the pencil pass with flat ones.
template <typename T, bool G = false> struct StateBuf {
  typedef __attribute__((address_space(1))) char gchar;
  typedef T pair_t __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(1))) pair_t gelem;
  const char *base;
  __device__ __forceinline__ explicit StateBuf(const void *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    base = (const char *)(((uint64_t)hi << 32) | lo);
  }
  __device__ __forceinline__ gchar *grow(uint32_t soff) const {
    asm volatile("" : "+s"(soff));
    return (gchar *)base + soff;
  }
  __device__ __forceinline__ C<T> load(uint32_t voff, uint32_t soff) const {
    if constexpr (G) {
      const pair_t v = *(const gelem *)(grow(soff) + voff);
      return mkc<T>(v.x, v.y);
    } else {
      return *(const C<T> *)(base + soff + voff);
    }
  }
  __device__ __forceinline__ void store(C<T> x, uint32_t voff, uint32_t soff) const {
    if constexpr (G) {
      pair_t v;
      v.x = x.x;
      v.y = x.y;
      *(gelem *)(grow(soff) + voff) = v;
    } else {
      *(C<T> *)(const_cast<char *>(base) + soff + voff) = x;
    }
  }
};

// Slab pass on tile (plane group p, fast x2 digit b), for each state of the member in turn, so that
// the potential factor rows of the tile are read from HBM once for all k states (or, with the
// entry's aux = 1, for one state per tile: k times the tiles, each reading the factor rows).  The
// tile's LDS holds row a of the group's plane j as line j N1 + a.  Steady mode
// (M_INV | M_MID | M_FWD, EDGE false): A^-1 from HBM, inverse x3, x h^2 (fused with the last
// inverse and first forward stages), forward x3, A to HBM.  The other modes (EDGE true, a kernel of
// its own so that its registers do not weigh on the steady pass): chunk start (M_PRE | M_FWD: x h,
// forward x3, A), chunk end (M_INV | M_POST: A^-1, inverse x3, x h) and plain transforms.  M_INV
// reads the split order, M_FWD writes it; otherwise the state is read or written in natural order.
template <typename T, int N, int N1, int NT, int XI, bool EDGE>
__device__ __forceinline__ void slab_body(const LaunchList &L, int e, int t, unsigned char *smem) {
  constexpr int N2 = N / N1;
  constexpr int P = padded_len(N);
  constexpr int NR = XI * N1;               // LDS lines of a tile
  constexpr int NH = N / XI;                // columns of each plane in one row slot
  constexpr int NP = XI * N;                // (row slot, element) positions of one row
  constexpr int CQ = (NP + NT - 1) / NT;    // positions per thread in the A stages
  constexpr int TPS = (N / XI) * N2;        // tiles per state
  using Rows = SlabGeo<NR, P, N1, XI>;
  constexpr RPlan PL = plan_of<T, N, false>();
  constexpr int M = PL.n - 1;
  static_assert(N % N1 == 0 && N % XI == 0 && PL.n >= 2, "slab pass needs N1 | N, XI | N and a plan of two or more stages");
  static_assert(sizeof(T) == 4 && (size_t)N * N * N * 8 < (1ull << 31), "complex64 states below 2 GiB");
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  // aux 1: one state per tile (tiles of state s follow those of state s - 1), else all k states
  int s0 = 0, s1 = d.k;
  if (L.aux[e] == 1) {
    s0 = t / TPS;
    s1 = s0 + 1;
    t -= s0 * TPS;
  }
  const int p = t / N2, b = t - (t / N2) * N2;
  // the twiddle tables first, so that their addresses fit the LDS instructions' offset field
  C<T> *tw = (C<T> *)smem;
  C<T> *wab = tw + tw_total<T, N>();       // W_N^{b k1}, k1 < N1: the twiddles of A
  C<T> *buf = wab + N1;
  load_tw<T, N, NT>(tw, d);
  for (int k1 = threadIdx.x; k1 < N1; k1 += NT) wab[k1] = ((const C<T> *)d.tw)[(b * k1) % N];
  constexpr size_t N3 = (size_t)N * N * N;
  const size_t voff = (size_t)XI * p * N * N;    // the group's first plane
  const bool vc = d.vcomplex != 0;
  // offset from the group's first plane of row N2 a + b of plane (or row slot) j, element n
  auto site = [&](int j, int a, int n) -> size_t { return ((size_t)j * N + N2 * a + b) * N + n; };
  auto fac = [&](const void *f, size_t o) -> C<T> {
    return vc ? ((const C<T> *)f)[voff + o] : mkc<T>(((const T *)f)[voff + o], 0);
  };
  // A^-1: the N1 values of each (row slot, element) position, conj twiddles, inverse DFT over k1,
  // to the LDS lines of the position's plane and column
  auto a_inverse_to_lds = [&](const C<T> *g) {
    const StateBuf<T, true> sb(g);
#pragma unroll
    for (int q = 0; q < CQ; ++q) {
      const int pos = (int)threadIdx.x + q * NT;
      if (NP % NT == 0 || pos < NP) {
        const int j = pos / N, w = pos - (pos / N) * N;
        const int pl = w % XI, col = j * NH + w / XI;
        C<T> v[N1];
        const uint32_t vo = (uint32_t)(site(j, 0, w) * sizeof(C<T>));
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) v[k1] = sb.load(vo, (uint32_t)(k1 * N2 * N * sizeof(C<T>)));
#pragma unroll
        for (int k1 = 1; k1 < N1; ++k1) {
          C<T> w1 = wab[k1];
          w1.y = -w1.y;
          v[k1] = cmul(v[k1], w1);
        }
        Dft<N1, true, C<T>>::run(v);
#pragma unroll
        for (int a = 0; a < N1; ++a) buf[Rows::at(pl * N1 + a, col)] = v[a];
      }
    }
  };
  // A: columns from the LDS lines, DFT over a, twiddles, to HBM at rows N2 k1 + b
  auto a_forward_from_lds = [&](C<T> *g) {
    const StateBuf<T, true> sb(g);
#pragma unroll
    for (int q = 0; q < CQ; ++q) {
      const int pos = (int)threadIdx.x + q * NT;
      if (NP % NT == 0 || pos < NP) {
        const int j = pos / N, w = pos - (pos / N) * N;
        const int pl = w % XI, col = j * NH + w / XI;
        C<T> v[N1];
#pragma unroll
        for (int a = 0; a < N1; ++a) v[a] = buf[Rows::at(pl * N1 + a, col)];
        Dft<N1, false, C<T>>::run(v);
#pragma unroll
        for (int k1 = 1; k1 < N1; ++k1) v[k1] = cmul(v[k1], wab[k1]);
        const uint32_t vo = (uint32_t)(site(j, 0, w) * sizeof(C<T>));
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) sb.store(v[k1], vo, (uint32_t)(k1 * N2 * N * sizeof(C<T>)));
      }
    }
  };
  if constexpr (!EDGE) {
  // every mode; the steady one fused (the API sends the other modes to the EDGE kernel)
  if (mode == (M_INV | M_MID | M_FWD)) {
    constexpr int RM = PL.r[M];
    using SS = SG<Rows, N, RM, NT>;
    // potential factors of the fused middle stage, held in registers for all k states (one
    // fetch per tile)
    C<T> hq[SS::CAPQ][RM];
#pragma unroll
    for (int q = 0; q < SS::CAPQ; ++q) {
      if (SS::active(q)) {
        int j, bl;
        SS::jb(q, j, bl);
        const int pl = bl / N1, a = bl - (bl / N1) * N1;
#pragma unroll
        for (int r = 0; r < RM; ++r) hq[q][r] = fac(d.h2fac, site(pl, a, j + r * SS::NR));
      }
    }
    for (int s = s0; s < s1; ++s) {
      C<T> *g = (C<T> *)d.psi + (size_t)s * N3 + voff;
      __syncthreads();     // the twiddle tables; the previous state's reads of the LDS rows
      a_inverse_to_lds(g);
      __syncthreads();
      lds_stages<T, N, false, true, Rows, NT, 0, M>(buf, tw);
      {
        constexpr int NSL = ns_before<T, N, false, M>();
        C<T> v[SS::CAPQ][RM];
        st_read<T, N, RM, NSL, true, Rows, NT, tw_off<T, N, false, M>()>(
            v, tw, [&](int bl, int n) { return buf[Rows::at(bl, n)]; });
        __syncthreads();
#pragma unroll
        for (int q = 0; q < SS::CAPQ; ++q) {
          if (SS::active(q)) {
#pragma unroll
            for (int r = 0; r < RM; ++r) v[q][r] = vc ? cmul(v[q][r], hq[q][r]) : cscale(v[q][r], hq[q][r].x);
            Dft<RM, false, C<T>>::run(v[q]);
          }
        }
        st_write<T, N, RM, 1, Rows, NT>(v, [&](int bl, int n, C<T> x) { buf[Rows::at(bl, n)] = x; });
        __syncthreads();
      }
      lds_stages<T, N, true, false, Rows, NT, 1, PL.n>(buf, tw);
      a_forward_from_lds(g);
    }
    return;
  }
  for (int s = s0; s < s1; ++s) {
    C<T> *g = (C<T> *)d.psi + (size_t)s * N3 + voff;
    __syncthreads();       // the twiddle tables; the previous state's reads of the LDS rows
    if (mode & M_INV) {
      a_inverse_to_lds(g);
    } else {
      for (int idx = threadIdx.x; idx < NR * N; idx += NT) {
        const int bl = idx / N, n = idx - bl * N;
        const int pl = bl / N1, a = bl - pl * N1;
        C<T> v = g[site(pl, a, n)];
        if (mode & M_PRE) {
          const C<T> h = fac(d.hfac, site(pl, a, n));
          v = vc ? cmul(v, h) : cscale(v, h.x);
        }
        buf[Rows::at(bl, n)] = v;
      }
    }
    __syncthreads();
    if (mode & M_INV) fft_lines_t<T, N, true, Rows, NT>(buf, tw);
    if (mode & (M_MID | M_POST)) {
      for (int idx = threadIdx.x; idx < NR * N; idx += NT) {
        const int bl = idx / N, n = idx - bl * N;
        const int pl = bl / N1, a = bl - pl * N1;
        const C<T> h = fac((mode & M_MID) ? d.h2fac : d.hfac, site(pl, a, n));
        const int o = Rows::at(bl, n);
        buf[o] = vc ? cmul(buf[o], h) : cscale(buf[o], h.x);
      }
      __syncthreads();
    }
    if (mode & M_FWD) {
      fft_lines_t<T, N, false, Rows, NT>(buf, tw);
      a_forward_from_lds(g);
    } else {
      for (int idx = threadIdx.x; idx < NR * N; idx += NT) {
        const int bl = idx / N, n = idx - bl * N;
        const int pl = bl / N1, a = bl - pl * N1;
        g[site(pl, a, n)] = buf[Rows::at(bl, n)];
      }
    }
  }
  } else {
  // Natural-order tile accesses (chunk edges, plain transforms): each thread takes elements
  // threadIdx.x + it NT, UB at a time, with all UB global loads issued before they are used.
  constexpr int NE = NR * N;
  constexpr int EPT = (NE + NT - 1) / NT;
  constexpr int UB = EPT < 8 ? EPT : 8;
  // state rows (times the factor f if given) to the LDS lines
  auto natural_to_lds = [&](const C<T> *g, const void *f) {
    const StateBuf<T, true> sb(g);
#pragma unroll 1
    for (int it0 = 0; it0 < EPT; it0 += UB) {
      C<T> v[UB], h[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int idx = (int)threadIdx.x + (it0 + u) * NT;
        if (it0 + u < EPT && (NE % NT == 0 || idx < NE)) {
          const int bl = idx / N, n = idx - bl * N, pl = bl / N1, a = bl - pl * N1;
          v[u] = sb.load((uint32_t)(site(pl, a, n) * sizeof(C<T>)), 0);
          if (f) h[u] = fac(f, site(pl, a, n));
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int idx = (int)threadIdx.x + (it0 + u) * NT;
        if (it0 + u < EPT && (NE % NT == 0 || idx < NE)) {
          const int bl = idx / N, n = idx - bl * N;
          C<T> x = v[u];
          if (f) x = vc ? cmul(x, h[u]) : cscale(x, h[u].x);
          buf[Rows::at(bl, n)] = x;
        }
      }
    }
  };
  // LDS lines (times the factor f if given) to the state rows
  auto lds_to_natural = [&](C<T> *g, const void *f) {
    const StateBuf<T, true> sb(g);
#pragma unroll 1
    for (int it0 = 0; it0 < EPT; it0 += UB) {
      C<T> h[UB];
      if (f) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int idx = (int)threadIdx.x + (it0 + u) * NT;
          if (it0 + u < EPT && (NE % NT == 0 || idx < NE)) {
            const int bl = idx / N, n = idx - bl * N, pl = bl / N1, a = bl - pl * N1;
            h[u] = fac(f, site(pl, a, n));
          }
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int idx = (int)threadIdx.x + (it0 + u) * NT;
        if (it0 + u < EPT && (NE % NT == 0 || idx < NE)) {
          const int bl = idx / N, n = idx - bl * N, pl = bl / N1, a = bl - pl * N1;
          C<T> x = buf[Rows::at(bl, n)];
          if (f) x = vc ? cmul(x, h[u]) : cscale(x, h[u].x);
          sb.store(x, (uint32_t)(site(pl, a, n) * sizeof(C<T>)), 0);
        }
      }
    }
  };
  const void *fmid = (mode & M_MID) ? d.h2fac : (mode & M_POST) ? d.hfac : nullptr;
  for (int s = s0; s < s1; ++s) {
    C<T> *g = (C<T> *)d.psi + (size_t)s * N3 + voff;
    __syncthreads();       // the twiddle tables; the previous state's reads of the LDS rows
    if (mode & M_INV) a_inverse_to_lds(g);
    else natural_to_lds(g, (mode & M_PRE) ? d.hfac : nullptr);
    __syncthreads();
    if (mode & M_INV) fft_lines_t<T, N, true, Rows, NT>(buf, tw);
    if (mode & M_FWD) {
      if (fmid) {
        for (int idx = threadIdx.x; idx < NE; idx += NT) {
          const int bl = idx / N, n = idx - bl * N;
          const int pl = bl / N1, a = bl - pl * N1;
          const C<T> h = fac(fmid, site(pl, a, n));
          const int o = Rows::at(bl, n);
          buf[o] = vc ? cmul(buf[o], h) : cscale(buf[o], h.x);
        }
        __syncthreads();
      }
      fft_lines_t<T, N, false, Rows, NT>(buf, tw);
      a_forward_from_lds(g);
    } else {
      // the factor of the chunk end (or a middle factor) is applied on the way out
      lds_to_natural(g, fmid);
    }
  }
  }
}

// Pencil pass on tile (state s, slow x2 frequency k1, x3 columns c0 .. c0 + TT - 1), steady
// mode only (B, forward x1, x e^{-dt T(k)}/N^3, inverse x1, B^-1): the chunk's slab passes
// bracket every pencil pass.  The state is in split order with plane groups of XI.
template <typename T, int N, int N2, int TT, int NT, int XI>
__device__ __forceinline__ void pencil_body(const LaunchList &L, int e, int t, unsigned char *smem) {
  constexpr int N1 = N / N2;
  constexpr int NH = N / XI;
  constexpr int NL = N2 * TT;
  constexpr int PC = pencil_pitch<N2, TT>();
  constexpr int NCB = N / TT;
  constexpr int PPT = (N * TT + NT - 1) / NT;    // (x1, column) positions per thread in the B stages
  using Geo = TileGeo<NL, PC>;
  constexpr RPlan PL = plan_of<T, N, false>();
  constexpr int M = PL.n - 1;
  static_assert(N % N2 == 0 && N % TT == 0 && N % XI == 0 && N % 2 == 0 && PL.n >= 2, "pencil tile must divide the lattice");
  static_assert(sizeof(T) == 4 && (size_t)N * N * N * 8 < (1ull << 31), "complex64 states below 2 GiB");
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const int cb = t % NCB;
  const int u = t / NCB;
  const int k1 = u % N1, s = u / N1;
  const int c0 = cb * TT;
  // the twiddle and kinetic tables first, so that their addresses fit the LDS instructions'
  // offset field
  C<T> *tw = (C<T> *)smem;
  T *ktl = (T *)(tw + tw_total<T, N>());      // the per-axis kinetic table
  C<T> *buf = (C<T> *)(ktl + N);
  load_tw<T, N, NT>(tw, d);
  for (int i = threadIdx.x; i < N; i += NT) ktl[i] = ((const T *)d.ktab)[i];
  constexpr size_t N3 = (size_t)N * N * N;
  const StateBuf<T> sb((C<T> *)d.psi + (size_t)s * N3);
  // the k-space factor of kin_factor_t, with the table read from LDS
  const bool rel = d.kin == KIN_REL, ab = d.scheme == SCHEME_AB;
  const T mm = (T)d.m, dtT = (T)d.dt, in3 = (T)d.inv_n3, dtn = (T)(d.dt * d.inv_n3);
  auto kfac = [&](int i1, int i2, int i3) -> T {
    if (rel) {
      const T p2 = ktl[i1] + ktl[i2] + ktl[i3];
      const float r = __builtin_amdgcn_sqrtf(p2 + mm * mm);
      if (ab) return p2 * __builtin_amdgcn_rcpf(r + mm) * dtn;
      return __builtin_amdgcn_exp2f(-dtT * 1.4426950408889634f * (r - mm)) * in3;
    }
    if (ab) return (ktl[i1] + ktl[i2] + ktl[i3]) * dtn;
    return ktl[i1] * ktl[i2] * ktl[i3] * in3;
  };
  // byte offset of (x1 plane i1, row N2 k1, column c0 + c): row slot (c0 + c) / NH of the plane
  // group, element XI ((c0 + c) mod NH) + i1 mod XI; rows b apart by b N elements
  auto at = [&](int i1, int c) -> uint32_t {
    const int col = c0 + c, j = col / NH, w = XI * (col - j * NH) + i1 % XI;
    return (uint32_t)((((size_t)(i1 - i1 % XI + j) * N + (size_t)(N2 * k1)) * N + w) * sizeof(C<T>));
  };
  __syncthreads();       // the twiddle tables
  // B: DFT over the N2 rows of each (x1, column) position, outputs to the x1 lines (k2, c)
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pos = (int)threadIdx.x + q * NT;
    if ((N * TT) % NT == 0 || pos < N * TT) {
      const int i1 = pos / TT, c = pos - (pos / TT) * TT;
      C<T> v[N2];
#pragma unroll
      for (int bb = 0; bb < N2; ++bb) v[bb] = sb.load(at(i1, c), (uint32_t)(bb * N * sizeof(C<T>)));
      Dft<N2, false, C<T>>::run(v);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) buf[Geo::at(k2 * TT + c, i1)] = v[k2];
    }
  }
  __syncthreads();
  lds_stages<T, N, false, false, Geo, NT, 0, M>(buf, tw);
  {
    constexpr int R = PL.r[M];
    constexpr int NSL = ns_before<T, N, false, M>();
    using SS = SG<Geo, N, R, NT>;
    C<T> v[SS::CAPQ][R];
    st_read<T, N, R, NSL, false, Geo, NT, tw_off<T, N, false, M>()>(v, tw, [&](int l, int n) { return buf[Geo::at(l, n)]; });
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SS::CAPQ; ++q) {
      if (SS::active(q)) {
        int j, l;
        SS::jb(q, j, l);
        const int k2 = l / TT, c = l - (l / TT) * TT;
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = cscale(v[q][r], kfac(j + r * SS::NR, k1 + N1 * k2, c0 + c));
        Dft<R, true, C<T>>::run(v[q]);
      }
    }
    st_write<T, N, R, 1, Geo, NT>(v, [&](int l, int n, C<T> x) { buf[Geo::at(l, n)] = x; });
    __syncthreads();
  }
  lds_stages<T, N, true, true, Geo, NT, 1, PL.n>(buf, tw);
  // B^-1: inverse DFT over k2 of each position, to the N2 rows in HBM
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pos = (int)threadIdx.x + q * NT;
    if ((N * TT) % NT == 0 || pos < N * TT) {
      const int i1 = pos / TT, c = pos - (pos / TT) * TT;
      C<T> v[N2];
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) v[k2] = buf[Geo::at(k2 * TT + c, i1)];
      Dft<N2, true, C<T>>::run(v);
#pragma unroll
      for (int bb = 0; bb < N2; ++bb) sb.store(v[bb], at(i1, c), (uint32_t)(bb * N * sizeof(C<T>)));
    }
  }
}

// Split-x2 shapes per size and variant (complex64): x2 = N1 x N2 (N1 stride rows per slab tile,
// N2 consecutive rows per pencil tile; both radices have register butterflies), TT x3 columns per
// pencil tile, and plane groups of XI (split_xi).  A pencil tile's (x1, row) pieces are
// XI TT 8 bytes.
//   variant 0: the size's default N1; 4 columns where 4 divides N (144 KiB of LDS at N = 256,
//              one tile per CU), else 2;
//   variant 1: the same N1; 2 columns (77 KiB at N = 256, two tiles per CU);
//   variant 2 (N = 128, 256): 8 consecutive rows (x2 = 16 x 8, 32 x 8) with 8 columns
//              (139 KiB at N = 256);
//   variant 3: the default factors swapped (x2 = N2 x N1: fewer rows per slab tile, more per
//              pencil tile), where they differ; columns as in variant 0 up to 16 pencil rows,
//              else 2.
// A slab tile has one thread per (row slot, element) position in its A stages (XI times 256 or
// 128 threads); a pencil tile one per (x1, column) position, at most 1024 (two positions per
// thread beyond).  Sizes or variants without a shape (N1 = 0) have no split-x2 kernels.
constexpr int SPLIT_VARIANTS = 4;
__host__ __device__ constexpr int split_n1_default(int N) {
  switch (N) {
    case 96: return 16;    // 16 x 6
    case 100: return 10;   // 10 x 10
    case 108: return 12;   // 12 x 9
    case 120: return 12;   // 12 x 10
    case 128: return 16;   // 16 x 8
    case 144: return 16;   // 16 x 9
    case 150: return 15;   // 15 x 10
    case 160: return 16;   // 16 x 10
    case 162: return 18;   // 18 x 9
    case 180: return 18;   // 18 x 10
    case 192: return 16;   // 16 x 12
    case 200: return 20;   // 20 x 10
    case 216: return 18;   // 18 x 12
    case 240: return 16;   // 16 x 15
    case 250: return 25;   // 25 x 10
    case 256: return 16;   // 16 x 16
    default: return 0;
  }
}
__host__ __device__ constexpr int split_n1(int N, int V) {
  if (V == 2) return N == 256 ? 32 : N == 128 ? 16 : 0;
  const int n1 = split_n1_default(N);
  if (V == 3) return (n1 > 0 && N / n1 != n1) ? N / n1 : 0;
  return n1;
}
// Planes per group of the split order (and per slab tile): pairs at the sizes where they measured
// faster.  With pairs the 2-column pencil tiles read 32-byte pieces two tiles per CU, and the slab
// tiles have twice the threads; at 192, 240 and 250 a pair tile's slab needs more than 128 VGPRs
// (one tile per CU) and at 150 and 180 pairs measured slower.
__host__ __device__ constexpr int split_xi(int N) { return (N == 128 || N == 160 || N == 256) ? 2 : 1; }
template <int N, int V> struct SplitShape {
  static constexpr int N1 = split_n1(N, V);
  static constexpr bool ok = N1 > 0;
  static constexpr int N2 = ok ? N / N1 : 1;
  static constexpr int XI = split_xi(N);
  static constexpr int SLAB_NT = XI * (N <= 128 ? 128 : 256);
  static constexpr int TT = V == 2 ? 8 : ((V == 0 || (V == 3 && N2 <= 16)) && N % 4 == 0) ? 4 : 2;
  static constexpr int PENCIL_NT = N * TT <= 1024 ? N * TT : 1024;
};

// Pencil block order: runs of consecutive x3 tiles per XCD, so that the pieces of one 128-byte
// row segment are fetched by blocks that share an L2.
constexpr int PENCIL_XCD_RUN = 128;

template <typename T, int N, int V>
__global__ void __launch_bounds__((SplitShape<N, V>::SLAB_NT)) k_slab_t(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  using SH = SplitShape<N, V>;
  const int e = find_entry(L, blockIdx.x);
  slab_body<T, N, SH::N1, SH::SLAB_NT, SH::XI, false>(L, e, blockIdx.x - L.tile_start[e], smem);
}
template <typename T, int N, int V>
__global__ void __launch_bounds__((SplitShape<N, V>::SLAB_NT)) k_slab_edge_t(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  using SH = SplitShape<N, V>;
  const int e = find_entry(L, blockIdx.x);
  slab_body<T, N, SH::N1, SH::SLAB_NT, SH::XI, true>(L, e, blockIdx.x - L.tile_start[e], smem);
}

template <typename T, int N, int V>
__global__ void __launch_bounds__((SplitShape<N, V>::PENCIL_NT)) k_pencil_t(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  using SH = SplitShape<N, V>;
  const int blk = xcd_block_chunked(blockIdx.x, gridDim.x, PENCIL_XCD_RUN);
  const int e = find_entry(L, blk);
  pencil_body<T, N, SH::N2, SH::TT, SH::PENCIL_NT, SH::XI>(L, e, blk - L.tile_start[e], smem);
}

template <int N, int V> void register_split(FftKernels &k) {
  if constexpr (SplitShape<N, V>::ok) {
    using SH = SplitShape<N, V>;
    k.slab[V] = (const void *)k_slab_t<float, N, V>;
    k.slab_edge[V] = (const void *)k_slab_edge_t<float, N, V>;
    k.slab_nt[V] = SH::SLAB_NT;
    k.slab_lds[V] = slab_lds_t<float, N, SH::N1, SH::XI>();
    k.split_n1[V] = SH::N1;
    k.split_xi[V] = SH::XI;
    k.pencil[V] = (const void *)k_pencil_t<float, N, V>;
    k.pencil_lds[V] = pencil_lds_t<float, N, SH::N2, SH::TT>();
    k.pencil_nt[V] = SH::PENCIL_NT;
    k.pencil_tt[V] = SH::TT;
  }
}

// ------------------------------------------------------------ dispatch table


template <int N> void register_size(FftKernels *tab) {
  static_assert(N > 128 || plane_fits<float, N>(), "complex64 planes up to N = 128 must fit LDS");
  static_assert(N > 96 || plane_fits<double, N>(), "complex128 planes up to N = 96 must fit LDS");
  FftKernels &k = tab[N];
  if constexpr (plane_fits<float, N>()) {
    k.plane[0] = (const void *)k_plane_t<float, N>;
    k.plane_lds[0] = plane_lds_t<float, N>();
  }
  if constexpr (plane_fits<double, N>()) {
    k.plane[1] = (const void *)k_plane_t<double, N>;
    k.plane_lds[1] = plane_lds_t<double, N>();
  }
  k.plane_nt = plane_threads<N>();
  k.row[0] = (const void *)k_row_t<float, N>;
  k.row[1] = (const void *)k_row_t<double, N>;
  k.row_lds[0] = row_lds_t<float, N>();
  k.row_lds[1] = row_lds_t<double, N>();
  k.col[0] = (const void *)k_col_t<float, N>;
  k.col[1] = (const void *)k_col_t<double, N>;
  k.col_lds[0] = col_lds_t<float, N>();
  k.col_lds[1] = col_lds_t<double, N>();
  register_split<N, 0>(k);
  register_split<N, 1>(k);
  register_split<N, 2>(k);
  register_split<N, 3>(k);
}

}  // namespace qf
