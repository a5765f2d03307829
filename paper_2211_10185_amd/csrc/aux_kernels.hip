// Setup, stencil, projection and FP64 measurement kernels.
//
//  k_twiddles     FP64 generation of roots of unity and kinetic symbols  (Sec. 2, text after HK3)
//  k_potential    FP64 V(r) on the lattice (harmonic, Cornell, Coulomb, radial spline, grid)
//  k_dt_tables    e^{-dt V/2}, e^{-dt V}, e^{-dt t(k_j)} for the current dt (FP64, stored
//                 in the state precision)
//  k_stencil      H_K^(0) step psi' = A psi + B dt/(2 M a^2) L psi            (Sec. 2, eq. HK0)
//  k_parity       P^+, P^-, P^-_{p_k} over reflection orbits                  (Sec. 3, Fig. 1 text)
//  k_gram ...     FP64 Gram matrix, Cholesky, Psi <- Psi R^{-1}              (Sec. 1: orthogonal projection)
//  k_energy_*     FP64 <psi|V|psi>, <psi|H_K|psi>, <psi|psi>                (Sec. 2, general solution)
//
// All reductions are two-level with a fixed grid and a fixed summation order,
// so repeated runs, and a member run alone or inside a batch, give identical bits.
#include "common.h"

namespace qf {

constexpr int EW_PER_THREAD = 4;   // sites per thread of the elementwise kernels

__host__ __device__ inline int ew_tiles(long long n) {
  long long per = (long long)RED_THREADS * EW_PER_THREAD;
  return (int)((n + per - 1) / per);
}

// ------------------------------------------------------------------ tables

// roots of unity w^m = e^{-2 pi i m/N}, FP64 and state precision; kinetic per-axis symbols
template <typename T>
__global__ void k_twiddles(C<T> *tw, double2 *tw64, double *ksym64, int N, int kin, double a, double m) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double s, c;
  sincospi(2.0 * (double)j / (double)N, &s, &c);
  tw64[j] = make_double2(c, -s);
  tw[j] = mkc<T>((T)c, (T)-s);
  // lattice momentum k = 2 pi j'/N with j' in (-N/2, N/2]
  const int jp = (j <= N / 2) ? j : j - N;
  const double k = 2.0 * M_PI * (double)jp / (double)N;
  const double sh = sinpi((double)jp / (double)N);   // sin(k/2)
  double v = 0.0;
  if (kin == KIN_P2) v = k * k / (2.0 * m * a * a);
  else if (kin == KIN_SIN2) v = 4.0 * sh * sh / (2.0 * m * a * a);
  else if (kin == KIN_REL) v = 4.0 * sh * sh / (a * a);
  ksym64[j] = v;
}

// Potential kinds (match the public header)
enum { PV_GRID = 0, PV_HARMONIC = 1, PV_CORNELL = 2, PV_COULOMB = 3, PV_SPLINE = 4 };

// knots: [nk] r, [nk] V, [nk] second derivatives of the natural spline
__device__ double spline_eval(const double *kn, int nk, double r) {
  const double *xr = kn, *yv = kn + nk, *M = kn + 2 * nk;
  int lo = 0, hi = nk - 2;
  while (lo < hi) {       // largest j <= nk-2 with x_j <= r (j = 0 below the first knot)
    int mid = (lo + hi + 1) >> 1;
    if (xr[mid] <= r) lo = mid; else hi = mid - 1;
  }
  const int j = lo;
  const double h = xr[j + 1] - xr[j];
  const double t0 = xr[j + 1] - r, t1 = r - xr[j];
  return (M[j] * t0 * t0 * t0 + M[j + 1] * t1 * t1 * t1) / (6.0 * h) + (yv[j] / h - M[j] * h / 6.0) * t0 +
         (yv[j + 1] / h - M[j + 1] * h / 6.0) * t1;
}

// v64: real [N^3] (vcomplex = 0) or complex [N^3] (vcomplex = 1); add: complex grid or null
__global__ void k_potential(double *v64, int vcomplex, int N, double a, int kind, double p0, double p1,
                            double p2, const double *knots, int nk, const double2 *add) {
  const size_t N3 = (size_t)N * N * N;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N3) return;
  const int i3 = (int)(g % N), i2 = (int)((g / N) % N), i1 = (int)(g / ((size_t)N * N));
  const double x1 = (i1 - N / 2) * a, x2 = (i2 - N / 2) * a, x3 = (i3 - N / 2) * a;
  const double r = sqrt(x1 * x1 + x2 * x2 + x3 * x3);
  double vr = 0.0, vi = 0.0;
  switch (kind) {
    case PV_HARMONIC: vr = 0.5 * p0 * r * r; break;
    case PV_CORNELL: { const double rf = fmax(r, p2); vr = -p0 / rf + p1 * rf; } break;
    case PV_COULOMB: { const double rf = fmax(r, p1); vr = -p0 / rf; } break;
    case PV_SPLINE: vr = spline_eval(knots, nk, r); break;
    default: break;
  }
  if (add) { vr += add[g].x; vi += add[g].y; }
  if (vcomplex) { v64[2 * g] = vr; v64[2 * g + 1] = vi; }
  else v64[g] = vr;
}

// state-precision V (FDTD), and e^{-dt V/2}, e^{-dt V} (FFT kinds) from the FP64 table
template <typename T>
__global__ void k_dt_tables(const double *v64, int vcomplex, size_t N3, double dt, void *vtab, void *hfac,
                            void *h2fac, T *ktab, const double *ksym64, int N, int kin, int scheme) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < (size_t)N && ktab) {
    // separable symbols: e^{-dt t(k_j)} (split step) or t(k_j) (A/B update);
    // relativistic: the lattice p^2 table itself
    const double ks = ksym64[g];
    ktab[g] = (T)((kin == KIN_REL || scheme == SCHEME_AB) ? ks : exp(-dt * ks));
  }
  if (g >= N3) return;
  const double vr = vcomplex ? v64[2 * g] : v64[g];
  const double vi = vcomplex ? v64[2 * g + 1] : 0.0;
  if (vtab) {
    if (vcomplex) ((C<T> *)vtab)[g] = mkc<T>((T)vr, (T)vi);
    else ((T *)vtab)[g] = (T)vr;
  }
  if (hfac) {
    const double e1 = exp(-0.5 * dt * vr), e2 = exp(-dt * vr);
    if (vcomplex) {
      double s1, c1, s2, c2;
      sincos(0.5 * dt * vi, &s1, &c1);
      sincos(dt * vi, &s2, &c2);
      ((C<T> *)hfac)[g] = mkc<T>((T)(e1 * c1), (T)(-e1 * s1));
      ((C<T> *)h2fac)[g] = mkc<T>((T)(e2 * c2), (T)(-e2 * s2));
    } else {
      ((T *)hfac)[g] = (T)e1;
      ((T *)h2fac)[g] = (T)e2;
    }
  }
}

// --------------------------------------------------------------- stencil

// psi' = A psi + B c (sum of 6 neighbours - 6 psi), c = dt/(2 m a^2),
// A = (1 - dt V/2)/(1 + dt V/2), B = 1/(1 + dt V/2); walls are ghost zeros.
//
// Tile = 64 (x3) x 16 (x2) columns of one state over ST_CZ planes along x1.
// Each wave owns 4 consecutive x2 rows, one x3 column per lane, and marches
// along x1 keeping psi at i1-1, i1, i1+1 of its 4 sites in registers.  x2
// neighbours come from the thread's own rows (memory only for the rows just
// outside its 4), x3 neighbours from the adjacent lanes by wavefront shifts
// (memory only at the tile's x3 edges), so each site is read from memory about
// once per sweep.  Loads of ST_ZU planes are issued together.
constexpr int ST_TX = 64, ST_RPT = 4, ST_TY = (RED_THREADS / 64) * ST_RPT, ST_CZ = 8, ST_ZU = 2;

__host__ __device__ inline int stencil_tiles(int N, int k) {
  return k * ((N + ST_TX - 1) / ST_TX) * ((N + ST_TY - 1) / ST_TY) * ((N + ST_CZ - 1) / ST_CZ);
}

// value of lane l-1 (DPP wave shift right by one; lane 0 gets 0)
__device__ __forceinline__ float lane_prev(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));
}
// value of lane l+1 (DPP wave shift left by one; lane 63 gets 0)
__device__ __forceinline__ float lane_next(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_prev(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_next(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, bool VC> struct VType { using type = T; };
template <typename T> struct VType<T, true> { using type = C<T>; };

template <typename T, bool VC>
__device__ __forceinline__ C<T> fdtd_update(C<T> cur, C<T> acc, typename VType<T, VC>::type V, T c, T hdt) {
  if constexpr (VC) {
    // B = 1/(1 + dt V/2), A = (1 - dt V/2) B
    const T dr = fmaT(hdt, V.x, (T)1), di = hdt * V.y;
    const T den = (T)1 / fmaT(dr, dr, di * di);
    const C<T> B = mkc<T>(dr * den, -di * den);
    const C<T> A = cmul(mkc<T>(fmaT(-hdt, V.x, (T)1), -hdt * V.y), B);
    return cadd(cmul(A, cur), cmul(B, cscale(acc, c)));
  } else {
    const T B = (T)1 / fmaT(hdt, V, (T)1);
    const T A = fmaT(-hdt, V, (T)1) * B;
    const T Bc = B * c;
    return mkc<T>(fmaT(A, cur.x, Bc * acc.x), fmaT(A, cur.y, Bc * acc.y));
  }
}

template <typename T, bool VC>
__device__ __forceinline__ typename VType<T, VC>::type load_v(const void *__restrict__ vtab, int off) {
  return ((const typename VType<T, VC>::type *)vtab)[off];
}

template <typename T, bool VC>
__device__ __forceinline__ void stencil_tile(const C<T> *__restrict__ sp, C<T> *__restrict__ dp,
                                             const void *__restrict__ vtab, int N, int y0, int i3, int lane,
                                             int z0, int z1, T c, T hdt) {
  const int N2 = N * N;
  const C<T> zero = mkc<T>(0, 0);
  const bool xin = i3 < N;
  bool rin[ST_RPT];
#pragma unroll
  for (int r = 0; r < ST_RPT; ++r) rin[r] = xin && (y0 + r < N);
  const bool up_ok = xin && y0 > 0, dn_ok = xin && y0 + ST_RPT < N;
  // x3 neighbour outside the wave: lane 0 needs i3-1, lane 63 needs i3+1
  const int xe_off = lane == 0 ? -1 : 1;
  const bool xe_mem = (lane == 0 && xin && i3 > 0) || (lane == 63 && i3 + 1 < N);
  const bool xr_wall = i3 + 1 >= N;
  using VT = typename VType<T, VC>::type;
  VT vzero;
  if constexpr (VC) vzero = zero; else vzero = (T)0;
  int off0 = (z0 * N + y0) * N + i3;                           // site (z0, y0, i3)
  C<T> prev[ST_RPT], cur[ST_RPT];
#pragma unroll
  for (int r = 0; r < ST_RPT; ++r) {
    prev[r] = (rin[r] && z0 > 0) ? sp[off0 + r * N - N2] : zero;
    cur[r] = rin[r] ? sp[off0 + r * N] : zero;
  }
  for (int z = z0; z < z1; z += ST_ZU) {
    C<T> nx[ST_ZU][ST_RPT], up[ST_ZU], dn[ST_ZU], xe[ST_ZU][ST_RPT];
    VT V[ST_ZU][ST_RPT];
#pragma unroll
    for (int u = 0; u < ST_ZU; ++u) {
      const int zz = z + u;
      const int o = off0 + (zz - z0) * N2;
      const bool zin = zz < z1;
#pragma unroll
      for (int r = 0; r < ST_RPT; ++r) {
        nx[u][r] = (rin[r] && zz + 1 < N && zin) ? sp[o + r * N + N2] : zero;
        V[u][r] = (rin[r] && zin) ? load_v<T, VC>(vtab, o + r * N) : vzero;
        xe[u][r] = (rin[r] && zin && xe_mem) ? sp[o + r * N + xe_off] : zero;
      }
      up[u] = (up_ok && zin) ? sp[o - N] : zero;
      dn[u] = (dn_ok && zin) ? sp[o + ST_RPT * N] : zero;
    }
#pragma unroll
    for (int u = 0; u < ST_ZU; ++u) {
      if (z + u >= z1) break;
      const int o = off0 + (z + u - z0) * N2;
#pragma unroll
      for (int r = 0; r < ST_RPT; ++r) {
        // x3 neighbours: adjacent lanes, or memory at the wave's edges, or the wall
        C<T> l = mkc<T>(lane_prev(cur[r].x), lane_prev(cur[r].y));
        C<T> rr = mkc<T>(lane_next(cur[r].x), lane_next(cur[r].y));
        if (lane == 0) l = xe[u][r];
        if (lane == 63) rr = xe[u][r];
        if (xr_wall) rr = zero;
        const C<T> yu = r > 0 ? cur[r - 1] : up[u];
        const C<T> yd = r < ST_RPT - 1 ? cur[r + 1] : dn[u];
        C<T> acc = csub(cadd(prev[r], nx[u][r]), cscale(cur[r], (T)6));
        acc = cadd(acc, cadd(cadd(l, rr), cadd(yu, yd)));
        if (rin[r]) dp[o + r * N] = fdtd_update<T, VC>(cur[r], acc, V[u][r], c, hdt);
      }
#pragma unroll
      for (int r = 0; r < ST_RPT; ++r) {
        prev[r] = cur[r];
        cur[r] = nx[u][r];
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_stencil(const LaunchList L) {
  // runs of 48 tiles per XCD: the states of a tile and its x2/x1 neighbours
  // meet in one L2 (shorter runs lose that at 128^3, one run per XCD loses
  // HBM-side balance at 256^3)
  const int blk = xcd_block_chunked(blockIdx.x, gridDim.x, 48);
  const int e = find_entry(L, blk);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const int N = d.N;
  const int ntx = (N + ST_TX - 1) / ST_TX, nty = (N + ST_TY - 1) / ST_TY;
  // states of one tile are adjacent in logical block order, so the potential
  // (shared by all states) and the halo rows of neighbouring tiles are re-read
  // from L2
  int t = blk - L.tile_start[e];
  const int s = t % d.k; t /= d.k;
  const int bx = t % ntx; t /= ntx;
  const int by = t % nty; t /= nty;
  const int bz = t;
  const int lane = threadIdx.x & 63;
  const int i3 = bx * ST_TX + lane;
  const int y0 = by * ST_TY + (threadIdx.x >> 6) * ST_RPT;
  const size_t N3 = (size_t)N * N * N;
  const C<T> *sp = (const C<T> *)((mode & M_SWAP) ? d.alt : d.psi) + (size_t)s * N3;
  C<T> *dp = (C<T> *)((mode & M_SWAP) ? d.psi : d.alt) + (size_t)s * N3;
  const T c = (T)d.stencil_c, hdt = (T)(0.5 * d.dt);
  const int z0 = bz * ST_CZ;
  const int z1 = (z0 + ST_CZ < N) ? z0 + ST_CZ : N;
  // every lane of the wave takes part (the lane shifts need the whole wave),
  // lanes and rows outside the lattice neither load nor store
  if (d.vcomplex) stencil_tile<T, true>(sp, dp, d.vtab, N, y0, i3, lane, z0, z1, c, hdt);
  else stencil_tile<T, false>(sp, dp, d.vtab, N, y0, i3, lane, z0, z1, c, hdt);
}

// ------------------------------------------------ two fused stencil steps (complex64)
//
// psi'' = S(S(psi)) for the H_K^(0) step S above, in one sweep.  A block owns an output tile
// of S2_TX (x3) x S2_TY (x2) sites over S2_CZ planes along x1 and marches along x1.  At plane
// zp it
//   - writes psi(zp) over the tile and a frame of width 2 in x2 and x3 to LDS;
//   - computes psi'(zp) over the tile and a frame of width 1 (x1 neighbours from registers,
//     x2 and x3 neighbours from LDS);
//   - computes psi''(zp - 1) over the tile from psi'(zp - 2), psi'(zp) in registers and
//     psi'(zp - 1) in LDS, and stores it.
// Every site is updated with the operations of S in the same order, so the fused pass gives
// the bits of two single passes.  psi' is zero outside the lattice (the walls).  Per step the
// lattice is read and written half as often as by single passes.
constexpr int S2_TX = 64, S2_TY = 16, S2_CZ = 8;   // S2_THREADS: common.h
constexpr int S2_PX = S2_TX + 4, S2_PY = S2_TY + 4;                // psi plane in LDS
constexpr int S2_QX = S2_TX + 2, S2_QY = S2_TY + 2;                // psi' plane in LDS
constexpr int S2_QN = S2_QX * S2_QY;
constexpr int S2_OWN = (S2_QN + S2_THREADS - 1) / S2_THREADS;      // psi' sites per thread
constexpr int S2_RING = S2_PX * S2_PY - S2_QN;                     // psi sites outside the psi' tile
static_assert(S2_RING <= S2_THREADS, "one frame site per thread");

__host__ __device__ inline int stencil2_tiles(int N, int k) {
  return k * ((N + S2_TX - 1) / S2_TX) * ((N + S2_TY - 1) / S2_TY) * ((N + S2_CZ - 1) / S2_CZ);
}

// psi-plane coordinates of frame site j: rows 0 and S2_PY - 1, then columns 0 and S2_PX - 1
// of the rows in between
__device__ __forceinline__ void s2_frame_site(int j, int &py, int &px) {
  if (j < S2_PX) { py = 0; px = j; }
  else if (j < 2 * S2_PX) { py = S2_PY - 1; px = j - S2_PX; }
  else { const int jj = j - 2 * S2_PX; py = 1 + (jj >> 1); px = (jj & 1) ? S2_PX - 1 : 0; }
}

template <bool VC>
__device__ __forceinline__ void stencil2_tile(const float2 *__restrict__ sp, float2 *__restrict__ dp,
                                              const void *__restrict__ vtab, int N, int x0, int y0, int z0,
                                              int z1, float c, float hdt, float2 *P, float2 *Q) {
  using VT = typename VType<float, VC>::type;
  const int N2 = N * N;
  const float2 zero = make_float2(0.f, 0.f);
  VT vzero;
  if constexpr (VC) vzero = zero; else vzero = 0.f;
  const int t = threadIdx.x;
  // psi' sites of this thread: i = t + q S2_THREADS over the (S2_QY x S2_QX) tile
  int qoff[S2_OWN], pa[S2_OWN], qa[S2_OWN];
  bool own[S2_OWN], lat[S2_OWN], out[S2_OWN];
#pragma unroll
  for (int q = 0; q < S2_OWN; ++q) {
    const int i = t + q * S2_THREADS;
    own[q] = i < S2_QN;
    const int qy = own[q] ? i / S2_QX : 0, qx = own[q] ? i - (i / S2_QX) * S2_QX : 0;
    const int y = y0 - 1 + qy, x = x0 - 1 + qx;
    lat[q] = own[q] && y >= 0 && y < N && x >= 0 && x < N;
    out[q] = lat[q] && qy >= 1 && qy <= S2_TY && qx >= 1 && qx <= S2_TX;
    qoff[q] = lat[q] ? y * N + x : 0;
    pa[q] = (qy + 1) * S2_PX + qx + 1;     // its psi-plane address
    qa[q] = qy * S2_QX + qx;               // its psi'-plane address
  }
  // frame site of this thread (psi only)
  int fa = 0, foff = 0;
  bool flat = false;
  if (t < S2_RING) {
    int py, px;
    s2_frame_site(t, py, px);
    const int y = y0 - 2 + py, x = x0 - 2 + px;
    flat = y >= 0 && y < N && x >= 0 && x < N;
    foff = flat ? y * N + x : 0;
    fa = py * S2_PX + px;
  }
  auto ld = [&](int z, int off, bool ok) -> float2 {
    return (ok && z >= 0 && z < N) ? sp[z * N2 + off] : zero;
  };
  // registers per psi' site: psi at zp - 1 and zp, psi' at zp - 2 and zp - 1, V at zp - 1
  float2 pp[S2_OWN], pc[S2_OWN], qm2[S2_OWN], qm1[S2_OWN];
  VT vm1[S2_OWN];
#pragma unroll
  for (int q = 0; q < S2_OWN; ++q) {
    pp[q] = ld(z0 - 2, qoff[q], lat[q]);
    pc[q] = ld(z0 - 1, qoff[q], lat[q]);
    qm2[q] = zero;
    qm1[q] = zero;
    vm1[q] = vzero;
  }
  for (int zp = z0 - 1; zp <= z1; ++zp) {
    const bool zin = zp >= 0 && zp < N;
    float2 pn[S2_OWN];
    VT v0[S2_OWN];
#pragma unroll
    for (int q = 0; q < S2_OWN; ++q) {
      pn[q] = ld(zp + 1, qoff[q], lat[q]);
      v0[q] = (lat[q] && zin) ? load_v<float, VC>(vtab, zp * N2 + qoff[q]) : vzero;
    }
    const float2 fv = t < S2_RING ? ld(zp, foff, flat) : zero;
    // psi(zp) over the tile and its frame of width 2
#pragma unroll
    for (int q = 0; q < S2_OWN; ++q)
      if (own[q]) P[pa[q]] = pc[q];
    if (t < S2_RING) P[fa] = fv;
    __syncthreads();
    // psi'(zp) over the tile and its frame of width 1
    float2 q0[S2_OWN];
#pragma unroll
    for (int q = 0; q < S2_OWN; ++q) {
      q0[q] = zero;
      if (lat[q] && zin) {
        const int a = pa[q];
        const float2 l = P[a - 1], rr = P[a + 1], yu = P[a - S2_PX], yd = P[a + S2_PX];
        float2 acc = csub(cadd(pp[q], pn[q]), cscale(pc[q], 6.f));
        acc = cadd(acc, cadd(cadd(l, rr), cadd(yu, yd)));
        q0[q] = fdtd_update<float, VC>(pc[q], acc, v0[q], c, hdt);
      }
    }
    // psi''(zp - 1) over the tile; the psi' plane in LDS holds psi'(zp - 1)
    const int zo = zp - 1;
    if (zo >= z0) {
#pragma unroll
      for (int q = 0; q < S2_OWN; ++q) {
        if (out[q]) {
          const int a = qa[q];
          const float2 l = Q[a - 1], rr = Q[a + 1], yu = Q[a - S2_QX], yd = Q[a + S2_QX];
          float2 acc = csub(cadd(qm2[q], q0[q]), cscale(qm1[q], 6.f));
          acc = cadd(acc, cadd(cadd(l, rr), cadd(yu, yd)));
          dp[zo * N2 + qoff[q]] = fdtd_update<float, VC>(qm1[q], acc, vm1[q], c, hdt);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < S2_OWN; ++q) {
      if (own[q]) Q[qa[q]] = q0[q];
      pp[q] = pc[q];
      pc[q] = pn[q];
      qm2[q] = qm1[q];
      qm1[q] = q0[q];
      vm1[q] = v0[q];
    }
  }
}

__global__ void __launch_bounds__(S2_THREADS) k_stencil2(const LaunchList L) {
  __shared__ float2 P[S2_PX * S2_PY];
  __shared__ float2 Q[S2_QN];
  // tiles are ordered as those of the single-step stencil (states of a tile adjacent, runs of
  // 48 tiles per XCD)
  const int blk = xcd_block_chunked(blockIdx.x, gridDim.x, 48);
  const int e = find_entry(L, blk);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const int N = d.N;
  const int ntx = (N + S2_TX - 1) / S2_TX, nty = (N + S2_TY - 1) / S2_TY;
  int t = blk - L.tile_start[e];
  const int s = t % d.k; t /= d.k;
  const int bx = t % ntx; t /= ntx;
  const int by = t % nty; t /= nty;
  const int bz = t;
  const size_t N3 = (size_t)N * N * N;
  const float2 *sp = (const float2 *)((mode & M_SWAP) ? d.alt : d.psi) + (size_t)s * N3;
  float2 *dp = (float2 *)((mode & M_SWAP) ? d.psi : d.alt) + (size_t)s * N3;
  const float c = (float)d.stencil_c, hdt = (float)(0.5 * d.dt);
  const int z0 = bz * S2_CZ;
  const int z1 = (z0 + S2_CZ < N) ? z0 + S2_CZ : N;
  if (d.vcomplex) stencil2_tile<true>(sp, dp, d.vtab, N, bx * S2_TX, by * S2_TY, z0, z1, c, hdt, P, Q);
  else stencil2_tile<false>(sp, dp, d.vtab, N, bx * S2_TX, by * S2_TY, z0, z1, c, hdt, P, Q);
}

// ---------------------------------------------------------------- parity

// reflection of index i on axis: periodic (N - i) mod N; walled N - i (N = wall)
__device__ __forceinline__ int mirror(int i, int N, bool periodic) {
  const int m = N - i;
  return periodic ? (m == N ? 0 : m) : m;
}

// Each thread takes sites gi; a projected state is processed by reflection orbits: the site of
// the orbit with the smallest index reads the orbit's values once and writes every member's
// output (the other members' threads do nothing), so each value is read and written once.  A
// member's output is the same expression of its own value and its own images as for a single
// site, so results do not depend on the grouping.  P^+/P^-: orbit {x, R x} (R reflects all three
// axes); P^-_{p_k}: {x, R_k x, R_o x, R x} (R_k reflects axis k, R_o the other two).
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_parity(const LaunchList L) {
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  // site indices in 32 bits: k N^3 <= 8 * 512^3 = 2^30
  const uint32_t N = (uint32_t)d.N;
  const uint32_t N3 = N * N * N;
  const C<T> *__restrict__ src = (const C<T> *)((mode & M_SWAP) ? d.alt : d.psi);
  C<T> *__restrict__ dst = (C<T> *)((mode & M_SWAP) ? d.psi : d.alt);
  const bool periodic = d.kin != KIN_FDTD;
  const uint32_t base = (uint32_t)(blockIdx.x - L.tile_start[e]) * RED_THREADS * EW_PER_THREAD;
  const uint32_t total = (uint32_t)d.k * N3;
#pragma unroll
  for (int q = 0; q < EW_PER_THREAD; ++q) {
    const uint32_t gi = base + q * RED_THREADS + threadIdx.x;
    if (gi >= total) break;
    const uint32_t s = gi / N3;
    const uint32_t x = gi - s * N3, sb = s * N3;
    const uint32_t r = x / N, i3 = x - r * N, i1 = r / N, i2 = r - i1 * N;
    const int sec = d.sector[s];
    if (sec == 0) { dst[gi] = src[gi]; continue; }
    // walled lattice: a site with some i_l = 0 mirrors onto the wall, so a state of definite
    // parity vanishes there (the projector stays idempotent); the other sites' images stay inside
    if (!periodic && (i1 == 0 || i2 == 0 || i3 == 0)) { dst[gi] = mkc<T>(0, 0); continue; }
    const uint32_t m1 = mirror(i1, N, periodic), m2 = mirror(i2, N, periodic), m3 = mirror(i3, N, periodic);
    auto idx = [&](uint32_t j1, uint32_t j2, uint32_t j3) -> uint32_t { return sb + (j1 * N + j2) * N + j3; };
    const uint32_t xa = idx(m1, m2, m3);
    if (sec == 1 || sec == 2) {
      if (xa < gi) continue;                     // the orbit's first site handles it
      const C<T> v = src[gi], w = src[xa];
      if (sec == 1) {
        dst[gi] = cscale(cadd(v, w), (T)0.5);
        if (xa != gi) dst[xa] = cscale(cadd(w, v), (T)0.5);
      } else {
        dst[gi] = cscale(csub(v, w), (T)0.5);
        if (xa != gi) dst[xa] = cscale(csub(w, v), (T)0.5);
      }
      continue;
    }
    // P^-_{p_k} = (1 + R_o)(1 - R_k)/4; member z: (v(z) + v(R_o z)) - (v(R_k z) + v(R z))
    uint32_t xk, xo;
    if (sec == 3) { xk = idx(m1, i2, i3); xo = idx(i1, m2, m3); }
    else if (sec == 4) { xk = idx(i1, m2, i3); xo = idx(m1, i2, m3); }
    else { xk = idx(i1, i2, m3); xo = idx(m1, m2, i3); }
    if (xk < gi || xo < gi || xa < gi) continue;
    const C<T> a = src[gi], b = src[xk], c = src[xo], f = src[xa];
    dst[gi] = cscale(csub(cadd(a, c), cadd(b, f)), (T)0.25);
    if (xk != gi) dst[xk] = cscale(csub(cadd(b, f), cadd(a, c)), (T)0.25);
    if (xo != gi && xo != xk) dst[xo] = cscale(csub(cadd(c, a), cadd(f, b)), (T)0.25);
    if (xa != gi && xa != xk && xa != xo) dst[xa] = cscale(csub(cadd(f, b), cadd(c, a)), (T)0.25);
  }
}

// ------------------------------------------------------------- reductions

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double *out) {
  __shared__ double red[RED_THREADS / 64][NV > 0 ? NV : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[w][q] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NV; q += blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int ww = 0; ww < RED_THREADS / 64; ++ww) v += red[ww][q];
    out[q] = v;
  }
}

// Gram partials G_ij = sum conj(psi_i) psi_j, i <= j, over block blk's range of the N3 sites
// (nblk blocks), written to out[0 .. 2 NP).
template <typename T, int KS>
__device__ __forceinline__ void gram_partials(const C<T> *src, size_t N3, int nblk, int blk, double *out) {
  constexpr int NP = KS * (KS + 1) / 2;
  const size_t chunk = (N3 + nblk - 1) / nblk;
  const size_t lo = blk * chunk, hi = (lo + chunk < N3) ? lo + chunk : N3;
  double acc[2 * NP];
#pragma unroll
  for (int q = 0; q < 2 * NP; ++q) acc[q] = 0.0;
  for (size_t x = lo + threadIdx.x; x < hi; x += RED_THREADS) {
    double2 v[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) {
      const C<T> u = src[(size_t)i * N3 + x];
      v[i] = make_double2((double)u.x, (double)u.y);
    }
    int p = 0;
#pragma unroll
    for (int i = 0; i < KS; ++i)
#pragma unroll
      for (int j = i; j < KS; ++j, ++p) {
        acc[2 * p] += v[i].x * v[j].x + v[i].y * v[j].y;
        acc[2 * p + 1] += v[i].x * v[j].y - v[i].y * v[j].x;
      }
  }
  block_reduce_store<2 * NP>(acc, out);
}

template <typename T, int KS>
__global__ void __launch_bounds__(RED_THREADS) k_gram(const LaunchList L) {
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const int blk = blockIdx.x - L.tile_start[e];
  const size_t N3 = (size_t)d.N * d.N * d.N;
  const C<T> *src = (const C<T> *)((mode & M_SWAP) ? d.alt : d.psi);
  gram_partials<T, KS>(src, N3, d.nblk_red, blk, d.partials + (size_t)blk * (2 * MAX_PAIRS));
}

// The same partials for k states given by a plain pointer ([k][n] interleaved complex).
template <typename T, int KS>
__global__ void __launch_bounds__(RED_THREADS) k_gram_flat(const C<T> *psi, size_t n, int nblk, double *partials) {
  gram_partials<T, KS>(psi, n, nblk, blockIdx.x, partials + (size_t)blockIdx.x * (2 * MAX_PAIRS));
}

__device__ __forceinline__ int pair_index(int i, int j, int KS) { return i * KS - i * (i - 1) / 2 + (j - i); }

// Sums of columns q0 .. q0 + nq - 1 (nq <= SUMQ) of a [nb][2*MAX_PAIRS] partials array over its
// nb rows, all at once, with all threads of the block: thread t adds rows t, t + RED_THREADS,
// ... in order, then a fixed-shape tree halves the thread sums.  The order of additions of a
// column never changes (and does not depend on nq or q0); the loads of all the columns are in
// flight together.  Thread j < nq writes the sum of column q0 + j to out[j].
constexpr int SUMQ = 12;
__device__ void block_sum_columns(const double *part, int nb, int q0, int nq, double *out) {
  __shared__ double red[SUMQ][RED_THREADS];
  double s[SUMQ];
#pragma unroll
  for (int j = 0; j < SUMQ; ++j) s[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += RED_THREADS) {
    const double *row = part + (size_t)b * (2 * MAX_PAIRS) + q0;
#pragma unroll
    for (int j = 0; j < SUMQ; ++j)
      if (j < nq) s[j] += row[j];
  }
#pragma unroll
  for (int j = 0; j < SUMQ; ++j)
    if (j < nq) red[j][threadIdx.x] = s[j];
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int j = 0; j < SUMQ; ++j)
        if (j < nq) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < nq) out[threadIdx.x] = red[threadIdx.x][0];
  __syncthreads();
}

// The Gram matrix itself: fixed-order sums of the partials into out[nq] (one block).
__global__ void __launch_bounds__(RED_THREADS) k_gram_sum(const double *partials, int nb, int nq, double *out) {
  for (int q0 = 0; q0 < nq; q0 += SUMQ)
    block_sum_columns(partials, nb, q0, nq - q0 < SUMQ ? nq - q0 : SUMQ, out + q0);
}

// The k x k Gram matrix from nb rows of partials: the pair sums in the fixed order of
// k_gram_sum, then the Hermitian matrix G[i][j] = (re, im), row-major, as qfdtd_gram_matrix
// returns it.
__global__ void __launch_bounds__(RED_THREADS) k_gram_full(const double *partials, int nb, int KS, double *G) {
  __shared__ double Gs[MAX_PAIRS * 2];
  const int NP = KS * (KS + 1) / 2;
  for (int q0 = 0; q0 < 2 * NP; q0 += SUMQ)
    block_sum_columns(partials, nb, q0, 2 * NP - q0 < SUMQ ? 2 * NP - q0 : SUMQ, Gs + q0);
  for (int t = threadIdx.x; t < KS * KS; t += blockDim.x) {
    const int i = t / KS, j = t - (t / KS) * KS;
    const int p = i <= j ? pair_index(i, j, KS) : pair_index(j, i, KS);
    G[2 * t] = Gs[2 * p];
    G[2 * t + 1] = i <= j ? Gs[2 * p + 1] : -Gs[2 * p + 1];
  }
}

// Sum the partials (fixed order), Cholesky G = R^H R per sector, coef = R^{-1}.
__global__ void __launch_bounds__(RED_THREADS) k_gram_finalize(const LaunchList L) {
  const int e = blockIdx.x;
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const int KS = d.k;
  const int NP = KS * (KS + 1) / 2;
  __shared__ double G[MAX_PAIRS * 2];
  for (int q0 = 0; q0 < 2 * NP; q0 += SUMQ)
    block_sum_columns(d.partials, d.nblk_red, q0, 2 * NP - q0 < SUMQ ? 2 * NP - q0 : SUMQ, G + q0);
  // the factor and its inverse in LDS: one thread works on them with indices known only at run
  // time (the states of each sector), which would otherwise put them in scratch memory
  __shared__ double Rr[MAX_STATES][MAX_STATES], Ri[MAX_STATES][MAX_STATES];
  __shared__ double Xr[MAX_STATES][MAX_STATES], Xi[MAX_STATES][MAX_STATES];
  if (threadIdx.x != 0) return;
  for (int i = 0; i < MAX_STATES; ++i)
    for (int j = 0; j < MAX_STATES; ++j) { Rr[i][j] = Ri[i][j] = Xr[i][j] = Xi[i][j] = 0.0; }
  int bad = 0;
  const bool residuals = L.aux[e] == 1;   // only report the diagonal of R (see below)
  double rdiag[MAX_STATES] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool done[MAX_STATES] = {false, false, false, false, false, false, false, false};
  for (int first = 0; first < KS; ++first) {
    if (done[first]) continue;
    int idx[MAX_STATES], n = 0;
    for (int s = first; s < KS; ++s)
      if (d.sector[s] == d.sector[first]) { idx[n++] = s; done[s] = true; }
    for (int jj = 0; jj < n; ++jj) {
      const int j = idx[jj];
      for (int ii = 0; ii < jj; ++ii) {
        const int i = idx[ii];
        const int p = pair_index(i, j, KS);
        double sr = G[2 * p], si = G[2 * p + 1];
        for (int ll = 0; ll < ii; ++ll) {
          const int l = idx[ll];
          // conj(R_li) R_lj
          sr -= Rr[l][i] * Rr[l][j] + Ri[l][i] * Ri[l][j];
          si -= Rr[l][i] * Ri[l][j] - Ri[l][i] * Rr[l][j];
        }
        Rr[i][j] = sr / Rr[i][i];
        Ri[i][j] = si / Rr[i][i];
      }
      const int p = pair_index(j, j, KS);
      double dd = G[2 * p];
      const double gjj = dd;
      for (int ll = 0; ll < jj; ++ll) {
        const int l = idx[ll];
        dd -= Rr[l][j] * Rr[l][j] + Ri[l][j] * Ri[l][j];
      }
      rdiag[j] = (dd > 0.0 && isfinite(dd)) ? sqrt(dd) : 0.0;
      if (!(gjj > 0.0) || !isfinite(gjj) || !(dd > 1e-24 * gjj) || !isfinite(dd)) { bad = 1; dd = 1.0; }
      Rr[j][j] = sqrt(dd);
      Ri[j][j] = 0.0;
    }
    // X = R^{-1} (upper triangular within the sector)
    for (int jj = 0; jj < n; ++jj) {
      const int j = idx[jj];
      Xr[j][j] = 1.0 / Rr[j][j];
      for (int ii = jj - 1; ii >= 0; --ii) {
        const int i = idx[ii];
        double sr = 0.0, si = 0.0;
        for (int ll = ii + 1; ll <= jj; ++ll) {
          const int l = idx[ll];
          sr += Rr[i][l] * Xr[l][j] - Ri[i][l] * Xi[l][j];
          si += Rr[i][l] * Xi[l][j] + Ri[i][l] * Xr[l][j];
        }
        Xr[i][j] = -sr / Rr[i][i];
        Xi[i][j] = -si / Rr[i][i];
      }
    }
  }
  if (residuals) {
    // R_jj = the norm of state j after projection against the earlier states of its sector
    // (G = R^H R per sector); qfdtd_gram_residuals reads it, nothing else changes
    for (int j = 0; j < KS; ++j) d.energy[ENERGY_RDIAG + j] = rdiag[j];
    return;
  }
  for (int i = 0; i < KS; ++i)
    for (int j = 0; j < KS; ++j) {
      d.coef[(i * MAX_STATES + j) * 2] = Xr[i][j];
      d.coef[(i * MAX_STATES + j) * 2 + 1] = Xi[i][j];
    }
  if (bad) d.energy[2 * MAX_STATES] = 1.0;
}

// psi_j <- sum_{i <= j} src_i coef_ij  (in place when src is psi)
template <typename T, int KS>
__global__ void __launch_bounds__(RED_THREADS) k_apply(const LaunchList L) {
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const size_t N3 = (size_t)d.N * d.N * d.N;
  const C<T> *src = (const C<T> *)((mode & M_SWAP) ? d.alt : d.psi);
  C<T> *dst = (C<T> *)d.psi;
  C<T> cf[KS][KS];
#pragma unroll
  for (int i = 0; i < KS; ++i)
#pragma unroll
    for (int j = 0; j < KS; ++j)
      cf[i][j] = mkc<T>((T)d.coef[(i * MAX_STATES + j) * 2], (T)d.coef[(i * MAX_STATES + j) * 2 + 1]);
  const long long base = (long long)(blockIdx.x - L.tile_start[e]) * RED_THREADS * EW_PER_THREAD;
#pragma unroll
  for (int q = 0; q < EW_PER_THREAD; ++q) {
    const long long x = base + q * RED_THREADS + threadIdx.x;
    if (x >= (long long)N3) break;
    C<T> v[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) v[i] = src[(size_t)i * N3 + x];
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      C<T> o = mkc<T>(0, 0);
#pragma unroll
      for (int i = 0; i <= j; ++i) o = cadd(o, cmul(v[i], cf[i][j]));
      dst[(size_t)j * N3 + x] = o;
    }
  }
}

// ------------------------------------------------------------- energies

// per state: |psi|^2, V |psi|^2 (re, im) and, for H_K^(0), conj(psi) H_K psi (re, im)
template <typename T, int KS>
__global__ void __launch_bounds__(RED_THREADS) k_energy_partials(const LaunchList L) {
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const int blk = blockIdx.x - L.tile_start[e];
  const int N = d.N;
  const size_t N3 = (size_t)N * N * N;
  const C<T> *src = (const C<T> *)d.psi;
  const size_t chunk = (N3 + d.nblk_red - 1) / d.nblk_red;
  const size_t lo = blk * chunk, hi = (lo + chunk < N3) ? lo + chunk : N3;
  const bool fdtd = d.kin == KIN_FDTD;
  const double kc = 1.0 / (2.0 * d.m * d.a * d.a);
  double acc[5 * KS];
#pragma unroll
  for (int q = 0; q < 5 * KS; ++q) acc[q] = 0.0;
  for (size_t x = lo + threadIdx.x; x < hi; x += RED_THREADS) {
    double vr, vi = 0.0;
    if (d.vcomplex) { vr = d.v64[2 * x]; vi = d.v64[2 * x + 1]; }
    else vr = d.v64[x];
    const int i3 = (int)(x % N), i2 = (int)((x / N) % N), i1 = (int)(x / ((size_t)N * N));
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const C<T> *sp = src + (size_t)s * N3;
      const C<T> u = sp[x];
      const double ur = u.x, ui = u.y;
      const double n2 = ur * ur + ui * ui;
      acc[5 * s] += n2;
      acc[5 * s + 1] += vr * n2;
      acc[5 * s + 2] += vi * n2;
      if (fdtd) {
        double lr = -6.0 * ur, li = -6.0 * ui;
        C<T> w;
        if (i3 > 0) { w = sp[x - 1]; lr += w.x; li += w.y; }
        if (i3 < N - 1) { w = sp[x + 1]; lr += w.x; li += w.y; }
        if (i2 > 0) { w = sp[x - N]; lr += w.x; li += w.y; }
        if (i2 < N - 1) { w = sp[x + N]; lr += w.x; li += w.y; }
        if (i1 > 0) { w = sp[x - (size_t)N * N]; lr += w.x; li += w.y; }
        if (i1 < N - 1) { w = sp[x + (size_t)N * N]; lr += w.x; li += w.y; }
        // conj(u) * (-L u) / (2 m a^2)
        acc[5 * s + 3] += -kc * (ur * lr + ui * li);
        acc[5 * s + 4] += -kc * (ur * li - ui * lr);
      }
    }
  }
  block_reduce_store<5 * KS>(acc, d.partials + (size_t)blk * (2 * MAX_PAIRS));
}

// state precision -> FP64 copy of all states (input of the FP64 energy transform)
template <typename T>
__global__ void __launch_bounds__(RED_THREADS) k_to64(const LaunchList L) {
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const long long total = (long long)d.k * d.N * d.N * d.N;
  const long long base = (long long)(blockIdx.x - L.tile_start[e]) * RED_THREADS * EW_PER_THREAD;
  const C<T> *src = (const C<T> *)d.psi;
#pragma unroll
  for (int q = 0; q < EW_PER_THREAD; ++q) {
    const long long gi = base + q * RED_THREADS + threadIdx.x;
    if (gi >= total) break;
    const C<T> u = src[gi];
    d.scratch64[gi] = make_double2((double)u.x, (double)u.y);
  }
}

// sum_k T(k) |psi^(k)|^2 / N^3 per state, from the FP64 forward transform in scratch64
template <int KS>
__global__ void __launch_bounds__(RED_THREADS) k_kin_partials(const LaunchList L) {
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const int blk = blockIdx.x - L.tile_start[e];
  const int N = d.N;
  const size_t N3 = (size_t)N * N * N;
  const size_t chunk = (N3 + d.nblk_red - 1) / d.nblk_red;
  const size_t lo = blk * chunk, hi = (lo + chunk < N3) ? lo + chunk : N3;
  const double m = d.m;
  double acc[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) acc[s] = 0.0;
  for (size_t x = lo + threadIdx.x; x < hi; x += RED_THREADS) {
    const int i3 = (int)(x % N), i2 = (int)((x / N) % N), i1 = (int)(x / ((size_t)N * N));
    const double ks = d.ksym64[i1] + d.ksym64[i2] + d.ksym64[i3];
    const double tk = (d.kin == KIN_REL) ? ks / (sqrt(ks + m * m) + m) : ks;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const double2 u = d.scratch64[(size_t)s * N3 + x];
      acc[s] += tk * (u.x * u.x + u.y * u.y);
    }
  }
  block_reduce_store<KS>(acc, d.partials + (size_t)(d.nblk_red + blk) * (2 * MAX_PAIRS));
}

// E_s = (<V> + <H_K>)/<psi|psi>; aux = trace slot (or -1)
__global__ void __launch_bounds__(RED_THREADS) k_energy_finalize(const LaunchList L) {
  const int e = blockIdx.x;
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const int KS = d.k;
  const bool fdtd = d.kin == KIN_FDTD;
  __shared__ double S[6 * MAX_STATES];
  for (int q0 = 0; q0 < 5 * KS; q0 += SUMQ)
    block_sum_columns(d.partials, d.nblk_red, q0, 5 * KS - q0 < SUMQ ? 5 * KS - q0 : SUMQ, S + q0);
  if (!fdtd) {
    for (int q0 = 0; q0 < KS; q0 += SUMQ)
      block_sum_columns(d.partials + (size_t)d.nblk_red * (2 * MAX_PAIRS), d.nblk_red, q0,
                        KS - q0 < SUMQ ? KS - q0 : SUMQ, S + 5 * KS + q0);
  }
  if (threadIdx.x != 0) return;
  const int slot = L.aux[e];
  for (int s = 0; s < KS; ++s) {
    const double nrm = S[5 * s];
    double er = S[5 * s + 1], ei = S[5 * s + 2];
    if (fdtd) { er += S[5 * s + 3]; ei += S[5 * s + 4]; }
    else er += S[5 * KS + s] * d.inv_n3;
    er /= nrm;
    ei /= nrm;
    d.energy[2 * s] = er;
    d.energy[2 * s + 1] = ei;
    if (slot >= 0 && d.trace) {
      d.trace[((size_t)slot * KS + s) * 2] = er;
      d.trace[((size_t)slot * KS + s) * 2 + 1] = ei;
    }
    if (!isfinite(er) || !isfinite(ei) || !(nrm > 0.0)) d.energy[2 * MAX_STATES] = 1.0;
  }
}

// host <-> state conversions through an FP64 staging buffer
// Seeded complex Gaussian noise for an initial state: Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, SC 2011), counter (x mod 2^32, x div 2^32, slot, 0) for site x, key (seed lo, seed hi);
// two 53-bit uniforms in (0, 1] from the four words, Box-Muller in FP64, stored in the state
// precision.
__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

template <typename T>
__global__ void k_noise(C<T> *dst, size_t n, uint32_t k0, uint32_t k1, uint32_t slot) {
  const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  uint32_t c[4] = {(uint32_t)x, (uint32_t)(x >> 32), slot, 0u};
  philox4x32_10(c, k0, k1);
  const uint64_t a = (((uint64_t)c[0] << 21) | (c[1] >> 11)) + 1;
  const uint64_t b = (((uint64_t)c[2] << 21) | (c[3] >> 11)) + 1;
  const double u1 = (double)a * 0x1p-53, u2 = (double)b * 0x1p-53;
  const double r = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  dst[x] = mkc<T>((T)(r * cs), (T)(r * sn));
}

template <typename T>
__global__ void k_from64_slot(C<T> *dst, const double2 *src, size_t n) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) dst[g] = mkc<T>((T)src[g].x, (T)src[g].y);
}
template <typename T>
__global__ void k_to64_slot(double2 *dst, const C<T> *src, size_t n) {
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) dst[g] = make_double2((double)src[g].x, (double)src[g].y);
}

// ------------------------------------------------------------- launchers

template <typename T>
void launch_tables_t(void *tw, double2 *tw64, double *ksym64, int N, int kin, double a, double m, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles<T>, dim3((N + 255) / 256), dim3(256), 0, st, (C<T> *)tw, tw64, ksym64, N, kin, a, m);
}
void launch_tables(bool dbl, void *tw, double2 *tw64, double *ksym64, int N, int kin, double a, double m, hipStream_t st) {
  if (dbl) launch_tables_t<double>(tw, tw64, ksym64, N, kin, a, m, st);
  else launch_tables_t<float>(tw, tw64, ksym64, N, kin, a, m, st);
}
void launch_potential(double *v64, int vcomplex, int N, double a, int kind, const double *p, const double *knots, int nk,
                      const double2 *add, hipStream_t st) {
  const size_t N3 = (size_t)N * N * N;
  hipLaunchKernelGGL(k_potential, dim3((unsigned)((N3 + 255) / 256)), dim3(256), 0, st, v64, vcomplex, N, a, kind, p[0],
                     p[1], p[2], knots, nk, add);
}
void launch_dt_tables(bool dbl, const double *v64, int vcomplex, int N, double dt, void *vtab, void *hfac, void *h2fac,
                      void *ktab, const double *ksym64, int kin, int scheme, hipStream_t st) {
  const size_t N3 = (size_t)N * N * N;
  const size_t n = N3 > (size_t)N ? N3 : (size_t)N;
  if (dbl)
    hipLaunchKernelGGL(k_dt_tables<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v64, vcomplex, N3, dt,
                       vtab, hfac, h2fac, (double *)ktab, ksym64, N, kin, scheme);
  else
    hipLaunchKernelGGL(k_dt_tables<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v64, vcomplex, N3, dt,
                       vtab, hfac, h2fac, (float *)ktab, ksym64, N, kin, scheme);
}
void launch_noise(bool dbl, void *dst, size_t n, uint64_t seed, int slot, hipStream_t st) {
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  if (dbl) hipLaunchKernelGGL(k_noise<double>, g, b, 0, st, (double2 *)dst, n, k0, k1, (uint32_t)slot);
  else hipLaunchKernelGGL(k_noise<float>, g, b, 0, st, (float2 *)dst, n, k0, k1, (uint32_t)slot);
}
void launch_from64_slot(bool dbl, void *dst, const double2 *src, size_t n, hipStream_t st) {
  if (dbl) hipLaunchKernelGGL(k_from64_slot<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (double2 *)dst, src, n);
  else hipLaunchKernelGGL(k_from64_slot<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (float2 *)dst, src, n);
}
void launch_to64_slot(bool dbl, double2 *dst, const void *src, size_t n, hipStream_t st) {
  if (dbl) hipLaunchKernelGGL(k_to64_slot<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, (const double2 *)src, n);
  else hipLaunchKernelGGL(k_to64_slot<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, (const float2 *)src, n);
}

int ew_tiles_host(long long n) { return ew_tiles(n); }
int stencil_tiles_host(int N, int k) { return stencil_tiles(N, k); }
int stencil2_tiles_host(int N, int k) { return stencil2_tiles(N, k); }
const void *stencil2_kernel() { return (const void *)k_stencil2; }

const void *stencil_kernel(bool dbl) {
  return dbl ? (const void *)k_stencil<double> : (const void *)k_stencil<float>;
}
void launch_parity(const LaunchList &L, int total, bool dbl, hipStream_t st) {
  if (dbl) hipLaunchKernelGGL(k_parity<double>, dim3(total), dim3(RED_THREADS), 0, st, L);
  else hipLaunchKernelGGL(k_parity<float>, dim3(total), dim3(RED_THREADS), 0, st, L);
}
void launch_to64(const LaunchList &L, int total, bool dbl, hipStream_t st) {
  if (dbl) hipLaunchKernelGGL(k_to64<double>, dim3(total), dim3(RED_THREADS), 0, st, L);
  else hipLaunchKernelGGL(k_to64<float>, dim3(total), dim3(RED_THREADS), 0, st, L);
}

#define QF_KS_SWITCH(KS, MACRO) \
  switch (KS) {                 \
    case 1: MACRO(1); break;    \
    case 2: MACRO(2); break;    \
    case 3: MACRO(3); break;    \
    case 4: MACRO(4); break;    \
    case 5: MACRO(5); break;    \
    case 6: MACRO(6); break;    \
    case 7: MACRO(7); break;    \
    default: MACRO(8); break;   \
  }

void launch_gram(const LaunchList &L, int total, int KS, bool dbl, hipStream_t st) {
#define G_(K)                                                                                  \
  if (dbl) hipLaunchKernelGGL((k_gram<double, K>), dim3(total), dim3(RED_THREADS), 0, st, L); \
  else hipLaunchKernelGGL((k_gram<float, K>), dim3(total), dim3(RED_THREADS), 0, st, L);
  QF_KS_SWITCH(KS, G_)
#undef G_
}
void launch_apply(const LaunchList &L, int total, int KS, bool dbl, hipStream_t st) {
#define A_(K)                                                                                   \
  if (dbl) hipLaunchKernelGGL((k_apply<double, K>), dim3(total), dim3(RED_THREADS), 0, st, L); \
  else hipLaunchKernelGGL((k_apply<float, K>), dim3(total), dim3(RED_THREADS), 0, st, L);
  QF_KS_SWITCH(KS, A_)
#undef A_
}
void launch_energy_partials(const LaunchList &L, int total, int KS, bool dbl, hipStream_t st) {
#define E_(K)                                                                                             \
  if (dbl) hipLaunchKernelGGL((k_energy_partials<double, K>), dim3(total), dim3(RED_THREADS), 0, st, L); \
  else hipLaunchKernelGGL((k_energy_partials<float, K>), dim3(total), dim3(RED_THREADS), 0, st, L);
  QF_KS_SWITCH(KS, E_)
#undef E_
}
void launch_kin_partials(const LaunchList &L, int total, int KS, hipStream_t st) {
#define K_(K) hipLaunchKernelGGL((k_kin_partials<K>), dim3(total), dim3(RED_THREADS), 0, st, L);
  QF_KS_SWITCH(KS, K_)
#undef K_
}
void launch_gram_sum(const double *partials, int nb, int nq, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_sum, dim3(1), dim3(RED_THREADS), 0, st, partials, nb, nq, out);
}
void launch_gram_finalize(const LaunchList &L, hipStream_t st) {
  hipLaunchKernelGGL(k_gram_finalize, dim3(L.n), dim3(RED_THREADS), 0, st, L);
}
void launch_energy_finalize(const LaunchList &L, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_finalize, dim3(L.n), dim3(RED_THREADS), 0, st, L);
}

// ------------------------------------------------ Gram matrix without allocation

// Device memory of qfdtd_gram_matrix_noalloc: the FP64 partial sums of one Gram sweep.  A
// file-scope array, so that the entry point allocates nothing; every call on a GPU uses that
// GPU's copy.  In host code `scratch` names a host-side stand-in, not device memory: its
// device address comes from hipGetSymbolAddress, once per device (gram_scratch_ptr).
static __device__ __align__(256) double scratch[MAX_RED_BLOCKS * 2 * MAX_PAIRS];

}  // namespace qf

#include <mutex>
#include <string>
#include "qfdtd.h"

extern thread_local std::string g_create_error;

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {nullptr};

// Device address of `scratch` on the current device, looked up on the first call there.
qfdtd_status gram_scratch_ptr(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    g_create_error = std::string("qfdtd_gram_matrix_noalloc: no current device: ") + hipGetErrorString(e);
    return QFDTD_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(qf::scratch));
    if (e != hipSuccess || !p) {
      g_create_error = std::string("qfdtd_gram_matrix_noalloc: scratch address: ") + hipGetErrorString(e);
      return QFDTD_E_DEVICE;
    }
    g_scratch_dev[dev] = p;
  }
  *out = (double *)g_scratch_dev[dev];
  return QFDTD_OK;
}

}  // namespace

extern "C" qfdtd_status qfdtd_gram_matrix_noalloc(const void *psi, int64_t n_sites, int32_t k, int32_t precision,
                                                  double *G, void *hip_stream) {
  using namespace qf;
  if (!psi || !G) {
    g_create_error = "qfdtd_gram_matrix_noalloc: NULL pointer";
    return QFDTD_E_INVALID;
  }
  if (k < 1 || k > MAX_STATES) {
    g_create_error = "qfdtd_gram_matrix_noalloc: k must be 1..8";
    return QFDTD_E_INVALID;
  }
  if (precision != 0 && precision != 1) {
    g_create_error = "qfdtd_gram_matrix_noalloc: precision must be 0 or 1";
    return QFDTD_E_INVALID;
  }
  if (n_sites < 1 || n_sites > QFDTD_NOALLOC_MAX_SITES) {
    g_create_error = "qfdtd_gram_matrix_noalloc: n_sites must be 1..QFDTD_NOALLOC_MAX_SITES (2^27)";
    return QFDTD_E_INVALID;
  }
  double *part = nullptr;
  qfdtd_status st = gram_scratch_ptr(&part);
  if (st != QFDTD_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t n = (size_t)n_sites;
  const int nb = red_blocks(n);
#define GF_(K)                                                                                                 \
  if (precision) hipLaunchKernelGGL((k_gram_flat<double, K>), dim3(nb), dim3(RED_THREADS), 0, s, (const double2 *)psi, n, nb, part); \
  else hipLaunchKernelGGL((k_gram_flat<float, K>), dim3(nb), dim3(RED_THREADS), 0, s, (const float2 *)psi, n, nb, part);
  QF_KS_SWITCH(k, GF_)
#undef GF_
  hipLaunchKernelGGL(k_gram_full, dim3(1), dim3(RED_THREADS), 0, s, (const double *)part, nb, (int)k, G);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_create_error = std::string("qfdtd_gram_matrix_noalloc: kernel launch: ") + hipGetErrorString(e);
    return QFDTD_E_DEVICE;
  }
  return QFDTD_OK;
}
