// Transform passes of the split-operator step on gfx950.
//
// One step of an FFT kinetic term (Sec. 2, eqs. HK1-HK3, with the symmetric
// split h F^-1[e^{-dt T} F[h psi]]) is carried out as passes over HBM, each
// reading and writing the state once:
//
//   plane pass  (N^2 plane in LDS): inverse x2,x3 -> x h^2 -> forward x3,x2
//   row pass    (rows of x3 in LDS): inverse x3 -> x h^2 -> forward x3
//   column pass (tile of contiguous x3 columns along x1 or x2 in LDS):
//               forward -> x e^{-dt T(k)}/N^3 -> inverse
//
// The 1D transforms are Stockham autosort FFTs (mixed radix 2, 3, 4, 5, 8 as
// given by the member's plan) on lines held in LDS; each radix stage reads its
// inputs to registers, synchronises, and writes its outputs, so one LDS buffer
// suffices.  Twiddles are the N-th roots of unity generated in FP64 on the
// device and stored in the state precision; they are staged to LDS per block.
#include "common.h"

namespace qf {

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

template <bool INV, typename V> struct Dft<8, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    using T = decltype(v[0].x);
    const T r2 = (T)0.70710678118654752440;
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV, V>::run(e);
    Dft<4, INV, V>::run(o);
    // o[q] *= w8^q, w8 = e^{-+ i pi/4}
    V o1;
    if (INV) { o1.x = (o[1].x - o[1].y) * r2; o1.y = (o[1].x + o[1].y) * r2; }
    else     { o1.x = (o[1].x + o[1].y) * r2; o1.y = (o[1].y - o[1].x) * r2; }
    V o2 = mul_mi<INV>(o[2]);
    V o3;
    if (INV) { o3.x = (-o[3].x - o[3].y) * r2; o3.y = (o[3].x - o[3].y) * r2; }
    else     { o3.x = (o[3].y - o[3].x) * r2; o3.y = (-o[3].x - o[3].y) * r2; }
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
  }
};

template <bool INV, typename V> struct Dft<3, INV, V> {
  static __device__ __forceinline__ void run(V *v) {
    using T = decltype(v[0].x);
    const T s = (T)0.86602540378443864676;
    V t = cadd(v[1], v[2]);
    V u = cscale(csub(v[1], v[2]), s);
    V a = csub(v[0], cscale(t, (T)0.5));
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
    V a1 = cadd(v[0], cadd(cscale(t1, c1), cscale(t2, c2)));
    V a2 = cadd(v[0], cadd(cscale(t1, c2), cscale(t2, c1)));
    V b1 = mul_mi<INV>(cadd(cscale(u1, s1), cscale(u2, s2)));
    V b2 = mul_mi<INV>(csub(cscale(u1, s2), cscale(u2, s1)));
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// ------------------------------------------------------ Stockham line stage

// Lines in LDS: element n of line b at buf[b*ls + n*es].  With `linefast`
// consecutive threads take consecutive lines (use when es > 1), otherwise
// consecutive butterflies of one line (use when es == 1).
struct LineGeom {
  int nlines, es, ls;
  bool linefast;
};

// One radix-R Stockham stage over all lines.  Kept out of line: with the five
// radix variants inlined into one kernel the register allocator spills to
// scratch; as separate functions each keeps its own small register set.
template <typename T, int R, bool INV, int CAPQ>
__device__ __attribute__((noinline)) void stage(C<T> *buf, const LineGeom g, int N, int Ns, const C<T> *tw) {
  const int NR = N / R;
  const int total = g.nlines * NR;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int twstep = N / (Ns * R);
  C<T> v[CAPQ][R];
  int doff[CAPQ];
#pragma unroll
  for (int q = 0; q < CAPQ; ++q) {
    const int f = tid + q * nt;
    if (f < total) {
      int j, b;
      if (g.linefast) { b = f % g.nlines; j = f / g.nlines; }
      else            { j = f % NR; b = f / NR; }
      const int kk = j % Ns;
      const int lb = b * g.ls;
      const C<T> *src = buf + lb + j * g.es;
      doff[q] = lb + ((j - kk) * R + kk) * g.es;
      v[q][0] = src[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C<T> x = src[r * NR * g.es];
        C<T> w = tw[r * kk * twstep];
        if (INV) w.y = -w.y;
        v[q][r] = cmul(x, w);
      }
      Dft<R, INV, C<T>>::run(v[q]);
    }
  }
  __syncthreads();
  const int ws = Ns * g.es;
#pragma unroll
  for (int q = 0; q < CAPQ; ++q) {
    if (tid + q * nt < total) {
      C<T> *dst = buf + doff[q];
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * ws] = v[q][r];
    }
  }
  __syncthreads();
}

// Full 1D transform of every line; CAPE = max elements per thread.
template <typename T, bool INV, int CAPE>
__device__ void fft_lines(C<T> *buf, const LineGeom g, const PassDesc &d, const C<T> *tw) {
  const int N = d.N;
  int Ns = 1;
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.radix[s];
    switch (R) {
      case 8: stage<T, 8, INV, (CAPE + 7) / 8>(buf, g, N, Ns, tw); break;
      case 4: stage<T, 4, INV, (CAPE + 3) / 4>(buf, g, N, Ns, tw); break;
      case 2: stage<T, 2, INV, (CAPE + 1) / 2>(buf, g, N, Ns, tw); break;
      case 5: stage<T, 5, INV, (CAPE + 4) / 5>(buf, g, N, Ns, tw); break;
      default: stage<T, 3, INV, (CAPE + 2) / 3>(buf, g, N, Ns, tw); break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------- pointwise factors

// psi * f where f is real (T) or complex (C<T>) at site `off`.
template <typename T>
__device__ __forceinline__ C<T> vmul(C<T> v, const void *f, int vcomplex, size_t off) {
  if (vcomplex) return cmul(v, ((const C<T> *)f)[off]);
  return cscale(v, ((const T *)f)[off]);
}

// e^{-dt T(k)} / N^3 at FFT indices (i1, i2, i3).
template <typename T>
__device__ __forceinline__ T kin_factor(const PassDesc &d, int i1, int i2, int i3) {
  const T *kt = (const T *)d.ktab;
  if (d.kin == KIN_REL) {
    const T p2 = kt[i1] + kt[i2] + kt[i3];
    const T m = (T)d.m;
    const T tk = p2 / (sqrt(p2 + m * m) + m);   // sqrt(p^2 + m^2) - m without cancellation
    return exp(-(T)d.dt * tk) * (T)d.inv_n3;
  }
  return kt[i1] * kt[i2] * kt[i3] * (T)d.inv_n3;
}

template <typename T>
__device__ __forceinline__ void load_twiddles(C<T> *tw, const PassDesc &d) {
  const C<T> *src = (const C<T> *)d.tw;
  for (int i = threadIdx.x; i < d.N; i += blockDim.x) tw[i] = src[i];
}

// ------------------------------------------------------------- plane pass

// Tile = one x2-x3 plane (state s, i1) held in LDS with a padded row pitch.
template <typename T>
__global__ void __launch_bounds__(PLANE_THREADS) k_plane(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const int N = d.N, P = N + 1;
  const int t = blockIdx.x - L.tile_start[e];
  const int s = t / N, i1 = t - s * N;
  C<T> *pl = (C<T> *)smem;
  C<T> *tw = pl + N * P;
  load_twiddles<T>(tw, d);
  const size_t N2 = (size_t)N * N;
  C<T> *g = (C<T> *)d.psi + ((size_t)s * N + i1) * N2;
  const size_t voff = (size_t)i1 * N2;
  const int NN = N * N;
  for (int idx = threadIdx.x; idx < NN; idx += blockDim.x) {
    const int r = idx / N, c = idx - r * N;
    C<T> v = g[idx];
    if (mode & M_PRE) v = vmul<T>(v, d.hfac, d.vcomplex, voff + idx);
    pl[r * P + c] = v;
  }
  __syncthreads();
  const LineGeom gx3 = {N, 1, P, false};
  const LineGeom gx2 = {N, P, 1, true};
  if (mode & M_INV) {
    fft_lines<T, true, 16>(pl, gx2, d, tw);
    fft_lines<T, true, 16>(pl, gx3, d, tw);
  }
  if (mode & M_MID) {
    for (int idx = threadIdx.x; idx < NN; idx += blockDim.x) {
      const int r = idx / N, c = idx - r * N;
      pl[r * P + c] = vmul<T>(pl[r * P + c], d.h2fac, d.vcomplex, voff + idx);
    }
    __syncthreads();
  }
  if (mode & M_FWD) {
    fft_lines<T, false, 16>(pl, gx3, d, tw);
    fft_lines<T, false, 16>(pl, gx2, d, tw);
  }
  for (int idx = threadIdx.x; idx < NN; idx += blockDim.x) {
    const int r = idx / N, c = idx - r * N;
    C<T> v = pl[r * P + c];
    if (mode & M_POST) v = vmul<T>(v, d.hfac, d.vcomplex, voff + idx);
    g[idx] = v;
  }
}

// --------------------------------------------------------------- row pass

__host__ __device__ __forceinline__ int row_block(int N) {
  int rb = 4096 / N;
  return rb < 1 ? 1 : rb;
}

// Tile = RB consecutive x3 rows (over all states).
template <typename T>
__global__ void __launch_bounds__(LINE_THREADS) k_row(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const int N = d.N, P = N + 1;
  const int RB = row_block(N);
  const int t = blockIdx.x - L.tile_start[e];
  const long long rows_total = (long long)d.k * N * N;
  const long long row0 = (long long)t * RB;
  const int nrows = (int)((rows_total - row0) < RB ? (rows_total - row0) : RB);
  C<T> *buf = (C<T> *)smem;
  C<T> *tw = buf + RB * P;
  load_twiddles<T>(tw, d);
  const size_t N3 = (size_t)N * N * N;
  C<T> *g = (C<T> *)d.psi + (size_t)row0 * N;
  const int ne = nrows * N;
  for (int idx = threadIdx.x; idx < ne; idx += blockDim.x) {
    const int r = idx / N, c = idx - r * N;
    C<T> v = g[idx];
    if (mode & M_PRE) v = vmul<T>(v, d.hfac, d.vcomplex, ((size_t)row0 * N + idx) % N3);
    buf[r * P + c] = v;
  }
  __syncthreads();
  const LineGeom gr = {nrows, 1, P, false};
  if (mode & M_INV) fft_lines<T, true, 16>(buf, gr, d, tw);
  if (mode & M_MID) {
    for (int idx = threadIdx.x; idx < ne; idx += blockDim.x) {
      const int r = idx / N, c = idx - r * N;
      buf[r * P + c] = vmul<T>(buf[r * P + c], d.h2fac, d.vcomplex, ((size_t)row0 * N + idx) % N3);
    }
    __syncthreads();
  }
  if (mode & M_FWD) fft_lines<T, false, 16>(buf, gr, d, tw);
  for (int idx = threadIdx.x; idx < ne; idx += blockDim.x) {
    const int r = idx / N, c = idx - r * N;
    C<T> v = buf[r * P + c];
    if (mode & M_POST) v = vmul<T>(v, d.hfac, d.vcomplex, ((size_t)row0 * N + idx) % N3);
    g[idx] = v;
  }
}

// ------------------------------------------------------------ column pass

template <typename T> __host__ __device__ constexpr int col_tile() { return sizeof(T) == 4 ? 16 : 8; }

// Tile = TC contiguous x3 columns at one position of the other transverse axis,
// all N elements along the transform axis (x1 if M_AXIS1, else x2).
template <typename T>
__global__ void __launch_bounds__(LINE_THREADS) k_col(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int TC = col_tile<T>();
  const int e = find_entry(L, blockIdx.x);
  const PassDesc &d = *(const PassDesc *)L.descp[e];
  const uint32_t mode = L.mode[e];
  const int N = d.N;
  const int ncb = (N + TC - 1) / TC;
  const int t = blockIdx.x - L.tile_start[e];
  const int per_state = N * ncb;
  const int s = t / per_state;
  const int rem = t - s * per_state;
  const int o = rem / ncb, cb = rem - o * ncb;
  const bool ax1 = (mode & M_AXIS1) != 0;
  const size_t S = ax1 ? (size_t)N * N : (size_t)N;     // stride along the transform axis
  const size_t OS = ax1 ? (size_t)N : (size_t)N * N;    // stride of the outer axis
  const int c0 = cb * TC;
  const int nc = (N - c0) < TC ? (N - c0) : TC;
  C<T> *buf = (C<T> *)smem;
  C<T> *tw = buf + N * TC;
  load_twiddles<T>(tw, d);
  C<T> *g = (C<T> *)d.psi + (size_t)s * N * N * N + (size_t)o * OS + c0;
  const int ne = N * TC;
  for (int idx = threadIdx.x; idx < ne; idx += blockDim.x) {
    const int n = idx / TC, c = idx - n * TC;
    C<T> v = mkc<T>(0, 0);
    if (c < nc) v = g[(size_t)n * S + c];
    buf[idx] = v;
  }
  __syncthreads();
  const LineGeom gc = {TC, TC, 1, true};
  if (mode & M_FWD) fft_lines<T, false, 16>(buf, gc, d, tw);
  if (mode & M_KIN) {
    for (int idx = threadIdx.x; idx < ne; idx += blockDim.x) {
      const int n = idx / TC, c = idx - n * TC;
      const int i1 = ax1 ? n : o, i2 = ax1 ? o : n;
      const int i3 = c0 + (c < nc ? c : 0);
      buf[idx] = cscale(buf[idx], kin_factor<T>(d, i1, i2, i3));
    }
    __syncthreads();
  }
  if (mode & M_INV) fft_lines<T, true, 16>(buf, gc, d, tw);
  const T post = (mode & M_SCALE) ? (T)d.inv_n3 : (T)1;
  for (int idx = threadIdx.x; idx < ne; idx += blockDim.x) {
    const int n = idx / TC, c = idx - n * TC;
    if (c < nc) g[(size_t)n * S + c] = cscale(buf[idx], post);
  }
}

// ------------------------------------------------------------- host side

size_t plane_lds(int N, bool dbl) { return (size_t)(N * (N + 1) + N) * (dbl ? 16 : 8); }
size_t row_lds(int N, bool dbl) { return (size_t)(row_block(N) * (N + 1) + N) * (dbl ? 16 : 8); }
size_t col_lds(int N, bool dbl) { return (size_t)(N * (dbl ? col_tile<double>() : col_tile<float>()) + N) * (dbl ? 16 : 8); }
int plane_tiles(int N, int k) { return k * N; }
int row_tiles(int N, int k) {
  long long rows = (long long)k * N * N;
  int rb = row_block(N);
  return (int)((rows + rb - 1) / rb);
}
int col_tiles(int N, int k, bool dbl) {
  int tc = dbl ? col_tile<double>() : col_tile<float>();
  return k * N * ((N + tc - 1) / tc);
}

hipError_t fft_kernels_init() {
  hipError_t e;
  const int big = 160 * 1024;
  if ((e = hipFuncSetAttribute((const void *)k_plane<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return e;
  if ((e = hipFuncSetAttribute((const void *)k_plane<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return e;
  if ((e = hipFuncSetAttribute((const void *)k_row<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return e;
  if ((e = hipFuncSetAttribute((const void *)k_row<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return e;
  if ((e = hipFuncSetAttribute((const void *)k_col<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return e;
  if ((e = hipFuncSetAttribute((const void *)k_col<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return e;
  return hipSuccess;
}

void launch_plane(const LaunchList &L, int total, size_t lds, bool dbl, hipStream_t st) {
  if (dbl) hipLaunchKernelGGL(k_plane<double>, dim3(total), dim3(PLANE_THREADS), lds, st, L);
  else     hipLaunchKernelGGL(k_plane<float>, dim3(total), dim3(PLANE_THREADS), lds, st, L);
}
void launch_row(const LaunchList &L, int total, size_t lds, bool dbl, hipStream_t st) {
  if (dbl) hipLaunchKernelGGL(k_row<double>, dim3(total), dim3(LINE_THREADS), lds, st, L);
  else     hipLaunchKernelGGL(k_row<float>, dim3(total), dim3(LINE_THREADS), lds, st, L);
}
void launch_col(const LaunchList &L, int total, size_t lds, bool dbl, hipStream_t st) {
  if (dbl) hipLaunchKernelGGL(k_col<double>, dim3(total), dim3(LINE_THREADS), lds, st, L);
  else     hipLaunchKernelGGL(k_col<float>, dim3(total), dim3(LINE_THREADS), lds, st, L);
}

}  // namespace qf
