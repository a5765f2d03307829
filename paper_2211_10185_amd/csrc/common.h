// Shared device/host definitions of the gfx950 imaginary-time solver.
//
// Data layout in HBM (one solve, "member"):
//   psi   [k][N][N][N] interleaved complex (float2 for complex64 states,
//         double2 for complex128), x3 fastest: site (i1,i2,i3) of state s at
//         s*N^3 + (i1*N + i2)*N + i3.
//   alt   same shape; ping-pong target of the FDTD stencil and of the parity
//         projection (allocated only when needed).
//   vtab  V in the state precision, real [N^3] or complex [N^3].
//   hfac  e^{-dt V/2}, h2fac e^{-dt V}: same type as vtab (FFT kinds).
//   ktab  [N] per-axis kinetic table in the state precision: e^{-dt t(k_j)}
//         for the separable symbols of eqs. (HK1)/(HK2), 4 sin^2(k_j/2)/a^2 for
//         eq. (HK3).
//   tw    [N] roots of unity e^{-2 pi i m/N} in the state precision.
//   tw64, ksym64: FP64 copies used by the FP64 energy measurement.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qf {

template <typename T> struct CT;
template <> struct CT<float> { using type = float2; };
template <> struct CT<double> { using type = double2; };
template <typename T> using C = typename CT<T>::type;

template <typename T> __host__ __device__ __forceinline__ C<T> mkc(T x, T y) { C<T> r; r.x = x; r.y = y; return r; }
template <typename V> __host__ __device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __host__ __device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
// Fused multiply-add written out: device code is compiled with
// -ffp-contract=off, so the rounding of every expression is fixed by the
// source and identical in every kernel instantiation (a member advanced by a
// single-size kernel or by a multi-size kernel gets the same bits).
__host__ __device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }

template <typename V> __host__ __device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = fmaT(a.x, b.x, -(a.y * b.y));
  r.y = fmaT(a.x, b.y, a.y * b.x);
  return r;
}
template <typename V, typename S> __host__ __device__ __forceinline__ V cscale(V a, S s) { V r; r.x = a.x * s; r.y = a.y * s; return r; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V> __host__ __device__ __forceinline__ V mul_mi(V a) {
  V r;
  if (INV) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
  return r;
}

// ------------------------------------------------------------- radix plans

struct RPlan {
  int n;
  int r[8];
};

// Stages of an N-point transform (N = 2^a 3^b 5^c): powers of two grouped into as few
// radix-16/8/4/2 stages as possible, threes paired into radix 9 (a leftover 3 alone), fives as
// radix 5.  Fewer stages mean fewer LDS exchanges and barriers; larger radices cost registers,
// which complex128 (dbl) pays twice over, so some merges are for complex64 only:
//   - a single factor 2 merges into a leftover 3 (radix 6) or a 5 (radix 10) when at least two
//     stages remain, and for complex64 into a 9 (radix 18, N = 162);
//   - 60 = 6 x 10 and 96 = 16 x 6; for complex64 also 100 = 10 x 10, 108 = 12 x 9, 120 = 8 x 15
//     and 160 = 16 x 10.
// The complex64-only merges ran 5-13% faster in complex64 and 3-8% slower in complex128.
__host__ __device__ constexpr RPlan make_rplan(int N, bool dbl) {
  RPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0}};
  int m = N, a = 0, b = 0, c = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  while (m % 5 == 0) { m /= 5; ++c; }
  if (a == 2 && b == 1 && c == 1) { p.r[p.n++] = 6; p.r[p.n++] = 10; return p; }
  if (a == 5 && b == 1 && c == 0) { p.r[p.n++] = 16; p.r[p.n++] = 6; return p; }
  if (!dbl) {
    // complex64: two stages with the composite radices 10, 12, 15 (measured faster; 150 = 15 x 10,
    // 180 = 20 x 9, 192 = 16 x 12, 200 = 20 x 10 and 216 = 24 x 9 were 3-17% slower, 240 = 16 x 15
    // no faster, so those keep three stages)
    struct Two { int n, r0, r1; };
    const Two two[] = {{100, 10, 10}, {160, 16, 10}, {108, 12, 9}, {120, 8, 15}};
    for (const Two &t : two)
      if (t.n == N) { p.r[p.n++] = t.r0; p.r[p.n++] = t.r1; return p; }
  }
  int nines = b / 2, threes = b % 2, fives = c;
  const bool merge2 = a == 1 && (threes || fives || !dbl) && nines + threes + fives >= 2;
  const int twos[9][2] = {{0, 0}, {2, 0}, {4, 0}, {8, 0}, {16, 0}, {8, 4}, {8, 8}, {16, 8}, {16, 16}};
  if (merge2) {
    if (threes) { p.r[p.n++] = 6; threes = 0; }
    else if (fives) { p.r[p.n++] = 10; --fives; }
    else { p.r[p.n++] = 18; --nines; }
  } else {
    for (int i = 0; i < 2; ++i)
      if (a <= 8 && twos[a][i]) p.r[p.n++] = twos[a][i];
  }
  for (int i = 0; i < nines; ++i) p.r[p.n++] = 9;
  if (threes) p.r[p.n++] = 3;
  for (int i = 0; i < fives; ++i) p.r[p.n++] = 5;
  return p;
}

constexpr int MAX_STAGES = 12;
constexpr int MAX_STATES = 8;
constexpr int MAX_PAIRS = MAX_STATES * (MAX_STATES + 1) / 2;
constexpr int MAX_LAUNCH = 64;       // members per launch list
constexpr int ENERGY_RDIAG = 2 * MAX_STATES + 8;           // offset of the Cholesky diagonal
constexpr int ENERGY_WORDS = ENERGY_RDIAG + MAX_STATES;    // doubles in PassDesc::energy

// Blocks of an FP64 reduction sweep over n sites: one per 2048 sites, at most MAX_RED_BLOCKS.
// The grid, and with it the order of every FP64 sum, depends only on the site count.
constexpr int MAX_RED_BLOCKS = 1024;
__host__ __device__ inline int red_blocks(size_t n) {
  size_t b = (n + 2047) / 2048;
  if (b > (size_t)MAX_RED_BLOCKS) b = MAX_RED_BLOCKS;
  return b < 1 ? 1 : (int)b;
}

// Kinetic kinds (eqs. HK0..HK3)
enum { KIN_FDTD = 0, KIN_P2 = 1, KIN_SIN2 = 2, KIN_REL = 3 };

// Mode bits of a real-space (plane or row) pass and of a column pass.
enum : uint32_t {
  M_PRE = 1u,    // x h before the forward transform (chunk start)
  M_INV = 2u,    // inverse transform first
  M_MID = 4u,    // x h^2 between inverse and forward (steady state)
  M_FWD = 8u,    // forward transform
  M_POST = 16u,  // x h after the inverse transform (chunk end)
  M_KIN = 32u,   // column pass: x e^{-dt T(k)}/N^3 between forward and inverse
  M_AXIS1 = 64u, // column pass along x1 (else x2)
  M_SWAP = 128u, // stencil: read alt, write psi (else read psi, write alt)
  M_SCALE = 256u, // column pass: x 1/N^3 after the last transform
  // A/B update of the FFT kinetic terms (the legacy iteration with H_K^(1..3)):
  M_COMB = 512u,  // real-space pass: input dt H_K psi (transformed) from alt; after the inverse,
                  // psi' = A psi - B (dt H_K psi) with psi read from and psi' written to psi
  M_ALT = 1024u   // transforms work on alt: column passes read/write alt, a real-space pass
                  // without M_COMB reads psi and writes its forward transform to alt
};

// Step of the FFT kinetic terms
enum { SCHEME_SPLIT = 0, SCHEME_AB = 1 };

// Everything a kernel needs to know about one member (one solve).  Lives in
// device memory; kernels index it through a launch list.
struct PassDesc {
  void *psi;
  void *alt;
  const void *vtab;
  const void *hfac;
  const void *h2fac;
  const void *ktab;
  const void *tw;
  const void *tw64;
  const double *ksym64;   // [N] t(k_j) (HK1/HK2) or 4 sin^2(k_j/2)/a^2 (HK3), FP64
  const double *v64;      // [N^3] V in FP64, real or (re, im) interleaved
  double2 *scratch64;     // [k][N^3] FP64 copy for the energy transform
  double *partials;       // [2][nblk_red][MAX_PAIRS][2] FP64 reduction partials
  double *coef;           // [MAX_STATES][MAX_STATES][2] FP64 orthonormalisation coefficients
  double *energy;         // [MAX_STATES][2] last energies; [2*MAX_STATES] status word;
                          // [ENERGY_RDIAG + j] Gram-Cholesky diagonal of state j (residual mode)
  double *trace;          // [cap][k][2] energy trace (or null)
  int32_t N, k, kin, vcomplex;
  int32_t nst;
  int32_t radix[MAX_STAGES];
  int32_t sector[MAX_STATES];
  int32_t nblk_red;       // reduction blocks per state sweep
  int32_t scheme;         // SCHEME_SPLIT or SCHEME_AB (FFT kinetic terms)
  double a, m, dt;
  double stencil_c;       // dt / (2 m a^2)
  double inv_n3;
};

// One launch: which members take part, with which mode, and where their tiles
// start in the flattened grid.  Passed by value (kernel arguments), so it is
// captured as-is by a HIP graph.
struct LaunchList {
  int32_t n;
  int32_t tile_start[MAX_LAUNCH + 1];
  const void *descp[MAX_LAUNCH];   // device PassDesc of each entry
  uint16_t mode[MAX_LAUNCH];
  int32_t aux[MAX_LAUNCH];         // per-entry extra (trace slot, ...)
};

// The dispatcher deals consecutive blocks of a grid to the chip's 8 XCDs in
// turn, and each XCD has its own L2.  xcd_block maps the hardware block index
// to a logical one so that every XCD receives one contiguous run of logical
// blocks (a bijection on [0, G) for any G): tiles that share data (neighbours'
// halos, one potential shared by several states) then meet in the same L2.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int q = G / NUM_XCD, r = G - q * NUM_XCD;
  const int x = b % NUM_XCD, i = b / NUM_XCD;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}
// Same in runs of `chunk` logical blocks: each group of NUM_XCD * chunk
// hardware blocks gives every XCD `chunk` consecutive logical blocks; the
// last, partial group falls back to xcd_block over its own range.
__device__ __forceinline__ int xcd_block_chunked(int b, int G, int chunk) {
  const int span = NUM_XCD * chunk;
  const int full = (G / span) * span;
  if (b >= full) return full + xcd_block(b - full, G - full);
  const int g = b / span, w = b - g * span;
  return g * span + (w % NUM_XCD) * chunk + w / NUM_XCD;
}

__device__ __forceinline__ int find_entry(const LaunchList &L, int blk) {
  int lo = 0, hi = L.n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (L.tile_start[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Transform-pass kernels instantiated for one lattice size (index 0: complex64,
// 1: complex128); plane entries are null where an N^2 plane does not fit LDS.
struct FftKernels {
  const void *plane[2];
  const void *row[2];
  const void *col[2];
  size_t plane_lds[2], row_lds[2], col_lds[2];
  int plane_nt;
  // split-x2 two-pass schedule (slab and pencil passes, complex64), where instantiated, by
  // variant (x2 = N1 x N2 and the pencil tile width)
  const void *slab[4], *slab_edge[4];   // steady pass; chunk-edge and plain-transform passes
  size_t slab_lds[4];
  int slab_nt[4], split_n1[4], split_xi[4];
  const void *pencil[4];
  size_t pencil_lds[4];
  int pencil_nt[4], pencil_tt[4];
};

// Multi-size transform-pass kernels of one size group (see fft_inst.hip).
struct GroupKernels {
  const void *plane[2];
  const void *row[2];
  const void *col[2];
  int plane_nt[2];
};

// Size group of a lattice size (groups of fft_inst.hip).
__host__ __device__ inline int size_group(int N) {
  return N <= 32 ? 0 : (N <= 80 ? 1 : (N <= 128 ? 2 : (N <= 180 ? 3 : 4)));
}

// Threads per block of each kernel family.
constexpr int LINE_THREADS = 256;
constexpr int RED_THREADS = 256;
constexpr int S2_THREADS = 256;      // block of the two-step stencil

// Rows of N sites per row-pass block, and x3 columns per column-pass tile; the kernels and the
// host's grid sizes use these same functions.  A row block holds enough rows that the largest
// radix stage of the transform (radices 16/8/4/2 for the powers of two, then 3, 5) gives each
// of the 256 threads a butterfly, but no more than keep its LDS tile under 72 KiB (two blocks
// per CU).  Measured against a fixed 4096 sites per block: 14-37% faster row passes at most
// sizes from 150 to 250 (complex64) and 100 to 160 (complex128), the same elsewhere.
__host__ __device__ constexpr int row_block(int N, bool dbl) {
  const RPlan p = make_rplan(N, dbl);
  int rmax = 1;
  for (int i = 0; i < p.n; ++i)
    if (p.r[i] > rmax) rmax = p.r[i];
  int rb = 256 * rmax / N;
  const int cap = 72 * 1024 / ((N + (N >> 4)) * (dbl ? 16 : 8));
  if (rb > cap) rb = cap;
  return rb < 1 ? 1 : rb;
}
__host__ __device__ constexpr int col_tile(bool dbl) { return dbl ? 8 : 16; }

}  // namespace qf
