// Instantiations of the transform passes, one group of lattice sizes per
// compilation (the build compiles this file once per QF_GROUP value).
//
// Per size N: k_plane_t / k_row_t / k_col_t with the block shape tuned for N.
// Per group: multi-size kernels that switch on each member's N, so that one
// launch advances every member of the group whatever its size (used when a
// batch holds several sizes of the group).
#include "fft_passes.h"

#if QF_GROUP == 0
#define QF_SIZES(X) X(8) X(10) X(12) X(16) X(18) X(20) X(24) X(30) X(32)
#define QF_MIN_N 8
#define QF_PLANE_NT 64
#define QF_PLANE_NT_D 64
#elif QF_GROUP == 1
#define QF_SIZES(X) X(36) X(40) X(48) X(50) X(54) X(60) X(64) X(72) X(80)
#define QF_MIN_N 36
#define QF_PLANE_NT 448
#define QF_PLANE_NT_D 448
#elif QF_GROUP == 2
#define QF_SIZES(X) X(90) X(96) X(100) X(108) X(120) X(128)
#define QF_MIN_N 90
#define QF_PLANE_NT 1024
#define QF_PLANE_NT_D 576
#elif QF_GROUP == 3
#define QF_SIZES(X) X(144) X(150) X(160) X(162) X(180)
#define QF_MIN_N 144
#define QF_PLANE_NT 64
#define QF_PLANE_NT_D 64
#else
#define QF_SIZES(X) X(192) X(200) X(216) X(240) X(250) X(256)
#define QF_MIN_N 192
#define QF_PLANE_NT 64
#define QF_PLANE_NT_D 64
#endif

#define QF_CAT2(a, b) a##b
#define QF_CAT(a, b) QF_CAT2(a, b)

namespace qf {

#define PLANE_CASE(n) \
  case n: if constexpr (plane_fits<T, n>()) plane_body<T, n, NT>(L, e, t, smem); break;
#define ROW_CASE(n) \
  case n: row_body<T, n, LINE_THREADS>(L, e, t, smem); break;
#define COL_CASE(n) \
  case n: col_body<T, n, LINE_THREADS>(L, e, t, smem); break;

template <typename T, int NT>
__global__ void __launch_bounds__(NT) QF_CAT(k_plane_multi_g, QF_GROUP)(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int e = find_entry(L, blockIdx.x);
  const int t = blockIdx.x - L.tile_start[e];
  switch (((const PassDesc *)L.descp[e])->N) { QF_SIZES(PLANE_CASE) default: break; }
}

template <typename T>
__global__ void __launch_bounds__(LINE_THREADS) QF_CAT(k_row_multi_g, QF_GROUP)(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int e = find_entry(L, blockIdx.x);
  const int t = blockIdx.x - L.tile_start[e];
  switch (((const PassDesc *)L.descp[e])->N) { QF_SIZES(ROW_CASE) default: break; }
}

template <typename T>
__global__ void __launch_bounds__(LINE_THREADS) QF_CAT(k_col_multi_g, QF_GROUP)(const LaunchList L) {
  extern __shared__ __align__(16) unsigned char smem[];
  // the block order of the group's smallest size (the group never straddles COL_XCD_MIN_N)
  const int blk = col_block(QF_MIN_N);
  const int e = find_entry(L, blk);
  const int t = blk - L.tile_start[e];
  switch (((const PassDesc *)L.descp[e])->N) { QF_SIZES(COL_CASE) default: break; }
}

#define REG_SIZE(n) register_size<n>(t);
#define ANY_PLANE_F(n) || plane_fits<float, n>()
#define ANY_PLANE_D(n) || plane_fits<double, n>()

void QF_CAT(register_fft_group, QF_GROUP)(FftKernels *t, GroupKernels *g) {
  QF_SIZES(REG_SIZE)
  if constexpr (false QF_SIZES(ANY_PLANE_F)) {
    g->plane[0] = (const void *)QF_CAT(k_plane_multi_g, QF_GROUP)<float, QF_PLANE_NT>;
    g->plane_nt[0] = QF_PLANE_NT;
  }
  if constexpr (false QF_SIZES(ANY_PLANE_D)) {
    g->plane[1] = (const void *)QF_CAT(k_plane_multi_g, QF_GROUP)<double, QF_PLANE_NT_D>;
    g->plane_nt[1] = QF_PLANE_NT_D;
  }
  g->row[0] = (const void *)QF_CAT(k_row_multi_g, QF_GROUP)<float>;
  g->row[1] = (const void *)QF_CAT(k_row_multi_g, QF_GROUP)<double>;
  g->col[0] = (const void *)QF_CAT(k_col_multi_g, QF_GROUP)<float>;
  g->col[1] = (const void *)QF_CAT(k_col_multi_g, QF_GROUP)<double>;
}

}  // namespace qf
