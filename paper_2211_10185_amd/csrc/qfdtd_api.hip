// C ABI of the solver: context lifecycle, the per-chunk pass schedule, the
// measurement (orthonormalisation and FP64 energies) and launch timing.
//
// Schedules (per member; k states are carried together through every pass):
//   FFT kinds, plane fits LDS (complex64 N <= 128, complex128 N <= 96):
//     chunk of n steps = plane[h, F23] ; { col1[F1, e^{-dt T}, F1^-1] ; plane[F23^-1, h^2, F23] } x (n-1)
//                        ; col1[...] ; plane[F23^-1, h]                 -> 2n + 1 passes
//   FFT kinds, larger N:
//     row[h, F3] ; col2[F2] ; { col1[...] ; col2[F2^-1] ; row[F3^-1, h^2, F3] ; col2[F2] } x (n-1)
//                        ; col1[...] ; col2[F2^-1] ; row[F3^-1, h]       -> 4n + 1 passes
//   H_K^(0): n stencil passes (ping-pong between psi and alt).
// After every chunk: parity projection (if any sector is set), FP64 Gram
// matrix, Cholesky per sector, psi <- psi R^{-1}.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <mutex>
#include <atomic>

#include "common.h"
#include "qfdtd.h"
#include <hip/hip_ext.h>

namespace qf {
void register_fft_group0(FftKernels *t, GroupKernels *g);
void register_fft_group1(FftKernels *t, GroupKernels *g);
void register_fft_group2(FftKernels *t, GroupKernels *g);
void register_fft_group3(FftKernels *t, GroupKernels *g);
void register_fft_group4(FftKernels *t, GroupKernels *g);
void launch_tables(bool dbl, void *tw, double2 *tw64, double *ksym64, int N, int kin, double a, double m, hipStream_t st);
void launch_potential(double *v64, int vcomplex, int N, double a, int kind, const double *p, const double *knots, int nk,
                      const double2 *add, hipStream_t st);
void launch_dt_tables(bool dbl, const double *v64, int vcomplex, int N, double dt, void *vtab, void *hfac, void *h2fac,
                      void *ktab, const double *ksym64, int kin, int scheme, hipStream_t st);
void launch_from64_slot(bool dbl, void *dst, const double2 *src, size_t n, hipStream_t st);
void launch_noise(bool dbl, void *dst, size_t n, uint64_t seed, int slot, hipStream_t st);
void launch_to64_slot(bool dbl, double2 *dst, const void *src, size_t n, hipStream_t st);
int ew_tiles_host(long long n);
int stencil_tiles_host(int N, int k);
int stencil2_tiles_host(int N, int k);
const void *stencil2_kernel();
const void *stencil_kernel(bool dbl);
void launch_parity(const LaunchList &L, int total, bool dbl, hipStream_t st);
void launch_to64(const LaunchList &L, int total, bool dbl, hipStream_t st);
void launch_gram(const LaunchList &L, int total, int KS, bool dbl, hipStream_t st);
void launch_apply(const LaunchList &L, int total, int KS, bool dbl, hipStream_t st);
void launch_energy_partials(const LaunchList &L, int total, int KS, bool dbl, hipStream_t st);
void launch_kin_partials(const LaunchList &L, int total, int KS, hipStream_t st);
void launch_gram_finalize(const LaunchList &L, hipStream_t st);
void launch_gram_sum(const double *partials, int nb, int nq, double *out, hipStream_t st);
void launch_energy_finalize(const LaunchList &L, hipStream_t st);
}  // namespace qf

using namespace qf;

// message of the last failing context-free call on this thread; defined with the
// potential file I/O (host-only source)
extern thread_local std::string g_create_error;

namespace {

enum { TC_PLANE = 0, TC_ROW = 1, TC_COL = 2, TC_STENCIL = 3, TC_MEAS = 4, TC_SLAB = 5, TC_PENCIL = 6, TC_N = 7 };

struct Timer {
  int every = 0;
  long long seen[TC_N] = {0, 0, 0, 0, 0, 0, 0};
  struct Rec { hipEvent_t a, b; int cls; double bytes; };
  std::vector<Rec> pool;
  size_t used = 0;
  long long count[TC_N] = {0, 0, 0, 0, 0, 0, 0};
  double sum_ms[TC_N] = {0, 0, 0, 0, 0, 0, 0};
  double sum_bytes[TC_N] = {0, 0, 0, 0, 0, 0, 0};
};

bool smooth235(int n) {
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

int make_plan(int N, int32_t *radix) {
  int n = N, s = 0;
  while (n % 8 == 0 && n / 8 >= 2) { radix[s++] = 8; n /= 8; }
  while (n % 4 == 0) { radix[s++] = 4; n /= 4; }
  while (n % 8 == 0) { radix[s++] = 8; n /= 8; }
  while (n % 2 == 0) { radix[s++] = 2; n /= 2; }
  while (n % 5 == 0) { radix[s++] = 5; n /= 5; }
  while (n % 3 == 0) { radix[s++] = 3; n /= 3; }
  return s;
}

FftKernels g_fft[257];
GroupKernels g_grp[5];
size_t g_grp_lds[5][3][2];   // per group, kind (plane, row, col), precision: largest LDS of its sizes

hipError_t fft_table_init() {
  // once per process; contexts may be created from several host threads
  static std::mutex mu;
  static bool done = false;
  std::lock_guard<std::mutex> lk(mu);
  if (done) return hipSuccess;
  std::memset(g_fft, 0, sizeof(g_fft));
  std::memset(g_grp, 0, sizeof(g_grp));
  std::memset(g_grp_lds, 0, sizeof(g_grp_lds));
  register_fft_group0(g_fft, &g_grp[0]);
  register_fft_group1(g_fft, &g_grp[1]);
  register_fft_group2(g_fft, &g_grp[2]);
  register_fft_group3(g_fft, &g_grp[3]);
  register_fft_group4(g_fft, &g_grp[4]);
  for (int n = 8; n <= 256; ++n)
    for (int w = 0; w < 2; ++w) {
      const int gi = size_group(n);
      if (g_fft[n].plane[w]) g_grp_lds[gi][0][w] = std::max(g_grp_lds[gi][0][w], g_fft[n].plane_lds[w]);
      if (g_fft[n].row[w]) g_grp_lds[gi][1][w] = std::max(g_grp_lds[gi][1][w], g_fft[n].row_lds[w]);
      if (g_fft[n].col[w]) g_grp_lds[gi][2][w] = std::max(g_grp_lds[gi][2][w], g_fft[n].col_lds[w]);
    }
  for (int gi = 0; gi < 5; ++gi)
    for (int w = 0; w < 2; ++w) {
      const void *fs[3] = {g_grp[gi].plane[w], g_grp[gi].row[w], g_grp[gi].col[w]};
      for (int q = 0; q < 3; ++q)
        if (fs[q]) {
          hipError_t e = hipFuncSetAttribute(fs[q], hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)g_grp_lds[gi][q][w]);
          if (e != hipSuccess) return e;
        }
    }
  for (int n = 0; n <= 256; ++n)
    for (int w = 0; w < 2; ++w) {
      const void *fs[3] = {g_fft[n].plane[w], g_fft[n].row[w], g_fft[n].col[w]};
      const size_t ls[3] = {g_fft[n].plane_lds[w], g_fft[n].row_lds[w], g_fft[n].col_lds[w]};
      for (int q = 0; q < 3; ++q)
        if (fs[q]) {
          hipError_t e = hipFuncSetAttribute(fs[q], hipFuncAttributeMaxDynamicSharedMemorySize, (int)ls[q]);
          if (e != hipSuccess) return e;
        }
    }
  for (int n = 0; n <= 256; ++n)
    for (int v = 0; v < 4; ++v) {
      const void *fs[3] = {g_fft[n].slab[v], g_fft[n].slab_edge[v], g_fft[n].pencil[v]};
      const size_t ls[3] = {g_fft[n].slab_lds[v], g_fft[n].slab_lds[v], g_fft[n].pencil_lds[v]};
      for (int q = 0; q < 3; ++q)
        if (fs[q]) {
          hipError_t e = hipFuncSetAttribute(fs[q], hipFuncAttributeMaxDynamicSharedMemorySize, (int)ls[q]);
          if (e != hipSuccess) return e;
        }
    }
  done = true;
  return hipSuccess;
}

// Captured chunks of multi-member batches: key = (member serial, steps) for
// every member in batch order.  A key seen once is only recorded (exec null);
// its second use captures, later uses replay, so chunk shapes that occur once
// (a serving loop between admissions) never pay for a capture.  Entries that
// hold a destroyed member are dropped; the cache keeps at most MAX_BATCH_GRAPHS.
struct BatchGraph {
  std::vector<std::pair<uint64_t, int>> key;
  hipGraphExec_t exec;
};
constexpr size_t MAX_BATCH_GRAPHS = 128;
std::vector<BatchGraph> g_batch_graphs;
std::mutex g_batch_mu;
std::atomic<uint64_t> g_next_serial{1};

void drop_batch_graphs(uint64_t serial) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (size_t i = 0; i < g_batch_graphs.size();) {
    bool hit = false;
    for (auto &kv : g_batch_graphs[i].key) hit = hit || kv.first == serial;
    if (hit) {
      if (g_batch_graphs[i].exec) (void)hipGraphExecDestroy(g_batch_graphs[i].exec);
      g_batch_graphs.erase(g_batch_graphs.begin() + i);
    } else {
      ++i;
    }
  }
}

int plane_tiles(int N, int k) { return k * N; }
int row_tiles(int N, int k, bool dbl) {
  const long long rows = (long long)k * N * N;
  const int rb = row_block(N, dbl);
  return (int)((rows + rb - 1) / rb);
}
int col_tiles(int N, int k, bool dbl) {
  const int tc = col_tile(dbl);
  return k * N * ((N + tc - 1) / tc);
}
// split-x2 schedule: slab tiles (group of split_xi x1 planes, fast x2 digit; a tile carries every
// state), pencil tiles (state, slow x2 frequency, x3 column block)
int slab_tiles(int N, int v) { return N / g_fft[N].split_xi[v] * (N / g_fft[N].split_n1[v]); }
// At small N the slab tiles are few (N * N2, each taking all k states in turn), so up to this size
// each state gets tiles of its own (aux 1), which reread the factor rows from cache.  Measured at
// k = 3 on one stream: 42.7 -> 35.5 us per step at 96, 48.1 -> 45.4 at 108, but 60.0 -> 65.9 at
// 120 and 58.0 -> 58.8 at 128.
constexpr int SLAB_STATE_TILES_MAX_N = 108;
int pencil_tiles(int N, int k, int v) { return k * g_fft[N].split_n1[v] * (N / g_fft[N].pencil_tt[v]); }

}  // namespace

constexpr int MAX_GROUPS = 3;   // state groups of one FFT solve on their own streams

struct qfdtd_ctx {
  int N = 0, kin = 0, prec = 0, k = 0, K = 50;
  double a = 0, m = 0;
  int sectors[MAX_STATES] = {0};
  bool any_parity = false, vcomplex = false, dbl = false, plane = false, plane64 = false;
  bool split = false;           // FFT kinds: the two-pass split-x2 schedule (slab and pencil passes)
  int split_v = 0;              // split-x2 variant (x2 = N1 x N2 and the pencil tile width)
  int scheme = SCHEME_SPLIT;    // FFT kinds: split-operator step or A/B update
  hipStream_t st = nullptr;
  qfdtd_alloc_fn af = nullptr;
  qfdtd_free_fn ff = nullptr;
  void *au = nullptr;
  std::string err;
  std::vector<void *> allocs;
  void *psi = nullptr, *alt = nullptr, *vtab = nullptr, *hfac = nullptr, *h2fac = nullptr, *ktab = nullptr, *tw = nullptr;
  double2 *tw64 = nullptr, *scratch64 = nullptr;
  double *ksym64 = nullptr, *v64 = nullptr, *partials = nullptr, *coef = nullptr, *energy = nullptr, *trace = nullptr;
  PassDesc *d_desc = nullptr;   // [0] main, [1] FP64 measurement copy, [2], [3] state groups
  PassDesc hd[2 + MAX_GROUPS];
  int ngroups = 1;              // 2 or 3: states split into groups pipelined on their own streams
  int gk[MAX_GROUPS] = {0, 0, 0};   // states per group
  hipStream_t gst[MAX_GROUPS] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[MAX_GROUPS] = {nullptr, nullptr, nullptr};
  uint64_t serial = 0;          // unique per context, never reused (keys of batch graphs)
  bool graphs = true;           // capture a steady chunk (passes + orthonormalisation) once, replay it
  std::vector<std::pair<int, hipGraphExec_t>> chunk_graphs;   // keyed by steps in the chunk
  int nblk_red = 1;
  double cur_dt = -1.0;
  bool fresh = true;
  uint32_t set_mask = 0;
  bool poisoned = false;
  int cur = 0;                  // H_K^(0): 1 when the state sits in alt
  bool stencil2 = false;        // H_K^(0), complex64: two fused steps per stencil pass
  int trace_on = 0;
  int64_t trace_cap = 0, trace_n = 0;
  double *h_status = nullptr;   // pinned
  hipEvent_t status_ev = nullptr;
  bool status_pending = false;
  Timer timer;

  size_t n3() const { return (size_t)N * N * N; }
  size_t csz() const { return dbl ? 16 : 8; }
  size_t rsz() const { return dbl ? 8 : 4; }
  bool fft() const { return kin != KIN_FDTD; }
};

namespace {

void *dalloc(qfdtd_ctx *c, size_t bytes) {
  void *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (c->af) p = c->af(bytes, c->au);
  else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  if (p) c->allocs.push_back(p);
  return p;
}

void free_all(qfdtd_ctx *c) {
  for (void *p : c->allocs) {
    if (c->ff) c->ff(p, c->au);
    else (void)hipFree(p);
  }
  c->allocs.clear();
}

qfdtd_status fail(qfdtd_ctx *c, qfdtd_status s, const std::string &msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return s;
}

#define QF_HIP(c, call)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail(c, QFDTD_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

#define QF_LAUNCHED(c)                                                                           \
  do {                                                                                           \
    hipError_t e_ = hipGetLastError();                                                           \
    if (e_ != hipSuccess) return fail(c, QFDTD_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

#define QF_TRY(x)                          \
  do {                                     \
    qfdtd_status s_ = (x);                 \
    if (s_ != QFDTD_OK) return s_;         \
  } while (0)

// ------------------------------------------------------------- timing

// A timed launch carries a start/stop event pair in its own dispatch
// (hipExtLaunchKernel), so the measured interval is the kernel's execution.
int tbegin(qfdtd_ctx *c, int cls, double bytes, hipStream_t st) {
  Timer &t = c->timer;
  if (t.every <= 0) return -1;
  if ((t.seen[cls]++ % t.every) != 0) return -1;
  if (t.used == t.pool.size()) {
    if (t.pool.size() >= 8192) return -1;
    Timer::Rec r;
    if (hipEventCreate(&r.a) != hipSuccess) return -1;
    if (hipEventCreate(&r.b) != hipSuccess) { (void)hipEventDestroy(r.a); return -1; }
    t.pool.push_back(r);
  }
  Timer::Rec &r = t.pool[t.used];
  r.cls = cls;
  r.bytes = bytes;
  (void)st;
  return (int)t.used++;
}

void tcollect(qfdtd_ctx *c) {
  Timer &t = c->timer;
  for (size_t i = 0; i < t.used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.pool[i].a, t.pool[i].b) == hipSuccess) {
      t.count[t.pool[i].cls] += 1;
      t.sum_ms[t.pool[i].cls] += ms;
      t.sum_bytes[t.pool[i].cls] += t.pool[i].bytes;
    }
  }
  t.used = 0;
}

// ------------------------------------------------------------- launch lists

struct Entry {
  qfdtd_ctx *c;
  int which;        // 0 main desc, 1 FP64 measurement desc
  uint32_t mode;
  int tiles;
  int aux;
};

// F_SLAB: slab passes of any mode (split below into the steady kernel and F_SLAB_EDGE, the kernel
// of the chunk-edge and plain-transform modes)
enum Fam { F_PLANE, F_ROW, F_COL, F_STENCIL, F_STENCIL2, F_PARITY, F_TO64, F_GRAM, F_APPLY, F_EPART, F_KPART, F_GFIN, F_EFIN,
           F_SLAB, F_PENCIL, F_SLAB_EDGE };

// Algorithmic bytes moved by one member's share of a launch (for timing): every state is read
// and written once, and the per-site potential factor, which all k states of the member share,
// is read once per launch.
double entry_bytes(const Entry &e, Fam f) {
  const qfdtd_ctx *c = e.c;
  const bool meas = e.which == 1;
  const int k = e.which >= 2 ? c->gk[e.which - 2] : c->k;
  const double n = (double)k * c->n3();
  const double n3 = (double)c->n3();
  const double s = meas ? 16.0 : (double)c->csz();
  const double fsz = (c->vcomplex ? 2.0 : 1.0) * (meas ? 8.0 : (double)c->rsz());
  switch (f) {
    case F_PLANE:
    case F_ROW:
    case F_SLAB:
    case F_SLAB_EDGE:
      // A/B combine: read alt and psi and V, write psi (and alt when the forward follows)
      if (e.mode & M_COMB) return n * (3 * s + ((e.mode & M_FWD) ? s : 0.0)) + n3 * fsz;
      return n * 2 * s + ((e.mode & (M_PRE | M_MID | M_POST)) ? n3 * fsz : 0.0);
    case F_COL:
    case F_PENCIL: return n * 2 * s;
    case F_STENCIL: return n * 2 * s + n3 * fsz;
    case F_STENCIL2: return 2 * (n * 2 * s + n3 * fsz);    // two steps per launch
    default: return n * 2 * s;
  }
}

qfdtd_status run_family(Fam f, std::vector<Entry> &es, bool dbl, int KS = 0, hipStream_t sto = nullptr);

// Transform passes are instantiated per lattice size.  Entries are split by
// size group; a group with one size uses that size's kernel, a group with
// several sizes its multi-size kernel (KS = -2 - group), one launch per group.
qfdtd_status run_fft_family(Fam f, std::vector<Entry> &es, bool dbl, hipStream_t sto) {
  for (int gi = 0; gi < 5; ++gi) {
    std::vector<Entry> sub;
    int n0 = -1;
    bool multi = false;
    for (auto &e : es)
      if (size_group(e.c->N) == gi) {
        sub.push_back(e);
        if (n0 < 0) n0 = e.c->N;
        else if (e.c->N != n0) multi = true;
      }
    if (sub.empty()) continue;
    if (multi && f == F_PLANE && !g_grp[gi].plane[dbl]) multi = false;
    if (!multi) {
      std::vector<int> sizes;
      for (auto &e : sub)
        if (std::find(sizes.begin(), sizes.end(), e.c->N) == sizes.end()) sizes.push_back(e.c->N);
      for (int N : sizes) {
        std::vector<Entry> one;
        for (auto &e : sub)
          if (e.c->N == N) one.push_back(e);
        QF_TRY(run_family(f, one, dbl, -1, sto));
      }
    } else {
      QF_TRY(run_family(f, sub, dbl, -2 - gi, sto));
    }
  }
  return QFDTD_OK;
}

qfdtd_status run_family(Fam f, std::vector<Entry> &es, bool dbl, int KS, hipStream_t sto) {
  if (es.empty()) return QFDTD_OK;
  if (f == F_SLAB) {
    // steady slab passes and the other modes run in separate kernels
    const uint32_t steady = M_INV | M_MID | M_FWD;
    std::vector<Entry> st_es, ed_es;
    for (auto &e : es) (e.mode == steady ? st_es : ed_es).push_back(e);
    if (!ed_es.empty()) {
      if (!st_es.empty()) QF_TRY(run_family(F_SLAB, st_es, dbl, KS, sto));
      return run_family(F_SLAB_EDGE, ed_es, dbl, KS, sto);
    }
  }
  if ((f == F_PLANE || f == F_ROW || f == F_COL) && KS >= 0) return run_fft_family(f, es, dbl, sto);
  const int grp = KS <= -2 ? -2 - KS : -1;   // multi-size kernel of this group
  qfdtd_ctx *c0 = es[0].c;
  hipStream_t st = sto ? sto : c0->st;
  for (size_t base = 0; base < es.size(); base += MAX_LAUNCH) {
    LaunchList L;
    std::memset(&L, 0, sizeof(L));
    const size_t cnt = (es.size() - base) < (size_t)MAX_LAUNCH ? es.size() - base : MAX_LAUNCH;
    int total = 0;
    size_t lds = 0;
    double bytes = 0;
    for (size_t i = 0; i < cnt; ++i) {
      const Entry &e = es[base + i];
      L.tile_start[i] = total;
      L.descp[i] = (const void *)(e.c->d_desc + e.which);
      L.mode[i] = (uint16_t)e.mode;
      L.aux[i] = e.aux;
      total += e.tiles;
      const FftKernels &K = g_fft[e.c->N];
      size_t l = 0;
      if (f == F_PLANE) l = K.plane_lds[dbl];
      else if (f == F_ROW) l = K.row_lds[dbl];
      else if (f == F_COL) l = K.col_lds[dbl];
      else if (f == F_SLAB || f == F_SLAB_EDGE) l = K.slab_lds[e.c->split_v];
      else if (f == F_PENCIL) l = K.pencil_lds[e.c->split_v];
      if (l > lds) lds = l;
      if (grp >= 0 && (f == F_PLANE || f == F_ROW || f == F_COL))
        lds = g_grp_lds[grp][f == F_PLANE ? 0 : (f == F_ROW ? 1 : 2)][dbl];
      bytes += entry_bytes(e, f);
    }
    L.n = (int)cnt;
    L.tile_start[cnt] = total;
    int cls = -1;
    // only the pass kernels launched below with an event pair are timed; transforms of the FP64
    // measurement copy count as measurement
    bool meas_copy = false;
    for (size_t i = 0; i < cnt; ++i) meas_copy = meas_copy || es[base + i].which == 1;
    if (f == F_PLANE || f == F_ROW || f == F_COL)
      cls = meas_copy ? TC_MEAS : (f == F_PLANE ? TC_PLANE : f == F_ROW ? TC_ROW : TC_COL);
    else if (f == F_STENCIL || f == F_STENCIL2) cls = TC_STENCIL;
    else if (f == F_SLAB || f == F_SLAB_EDGE) cls = TC_SLAB;
    else if (f == F_PENCIL) cls = TC_PENCIL;
    const int tix = cls >= 0 ? tbegin(c0, cls, bytes, st) : -1;
    const FftKernels &K = g_fft[es[base].c->N];
    void *kargs[] = {(void *)&L};
    hipEvent_t ea = tix >= 0 ? c0->timer.pool[tix].a : nullptr;
    hipEvent_t eb = tix >= 0 ? c0->timer.pool[tix].b : nullptr;
    const void *fplane = grp >= 0 ? g_grp[grp].plane[dbl] : K.plane[dbl];
    const int ntplane = grp >= 0 ? g_grp[grp].plane_nt[dbl] : K.plane_nt;
    const void *frow = grp >= 0 ? g_grp[grp].row[dbl] : K.row[dbl];
    const void *fcol = grp >= 0 ? g_grp[grp].col[dbl] : K.col[dbl];
    // timed launches carry their event pair in the dispatch; untimed ones use the
    // plain launch, which can also be captured into a graph
    auto go = [&](const void *fn, int nt, size_t sh) {
      if (tix >= 0) (void)hipExtLaunchKernel(fn, dim3(total), dim3(nt), kargs, sh, st, ea, eb, 0);
      else (void)hipLaunchKernel(fn, dim3(total), dim3(nt), kargs, sh, st);
    };
    switch (f) {
      case F_PLANE: go(fplane, ntplane, lds); break;
      case F_ROW: go(frow, LINE_THREADS, lds); break;
      case F_COL: go(fcol, LINE_THREADS, lds); break;
      case F_SLAB: go(K.slab[c0->split_v], K.slab_nt[c0->split_v], lds); break;
      case F_SLAB_EDGE: go(K.slab_edge[c0->split_v], K.slab_nt[c0->split_v], lds); break;
      case F_PENCIL: go(K.pencil[c0->split_v], K.pencil_nt[c0->split_v], lds); break;
      case F_STENCIL: go(stencil_kernel(dbl), RED_THREADS, 0); break;
      case F_STENCIL2: go(stencil2_kernel(), S2_THREADS, 0); break;
      case F_PARITY: launch_parity(L, total, dbl, st); break;
      case F_TO64: launch_to64(L, total, dbl, st); break;
      case F_GRAM: launch_gram(L, total, KS, dbl, st); break;
      case F_APPLY: launch_apply(L, total, KS, dbl, st); break;
      case F_EPART: launch_energy_partials(L, total, KS, dbl, st); break;
      case F_KPART: launch_kin_partials(L, total, KS, st); break;
      case F_GFIN: launch_gram_finalize(L, st); break;
      case F_EFIN: launch_energy_finalize(L, st); break;
    }
    QF_LAUNCHED(c0);
  }
  return QFDTD_OK;
}


// run a family separately for each distinct k (kernels templated on k)
qfdtd_status run_by_k(Fam f, std::vector<Entry> &es, bool dbl) {
  for (int KS = 1; KS <= MAX_STATES; ++KS) {
    std::vector<Entry> sub;
    for (auto &e : es)
      if (e.c->k == KS) sub.push_back(e);
    QF_TRY(run_family(f, sub, dbl, KS));
  }
  return QFDTD_OK;
}

// run a single-size kernel family once per distinct N and split variant (split-x2 passes)
qfdtd_status run_by_size(Fam f, std::vector<Entry> &es, bool dbl) {
  std::vector<int> keys;
  auto key_of = [&](const Entry &e) { return e.c->N * 4 + e.c->split_v; };
  for (auto &e : es)
    if (std::find(keys.begin(), keys.end(), key_of(e)) == keys.end()) keys.push_back(key_of(e));
  for (int kk : keys) {
    std::vector<Entry> one;
    for (auto &e : es)
      if (key_of(e) == kk) one.push_back(e);
    QF_TRY(run_family(f, one, dbl, -1));
  }
  return QFDTD_OK;
}

// ------------------------------------------------------------- measurement

// parity projection + orthonormalisation; leaves every state in psi
qfdtd_status orthonormalise(std::vector<qfdtd_ctx *> &ms) {
  if (ms.empty()) return QFDTD_OK;
  const bool dbl = ms[0]->dbl;
  std::vector<Entry> par, gram, fin, app;
  for (auto *c : ms) {
    const long long tot = (long long)c->k * c->n3();
    int src = c->cur;    // 0: psi, 1: alt
    if (c->any_parity) {
      par.push_back({c, 0, src ? (uint32_t)M_SWAP : 0u, ew_tiles_host(tot), 0});
      src = 1 - src;
    }
    gram.push_back({c, 0, src ? (uint32_t)M_SWAP : 0u, c->nblk_red, 0});
    fin.push_back({c, 0, 0u, 1, 0});
    app.push_back({c, 0, src ? (uint32_t)M_SWAP : 0u, ew_tiles_host((long long)c->n3()), 0});
    c->cur = 0;
    c->fresh = false;
  }
  QF_TRY(run_family(F_PARITY, par, dbl));
  QF_TRY(run_by_k(F_GRAM, gram, dbl));
  QF_TRY(run_family(F_GFIN, fin, dbl));
  QF_TRY(run_by_k(F_APPLY, app, dbl));
  return QFDTD_OK;
}

// FP64 forward transform of the scratch copy (FFT members)
qfdtd_status fwd64(std::vector<qfdtd_ctx *> &ms) {
  std::vector<Entry> pl, rw, c2, c1;
  for (auto *c : ms) {
    if (c->plane64) pl.push_back({c, 1, M_FWD, plane_tiles(c->N, c->k), 0});
    else {
      rw.push_back({c, 1, M_FWD, row_tiles(c->N, c->k, true), 0});
      c2.push_back({c, 1, M_FWD, col_tiles(c->N, c->k, true), 0});
    }
    c1.push_back({c, 1, M_FWD | M_AXIS1, col_tiles(c->N, c->k, true), 0});
  }
  QF_TRY(run_family(F_PLANE, pl, true));
  QF_TRY(run_family(F_ROW, rw, true));
  QF_TRY(run_family(F_COL, c2, true));
  QF_TRY(run_family(F_COL, c1, true));
  return QFDTD_OK;
}

// E_i = <psi_i|H|psi_i>/<psi_i|psi_i> in FP64; `slot` >= 0 also records a trace row
qfdtd_status energies(std::vector<qfdtd_ctx *> &ms, bool with_trace) {
  if (ms.empty()) return QFDTD_OK;
  const bool dbl = ms[0]->dbl;
  std::vector<Entry> ep, to, kp, fin;
  std::vector<qfdtd_ctx *> ffts;
  for (auto *c : ms) {
    ep.push_back({c, 0, 0u, c->nblk_red, 0});
    if (c->fft()) {
      to.push_back({c, 0, 0u, ew_tiles_host((long long)c->k * c->n3()), 0});
      kp.push_back({c, 1, 0u, c->nblk_red, 0});
      ffts.push_back(c);
    }
    int slot = -1;
    if (with_trace && c->trace_on && c->trace_n < c->trace_cap) slot = (int)c->trace_n++;
    fin.push_back({c, 0, 0u, 1, slot});
  }
  QF_TRY(run_by_k(F_EPART, ep, dbl));
  QF_TRY(run_family(F_TO64, to, dbl));
  QF_TRY(fwd64(ffts));
  QF_TRY(run_by_k(F_KPART, kp, true));
  QF_TRY(run_family(F_EFIN, fin, dbl));
  return QFDTD_OK;
}

// ------------------------------------------------------------- one chunk

// One FFT member with its states split into two or three groups, each group's pass
// chain on its own stream: a group's plane pass (transform arithmetic bound)
// overlaps the other group's column pass (memory bound); with the split-x2
// schedule a group's pencil pass (one tile per CU, its loads, transforms and
// stores in turn) overlaps the other group's slab pass.  Forked from and joined
// to the context stream, so ordering with the caller is unchanged.
qfdtd_status run_chunk_grouped(qfdtd_ctx *c, int n) {
  const bool dbl = c->dbl;
  QF_HIP(c, hipEventRecord(c->ev_fork, c->st));
  for (int g = 0; g < c->ngroups; ++g) QF_HIP(c, hipStreamWaitEvent(c->gst[g], c->ev_fork, 0));
  for (int g = 0; g < c->ngroups; ++g) {
    const int which = 2 + g, kg = c->gk[g];
    hipStream_t st = c->gst[g];
    if (c->split) {
      const int v = c->split_v;
      const int ps = (c->N <= SLAB_STATE_TILES_MAX_N && kg > 1) ? kg : 1;
      std::vector<Entry> s0{{c, which, M_PRE | M_FWD, ps * slab_tiles(c->N, v), ps > 1 ? 1 : 0}};
      QF_TRY(run_family(F_SLAB, s0, dbl, 0, st));
      for (int s = 0; s < n; ++s) {
        std::vector<Entry> pe{{c, which, M_FWD | M_KIN | M_INV, pencil_tiles(c->N, kg, v), 0}};
        const uint32_t rs = (s == n - 1) ? (M_INV | M_POST) : (M_INV | M_MID | M_FWD);
        std::vector<Entry> s1{{c, which, rs, ps * slab_tiles(c->N, v), ps > 1 ? 1 : 0}};
        QF_TRY(run_family(F_PENCIL, pe, dbl, 0, st));
        QF_TRY(run_family(F_SLAB, s1, dbl, 0, st));
      }
      QF_HIP(c, hipEventRecord(c->ev_join[g], st));
      continue;
    }
    std::vector<Entry> pl{{c, which, M_PRE | M_FWD, plane_tiles(c->N, kg), 0}};
    QF_TRY(run_family(F_PLANE, pl, dbl, 0, st));
    for (int s = 0; s < n; ++s) {
      std::vector<Entry> c1{{c, which, M_FWD | M_KIN | M_INV | M_AXIS1, col_tiles(c->N, kg, dbl), 0}};
      const uint32_t rs = (s == n - 1) ? (M_INV | M_POST) : (M_INV | M_MID | M_FWD);
      std::vector<Entry> p2{{c, which, rs, plane_tiles(c->N, kg), 0}};
      QF_TRY(run_family(F_COL, c1, dbl, 0, st));
      QF_TRY(run_family(F_PLANE, p2, dbl, 0, st));
    }
    QF_HIP(c, hipEventRecord(c->ev_join[g], st));
  }
  for (int g = 0; g < c->ngroups; ++g) QF_HIP(c, hipStreamWaitEvent(c->st, c->ev_join[g], 0));
  return QFDTD_OK;
}

Entry slab_entry(qfdtd_ctx *c, uint32_t mode) {
  const int ps = (c->N <= SLAB_STATE_TILES_MAX_N && c->k > 1) ? c->k : 1;
  return {c, 0, mode, ps * slab_tiles(c->N, c->split_v), ps > 1 ? 1 : 0};
}

qfdtd_status run_chunk(std::vector<qfdtd_ctx *> &ms, std::vector<int> &n) {
  if (ms.empty()) return QFDTD_OK;
  // while launches are timed the state groups run on one stream, so that every timed launch
  // has the device to itself (as under a profiler) and its duration is the kernel's own
  if (ms.size() == 1 && ms[0]->ngroups >= 2 && n[0] > 0 && ms[0]->timer.every <= 0)
    return run_chunk_grouped(ms[0], n[0]);
  const bool dbl = ms[0]->dbl;
  int maxn = 0;
  for (int v : n) maxn = v > maxn ? v : maxn;
  std::vector<Entry> pl, rw, c2, c1, sten, sten2, sl, pen;
  // chunk start: h then forward transforms along x3 (and x2)
  for (size_t j = 0; j < ms.size(); ++j) {
    qfdtd_ctx *c = ms[j];
    if (!c->fft() || n[j] <= 0) continue;
    if (c->split) {
      sl.push_back(slab_entry(c, M_PRE | M_FWD));
      continue;
    }
    // A/B update: the forward transform of psi goes to alt; psi stays for the combine
    const uint32_t start = c->scheme == SCHEME_AB ? (uint32_t)(M_FWD | M_ALT) : (uint32_t)(M_PRE | M_FWD);
    const uint32_t onalt = c->scheme == SCHEME_AB ? (uint32_t)M_ALT : 0u;
    if (c->plane) pl.push_back({c, 0, start, plane_tiles(c->N, c->k), 0});
    else {
      rw.push_back({c, 0, start, row_tiles(c->N, c->k, dbl), 0});
      c2.push_back({c, 0, M_FWD | onalt, col_tiles(c->N, c->k, dbl), 0});
    }
  }
  QF_TRY(run_by_size(F_SLAB, sl, dbl));
  QF_TRY(run_family(F_PLANE, pl, dbl));
  QF_TRY(run_family(F_ROW, rw, dbl));
  QF_TRY(run_family(F_COL, c2, dbl));
  for (int s = 0; s < maxn; ++s) {
    c1.clear(); c2.clear(); pl.clear(); rw.clear(); sten.clear(); sten2.clear(); sl.clear(); pen.clear();
    std::vector<Entry> c2f;
    for (size_t j = 0; j < ms.size(); ++j) {
      qfdtd_ctx *c = ms[j];
      if (s >= n[j]) continue;
      if (!c->fft()) {
        // two fused steps at even s while two steps remain; a chunk of odd length ends with
        // one single step
        const uint32_t sw = c->cur ? (uint32_t)M_SWAP : 0u;
        if (c->stencil2 && (s & 1)) continue;                // advanced by the pass at s - 1
        if (c->stencil2 && s + 1 < n[j]) sten2.push_back({c, 0, sw, stencil2_tiles_host(c->N, c->k), 0});
        else sten.push_back({c, 0, sw, stencil_tiles_host(c->N, c->k), 0});
        c->cur ^= 1;
        continue;
      }
      const bool last = (s == n[j] - 1);
      if (c->split) {
        pen.push_back({c, 0, M_FWD | M_KIN | M_INV, pencil_tiles(c->N, c->k, c->split_v), 0});
        sl.push_back(slab_entry(c, last ? (uint32_t)(M_INV | M_POST) : (uint32_t)(M_INV | M_MID | M_FWD)));
        continue;
      }
      const bool ab = c->scheme == SCHEME_AB;
      const uint32_t onalt = ab ? (uint32_t)M_ALT : 0u;
      uint32_t rs = last ? (M_INV | M_POST) : (M_INV | M_MID | M_FWD);
      if (ab) rs = last ? (uint32_t)(M_INV | M_COMB) : (uint32_t)(M_INV | M_COMB | M_FWD | M_ALT);
      c1.push_back({c, 0, M_FWD | M_KIN | M_INV | M_AXIS1 | onalt, col_tiles(c->N, c->k, dbl), 0});
      if (c->plane) pl.push_back({c, 0, rs, plane_tiles(c->N, c->k), 0});
      else {
        c2.push_back({c, 0, M_INV | onalt, col_tiles(c->N, c->k, dbl), 0});
        rw.push_back({c, 0, rs, row_tiles(c->N, c->k, dbl), 0});
        if (!last) c2f.push_back({c, 0, M_FWD | onalt, col_tiles(c->N, c->k, dbl), 0});
      }
    }
    QF_TRY(run_family(F_COL, c1, dbl));
    QF_TRY(run_family(F_COL, c2, dbl));
    QF_TRY(run_by_size(F_PENCIL, pen, dbl));
    QF_TRY(run_by_size(F_SLAB, sl, dbl));
    QF_TRY(run_family(F_PLANE, pl, dbl));
    QF_TRY(run_family(F_ROW, rw, dbl));
    QF_TRY(run_family(F_COL, c2f, dbl));
    QF_TRY(run_family(F_STENCIL2, sten2, dbl));
    QF_TRY(run_family(F_STENCIL, sten, dbl));
  }
  return QFDTD_OK;
}

qfdtd_status upload_desc(qfdtd_ctx *c) {
  QF_HIP(c, hipMemcpyAsync(c->d_desc, c->hd, sizeof(c->hd), hipMemcpyHostToDevice, c->st));
  return QFDTD_OK;
}

qfdtd_status set_dt(qfdtd_ctx *c, double dt) {
  if (dt == c->cur_dt) return QFDTD_OK;
  launch_dt_tables(c->dbl, c->v64, c->vcomplex ? 1 : 0, c->N, dt, c->vtab, c->hfac, c->h2fac, c->ktab, c->ksym64,
                   c->kin, c->scheme, c->st);
  QF_LAUNCHED(c);
  for (int w = 0; w < 2 + MAX_GROUPS; ++w) {
    c->hd[w].dt = dt;
    c->hd[w].stencil_c = dt / (2.0 * c->m * c->a * c->a);
  }
  QF_TRY(upload_desc(c));
  // the descriptor upload reads host memory that may change again: wait for it
  QF_HIP(c, hipStreamSynchronize(c->st));
  c->cur_dt = dt;
  return QFDTD_OK;
}

qfdtd_status check_status(qfdtd_ctx *c, bool wait) {
  if (!c->status_pending) return QFDTD_OK;
  if (wait) QF_HIP(c, hipEventSynchronize(c->status_ev));
  else if (hipEventQuery(c->status_ev) != hipSuccess) return QFDTD_OK;
  c->status_pending = false;
  if (*c->h_status != 0.0) {
    c->poisoned = true;
    c->set_mask = 0;
    return fail(c, QFDTD_E_NUMERIC, "non-finite value or collapsed norm during orthonormalisation");
  }
  return QFDTD_OK;
}

qfdtd_status post_status(qfdtd_ctx *c) {
  QF_HIP(c, hipMemcpyAsync(c->h_status, c->energy + 2 * MAX_STATES, sizeof(double), hipMemcpyDeviceToHost, c->st));
  QF_HIP(c, hipEventRecord(c->status_ev, c->st));
  c->status_pending = true;
  return QFDTD_OK;
}

qfdtd_status validate_common(qfdtd_ctx *c) {
  if (c->poisoned) return fail(c, QFDTD_E_STATE, "context poisoned by an earlier numeric failure; set every state again");
  const uint32_t all = (c->k >= 32) ? 0xffffffffu : ((1u << c->k) - 1u);
  if ((c->set_mask & all) != all) return fail(c, QFDTD_E_STATE, "not every state has been set");
  return QFDTD_OK;
}

// Largest stable dt of the A/B update with an FFT kinetic term: dt max T <= 2,
// max T at k = (pi, pi, pi) (eqs. HK1-HK3).
double ab_dt_bound(int kin, double a, double m) {
  double tmax;
  if (kin == KIN_P2) tmax = 3.0 * M_PI * M_PI / (2.0 * m * a * a);
  else if (kin == KIN_REL) tmax = std::sqrt(12.0 / (a * a) + m * m) - m;
  else tmax = 6.0 / (m * a * a);
  return 2.0 / tmax;
}

qfdtd_status batch_evolve_impl(qfdtd_ctx *const *members, int32_t n, const int64_t *steps, const double *dt) {
  std::vector<qfdtd_ctx *> ms;
  std::vector<int64_t> rem;
  for (int j = 0; j < n; ++j) {
    qfdtd_ctx *c = members[j];
    QF_TRY(check_status(c, false));
    QF_TRY(validate_common(c));
    if (!(dt[j] > 0.0) || !std::isfinite(dt[j])) return fail(c, QFDTD_E_UNSTABLE_DT, "dt must be positive and finite");
    if (c->kin == KIN_FDTD && dt[j] > c->m * c->a * c->a / 3.0)
      return fail(c, QFDTD_E_UNSTABLE_DT, "H_K^(0) needs dt <= m a^2 / 3");
    if (c->kin != KIN_FDTD && c->scheme == SCHEME_AB && dt[j] > ab_dt_bound(c->kin, c->a, c->m))
      return fail(c, QFDTD_E_UNSTABLE_DT, "the A/B update needs dt <= 2 / max T(k)");
    if (steps[j] < 0) return fail(c, QFDTD_E_INVALID, "steps must be >= 0");
    if (j > 0 && (c->dbl != members[0]->dbl || c->st != members[0]->st))
      return fail(c, QFDTD_E_INVALID, "batch members need the same precision and stream");
    for (int i = 0; i < j; ++i)
      if (members[i] == c) return fail(c, QFDTD_E_INVALID, "a context appears twice in the batch");
  }
  for (int j = 0; j < n; ++j) {
    QF_TRY(set_dt(members[j], dt[j]));
    ms.push_back(members[j]);
    rem.push_back(steps[j]);
  }
  std::vector<qfdtd_ctx *> fr;
  for (auto *c : ms)
    if (c->fresh) fr.push_back(c);
  QF_TRY(orthonormalise(fr));
  // A single context replays a captured graph of each chunk shape (steps in
  // the chunk) after its first use; kernel arguments are captured by value and
  // point at buffers that live as long as the context.
  if (n == 1 && ms[0]->graphs && !ms[0]->trace_on && ms[0]->timer.every <= 0) {
    qfdtd_ctx *c = ms[0];
    int64_t rem0 = rem[0];
    while (rem0 > 0) {
      const int cn = (int)(rem0 < c->K ? rem0 : c->K);
      hipGraphExec_t ex = nullptr;
      for (auto &g : c->chunk_graphs)
        if (g.first == cn) ex = g.second;
      if (!ex) {
        hipGraph_t gr = nullptr;
        if (hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          (void)hipGetLastError();
          c->graphs = false;
          break;
        }
        std::vector<qfdtd_ctx *> one{c};
        std::vector<int> nn{cn};
        qfdtd_status st1 = run_chunk(one, nn);
        if (st1 == QFDTD_OK) st1 = orthonormalise(one);
        hipError_t ee = hipStreamEndCapture(c->st, &gr);
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(c->st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
          hipGraph_t junk = nullptr;
          (void)hipStreamEndCapture(c->st, &junk);
          if (junk) (void)hipGraphDestroy(junk);
          ee = hipErrorUnknown;
        }
        if (st1 != QFDTD_OK || ee != hipSuccess || !gr ||
            hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess) {
          if (gr) (void)hipGraphDestroy(gr);
          (void)hipGetLastError();
          c->graphs = false;   // fall back to direct launches for this context
          c->cur = 0;          // nothing captured ran; the states are where the chunk found them
          c->err.clear();
          break;
        }
        (void)hipGraphDestroy(gr);
        c->chunk_graphs.push_back({cn, ex});
      }
      QF_HIP(c, hipGraphLaunch(ex, c->st));
      rem0 -= cn;
    }
    rem[0] = rem0;
  }
  // Several members: capture each distinct chunk shape (active members and their
  // step counts) once and replay it, when every member allows graphs.
  bool bgraph = n > 1;
  for (auto *c : ms) bgraph = bgraph && c->graphs && !c->trace_on && c->timer.every <= 0;
  for (;;) {
    std::vector<qfdtd_ctx *> act;
    std::vector<int> cn;
    for (size_t j = 0; j < ms.size(); ++j)
      if (rem[j] > 0) {
        act.push_back(ms[j]);
        cn.push_back((int)(rem[j] < ms[j]->K ? rem[j] : ms[j]->K));
      }
    if (act.empty()) break;
    if (bgraph) {
      std::vector<std::pair<uint64_t, int>> key;
      for (size_t j = 0; j < act.size(); ++j) key.push_back({act[j]->serial, cn[j]});
      std::lock_guard<std::mutex> lk(g_batch_mu);
      BatchGraph *hit = nullptr;
      for (auto &bg : g_batch_graphs)
        if (bg.key == key) hit = &bg;
      bool replay = false;
      if (!hit) {
        if (g_batch_graphs.size() >= MAX_BATCH_GRAPHS) {
          if (g_batch_graphs.front().exec) (void)hipGraphExecDestroy(g_batch_graphs.front().exec);
          g_batch_graphs.erase(g_batch_graphs.begin());
        }
        g_batch_graphs.push_back({key, nullptr});     // first sighting: direct launches below
      } else if (hit->exec) {
        replay = true;
      } else {
        hipStream_t st0 = act[0]->st;
        hipGraph_t gr = nullptr;
        hipGraphExec_t ex = nullptr;
        std::vector<int> saved_cur;
        for (auto *c : act) saved_cur.push_back(c->cur);
        bool ok = hipStreamBeginCapture(st0, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
          qfdtd_status s1 = run_chunk(act, cn);
          if (s1 == QFDTD_OK) s1 = orthonormalise(act);
          hipError_t ee = hipStreamEndCapture(st0, &gr);
          hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
          if (hipStreamIsCapturing(st0, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
            hipGraph_t junk = nullptr;
            (void)hipStreamEndCapture(st0, &junk);
            if (junk) (void)hipGraphDestroy(junk);
            ee = hipErrorUnknown;
          }
          ok = s1 == QFDTD_OK && ee == hipSuccess && gr &&
               hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) == hipSuccess;
          if (gr) (void)hipGraphDestroy(gr);
        }
        if (!ok) {
          // nothing captured ran: the states are where the chunk found them
          for (size_t j = 0; j < act.size(); ++j) { act[j]->cur = saved_cur[j]; act[j]->err.clear(); }
          (void)hipGetLastError();
          bgraph = false;     // this call continues with direct launches
        } else {
          hit->exec = ex;
          replay = true;
        }
      }
      if (replay) {
        QF_HIP(act[0], hipGraphLaunch(hit->exec, act[0]->st));
        size_t q = 0;
        for (size_t j = 0; j < ms.size(); ++j)
          if (rem[j] > 0) rem[j] -= cn[q++];
        continue;
      }
    }
    QF_TRY(run_chunk(act, cn));
    QF_TRY(orthonormalise(act));
    std::vector<qfdtd_ctx *> tr;
    for (auto *c : act)
      if (c->trace_on) tr.push_back(c);
    QF_TRY(energies(tr, true));
    size_t q = 0;
    for (size_t j = 0; j < ms.size(); ++j)
      if (rem[j] > 0) rem[j] -= cn[q++];
  }
  for (auto *c : ms) QF_TRY(post_status(c));
  return QFDTD_OK;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

size_t qfdtd_footprint(int32_t N, int32_t kinetic, int32_t precision, int32_t n_states) {
  if (N <= 0 || n_states <= 0) return 0;
  const size_t n3 = (size_t)N * N * N, k = (size_t)n_states;
  const size_t cs = precision ? 16 : 8, rs = precision ? 8 : 4;
  size_t b = k * n3 * cs;                                  // psi
  b += k * n3 * cs;                                        // alt (upper bound)
  b += n3 * 16;                                            // v64 (upper bound: complex)
  b += (kinetic == KIN_FDTD ? 1 : 2) * n3 * 2 * rs;        // vtab or h, h^2 (upper bound: complex)
  b += k * n3 * 16;                                        // FP64 scratch
  b += 2 * 1024 * MAX_PAIRS * 2 * 8 + 64 * 1024;           // partials, small tables
  return b;
}

qfdtd_status qfdtd_create(qfdtd_ctx **out, int32_t N, double a, double m, int32_t kinetic, const qfdtd_potential *V,
                          const qfdtd_options *opt) {
  if (!out) return fail(nullptr, QFDTD_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!V) return fail(nullptr, QFDTD_E_INVALID, "potential is NULL");
  if (kinetic < 0 || kinetic > 3) return fail(nullptr, QFDTD_E_INVALID, "kinetic must be 0..3");
  if (!(a > 0.0) || !std::isfinite(a)) return fail(nullptr, QFDTD_E_INVALID, "a must be > 0");
  if (!(m > 0.0) || !std::isfinite(m)) return fail(nullptr, QFDTD_E_INVALID, "m must be > 0");
  if (N < 8 || (N & 1)) return fail(nullptr, QFDTD_E_UNSUPPORTED_N, "N must be even and >= 8");
  if (kinetic != KIN_FDTD && (N > 256 || !smooth235(N)))
    return fail(nullptr, QFDTD_E_UNSUPPORTED_N, "FFT kinetic terms need N <= 256 with factors 2, 3, 5 only");
  if (kinetic == KIN_FDTD && N > 512) return fail(nullptr, QFDTD_E_UNSUPPORTED_N, "N must be <= 512");
  qfdtd_options o;
  std::memset(&o, 0, sizeof(o));
  o.n_states = 3;
  if (opt) o = *opt;
  if (o.precision != 0 && o.precision != 1) return fail(nullptr, QFDTD_E_INVALID, "precision must be 0 or 1");
  if (o.n_states < 1 || o.n_states > MAX_STATES) return fail(nullptr, QFDTD_E_INVALID, "n_states must be 1..8");
  if (o.measure_every < 0) return fail(nullptr, QFDTD_E_INVALID, "measure_every must be >= 0");
  if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr))
    return fail(nullptr, QFDTD_E_INVALID, "dev_alloc and dev_free must be given together");
  if (V->kind < 0 || V->kind > 4) return fail(nullptr, QFDTD_E_INVALID, "unknown potential kind");
  if (V->kind == 0 && !V->grid) return fail(nullptr, QFDTD_E_INVALID, "QFDTD_V_GRID needs grid");
  if (V->kind == 4) {
    if (!V->knots || V->n_knots < 3 || V->n_knots > 4096) return fail(nullptr, QFDTD_E_INVALID, "spline needs 3..4096 knots");
    for (int j = 1; j < V->n_knots; ++j)
      if (!(V->knots[2 * j] > V->knots[2 * (j - 1)])) return fail(nullptr, QFDTD_E_INVALID, "spline knots must increase in r");
  }
  for (int i = 0; i < o.n_states && o.sectors; ++i)
    if (o.sectors[i] < 0 || o.sectors[i] > 5) return fail(nullptr, QFDTD_E_INVALID, "sector must be 0..5");
  {
    hipError_t e = fft_table_init();
    if (e != hipSuccess) return fail(nullptr, QFDTD_E_DEVICE, std::string("kernel attributes: ") + hipGetErrorString(e));
  }
  qfdtd_ctx *c = new qfdtd_ctx();
  c->N = N; c->a = a; c->m = m; c->kin = kinetic;
  c->prec = o.precision; c->dbl = o.precision == 1;
  c->k = o.n_states;
  c->K = o.measure_every > 0 ? o.measure_every : 50;
  c->st = (hipStream_t)o.hip_stream;
  c->af = o.dev_alloc; c->ff = o.dev_free; c->au = o.alloc_user;
  for (int i = 0; i < c->k; ++i) {
    const int s = o.sectors ? o.sectors[i] : 0;
    if (s < 0 || s > 5) { delete c; return fail(nullptr, QFDTD_E_INVALID, "sector must be 0..5"); }
    c->sectors[i] = s;
    if (s) c->any_parity = true;
  }
  const size_t n3 = c->n3();
  // complex potential?
  if (V->grid) {
    for (size_t g = 0; g < n3; ++g)
      if (V->grid[2 * g + 1] != 0.0) { c->vcomplex = true; break; }
  }
  if (c->fft() && !g_fft[N].col[0]) {
    delete c;
    return fail(nullptr, QFDTD_E_UNSUPPORTED_N, "no transform kernels for this N");
  }
  c->scheme = (c->fft() && (o.flags & QFDTD_F_AB_SCHEME)) ? SCHEME_AB : SCHEME_SPLIT;
  c->split_v = (int)QFDTD_SPLIT_VARIANT(o.flags);
  c->split = c->fft() && c->scheme == SCHEME_SPLIT && (o.flags & QFDTD_F_SPLIT_X2) && !c->dbl &&
             g_fft[N].slab[c->split_v] != nullptr;
  c->plane = c->fft() && g_fft[N].plane[c->dbl ? 1 : 0] != nullptr && !(o.flags & QFDTD_F_ROWCOL) && !c->split;
  c->plane64 = c->fft() && g_fft[N].plane[1] != nullptr;
  c->nblk_red = red_blocks(n3);
  c->trace_on = o.trace_energies ? 1 : 0;
  c->graphs = !(o.flags & QFDTD_F_NO_GRAPH);
  c->stencil2 = !c->fft() && !c->dbl && !(o.flags & QFDTD_F_STENCIL_1STEP);
  c->serial = g_next_serial.fetch_add(1);
  c->trace_cap = c->trace_on ? 4096 : 0;

  auto bail = [&](qfdtd_status s, const std::string &msg) {
    for (int g = 0; g < MAX_GROUPS; ++g) {
      if (c->gst[g]) (void)hipStreamDestroy(c->gst[g]);
      if (c->ev_join[g]) (void)hipEventDestroy(c->ev_join[g]);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    free_all(c);
    if (c->h_status) (void)hipHostFree(c->h_status);
    if (c->status_ev) (void)hipEventDestroy(c->status_ev);
    delete c;
    return fail(nullptr, s, msg);
  };
  const size_t cs = c->csz(), rs = c->rsz();
  const size_t fsz = (c->vcomplex ? 2 : 1) * rs;
  c->psi = dalloc(c, c->k * n3 * cs);
  const bool ab = c->scheme == SCHEME_AB;
  if (!c->fft() || c->any_parity || ab) c->alt = dalloc(c, c->k * n3 * cs);
  c->v64 = (double *)dalloc(c, n3 * 8 * (c->vcomplex ? 2 : 1));
  if (!c->fft() || ab) c->vtab = dalloc(c, n3 * fsz);
  else { c->hfac = dalloc(c, n3 * fsz); c->h2fac = dalloc(c, n3 * fsz); }
  c->ktab = dalloc(c, N * rs);
  c->tw = dalloc(c, N * cs);
  c->tw64 = (double2 *)dalloc(c, N * 16);
  c->ksym64 = (double *)dalloc(c, N * 8);
  c->scratch64 = (double2 *)dalloc(c, c->k * n3 * 16);
  c->partials = (double *)dalloc(c, 2 * (size_t)c->nblk_red * MAX_PAIRS * 2 * 8);
  c->coef = (double *)dalloc(c, MAX_STATES * MAX_STATES * 2 * 8);
  c->energy = (double *)dalloc(c, ENERGY_WORDS * 8);
  if (c->trace_on) c->trace = (double *)dalloc(c, (size_t)c->trace_cap * c->k * 2 * 8);
  c->d_desc = (PassDesc *)dalloc(c, sizeof(c->hd));
  bool ok = c->psi && c->v64 && c->ktab && c->tw && c->tw64 && c->ksym64 && c->scratch64 && c->partials && c->coef &&
            c->energy && c->d_desc && ((c->fft() && !ab) || (c->alt && c->vtab)) &&
            (!c->fft() || ab || (c->hfac && c->h2fac)) &&
            (!c->any_parity || c->alt) && (!c->trace_on || c->trace);
  if (!ok) return bail(QFDTD_E_NOMEM, "device allocation failed");
  if (hipHostMalloc((void **)&c->h_status, sizeof(double)) != hipSuccess) return bail(QFDTD_E_NOMEM, "pinned allocation failed");
  *c->h_status = 0.0;
  if (hipEventCreateWithFlags(&c->status_ev, hipEventDisableTiming) != hipSuccess)
    return bail(QFDTD_E_DEVICE, "event creation failed");

  // ---- potential (FP64, on the device)
  double *d_knots = nullptr;
  int nk = 0;
  if (V->kind == 4) {
    nk = V->n_knots;
    std::vector<double> h(3 * nk);
    std::vector<double> x(nk), y(nk), M(nk, 0.0);
    for (int j = 0; j < nk; ++j) { x[j] = V->knots[2 * j]; y[j] = V->knots[2 * j + 1]; }
    // natural spline: second derivatives from the tridiagonal system (Thomas algorithm)
    std::vector<double> cp(nk, 0.0), dp(nk, 0.0);
    for (int j = 1; j < nk - 1; ++j) {
      const double h0 = x[j] - x[j - 1], h1 = x[j + 1] - x[j];
      const double sub = h0, diag = 2.0 * (h0 + h1), sup = h1;
      const double rhs = 6.0 * ((y[j + 1] - y[j]) / h1 - (y[j] - y[j - 1]) / h0);
      const double den = diag - sub * cp[j - 1];
      cp[j] = sup / den;
      dp[j] = (rhs - sub * dp[j - 1]) / den;
    }
    for (int j = nk - 2; j >= 1; --j) M[j] = dp[j] - cp[j] * M[j + 1];
    for (int j = 0; j < nk; ++j) { h[j] = x[j]; h[nk + j] = y[j]; h[2 * nk + j] = M[j]; }
    if (hipMalloc(&d_knots, h.size() * 8) != hipSuccess) return bail(QFDTD_E_NOMEM, "knot buffer");
    if (hipMemcpy(d_knots, h.data(), h.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d_knots);
      return bail(QFDTD_E_DEVICE, "knot upload");
    }
  }
  const double2 *d_add = nullptr;
  if (V->grid) {
    if (hipMemcpyAsync(c->scratch64, V->grid, n3 * 16, hipMemcpyHostToDevice, c->st) != hipSuccess) {
      if (d_knots) (void)hipFree(d_knots);
      return bail(QFDTD_E_DEVICE, "potential grid upload");
    }
    d_add = c->scratch64;
  }
  (void)hipGetLastError();    // clear an error an earlier call on this thread left behind
  launch_potential(c->v64, c->vcomplex ? 1 : 0, N, a, V->kind, V->p, d_knots, nk, d_add, c->st);
  launch_tables(c->dbl, c->tw, c->tw64, c->ksym64, N, kinetic, a, m, c->st);
  hipError_t le = hipGetLastError();
  hipError_t se = hipStreamSynchronize(c->st);
  if (d_knots) (void)hipFree(d_knots);
  if (le != hipSuccess || se != hipSuccess)
    return bail(QFDTD_E_DEVICE, std::string("setup kernels: ") + hipGetErrorString(le != hipSuccess ? le : se));

  // ---- descriptors
  for (int w = 0; w < 2; ++w) {
    PassDesc &d = c->hd[w];
    std::memset(&d, 0, sizeof(d));
    d.psi = w ? (void *)c->scratch64 : c->psi;
    d.alt = c->alt;
    d.vtab = c->vtab;
    d.hfac = c->hfac;
    d.h2fac = c->h2fac;
    d.ktab = c->ktab;
    d.tw = w ? (const void *)c->tw64 : c->tw;
    d.tw64 = c->tw64;
    d.ksym64 = c->ksym64;
    d.v64 = c->v64;
    d.scratch64 = c->scratch64;
    d.partials = c->partials;
    d.coef = c->coef;
    d.energy = c->energy;
    d.trace = c->trace;
    d.N = N; d.k = c->k; d.kin = kinetic; d.vcomplex = c->vcomplex ? 1 : 0;
    d.nst = make_plan(N, d.radix);
    for (int i = 0; i < c->k; ++i) d.sector[i] = c->sectors[i];
    d.nblk_red = c->nblk_red;
    d.scheme = c->scheme;
    d.a = a; d.m = m; d.dt = 0.0; d.stencil_c = 0.0;
    d.inv_n3 = 1.0 / (double)n3;
  }
  // state groups for the two-stream schedule (plane or split-x2 schedule, k >= 2)
  for (int g = 0; g < MAX_GROUPS; ++g) c->hd[2 + g] = c->hd[0];
  if (c->fft() && (c->plane || c->split) && c->k >= 2 && !(o.flags & QFDTD_F_SINGLE_STREAM) && !ab) {
    c->ngroups = ((o.flags & QFDTD_F_THREE_GROUPS) && c->k >= 3) ? 3 : 2;
    size_t first = 0;
    bool okg = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int g = 0; g < c->ngroups; ++g) {
      // states split as evenly as possible, the larger groups first
      c->gk[g] = c->k / c->ngroups + (g < c->k % c->ngroups ? 1 : 0);
      c->hd[2 + g].psi = (char *)c->psi + first * n3 * cs;
      c->hd[2 + g].k = c->gk[g];
      first += (size_t)c->gk[g];
      okg = okg && hipStreamCreateWithFlags(&c->gst[g], hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&c->ev_join[g], hipEventDisableTiming) == hipSuccess;
    }
    if (!okg) return bail(QFDTD_E_DEVICE, "stream creation failed");
  }
  if (upload_desc(c) != QFDTD_OK || hipMemsetAsync(c->energy, 0, ENERGY_WORDS * 8, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess)
    return bail(QFDTD_E_DEVICE, "descriptor upload");
  *out = c;
  return QFDTD_OK;
}

qfdtd_status qfdtd_set_state(qfdtd_ctx *c, int32_t i, const double *psi) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (!psi) return fail(c, QFDTD_E_INVALID, "psi is NULL");
  if (i < 0 || i >= c->k) return fail(c, QFDTD_E_INVALID, "state index out of range");
  QF_TRY(check_status(c, true));
  const size_t n3 = c->n3();
  QF_HIP(c, hipMemcpyAsync(c->scratch64, psi, n3 * 16, hipMemcpyHostToDevice, c->st));
  launch_from64_slot(c->dbl, (char *)c->psi + (size_t)i * n3 * c->csz(), c->scratch64, n3, c->st);
  QF_LAUNCHED(c);
  QF_HIP(c, hipStreamSynchronize(c->st));
  c->set_mask |= 1u << i;
  c->fresh = true;
  const uint32_t all = (1u << c->k) - 1u;
  if ((c->set_mask & all) == all && c->poisoned) {
    c->poisoned = false;
    QF_HIP(c, hipMemsetAsync(c->energy + 2 * MAX_STATES, 0, 8, c->st));
  }
  return QFDTD_OK;
}

qfdtd_status qfdtd_set_state_noise(qfdtd_ctx *c, int32_t i, uint64_t seed) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (i < 0 || i >= c->k) return fail(c, QFDTD_E_INVALID, "state index out of range");
  QF_TRY(check_status(c, false));
  launch_noise(c->dbl, (char *)c->psi + (size_t)i * c->n3() * c->csz(), c->n3(), seed, i, c->st);
  QF_LAUNCHED(c);
  c->set_mask |= 1u << i;
  c->fresh = true;
  const uint32_t all = (1u << c->k) - 1u;
  if ((c->set_mask & all) == all && c->poisoned) {
    c->poisoned = false;
    QF_HIP(c, hipMemsetAsync(c->energy + 2 * MAX_STATES, 0, 8, c->st));
  }
  return QFDTD_OK;
}

qfdtd_status qfdtd_set_state_device(qfdtd_ctx *c, int32_t i, const void *psi_dev) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (!psi_dev) return fail(c, QFDTD_E_INVALID, "psi_dev is NULL");
  if (i < 0 || i >= c->k) return fail(c, QFDTD_E_INVALID, "state index out of range");
  QF_TRY(check_status(c, false));
  const size_t bytes = c->n3() * c->csz();
  QF_HIP(c, hipMemcpyAsync((char *)c->psi + (size_t)i * bytes, psi_dev, bytes, hipMemcpyDeviceToDevice, c->st));
  c->set_mask |= 1u << i;
  c->fresh = true;
  const uint32_t all = (1u << c->k) - 1u;
  if ((c->set_mask & all) == all && c->poisoned) {
    c->poisoned = false;
    QF_HIP(c, hipMemsetAsync(c->energy + 2 * MAX_STATES, 0, 8, c->st));
  }
  return QFDTD_OK;
}

qfdtd_status qfdtd_evolve(qfdtd_ctx *c, int64_t steps, double dt) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  qfdtd_ctx *m[1] = {c};
  return batch_evolve_impl(m, 1, &steps, &dt);
}

qfdtd_status qfdtd_batch_evolve(qfdtd_ctx *const *members, int32_t n, const int64_t *steps, const double *dt) {
  if (!members || !steps || !dt || n < 1) return fail(nullptr, QFDTD_E_INVALID, "bad batch arguments");
  for (int j = 0; j < n; ++j)
    if (!members[j]) return fail(nullptr, QFDTD_E_INVALID, "NULL batch member");
  return batch_evolve_impl(members, n, steps, dt);
}

static qfdtd_status measure_host(qfdtd_ctx *c) {
  QF_TRY(check_status(c, true));
  QF_TRY(validate_common(c));
  std::vector<qfdtd_ctx *> one{c};
  if (c->fresh) QF_TRY(orthonormalise(one));
  QF_TRY(energies(one, false));
  QF_TRY(post_status(c));
  QF_TRY(check_status(c, true));
  return QFDTD_OK;
}

qfdtd_status qfdtd_states(qfdtd_ctx *c, int32_t k, double *en, double *psi) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (k < 1 || k > c->k) return fail(c, QFDTD_E_INVALID, "k out of range");
  QF_TRY(measure_host(c));
  std::vector<double> e(2 * MAX_STATES);
  QF_HIP(c, hipMemcpyAsync(e.data(), c->energy, 2 * MAX_STATES * 8, hipMemcpyDeviceToHost, c->st));
  QF_HIP(c, hipStreamSynchronize(c->st));
  if (en) std::memcpy(en, e.data(), (size_t)2 * k * 8);
  if (psi) {
    const size_t n3 = c->n3();
    for (int i = 0; i < k; ++i) {
      const void *src = (const char *)c->psi + (size_t)i * n3 * c->csz();
      if (c->dbl) {
        QF_HIP(c, hipMemcpyAsync(psi + (size_t)i * 2 * n3, src, n3 * 16, hipMemcpyDeviceToHost, c->st));
      } else {
        launch_to64_slot(false, c->scratch64, src, n3, c->st);
        QF_LAUNCHED(c);
        QF_HIP(c, hipMemcpyAsync(psi + (size_t)i * 2 * n3, c->scratch64, n3 * 16, hipMemcpyDeviceToHost, c->st));
      }
    }
    QF_HIP(c, hipStreamSynchronize(c->st));
  }
  return QFDTD_OK;
}

qfdtd_status qfdtd_states_device(qfdtd_ctx *c, int32_t k, double *en, void *psi_dev) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (k < 1 || k > c->k) return fail(c, QFDTD_E_INVALID, "k out of range");
  QF_TRY(measure_host(c));
  if (en) {
    std::vector<double> e(2 * MAX_STATES);
    QF_HIP(c, hipMemcpyAsync(e.data(), c->energy, 2 * MAX_STATES * 8, hipMemcpyDeviceToHost, c->st));
    QF_HIP(c, hipStreamSynchronize(c->st));
    std::memcpy(en, e.data(), (size_t)2 * k * 8);
  }
  if (psi_dev) QF_HIP(c, hipMemcpyAsync(psi_dev, c->psi, (size_t)k * c->n3() * c->csz(), hipMemcpyDeviceToDevice, c->st));
  return QFDTD_OK;
}

qfdtd_status qfdtd_gram_matrix(qfdtd_ctx *c, double *G) {
  if (!c || !G) return fail(c, QFDTD_E_INVALID, "NULL argument");
  QF_TRY(check_status(c, false));
  QF_TRY(validate_common(c));
  std::vector<Entry> gram{{c, 0, c->cur ? (uint32_t)M_SWAP : 0u, c->nblk_red, 0}};
  QF_TRY(run_by_k(F_GRAM, gram, c->dbl));
  // the orthonormalisation coefficients are rewritten before every use, so their buffer
  // holds the sums here
  const int NP = c->k * (c->k + 1) / 2;
  launch_gram_sum(c->partials, c->nblk_red, 2 * NP, c->coef, c->st);
  QF_LAUNCHED(c);
  std::vector<double> g(2 * NP);
  QF_HIP(c, hipMemcpyAsync(g.data(), c->coef, (size_t)2 * NP * 8, hipMemcpyDeviceToHost, c->st));
  QF_HIP(c, hipStreamSynchronize(c->st));
  int p = 0;
  for (int i = 0; i < c->k; ++i)
    for (int j = i; j < c->k; ++j, ++p) {
      G[2 * (i * c->k + j)] = g[2 * p];
      G[2 * (i * c->k + j) + 1] = g[2 * p + 1];
      G[2 * (j * c->k + i)] = g[2 * p];
      G[2 * (j * c->k + i) + 1] = -g[2 * p + 1];
    }
  return QFDTD_OK;
}

qfdtd_status qfdtd_gram_residuals(qfdtd_ctx *c, double *r) {
  if (!c || !r) return fail(c, QFDTD_E_INVALID, "NULL argument");
  QF_TRY(check_status(c, false));
  QF_TRY(validate_common(c));
  std::vector<Entry> gram{{c, 0, c->cur ? (uint32_t)M_SWAP : 0u, c->nblk_red, 0}};
  QF_TRY(run_by_k(F_GRAM, gram, c->dbl));
  // aux = 1: the finalize kernel writes the Cholesky diagonal and leaves the orthonormalisation
  // coefficients and the status word alone
  std::vector<Entry> fin{{c, 0, 0u, 1, 1}};
  QF_TRY(run_family(F_GFIN, fin, c->dbl));
  std::vector<double> d(MAX_STATES);
  QF_HIP(c, hipMemcpyAsync(d.data(), c->energy + ENERGY_RDIAG, MAX_STATES * 8, hipMemcpyDeviceToHost, c->st));
  QF_HIP(c, hipStreamSynchronize(c->st));
  std::memcpy(r, d.data(), (size_t)c->k * 8);
  return QFDTD_OK;
}

qfdtd_status qfdtd_batch_energies(qfdtd_ctx *const *members, int32_t n, double *en) {
  if (!members || n < 1 || !en) return fail(nullptr, QFDTD_E_INVALID, "bad batch arguments");
  std::vector<qfdtd_ctx *> ms, fr;
  int kmax = 0;
  for (int j = 0; j < n; ++j) {
    qfdtd_ctx *c = members[j];
    if (!c) return fail(nullptr, QFDTD_E_INVALID, "NULL batch member");
    QF_TRY(check_status(c, false));
    QF_TRY(validate_common(c));
    if (c->dbl != members[0]->dbl || c->st != members[0]->st)
      return fail(c, QFDTD_E_INVALID, "batch members need the same precision and stream");
    ms.push_back(c);
    if (c->fresh) fr.push_back(c);
    kmax = c->k > kmax ? c->k : kmax;
  }
  QF_TRY(orthonormalise(fr));
  QF_TRY(energies(ms, false));
  std::vector<double> e(2 * MAX_STATES + 8);
  for (int j = 0; j < n; ++j) {
    qfdtd_ctx *c = ms[j];
    QF_HIP(c, hipMemcpyAsync(e.data(), c->energy, (2 * MAX_STATES + 1) * 8, hipMemcpyDeviceToHost, c->st));
    QF_HIP(c, hipStreamSynchronize(c->st));
    if (e[2 * MAX_STATES] != 0.0) {
      c->poisoned = true;
      c->set_mask = 0;
      return fail(c, QFDTD_E_NUMERIC, "non-finite energy or collapsed norm");
    }
    for (int i = 0; i < kmax; ++i) {
      en[2 * ((size_t)j * kmax + i)] = i < c->k ? e[2 * i] : 0.0;
      en[2 * ((size_t)j * kmax + i) + 1] = i < c->k ? e[2 * i + 1] : 0.0;
    }
  }
  return QFDTD_OK;
}

qfdtd_status qfdtd_energy_trace(qfdtd_ctx *c, double *out, int64_t cap, int64_t *n) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (!n) return fail(c, QFDTD_E_INVALID, "n is NULL");
  QF_HIP(c, hipStreamSynchronize(c->st));
  *n = c->trace_n;
  const int64_t rows = cap < c->trace_n ? cap : c->trace_n;
  if (out && rows > 0 && c->trace)
    QF_HIP(c, hipMemcpy(out, c->trace, (size_t)rows * c->k * 2 * 8, hipMemcpyDeviceToHost));
  return QFDTD_OK;
}

qfdtd_status qfdtd_enable_kernel_timing(qfdtd_ctx *c, int32_t every) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (every < 0) return fail(c, QFDTD_E_INVALID, "every must be >= 0");
  QF_HIP(c, hipStreamSynchronize(c->st));
  tcollect(c);
  Timer &t = c->timer;
  t.every = every;
  for (int i = 0; i < TC_N; ++i) { t.seen[i] = 0; t.count[i] = 0; t.sum_ms[i] = 0; t.sum_bytes[i] = 0; }
  return QFDTD_OK;
}

qfdtd_status qfdtd_kernel_stats(qfdtd_ctx *c, int32_t cls, int64_t *count, double *mean_ms, double *bytes) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (cls < 0 || cls >= TC_N) return fail(c, QFDTD_E_INVALID, "class out of range");
  QF_HIP(c, hipStreamSynchronize(c->st));
  tcollect(c);
  const Timer &t = c->timer;
  if (count) *count = t.count[cls];
  if (mean_ms) *mean_ms = t.count[cls] ? t.sum_ms[cls] / (double)t.count[cls] : 0.0;
  if (bytes) *bytes = t.count[cls] ? t.sum_bytes[cls] / (double)t.count[cls] : 0.0;
  return QFDTD_OK;
}

qfdtd_status qfdtd_transform_state(qfdtd_ctx *c, int32_t i, int32_t sign) {
  if (!c) return fail(nullptr, QFDTD_E_INVALID, "ctx is NULL");
  if (!c->fft()) return fail(c, QFDTD_E_INVALID, "transform needs an FFT kinetic term");
  if (i < 0 || i >= c->k || (sign != 1 && sign != -1)) return fail(c, QFDTD_E_INVALID, "bad state index or sign");
  // a one-state view of slot i: temporarily point the main descriptor at it
  PassDesc save = c->hd[0];
  c->hd[0].psi = (char *)c->psi + (size_t)i * c->n3() * c->csz();
  c->hd[0].k = 1;
  QF_TRY(upload_desc(c));
  std::vector<Entry> pl, rw, c2, c1;
  const uint32_t dir = sign < 0 ? M_FWD : M_INV;
  const bool dbl = c->dbl;
  if (c->plane) pl.push_back({c, 0, dir, plane_tiles(c->N, 1), 0});
  else {
    rw.push_back({c, 0, dir, row_tiles(c->N, 1, dbl), 0});
    c2.push_back({c, 0, dir, col_tiles(c->N, 1, dbl), 0});
  }
  c1.push_back({c, 0, dir | M_AXIS1 | (sign > 0 ? (uint32_t)M_SCALE : 0u), col_tiles(c->N, 1, dbl), 0});
  qfdtd_status s = QFDTD_OK;
  if (s == QFDTD_OK) s = run_family(F_PLANE, pl, dbl);
  if (s == QFDTD_OK) s = run_family(F_ROW, rw, dbl);
  if (s == QFDTD_OK) s = run_family(F_COL, c2, dbl);
  if (s == QFDTD_OK) s = run_family(F_COL, c1, dbl);
  QF_HIP(c, hipStreamSynchronize(c->st));
  c->hd[0] = save;
  QF_TRY(upload_desc(c));
  QF_HIP(c, hipStreamSynchronize(c->st));
  return s;
}

qfdtd_status qfdtd_state_pointer(qfdtd_ctx *c, int32_t i, void **ptr) {
  if (!c || !ptr) return fail(c, QFDTD_E_INVALID, "NULL argument");
  if (i < 0 || i >= c->k) return fail(c, QFDTD_E_INVALID, "state index out of range");
  *ptr = (char *)c->psi + (size_t)i * c->n3() * c->csz();
  return QFDTD_OK;
}

void qfdtd_destroy(qfdtd_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  for (auto &r : c->timer.pool) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto &g : c->chunk_graphs) (void)hipGraphExecDestroy(g.second);
  c->chunk_graphs.clear();
  drop_batch_graphs(c->serial);
  for (int g = 0; g < MAX_GROUPS; ++g) {
    if (c->gst[g]) { (void)hipStreamSynchronize(c->gst[g]); (void)hipStreamDestroy(c->gst[g]); }
    if (c->ev_join[g]) (void)hipEventDestroy(c->ev_join[g]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  free_all(c);
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->status_ev) (void)hipEventDestroy(c->status_ev);
  delete c;
}

const char *qfdtd_last_error(const qfdtd_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }


}  // extern "C"
