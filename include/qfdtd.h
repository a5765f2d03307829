/*
 * qfdtd.h -- C ABI of the MI355X (gfx950) imaginary-time Schroedinger solver.
 *
 * The library evolves k wavefunctions on a periodic or walled N^3 lattice in
 * imaginary time and extracts the lowest states and their energies, as
 * described in arXiv:2211.10185 (QuantumFDTD v3):
 *
 *   H = H_K + V                                        Sec. 2, eq. (eq_schro)
 *   H_K^(0) 7-point finite differences, Dirichlet      Sec. 2, eq. (HK0); Sec. 1
 *   H_K^(1) FFT, sum k_l^2 / (2 A^2 M)                 Sec. 2, eq. (HK1)
 *   H_K^(2) FFT, 4 sum sin^2(k_l/2) / (2 A^2 M)        Sec. 2, eq. (HK2)
 *   H_K^(3) FFT, sqrt(4 sum sin^2(k_l/2) + (AM)^2)/A   Sec. 2, eq. (HK3)
 *   k_l = A p_l in {-pi + 2pi/N, ..., pi}              Sec. 2, after (HK3)
 *   -d/dtau Psi = H Psi; Psi = sum a_n Psi_n e^{-E_n tau}   Sec. 2, eq. (eq_iterat)
 *   excited states by orthogonal projection            Sec. 1
 *   parity projectors P^+, P^-, P^-_{p_k}              Sec. 3, beside Fig. 1
 *
 * Readings taken where the paper defers to its references:
 *   - FFT kinds use the symmetric split step  h F^-1[e^{-dt T} F[h psi]],
 *     h = e^{-dt V/2};  H_K^(0) uses psi <- A psi - B dt H_K^(0) psi with
 *     A = (1 - dt V/2)/(1 + dt V/2), B = 1/(1 + dt V/2).  The same A/B update with
 *     an FFT kinetic term is available as a second scheme (QFDTD_F_AB_SCHEME).
 *   - H_K^(0) is the standard 7-point Laplacian over A^2, times -1/(2M).
 *   - H_K^(3) is evolved and reported with the rest mass removed (T - M).
 *   - Site i_l has coordinate x_l = (i_l - N/2) A (origin on site N/2).
 *   - The k states are orthonormalised (Gram-Schmidt in state order, within
 *     each parity sector) every `measure_every` steps and after the last one.
 *   - Energies are the Rayleigh quotients <psi_i|H|psi_i>, complex when V is.
 *
 * Conventions
 *   - Every call returns a qfdtd_status; nothing throws across the ABI.
 *   - Host arrays are complex128, interleaved (re, im), C order with x3
 *     fastest: element (i1, i2, i3) at 2*((i1*N + i2)*N + i3).
 *   - The context owns all device memory it allocates (through the optional
 *     allocator hook, else hipMalloc).  Input arrays are copied during the
 *     call and stay owned by the caller; output arrays are caller-owned.
 *   - All device work is ordered on the context's stream.  Calls that return
 *     host data synchronise that stream before returning.
 *   - One context must not be used from two host threads at once.
 *   - After QFDTD_E_NUMERIC (NaN/Inf or a collapsed norm) or QFDTD_E_DEVICE
 *     the context is poisoned: qfdtd_evolve returns QFDTD_E_STATE until every
 *     state has been replaced with qfdtd_set_state.
 */
#ifndef QFDTD_H
#define QFDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QFDTD_OK = 0,
  QFDTD_E_INVALID = -1,        /* bad argument (null pointer, a <= 0, k out of range, ...) */
  QFDTD_E_UNSUPPORTED_N = -2,  /* N odd, N < 8, N > 512, or (FFT kinds) N not 2^a 3^b 5^c */
  QFDTD_E_UNSTABLE_DT = -3,    /* dt <= 0, H_K^(0) with dt > M A^2 / 3, or the A/B update of an
                                  FFT kind above its bound (QFDTD_F_AB_SCHEME) */
  QFDTD_E_NOMEM = -4,          /* device allocation failed */
  QFDTD_E_DEVICE = -5,         /* a HIP runtime call failed */
  QFDTD_E_NUMERIC = -6,        /* NaN/Inf or non-positive norm met during orthonormalisation */
  QFDTD_E_STATE = -7           /* context poisoned, or states not set */
} qfdtd_status;

/* H_K^(0..3), Sec. 2 eqs. (HK0)-(HK3). */
typedef enum {
  QFDTD_K_FDTD = 0,
  QFDTD_K_NR_P2 = 1,
  QFDTD_K_NR_SIN2 = 2,
  QFDTD_K_REL = 3
} qfdtd_kinetic;

typedef enum {
  QFDTD_V_GRID = 0,           /* V is `grid` */
  QFDTD_V_HARMONIC = 1,       /* V = p[0] r^2 / 2 */
  QFDTD_V_CORNELL = 2,        /* V = -p[0]/r_f + p[1] r_f,  r_f = max(r, p[2]) */
  QFDTD_V_COULOMB = 3,        /* V = -p[0]/r_f,             r_f = max(r, p[1]) */
  QFDTD_V_RADIAL_SPLINE = 4   /* natural cubic spline through (knots[2j], knots[2j+1]) = (r_j, V_j) */
} qfdtd_vkind;

/* Parity sectors (Sec. 3).  Reflection R_l maps site i_l to N - i_l
 * (mod N on the periodic lattice; onto the wall, where psi = 0, for FDTD).
 *   P^+ = (1 + R)/2, P^- = (1 - R)/2 with R = R_1 R_2 R_3,
 *   P^-_{p_k} = (1 + R_i R_j)(1 - R_k)/4, {i, j, k} = {1, 2, 3}.
 * On the walled lattice a site with some i_l = 0 mirrors onto the wall, so a state of
 * definite parity vanishes there: the projection sets those sites to zero, which keeps
 * the projectors idempotent. */
typedef enum {
  QFDTD_S_NONE = 0,
  QFDTD_S_PLUS = 1,
  QFDTD_S_MINUS = 2,
  QFDTD_S_PK1 = 3,
  QFDTD_S_PK2 = 4,
  QFDTD_S_PK3 = 5
} qfdtd_sector;

typedef struct {
  int32_t kind;              /* qfdtd_vkind */
  double p[4];               /* parameters, see qfdtd_vkind */
  const double *knots;       /* QFDTD_V_RADIAL_SPLINE: n_knots (r, V) pairs, r strictly increasing; host, copied */
  int32_t n_knots;           /* >= 3 */
  const double *grid;        /* host complex128 N^3 (re, im): the potential for QFDTD_V_GRID, otherwise
                                an addition to the analytic V (e.g. an imaginary part); NULL = none; copied */
} qfdtd_potential;

typedef void *(*qfdtd_alloc_fn)(size_t bytes, void *user);
typedef void (*qfdtd_free_fn)(void *ptr, void *user);

typedef struct {
  int32_t precision;          /* 0: complex64 states, FP32 transforms, FP64 reductions; 1: complex128 throughout */
  int32_t n_states;           /* k, 1..8 */
  const int32_t *sectors;     /* k qfdtd_sector values, or NULL for all QFDTD_S_NONE; copied */
  int32_t measure_every;      /* K >= 1: orthonormalise every K steps (0 = default 50) */
  int32_t trace_energies;     /* nonzero: also record E_i after every K-step chunk (qfdtd_energy_trace) */
  void *hip_stream;           /* hipStream_t for all work; NULL = the null stream */
  qfdtd_alloc_fn dev_alloc;   /* optional device allocator (e.g. a framework caching allocator) */
  qfdtd_free_fn dev_free;     /* must be given together with dev_alloc */
  void *alloc_user;           /* passed to dev_alloc / dev_free */
  uint32_t flags;             /* QFDTD_F_* bits */
} qfdtd_options;

/* qfdtd_options.flags */
#define QFDTD_F_SINGLE_STREAM 1u  /* do not split the states of an FFT solve into groups
                                     evolved on internal streams of their own */
#define QFDTD_F_ROWCOL 2u         /* FFT kinds: use the row + three column pass schedule even
                                     where an x2-x3 plane fits in LDS (schedule autotuning) */
#define QFDTD_F_NO_GRAPH 4u       /* qfdtd_evolve: launch every chunk directly instead of capturing
                                     a chunk into a HIP graph once and replaying it */
#define QFDTD_F_THREE_GROUPS 16u  /* FFT kinds, k >= 3: split the states into three groups on three
                                     internal streams instead of two (schedule autotuning) */
#define QFDTD_F_STENCIL_1STEP 32u /* H_K^(0) with complex64 states: one step per stencil pass.
                                     By default a pass advances two steps at once (eq. HK0
                                     applied twice in one sweep, the same operations per site,
                                     so the results are bit-identical) and halves the memory
                                     traffic per step; a chunk of odd length ends with a
                                     single step. */
#define QFDTD_F_SPLIT_X2 64u     /* FFT kinds, complex64, sizes with a split-x2 instantiation
                                     (N = 96, 100, 108, 120, 128, 144, 150, 160, 162, 180, 192,
                                     200, 216, 240, 250, 256):
                                     the two-pass schedule.  The x2 transform is split four-step
                                     style (N = N1 N2); a slab pass holds N1 rows of one x1 plane
                                     (of two at N = 128, 160 and 256, whose rows the state holds
                                     interleaved between the passes of a chunk)
                                     and does the x3 transforms around the potential factor and
                                     the stride-N2 part of x2, a pencil pass holds N2 consecutive
                                     rows of a few x3 columns over all x1 and does the other part
                                     of x2 and the x1 transforms around the kinetic factor.  Two
                                     passes over the state per step instead of four (schedule
                                     autotuning; ignored with QFDTD_F_AB_SCHEME). */
/* Flag bits 7-8: the split-x2 variant (schedule autotuning), read as QFDTD_SPLIT_VARIANT(flags):
 *   0: the size's default x2 = N1 x N2 with pencil tiles of 4 x3 columns (2 where 4 does not
 *      divide N);
 *   1 (QFDTD_F_SPLIT_NARROW): the same factors, pencil tiles of 2 columns (half the on-chip
 *      memory per tile, so two tiles share a compute unit);
 *   2 (QFDTD_F_SPLIT_WIDE), N = 128 and 256: 8 consecutive rows per pencil tile and 8 columns
 *      (row pieces twice as long as with 4 columns);
 *   3 (QFDTD_F_SPLIT_SWAPPED): the default factors swapped, x2 = N2 x N1 (fewer rows per slab
 *      tile, more per pencil tile), at the sizes where they differ.
 * A variant a size does not have runs the schedule the other flags select. */
#define QFDTD_F_SPLIT_NARROW 128u
#define QFDTD_F_SPLIT_WIDE 256u
#define QFDTD_F_SPLIT_SWAPPED 384u
#define QFDTD_SPLIT_VARIANT(flags) (((flags) >> 7) & 3u)
#define QFDTD_F_AB_SCHEME 8u      /* FFT kinds: step with the legacy update of H_K^(0) with the
                                     FFT kinetic term swapped in (Sec. 2, the update the paper
                                     keeps while changing H_K):  psi' = A psi - B dt H_K psi,
                                     A = (1 - dt V/2)/(1 + dt V/2), B = 1/(1 + dt V/2), with
                                     H_K psi = F^-1[T F[psi]].  Needs dt <= 2 / max T:
                                     4 m a^2/(3 pi^2) (H_K^(1)), m a^2/3 (H_K^(2)),
                                     2/(sqrt(12/a^2 + m^2) - m) (H_K^(3)); else
                                     qfdtd_evolve returns QFDTD_E_UNSTABLE_DT.  Ignored for
                                     H_K^(0), which always steps this way.  Default: the
                                     symmetric split-operator step. */

typedef struct qfdtd_ctx qfdtd_ctx;

/* Create a solver for an N^3 lattice of spacing a and mass m with kinetic term
 * `kinetic` and potential `V` (Sec. 2).  V is evaluated on the device in FP64 at
 * x_l = (i_l - N/2) a.  The states are unset until qfdtd_set_state.  On failure
 * *out is NULL and nothing is leaked.  opt may be NULL (complex64, k = 3, K = 50). */
qfdtd_status qfdtd_create(qfdtd_ctx **out, int32_t N, double a, double m, int32_t kinetic,
                          const qfdtd_potential *V, const qfdtd_options *opt);

/* Replace state i (0 <= i < k) with the host complex128 array psi (N^3 (re, im)).
 * The states are projected onto their sectors and orthonormalised before the next
 * evolution step (so the array need not be normalised).  Clears a poisoned context
 * once every state has been set again. */
qfdtd_status qfdtd_set_state(qfdtd_ctx *c, int32_t i, const double *psi);

/* Same, from a device buffer in the context's state precision (complex64 or
 * complex128, interleaved, N^3 elements).  Stream-ordered; no synchronisation. */
qfdtd_status qfdtd_set_state_device(qfdtd_ctx *c, int32_t i, const void *psi_dev);

/* Replace state i with seeded complex Gaussian noise generated on the device (Re and Im
 * independent N(0, 1) per site): Philox4x32-10 (Salmon et al., SC 2011) with counter
 * (x mod 2^32, x div 2^32, i, 0) for site x in C order and key (seed mod 2^32, seed div 2^32);
 * the four words give u1 = ((w0 2^21 + w1 div 2^11) + 1) 2^-53 and u2 likewise from w2, w3, and
 * the Box-Muller transform sqrt(-2 ln u1) (cos 2 pi u2 + i sin 2 pi u2) in FP64, stored in the
 * state precision.  A random initial guess without a host array (Sec. 2: any start with a
 * ground-state component converges).  Stream-ordered; no synchronisation. */
qfdtd_status qfdtd_set_state_noise(qfdtd_ctx *c, int32_t i, uint64_t seed);

/* Advance all k states by `steps` imaginary-time steps of size dt (Sec. 2, eq.
 * (eq_iterat)), orthonormalising every K steps and after the last one.  Enqueued on
 * the stream; returns without waiting, except that a NaN/Inf found by an earlier
 * call is reported here.  QFDTD_E_UNSTABLE_DT for H_K^(0) when dt > m a^2 / 3 and,
 * with QFDTD_F_AB_SCHEME, for an FFT kind when dt exceeds its bound (see the flag). */
qfdtd_status qfdtd_evolve(qfdtd_ctx *c, int64_t steps, double dt);

/* Energies of states 0..k-1 (energies[2i], energies[2i+1] = Re, Im of E_i; H_K^(3)
 * energies exclude the rest mass) and, if psi is not NULL, the states as host
 * complex128 [k][N^3] normalised to sum |psi|^2 = 1.  Synchronises the stream. */
qfdtd_status qfdtd_states(qfdtd_ctx *c, int32_t k, double *energies, double *psi);

/* Energies to host as above (synchronising), states copied device-to-device into
 * psi_dev ([k][N^3] in the state precision) on the stream. */
qfdtd_status qfdtd_states_device(qfdtd_ctx *c, int32_t k, double *energies, void *psi_dev);

/* Energies recorded after each chunk when trace_energies was set: out[(t*k + i)*2 + {0,1}]
 * for t < min(cap, recorded); *n = number of recorded chunks.  Synchronises. */
qfdtd_status qfdtd_energy_trace(qfdtd_ctx *c, double *out, int64_t cap, int64_t *n);

/* Evolve several contexts together: member j advances steps[j] steps of dt[j].  Each
 * pass of the step is one launch over the tiles of every member that takes it, so
 * lattices of different N, kinetic term and potential share the GPU.  All members
 * must have the same precision and the same stream.  Results are identical to
 * calling qfdtd_evolve on each member alone. */
qfdtd_status qfdtd_batch_evolve(qfdtd_ctx *const *members, int32_t n, const int64_t *steps,
                                const double *dt);

/* FP64 Gram matrix of the context's current states (Sec. 1: the overlaps that the
 * orthogonal projection removes):  G_ij = <psi_i|psi_j> = sum_x conj(psi_i(x)) psi_j(x),
 * reduced in FP64 in a fixed order.  The states are read as they are: as set (before any
 * orthonormalisation) or as left by the last evolve.  G: host, [k][k][2] (re, im), row-major,
 * caller-owned.  Synchronises the stream.  QFDTD_E_STATE if a state is unset. */
qfdtd_status qfdtd_gram_matrix(qfdtd_ctx *c, double *G);

/* Projected norms of the current states (Sec. 1: the orthogonal projection of snapshots):
 * r[j] = || psi_j - (projection of psi_j on the span of the earlier states of its sector) ||,
 * the diagonal of the FP64 Cholesky factor R of the sector's Gram matrix (G = R^H R), computed
 * on the device in a fixed summation order.  Its absolute error is about 1e-16 / r[j], so values
 * below about 1e-8 are rounding.  r: host, k doubles, caller-owned.  Synchronises the stream;
 * the states are not changed. */
qfdtd_status qfdtd_gram_residuals(qfdtd_ctx *c, double *r);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the FP64 Gram matrix of qfdtd_gram_matrix, of k
 * states given by a device pointer, with no context and no allocation.  Its partial sums live
 * in a fixed device array inside the library (576 KiB on each GPU that runs it, held until the
 * process ends); every call on a GPU uses that GPU's array, so calls that overlap in time on
 * one GPU (two streams, two host threads) race and must be serialised by the caller.
 *   psi:       device, [k][n_sites] interleaved complex64 (precision 0) or complex128 (1),
 *              caller-owned, read only.
 *   n_sites:   1 .. QFDTD_NOALLOC_MAX_SITES; k: 1..8.
 *   G:         device, [k][k][2] FP64 (re, im), row-major, caller-owned; written on the stream.
 *   hip_stream: hipStream_t (NULL = null stream).  Stream-ordered; nothing is synchronised.
 * Same summation order as qfdtd_gram_matrix for the same states, so the same bits.
 * QFDTD_E_INVALID for a NULL pointer or a size beyond these limits (message in
 * qfdtd_last_error(NULL)); QFDTD_E_DEVICE if the launch fails. */
#define QFDTD_NOALLOC_MAX_SITES (1ll << 27)
qfdtd_status qfdtd_gram_matrix_noalloc(const void *psi, int64_t n_sites, int32_t k, int32_t precision,
                                       double *G, void *hip_stream);

/* Batched energy readout: energies[2*(j*kmax + i) + {0,1}] for member j, state i < k_j.
 * kmax = largest k among the members.  Synchronises the (common) stream. */
qfdtd_status qfdtd_batch_energies(qfdtd_ctx *const *members, int32_t n, double *energies);

/* Device bytes the context for this problem would hold (for admission control). */
size_t qfdtd_footprint(int32_t N, int32_t kinetic, int32_t precision, int32_t n_states);

/* Complex potentials from ASCII files of numbers (Sec. 1: arbitrary complex potentials
 * loaded from ASCII files), for qfdtd_potential.grid with kind QFDTD_V_GRID.  Host only
 * (no device work).  A record is a line; '#' starts a comment; fields are separated by
 * blanks, tabs or commas; every record has the same number of fields:
 *   1: re    2: re im               N^3 records in C order (x3 fastest)
 *   4: i1 i2 i3 re    5: i1 i2 i3 re im   every site exactly once, in any order
 * grid: host, N^3 complex128 (re, im), caller-owned, filled on success.  QFDTD_E_INVALID
 * (message in qfdtd_last_error(NULL)) for a missing file, a malformed or non-finite number,
 * an index out of range, a repeated or missing site, or a wrong record count. */
qfdtd_status qfdtd_read_potential_ascii(const char *path, int32_t N, double *grid);

/* Write N^3 complex128 values as "re im" records in C order (17 significant digits, so
 * qfdtd_read_potential_ascii returns the same doubles).  QFDTD_E_INVALID if the file cannot
 * be written. */
qfdtd_status qfdtd_write_potential_ascii(const char *path, int32_t N, const double *grid);

/* Launch-level timing of the evolution kernels: when enabled, the context records a
 * pair of HIP events on its stream around every sampled launch, per kernel class.
 * qfdtd_kernel_stats returns, for class `cls` (0 plane, 1 row, 2 column, 3 stencil,
 * 4 measurement, 5 slab, 6 pencil), the number of timed launches, their mean duration in ms and the
 * algorithmic bytes one launch of that class moves: every state read once and written once,
 * plus the per-site potential factor, shared by the k states of a solve, read once.
 * While timing is enabled the states of an FFT solve are not split over internal
 * streams, so timed launches never overlap other kernels of the context.  every <= 0
 * disables timing.  Synchronises the stream. */
qfdtd_status qfdtd_enable_kernel_timing(qfdtd_ctx *c, int32_t every);
qfdtd_status qfdtd_kernel_stats(qfdtd_ctx *c, int32_t cls, int64_t *count, double *mean_ms,
                                double *bytes_per_launch);

/* Forward (sign = -1) or inverse (sign = +1, including 1/N^3) 3D DFT of state i in
 * place, in the state precision, with the library's transform kernels.  For checks
 * of the transform against a reference; FFT kinds only. */
qfdtd_status qfdtd_transform_state(qfdtd_ctx *c, int32_t i, int32_t sign);

/* Device pointer of state i (state precision, N^3 interleaved complex). */
qfdtd_status qfdtd_state_pointer(qfdtd_ctx *c, int32_t i, void **ptr);

void qfdtd_destroy(qfdtd_ctx *c);

/* Message for the last failing call on c, or, when c is NULL, of the last failing
 * context-free call on this host thread (qfdtd_create, the potential file functions). */
const char *qfdtd_last_error(const qfdtd_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* QFDTD_H */
