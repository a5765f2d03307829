/* Batched 16-point DFT stage on the two gfx950 execution units that could run it.
 *
 * The transform passes of the solver build their 128-point (and other) transforms from
 * radix-16/8/4/2/3/5 butterflies on the FP32 vector ALUs.  A matrix-core alternative computes
 * a radix-16 stage as a dense complex product Y = F16 X (F16 the 16 x 16 DFT matrix) with FP32
 * MFMA.  This library times both on the same data so that the choice between them rests on a
 * measurement.  It is a measurement tool beside the solver (libdftstage.so), not part of the
 * solver's C ABI.
 *
 * Operation (the discrete Fourier transform of the split-step, Sec. 2): for every vector v
 *   Y_v[i] = sum_k exp(-+2 pi i i k / 16) X_v[k],  i, k = 0..15
 * applied `reps` times in place on data held in registers: even repetitions forward (-),
 * odd ones inverse (+) followed by a multiply by 1/16, so an even count returns the input up
 * to rounding and an odd count gives the forward DFT.
 *
 * Layout: in and out are device arrays of nvec vectors x 16 points of interleaved complex
 * FP32 (re, im): point k of vector v at float offset 2 (16 v + k).  They may not overlap.
 *
 * Variants: DFT16_VALU (0) one vector per lane, the solver's radix-4 x 4 butterfly;
 *           DFT16_MFMA (1) 16 vectors per 16x16 tile, 16 v_mfma_f32_16x16x4_f32 per tile
 *           (four real products Fr Xr, Fi Xi, Fr Xi, Fi Xr in k-chunks of four).
 *
 * Errors (return value): 0 success; -1 invalid argument (unknown variant, nvec not a positive
 * multiple of 256, reps < 1, iters < 1, NULL pointer); -5 a HIP call failed.
 * dft16_stage_last_error() describes the last failure of the calling thread.
 */
#ifndef DFT_STAGE_H
#define DFT_STAGE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DFT16_VALU = 0, DFT16_MFMA = 1 };

/* One launch on `stream` (hipStream_t, NULL = default stream); stream-ordered, no host sync. */
int dft16_stage_run(int32_t variant, const void *in, void *out, int64_t nvec, int32_t reps, void *stream);

/* `iters` back-to-back launches bracketed by HIP events on `stream`; synchronises and writes
 * the mean milliseconds per launch to *ms_per_launch. */
int dft16_stage_time(int32_t variant, const void *in, void *out, int64_t nvec, int32_t reps, int32_t iters,
                     void *stream, double *ms_per_launch);

const char *dft16_stage_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
