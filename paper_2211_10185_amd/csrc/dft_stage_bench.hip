// Batched 16-point DFT stage: FP32 vector ALUs against FP32 matrix cores (gfx950).
//
// A measurement tool beside the solver: it decides whether a radix-16 stage of the transform
// passes would run faster as a dense 16 x 16 complex matrix product on MFMA than as the FFT
// butterfly the passes use.  Both kernels hold the data in registers and repeat the stage
// `reps` times (forward, then inverse with a 1/16 scale, alternately), so a large count times
// the arithmetic alone and reps = 1 a single stage between an HBM read and write.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <string>

#include "dft_stage.h"
#include "fft_core.h"

namespace {

using qf::C;
constexpr int BLOCK = 256;   // vectors per block in both variants (4 waves of 64)

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

// ---------------------------------------------------------------- VALU: one vector per lane
// The solver's radix-16 butterfly (4 x 4 with internal twiddles), on 16 values in registers.
__global__ void __launch_bounds__(BLOCK) k_dft16_valu(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                      int reps) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const float4 *src = reinterpret_cast<const float4 *>(in + v * 16);
  float2 x[16];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float4 q = src[i];
    x[2 * i] = make_float2(q.x, q.y);
    x[2 * i + 1] = make_float2(q.z, q.w);
  }
  int r = 0;
  for (; r + 1 < reps; r += 2) {
    qf::Dft<16, false, float2>::run(x);
    qf::Dft<16, true, float2>::run(x);
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = qf::cscale(x[i], 0.0625f);
  }
  if (r < reps) qf::Dft<16, false, float2>::run(x);
  float4 *dst = reinterpret_cast<float4 *>(out + v * 16);
#pragma unroll
  for (int i = 0; i < 8; ++i) dst[i] = make_float4(x[2 * i].x, x[2 * i].y, x[2 * i + 1].x, x[2 * i + 1].y);
}

// ---------------------------------------------------------------- MFMA: 16 vectors per tile
// v_mfma_f32_16x16x4_f32 computes D = A (16 x 4) B (4 x 16) + C.  Lane l = j + 16 q
// (j = l mod 16, q = l / 16) supplies A[j][q] and B[q][j] and receives D[4 q + r][j] in
// accumulator register r.  Product c (c = 0..3) of a tile contracts the DFT index
// k = 4 q + c: A[i][q] = F[i][4 q + c], B[q][j] = X[4 q + c][vector j].  The result
// register r of lane (j, q) then holds Y[4 q + r][vector j], which is exactly the operand
// B of product c = r for the next repetition: the stage chains without data movement.
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Y = F X for the four tiles of a wave; INV selects conj(F) (then Yr = Fr Xr + Fi Xi,
// Yi = Fr Xi - Fi Xr with fi the forward sine part).
template <bool INV>
__device__ __forceinline__ void tile_dft(float (&xr)[4][4], float (&xi)[4][4], const float (&fr)[4],
                                         const float (&fi)[4], const float (&nfi)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      yr = mfma(fr[c], xr[t][c], yr);
      yr = mfma(INV ? fi[c] : nfi[c], xi[t][c], yr);
      yi = mfma(fr[c], xi[t][c], yi);
      yi = mfma(INV ? nfi[c] : fi[c], xr[t][c], yi);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      xr[t][c] = yr[c];
      xi[t][c] = yi[c];
    }
  }
}

__global__ void __launch_bounds__(BLOCK) k_dft16_mfma(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                      int reps) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, q = lane >> 4;
  const int64_t v0 = ((int64_t)blockIdx.x * (BLOCK / 64) + wave) * 64;   // first vector of the wave
  // operand A: F[i = j][k = 4 q + c] = exp(-2 pi i j k / 16), generated in FP64
  float fr[4], fi[4], nfi[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int m = (j * (4 * q + c)) & 15;
    double s, co;
    sincos(-2.0 * M_PI * m / 16.0, &s, &co);
    fr[c] = (float)co;
    fi[c] = (float)s;
    nfi[c] = (float)-s;
  }
  float xr[4][4], xi[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float4 *src = reinterpret_cast<const float4 *>(in + (v0 + 16 * t + j) * 16 + 4 * q);
    const float4 a = src[0], b = src[1];
    xr[t][0] = a.x; xi[t][0] = a.y; xr[t][1] = a.z; xi[t][1] = a.w;
    xr[t][2] = b.x; xi[t][2] = b.y; xr[t][3] = b.z; xi[t][3] = b.w;
  }
  int r = 0;
  for (; r + 1 < reps; r += 2) {
    tile_dft<false>(xr, xi, fr, fi, nfi);
    tile_dft<true>(xr, xi, fr, fi, nfi);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        xr[t][c] *= 0.0625f;
        xi[t][c] *= 0.0625f;
      }
  }
  if (r < reps) tile_dft<false>(xr, xi, fr, fi, nfi);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float4 *dst = reinterpret_cast<float4 *>(out + (v0 + 16 * t + j) * 16 + 4 * q);
    dst[0] = make_float4(xr[t][0], xi[t][0], xr[t][1], xi[t][1]);
    dst[1] = make_float4(xr[t][2], xi[t][2], xr[t][3], xi[t][3]);
  }
}

int check(int32_t variant, const void *in, const void *out, int64_t nvec, int32_t reps) {
  if (variant != DFT16_VALU && variant != DFT16_MFMA) return fail(-1, "unknown variant");
  if (!in || !out) return fail(-1, "in or out is NULL");
  if (nvec <= 0 || nvec % BLOCK != 0) return fail(-1, "nvec must be a positive multiple of 256");
  if (nvec / BLOCK > 0x7fffffffLL) return fail(-1, "nvec too large");
  if (reps < 1) return fail(-1, "reps must be >= 1");
  return 0;
}

int launch(int32_t variant, const void *in, void *out, int64_t nvec, int32_t reps, hipStream_t st) {
  // every block covers exactly 256 whole vectors (nvec is a multiple of 256): no tail
  const dim3 grid((unsigned)(nvec / BLOCK)), block(BLOCK);
  if (variant == DFT16_VALU)
    hipLaunchKernelGGL(k_dft16_valu, grid, block, 0, st, (const float2 *)in, (float2 *)out, (int)reps);
  else
    hipLaunchKernelGGL(k_dft16_mfma, grid, block, 0, st, (const float2 *)in, (float2 *)out, (int)reps);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : fail(-5, std::string("launch: ") + hipGetErrorString(e));
}

}  // namespace

extern "C" {

int dft16_stage_run(int32_t variant, const void *in, void *out, int64_t nvec, int32_t reps, void *stream) {
  if (int e = check(variant, in, out, nvec, reps)) return e;
  return launch(variant, in, out, nvec, reps, (hipStream_t)stream);
}

int dft16_stage_time(int32_t variant, const void *in, void *out, int64_t nvec, int32_t reps, int32_t iters,
                     void *stream, double *ms_per_launch) {
  if (int e = check(variant, in, out, nvec, reps)) return e;
  if (iters < 1 || !ms_per_launch) return fail(-1, "iters must be >= 1 and ms_per_launch non-NULL");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(-5, "hipEventCreate");
  }
  int rc = 0;
  if (hipEventRecord(e0, st) != hipSuccess) rc = fail(-5, "hipEventRecord");
  for (int i = 0; i < iters && rc == 0; ++i) rc = launch(variant, in, out, nvec, reps, st);
  if (rc == 0 && hipEventRecord(e1, st) != hipSuccess) rc = fail(-5, "hipEventRecord");
  float ms = 0.f;
  if (rc == 0 && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = fail(-5, "event timing");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == 0) *ms_per_launch = (double)ms / iters;
  return rc;
}

const char *dft16_stage_last_error(void) { return g_err.c_str(); }

}  // extern "C"
