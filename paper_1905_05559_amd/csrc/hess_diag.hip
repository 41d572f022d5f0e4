// Sustained MFMA rate (register-only stream); see include/hess_diag.h.
#include <algorithm>

#include "api_internal.h"
#include "hess_diag.h"
#include "mfma.h"

namespace hs {
namespace {

typedef float f16v_t __attribute__((ext_vector_type(16)));

// One kernel per instruction, each holding only its own accumulators (a shared body
// made the compiler shuttle every accumulator through other registers each iteration).
__global__ __launch_bounds__(256) void k_stream_f32(float* sink, int64_t iters) {
  const int l = threadIdx.x & 63;
  f4_t acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = f4_t{0.f, 0.f, 0.f, 0.f};
  const float a = 1e-3f * (float)l, b = 2e-3f;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i][0];
  if (s == -1.0e30f) sink[0] = s;  // never true: keeps the accumulators live
}

__device__ __forceinline__ void stream_operands(bf8_t& av, bf8_t& bv) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    av[i] = (__bf16)(1e-3f * (float)(l + i));
    bv[i] = (__bf16)(1e-3f * (float)i);
  }
}

__global__ __launch_bounds__(256, 2) void k_stream_bf16_16(float* sink, int64_t iters) {
  f4_t acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = f4_t{0.f, 0.f, 0.f, 0.f};
  bf8_t av, bv;
  stream_operands(av, bv);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i][0];
  if (s == -1.0e30f) sink[0] = s;
}

__global__ __launch_bounds__(256, 2) void k_stream_bf16_32(float* sink, int64_t iters) {
  f16v_t acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f16v_t{};
  bf8_t av, bv;
  stream_operands(av, bv);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) s += acc[i][0];
  if (s == -1.0e30f) sink[0] = s;
}

__global__ __launch_bounds__(256, 2) void k_stream_f64(float* sink, int64_t iters) {
  const int l = threadIdx.x & 63;
  d4_t acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = d4_t{0.0, 0.0, 0.0, 0.0};
  const double a = 1e-3 * (double)l, b = 2e-3;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i][0];
  if (s == -1.0e30) sink[0] = (float)s;
}

}  // namespace
}  // namespace hs

using namespace hs;

extern "C" hess_status hess_mfma_stream_rate(hess_ctx* ctx, int kind, int64_t iters, void* sink_v, double* tflops) {
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  if (kind < 0 || kind > 3 || iters < 1 || !tflops || !sink_v) return fail(ctx, HESS_E_ARG, "bad kind, iters or pointers");
  float* sink = static_cast<float*>(sink_v);
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int blocks = 8 * std::max(cus, 1);  // 8 workgroups of 4 wavefronts per compute unit
  // one flops-per-iteration count per kind, per wavefront
  const double per_iter[4] = {16.0 * 16 * 4 * 2 * 16, 16.0 * 16 * 32 * 2 * 16, 32.0 * 32 * 16 * 2 * 4,
                              16.0 * 16 * 4 * 2 * 16};
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float ms = 0.f;
  for (int rep = 0; rep < 2; ++rep) {
    (void)hipEventRecord(e0, ex.stream);
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_stream_f32, dim3(blocks), dim3(256), 0, ex.stream, sink, iters); break;
      case 1: hipLaunchKernelGGL(k_stream_bf16_16, dim3(blocks), dim3(256), 0, ex.stream, sink, iters); break;
      case 2: hipLaunchKernelGGL(k_stream_bf16_32, dim3(blocks), dim3(256), 0, ex.stream, sink, iters); break;
      default: hipLaunchKernelGGL(k_stream_f64, dim3(blocks), dim3(256), 0, ex.stream, sink, iters); break;
    }
    (void)hipEventRecord(e1, ex.stream);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&ms, e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess || ms <= 0.f) return fail(ctx, HESS_E_DEVICE, "MFMA stream kernel failed");
  *tflops = per_iter[kind] * (double)iters * (double)blocks * 4.0 / ((double)ms * 1e9);
  return HESS_OK;
}
