// Sustained MFMA rate (register-only stream); see include/hess_diag.h.
#include <algorithm>

#include "api_internal.h"
#include "hess_diag.h"
#include "mfma.h"

namespace hs {
namespace {

typedef float f16v_t __attribute__((ext_vector_type(16)));

template <int KIND>
__global__ __launch_bounds__(256) void k_mfma_stream(float* sink, int64_t iters) {
  const int l = threadIdx.x & 63;
  f4_t acc[16];
  d4_t dacc[16];
  f16v_t acc32[4];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    acc[i] = f4_t{0.f, 0.f, 0.f, 0.f};
    dacc[i] = d4_t{0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) acc32[i] = f16v_t{};
  const float a = 1e-3f * (float)l, b = 2e-3f;
  bf8_t av, bv;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    av[i] = (__bf16)(1e-3f * (float)(l + i));
    bv[i] = (__bf16)(1e-3f * (float)i);
  }
  for (int64_t it = 0; it < iters; ++it) {
    if (KIND == 0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
    } else if (KIND == 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
    } else if (KIND == 2) {
#pragma unroll
      for (int i = 0; i < 4; ++i) acc32[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc32[i], 0, 0, 0);
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) dacc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, (double)b, dacc[i], 0, 0, 0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i][0] + (float)dacc[i][0];
#pragma unroll
  for (int i = 0; i < 4; ++i) s += acc32[i][0];
  if (s == -1.0e30f) sink[0] = s;  // never true: keeps the accumulators live
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
      case 0: hipLaunchKernelGGL(k_mfma_stream<0>, dim3(blocks), dim3(256), 0, ex.stream, sink, iters); break;
      case 1: hipLaunchKernelGGL(k_mfma_stream<1>, dim3(blocks), dim3(256), 0, ex.stream, sink, iters); break;
      case 2: hipLaunchKernelGGL(k_mfma_stream<2>, dim3(blocks), dim3(256), 0, ex.stream, sink, iters); break;
      default: hipLaunchKernelGGL(k_mfma_stream<3>, dim3(blocks), dim3(256), 0, ex.stream, sink, iters); break;
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
