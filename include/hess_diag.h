/* Diagnostics for roofline context (not an operation of the method).
 *
 * hess_mfma_stream_rate: sustained rate of one MFMA instruction on this device,
 * measured by a kernel that keeps 16 independent accumulators per wavefront in
 * registers (no memory traffic) on every compute unit for `iters` iterations; the
 * result is what the matrix cores deliver at the clock they sustain under that load,
 * the practical ceiling beside the vendor peak.  kind: 0 = v_mfma_f32_16x16x4_f32,
 * 1 = v_mfma_f32_16x16x32_bf16, 2 = v_mfma_f32_32x32x16_bf16, 3 = v_mfma_f64_16x16x4_f64.
 * sink: device buffer of at least 4 bytes, owned by the caller (written only if the
 * accumulators reach an impossible value, so it only keeps the stream from being
 * optimised away).  *tflops (host) receives the algorithmic rate (2 flops per
 * multiply-add).  Synchronises the context's stream.  Errors: HESS_E_ARG (bad kind,
 * iters < 1, NULL pointers), HESS_E_DEVICE. */
#pragma once

#include "hess.h"

#ifdef __cplusplus
extern "C" {
#endif

hess_status hess_mfma_stream_rate(hess_ctx* ctx, int kind, int64_t iters, void* sink, double* tflops);

#ifdef __cplusplus
}
#endif
