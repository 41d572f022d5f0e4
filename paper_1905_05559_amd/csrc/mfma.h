// MFMA wrappers for gfx950 (CDNA4), 64-wide wavefronts.
//
// 16x16x4 (f32 and f64): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
// The 16x16 result is held as D[row_of(l / 16, v)][l % 16], v = 0..3, where
// row_of(q, v) = 4q + v for f32 and q + 4v for f64 (measured on gfx950).
// 16x16x32 bf16: lane l supplies A[l % 16][8 * (l / 16) + 0..7] and
// B[8 * (l / 16) + 0..7][l % 16]; the result layout is the same as above.
#pragma once

#include "common.h"

namespace hs {

template <typename T>
struct MfmaOp;

template <>
struct MfmaOp<float> {
  using acc_t = f4_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ int row_of(int q, int v) { return 4 * q + v; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <>
struct MfmaOp<double> {
  using acc_t = d4_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ int row_of(int q, int v) { return q + 4 * v; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ f4_t mma_bf16(bf8_t a, bf8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Map a dispatch-order workgroup id to a logical tile id so that each of the 8
// XCDs (which receive workgroups round-robin) works on one contiguous range of
// logical tiles; neighbouring tiles then share operand panels in that XCD's L2.
// Returns -1 for padding workgroups.  grid must be a multiple of 8.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t grid, int64_t ntiles) {
  const int64_t per = grid >> 3;
  const int64_t t = (bid & 7) * per + (bid >> 3);
  return t < ntiles ? t : -1;
}

inline int64_t xcd_grid(int64_t ntiles) { return (ntiles + 7) & ~int64_t(7); }

}  // namespace hs
