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

// x = h + m + l with h, m, l BF16: h = RNE(x), m = RNE(x - h), l = RNE(x - h - m); both
// differences are exact in FP32, so |x - h - m - l| <= 2^-24 |x| (up to underflow).
// Two values at a time: one packed conversion per part.
typedef float f2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
// The residuals x - h are formed by v_dot2c_f32_bf16 as x + h.lo * (-1) + h.hi * 0 (and
// the mirror for the high half): one instruction per value instead of a widening and a
// subtraction; the result is exact (x - h is representable).  The two packed multipliers
// are produced by s_mov in SGPRs (SplitC): folded as an inline constant, the compiler's
// encoding of the pair (-1, 0) did not multiply by -1.
struct SplitC {
  bf2_t nlo, nhi;  // (-1, 0) and (0, -1)
};
__device__ __forceinline__ SplitC split_consts() {
  unsigned lo, hi;
  asm volatile("s_mov_b32 %0, 0x0000bf80" : "=s"(lo));
  asm volatile("s_mov_b32 %0, 0xbf800000" : "=s"(hi));
  return SplitC{__builtin_bit_cast(bf2_t, lo), __builtin_bit_cast(bf2_t, hi)};
}
__device__ __forceinline__ void split3x2(f2_t x, bf2_t& h, bf2_t& m, bf2_t& l, const SplitC& c) {
  h = __builtin_convertvector(x, bf2_t);
  const float r0 = __builtin_amdgcn_fdot2_f32_bf16(h, c.nlo, x[0], false);
  const float r1 = __builtin_amdgcn_fdot2_f32_bf16(h, c.nhi, x[1], false);
  m = __builtin_convertvector(f2_t{r0, r1}, bf2_t);
  const float s0 = __builtin_amdgcn_fdot2_f32_bf16(m, c.nlo, r0, false);
  const float s1 = __builtin_amdgcn_fdot2_f32_bf16(m, c.nhi, r1, false);
  l = __builtin_convertvector(f2_t{s0, s1}, bf2_t);
}
// operand parts of the six products, in order m m, l h, h l, m h, h m, h h (smallest first)
__device__ __forceinline__ const bf8_t& pr_x(int pr, const bf8_t& h, const bf8_t& m, const bf8_t& l) {
  return pr == 0 ? m : pr == 1 ? l : pr == 2 ? h : pr == 3 ? m : h;
}
__device__ __forceinline__ const bf8_t& pr_y(int pr, const bf8_t& h, const bf8_t& m, const bf8_t& l) {
  return pr == 0 ? m : pr == 1 ? h : pr == 2 ? l : pr == 3 ? h : pr == 4 ? m : h;
}
// the three BF16 parts of 8 values v[0..7] as MFMA operands
__device__ __forceinline__ void split3x8(const float (&v)[8], bf8_t& h, bf8_t& m, bf8_t& l, const SplitC& c) {
  bf2_t hh[4], mm[4], ll[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) split3x2(f2_t{v[2 * p], v[2 * p + 1]}, hh[p], mm[p], ll[p], c);
  h = bf8_t{hh[0][0], hh[0][1], hh[1][0], hh[1][1], hh[2][0], hh[2][1], hh[3][0], hh[3][1]};
  m = bf8_t{mm[0][0], mm[0][1], mm[1][0], mm[1][1], mm[2][0], mm[2][1], mm[3][0], mm[3][1]};
  l = bf8_t{ll[0][0], ll[0][1], ll[1][0], ll[1][1], ll[2][0], ll[2][1], ll[3][0], ll[3][1]};
}

// Element (row, k) of one BF16 plane of a pre-split operand (the split-product GEMM on
// pre-split operands): blocks of 16 rows x 32 k (1 KB), block (row / 16, k / 32) at
// ((k / 32) nrb + row / 16) 512, nrb = row blocks; inside a block, lane l = 16 (k % 32 / 8) +
// row % 16 holds k % 8 = 0..7 at 8 l .. 8 l + 7, the operand order of
// v_mfma_f32_16x16x32_bf16, so that a block is copied and read 16 bytes a lane, in order.
__device__ __forceinline__ int64_t ps_off(int64_t row, int64_t k, int64_t nrb) {
  return (((k >> 5) * nrb + (row >> 4)) << 9) + ((((k & 31) >> 3) * 16 + (row & 15)) << 3) + (k & 7);
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

// Grouped tile orders: consecutive tile ids walk TILE_GROUP row panels column by column,
// so the tiles an XCD runs at once (a contiguous id range, see xcd_tile) share a few row
// and column panels in its L2 instead of one row panel and many column panels.
// Measured on the MNIST-shaped step: the BF16 Gram takes G = 4 (318 ms; 323 at 8, 336 at 16),
// the Khatri-Rao contractions G = 16 (their dominant launch 1 581 ms; 1 598 at 8, 1 584 at 32).
constexpr int64_t TILE_GROUP = 8;

// Full tiles_r x tiles_c grid.
template <int64_t G = TILE_GROUP>
__device__ __forceinline__ void grouped_full_tile(int64_t t, int64_t tiles_c, int64_t tiles_r, int64_t& tr,
                                                  int64_t& tc) {
  const int64_t g = t / (G * tiles_c), u = t - g * G * tiles_c;
  const int64_t Gg = tiles_r - g * G < G ? tiles_r - g * G : G;
  tc = u / Gg;
  tr = g * G + u % Gg;
}

// Lower triangle (tc <= tr) of a tiles_r x tiles_r grid: group g (rows gG .. gG + Gg - 1)
// holds gG full columns of Gg tiles and then a lower triangle of Gg columns.
template <int64_t G = TILE_GROUP>
__device__ __forceinline__ void grouped_lower_tile(int64_t t, int64_t tiles_r, int64_t& tr, int64_t& tc) {
  // tiles before group g (all full): G^2 g (g - 1) / 2 + g G (G + 1) / 2
  auto before = [](int64_t g) { return G * G * g * (g - 1) / 2 + g * G * (G + 1) / 2; };
  int64_t g = (int64_t)(sqrt(2.0 * (double)t) / (double)G);
  while (g > 0 && before(g) > t) --g;
  while (before(g + 1) <= t && (g + 1) * G < tiles_r) ++g;
  int64_t u = t - before(g);
  const int64_t Gg = tiles_r - g * G < G ? tiles_r - g * G : G, r0 = g * G;
  if (u < r0 * Gg) {
    tc = u / Gg;
    tr = r0 + u % Gg;
    return;
  }
  u -= r0 * Gg;
  int64_t c = 0;
  while (u >= Gg - c) {
    u -= Gg - c;
    ++c;
  }
  tc = r0 + c;
  tr = r0 + c + u;
}

}  // namespace hs
