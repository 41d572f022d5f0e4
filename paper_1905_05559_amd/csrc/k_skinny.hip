// Dense operator applied to a thin block: Y = Q M for b <= 64 row vectors Q (FP32,
// b x P) and a dense symmetric FP32 matrix M (P x P), the products of the block
// Lanczos eigensolver on a formed H or OPG (paper, Sec. 5.3).  With b this small the
// product reads M once (4 P^2 bytes) for 2 b P^2 flops, so it is bound by HBM for
// b <~ 32: the tile is SR (= 16, 32 or 64) rows x 256 columns of M, streamed through LDS in
// chunks of 16 rows of M, double-buffered, one barrier per chunk.  The contraction over
// P is split into slices (one workgroup per column block and slice); partial products
// go to part[slice][b][P] and are summed in slice order by the caller.
//
// MFMA v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] (Q, rows = vectors)
// and B[l / 16][l % 16] (M, columns); D[4 (l / 16) + v][l % 16].  Each of the four
// wavefronts owns 64 columns of the tile and all SR rows.
#include <algorithm>

#include "api_internal.h"
#include "mfma.h"

namespace hs {

namespace {

constexpr int SC = 256;       // columns of M per tile
constexpr int SKC = 16;       // rows of M (contraction index) per chunk
constexpr int MSTR = SC + 16;  // LDS row stride of the M chunk: rows q, q + 1 fall in opposite bank halves

template <int SR>
struct SkinnyLds {
  static constexpr int QSTR = SR + 16;
  static constexpr int M = SKC * MSTR, Q = SKC * QSTR, STAGE = M + Q;
};

template <int SR>
__global__ __launch_bounds__(256, SR <= 32 ? 4 : 2) void k_skinny_f32(const float* __restrict__ Q, int64_t ldq, int64_t b,
                                                       int64_t P, const float* __restrict__ M, int64_t ldm,
                                                       float* __restrict__ part, int64_t kslice, int64_t ncb,
                                                       int64_t ntiles) {
  using L = SkinnyLds<SR>;
  constexpr int RB = SR / 16;                // 16-row blocks
  constexpr int QPT = SR * SKC / 256;        // Q values loaded per thread per chunk
  __shared__ __attribute__((aligned(16))) float sm[2 * L::STAGE];
  const int64_t t = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (t < 0) return;
  const int64_t sp = t / ncb, cb = t - sp * ncb;
  const int64_t c0 = cb * SC, r0 = (int64_t)blockIdx.y * SR;
  const int64_t k0 = sp * kslice, k1 = std::min<int64_t>(P, k0 + kslice);
  const int nch = (int)((k1 - k0 + SKC - 1) / SKC);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;

  // Buffer loads: an offset past the resource's extent reads 0, so every load is issued
  // unconditionally (no per-row branch and wait).  The M resource covers the chunk's
  // rows only (none past the slice); invalid columns and rows get offsets beyond it.
  const __amdgpu_buffer_rsrc_t rq =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Q), (short)0, (int)(b * ldq * 4), 0x00020000);
  // M: each lane loads 16 bytes (4 columns) of 4 rows of the chunk (rows 4 w .. 4 w + 3):
  // one 1 KB row segment per wavefront load instead of four.  Columns past P in a row
  // before the last read the next row's first entries and feed only output columns that
  // are never stored; past the resource's extent the load reads zeros.
  const int64_t col4 = c0 + 4 * lane;
  const uint32_t coff = col4 < P ? (uint32_t)(col4 * 4) : 0x80000000u;
  constexpr int RPW = SKC / 4;  // rows of a chunk per wavefront
  struct Regs {
    f4_t m[RPW];
    float q[QPT];
  };
  auto load = [&](int ch, Regs& g) {
    const int64_t kk = k0 + (int64_t)ch * SKC;
    const int64_t rows = k1 - kk < SKC ? (k1 - kk > 0 ? k1 - kk : 0) : SKC;
    const __amdgpu_buffer_rsrc_t rm = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(M + (rows > 0 ? kk : k0) * ldm), (short)0, (int)(rows * ldm * 4), 0x00020000);
#pragma unroll
    for (int r = 0; r < RPW; ++r)
      g.m[r] = __builtin_bit_cast(
          f4_t, __builtin_amdgcn_raw_buffer_load_b128(rm, coff + (uint32_t)((RPW * w + r) * ldm * 4), 0, 0));
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      const int e = tid + 256 * i;               // e = row * SKC + kq
      const int row = e / SKC, kq = e % SKC;
      const int64_t k = kk + kq, rr = r0 + row;
      const uint32_t off = (k < k1 && rr < b) ? (uint32_t)((rr * ldq + k) * 4) : 0xfffffff0u;
      g.q[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rq, off, 0, 0));
    }
  };
  auto store = [&](const Regs& g, int buf) {
    float* ms = sm + buf * L::STAGE;
    float* qs = ms + L::M;
#pragma unroll
    for (int r = 0; r < RPW; ++r) *reinterpret_cast<f4_t*>(&ms[(RPW * w + r) * MSTR + 4 * lane]) = g.m[r];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      const int e = tid + 256 * i;
      qs[(e % SKC) * L::QSTR + e / SKC] = g.q[i];
    }
  };

  f4_t acc[RB][4];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](int buf) {
    const float* ms = sm + buf * L::STAGE;
    const float* qs = ms + L::M;
#pragma unroll
    for (int ks = 0; ks < SKC / 4; ++ks) {
      const int kr = 4 * ks + lq;
      float a[RB], bv[4];
#pragma unroll
      for (int i = 0; i < RB; ++i) a[i] = qs[kr * L::QSTR + 16 * i + li];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = ms[kr * MSTR + 64 * w + 16 * j + li];
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bv[j], acc[i][j], 0, 0, 0);
    }
  };

  // Two chunks in flight: while chunk c is multiplied from LDS, chunk c + 1 waits in
  // registers and chunk c + 2 is being loaded.  The loop runs an even number of chunks
  // (an extra chunk past the slice reads zeros).
  Regs ga, gb;
  load(0, ga);
  load(1, gb);
  store(ga, 0);
  __syncthreads();
  // (the scheduling barriers keep each chunk's loads ahead of the multiply of the chunk
  // before it; without them the loads sink below the LDS stores and every store waits for all)
  for (int ch = 0; ch < nch; ch += 2) {
    load(ch + 2, ga);
    __builtin_amdgcn_sched_barrier(0);
    compute(0);
    store(gb, 1);
    __syncthreads();
    load(ch + 3, gb);
    __builtin_amdgcn_sched_barrier(0);
    compute(1);
    store(ga, 0);
    __syncthreads();
  }
  float* out = part + sp * b * P;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = c0 + 64 * w + 16 * j + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 16 * i + 4 * lq + v;
        if (row < b && col < P) out[row * P + col] = acc[i][j][v];
      }
    }
}

}  // namespace

// Slices of the contraction: the count whose tiles fill whole rounds of the device's
// resident workgroups best (4 per compute unit for b <= 32, 2 above), each slice a
// multiple of the chunk length and at least 1024 rows of M.
void skinny_slices(int64_t P, int64_t b, int64_t& ks, int64_t& kslice) {
  static const int64_t cus = [] {
    int dev = 0, n = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return (int64_t)std::max(n, 1);
  }();
  const int64_t slots = (b <= 32 ? 4 : 2) * cus;
  const int64_t ncb = (P + SC - 1) / SC, nrt = b <= 32 ? 1 : (b + 63) / 64;
  int64_t best = 1;
  double best_eff = -1.0;
  for (int64_t k = 1; k <= 16 && (k == 1 || P / k >= 1024); ++k) {
    const int64_t w = ncb * nrt * k, rounds = (w + slots - 1) / slots;
    const double eff = (double)w / (double)(rounds * slots);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = k;
    }
  }
  kslice = rup((P + best - 1) / best, SKC);
  ks = (P + kslice - 1) / kslice;
}

void skinny_apply_f32(Exec& ex, const float* Q, int64_t b, int64_t P, const float* M, float* part, int64_t ks,
                      int64_t kslice) {
  if (!launch_ok(ex)) return;
  // buffer extents: the block (b P floats) and one chunk of rows of M in 32-bit byte offsets
  if (b * P * 4 >= 0x7fffffffLL || 16 * P * 4 + P * 4 >= 0x7fffffffLL) {
    ex.ctx->fault_hit = true;
    return;
  }
  const int64_t ncb = (P + SC - 1) / SC, ntiles = ncb * ks;
  const int tok = prof_begin(ex, "dense_apply_skinny_f32", 2.0 * b * (double)P * P,
                             4.0 * (double)P * P + 4.0 * b * P * (1 + ks));
  if (b <= 16) {
    hipLaunchKernelGGL(k_skinny_f32<16>, dim3((unsigned)xcd_grid(ntiles), 1), dim3(256), 0, ex.stream, Q, P, b, P, M,
                       P, part, kslice, ncb, ntiles);
  } else if (b <= 32) {
    hipLaunchKernelGGL(k_skinny_f32<32>, dim3((unsigned)xcd_grid(ntiles), 1), dim3(256), 0, ex.stream, Q, P, b, P, M,
                       P, part, kslice, ncb, ntiles);
  } else {
    hipLaunchKernelGGL(k_skinny_f32<64>, dim3((unsigned)xcd_grid(ntiles), (unsigned)((b + 63) / 64)), dim3(256), 0,
                       ex.stream, Q, P, b, P, M, P, part, kslice, ncb, ntiles);
  }
  prof_end(ex, tok);
}

}  // namespace hs
