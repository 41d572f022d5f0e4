// BF16 variant of the Khatri-Rao Gram contraction for the OPG (RANK1 mode only):
// the per-example gradient tiles J[n, p] = delta^(l)_{n,i} abar^(l-1)_{n,j} are formed
// in FP32 while staging, rounded to BF16 (round to nearest even) into LDS and
// contracted with v_mfma_f32_16x16x32_bf16 into FP32 accumulators.
//
// Tile: 128 x 128 per workgroup, 4 wavefronts in 2 x 2, each 64 x 64 = 4 x 4 blocks;
// K chunk 32 = one MFMA step per block.  LDS rows hold 32 k values (+8 padding).
#include "mfma.h"

namespace hs {

namespace {

constexpr int BM = 128, BN = 128, KC = 32, KP = KC + 8;

__device__ __forceinline__ int64_t flat_index(int32_t perm, int64_t off, int32_t Tin, int32_t Tout,
                                              int64_t u, int64_t s) {
  const int64_t i = perm ? s : u, j = perm ? u : s;
  return j < Tin ? off + i * Tin + j : off + (int64_t)Tout * Tin + i;
}

__global__ __launch_bounds__(256) void krg_bf16_kernel(KrgArgs<float, float> a, int64_t tiles_c,
                                                       int64_t ntiles) {
  __shared__ __attribute__((aligned(16))) __bf16 As[BM * KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN * KP];

  const int64_t t = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (t < 0) return;
  int64_t tr, tc;
  if (a.symmetric) {
    int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    tr = r;
    tc = t - r * (r + 1) / 2;
  } else {
    tr = t / tiles_c;
    tc = t % tiles_c;
  }
  const int64_t r0 = tr * BM, c0 = tc * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  const int srow = tid & 127, sk0 = (tid >> 7) * 16;
  const int64_t gr = r0 + srow, gc = c0 + srow;
  const int64_t sur = gr / a.r.pad, ssr = gr % a.r.pad;
  const int64_t suc = gc / a.c.pad, ssc = gc % a.c.pad;
  const bool rvalid = sur < a.r.n_units && ssr < a.r.len;
  const bool cvalid = suc < a.c.n_units && ssc < a.c.len;
  float ra[16], rbv[16];

  auto load = [&](int64_t n0) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t n = n0 + sk0 + i;
      float va = 0.f, vb = 0.f;
      if (n < a.N) {
        if (rvalid) {
          va = a.r.src[n * a.r.ld + ssr];
          if (a.r.scale) va *= a.r.scale[n * a.r.ld_scale + sur];
        }
        if (cvalid) {
          vb = a.c.src[n * a.c.ld + ssc];
          if (a.c.scale) vb *= a.c.scale[n * a.c.ld_scale + suc];
        }
      }
      ra[i] = va;
      rbv[i] = vb;
    }
  };
  auto store = [&]() {
    bf8_t x0, x1, y0, y1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      x0[i] = (__bf16)ra[i];
      x1[i] = (__bf16)ra[8 + i];
      y0[i] = (__bf16)rbv[i];
      y1[i] = (__bf16)rbv[8 + i];
    }
    *reinterpret_cast<bf8_t*>(&As[srow * KP + sk0]) = x0;
    *reinterpret_cast<bf8_t*>(&As[srow * KP + sk0 + 8]) = x1;
    *reinterpret_cast<bf8_t*>(&Bs[srow * KP + sk0]) = y0;
    *reinterpret_cast<bf8_t*>(&Bs[srow * KP + sk0 + 8]) = y1;
  };

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int row = lane & 15, q = lane >> 4;
  const int64_t nk = (a.N + KC - 1) / KC;
  load(0);
  store();
  __syncthreads();
  for (int64_t kc = 0; kc < nk; ++kc) {
    if (kc + 1 < nk) load((kc + 1) * KC);
    bf8_t av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const bf8_t*>(&As[(wr * 64 + i * 16 + row) * KP + 8 * q]);
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = *reinterpret_cast<const bf8_t*>(&Bs[(wc * 64 + j * 16 + row) * KP + 8 * q]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = mma_bf16(av[i], bv[j], acc[i][j]);
    __syncthreads();
    if (kc + 1 < nk) {
      store();
      __syncthreads();
    }
  }

  int64_t fcol[4], ccomp[4];
  bool cok[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = c0 + wc * 64 + j * 16 + row;
    const int64_t uc = c / a.c.pad, sc = c % a.c.pad;
    ccomp[j] = c;
    cok[j] = uc < a.c.n_units && sc < a.c.len;
    fcol[j] = cok[j] ? flat_index(a.c.perm, a.c.off, a.c.Tin, a.c.Tout, uc, sc) : 0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = r0 + wr * 64 + i * 16 + 4 * q + v;
      const int64_t ur = r / a.r.pad, sr = r % a.r.pad;
      if (!(ur < a.r.n_units && sr < a.r.len)) continue;
      const int64_t fr = flat_index(a.r.perm, a.r.off, a.r.Tin, a.r.Tout, ur, sr);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!cok[j]) continue;
        if (a.symmetric && r < ccomp[j]) continue;
        const float val = (float)(a.scale * (double)acc[i][j][v]);
        a.out[fr * a.ldo + fcol[j]] = val;
        if (a.mirror && !(a.symmetric && r == ccomp[j])) a.out[fcol[j] * a.ldo + fr] = val;
      }
    }
}

}  // namespace

void krg_bf16(Exec& ex, const KrgArgs<float, float>& a) {
  const int64_t rows = (int64_t)a.r.n_units * a.r.pad, cols = (int64_t)a.c.n_units * a.c.pad;
  const int64_t tr = (rows + BM - 1) / BM, tc = (cols + BN - 1) / BN;
  const int64_t nt = a.symmetric ? tr * (tr + 1) / 2 : tr * tc;
  if (nt <= 0) return;
  if (!launch_ok(ex)) return;
  hipLaunchKernelGGL(krg_bf16_kernel, dim3((unsigned)xcd_grid(nt)), dim3(256), 0, ex.stream, a, tc, nt);
}

}  // namespace hs
