// BF16 OPG: OPG = J^T J / N with the per-example gradient matrix J formed once in
// BF16 and contracted as one symmetric Gram product on BF16 MFMA.
//
// 1) jt_bf16: Jt[p][n] = bf16_rne(delta^(l)_{n,i} * abar^(l-1)_{n,j}) for the flat
//    parameter p = (layer l, unit i, input j) (j = T_{l-1} is the bias, abar = 1);
//    columns n >= N are zero.  Jt is p-major so that the contraction index n is
//    contiguous for the MFMA operands.  (On a 288 GB part the BF16 J of the
//    MNIST-shaped workload, 9.5 GB, fits comfortably in the workspace.)
// 2) gram_bf16: C[p][q] = scale * sum_n Jt[p][n] Jt[q][n] for the lower triangle of
//    256 x 256 tiles, mirrored, FP32 accumulation (v_mfma_f32_16x16x32_bf16).
//    4 wavefronts (2 x 2), each 128 x 128 = 8 x 8 MFMA blocks; K staged through LDS
//    in chunks of 32 by direct HBM -> LDS copies, several chunks ahead, with the MFMA
//    operands of the next chunk read from LDS while the current chunk's MFMAs run.
#include <algorithm>
#include <string>

#include "mfma.h"

namespace hs {

namespace {

constexpr int JP = 64, JN = 64;   // jt_bf16 tile (params x examples)

__global__ __launch_bounds__(256) void jt_bf16_kernel(JtArgs a) {
  __shared__ __bf16 tile[JP][JN + 8];
  const int64_t tiles_n = a.ldk / JN;
  const int64_t p0 = (blockIdx.x / tiles_n) * JP, n0 = (blockIdx.x % tiles_n) * JN;
  const int tid = threadIdx.x;
  // phase 1: each thread forms 16 entries (one parameter, 16 examples)
  const int pp = tid & 63, nb = (tid >> 6) * 16;
  const int64_t p = p0 + pp;
  int lay = -1;
  int64_t i = 0, j = 0;
  if (p < a.P) {
    for (int k = 0; k < a.nlayers; ++k) {
      const int64_t ow = a.offW[k], ob = ow + (int64_t)a.Tout[k] * a.Tin[k];
      if (p >= ow && p < ob + a.Tout[k]) {
        lay = k;
        if (p < ob) {
          i = (p - ow) / a.Tin[k];
          j = (p - ow) % a.Tin[k];
        } else {
          i = p - ob;
          j = a.Tin[k];
        }
        break;
      }
    }
  }
  // all 16 examples' loads issued before any product (full unroll: 32 loads in flight)
  float dv[16], xv[16];
  if (lay >= 0) {
    const float* dl = a.delta[lay] + i;
    const float* xl = a.abar[lay] + j;
    const int64_t ldd = a.ld_delta[lay], ldx = a.ld_abar[lay];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int64_t n = min(n0 + nb + t, a.N - 1);  // clamped in-range read; zeroed below
      dv[t] = dl[n * ldd];
      xv[t] = xl[n * ldx];
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const bool ok = lay >= 0 && n0 + nb + t < a.N;
    tile[pp][nb + t] = (__bf16)(ok ? dv[t] * xv[t] : 0.f);
  }
  __syncthreads();
  // phase 2: write 64 rows x 128 bytes, 16 bytes per thread
  for (int e = tid; e < JP * (JN / 8); e += 256) {
    const int r = e / (JN / 8), seg = e % (JN / 8);
    const int64_t pr = p0 + r;
    if (pr < a.P)
      *reinterpret_cast<bf8_t*>(&a.Jt[pr * a.ldk + n0 + seg * 8]) =
          *reinterpret_cast<const bf8_t*>(&tile[r][seg * 8]);
  }
}

constexpr int GB = 256, GK = 64, GKP = GK + 8;

__global__ __launch_bounds__(256) void gram_bf16_kernel(const __bf16* __restrict__ Jt, int64_t P, int64_t ldk,
                                                        int64_t nk, float scale, float* __restrict__ C,
                                                        int64_t ldc, int64_t ntiles) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __bf16* As = reinterpret_cast<__bf16*>(smem);
  __bf16* Bs = As + GB * GKP;

  const int64_t t = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (t < 0) return;
  int64_t tr = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (tr * (tr + 1) / 2 > t) --tr;
  while ((tr + 1) * (tr + 2) / 2 <= t) ++tr;
  const int64_t tc = t - tr * (tr + 1) / 2;
  const int64_t r0 = tr * GB, c0 = tc * GB;
  const bool diag = (tr == tc);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // staging: 256 rows x 8 segments of 8 bf16 per side; thread -> 8 segments per side
  bf8_t ra[8], rb[8];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + i * 256;
      const int row = e >> 3, seg = e & 7;
      const int64_t gr = r0 + row, gc = c0 + row;
      bf8_t z = {};
      ra[i] = gr < P ? *reinterpret_cast<const bf8_t*>(&Jt[gr * ldk + k0 + seg * 8]) : z;
      if (!diag) rb[i] = gc < P ? *reinterpret_cast<const bf8_t*>(&Jt[gc * ldk + k0 + seg * 8]) : z;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + i * 256;
      const int row = e >> 3, seg = e & 7;
      *reinterpret_cast<bf8_t*>(&As[row * GKP + seg * 8]) = ra[i];
      if (!diag) *reinterpret_cast<bf8_t*>(&Bs[row * GKP + seg * 8]) = rb[i];
    }
  };
  const __bf16* Bsrc = diag ? As : Bs;

  f4_t acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int row = lane & 15, q = lane >> 4;
  load(0);
  store();
  __syncthreads();
  for (int64_t kc = 0; kc < nk; ++kc) {
    if (kc + 1 < nk) load((kc + 1) * GK);
#pragma unroll
    for (int ks = 0; ks < GK / 32; ++ks) {
      bf8_t av[8], bv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        av[i] = *reinterpret_cast<const bf8_t*>(&As[(wr * 128 + i * 16 + row) * GKP + ks * 32 + 8 * q]);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        bv[j] = *reinterpret_cast<const bf8_t*>(&Bsrc[(wc * 128 + j * 16 + row) * GKP + ks * 32 + 8 * q]);
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = mma_bf16(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
    if (kc + 1 < nk) {
      store();
      __syncthreads();
    }
  }

#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = r0 + wr * 128 + i * 16 + 4 * q + v;
      if (r >= P) continue;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t c = c0 + wc * 128 + j * 16 + row;
        if (c >= P || (diag && r < c)) continue;
        const float val = scale * acc[i][j][v];
        C[r * ldc + c] = val;
        if (r != c) C[c * ldc + r] = val;
      }
    }
}

// ---------------------------------------------------------------------------
// Gram product with direct HBM -> LDS staging (buffer_load_dwordx4 ... lds).
//
// Same 256 x 256 tiles and wavefront layout as above; K chunks of GD examples in GS LDS
// stages, one barrier per chunk, the copies of a chunk issued GS - 1 chunks ahead.  Tiles
// are visited in the grouped lower-triangle order, so the tiles an XCD runs at once share
// eight row panels and a few column panels in its L2.  A stage holds the two 256-row
// panels, GD / 8 segments of 8 BF16 (16 bytes) per row.  Each lane copies one segment,
// stored at position row * (GD / 8) + (seg ^ swz(row)): the swizzle puts the lanes of an
// MFMA operand read (16 consecutive rows, one segment) on distinct bank groups whether
// the LDS serves 8 lanes per 128-byte cycle or 16 lanes per 256-byte cycle.  Rows past P
// are clamped to row P - 1 (their outputs are discarded); Jt columns n >= N are zero.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0f70);
}

// Segment swizzle of a row (tile-local row index, bits 0..3 used): with GD = 32 (4
// segments) and GD = 64 (8 segments) the 8 lanes of a 128-byte LDS cycle and the 16 lanes
// of a 256-byte cycle both hit distinct bank groups.
template <int GD>
__device__ __forceinline__ int seg_swz(int row) {
  return GD == 32 ? (((row >> 1) ^ ((row >> 3) & 1)) & 3) : ((row ^ ((row >> 3) & 1)) & 7);
}

extern __shared__ __attribute__((aligned(16))) unsigned char gram_smem[];

// Stores of a 256 x 256 tile's accumulators (wavefront (wr, wc), lane (row16, q)): entry
// (r, c) = (r0 + 128 wr + 16 i + 4 q + v, c0 + 128 wc + 16 j + row16) goes to C[r][c] and,
// mirrored, to C[c][r].  A lane's four v of one block are four consecutive r, so on interior
// off-diagonal tiles the mirror is written as one 16-byte store (two 8-byte stores when the
// rows are only 8-byte aligned) instead of four scattered floats; diagonal and edge tiles keep
// the per-entry form.
__device__ __forceinline__ void gram_store(const f4_t (&acc)[8][8], int64_t P, int64_t r0, int64_t c0, bool diag,
                                           int wr, int wc, int row16, int q, float scale, float* __restrict__ C,
                                           int64_t ldc) {
  if (!diag && r0 + GB <= P && c0 + GB <= P) {
    const uintptr_t base = reinterpret_cast<uintptr_t>(C);
    const bool a16 = (ldc & 3) == 0 && (base & 15) == 0, a8 = (ldc & 1) == 0 && (base & 7) == 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t rb = r0 + wr * 128 + i * 16 + 4 * q, c = c0 + wc * 128 + j * 16 + row16;
        const f4_t val = scale * acc[i][j];
#pragma unroll
        for (int v = 0; v < 4; ++v) C[(rb + v) * ldc + c] = val[v];
        float* m = C + c * ldc + rb;
        if (a16) {
          *reinterpret_cast<f4_t*>(m) = val;
        } else if (a8) {
          reinterpret_cast<f2_t*>(m)[0] = f2_t{val[0], val[1]};
          reinterpret_cast<f2_t*>(m)[1] = f2_t{val[2], val[3]};
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) m[v] = val[v];
        }
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = r0 + wr * 128 + i * 16 + 4 * q + v;
      if (r >= P) continue;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t c = c0 + wc * 128 + j * 16 + row16;
        if (c >= P || (diag && r < c)) continue;
        const float val = scale * acc[i][j][v];
        C[r * ldc + c] = val;
        if (r != c) C[c * ldc + r] = val;
      }
    }
}

// DIST: the next chunk's copies are spread over the current chunk's MFMA rows (one copy
// after each row of 8 MFMAs) instead of issued together after the barrier: a full copy
// queue then holds up a few MFMAs instead of the whole chunk's.
template <int GD, int GS, bool DIST = false>
__device__ __forceinline__ void gram_dma_tile(const __bf16* __restrict__ Jt, int64_t P, int64_t ldk, float scale,
                                              float* __restrict__ C, int64_t ldc, int64_t ntiles) {
  constexpr int NSEG = GD / 8;            // 16-byte segments per row and chunk
  constexpr int RPC = 64 / NSEG;          // rows per copy (64 lanes)
  constexpr int CPW = GB / RPC / 4;       // copies per panel and wavefront
  constexpr int GSTAGE = 2 * GB * GD;     // BF16 elements per stage
  __bf16* S = reinterpret_cast<__bf16*>(gram_smem);

  const int64_t t = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (t < 0) return;
  int64_t tr, tc;
  grouped_lower_tile<4>(t, (P + GB - 1) / GB, tr, tc);
  const int64_t r0 = tr * GB, c0 = tc * GB;
  const bool diag = (tr == tc);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int row16 = lane & 15, q = lane >> 4;

  // copy m of this wavefront moves rows RPC * (CPW * wave + m) .. + RPC - 1 of a panel
  int voffA[CPW], voffB[CPW];
#pragma unroll
  for (int m = 0; m < CPW; ++m) {
    const int row = RPC * (CPW * wave + m) + lane / NSEG;
    const int seg = (lane % NSEG) ^ seg_swz<GD>(row);
    const int64_t ra = std::min<int64_t>(r0 + row, P - 1) - r0, rb = std::min<int64_t>(c0 + row, P - 1) - c0;
    voffA[m] = (int)((ra * ldk + seg * 8) * 2);
    voffB[m] = (int)((rb * ldk + seg * 8) * 2);
  }
  const int64_t nk = ldk / GD;
  auto issue = [&](int st, int64_t k0) {
    __bf16* D = S + st * GSTAGE;
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<__bf16*>(Jt + r0 * ldk + k0), (short)0, 0x7ffffff0, 0x00020000);
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<__bf16*>(Jt + c0 * ldk + k0), (short)0, 0x7ffffff0, 0x00020000);
#pragma unroll
    for (int m = 0; m < CPW; ++m)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          ra, (__attribute__((address_space(3))) void*)(D + (CPW * wave + m) * RPC * GD), 16, voffA[m], 0, 0, 0);
#pragma unroll
    for (int m = 0; m < CPW; ++m)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rb, (__attribute__((address_space(3))) void*)(D + GB * GD + (CPW * wave + m) * RPC * GD), 16, voffB[m], 0, 0,
          0);
  };
  // DIST: copy s of a chunk (s = 0 .. 2 CPW - 1): A copy s / 2 for even s, B copy s / 2 for
  // odd s.  Issued without a branch (a branch among the MFMAs makes the compiler move the
  // accumulators): past the last chunk the buffer is empty and the copy writes zeros into
  // the stage that is no longer read.
  static_assert(!DIST || 2 * CPW == (GD / 32) * 8, "one copy per MFMA row");
  auto issue_one = [&](int st, int64_t k0, int s, bool live) {
    __bf16* D = S + st * GSTAGE;
    const int m = s >> 1;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<__bf16*>(Jt + ((s & 1) ? c0 : r0) * ldk + (live ? k0 : 0)), (short)0, live ? 0x7ffffff0 : 0,
        0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        r, (__attribute__((address_space(3))) void*)(D + ((s & 1) ? GB * GD : 0) + (CPW * wave + m) * RPC * GD), 16,
        (s & 1) ? voffB[m] : voffA[m], 0, 0, 0);
  };

  f4_t acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int sw = seg_swz<GD>(row16);  // operand rows r satisfy r % 16 == row16
#pragma unroll
  for (int c = 0; c < GS - 1; ++c)
    if (c < nk) issue(c, (int64_t)c * GD);
  for (int64_t kc = 0; kc < nk; ++kc) {
    // chunk kc's copies are the oldest in flight; up to GS - 2 later chunks may stay pending
    const int64_t later = std::min<int64_t>(GS - 2, nk - 1 - kc);
    if (later >= 2) wait_vmcnt<4 * CPW>(); else if (later == 1) wait_vmcnt<2 * CPW>(); else wait_vmcnt<0>();
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    const bool more = kc + GS - 1 < nk;
    const int nst = (int)((kc + GS - 1) % GS);
    const int64_t nk0 = (kc + GS - 1) * GD;
    if (!DIST && more) issue(nst, nk0);
    const __bf16* As = S + (kc % GS) * GSTAGE;
    const __bf16* Bs = diag ? As : As + GB * GD;
#pragma unroll
    for (int ks = 0; ks < GD / 32; ++ks) {
      const int off = ((4 * ks + q) ^ sw) * 8;  // segment of k = 32 ks + 8q .. + 7
      bf8_t av[8], bv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) av[i] = *reinterpret_cast<const bf8_t*>(&As[(wr * 128 + i * 16 + row16) * GD + off]);
#pragma unroll
      for (int j = 0; j < 8; ++j) bv[j] = *reinterpret_cast<const bf8_t*>(&Bs[(wc * 128 + j * 16 + row16) * GD + off]);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = mma_bf16(av[i], bv[j], acc[i][j]);
        if constexpr (DIST) {
          __builtin_amdgcn_sched_barrier(0);
          issue_one(nst, nk0, ks * 8 + i, more);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  }

  gram_store(acc, P, r0, c0, diag, wr, wc, row16, q, scale, C, ldc);
}

// Software-pipelined form: chunks of 32 examples in GS >= 3 stages.  The barrier at the top
// of chunk kc also covers chunk kc + 1 (its copies are waited for one chunk early), so each
// wavefront reads its MFMA operands of chunk kc + 1 from LDS while the MFMAs of chunk kc run
// on the operands read during chunk kc - 1: no LDS latency between the barrier and the first
// MFMA.  The copies of chunk kc + GS - 1 are spread over the MFMA rows of chunk kc; they refill
// the stage of chunk kc - 1, whose operand reads (issued during chunk kc - 2) completed before
// the barrier of chunk kc - 1.  Same products in the same order as gram_dma_tile.
template <int GS>
__device__ __forceinline__ void gram_pipe_tile(const __bf16* __restrict__ Jt, int64_t P, int64_t ldk, float scale,
                                               float* __restrict__ C, int64_t ldc, int64_t ntiles) {
  static_assert(GS >= 3, "the pipelined form needs three stages or more");
  constexpr int GD = 32, NSEG = 4, RPC = 16, CPW = GB / RPC / 4;  // 4 copies per panel and wavefront
  constexpr int GSTAGE = 2 * GB * GD;
  __bf16* S = reinterpret_cast<__bf16*>(gram_smem);

  const int64_t t = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (t < 0) return;
  int64_t tr, tc;
  grouped_lower_tile<4>(t, (P + GB - 1) / GB, tr, tc);
  const int64_t r0 = tr * GB, c0 = tc * GB;
  const bool diag = (tr == tc);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int row16 = lane & 15, q = lane >> 4;

  int voffA[CPW], voffB[CPW];
#pragma unroll
  for (int m = 0; m < CPW; ++m) {
    const int row = RPC * (CPW * wave + m) + lane / NSEG;
    const int seg = (lane % NSEG) ^ seg_swz<GD>(row);
    const int64_t ra = std::min<int64_t>(r0 + row, P - 1) - r0, rb = std::min<int64_t>(c0 + row, P - 1) - c0;
    voffA[m] = (int)((ra * ldk + seg * 8) * 2);
    voffB[m] = (int)((rb * ldk + seg * 8) * 2);
  }
  const int64_t nk = ldk / GD;
  // copy s (0 .. 2 CPW - 1) of chunk k0 / GD into stage st: A copy s / 2 for even s, B copy
  // s / 2 for odd s; past the last chunk the buffer is empty and the copy writes zeros into a
  // stage that is not read again
  auto issue_one = [&](int st, int64_t k0, int s, bool live) {
    __bf16* D = S + st * GSTAGE;
    const int m = s >> 1;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<__bf16*>(Jt + ((s & 1) ? c0 : r0) * ldk + (live ? k0 : 0)), (short)0, live ? 0x7ffffff0 : 0,
        0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        r, (__attribute__((address_space(3))) void*)(D + ((s & 1) ? GB * GD : 0) + (CPW * wave + m) * RPC * GD), 16,
        (s & 1) ? voffB[m] : voffA[m], 0, 0, 0);
  };
  const int sw = seg_swz<GD>(row16);
  const int off = (q ^ sw) * 8;
  auto read_ops = [&](int st, bf8_t (&av)[8], bf8_t (&bv)[8]) {
    const __bf16* As = S + st * GSTAGE;
    const __bf16* Bs = diag ? As : As + GB * GD;
#pragma unroll
    for (int i = 0; i < 8; ++i) av[i] = *reinterpret_cast<const bf8_t*>(&As[(wr * 128 + i * 16 + row16) * GD + off]);
#pragma unroll
    for (int j = 0; j < 8; ++j) bv[j] = *reinterpret_cast<const bf8_t*>(&Bs[(wc * 128 + j * 16 + row16) * GD + off]);
  };

  f4_t acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int c = 0; c < GS - 1; ++c)
#pragma unroll
    for (int s = 0; s < 2 * CPW; ++s) issue_one(c, (int64_t)c * GD, s, c < nk);
  // chunk 0 landed (GS - 2 later chunks may stay in flight)
  wait_vmcnt<(GS - 2) * 2 * CPW>();
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  // two operand sets, alternated by unrolling two chunks per iteration (no register moves);
  // st = stage of chunk kc
  bf8_t a0[8], b0[8], a1[8], b1[8];
  read_ops(0, a0, b0);
  auto step = [&](int64_t kc, int st, bf8_t (&ac)[8], bf8_t (&bc)[8], bf8_t (&an)[8], bf8_t (&bn)[8]) {
    // chunk kc + 1 landed: of the copies issued so far (through chunk kc + GS - 2, every one
    // issued, live or not) those of chunks kc + 2 .. kc + GS - 2 may stay in flight
    wait_vmcnt<(GS - 3) * 2 * CPW>();
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    read_ops(st + 1 == GS ? 0 : st + 1, an, bn);
    const bool more = kc + GS - 1 < nk;
    const int nst = st == 0 ? GS - 1 : st - 1;  // stage of chunk kc + GS - 1 (= that of kc - 1)
    const int64_t nk0 = (kc + GS - 1) * GD;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = mma_bf16(ac[i], bc[j], acc[i][j]);
      __builtin_amdgcn_sched_barrier(0);
      issue_one(nst, nk0, i, more);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  int st = 0;
  int64_t kc = 0;
  for (; kc + 1 < nk; kc += 2) {
    step(kc, st, a0, b0, a1, b1);
    st = st + 1 == GS ? 0 : st + 1;
    step(kc + 1, st, a1, b1, a0, b0);
    st = st + 1 == GS ? 0 : st + 1;
  }
  if (kc < nk) step(kc, st, a0, b0, a1, b1);
  gram_store(acc, P, r0, c0, diag, wr, wc, row16, q, scale, C, ldc);
}

template <int GS>
__global__ __launch_bounds__(256) void gram_bf16_pipe_kernel(const __bf16* __restrict__ Jt, int64_t P, int64_t ldk,
                                                             float scale, float* __restrict__ C, int64_t ldc,
                                                             int64_t ntiles) {
  gram_pipe_tile<GS>(Jt, P, ldk, scale, C, ldc, ntiles);
}

template <int GS>
void launch_gram_pipe(Exec& ex, const __bf16* Jt, int64_t P, int64_t ldk, float scale, float* C, int64_t ldc,
                      int64_t nt) {
  constexpr int shm = GS * 2 * GB * 32 * (int)sizeof(__bf16);
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)gram_bf16_pipe_kernel<GS>, hipFuncAttributeMaxDynamicSharedMemorySize, shm);
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((gram_bf16_pipe_kernel<GS>), dim3((unsigned)xcd_grid(nt)), dim3(256), shm, ex.stream, Jt, P, ldk,
                     scale, C, ldc, nt);
}

template <int GD, int GS, bool DIST>
__global__ __launch_bounds__(256) void gram_bf16_dma_kernel(const __bf16* __restrict__ Jt, int64_t P, int64_t ldk,
                                                            float scale, float* __restrict__ C, int64_t ldc,
                                                            int64_t ntiles) {
  gram_dma_tile<GD, GS, DIST>(Jt, P, ldk, scale, C, ldc, ntiles);
}

template <int GD, int GS, bool DIST = false>
void launch_gram_dma(Exec& ex, const __bf16* Jt, int64_t P, int64_t ldk, float scale, float* C, int64_t ldc,
                     int64_t nt) {
  constexpr int shm = GS * 2 * GB * GD * (int)sizeof(__bf16);
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)gram_bf16_dma_kernel<GD, GS, DIST>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, shm);
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((gram_bf16_dma_kernel<GD, GS, DIST>), dim3((unsigned)xcd_grid(nt)), dim3(256), shm, ex.stream,
                     Jt, P, ldk, scale, C, ldc, nt);
}

}  // namespace

void jt_bf16(Exec& ex, const JtArgs& a) {
  const int64_t tiles = ((a.P + JP - 1) / JP) * (a.ldk / JN);
  if (tiles <= 0) return;
  if (!launch_ok(ex)) return;
  const int tok = prof_begin(ex, "jt_bf16", 2.0 * 0.5 * a.P * a.N, (double)a.P * a.ldk * 2.0);
  hipLaunchKernelGGL(jt_bf16_kernel, dim3((unsigned)tiles), dim3(256), 0, ex.stream, a);
  prof_end(ex, tok);
}

int64_t jt_ld(int64_t N) { return (N + GK - 1) / GK * GK; }

void gram_bf16_variant(Exec& ex, const __bf16* Jt, int64_t P, int64_t ldk, int64_t N, float scale, float* C,
                       int64_t ldc, int variant) {
  const int64_t tr = (P + GB - 1) / GB;
  const int64_t nt = tr * (tr + 1) / 2;
  if (nt <= 0) return;
  if (!launch_ok(ex)) return;
  const double entries = (double)P * (P + 1) / 2;
  // LDS-staged form needs every copy offset below 2^31 bytes (255 rows of ldk BF16)
  const bool dma = variant != 1 && (int64_t)GB * ldk * 2 < 0x7fff0000;
  // configuration of the LDS-staged form: 0 = software-pipelined chunks of 32 in 4 stages
  // (measured 321 ms on the MNIST-shaped OPG), 1 = (32 examples, 4 stages), 2 = (64, 2) with
  // the copies spread over the MFMA rows (338 ms); all bitwise equal
  auto go = [&](int cfg, int64_t ntl) {
    if (cfg == 1) launch_gram_dma<32, 4>(ex, Jt, P, ldk, scale, C, ldc, ntl);
    else if (cfg == 2) launch_gram_dma<64, 2, true>(ex, Jt, P, ldk, scale, C, ldc, ntl);
    else launch_gram_pipe<4>(ex, Jt, P, ldk, scale, C, ldc, ntl);
  };
  int cfg = variant == 2 ? 1 : (variant == 3 ? 2 : 0);
  if (dma && variant == 0 && ex.ctx->autotune) {
    // probe on the first two device rounds of tiles (one workgroup per compute unit)
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t ntp = std::min<int64_t>(nt, 2 * (int64_t)std::max(cus, 1));
    auto lg = [](int64_t v) { int b = 0; while (v > 1) { v >>= 1; ++b; } return b; };
    const std::string key = "gram_bf16 P2^" + std::to_string(lg(P)) + " N2^" + std::to_string(lg(ldk));
    static const char* const cfgs[3] = {"pipe32x4", "chunk32x4", "chunk64x2"};
    cfg = autotune_pick(ex, key, 3, cfgs, [&](int i) { go(i, ntp); });
  }
  const int tok = prof_begin(ex, "gram_bf16_sym", 2.0 * N * entries, (double)P * ldk * 2.0 + (double)P * P * 4.0);
  if (dma) {
    go(cfg, nt);
  } else {
    const size_t shm = 2 * GB * GKP * sizeof(__bf16);
    static const bool attr = [shm] {
      (void)hipFuncSetAttribute((const void*)gram_bf16_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      return true;
    }();
    (void)attr;
    hipLaunchKernelGGL(gram_bf16_kernel, dim3((unsigned)xcd_grid(nt)), dim3(256), shm, ex.stream, Jt, P, ldk,
                       ldk / GK, scale, C, ldc, nt);
  }
  prof_end(ex, tok);
}

void gram_bf16(Exec& ex, const __bf16* Jt, int64_t P, int64_t ldk, int64_t N, float scale, float* C,
               int64_t ldc) {
  gram_bf16_variant(ex, Jt, P, ldk, N, scale, C, ldc, 0);
}

}  // namespace hs
