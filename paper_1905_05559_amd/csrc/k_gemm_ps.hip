// FP32 GEMM on pre-split operands: C = alpha A B^T + beta C, where A (M x K) and B (N x K)
// are each given as three BF16 planes h, m, l with x = h + m + l (the compensated split of
// the FP32 values, round-to-nearest-even of the running remainder; split3x2 in mfma.h), k
// contiguous, K padded with zeros to a multiple of 32.  Each product is accumulated in
// FP32 from the six BF16 products h h, h m, m h, h l, l h, m m (smallest first) by
// v_mfma_f32_16x16x32_bf16, in the same order as the split-product GEMM that splits its
// operands in the tile, so both give the same bits; here no split work is left in the
// tile, which only streams parts and issues MFMAs.
//
// Used where one operand is shared by many products: the Hessian-vector sweep splits the
// direction block V once per call and the example chunk abar once per chunk, instead of
// once per tile (Sec. 5.1 / Appendix A.1 products R{Z} = abar Vbar^T and the accumulation
// R{delta}^T abar).
#include <algorithm>

#include "api_internal.h"
#include "mfma.h"

namespace hs {

namespace {

constexpr int TPB = 256;
inline unsigned grid_for(int64_t n) {
  int64_t g = (n + TPB - 1) / TPB;
  if (g > (1 << 20)) g = 1 << 20;
  return (unsigned)(g < 1 ? 1 : g);
}
#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ---- split passes ----------------------------------------------------------

// planes of dst (rows x kpad in the ps_off layout with nrb row blocks, plane stride pl): the
// split of src[r * lds + k] for k < K, zero for K <= k < kpad; one thread per pair of k.
__global__ void k_split_rows(const float* __restrict__ src, int64_t rows, int64_t K, int64_t lds, int64_t kpad,
                             uint32_t* __restrict__ dst, int64_t nrb, int64_t pl) {
  const SplitC sc = split_consts();
  const int64_t hp = kpad / 2;
  GRID_STRIDE(e, rows * hp) {
    const int64_t r = e / hp, k = 2 * (e - r * hp);
    const float x0 = k < K ? src[r * lds + k] : 0.f;
    const float x1 = k + 1 < K ? src[r * lds + k + 1] : 0.f;
    bf2_t h, m, l;
    split3x2(f2_t{x0, x1}, h, m, l, sc);
    const int64_t o = ps_off(r, k, nrb) / 2;
    dst[o] = __builtin_bit_cast(uint32_t, h);
    dst[o + pl / 2] = __builtin_bit_cast(uint32_t, m);
    dst[o + pl] = __builtin_bit_cast(uint32_t, l);
  }
}

// planes of dst (cols x rpad in the ps_off layout, plane stride pl): the split of the
// transpose, dst[c][r] = split(src[r * lds + c]) for r < R, zero for R <= r < rpad; 64 x 64
// tiles through LDS (reads coalesced along c, writes along r).
__global__ __launch_bounds__(256) void k_split_transpose(const float* __restrict__ src, int64_t R, int64_t Cc,
                                                         int64_t lds, int64_t rpad, uint32_t* __restrict__ dst,
                                                         int64_t nrb, int64_t pl) {
  __shared__ float tile[64][65];
  const int64_t tr = (rpad + 63) / 64;
  const int64_t r0 = (int64_t)(blockIdx.x % tr) * 64, c0 = (int64_t)(blockIdx.x / tr) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int y = ty; y < 64; y += 4) {
    const int64_t r = r0 + y, c = c0 + tx;
    tile[y][tx] = (r < R && c < Cc) ? src[r * lds + c] : 0.f;
  }
  __syncthreads();
  const SplitC sc = split_consts();
  const int p = threadIdx.x & 31;  // pair of rows 2p, 2p + 1 of the tile
  for (int cc = threadIdx.x >> 5; cc < 64; cc += 8) {
    const int64_t c = c0 + cc, r = r0 + 2 * p;
    if (c >= Cc || r >= rpad) continue;
    bf2_t h, m, l;
    split3x2(f2_t{tile[2 * p][cc], tile[2 * p + 1][cc]}, h, m, l, sc);
    const int64_t o = ps_off(c, r, nrb) / 2;
    dst[o] = __builtin_bit_cast(uint32_t, h);
    dst[o + pl / 2] = __builtin_bit_cast(uint32_t, m);
    dst[o + pl] = __builtin_bit_cast(uint32_t, l);
  }
}

}  // namespace

// ---- the GEMM tile -----------------------------------------------------------

//
// Tile BM x 128 (BM = 128 or 256) with BM / 32 wavefronts of 64 x 64 (4 x 4 blocks of
// 16 x 16); chunks of 32 k in two LDS stages, copied by buffer_load_dwordx4 ... lds.  At
// BM = 256 a stage is 72 KB: one workgroup of 8 wavefronts per CU, two per SIMD.

constexpr int PN = 128;           // tile columns (B rows)
constexpr int PKC = 32;           // k per chunk
constexpr int PSEG = PKC / 8;     // 16-byte segments per row, part and chunk
constexpr int PSTAGES = 2;
template <int BM>
struct PsTile {
  static constexpr int W = BM / 32;                       // wavefronts
  static constexpr int A_PART = BM * PKC * 2;             // bytes of one part of A per chunk
  static constexpr int B_PART = PN * PKC * 2;
  static constexpr int STAGE = 3 * (A_PART + B_PART);
  static constexpr int LDS = PSTAGES * STAGE;
  static constexpr int GA = BM / 16 / W, GB = PN / 16 / W;  // 16-row copy groups per wavefront
};


extern __shared__ __attribute__((aligned(16))) unsigned char ps_smem[];

struct PsArgs {
  const __bf16* A;  // part x of A(m, k) at A[x * pa + ps_off(m, k, nrba)]
  const __bf16* B;  // part x of B(n, k) at B[x * pb + ps_off(n, k, nrbb)]
  int64_t nrba, nrbb, pa, pb;
  int64_t M, N, K;  // K a multiple of 32 (parts zero past the true contraction length)
  float* C;
  int64_t scm, scn;
  float alpha, beta;
};

template <int BM>
__device__ __forceinline__ void gemm_ps_tile(const PsArgs& g, int64_t tiles_n, int64_t ntiles) {
  using TL = PsTile<BM>;
  const int64_t t = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (t < 0) return;
  const int64_t m0 = (t / tiles_n) * BM, n0 = (t % tiles_n) * PN;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int row16 = lane & 15, q = lane >> 4;

  // copies: one 1 KB block (16 rows x 32 k of one part, in MFMA operand order) per
  // instruction, 16 bytes a lane; wavefront w moves A row blocks GA w .. GA w + GA - 1 and
  // B row blocks GB w .. of every part.  Blocks past M (N) read the last block (outputs
  // discarded).
  int64_t rbA[TL::GA], rbB[TL::GB];
#pragma unroll
  for (int ga = 0; ga < TL::GA; ++ga) rbA[ga] = std::min<int64_t>(m0 / 16 + TL::GA * wave + ga, g.nrba - 1);
#pragma unroll
  for (int gb = 0; gb < TL::GB; ++gb) rbB[gb] = std::min<int64_t>(n0 / 16 + TL::GB * wave + gb, g.nrbb - 1);
  auto issue = [&](int st, int64_t kc) {
    unsigned char* D = ps_smem + st * TL::STAGE;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<__bf16*>(g.A + x * g.pa + kc * g.nrba * 512), (short)0, 0x7ffffff0, 0x00020000);
      const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<__bf16*>(g.B + x * g.pb + kc * g.nrbb * 512), (short)0, 0x7ffffff0, 0x00020000);
#pragma unroll
      for (int ga = 0; ga < TL::GA; ++ga)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            ra, (__attribute__((address_space(3))) void*)(D + x * TL::A_PART + (TL::GA * wave + ga) * 1024), 16,
            (int)(rbA[ga] * 1024 + 16 * lane), 0, 0, 0);
#pragma unroll
      for (int gb = 0; gb < TL::GB; ++gb)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rb,
            (__attribute__((address_space(3))) void*)(D + 3 * TL::A_PART + x * TL::B_PART + (TL::GB * wave + gb) * 1024),
            16, (int)(rbB[gb] * 1024 + 16 * lane), 0, 0, 0);
    }
  };

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  const int64_t nk = g.K / PKC;
  issue(0, 0);
  for (int64_t kc = 0; kc < nk; ++kc) {
    // this chunk's copies have landed and every wavefront is done reading the stage that
    // is refilled next
    asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (kc + 1 < nk) issue((int)((kc + 1) % PSTAGES), kc + 1);
    const unsigned char* S = ps_smem + (kc % PSTAGES) * TL::STAGE;
    const unsigned char* SB = S + 3 * TL::A_PART;
    const int lo = 16 * lane;  // this lane's 16 bytes of a block
    bf8_t bh[4], bm[4], bl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int blk = wc * 4 + j;
      bh[j] = *reinterpret_cast<const bf8_t*>(SB + 0 * TL::B_PART + blk * 1024 + lo);
      bm[j] = *reinterpret_cast<const bf8_t*>(SB + 1 * TL::B_PART + blk * 1024 + lo);
      bl[j] = *reinterpret_cast<const bf8_t*>(SB + 2 * TL::B_PART + blk * 1024 + lo);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int blk = wr * 4 + i;
      const bf8_t ah = *reinterpret_cast<const bf8_t*>(S + 0 * TL::A_PART + blk * 1024 + lo);
      const bf8_t am = *reinterpret_cast<const bf8_t*>(S + 1 * TL::A_PART + blk * 1024 + lo);
      const bf8_t al = *reinterpret_cast<const bf8_t*>(S + 2 * TL::A_PART + blk * 1024 + lo);
#pragma unroll
      for (int pr = 0; pr < 6; ++pr)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mma_bf16(pr_x(pr, ah, am, al), pr_y(pr, bh[j], bm[j], bl[j]), acc[i][j]);
    }
  }
  // output: row 4 q + v of block i, column row16 of block j
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wr * 64 + i * 16 + 4 * q + v;
        const int64_t n = n0 + wc * 64 + j * 16 + row16;
        if (m < g.M && n < g.N) {
          float* c = g.C + m * g.scm + n * g.scn;
          const float val = g.alpha * acc[i][j][v];
          *c = (g.beta != 0.f) ? val + g.beta * (*c) : val;
        }
      }
}

// the kernel body is a device template, so that the host stubs of the instances are emitted
template <int BM>
__global__ __launch_bounds__(BM * 2, 1) void gemm_ps_kernel(PsArgs g, int64_t tiles_n, int64_t ntiles) {
  gemm_ps_tile<BM>(g, tiles_n, ntiles);
}

namespace {

template <int BM>
void launch_ps(Exec& ex, const PsArgs& g) {
  constexpr int bytes = PsTile<BM>::LDS;
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)gemm_ps_kernel<BM>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return true;
  }();
  (void)attr;
  const int64_t tm = (g.M + BM - 1) / BM, tn = (g.N + PN - 1) / PN, nt = tm * tn;
  hipLaunchKernelGGL((gemm_ps_kernel<BM>), dim3((unsigned)xcd_grid(nt)), dim3(BM * 2), bytes, ex.stream, g, tn, nt);
}

}  // namespace

SplitMat take_split(Arena& ar, int64_t rows, int64_t kpad) {
  SplitMat s;
  s.nrb = (rows + 15) / 16;
  s.plane = s.nrb * 16 * kpad;
  s.kpad = kpad;
  s.p = ar.take<__bf16>(3 * s.plane);
  return s;
}

void split_rows(Exec& ex, const float* src, int64_t rows, int64_t K, int64_t lds, SplitMat dst) {
  if (rows <= 0 || !launch_ok(ex)) return;
  hipLaunchKernelGGL(k_split_rows, dim3(grid_for(rows * (dst.kpad / 2))), dim3(TPB), 0, ex.stream, src, rows, K, lds,
                     dst.kpad, reinterpret_cast<uint32_t*>(dst.p), dst.nrb, dst.plane);
}

void split_transpose(Exec& ex, const float* src, int64_t R, int64_t Cc, int64_t lds, SplitMat dst) {
  if (Cc <= 0 || !launch_ok(ex)) return;
  const int64_t blocks = ((dst.kpad + 63) / 64) * ((Cc + 63) / 64);
  hipLaunchKernelGGL(k_split_transpose, dim3((unsigned)blocks), dim3(256), 0, ex.stream, src, R, Cc, lds, dst.kpad,
                     reinterpret_cast<uint32_t*>(dst.p), dst.nrb, dst.plane);
}

void gemm_presplit(Exec& ex, int64_t M, int64_t N, const SplitMat& A, const SplitMat& B, float alpha, float beta,
                   float* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return;
  if (!launch_ok(ex)) return;
  PsArgs g;
  g.A = A.p; g.nrba = A.nrb; g.pa = A.plane;
  g.B = B.p; g.nrbb = B.nrb; g.pb = B.plane;
  g.M = M; g.N = N; g.K = A.kpad;
  g.C = C; g.scm = ldc; g.scn = 1;
  g.alpha = alpha; g.beta = beta;
  const int tok = prof_begin(ex, "gemm_bf16x6_presplit", 2.0 * M * N * A.kpad,
                             (double)(M + N) * A.kpad * 6.0 + (double)M * N * 4.0 * (beta != 0.f ? 2 : 1));
  if (M >= 256)
    launch_ps<256>(ex, g);
  else
    launch_ps<128>(ex, g);
  prof_end(ex, tok);
}

}  // namespace hs
