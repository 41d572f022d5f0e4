// Generic strided GEMM on MFMA (FP64 and FP32), used for the forward and backward
// passes, the curvature-factor propagation, the R-operator passes of dense
// Hessian-vector products and the subspace-iteration products.
//
// Tiling: 256 threads = 4 wavefronts in a 2 x 2 grid; each wavefront owns a
// (BM/2) x (BN/2) sub-tile made of 16 x 16 MFMA blocks.  The K dimension is staged
// through two LDS stages in chunks of 16 (one barrier per chunk), stored k-contiguous
// per row so that each lane picks
// up its four k values of a chunk with one vector read; the sum over k inside a
// chunk is permuted (lane group q takes k = 4q..4q+3 over the four MFMA steps),
// which is legal because A and B use the same permutation.
#include "mfma.h"

namespace hs {

namespace {

constexpr int KC = 16;
constexpr int KP = KC + 4;  // padded row length in LDS (bank spread)

// Raw buffer load of one element; an offset at or past num_records reads 0.
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// BUF: operands read through buffer resources (the host checks that every element of A
// and B lies within 2^31 bytes of its batch base), so an element outside M x K (N x K)
// gets an out-of-range offset and reads 0 with no branch; a guarded plain load compiles
// to a branch and a full wait per element.
template <typename T, int BM, int BN, bool BUF>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs<T> g, int64_t tiles_n, int64_t ntiles) {
  using Op = MfmaOp<T>;
  using acc_t = typename Op::acc_t;
  // two LDS stages: chunk c + 1 is stored into the other stage while chunk c is multiplied
  __shared__ __attribute__((aligned(16))) T As[2][BM * KP];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN * KP];

  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (tile < 0) return;
  const int64_t bz = blockIdx.y;
  const T* A = g.A + bz * g.sab;
  const T* B = g.B + bz * g.sbb;
  T* C = g.C + bz * g.scb;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  constexpr int WM = BM / 2, WN = BN / 2, RB = WM / 16, CB = WN / 16;
  const int64_t m0 = (tile / tiles_n) * BM, n0 = (tile % tiles_n) * BN;

  constexpr int AE = BM * KC / 256, BE = BN * KC / 256;
  const bool a_kfast = (g.sak == 1);
  const bool b_kfast = (g.sbk == 1);
  T ra[AE], rb[BE];

  auto idx_a = [&](int e, int& m, int& k) {
    if (a_kfast) { m = e / KC; k = e % KC; } else { k = e / BM; m = e % BM; }
  };
  auto idx_b = [&](int e, int& n, int& k) {
    if (b_kfast) { n = e / KC; k = e % KC; } else { k = e / BN; n = e % BN; }
  };
  __amdgpu_buffer_rsrc_t rsa, rsb;
  if constexpr (BUF) {
    rsa = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(A), (short)0, 0x7fffffff, 0x00020000);
    rsb = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(B), (short)0, 0x7fffffff, 0x00020000);
  }
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      int m, k;
      idx_a(tid + i * 256, m, k);
      const int64_t gm = m0 + m, gk = k0 + k;
      if constexpr (BUF) {
        const uint32_t off = (gm < g.M && gk < g.K) ? (uint32_t)((gm * g.sam + gk * g.sak) * (int64_t)sizeof(T))
                                                    : 0xfffffff0u;
        ra[i] = buf_load<T>(rsa, off);
      } else {
        ra[i] = (gm < g.M && gk < g.K) ? A[gm * g.sam + gk * g.sak] : T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      int n, k;
      idx_b(tid + i * 256, n, k);
      const int64_t gn = n0 + n, gk = k0 + k;
      if constexpr (BUF) {
        const uint32_t off = (gn < g.N && gk < g.K) ? (uint32_t)((gk * g.sbk + gn * g.sbn) * (int64_t)sizeof(T))
                                                    : 0xfffffff0u;
        rb[i] = buf_load<T>(rsb, off);
      } else {
        rb[i] = (gn < g.N && gk < g.K) ? B[gk * g.sbk + gn * g.sbn] : T(0);
      }
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      int m, k;
      idx_a(tid + i * 256, m, k);
      As[st][m * KP + k] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      int n, k;
      idx_b(tid + i * 256, n, k);
      Bs[st][n * KP + k] = rb[i];
    }
  };

  acc_t acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = Op::zero();

  const int row = lane & 15, q = lane >> 4;
  const int64_t nk = (g.K + KC - 1) / KC;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t kc = 0; kc < nk; ++kc) {
    const int st = (int)(kc & 1);
    if (kc + 1 < nk) load((kc + 1) * KC);
    T a[RB][4], b[CB][4];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int s = 0; s < 4; ++s) a[i][s] = As[st][(wr * WM + i * 16 + row) * KP + 4 * q + s];
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int s = 0; s < 4; ++s) b[j][s] = Bs[st][(wc * WN + j * 16 + row) * KP + 4 * q + s];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = Op::mma(a[i][s], b[j][s], acc[i][j]);
    // the other stage was last read in the previous chunk, before the barrier below
    if (kc + 1 < nk) store(st ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wr * WM + i * 16 + Op::row_of(q, v);
        const int64_t n = n0 + wc * WN + j * 16 + row;
        if (m < g.M && n < g.N) {
          T* c = C + m * g.scm + n * g.scn;
          const T val = g.alpha * acc[i][j][v];
          *c = (g.beta != T(0)) ? val + g.beta * (*c) : val;
        }
      }
}

// Byte extent of a strided operand (rows x k) from its batch base; strides are >= 0.
inline int64_t extent_bytes(int64_t rows, int64_t k, int64_t s_row, int64_t s_k, size_t elem) {
  return ((rows - 1) * s_row + (k - 1) * s_k + 1) * (int64_t)elem;
}

// FP32 GEMM with each product taken from BF16 MFMAs on three-way split operands
// (x = h + m + l by round-to-nearest-even of the remainder; products h h, h m, m h, h l,
// l h, m m accumulated in FP32 by v_mfma_f32_16x16x32_bf16): chunks of 32 k staged in two
// LDS stages, k-contiguous per row, so a lane's 8 consecutive k of a row are two 16-byte
// reads; the same tiling and output layout as the FP32 kernel.
constexpr int SKC = 32, SKP = SKC + 4;

template <int BM, int BN, bool BUF>
__global__ __launch_bounds__(256, 2) void gemm_split_kernel(GemmArgs<float> g, int64_t tiles_n, int64_t ntiles) {
  __shared__ __attribute__((aligned(16))) float As[2][BM * SKP];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN * SKP];
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (tile < 0) return;
  const int64_t bz = blockIdx.y;
  const float* A = g.A + bz * g.sab;
  const float* B = g.B + bz * g.sbb;
  float* C = g.C + bz * g.scb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  constexpr int WM = BM / 2, WN = BN / 2, RB = WM / 16, CB = WN / 16;
  const int64_t m0 = (tile / tiles_n) * BM, n0 = (tile % tiles_n) * BN;
  constexpr int AE = BM * SKC / 256, BE = BN * SKC / 256;
  const bool a_kfast = (g.sak == 1), b_kfast = (g.sbk == 1);
  float ra[AE], rb[BE];
  __amdgpu_buffer_rsrc_t rsa, rsb;
  if constexpr (BUF) {
    rsa = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(A), (short)0, 0x7fffffff, 0x00020000);
    rsb = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(B), (short)0, 0x7fffffff, 0x00020000);
  }
  auto idx_a = [&](int e, int& m, int& k) {
    if (a_kfast) { m = e / SKC; k = e % SKC; } else { k = e / BM; m = e % BM; }
  };
  auto idx_b = [&](int e, int& n, int& k) {
    if (b_kfast) { n = e / SKC; k = e % SKC; } else { k = e / BN; n = e % BN; }
  };
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      int m, k;
      idx_a(tid + i * 256, m, k);
      const int64_t gm = m0 + m, gk = k0 + k;
      if constexpr (BUF) {
        const uint32_t off = (gm < g.M && gk < g.K) ? (uint32_t)((gm * g.sam + gk * g.sak) * 4) : 0xfffffff0u;
        ra[i] = buf_load<float>(rsa, off);
      } else {
        ra[i] = (gm < g.M && gk < g.K) ? A[gm * g.sam + gk * g.sak] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      int n, k;
      idx_b(tid + i * 256, n, k);
      const int64_t gn = n0 + n, gk = k0 + k;
      if constexpr (BUF) {
        const uint32_t off = (gn < g.N && gk < g.K) ? (uint32_t)((gk * g.sbk + gn * g.sbn) * 4) : 0xfffffff0u;
        rb[i] = buf_load<float>(rsb, off);
      } else {
        rb[i] = (gn < g.N && gk < g.K) ? B[gk * g.sbk + gn * g.sbn] : 0.f;
      }
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      int m, k;
      idx_a(tid + i * 256, m, k);
      As[st][m * SKP + k] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      int n, k;
      idx_b(tid + i * 256, n, k);
      Bs[st][n * SKP + k] = rb[i];
    }
  };
  f4_t acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  const int row = lane & 15, q = lane >> 4;
  const int64_t nk = (g.K + SKC - 1) / SKC;
  const SplitC sc = split_consts();
  load(0);
  store(0);
  __syncthreads();
  for (int64_t kc = 0; kc < nk; ++kc) {
    const int st = (int)(kc & 1);
    if (kc + 1 < nk) load((kc + 1) * SKC);
    bf8_t bh[CB], bm[CB], bl[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      float v[8];
      const f4_t* p = (const f4_t*)&Bs[st][(wc * WN + j * 16 + row) * SKP + 8 * q];
      const f4_t v0 = p[0], v1 = p[1];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        v[s] = v0[s];
        v[4 + s] = v1[s];
      }
      split3x8(v, bh[j], bm[j], bl[j], sc);
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      float v[8];
      const f4_t* p = (const f4_t*)&As[st][(wr * WM + i * 16 + row) * SKP + 8 * q];
      const f4_t v0 = p[0], v1 = p[1];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        v[s] = v0[s];
        v[4 + s] = v1[s];
      }
      bf8_t ah, am, al;
      split3x8(v, ah, am, al, sc);
#pragma unroll
      for (int pr = 0; pr < 6; ++pr)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = mma_bf16(pr_x(pr, ah, am, al), pr_y(pr, bh[j], bm[j], bl[j]), acc[i][j]);
    }
    if (kc + 1 < nk) store(st ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wr * WM + i * 16 + 4 * q + v;
        const int64_t n = n0 + wc * WN + j * 16 + row;
        if (m < g.M && n < g.N) {
          float* c = C + m * g.scm + n * g.scn;
          const float val = g.alpha * acc[i][j][v];
          *c = (g.beta != 0.f) ? val + g.beta * (*c) : val;
        }
      }
}

template <typename T, int BM, int BN>
void launch(Exec& ex, const GemmArgs<T>& g) {
  const int64_t tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  const int64_t nt = tm * tn;
  dim3 grid((unsigned)xcd_grid(nt), (unsigned)g.batch);
  if (!launch_ok(ex)) return;
  const double b = (double)g.batch;
  // split products for FP32 under ex.split, except short contractions (K <= 128), which
  // keep the FP32 MFMA tile: the split form pads K to chunks of 32 and its six products
  // and splits cost more than they save there
  const bool split = sizeof(T) == 4 && ex.split && g.K > 128;
  const int tok = prof_begin(ex, sizeof(T) == 8 ? "gemm_f64" : (split ? "gemm_bf16x6" : "gemm_f32"),
                             2.0 * g.M * g.N * g.K * b,
                             (double)(g.M * g.K + g.K * g.N + g.M * g.N) * sizeof(T) * b);
  const int64_t lim = 0x7fffff00;
  const bool buf = g.sam >= 0 && g.sak >= 0 && g.sbk >= 0 && g.sbn >= 0 &&
                   extent_bytes(g.M, g.K, g.sam, g.sak, sizeof(T)) < lim &&
                   extent_bytes(g.N, g.K, g.sbn, g.sbk, sizeof(T)) < lim;
  if constexpr (sizeof(T) == 4) {
    if (split) {  // FP32 products from split-BF16 MFMAs: tiles of BM x BN/2 (register budget)
      constexpr int SBN = BN / 2;
      const int64_t stn = (g.N + SBN - 1) / SBN, snt = tm * stn;
      const dim3 sgrid((unsigned)xcd_grid(snt), (unsigned)g.batch);
      if (buf)
        hipLaunchKernelGGL((gemm_split_kernel<BM, SBN, true>), sgrid, dim3(256), 0, ex.stream, g, stn, snt);
      else
        hipLaunchKernelGGL((gemm_split_kernel<BM, SBN, false>), sgrid, dim3(256), 0, ex.stream, g, stn, snt);
      prof_end(ex, tok);
      return;
    }
  }
  if (buf)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, true>), grid, dim3(256), 0, ex.stream, g, tn, nt);
  else
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, false>), grid, dim3(256), 0, ex.stream, g, tn, nt);
  prof_end(ex, tok);
}

}  // namespace

template <typename T>
void gemm(Exec& ex, const GemmArgs<T>& g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  if (g.M >= 128 && g.N >= 128)
    launch<T, 128, 128>(ex, g);
  else
    launch<T, 64, 64>(ex, g);
}

template <typename T>
void gemm_rm(Exec& ex, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, const T* A,
             int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc) {
  GemmArgs<T> g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.sam = ta ? 1 : lda; g.sak = ta ? lda : 1; g.sab = 0;
  g.B = B; g.sbk = tb ? 1 : ldb; g.sbn = tb ? ldb : 1; g.sbb = 0;
  g.C = C; g.scm = ldc; g.scn = 1; g.scb = 0;
  g.alpha = alpha; g.beta = beta; g.batch = 1;
  gemm<T>(ex, g);
}

template void gemm<float>(Exec&, const GemmArgs<float>&);
template void gemm<double>(Exec&, const GemmArgs<double>&);
template void gemm_rm<float>(Exec&, bool, bool, int64_t, int64_t, int64_t, float, const float*,
                             int64_t, const float*, int64_t, float, float*, int64_t);
template void gemm_rm<double>(Exec&, bool, bool, int64_t, int64_t, int64_t, double, const double*,
                              int64_t, const double*, int64_t, double, double*, int64_t);

}  // namespace hs
