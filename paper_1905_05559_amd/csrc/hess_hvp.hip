// Hessian-vector products for B dense directions (paper, Sec. 5.1 and Appendix A.1),
// by forward-over-reverse R-operator propagation through every layer's W, b and sigma:
//
//   R{Z^(l)}     = R{A^(l-1)} W^(l-1)^T + Abar^(l-1) Vbar^(l-1)^T          (R{A^(1)} = 0)
//   R{A^(l)}     = sigma'(Z^(l)) * R{Z^(l)}
//   R{delta^(L)} = Yhat * (R{Z^(L)} - sum(Yhat * R{Z^(L)}))
//   R{delta^(l)} = sigma''(Z^(l)) E^(l) * R{Z^(l)}
//                  + sigma'(Z^(l)) * (R{delta^(l+1)} W^(l) + delta^(l+1) V_W^(l))
//   (HV)_{Wbar^(l-1)} = (1/N) [ R{delta^(l)}^T Abar^(l-1) + delta^(l)^T R{A^(l-1)} ]
//
// (Vbar = [V_W | V_b]; the ones column of Abar turns the weight formula into the bias
// one.)  R tensors are laid out [n][b][unit] so the W products are plain GEMMs over
// (n, b) rows and the direction-dependent products are GEMMs batched over b.  The
// example range is processed in chunks to bound the workspace; the accumulation over
// chunks is the sum over n of the definition.
#include <algorithm>
#include <cmath>

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

// Vbar[(b, i)][j] = V[b][offW + i*Tin + j] (j < Tin), V[b][offb + i] (j == Tin)
template <typename T>
__global__ void k_pack_vbar(const T* V, int64_t B, int64_t P, int64_t offW, int64_t offb, int64_t Tout,
                            int64_t Tin, T* Vbar) {
  GRID_STRIDE(e, B * Tout * (Tin + 1)) {
    const int64_t j = e % (Tin + 1), bi = e / (Tin + 1), i = bi % Tout, b = bi / Tout;
    Vbar[e] = V[b * P + (j < Tin ? offW + i * Tin + j : offb + i)];
  }
}

template <typename T>
__global__ void k_unpack_hv(const T* HVbar, int64_t B, int64_t P, int64_t offW, int64_t offb, int64_t Tout,
                            int64_t Tin, T* HV) {
  GRID_STRIDE(e, B * Tout * (Tin + 1)) {
    const int64_t j = e % (Tin + 1), bi = e / (Tin + 1), i = bi % Tout, b = bi / Tout;
    HV[b * P + (j < Tin ? offW + i * Tin + j : offb + i)] = HVbar[e];
  }
}

// HVbar_b[i][j] += Tacc[i][b T_in + j] for the weight columns j < T_in of every direction b
template <typename T>
__global__ void k_add_wcols(const T* Tacc, int64_t B, int64_t Tl, int64_t Tin, T* HVbar) {
  GRID_STRIDE(e, Tl * B * Tin) {
    const int64_t i = e / (B * Tin), r = e % (B * Tin), b = r / Tin, j = r % Tin;
    HVbar[(b * Tl + i) * (Tin + 1) + j] += Tacc[e];
  }
}

// RA[n][b][t] = D1[n][t] * RZ[n][b][t]
template <typename T>
__global__ void k_ra(const T* RZ, const T* D1, int64_t Nc, int64_t B, int64_t Tl, T* RA) {
  GRID_STRIDE(e, Nc * B * Tl) {
    const int64_t t = e % Tl, n = e / (B * Tl);
    RA[e] = D1[n * Tl + t] * RZ[e];
  }
}

// RD[n][b][:] = Yhat[n] * (RZ[n][b][:] - sum_t Yhat[n][t] RZ[n][b][t]), one thread per (n, b)
template <typename T>
__global__ void k_ryhat(const T* RZ, const T* Yh, int64_t Nc, int64_t B, int64_t TL, T* RD) {
  GRID_STRIDE(e, Nc * B) {
    const int64_t n = e / B;
    const T* z = RZ + e * TL;
    const T* p = Yh + n * TL;
    T s = 0;
    for (int64_t t = 0; t < TL; ++t) s += p[t] * z[t];
    for (int64_t t = 0; t < TL; ++t) RD[e * TL + t] = p[t] * (z[t] - s);
  }
}

// RD[n][b][t] = D1[n][t] * RD[n][b][t] + CE[n][t] * RZ[n][b][t]
template <typename T>
__global__ void k_rdelta(T* RD, const T* RZ, const T* D1, const T* CE, int64_t Nc, int64_t B, int64_t Tl) {
  GRID_STRIDE(e, Nc * B * Tl) {
    const int64_t t = e % Tl, n = e / (B * Tl);
    RD[e] = D1[n * Tl + t] * RD[e] + CE[n * Tl + t] * RZ[e];
  }
}

// R{delta^(l)} of one example chunk when the next layer has at most RDS_TN units, computed
// in one pass and written directly as the split transpose that the accumulation product
// R{delta^(l)}^T abar^(l-1) reads (row c = b T_l + t, k = n; the three BF16 planes of the
// compensated split, zero for Nc <= n < rpad):
//   RD[n][b][t] = D1[n][t] (sum_k RDn[n][b][k] Wn[k][t] + sum_k dn[n][k] Vn_b[k][t])
//                 + CE[n][t] RZ[n][b][t]
// (the two K = T_{l+1} products and the sigma' / sigma'' terms of the R-backward step,
// which otherwise take two GEMMs, an elementwise pass and a transpose pass over the
// N_c x B T_l tensor).  Tiles of 64 examples x 64 columns (T_l >= 32, so a tile spans at
// most three directions b): a lane owns one column c and keeps its W and V_b columns in
// registers; the tile's rows of RDn (its directions) and of dn are staged in LDS and read
// as broadcasts; RZ, D1 and CE are read along c; the finished tile is split and written
// transposed through LDS as in k_split_transpose.
constexpr int RDS_TN = 32;
constexpr int RDS_SUB = 1;  // 64-example subtiles of a workgroup (4 measured slower: 21 against 16 ms per 512 HVPs)
template <int TN>
__global__ __launch_bounds__(256) void k_rdelta_split(const float* __restrict__ RZ, const float* __restrict__ RDn,
                                                      const float* __restrict__ Wn, const float* __restrict__ dn,
                                                      const float* __restrict__ Vn, const float* __restrict__ D1,
                                                      const float* __restrict__ CE, int64_t Nc, int64_t B, int Tl,
                                                      int Tn, int64_t rpad, uint32_t* __restrict__ dst, int64_t nrb,
                                                      int64_t pl, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) float rdn_s[64][3 * TN];
  __shared__ __attribute__((aligned(16))) float dn_s[64][TN];
  __shared__ float tile[64][65];
  __shared__ float red[4][TN][64];
  const int64_t BT = B * Tl;
  const int64_t tn = (rpad + 64 * RDS_SUB - 1) / (64 * RDS_SUB);
  const int64_t grp = (int64_t)(blockIdx.x % tn), c0 = (int64_t)(blockIdx.x / tn) * 64;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t blo = c0 / Tl;
  const int nbt = (int)(std::min(c0 + 63, BT - 1) / Tl - blo + 1);  // directions in the tile (<= 3)
  const int64_t c = c0 + lane;
  const bool cok = c < BT;
  const int64_t b = cok ? c / Tl : blo;
  const int t = cok ? (int)(c - b * Tl) : 0;
  const int bb = (int)(b - blo);
  float wr[TN], vr[TN];
#pragma unroll
  for (int k = 0; k < TN; ++k) {
    wr[k] = cok && k < Tn ? Wn[(int64_t)k * Tl + t] : 0.f;
    vr[k] = cok && k < Tn ? Vn[(b * Tn + k) * (Tl + 1) + t] : 0.f;
  }
  const int nq = (Tn + 3) / 4;
  float pacc[TN];  // this wavefront's rows of sum_n dn[n][k] R{A}[n][c] (R{A} = D1 * RZ)
#pragma unroll
  for (int k = 0; k < TN; ++k) pacc[k] = 0.f;
  const SplitC sc = split_consts();
  constexpr int RE = 64 * 3 * TN / 256, DE = 64 * TN / 256;
  for (int sub = 0; sub < RDS_SUB; ++sub) {
    const int64_t n0 = (grp * RDS_SUB + sub) * 64;
    if (n0 >= rpad) break;
    // every global read of the subtile is issued before any is used (fully unrolled loops),
    // so a wavefront waits for memory once rather than once per row
    float rv[RE], dv[DE];
#pragma unroll
    for (int x = 0; x < RE; ++x) {
      const int e = threadIdx.x + 256 * x;
      const int y = e / (3 * TN), j = e - y * (3 * TN), bq = j / TN, k = j - bq * TN;
      const int64_t n = n0 + y;
      rv[x] = (n < Nc && bq < nbt && k < Tn) ? RDn[(n * B + blo + bq) * Tn + k] : 0.f;
    }
#pragma unroll
    for (int x = 0; x < DE; ++x) {
      const int e = threadIdx.x + 256 * x;
      const int y = e / TN, k = e - y * TN;
      const int64_t n = n0 + y;
      dv[x] = (n < Nc && k < Tn) ? dn[n * Tn + k] : 0.f;
    }
    // this wavefront's rows y = wave + 4 i
    float zr[16], d1r[16], cer[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t n = n0 + wave + 4 * i;
      const bool ok = cok && n < Nc;
      zr[i] = ok ? RZ[n * BT + c] : 0.f;
      d1r[i] = ok ? D1[n * Tl + t] : 0.f;
      cer[i] = ok ? CE[n * Tl + t] : 0.f;
    }
    __syncthreads();  // the previous subtile's LDS reads are done
#pragma unroll
    for (int x = 0; x < RE; ++x) (&rdn_s[0][0])[threadIdx.x + 256 * x] = rv[x];
#pragma unroll
    for (int x = 0; x < DE; ++x) (&dn_s[0][0])[threadIdx.x + 256 * x] = dv[x];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int y = wave + 4 * i;
      const f4_t* rp = reinterpret_cast<const f4_t*>(&rdn_s[y][bb * TN]);
      const f4_t* dp = reinterpret_cast<const f4_t*>(&dn_s[y][0]);
      if (part) {
        const float ra = d1r[i] * zr[i];
#pragma unroll
        for (int qd = 0; qd < TN / 4; ++qd) {
          if (qd < nq) {
            const f4_t d4 = dp[qd];
            pacc[4 * qd] += d4[0] * ra;
            pacc[4 * qd + 1] += d4[1] * ra;
            pacc[4 * qd + 2] += d4[2] * ra;
            pacc[4 * qd + 3] += d4[3] * ra;
          }
        }
      }
      float acc = 0.f;
#pragma unroll
      for (int qd = 0; qd < TN / 4; ++qd) {
        if (qd < nq) {
          const f4_t r4 = rp[qd];
          acc += r4[0] * wr[4 * qd] + r4[1] * wr[4 * qd + 1] + r4[2] * wr[4 * qd + 2] + r4[3] * wr[4 * qd + 3];
        }
      }
#pragma unroll
      for (int qd = 0; qd < TN / 4; ++qd) {
        if (qd < nq) {
          const f4_t d4 = dp[qd];
          acc += d4[0] * vr[4 * qd] + d4[1] * vr[4 * qd + 1] + d4[2] * vr[4 * qd + 2] + d4[3] * vr[4 * qd + 3];
        }
      }
      tile[y][lane] = d1r[i] * acc + cer[i] * zr[i];  // zero outside the chunk and past the columns
    }
    __syncthreads();
    const int pr = threadIdx.x & 31;  // pair of rows 2 pr, 2 pr + 1 of the tile
    for (int cc = threadIdx.x >> 5; cc < 64; cc += 8) {
      const int64_t col = c0 + cc, r = n0 + 2 * pr;
      if (col >= BT || r >= rpad) continue;
      bf2_t h, m, l;
      split3x2(f2_t{tile[2 * pr][cc], tile[2 * pr + 1][cc]}, h, m, l, sc);
      const int64_t o = ps_off(col, r, nrb) / 2;
      dst[o] = __builtin_bit_cast(uint32_t, h);
      dst[o + pl / 2] = __builtin_bit_cast(uint32_t, m);
      dst[o + pl] = __builtin_bit_cast(uint32_t, l);
    }
  }
  if (part) {
#pragma unroll
    for (int k = 0; k < TN; ++k) red[wave][k][lane] = pacc[k];
    __syncthreads();
    // the group's partial over its examples: waves summed in order
    if (cok)
      for (int k = wave; k < Tn; k += 4)
        part[(grp * Tn + k) * BT + c] = ((red[0][k][lane] + red[1][k][lane]) + red[2][k][lane]) + red[3][k][lane];
  }
}

// HVbar_next_b[k][t] += invN sum_j part[j][k][b T_l + t] for the weight columns t < T_l of the
// next layer's block of every direction b: the delta^(l+1)^T R{A^(l)} term of the accumulation,
// summed over the example tiles of a chunk in tile order.
__global__ __launch_bounds__(256) void k_sum_rapart(const float* __restrict__ part, int64_t ntiles, int Tn,
                                                    int64_t B, int Tl, float invN, float* __restrict__ HVn) {
  const int64_t BT = B * Tl;
  GRID_STRIDE(e, (int64_t)Tn * BT) {
    const int64_t k = e / BT, c = e - k * BT, b = c / Tl, t = c - b * Tl;
    float sum = 0.f;
    for (int64_t j = 0; j < ntiles; ++j) sum += part[(j * Tn + k) * BT + c];
    HVn[(b * Tn + k) * (Tl + 1) + t] += invN * sum;
  }
}

// RZn[r][k] += sum_t D1[n][t] RZ[r][t] Wn[k][t] for the rows r = n B + b of a chunk: the
// R{A^(l)} W^(l)^T term of the next layer's R{Z} with R{A^(l)} = sigma'(Z^(l)) * R{Z^(l)} formed
// on the fly.  A wavefront owns 64 rows (a lane one row and its T_{l+1} <= TN sums); chunks
// of 32 of the T_l columns of its rows and of sigma' are staged in LDS with reads along t.
template <int TN>
__global__ __launch_bounds__(256) void k_rz_next(const float* __restrict__ RZ, const float* __restrict__ D1,
                                                 const float* __restrict__ Wn, int64_t rows, int64_t B, int Tl, int Tn,
                                                 float* __restrict__ RZn) {
  __shared__ float ras[4][64][33];  // R{A} of this wavefront's rows, 32 columns at a time
  __shared__ float ws[TN][32];
  __shared__ int64_t nrow[4][64];   // example of each row
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = (int64_t)blockIdx.x * 256 + wave * 64;
  nrow[wave][lane] = (r0 + lane) / B;
  float acc[TN];
#pragma unroll
  for (int k = 0; k < TN; ++k) acc[k] = 0.f;
  for (int t0 = 0; t0 < Tl; t0 += 32) {
    __syncthreads();
    for (int e = threadIdx.x; e < TN * 32; e += 256) {
      const int k = e >> 5, tt = e & 31;
      ws[k][tt] = (k < Tn && t0 + tt < Tl) ? Wn[(int64_t)k * Tl + t0 + tt] : 0.f;
    }
    // all 32 reads of R{Z} and of sigma' issued before any is used
    float zv[32], dv[32];
#pragma unroll
    for (int x = 0; x < 32; ++x) {
      const int e = lane + 64 * x, i = e >> 5, tt = e & 31;
      const int64_t rr = r0 + i;
      const bool ok = rr < rows && t0 + tt < Tl;
      zv[x] = ok ? RZ[rr * Tl + t0 + tt] : 0.f;
      dv[x] = ok ? D1[nrow[wave][i] * Tl + t0 + tt] : 0.f;
    }
#pragma unroll
    for (int x = 0; x < 32; ++x) {
      const int e = lane + 64 * x;
      ras[wave][e >> 5][e & 31] = dv[x] * zv[x];
    }
    __syncthreads();
#pragma unroll 8
    for (int tt = 0; tt < 32; ++tt) {
      const float ra = ras[wave][lane][tt];
#pragma unroll
      for (int k = 0; k < TN; ++k) acc[k] += ra * ws[k][tt];
    }
  }
  const int64_t r = r0 + lane;
  if (r < rows)
    for (int k = 0; k < Tn; ++k) RZn[r * Tn + k] += acc[k];
}

// S[n][b] = sum_i delta2[n][i] U2[n][b][i] + (same for layers 3 and 4 when present)
template <typename T>
__global__ void k_jv(const T* U2, const T* U3, const T* U4, const T* d2, const T* d3, const T* d4, int64_t T2,
                     int64_t T3, int64_t T4, int64_t Nc, int64_t B, T* S) {
  GRID_STRIDE(e, Nc * B) {
    const int64_t n = e / B;
    T s = 0;
    for (int64_t i = 0; i < T2; ++i) s += d2[n * T2 + i] * U2[e * T2 + i];
    if (d3)
      for (int64_t i = 0; i < T3; ++i) s += d3[n * T3 + i] * U3[e * T3 + i];
    if (d4)
      for (int64_t i = 0; i < T4; ++i) s += d4[n * T4 + i] * U4[e * T4 + i];
    S[e] = s;
  }
}

template <typename T>
__global__ void k_jv_add(const T* U, const T* d, int64_t Tl, int64_t Nc, int64_t B, T* S) {
  GRID_STRIDE(e, Nc * B) {
    const int64_t n = e / B;
    T s = 0;
    for (int64_t i = 0; i < Tl; ++i) s += d[n * Tl + i] * U[e * Tl + i];
    S[e] += s;
  }
}

// D[n][b][i] = delta[n][i] * S[n][b]
template <typename T>
__global__ void k_dscale(const T* d, const T* S, int64_t Nc, int64_t B, int64_t Tl, T* D) {
  GRID_STRIDE(e, Nc * B * Tl) {
    const int64_t i = e % Tl, nb = e / Tl, n = nb / B;
    D[e] = d[n * Tl + i] * S[nb];
  }
}

#define LAUNCH(kernel, n, ...)                                                                 \
  do {                                                                                         \
    if (!launch_ok(ex)) return;                                                                \
    hipLaunchKernelGGL(kernel, dim3(grid_for(n)), dim3(TPB), 0, ex.stream, __VA_ARGS__);       \
  } while (0)

int64_t hvp_chunk(const Model& m, int64_t N, int64_t B, size_t esz) {
  int64_t sumT = 0;
  for (int l = 2; l <= m.L; ++l) sumT += m.T[l - 1];
  const double budget = 6.0e9;  // bytes of R tensors per chunk
  int64_t nc = (int64_t)(budget / ((double)B * sumT * 3.0 * esz));
  nc = std::max<int64_t>(64, nc / 64 * 64);
  return std::min(N, nc);
}

}  // namespace

// Products of the sweep that take pre-split operands (split products, FP32): R{Z^(l)} when
// its contraction (T_{l-1} + 1 inputs) is longer than 128 (shorter ones keep the FP32 MFMA
// tile), and the accumulation over a chunk of examples when the chunk is.
static bool presplit_rz(const Model& m, int l) { return m.T[l - 2] + 1 > 128; }
// The accumulation takes pre-split operands when the chunk is longer than 128 examples and
// its output (B T_l x (T_{l-1} + 1)) has enough 256 x 128 tiles to fill the device; a small
// output (the output layer of a classifier) keeps the FP32 tile, which spreads it over more
// workgroups.
static bool presplit_acc(int64_t Nc, int64_t rows, int64_t cols) {
  return Nc > 128 && ((rows + 255) / 256) * ((cols + 127) / 128) >= 128;
}
// R{delta^(2)} of a chunk formed and split in one pass (k_rdelta_split) when its
// accumulation takes pre-split operands and the next layer is narrow.
static bool fused_rdelta(const Model& m, int l, int64_t Nc, int64_t B) {
  return l == 2 && m.L >= 3 && m.T[l] <= RDS_TN && m.T[l - 1] >= 32 && presplit_acc(Nc, B * m.T[l - 1], m.T[l - 2] + 1);
}
// ... and, when that layer is the last hidden one, R{A^(2)} = sigma' * R{Z^(2)} is never
// stored: the output layer's R{Z} reads R{Z^(2)} and sigma' (k_rz_next) and the one-pass
// step leaves the partials of delta^(3)^T R{A^(2)} (k_sum_rapart).
static bool fused_ra(const Model& m, int64_t Nc, int64_t B) { return m.L == 3 && fused_rdelta(m, 2, Nc, B); }
static int64_t rapart_tiles(int64_t Nc) { return (rup(Nc, 32) + 64 * RDS_SUB - 1) / (64 * RDS_SUB); }

template <typename T>
size_t plan_hvp(Arena& ar, const Model& m, int64_t N, int64_t B, Prep& p, HvpBufs<T>& h, bool split) {
  const int L = m.L;
  plan_prep(ar, m, N, p, false);
  h.abar.assign(L + 1, nullptr);
  h.delta.assign(L + 1, nullptr);
  h.D1.assign(L + 1, nullptr);
  h.CE.assign(L + 1, nullptr);
  h.W.assign(L + 1, nullptr);
  h.Vbar.assign(L + 1, nullptr);
  h.HVbar.assign(L + 1, nullptr);
  h.RZ.assign(L + 1, nullptr);
  h.RA.assign(L + 1, nullptr);
  h.RD.assign(L + 1, nullptr);
  const bool same = sizeof(T) == 8;
  for (int l = 1; l <= L - 1; ++l) h.abar[l] = same ? nullptr : ar.take<T>(N * p.lda[l]);
  for (int l = 2; l <= L; ++l) h.delta[l] = same ? nullptr : ar.take<T>(N * m.T[l - 1]);
  for (int l = 2; l <= L - 1; ++l) {
    h.D1[l] = same ? nullptr : ar.take<T>(N * m.T[l - 1]);
    h.CE[l] = ar.take<T>(N * m.T[l - 1]);
  }
  h.Yhat = same ? nullptr : ar.take<T>(N * m.T[L - 1]);
  for (int l = 2; l <= L; ++l) {
    h.W[l] = same ? nullptr : ar.take<T>(m.T[l - 1] * m.T[l - 2]);
    h.Vbar[l] = ar.take<T>(B * m.T[l - 1] * (m.T[l - 2] + 1));
    h.HVbar[l] = ar.take<T>(B * m.T[l - 1] * (m.T[l - 2] + 1));
  }
  h.Nc = hvp_chunk(m, N, B, sizeof(T));
  for (int l = 2; l <= L; ++l) {
    h.RZ[l] = ar.take<T>(h.Nc * B * m.T[l - 1]);
    h.RD[l] = ar.take<T>(h.Nc * B * m.T[l - 1]);
    if (l < L) h.RA[l] = ar.take<T>(h.Nc * B * m.T[l - 1]);
  }
  h.S = ar.take<T>(h.Nc * B);
  int64_t tacc = 0;
  for (int l = 3; l <= L; ++l) tacc = std::max<int64_t>(tacc, m.T[l - 1] * B * m.T[l - 2]);
  h.Tacc = tacc > 0 ? ar.take<T>(tacc) : nullptr;
  h.Bmax = B;
  h.split = split && sizeof(T) == 4;
  h.Vps.assign(L + 1, SplitMat());
  h.Aps.assign(L + 1, SplitMat());
  h.ATps.assign(L + 1, SplitMat());
  h.RDps = SplitMat();
  if (h.split) {
    int64_t rd_rows = 0;
    for (int l = 2; l <= L; ++l) {
      const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
      if (presplit_rz(m, l)) {
        h.Vps[l] = take_split(ar, B * Tl, rup(Tin + 1, 32));
        h.Aps[l] = take_split(ar, h.Nc, rup(Tin + 1, 32));
      }
      if (presplit_acc(h.Nc, B * Tl, Tin + 1)) {
        h.ATps[l] = take_split(ar, Tin + 1, rup(h.Nc, 32));
        rd_rows = std::max(rd_rows, B * Tl);
      }
    }
    if (rd_rows > 0) h.RDps = take_split(ar, rd_rows, rup(h.Nc, 32));
    if (fused_ra(m, h.Nc, B)) h.RApart = ar.take<T>(rapart_tiles(h.Nc) * m.T[2] * B * m.T[1]);
  }
  return ar.used;
}

// Operands of the R-operator passes in the arithmetic precision (once per call).
template <typename T>
void hvp_setup(Exec& ex, const Model& m, int64_t N, Prep& p, HvpBufs<T>& h) {
  const int L = m.L;
  const bool same = sizeof(T) == 8;
  // operands in the arithmetic precision
  for (int l = 1; l <= L - 1; ++l) {
    if (same)
      h.abar[l] = reinterpret_cast<T*>(p.Abar[l]);
    else
      cast_copy<T>(ex, p.Abar[l], h.abar[l], N * p.lda[l]);
  }
  for (int l = 2; l <= L; ++l) {
    if (same)
      h.delta[l] = reinterpret_cast<T*>(p.delta[l]);
    else
      cast_copy<T>(ex, p.delta[l], h.delta[l], N * m.T[l - 1]);
  }
  for (int l = 2; l <= L - 1; ++l) {
    const int64_t n = N * m.T[l - 1];
    mul(ex, p.D2[l], p.E[l], p.Z, n);  // sigma'' E in FP64, then cast
    cast_copy<T>(ex, p.Z, h.CE[l], n);
    if (same)
      h.D1[l] = reinterpret_cast<T*>(p.D1[l]);
    else
      cast_copy<T>(ex, p.D1[l], h.D1[l], n);
  }
  if (same)
    h.Yhat = reinterpret_cast<T*>(p.Yhat);
  else
    cast_copy<T>(ex, p.Yhat, h.Yhat, N * m.T[L - 1]);
  for (int l = 2; l <= L; ++l) {
    const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
    if (same)
      h.W[l] = reinterpret_cast<T*>(p.W64[l - 2]);
    else
      cast_copy<T>(ex, p.W64[l - 2], h.W[l], Tl * Tin);
  }
}

// HV[b, :] = H V[b, :] for b < B (rows of V and HV have stride ldv).
template <typename T>
void hvp_apply(Exec& ex, const Model& m, int64_t N, int64_t B, Prep& p, HvpBufs<T>& h, const T* V, int64_t ldv,
               T* HV) {
  const int L = m.L;
  for (int l = 2; l <= L; ++l) {
    const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
    LAUNCH(k_pack_vbar<T>, B * Tl * (Tin + 1), V, B, ldv, m.offW[l - 2], m.offb[l - 2], Tl, Tin, h.Vbar[l]);
  }

  const T invN = (T)(1.0 / (double)N);
  if constexpr (sizeof(T) == 4) {  // the direction block, split once for all chunks
    for (int l = 2; l <= L; ++l)
      if (h.Vps[l].p) split_rows(ex, h.Vbar[l], B * m.T[l - 1], m.T[l - 2] + 1, m.T[l - 2] + 1, h.Vps[l]);
  }
  for (int64_t n0 = 0; n0 < N; n0 += h.Nc) {
    const int64_t Nc = std::min(h.Nc, N - n0);
    const T beta_acc = n0 == 0 ? T(0) : T(1);
    const bool fra = sizeof(T) == 4 && h.RApart && h.ATps[2].p && fused_ra(m, Nc, B);
    // ---- R-forward
    for (int l = 2; l <= L; ++l) {
      const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
      // R{Z^(l)} = Abar^(l-1) Vbar^T  (N_c x (B T_l)) ...
      bool done = false;
      if constexpr (sizeof(T) == 4) {
        if (h.Vps[l].p) {
          split_rows(ex, h.abar[l - 1] + n0 * p.lda[l - 1], Nc, Tin + 1, p.lda[l - 1], h.Aps[l]);
          gemm_presplit(ex, Nc, B * Tl, h.Aps[l], h.Vps[l], 1.f, 0.f, h.RZ[l], B * Tl);
          done = true;
        }
      }
      if (!done)
        gemm_rm<T>(ex, false, true, Nc, B * Tl, Tin + 1, T(1), h.abar[l - 1] + n0 * p.lda[l - 1], p.lda[l - 1],
                   h.Vbar[l], Tin + 1, T(0), h.RZ[l], B * Tl);
      // ... + R{A^(l-1)} W^(l-1)^T  ((N_c B) x T_l)
      if constexpr (sizeof(T) == 4) {
        if (l == 3 && fra) {
          const int64_t rows = Nc * B;
          if (!launch_ok(ex)) return;
          auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, ex.stream, h.RZ[2],
                               h.D1[2] + n0 * Tin, h.W[3], rows, B, (int)Tin, (int)Tl, h.RZ[3]);
          };
          if (Tl <= 16) go(k_rz_next<16>); else go(k_rz_next<RDS_TN>);
          continue;  // (l == L: no R{A^(3)})
        }
      }
      if (l >= 3)
        gemm_rm<T>(ex, false, true, Nc * B, Tl, Tin, T(1), h.RA[l - 1], Tin, h.W[l], Tin, T(1), h.RZ[l], Tl);
      if (l < L && !fra) LAUNCH(k_ra<T>, Nc * B * Tl, h.RZ[l], h.D1[l] + n0 * Tl, Nc, B, Tl, h.RA[l]);
    }
    // ---- R-backward
    LAUNCH(k_ryhat<T>, Nc * B, h.RZ[L], h.Yhat + n0 * m.T[L - 1], Nc, B, m.T[L - 1], h.RD[L]);
    for (int l = L - 1; l >= 2; --l) {
      const int64_t Tl = m.T[l - 1], Tn = m.T[l];
      if constexpr (sizeof(T) == 4) {
        if (h.ATps[l].p && fused_rdelta(m, l, Nc, B)) {
          // formed, split and transposed at once into the accumulation operand
          SplitMat a = h.RDps;
          a.kpad = rup(Nc, 32);
          const int64_t blocks = ((a.kpad + 64 * RDS_SUB - 1) / (64 * RDS_SUB)) * ((B * Tl + 63) / 64);
          if (!launch_ok(ex)) return;
          auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, ex.stream, h.RZ[l], h.RD[l + 1],
                               h.W[l + 1], h.delta[l + 1] + n0 * Tn, h.Vbar[l + 1], h.D1[l] + n0 * Tl,
                               h.CE[l] + n0 * Tl, Nc, B, (int)Tl, (int)Tn, a.kpad,
                               reinterpret_cast<uint32_t*>(a.p), a.nrb, a.plane, fra ? h.RApart : nullptr);
          };
          if (Tn <= 16) go(k_rdelta_split<16>); else go(k_rdelta_split<RDS_TN>);
          continue;
        }
      }
      // R{delta^(l+1)} W^(l)   ((N_c B) x T_l)
      gemm_rm<T>(ex, false, false, Nc * B, Tl, Tn, T(1), h.RD[l + 1], Tn, h.W[l + 1], Tl, T(0), h.RD[l], Tl);
      // + delta^(l+1) V_W^(l)_b, batched over directions b
      GemmArgs<T> g;
      g.M = Nc; g.N = Tl; g.K = Tn;
      g.A = h.delta[l + 1] + n0 * Tn; g.sam = Tn; g.sak = 1; g.sab = 0;
      g.B = h.Vbar[l + 1]; g.sbk = Tl + 1; g.sbn = 1; g.sbb = Tn * (Tl + 1);
      g.C = h.RD[l]; g.scm = B * Tl; g.scn = 1; g.scb = Tl;
      g.alpha = T(1); g.beta = T(1); g.batch = B;
      gemm<T>(ex, g);
      LAUNCH(k_rdelta<T>, Nc * B * Tl, h.RD[l], h.RZ[l], h.D1[l] + n0 * Tl, h.CE[l] + n0 * Tl, Nc, B, Tl);
    }
    // ---- accumulation over the examples of this chunk
    for (int l = 2; l <= L; ++l) {
      const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
      // R{delta^(l)}^T Abar^(l-1): ((B T_l) x (T_in + 1)), contraction over n
      bool done = false;
      if constexpr (sizeof(T) == 4) {
        if (h.ATps[l].p && presplit_acc(Nc, B * Tl, Tin + 1)) {
          SplitMat a = h.RDps, b = h.ATps[l];
          a.kpad = b.kpad = rup(Nc, 32);
          if (!fused_rdelta(m, l, Nc, B)) split_transpose(ex, h.RD[l], Nc, B * Tl, B * Tl, a);
          split_transpose(ex, h.abar[l - 1] + n0 * p.lda[l - 1], Nc, Tin + 1, p.lda[l - 1], b);
          gemm_presplit(ex, B * Tl, Tin + 1, a, b, invN, beta_acc, h.HVbar[l], Tin + 1);
          done = true;
        }
      }
      if (!done)
        gemm_rm<T>(ex, true, false, B * Tl, Tin + 1, Nc, invN, h.RD[l], B * Tl, h.abar[l - 1] + n0 * p.lda[l - 1],
                   p.lda[l - 1], beta_acc, h.HVbar[l], Tin + 1);
      if constexpr (sizeof(T) == 4) {
        if (l == 3 && fra) {  // + delta^(3)^T R{A^(2)}_b from the one-pass step's partials
          const int64_t tot = Tl * B * Tin;
          if (!launch_ok(ex)) return;
          hipLaunchKernelGGL(k_sum_rapart, dim3(grid_for(tot)), dim3(TPB), 0, ex.stream, h.RApart,
                             rapart_tiles(Nc), (int)Tl, B, (int)Tin, (float)invN, h.HVbar[3]);
          continue;
        }
      }
      if (l >= 3) {
        // + delta^(l)^T R{A^(l-1)}_b for all directions at once: R{A} of the chunk is
        // N_c x (B T_in), so this is one T_l x (B T_in) product (rather than B products of
        // T_l x T_in, each a mostly empty tile); the result is added into the weight
        // columns of each direction's block
        gemm_rm<T>(ex, true, false, Tl, B * Tin, Nc, invN, h.delta[l] + n0 * Tl, Tl, h.RA[l - 1], B * Tin, T(0),
                   h.Tacc, B * Tin);
        LAUNCH(k_add_wcols<T>, Tl * B * Tin, h.Tacc, B, Tl, Tin, h.HVbar[l]);
      }
    }
  }
  for (int l = 2; l <= L; ++l) {
    const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
    LAUNCH(k_unpack_hv<T>, B * Tl * (Tin + 1), h.HVbar[l], B, ldv, m.offW[l - 2], m.offb[l - 2], Tl, Tin, HV);
  }
}

// OPG V without forming the OPG: (J^T (J v_b)) / N.  (J v_b)_n = sum_l delta^(l)_n . (Vbar_b^(l) abar^(l-1)_n),
// then the accumulation GEMM of the R-operator path with R{delta^(l)} replaced by delta^(l)_n (J v_b)_n.
template <typename T>
void opg_apply(Exec& ex, const Model& m, int64_t N, int64_t B, Prep& p, HvpBufs<T>& h, const T* V, int64_t ldv,
               T* GV) {
  const int L = m.L;
  for (int l = 2; l <= L; ++l) {
    const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
    LAUNCH(k_pack_vbar<T>, B * Tl * (Tin + 1), V, B, ldv, m.offW[l - 2], m.offb[l - 2], Tl, Tin, h.Vbar[l]);
  }
  const T invN = (T)(1.0 / (double)N);
  for (int64_t n0 = 0; n0 < N; n0 += h.Nc) {
    const int64_t Nc = std::min(h.Nc, N - n0);
    const T beta_acc = n0 == 0 ? T(0) : T(1);
    for (int l = 2; l <= L; ++l) {
      const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
      gemm_rm<T>(ex, false, true, Nc, B * Tl, Tin + 1, T(1), h.abar[l - 1] + n0 * p.lda[l - 1], p.lda[l - 1],
                 h.Vbar[l], Tin + 1, T(0), h.RZ[l], B * Tl);
    }
    LAUNCH(k_jv<T>, Nc * B, h.RZ[2], h.RZ[3 <= L ? 3 : 2], h.RZ[4 <= L ? 4 : 2], h.delta[2] + n0 * m.T[1],
           L >= 3 ? h.delta[3] + n0 * m.T[2] : nullptr, L >= 4 ? h.delta[4] + n0 * m.T[3] : nullptr,
           m.T[1], L >= 3 ? m.T[2] : 0, L >= 4 ? m.T[3] : 0, Nc, B, h.S);
    for (int l = 5; l <= L; ++l)
      LAUNCH(k_jv_add<T>, Nc * B, h.RZ[l], h.delta[l] + n0 * m.T[l - 1], m.T[l - 1], Nc, B, h.S);
    for (int l = 2; l <= L; ++l) {
      const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
      LAUNCH(k_dscale<T>, Nc * B * Tl, h.delta[l] + n0 * Tl, h.S, Nc, B, Tl, h.RD[l]);
      gemm_rm<T>(ex, true, false, B * Tl, Tin + 1, Nc, invN, h.RD[l], B * Tl, h.abar[l - 1] + n0 * p.lda[l - 1],
                 p.lda[l - 1], beta_acc, h.HVbar[l], Tin + 1);
    }
  }
  for (int l = 2; l <= L; ++l) {
    const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
    LAUNCH(k_unpack_hv<T>, B * Tl * (Tin + 1), h.HVbar[l], B, ldv, m.offW[l - 2], m.offb[l - 2], Tl, Tin, GV);
  }
}

template <typename T>
void jv_apply(Exec& ex, const Model& m, int64_t N, int64_t B, Prep& p, HvpBufs<T>& h, const T* V, int64_t ldv,
              T* JV) {
  const int L = m.L;
  for (int l = 2; l <= L; ++l) {
    const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
    LAUNCH(k_pack_vbar<T>, B * Tl * (Tin + 1), V, B, ldv, m.offW[l - 2], m.offb[l - 2], Tl, Tin, h.Vbar[l]);
  }
  for (int64_t n0 = 0; n0 < N; n0 += h.Nc) {
    const int64_t Nc = std::min(h.Nc, N - n0);
    for (int l = 2; l <= L; ++l) {
      const int64_t Tl = m.T[l - 1], Tin = m.T[l - 2];
      gemm_rm<T>(ex, false, true, Nc, B * Tl, Tin + 1, T(1), h.abar[l - 1] + n0 * p.lda[l - 1], p.lda[l - 1],
                 h.Vbar[l], Tin + 1, T(0), h.RZ[l], B * Tl);
    }
    T* out = JV + n0 * B;
    LAUNCH(k_jv<T>, Nc * B, h.RZ[2], h.RZ[3 <= L ? 3 : 2], h.RZ[4 <= L ? 4 : 2], h.delta[2] + n0 * m.T[1],
           L >= 3 ? h.delta[3] + n0 * m.T[2] : nullptr, L >= 4 ? h.delta[4] + n0 * m.T[3] : nullptr,
           m.T[1], L >= 3 ? m.T[2] : 0, L >= 4 ? m.T[3] : 0, Nc, B, out);
    for (int l = 5; l <= L; ++l)
      LAUNCH(k_jv_add<T>, Nc * B, h.RZ[l], h.delta[l] + n0 * m.T[l - 1], m.T[l - 1], Nc, B, out);
  }
}

template void jv_apply<double>(Exec&, const Model&, int64_t, int64_t, Prep&, HvpBufs<double>&, const double*,
                               int64_t, double*);
template size_t plan_hvp<float>(Arena&, const Model&, int64_t, int64_t, Prep&, HvpBufs<float>&, bool);
template size_t plan_hvp<double>(Arena&, const Model&, int64_t, int64_t, Prep&, HvpBufs<double>&, bool);
template void hvp_setup<float>(Exec&, const Model&, int64_t, Prep&, HvpBufs<float>&);
template void hvp_setup<double>(Exec&, const Model&, int64_t, Prep&, HvpBufs<double>&);
template void hvp_apply<float>(Exec&, const Model&, int64_t, int64_t, Prep&, HvpBufs<float>&, const float*,
                               int64_t, float*);
template void hvp_apply<double>(Exec&, const Model&, int64_t, int64_t, Prep&, HvpBufs<double>&, const double*,
                                int64_t, double*);
template void opg_apply<float>(Exec&, const Model&, int64_t, int64_t, Prep&, HvpBufs<float>&, const float*,
                               int64_t, float*);
template void opg_apply<double>(Exec&, const Model&, int64_t, int64_t, Prep&, HvpBufs<double>&, const double*,
                                int64_t, double*);

namespace {

// ---- exact H columns through basis-direction HVPs ----
constexpr int64_t EXC_B = 512;  // columns per block

template <typename T>
__global__ void k_basis(T* V, int64_t B, int64_t P, int64_t c0) {
  GRID_STRIDE(i, B * P) { V[i] = (i % P == c0 + i / P) ? T(1) : T(0); }
}

// out[p * ldo + b] = HV[b * P + p] for b < B, p < P (32 x 32 tiles through LDS)
template <typename T>
__global__ void k_cols_from_rows(const T* HV, int64_t B, int64_t P, T* out, int64_t ldo) {
  __shared__ T tile[32][33];
  const int64_t p0 = (int64_t)blockIdx.x * 32, b0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int64_t b = b0 + y, p = p0 + tx;
    if (b < B && p < P) tile[y][tx] = HV[b * P + p];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t p = p0 + y, b = b0 + tx;
    if (b < B && p < P) out[p * ldo + b] = tile[tx][y];
  }
}

template <typename T>
size_t plan_exact_cols(Arena& ar, const Model& m, int64_t N, int64_t ncols, Prep& p, HvpBufs<T>& h, T*& V, T*& HV,
                       bool split) {
  const int64_t B = std::min(ncols, EXC_B);
  plan_hvp<T>(ar, m, N, B, p, h, split);
  V = ar.take<T>(B * m.P);
  HV = ar.take<T>(B * m.P);
  return ar.used;
}

template <typename T>
void run_exact_cols(Exec& ex, const Model& m, int64_t N, Prep& p, HvpBufs<T>& h, T* V, T* HV, int64_t col0,
                    int64_t ncols, T* out) {
  hvp_setup<T>(ex, m, N, p, h);
  for (int64_t cb = 0; cb < ncols; cb += EXC_B) {
    const int64_t B = std::min(EXC_B, ncols - cb);
    LAUNCH(k_basis<T>, B * m.P, V, B, m.P, col0 + cb);
    hvp_apply<T>(ex, m, N, B, p, h, V, m.P, HV);
    if (!launch_ok(ex)) return;
    hipLaunchKernelGGL(k_cols_from_rows<T>, dim3((unsigned)((m.P + 31) / 32), (unsigned)((B + 31) / 32)), dim3(256), 0,
                       ex.stream, HV, B, m.P, out + cb, ncols);
  }
}

size_t ws_exact_cols(const Model& m, int64_t N, int prec, int64_t ncols) {
  Arena ar(nullptr);
  Prep p;
  if (prec == HESS_P_F64) {
    HvpBufs<double> h;
    double *V, *HV;
    return plan_exact_cols<double>(ar, m, N, ncols, p, h, V, HV, false);
  }
  HvpBufs<float> h;
  float *V, *HV;
  return plan_exact_cols<float>(ar, m, N, ncols, p, h, V, HV, prec == HESS_P_F32_SPLIT);
}

size_t ws_hvp(const Model& m, int64_t N, int prec, int64_t B) {
  Arena ar(nullptr);
  Prep p;
  if (prec == HESS_P_F64) {
    HvpBufs<double> h;
    return plan_hvp<double>(ar, m, N, B, p, h);
  }
  HvpBufs<float> h;
  return plan_hvp<float>(ar, m, N, B, p, h, prec == HESS_P_F32_SPLIT);
}

}  // namespace

hess_status exact_cols_workspace(hess_ctx* ctx, const Model& m, int64_t N, int prec, int64_t ncols, size_t* bytes) {
  if (prec != HESS_P_F64 && prec != HESS_P_F32 && prec != HESS_P_F32_SPLIT)
    return fail(ctx, HESS_E_UNSUPPORTED, "H columns: F64, F32 or F32_SPLIT only");
  if (ncols < 1) return fail(ctx, HESS_E_SHAPE, "ncols must be positive");
  *bytes = ws_exact_cols(m, N, prec, ncols);
  return HESS_OK;
}

hess_status hvp_workspace(hess_ctx* ctx, const Model& m, int64_t N, int prec, int64_t B, size_t* bytes) {
  if (prec != HESS_P_F64 && prec != HESS_P_F32 && prec != HESS_P_F32_SPLIT)
    return fail(ctx, HESS_E_UNSUPPORTED, "HVP: F64, F32 or F32_SPLIT only");
  if (B < 1 || B > 65535) return fail(ctx, HESS_E_SHAPE, "B out of range (1..65535)");
  *bytes = ws_hvp(m, N, prec, B);
  return HESS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" hess_status hess_hvp(hess_ctx* ctx, const hess_mlp* mlp, const hess_data* d, int prec, int64_t B,
                                const void* V, void* HV, void* ws, size_t ws_bytes) {
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  Model m;
  if ((s = validate_mlp(ctx, mlp, m, true)) != HESS_OK) return s;
  if ((s = validate_data(ctx, d, true)) != HESS_OK) return s;
  if (prec != HESS_P_F64 && prec != HESS_P_F32 && prec != HESS_P_F32_SPLIT)
    return fail(ctx, HESS_E_UNSUPPORTED, "HVP: F64, F32 or F32_SPLIT only");
  if (B < 1 || B > 65535) return fail(ctx, HESS_E_SHAPE, "B out of range (1..65535)");
  if (!V || !HV) return fail(ctx, HESS_E_ARG, "V or HV is NULL");
  ex.split = prec == HESS_P_F32_SPLIT;
  const size_t need = ws_hvp(m, d->N, prec, B);
  if ((s = check_ws(ctx, need, ws, ws_bytes, (size_t)B * m.P * (prec == HESS_P_F64 ? 16 : 8))) != HESS_OK)
    return s;
  Arena ar(ws);
  Prep p;
  if (prec == HESS_P_F64) {
    HvpBufs<double> h;
    plan_hvp<double>(ar, m, d->N, B, p, h);
    if ((s = check_inputs(ex, m, d, p)) != HESS_OK) return s;
    run_prep(ex, m, d, p, false);
    hvp_setup<double>(ex, m, d->N, p, h);
    hvp_apply<double>(ex, m, d->N, B, p, h, static_cast<const double*>(V), m.P, static_cast<double*>(HV));
  } else {
    HvpBufs<float> h;
    plan_hvp<float>(ar, m, d->N, B, p, h, prec == HESS_P_F32_SPLIT);
    if ((s = check_inputs(ex, m, d, p)) != HESS_OK) return s;
    run_prep(ex, m, d, p, false);
    hvp_setup<float>(ex, m, d->N, p, h);
    hvp_apply<float>(ex, m, d->N, B, p, h, static_cast<const float*>(V), m.P, static_cast<float*>(HV));
  }
  return finish(ex, "hess_hvp");
}

extern "C" hess_status hess_exact_cols(hess_ctx* ctx, const hess_mlp* mlp, const hess_data* d, int prec, int64_t col0,
                                       int64_t ncols, void* Hcols, void* ws, size_t ws_bytes) {
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  Model m;
  if ((s = validate_mlp(ctx, mlp, m, true)) != HESS_OK) return s;
  if ((s = validate_data(ctx, d, true)) != HESS_OK) return s;
  if (prec != HESS_P_F64 && prec != HESS_P_F32 && prec != HESS_P_F32_SPLIT)
    return fail(ctx, HESS_E_UNSUPPORTED, "H columns: F64, F32 or F32_SPLIT only");
  if (ncols < 1 || col0 < 0 || col0 > m.P - ncols) return fail(ctx, HESS_E_SHAPE, "column range outside [0, P)");
  if (!Hcols) return fail(ctx, HESS_E_ARG, "Hcols is NULL");
  ex.split = prec == HESS_P_F32_SPLIT;
  const size_t need = ws_exact_cols(m, d->N, prec, ncols);
  if ((s = check_ws(ctx, need, ws, ws_bytes, (size_t)ncols * m.P * (prec == HESS_P_F64 ? 8 : 4))) != HESS_OK)
    return s;
  Arena ar(ws);
  Prep p;
  if (prec == HESS_P_F64) {
    HvpBufs<double> h;
    double *V, *HV;
    plan_exact_cols<double>(ar, m, d->N, ncols, p, h, V, HV, false);
    if ((s = check_inputs(ex, m, d, p)) != HESS_OK) return s;
    run_prep(ex, m, d, p, false);
    run_exact_cols<double>(ex, m, d->N, p, h, V, HV, col0, ncols, static_cast<double*>(Hcols));
  } else {
    HvpBufs<float> h;
    float *V, *HV;
    plan_exact_cols<float>(ar, m, d->N, ncols, p, h, V, HV, prec == HESS_P_F32_SPLIT);
    if ((s = check_inputs(ex, m, d, p)) != HESS_OK) return s;
    run_prep(ex, m, d, p, false);
    run_exact_cols<float>(ex, m, d->N, p, h, V, HV, col0, ncols, static_cast<float*>(Hcols));
  }
  return finish(ex, "hess_exact_cols");
}

struct hess_hvp_op {
  Model m;
  int64_t N = 0, maxB = 0;
  int prec = HESS_P_F32;
  Prep p;
  HvpBufs<float> hf;
  HvpBufs<double> hd;
};

extern "C" hess_status hess_hvp_prepare(hess_ctx* ctx, const hess_mlp* mlp, const hess_data* d, int prec,
                                        int64_t max_B, void* ws, size_t ws_bytes, hess_hvp_op** op) {
  if (!op) return fail(ctx, HESS_E_ARG, "op is NULL");
  *op = nullptr;
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  Model m;
  if ((s = validate_mlp(ctx, mlp, m, true)) != HESS_OK) return s;
  if ((s = validate_data(ctx, d, true)) != HESS_OK) return s;
  if (prec != HESS_P_F64 && prec != HESS_P_F32 && prec != HESS_P_F32_SPLIT)
    return fail(ctx, HESS_E_UNSUPPORTED, "HVP: F64, F32 or F32_SPLIT only");
  if (max_B < 1 || max_B > 65535) return fail(ctx, HESS_E_SHAPE, "max_B out of range (1..65535)");
  ex.split = prec == HESS_P_F32_SPLIT;
  const size_t need = ws_hvp(m, d->N, prec, max_B);
  if ((s = check_ws(ctx, need, ws, ws_bytes, 0)) != HESS_OK) return s;
  hess_hvp_op* o = new hess_hvp_op();
  o->m = m;
  o->N = d->N;
  o->maxB = max_B;
  o->prec = prec;
  Arena ar(ws);
  if (prec == HESS_P_F64) {
    plan_hvp<double>(ar, o->m, d->N, max_B, o->p, o->hd);
  } else {
    plan_hvp<float>(ar, o->m, d->N, max_B, o->p, o->hf, prec == HESS_P_F32_SPLIT);
  }
  if ((s = check_inputs(ex, o->m, d, o->p)) != HESS_OK) {
    delete o;
    return s;
  }
  run_prep(ex, o->m, d, o->p, false);
  if (prec == HESS_P_F64)
    hvp_setup<double>(ex, o->m, d->N, o->p, o->hd);
  else
    hvp_setup<float>(ex, o->m, d->N, o->p, o->hf);
  s = finish(ex, "hess_hvp_prepare");
  if (s != HESS_OK) {
    delete o;
    return s;
  }
  *op = o;
  return HESS_OK;
}

extern "C" hess_status hess_hvp_apply(hess_ctx* ctx, hess_hvp_op* op, int64_t B, const void* V, void* HV) {
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  if (!op) return fail(ctx, HESS_E_ARG, "op is NULL");
  if (B < 1 || B > op->maxB) return fail(ctx, HESS_E_SHAPE, "B outside 1..max_B");
  if (!V || !HV) return fail(ctx, HESS_E_ARG, "V or HV is NULL");
  ex.split = op->prec == HESS_P_F32_SPLIT;
  if (op->prec == HESS_P_F64)
    hvp_apply<double>(ex, op->m, op->N, B, op->p, op->hd, static_cast<const double*>(V), op->m.P,
                      static_cast<double*>(HV));
  else
    hvp_apply<float>(ex, op->m, op->N, B, op->p, op->hf, static_cast<const float*>(V), op->m.P,
                     static_cast<float*>(HV));
  return finish(ex, "hess_hvp_apply");
}

extern "C" hess_status hess_hvp_release(hess_hvp_op* op) {
  delete op;
  return HESS_OK;
}
