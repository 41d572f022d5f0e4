// Khatri-Rao Gram contraction: the P x P tiles of the OPG and of the exact Hessian.
//
// Both matrices are sums over the N examples of products of per-example factors
// that are indexed by (unit, input) pairs of two layers.  For a row parameter
// (layer l, unit i', input j') and a column parameter (layer m, unit i, input j):
//
//   OPG:  (1/N) sum_n  delta^(l)_{n,i'} abar^(l-1)_{n,j'}  delta^(m)_{n,i} abar^(m-1)_{n,j}
//   H:    (1/N) sum_n  G^(l,m)_n[i',i] abar^(l-1)_{n,j'} abar^(m-1)_{n,j}  (+ cross-layer term)
//
// (abar = activations with a trailing 1 for the bias.)  The per-example gradient
// matrix J of the OPG definition is never stored: its tiles are formed in LDS
// from delta and abar (RANK1 mode).  For H the per-example unit-pair weights
// G_n[i',i] come from the R-operator propagation of unit directions and are
// applied to the B fragments in registers (PAIR modes).
//
// Tile: 128 x 128 outputs per workgroup of 4 wavefronts (2 x 2), each wavefront
// 64 x 64 = 4 x 4 MFMA blocks of 16 x 16.  Units are padded to a multiple of 16
// slots in compute space so every MFMA block lies inside one (row unit, column
// unit) pair.  K (the example index) is staged through LDS in chunks of KC with the
// k-permutation of the generic GEMM (lane group q takes 4 consecutive k per 16),
// with STAGES LDS buffers: with two, the next chunk is written while the current
// one is read and one barrier per chunk suffices.  Symmetric blocks enumerate only
// the lower triangle of tiles and mirror every stored entry, so the result is
// exactly symmetric.
#include <algorithm>
#include <string>
#include <type_traits>
#include <vector>

#include "mfma.h"

namespace hs {

namespace {

constexpr int BM = 128, BN = 128;
constexpr int MAXU = BM / 16 + 1;  // units a tile can touch (pad >= 16)

__device__ __forceinline__ int64_t flat_index(int32_t perm, int64_t off, int32_t Tin, int32_t Tout,
                                              int64_t u, int64_t s) {
  const int64_t i = perm ? s : u, j = perm ? u : s;
  return j < Tin ? off + i * Tin + j : off + (int64_t)Tout * Tin + i;
}

template <int64_t G = 16>
__device__ __forceinline__ void tile_of(int64_t t, bool symmetric, int64_t tiles_c, int64_t tiles_r, int64_t& tr,
                                        int64_t& tc) {
  if (symmetric)
    grouped_lower_tile<G>(t, tiles_r, tr, tc);
  else
    grouped_full_tile<G>(t, tiles_c, tiles_r, tr, tc);
}

template <typename TOut>
__device__ __forceinline__ void store_out(TOut* out, int64_t idx, double v, int32_t accumulate) {
  if (accumulate)
    out[idx] = (TOut)((double)out[idx] + v);
  else
    out[idx] = (TOut)v;
}

template <typename T, int WMODE, int KC, int STAGES>
struct KrgSmem {
  static constexpr int KP = KC + 4;
  static constexpr int WSZ = (WMODE == KRG_RANK1) ? 4 : MAXU * MAXU * KC;
  static constexpr int A = 0, B = STAGES * BM * KP, W = B + STAGES * BN * KP;
  static constexpr int SIZE = W + STAGES * WSZ;
};

// One 128 x 128 output tile t of the contraction described by `a` (smem: KrgSmem::SIZE elements).
template <typename T, typename TOut, int WMODE, bool SYM, int KC, int STAGES>
__device__ __forceinline__ void krg_tile(const KrgArgs<T, TOut>& a, int64_t t, int64_t tiles_c, T* smem) {
  using Op = MfmaOp<T>;
  using acc_t = typename Op::acc_t;
  using SM = KrgSmem<T, WMODE, KC, STAGES>;
  constexpr int KP = SM::KP;
  constexpr int WSZ = SM::WSZ;
  T* As_ = smem + SM::A;
  T* Bs_ = smem + SM::B;
  T* Ws_ = smem + SM::W;
  auto As = [&](int s) { return As_ + s * BM * KP; };
  auto Bs = [&](int s) { return Bs_ + s * BN * KP; };
  auto Ws = [&](int s) { return Ws_ + s * WSZ; };

  int64_t tr, tc;
  const int64_t tiles_r = ((int64_t)a.r.n_units * a.r.pad + BM - 1) / BM;
  tile_of(t, SYM, tiles_c, tiles_r, tr, tc);
  const int64_t r0 = tr * BM, c0 = tc * BN;
  const int64_t ur_lo = r0 / a.r.pad, uc_lo = c0 / a.c.pad;
  const int64_t ur_hi = min((int64_t)a.r.n_units - 1, (r0 + BM - 1) / a.r.pad);
  const int64_t uc_hi = min((int64_t)a.c.n_units - 1, (c0 + BN - 1) / a.c.pad);
  if (WMODE == KRG_PAIR_DIAG && (ur_hi < uc_lo || uc_hi < ur_lo)) return;
  const int nur = (int)(ur_hi - ur_lo + 1), nuc = (int)(uc_hi - uc_lo + 1);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // Staging assignment: thread -> one row (column) of the tile and KC/2 consecutive k.
  constexpr int SK = KC / 2;
  const int srow = tid & 127, sk0 = (tid >> 7) * SK;
  const int64_t gr = r0 + srow, gc = c0 + srow;
  const int64_t sur = gr / a.r.pad, ssr = gr % a.r.pad;
  const int64_t suc = gc / a.c.pad, ssc = gc % a.c.pad;
  const bool rvalid = sur < a.r.n_units && ssr < a.r.len;
  const bool cvalid = suc < a.c.n_units && ssc < a.c.len;
  const T* rsrc = a.r.src + ssr;
  const T* csrc = a.c.src + ssc;
  T ra[SK], rbv[SK];
  constexpr int WE = (WMODE == KRG_RANK1) ? 1 : (WSZ + 255) / 256;
  T rw[WE];
  const int nw = nur * nuc * KC;

  auto load = [&](int64_t n0) {
#pragma unroll
    for (int i = 0; i < SK; ++i) {
      const int64_t n = n0 + sk0 + i;
      T va = T(0), vb = T(0);
      if (n < a.N) {
        if (rvalid) {
          va = rsrc[n * a.r.ld];
          if (WMODE == KRG_RANK1 && a.r.scale) va *= a.r.scale[n * a.r.ld_scale + sur];
        }
        if (cvalid) {
          vb = csrc[n * a.c.ld];
          if (WMODE == KRG_RANK1 && a.c.scale) vb *= a.c.scale[n * a.c.ld_scale + suc];
        }
      }
      ra[i] = va;
      rbv[i] = vb;
    }
    if (WMODE != KRG_RANK1) {
#pragma unroll
      for (int i = 0; i < WE; ++i) {
        const int e = tid + i * 256;
        T w = T(0);
        if (e < nw) {
          const int kk = e % KC, p = e / KC;
          const int64_t ur = ur_lo + p / nuc, uc = uc_lo + p % nuc;
          const int64_t n = n0 + kk;
          if (n < a.N) {
            if (WMODE == KRG_PAIR_FULL)
              w = a.wts[(ur * a.c.n_units + uc) * a.ldw + n];
            else if (ur == uc)
              w = a.wts[ur * a.ldw + n];
          }
        }
        rw[i] = w;
      }
    }
  };
  auto store = [&](int s) {
#pragma unroll
    for (int i = 0; i < SK; ++i) {
      As(s)[srow * KP + sk0 + i] = ra[i];
      Bs(s)[srow * KP + sk0 + i] = rbv[i];
    }
    if (WMODE != KRG_RANK1) {
#pragma unroll
      for (int i = 0; i < WE; ++i) {
        const int e = tid + i * 256;
        if (e < nw) {
          const int kk = e % KC, p = e / KC;
          Ws(s)[((p / nuc) * MAXU + (p % nuc)) * KC + kk] = rw[i];
        }
      }
    }
  };

  // Unit pair of every MFMA block of this wavefront (wave-uniform).
  int pu[4], pc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    pu[i] = (int)((r0 + wr * 64 + i * 16) / a.r.pad - ur_lo);
    pc[i] = (int)((c0 + wc * 64 + i * 16) / a.c.pad - uc_lo);
  }

  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = Op::zero();

  const int row = lane & 15, q = lane >> 4;
  // All four column blocks of this wavefront in one column unit (the common case when
  // units are wider than 64 slots): the pair weight then depends on the row block only
  // and is applied once to each A fragment instead of once per MFMA block.
  const bool one_cunit = pc[0] == pc[3];
  auto compute = [&](int s) {
#pragma unroll
    for (int ks = 0; ks < KC / 16; ++ks) {
      const int ko = ks * 16 + 4 * q;
      T av[4][4], bv[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) av[i][u] = As(s)[(wr * 64 + i * 16 + row) * KP + ko + u];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int u = 0; u < 4; ++u) bv[j][u] = Bs(s)[(wc * 64 + j * 16 + row) * KP + ko + u];
      if (WMODE == KRG_RANK1) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = Op::mma(av[i][u], bv[j][u], acc[i][j]);
      } else if (one_cunit) {
        T w[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool live = WMODE != KRG_PAIR_DIAG || (pu[i] + ur_lo) == (pc[0] + uc_lo);
          const T* wp = &Ws(s)[(pu[i] * MAXU + pc[0]) * KC + ko];
#pragma unroll
          for (int u = 0; u < 4; ++u) w[i][u] = live ? wp[u] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const T aw = av[i][u] * w[i][u];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = Op::mma(aw, bv[j][u], acc[i][j]);
          }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (WMODE == KRG_PAIR_DIAG && (pu[i] + ur_lo) != (pc[j] + uc_lo)) continue;
            const T* wp = &Ws(s)[(pu[i] * MAXU + pc[j]) * KC + ko];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[i][j] = Op::mma(av[i][u], bv[j][u] * wp[u], acc[i][j]);
          }
      }
    }
  };

  const int64_t nk = (a.N + KC - 1) / KC;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t kc = 0; kc < nk; ++kc) {
    const bool more = kc + 1 < nk;
    if (more) load((kc + 1) * KC);
    if (STAGES == 2) {
      compute((int)(kc & 1));
      if (more) store((int)((kc + 1) & 1));
      __syncthreads();
    } else {
      compute(0);
      __syncthreads();
      if (more) {
        store(0);
        __syncthreads();
      }
    }
  }

  // Epilogue: scale by 1/N, map compute indices to flat parameter indices.
  int64_t fcol[4];
  bool cok[4];
  int64_t ccomp[4];
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
      const int64_t r = r0 + wr * 64 + i * 16 + Op::row_of(q, v);
      const int64_t ur = r / a.r.pad, sr = r % a.r.pad;
      if (!(ur < a.r.n_units && sr < a.r.len)) continue;
      const int64_t fr = flat_index(a.r.perm, a.r.off, a.r.Tin, a.r.Tout, ur, sr);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!cok[j]) continue;
        if (SYM && r < ccomp[j]) continue;
        const double val = a.scale * (double)acc[i][j][v];
        store_out<TOut>(a.out, fr * a.ldo + fcol[j], val, a.accumulate);
        if (a.mirror && !(SYM && r == ccomp[j])) store_out<TOut>(a.out, fcol[j] * a.ldo + fr, val, a.accumulate);
      }
    }
}

// ---------------------------------------------------------------------------
// FP32 tile with direct HBM -> LDS staging (buffer_load ... lds).
//
// The operands never pass through registers on their way to LDS: every chunk of
// KC examples is copied by the vector memory unit straight into one of NST LDS
// stages (the copies of chunk c + NST - 1 are issued right after the barrier that
// opens chunk c), so the K loop issues only the copies, the LDS operand reads, the
// pair weight products and the MFMAs.  Example ranges can be split into slices that
// run in the same launch and write separate partial results.  A stage holds A and B k-major (As[k][r], row
// stride DLD floats; DLD = 132 puts the four lane groups of a 16x16x4 MFMA step,
// which read k = 16 g + 4q + s, on disjoint LDS banks) and the per-chunk pair weights
// (PAIR_FULL: [row unit][column unit][k], PAIR_DIAG: [unit][k], RANK1: the row
// and column scale factors [unit][k]).  Each lane copies one float: its address
// clamps the slot to the unit's valid range (so every read stays inside the
// source row), and the buffer range check (num_records = the chunk's valid
// examples) turns examples past N into zeros.  Weights read past N are replaced
// by zeros in registers.  Units beyond a side's last unit are clamped: they only
// feed outputs that the epilogue discards.
//
// Wavefront tile 64 x 64 = 4 x 4 MFMA blocks.  When the wavefront's 64 columns lie
// in one column unit (the common case for wide units) the pair weight depends on
// the row only: A is read interleaved (block i holds rows 4 * row16 + i, so one
// 128-bit read gives all four blocks) and the weight is applied to A.  Otherwise A
// blocks are 16 consecutive rows (one row unit each) and the weight, which then
// depends on the block's row unit and the lane's column unit, is applied to B.
// B is always read interleaved (lane columns 4 * col16 + j, one column unit).
// ---------------------------------------------------------------------------
constexpr int DLD = 132;

// chunk of examples per stage and number of LDS stages (prefetch distance NST - 1);
// SPLIT: FP32 products from BF16 MFMAs on three-way split operands (chunks of 32);
// BPS: the column operand arrives already split (bsplit layout) and is copied into LDS
// as BF16 parts in MFMA operand order; A rows are unpadded (128-bit reads of 16 lanes
// cover 256 contiguous bytes) and the pair weights go to registers, so that two
// workgroups (2 x 80 KB) share a CU
// LIST: the tile sums over an example list (its unit pair's, its row tile's or its column
// tile's; see KrgArgs): rows of both sources and the pair weights are gathered by example index
template <int KC_, int NST_, bool SPLIT_ = false, bool BPS_ = false, bool LIST_ = false>
struct DmaCfg {
  static constexpr int KC = KC_, NST = NST_;
  static constexpr bool SPLIT = SPLIT_, BPS = BPS_, LIST = LIST_;
  static_assert(!BPS || (SPLIT && KC == 32), "pre-split columns need split products on chunks of 32");
  static_assert(!LIST || (SPLIT && !BPS && KC == 32 && NST == 2), "example lists: split products in the tile");
};
// Row panels per tile group of the example-list tile (grouped lower-triangle order): tiles of
// one unit pair share a list, and long groups keep more of the gathered rows in L2; measured
// on the MNIST-shaped block (625 row panels): 16 -> 807 ms, 32 -> 762, 48 -> 714, 64 -> 750,
// 100 -> 701, 128 -> 693-700, 200 -> 707, 320 -> 760, 640 -> 834
constexpr int64_t KRG_LIST_GROUP = 128;
using DmaDefault = DmaCfg<16, 2>;  // measured: (16, 2) 131, (16, 3) 129, (32, 2) 126 TFLOP/s

template <int WMODE, int MAXU, class C = DmaDefault>
struct DmaSmem {
  static constexpr int DKC = C::KC;
  // row strides (floats) of A and B: unpadded where every read is a 128-bit read of 16 lanes
  // on 256 contiguous bytes (pre-split columns, example lists), DLD otherwise
  static constexpr int ALD = (C::BPS || C::LIST) ? 128 : DLD;
  static constexpr int BLD = C::LIST ? 128 : DLD;
  static constexpr int AB = DKC * ALD;
  static constexpr int WN1 = WMODE == KRG_PAIR_FULL ? MAXU * MAXU * DKC : MAXU * DKC;  // floats per weight array
  static constexpr int NW = WMODE == KRG_RANK1 ? 2 : 1;                              // weight arrays
  static constexpr int WI1 = (WN1 + 63) / 64;                                         // copies per array
  static constexpr int WI = NW * WI1;
  // B: FP32 like A, or (BPS) the three BF16 parts of the tile's 128 columns as 24
  // fragments of 64 lanes x 16 bytes, fragment ((wc * 4 + j) * 3 + part)
  static constexpr int BSZ = C::BPS ? 24 * 256 : AB;
  static constexpr int WOFF = AB + BSZ;  // weights after A and B (none for BPS)
  static constexpr int STAGE = AB + BSZ + (C::BPS ? 0 : NW * WN1);
  static constexpr int SIZE = C::NST * STAGE;
  // copies every wavefront issues per chunk: KC / 2 for A, KC / 2 for B (24 for BPS),
  // and its share of the weight copies (a lower bound when RANK1 scale factors may be absent)
  static constexpr int VMC = DKC / 2 + (C::BPS ? 24 : DKC / 2) + (C::BPS || WMODE == KRG_RANK1 ? 0 : WI / 4);
  static constexpr int WPW = (WI + 3) / 4;  // weight copies one wavefront may issue
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;


__device__ __forceinline__ int64_t mn64(int64_t x, int64_t y) { return x < y ? x : y; }
// A value known to be the same in every lane, moved to scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
}

// Raw buffer over `elems` (>= 0) floats from base; the byte count is capped below 2^31
// (copy offsets are checked on the host to stay below the cap).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* base, int64_t elems) {
  const uint64_t e = (uint64_t)elems;
  const uint32_t nrec = e >= 0x1ffffffcull ? 0x7ffffff0u : (uint32_t)e * 4u;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nrec, 0x00020000);
}

__device__ __forceinline__ void copy_lds(__amdgpu_buffer_rsrc_t r, float* dst, int voff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr_t)dst, 4, voff, 0, 0, 0);
}
// the same with a wavefront-uniform byte offset added by the scalar offset operand
__device__ __forceinline__ void copy_lds_s(__amdgpu_buffer_rsrc_t r, float* dst, int voff, int soff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr_t)dst, 4, voff, soff, 0, 0);
}

// s_waitcnt vmcnt(N) with expcnt and lgkmcnt left free (gfx9 encoding: vmcnt bits 3:0 and 15:14)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0f70);
}

template <int WMODE, bool SYM, int MAXU, class C = DmaDefault>
__device__ __forceinline__ void krg_tile_dma(const KrgArgs<float, float>& a, int64_t t, int64_t tiles_c,
                                             float* smem) {
  using SM = DmaSmem<WMODE, MAXU, C>;
  constexpr int DKC = C::KC, DST = C::NST, KH = DKC / 2;
  int64_t tr, tc;
  const int64_t tiles_r = ((int64_t)a.r.n_units * a.r.pad + BM - 1) / BM;
  tile_of<C::LIST ? KRG_LIST_GROUP : 16>(t, SYM, tiles_c, tiles_r, tr, tc);
  const int64_t r0 = tr * BM, c0 = tc * BN;
  const int ur_lo = (int)(r0 / a.r.pad), uc_lo = (int)(c0 / a.c.pad);
  const int ur_hi = (int)min((int64_t)a.r.n_units - 1, (r0 + BM - 1) / a.r.pad);
  const int uc_hi = (int)min((int64_t)a.c.n_units - 1, (c0 + BN - 1) / a.c.pad);
  if (WMODE == KRG_PAIR_DIAG && (ur_hi < uc_lo || uc_hi < ur_lo)) return;
  // examples summed by this tile: all N, or (LIST) its unit pair's list when its rows and its
  // columns each lie in one unit (symmetric), else the shorter of its row tile's (symmetric)
  // and column tile's lists
  int64_t NE = a.N;
  const int32_t* klist = nullptr;
  if constexpr (C::LIST) {
    if (SYM && a.plist && ur_lo == ur_hi && uc_lo == uc_hi) {  // one unit pair: its own list
      const int64_t pi = (int64_t)ur_lo * (ur_lo + 1) / 2 + uc_lo;
      klist = a.plist + pi * a.ldl;
      NE = a.pcnt[pi];
    } else if (SYM && a.rlist && a.rcnt[tr] < a.kcnt[tc]) {  // the row tile's list is shorter
      klist = a.rlist + tr * a.ldl;
      NE = a.rcnt[tr];
    } else {
      klist = a.klist + tc * a.ldl;
      NE = a.kcnt[tc];
    }
  }

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int row16 = lane & 15, q = lane >> 4;

  // ---- per-lane copy offsets (bytes, relative to the chunk's base pointers) ----
  int voffA[KH], voffB[KH];
#pragma unroll
  for (int m = 0; m < KH; ++m) {
    const int k = (DKC / 4) * wave + (m >> 1);
    const int64_t r = r0 + (m & 1) * 64 + lane, c = c0 + (m & 1) * 64 + lane;
    const int sr = (int)mn64(r % a.r.pad, a.r.len - 1), sc = (int)mn64(c % a.c.pad, a.c.len - 1);
    voffA[m] = (int)(((C::LIST ? 0 : k) * a.r.ld + sr) * 4);  // LIST: the example rides in the scalar offset
    voffB[m] = (int)(((C::LIST ? 0 : k) * a.c.ld + sc) * 4);
  }
  // BPS: byte offsets of the tile's four 32-column groups (column half h, group g) in a
  // pre-split chunk.  With BPS, block j of a wavefront holds its columns 16 j .. 16 j + 15,
  // so blocks 0, 1 lie in group 0 and blocks 2, 3 in group 1; a group never crosses a
  // unit (pad is a multiple of 32).
  int bpo[4] = {0, 0, 0, 0};
  if constexpr (C::BPS) {
    const int64_t vcols = (int64_t)a.c.n_units * a.c.pad;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      int64_t cb = c0 + 32 * x;
      if (cb >= vcols) cb = 0;  // beyond the last unit: any group (outputs discarded)
      bpo[x] = (int)((cb % a.c.pad) / 32 * 512 * 4);
    }
  }
  int voffW[SM::WPW];
  bool wlive[SM::WPW];
#pragma unroll
  for (int x = 0; x < SM::WPW; ++x) {
    const int g = wave + 4 * x;              // copy index over all weight arrays
    const int arr = g / SM::WI1;             // RANK1: 0 = row scales, 1 = column scales
    const int e = (g % SM::WI1) * 64 + lane;  // element within the array
    wlive[x] = g < SM::WI && e < SM::WN1;
    int off = 0;
    if (WMODE == KRG_PAIR_FULL) {
      const int p = e / DKC, k = C::LIST ? 0 : e % DKC;  // LIST: example e % DKC added at the copy
      const int ur = min(ur_lo + p / MAXU, a.r.n_units - 1), uc = min(uc_lo + p % MAXU, a.c.n_units - 1);
      off = (int)((((int64_t)(ur - ur_lo) * a.c.n_units + (uc - uc_lo)) * a.ldw + k) * 4);
    } else if (WMODE == KRG_PAIR_DIAG) {
      const int d = e / DKC, k = e % DKC;
      const int u = min(ur_lo + d, min(a.r.n_units, a.c.n_units) - 1);
      off = (int)(((int64_t)(u - ur_lo) * a.ldw + k) * 4);
    } else {
      const int d = e / DKC, k = e % DKC;
      if (arr == 0) {
        const int u = min(ur_lo + d, a.r.n_units - 1);
        off = (int)((k * a.r.ld_scale + (u - ur_lo)) * 4);
      } else {
        const int u = min(uc_lo + d, a.c.n_units - 1);
        off = (int)((k * a.c.ld_scale + (u - uc_lo)) * 4);
      }
    }
    voffW[x] = off;
  }
  const bool has_sa = WMODE == KRG_RANK1 && a.r.scale != nullptr;
  const bool has_sb = WMODE == KRG_RANK1 && a.c.scale != nullptr;
  int64_t wtot = 0;  // elements of the weight buffer (for the range check)
  if (WMODE == KRG_PAIR_FULL) wtot = ((int64_t)a.r.n_units * a.c.n_units - 1) * a.ldw + a.N;
  if (WMODE == KRG_PAIR_DIAG) wtot = ((int64_t)min(a.r.n_units, a.c.n_units) - 1) * a.ldw + a.N;

  // ---- one chunk's copies into stage st ----
  // LIST: example indices of the chunk being copied, lane l holding entry l % 32
  int ixv = 0;
  auto issue = [&](int st, int64_t n0) {
    float* S = smem + st * SM::STAGE;
    if constexpr (C::LIST) {
      // copy row k of the chunk is example klist[n0 + k]: its row offset in the scalar operand
      // (the buffers span all N rows, every index is below N), the slot in the vector offset;
      // weight lane e takes example e % 32 of the chunk
      static_assert(WMODE == KRG_PAIR_FULL, "example lists are built for pair weights");
      const __amdgpu_buffer_rsrc_t ga = rsrc_of(a.r.src, a.N * a.r.ld), gb = rsrc_of(a.c.src, a.N * a.c.ld);
#pragma unroll
      for (int m = 0; m < KH; ++m) {
        const int k = (DKC / 4) * wave + (m >> 1);
        const int ex = __builtin_amdgcn_readlane(ixv, k);
        copy_lds_s(ga, S + k * SM::ALD + (m & 1) * 64, voffA[m], (int)((int64_t)ex * a.r.ld * 4));
        copy_lds_s(gb, S + SM::AB + k * SM::BLD + (m & 1) * 64, voffB[m], (int)((int64_t)ex * a.c.ld * 4));
      }
      const int64_t base = ((int64_t)ur_lo * a.c.n_units + uc_lo) * a.ldw;
      const __amdgpu_buffer_rsrc_t rw = rsrc_of(a.wts + base, wtot - base);
      float* W = S + SM::WOFF;
#pragma unroll
      for (int x = 0; x < SM::WPW; ++x) {
        const int g = wave + 4 * x;
        if (g < SM::WI && wlive[x]) copy_lds(rw, W + g * 64, voffW[x] + 4 * ixv);
      }
      return;
    }
    const int kv = (int)mn64(DKC, a.N - n0);
    const __amdgpu_buffer_rsrc_t ra = rsrc_of(a.r.src + n0 * a.r.ld, (int64_t)kv * a.r.ld);
    const __amdgpu_buffer_rsrc_t rb = rsrc_of(a.c.src + n0 * a.c.ld, (int64_t)kv * a.c.ld);
    if constexpr (C::BPS) {
      // voffA[m] = voffA[m & 1] + (m / 2) rows of the source: the row part is uniform and
      // rides in the scalar offset.  The buffer range check leaves the scalar offset out,
      // so the rows of a partial chunk past N are read from the source's padding: the row
      // sources of this tile hold whole chunks of 32 examples, zero past N (cast_ops).
#pragma unroll
      for (int m = 0; m < KH; ++m)
        copy_lds_s(ra, S + ((DKC / 4) * wave + (m >> 1)) * SM::ALD + (m & 1) * 64, voffA[m & 1],
                   (int)((m >> 1) * a.r.ld * 4));
    } else {
#pragma unroll
      for (int m = 0; m < KH; ++m) copy_lds(ra, S + ((DKC / 4) * wave + (m >> 1)) * SM::ALD + (m & 1) * 64, voffA[m]);
    }
    if constexpr (C::BPS) {
      // 96 fragment row blocks of 256 bytes (2 halves x 4 j x 3 parts x 4 row blocks), 24 per
      // wavefront, each 256 contiguous bytes of chunk n0 / 32 of the pre-split source
      const int64_t cs = (int64_t)3 * a.bp_nblk * 512;  // dwords per chunk
      const __amdgpu_buffer_rsrc_t rp = rsrc_of(a.bparts + (n0 / DKC) * cs, cs);
#pragma unroll
      for (int x = 0; x < 24; ++x) {  // (half, j, part) fixed per x; wavefront w copies row block w
        const int part = x % 3, j = (x / 3) & 3, h = x / 12, mb = wave;
        copy_lds(rp, S + SM::AB + ((h * 4 + j) * 3 + part) * 256 + mb * 64,
                 bpo[2 * h + (j >> 1)] + 4 * (part * a.bp_nblk * 512 + (j & 1) * 256 + mb * 64 + lane));
      }
    } else {
#pragma unroll
      for (int m = 0; m < KH; ++m)
        copy_lds(rb, S + SM::AB + ((DKC / 4) * wave + (m >> 1)) * SM::BLD + (m & 1) * 64, voffB[m]);
    }
    float* W = S + SM::WOFF;
    if (C::BPS) {
      // pair weights are loaded into registers by the tile (wload)
    } else if (WMODE == KRG_PAIR_FULL || WMODE == KRG_PAIR_DIAG) {
      const int64_t base = (WMODE == KRG_PAIR_FULL ? ((int64_t)ur_lo * a.c.n_units + uc_lo) : (int64_t)ur_lo) * a.ldw + n0;
      const __amdgpu_buffer_rsrc_t rw = rsrc_of(a.wts + base, wtot - base);
#pragma unroll
      for (int x = 0; x < SM::WPW; ++x) {
        const int g = wave + 4 * x;
        if (g < SM::WI && wlive[x]) copy_lds(rw, W + g * 64, voffW[x]);
      }
    } else {
      const __amdgpu_buffer_rsrc_t rsa =
          rsrc_of(has_sa ? a.r.scale + n0 * a.r.ld_scale + ur_lo : a.r.src, has_sa ? (int64_t)kv * a.r.ld_scale - ur_lo : 0);
      const __amdgpu_buffer_rsrc_t rsb =
          rsrc_of(has_sb ? a.c.scale + n0 * a.c.ld_scale + uc_lo : a.c.src, has_sb ? (int64_t)kv * a.c.ld_scale - uc_lo : 0);
#pragma unroll
      for (int x = 0; x < SM::WPW; ++x) {
        const int g = wave + 4 * x;
        if (g >= SM::WI) continue;
        const int arr = g / SM::WI1;
        if ((arr == 0 ? has_sa : has_sb) && wlive[x]) copy_lds(arr == 0 ? rsa : rsb, W + g * 64 - arr * (SM::WI1 * 64 - SM::WN1), voffW[x]);
      }
    }
  };

  // weights of (row unit urel, column unit ucrel) for this lane's k = k0 + 4q .. k0 + 4q + 3
  auto wt4 = [&](const float* W, int urel, int ucrel, int k0, int kv) -> f4_t {
    const int kk = k0 + 4 * q;
    f4_t w;
    if (WMODE == KRG_PAIR_FULL) {
      w = *(const f4_t*)&W[(urel * MAXU + ucrel) * DKC + kk];
    } else if (WMODE == KRG_PAIR_DIAG) {
      w = (ur_lo + urel == uc_lo + ucrel) ? *(const f4_t*)&W[urel * DKC + kk] : f4_t{0.f, 0.f, 0.f, 0.f};
    } else {
      w = f4_t{1.f, 1.f, 1.f, 1.f};
      if (has_sa) w *= *(const f4_t*)&W[urel * DKC + kk];
      if (has_sb) w *= *(const f4_t*)&W[SM::WN1 + ucrel * DKC + kk];
    }
    if (kv < DKC) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (kk + s >= kv) w[s] = 0.f;
    }
    return w;
  };

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  // column unit of this lane's interleaved columns (4 * col16 + j share it)
  const int uc_lane = (int)((c0 + wc * 64 + 4 * row16) / a.c.pad) - uc_lo;
  const bool one_cunit = (c0 + wc * 64) / a.c.pad == (c0 + wc * 64 + 63) / a.c.pad;
  const int ur_lane = (int)((r0 + wr * 64 + 4 * row16) / a.r.pad) - ur_lo;  // rows 4 * row16 + i share it
  int ur_blk[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) ur_blk[i] = (int)((r0 + wr * 64 + 16 * i) / a.r.pad) - ur_lo;

  const int64_t nk = (NE + DKC - 1) / DKC;
  // BPS: this lane's pair weights of examples n0 + 8 q .. n0 + 8 q + 7 for its row unit and
  // column unit u (relative), read straight into registers through one wavefront-uniform
  // buffer that starts at the tile's first unit pair (the lane's pair is in the offset, as
  // for the weight copies); examples past N read as zero
  const int64_t wb0 = ((int64_t)ur_lo * a.c.n_units + uc_lo) * a.ldw;
  auto wload = [&](int64_t n0, int u, float (&w)[8]) {
    const int ur = min(ur_lo + ur_lane, a.r.n_units - 1), uc = min(uc_lo + u, a.c.n_units - 1);
    const int vo = (int)((((int64_t)(ur - ur_lo) * a.c.n_units + (uc - uc_lo)) * a.ldw + 8 * q) * 4);
    const __amdgpu_buffer_rsrc_t rw = rsrc_of(a.wts + wb0 + n0, wtot - wb0 - n0);
#pragma unroll
    for (int s = 0; s < 8; ++s) w[s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rw, vo + 4 * s, 0, 0));
    if (n0 + DKC > a.N) {
#pragma unroll
      for (int s = 0; s < 8; ++s)
        if (n0 + 8 * q + s >= a.N) w[s] = 0.f;
    }
  };
  auto kloop = [&](auto oc) {
    constexpr bool ONE = decltype(oc)::value;
    // BPS: the rows are weighted for one column unit, or for two when the wavefront's
    // columns lie in two units (units ubase and ubase + 1, split at its 32nd column)
    constexpr int NPB = ONE ? 1 : 2;
    const int ubase = ONE ? uc_lane : (int)((c0 + wc * 64) / a.c.pad) - uc_lo;
    float wcur[NPB][8], wnxt[NPB][8];
    if constexpr (C::BPS) {
#pragma unroll
      for (int ps = 0; ps < NPB; ++ps) wload(0, ubase + ps, wnxt[ps]);
    }
    int ixn = 0;  // LIST: indices of the next chunk to copy, loaded a chunk ahead
    if constexpr (C::LIST) {
      if (nk > 0) ixv = klist[lane & 31];
      if (nk > 1) ixn = klist[DKC + (lane & 31)];
    }
#pragma unroll
    for (int c = 0; c < DST - 1; ++c)
      if (c < nk) issue(c, (int64_t)c * DKC);
    for (int64_t kc = 0; kc < nk; ++kc) {
      // wait for this chunk's copies; with three stages the next chunk may stay in flight
      if (DST > 2 && kc + 1 < nk) wait_vm<(DST > 2 ? SM::VMC : 0)>(); else wait_vm<0>();
      // every wavefront's copies of this chunk have landed and its reads of the stage
      // about to be refilled are complete
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
      if constexpr (C::LIST) {
        if (kc + 1 < nk) {
          ixv = ixn;
          issue((int)((kc + 1) % DST), (kc + 1) * DKC);
          if (kc + 2 < nk) ixn = klist[(kc + 2) * DKC + (lane & 31)];
        }
      } else if (kc + DST - 1 < nk) {
        issue((int)((kc + DST - 1) % DST), (kc + DST - 1) * DKC);
      }
      if constexpr (C::BPS) {  // this chunk's weights landed with its copies; fetch the next
#pragma unroll
        for (int ps = 0; ps < NPB; ++ps)
#pragma unroll
          for (int s = 0; s < 8; ++s) wcur[ps][s] = wnxt[ps][s];
        if (kc + 1 < nk) {
#pragma unroll
          for (int ps = 0; ps < NPB; ++ps) wload((kc + 1) * DKC, ubase + ps, wnxt[ps]);
        }
      }
      const int st = (int)(kc % DST);
      const float* As = smem + st * SM::STAGE;
      const float* Bs = As + SM::AB;
      const float* W = As + SM::WOFF;
      const int kv = (int)mn64(DKC, NE - kc * DKC);
      if constexpr (C::BPS) {
        // The columns arrive split: 12 fragment reads (lane = 16 q + row16 holds examples
        // 8 q .. 8 q + 7 of column 16 j + row16).  The rows are weighted and split here,
        // once per column unit: blocks 0, 1 take the weights of group 0's unit and blocks
        // 2, 3 those of group 1's unit (the same unit unless the wavefront straddles two).
        const SplitC sc = split_consts();
        const bf8_t* Bq = reinterpret_cast<const bf8_t*>(Bs);
        bf8_t bh[4], bm[4], bl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bh[j] = Bq[((wc * 4 + j) * 3 + 0) * 64 + lane];
          bm[j] = Bq[((wc * 4 + j) * 3 + 1) * 64 + lane];
          bl[j] = Bq[((wc * 4 + j) * 3 + 2) * 64 + lane];
        }
        float ax[4][8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const f4_t a4 = *(const f4_t*)&As[(8 * q + s) * SM::ALD + wr * 64 + 4 * row16];
#pragma unroll
          for (int i = 0; i < 4; ++i) ax[i][s] = a4[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int ps = 0; ps < NPB; ++ps) {
            float av[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) av[s] = ax[i][s] * wcur[ps][s];
            bf8_t ah, am, al;
            split3x8(av, ah, am, al, sc);
            constexpr int J0 = 0, JN = 4 / NPB;
#pragma unroll
            for (int pr = 0; pr < 6; ++pr)
#pragma unroll
              for (int jj = J0; jj < JN; ++jj) {
                const int j = ps * JN + jj;
                acc[i][j] = mma_bf16(pr_x(pr, ah, am, al), pr_y(pr, bh[j], bm[j], bl[j]), acc[i][j]);
              }
          }
        }
        continue;
      }
      if constexpr (ONE && C::SPLIT) {
        // the chunk's 32 examples at once: this lane supplies k = 8 q + s (s = 0..7) of
        // its four rows (A, weighted) and four columns (B); each value is split in three
        // BF16 parts and the products h h, h m, m h, h l, l h, m m of A and B parts are
        // accumulated in FP32 by v_mfma_f32_16x16x32_bf16 (same output layout as the
        // FP32 instruction).  The dropped m l, l m, l l terms are below 2^-32 relative.
        static_assert(DKC == 32, "split products take chunks of 32 examples");
        const SplitC sc = split_consts();
        const f4_t wlo = wt4(W, ur_lane, uc_lane, 4 * q, kv), whi = wt4(W, ur_lane, uc_lane, 4 * q + 4, kv);
        float av[4][8], bv[4][8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = 8 * q + s;
          const float ws = s < 4 ? wlo[s] : whi[s - 4];
          const f4_t a4 = *(const f4_t*)&As[k * SM::ALD + wr * 64 + 4 * row16] * ws;
          const f4_t b4 = *(const f4_t*)&Bs[k * SM::BLD + wc * 64 + 4 * row16];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            av[i][s] = a4[i];
            bv[i][s] = b4[i];
          }
        }
        bf8_t bh[4], bm[4], bl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) split3x8(bv[j], bh[j], bm[j], bl[j], sc);
        // row block by row block; consecutive MFMAs on one accumulator are 4 apart
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          bf8_t ah, am, al;
          split3x8(av[i], ah, am, al, sc);
#pragma unroll
          for (int pr = 0; pr < 6; ++pr)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mma_bf16(pr_x(pr, ah, am, al), pr_y(pr, bh[j], bm[j], bl[j]), acc[i][j]);
        }
        continue;
      }
#pragma unroll
      for (int k0 = 0; k0 < DKC; k0 += 16) {
        if (ONE) {
          const f4_t w = wt4(W, ur_lane, uc_lane, k0, kv);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * q + s;
            const f4_t av = *(const f4_t*)&As[k * SM::ALD + wr * 64 + 4 * row16] * w[s];
            const f4_t bv = *(const f4_t*)&Bs[k * SM::BLD + wc * 64 + 4 * row16];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
          }
        } else {
          f4_t w[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) w[i] = wt4(W, ur_blk[i], uc_lane, k0, kv);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * q + s;
            const f4_t bv = *(const f4_t*)&Bs[k * SM::BLD + wc * 64 + 4 * row16];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float av = As[k * SM::ALD + wr * 64 + 16 * i + row16];
              const f4_t bw = bv * w[i][s];
#pragma unroll
              for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bw[j], acc[i][j], 0, 0, 0);
            }
          }
        }
      }
    }
  };
  if (one_cunit) kloop(std::integral_constant<bool, true>());
  else kloop(std::integral_constant<bool, false>());

  // ---- epilogue: 1/N scale, flat indices, symmetric mirror ----
  int64_t fcol[4];
  bool cok[4];
  int64_t ccomp[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = c0 + wc * 64 + (C::BPS ? 16 * j + row16 : 4 * row16 + j);
    const int64_t uc = c / a.c.pad, sc = c % a.c.pad;
    ccomp[j] = c;
    cok[j] = uc < a.c.n_units && sc < a.c.len;
    fcol[j] = cok[j] ? flat_index(a.c.perm, a.c.off, a.c.Tin, a.c.Tout, uc, sc) : 0;
  }
  // With the row mapping 16 q + 4 v + i a lane holds 16 consecutive rows of each of its
  // columns.  When they are 16 weights of one unit (consecutive flat indices) and every
  // (r, c) of the tile is stored (off the diagonal of a symmetric contraction), the mirrored
  // entries of a column are 64 contiguous bytes, written as 8-byte pairs instead of 16
  // scattered floats.  Otherwise (bias or padding slots, transposed index map, diagonal
  // tiles, accumulation) every entry takes the general path.
  if constexpr (C::BPS) {
    const int64_t rf = r0 + wr * 64 + 16 * q;
    const int64_t urf = rf / a.r.pad, srf = rf % a.r.pad;
    const bool vec = a.mirror && !a.accumulate && a.r.perm == 0 && (a.ldo & 1) == 0 &&
                     (reinterpret_cast<uintptr_t>(a.out) & 7) == 0 && !(SYM && r0 == c0) && urf < a.r.n_units &&
                     srf + 15 < a.r.len && srf + 15 < a.r.Tin;
    if (vec) {
      const int64_t fr0 = a.r.off + urf * a.r.Tin + srf;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!cok[j]) continue;
        float val[16];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int i = 0; i < 4; ++i) val[4 * v + i] = (float)(a.scale * (double)acc[i][j][v]);
#pragma unroll
        for (int e = 0; e < 16; ++e) a.out[(fr0 + e) * a.ldo + fcol[j]] = val[e];
        f2_t* m = reinterpret_cast<f2_t*>(a.out + fcol[j] * a.ldo + fr0);
#pragma unroll
        for (int e = 0; e < 8; ++e) m[e] = f2_t{val[2 * e], val[2 * e + 1]};
      }
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = r0 + wr * 64 + ((C::BPS || one_cunit) ? 16 * q + 4 * v + i : 16 * i + 4 * q + v);
      const int64_t ur = r / a.r.pad, sr = r % a.r.pad;
      if (!(ur < a.r.n_units && sr < a.r.len)) continue;
      const int64_t fr = flat_index(a.r.perm, a.r.off, a.r.Tin, a.r.Tout, ur, sr);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!cok[j]) continue;
        if (SYM && r < ccomp[j]) continue;
        const double val = a.scale * (double)acc[i][j][v];
        store_out<float>(a.out, fr * a.ldo + fcol[j], val, a.accumulate);
        if (a.mirror && !(SYM && r == ccomp[j])) store_out<float>(a.out, fcol[j] * a.ldo + fr, val, a.accumulate);
      }
    }
}

extern __shared__ __attribute__((aligned(16))) float dma_smem[];

template <int WMODE, bool SYM, int MAXU, class C>
__global__ __launch_bounds__(256, 2) void krg_kernel_dma(KrgArgs<float, float> a, int64_t tiles_c, int64_t ntiles) {
  int64_t t = xcd_tile(blockIdx.x, gridDim.x, ntiles * a.ksplit);
  if (t < 0) return;
  if (a.ksplit > 1) {  // slice of the example range: shift every per-example operand
    const int64_t sp = t / ntiles, k0 = sp * a.kslice;
    t -= sp * ntiles;
    a.r.src += k0 * a.r.ld;
    a.c.src += k0 * a.c.ld;
    if (a.r.scale) a.r.scale += k0 * a.r.ld_scale;
    if (a.c.scale) a.c.scale += k0 * a.c.ld_scale;
    if (a.wts) a.wts += k0;
    if (a.bparts) a.bparts += (k0 / 32) * (int64_t)3 * a.bp_nblk * 512;  // kslice is a multiple of 32
    a.N = mn64(a.kslice, a.N - k0);
    a.out += sp * a.out_split;
  }
  krg_tile_dma<WMODE, SYM, MAXU, C>(a, t, tiles_c, dma_smem);
}

// Units of one side that a 128-row tile can touch: pad >= 128 -> 2, >= 32 -> 5, else 9.
int dma_maxu(int pad) { return pad >= 128 ? 2 : (pad >= 32 ? 5 : 9); }

// The copy offsets of the LDS-staged tile are signed 32-bit byte offsets from
// per-chunk base pointers; contractions whose offsets could exceed that use the
// register-staged tile.
bool dma_fits(const KrgArgs<float, float>& a, int maxu) {
  const int64_t lim = 0x7fff0000, DKC = 32;  // largest chunk of any configuration
  if (a.r.len > a.r.ld || a.c.len > a.c.ld) return false;
  if ((int64_t)DKC * std::max(a.r.ld, a.c.ld) * 4 > lim) return false;
  if (a.wmode == KRG_PAIR_FULL && (((int64_t)(maxu - 1) * a.c.n_units + maxu) * a.ldw + DKC) * 4 > lim) return false;
  if (a.wmode == KRG_PAIR_DIAG && ((int64_t)maxu * a.ldw + DKC) * 4 > lim) return false;
  if (a.wmode == KRG_RANK1 && ((int64_t)DKC * std::max(a.r.ld_scale, a.c.ld_scale) + maxu) * 4 > lim) return false;
  return true;
}

template <int WMODE, bool SYM, int MAXU, class C>
void launch_dma_one(Exec& ex, const KrgArgs<float, float>& a, dim3 grid, int64_t tc, int64_t nt) {
  constexpr int bytes = DmaSmem<WMODE, MAXU, C>::SIZE * 4;
  static const bool attr = [] {  // once per process (thread-safe static initialisation)
    (void)hipFuncSetAttribute((const void*)krg_kernel_dma<WMODE, SYM, MAXU, C>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((krg_kernel_dma<WMODE, SYM, MAXU, C>), grid, dim3(256), bytes, ex.stream, a, tc, nt);
}

template <int MAXU, class C = DmaDefault>
void launch_dma(Exec& ex, const KrgArgs<float, float>& a, dim3 grid, int64_t tc, int64_t nt) {
  if (a.wmode == KRG_RANK1) {
    if (a.symmetric) launch_dma_one<KRG_RANK1, true, MAXU, C>(ex, a, grid, tc, nt);
    else launch_dma_one<KRG_RANK1, false, MAXU, C>(ex, a, grid, tc, nt);
  } else if (a.wmode == KRG_PAIR_FULL) {
    if (a.symmetric) launch_dma_one<KRG_PAIR_FULL, true, MAXU, C>(ex, a, grid, tc, nt);
    else launch_dma_one<KRG_PAIR_FULL, false, MAXU, C>(ex, a, grid, tc, nt);
  } else {
    launch_dma_one<KRG_PAIR_DIAG, false, MAXU, C>(ex, a, grid, tc, nt);
  }
}

// FP32 with K chunk 16 is held to two wavefronts per SIMD (228 registers, no spills):
// the kernel is latency-sensitive and the second wavefront hides the staging loads.
template <typename T, typename TOut, int WMODE, bool SYM, int KC, int STAGES>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && KC == 16) ? 2 : 1) void krg_kernel(KrgArgs<T, TOut> a,
                                                                                         int64_t tiles_c,
                                                                                         int64_t ntiles) {
  __shared__ __attribute__((aligned(16))) T smem[KrgSmem<T, WMODE, KC, STAGES>::SIZE];
  const int64_t t = xcd_tile(blockIdx.x, gridDim.x, ntiles);
  if (t < 0) return;
  krg_tile<T, TOut, WMODE, SYM, KC, STAGES>(a, t, tiles_c, smem);
}

// Persistent form for many contractions (several networks): every workgroup takes tiles
// from global counters until all tiles of all jobs are done; a tile's job is found by
// binary search over the jobs' first-tile offsets.  The tile range is cut into 8
// contiguous parts, one per XCD (workgroups reach the XCDs round-robin): a workgroup
// takes the next tile of its own XCD's part and, once that part is exhausted, helps the
// following parts, so neighbouring tiles (which share operand panels) mostly run in one
// XCD's L2.  One kernel instance per units-per-tile bound and tile configuration; each
// tile is computed by exactly one workgroup with the single-launch tile code, so results
// do not depend on the schedule and equal single-contraction launches bitwise.
template <int MAXU, class C>
constexpr int persist_lds_bytes() {
  return std::max(std::max(DmaSmem<KRG_PAIR_FULL, MAXU, C>::SIZE, DmaSmem<KRG_RANK1, MAXU, C>::SIZE),
                  DmaSmem<KRG_PAIR_DIAG, MAXU, C>::SIZE) * 4;
}
constexpr int PERSIST_PARTS = 8;

// Next tile of a persistent launch for this workgroup (the same value in every lane), or -1
// once every part is exhausted.  visited: parts found exhausted so far (thread 0's copy).
__device__ __forceinline__ int64_t persistent_next(int64_t total, unsigned long long* counters, int& visited,
                                                   int64_t* tsh) {
  const int64_t per = (total + PERSIST_PARTS - 1) / PERSIST_PARTS;
  const int home = (int)(blockIdx.x % PERSIST_PARTS);
  if (threadIdx.x == 0) {
    int64_t t = -1;
    while (visited < PERSIST_PARTS) {
      const int x = (home + visited) % PERSIST_PARTS;
      const int64_t lo = x * per, hi = min(total, lo + per);
      if (lo < hi) {
        const int64_t k = (int64_t)atomicAdd(&counters[x], 1ull);
        if (lo + k < hi) {
          t = lo + k;
          break;
        }
      }
      ++visited;
    }
    *tsh = t;
  }
  __syncthreads();
  // the tile (hence the job and its arguments) is the same for the whole workgroup:
  // uniform values let the job's arguments live in scalar registers
  const int64_t t = uniform64(*tsh);
  __syncthreads();
  return t;
}

// The job list is read through the constant address space: with a workgroup-uniform job
// index its fields are scalar loads, so the buffer descriptors the tile builds from them
// are uniform (a descriptor the compiler cannot prove uniform costs a loop around every
// buffer load).
typedef const __attribute__((address_space(4))) KrgJob* cjob_ptr;

// Job of tile t: the last job whose first tile is at most t.
__device__ __forceinline__ const KrgJob& persistent_job(const KrgJob* jobs, int njobs, int64_t t) {
  cjob_ptr cj = (cjob_ptr)jobs;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (cj[mid].first <= t) lo = mid; else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  return *(const KrgJob*)(cj + lo);
}

template <int MAXU, class C>
__global__ __launch_bounds__(256, 2) void krg_persistent(const KrgJob* jobs, int njobs, int64_t total,
                                                         unsigned long long* counters) {
  __shared__ int64_t tsh;
  int visited = 0;
  for (;;) {
    const int64_t t = persistent_next(total, counters, visited, &tsh);
    if (t < 0) break;
    const KrgJob& J = persistent_job(jobs, njobs, t);
    const int64_t lt = t - J.first;
    switch (J.mode * 2 + (J.a.symmetric ? 1 : 0)) {
      case KRG_RANK1 * 2 + 0: krg_tile_dma<KRG_RANK1, false, MAXU, C>(J.a, lt, J.tiles_c, dma_smem); break;
      case KRG_RANK1 * 2 + 1: krg_tile_dma<KRG_RANK1, true, MAXU, C>(J.a, lt, J.tiles_c, dma_smem); break;
      case KRG_PAIR_FULL * 2 + 0: krg_tile_dma<KRG_PAIR_FULL, false, MAXU, C>(J.a, lt, J.tiles_c, dma_smem); break;
      case KRG_PAIR_FULL * 2 + 1: krg_tile_dma<KRG_PAIR_FULL, true, MAXU, C>(J.a, lt, J.tiles_c, dma_smem); break;
      default: krg_tile_dma<KRG_PAIR_DIAG, false, MAXU, C>(J.a, lt, J.tiles_c, dma_smem); break;
    }
    __syncthreads();
  }
}

__global__ void k_zero_counters(unsigned long long* c) {
  if (threadIdx.x < PERSIST_PARTS) c[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) p[t] = 0.f;
}

// One thread per dword of the pre-split layout (see bsplit in common.h): two consecutive
// examples of one slot, split by the same arithmetic as the tile's split3x2.
__global__ __launch_bounds__(256) void k_bsplit(const float* __restrict__ src, int64_t ld, int32_t len, int32_t nblk,
                                                int64_t N, int64_t total, uint32_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  const int e = (int)(t & 511);
  const int64_t cb = t >> 9;  // chunk * nblk + block
  const int64_t chunk = cb / nblk;
  const int bi = (int)(cb - chunk * nblk);
  const int jj = e >> 8, q = (e >> 6) & 3, s16 = (e >> 2) & 15, w = e & 3;
  const int sc = bi * 32 + 16 * jj + s16;
  const int64_t k = chunk * 32 + 8 * q + 2 * w;
  float x0 = 0.f, x1 = 0.f;
  if (sc < len) {
    if (k < N) x0 = src[k * ld + sc];
    if (k + 1 < N) x1 = src[(k + 1) * ld + sc];
  }
  bf2_t h, m, l;
  split3x2(f2_t{x0, x1}, h, m, l, split_consts());
  const int64_t ps = (int64_t)nblk * 512;
  const int64_t o = (chunk * 3 * nblk + bi) * 512 + e;
  out[o] = __builtin_bit_cast(uint32_t, h);
  out[o + ps] = __builtin_bit_cast(uint32_t, m);
  out[o + 2 * ps] = __builtin_bit_cast(uint32_t, l);
}

template <typename T, typename TOut, int KC, int STAGES>
void launch_cfg(Exec& ex, const KrgArgs<T, TOut>& a, dim3 grid, int64_t tc, int64_t nt) {
#define KRG_LAUNCH(MODE, SYMV) \
  hipLaunchKernelGGL((krg_kernel<T, TOut, MODE, SYMV, KC, STAGES>), grid, dim3(256), 0, ex.stream, a, tc, nt)
  if (a.wmode == KRG_RANK1) {
    if (a.symmetric) KRG_LAUNCH(KRG_RANK1, true); else KRG_LAUNCH(KRG_RANK1, false);
  } else if (a.wmode == KRG_PAIR_FULL) {
    if (a.symmetric) KRG_LAUNCH(KRG_PAIR_FULL, true); else KRG_LAUNCH(KRG_PAIR_FULL, false);
  } else {
    KRG_LAUNCH(KRG_PAIR_DIAG, false);
  }
#undef KRG_LAUNCH
}

}  // namespace

// variant: 0 = default for the precision; register-staged tile 1 = (KC 16, 1 stage), 2 = (16, 2),
// 3 = (32, 1), 4 = (32, 2); FP32 LDS-staged tile 5 = (32 examples, 2 stages), 6 = (16, 3);
// split products 7 = columns split in the tile, 8 = pre-split columns (needs a.bparts)
// ---------------------------------------------------------------------------
// Example lists of a pair-weighted contraction.  flags[u][n] = 1 when some row unit has a
// nonzero weight with column unit u at example n; a column tile lists, in increasing order,
// the examples flagged for any unit its 128 columns touch.  (With ReLU units the weights of
// an inactive column unit are exact zeros, about half of them.)
// ---------------------------------------------------------------------------
// rows = 0: flags[u][n] = some row unit r has w[r][u][n] != 0 (u a column unit, nr row
// units); rows = 1: flags[u][n] = some column unit v has w[u][v][n] != 0 (u a row unit, nr
// column units)
__global__ __launch_bounds__(256) void k_list_flags(const float* __restrict__ w, int64_t ldw, int32_t nr,
                                                    int32_t nu, int64_t N, int rows, uint8_t* __restrict__ flags) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int u = blockIdx.y;
  if (n >= N) return;
  bool f = false;
  for (int r = 0; r < nr; ++r)
    f |= w[(rows ? (int64_t)u * nr + r : (int64_t)r * nu + u) * ldw + n] != 0.f;
  flags[(int64_t)u * N + n] = f ? 1 : 0;
}

// one workgroup per column tile: ordered compaction of the flagged examples (a wavefront
// ballot for positions within 64 examples, the four wavefronts' counts through LDS), then
// example 0 up to the next multiple of 32
__global__ __launch_bounds__(256) void k_list_build(const uint8_t* __restrict__ flags, int64_t N, int32_t pad,
                                                    int32_t nu, int64_t ldl, int32_t* __restrict__ lists,
                                                    int64_t* __restrict__ cnt) {
  __shared__ int wsum[4];
  const int64_t t = blockIdx.x;
  const int u0 = (int)(t * BN / pad), u1 = (int)min((int64_t)nu - 1, (t * BN + BN - 1) / pad);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t* L = lists + t * ldl;
  int64_t base = 0;
  for (int64_t n0 = 0; n0 < N; n0 += 256) {
    const int64_t n = n0 + threadIdx.x;
    const bool f = n < N && (flags[(int64_t)u0 * N + n] | flags[(int64_t)u1 * N + n]);
    const unsigned long long b = __ballot(f);
    const int before = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(b);
    __syncthreads();
    int off = 0;
    for (int x = 0; x < wave; ++x) off += wsum[x];
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (f) L[base + off + before] = (int32_t)n;
    base += tot;
    __syncthreads();
  }
  const int64_t end = (base + 31) / 32 * 32;
  for (int64_t i = base + threadIdx.x; i < end; i += 256) L[i] = 0;
  if (threadIdx.x == 0) cnt[t] = base;
}

// one workgroup per unit pair (u >= v): ordered compaction of the examples with w[u][v][n] != 0
__global__ __launch_bounds__(256) void k_pair_list_build(const float* __restrict__ w, int64_t ldw, int32_t nu,
                                                         int64_t N, int64_t ldl, int32_t* __restrict__ lists,
                                                         int64_t* __restrict__ cnt) {
  __shared__ int wsum[4];
  const int64_t pi = blockIdx.x;
  int u = (int)((sqrt(8.0 * (double)pi + 1.0) - 1.0) * 0.5);
  while ((int64_t)u * (u + 1) / 2 > pi) --u;
  while ((int64_t)(u + 1) * (u + 2) / 2 <= pi) ++u;
  const int v = (int)(pi - (int64_t)u * (u + 1) / 2);
  const float* wr = w + ((int64_t)u * nu + v) * ldw;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t* L = lists + pi * ldl;
  int64_t base = 0;
  for (int64_t n0 = 0; n0 < N; n0 += 256) {
    const int64_t n = n0 + threadIdx.x;
    const bool f = n < N && wr[n] != 0.f;
    const unsigned long long b = __ballot(f);
    const int before = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(b);
    __syncthreads();
    int off = 0;
    for (int x = 0; x < wave; ++x) off += wsum[x];
    const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (f) L[base + off + before] = (int32_t)n;
    base += tot;
    __syncthreads();
  }
  const int64_t end = (base + 31) / 32 * 32;
  for (int64_t i = base + threadIdx.x; i < end; i += 256) L[i] = 0;
  if (threadIdx.x == 0) cnt[pi] = base;
}

void krg_build_row_lists(Exec& ex, const KrgArgs<float, float>& a, uint8_t* flags, int32_t* lists, int64_t* cnt,
                         int64_t ldl) {
  const int64_t tr = ((int64_t)a.r.n_units * a.r.pad + BM - 1) / BM;
  if (tr <= 0 || a.N <= 0 || !launch_ok(ex)) return;
  hipLaunchKernelGGL(k_list_flags, dim3((unsigned)((a.N + 255) / 256), (unsigned)a.r.n_units), dim3(256), 0,
                     ex.stream, a.wts, a.ldw, a.c.n_units, a.c.n_units, a.N, 1, flags);
  hipLaunchKernelGGL(k_list_build, dim3((unsigned)tr), dim3(256), 0, ex.stream, flags, a.N, a.r.pad, a.r.n_units,
                     ldl, lists, cnt);
}

void krg_build_pair_lists(Exec& ex, const KrgArgs<float, float>& a, int32_t* lists, int64_t* cnt, int64_t ldl) {
  const int64_t np = (int64_t)a.c.n_units * (a.c.n_units + 1) / 2;
  if (np <= 0 || a.N <= 0 || !launch_ok(ex)) return;
  hipLaunchKernelGGL(k_pair_list_build, dim3((unsigned)np), dim3(256), 0, ex.stream, a.wts, a.ldw, a.c.n_units, a.N,
                     ldl, lists, cnt);
}

int64_t krg_list_tiles(const KrgArgs<float, float>& a) { return ((int64_t)a.c.n_units * a.c.pad + BN - 1) / BN; }

void krg_build_lists(Exec& ex, const KrgArgs<float, float>& a, uint8_t* flags, int32_t* lists, int64_t* cnt,
                     int64_t ldl) {
  const int64_t tc = krg_list_tiles(a);
  if (tc <= 0 || a.N <= 0 || !launch_ok(ex)) return;
  hipLaunchKernelGGL(k_list_flags, dim3((unsigned)((a.N + 255) / 256), (unsigned)a.c.n_units), dim3(256), 0,
                     ex.stream, a.wts, a.ldw, a.r.n_units, a.c.n_units, a.N, 0, flags);
  hipLaunchKernelGGL(k_list_build, dim3((unsigned)tc), dim3(256), 0, ex.stream, flags, a.N, a.c.pad, a.c.n_units,
                     ldl, lists, cnt);
}

// Share of the full example sum that the listed tiles compute: each tile's list length over N,
// weighted by the tile's entries (valid slots; on or below the diagonal when symmetric).
// Reads the counts back (the profile's flop count only).
double krg_list_share(Exec& ex, const KrgArgs<float, float>& a) {
  const int64_t tcn = krg_list_tiles(a);
  const int64_t np = a.plist ? (int64_t)a.c.n_units * (a.c.n_units + 1) / 2 : 0;
  const int64_t trn0 = ((int64_t)a.r.n_units * a.r.pad + BM - 1) / BM, nr = a.rlist ? trn0 : 0;
  std::vector<int64_t> cnt((size_t)tcn), pc((size_t)np), rc((size_t)nr);
  if (hipMemcpyAsync(cnt.data(), a.kcnt, tcn * sizeof(int64_t), hipMemcpyDeviceToHost, ex.stream) != hipSuccess ||
      (np > 0 && hipMemcpyAsync(pc.data(), a.pcnt, np * sizeof(int64_t), hipMemcpyDeviceToHost, ex.stream) !=
                     hipSuccess) ||
      (nr > 0 && hipMemcpyAsync(rc.data(), a.rcnt, nr * sizeof(int64_t), hipMemcpyDeviceToHost, ex.stream) !=
                     hipSuccess) ||
      hipStreamSynchronize(ex.stream) != hipSuccess)
    return 1.0;
  // valid slots of a 128-wide tile of one side
  auto valid = [](const KrgSide<float>& sd, int64_t t0) {
    int64_t v = 0;
    for (int64_t i = t0; i < std::min<int64_t>(t0 + BM, (int64_t)sd.n_units * sd.pad); ++i) v += (i % sd.pad) < sd.len;
    return v;
  };
  const int64_t trn = ((int64_t)a.r.n_units * a.r.pad + BM - 1) / BM;
  std::vector<int64_t> vr((size_t)trn), vc((size_t)tcn);
  for (int64_t t = 0; t < trn; ++t) vr[t] = valid(a.r, t * BM);
  for (int64_t t = 0; t < tcn; ++t) vc[t] = valid(a.c, t * BN);
  const double N = (double)std::max<int64_t>(1, a.N);
  double all = 0, done = 0;
  for (int64_t tr = 0; tr < trn; ++tr)
    for (int64_t tc = 0; tc < (a.symmetric ? tr + 1 : tcn); ++tc) {
      const double e = (a.symmetric && tr == tc) ? 0.5 * vr[tr] * (vr[tr] + 1) : (double)vr[tr] * vc[tc];
      int64_t c = cnt[tc];
      if (np > 0) {
        const int64_t r0 = tr * BM, c0 = tc * BN;
        const int64_t ul = r0 / a.r.pad, uh = std::min<int64_t>(a.r.n_units - 1, (r0 + BM - 1) / a.r.pad);
        const int64_t vl = c0 / a.c.pad, vh = std::min<int64_t>(a.c.n_units - 1, (c0 + BN - 1) / a.c.pad);
        if (ul == uh && vl == vh) c = pc[ul * (ul + 1) / 2 + vl];
        else if (nr > 0 && rc[tr] < c) c = rc[tr];
      }
      all += e;
      done += e * (double)c / N;
    }
  return all > 0 ? done / all : 1.0;
}

template <typename T, typename TOut>
void krg_variant(Exec& ex, const KrgArgs<T, TOut>& a, int variant) {
  const int64_t rows = (int64_t)a.r.n_units * a.r.pad, cols = (int64_t)a.c.n_units * a.c.pad;
  const int64_t tr = (rows + BM - 1) / BM, tc = (cols + BN - 1) / BN;
  const int64_t nt = a.symmetric ? tr * (tr + 1) / 2 : tr * tc;
  if (nt <= 0) return;
  if (!launch_ok(ex)) return;
  // algorithmic work of this launch (for the per-kernel profile)
  const double Pr = (double)a.r.n_units * a.r.len, Pc = (double)a.c.n_units * a.c.len;
  double entries = a.symmetric ? Pr * (Pr + 1) / 2 : Pr * Pc;
  if (a.wmode == KRG_PAIR_DIAG) entries = (double)std::min(a.r.n_units, a.c.n_units) * a.r.len * a.c.len;
  double wbytes = 0;
  if (a.wmode == KRG_PAIR_FULL) wbytes = (double)a.r.n_units * a.c.n_units * a.N * sizeof(T);
  if (a.wmode == KRG_PAIR_DIAG) wbytes = (double)a.r.n_units * a.N * sizeof(T);
  if (a.wmode == KRG_RANK1) wbytes = (double)a.N * (a.r.n_units + a.c.n_units) * sizeof(T);
  const double src = (double)a.N * (a.r.ld + (a.symmetric ? 0 : a.c.ld)) * sizeof(T);
  const double obytes = entries * sizeof(TOut) * (a.mirror ? 2 : 1) * (a.accumulate ? 2 : 1);
  const char* names[2][3][2] = {{{"krg_f32_rank1", "krg_f32_rank1_sym"}, {"krg_f32_pair", "krg_f32_pair_sym"},
                                 {"krg_f32_pairdiag", "krg_f32_pairdiag_sym"}},
                                {{"krg_f64_rank1", "krg_f64_rank1_sym"}, {"krg_f64_pair", "krg_f64_pair_sym"},
                                 {"krg_f64_pairdiag", "krg_f64_pairdiag_sym"}}};
  const int ks = std::max(1, a.ksplit);
  // FP32 default: the LDS-staged tile, one kernel instance per units-per-tile bound; the
  // profile name carries that bound so that a profile class is one kernel instance
  const int maxu = dma_maxu(std::min(a.r.pad, a.c.pad));
  bool dma = false;
  if constexpr (sizeof(T) == 4) dma = (variant == 0 || variant >= 5) && dma_fits(a, maxu);
  std::string label = a.label ? a.label : names[sizeof(T) == 8][a.wmode][a.symmetric ? 1 : 0];
  if (dma && !a.label) label += "_u" + std::to_string(maxu);
  dim3 grid((unsigned)xcd_grid(nt * ks));
  if constexpr (sizeof(T) == 4) {
    if (dma) {
      // configuration: 0 = (16 examples, 2 stages), 1 = (16, 3), 2 = (32, 2)
      auto go = [&](int cfg, dim3 g, int64_t ntl) {
        auto run = [&](auto c) {
          using C = decltype(c);
          if constexpr (C::LIST) {  // pair-weighted form: symmetric with two units per tile side, or not
            if (a.symmetric) launch_dma_one<KRG_PAIR_FULL, true, 2, C>(ex, a, g, tc, ntl);
            else if (maxu == 2) launch_dma_one<KRG_PAIR_FULL, false, 2, C>(ex, a, g, tc, ntl);
            else launch_dma_one<KRG_PAIR_FULL, false, 5, C>(ex, a, g, tc, ntl);
          } else if constexpr (C::BPS) {  // only the pair-weighted form, two column units per tile
            if (a.symmetric) launch_dma_one<KRG_PAIR_FULL, true, 2, C>(ex, a, g, tc, ntl);
            else if (maxu == 2) launch_dma_one<KRG_PAIR_FULL, false, 2, C>(ex, a, g, tc, ntl);
            else launch_dma_one<KRG_PAIR_FULL, false, 5, C>(ex, a, g, tc, ntl);
          } else {
            if (maxu == 2) launch_dma<2, C>(ex, a, g, tc, ntl);
            else if (maxu == 5) launch_dma<5, C>(ex, a, g, tc, ntl);
            else launch_dma<9, C>(ex, a, g, tc, ntl);
          }
        };
        if (cfg == 1) run(DmaCfg<16, 3>());
        else if (cfg == 2) run(DmaCfg<32, 2>());
        else if (cfg == 3) run(DmaCfg<32, 2, true>());
        else if (cfg == 4) run(DmaCfg<32, 2, true, true>());
        else if (cfg == 5) run(DmaCfg<32, 2, true, false, true>());
        else run(DmaDefault());
      };
      int cfg = variant == 5 ? 2 : (variant == 6 ? 1 : (variant >= 7 || ex.split ? 3 : 0));
      // split products on pre-split columns (variant 8 asks for it explicitly)
      // (the rows may span up to 5 units of a tile: each lane's rows lie in one unit)
      const bool bps = a.bparts && a.wmode == KRG_PAIR_FULL && a.c.pad >= 128 && a.c.pad % 32 == 0 &&
                       (maxu == 2 || (maxu == 5 && !a.symmetric)) && a.bp_nblk == a.c.pad / 32 &&
                       (ks == 1 || a.kslice % 32 == 0);
      // split products over the column tiles' example lists (their gathered row offsets and
      // weight offsets stay below 2^31 bytes)
      const int64_t lim = 0x7fff0000;
      const bool lst = a.klist && a.kcnt && a.wmode == KRG_PAIR_FULL && ks == 1 &&
                       (a.symmetric ? maxu == 2 : (maxu == 2 || maxu == 5)) &&
                       a.N * std::max(a.r.ld, a.c.ld) * 4 <= lim &&
                       (((int64_t)a.c.n_units + 2) * a.ldw + a.N) * 4 <= lim;
      double done = 1.0;  // share of the examples the tiles sum over (profile only)
      if (cfg == 3 && lst && variant != 7) {
        cfg = 5;
        if (ex.ctx->profile) done = krg_list_share(ex, a);
      } else if (cfg == 3 && bps && variant != 7) {
        cfg = 4;
      }
      if (cfg >= 3 && label.compare(0, 7, "krg_f32") == 0) label = "krg_bf16x6" + label.substr(7);
      // Probes write into the output, which the full launch then overwrites; a launch that
      // accumulates into its output keeps the default configuration.
      if (variant == 0 && !ex.split && ex.ctx->autotune && !a.accumulate && launch_ok(ex)) {
        // probe on the first two device rounds of tiles (all of them if fewer)
        static const int64_t slots = [] {
          int dev = 0, cus = 256;
          (void)hipGetDevice(&dev);
          (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
          return 3 * (int64_t)std::max(cus, 1);
        }();
        const int64_t ntp = std::min(nt, std::max<int64_t>(1, 2 * slots / ks));
        const dim3 gp((unsigned)xcd_grid(ntp * ks));
        auto lg = [](int64_t v) { int b = 0; while (v > 1) { v >>= 1; ++b; } return b; };
        const std::string key = "krg_f32 mode" + std::to_string(a.wmode) + (a.symmetric ? " sym" : "") + " u" +
                                std::to_string(maxu) + " slices" + std::to_string(ks) + " tiles2^" +
                                std::to_string(lg(nt)) + " N2^" + std::to_string(lg(a.N));
        static const char* const cfgs[3] = {"chunk16x2", "chunk16x3", "chunk32x2"};
        cfg = autotune_pick(ex, key, 3, cfgs, [&](int i) { go(i, gp, ntp); });
      }
      const int tok = prof_begin(ex, label.c_str(), 2.0 * a.N * entries * done, src * done + wbytes + obytes * ks);
      go(cfg, grid, nt);
      prof_end(ex, tok);
      return;
    }
  }
  const int tok = prof_begin(ex, label.c_str(), 2.0 * a.N * entries, src + wbytes + obytes * ks);
  if (ks > 1) {  // register-staged tile: one launch per slice of the example range
    grid = dim3((unsigned)xcd_grid(nt));
    for (int sp = 0; sp < ks; ++sp) {
      KrgArgs<T, TOut> b = a;
      const int64_t k0 = sp * a.kslice;
      b.ksplit = 1;
      b.r.src += k0 * a.r.ld;
      b.c.src += k0 * a.c.ld;
      if (b.r.scale) b.r.scale += k0 * a.r.ld_scale;
      if (b.c.scale) b.c.scale += k0 * a.c.ld_scale;
      if (b.wts) b.wts += k0;
      b.N = std::max<int64_t>(0, std::min(a.kslice, a.N - k0));
      b.out += sp * a.out_split;
      if (variant == 2) launch_cfg<T, TOut, 16, 2>(ex, b, grid, tc, nt);
      else launch_cfg<T, TOut, 16, 1>(ex, b, grid, tc, nt);
    }
    prof_end(ex, tok);
    return;
  }
  if (variant == 0) variant = 1;  // register-staged tile: K chunk 16, one stage
  if constexpr (sizeof(T) == 8) {  // FP64 tiles need twice the LDS: K chunk 16 only
    if (variant == 2)
      launch_cfg<T, TOut, 16, 2>(ex, a, grid, tc, nt);
    else
      launch_cfg<T, TOut, 16, 1>(ex, a, grid, tc, nt);
  } else {
    switch (variant) {
      case 1: launch_cfg<T, TOut, 16, 1>(ex, a, grid, tc, nt); break;
      case 2: launch_cfg<T, TOut, 16, 2>(ex, a, grid, tc, nt); break;
      case 3: launch_cfg<T, TOut, 32, 1>(ex, a, grid, tc, nt); break;
      default: launch_cfg<T, TOut, 32, 2>(ex, a, grid, tc, nt); break;
    }
  }
  prof_end(ex, tok);
}


// ---- pair-diagonal contraction as one product ----
namespace {
__global__ __launch_bounds__(256) void k_pd_form(const float* __restrict__ rsrc, int64_t rld, int32_t lr,
                                                 const float* __restrict__ w, int64_t ldw, int32_t U, int64_t N,
                                                 float* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x, row = (int64_t)U * lr;
  if (t >= N * row) return;
  const int64_t n = t / row;
  const int e = (int)(t - n * row), u = e / lr, sl = e - u * lr;
  Y[t] = w[u * ldw + n] * rsrc[n * rld + sl];
}

__global__ __launch_bounds__(256) void k_pd_scatter(const float* __restrict__ Cp, int64_t part, int32_t lr,
                                                    int32_t lc, int32_t U, KrgArgs<float, float> a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)U * lr * lc) return;
  const int b = (int)(t % lc);
  const int64_t m = t / lc;
  const int u = (int)(m / lr), sl = (int)(m % lr);
  float acc = 0.f;
#pragma unroll
  for (int sp = 0; sp < PD_SLICES; ++sp) acc += Cp[sp * part + t];
  const int64_t fr = flat_index(a.r.perm, a.r.off, a.r.Tin, a.r.Tout, u, sl);
  const int64_t fc = flat_index(a.c.perm, a.c.off, a.c.Tin, a.c.Tout, u, b);
  const double v = a.scale * (double)acc;
  store_out<float>(a.out, fr * a.ldo + fc, v, a.accumulate);
  if (a.mirror) store_out<float>(a.out, fc * a.ldo + fr, v, a.accumulate);
}
}  // namespace

int64_t pairdiag_floats(int64_t N, int64_t U, int64_t len_r, int64_t len_c) {
  return N * U * len_r + (int64_t)PD_SLICES * U * len_r * len_c;
}

void krg_pairdiag_gemm(Exec& ex, const KrgArgs<float, float>& a, float* ws) {
  const int32_t U = std::min(a.r.n_units, a.c.n_units), lr = a.r.len, lc = a.c.len;
  const int64_t N = a.N, M = (int64_t)U * lr, part = M * lc;
  if (U <= 0 || N <= 0 || !launch_ok(ex)) return;
  float* Y = ws;
  float* Cp = ws + N * M;
  const int tok = prof_begin(ex, "krg_pairdiag_gemm", 2.0 * N * (double)M * lc,
                             (double)N * (a.r.ld + a.c.ld + U) * 4 + (double)N * M * 8 + (double)part * 4 * 3);
  hipLaunchKernelGGL(k_pd_form, dim3((unsigned)((N * M + 255) / 256)), dim3(256), 0, ex.stream, a.r.src, a.r.ld, lr,
                     a.wts, a.ldw, U, N, Y);
  // partial products over PD_SLICES slices of the examples: PD_SLICES - 1 equal slices in
  // one batched call, the rest in a second call
  const int64_t ks = N / PD_SLICES, klast = N - (PD_SLICES - 1) * ks;
  if (ks > 0) {
    GemmArgs<float> g;
    g.M = M; g.N = lc; g.K = ks;
    g.A = Y; g.sam = 1; g.sak = M; g.sab = ks * M;
    g.B = a.c.src; g.sbk = a.c.ld; g.sbn = 1; g.sbb = ks * a.c.ld;
    g.C = Cp; g.scm = lc; g.scn = 1; g.scb = part;
    g.alpha = 1.f; g.beta = 0.f; g.batch = PD_SLICES - 1;
    gemm<float>(ex, g);
  } else {
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((part * (PD_SLICES - 1) + 255) / 256)), dim3(256), 0, ex.stream,
                       Cp, part * (PD_SLICES - 1));
  }
  const int64_t k0 = (PD_SLICES - 1) * ks;
  gemm_rm<float>(ex, true, false, M, lc, klast, 1.f, Y + k0 * M, M, a.c.src + k0 * a.c.ld, a.c.ld, 0.f,
                 Cp + (PD_SLICES - 1) * part, lc);
  hipLaunchKernelGGL(k_pd_scatter, dim3((unsigned)((part + 255) / 256)), dim3(256), 0, ex.stream, Cp, part, lr, lc, U,
                     a);
  prof_end(ex, tok);
}

int64_t bsplit_dwords(int64_t N, int32_t pad) { return (N + 31) / 32 * 3 * (int64_t)(pad / 32) * 512; }

void bsplit(Exec& ex, const float* src, int64_t ld, int32_t len, int32_t pad, int64_t N, uint32_t* out) {
  const int64_t nblk = pad / 32, total = (N + 31) / 32 * nblk * 512;
  if (total <= 0 || pad % 32 != 0 || len > pad) return;
  if (!launch_ok(ex)) return;
  const int tok = prof_begin(ex, "bsplit", 0.0, (double)N * len * 4 + (double)total * 12);
  hipLaunchKernelGGL(k_bsplit, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, ex.stream, src, ld, len,
                     (int32_t)nblk, N, total, out);
  prof_end(ex, tok);
}

int64_t krg_tiles(const KrgArgs<float, float>& a, int64_t* tiles_c) {
  const int64_t rows = (int64_t)a.r.n_units * a.r.pad, cols = (int64_t)a.c.n_units * a.c.pad;
  const int64_t tr = (rows + BM - 1) / BM, tc = (cols + BN - 1) / BN;
  *tiles_c = tc;
  return a.symmetric ? tr * (tr + 1) / 2 : tr * tc;
}

namespace {
template <int MAXU, class C>
void persistent_one(Exec& ex, const KrgJob* jobs_dev, int njobs, int64_t total, unsigned long long* counters,
                    int64_t grid) {
  constexpr int bytes = persist_lds_bytes<MAXU, C>();
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)krg_persistent<MAXU, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              bytes);
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL((krg_persistent<MAXU, C>), dim3((unsigned)grid), dim3(256), bytes, ex.stream, jobs_dev, njobs,
                     total, counters);
}
template <class C>
void persistent_u(Exec& ex, int maxu, const KrgJob* jobs_dev, int njobs, int64_t total, unsigned long long* counters,
                  int64_t grid) {
  if (maxu == 2) persistent_one<2, C>(ex, jobs_dev, njobs, total, counters, grid);
  else if (maxu == 5) persistent_one<5, C>(ex, jobs_dev, njobs, total, counters, grid);
  else persistent_one<9, C>(ex, jobs_dev, njobs, total, counters, grid);
}
}  // namespace

int krg_persistent_maxu(const KrgArgs<float, float>& a) { return dma_maxu(std::min(a.r.pad, a.c.pad)); }

bool krg_persistent_fits(const KrgArgs<float, float>& a) { return dma_fits(a, krg_persistent_maxu(a)); }

void krg_persistent_launch(Exec& ex, const KrgJob* jobs_dev, int njobs, int64_t total, unsigned long long* counters,
                           double flops, double bytes, int maxu, int cfg) {
  if (total <= 0) return;
  if (!launch_ok(ex)) return;
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, ex.stream, counters);
  if (!launch_ok(ex)) return;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t grid = std::min<int64_t>(xcd_grid(total), xcd_grid((int64_t)cus * 2));
  std::string label = std::string(cfg == 3 ? "krg_bf16x6_persistent_u" : "krg_f32_persistent_u") + std::to_string(maxu);
  const int tok = prof_begin(ex, label.c_str(), flops, bytes);
  switch (cfg) {
    case 1: persistent_u<DmaCfg<16, 3>>(ex, maxu, jobs_dev, njobs, total, counters, grid); break;
    case 2: persistent_u<DmaCfg<32, 2>>(ex, maxu, jobs_dev, njobs, total, counters, grid); break;
    case 3: persistent_u<DmaCfg<32, 2, true>>(ex, maxu, jobs_dev, njobs, total, counters, grid); break;
    default: persistent_u<DmaDefault>(ex, maxu, jobs_dev, njobs, total, counters, grid); break;
  }
  prof_end(ex, tok);
}

template <typename T, typename TOut>
void krg(Exec& ex, const KrgArgs<T, TOut>& a) {
  krg_variant<T, TOut>(ex, a, 0);
}

template void krg<double, double>(Exec&, const KrgArgs<double, double>&);
template void krg<float, float>(Exec&, const KrgArgs<float, float>&);
template void krg_variant<float, float>(Exec&, const KrgArgs<float, float>&, int);

}  // namespace hs
