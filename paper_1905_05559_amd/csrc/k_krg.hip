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

// Grouped tile order: consecutive tile ids walk GROUP row panels column by column, so
// the ~64 tiles an XCD runs at once share 8 row panels and 8 column panels in its L2
// instead of one row panel and 64 column panels.  Symmetric blocks enumerate only
// tiles with tc <= tr: group g (rows gG .. gG+Gg-1) holds gG full columns of Gg tiles
// and then a lower triangle of Gg columns.
constexpr int64_t GROUP = 8;

__device__ __forceinline__ void tile_of(int64_t t, bool symmetric, int64_t tiles_c, int64_t tiles_r, int64_t& tr,
                                        int64_t& tc) {
  if (!symmetric) {
    const int64_t g = t / (GROUP * tiles_c), u = t - g * GROUP * tiles_c;
    const int64_t Gg = min(GROUP, tiles_r - g * GROUP);
    tc = u / Gg;
    tr = g * GROUP + u % Gg;
    return;
  }
  // tiles before group g (all full): G^2 g (g - 1) / 2 + g G (G + 1) / 2
  auto before = [](int64_t g) { return GROUP * GROUP * g * (g - 1) / 2 + g * GROUP * (GROUP + 1) / 2; };
  int64_t g = (int64_t)(sqrt(2.0 * (double)t) / (double)GROUP);
  while (g > 0 && before(g) > t) --g;
  while (before(g + 1) <= t && (g + 1) * GROUP < tiles_r) ++g;
  int64_t u = t - before(g);
  const int64_t Gg = min(GROUP, tiles_r - g * GROUP), r0 = g * GROUP;
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

// Persistent form for many contractions (several networks): every workgroup takes the
// next tile from a global counter until all tiles of all jobs are done; a tile's job is
// found by binary search over the jobs' first-tile offsets.  Each tile is computed by
// exactly one workgroup, so results do not depend on the schedule.
__global__ __launch_bounds__(256, 2) void krg_persistent(const KrgJob* jobs, int njobs, int64_t total,
                                                         unsigned long long* counter) {
  constexpr int SZ = KrgSmem<float, KRG_PAIR_FULL, 16, 1>::SIZE;
  __shared__ __attribute__((aligned(16))) float smem[SZ];
  __shared__ int64_t tsh;
  for (;;) {
    if (threadIdx.x == 0) tsh = (int64_t)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t t = tsh;
    __syncthreads();
    if (t >= total) break;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (jobs[mid].first <= t) lo = mid; else hi = mid - 1;
    }
    const KrgJob& J = jobs[lo];
    const int64_t lt = t - J.first;
    switch (J.mode * 2 + (J.a.symmetric ? 1 : 0)) {
      case KRG_RANK1 * 2 + 0: krg_tile<float, float, KRG_RANK1, false, 16, 1>(J.a, lt, J.tiles_c, smem); break;
      case KRG_RANK1 * 2 + 1: krg_tile<float, float, KRG_RANK1, true, 16, 1>(J.a, lt, J.tiles_c, smem); break;
      case KRG_PAIR_FULL * 2 + 0: krg_tile<float, float, KRG_PAIR_FULL, false, 16, 1>(J.a, lt, J.tiles_c, smem); break;
      case KRG_PAIR_FULL * 2 + 1: krg_tile<float, float, KRG_PAIR_FULL, true, 16, 1>(J.a, lt, J.tiles_c, smem); break;
      default: krg_tile<float, float, KRG_PAIR_DIAG, false, 16, 1>(J.a, lt, J.tiles_c, smem); break;
    }
    __syncthreads();
  }
}

__global__ void k_zero_counter(unsigned long long* c) { *c = 0ull; }

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

// variant: 0 = default for the precision; 1 = (KC 16, 1 stage); 2 = (16, 2); 3 = (32, 1); 4 = (32, 2)
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
  const int tok = prof_begin(ex, names[sizeof(T) == 8][a.wmode][a.symmetric ? 1 : 0], 2.0 * a.N * entries,
                             src + wbytes + obytes);
  dim3 grid((unsigned)xcd_grid(nt));
  if (variant == 0) variant = 1;  // measured best on the MNIST-shaped H block (K chunk 16, one stage)
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

int64_t krg_tiles(const KrgArgs<float, float>& a, int64_t* tiles_c) {
  const int64_t rows = (int64_t)a.r.n_units * a.r.pad, cols = (int64_t)a.c.n_units * a.c.pad;
  const int64_t tr = (rows + BM - 1) / BM, tc = (cols + BN - 1) / BN;
  *tiles_c = tc;
  return a.symmetric ? tr * (tr + 1) / 2 : tr * tc;
}

void krg_persistent_launch(Exec& ex, const KrgJob* jobs_dev, int njobs, int64_t total, unsigned long long* counter,
                           double flops, double bytes) {
  if (total <= 0) return;
  if (!launch_ok(ex)) return;
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, ex.stream, counter);
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t grid = std::min<int64_t>(total, (int64_t)cus * 2);
  const int tok = prof_begin(ex, "krg_f32_persistent", flops, bytes);
  hipLaunchKernelGGL(krg_persistent, dim3((unsigned)grid), dim3(256), 0, ex.stream, jobs_dev, njobs, total, counter);
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
