// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <functional>
#include <string>
#include <vector>

#include "hess.h"

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

namespace hs {

// ---------------------------------------------------------------------------
// Workspace arena: a bump allocator over the caller's buffer.  With base ==
// nullptr it only counts, which is how hess_workspace_size is answered with the
// same planning code that later carves the real buffer.
// ---------------------------------------------------------------------------
struct Arena {
  char* base;
  size_t used = 0;
  explicit Arena(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

// Launch bookkeeping for one API call.
struct Exec {
  hipStream_t stream;
  hess_ctx* ctx;
  bool split = false;  // FP32 contractions take their products from split-BF16 MFMAs
};

bool launch_ok(Exec& ex);   // fault-injection hook + hipGetLastError check

// Autotuning: for a shape-class key, run each candidate launch (in-bounds, on a bounded
// sample of the work) twice, time the second run with HIP events on the call's stream
// and keep the fastest; the decision is cached per context.  Returns the candidate index.
int autotune_pick(Exec& ex, const std::string& key, int ncand, const char* const* names,
                  const std::function<void(int)>& launch);

// Profiling brackets around one launch (no-ops unless HESS_OPT_PROFILE is set).
int prof_begin(Exec& ex, const char* name, double flops, double bytes);
void prof_end(Exec& ex, int token);

// ---------------------------------------------------------------------------
// Generic strided GEMM on MFMA:  C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n)
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], C(m,n) = C[m*scm + n*scn],
// optional batch over blockIdx.z with element strides sab, sbb, scb.
// ---------------------------------------------------------------------------
template <typename T>
struct GemmArgs {
  int64_t M, N, K;
  const T* A; int64_t sam, sak, sab;
  const T* B; int64_t sbk, sbn, sbb;
  T* C; int64_t scm, scn, scb;
  T alpha, beta;
  int64_t batch;
};
template <typename T>
void gemm(Exec& ex, const GemmArgs<T>& g);

// Convenience: row-major C[M x N] = alpha * op(A) op(B) + beta C with leading dims.
template <typename T>
void gemm_rm(Exec& ex, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha,
             const T* A, int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc);

// ---------------------------------------------------------------------------
// Khatri-Rao Gram contraction (the H and OPG tiles).
//
// Compute space: a row index r = ur * r.pad + sr names unit ur and slot sr of the
// row side (likewise for columns).  For every valid (r, c):
//   acc(r,c) = sum_n w_n(ur,uc) * Rsrc[n, sr] * Csrc[n, sc]
// where w_n(ur,uc) is
//   RANK1:     rscale[n, ur] * cscale[n, uc]  (either factor may be absent = 1)
//   PAIR_FULL: wts[(ur * c.n_units + uc) * ldw + n]
//   PAIR_DIAG: wts[ur * ldw + n] if ur == uc, else 0
// and the result scale * acc is stored to out[flat_r * ldo + flat_c] (and mirrored
// to out[flat_c * ldo + flat_r]).  flat(u, s) is the flat parameter index of
// (unit i, input j) in a layer with Tout units and Tin inputs: with perm = 0,
// (i, j) = (u, s), with perm = 1, (i, j) = (s, u); j == Tin denotes the bias.
// ---------------------------------------------------------------------------
enum { KRG_RANK1 = 0, KRG_PAIR_FULL = 1, KRG_PAIR_DIAG = 2 };

template <typename T>
struct KrgSide {
  const T* src; int64_t ld;       // N x ld source rows
  int32_t n_units, len, pad;      // units, valid slots per unit, padded slots per unit
  const T* scale; int64_t ld_scale;  // RANK1 per-(n, unit) factor or nullptr
  int32_t perm; int64_t off; int32_t Tin, Tout;  // output index map
};

template <typename T, typename TOut>
struct KrgArgs {
  KrgSide<T> r, c;
  int32_t wmode;
  const T* wts; int64_t ldw;
  TOut* out; int64_t ldo;
  int32_t symmetric, accumulate, mirror;
  double scale;
  int64_t N;
  // Split over examples: slice s covers examples [s * kslice, min(N, (s + 1) * kslice))
  // and writes its partial result at out + s * out_split (one launch for all slices).
  int32_t ksplit = 1;
  int64_t kslice = 0, out_split = 0;
  const char* label = nullptr;  // profile name (default: by weight mode and precision)
  // Column source already split into three BF16 parts (bsplit layout, blocks of 32
  // slots; bp_nblk = c.pad / 32), read by the split-product tile instead of splitting
  // the FP32 columns in every wavefront; nullptr: split in the tile.
  const uint32_t* bparts = nullptr;
  int32_t bp_nblk = 0;
  // Per column tile (128 columns) the examples with a nonzero weight for some pair of the
  // tile, in increasing order: klist[t * ldl + i] for i < kcnt[t], padded with example 0
  // to whole chunks of 32 (ldl a multiple of 32, at least N rounded up).  With split products
  // on a pair-weighted contraction the tile then sums over those examples only (the others
  // contribute exact zeros); nullptr: every example.
  const int32_t* klist = nullptr;
  const int64_t* kcnt = nullptr;
  int64_t ldl = 0;
  // Symmetric contractions: per unit pair (u >= v, index u (u + 1) / 2 + v) the examples with
  // a nonzero weight w[u][v][n], same layout (row stride ldl); a tile whose rows lie in one
  // unit and columns in one unit sums over its pair's list instead; nullptr: column lists only.
  const int32_t* plist = nullptr;
  const int64_t* pcnt = nullptr;
  // Symmetric contractions: per row tile the examples where one of its row units has a
  // nonzero weight with some column unit (same layout); a tile that spans two units on a side
  // sums over the shorter of its row tile's and column tile's lists; nullptr: column lists.
  const int32_t* rlist = nullptr;
  const int64_t* rcnt = nullptr;
};
// The example lists above for a pair-weighted contraction, from its weights: flags (column
// units x N bytes) marks the examples of each column unit with a nonzero weight for some row
// unit, then each column tile gathers the examples flagged for any of its units.
int64_t krg_list_tiles(const KrgArgs<float, float>& a);
void krg_build_lists(Exec& ex, const KrgArgs<float, float>& a, uint8_t* flags, int32_t* lists, int64_t* cnt,
                     int64_t ldl);
// The row-tile lists above (symmetric contraction: r and c the same units), through flags.
void krg_build_row_lists(Exec& ex, const KrgArgs<float, float>& a, uint8_t* flags, int32_t* lists, int64_t* cnt,
                         int64_t ldl);
// The unit-pair lists above (symmetric contraction: r and c the same units).
void krg_build_pair_lists(Exec& ex, const KrgArgs<float, float>& a, int32_t* lists, int64_t* cnt, int64_t ldl);
// Pair-diagonal contraction (KRG_PAIR_DIAG, FP32) as one product instead of tiles:
// out[row(u, s)][col(u, b)] (+)= scale * sum_n w[u][n] r.src[n][s] c.src[n][b] for units
// u < min(r.n_units, c.n_units), through Y[n][u len_r + s] = w[u][n] r.src[n][s] (N x U len_r),
// PD_SLICES partial products Y^T c.src over slices of the examples, and a scatter that sums
// them (mirrored if a.mirror).  Workspace: pairdiag_floats(a) floats.
constexpr int PD_SLICES = 8;
int64_t pairdiag_floats(int64_t N, int64_t U, int64_t len_r, int64_t len_c);
void krg_pairdiag_gemm(Exec& ex, const KrgArgs<float, float>& a, float* ws);
// Three-way BF16 split of an N x len column source (row stride ld) into the chunked
// fragment layout read by the split-product tile: per chunk of 32 examples, per part
// (h, m, l), per block of 32 slots, 512 dwords ordered [slot / 16 % 2][example / 8 % 4]
// [slot % 16][example pair % 4], each dword two BF16 values of consecutive examples.
// Slots >= len and examples >= N are zero.  Size: bsplit_dwords(N, pad) dwords.
int64_t bsplit_dwords(int64_t N, int32_t pad);
void bsplit(Exec& ex, const float* src, int64_t ld, int32_t len, int32_t pad, int64_t N, uint32_t* out);
template <typename T, typename TOut>
void krg(Exec& ex, const KrgArgs<T, TOut>& a);
// Several contractions (FP32) through one persistent launch; jobs_dev is a device array.
struct KrgJob {
  KrgArgs<float, float> a;
  int64_t tiles_c, first;  // column tiles; index of the job's first tile in the global order
  int32_t mode;            // KRG_* weight mode
};
int64_t krg_tiles(const KrgArgs<float, float>& a, int64_t* tiles_c);
// Units-per-tile bound of a contraction's tile (2, 5 or 9); the persistent launch runs
// jobs of one bound together.
int krg_persistent_maxu(const KrgArgs<float, float>& a);
// Whether a contraction can run in the persistent launch (its copy offsets fit 32 bits).
bool krg_persistent_fits(const KrgArgs<float, float>& a);
// One persistent launch over jobs of one units-per-tile bound maxu; counters: 8 device
// words (zeroed by the launch).  cfg: 0 = (16 examples, 2 stages), 1 = (16, 3),
// 2 = (32, 2), 3 = split-BF16 products (32, 2); every FP32 configuration gives the same bits.
void krg_persistent_launch(Exec& ex, const KrgJob* jobs_dev, int njobs, int64_t total, unsigned long long* counters,
                           double flops, double bytes, int maxu, int cfg);
// Tile-configuration variants (tuning and tests): register-staged tile 1..4 = (K chunk,
// LDS stages) in {(16,1), (16,2), (32,1), (32,2)}; FP32 LDS-staged tile 5 = (32, 2),
// 6 = (16, 3); split products 7 = columns split in the tile, 8 = pre-split columns
// (a.bparts); 0 = the default for the precision (FP32: LDS-staged (16, 2)).
template <typename T, typename TOut>
void krg_variant(Exec& ex, const KrgArgs<T, TOut>& a, int variant);
// BF16 OPG: materialise Jt (P x ldk, BF16, p-major) then one symmetric Gram product.
constexpr int JT_MAXL = 16;
struct JtArgs {
  __bf16* Jt; int64_t ldk; int64_t P; int64_t N; int nlayers;
  const float* delta[JT_MAXL]; int64_t ld_delta[JT_MAXL];   // per weight layer k: delta^(k+2) (N x T)
  const float* abar[JT_MAXL]; int64_t ld_abar[JT_MAXL];     // abar^(k+1) (N x lda, bias column = 1)
  int64_t offW[JT_MAXL]; int32_t Tin[JT_MAXL], Tout[JT_MAXL];
};
void jt_bf16(Exec& ex, const JtArgs& a);
int64_t jt_ld(int64_t N);
void gram_bf16(Exec& ex, const __bf16* Jt, int64_t P, int64_t ldk, int64_t N, float scale, float* C, int64_t ldc);
// variant 1: register-staged Gram kernel; 2: LDS-staged with 32-example chunks in 4 stages;
// 3: LDS-staged (64, 2) with each chunk's copies issued together after the barrier;
// otherwise LDS-staged (64, 2) with the copies spread over the MFMA rows (default)
void gram_bf16_variant(Exec& ex, const __bf16* Jt, int64_t P, int64_t ldk, int64_t N, float scale, float* C,
                       int64_t ldc, int variant);

// ---------------------------------------------------------------------------
// Element-wise and small kernels (k_elem.hip).
// ---------------------------------------------------------------------------
void check_finite(Exec& ex, const void* p, int dtype, int64_t n, int* flag);
void check_onehot(Exec& ex, const void* Y, int dtype, int64_t N, int64_t C, int* flag);
void check_cls(Exec& ex, const int32_t* cls, int64_t n, int64_t C, int* flag);
// dst[n*ldd + j] = (double) src[n*lds + j] for j < cols; optional bias column of ones at j == cols
void to_f64_rows(Exec& ex, const void* src, int dtype, int64_t rows, int64_t cols, int64_t lds,
                 double* dst, int64_t ldd, int bias_one);
// Wbar = [W | b] (Tout x (Tin+1)) in FP64
void make_wbar(Exec& ex, const void* W, const void* b, int dtype, int64_t Tout, int64_t Tin,
               double* Wbar);
// hidden activation: from Z (N x T) write Abar (N x ldab, bias column = 1), D1, D2 (N x T)
void activate(Exec& ex, int act, const double* Z, int64_t N, int64_t T, double* Abar,
              int64_t ldab, double* D1, double* D2);
// softmax rows (one wavefront per row): Yhat = softmax(Z)
void softmax_rows(Exec& ex, const double* Z, int64_t N, int64_t T, double* Yhat);
// delta^(L) = Yhat - Y
void output_delta(Exec& ex, const double* Yhat, const void* Y, int dtype, int64_t N, int64_t T,
                  double* delta);
// c[i] = a[i] * b[i]
void mul(Exec& ex, const double* a, const double* b, double* c, int64_t n);
// dst (cols x rows) = transpose of src (rows x cols, leading dim lds), optional elementwise product with src2
void transpose(Exec& ex, const double* src, int64_t rows, int64_t cols, int64_t lds, double* dst,
               int64_t ldd);
template <typename TD>
void cast_copy(Exec& ex, const double* src, TD* dst, int64_t n);
// dst[0 .. n) = 0 (a kernel, so that it may also run inside captured sequences); n may be 0
template <typename TD>
void fill_zero(Exec& ex, TD* dst, int64_t n);
// examples per chunk of the split-product tile; its FP32 row sources hold whole chunks
constexpr int64_t kSrcRows = 32;
// strided 2D cast: dst[r*ldd + c] = (TD) src[r*lds + c]
template <typename TD>
void cast_2d(Exec& ex, const double* src, int64_t rows, int64_t cols, int64_t lds, TD* dst, int64_t ldd);
// Curvature-factor helpers on the [T_a][T_m][N] layout (n fastest, N examples of a chunk);
// the per-example caches D1T, CT, PT are [T][ldc] (ldc = the full example count), passed
// already offset to the chunk's first example.
// F[i2][i][n] = W[i2*ldw + i] * D1T[i][n]
void factor_first(Exec& ex, const double* W, int64_t T2, int64_t Tm, const double* D1T, int64_t ldc, int64_t N,
                  double* F);
// K[k][i][n] = D1T[k][n] * F[k][i][n]
void factor_rowscale(Exec& ex, const double* F, int64_t Tk, int64_t Tm, const double* D1T, int64_t ldc, int64_t N,
                     double* K);
// G[k][i][n] = p[k][n] * (F[k][i][n] - sum_k' p[k'][n] F[k'][i][n]); F == nullptr means identity
void factor_softmax(Exec& ex, const double* F, int64_t TL, int64_t Tm, const double* PT, int64_t ldc, int64_t N,
                    double* G);
// G[k][i][n] = D1T[k][n] * G[k][i][n] + CT[k][n] * (F ? F[k][i][n] : (k == i))
void factor_combine(Exec& ex, double* G, int64_t Tk, int64_t Tm, const double* D1T,
                    const double* CT, int64_t ldc, const double* F, int64_t N);

}  // namespace hs

struct hess_prof_rec {
  int agg;
  hipEvent_t a, b;
  double flops, bytes;
};
struct hess_prof_agg {
  std::string name;
  int64_t launches = 0;
  double ms = 0, flops = 0, bytes = 0;
};

struct hess_ctx {
  int profile = 0;
  std::vector<hess_prof_rec> pending;
  std::vector<hipEvent_t> event_pool;
  std::vector<hess_prof_agg> aggs;
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  int check_inputs = 1;
  int64_t hbm_budget = 0;
  int64_t fault_after = -1;
  int64_t launches = 0;
  bool fault_hit = false;
  int graphs = 1;                       // capture repeated operator applications as HIP graphs
  int autotune = 0;                     // time the tile configurations per shape class
  int64_t factor_cap = 0;               // hess_exact factor-region cap in bytes (0 = default)
  std::vector<std::pair<std::string, int>> tuned;  // shape class -> chosen configuration
  std::string tune_log;                 // one line per decision
  hipStream_t capture_stream = nullptr;  // created on first capture (graphs cannot be captured on the null stream)
};
