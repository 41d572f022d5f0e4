// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace hs {

// Validated host view of a hess_mlp.
struct Model {
  int L = 0;
  int dtype = 0;
  std::vector<int64_t> T;
  std::vector<int> act;
  std::vector<const void*> W, b;
  std::vector<int64_t> offW, offb;  // flat offsets of W^(k+1) and b^(k+2)
  int64_t P = 0;
};

// FP64 per-example arrays.  Indexed by layer l (1-based); unused entries null.
struct Prep {
  int64_t N = 0;
  std::vector<double*> Abar;   // l = 1..L-1: N x lda[l], column T_l holds 1 (bias)
  std::vector<int64_t> lda;
  std::vector<double*> D1, D2, E;  // hidden l: N x T_l (sigma', sigma'', delta^(l+1) W^(l))
  std::vector<double*> delta;  // l = 2..L: N x T_l
  std::vector<double*> D1T, CT;  // hidden l: T_l x N (sigma', sigma'' * E), transposed
  std::vector<double*> W64, Wbar;  // k = 0..L-2: W^(k+1) (T x T) and [W | b]
  double* Yhat = nullptr;      // N x T_L
  double* PT = nullptr;        // T_L x N
  double* Z = nullptr;         // N x max T scratch
  int* flags = nullptr;
};

int64_t rup(int64_t x, int64_t m);
hess_status fail(hess_ctx* ctx, hess_status s, const std::string& msg);
hess_status validate_mlp(hess_ctx* ctx, const hess_mlp* m, Model& out, bool need_ptrs);
hess_status validate_data(hess_ctx* ctx, const hess_data* d, bool need_ptrs);
void plan_prep(Arena& ar, const Model& m, int64_t N, Prep& p, bool want_transposes);
hess_status check_inputs(Exec& ex, const Model& m, const hess_data* d, Prep& p);
void run_prep(Exec& ex, const Model& m, const hess_data* d, Prep& p, bool want_transposes);
void run_forward(Exec& ex, const Model& m, const void* X, int xdtype, Prep& p);
void run_backward(Exec& ex, const Model& m, Prep& p);
hess_status finish(Exec& ex, const char* what);
hess_status begin(hess_ctx* ctx, Exec& ex);
hess_status check_ws(hess_ctx* ctx, size_t need, void* ws, size_t ws_bytes, size_t out_bytes);

// Operands of the P x P contractions in the arithmetic precision.
template <typename T>
struct OpgBufs {
  std::vector<T*> abar, delta;
  __bf16* Jt = nullptr;
  int64_t ldk = 0;
};
template <typename T>
void plan_opg_ops(Arena& ar, const Model& m, int64_t N, const Prep& p, OpgBufs<T>& b);
template <typename T>
void cast_ops(Exec& ex, const Model& m, const Prep& p, OpgBufs<T>& b);
// Row/column side of the contraction for layer l (params W^(l-1), b^(l)).
template <typename T>
KrgSide<T> side_layer(const Model& m, int l, const T* abar, int64_t lda, const T* scale, int64_t ld_scale);
// Pair-diagonal block of column layer mm (the K term with l = mm + 1; units T_m, row slots
// T_{m+1}, column slots T_{m-1} + 1): FP32 workspace of its one-product form, which is used
// when that stays within kPairdiagMaxBytes (single and batched Hessians alike, so that the
// two agree bitwise).
int64_t pairdiag_block_floats(const Model& m, int64_t N, int mm);
constexpr int64_t kPairdiagMaxBytes = int64_t(2) << 30;

// Unit-direction R-operator factors of one column layer; see hess_api.hip.
struct HFactors {
  std::vector<double*> F, K, G;   // indexed by layer, layout [T_a][T_m][N]
};
void compute_factors(Exec& ex, const Model& m, int64_t Nc, int64_t n0, Prep& p, HFactors& f, int mm);

// A matrix split in three BF16 planes (h, m, l; x = h + m + l): part x of element (r, k)
// at p[x * plane + ps_off(r, k, nrb)] (blocks of 16 rows x 32 k in MFMA operand order, see
// mfma.h); k runs over kpad (a multiple of 32), zero past the true length; rows of the last
// block past the true count are never written.  See k_gemm_ps.hip.
struct SplitMat {
  __bf16* p = nullptr;
  int64_t nrb = 0, plane = 0, kpad = 0;  // row blocks of 16 (ps_off layout), plane length, k extent
};
// Takes the planes of a rows x kpad split matrix from an arena.
SplitMat take_split(Arena& ar, int64_t rows, int64_t kpad);
// dst = split of src (rows x K, row stride lds), k padded with zeros to dst.kpad.
void split_rows(Exec& ex, const float* src, int64_t rows, int64_t K, int64_t lds, SplitMat dst);
// dst = split of src^T (src: R x Cc, row stride lds; dst: Cc rows, k over R padded to dst.kpad).
void split_transpose(Exec& ex, const float* src, int64_t R, int64_t Cc, int64_t lds, SplitMat dst);
// C (M x N, row stride ldc) = alpha A B^T + beta C with A (M x K) and B (N x K) pre-split,
// K = A.kpad = B.kpad; FP32 accumulation of the six BF16 products of each product.
void gemm_presplit(Exec& ex, int64_t M, int64_t N, const SplitMat& A, const SplitMat& B, float alpha, float beta,
                   float* C, int64_t ldc);

// Buffers of the R-operator (dense-direction) passes; see hess_hvp.hip.
template <typename T>
struct HvpBufs {
  std::vector<T*> abar, delta, D1, CE, W, Vbar, HVbar, RZ, RA, RD;
  T* Yhat = nullptr;
  T* S = nullptr;
  T* Tacc = nullptr;  // T_l x (B T_{l-1}) partial of the delta^T R{A} accumulation
  int64_t Nc = 0, Bmax = 0;
  // split products (FP32 only): the shared operands of the large products split once,
  // per call (Vps: Vbar^(l)) or per chunk of examples (Aps: abar^(l-1) rows, ATps: its
  // transpose, RDps: R{delta^(l)} transposed, one layer at a time); empty where unused
  bool split = false;
  std::vector<SplitMat> Vps, Aps, ATps;
  SplitMat RDps;
  // one-pass R-backward step of a last hidden layer (FP32 split products): per-tile partials
  // of delta^(L)^T R{A^(L-1)} over 64-example tiles, summed by the accumulation
  T* RApart = nullptr;
};
template <typename T>
size_t plan_hvp(Arena& ar, const Model& m, int64_t N, int64_t B, Prep& p, HvpBufs<T>& h, bool split = false);
template <typename T>
void hvp_setup(Exec& ex, const Model& m, int64_t N, Prep& p, HvpBufs<T>& h);
template <typename T>
void hvp_apply(Exec& ex, const Model& m, int64_t N, int64_t B, Prep& p, HvpBufs<T>& h, const T* V, int64_t ldv,
               T* HV);
template <typename T>
void opg_apply(Exec& ex, const Model& m, int64_t N, int64_t B, Prep& p, HvpBufs<T>& h, const T* V, int64_t ldv,
               T* GV);
// JV[n][b] = (J v_b)_n = grad C_n . v_b for the per-example gradients held in the buffers.
template <typename T>
void jv_apply(Exec& ex, const Model& m, int64_t N, int64_t B, Prep& p, HvpBufs<T>& h, const T* V, int64_t ldv,
              T* JV);

// Workspace queries of the other translation units.
hess_status exact_cols_workspace(hess_ctx* ctx, const Model& m, int64_t N, int prec, int64_t ncols, size_t* bytes);
hess_status curvature_workspace(hess_ctx* ctx, int64_t K, int64_t nx, size_t* bytes);

// Dense symmetric eigen-decomposition (n <= 512), hess_syev.hip: w descending, U rows
// = eigenvectors (ldu), sign-normalised.  run_syev synchronises the stream once per
// recorded rotation chunk and returns false on a device error or QL non-convergence.
struct SyevBufs {
  int n = 0;
  double *A = nullptr, *Q = nullptr, *d = nullptr, *e = nullptr, *tau = nullptr, *rot = nullptr;
  int *st = nullptr, *perm = nullptr;
  int64_t cap = 0;
};
void plan_syev(Arena& ar, int n, SyevBufs& s);
bool run_syev(Exec& ex, const double* A, int64_t lda, double* w, double* U, int64_t ldu, SyevBufs& s);
hess_status syev_workspace(hess_ctx* ctx, int64_t n, size_t* bytes);

// Y part = Q M for a thin FP32 block (k_skinny.hip): part[s][b][P] over ks slices of
// kslice rows of M (P x P, row-major); the caller sums the slices in order.
void skinny_slices(int64_t P, int64_t b, int64_t& ks, int64_t& kslice);
void skinny_apply_f32(Exec& ex, const float* Q, int64_t b, int64_t P, const float* M, float* part, int64_t ks,
                      int64_t kslice);
hess_status hvp_workspace(hess_ctx* ctx, const Model& m, int64_t N, int prec, int64_t B, size_t* bytes);
hess_status topk_workspace(hess_ctx* ctx, const hess_mlp* mlp, const hess_data* d, int64_t K,
                           const hess_eig_opts* o, size_t* bytes);
hess_status predvar_workspace(hess_ctx* ctx, const Model& m, int prec, int64_t nq, size_t* bytes);
hess_status batched_workspace(hess_ctx* ctx, int64_t M, const hess_mlp* models, const hess_data* datas,
                              size_t* bytes);

}  // namespace hs
