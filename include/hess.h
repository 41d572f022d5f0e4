/*
 * hess.h -- C ABI of the MI355X (gfx950) library for the exact Hessian, the
 * Outer-Product-of-Gradients (OPG) matrix and their leading eigenpairs for the
 * mean softmax cross-entropy cost of a dense feed-forward network.
 *
 * Model and notation (paper, Sec. 2): layers l = 1..L with widths T_l; weights
 * W^(l-1) in R^{T_l x T_{l-1}}, biases b^(l) in R^{T_l}; hidden activations
 * sigma^(l) (l = 2..L-1); softmax output; cost C = (1/N) sum_n C_n, the mean
 * per-example cross-entropy against one-hot targets y_n.
 *
 * Parameter layout (paper, Sec. 2, the flatten definition): every P-vector and
 * every P x P matrix uses the flat order W^(1) row-major (index i*T_1 + j, i the
 * output unit, j the input unit), then b^(2), then W^(2), b^(3), ...
 * P = T_1 T_2 + T_2 + ... + T_{L-1} T_L + T_L.
 *
 * Conventions for every entry point:
 *   - All array arguments marked "device" are device pointers on the context's
 *     device; the caller owns them.  "host" arrays are read during the call only.
 *   - Work is issued on the context's stream.  Every call returns after its
 *     results are in device memory (it synchronises the stream), so results can be
 *     read on any stream afterwards.
 *   - Scratch memory is supplied by the caller as (ws, ws_bytes); the required size
 *     comes from hess_workspace_size.  The library allocates no device memory.
 *   - Arguments are validated before any work is launched.  On any error the
 *     outputs are unspecified, nothing else changes, and hess_last_error gives a
 *     message.  A context is not thread-safe: use one context per host thread.
 */
#ifndef HESS_H
#define HESS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hess_ctx hess_ctx;

typedef enum {
  HESS_OK = 0,
  HESS_E_ARG = 1,         /* null pointer or enum out of range */
  HESS_E_SHAPE = 2,       /* L < 2, a width < 1, N < 1, K/B out of range, P overflow */
  HESS_E_LABEL = 3,       /* a row of Y is not exactly one-hot */
  HESS_E_NONFINITE = 4,   /* NaN or Inf in an input array */
  HESS_E_WORKSPACE = 5,   /* ws is NULL or ws_bytes below hess_workspace_size */
  HESS_E_BUDGET = 6,      /* footprint above the context's HBM budget */
  HESS_E_DEVICE = 7,      /* HIP runtime error (or the injected test fault) */
  HESS_E_NOCONV = 8,      /* eigensolver reached max_iter; best iterate returned */
  HESS_E_NOTPD = 9,       /* lambda_k + delta <= 0 in the damped query */
  HESS_E_UNSUPPORTED = 10 /* precision not offered for this operation */
} hess_status;

typedef enum { HESS_TANH = 0, HESS_SIGMOID = 1, HESS_RELU = 2 } hess_act;

/* Storage type of W, b, X, Y (and V, Q where stated). */
typedef enum { HESS_F64 = 0, HESS_F32 = 1 } hess_dtype;

/* Arithmetic of the P x P contractions.  The per-example forward/backward
 * passes and curvature factors are always computed in FP64.
 *   HESS_P_F64   FP64 MFMA, FP64 output
 *   HESS_P_F32   FP32 MFMA with FP32 accumulation, FP32 output
 *   HESS_P_BF16  OPG only: per-example gradient tiles rounded to BF16 (round to
 *                nearest even), BF16 MFMA with FP32 accumulation, FP32 output
 *   HESS_P_F32_SPLIT  hess_exact and hess_opg: as HESS_P_F32 (FP32 operands, FP32
 *                accumulation and output), but the FP32 contractions take each product
 *                from BF16 MFMAs on compensated three-way splits of the FP32 operands
 *                (x = h + m + l, each part the round-to-nearest-even BF16 of the remainder;
 *                products h h, h m, m h, h l, l h, m m), which keeps FP32-level error.
 *                hess_hvp, hess_hvp_prepare, hess_exact_cols and the matrix-free operator
 *                of hess_topk_eig accept it too (their FP32 GEMMs take split products,
 *                except contractions of at most 128 terms, which use FP32 MFMAs), and so
 *                does hess_batched. */
typedef enum { HESS_P_F64 = 0, HESS_P_F32 = 1, HESS_P_BF16 = 2, HESS_P_F32_SPLIT = 3 } hess_prec;

typedef struct {
  int32_t L;               /* number of layers including the input layer, L >= 2 */
  const int64_t* T;        /* host, T[0..L-1] = T_1..T_L, each >= 1 */
  const int32_t* act;      /* host, act[0..L-3] = sigma^(2)..sigma^(L-1) (hess_act) */
  int32_t dtype;           /* hess_dtype of every W[k] and b[k] */
  const void* const* W;    /* host array of L-1 device pointers: W[k] = W^(k+1), T_{k+2} x T_{k+1} row-major */
  const void* const* b;    /* host array of L-1 device pointers: b[k] = b^(k+2), T_{k+2} entries */
} hess_mlp;

typedef struct {
  int64_t N;               /* number of examples, >= 1 */
  int32_t dtype;           /* hess_dtype of X and Y */
  const void* X;           /* device, N x T_1 row-major */
  const void* Y;           /* device, N x T_L row-major, every row exactly one-hot */
} hess_data;

/* Operation codes for hess_workspace_size. */
typedef enum {
  HESS_OP_EXACT = 0, HESS_OP_OPG = 1, HESS_OP_HVP = 2, HESS_OP_TOPK = 3, HESS_OP_PREDVAR = 4,
  HESS_OP_BATCHED = 5, HESS_OP_EXACT_COLS = 6, HESS_OP_CURVATURE = 7, HESS_OP_SYEV = 8
} hess_op;

/* Create a context on `device`; `stream` is a hipStream_t (NULL = the null stream). */
hess_status hess_create(hess_ctx** ctx, int device, void* stream);
hess_status hess_destroy(hess_ctx* ctx);
const char* hess_status_str(hess_status s);
/* Message describing the last error on this context ("" if none). */
const char* hess_last_error(const hess_ctx* ctx);

/* Context options.  HESS_OPT_CHECK_INPUTS (default 1): run the device-side
 * finiteness / one-hot check pass before each call.  HESS_OPT_HBM_BUDGET: bytes of
 * outputs + workspace a call may touch (0 = unlimited); above it a call returns
 * HESS_E_BUDGET before launching anything.  HESS_OPT_FAULT_AFTER: test hook; when
 * >= 0, the call during which that many kernel launches have been issued on this
 * context reports HESS_E_DEVICE (no kernel faults; the launch is skipped). */
/* HESS_OPT_GRAPHS (default 1): inside hess_topk_eig, the operator application (the
 * sweep of Hessian-vector products, OPG products or the dense product) for each pair
 * of block buffers is captured once as a HIP graph and replayed for every later
 * application; results are bitwise the same as without graphs.  Graphs are not used
 * while HESS_OPT_PROFILE or HESS_OPT_FAULT_AFTER is active.
 * HESS_OPT_AUTOTUNE (default 0): the first FP32 contraction launch and the first BF16
 * Gram product of each shape class times every tile configuration of that kernel
 * (example chunk and LDS stage count) on a bounded sample of its tiles, synchronising
 * the stream, and caches the choice for the context: the default configuration unless
 * another is at least 3% faster on the sample (contractions that accumulate into their
 * output keep the default); all configurations give bitwise identical results.
 * hess_autotune_report lists the decisions. */
/* HESS_OPT_FACTOR_BYTES (default 0 = 32 GiB): cap on the bytes of hess_exact's per-example
 * curvature factors (about sum T_l T_m N doubles per column layer m).  Above it hess_exact
 * runs the factor computation and the contraction over chunks of examples (a multiple of
 * 32, at least 32) and accumulates H chunk by chunk, the mini-batch sum of Sec. 5.1; the
 * workspace then holds one chunk's factors.  Results agree with the one-pass H to FP
 * rounding (the sum over examples is split at the chunk boundaries). */
typedef enum {
  HESS_OPT_CHECK_INPUTS = 0, HESS_OPT_HBM_BUDGET = 1, HESS_OPT_FAULT_AFTER = 2, HESS_OPT_PROFILE = 3,
  HESS_OPT_GRAPHS = 4, HESS_OPT_AUTOTUNE = 5, HESS_OPT_FACTOR_BYTES = 6
} hess_opt;
hess_status hess_set_option(hess_ctx* ctx, int opt, int64_t value);

/* Text report of the autotuning decisions of this context, one line per shape class
 * (candidate times in ms and the choice).  Writes at most len bytes including the
 * terminating NUL into buf (host memory, may be NULL); *needed (may be NULL) receives
 * the full length + 1. */
hess_status hess_autotune_report(hess_ctx* ctx, char* buf, size_t len, size_t* needed);

/* Per-kernel timing.  With HESS_OPT_PROFILE = 1 every P x P contraction and every
 * GEMM launch is bracketed by HIP events on the context stream; the elapsed times
 * are collected when the call synchronises.  hess_profile_read copies up to
 * max_entries aggregates (one per kernel class, since the last reset) to `out`
 * and returns the number of classes; flops and bytes are the algorithmic counts
 * of the launches (2 flops per multiply-add; bytes = operands read once plus
 * outputs written). */
typedef struct {
  char name[48];
  int64_t launches;
  double ms;
  double flops;
  double bytes;
} hess_prof_entry;
int hess_profile_read(hess_ctx* ctx, hess_prof_entry* out, int max_entries);
hess_status hess_profile_reset(hess_ctx* ctx);

/* P of the model (Sec. 2).  Host-only; validates the widths. */
hess_status hess_num_params(const hess_mlp* m, int64_t* P);

/* Bytes of workspace `op` needs.  `arg` is B for HESS_OP_HVP, ncols for
 * HESS_OP_EXACT_COLS, nx for HESS_OP_CURVATURE (opts: const int64_t* K), n for HESS_OP_SYEV,
 * K for HESS_OP_TOPK,
 * the number of queries for HESS_OP_PREDVAR, the number of networks M for
 * HESS_OP_BATCHED (then `m` and `d` point to arrays of M entries), unused otherwise.
 * For HESS_OP_TOPK `opts` is a const hess_eig_opts*, else NULL.  `data` may be NULL
 * for HESS_OP_PREDVAR and for HESS_OP_TOPK with a dense source. */
hess_status hess_workspace_size(hess_ctx* ctx, int op, const hess_mlp* m, const hess_data* d,
                                int prec, int64_t arg, const void* opts, size_t* bytes);

/* Exact Hessian H = (1/N) sum_n d^2 C_n / d omega d omega^T (paper, Sec. 3, the
 * Hessian definition), assembled from forward-over-reverse Hessian-vector products
 * (Sec. 5.1, Appendix A.1) through every layer's W, b and sigma.
 * H: device, P x P row-major, FP64 for HESS_P_F64 else FP32; exactly symmetric
 * (every entry below the diagonal is computed once and mirrored).
 * prec: HESS_P_F64, HESS_P_F32 or HESS_P_F32_SPLIT (HESS_P_BF16 -> HESS_E_UNSUPPORTED).
 * With FP32 operands the workspace also holds the block between a layer's weights and
 * the previous layer's weights as one product (N T_m T_{m+1} + 8 T_m T_{m+1} (T_{m-1} + 1)
 * floats, where that stays within 2 GiB).  With HESS_P_F32_SPLIT it also holds one
 * layer's inputs at a time split into BF16 parts, sized for the largest layer that
 * qualifies (inputs plus bias padded to a multiple of 32 and at least 128): about
 * 6 N (T_{m-1} + 1) bytes.  For a ReLU hidden layer m of that kind it also holds, per
 * 128-column tile and per unit pair, the list of examples with a nonzero curvature weight
 * (about 4 N (T_m (T_{m-1} + 1) / 128 + T_m (T_m + 1) / 2) + N T_m bytes): the weighted
 * sums of those blocks skip the examples where a unit is inactive, whose weights are
 * exact zeros (the result changes only by the grouping of FP32 additions). */
hess_status hess_exact(hess_ctx* ctx, const hess_mlp* m, const hess_data* d, int prec,
                       void* H, void* ws, size_t ws_bytes);

/* OPG = (1/N) sum_n grad C_n grad C_n^T = J^T J / N with J[n,:] = grad C_n
 * (paper, Sec. 3, the OPG definition and its Jacobian form).  For HESS_P_F64 and
 * HESS_P_F32 the tiles of J are formed in LDS from the per-example factors and J
 * is never stored; for HESS_P_BF16 J^T is formed once in BF16 in the workspace
 * (P x N x 2 bytes) and contracted as one symmetric Gram product.
 * G: device, P x P row-major, FP64 for HESS_P_F64 else FP32, exactly symmetric. */
hess_status hess_opg(hess_ctx* ctx, const hess_mlp* m, const hess_data* d, int prec,
                     void* G, void* ws, size_t ws_bytes);

/* Hessian-vector products for B directions (paper, Sec. 5.1 and Appendix A.1):
 * HV[b,:] = H V[b,:].  V, HV: device, B x P row-major (direction-contiguous), FP64
 * for HESS_P_F64 else FP32.  prec: HESS_P_F64, HESS_P_F32 or HESS_P_F32_SPLIT
 * (HESS_P_BF16 -> HESS_E_UNSUPPORTED). */
hess_status hess_hvp(hess_ctx* ctx, const hess_mlp* m, const hess_data* d, int prec,
                     int64_t B, const void* V, void* HV, void* ws, size_t ws_bytes);

/* Curvature operators from K eigenpairs (lambda descending, Q K x P row-major, FP64,
 * e.g. from hess_topk_eig) applied to nx vectors X (nx x P row-major, FP64), never
 * forming a P x P matrix.  Low rank (paper, Sec. 5.5): H~ = Q^T diag(lambda) Q.  Full
 * rank (Sec. 5.6, App. A.2): H~~ = H~ + lt (I - Q^T Q), lt = lam_tilde (the paper's
 * choice is lambda_K); Q's rows must be orthonormal.  Modes:
 *   HESS_CURV_LOW_QUAD    out[i] = x_i^T H~ x_i          (out: nx)
 *   HESS_CURV_FULL_QUAD   out[i] = x_i^T H~~ x_i         (out: nx)
 *   HESS_CURV_LOW_APPLY   out[i,:] = H~ x_i              (out: nx x P)
 *   HESS_CURV_FULL_APPLY  out[i,:] = H~~ x_i             (out: nx x P)
 *   HESS_CURV_FULL_INV    out[i,:] = H~~^{-1} x_i        (out: nx x P)
 * All device pointers; ws: hess_workspace_size(HESS_OP_CURVATURE, arg = nx, opts = const
 * int64_t* K).  Errors: HESS_E_SHAPE (K < 1, P < K, nx < 1), HESS_E_NONFINITE (lambda or
 * lam_tilde), HESS_E_NOTPD (inverse with some lambda_k <= 0 or lam_tilde <= 0). */
typedef enum {
  HESS_CURV_LOW_QUAD = 0, HESS_CURV_FULL_QUAD = 1, HESS_CURV_LOW_APPLY = 2, HESS_CURV_FULL_APPLY = 3,
  HESS_CURV_FULL_INV = 4
} hess_curv_mode;
hess_status hess_curvature(hess_ctx* ctx, int mode, int64_t K, int64_t P, const double* lambda, const double* Q,
                           double lam_tilde, int64_t nx, const double* X, double* out, void* ws, size_t ws_bytes);

/* hess_curvature without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same modes, arguments, results and errors as hess_curvature, computed by
 * the same kernels; the scratch (2 nx K + nx doubles, 256-byte aligned per array) lives
 * in a library-owned 16 MiB device array, one per device, held until the process ends.
 * HESS_E_WORKSPACE if 2 nx K + nx doubles exceed it (e.g. nx K above about 1.04e6).
 * The call allocates nothing.  Every call on a device shares that device's array:
 * calls that overlap on one device (other host threads, other contexts) race and must
 * be serialised by the caller. */
hess_status hess_curvature_noalloc(hess_ctx* ctx, int mode, int64_t K, int64_t P, const double* lambda,
                                   const double* Q, double lam_tilde, int64_t nx, const double* X, double* out);

/* Eigen-decomposition of a dense symmetric n x n FP64 matrix on the device, the
 * projected problem of the Lanczos eigensolver (paper, Sec. 5.3), 1 <= n <= 512.
 * A: device, row-major with row stride lda >= n, used as (A + A^T) / 2, not modified.
 * w: device, n eigenvalues, descending.  U: device, n x n row-major, row j = unit
 * eigenvector of w[j], largest-magnitude component positive.  Householder
 * tridiagonalisation, then implicit-shift QL; synchronises the call's stream.
 * ws: hess_workspace_size(HESS_OP_SYEV, arg = n).  Errors: HESS_E_SHAPE (n, lda),
 * HESS_E_NOCONV (more than 60 QL iterations for one eigenvalue, e.g. non-finite A). */
hess_status hess_syev(hess_ctx* ctx, int64_t n, const double* A, int64_t lda, double* w, double* U, void* ws,
                      size_t ws_bytes);

/* Prepared HVP operator: the per-example passes of hess_hvp (forward and backward over
 * all N examples, paper Sec. 2-3) run once, then hess_hvp_apply forms H V for any number
 * of blocks of up to max_B directions without repeating them (paper, Sec. 5.1 and
 * Appendix A.1).  ws (device, caller-owned, size hess_workspace_size(HESS_OP_HVP) with
 * arg = max_B) holds the prepared state and must stay allocated and untouched until
 * hess_hvp_release; m's weights and d's X, Y are not read after hess_hvp_prepare.
 * V, HV: device, B x P row-major, FP64 for HESS_P_F64 else FP32, B <= max_B.
 * Errors: as hess_hvp; HESS_E_SHAPE for B outside 1..max_B. */
typedef struct hess_hvp_op hess_hvp_op;
hess_status hess_hvp_prepare(hess_ctx* ctx, const hess_mlp* m, const hess_data* d, int prec, int64_t max_B,
                             void* ws, size_t ws_bytes, hess_hvp_op** op);
hess_status hess_hvp_apply(hess_ctx* ctx, hess_hvp_op* op, int64_t B, const void* V, void* HV);
hess_status hess_hvp_release(hess_hvp_op* op);

/* Columns col0 .. col0 + ncols - 1 of the exact H (paper, Sec. 5.1: the Hessian-vector
 * product with the j-th unit vector is column j of H), computed as HVPs with basis
 * directions in blocks of up to 512 columns.  Hcols: device, P x ncols row-major, FP64
 * for HESS_P_F64 else FP32.  prec: HESS_P_F64, HESS_P_F32 or HESS_P_F32_SPLIT.
 * Errors: HESS_E_SHAPE if the column range is empty or leaves [0, P); otherwise as
 * hess_hvp. */
hess_status hess_exact_cols(hess_ctx* ctx, const hess_mlp* m, const hess_data* d, int prec,
                            int64_t col0, int64_t ncols, void* Hcols, void* ws, size_t ws_bytes);

typedef struct {
  int32_t which;        /* 0 = H, 1 = OPG (used when source == 0) */
  int32_t source;       /* 0 = matrix-free operator from (m, d); 1 = dense symmetric M */
  const void* M;        /* source == 1: device, P x P row-major symmetric */
  int32_t M_dtype;      /* source == 1: hess_dtype of M */
  int32_t prec;         /* source == 0: hess_prec of the operator (HESS_P_F64, HESS_P_F32 or
                           HESS_P_F32_SPLIT) */
  int64_t P;            /* source == 1: order of M (m may be NULL) */
  int64_t oversample;   /* block size b = roundup(K + oversample, 16); default 10 if < 0 */
  int32_t max_iter;     /* cap on subspace iterations (default 200 if <= 0) */
  double tol;           /* stop when max_k ||M q_k - theta_k q_k|| <= tol * |theta_1| */
  uint64_t seed;        /* seed of the counter-based start block */
  int32_t method;       /* 0 = filtered subspace iteration; 1 = thick-restart block Lanczos */
  int32_t block;        /* method 1: Lanczos block size (default 32 if <= 0, at most 128) */
} hess_eig_opts;

typedef struct {
  int32_t iters;             /* subspace iterations run (method 1: restarts) */
  int32_t applies;           /* operator applications (block products; method 1: blocks of `block`) */
  double max_rel_residual;   /* max_k ||M q_k - theta_k q_k|| / |theta_1| at exit */
  double shift_used;         /* spectral shift used for the algebraically-largest search */
} hess_eig_info;

/* K algebraically largest eigenpairs of H or the OPG (paper, Sec. 4.1, 5.3, 5.4:
 * which='LA', sorted descending).  method 0: randomized subspace iteration with a
 * Chebyshev filter, FP64 Cholesky-QR re-orthogonalisation and FP64 Rayleigh-Ritz
 * (K + oversample <= 128).  method 1: block Lanczos (the paper's solver, Sec. 5.3)
 * with full FP64 re-orthogonalisation, thick restarts and locking of converged
 * pairs; window min(512, 3K + 3b, P - b) basis vectors (must be >= K + 2b), a final
 * Rayleigh-Ritz over the K locked vectors gives the reported pairs and residuals;
 * max_iter caps the restarts.
 * lambda: device, K doubles, descending.  Q: device, K x P row-major doubles
 * (row k = eigenvector k, orthonormal, largest-|.| component positive).
 * Returns HESS_E_NOCONV (with the best iterate written) at max_iter. */
hess_status hess_topk_eig(hess_ctx* ctx, const hess_mlp* m, const hess_data* d, int64_t K,
                          const hess_eig_opts* opts, double* lambda, double* Q,
                          hess_eig_info* info, void* ws, size_t ws_bytes);

/* Damped curvature query (Laplace-style predictive variance) for nq inputs:
 * s_q = g_q^T (Q^T diag(lambda) Q + delta I)^{-1} g_q with g_q = d z^(L)_{c_q}(x_q)/d omega,
 * evaluated as sum_k (q_k.g)^2/(lambda_k+delta) + (|g|^2 - sum_k (q_k.g)^2)/delta
 * (the full-rank construction of Sec. 4.2 / Appendix A.2 with the complement
 * eigenvalue delta).  Xq: device, nq x T_1 (dtype m->dtype); cls: device int32
 * nq entries (-1 = arg-max of the prediction, lowest index on ties) or NULL
 * (all arg-max); lambda: device K doubles; Q: device K x P row-major doubles
 * (orthonormal rows); s: device nq doubles.  HESS_E_NOTPD if lambda_k + delta <= 0. */
hess_status hess_predvar(hess_ctx* ctx, const hess_mlp* m, int64_t K, const double* lambda,
                         const double* Q, double delta, int64_t nq, const void* Xq,
                         const int32_t* cls, double* s, void* ws, size_t ws_bytes);

/* Exact H and/or OPG of M independent networks with their own data sets (widths and
 * N may differ), FP32 output; prec HESS_P_F32 or HESS_P_F32_SPLIT.  Same definitions as
 * hess_exact and hess_opg (paper, Sec. 3); the per-example passes of each network run as
 * small launches and all P x P tiles of all networks go through persistent launches, one
 * per tile units bound (2, 5 or 9 units of a layer per 128-wide tile side), plus one per
 * bound for the cross-layer term of H.  With HESS_OPT_AUTOTUNE the tile configuration of
 * the first-phase launches is tuned like the single-network contractions.
 * models, datas: host arrays of M entries; H, G: host arrays of M device pointers
 * (P_i x P_i FP32 row-major); H or G (the array) may be NULL, and so may single entries,
 * to skip that output.  With HESS_P_F32 the results equal those of the single-network
 * calls bitwise; with HESS_P_F32_SPLIT every block takes split products with the columns
 * split in the tile (the single-network calls read some blocks' columns pre-split) and
 * holds the FP32 tolerance. */
hess_status hess_batched(hess_ctx* ctx, int64_t M, const hess_mlp* models, const hess_data* datas, int prec,
                         void* const* H, void* const* G, void* ws, size_t ws_bytes);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of curvature requests on one device.
 * A server owns n_slots worker slots (each with its own context and HIP stream)
 * and carves every request's workspace from the caller's device pool.  A request is
 * admitted when a slot is free and its footprint fits in the unused pool, so requests
 * that arrive while others run overlap with them on the device.  With coalesce = 1 a
 * slot that takes a damped query also takes the queued queries against the same model
 * and eigenpairs (up to 4096 inputs) and answers them with one hess_predvar call; each
 * query is computed independently, so its result does not depend on the mix.
 * Requests are computed in FP32 (H, OPG, matrix-free top-k) or as hess_predvar.
 * The caller keeps every device buffer a request names alive until hess_server_wait
 * returns for it; host arrays of the model are copied at submission.
 * --------------------------------------------------------------------------- */
typedef struct hess_server hess_server;
typedef enum { HESS_REQ_FULL = 0, HESS_REQ_TOPK = 1, HESS_REQ_PREDVAR = 2, HESS_REQ_CURVATURE = 3 } hess_req_kind;
typedef struct {
  int32_t kind;          /* hess_req_kind */
  hess_mlp model;
  hess_data data;        /* FULL, TOPK: the network's data set */
  void* H;               /* FULL: P x P FP32 output, or NULL */
  void* G;               /* FULL: P x P FP32 OPG output, or NULL */
  int64_t K;             /* TOPK: pairs wanted; PREDVAR, CURVATURE: pairs held in lambda, Q */
  double* lambda;        /* TOPK: output (K); PREDVAR, CURVATURE: input (K), device FP64 */
  double* Q;             /* TOPK: output (K x P); PREDVAR, CURVATURE: input (K x P), device FP64 */
  double tol;            /* TOPK: relative residual tolerance */
  uint64_t seed;         /* TOPK: start-block seed */
  double delta;          /* PREDVAR: damping */
  int64_t nq;            /* PREDVAR: number of query inputs; CURVATURE: number of vectors */
  const void* Xq;        /* PREDVAR: nq x T_1 (model dtype); CURVATURE: nq x P FP64; device */
  const int32_t* cls;    /* PREDVAR: classes (device) or NULL for arg-max */
  double* s;             /* PREDVAR: nq outputs; CURVATURE: nq or nq x P outputs; device FP64 */
  int32_t curv_mode;     /* CURVATURE: hess_curv_mode (the model gives P) */
  double lam_tilde;      /* CURVATURE: full-rank level */
  int32_t fault_launch;  /* test hook, 0 = off: n > 0 makes this request's n-th kernel launch
                            report HESS_E_DEVICE without launching (HESS_OPT_FAULT_AFTER on the
                            slot's context for this request only); such a request is never
                            coalesced with others */
} hess_request;

hess_status hess_server_create(hess_server** srv, int device, int n_slots, void* pool, size_t pool_bytes,
                               int coalesce);
/* Queue a request; HESS_E_BUDGET if its footprint exceeds the whole pool. */
hess_status hess_server_submit(hess_server* srv, const hess_request* req, uint64_t* id);
/* Block until request `id` completes; returns its status and the submit-to-result
 * latency (results in device memory) in milliseconds. */
hess_status hess_server_wait(hess_server* srv, uint64_t id, double* latency_ms);
/* out[0..3] = submitted, completed, failed, coalesced query batches. */
hess_status hess_server_stats(hess_server* srv, int64_t* out);
/* Finish all queued requests, then stop the slots. */
hess_status hess_server_destroy(hess_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* HESS_H */
