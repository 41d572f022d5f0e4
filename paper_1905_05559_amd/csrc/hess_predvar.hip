// Damped curvature query (Laplace-style predictive variance) for a batch of inputs:
//   s_q = g_q^T (Q^T diag(lambda) Q + delta I)^{-1} g_q,   g_q = d z^(L)_{c_q}(x_q) / d omega,
// evaluated in FP64 through the full-rank construction of Sec. 4.2 / Appendix A.2
// (the complement of span(Q) carries the eigenvalue delta):
//   s_q = sum_k (q_k . g_q)^2 / (lambda_k + delta) + (|g_q|^2 - sum_k (q_k . g_q)^2) / delta.
// g_q is never formed: q_k . g_q = sum_l delta^(l)_q . (Qbar_k^(l) abar^(l-1)_q) (one GEMM
// per layer plus a reduction) and |g_q|^2 = sum_l |delta^(l)_q|^2 |abar^(l-1)_q|^2, since
// each layer block of g_q is an outer product.  delta^(l)_q comes from backprop seeded
// with the unit vector e_c at the output pre-activations.
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

// delta^(L)_q = e_c with c = cls[q], or the arg-max of z^(L)_q (lowest index on ties)
__global__ void k_logit_seed(const double* Z, int64_t nq, int64_t TL, const int32_t* cls, double* delta) {
  GRID_STRIDE(q, nq) {
    int64_t c = cls ? cls[q] : -1;
    if (c < 0) {
      c = 0;
      for (int64_t t = 1; t < TL; ++t)
        if (Z[q * TL + t] > Z[q * TL + c]) c = t;
    }
    for (int64_t t = 0; t < TL; ++t) delta[q * TL + t] = (t == c) ? 1.0 : 0.0;
  }
}

constexpr int MAXL = 64;
struct NormArgs {
  int nl;
  const double* d[MAXL];
  int64_t Td[MAXL];
  const double* a[MAXL];
  int64_t lda[MAXL], Ta[MAXL];
};

__global__ void k_gnorm(NormArgs na, int64_t nq, double* g2) {
  GRID_STRIDE(q, nq) {
    double s = 0.0;
    for (int k = 0; k < na.nl; ++k) {
      double dd = 0.0, aa = 0.0;
      for (int64_t i = 0; i < na.Td[k]; ++i) dd += na.d[k][q * na.Td[k] + i] * na.d[k][q * na.Td[k] + i];
      for (int64_t j = 0; j < na.Ta[k]; ++j) aa += na.a[k][q * na.lda[k] + j] * na.a[k][q * na.lda[k] + j];
      s += dd * aa;
    }
    g2[q] = s;
  }
}

__global__ void k_predvar(const double* proj, const double* g2, const double* lam, int64_t K, double delta,
                          int64_t nq, double* s) {
  GRID_STRIDE(q, nq) {
    double a = 0.0, p2 = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      const double p = proj[q * K + k];
      a += p * p / (lam[k] + delta);
      p2 += p * p;
    }
    s[q] = a + (g2[q] - p2) / delta;
  }
}

struct PvBufs {
  HvpBufs<double> h;
  Prep p;
  double *proj = nullptr, *g2 = nullptr;
};

size_t plan_pv(Arena& ar, const Model& m, int64_t K, int64_t nq, PvBufs& b) {
  plan_hvp<double>(ar, m, nq, K, b.p, b.h);
  b.proj = ar.take<double>(nq * K);
  b.g2 = ar.take<double>(nq);
  return ar.used;
}

}  // namespace

hess_status predvar_workspace(hess_ctx* ctx, const Model& m, int prec, int64_t nq, size_t* bytes) {
  (void)prec;
  if (nq < 1) return fail(ctx, HESS_E_SHAPE, "nq must be >= 1");
  // the block of eigenvectors is at most 128 wide in this library (hess_topk_eig)
  Arena ar(nullptr);
  PvBufs b;
  *bytes = plan_pv(ar, m, 128, nq, b);
  return HESS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" hess_status hess_predvar(hess_ctx* ctx, const hess_mlp* mlp, int64_t K, const double* lambda,
                                    const double* Q, double delta, int64_t nq, const void* Xq, const int32_t* cls,
                                    double* s, void* ws, size_t ws_bytes) {
  Exec ex;
  hess_status st = begin(ctx, ex);
  if (st != HESS_OK) return st;
  Model m;
  if ((st = validate_mlp(ctx, mlp, m, true)) != HESS_OK) return st;
  if (m.L - 1 > MAXL) return fail(ctx, HESS_E_SHAPE, "too many layers");
  if (K < 1 || K > 128 || K > m.P) return fail(ctx, HESS_E_SHAPE, "K out of range (1..128, <= P)");
  if (nq < 1 || nq > ((int64_t)1 << 24)) return fail(ctx, HESS_E_SHAPE, "nq out of range");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(ctx, HESS_E_ARG, "delta must be positive and finite");
  if (!lambda || !Q || !Xq || !s) return fail(ctx, HESS_E_ARG, "NULL array");
  Arena probe(nullptr);
  PvBufs b0;
  const size_t need = plan_pv(probe, m, K, nq, b0);
  if ((st = check_ws(ctx, need, ws, ws_bytes, (size_t)nq * 8)) != HESS_OK) return st;
  Arena ar(ws);
  PvBufs b;
  plan_pv(ar, m, K, nq, b);
  // lambda_k + delta > 0 (the damped matrix must be positive definite)
  std::vector<double> lam(K);
  hipMemcpyAsync(lam.data(), lambda, K * sizeof(double), hipMemcpyDeviceToHost, ex.stream);
  if (hipStreamSynchronize(ex.stream) != hipSuccess) return fail(ctx, HESS_E_DEVICE, "reading lambda failed");
  for (int64_t k = 0; k < K; ++k) {
    if (!std::isfinite(lam[k])) return fail(ctx, HESS_E_NONFINITE, "non-finite lambda");
    if (!(lam[k] + delta > 0.0)) return fail(ctx, HESS_E_NOTPD, "lambda_k + delta <= 0 for k = " + std::to_string(k));
  }
  Prep& p = b.p;
  if (ctx->check_inputs) {
    hipMemsetAsync(p.flags, 0, 8 * sizeof(int), ex.stream);
    for (int k = 0; k < m.L - 1; ++k) {
      check_finite(ex, m.W[k], m.dtype, m.T[k + 1] * m.T[k], p.flags);
      check_finite(ex, m.b[k], m.dtype, m.T[k + 1], p.flags);
    }
    check_finite(ex, Xq, m.dtype, nq * m.T[0], p.flags);
    check_finite(ex, Q, HESS_F64, K * m.P, p.flags);
    if (cls) check_cls(ex, cls, nq, m.T[m.L - 1], p.flags + 1);
    int h[8] = {0};
    hipMemcpyAsync(h, p.flags, 8 * sizeof(int), hipMemcpyDeviceToHost, ex.stream);
    if (hipStreamSynchronize(ex.stream) != hipSuccess) return fail(ctx, HESS_E_DEVICE, "input check failed");
    if (ctx->fault_hit) return fail(ctx, HESS_E_DEVICE, "injected device fault");
    if (h[0]) return fail(ctx, HESS_E_NONFINITE, "non-finite value in W, b, Xq or Q");
    if (h[1]) return fail(ctx, HESS_E_ARG, "class index out of range");
  }
  const int L = m.L;
  run_forward(ex, m, Xq, m.dtype, p);
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_logit_seed, dim3(grid_for(nq)), dim3(TPB), 0, ex.stream, p.Z, nq, m.T[L - 1], cls,
                       p.delta[L]);
  run_backward(ex, m, p);
  hvp_setup<double>(ex, m, nq, p, b.h);
  jv_apply<double>(ex, m, nq, K, p, b.h, Q, m.P, b.proj);
  NormArgs na;
  na.nl = L - 1;
  for (int k = 0; k < L - 1; ++k) {
    const int l = k + 2;
    na.d[k] = p.delta[l];
    na.Td[k] = m.T[l - 1];
    na.a[k] = p.Abar[l - 1];
    na.lda[k] = p.lda[l - 1];
    na.Ta[k] = m.T[l - 2] + 1;
  }
  if (launch_ok(ex)) hipLaunchKernelGGL(k_gnorm, dim3(grid_for(nq)), dim3(TPB), 0, ex.stream, na, nq, b.g2);
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_predvar, dim3(grid_for(nq)), dim3(TPB), 0, ex.stream, b.proj, b.g2, lambda, K, delta, nq,
                       s);
  return finish(ex, "hess_predvar");
}
