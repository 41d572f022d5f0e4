// Low- and full-rank curvature operators from K eigenpairs (paper, Sec. 5.5-5.6 and
// Appendix A.2), applied to a batch of vectors without forming a P x P matrix:
//   p_i = Q x_i (K), H~ x = Q^T (lam p), H~~ x = Q^T (lam p) + lt (x - Q^T p),
//   H~~^{-1} x = Q^T (p / lam) + (x - Q^T p) / lt, and the quadratic forms x^T H~ x,
//   x^T H~~ x.  All FP64: the projections and back-projections are MFMA GEMMs.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "api_internal.h"
#include "mfma.h"

namespace hs {
namespace {

constexpr int TPB = 256;
inline unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + TPB - 1) / TPB, 65535); }
#define GRID_STRIDE(i, n) \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ||x_i||^2 for the rows of X (nx x P), one workgroup per row, fixed reduction order.
__global__ void k_rownorm2(const double* X, int64_t P, double* out) {
  __shared__ double red[TPB];
  const int64_t i = blockIdx.x;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < P; j += TPB) {
    const double v = X[i * P + j];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// quadratic forms: s_i = sum_k lam_k p_ik^2 (+ lt (||x_i||^2 - sum_k p_ik^2) when full)
__global__ void k_quad(const double* proj, const double* x2, const double* lam, int64_t K, double lt, int full,
                       int64_t nx, double* s) {
  GRID_STRIDE(i, nx) {
    double a = 0.0, p2 = 0.0;
    for (int64_t k = 0; k < K; ++k) {
      const double p = proj[i * K + k];
      a += lam[k] * p * p;
      p2 += p * p;
    }
    s[i] = full ? a + lt * (x2[i] - p2) : a;
  }
}

// coefficients of the back-projection: c_ik = f(lam_k) p_ik - g p_ik, with f = lam (apply)
// or 1 / lam (inverse), g = the complement factor (0 for the low-rank apply)
__global__ void k_coef(const double* proj, const double* lam, int64_t K, int inverse, double g, int64_t nx,
                       double* coef) {
  GRID_STRIDE(e, nx * K) {
    const int64_t k = e % K;
    const double f = inverse ? 1.0 / lam[k] : lam[k];
    coef[e] = (f - g) * proj[e];
  }
}

__global__ void k_scale(const double* X, double g, int64_t n, double* Y) {
  GRID_STRIDE(e, n) { Y[e] = g * X[e]; }
}

void plan_curv(Arena& ar, int64_t K, int64_t nx, double*& proj, double*& coef, double*& x2) {
  proj = ar.take<double>(nx * K);
  coef = ar.take<double>(nx * K);
  x2 = ar.take<double>(nx);
}

}  // namespace

hess_status curvature_workspace(hess_ctx* ctx, int64_t K, int64_t nx, size_t* bytes) {
  if (K < 1 || nx < 1) return fail(ctx, HESS_E_SHAPE, "K and nx must be positive");
  Arena ar(nullptr);
  double *proj, *coef, *x2;
  plan_curv(ar, K, nx, proj, coef, x2);
  *bytes = ar.used;
  return HESS_OK;
}

namespace {

// Library-owned scratch of hess_curvature_noalloc: projections, coefficients and row
// norms (2 nx K + nx doubles, each array 256-byte aligned).  Every device the library
// runs on holds its own copy until the process ends.  In host code `scratch` is only a
// stand-in for the symbol; its device address comes from hipGetSymbolAddress, once per
// device, and only that address is handed to kernels.
constexpr size_t kCurvScratchBytes = size_t(16) << 20;
__device__ __align__(256) unsigned char scratch[kCurvScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the device is current); nullptr on failure.
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

hess_status curvature_run(Exec& ex, int mode, int64_t K, int64_t P, const double* lambda, const double* Q,
                          double lam_tilde, int64_t nx, const double* X, double* out, void* ws, size_t ws_bytes);

}  // namespace
}  // namespace hs

using namespace hs;

extern "C" hess_status hess_curvature(hess_ctx* ctx, int mode, int64_t K, int64_t P, const double* lambda,
                                      const double* Q, double lam_tilde, int64_t nx, const double* X, double* out,
                                      void* ws, size_t ws_bytes) {
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  return curvature_run(ex, mode, K, P, lambda, Q, lam_tilde, nx, X, out, ws, ws_bytes);
}

extern "C" hess_status hess_curvature_noalloc(hess_ctx* ctx, int mode, int64_t K, int64_t P, const double* lambda,
                                              const double* Q, double lam_tilde, int64_t nx, const double* X,
                                              double* out) {
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  size_t need = 0;
  if ((s = curvature_workspace(ctx, K, nx, &need)) != HESS_OK) return s;
  if (need > kCurvScratchBytes)
    return fail(ctx, HESS_E_WORKSPACE, "hess_curvature_noalloc: " + std::to_string(need) +
                                           " B of scratch needed (2 nx K + nx doubles), above the library's " +
                                           std::to_string(kCurvScratchBytes) + " B");
  void* ptr = scratch_address(ctx->device);
  if (!ptr) return fail(ctx, HESS_E_DEVICE, "hess_curvature_noalloc: hipGetSymbolAddress of the scratch failed");
  return curvature_run(ex, mode, K, P, lambda, Q, lam_tilde, nx, X, out, ptr, kCurvScratchBytes);
}

namespace hs {
namespace {

hess_status curvature_run(Exec& ex, int mode, int64_t K, int64_t P, const double* lambda, const double* Q,
                          double lam_tilde, int64_t nx, const double* X, double* out, void* ws, size_t ws_bytes) {
  hess_ctx* ctx = ex.ctx;
  hess_status s;
  if (mode < 0 || mode > 4) return fail(ctx, HESS_E_ARG, "unknown curvature mode");
  if (K < 1 || P < K || nx < 1) return fail(ctx, HESS_E_SHAPE, "need 1 <= K <= P and nx >= 1");
  if (!lambda || !Q || !X || !out) return fail(ctx, HESS_E_ARG, "NULL pointer");
  const bool full = mode == HESS_CURV_FULL_QUAD || mode == HESS_CURV_FULL_APPLY || mode == HESS_CURV_FULL_INV;
  // the eigenvalues (K values) decide validity: read them to the host
  std::vector<double> lam(K);
  hipMemcpyAsync(lam.data(), lambda, K * sizeof(double), hipMemcpyDeviceToHost, ex.stream);
  if (hipStreamSynchronize(ex.stream) != hipSuccess) return fail(ctx, HESS_E_DEVICE, "reading lambda failed");
  for (double v : lam)
    if (!std::isfinite(v)) return fail(ctx, HESS_E_NONFINITE, "non-finite eigenvalue");
  if (full && !(std::isfinite(lam_tilde))) return fail(ctx, HESS_E_NONFINITE, "non-finite lam_tilde");
  if (mode == HESS_CURV_FULL_INV) {
    if (!(lam_tilde > 0.0)) return fail(ctx, HESS_E_NOTPD, "lam_tilde <= 0: the full-rank operator is singular");
    for (double v : lam)
      if (!(v > 0.0)) return fail(ctx, HESS_E_NOTPD, "an eigenvalue <= 0: the full-rank operator is singular");
  }
  Arena probe(nullptr);
  double *proj, *coef, *x2;
  plan_curv(probe, K, nx, proj, coef, x2);
  const size_t outb = (size_t)nx * (mode == HESS_CURV_LOW_QUAD || mode == HESS_CURV_FULL_QUAD ? 1 : P) * 8;
  if ((s = check_ws(ctx, probe.used, ws, ws_bytes, outb)) != HESS_OK) return s;
  Arena ar(ws);
  plan_curv(ar, K, nx, proj, coef, x2);
  // p = X Q^T  (nx x K)
  gemm_rm<double>(ex, false, true, nx, K, P, 1.0, X, P, Q, P, 0.0, proj, K);
  if (mode == HESS_CURV_LOW_QUAD || mode == HESS_CURV_FULL_QUAD) {
    if (full && launch_ok(ex)) hipLaunchKernelGGL(k_rownorm2, dim3((unsigned)nx), dim3(TPB), 0, ex.stream, X, P, x2);
    if (launch_ok(ex))
      hipLaunchKernelGGL(k_quad, dim3(grid_for(nx)), dim3(TPB), 0, ex.stream, proj, x2, lambda, K, lam_tilde,
                         full ? 1 : 0, nx, out);
    return finish(ex, "hess_curvature");
  }
  // Y = C Q + g X with C = (f(lam) - g) p, g = lt (apply), 1 / lt (inverse), 0 (low rank)
  const int inverse = mode == HESS_CURV_FULL_INV;
  const double g = mode == HESS_CURV_LOW_APPLY ? 0.0 : (inverse ? 1.0 / lam_tilde : lam_tilde);
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_coef, dim3(grid_for(nx * K)), dim3(TPB), 0, ex.stream, proj, lambda, K, inverse, g, nx, coef);
  if (launch_ok(ex)) hipLaunchKernelGGL(k_scale, dim3(grid_for(nx * P)), dim3(TPB), 0, ex.stream, X, g, nx * P, out);
  gemm_rm<double>(ex, false, false, nx, P, K, 1.0, coef, K, Q, P, 1.0, out, P);
  return finish(ex, "hess_curvature");
}

}  // namespace
}  // namespace hs
