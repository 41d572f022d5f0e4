// Element-wise and row-wise kernels of the per-example passes: input checks,
// casts, activations with their first two derivatives, the row softmax (one
// wavefront per row, shuffle reductions), the output error signal and the
// per-example curvature-factor updates of the R-operator propagation.
#include <cmath>

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

template <typename T>
__device__ __forceinline__ double ld(const void* p, int64_t i) {
  return (double)static_cast<const T*>(p)[i];
}
__device__ __forceinline__ double ldd(const void* p, int dtype, int64_t i) {
  return dtype == HESS_F64 ? ld<double>(p, i) : ld<float>(p, i);
}

__global__ void k_check_finite(const void* p, int dtype, int64_t n, int* flag) {
  GRID_STRIDE(i, n) {
    if (!isfinite(ldd(p, dtype, i))) *flag = 1;
  }
}

__global__ void k_check_onehot(const void* Y, int dtype, int64_t N, int64_t C, int* flag) {
  GRID_STRIDE(n, N) {
    int ones = 0;
    bool bad = false;
    for (int64_t c = 0; c < C; ++c) {
      const double v = ldd(Y, dtype, n * C + c);
      if (v == 1.0)
        ++ones;
      else if (v != 0.0)
        bad = true;
    }
    if (bad || ones != 1) *flag = 1;
  }
}

__global__ void k_check_cls(const int32_t* cls, int64_t n, int64_t C, int* flag) {
  GRID_STRIDE(i, n) {
    const int32_t c = cls[i];
    if (c < -1 || c >= C) *flag = 1;
  }
}

__global__ void k_to_f64_rows(const void* src, int dtype, int64_t rows, int64_t cols, int64_t lds,
                              double* dst, int64_t ldd_, int bias_one) {
  const int64_t w = cols + (bias_one ? 1 : 0);
  GRID_STRIDE(i, rows * w) {
    const int64_t r = i / w, c = i % w;
    dst[r * ldd_ + c] = (c < cols) ? ldd(src, dtype, r * lds + c) : 1.0;
  }
}

__global__ void k_make_wbar(const void* W, const void* b, int dtype, int64_t Tout, int64_t Tin,
                            double* Wbar) {
  GRID_STRIDE(i, Tout * (Tin + 1)) {
    const int64_t r = i / (Tin + 1), c = i % (Tin + 1);
    Wbar[i] = (c < Tin) ? ldd(W, dtype, r * Tin + c) : ldd(b, dtype, r);
  }
}

__device__ __forceinline__ void act_eval(int act, double z, double& s, double& d1, double& d2) {
  if (act == HESS_TANH) {
    const double t = tanh(z);
    s = t;
    d1 = 1.0 - t * t;
    d2 = -2.0 * t * d1;
  } else if (act == HESS_SIGMOID) {
    const double e = 1.0 / (1.0 + exp(-z));
    s = e;
    d1 = e * (1.0 - e);
    d2 = d1 * (1.0 - 2.0 * e);
  } else {  // ReLU: sigma'(0) = 0, sigma'' = 0
    s = z > 0.0 ? z : 0.0;
    d1 = z > 0.0 ? 1.0 : 0.0;
    d2 = 0.0;
  }
}

__global__ void k_activate(int act, const double* Z, int64_t N, int64_t T, double* Abar, int64_t ldab,
                           double* D1, double* D2) {
  GRID_STRIDE(i, N * (T + 1)) {
    const int64_t n = i / (T + 1), j = i % (T + 1);
    if (j == T) {
      Abar[n * ldab + T] = 1.0;
    } else {
      double s, d1, d2;
      act_eval(act, Z[n * T + j], s, d1, d2);
      Abar[n * ldab + j] = s;
      D1[n * T + j] = d1;
      D2[n * T + j] = d2;
    }
  }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One wavefront per row: row max and exp-sum by xor-shuffle reductions.
__global__ void k_softmax_rows(const double* Z, int64_t N, int64_t T, double* Yhat) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x / 64;
  for (int64_t n = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); n < N; n += (int64_t)gridDim.x * wpb) {
    const double* z = Z + n * T;
    double m = -INFINITY;
    for (int64_t j = lane; j < T; j += 64) m = fmax(m, z[j]);
    m = wave_max(m);
    double s = 0.0;
    for (int64_t j = lane; j < T; j += 64) s += exp(z[j] - m);
    s = wave_sum(s);
    const double inv = 1.0 / s;
    for (int64_t j = lane; j < T; j += 64) Yhat[n * T + j] = exp(z[j] - m) * inv;
  }
}

__global__ void k_output_delta(const double* Yhat, const void* Y, int dtype, int64_t n, double* d) {
  GRID_STRIDE(i, n) { d[i] = Yhat[i] - ldd(Y, dtype, i); }
}

__global__ void k_mul(const double* a, const double* b, double* c, int64_t n) {
  GRID_STRIDE(i, n) { c[i] = a[i] * b[i]; }
}

__global__ void k_transpose(const double* src, int64_t rows, int64_t cols, int64_t lds, double* dst,
                            int64_t ldd_) {
  __shared__ double tile[32][33];
  const int64_t tiles_c = (cols + 31) / 32;
  const int64_t tr = blockIdx.x / tiles_c, tc = blockIdx.x % tiles_c;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = tr * 32 + k, c = tc * 32 + tx;
    if (r < rows && c < cols) tile[k][tx] = src[r * lds + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = tc * 32 + k, r = tr * 32 + tx;
    if (r < rows && c < cols) dst[c * ldd_ + r] = tile[tx][k];
  }
}

template <typename TD>
__global__ void k_cast(const double* src, TD* dst, int64_t n) {
  GRID_STRIDE(i, n) { dst[i] = (TD)src[i]; }
}

template <typename TD>
__global__ void k_cast2d(const double* src, int64_t rows, int64_t cols, int64_t lds, TD* dst, int64_t ldd_) {
  GRID_STRIDE(i, rows * cols) {
    const int64_t r = i / cols, c = i % cols;
    dst[r * ldd_ + c] = (TD)src[r * lds + c];
  }
}

__global__ void k_factor_first(const double* W, int64_t T2, int64_t Tm, const double* D1T, int64_t ldc, int64_t N,
                               double* F) {
  GRID_STRIDE(idx, T2 * Tm * N) {
    const int64_t n = idx % N, i = (idx / N) % Tm, i2 = idx / (N * Tm);
    F[idx] = W[i2 * Tm + i] * D1T[i * ldc + n];
  }
}

__global__ void k_factor_rowscale(const double* F, int64_t Tk, int64_t Tm, const double* D1T, int64_t ldc,
                                  int64_t N, double* K) {
  GRID_STRIDE(idx, Tk * Tm * N) {
    const int64_t n = idx % N, k = idx / (N * Tm);
    K[idx] = D1T[k * ldc + n] * F[idx];
  }
}

// G = S_n F with S_n = diag(p_n) - p_n p_n^T (the softmax Jacobian), per (i, n).
__global__ void k_factor_softmax(const double* F, int64_t TL, int64_t Tm, const double* PT, int64_t ldc,
                                 int64_t N, double* G) {
  GRID_STRIDE(idx, Tm * N) {
    const int64_t n = idx % N, i = idx / N;
    double s = 0.0;
    if (F) {
      for (int64_t k = 0; k < TL; ++k) s += PT[k * ldc + n] * F[(k * Tm + i) * N + n];
    } else {
      s = PT[i * ldc + n];
    }
    for (int64_t k = 0; k < TL; ++k) {
      const double f = F ? F[(k * Tm + i) * N + n] : (k == i ? 1.0 : 0.0);
      G[(k * Tm + i) * N + n] = PT[k * ldc + n] * (f - s);
    }
  }
}

__global__ void k_factor_combine(double* G, int64_t Tk, int64_t Tm, const double* D1T, const double* CT,
                                 int64_t ldc, const double* F, int64_t N) {
  GRID_STRIDE(idx, Tk * Tm * N) {
    const int64_t n = idx % N, i = (idx / N) % Tm, k = idx / (N * Tm);
    const double f = F ? F[idx] : (k == i ? 1.0 : 0.0);
    G[idx] = D1T[k * ldc + n] * G[idx] + CT[k * ldc + n] * f;
  }
}

}  // namespace

#define LAUNCH(kernel, n, ...)                                                     \
  do {                                                                             \
    if (!launch_ok(ex)) return;                                                    \
    hipLaunchKernelGGL(kernel, dim3(grid_for(n)), dim3(TPB), 0, ex.stream, __VA_ARGS__); \
  } while (0)

void check_finite(Exec& ex, const void* p, int dtype, int64_t n, int* flag) {
  if (n > 0) LAUNCH(k_check_finite, n, p, dtype, n, flag);
}
void check_onehot(Exec& ex, const void* Y, int dtype, int64_t N, int64_t C, int* flag) {
  LAUNCH(k_check_onehot, N, Y, dtype, N, C, flag);
}
void check_cls(Exec& ex, const int32_t* cls, int64_t n, int64_t C, int* flag) {
  LAUNCH(k_check_cls, n, cls, n, C, flag);
}
void to_f64_rows(Exec& ex, const void* src, int dtype, int64_t rows, int64_t cols, int64_t lds,
                 double* dst, int64_t ldd_, int bias_one) {
  LAUNCH(k_to_f64_rows, rows * (cols + 1), src, dtype, rows, cols, lds, dst, ldd_, bias_one);
}
void make_wbar(Exec& ex, const void* W, const void* b, int dtype, int64_t Tout, int64_t Tin,
               double* Wbar) {
  LAUNCH(k_make_wbar, Tout * (Tin + 1), W, b, dtype, Tout, Tin, Wbar);
}
void activate(Exec& ex, int act, const double* Z, int64_t N, int64_t T, double* Abar, int64_t ldab,
              double* D1, double* D2) {
  LAUNCH(k_activate, N * (T + 1), act, Z, N, T, Abar, ldab, D1, D2);
}
void softmax_rows(Exec& ex, const double* Z, int64_t N, int64_t T, double* Yhat) {
  if (!launch_ok(ex)) return;
  int64_t g = (N + 3) / 4;
  if (g > (1 << 20)) g = 1 << 20;
  hipLaunchKernelGGL(k_softmax_rows, dim3((unsigned)g), dim3(256), 0, ex.stream, Z, N, T, Yhat);
}
void output_delta(Exec& ex, const double* Yhat, const void* Y, int dtype, int64_t N, int64_t T,
                  double* delta) {
  LAUNCH(k_output_delta, N * T, Yhat, Y, dtype, N * T, delta);
}
void mul(Exec& ex, const double* a, const double* b, double* c, int64_t n) {
  LAUNCH(k_mul, n, a, b, c, n);
}
void transpose(Exec& ex, const double* src, int64_t rows, int64_t cols, int64_t lds, double* dst,
               int64_t ldd_) {
  if (!launch_ok(ex)) return;
  const int64_t nb = ((rows + 31) / 32) * ((cols + 31) / 32);
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)nb), dim3(256), 0, ex.stream, src, rows, cols, lds, dst,
                     ldd_);
}
template <typename TD>
void cast_copy(Exec& ex, const double* src, TD* dst, int64_t n) {
  LAUNCH(k_cast<TD>, n, src, dst, n);
}
template <typename TD>
void cast_2d(Exec& ex, const double* src, int64_t rows, int64_t cols, int64_t lds, TD* dst, int64_t ldd_) {
  LAUNCH(k_cast2d<TD>, rows * cols, src, rows, cols, lds, dst, ldd_);
}
template <typename TD>
__global__ void k_zero(TD* dst, int64_t n) {
  GRID_STRIDE(i, n) { dst[i] = TD(0); }
}
template <typename TD>
void fill_zero(Exec& ex, TD* dst, int64_t n) {
  if (n > 0) LAUNCH(k_zero<TD>, n, dst, n);
}
template void fill_zero<float>(Exec&, float*, int64_t);
template void fill_zero<double>(Exec&, double*, int64_t);
template void cast_copy<float>(Exec&, const double*, float*, int64_t);
template void cast_copy<double>(Exec&, const double*, double*, int64_t);
template void cast_2d<float>(Exec&, const double*, int64_t, int64_t, int64_t, float*, int64_t);
template void cast_2d<double>(Exec&, const double*, int64_t, int64_t, int64_t, double*, int64_t);

void factor_first(Exec& ex, const double* W, int64_t T2, int64_t Tm, const double* D1T, int64_t ldc, int64_t N,
                  double* F) {
  LAUNCH(k_factor_first, T2 * Tm * N, W, T2, Tm, D1T, ldc, N, F);
}
void factor_rowscale(Exec& ex, const double* F, int64_t Tk, int64_t Tm, const double* D1T, int64_t ldc, int64_t N,
                     double* K) {
  LAUNCH(k_factor_rowscale, Tk * Tm * N, F, Tk, Tm, D1T, ldc, N, K);
}
void factor_softmax(Exec& ex, const double* F, int64_t TL, int64_t Tm, const double* PT, int64_t ldc, int64_t N,
                    double* G) {
  LAUNCH(k_factor_softmax, Tm * N, F, TL, Tm, PT, ldc, N, G);
}
void factor_combine(Exec& ex, double* G, int64_t Tk, int64_t Tm, const double* D1T, const double* CT, int64_t ldc,
                    const double* F, int64_t N) {
  LAUNCH(k_factor_combine, Tk * Tm * N, G, Tk, Tm, D1T, CT, ldc, F, N);
}

}  // namespace hs
