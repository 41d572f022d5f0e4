// Leading (algebraically largest) eigenpairs of H or of the OPG (paper, Sec. 4.1,
// 5.3, 5.4): randomized block subspace iteration accelerated by a Chebyshev
// polynomial filter, with FP64 re-orthogonalisation (shifted Cholesky-QR, three
// passes) and FP64 Rayleigh-Ritz (cyclic Jacobi on the b x b projected matrix).
//
// The paper asks the Lanczos solver for which='LA' and sorts the pairs in
// descending order; H is indefinite away from a minimum, so plain power-type
// subspace iteration (which converges to the largest |lambda|) would answer a
// different question.  The filter T_d((x - c) / e) with c, e mapping
// [lambda_lb, a] onto [-1, 1] is bounded by 1 on that interval and grows quickly
// above the cut a (the smallest Ritz value of the block), so the block converges
// to the algebraically largest eigenvalues.  lambda_lb is a lower bound of the
// spectrum from the spectral radius estimated by a few unfiltered block steps.
//
// Block vectors are stored b x Ppad (row k = vector k, zero-padded columns) in FP64.
// The operator is applied in its own precision: a dense M (FP64 or FP32) through the
// MFMA GEMM, or the matrix-free H (R-operator) or OPG (J^T J v / N) products.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "api_internal.h"
#include "mfma.h"

namespace hs {

namespace {

constexpr int TPB = 256;
constexpr int BMAX = 128;     // largest block size (Jacobi and Cholesky run in LDS)
constexpr int64_t KSPLIT = 1024;  // columns per split of the Gram products (block rows are padded to it)

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + TPB - 1) / TPB;
  if (g > (1 << 20)) g = 1 << 20;
  return (unsigned)(g < 1 ? 1 : g);
}
#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)
#define LAUNCH(kernel, n, ...)                                                                 \
  do {                                                                                         \
    if (!launch_ok(ex)) return;                                                                \
    hipLaunchKernelGGL(kernel, dim3(grid_for(n)), dim3(TPB), 0, ex.stream, __VA_ARGS__);       \
  } while (0)

// SplitMix64 finaliser (Steele, Lea & Flood, 2014) used as a counter-based generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Q[k][p] ~ N(0, 1) by Box-Muller on two counter-derived uniforms; zero in the padding.
__global__ void k_randn(uint64_t seed, int64_t b, int64_t P, int64_t ldp, double* Q) {
  GRID_STRIDE(e, b * ldp) {
    const int64_t k = e / ldp, p = e % ldp;
    if (p >= P) {
      Q[e] = 0.0;
      continue;
    }
    const uint64_t c = (uint64_t)(k * P + p);
    const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * c));
    const uint64_t h2 = splitmix64(seed ^ splitmix64(2 * c + 1));
    const double u1 = ((double)(h1 >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(h2 >> 11) * 0x1.0p-53;
    Q[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

__global__ void k_fill(double* x, int64_t n, double v) {
  GRID_STRIDE(i, n) { x[i] = v; }
}

__global__ void k_f32_to_f64_2d(const float* src, int64_t rows, int64_t cols, int64_t lds, double* dst,
                                int64_t ldd) {
  GRID_STRIDE(i, rows * cols) {
    const int64_t r = i / cols, c = i % cols;
    dst[r * ldd + c] = (double)src[r * lds + c];
  }
}

// dst (cols x rows, FP32) = src^T, src rows x cols FP64 with leading dimension lds
__global__ void k_cast_t(const double* src, int64_t rows, int64_t cols, int64_t lds, float* dst) {
  __shared__ float tile[32][33];
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + y, c = c0 + tx;
    if (r < rows && c < cols) tile[y][tx] = (float)src[r * lds + c];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t c = c0 + y, r = r0 + tx;
    if (r < rows && c < cols) dst[c * rows + r] = tile[tx][y];
  }
}

// Y (rows x cols, FP64, leading dimension ldy) = sum_s part[s] (FP32 rows x cols), in split order
__global__ void k_sum_splits_f32(const float* part, int64_t S, int64_t rows, int64_t cols, double* Y, int64_t ldy) {
  GRID_STRIDE(i, rows * cols) {
    double v = 0.0;
    for (int64_t k = 0; k < S; ++k) v += (double)part[k * rows * cols + i];
    Y[(i / cols) * ldy + i % cols] = v;
  }
}

// out[i] = sum_s part[s * n + i], summed in split order (deterministic)
__global__ void k_sum_splits(const double* part, int64_t S, int64_t n, double* out) {
  GRID_STRIDE(i, n) {
    double s = 0.0;
    for (int64_t k = 0; k < S; ++k) s += part[k * n + i];
    out[i] = s;
  }
}

// out = alpha * A + beta * B + gamma * C  (elementwise)
__global__ void k_axpbypcz(double alpha, const double* A, double beta, const double* B, double gamma,
                           const double* C, int64_t n, double* out) {
  GRID_STRIDE(i, n) {
    double v = alpha * A[i] + beta * B[i];
    if (C) v += gamma * C[i];
    out[i] = v;
  }
}

// W = L L^T (b x b, b <= BMAX) with an optional diagonal shift; writes L^{-1} (lower).
// shift_mode 1 adds 11 (P b + b (b + 1)) u trace(W) to the diagonal (shifted
// Cholesky-QR, Fukaya et al. 2020).  info[0] = 1 on a non-positive pivot.
__global__ __launch_bounds__(256) void k_chol_inv(const double* W, int b, int64_t P, int shift_mode,
                                                  double* Linv, int* info) {
  extern __shared__ double As[];  // b x (b + 1)
  const int ld = b + 1, tid = threadIdx.x;
  __shared__ double trace;
  __shared__ int bad;
  for (int e = tid; e < b * b; e += blockDim.x) As[(e / b) * ld + e % b] = W[e];
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < b; ++i) t += W[i * b + i];
    trace = t;
    bad = 0;
  }
  __syncthreads();
  if (shift_mode) {
    const double s = 11.0 * ((double)P * b + (double)b * (b + 1)) * 1.1102230246251565e-16 * trace;
    for (int i = tid; i < b; i += blockDim.x) As[i * ld + i] += s;
  }
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    if (tid == 0) {
      const double d = As[j * ld + j];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
        As[j * ld + j] = 1.0;
      } else {
        As[j * ld + j] = sqrt(d);
      }
    }
    __syncthreads();
    const double piv = As[j * ld + j];
    for (int i = j + 1 + tid; i < b; i += blockDim.x) As[i * ld + j] /= piv;
    __syncthreads();
    const int n = b - j - 1;
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int i = j + 1 + e / n, k = j + 1 + e % n;
      if (k <= i) As[i * ld + k] -= As[i * ld + j] * As[k * ld + j];
    }
    __syncthreads();
  }
  // column c of L^{-1} by forward substitution (one thread per column)
  for (int c = tid; c < b; c += blockDim.x) {
    for (int i = 0; i < c; ++i) Linv[i * b + c] = 0.0;
    for (int i = c; i < b; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= As[i * ld + k] * Linv[k * b + c];
      Linv[i * b + c] = s / As[i * ld + i];
    }
  }
  if (tid == 0 && bad) info[0] = 1;
}

// Cyclic Jacobi for the symmetric b x b matrix (T + T^T) / 2 with round-robin parallel
// ordering; eigenvalues sorted descending in ev, eigenvectors in the columns of U.
__global__ __launch_bounds__(256) void k_jacobi(const double* Tm, int b, int max_sweeps, double* ev, double* U,
                                                int* sweeps_out) {
  extern __shared__ double A[];  // n x (n + 1), n = b rounded up to even
  __shared__ double red[256];
  __shared__ double cs[BMAX / 2][2];
  __shared__ int pr[BMAX / 2][2];
  __shared__ int perm[BMAX];
  const int n = (b + 1) & ~1, ld = n + 1, tid = threadIdx.x;
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    double v = 0.0;
    if (i < b && j < b) v = 0.5 * (Tm[i * b + j] + Tm[j * b + i]);
    A[i * ld + j] = v;
  }
  for (int e = tid; e < b * b; e += blockDim.x) U[e] = (e / b == e % b) ? 1.0 : 0.0;
  __syncthreads();
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < b * b; e += blockDim.x) {
      const int i = e / b, j = e % b;
      const double v = A[i * ld + j] * A[i * ld + j];
      tot += v;
      if (i != j) off += v;
    }
    red[tid] = off;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const double tots = red[0];
    __syncthreads();
    if (offs <= 1e-30 * tots || tots == 0.0) break;
    for (int r = 0; r < n - 1; ++r) {
      const int np = n / 2;
      if (tid < np) {
        int p, q;
        if (tid == 0) {
          p = r;
          q = n - 1;
        } else {
          p = (r + tid) % (n - 1);
          q = (r - tid + n - 1) % (n - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < b) {
          const double apq = A[p * ld + q];
          if (apq != 0.0) {
            const double tau = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
            const double t = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau)) : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pr[tid][0] = p;
        pr[tid][1] = q;
        cs[tid][0] = c;
        cs[tid][1] = s;
      }
      __syncthreads();
      // rows p, q  <-  J^T A
      for (int e = tid; e < np * n; e += blockDim.x) {
        const int k = e / n, j = e % n;
        const int p = pr[k][0], q = pr[k][1];
        const double c = cs[k][0], s = cs[k][1];
        const double apj = A[p * ld + j], aqj = A[q * ld + j];
        A[p * ld + j] = c * apj - s * aqj;
        A[q * ld + j] = s * apj + c * aqj;
      }
      __syncthreads();
      // columns p, q  <-  A J ; U <- U J
      for (int e = tid; e < np * n; e += blockDim.x) {
        const int k = e / n, i = e % n;
        const int p = pr[k][0], q = pr[k][1];
        const double c = cs[k][0], s = cs[k][1];
        const double aip = A[i * ld + p], aiq = A[i * ld + q];
        A[i * ld + p] = c * aip - s * aiq;
        A[i * ld + q] = s * aip + c * aiq;
        if (i < b && q < b) {
          const double uip = U[i * b + p], uiq = U[i * b + q];
          U[i * b + p] = c * uip - s * uiq;
          U[i * b + q] = s * uip + c * uiq;
        }
      }
      __syncthreads();
    }
  }
  // sort descending (stable: lower index first on ties)
  if (tid == 0) {
    for (int i = 0; i < b; ++i) perm[i] = i;
    for (int i = 0; i < b; ++i) {
      int best = i;
      for (int j = i + 1; j < b; ++j)
        if (A[perm[j] * ld + perm[j]] > A[perm[best] * ld + perm[best]]) best = j;
      const int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
    *sweeps_out = sweep;
  }
  __syncthreads();
  for (int i = tid; i < b; i += blockDim.x) ev[i] = A[perm[i] * ld + perm[i]];
  // permute columns of U through the LDS matrix (A no longer needed)
  __syncthreads();
  for (int e = tid; e < b * b; e += blockDim.x) A[(e / b) * ld + e % b] = U[e];
  __syncthreads();
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    U[e] = A[i * ld + perm[j]];
  }
}

// res[k] = || MX[k] - theta[k] X[k] ||_2, one workgroup per row
__global__ __launch_bounds__(256) void k_resid(const double* MX, const double* X, const double* theta, int64_t P,
                                               int64_t ldp, double* res) {
  __shared__ double red[256];
  const int64_t k = blockIdx.x;
  const double th = theta[k];
  double s = 0.0;
  for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
    const double r = MX[k * ldp + p] - th * X[k * ldp + p];
    s += r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) res[k] = sqrt(red[0]);
}

// Flip row k so that its largest-|.| entry (lowest index on ties) is positive; copy to out.
__global__ __launch_bounds__(256) void k_sign_copy(const double* X, int64_t P, int64_t ldp, double* out) {
  __shared__ double vmax[256];
  __shared__ int64_t imax[256];
  const int64_t k = blockIdx.x;
  double best = -1.0;
  int64_t bi = P;
  for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
    const double a = fabs(X[k * ldp + p]);
    if (a > best) {
      best = a;
      bi = p;
    }
  }
  vmax[threadIdx.x] = best;
  imax[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = vmax[threadIdx.x + w];
      const int64_t oi = imax[threadIdx.x + w];
      if (o > vmax[threadIdx.x] || (o == vmax[threadIdx.x] && oi < imax[threadIdx.x])) {
        vmax[threadIdx.x] = o;
        imax[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = (imax[0] < P && X[k * ldp + imax[0]] < 0.0) ? -1.0 : 1.0;
  for (int64_t p = threadIdx.x; p < P; p += blockDim.x) out[k * P + p] = sg * X[k * ldp + p];
}

struct EigBufs {
  int64_t b = 0, P = 0, ldp = 0, S = 0;
  double *Q, *Y, *Yp, *Z, *MQ, *X, *MX;
  float *Qf, *Yf;
  float* Ypart = nullptr;      // dense FP32 operator: per-slice partial products
  int64_t ks = 1, kslice = 0;  // slices of the contraction over P
  bool skinny = false;         // dense FP32 operator with b <= 64: thin-block kernel
  double *part, *W, *Linv, *T, *U, *theta, *res;
  int* info;
  Prep p;
  HvpBufs<double> hd;
  HvpBufs<float> hf;
};

}  // namespace

// Slices of the dense FP32 apply (b x P times P x P): the output alone has few 128 x 128
// tiles, so the contraction over P is split into slices; the count is chosen so that the
// workgroups fill whole rounds of the device's resident slots (three per compute unit).
static void dense_slices(int64_t P, int64_t b, int64_t& ks, int64_t& kslice) {
  static const int64_t slots = [] {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return 3 * (int64_t)std::max(cus, 1);
  }();
  const int64_t tiles = ((b + 127) / 128) * ((P + 127) / 128);
  int64_t best = 1;
  double best_eff = -1.0;
  for (int64_t k = 1; k <= 12 && (k == 1 || P / k >= 1024); ++k) {
    const int64_t w = tiles * k, rounds = (w + slots - 1) / slots;
    // fraction of slot time doing work; one round or fewer is charged as under-filled
    const double eff = (double)w / (double)(std::max<int64_t>(rounds, 2) * slots);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = k;
    }
  }
  kslice = rup((P + best - 1) / best, 32);
  ks = (P + kslice - 1) / kslice;
}

static size_t plan_eig(Arena& ar, const Model* m, int64_t N, int64_t P, int64_t b, int source, int prec,
                       int mdtype, EigBufs& e) {
  e.b = b;
  e.P = P;
  e.ldp = rup(P, KSPLIT);
  e.S = e.ldp / KSPLIT;
  const int64_t nb = b * e.ldp;
  for (double** x : {&e.Q, &e.Y, &e.Yp, &e.Z, &e.MQ, &e.X, &e.MX}) *x = ar.take<double>(nb);
  e.Qf = ar.take<float>(b * P);
  e.Yf = ar.take<float>(b * P);
  e.part = ar.take<double>(e.S * b * b);
  if (source == 1 && mdtype == HESS_F32) {
    e.skinny = b <= 64;
    if (e.skinny)
      skinny_slices(P, b, e.ks, e.kslice);
    else
      dense_slices(P, b, e.ks, e.kslice);
    e.Ypart = ar.take<float>(e.ks * b * P);
  }
  for (double** x : {&e.W, &e.Linv, &e.T, &e.U}) *x = ar.take<double>(b * b);
  e.theta = ar.take<double>(b);
  e.res = ar.take<double>(b);
  e.info = ar.take<int>(16);
  if (source == 0) {
    if (prec == HESS_P_F64)
      plan_hvp<double>(ar, *m, N, b, e.p, e.hd);
    else
      plan_hvp<float>(ar, *m, N, b, e.p, e.hf, prec == HESS_P_F32_SPLIT);
  }
  return ar.used;
}

namespace {

// The Cholesky and Jacobi kernels keep a b x (b + 1) FP64 matrix in LDS (up to 132 KB).
void set_lds_limits() {
  static bool done = false;
  if (done) return;
  const int lim = 150 * 1024;
  (void)hipFuncSetAttribute((const void*)k_chol_inv, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  done = true;
}

struct GraphCache;

struct EigRun {
  Exec* ex;
  EigBufs* e;
  const Model* m;
  int64_t N;
  int source, which, prec, Mdtype;
  const void* M;
  GraphCache* gc = nullptr;  // captured operator applications (nullptr: always eager)
};

// Y = Op Q (rows), both b x ldp FP64
void op_apply(EigRun& r, const double* Q, double* Y) {
  Exec& ex = *r.ex;
  EigBufs& e = *r.e;
  const int64_t b = e.b, P = e.P, ldp = e.ldp;
  if (r.source == 1) {
    if (r.Mdtype == HESS_F64) {
      gemm_rm<double>(ex, false, false, b, P, P, 1.0, Q, ldp, static_cast<const double*>(r.M), P, 0.0, Y, ldp);
    } else {
      // Y = Q M through the Khatri-Rao contraction with one unit per side: rows are the
      // b block vectors (source Q^T, P x b), columns the P columns of M (source M: row k
      // of M holds M[k][c] for all c); the contraction over k is split into slices whose
      // partial products are summed in slice order.
      if (!launch_ok(ex)) return;
      if (e.skinny) {  // thin block: M streamed once per application
        cast_2d<float>(ex, Q, b, P, ldp, e.Qf, P);
        skinny_apply_f32(ex, e.Qf, b, P, static_cast<const float*>(r.M), e.Ypart, e.ks, e.kslice);
        LAUNCH(k_sum_splits_f32, b * P, e.Ypart, e.ks, b, P, Y, ldp);
        return;
      }
      hipLaunchKernelGGL(k_cast_t, dim3((unsigned)((P + 31) / 32), (unsigned)((b + 31) / 32)), dim3(256), 0,
                         ex.stream, Q, b, P, ldp, e.Qf);
      KrgArgs<float, float> a;
      a.r = KrgSide<float>{e.Qf, b, 1, (int32_t)b, (int32_t)rup(b, 16), nullptr, 0, 0, 0, (int32_t)b, 1};
      a.c = KrgSide<float>{static_cast<const float*>(r.M), P, 1, (int32_t)P, (int32_t)rup(P, 16), nullptr, 0, 0, 0,
                           (int32_t)P, 1};
      a.wmode = KRG_RANK1;
      a.wts = nullptr;
      a.ldw = 0;
      a.out = e.Ypart;
      a.ldo = P;
      a.symmetric = 0;
      a.accumulate = 0;
      a.mirror = 0;
      a.scale = 1.0;
      a.N = P;
      a.ksplit = (int32_t)e.ks;
      a.kslice = e.kslice;
      a.out_split = b * P;
      a.label = "dense_apply_f32";
      krg<float, float>(ex, a);
      LAUNCH(k_sum_splits_f32, b * P, e.Ypart, e.ks, b, P, Y, ldp);
    }
    return;
  }
  if (r.prec == HESS_P_F64) {
    if (r.which == 0)
      hvp_apply<double>(ex, *r.m, r.N, b, e.p, e.hd, Q, ldp, Y);
    else
      opg_apply<double>(ex, *r.m, r.N, b, e.p, e.hd, Q, ldp, Y);
  } else {
    cast_2d<float>(ex, Q, b, P, ldp, e.Qf, P);
    if (r.which == 0)
      hvp_apply<float>(ex, *r.m, r.N, b, e.p, e.hf, e.Qf, P, e.Yf);
    else
      opg_apply<float>(ex, *r.m, r.N, b, e.p, e.hf, e.Qf, P, e.Yf);
    LAUNCH(k_f32_to_f64_2d, b * P, e.Yf, b, P, P, Y, ldp);
  }
}

// Operator applications captured as HIP graphs: the first application for a (Q, Y) pair
// runs eagerly, the second is captured on the context's capture stream (the null stream
// cannot be captured) and launched on the call's stream, later ones replay the graph.
// The captured sequence holds kernel launches only (no memsets, copies or host waits).
struct GraphCache {
  struct Ent {
    const double* q;
    double* y;
    int uses;
    hipGraphExec_t exec;
  };
  std::vector<Ent> ents;
  bool disabled = false;
  ~GraphCache() {
    for (auto& e : ents)
      if (e.exec) (void)hipGraphExecDestroy(e.exec);
  }
};

void apply_op(EigRun& r, GraphCache* gc, const double* Q, double* Y) {
  Exec& ex = *r.ex;
  hess_ctx* c = ex.ctx;
  if (!gc || gc->disabled || c->profile || c->fault_after >= 0) {
    op_apply(r, Q, Y);
    return;
  }
  GraphCache::Ent* ent = nullptr;
  for (auto& e : gc->ents)
    if (e.q == Q && e.y == Y) ent = &e;
  if (!ent) {
    gc->ents.push_back(GraphCache::Ent{Q, Y, 0, nullptr});
    ent = &gc->ents.back();
  }
  ent->uses++;
  if (ent->exec) {
    if (hipGraphLaunch(ent->exec, ex.stream) != hipSuccess) {
      (void)hipGetLastError();
      ex.ctx->fault_hit = true;
    }
    return;
  }
  if (ent->uses == 1) {
    op_apply(r, Q, Y);
    return;
  }
  if (!c->capture_stream && hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    c->capture_stream = nullptr;
    gc->disabled = true;
    op_apply(r, Q, Y);
    return;
  }
  const hipStream_t run = ex.stream;
  hipGraph_t g = nullptr;
  bool ok = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    ex.stream = c->capture_stream;
    op_apply(r, Q, Y);
    ex.stream = run;
    ok = hipStreamEndCapture(c->capture_stream, &g) == hipSuccess && g;
  }
  if (ok) ok = hipGraphInstantiate(&ent->exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!ok) {  // capture unavailable: stay eager for this call
    (void)hipGetLastError();
    ent->exec = nullptr;
    gc->disabled = true;
    op_apply(r, Q, Y);
    return;
  }
  if (hipGraphLaunch(ent->exec, run) != hipSuccess) {
    (void)hipGetLastError();
    ex.ctx->fault_hit = true;
  }
}

// C (b x b) = A B^T over ldp columns, split over KSPLIT columns and summed in order
void gram(EigRun& r, const double* A, const double* B, double* C) {
  Exec& ex = *r.ex;
  EigBufs& e = *r.e;
  GemmArgs<double> g;
  g.M = e.b; g.N = e.b; g.K = KSPLIT;
  g.A = A; g.sam = e.ldp; g.sak = 1; g.sab = KSPLIT;
  g.B = B; g.sbk = 1; g.sbn = e.ldp; g.sbb = KSPLIT;
  g.C = e.part; g.scm = e.b; g.scn = 1; g.scb = e.b * e.b;
  g.alpha = 1.0; g.beta = 0.0; g.batch = e.S;
  gemm<double>(ex, g);
  LAUNCH(k_sum_splits, e.b * e.b, e.part, e.S, e.b * e.b, C);
}

// Q = orthonormal rows spanning Y: shifted Cholesky-QR, then plain passes (three passes
// in all by default; with first_plain the first pass is unshifted too).  Y is overwritten;
// with an odd number of passes the result is in Q.
void orth(EigRun& r, double* Y, double* Q, int passes = 3, bool first_plain = false) {
  Exec& ex = *r.ex;
  EigBufs& e = *r.e;
  const int b = (int)e.b;
  const size_t shm = (size_t)b * (b + 1) * sizeof(double);
  for (int pass = 0; pass < passes; ++pass) {
    double* src = pass == 1 ? Q : Y;
    double* dst = pass == 1 ? Y : Q;
    gram(r, src, src, e.W);
    if (!launch_ok(ex)) return;
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), shm, ex.stream, e.W, b, e.P,
                       (pass == 0 && !first_plain) ? 1 : 0, e.Linv, e.info);
    gemm_rm<double>(ex, false, false, b, e.ldp, b, 1.0, e.Linv, b, src, e.ldp, 0.0, dst, e.ldp);
  }
}

// Rayleigh-Ritz on the orthonormal block Q: X, MX, theta (descending), res.
void rayleigh_ritz(EigRun& r, int* sweeps) {
  Exec& ex = *r.ex;
  EigBufs& e = *r.e;
  const int b = (int)e.b;
  apply_op(r, r.gc, e.Q, e.MQ);
  gram(r, e.Q, e.MQ, e.T);
  const int n = (b + 1) & ~1;
  const size_t shm = (size_t)n * (n + 1) * sizeof(double);
  if (!launch_ok(ex)) return;
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), shm, ex.stream, e.T, b, 60, e.theta, e.U, e.info + 4);
  gemm_rm<double>(ex, true, false, b, e.ldp, b, 1.0, e.U, b, e.Q, e.ldp, 0.0, e.X, e.ldp);
  gemm_rm<double>(ex, true, false, b, e.ldp, b, 1.0, e.U, b, e.MQ, e.ldp, 0.0, e.MX, e.ldp);
  if (!launch_ok(ex)) return;
  hipLaunchKernelGGL(k_resid, dim3(b), dim3(256), 0, ex.stream, e.MX, e.X, e.theta, e.P, e.ldp, e.res);
  (void)sweeps;
}

bool read_back(Exec& ex, EigBufs& e, std::vector<double>& theta, std::vector<double>& res, int* info) {
  theta.assign(e.b, 0.0);
  res.assign(e.b, 0.0);
  hipMemcpyAsync(theta.data(), e.theta, e.b * sizeof(double), hipMemcpyDeviceToHost, ex.stream);
  hipMemcpyAsync(res.data(), e.res, e.b * sizeof(double), hipMemcpyDeviceToHost, ex.stream);
  hipMemcpyAsync(info, e.info, 16 * sizeof(int), hipMemcpyDeviceToHost, ex.stream);
  return hipStreamSynchronize(ex.stream) == hipSuccess && !ex.ctx->fault_hit;
}

// ---------------------------------------------------------------------------
// Thick-restart block Lanczos with locking (method 1).
//
// The window W holds n orthonormal rows (n <= win): kept Ritz vectors followed by
// Lanczos blocks; T = W Op W^T is kept explicitly (n x n, row stride win).  Each step
// applies Op to the open block (the last one), re-orthogonalises the product against
// W and the locked vectors L with two classical Gram-Schmidt passes (their
// coefficients give T's column block), and orthonormalises the remainder into the
// next block; T's coupling block is V_new Z^T.  When the window is full, T is
// diagonalised (Rayleigh-Ritz); residual norms of the Ritz pairs follow from the
// remainder Z of the last block without another product.  The leading Ritz pairs with
// residual below half the tolerance are locked; the next `keep` Ritz vectors plus the
// orthonormalised remainder start the next window (T = diag(theta) with the coupling
// row).  Once K pairs are locked, a Rayleigh-Ritz over L gives the reported pairs and
// their true residuals.
// ---------------------------------------------------------------------------

// T[i][o + j] = T[o + j][i] = C[i][j] for i < n, j < b; the open block's diagonal
// block is symmetrised.
__global__ void k_put_cols(double* T, int64_t ldt, int64_t n, int64_t o, int64_t b, const double* C) {
  GRID_STRIDE(e, n * b) {
    const int64_t i = e / b, j = e % b;
    double v = C[e];
    if (i >= o && i < o + b) v = 0.5 * (v + C[(o + j) * b + (i - o)]);
    T[i * ldt + o + j] = v;
    T[(o + j) * ldt + i] = v;
  }
}

// T[r0 + x][o + a] = T[o + a][r0 + x] = G[x][a]
__global__ void k_put_coupling(double* T, int64_t ldt, int64_t r0, int64_t o, int64_t b, const double* G) {
  GRID_STRIDE(e, b * b) {
    const int64_t x = e / b, a = e % b;
    T[(r0 + x) * ldt + o + a] = G[e];
    T[(o + a) * ldt + r0 + x] = G[e];
  }
}

// res[j] = sqrt(u_j^T Zg u_j), u_j = U[j][o .. o + b): residual norm of Ritz pair j
__global__ void k_res_est(const double* U, int64_t ldu, int64_t n, int64_t o, int64_t b, const double* Zg,
                          double* res) {
  GRID_STRIDE(j, n) {
    const double* u = U + j * ldu + o;
    double acc = 0.0;
    for (int64_t a = 0; a < b; ++a) {
      double t = 0.0;
      for (int64_t c = 0; c < b; ++c) t += Zg[a * b + c] * u[c];
      acc += u[a] * t;
    }
    res[j] = sqrt(acc > 0.0 ? acc : 0.0);
  }
}

// restarted T (zeroed before): T[j][j] = theta[j] (j < kk); coupling of the new block
// T[kk + x][j] = T[j][kk + x] = sum_a G[x][a] U[j0 + j][o + a]
__global__ void k_restart_t(double* T, int64_t ldt, int64_t kk, int64_t b, const double* theta, const double* U,
                            int64_t ldu, int64_t j0, int64_t o, const double* G) {
  GRID_STRIDE(e, (b + 1) * kk) {
    const int64_t x = e / kk, j = e % kk;
    if (x == b) {
      T[j * ldt + j] = theta[j];
    } else {
      double acc = 0.0;
      for (int64_t a = 0; a < b; ++a) acc += G[x * b + a] * U[(j0 + j) * ldu + o + a];
      T[(kk + x) * ldt + j] = acc;
      T[j * ldt + kk + x] = acc;
    }
  }
}

struct LzBufs {
  int64_t b = 0, win = 0, keep = 0, K = 0;
  double *W, *W2, *L, *C, *Cp, *part, *T, *U, *w, *res, *G, *Zg;
  SyevBufs sy;
};

void plan_lanczos(Arena& ar, int64_t ldp, int64_t S, int64_t b, int64_t win, int64_t keep, int64_t K, LzBufs& z) {
  z.b = b;
  z.win = win;
  z.keep = keep;
  z.K = K;
  z.W = ar.take<double>(win * ldp);
  z.W2 = ar.take<double>(win * ldp);
  z.L = ar.take<double>(K * ldp);
  z.C = ar.take<double>(win * b);
  z.Cp = ar.take<double>(std::max(win, K) * b);
  z.part = ar.take<double>(S * std::max(win * b, K * K));
  z.T = ar.take<double>(win * win);
  z.U = ar.take<double>(win * win);
  z.w = ar.take<double>(win);
  z.res = ar.take<double>(win);
  z.G = ar.take<double>(b * b);
  z.Zg = ar.take<double>(b * b);
  plan_syev(ar, (int)win, z.sy);
}

// C (M x N, row-major) = A B^T over the ldp columns of the row blocks A (M rows) and
// B (N rows); split over KSPLIT columns, partials summed in split order.
void gram_mn(EigRun& r, const double* A, int64_t M, const double* B, int64_t N, double* part, double* C) {
  Exec& ex = *r.ex;
  EigBufs& e = *r.e;
  GemmArgs<double> g;
  g.M = M; g.N = N; g.K = KSPLIT;
  g.A = A; g.sam = e.ldp; g.sak = 1; g.sab = KSPLIT;
  g.B = B; g.sbk = 1; g.sbn = e.ldp; g.sbb = KSPLIT;
  g.C = part; g.scm = N; g.scn = 1; g.scb = M * N;
  g.alpha = 1.0; g.beta = 0.0; g.batch = e.S;
  gemm<double>(ex, g);
  LAUNCH(k_sum_splits, M * N, part, e.S, M * N, C);
}

// Z -= C^T A: removes from the b rows of Z their components along the M rows of A
void project_out(EigRun& r, const double* C, const double* A, int64_t M, double* Z) {
  EigBufs& e = *r.e;
  gemm_rm<double>(*r.ex, true, false, e.b, e.ldp, M, -1.0, C, e.b, A, e.ldp, 1.0, Z, e.ldp);
}

SyevBufs syev_view(const SyevBufs& s, int n) {
  SyevBufs v = s;
  v.n = n;
  v.cap = 3 * (int64_t)n * n + 4 * (int64_t)n + 16;
  return v;
}

// e.Q = orthonormal rows spanning e.Z's rows, orthogonal to the nw rows of Wb and the
// nl rows of z.L; z.G = e.Q e.Z^T.  Two Cholesky-QR passes (the first shifted), one more
// projection against Wb and L (which matters when Z is tiny, i.e. near an invariant
// subspace), two plain Cholesky-QR passes.
void lz_new_block(EigRun& r, LzBufs& z, const double* Wb, int64_t nw, int64_t nl) {
  Exec& ex = *r.ex;
  EigBufs& e = *r.e;
  const int64_t nb = e.b * e.ldp;
  hipMemcpyAsync(e.Y, e.Z, nb * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
  orth(r, e.Y, e.Q, 2);  // result in e.Y
  gram_mn(r, Wb, nw, e.Y, e.b, z.part, z.Cp);
  project_out(r, z.Cp, Wb, nw, e.Y);
  if (nl > 0) {
    gram_mn(r, z.L, nl, e.Y, e.b, z.part, z.Cp);
    project_out(r, z.Cp, z.L, nl, e.Y);
  }
  orth(r, e.Y, e.Q, 2, true);  // result in e.Y
  hipMemcpyAsync(e.Q, e.Y, nb * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
  gram_mn(r, e.Q, e.b, e.Z, e.b, z.part, z.G);
}

struct LzResult {
  int restarts = 0, applies = 0;
  double maxrel = 0.0;
  bool converged = false, ok = true;
};

LzResult lanczos_topk(EigRun& r, LzBufs& z, int64_t K, double tol, int max_restarts, uint64_t seed, double* lambda,
                      double* Qout) {
  Exec& ex = *r.ex;
  EigBufs& e = *r.e;
  LzResult out;
  const int64_t b = e.b, ldp = e.ldp, P = e.P, win = z.win, nb = b * ldp;
  const double margin = 0.5;
  for (double* x : {e.Q, e.Y, e.Z})
    if (launch_ok(ex)) hipLaunchKernelGGL(k_fill, dim3(grid_for(nb)), dim3(TPB), 0, ex.stream, x, nb, 0.0);
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_fill, dim3(grid_for(win * win)), dim3(TPB), 0, ex.stream, z.T, win * win, 0.0);
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_randn, dim3(grid_for(nb)), dim3(TPB), 0, ex.stream, seed, b, P, ldp, e.Y);
  orth(r, e.Y, e.Q);
  hipMemcpyAsync(z.W, e.Q, nb * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
  int64_t n = b, o = 0, nl = 0;
  double scale = 0.0;
  std::vector<double> w, res;
  for (;;) {
    apply_op(r, r.gc, e.Q, e.Z);
    ++out.applies;
    for (int pass = 0; pass < 2; ++pass) {
      double* c = pass == 0 ? z.C : z.Cp;
      gram_mn(r, z.W, n, e.Z, b, z.part, c);
      project_out(r, c, z.W, n, e.Z);
      if (pass == 1 && launch_ok(ex))
        hipLaunchKernelGGL(k_axpbypcz, dim3(grid_for(n * b)), dim3(TPB), 0, ex.stream, 1.0, z.C, 1.0, z.Cp, 0.0,
                           nullptr, n * b, z.C);
      if (nl > 0) {
        gram_mn(r, z.L, nl, e.Z, b, z.part, z.Cp);
        project_out(r, z.Cp, z.L, nl, e.Z);
      }
    }
    if (launch_ok(ex))
      hipLaunchKernelGGL(k_put_cols, dim3(grid_for(n * b)), dim3(TPB), 0, ex.stream, z.T, win, n, o, b, z.C);
    if (n + b <= win) {
      lz_new_block(r, z, z.W, n, nl);
      if (launch_ok(ex))
        hipLaunchKernelGGL(k_put_coupling, dim3(grid_for(b * b)), dim3(TPB), 0, ex.stream, z.T, win, n, o, b, z.G);
      hipMemcpyAsync(z.W + n * ldp, e.Q, nb * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
      o = n;
      n += b;
      continue;
    }
    // Rayleigh-Ritz on the full window
    ++out.restarts;
    SyevBufs sv = syev_view(z.sy, (int)n);
    if (!run_syev(ex, z.T, win, z.w, z.U, n, sv)) {
      out.ok = false;
      return out;
    }
    gram_mn(r, e.Z, b, e.Z, b, z.part, z.Zg);
    if (launch_ok(ex))
      hipLaunchKernelGGL(k_res_est, dim3(grid_for(n)), dim3(TPB), 0, ex.stream, z.U, n, n, o, b, z.Zg, z.res);
    w.assign(n, 0.0);
    res.assign(n, 0.0);
    hipMemcpyAsync(w.data(), z.w, n * sizeof(double), hipMemcpyDeviceToHost, ex.stream);
    hipMemcpyAsync(res.data(), z.res, n * sizeof(double), hipMemcpyDeviceToHost, ex.stream);
    if (hipStreamSynchronize(ex.stream) != hipSuccess || ex.ctx->fault_hit) {
      out.ok = false;
      return out;
    }
    scale = std::max(scale, std::fabs(w[0]));
    const int64_t need = K - nl;
    int64_t nc = 0;
    while (nc < need && std::isfinite(res[nc]) && res[nc] <= margin * tol * scale) ++nc;
    const bool last = nl + nc >= K || out.restarts >= max_restarts || !std::isfinite(w[0]);
    // at the restart cap, the leading unconverged Ritz vectors fill the remaining slots
    const int64_t take = last ? need : nc;
    if (take > 0) gemm_rm<double>(ex, false, false, take, ldp, n, 1.0, z.U, n, z.W, ldp, 0.0, z.L + nl * ldp, ldp);
    nl += take;
    if (last) {
      out.converged = nc >= need;
      break;
    }
    const int64_t kk = std::min<int64_t>(z.keep, n - nc);
    gemm_rm<double>(ex, false, false, kk, ldp, n, 1.0, z.U + nc * n, n, z.W, ldp, 0.0, z.W2, ldp);
    std::swap(z.W, z.W2);
    lz_new_block(r, z, z.W, kk, nl);
    if (launch_ok(ex))
      hipLaunchKernelGGL(k_fill, dim3(grid_for(win * win)), dim3(TPB), 0, ex.stream, z.T, win * win, 0.0);
    if (launch_ok(ex))
      hipLaunchKernelGGL(k_restart_t, dim3(grid_for((b + 1) * kk)), dim3(TPB), 0, ex.stream, z.T, win, kk, b,
                         z.w + nc, z.U, n, nc, o, z.G);
    hipMemcpyAsync(z.W + kk * ldp, e.Q, nb * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
    o = kk;
    n = kk + b;
  }
  // final Rayleigh-Ritz over the K locked vectors: M L into W2, in blocks of b rows
  for (int64_t c0 = 0; c0 < K; c0 += b) {
    const int64_t rows = std::min<int64_t>(b, K - c0);
    if (rows < b && launch_ok(ex))
      hipLaunchKernelGGL(k_fill, dim3(grid_for(nb)), dim3(TPB), 0, ex.stream, e.Q, nb, 0.0);
    hipMemcpyAsync(e.Q, z.L + c0 * ldp, rows * ldp * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
    apply_op(r, r.gc, e.Q, e.Z);
    ++out.applies;
    hipMemcpyAsync(z.W2 + c0 * ldp, e.Z, rows * ldp * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
  }
  gram_mn(r, z.L, K, z.W2, K, z.part, z.T);
  SyevBufs sv = syev_view(z.sy, (int)K);
  if (!run_syev(ex, z.T, K, z.w, z.U, K, sv)) {
    out.ok = false;
    return out;
  }
  gemm_rm<double>(ex, false, false, K, ldp, K, 1.0, z.U, K, z.L, ldp, 0.0, z.W, ldp);   // X
  gemm_rm<double>(ex, false, false, K, ldp, K, 1.0, z.U, K, z.W2, ldp, 0.0, z.L, ldp);  // M X
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_resid, dim3((unsigned)K), dim3(256), 0, ex.stream, z.L, z.W, z.w, P, ldp, z.res);
  w.assign(K, 0.0);
  res.assign(K, 0.0);
  hipMemcpyAsync(w.data(), z.w, K * sizeof(double), hipMemcpyDeviceToHost, ex.stream);
  hipMemcpyAsync(res.data(), z.res, K * sizeof(double), hipMemcpyDeviceToHost, ex.stream);
  hipMemcpyAsync(lambda, z.w, K * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_sign_copy, dim3((unsigned)K), dim3(256), 0, ex.stream, z.W, P, ldp, Qout);
  if (hipStreamSynchronize(ex.stream) != hipSuccess || ex.ctx->fault_hit) {
    out.ok = false;
    return out;
  }
  const double sc = std::max(std::fabs(w[0]), 1e-300);
  for (int64_t k = 0; k < K; ++k) out.maxrel = std::max(out.maxrel, res[k] / sc);
  if (!std::isfinite(out.maxrel) || out.maxrel > tol) out.converged = false;
  return out;
}

}  // namespace

struct TopkPlan {
  Model m;
  bool has_model = false;
  int64_t N = 0, P = 0, b = 0;
  int source = 0, which = 0, prec = 1, Mdtype = 0, max_iter = 200;
  double tol = 1e-5;
  int64_t oversample = 10;
  int method = 0;
  int64_t win = 0, keep = 0;  // method 1: window and kept Ritz vectors (b = block size)
};

static hess_status topk_validate(hess_ctx* ctx, const hess_mlp* mlp, const hess_data* d, int64_t K,
                                 const hess_eig_opts* o, TopkPlan& t, bool need_ptrs) {
  if (!o) return fail(ctx, HESS_E_ARG, "opts is NULL");
  t.source = o->source;
  t.which = o->which;
  if (t.source != 0 && t.source != 1) return fail(ctx, HESS_E_ARG, "opts.source must be 0 or 1");
  if (t.which != 0 && t.which != 1) return fail(ctx, HESS_E_ARG, "opts.which must be 0 or 1");
  hess_status s;
  if (t.source == 1) {
    if (need_ptrs && !o->M) return fail(ctx, HESS_E_ARG, "opts.M is NULL");
    if (o->M_dtype != HESS_F64 && o->M_dtype != HESS_F32) return fail(ctx, HESS_E_ARG, "bad opts.M_dtype");
    if (o->P < 1 || o->P > ((int64_t)1 << 31)) return fail(ctx, HESS_E_SHAPE, "opts.P out of range");
    t.P = o->P;
    t.Mdtype = o->M_dtype;
  } else {
    if ((s = validate_mlp(ctx, mlp, t.m, need_ptrs)) != HESS_OK) return s;
    if ((s = validate_data(ctx, d, need_ptrs)) != HESS_OK) return s;
    if (o->prec != HESS_P_F64 && o->prec != HESS_P_F32 && o->prec != HESS_P_F32_SPLIT)
      return fail(ctx, HESS_E_UNSUPPORTED, "matrix-free operator: F64 or F32");
    t.has_model = true;
    t.N = d->N;
    t.P = t.m.P;
    t.prec = o->prec;
  }
  t.oversample = o->oversample < 0 ? 10 : o->oversample;
  t.max_iter = o->max_iter <= 0 ? 200 : o->max_iter;
  t.tol = o->tol > 0 ? o->tol : 1e-5;
  if (K < 1 || K > t.P) return fail(ctx, HESS_E_SHAPE, "K out of range");
  t.method = o->method;
  if (t.method != 0 && t.method != 1) return fail(ctx, HESS_E_ARG, "opts.method must be 0 or 1");
  if (t.method == 1) {
    // block b <= (P - K) / 3 so that a window of K + 2b rows leaves room for one more block
    int64_t b = o->block > 0 ? o->block : 32;
    b = std::min<int64_t>(std::min<int64_t>(b, BMAX), (t.P - K) / 3);
    if (b < 1) return fail(ctx, HESS_E_SHAPE, "Lanczos: P must be at least K + 3");
    t.b = b;
    t.win = std::min<int64_t>(std::min<int64_t>(512, 3 * K + 3 * b), t.P - b);
    if (t.win < K + 2 * b) return fail(ctx, HESS_E_SHAPE, "Lanczos: K + 2 block must fit in a 512-row window");
    t.keep = std::min<int64_t>(2 * K + b, t.win - 2 * b);
    return HESS_OK;
  }
  t.b = std::min<int64_t>(rup(K + t.oversample, 16), t.P);
  if (t.b > BMAX) return fail(ctx, HESS_E_SHAPE, "K + oversample must not exceed 128");
  return HESS_OK;
}

hess_status topk_workspace(hess_ctx* ctx, const hess_mlp* mlp, const hess_data* d, int64_t K,
                           const hess_eig_opts* o, size_t* bytes) {
  TopkPlan t;
  hess_status s = topk_validate(ctx, mlp, d, K, o, t, false);
  if (s != HESS_OK) return s;
  Arena ar(nullptr);
  EigBufs e;
  *bytes = plan_eig(ar, t.has_model ? &t.m : nullptr, t.N, t.P, t.b, t.source, t.prec, t.Mdtype, e);
  if (t.method == 1) {
    LzBufs z;
    plan_lanczos(ar, e.ldp, e.S, t.b, t.win, t.keep, K, z);
    *bytes = ar.used;
  }
  return HESS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" hess_status hess_topk_eig(hess_ctx* ctx, const hess_mlp* mlp, const hess_data* d, int64_t K,
                                     const hess_eig_opts* opts, double* lambda, double* Qout,
                                     hess_eig_info* info, void* ws, size_t ws_bytes) {
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  TopkPlan t;
  if ((s = topk_validate(ctx, mlp, d, K, opts, t, true)) != HESS_OK) return s;
  if (!lambda || !Qout) return fail(ctx, HESS_E_ARG, "lambda or Q is NULL");
  Arena probe(nullptr);
  EigBufs e0;
  size_t need = plan_eig(probe, t.has_model ? &t.m : nullptr, t.N, t.P, t.b, t.source, t.prec, t.Mdtype, e0);
  LzBufs z;
  if (t.method == 1) {
    plan_lanczos(probe, e0.ldp, e0.S, t.b, t.win, t.keep, K, z);
    need = probe.used;
  }
  if ((s = check_ws(ctx, need, ws, ws_bytes, (size_t)K * (t.P + 1) * 8)) != HESS_OK) return s;
  Arena ar(ws);
  EigBufs e;
  plan_eig(ar, t.has_model ? &t.m : nullptr, t.N, t.P, t.b, t.source, t.prec, t.Mdtype, e);
  if (t.method == 1) plan_lanczos(ar, e.ldp, e.S, t.b, t.win, t.keep, K, z);
  if (t.source == 0) {
    if ((s = check_inputs(ex, t.m, d, e.p)) != HESS_OK) return s;
    run_prep(ex, t.m, d, e.p, false);
    if (t.prec == HESS_P_F64)
      hvp_setup<double>(ex, t.m, t.N, e.p, e.hd);
    else
      hvp_setup<float>(ex, t.m, t.N, e.p, e.hf);
  }
  set_lds_limits();
  // matrix-free FP32 operator with split-BF16 products in its GEMMs
  ex.split = t.source == 0 && t.prec == HESS_P_F32_SPLIT;
  EigRun r{&ex, &e, t.has_model ? &t.m : nullptr, t.N, t.source, t.which, t.prec, t.Mdtype,
           t.source == 1 ? opts->M : nullptr};
  GraphCache graphs;  // destroyed after the call has synchronised (finish)
  if (ctx->graphs) r.gc = &graphs;
  if (t.method == 1) {
    const LzResult lr = lanczos_topk(r, z, K, t.tol, t.max_iter, (uint64_t)opts->seed, lambda, Qout);
    if (info) {
      info->iters = lr.restarts;
      info->applies = lr.applies;
      info->max_rel_residual = lr.maxrel;
      info->shift_used = 0.0;
    }
    s = finish(ex, "hess_topk_eig");
    if (s != HESS_OK) return s;
    if (!lr.ok) return fail(ctx, HESS_E_NOCONV, "Lanczos: projected eigenproblem did not converge");
    if (!lr.converged)
      return fail(ctx, HESS_E_NOCONV,
                  "no convergence within max_iter restarts (max rel residual " + std::to_string(lr.maxrel) + ")");
    return HESS_OK;
  }
  const int64_t nb = e.b * e.ldp;
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_fill, dim3(grid_for(16)), dim3(TPB), 0, ex.stream, reinterpret_cast<double*>(e.info),
                       (int64_t)8, 0.0);
  for (double* x : {e.Y, e.Yp, e.Z, e.MQ, e.X, e.MX})
    if (launch_ok(ex)) hipLaunchKernelGGL(k_fill, dim3(grid_for(nb)), dim3(TPB), 0, ex.stream, x, nb, 0.0);
  if (launch_ok(ex))
    hipLaunchKernelGGL(k_randn, dim3(grid_for(nb)), dim3(TPB), 0, ex.stream, (uint64_t)opts->seed, e.b, e.P,
                       e.ldp, e.Y);
  orth(r, e.Y, e.Q);
  int applies = 0;
  // a few unfiltered block steps: estimate of the spectral radius
  for (int it = 0; it < 3; ++it) {
    apply_op(r, r.gc, e.Q, e.Y);
    ++applies;
    orth(r, e.Y, e.Q);
  }
  rayleigh_ritz(r, nullptr);
  ++applies;
  std::vector<double> theta, res;
  int hinfo[16];
  if (!read_back(ex, e, theta, res, hinfo)) return finish(ex, "hess_topk_eig");
  double rho = 0.0;
  for (int64_t k = 0; k < e.b; ++k) rho = std::max(rho, std::fabs(theta[k]) + res[k]);
  const double lb = t.which == 1 ? -0.01 * rho : -1.5 * rho;  // the OPG is positive semidefinite
  const int degree = 8;
  int iters = 0;
  double maxrel = 0.0;
  bool converged = false;
  for (;;) {
    maxrel = 0.0;
    const double scale = std::max(std::fabs(theta[0]), 1e-300);
    for (int64_t k = 0; k < K; ++k) maxrel = std::max(maxrel, res[k] / scale);
    if (!std::isfinite(maxrel)) break;
    if (maxrel <= t.tol) {
      converged = true;
      break;
    }
    if (iters >= t.max_iter) break;
    ++iters;
    // Chebyshev filter on [lb, a]: Y_1 = (M X - c X) / e, Y_{j+1} = 2 (M Y_j - c Y_j) / e - Y_{j-1}
    double a = theta[e.b - 1];
    if (!(a > lb)) a = lb + 0.1 * (rho - lb);
    const double c = 0.5 * (a + lb), hw = 0.5 * (a - lb);
    // The filter grows the top of the spectrum by about T_m(mu_1), mu_1 = (rho - c) / hw,
    // against at most 1 on [lb, a].  A large growth (a narrow interval far below rho, as
    // for the OPG with its small trailing eigenvalues) would push the block's wanted
    // directions near a below the FP64 rounding of the leading ones, and the
    // orthonormalisation would lose them; so the degree keeps T_m(mu_1) below about 1e8.
    const double mu1 = (rho - c) / hw;
    const int deg = mu1 > 1.0 ? std::max(2, std::min(degree, (int)std::floor(std::log(2e8) / std::acosh(mu1))))
                              : degree;
    if (launch_ok(ex))
      hipLaunchKernelGGL(k_axpbypcz, dim3(grid_for(nb)), dim3(TPB), 0, ex.stream, 1.0 / hw, e.MX, -c / hw, e.X,
                         0.0, nullptr, nb, e.Y);
    hipMemcpyAsync(e.Yp, e.X, nb * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
    for (int j = 1; j < deg; ++j) {
      apply_op(r, r.gc, e.Y, e.Z);
      ++applies;
      // Z <- 2 (Z - c Y) / hw - Yp ; then rotate (Yp, Y) <- (Y, Z)
      if (launch_ok(ex))
        hipLaunchKernelGGL(k_axpbypcz, dim3(grid_for(nb)), dim3(TPB), 0, ex.stream, 2.0 / hw, e.Z, -2.0 * c / hw,
                           e.Y, -1.0, e.Yp, nb, e.Z);
      std::swap(e.Yp, e.Y);
      std::swap(e.Y, e.Z);
    }
    orth(r, e.Y, e.Q);
    rayleigh_ritz(r, nullptr);
    ++applies;
    if (!read_back(ex, e, theta, res, hinfo)) return finish(ex, "hess_topk_eig");
  }
  // outputs: lambda (K), Q (K x P) sign-normalised
  hipMemcpyAsync(lambda, e.theta, K * sizeof(double), hipMemcpyDeviceToDevice, ex.stream);
  if (launch_ok(ex)) hipLaunchKernelGGL(k_sign_copy, dim3((unsigned)K), dim3(256), 0, ex.stream, e.X, e.P, e.ldp, Qout);
  if (info) {
    info->iters = iters;
    info->applies = applies;
    info->max_rel_residual = maxrel;
    info->shift_used = lb;
  }
  s = finish(ex, "hess_topk_eig");
  if (s != HESS_OK) return s;
  if (!converged)
    return fail(ctx, HESS_E_NOCONV, "no convergence within max_iter (max rel residual " + std::to_string(maxrel) + ")");
  return HESS_OK;
}
