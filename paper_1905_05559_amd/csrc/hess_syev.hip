// Eigen-decomposition of a small dense symmetric FP64 matrix (n <= 512) on the device:
// the projected (Rayleigh-Ritz) problem of the block Lanczos eigensolver (paper,
// Sec. 5.3: the K leading eigenpairs come from the Lanczos projection of H), also
// exported on its own.
//
//  1. Householder reduction to tridiagonal form T_t = Q^T A Q (one workgroup; the
//     n x n working copy stays in L2).  Reflector k is v_k = e_1 + ..., stored in row
//     k of the working copy, with H_k = I - tau_k v_k v_k^T.
//  2. Q = H_0 H_1 ... H_{n-3} by backward accumulation, 32 columns per workgroup
//     held in LDS.
//  3. Implicit-shift QL on T_t (Wilkinson-type shift, deflation when
//     |e_m| <= eps (|d_m| + |d_{m+1}|)).  One lane runs the serial rotation chain and
//     records every rotation; the recorded sequence is then applied to the rows of Q,
//     32 rows per workgroup held in LDS, one lane per row.  Recording happens in
//     chunks of bounded length, alternating with the application.
//  4. Eigenvalues sorted descending (ties by index), eigenvectors written as rows and
//     sign-normalised (largest-magnitude component positive, first index on ties).
#include <algorithm>
#include <cmath>
#include <vector>

#include "api_internal.h"

namespace hs {

namespace {

constexpr int NMAX = 512;
constexpr int TRED_T = 1024;  // threads of the reduction workgroup (16 wavefronts)
constexpr int COLS = 32;      // columns (Q accumulation) or rows (rotations) per workgroup
constexpr int QSTR = COLS + 1;  // LDS row stride of the column blocks (bank spread)

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 1024 threads in a fixed order; every thread gets the same value.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < TRED_T / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// W = (A + A^T) / 2, n x n, from A with row stride lda.
__global__ void k_sym_copy(const double* A, int64_t lda, int n, double* W) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    W[e] = 0.5 * (A[i * lda + j] + A[j * lda + i]);
  }
}

// Householder tridiagonalisation in place; d (n), e (n, e[i] couples i and i+1), tau.
__global__ __launch_bounds__(TRED_T) void k_tred(double* A, int n, double* d, double* e, double* tau) {
  __shared__ double v[NMAX];
  __shared__ double p[NMAX];
  __shared__ double red[TRED_T / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int k = 0; k < n - 2; ++k) {
    const int m = n - k - 1;
    double* xr = A + (int64_t)k * n + (k + 1);  // row k right of the diagonal = column k below it
    double s = 0.0;
    for (int j = 1 + t; j < m; j += TRED_T) {
      const double x = xr[j];
      s += x * x;
    }
    s = block_sum(s, red);
    const double alpha = xr[0];
    double tk = 0.0, beta = alpha, sc = 0.0;
    if (s != 0.0) {
      const double nrm = sqrt(alpha * alpha + s);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tk = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    for (int j = t; j < m; j += TRED_T) v[j] = j == 0 ? 1.0 : xr[j] * sc;
    __syncthreads();
    for (int j = t; j < m; j += TRED_T) xr[j] = v[j];
    if (t == 0) {
      d[k] = A[(int64_t)k * n + k];
      e[k] = beta;
      tau[k] = tk;
    }
    if (tk != 0.0) {
      double* A22 = A + (int64_t)(k + 1) * n + (k + 1);
      // p = tau A22 v
      for (int i = wv; i < m; i += TRED_T / 64) {
        const double* row = A22 + (int64_t)i * n;
        double acc = 0.0;
        for (int j = lane; j < m; j += 64) acc += row[j] * v[j];
        acc = wave_sum(acc);
        if (lane == 0) p[i] = tk * acc;
      }
      __syncthreads();
      double pv = 0.0;
      for (int i = t; i < m; i += TRED_T) pv += p[i] * v[i];
      pv = block_sum(pv, red);
      const double kc = 0.5 * tk * pv;
      for (int i = t; i < m; i += TRED_T) p[i] -= kc * v[i];  // p becomes w
      __syncthreads();
      // A22 -= v w^T + w v^T
      for (int i = wv; i < m; i += TRED_T / 64) {
        double* row = A22 + (int64_t)i * n;
        const double vi = v[i], wi = p[i];
        for (int j = lane; j < m; j += 64) row[j] -= vi * p[j] + wi * v[j];
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    if (n >= 2) {
      d[n - 2] = A[(int64_t)(n - 2) * n + (n - 2)];
      e[n - 2] = A[(int64_t)(n - 2) * n + (n - 1)];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = A[(int64_t)(n - 1) * n + (n - 1)];
    e[n - 1] = 0.0;
    tau[n - 1] = 0.0;
  }
}

// Q = H_0 ... H_{n-3}: columns [32 blockIdx.x, +32) accumulated in LDS (n x 33 doubles).
__global__ __launch_bounds__(256) void k_form_q(const double* A, const double* tau, int n, double* Q) {
  extern __shared__ double sm[];
  double* ql = sm;                     // n x QSTR
  double* v = sm + (size_t)n * QSTR;   // n
  const int c0 = blockIdx.x * COLS;
  const int t = threadIdx.x, c = t >> 3, part = t & 7;
  for (int e = t; e < n * COLS; e += blockDim.x) {
    const int r = e / COLS, cc = e % COLS;
    ql[r * QSTR + cc] = (r == c0 + cc) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    if (tau[k] == 0.0 || c0 + COLS - 1 < k + 1) continue;  // uniform in the workgroup
    const int m = n - k - 1;
    const double* vr = A + (int64_t)k * n + (k + 1);
    for (int j = t; j < m; j += blockDim.x) v[j] = vr[j];
    __syncthreads();
    double acc = 0.0;
    for (int i = part; i < m; i += 8) acc += v[i] * ql[(k + 1 + i) * QSTR + c];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    const double f = tau[k] * acc;
    for (int i = part; i < m; i += 8) ql[(k + 1 + i) * QSTR + c] -= f * v[i];
    __syncthreads();
  }
  for (int e = t; e < n * COLS; e += blockDim.x) {
    const int r = e / COLS, cc = e % COLS;
    if (c0 + cc < n) Q[(int64_t)r * n + c0 + cc] = ql[r * QSTR + cc];
  }
}

// State of the QL iteration kept between chunks (ints): done, error, l, iterations
// at l, entries written in the current chunk.
enum { ST_DONE = 0, ST_ERR = 1, ST_L = 2, ST_IT = 3, ST_LEN = 4, ST_N = 8 };
constexpr int QL_MAXIT = 60;

// r = sqrt(f^2 + g^2) and ir = 1 / r from the hardware reciprocal square root refined by
// two Newton steps (y <- y + y (1 - q y^2) / 2; each step doubles the correct bits).
// Returns false (r = the scaled hypot, ir unset) where q = f^2 + g^2 is zero, tiny or
// not finite, so the caller falls back to a division.
__device__ __forceinline__ bool rot_rsqrt(double f, double g, double& r, double& ir) {
  const double q = f * f + g * g;
  if (q > 1e-280 && q < 1e280) {
    double y = __builtin_amdgcn_rsq(q);
    double h = fma(-q * y, y, 1.0);
    y = fma(0.5 * h, y, y);
    h = fma(-q * y, y, 1.0);
    y = fma(0.5 * h, y, y);
    ir = y;
    r = q * y;
    return true;
  }
  const double af = fabs(f), ag = fabs(g), mx = af > ag ? af : ag, mn = af > ag ? ag : af;
  r = mx == 0.0 ? 0.0 : mx * sqrt(1.0 + (mn / mx) * (mn / mx));
  return false;
}

__global__ void k_ql_init(int* st) {
  if (threadIdx.x < ST_N) st[threadIdx.x] = 0;
}

// Implicit-shift QL on (d, e), lane 0 only; records rotations as double2 entries:
// a header {first index i0, count} followed by count entries {c, s} for i = i0, i0-1, ...
// Stops before an iteration that might not fit in cap entries.
__global__ __launch_bounds__(64) void k_ql_chain(double* dg, double* eg, int n, double2* rot, int64_t cap, int* st) {
  __shared__ double d[NMAX];
  __shared__ double e[NMAX];
  if (st[ST_DONE] || st[ST_ERR]) {
    if (threadIdx.x == 0) st[ST_LEN] = 0;
    return;
  }
  for (int i = threadIdx.x; i < n; i += 64) {
    d[i] = dg[i];
    e[i] = eg[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double eps = 2.220446049250313e-16;
    int l = st[ST_L], it = st[ST_IT];
    int64_t pos = 0;
    bool full = false;
    while (l < n && !full) {
      int m = l;
      while (m < n - 1) {
        const double dd = fabs(d[m]) + fabs(d[m + 1]);
        if (fabs(e[m]) <= eps * dd) break;
        ++m;
      }
      if (m == l) {
        ++l;
        it = 0;
        continue;
      }
      if (pos + (m - l) + 1 > cap) {
        full = true;
        break;
      }
      if (++it > QL_MAXIT) {
        st[ST_ERR] = 1;
        break;
      }
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = sqrt(g * g + 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      const int64_t hdr = pos++;
      int cnt = 0;
      bool under = false;
      // d[i + 1] is carried in a register; e[i], d[i] are read one step ahead
      double di1 = d[m], ei = e[m - 1], di = d[m - 1];
      for (int i = m - 1; i >= l; --i) {
        const int ip = i > l ? i - 1 : i;  // unconditional read (the value is unused at i = l)
        const double en = e[ip], dn = d[ip];
        const double f = s * ei, b = c * ei;
        double ir;
        if (!rot_rsqrt(f, g, r, ir)) {
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] = di1 - p;
            e[m] = 0.0;
            under = true;
            break;
          }
          ir = 1.0 / r;
        }
        e[i + 1] = r;
        s = f * ir;
        c = g * ir;
        g = di1 - p;
        r = (di - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        rot[pos++] = make_double2(c, s);
        ++cnt;
        di1 = di;
        ei = en;
        di = dn;
      }
      rot[hdr] = make_double2((double)(m - 1), (double)cnt);
      if (under) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
    st[ST_L] = l;
    st[ST_IT] = it;
    st[ST_LEN] = (int)pos;
    if (l >= n) st[ST_DONE] = 1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 64) {
    dg[i] = d[i];
    eg[i] = e[i];
  }
}

// Applies the recorded rotations to rows [32 blockIdx.x, +32) of Q (held in LDS as
// z[column][row]); rotation (c, s) at i maps columns (i, i+1) to
// (c z_i - s z_{i+1}, s z_i + c z_{i+1}).
__global__ __launch_bounds__(64) void k_ql_apply(double* Q, int n, const double2* rot, const int* st) {
  extern __shared__ double z[];  // n x COLS
  const int len = st[ST_LEN];
  if (len == 0) return;
  const int r0 = blockIdx.x * COLS, t = threadIdx.x;
  for (int e = t; e < n * COLS; e += 64) {
    const int col = e / COLS, rr = e % COLS;
    z[e] = (r0 + rr < n) ? Q[(int64_t)(r0 + rr) * n + col] : 0.0;
  }
  __syncthreads();
  if (t < COLS) {
    int pos = 0;
    while (pos < len) {
      const double2 h = rot[pos++];
      const int i0 = (int)h.x, cnt = (int)h.y;
      double carry = z[(i0 + 1) * COLS + t];
      int q = 0;
      for (; q + 8 <= cnt; q += 8) {
        double2 g[8];
        double zz[8];
        const int i = i0 - q;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          g[u] = rot[pos + q + u];
          zz[u] = z[(i - u) * COLS + t];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          z[(i - u + 1) * COLS + t] = g[u].y * zz[u] + g[u].x * carry;
          carry = g[u].x * zz[u] - g[u].y * carry;
        }
      }
      for (; q < cnt; ++q) {
        const double2 g = rot[pos + q];
        const int i = i0 - q;
        const double zi = z[i * COLS + t];
        z[(i + 1) * COLS + t] = g.y * zi + g.x * carry;
        carry = g.x * zi - g.y * carry;
      }
      z[(i0 - cnt + 1) * COLS + t] = carry;
      pos += cnt;
    }
  }
  __syncthreads();
  for (int e = t; e < n * COLS; e += 64) {
    const int col = e / COLS, rr = e % COLS;
    if (r0 + rr < n) Q[(int64_t)(r0 + rr) * n + col] = z[e];
  }
}

// Descending order of d (ties by index): perm[rank] = i, w[rank] = d[i].
__global__ void k_sort_desc(const double* d, int n, int* perm, double* w) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double di = d[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = d[j];
      rank += (dj > di || (dj == di && j < i)) ? 1 : 0;
    }
    perm[rank] = i;
    w[rank] = di;
  }
}

// U[r][c] = s_r Q[c][perm[r]], s_r making the largest-magnitude entry of row r positive.
__global__ __launch_bounds__(256) void k_rows_out(const double* Q, int n, const int* perm, double* U, int64_t ldu) {
  __shared__ double vmax[256];
  __shared__ int imax[256];
  const int r = blockIdx.x, col = perm[r];
  double best = -1.0;
  int bi = n;
  for (int c = threadIdx.x; c < n; c += 256) {
    const double a = fabs(Q[(int64_t)c * n + col]);
    if (a > best) {
      best = a;
      bi = c;
    }
  }
  vmax[threadIdx.x] = best;
  imax[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = vmax[threadIdx.x + w];
      const int oi = imax[threadIdx.x + w];
      if (o > vmax[threadIdx.x] || (o == vmax[threadIdx.x] && oi < imax[threadIdx.x])) {
        vmax[threadIdx.x] = o;
        imax[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = (imax[0] < n && Q[(int64_t)imax[0] * n + col] < 0.0) ? -1.0 : 1.0;
  for (int c = threadIdx.x; c < n; c += 256) U[(int64_t)r * ldu + c] = sg * Q[(int64_t)c * n + col];
}

void set_syev_lds() {
  static bool done = false;
  if (done) return;
  const int lim = 150 * 1024;
  (void)hipFuncSetAttribute((const void*)k_form_q, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_ql_apply, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  done = true;
}

}  // namespace

void plan_syev(Arena& ar, int n, SyevBufs& s) {
  s.n = n;
  s.A = ar.take<double>((size_t)n * n);
  s.Q = ar.take<double>((size_t)n * n);
  s.d = ar.take<double>(n);
  s.e = ar.take<double>(n);
  s.tau = ar.take<double>(n);
  s.cap = 3 * (int64_t)n * n + 4 * (int64_t)n + 16;
  s.rot = ar.take<double>(2 * (size_t)s.cap);
  s.st = ar.take<int>(ST_N);
  s.perm = ar.take<int>(n);
}

// Runs steps 1-4 on the stream; returns false on a device error or when the QL
// iteration limit was reached (the host reads the state once per recorded chunk).
bool run_syev(Exec& ex, const double* A, int64_t lda, double* w, double* U, int64_t ldu, SyevBufs& s) {
  const int n = s.n;
  set_syev_lds();
  if (!launch_ok(ex)) return false;
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_sym_copy, dim3((unsigned)std::min<int64_t>((nn + 255) / 256, 4096)), dim3(256), 0, ex.stream,
                     A, lda, n, s.A);
  hipLaunchKernelGGL(k_tred, dim3(1), dim3(TRED_T), 0, ex.stream, s.A, n, s.d, s.e, s.tau);
  const unsigned nb = (unsigned)((n + COLS - 1) / COLS);
  hipLaunchKernelGGL(k_form_q, dim3(nb), dim3(256), (size_t)(n * QSTR + n) * sizeof(double), ex.stream, s.A, s.tau,
                     n, s.Q);
  hipLaunchKernelGGL(k_ql_init, dim3(1), dim3(64), 0, ex.stream, s.st);
  int st[ST_N] = {0};
  // chunks: typically one (about 1.1 n^2 rotations against a capacity of 3 n^2)
  for (int chunk = 0; chunk < 4 * QL_MAXIT; ++chunk) {
    if (!launch_ok(ex)) return false;
    hipLaunchKernelGGL(k_ql_chain, dim3(1), dim3(64), 0, ex.stream, s.d, s.e, n, reinterpret_cast<double2*>(s.rot),
                       s.cap, s.st);
    hipLaunchKernelGGL(k_ql_apply, dim3(nb), dim3(64), (size_t)n * COLS * sizeof(double), ex.stream, s.Q, n,
                       reinterpret_cast<const double2*>(s.rot), s.st);
    hipMemcpyAsync(st, s.st, sizeof(st), hipMemcpyDeviceToHost, ex.stream);
    if (hipStreamSynchronize(ex.stream) != hipSuccess) {
      ex.ctx->fault_hit = true;
      return false;
    }
    if (st[ST_DONE] || st[ST_ERR]) break;
  }
  if (!st[ST_DONE] || st[ST_ERR]) return false;
  if (!launch_ok(ex)) return false;
  hipLaunchKernelGGL(k_sort_desc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ex.stream, s.d, n, s.perm, w);
  hipLaunchKernelGGL(k_rows_out, dim3((unsigned)n), dim3(256), 0, ex.stream, s.Q, n, s.perm, U, ldu);
  return true;
}

hess_status syev_workspace(hess_ctx* ctx, int64_t n, size_t* bytes) {
  if (n < 1 || n > NMAX) return fail(ctx, HESS_E_SHAPE, "syev: n must be in 1..512");
  Arena ar(nullptr);
  SyevBufs s;
  plan_syev(ar, (int)n, s);
  *bytes = ar.used;
  return HESS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" hess_status hess_syev(hess_ctx* ctx, int64_t n, const double* A, int64_t lda, double* w, double* U,
                                 void* ws, size_t ws_bytes) {
  Exec ex;
  hess_status s = begin(ctx, ex);
  if (s != HESS_OK) return s;
  if (n < 1 || n > NMAX) return fail(ctx, HESS_E_SHAPE, "syev: n must be in 1..512");
  if (lda < n) return fail(ctx, HESS_E_SHAPE, "syev: lda < n");
  if (!A || !w || !U) return fail(ctx, HESS_E_ARG, "NULL pointer");
  Arena probe(nullptr);
  SyevBufs sb;
  plan_syev(probe, (int)n, sb);
  if ((s = check_ws(ctx, probe.used, ws, ws_bytes, (size_t)n * (n + 1) * 8)) != HESS_OK) return s;
  Arena ar(ws);
  plan_syev(ar, (int)n, sb);
  const bool ok = run_syev(ex, A, lda, w, U, n, sb);
  s = finish(ex, "hess_syev");
  if (s != HESS_OK) return s;
  if (!ok) return fail(ctx, HESS_E_NOCONV, "syev: QL iteration limit reached");
  return HESS_OK;
}
