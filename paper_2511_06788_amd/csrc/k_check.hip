// Set-up kernels outside the step: the positive-definiteness check of the
// operator (a Lanczos run on one vector), the Cholesky factor of an inner
// matrix for re-orthonormalising a block, and small device-scalar copies.
//
// Positive definiteness (the coercivity of a(u,v), Section 2.2, that makes
// G = H^{-1} exist): every Ritz value of a Krylov space of H lies in
// [lambda_min, lambda_max], so a Ritz value <= 0 proves H is not SPD.  The
// Lanczos recurrence on one vector from a seeded pseudo-random start,
//   w = H v_j - beta_{j-1} v_{j-1},  alpha_j = w.v_j,  w -= alpha_j v_j,
//   beta_j = |w|,  v_{j+1} = w / beta_j,
// runs here; the host takes the smallest and largest eigenvalues of the
// tridiagonal matrix (alpha, beta) by Sturm-sequence bisection.
#include <math.h>

#include "ope_internal.h"

namespace {

constexpr int LW = 256;        // threads of the vector kernels
constexpr int RW = 1024;       // threads of the one-work-group reductions

// 64-bit mix (SplitMix64 finaliser, Steele, Lea & Flood 2014) of a counter:
// the start vector is a function of the point index and the seed only.
__device__ __forceinline__ double start_value(uint64_t p, uint64_t seed) {
  uint64_t z = p + seed * 0x9E3779B97F4A7C15ull + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// v = start vector, partial sums of v.v
__global__ __launch_bounds__(LW) void k_lz_start(double* __restrict__ v, uint64_t n, uint64_t seed,
                                                 double* __restrict__ part) {
  __shared__ double sh[LW];
  double s = 0.0;
  for (uint64_t p = (uint64_t)blockIdx.x * LW + threadIdx.x; p < n; p += (uint64_t)gridDim.x * LW) {
    const double x = start_value(p, seed);
    v[p] = x;
    s += x * x;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// (H x)_p for one vector: d_p x_p - sum over axes of c_a (x_{p-s_a} + x_{p+s_a})
__device__ __forceinline__ double apply_point(const double* __restrict__ x, const double* __restrict__ diag,
                                              const OpeGrid& g, uint64_t p) {
  const uint32_t i0 = (uint32_t)(p % g.m0);
  const uint64_t r = p / g.m0;
  const uint32_t i1 = (uint32_t)(r % g.m1);
  const uint32_t i2 = (uint32_t)(r / g.m1);
  double nx = 0.0, ny = 0.0, nz = 0.0;
  if (i0 > 0) nx += x[p - 1];
  if (i0 + 1 < g.m0) nx += x[p + 1];
  if (i1 > 0) ny += x[p - g.s1];
  if (i1 + 1 < g.m1) ny += x[p + g.s1];
  if (g.dim == 3) {
    if (i2 > 0) nz += x[p - g.s2];
    if (i2 + 1 < g.m2) nz += x[p + g.s2];
  }
  return diag[p] * x[p] - (g.cx * nx + g.cy * ny + g.cz * nz);
}

// w = (H v) * sv - b * u with sv = 1 / scale[0] (the pending normalisation of
// v), b = beta[j-1] (0 at j = 0); partial sums of w.v * sv.
__global__ __launch_bounds__(LW) void k_lz_apply(const double* __restrict__ v, const double* __restrict__ u,
                                                 double* __restrict__ w, const double* __restrict__ diag, OpeGrid g,
                                                 uint64_t n, const double* __restrict__ vscale,
                                                 const double* __restrict__ bprev, double* __restrict__ part) {
  __shared__ double sh[LW];
  const double sv = 1.0 / vscale[0];
  const double b = bprev ? bprev[0] : 0.0;
  double s = 0.0;
  for (uint64_t p = (uint64_t)blockIdx.x * LW + threadIdx.x; p < n; p += (uint64_t)gridDim.x * LW) {
    const double hv = apply_point(v, diag, g, p) * sv;
    const double x = hv - (u ? b * u[p] : 0.0);
    w[p] = x;
    s += x * (v[p] * sv);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// w -= alpha v * sv, v <- v * sv (normalised in place); partial sums of w.w
__global__ __launch_bounds__(LW) void k_lz_orth(double* __restrict__ v, double* __restrict__ w, uint64_t n,
                                                const double* __restrict__ vscale, const double* __restrict__ alpha,
                                                double* __restrict__ part) {
  __shared__ double sh[LW];
  const double sv = 1.0 / vscale[0];
  const double a = alpha[0];
  double s = 0.0;
  for (uint64_t p = (uint64_t)blockIdx.x * LW + threadIdx.x; p < n; p += (uint64_t)gridDim.x * LW) {
    const double vn = v[p] * sv;
    v[p] = vn;
    const double x = w[p] - a * vn;
    w[p] = x;
    s += x * x;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[0] = sum of part (fixed order); mode 1: out = sqrt(sum) (a norm)
__global__ __launch_bounds__(RW) void k_lz_sum(const double* __restrict__ part, uint32_t count, int mode,
                                               double* __restrict__ out) {
  __shared__ double sh[RW];
  double s = 0.0;
  for (uint32_t k = threadIdx.x; k < count; k += RW) s += part[k];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = mode ? sqrt(s) : s;
}

// Cholesky factor of an SPD N x N matrix (row-major, in place in A: the lower
// triangle receives L with A = L L^T), then X = L^{-1} (lower triangular) and
// Rinv = X^T = R^{-1} for R = L^T.  One work-group, right-looking; bad = 1 if a
// pivot is not a finite positive number.
__global__ __launch_bounds__(RW) void k_chol_rinv(double* __restrict__ A, uint32_t N, double* __restrict__ Rinv,
                                                  OpeScalars* __restrict__ sc) {
  __shared__ double piv;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (uint32_t k = 0; k < N; ++k) {
    if (threadIdx.x == 0) {
      const double d = A[(uint64_t)k * N + k];
      if (!(d > 0.0) || !isfinite(d)) bad = 1;
      piv = d > 0.0 ? sqrt(d) : 1.0;
      A[(uint64_t)k * N + k] = piv;
    }
    __syncthreads();
    for (uint32_t i = k + 1 + threadIdx.x; i < N; i += RW) A[(uint64_t)i * N + k] /= piv;
    __syncthreads();
    const uint32_t m = N - k - 1;
    for (uint64_t q = threadIdx.x; q < (uint64_t)m * m; q += RW) {
      const uint32_t i = k + 1 + (uint32_t)(q / m), j = k + 1 + (uint32_t)(q % m);
      if (j <= i) A[(uint64_t)i * N + j] -= A[(uint64_t)i * N + k] * A[(uint64_t)j * N + k];
    }
    __syncthreads();
  }
  // column c of X = L^{-1}: forward substitution, one thread per column
  for (uint32_t c = threadIdx.x; c < N; c += RW) {
    for (uint32_t i = 0; i < N; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (uint32_t k = c; k < i; ++k) s -= A[(uint64_t)i * N + k] * Rinv[(uint64_t)c * N + k];
      Rinv[(uint64_t)c * N + i] = i < c ? 0.0 : s / A[(uint64_t)i * N + i];
    }
  }
  // Rinv currently holds X^T row-wise: Rinv[c][i] = X[i][c] = (R^{-1})[c][i]
  __syncthreads();
  if (threadIdx.x == 0 && bad && sc->err == 0) sc->err = OPE_ENOTSPD;
}

__global__ void k_scalar_copy(const OpeScalars* __restrict__ sc, int which, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  out[0] = which == 0 ? sc->energy : (which == 1 ? sc->residual : sc->drift);
}

}  // namespace

static hipError_t lz_launch_dims(uint64_t n, uint32_t* blocks) {
  uint64_t b = (n + LW - 1) / LW;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  *blocks = (uint32_t)b;
  return hipSuccess;
}

// Smallest and largest eigenvalue of the symmetric tridiagonal matrix with
// diagonal a[0..k) and off-diagonal b[0..k-1), by bisection on the Sturm count
// (number of eigenvalues below x = number of negative pivots of T - x I).
static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, int k, double x) {
  int cnt = 0;
  double q = a[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < k; ++i) {
    const double den = q != 0.0 ? q : 1e-300;
    q = a[i] - x - b[i - 1] * b[i - 1] / den;
    if (q < 0) ++cnt;
  }
  return cnt;
}

static void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, int k, double* lo_eig,
                             double* hi_eig) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  auto bis = [&](int target) {   // the target-th eigenvalue (0-based)
    double l = lo, h = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (l + h);
      if (mid == l || mid == h) break;
      if (sturm_count(a, b, k, mid) > target) h = mid;
      else l = mid;
    }
    return 0.5 * (l + h);
  };
  *lo_eig = bis(0);
  *hi_eig = bis(k - 1);
}

// Lanczos estimate of the extreme eigenvalues of the context's H (FP64).
// Works in three temporary n-vectors; stops when the smallest Ritz value is
// <= 0 (H is then certainly not SPD), when it changed by less than 1e-10
// relative over the last 25 iterations, at an invariant subspace, or after
// max_it iterations.
hipError_t lanczos_extremes(ope_ctx* c, int max_it, double* lmin, double* lmax, int* iters) {
  const uint64_t n = (uint64_t)c->n;
  double *buf = nullptr, *ab = nullptr;
  hipError_t e = hipMalloc((void**)&buf, sizeof(double) * (3 * n + 1024));
  if (e != hipSuccess) return e;
  e = hipMalloc((void**)&ab, sizeof(double) * (2 * (size_t)max_it + 2));
  if (e != hipSuccess) {
    (void)hipFree(buf);
    return e;
  }
  double* vec[3] = {buf, buf + n, buf + 2 * n};
  double* part = buf + 3 * n;
  double* alpha = ab;                     // alpha[j]
  double* beta = ab + max_it + 1;         // beta[0] = |start|, beta[j + 1] = |w_j|
  uint32_t blocks;
  lz_launch_dims(n, &blocks);
  hipStream_t s = c->stream;
  std::vector<double> ha(max_it), hb(max_it + 1);
  double prev = 0.0;
  int k = 0;
  // buffer roles: ic holds v_j (unnormalised, scale beta[j]), ip v_{j-1}
  // (normalised), iw receives w; they rotate every iteration
  int ip = 0, ic = 1, iw = 2;
  hipLaunchKernelGGL(k_lz_start, dim3(blocks), dim3(LW), 0, s, vec[ic], n, (uint64_t)0x5EED, part);
  hipLaunchKernelGGL(k_lz_sum, dim3(1), dim3(RW), 0, s, part, blocks, 1, beta);
  *lmin = 0.0;
  *lmax = 0.0;
  for (int j = 0; j < max_it; ++j) {
    hipLaunchKernelGGL(k_lz_apply, dim3(blocks), dim3(LW), 0, s, vec[ic], j > 0 ? vec[ip] : nullptr, vec[iw], c->diag,
                       c->g, n, beta + j, j > 0 ? beta + j : nullptr, part);
    hipLaunchKernelGGL(k_lz_sum, dim3(1), dim3(RW), 0, s, part, blocks, 0, alpha + j);
    hipLaunchKernelGGL(k_lz_orth, dim3(blocks), dim3(LW), 0, s, vec[ic], vec[iw], n, beta + j, alpha + j, part);
    hipLaunchKernelGGL(k_lz_sum, dim3(1), dim3(RW), 0, s, part, blocks, 1, beta + j + 1);
    if ((e = hipGetLastError()) != hipSuccess) break;
    const int t = ip;
    ip = ic;
    ic = iw;
    iw = t;
    k = j + 1;
    if (k % 25 == 0 || k == max_it) {
      if ((e = hipMemcpyAsync(ha.data(), alpha, sizeof(double) * k, hipMemcpyDeviceToHost, s)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(hb.data(), beta, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, s)) != hipSuccess) break;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
      std::vector<double> bb(hb.begin() + 1, hb.begin() + k);   // beta_1 .. beta_{k-1}
      double lo, hi;
      tridiag_extremes(ha, bb, k, &lo, &hi);
      *lmin = lo;
      *lmax = hi;
      const bool breakdown = !(hb[k] > 1e-13 * fabs(hi));
      if (lo <= 0.0 || breakdown || !isfinite(lo)) break;
      if (k > 25 && fabs(lo - prev) <= 1e-10 * fabs(lo)) break;
      prev = lo;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  (void)hipFree(ab);
  *iters = k;
  return e;
}

hipError_t launch_chol_rinv(ope_ctx* c, double* A, double* Rinv) {
  hipLaunchKernelGGL(k_chol_rinv, dim3(1), dim3(RW), 0, c->stream, A, (uint32_t)c->N, Rinv, c->sc);
  return hipGetLastError();
}

hipError_t launch_scalar_copy(ope_ctx* c, int which, double* out) {
  hipLaunchKernelGGL(k_scalar_copy, dim3(1), dim3(64), 0, c->stream, c->sc, which, out);
  return hipGetLastError();
}
