// FP64 kernels on N x N matrices: the small solve of
// Steps 2-3 (Section 4.1), the warm-start inverse Lam^{-1}, the per-step
// scalars, and Jacobi eigenvalues for the Ritz values.
//
// A 1024-thread work-group holds an N x N matrix in registers: thread t owns
// column j = t % 128 and rows i = t / 128 + 8 r, r = 0..15.  Gauss-Jordan
// elimination without pivoting runs four pivots per block step, with two
// barriers per step (the pivot columns and rows are published through
// double-buffered LDS); this is the path for N <= 128, larger N use the
// Newton-Schulz pieces below.  No
// pivoting is needed: the Step-2 matrix has symmetric part >= I (Lemma 3.1 and
// its generalisation to an inexact GU), and Lam = U^T H U is SPD, so every
// pivot of either is positive.
#include "ope_internal.h"

namespace {

constexpr int SW = 1024;      // threads of the small kernels
constexpr int RPT = 16;       // rows per thread (128 / 8)

struct Own {
  uint32_t j, q;
  __device__ Own() : j(threadIdx.x & 127u), q(threadIdx.x >> 7) {}
  __device__ uint32_t row(int r) const { return q + 8u * (uint32_t)r; }
};

// Deterministic work-group sum (fixed tree order).
__device__ double wg_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = SW / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// In-place Gauss-Jordan inversion of the register-resident matrix w, four
// pivots per block step (the arithmetic of four successive single pivots,
// regrouped):  with K the block's pivot indices, P = W[K,K] and
// X = P^{-1} [W[K,:] with W[K,K] replaced by I],
//   rows not in K:  W[i,:] <- W'[i,:] - W[i,K] X   (W' = W with columns K zeroed)
//   rows in K:      W[K,:] <- X.
// LDS per block step (double-buffered by step parity): the pivot columns
// F[c][q * 16 + r] (row q + 8 r, so a thread reads its rows contiguously), the
// pivot rows R[c][j], and X[c][j], which the 128 threads of row group 0 solve
// for their column from P by Gauss-Jordan (a 4 x 4 system per column: two
// barriers per step serve four pivots, instead of one barrier per pivot).  Sets *bad when a
// pivot of the elimination is not a finite number above 1e-300.
constexpr int GJB = 4;      // pivots per block step

struct GjLds {
  double F[2][GJB][128];
  double R[2][GJB][128];
  double X[2][GJB][128];
};

__device__ void gj_invert(double (&w)[RPT], uint32_t N, GjLds& L, int* bad) {
  const Own o;
  for (uint32_t k0 = 0, st = 0; k0 < N; k0 += GJB, st ^= 1u) {
    const uint32_t kb = min((uint32_t)GJB, N - k0);     // pivots of this step
    double(&F)[GJB][128] = L.F[st];
    double(&R)[GJB][128] = L.R[st];
    double(&X)[GJB][128] = L.X[st];
    const uint32_t kr = k0 >> 3;                         // register row of the pivot rows
    const uint32_t q0 = k0 & 7u;                         // their row groups: q0 .. q0 + kb - 1
    const bool krow = o.q >= q0 && o.q < q0 + kb;        // this wave holds a pivot row (as w[kr])
    // pivot rows first (they include the block), then the pivot columns,
    // which their lanes then zero
    if (krow && o.j < N) {
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if ((uint32_t)r == kr) R[o.q - q0][o.j] = w[r];
    }
    if (o.j >= k0 && o.j < k0 + kb) {
      const uint32_t c = o.j - k0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        F[c][o.q * 16u + r] = w[r];
        w[r] = 0.0;
      }
    }
    __syncthreads();
    if (o.q == 0 && o.j < N) {
      // solve P x = b for this column: b = R[:, j], or the unit vector of
      // column j when j is a pivot column
      double P[GJB][GJB], x[GJB];
#pragma unroll
      for (int c = 0; c < GJB; ++c) {
#pragma unroll
        for (int d = 0; d < GJB; ++d)
          P[c][d] = ((uint32_t)c < kb && (uint32_t)d < kb) ? R[c][k0 + d] : (c == d ? 1.0 : 0.0);
        const bool inK = o.j >= k0 && o.j < k0 + kb;
        x[c] = (uint32_t)c < kb ? (inK ? (o.j - k0 == (uint32_t)c ? 1.0 : 0.0) : R[c][o.j]) : 0.0;
      }
#pragma unroll
      for (int p = 0; p < GJB; ++p) {
        const double piv = P[p][p];
        const bool ok = isfinite(piv) && piv > 1e-300;
        if (!ok && (uint32_t)p < kb && o.j == 0) *bad = 1;
        const double pinv = ok ? 1.0 / piv : 0.0;
#pragma unroll
        for (int d = 0; d < GJB; ++d) P[p][d] *= pinv;
        x[p] *= pinv;
#pragma unroll
        for (int c = 0; c < GJB; ++c) {
          if (c == p) continue;
          const double f = P[c][p];
#pragma unroll
          for (int d = 0; d < GJB; ++d) P[c][d] = fma(-f, P[p][d], P[c][d]);
          x[c] = fma(-f, x[p], x[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < GJB; ++c) X[c][o.j] = x[c];
    }
    __syncthreads();
    if (o.j < N) {
      double xj[GJB];
#pragma unroll
      for (int c = 0; c < GJB; ++c) xj[c] = X[c][o.j];
#pragma unroll
      for (int c = 0; c < GJB; ++c) {
        if ((uint32_t)c >= kb) break;                    // slots past the last pivot hold no column
        const double2* F2 = reinterpret_cast<const double2*>(&F[c][o.q * 16u]);
#pragma unroll
        for (int r = 0; r < RPT / 2; ++r) {
          const double2 f = F2[r];
          w[2 * r] = fma(-f.x, xj[c], w[2 * r]);
          w[2 * r + 1] = fma(-f.y, xj[c], w[2 * r + 1]);
        }
      }
      if (krow) {
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          if ((uint32_t)r == kr) w[r] = xj[o.q - q0];
      }
    }
  }
  __syncthreads();
}

__device__ void load_own(const double* __restrict__ M, uint32_t N, double (&w)[RPT]) {
  const Own o;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const uint32_t i = o.row(r);
    w[r] = (i < N && o.j < N) ? M[(uint64_t)i * N + o.j] : 0.0;
  }
}

__device__ void store_own(double* __restrict__ M, uint32_t N, const double (&w)[RPT]) {
  const Own o;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const uint32_t i = o.row(r);
    if (i < N && o.j < N) M[(uint64_t)i * N + o.j] = w[r];
  }
}

// Energy, drift, |Lam|_F, column norms, and Lam^{-1} for the warm start.
__global__ __launch_bounds__(SW) void k_prep_small(const double* __restrict__ C, const double* __restrict__ Lam,
                                                   double* __restrict__ Linv, double* __restrict__ cnorm2,
                                                   uint32_t N, OpeScalars* __restrict__ sc, float* __restrict__ Lam32,
                                                   float* __restrict__ Linv32) {
  __shared__ double red[SW];
  __shared__ __align__(16) GjLds gl;
  __shared__ int bad;
  const Own o;
  if (threadIdx.x == 0) bad = 0;
  double w[RPT];
  double e = 0.0, lf = 0.0, dr = 0.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const uint32_t i = o.row(r);
    if (i < N && o.j < N) {
      const double lij = Lam[(uint64_t)i * N + o.j], lji = Lam[(uint64_t)o.j * N + i];
      const double cij = C[(uint64_t)i * N + o.j] - (i == o.j ? 1.0 : 0.0);
      w[r] = 0.5 * (lij + lji);
      if (Lam32) Lam32[(uint64_t)i * N + o.j] = (float)lij;
      lf += lij * lij;
      dr += cij * cij;
      if (i == o.j) {
        e += lij;
        cnorm2[i] = C[(uint64_t)i * N + i];
      }
    } else {
      w[r] = 0.0;
    }
  }
  e = wg_sum(e, red);
  lf = wg_sum(lf, red);
  dr = wg_sum(dr, red);
  gj_invert(w, N, gl, &bad);
  store_own(Linv, N, w);
  if (Linv32) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const uint32_t i = o.row(r);
      if (i < N && o.j < N) Linv32[(uint64_t)i * N + o.j] = (float)w[r];
    }
  }
  if (threadIdx.x == 0) {
    sc->energy = 0.5 * e;
    sc->lam_fro = sqrt(lf);
    sc->drift = sqrt(dr);
    int err = 0;
    if (!isfinite(e) || !isfinite(lf) || !isfinite(dr)) err = OPE_ENONFINITE;
    else if (bad) err = OPE_EPIVOT;
    sc->err = err;                 // first writer of the step: resets earlier errors
  }
}

// Outer residual, inner tolerance and CG start state (one step of Algorithm 1).
__global__ __launch_bounds__(SW) void k_cg_setup(const double* __restrict__ rcol, const double* __restrict__ rho0,
                                                 const double* __restrict__ cnorm2, double eta_rel, double eta_floor,
                                                 uint32_t N, double* __restrict__ rho, double* __restrict__ target,
                                                 double* __restrict__ alpha, double* __restrict__ beta,
                                                 int32_t* __restrict__ active, OpeScalars* __restrict__ sc) {
  __shared__ double red[SW];
  double s = 0.0;
  for (uint32_t j = threadIdx.x; j < N; j += SW) s += rcol[j];
  s = wg_sum(s, red);
  const double res = sqrt(s) / sc->lam_fro;
  double eta = eta_rel * res;
  if (!(eta > eta_floor)) eta = eta_floor;
  for (uint32_t j = threadIdx.x; j < N; j += SW) {
    const double t = eta * eta * cnorm2[j];
    target[j] = t;
    rho[j] = rho0[j];
    alpha[j] = 0.0;
    alpha[N + j] = 0.0;        // both iteration-parity halves
    beta[j] = 0.0;
    active[j] = rho0[j] > t ? 1 : 0;
  }
  if (threadIdx.x == 0) {
    sc->cg_iters = 0;
    sc->residual = res;
    sc->eta = eta;
    if (!isfinite(res) && sc->err == 0) sc->err = OPE_ENONFINITE;
  }
}

// Stand-alone Step 1: tolerance relative to the column norms of U.
__global__ __launch_bounds__(SW) void k_solve_setup(const double* __restrict__ rho0, const double* __restrict__ unorm2,
                                                    double tol, uint32_t N, double* __restrict__ rho,
                                                    double* __restrict__ target, double* __restrict__ alpha,
                                                    double* __restrict__ beta, int32_t* __restrict__ active,
                                                    OpeScalars* __restrict__ sc) {
  for (uint32_t j = threadIdx.x; j < N; j += SW) {
    const double t = tol * tol * unorm2[j];
    target[j] = t;
    rho[j] = rho0[j];
    alpha[j] = 0.0;
    alpha[N + j] = 0.0;        // both iteration-parity halves
    beta[j] = 0.0;
    active[j] = rho0[j] > t ? 1 : 0;
  }
  if (threadIdx.x == 0) {
    sc->err = 0;
    sc->cg_iters = 0;
  }
}

// The N x N products below run from LDS: a thread's row index is uniform over
// its wave, so that operand is a broadcast read; from global memory it would be
// a scalar load, and at most 15 of those can be outstanding.  smat holds one
// N x N FP64 matrix (dynamic LDS, N*N*8 bytes, at most 128 KiB).

// Steps 2-3: M = I + tau/2 (S_a - S_b) + tau^2/4 (T - S_a S_b), S_a = S_b^T,
// B = M^{-1}, A = 2/tau (I - B) + S_b B, Z = [I - tau A ; tau B].
__global__ __launch_bounds__(SW) void k_small_solve(const double* __restrict__ Sb, const double* __restrict__ T,
                                                    double tau, uint32_t N, double* __restrict__ Bws,
                                                    double* __restrict__ Z, double* __restrict__ Aout,
                                                    OpeScalars* __restrict__ sc) {
  extern __shared__ double smat[];
  __shared__ __align__(16) GjLds gl;
  __shared__ int bad;
  const Own o;
  if (threadIdx.x == 0) bad = 0;
  for (uint32_t e = threadIdx.x; e < N * N; e += SW) smat[e] = Sb[e];
  __syncthreads();
  const uint32_t jj = o.j < N ? o.j : 0u;
  double w[RPT];
  // M, with P = S_a S_b, P_ij = sum_k S_b[k][i] S_b[k][j]
  double P[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) P[r] = 0.0;
#pragma unroll 1
  for (uint32_t k = 0; k < N; ++k) {
    const double skj = smat[k * N + jj];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const uint32_t i = o.row(r);
      const double ski = smat[k * N + (i < N ? i : 0u)];
      P[r] += ski * skj;
    }
  }
  const double ht = 0.5 * tau, qt = 0.25 * tau * tau;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const uint32_t i = o.row(r);
    if (i < N && o.j < N) {
      const double sb = Sb[(uint64_t)i * N + o.j], sa = Sb[(uint64_t)o.j * N + i];
      w[r] = (i == o.j ? 1.0 : 0.0) + ht * (sa - sb) + qt * (T[(uint64_t)i * N + o.j] - P[r]);
    } else {
      w[r] = 0.0;
    }
  }
  gj_invert(w, N, gl, &bad);
  store_own(Bws, N, w);           // B
  __syncthreads();
  // A = 2/tau (I - B) + S_b B: B's rows staged through the elimination's LDS
  // (free now) in chunks of BCH rows, every thread loading its share at once
  double acc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
  constexpr uint32_t BCH = sizeof(GjLds) / (sizeof(double) * 128);     // rows of 128 per chunk
  double* bst = reinterpret_cast<double*>(&gl);
  for (uint32_t k0 = 0; k0 < N; k0 += BCH) {
    const uint32_t kn = min(BCH, N - k0);
    for (uint32_t e = threadIdx.x; e < kn * N; e += SW) bst[e] = Bws[(uint64_t)k0 * N + e];
    __syncthreads();
#pragma unroll 1
    for (uint32_t k = 0; k < kn; ++k) {
      const double bkj = bst[k * N + jj];
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const uint32_t i = o.row(r);
        acc[r] += smat[(i < N ? i : 0u) * N + k0 + k] * bkj;
      }
    }
    __syncthreads();
  }
  const double it = 2.0 / tau;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const uint32_t i = o.row(r);
    if (i < N && o.j < N) {
      const double dij = (i == o.j ? 1.0 : 0.0);
      const double a = it * (dij - w[r]) + acc[r];
      Z[(uint64_t)i * N + o.j] = dij - tau * a;
      Z[(uint64_t)(N + i) * N + o.j] = tau * w[r];
      if (Aout) Aout[(uint64_t)i * N + o.j] = a;
    }
  }
  if (threadIdx.x == 0 && bad && sc->err == 0) sc->err = OPE_EPIVOT;
}

// Mixed-precision Steps 2-3 in delta form.  With P = Y - U S_b and
// C = <U,U>, T - S_a S_b = P^T P - S_b^T (C - I) S_b, so the Step-2 matrix is
// M = I + tau/2 (S_a - S_b) + tau^2/4 (P^T P - S_b^T (C - I) S_b), B = M^{-1},
// and Step 4 is U' = U + U Z1 + P Z2 with Z1 = -2 (I - B), Z2 = tau B: the
// same map as the FP64 step for any U, written so that both products vanish
// at a fixed point (their BF16 rounding vanishes with them).  The
// S_b^T (C - I) S_b term keeps the step orthogonality-preserving when the
// FP32 iterate has drifted; without it the drift is amplified at large tau.
// Z is written in FP32 (2N x N) for the BF16 product; Wsm is N x N scratch.
__global__ __launch_bounds__(SW) void k_small_solve_delta(const double* __restrict__ Sb,
                                                          const double* __restrict__ Tp,
                                                          const double* __restrict__ C, double tau, uint32_t N,
                                                          double* __restrict__ Wsm, float* __restrict__ Z32,
                                                          OpeScalars* __restrict__ sc) {
  extern __shared__ double smat[];
  __shared__ __align__(16) GjLds gl;
  __shared__ int bad;
  const Own o;
  if (threadIdx.x == 0) bad = 0;
  for (uint32_t e = threadIdx.x; e < N * N; e += SW) smat[e] = C[e];
  __syncthreads();
  const uint32_t jj = o.j < N ? o.j : 0u;
  // Wsm = (C - I) S_b  (C from LDS, S_b's columns from global memory)
  double acc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
  double snx = Sb[jj];
#pragma unroll 1
  for (uint32_t l = 0; l < N; ++l) {
    const double slj = snx;
    snx = Sb[(uint64_t)(l + 1 < N ? l + 1 : l) * N + jj];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const uint32_t k = o.row(r) < N ? o.row(r) : 0u;
      acc[r] += (smat[k * N + l] - (k == l ? 1.0 : 0.0)) * slj;
    }
  }
  store_own(Wsm, N, acc);
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < N * N; e += SW) smat[e] = Sb[e];
  __syncthreads();
  // Q = S_b^T Wsm  (S_b from LDS, Wsm's columns from global memory)
  double qv[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) qv[r] = 0.0;
  double wnx = Wsm[jj];
#pragma unroll 1
  for (uint32_t k = 0; k < N; ++k) {
    const double wkj = wnx;
    wnx = Wsm[(uint64_t)(k + 1 < N ? k + 1 : k) * N + jj];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const uint32_t i = o.row(r) < N ? o.row(r) : 0u;
      qv[r] += smat[k * N + i] * wkj;
    }
  }
  double w[RPT];
  const double ht = 0.5 * tau, qt = 0.25 * tau * tau;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const uint32_t i = o.row(r);
    if (i < N && o.j < N) {
      const double sb = Sb[(uint64_t)i * N + o.j], sa = Sb[(uint64_t)o.j * N + i];
      w[r] = (i == o.j ? 1.0 : 0.0) + ht * (sa - sb) + qt * (Tp[(uint64_t)i * N + o.j] - qv[r]);
    } else {
      w[r] = 0.0;
    }
  }
  gj_invert(w, N, gl, &bad);
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const uint32_t i = o.row(r);
    if (i < N && o.j < N) {
      const double dij = (i == o.j ? 1.0 : 0.0);
      Z32[(uint64_t)i * N + o.j] = (float)(-2.0 * (dij - w[r]));
      Z32[(uint64_t)(N + i) * N + o.j] = (float)(tau * w[r]);
    }
  }
  if (threadIdx.x == 0 && bad && sc->err == 0) sc->err = OPE_EPIVOT;
}

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, uint64_t count) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < count; e += (uint64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

__global__ void k_to_f64(const float* __restrict__ src, double* __restrict__ dst, uint64_t count) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < count; e += (uint64_t)gridDim.x * blockDim.x)
    dst[e] = (double)src[e];
}

// Cyclic Jacobi (round-robin parallel ordering) on a symmetric N x N matrix
// (N <= 512) held in global workspace; eigenvalues sorted ascending into evals.
__global__ __launch_bounds__(SW) void k_jacobi(const double* __restrict__ Asrc, double* __restrict__ W,
                                               double* __restrict__ evals, uint32_t N) {
  __shared__ double red[SW];
  __shared__ double cs[256], sn[256];
  __shared__ uint32_t pp[256], qq[256];
  __shared__ double dg[512];
  const uint32_t Np = N + (N & 1u);             // even number of players (one dummy for odd N)
  const uint32_t npair = Np / 2, m = Np - 1;
  for (uint32_t e = threadIdx.x; e < N * N; e += SW) {
    const uint32_t i = e / N, j = e - i * N;
    W[e] = 0.5 * (Asrc[(uint64_t)i * N + j] + Asrc[(uint64_t)j * N + i]);
  }
  __syncthreads();
  double fro = 0.0;
  for (uint32_t e = threadIdx.x; e < N * N; e += SW) fro += W[e] * W[e];
  fro = wg_sum(fro, red);
  for (int sweep = 0; sweep < 40 && N > 1; ++sweep) {
    double off = 0.0;
    for (uint32_t e = threadIdx.x; e < N * N; e += SW) {
      const uint32_t i = e / N, j = e - i * N;
      if (i != j) off += W[e] * W[e];
    }
    off = wg_sum(off, red);
    if (off <= 1e-32 * fro) break;
    for (uint32_t rnd = 0; rnd < m; ++rnd) {
      if (threadIdx.x < npair) {
        const uint32_t s = threadIdx.x;
        const uint32_t a = (s == 0) ? 0u : ((s - 1 + rnd) % m) + 1;
        const uint32_t b = ((m - 1 - s + rnd) % m) + 1;
        const uint32_t p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, t = 0.0;
        if (q < N) {
          const double apq = W[(uint64_t)p * N + q];
          if (apq != 0.0) {
            const double theta = (W[(uint64_t)q * N + q] - W[(uint64_t)p * N + p]) / (2.0 * apq);
            t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
            if (theta < 0.0) t = -t;
            c = 1.0 / sqrt(t * t + 1.0);
          }
        }
        cs[s] = c;
        sn[s] = t * c;
        pp[s] = p;
        qq[s] = q;
      }
      __syncthreads();
      // W <- J^T W J in one pass over the 2 x 2 blocks of rows (p_a, q_a) and
      // columns (p_b, q_b) of two pairs a, b: the rows first,
      //   row_p' = c row_p - s row_q, row_q' = s row_p + c row_q,
      // then the columns of the result the same way (a dummy index of odd N,
      // q = N, leaves its row or column unrotated and is not stored)
      for (uint32_t e = threadIdx.x; e < npair * npair; e += SW) {
        const uint32_t a = e / npair, b = e - a * npair;
        const uint32_t pa = pp[a], qa = qq[a], pb = pp[b], qb = qq[b];
        const bool ra = qa < N, rb = qb < N;
        const double ca = ra ? cs[a] : 1.0, sa = ra ? sn[a] : 0.0;
        const double cb = rb ? cs[b] : 1.0, sb = rb ? sn[b] : 0.0;
        const double w00 = W[(uint64_t)pa * N + pb];
        const double w01 = rb ? W[(uint64_t)pa * N + qb] : 0.0;
        const double w10 = ra ? W[(uint64_t)qa * N + pb] : 0.0;
        const double w11 = (ra && rb) ? W[(uint64_t)qa * N + qb] : 0.0;
        const double r00 = ca * w00 - sa * w10, r01 = ca * w01 - sa * w11;
        const double r10 = sa * w00 + ca * w10, r11 = sa * w01 + ca * w11;
        W[(uint64_t)pa * N + pb] = cb * r00 - sb * r01;
        if (rb) W[(uint64_t)pa * N + qb] = sb * r00 + cb * r01;
        if (ra) W[(uint64_t)qa * N + pb] = cb * r10 - sb * r11;
        if (ra && rb) W[(uint64_t)qa * N + qb] = sb * r10 + cb * r11;
      }
      __syncthreads();
    }
  }
  for (uint32_t i = threadIdx.x; i < N; i += SW) dg[i] = W[(uint64_t)i * N + i];
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < N; i += SW) {
    const double v = dg[i];
    uint32_t rank = 0;
    for (uint32_t k = 0; k < N; ++k) rank += (dg[k] < v || (dg[k] == v && k < i)) ? 1u : 0u;
    evals[rank] = v;
  }
}


// ---------------------------------------------------------------------------
// N > 128: the same small phase from multi-work-group pieces.  Inverses by
// Newton-Schulz, X <- X (2I - M X), on the FP64 matrix cores (k_sqmm): it
// converges quadratically from X0 = M^T / (|M|_1 |M|_inf) for any
// non-singular M, and from X0 = I / |M|_inf for SPD M (Lam); the Step-2
// matrix has symmetric part >= I and Lam is SPD, so both are well
// conditioned.  A device-side state stops the iteration once
// |I - M X_k|_F <= 1e-10 (one more update then squares the error).
// ---------------------------------------------------------------------------

// one work-group: energy, |Lam|_F, drift, column norms, sym(Lam) into Ls,
// X0 = I / |Ls|_inf, and the Newton-Schulz state reset
__global__ __launch_bounds__(SW) void k_big_prep(const double* __restrict__ C, const double* __restrict__ Lam,
                                                 double* __restrict__ Ls, double* __restrict__ X0,
                                                 double* __restrict__ cnorm2, uint32_t N,
                                                 OpeScalars* __restrict__ sc, float* __restrict__ Lam32,
                                                 NsState* __restrict__ ns) {
  __shared__ double red[SW];
  double e = 0.0, lf = 0.0, dr = 0.0, rmax = 0.0;
  for (uint32_t i = threadIdx.x; i < N; i += SW) {
    double rs = 0.0;
    for (uint32_t j = 0; j < N; ++j) {
      const double lij = Lam[(uint64_t)i * N + j], lji = Lam[(uint64_t)j * N + i];
      const double ls = 0.5 * (lij + lji);
      Ls[(uint64_t)i * N + j] = ls;
      if (Lam32) Lam32[(uint64_t)i * N + j] = (float)lij;
      const double cij = C[(uint64_t)i * N + j] - (i == j ? 1.0 : 0.0);
      lf += lij * lij;
      dr += cij * cij;
      rs += fabs(ls);
    }
    e += Lam[(uint64_t)i * N + i];
    cnorm2[i] = C[(uint64_t)i * N + i];
    rmax = rs > rmax ? rs : rmax;
  }
  e = wg_sum(e, red);
  lf = wg_sum(lf, red);
  dr = wg_sum(dr, red);
  red[threadIdx.x] = rmax;
  __syncthreads();
  for (int s = SW / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double scale = red[0] > 0.0 ? 1.0 / red[0] : 0.0;
  for (uint32_t q = threadIdx.x; q < N * N; q += SW) X0[q] = (q % (N + 1) == 0) ? scale : 0.0;
  if (threadIdx.x == 0) {
    sc->energy = 0.5 * e;
    sc->lam_fro = sqrt(lf);
    sc->drift = sqrt(dr);
    int err = 0;
    if (!isfinite(e) || !isfinite(lf) || !isfinite(dr) || !(scale > 0.0)) err = OPE_ENONFINITE;
    sc->err = err;                 // first writer of the step: resets earlier errors
    ns->done = 0;
    ns->cur = 0;
    ns->upd_skip = 0;
    ns->iters = 0;
  }
}

// M = I + tau/2 (S_b^T - S_b) + tau^2/4 (T - P) (N^2 threads); with the
// transpose X0 = M^T / (|M|_1 |M|_inf) written by k_big_init.
__global__ void k_big_form_m(const double* __restrict__ Sb, const double* __restrict__ T,
                             const double* __restrict__ P, double tau, uint32_t N, double* __restrict__ M) {
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (uint64_t)N * N) return;
  const uint32_t i = (uint32_t)(q / N), j = (uint32_t)(q % N);
  M[q] = (i == j ? 1.0 : 0.0) + 0.5 * tau * (Sb[(uint64_t)j * N + i] - Sb[q]) + 0.25 * tau * tau * (T[q] - P[q]);
}

// one work-group: X0 = M^T / (|M|_1 |M|_inf), Newton-Schulz state reset
__global__ __launch_bounds__(SW) void k_big_init(const double* __restrict__ M, uint32_t N, double* __restrict__ X0,
                                                 NsState* __restrict__ ns, OpeScalars* __restrict__ sc) {
  __shared__ double red[SW];
  double rmax = 0.0, cmax = 0.0;
  for (uint32_t i = threadIdx.x; i < N; i += SW) {
    double rs = 0.0, cs = 0.0;
    for (uint32_t j = 0; j < N; ++j) {
      rs += fabs(M[(uint64_t)i * N + j]);
      cs += fabs(M[(uint64_t)j * N + i]);
    }
    rmax = rs > rmax ? rs : rmax;
    cmax = cs > cmax ? cs : cmax;
  }
  red[threadIdx.x] = rmax;
  __syncthreads();
  for (int s = SW / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double ninf = red[0];
  __syncthreads();
  red[threadIdx.x] = cmax;
  __syncthreads();
  for (int s = SW / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double n1 = red[0];
  const double a = (ninf > 0.0 && n1 > 0.0 && isfinite(ninf * n1)) ? 1.0 / (ninf * n1) : 0.0;
  for (uint32_t q = threadIdx.x; q < N * N; q += SW) {
    const uint32_t i = q / N, j = q % N;
    X0[q] = a * M[(uint64_t)j * N + i];
  }
  if (threadIdx.x == 0) {
    ns->done = 0;
    ns->cur = 0;
    ns->upd_skip = 0;
    ns->iters = 0;
    if (!(a > 0.0) && sc->err == 0) sc->err = OPE_EPIVOT;
  }
}

// after G = M X_k with its residual partials: |I - G|_F, the stop decision,
// and which buffer the update of iteration k writes
__global__ __launch_bounds__(256) void k_ns_check(const double* __restrict__ part, uint32_t nparts, uint32_t k,
                                                  NsState* __restrict__ ns) {
  __shared__ double red[256];
  if (ns->done) {
    if (threadIdx.x == 0) ns->upd_skip = 1;
    return;
  }
  double s = 0.0;
  for (uint32_t q = threadIdx.x; q < nparts; q += 256) s += part[q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = sqrt(red[0]);
    ns->res = r;
    ns->iters = (int32_t)k + 1;
    ns->upd_skip = 0;
    ns->cur = (int32_t)((k + 1) & 1u);
    if (!isfinite(r)) {
      ns->done = 2;              // failed: no further iterations
      ns->upd_skip = 1;
      ns->cur = (int32_t)(k & 1u);
    } else if (r <= 1e-10) {
      ns->done = 1;              // this iteration's update is the last
    }
  }
}

// the inverse into Dst from the buffer holding it; sets EPIVOT if the
// iteration did not converge
__global__ void k_ns_take(const double* __restrict__ X0, const double* __restrict__ X1, uint32_t N,
                          const NsState* __restrict__ ns, double* __restrict__ Dst, float* __restrict__ Dst32,
                          OpeScalars* __restrict__ sc) {
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double* X = ns->cur ? X1 : X0;
  if (q < (uint64_t)N * N) {
    Dst[q] = X[q];
    if (Dst32) Dst32[q] = (float)X[q];
  }
  if (q == 0 && ns->done != 1 && sc->err == 0) sc->err = OPE_EPIVOT;
}

// Z = [I - tau A ; tau B] (FP64) or, for the delta form, Z32 = [-2 (I - B) ; tau B]
__global__ void k_big_z(const double* __restrict__ A, const double* __restrict__ B, double tau, uint32_t N,
                        double* __restrict__ Z, float* __restrict__ Z32) {
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (uint64_t)N * N) return;
  const uint32_t i = (uint32_t)(q / N), j = (uint32_t)(q % N);
  const double d = i == j ? 1.0 : 0.0;
  if (Z) {
    Z[q] = d - tau * A[q];
    Z[(uint64_t)N * N + q] = tau * B[q];
  } else {
    Z32[q] = (float)(-2.0 * (d - B[q]));
    Z32[(uint64_t)N * N + q] = (float)(tau * B[q]);
  }
}

// Z = (I - C) / 2, the correction of U <- U + U Z = U (3I - C) / 2
__global__ void k_renorm(const double* __restrict__ C, uint32_t N, float* __restrict__ Z) {
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (uint64_t)N * N) return;
  const uint32_t i = (uint32_t)(q / N), j = (uint32_t)(q % N);
  Z[q] = (float)(0.5 * ((i == j ? 1.0 : 0.0) - C[q]));
}

// Drift check after a mixed-precision update: drift = |C - I|_F of the new
// iterate (C = U^T U accumulated in FP64); above thr the next predicated
// product applies U <- U + U (I - C) / 2 = U (3 I - C) / 2, one Newton-Schulz
// step toward the nearest orthonormal block (drift E -> O(E^2)).  Z receives
// the correction (I - C) / 2: formed as U + U Z, its small terms are summed
// among themselves before U is added; as U (3I - C)/2 in FP32 they would be
// absorbed one by one into an accumulator of the size of U.
__global__ __launch_bounds__(SW) void k_drift_check(const double* __restrict__ C, uint32_t N, double thr,
                                                    float* __restrict__ Z, OpeScalars* __restrict__ sc) {
  __shared__ double red[SW];
  double s = 0.0;
  const uint64_t nn = (uint64_t)N * N;
  for (uint64_t q = threadIdx.x; q < nn; q += SW) {
    const uint32_t i = (uint32_t)(q / N), j = (uint32_t)(q % N);
    const double d = C[q] - (i == j ? 1.0 : 0.0);
    s += d * d;
    Z[q] = (float)(-0.5 * d);
  }
  s = wg_sum(s, red);
  if (threadIdx.x == 0) {
    const double drift = sqrt(s);
    sc->drift_after = drift;
    const int on = drift > thr && sc->err == 0 && isfinite(drift);
    sc->renorm = on;
    sc->renorms += on;
  }
}

__global__ void k_copy_pred(const void* __restrict__ src, void* __restrict__ dst, uint64_t words,
                            const OpeScalars* __restrict__ sc, int pred) {
  if ((pred & ROWMM_IF_OK) && sc->err != 0) return;
  if ((pred & ROWMM_IF_RENORM) && sc->renorm == 0) return;
  const uint64_t* s = (const uint64_t*)src;
  uint64_t* d = (uint64_t*)dst;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < words; e += (uint64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

}  // namespace

// Newton-Schulz iterations on M (from X0 in ns_x[0]) in chunks of 8 with a
// host check of the device state between chunks; the inverse goes to Dst.
static hipError_t ns_invert(ope_ctx* c, const double* M, double* Dst, float* Dst32) {
  const uint32_t N = (uint32_t)c->N;
  const uint32_t t = (N + 63) / 64;
  hipError_t e;
  for (int k = 0; k < 96; ++k) {
    double* X = c->ns_x[k & 1];
    double* Xn = c->ns_x[(k + 1) & 1];
    if ((e = launch_sqmm(c, M, 0, X, 0, nullptr, 1.0, 0.0, 0.0, c->ns_g, N, &c->ns->done, c->ns_part)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_ns_check, dim3(1), dim3(256), 0, c->stream, c->ns_part, t * t, (uint32_t)k, c->ns);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // X_{k+1} = 2 X_k - X_k G
    if ((e = launch_sqmm(c, X, 0, c->ns_g, 0, X, -1.0, 2.0, 0.0, Xn, N, &c->ns->upd_skip, nullptr)) != hipSuccess)
      return e;
    if (k % 8 == 7) {
      if ((e = hipMemcpyAsync(c->hns, c->ns, sizeof(NsState), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return e;
      if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
      if (c->hns->done) break;
    }
  }
  const uint64_t nn = (uint64_t)N * N;
  hipLaunchKernelGGL(k_ns_take, dim3((uint32_t)((nn + 255) / 256)), dim3(256), 0, c->stream, c->ns_x[0], c->ns_x[1],
                     N, c->ns, Dst, Dst32, c->sc);
  return hipGetLastError();
}

static hipError_t big_prep(ope_ctx* c) {
  const uint32_t N = (uint32_t)c->N;
  hipLaunchKernelGGL(k_big_prep, dim3(1), dim3(SW), 0, c->stream, c->C, c->Lam, c->ns_m, c->ns_x[0], c->cnorm2, N,
                     c->sc, c->Lam32, c->ns);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return ns_invert(c, c->ns_m, c->Linv, c->Linv32);
}

// B = M^{-1} for M = I + tau/2 (S_b^T - S_b) + tau^2/4 (T' - P), P in ns_p
static hipError_t big_form_and_invert(ope_ctx* c, const double* Sb, const double* Tp, double tau, double* B) {
  const uint32_t N = (uint32_t)c->N;
  const uint64_t nn = (uint64_t)N * N;
  hipLaunchKernelGGL(k_big_form_m, dim3((uint32_t)((nn + 255) / 256)), dim3(256), 0, c->stream, Sb, Tp, c->ns_p, tau,
                     N, c->ns_m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_init, dim3(1), dim3(SW), 0, c->stream, c->ns_m, N, c->ns_x[0], c->ns, c->sc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return ns_invert(c, c->ns_m, B, nullptr);
}

static hipError_t big_small_solve(ope_ctx* c, const double* Sb, const double* T, double tau, double* Z, double* A,
                                  double* B) {
  const uint32_t N = (uint32_t)c->N;
  const uint64_t nn = (uint64_t)N * N;
  hipError_t e;
  // P = S_a S_b = S_b^T S_b
  if ((e = launch_sqmm(c, Sb, 1, Sb, 0, nullptr, 1.0, 0.0, 0.0, c->ns_p, N, nullptr, nullptr)) != hipSuccess) return e;
  if ((e = big_form_and_invert(c, Sb, T, tau, B)) != hipSuccess) return e;
  // A = 2/tau (I - B) + S_b B
  double* Aw = A ? A : c->A;
  if ((e = launch_sqmm(c, Sb, 0, B, 0, B, 1.0, -2.0 / tau, 2.0 / tau, Aw, N, nullptr, nullptr)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_big_z, dim3((uint32_t)((nn + 255) / 256)), dim3(256), 0, c->stream, Aw, B, tau, N, Z,
                     (float*)nullptr);
  return hipGetLastError();
}

static hipError_t big_small_solve_delta(ope_ctx* c, const double* Sb, const double* Tp, double tau) {
  const uint32_t N = (uint32_t)c->N;
  const uint64_t nn = (uint64_t)N * N;
  hipError_t e;
  // Wsm = (C - I) S_b = C S_b - S_b ; P = S_b^T Wsm
  if ((e = launch_sqmm(c, c->C, 0, Sb, 0, Sb, 1.0, -1.0, 0.0, c->Wsm, N, nullptr, nullptr)) != hipSuccess) return e;
  if ((e = launch_sqmm(c, Sb, 1, c->Wsm, 0, nullptr, 1.0, 0.0, 0.0, c->ns_p, N, nullptr, nullptr)) != hipSuccess)
    return e;
  if ((e = big_form_and_invert(c, Sb, Tp, tau, c->B)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_z, dim3((uint32_t)((nn + 255) / 256)), dim3(256), 0, c->stream, (const double*)nullptr,
                     c->B, tau, N, (double*)nullptr, c->Z32);
  return hipGetLastError();
}

hipError_t launch_renorm_matrix(ope_ctx* c, const double* C, float* Z32) {
  const uint64_t nn = (uint64_t)c->N * c->N;
  hipLaunchKernelGGL(k_renorm, dim3((uint32_t)((nn + 255) / 256)), dim3(256), 0, c->stream, C, (uint32_t)c->N, Z32);
  return hipGetLastError();
}

hipError_t launch_copy_pred(ope_ctx* c, const void* src, void* dst, uint64_t bytes, int pred) {
  uint64_t words = bytes / 8;
  uint64_t grid = (words + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_copy_pred, dim3((uint32_t)grid), dim3(256), 0, c->stream, src, dst, words, c->sc, pred);
  return hipGetLastError();
}

hipError_t launch_drift_check(ope_ctx* c, const double* C, float* Z32, double thr) {
  hipLaunchKernelGGL(k_drift_check, dim3(1), dim3(SW), 0, c->stream, C, (uint32_t)c->N, thr, Z32, c->sc);
  return hipGetLastError();
}

hipError_t launch_prep_small(ope_ctx* c) {
  if (c->N > OPE_MAX_N_ONE_WG) return big_prep(c);
  ProfScope ps(c, OPE_KERNEL_SMALL);
  hipLaunchKernelGGL(k_prep_small, dim3(1), dim3(SW), 0, c->stream, c->C, c->Lam, c->Linv, c->cnorm2, (uint32_t)c->N,
                     c->sc, c->Lam32, c->Linv32);
  return hipGetLastError();
}

hipError_t launch_small_solve_delta(ope_ctx* c, const double* Sb, const double* Tperp, double tau) {
  if (c->N > OPE_MAX_N_ONE_WG) return big_small_solve_delta(c, Sb, Tperp, tau);
  ProfScope ps(c, OPE_KERNEL_SMALL);
  hipLaunchKernelGGL(k_small_solve_delta, dim3(1), dim3(SW), (size_t)c->N * c->N * sizeof(double), c->stream, Sb,
                     Tperp, c->C, tau, (uint32_t)c->N, c->Wsm, c->Z32, c->sc);
  return hipGetLastError();
}

hipError_t launch_small_to_f32(ope_ctx* c, const double* src, float* dst, int64_t count) {
  hipLaunchKernelGGL(k_to_f32, dim3(64), dim3(256), 0, c->stream, src, dst, (uint64_t)count);
  return hipGetLastError();
}

hipError_t launch_convert(ope_ctx* c, const void* src, void* dst, int64_t count, int to_double) {
  const uint64_t n = (uint64_t)count;
  uint64_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  if (to_double)
    hipLaunchKernelGGL(k_to_f64, dim3((uint32_t)grid), dim3(256), 0, c->stream, (const float*)src, (double*)dst, n);
  else
    hipLaunchKernelGGL(k_to_f32, dim3((uint32_t)grid), dim3(256), 0, c->stream, (const double*)src, (float*)dst, n);
  return hipGetLastError();
}

hipError_t launch_cg_setup(ope_ctx* c, const double* rho0) {
  hipLaunchKernelGGL(k_cg_setup, dim3(1), dim3(SW), 0, c->stream, c->rcol, rho0, c->cnorm2, c->eta_rel, c->eta_floor,
                     (uint32_t)c->N, c->rho, c->target, c->alpha, c->beta, c->active, c->sc);
  return hipGetLastError();
}

hipError_t launch_solve_setup(ope_ctx* c, const double* rho0, double tol) {
  hipLaunchKernelGGL(k_solve_setup, dim3(1), dim3(SW), 0, c->stream, rho0, c->cnorm2, tol, (uint32_t)c->N, c->rho,
                     c->target, c->alpha, c->beta, c->active, c->sc);
  return hipGetLastError();
}

hipError_t launch_small_solve(ope_ctx* c, const double* Sb, const double* T, double tau, double* Z, double* A,
                              double* B) {
  if (c->N > OPE_MAX_N_ONE_WG) return big_small_solve(c, Sb, T, tau, Z, A, B ? B : c->B);
  ProfScope ps(c, OPE_KERNEL_SMALL);
  hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(SW), (size_t)c->N * c->N * sizeof(double), c->stream, Sb, T, tau,
                     (uint32_t)c->N, B ? B : c->B, Z, A, c->sc);
  return hipGetLastError();
}

hipError_t launch_jacobi_eig(ope_ctx* c, const double* Asym, double* evals) {
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(SW), 0, c->stream, Asym, c->Wsm, evals, (uint32_t)c->N);
  return hipGetLastError();
}
