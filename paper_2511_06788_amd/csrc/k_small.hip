// One-work-group FP64 kernels on N x N matrices (N <= 128): the small solve of
// Steps 2-3 (Section 4.1), the warm-start inverse Lam^{-1}, the per-step
// scalars, and Jacobi eigenvalues for the Ritz values.
//
// A 1024-thread work-group holds an N x N matrix in registers: thread t owns
// column j = t % 128 and rows i = t / 128 + 8 r, r = 0..15.  Gauss-Jordan
// elimination without pivoting runs with one barrier per pivot (the pivot
// column and pivot row are published through double-buffered LDS).  No
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

// In-place Gauss-Jordan inversion of the register-resident matrix w.
// Sets *bad when a pivot is not a finite number above 1e-300.
__device__ void gj_invert(double (&w)[RPT], uint32_t N, double* fcol, double* rowk, int* bad) {
  const Own o;
  for (uint32_t k = 0; k < N; ++k) {
    double* F = fcol + (k & 1u) * 128;
    double* R = rowk + (k & 1u) * 128;
    if (o.j == k) {
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (o.row(r) < N) F[o.row(r)] = w[r];
    }
    if (o.j < N) {
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (o.row(r) == k) R[o.j] = w[r];
    }
    __syncthreads();
    const double piv = F[k];
    const bool ok = isfinite(piv) && piv > 1e-300;
    if (!ok && threadIdx.x == 0) *bad = 1;
    const double pinv = ok ? 1.0 / piv : 0.0;
    const double rk = (o.j == k ? 1.0 : R[o.j & 127u]) * pinv;
    if (o.j < N) {
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const uint32_t i = o.row(r);
        if (i < N) w[r] = (i == k) ? rk : ((o.j == k ? 0.0 : w[r]) - F[i] * rk);
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
  __shared__ double fcol[256], rowk[256];
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
  gj_invert(w, N, fcol, rowk, &bad);
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
    beta[j] = 0.0;
    active[j] = rho0[j] > t ? 1 : 0;
  }
  if (threadIdx.x == 0) {
    sc->err = 0;
    sc->cg_iters = 0;
  }
}

// Steps 2-3: M = I + tau/2 (S_a - S_b) + tau^2/4 (T - S_a S_b), S_a = S_b^T,
// B = M^{-1}, A = 2/tau (I - B) + S_b B, Z = [I - tau A ; tau B].
__global__ __launch_bounds__(SW) void k_small_solve(const double* __restrict__ Sb, const double* __restrict__ T,
                                                    double tau, uint32_t N, double* __restrict__ Bws,
                                                    double* __restrict__ Z, double* __restrict__ Aout,
                                                    OpeScalars* __restrict__ sc) {
  __shared__ double fcol[256], rowk[256];
  __shared__ int bad;
  const Own o;
  if (threadIdx.x == 0) bad = 0;
  const uint32_t jj = o.j < N ? o.j : 0u;
  double w[RPT];
  // M, with P = S_a S_b, P_ij = sum_k S_b[k][i] S_b[k][j]
  double P[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) P[r] = 0.0;
  for (uint32_t k = 0; k < N; ++k) {
    const double skj = Sb[(uint64_t)k * N + jj];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const uint32_t i = o.row(r);
      const double ski = Sb[(uint64_t)k * N + (i < N ? i : 0u)];
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
  gj_invert(w, N, fcol, rowk, &bad);
  store_own(Bws, N, w);           // B
  __syncthreads();
  // A = 2/tau (I - B) + S_b B
  double acc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
  for (uint32_t k = 0; k < N; ++k) {
    const double bkj = Bws[(uint64_t)k * N + jj];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const uint32_t i = o.row(r);
      acc[r] += Sb[(uint64_t)(i < N ? i : 0u) * N + k] * bkj;
    }
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
  __shared__ double fcol[256], rowk[256];
  __shared__ int bad;
  const Own o;
  if (threadIdx.x == 0) bad = 0;
  const uint32_t jj = o.j < N ? o.j : 0u;
  // Wsm = (C - I) S_b
  double acc[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
  for (uint32_t l = 0; l < N; ++l) {
    const double slj = Sb[(uint64_t)l * N + jj];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const uint32_t k = o.row(r) < N ? o.row(r) : 0u;
      acc[r] += (C[(uint64_t)k * N + l] - (k == l ? 1.0 : 0.0)) * slj;
    }
  }
  store_own(Wsm, N, acc);
  __syncthreads();
  // Q = S_b^T Wsm
  double qv[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) qv[r] = 0.0;
  for (uint32_t k = 0; k < N; ++k) {
    const double wkj = Wsm[(uint64_t)k * N + jj];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const uint32_t i = o.row(r) < N ? o.row(r) : 0u;
      qv[r] += Sb[(uint64_t)k * N + i] * wkj;
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
  gj_invert(w, N, fcol, rowk, &bad);
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
// held in global workspace; eigenvalues sorted ascending into evals.
__global__ __launch_bounds__(SW) void k_jacobi(const double* __restrict__ Asrc, double* __restrict__ W,
                                               double* __restrict__ evals, uint32_t N) {
  __shared__ double red[SW];
  __shared__ double cs[64], sn[64];
  __shared__ uint32_t pp[64], qq[64];
  __shared__ double dg[128];
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
      // rows: row_p' = c row_p - s row_q ; row_q' = s row_p + c row_q
      for (uint32_t e = threadIdx.x; e < npair * N; e += SW) {
        const uint32_t s = e / N, j = e - s * N;
        const uint32_t p = pp[s], q = qq[s];
        if (q < N) {
          const double xp = W[(uint64_t)p * N + j], xq = W[(uint64_t)q * N + j];
          W[(uint64_t)p * N + j] = cs[s] * xp - sn[s] * xq;
          W[(uint64_t)q * N + j] = sn[s] * xp + cs[s] * xq;
        }
      }
      __syncthreads();
      // columns: col_p' = c col_p - s col_q ; col_q' = s col_p + c col_q
      for (uint32_t e = threadIdx.x; e < npair * N; e += SW) {
        const uint32_t s = e / N, i = e - s * N;
        const uint32_t p = pp[s], q = qq[s];
        if (q < N) {
          const double xp = W[(uint64_t)i * N + p], xq = W[(uint64_t)i * N + q];
          W[(uint64_t)i * N + p] = cs[s] * xp - sn[s] * xq;
          W[(uint64_t)i * N + q] = sn[s] * xp + cs[s] * xq;
        }
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

}  // namespace

hipError_t launch_prep_small(ope_ctx* c) {
  ProfScope ps(c, OPE_KERNEL_SMALL);
  hipLaunchKernelGGL(k_prep_small, dim3(1), dim3(SW), 0, c->stream, c->C, c->Lam, c->Linv, c->cnorm2, (uint32_t)c->N,
                     c->sc, c->Lam32, c->Linv32);
  return hipGetLastError();
}

hipError_t launch_small_solve_delta(ope_ctx* c, const double* Sb, const double* Tperp, double tau) {
  ProfScope ps(c, OPE_KERNEL_SMALL);
  hipLaunchKernelGGL(k_small_solve_delta, dim3(1), dim3(SW), 0, c->stream, Sb, Tperp, c->C, tau, (uint32_t)c->N,
                     c->Wsm, c->Z32, c->sc);
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
  ProfScope ps(c, OPE_KERNEL_SMALL);
  hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(SW), 0, c->stream, Sb, T, tau, (uint32_t)c->N, B ? B : c->B, Z, A,
                     c->sc);
  return hipGetLastError();
}

hipError_t launch_jacobi_eig(ope_ctx* c, const double* Asym, double* evals) {
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(SW), 0, c->stream, Asym, c->Wsm, evals, (uint32_t)c->N);
  return hipGetLastError();
}
