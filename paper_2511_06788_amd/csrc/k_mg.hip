// Multigrid V-cycle: the preconditioner of Step 1's preconditioned CG
// (ope_set_multigrid).  Step 1 of the scheme (Section 4.1) solves the N source
// problems H y_j = u_j; the paper leaves the solver open.  One symmetric
// V-cycle per CG iteration takes the iteration count of the warm-started
// Step 1 at 64^3 from about seventy to about five.
//
// Hierarchy (built on the host at set-up): level k+1 halves every axis with
// more than one node (m' = ceil(m / 2); coarse node I is the parent of fine
// nodes 2I and 2I + 1), doubles its spacing (c_a' = c_a / 4), and takes as
// potential the mean of V + shift over the existing children; the first level
// k >= 1 with at most 512 nodes is solved exactly with a dense inverse
// (Cholesky on the host).  Transfers per coarsened axis: prolongation
// 3/4 e_I + 1/4 e_J (J = I - 1 for even fine nodes, I + 1 for odd ones,
// missing J = 0), restriction R = P^T / 2^d.  V-cycle, damped Jacobi
// (omega = 0.8) once on each side of the coarse correction:
//   x0 = omega b / d;  r1 = b - H x0;  e = B_{k+1}(R r1);  x1 = x0 + P e;
//   z = x1 + omega (b - H x1) / d.
// Kernels, per level: k_mg_res (r1, one stencil over x0 formed on the fly
// from b), k_mg_restrict (R r1), k_mg_dense (coarsest), k_mg_prolong
// (x1 = x0 + P e), k_mg_post (z, one stencil over x1; on level 0 also the
// per-column partial sums of r^T z and r^T r that the PCG needs).
// Layout: every block is n x N row-major (a grid point's N values
// contiguous), x fastest, as everywhere in the library; a thread owns one
// 16-byte chunk (VW = 2 doubles) or one double of a point's row.  Columns
// whose CG has converged are skipped.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "ope_internal.h"

namespace {

constexpr double MG_OMEGA = 0.8;
constexpr int64_t MG_COARSEST_MAX = 512;
constexpr uint32_t MG_WG = 256;
constexpr uint32_t MG_POST_WGS = 2048;      // work-groups of the level-0 post-smoothing (partial rows)

struct MgGeom {
  uint32_t m0, m1, m2;
  double cx, cy, cz;
};

template <int VW>
__device__ __forceinline__ void ldr(const double* __restrict__ a, uint64_t row, uint32_t N, uint32_t v,
                                    double (&o)[VW]) {
  if constexpr (VW == 2) {
    const double2 t = *reinterpret_cast<const double2*>(a + row * N + 2u * v);
    o[0] = t.x;
    o[1] = t.y;
  } else {
    o[0] = a[row * N + v];
  }
}

template <int VW>
__device__ __forceinline__ void str(double* __restrict__ a, uint64_t row, uint32_t N, uint32_t v,
                                    const double (&o)[VW]) {
  if constexpr (VW == 2) {
    *reinterpret_cast<double2*>(a + row * N + 2u * v) = make_double2(o[0], o[1]);
  } else {
    a[row * N + v] = o[0];
  }
}

template <int VW>
__device__ __forceinline__ bool vec_active(const int32_t* __restrict__ active, uint32_t v) {
  if (!active) return true;
  bool a = false;
#pragma unroll
  for (int k = 0; k < VW; ++k) a |= active[v * VW + k] != 0;
  return a;
}

// x0 = omega b / d at point q (zero outside the grid is the caller's job)
template <int VW>
__device__ __forceinline__ void jac0(const double* __restrict__ b, const double* __restrict__ diag, uint64_t q,
                                     uint32_t N, uint32_t v, double omega, double (&o)[VW]) {
  ldr<VW>(b, q, N, v, o);
  const double d = diag[q];
#pragma unroll
  for (int k = 0; k < VW; ++k) o[k] = (omega * o[k]) / d;
}

// (H f)(p) for a field given point-wise by F(q, out): d f - sum_a c_a (f(p - e_a) + f(p + e_a))
template <int VW, typename F>
__device__ __forceinline__ void stencil(const MgGeom& g, const double* __restrict__ diag, uint32_t x, uint32_t y,
                                        uint32_t z, uint64_t p, F&& field, double (&hx)[VW]) {
  double c[VW], xm[VW], xp[VW], ym[VW], yp[VW], zm[VW], zp[VW];
  field(p, c);
  const uint64_t s1 = g.m0, s2 = (uint64_t)g.m0 * g.m1;
#pragma unroll
  for (int k = 0; k < VW; ++k) xm[k] = xp[k] = ym[k] = yp[k] = zm[k] = zp[k] = 0.0;
  if (x > 0) field(p - 1, xm);
  if (x + 1 < g.m0) field(p + 1, xp);
  if (y > 0) field(p - s1, ym);
  if (y + 1 < g.m1) field(p + s1, yp);
  if (z > 0) field(p - s2, zm);
  if (z + 1 < g.m2) field(p + s2, zp);
  const double d = diag[p];
#pragma unroll
  for (int k = 0; k < VW; ++k)
    hx[k] = d * c[k] - (g.cx * (xm[k] + xp[k]) + g.cy * (ym[k] + yp[k]) + g.cz * (zm[k] + zp[k]));
}

// r1 = b - H x0, x0 = omega b / d
template <int VW>
__global__ __launch_bounds__(MG_WG) void k_mg_res(const double* __restrict__ b, double* __restrict__ out, MgGeom g,
                                                 const double* __restrict__ diag, double omega,
                                                 const int32_t* __restrict__ active, uint32_t N, uint32_t NV,
                                                 uint64_t total) {
  const uint64_t e = (uint64_t)xcd_remap(blockIdx.x, gridDim.x) * MG_WG + threadIdx.x;
  if (e >= total) return;
  const uint32_t v = (uint32_t)(e % NV);
  const uint64_t p = e / NV;
  if (!vec_active<VW>(active, v)) return;
  const uint32_t x = (uint32_t)(p % g.m0), y = (uint32_t)((p / g.m0) % g.m1), z = (uint32_t)(p / ((uint64_t)g.m0 * g.m1));
  double hx[VW], bc[VW], o[VW];
  stencil<VW>(g, diag, x, y, z, p, [&](uint64_t q, double(&f)[VW]) { jac0<VW>(b, diag, q, N, v, omega, f); }, hx);
  ldr<VW>(b, p, N, v, bc);
#pragma unroll
  for (int k = 0; k < VW; ++k) o[k] = bc[k] - hx[k];
  str<VW>(out, p, N, v, o);
}

// Fine nodes and weights of coarse node I along one axis (4 at most); the
// factor 1/2 of R = P^T / 2^d is applied per coarsened axis.
__device__ __forceinline__ int restrict_taps(uint32_t I, uint32_t mf, uint32_t (&f)[4], double (&w)[4]) {
  if (mf == 1) {
    f[0] = I;
    w[0] = 1.0;
    return 1;
  }
  int k = 0;
  const int64_t c[4] = {2 * (int64_t)I - 1, 2 * (int64_t)I, 2 * (int64_t)I + 1, 2 * (int64_t)I + 2};
  const double cw[4] = {0.125, 0.375, 0.375, 0.125};
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (c[t] >= 0 && c[t] < (int64_t)mf) {
      f[k] = (uint32_t)c[t];
      w[k] = cw[t];
      ++k;
    }
  return k;
}

// coarse B = R T
template <int VW>
__global__ __launch_bounds__(MG_WG) void k_mg_restrict(const double* __restrict__ T, double* __restrict__ B,
                                                      MgGeom fg, MgGeom cg, const int32_t* __restrict__ active,
                                                      uint32_t N, uint32_t NV, uint64_t total) {
  const uint64_t e = (uint64_t)xcd_remap(blockIdx.x, gridDim.x) * MG_WG + threadIdx.x;
  if (e >= total) return;
  const uint32_t v = (uint32_t)(e % NV);
  const uint64_t P = e / NV;
  if (!vec_active<VW>(active, v)) return;
  const uint32_t I = (uint32_t)(P % cg.m0), J = (uint32_t)((P / cg.m0) % cg.m1),
                 K = (uint32_t)(P / ((uint64_t)cg.m0 * cg.m1));
  uint32_t fx[4], fy[4], fz[4];
  double wx[4], wy[4], wz[4];
  const int nx = restrict_taps(I, fg.m0, fx, wx), ny = restrict_taps(J, fg.m1, fy, wy),
            nz = restrict_taps(K, fg.m2, fz, wz);
  double acc[VW];
#pragma unroll
  for (int k = 0; k < VW; ++k) acc[k] = 0.0;
  for (int c = 0; c < nz; ++c) {
    double ay[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) ay[k] = 0.0;
    for (int b = 0; b < ny; ++b) {
      double ax[VW];
#pragma unroll
      for (int k = 0; k < VW; ++k) ax[k] = 0.0;
      const uint64_t row = ((uint64_t)fz[c] * fg.m1 + fy[b]) * fg.m0;
      for (int a = 0; a < nx; ++a) {
        double t[VW];
        ldr<VW>(T, row + fx[a], N, v, t);
#pragma unroll
        for (int k = 0; k < VW; ++k) ax[k] += wx[a] * t[k];
      }
#pragma unroll
      for (int k = 0; k < VW; ++k) ay[k] += wy[b] * ax[k];
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) acc[k] += wz[c] * ay[k];
  }
  str<VW>(B, P, N, v, acc);
}

// coarsest level: E = A^{-1} B with the dense inverse (row-major nc x nc)
template <int VW>
__global__ __launch_bounds__(MG_WG) void k_mg_dense(const double* __restrict__ Ainv, const double* __restrict__ B,
                                                   double* __restrict__ E, uint32_t nc,
                                                   const int32_t* __restrict__ active, uint32_t N, uint32_t NV,
                                                   uint64_t total) {
  const uint64_t e = (uint64_t)blockIdx.x * MG_WG + threadIdx.x;
  if (e >= total) return;
  const uint32_t v = (uint32_t)(e % NV);
  const uint32_t i = (uint32_t)(e / NV);
  if (!vec_active<VW>(active, v)) return;
  double acc[VW];
#pragma unroll
  for (int k = 0; k < VW; ++k) acc[k] = 0.0;
  const double* a = Ainv + (uint64_t)i * nc;
  for (uint32_t j = 0; j < nc; ++j) {
    double t[VW];
    ldr<VW>(B, j, N, v, t);
    const double w = a[j];
#pragma unroll
    for (int k = 0; k < VW; ++k) acc[k] += w * t[k];
  }
  str<VW>(E, i, N, v, acc);
}

// Coarse nodes and weights of fine node f along one axis (2 at most).
__device__ __forceinline__ int prolong_taps(uint32_t f, uint32_t mf, uint32_t mc, uint32_t (&I)[2], double (&w)[2]) {
  if (mf == 1) {
    I[0] = f;
    w[0] = 1.0;
    return 1;
  }
  I[0] = f / 2;
  w[0] = 0.75;
  const int64_t J = (f % 2 == 0) ? (int64_t)(f / 2) - 1 : (int64_t)(f / 2) + 1;
  if (J >= 0 && J < (int64_t)mc) {
    I[1] = (uint32_t)J;
    w[1] = 0.25;
    return 2;
  }
  return 1;
}

// T = x0 + P E (x0 = omega b / d), on the fine level of the pair
template <int VW>
__global__ __launch_bounds__(MG_WG) void k_mg_prolong(const double* __restrict__ b, const double* __restrict__ E,
                                                     double* __restrict__ T, MgGeom fg, MgGeom cg,
                                                     const double* __restrict__ diag, double omega,
                                                     const int32_t* __restrict__ active, uint32_t N, uint32_t NV,
                                                     uint64_t total) {
  const uint64_t e = (uint64_t)xcd_remap(blockIdx.x, gridDim.x) * MG_WG + threadIdx.x;
  if (e >= total) return;
  const uint32_t v = (uint32_t)(e % NV);
  const uint64_t p = e / NV;
  if (!vec_active<VW>(active, v)) return;
  const uint32_t x = (uint32_t)(p % fg.m0), y = (uint32_t)((p / fg.m0) % fg.m1),
                 z = (uint32_t)(p / ((uint64_t)fg.m0 * fg.m1));
  uint32_t Ix[2], Iy[2], Iz[2];
  double wx[2], wy[2], wz[2];
  const int nx = prolong_taps(x, fg.m0, cg.m0, Ix, wx), ny = prolong_taps(y, fg.m1, cg.m1, Iy, wy),
            nz = prolong_taps(z, fg.m2, cg.m2, Iz, wz);
  double pe[VW];
#pragma unroll
  for (int k = 0; k < VW; ++k) pe[k] = 0.0;
  for (int c = 0; c < nz; ++c) {
    double ay[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) ay[k] = 0.0;
    for (int bb = 0; bb < ny; ++bb) {
      double ax[VW];
#pragma unroll
      for (int k = 0; k < VW; ++k) ax[k] = 0.0;
      const uint64_t row = ((uint64_t)Iz[c] * cg.m1 + Iy[bb]) * cg.m0;
      for (int a = 0; a < nx; ++a) {
        double t[VW];
        ldr<VW>(E, row + Ix[a], N, v, t);
#pragma unroll
        for (int k = 0; k < VW; ++k) ax[k] += wx[a] * t[k];
      }
#pragma unroll
      for (int k = 0; k < VW; ++k) ay[k] += wy[bb] * ax[k];
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) pe[k] += wz[c] * ay[k];
  }
  double x0[VW], o[VW];
  jac0<VW>(b, diag, p, N, v, omega, x0);
#pragma unroll
  for (int k = 0; k < VW; ++k) o[k] = x0[k] + pe[k];
  str<VW>(T, p, N, v, o);
}

// z = x1 + omega (b - H x1) / d with x1 in T.  A work-group owns a contiguous
// range of `ppw` points; thread t < PL NV (PL = 256 / NV point lanes) owns
// vector t % NV of every PL-th point.  With DOTS, the work-group's sums of
// b z and b b per column (point lanes added in order) form row blockIdx.x of
// part (2N columns: r^T z, then r^T r).
template <int VW, bool DOTS>
__global__ __launch_bounds__(MG_WG) void k_mg_post(const double* __restrict__ b, const double* __restrict__ T,
                                                  double* __restrict__ out, MgGeom g,
                                                  const double* __restrict__ diag, double omega,
                                                  const int32_t* __restrict__ active, uint32_t N, uint32_t NV,
                                                  uint64_t n, uint64_t ppw, double* __restrict__ part) {
  const uint32_t PL = MG_WG / NV;
  const uint32_t t = threadIdx.x;
  const bool lane_ok = t < PL * NV;
  const uint32_t v = lane_ok ? t % NV : 0, pl = lane_ok ? t / NV : 0;
  const bool act = lane_ok && vec_active<VW>(active, v);
  const uint64_t p0 = (uint64_t)blockIdx.x * ppw;
  const uint64_t p1 = p0 + ppw < n ? p0 + ppw : n;
  double srz[VW], srr[VW];
#pragma unroll
  for (int k = 0; k < VW; ++k) srz[k] = srr[k] = 0.0;
  if (act) {
    for (uint64_t p = p0 + pl; p < p1; p += PL) {
      const uint32_t x = (uint32_t)(p % g.m0), y = (uint32_t)((p / g.m0) % g.m1),
                     z = (uint32_t)(p / ((uint64_t)g.m0 * g.m1));
      double hx[VW], bc[VW], xc[VW], o[VW];
      stencil<VW>(g, diag, x, y, z, p, [&](uint64_t q, double(&f)[VW]) { ldr<VW>(T, q, N, v, f); }, hx);
      ldr<VW>(b, p, N, v, bc);
      ldr<VW>(T, p, N, v, xc);
      const double d = diag[p];
#pragma unroll
      for (int k = 0; k < VW; ++k) o[k] = xc[k] + (omega * (bc[k] - hx[k])) / d;
      str<VW>(out, p, N, v, o);
      if constexpr (DOTS) {
#pragma unroll
        for (int k = 0; k < VW; ++k) {
          srz[k] += bc[k] * o[k];
          srr[k] += bc[k] * bc[k];
        }
      }
    }
  }
  if constexpr (DOTS) {
    __shared__ double red[2 * MG_WG * 2];
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      red[(t * VW + k) * 2 + 0] = srz[k];
      red[(t * VW + k) * 2 + 1] = srr[k];
    }
    __syncthreads();
    // thread c < N sums column c over the point lanes in order
    for (uint32_t c = t; c < N; c += MG_WG) {
      const uint32_t cv = c / VW, ck = c % VW;
      double a = 0.0, bsum = 0.0;
      for (uint32_t l = 0; l < PL; ++l) {
        const uint32_t th = l * NV + cv;
        a += red[(th * VW + ck) * 2 + 0];
        bsum += red[(th * VW + ck) * 2 + 1];
      }
      part[(uint64_t)blockIdx.x * 2 * N + c] = a;
      part[(uint64_t)blockIdx.x * 2 * N + N + c] = bsum;
    }
  }
}

// PCG start: rho = r^T z (the CG set-up has already set the targets and the
// convergence flags from |r|^2).
__global__ __launch_bounds__(MG_WG) void k_pcg_start(const double* __restrict__ dots, uint32_t N,
                                                    double* __restrict__ rho) {
  for (uint32_t j = threadIdx.x; j < N; j += MG_WG) rho[j] = dots[j];
}

// PCG after the preconditioning of the new residual: for a running column,
// beta = r^T z / rho, rho = r^T z, and it keeps running while |r|^2 > target
// (a non-positive r^T z, which an SPD preconditioner cannot give, stops it).
__global__ __launch_bounds__(MG_WG) void k_pcg_beta(const double* __restrict__ dots, uint32_t N,
                                                   double* __restrict__ rho, double* __restrict__ beta,
                                                   const double* __restrict__ target, int32_t* __restrict__ active,
                                                   OpeScalars* __restrict__ sc) {
  for (uint32_t j = threadIdx.x; j < N; j += MG_WG) {
    if (!active[j]) {
      beta[j] = 0.0;
      continue;
    }
    const double rz = dots[j], rr = dots[N + j];
    if (!isfinite(rz) || !isfinite(rr)) {
      if (sc->err == 0) sc->err = OPE_ENONFINITE;
      active[j] = 0;
      beta[j] = 0.0;
      continue;
    }
    beta[j] = rz / rho[j];
    rho[j] = rz;
    active[j] = (rr > target[j] && rz > 0.0) ? 1 : 0;
  }
}

inline MgGeom geom(const MgLevel& L) { return MgGeom{L.m0, L.m1, L.m2, L.cx, L.cy, L.cz}; }

inline uint32_t grid_of(uint64_t total) { return (uint32_t)((total + MG_WG - 1) / MG_WG); }

// Dense inverse of an SPD matrix (row-major, n x n) by Cholesky: A = L L^T,
// A^{-1} = L^{-T} L^{-1}.  False if A is not positive definite.
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / ljj;
    }
  }
  // Li = L^{-1} (lower triangular), by forward substitution per column
  std::vector<double> Li((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    for (int i = c; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) t -= L[(size_t)i * n + k] * Li[(size_t)k * n + c];
      Li[(size_t)i * n + c] = t / L[(size_t)i * n + i];
    }
  }
  // A^{-1} = Li^T Li
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double t = 0.0;
      for (int k = i; k < n; ++k) t += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
      A[(size_t)i * n + j] = t;
      A[(size_t)j * n + i] = t;
    }
  return true;
}

}  // namespace

void mg_free(ope_ctx* c) {
  for (int k = 1; k < c->mg_levels; ++k)
    if (c->mg[k].diag) (void)hipFree(c->mg[k].diag);
  if (c->mg_mem) (void)hipFree(c->mg_mem);
  if (c->mg_inv) (void)hipFree(c->mg_inv);
  if (c->mg_part) (void)hipFree(c->mg_part);
  if (c->mg_dots) (void)hipFree(c->mg_dots);
  c->mg_mem = nullptr;
  c->mg_inv = nullptr;
  c->mg_part = nullptr;
  c->mg_dots = nullptr;
  c->mg_Z = nullptr;
  for (int k = 0; k < OPE_MG_MAX_LEVELS; ++k) c->mg[k] = MgLevel{};
  c->mg_levels = 0;
  c->mg_on = 0;
}

ope_status mg_build(ope_ctx* c) {
  mg_free(c);
  const int64_t N = c->N;
  // level 0: the operator; its potential W = diag - 2 (cx + cy + cz)
  std::vector<double> W((size_t)c->n);
  if (hipMemcpy(W.data(), c->diag, sizeof(double) * c->n, hipMemcpyDeviceToHost) != hipSuccess) return OPE_EHIP;
  const double dsum0 = 2.0 * (c->g.cx + c->g.cy + c->g.cz);
  for (auto& w : W) w -= dsum0;
  std::vector<std::vector<double>> diags;
  MgLevel L0{};
  L0.m0 = c->g.m0;
  L0.m1 = c->g.m1;
  L0.m2 = c->g.m2;
  L0.cx = c->g.cx;
  L0.cy = c->g.cy;
  L0.cz = c->g.cz;
  L0.n = c->n;
  L0.diag = c->diag;
  MgLevel lv[OPE_MG_MAX_LEVELS];
  lv[0] = L0;
  int nl = 1;
  std::vector<double> Wc;
  while (nl == 1 || lv[nl - 1].n > MG_COARSEST_MAX) {
    const MgLevel& f = lv[nl - 1];
    MgLevel q{};
    q.m0 = f.m0 > 1 ? (f.m0 + 1) / 2 : 1;
    q.m1 = f.m1 > 1 ? (f.m1 + 1) / 2 : 1;
    q.m2 = f.m2 > 1 ? (f.m2 + 1) / 2 : 1;
    if (q.m0 == f.m0 && q.m1 == f.m1 && q.m2 == f.m2) break;
    if (nl == OPE_MG_MAX_LEVELS) return OPE_EUNSUPPORTED;
    q.cx = f.m0 > 1 ? f.cx / 4.0 : f.cx;
    q.cy = f.m1 > 1 ? f.cy / 4.0 : f.cy;
    q.cz = f.m2 > 1 ? f.cz / 4.0 : f.cz;
    q.n = (int64_t)q.m0 * q.m1 * q.m2;
    // coarse potential: mean over the existing children
    Wc.assign((size_t)q.n, 0.0);
    for (uint32_t K = 0; K < q.m2; ++K)
      for (uint32_t J = 0; J < q.m1; ++J)
        for (uint32_t I = 0; I < q.m0; ++I) {
          double s = 0.0;
          int cnt = 0;
          const uint32_t zs = f.m2 > 1 ? 2 * K : K, ze = f.m2 > 1 ? std::min(2 * K + 2, f.m2) : K + 1;
          const uint32_t ys = f.m1 > 1 ? 2 * J : J, ye = f.m1 > 1 ? std::min(2 * J + 2, f.m1) : J + 1;
          const uint32_t xs = f.m0 > 1 ? 2 * I : I, xe = f.m0 > 1 ? std::min(2 * I + 2, f.m0) : I + 1;
          for (uint32_t z = zs; z < ze; ++z)
            for (uint32_t y = ys; y < ye; ++y)
              for (uint32_t x = xs; x < xe; ++x) {
                s += W[((size_t)z * f.m1 + y) * f.m0 + x];
                ++cnt;
              }
          Wc[((size_t)K * q.m1 + J) * q.m0 + I] = s / cnt;
        }
    W.swap(Wc);
    std::vector<double> d((size_t)q.n);
    const double dsum = 2.0 * (q.cx + q.cy + q.cz);
    for (int64_t p = 0; p < q.n; ++p) d[(size_t)p] = W[(size_t)p] + dsum;
    diags.push_back(d);
    lv[nl++] = q;
  }
  if (nl < 2) return OPE_EUNSUPPORTED;
  // coarsest operator, dense, and its inverse
  const MgLevel& cl = lv[nl - 1];
  const int nc = (int)cl.n;
  std::vector<double> A((size_t)nc * nc, 0.0);
  const std::vector<double>& dc = diags.back();
  for (uint32_t z = 0; z < cl.m2; ++z)
    for (uint32_t y = 0; y < cl.m1; ++y)
      for (uint32_t x = 0; x < cl.m0; ++x) {
        const size_t p = ((size_t)z * cl.m1 + y) * cl.m0 + x;
        A[p * nc + p] = dc[p];
        if (x > 0) A[p * nc + p - 1] = -cl.cx;
        if (x + 1 < cl.m0) A[p * nc + p + 1] = -cl.cx;
        if (y > 0) A[p * nc + p - cl.m0] = -cl.cy;
        if (y + 1 < cl.m1) A[p * nc + p + cl.m0] = -cl.cy;
        if (z > 0) A[p * nc + p - (size_t)cl.m0 * cl.m1] = -cl.cz;
        if (z + 1 < cl.m2) A[p * nc + p + (size_t)cl.m0 * cl.m1] = -cl.cz;
      }
  if (!spd_inverse(A, nc)) return OPE_ENOTSPD;
  // device memory: level diagonals, blocks (level 0: T and Z; others: B, E, T)
  int64_t elems = 2 * c->n * N;
  for (int k = 1; k < nl; ++k) elems += 3 * lv[k].n * N;
  c->mg_rows = std::min<int64_t>(MG_POST_WGS, (c->n + 3) / 4);
  bool ok = hipMalloc(&c->mg_mem, sizeof(double) * (size_t)elems) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->mg_inv, sizeof(double) * (size_t)nc * nc) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->mg_part, sizeof(double) * (size_t)c->mg_rows * 2 * N) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->mg_dots, sizeof(double) * 2 * (size_t)N) == hipSuccess;
  for (int k = 1; k < nl && ok; ++k) ok = hipMalloc((void**)&lv[k].diag, sizeof(double) * lv[k].n) == hipSuccess;
  c->mg_levels = nl;
  for (int k = 0; k < nl; ++k) c->mg[k] = lv[k];
  if (!ok) {
    mg_free(c);
    return OPE_ENOMEM;
  }
  double* mem = (double*)c->mg_mem;
  c->mg[0].T = mem;
  mem += c->n * N;
  c->mg_Z = mem;
  mem += c->n * N;
  for (int k = 1; k < nl; ++k) {
    c->mg[k].B = mem;
    mem += c->mg[k].n * N;
    c->mg[k].E = mem;
    mem += c->mg[k].n * N;
    c->mg[k].T = mem;
    mem += c->mg[k].n * N;
  }
  ok = hipMemcpy(c->mg_inv, A.data(), sizeof(double) * (size_t)nc * nc, hipMemcpyHostToDevice) == hipSuccess;
  for (int k = 1; k < nl && ok; ++k)
    ok = hipMemcpy(c->mg[k].diag, diags[(size_t)k - 1].data(), sizeof(double) * c->mg[k].n,
                   hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    mg_free(c);
    return OPE_EHIP;
  }
  return OPE_OK;
}

template <int VW>
static hipError_t vcycle_t(ope_ctx* c, const double* r, double* z, const int32_t* active, bool dots) {
  const uint32_t N = (uint32_t)c->N, NV = N / VW;
  const int L = c->mg_levels;
  hipStream_t s = c->stream;
  for (int k = 0; k + 1 < L; ++k) {
    const MgLevel& f = c->mg[k];
    const MgLevel& q = c->mg[k + 1];
    const double* in = k == 0 ? r : f.B;
    const uint64_t tf = (uint64_t)f.n * NV, tc = (uint64_t)q.n * NV;
    hipLaunchKernelGGL(k_mg_res<VW>, dim3(grid_of(tf)), dim3(MG_WG), 0, s, in, f.T, geom(f), f.diag, MG_OMEGA, active,
                       N, NV, tf);
    hipLaunchKernelGGL(k_mg_restrict<VW>, dim3(grid_of(tc)), dim3(MG_WG), 0, s, f.T, q.B, geom(f), geom(q), active, N,
                       NV, tc);
  }
  const MgLevel& cl = c->mg[L - 1];
  const uint64_t tcl = (uint64_t)cl.n * NV;
  hipLaunchKernelGGL(k_mg_dense<VW>, dim3(grid_of(tcl)), dim3(MG_WG), 0, s, c->mg_inv, cl.B, cl.E, (uint32_t)cl.n,
                     active, N, NV, tcl);
  for (int k = L - 2; k >= 0; --k) {
    const MgLevel& f = c->mg[k];
    const MgLevel& q = c->mg[k + 1];
    const double* in = k == 0 ? r : f.B;
    double* out = k == 0 ? z : f.E;
    const uint64_t tf = (uint64_t)f.n * NV;
    hipLaunchKernelGGL(k_mg_prolong<VW>, dim3(grid_of(tf)), dim3(MG_WG), 0, s, in, q.E, f.T, geom(f), geom(q), f.diag,
                       MG_OMEGA, active, N, NV, tf);
    const uint32_t PL = MG_WG / NV;
    const uint64_t wgs = k == 0 ? (uint64_t)c->mg_rows : std::min<uint64_t>(4096, (f.n + PL - 1) / PL);
    uint64_t ppw = (f.n + wgs - 1) / wgs;
    ppw = (ppw + PL - 1) / PL * PL;
    const uint32_t grid = (uint32_t)((f.n + ppw - 1) / ppw);
    if (k == 0 && dots) {
      // rows past the last used work-group stay zero
      hipLaunchKernelGGL((k_mg_post<VW, true>), dim3(grid), dim3(MG_WG), 0, s, in, f.T, out, geom(f), f.diag, MG_OMEGA,
                         active, N, NV, (uint64_t)f.n, ppw, c->mg_part);
      c->mg_rows_used = grid;
    } else {
      hipLaunchKernelGGL((k_mg_post<VW, false>), dim3(grid), dim3(MG_WG), 0, s, in, f.T, out, geom(f), f.diag,
                         MG_OMEGA, active, N, NV, (uint64_t)f.n, ppw, nullptr);
    }
  }
  return hipGetLastError();
}

hipError_t mg_vcycle(ope_ctx* c, const double* r, double* z, const int32_t* active, bool dots) {
  ProfScope ps(c, OPE_KERNEL_MG);
  if (c->N % 2 == 0) return vcycle_t<2>(c, r, z, active, dots);
  return vcycle_t<1>(c, r, z, active, dots);
}

hipError_t launch_pcg_start(ope_ctx* c) {
  hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(MG_WG), 0, c->stream, c->mg_dots, (uint32_t)c->N, c->rho);
  return hipGetLastError();
}

hipError_t launch_pcg_beta(ope_ctx* c) {
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(MG_WG), 0, c->stream, c->mg_dots, (uint32_t)c->N, c->rho, c->beta,
                     c->target, c->active, c->sc);
  return hipGetLastError();
}
