// Stencil SpMM and the conjugate-gradient sweeps of Step 1 (Section 4.1) on gfx950.
//
// H = c (-Lap_h) + diag(V + sigma) on the interior nodes of a uniform grid with
// homogeneous Dirichlet boundary (the bilinear form a(u,v) of Section 2.2):
//   (H x)_p = d_p x_p - cx (x_{p-1} + x_{p+1}) - cy (x_{p-s1} + x_{p+s1}) - cz (x_{p-s2} + x_{p+s2}),
//   d_p = V_p + sigma + 2 (cx + cy + cz),  c_a = kinetic / h_a^2,
// with the neighbour terms dropped outside the grid.
//
// All kernels are HBM-bound streaming kernels.  A block row (the N orbitals of
// one grid point) is read by N/VW consecutive lanes with 16-byte loads, so a
// wavefront covers whole rows; the six neighbour rows are re-read through the
// caches.  Work-groups are mapped XCD-contiguously (xcd_remap) so that each
// XCD's L2 holds the neighbouring planes of the rows it streams.
//
// Step 1 solves the N source problems H y_j = u_j independently (one CG per
// column).  One CG iteration is two sweeps:
//   sweep A (cg_pap):    p = r + beta p_old (formed on the fly), sigma_j = p_j^T H p_j
//   sweep B (cg_update): p = r + beta p_old, y += alpha p, r' = r - alpha H p,
//                        rho'_j = r'_j^T r'_j, and p is written out
// so an iteration moves 8 block-passes (A reads r, p_old; B reads r, p_old, y
// and writes r', p, y) instead of materialising q = H p.  The per-column
// scalars alpha, beta, rho and the convergence flags live on the device and
// are produced by the fixed-order reductions at the end of this file.
#include "ope_internal.h"

namespace {

template <int VW>
__device__ __forceinline__ void ldv(const double* __restrict__ base, uint64_t off, double (&v)[VW]) {
  if constexpr (VW == 2) {
    const double2 t = *reinterpret_cast<const double2*>(base + off);
    v[0] = t.x;
    v[1] = t.y;
  } else {
    v[0] = base[off];
  }
}

template <int VW>
__device__ __forceinline__ void stv(double* __restrict__ base, uint64_t off, const double (&v)[VW]) {
  if constexpr (VW == 2) {
    *reinterpret_cast<double2*>(base + off) = make_double2(v[0], v[1]);
  } else {
    base[off] = v[0];
  }
}

struct PointCoord {
  uint32_t i0, i1, i2;
};

__device__ __forceinline__ PointCoord coords(uint32_t p, const OpeGrid& g) {
  PointCoord c;
  const uint32_t t = p / g.m0;
  c.i0 = p - t * g.m0;
  c.i2 = t / g.m1;
  c.i1 = t - c.i2 * g.m1;
  return c;
}

// Search direction value at element offset `off`: r + beta * p_old (r on the first iteration).
template <int VW, bool FIRST>
__device__ __forceinline__ void dirv(const double* __restrict__ r, const double* __restrict__ pold,
                                     uint64_t off, const double (&b)[VW], double (&out)[VW]) {
  double rv[VW];
  ldv<VW>(r, off, rv);
  if constexpr (FIRST) {
#pragma unroll
    for (int v = 0; v < VW; ++v) out[v] = rv[v];
  } else {
    double pv[VW];
    ldv<VW>(pold, off, pv);
#pragma unroll
    for (int v = 0; v < VW; ++v) out[v] = rv[v] + b[v] * pv[v];
  }
}

// (H x) at point p for the field produced by `get(off, out)`, given x_p = xc.
template <int VW, typename Get>
__device__ __forceinline__ void stencil_at(uint32_t p, uint64_t off, uint64_t rowlen, const OpeGrid& g,
                                           const double* __restrict__ diag, const double (&xc)[VW],
                                           Get&& get, double (&hx)[VW]) {
  const PointCoord pc = coords(p, g);
  const double d = diag[p];
  double nx[VW], ny[VW], nz[VW], t[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) nx[v] = ny[v] = nz[v] = 0.0;
  if (pc.i0 > 0) { get(off - rowlen, t); for (int v = 0; v < VW; ++v) nx[v] += t[v]; }
  if (pc.i0 + 1 < g.m0) { get(off + rowlen, t); for (int v = 0; v < VW; ++v) nx[v] += t[v]; }
  if (pc.i1 > 0) { get(off - rowlen * g.s1, t); for (int v = 0; v < VW; ++v) ny[v] += t[v]; }
  if (pc.i1 + 1 < g.m1) { get(off + rowlen * g.s1, t); for (int v = 0; v < VW; ++v) ny[v] += t[v]; }
  if (g.dim == 3) {
    if (pc.i2 > 0) { get(off - rowlen * g.s2, t); for (int v = 0; v < VW; ++v) nz[v] += t[v]; }
    if (pc.i2 + 1 < g.m2) { get(off + rowlen * g.s2, t); for (int v = 0; v < VW; ++v) nz[v] += t[v]; }
  }
#pragma unroll
  for (int v = 0; v < VW; ++v) hx[v] = d * xc[v] - (g.cx * nx[v] + g.cy * ny[v] + g.cz * nz[v]);
}

template <int VW>
__global__ __launch_bounds__(OPE_WG) void k_apply_h(const double* __restrict__ X, double* __restrict__ Yo,
                                                    const double* __restrict__ diag, OpeGrid g, uint32_t N,
                                                    uint32_t NV, uint64_t total) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  const uint64_t e = (uint64_t)b * OPE_WG + threadIdx.x;
  if (e >= total) return;
  const uint32_t p = (uint32_t)(e / NV);
  const uint32_t cv = (uint32_t)(e - (uint64_t)p * NV);
  const uint64_t off = (uint64_t)p * N + (uint64_t)cv * VW;
  double xc[VW], hx[VW];
  ldv<VW>(X, off, xc);
  stencil_at<VW>(p, off, N, g, diag, xc, [&](uint64_t o, double (&t)[VW]) { ldv<VW>(X, o, t); }, hx);
  stv<VW>(Yo, off, hx);
}

__device__ __forceinline__ bool any_active(const int32_t* __restrict__ active, uint32_t N) {
  int a = 0;
  for (uint32_t j = threadIdx.x; j < N; j += OPE_WG) a |= active[j];
  return __syncthreads_or(a) != 0;
}

// Writes the work-group's per-column sums of acc (one row of `part`).
template <int VW>
__device__ __forceinline__ void wg_colsum(double* red, const double (&acc)[VW], bool lane_ok, uint32_t lp_count,
                                          uint32_t NV, uint32_t N, double* __restrict__ part_row) {
#pragma unroll
  for (int v = 0; v < VW; ++v) red[threadIdx.x * VW + v] = lane_ok ? acc[v] : 0.0;
  __syncthreads();
  for (uint32_t c = threadIdx.x; c < NV; c += OPE_WG) {
    double s[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) s[v] = 0.0;
    for (uint32_t l = 0; l < lp_count; ++l) {
#pragma unroll
      for (int v = 0; v < VW; ++v) s[v] += red[(l * NV + c) * VW + v];
    }
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      const uint32_t col = c * VW + v;
      if (col < N) part_row[col] = s[v];
    }
  }
}

template <int VW, bool FIRST>
__global__ __launch_bounds__(OPE_WG) void k_cg_pap(const double* __restrict__ r, const double* __restrict__ pold,
                                                   const double* __restrict__ beta, const int32_t* __restrict__ active,
                                                   const double* __restrict__ diag, OpeGrid g, uint32_t n, uint32_t N,
                                                   uint32_t NV, uint32_t pts, double* __restrict__ part,
                                                   OpeScalars* __restrict__ sc) {
  __shared__ double red[OPE_WG * VW];
  if (!any_active(active, N)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->cg_iters += 1;
  const uint32_t wg = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t pp = OPE_WG / NV;                 // points per pass
  const uint32_t lp = threadIdx.x / NV, cv = threadIdx.x - lp * NV;
  const bool lane_ok = lp < pp;
  double b[VW], acc[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) {
    b[v] = FIRST ? 0.0 : beta[cv * VW + v];
    acc[v] = 0.0;
  }
  const uint32_t p0 = wg * pts;
  const uint32_t p1 = min(n, p0 + pts);
  if (lane_ok) {
    for (uint32_t p = p0 + lp; p < p1; p += pp) {
      const uint64_t off = (uint64_t)p * N + (uint64_t)cv * VW;
      double pc[VW], hp[VW];
      dirv<VW, FIRST>(r, pold, off, b, pc);
      stencil_at<VW>(p, off, N, g, diag, pc,
                     [&](uint64_t o, double (&t)[VW]) { dirv<VW, FIRST>(r, pold, o, b, t); }, hp);
#pragma unroll
      for (int v = 0; v < VW; ++v) acc[v] += pc[v] * hp[v];
    }
  }
  wg_colsum<VW>(red, acc, lane_ok, pp, NV, N, part + (uint64_t)wg * N);
}

template <int VW, bool FIRST>
__global__ __launch_bounds__(OPE_WG) void k_cg_update(const double* __restrict__ r, const double* __restrict__ pold,
                                                      double* __restrict__ rnew, double* __restrict__ pnew,
                                                      double* __restrict__ y, const double* __restrict__ alpha,
                                                      const double* __restrict__ beta, const int32_t* __restrict__ active,
                                                      const double* __restrict__ diag, OpeGrid g, uint32_t n,
                                                      uint32_t N, uint32_t NV, uint32_t pts, double* __restrict__ part) {
  __shared__ double red[OPE_WG * VW];
  if (!any_active(active, N)) return;
  const uint32_t wg = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t pp = OPE_WG / NV;
  const uint32_t lp = threadIdx.x / NV, cv = threadIdx.x - lp * NV;
  const bool lane_ok = lp < pp;
  double b[VW], a[VW], acc[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) {
    b[v] = FIRST ? 0.0 : beta[cv * VW + v];
    a[v] = alpha[cv * VW + v];
    acc[v] = 0.0;
  }
  const uint32_t p0 = wg * pts;
  const uint32_t p1 = min(n, p0 + pts);
  if (lane_ok) {
    for (uint32_t p = p0 + lp; p < p1; p += pp) {
      const uint64_t off = (uint64_t)p * N + (uint64_t)cv * VW;
      double pc[VW], hp[VW], rc[VW], yc[VW];
      dirv<VW, FIRST>(r, pold, off, b, pc);
      stencil_at<VW>(p, off, N, g, diag, pc,
                     [&](uint64_t o, double (&t)[VW]) { dirv<VW, FIRST>(r, pold, o, b, t); }, hp);
      ldv<VW>(r, off, rc);
      ldv<VW>(y, off, yc);
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        yc[v] += a[v] * pc[v];
        rc[v] -= a[v] * hp[v];
        acc[v] += rc[v] * rc[v];
      }
      stv<VW>(y, off, yc);
      stv<VW>(rnew, off, rc);
      stv<VW>(pnew, off, pc);
    }
  }
  wg_colsum<VW>(red, acc, lane_ok, pp, NV, N, part + (uint64_t)wg * N);
}

// r0 = U - H Y0 (HY given) or r0 = U with y zeroed (HY null); one partial row of
// 2N values per work-group: sums of r0^2 (first N) and of U^2 (next N).
template <int VW>
__global__ __launch_bounds__(OPE_WG) void k_resid0(const double* __restrict__ U, const double* __restrict__ HY,
                                                   double* __restrict__ R, double* __restrict__ y, uint32_t n,
                                                   uint32_t N, uint32_t NV, uint32_t pts, double* __restrict__ part) {
  __shared__ double red[OPE_WG * VW];
  const uint32_t wg = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t pp = OPE_WG / NV;
  const uint32_t lp = threadIdx.x / NV, cv = threadIdx.x - lp * NV;
  const bool lane_ok = lp < pp;
  double ar[VW], au[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) ar[v] = au[v] = 0.0;
  const uint32_t p0 = wg * pts;
  const uint32_t p1 = min(n, p0 + pts);
  if (lane_ok) {
    for (uint32_t p = p0 + lp; p < p1; p += pp) {
      const uint64_t off = (uint64_t)p * N + (uint64_t)cv * VW;
      double u[VW], r[VW];
      ldv<VW>(U, off, u);
      if (HY) {
        double t[VW];
        ldv<VW>(HY, off, t);
#pragma unroll
        for (int v = 0; v < VW; ++v) r[v] = u[v] - t[v];
      } else {
        double z[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          r[v] = u[v];
          z[v] = 0.0;
        }
        stv<VW>(y, off, z);
      }
      stv<VW>(R, off, r);
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        ar[v] += r[v] * r[v];
        au[v] += u[v] * u[v];
      }
    }
  }
  double* row = part + (uint64_t)wg * 2 * N;
  wg_colsum<VW>(red, ar, lane_ok, pp, NV, N, row);
  __syncthreads();
  wg_colsum<VW>(red, au, lane_ok, pp, NV, N, row + N);
}

// Column sums of a [nrows][ncols] partial array in a fixed order, split over
// gridDim.y work-groups per column group with a last-block second stage, and
// an optional CG finalisation per column.
template <int MODE>
__global__ __launch_bounds__(OPE_WG) void k_reduce_cols(const double* __restrict__ part, uint32_t nrows,
                                                        uint32_t ncols, double* __restrict__ out,
                                                        double* __restrict__ stage, uint32_t* __restrict__ counters,
                                                        double* __restrict__ alpha, double* __restrict__ beta,
                                                        double* __restrict__ rho, const double* __restrict__ target,
                                                        int32_t* __restrict__ active, OpeScalars* __restrict__ sc) {
  __shared__ double red[OPE_WG];
  __shared__ uint32_t ticket;
  // No early exit here even when every column has converged: the partials are
  // then stale, but inactive columns only ever receive alpha = beta = 0, and a
  // uniform exit keeps the last-block counters consistent.
  const uint32_t S = gridDim.y, s = blockIdx.y;
  const uint32_t lc = threadIdx.x & 63u, grp = threadIdx.x >> 6;
  const uint32_t col = blockIdx.x * 64u + lc;
  const uint32_t rps = (nrows + S - 1) / S;
  const uint32_t w0 = s * rps, w1 = min(nrows, w0 + rps);
  double acc = 0.0;
  if (col < ncols)
    for (uint32_t w = w0 + grp; w < w1; w += 4) acc += part[(uint64_t)w * ncols + col];
  red[threadIdx.x] = acc;
  __syncthreads();
  double tot = 0.0;
  if (grp == 0) tot = red[lc] + red[64 + lc] + red[128 + lc] + red[192 + lc];
  if (S > 1) {
    if (grp == 0 && col < ncols) stage[(uint64_t)s * ncols + col] = tot;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) ticket = atomicAdd(&counters[blockIdx.x], 1u);
    __syncthreads();
    if (ticket != S - 1) return;
    __threadfence();
    if (grp == 0) {
      tot = 0.0;
      if (col < ncols)
        for (uint32_t k = 0; k < S; ++k) tot += stage[(uint64_t)k * ncols + col];
    }
    if (threadIdx.x == 0) counters[blockIdx.x] = 0u;
  }
  if (grp != 0 || col >= ncols) return;
  if (MODE == RED_PLAIN) {
    out[col] = tot;
  } else if (MODE == RED_CG_ALPHA) {
    const bool act = active[col] != 0;
    if (act && !isfinite(tot)) sc->err = OPE_ENONFINITE;
    alpha[col] = (act && tot > 0.0 && isfinite(tot)) ? rho[col] / tot : 0.0;
  } else {  // RED_CG_BETA
    if (active[col]) {
      if (!isfinite(tot)) {
        sc->err = OPE_ENONFINITE;
        active[col] = 0;
        beta[col] = 0.0;
      } else {
        beta[col] = tot / rho[col];
        rho[col] = tot;
        active[col] = tot > target[col] ? 1 : 0;
      }
    } else {
      beta[col] = 0.0;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_apply_h(ope_ctx* c, const double* X, double* Yo) {
  const uint32_t N = (uint32_t)c->N;
  const uint32_t NV = N / c->vw;
  const uint64_t total = (uint64_t)c->n * NV;
  const uint32_t grid = (uint32_t)((total + OPE_WG - 1) / OPE_WG);
  if (c->vw == 2)
    hipLaunchKernelGGL((k_apply_h<2>), dim3(grid), dim3(OPE_WG), 0, c->stream, X, Yo, c->diag, c->g, N, NV, total);
  else
    hipLaunchKernelGGL((k_apply_h<1>), dim3(grid), dim3(OPE_WG), 0, c->stream, X, Yo, c->diag, c->g, N, NV, total);
  return hipGetLastError();
}

hipError_t launch_cg_pap(ope_ctx* c, const double* r, const double* pold, int first) {
  const uint32_t N = (uint32_t)c->N, NV = N / c->vw, n = (uint32_t)c->n;
  const dim3 grid(c->stream_wgs), blk(OPE_WG);
  const uint32_t pts = (uint32_t)c->stream_pts;
  if (c->vw == 2) {
    if (first)
      hipLaunchKernelGGL((k_cg_pap<2, true>), grid, blk, 0, c->stream, r, pold, c->beta, c->active, c->diag, c->g, n, N, NV, pts, c->part, c->sc);
    else
      hipLaunchKernelGGL((k_cg_pap<2, false>), grid, blk, 0, c->stream, r, pold, c->beta, c->active, c->diag, c->g, n, N, NV, pts, c->part, c->sc);
  } else {
    if (first)
      hipLaunchKernelGGL((k_cg_pap<1, true>), grid, blk, 0, c->stream, r, pold, c->beta, c->active, c->diag, c->g, n, N, NV, pts, c->part, c->sc);
    else
      hipLaunchKernelGGL((k_cg_pap<1, false>), grid, blk, 0, c->stream, r, pold, c->beta, c->active, c->diag, c->g, n, N, NV, pts, c->part, c->sc);
  }
  return hipGetLastError();
}

hipError_t launch_cg_update(ope_ctx* c, const double* r, const double* pold, double* rnew, double* pnew,
                            double* y, int first) {
  const uint32_t N = (uint32_t)c->N, NV = N / c->vw, n = (uint32_t)c->n;
  const dim3 grid(c->stream_wgs), blk(OPE_WG);
  const uint32_t pts = (uint32_t)c->stream_pts;
  if (c->vw == 2) {
    if (first)
      hipLaunchKernelGGL((k_cg_update<2, true>), grid, blk, 0, c->stream, r, pold, rnew, pnew, y, c->alpha, c->beta, c->active, c->diag, c->g, n, N, NV, pts, c->part);
    else
      hipLaunchKernelGGL((k_cg_update<2, false>), grid, blk, 0, c->stream, r, pold, rnew, pnew, y, c->alpha, c->beta, c->active, c->diag, c->g, n, N, NV, pts, c->part);
  } else {
    if (first)
      hipLaunchKernelGGL((k_cg_update<1, true>), grid, blk, 0, c->stream, r, pold, rnew, pnew, y, c->alpha, c->beta, c->active, c->diag, c->g, n, N, NV, pts, c->part);
    else
      hipLaunchKernelGGL((k_cg_update<1, false>), grid, blk, 0, c->stream, r, pold, rnew, pnew, y, c->alpha, c->beta, c->active, c->diag, c->g, n, N, NV, pts, c->part);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_cols(ope_ctx* c, const double* part, int64_t nrows, int64_t ncols, double* out, int mode) {
  const uint32_t ncg = (uint32_t)((ncols + 63) / 64);
  // enough rows per work-group to amortise, enough work-groups to spread the read
  uint32_t S = (uint32_t)((nrows + 255) / 256);
  if (S < 1) S = 1;
  if (S > 64) S = 64;
  if ((int64_t)S * ncols > c->stage_cap) S = 1;
  if (ncg > 4096) S = 1;
  const dim3 grid(ncg, S), blk(OPE_WG);
  switch (mode) {
    case RED_PLAIN:
      hipLaunchKernelGGL((k_reduce_cols<RED_PLAIN>), grid, blk, 0, c->stream, part, (uint32_t)nrows, (uint32_t)ncols,
                         out, c->stage, c->counters, c->alpha, c->beta, c->rho, c->target, c->active, c->sc);
      break;
    case RED_CG_ALPHA:
      hipLaunchKernelGGL((k_reduce_cols<RED_CG_ALPHA>), grid, blk, 0, c->stream, part, (uint32_t)nrows, (uint32_t)ncols,
                         out, c->stage, c->counters, c->alpha, c->beta, c->rho, c->target, c->active, c->sc);
      break;
    default:
      hipLaunchKernelGGL((k_reduce_cols<RED_CG_BETA>), grid, blk, 0, c->stream, part, (uint32_t)nrows, (uint32_t)ncols,
                         out, c->stage, c->counters, c->alpha, c->beta, c->rho, c->target, c->active, c->sc);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_resid0(ope_ctx* c, const double* U, const double* HY, double* R, double* y) {
  const uint32_t N = (uint32_t)c->N, NV = N / c->vw, n = (uint32_t)c->n;
  const dim3 grid(c->stream_wgs), blk(OPE_WG);
  const uint32_t pts = (uint32_t)c->stream_pts;
  if (c->vw == 2)
    hipLaunchKernelGGL((k_resid0<2>), grid, blk, 0, c->stream, U, HY, R, y, n, N, NV, pts, c->part);
  else
    hipLaunchKernelGGL((k_resid0<1>), grid, blk, 0, c->stream, U, HY, R, y, n, N, NV, pts, c->part);
  return hipGetLastError();
}
