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

// 16-byte (or narrower) row chunk of VW elements of type T.
template <typename T, int VW>
struct alignas(sizeof(T) * VW) RowVec {
  T v[VW];
};

template <typename T, int VW>
__device__ __forceinline__ void ldv(const T* __restrict__ base, uint64_t off, T (&v)[VW]) {
  const RowVec<T, VW> t = *reinterpret_cast<const RowVec<T, VW>*>(base + off);
#pragma unroll
  for (int k = 0; k < VW; ++k) v[k] = t.v[k];
}

template <typename T, int VW>
__device__ __forceinline__ void stv(T* __restrict__ base, uint64_t off, const T (&v)[VW]) {
  RowVec<T, VW> t;
#pragma unroll
  for (int k = 0; k < VW; ++k) t.v[k] = v[k];
  *reinterpret_cast<RowVec<T, VW>*>(base + off) = t;
}

// Store that is not kept in the caches (the rows are not read again by this sweep).
template <typename T, int VW>
__device__ __forceinline__ void stv_nt(T* __restrict__ base, uint64_t off, const T (&v)[VW]) {
#pragma unroll
  for (int k = 0; k < VW; ++k) __builtin_nontemporal_store(v[k], base + off + k);
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

// Plane-marching stencil sweep (2.5D).  A work-group owns one side line
// (y in 3D), one x segment, one chunk of columns and one range of the march
// axis (z in 3D, y in 2D).  It walks that range plane by plane, keeping the
// field at planes k-1, k, k+1 in registers, so each row is read from HBM once;
// x neighbours come from the current plane staged in LDS, side neighbours from
// the rows the adjacent work-groups of the same XCD stream at the same time
// (L2 hits).  The march is software-pipelined: while plane k is computed, the
// centre rows of plane k+2 and the side rows, diagonal and y of plane k+1 are
// already in flight, so no load latency sits on the per-plane critical path.
// MODE selects what is done with (H p) at each point:
//   SW_APPLY   out = H x
//   SW_PAP     sigma_j += p_j (H p)_j,          p = r + beta p_old
//   SW_UPDATE  y += alpha p, r' = r - alpha H p, p written, rho'_j += r'_j^2
enum { SW_APPLY = 0, SW_PAP = 1, SW_UPDATE = 2 };

template <typename T, int VW, int Q, int MODE, bool FIRST>
__global__ __launch_bounds__(OPE_WG) void k_march(const T* __restrict__ F0, const T* __restrict__ F1,
                                                  T* __restrict__ O0, T* __restrict__ O1,
                                                  T* __restrict__ Yv, const double* __restrict__ alpha,
                                                  const double* __restrict__ beta, const int32_t* __restrict__ active,
                                                  const T* __restrict__ diag, OpeGrid g, MarchShape ms,
                                                  uint32_t N, uint32_t NV, double* __restrict__ part,
                                                  OpeScalars* __restrict__ sc) {
  constexpr bool TWO = (MODE != SW_APPLY) && !FIRST;   // field is r + beta p_old (two loads per value)
  constexpr bool UPD = (MODE == SW_UPDATE);
  __shared__ T lds[2 * Q * OPE_WG * VW];
  __shared__ double red[OPE_WG * VW];
  if (MODE != SW_APPLY) {
    if (!any_active(active, N)) return;
    if (MODE == SW_PAP && blockIdx.x == 0 && threadIdx.x == 0) sc->cg_iters += 1;
  }
  uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t mchunk_id = t % ms.mc;
  t /= ms.mc;
  uint32_t cchunk, xs, line;
  if (ms.order == 0) {           // ((line * nxs + xs) * cc + chunk) * mc + m
    cchunk = t % ms.cc;
    t /= ms.cc;
    xs = t % ms.nxs;
    line = t / ms.nxs;
  } else {                       // ((chunk * lines + line) * nxs + xs) * mc + m
    xs = t % ms.nxs;
    t /= ms.nxs;
    line = t % ms.lines;
    cchunk = t / ms.lines;
  }
  const uint32_t cv = threadIdx.x % ms.ncv, slot = threadIdx.x / ms.ncv;
  const uint32_t colv = cchunk * ms.ncv + cv;
  const bool lane_ok = slot < ms.pp && colv < NV;
  const uint64_t coff = (uint64_t)colv * VW;
  const uint32_t z0 = mchunk_id * ms.mchunk;
  const uint32_t z1 = min(ms.mlen, z0 + ms.mchunk);
  const uint64_t lbase = (uint64_t)line * ms.side_stride;
  const bool side_lo = ms.has_side && line > 0;
  const bool side_hi = ms.has_side && line + 1 < ms.lines;
  const uint64_t sstride = (uint64_t)ms.side_stride * N;

  T b[VW], a[VW];
  double acc[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) {
    b[v] = (TWO && lane_ok) ? (T)beta[coff + v] : T(0);
    a[v] = (UPD && lane_ok) ? (T)alpha[coff + v] : T(0);
    acc[v] = 0.0;
  }
  const T cx = (T)g.cx, cs = (T)ms.cs, cm = (T)ms.cm;
  uint32_t xq[Q];
  bool okq[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint32_t xi = q * ms.pp + slot;
    xq[q] = xs * ms.xseg + xi;
    okq[q] = lane_ok && xi < ms.xseg && xq[q] < g.m0;
  }
  auto off_of = [&](uint32_t x, uint32_t z) -> uint64_t {
    return ((uint64_t)x + lbase + (uint64_t)z * ms.march_stride) * N + coff;
  };
  auto zero = [](T (&o)[VW]) {
#pragma unroll
    for (int v = 0; v < VW; ++v) o[v] = T(0);
  };
  // raw loads of one field value (r and p_old, or x); combined later
  auto ld_raw = [&](bool ok, uint64_t o, T (&r)[VW], T (&po)[VW]) {
    if (ok) {
      ldv<T, VW>(F0, o, r);
      if constexpr (TWO) ldv<T, VW>(F1, o, po);
    } else {
      zero(r);
      if constexpr (TWO) zero(po);
    }
  };
  auto comb = [&](const T (&r)[VW], const T (&po)[VW], T (&out)[VW]) {
#pragma unroll
    for (int v = 0; v < VW; ++v) out[v] = TWO ? r[v] + b[v] * po[v] : r[v];
  };

  // pipeline registers (per pass q)
  T pm[Q][VW], pz[Q][VW], p1[Q][VW];               // field at z-1, z, z+1
  T rz[Q][VW], r1[Q][VW];                           // r at z, z+1 (UPDATE)
  T smz[Q][VW], spz[Q][VW];                         // side neighbours at z
  T dz[Q], yz[Q][VW];                               // diagonal and y at z
  T c2r[Q][VW], c2p[Q][VW];                         // in flight: centre of z+2
  T s1r[Q][VW], s1p[Q][VW], t1r[Q][VW], t1p[Q][VW];  // in flight: side rows of z+1
  T d1[Q], y1[Q][VW];                               // in flight: diagonal, y of z+1

  // prologue: everything for plane z0 and the centre of z0+1
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    T tr[VW], tp[VW];
    const bool ok = okq[q] && z0 < z1;
    ld_raw(ok && z0 > 0, ok && z0 > 0 ? off_of(xq[q], z0 - 1) : 0, tr, tp);
    comb(tr, tp, pm[q]);
    ld_raw(ok, ok ? off_of(xq[q], z0) : 0, tr, tp);
    comb(tr, tp, pz[q]);
#pragma unroll
    for (int v = 0; v < VW; ++v) rz[q][v] = tr[v];
    ld_raw(ok && z0 + 1 < ms.mlen, ok && z0 + 1 < ms.mlen ? off_of(xq[q], z0 + 1) : 0, tr, tp);
    comb(tr, tp, p1[q]);
#pragma unroll
    for (int v = 0; v < VW; ++v) r1[q][v] = tr[v];
    const uint64_t o = ok ? off_of(xq[q], z0) : 0;
    ld_raw(ok && side_lo, o - (side_lo ? sstride : 0), tr, tp);
    comb(tr, tp, smz[q]);
    ld_raw(ok && side_hi, o + (side_hi ? sstride : 0), tr, tp);
    comb(tr, tp, spz[q]);
    dz[q] = ok ? diag[o / N] : T(0);
    if constexpr (UPD) {
      if (ok) ldv<T, VW>(Yv, o, yz[q]);
      else zero(yz[q]);
    }
  }

  for (uint32_t z = z0; z < z1; ++z) {
    // issue the loads of the next iterations
    const bool n2 = z + 2 < ms.mlen && z + 1 < z1;
    const bool n1 = z + 1 < z1;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const bool ok = okq[q];
      ld_raw(ok && n2, ok && n2 ? off_of(xq[q], z + 2) : 0, c2r[q], c2p[q]);
      const uint64_t o1 = (ok && n1) ? off_of(xq[q], z + 1) : 0;
      ld_raw(ok && n1 && side_lo, o1 - (ok && n1 && side_lo ? sstride : 0), s1r[q], s1p[q]);
      ld_raw(ok && n1 && side_hi, o1 + (ok && n1 && side_hi ? sstride : 0), t1r[q], t1p[q]);
      d1[q] = (ok && n1) ? diag[o1 / N] : T(0);
      if constexpr (UPD) {
        if (ok && n1) ldv<T, VW>(Yv, o1, y1[q]);
        else zero(y1[q]);
      }
    }
    // stage plane z for the x neighbours
    T* buf = lds + (z & 1u) * (Q * OPE_WG * VW);
    // lanes past the last whole slot (when ncv does not divide the work-group)
    // hold no point, and their index would alias the next pass's first slot
    if (slot < ms.pp) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int v = 0; v < VW; ++v) buf[((q * ms.pp + slot) * ms.ncv + cv) * VW + v] = pz[q][v];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (!okq[q]) continue;
      const uint32_t x = xq[q];
      const uint32_t xi = q * ms.pp + slot;
      const uint64_t o = off_of(x, z);
      T xm[VW], xp[VW];
      zero(xm);
      zero(xp);
      if (x > 0) {
        if (xi > 0) {
#pragma unroll
          for (int v = 0; v < VW; ++v) xm[v] = buf[((xi - 1) * ms.ncv + cv) * VW + v];
        } else {
          T tr[VW], tp[VW];
          ld_raw(true, o - N, tr, tp);
          comb(tr, tp, xm);
        }
      }
      if (x + 1 < g.m0) {
        if (xi + 1 < ms.xseg) {
#pragma unroll
          for (int v = 0; v < VW; ++v) xp[v] = buf[((xi + 1) * ms.ncv + cv) * VW + v];
        } else {
          T tr[VW], tp[VW];
          ld_raw(true, o + N, tr, tp);
          comb(tr, tp, xp);
        }
      }
      T hx[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v)
        hx[v] = dz[q] * pz[q][v] - (cx * (xm[v] + xp[v]) + cs * (smz[q][v] + spz[q][v]) + cm * (pm[q][v] + p1[q][v]));
      if constexpr (MODE == SW_APPLY) {
        if (ms.nt) stv_nt<T, VW>(O0, o, hx);
        else stv<T, VW>(O0, o, hx);
      } else if constexpr (MODE == SW_PAP) {
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] += (double)pz[q][v] * (double)hx[v];
      } else {
        T yv[VW], rnew[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          yv[v] = yz[q][v] + a[v] * pz[q][v];
          rnew[v] = rz[q][v] - a[v] * hx[v];
          acc[v] += (double)rnew[v] * (double)rnew[v];
        }
        if (ms.nt) {
          stv_nt<T, VW>(Yv, o, yv);
          stv_nt<T, VW>(O0, o, rnew);
          stv_nt<T, VW>(O1, o, pz[q]);
        } else {
          stv<T, VW>(Yv, o, yv);
          stv<T, VW>(O0, o, rnew);
          stv<T, VW>(O1, o, pz[q]);
        }
      }
    }
    // rotate the pipeline
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        pm[q][v] = pz[q][v];
        pz[q][v] = p1[q][v];
        rz[q][v] = r1[q][v];
        r1[q][v] = c2r[q][v];
        if constexpr (UPD) yz[q][v] = y1[q][v];
      }
      comb(c2r[q], c2p[q], p1[q]);
      comb(s1r[q], s1p[q], smz[q]);
      comb(t1r[q], t1p[q], spz[q]);
      dz[q] = d1[q];
    }
  }
  if constexpr (MODE != SW_APPLY) {
    // per-column sums over the work-group's slots -> one partial row per (line, segment, march chunk)
#pragma unroll
    for (int v = 0; v < VW; ++v) red[threadIdx.x * VW + v] = (slot < ms.pp) ? acc[v] : 0.0;
    __syncthreads();
    if (threadIdx.x < ms.ncv && colv < NV) {
      double s[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) s[v] = 0.0;
      for (uint32_t l = 0; l < ms.pp; ++l)
#pragma unroll
        for (int v = 0; v < VW; ++v) s[v] += red[(l * ms.ncv + cv) * VW + v];
      const uint64_t row = ((uint64_t)line * ms.nxs + xs) * ms.mc + mchunk_id;
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const uint64_t col = coff + v;
        if (col < N) part[row * N + col] = s[v];
      }
    }
  }
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
      ldv<double, VW>(U, off, u);
      if (HY) {
        double t[VW];
        ldv<double, VW>(HY, off, t);
#pragma unroll
        for (int v = 0; v < VW; ++v) r[v] = u[v] - t[v];
      } else {
        double z[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          r[v] = u[v];
          z[v] = 0.0;
        }
        stv<double, VW>(y, off, z);
      }
      stv<double, VW>(R, off, r);
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

// CG finalisation of one column from its dot product `tot` (after sweep A:
// alpha; after sweep B: beta, rho and the convergence flag).
template <int MODE>
__device__ __forceinline__ void cg_finalise(uint32_t col, double tot, double* __restrict__ alpha,
                                            double* __restrict__ beta, double* __restrict__ rho,
                                            const double* __restrict__ target, int32_t* __restrict__ active,
                                            OpeScalars* __restrict__ sc) {
  if (MODE == RED_CG_ALPHA) {
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
  if (MODE == RED_PLAIN) out[col] = tot;
  else cg_finalise<MODE>(col, tot, alpha, beta, rho, target, active, sc);
}

// The same column sums for few columns (ncols <= 128) by one work-group with
// no second stage: thread t sums column t % ncols over rows t / ncols,
// t / ncols + G, ... (G = 256 / ncols row groups, eight loads in flight), then
// the groups are added in order.  Avoids the cross-work-group fence of the
// split form, which writes back the L2 lines the preceding sweep left dirty.
template <int MODE>
__global__ __launch_bounds__(OPE_WG) void k_reduce_few(const double* __restrict__ part, uint32_t nrows,
                                                       uint32_t ncols, double* __restrict__ out,
                                                       double* __restrict__ alpha, double* __restrict__ beta,
                                                       double* __restrict__ rho, const double* __restrict__ target,
                                                       int32_t* __restrict__ active, OpeScalars* __restrict__ sc) {
  __shared__ double red[OPE_WG];
  const uint32_t G = OPE_WG / ncols;
  const uint32_t col = threadIdx.x % ncols, gi = threadIdx.x / ncols;
  double a = 0.0;
  if (gi < G) {
    double q[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    uint32_t w = gi;
    for (; w + 7 * G < nrows; w += 8 * G) {
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] += part[(uint64_t)(w + u * G) * ncols + col];
    }
    for (; w < nrows; w += G) q[0] += part[(uint64_t)w * ncols + col];
    a = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
  }
  red[threadIdx.x] = a;
  __syncthreads();
  if (gi != 0) return;
  double tot = 0.0;
  for (uint32_t k = 0; k < G; ++k) tot += red[k * ncols + col];
  if (MODE == RED_PLAIN) out[col] = tot;
  else cg_finalise<MODE>(col, tot, alpha, beta, rho, target, active, sc);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T, int VW, int Q, int MODE, bool FIRST>
static void launch_march_t(ope_ctx* c, const T* F0, const T* F1, T* O0, T* O1, T* Yv, const T* diag) {
  const uint32_t N = (uint32_t)c->N, NV = N / VW;
  const MarchShape& ms = c->ms;
  const uint32_t grid = ms.lines * ms.nxs * ms.cc * ms.mc;
  hipLaunchKernelGGL((k_march<T, VW, Q, MODE, FIRST>), dim3(grid), dim3(OPE_WG), 0, c->stream, F0, F1, O0, O1, Yv,
                     c->alpha, c->beta, c->active, diag, c->g, ms, N, NV, c->part, c->sc);
}

template <typename T, int VW, int MODE, bool FIRST>
static void launch_march_q(ope_ctx* c, const T* F0, const T* F1, T* O0, T* O1, T* Yv, const T* diag) {
  switch (c->ms.q) {
    case 1: launch_march_t<T, VW, 1, MODE, FIRST>(c, F0, F1, O0, O1, Yv, diag); break;
    case 2: launch_march_t<T, VW, 2, MODE, FIRST>(c, F0, F1, O0, O1, Yv, diag); break;
    default: launch_march_t<T, VW, 4, MODE, FIRST>(c, F0, F1, O0, O1, Yv, diag); break;
  }
}

template <int MODE, bool FIRST>
static hipError_t launch_march(ope_ctx* c, const void* F0, const void* F1, void* O0, void* O1, void* Yv) {
  if (c->prec == OPE_FP64) {
    using T = double;
    if (c->vw == 2)
      launch_march_q<T, 2, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag);
    else
      launch_march_q<T, 1, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag);
  } else {
    using T = float;
    if (c->vw == 4)
      launch_march_q<T, 4, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag32);
    else if (c->vw == 2)
      launch_march_q<T, 2, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag32);
    else
      launch_march_q<T, 1, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag32);
  }
  return hipGetLastError();
}

void march_shape(ope_ctx* c, int q_max, int mc_override, int order, int nt, int narrow) {
  MarchShape& ms = c->ms;
  ms.order = order ? 1u : 0u;
  ms.nt = nt ? 1u : 0u;
  const OpeGrid& g = c->g;
  const uint32_t NV = (uint32_t)(c->N / c->vw);
  // Column chunk of a work-group: whole rows when they have at most 32 vector
  // columns (one contiguous run of pp rows per pass, no partly idle chunk),
  // else 8 vector columns (one 128-byte line per grid point and work-group).
  ms.ncv = (NV <= 32u && !narrow) ? NV : (NV < 8u ? NV : 8u);
  ms.pp = OPE_WG / ms.ncv;
  // passes per plane (1, 2 or 4, at most q_max, default 2; a larger one only
  // while the smaller does not cover the x line): the one that leaves the
  // fewest idle lanes in the last x segment, the larger on a tie
  const uint32_t qcap = q_max > 0 ? (uint32_t)q_max : 2u;
  uint32_t q = 1;
  double best = -1.0;
  for (uint32_t qq = 1; qq <= qcap && qq <= 4u; qq *= 2) {
    if (qq > 1 && (qq / 2) * ms.pp >= g.m0) break;
    const uint32_t xs = qq * ms.pp, nx = (g.m0 + xs - 1) / xs;
    const double use = (double)g.m0 / (double)(nx * xs);
    if (use >= best - 1e-12) {
      q = qq;
      best = use > best ? use : best;
    }
  }
  ms.q = q;
  ms.xseg = q * ms.pp;
  ms.nxs = (g.m0 + ms.xseg - 1) / ms.xseg;
  ms.cc = (NV + ms.ncv - 1) / ms.ncv;
  if (g.dim == 3) {
    ms.lines = g.m1;
    ms.mlen = g.m2;
    ms.side_stride = g.m0;
    ms.march_stride = g.m0 * g.m1;
    ms.cm = g.cz;
    ms.cs = g.cy;
    ms.has_side = 1;
  } else {
    ms.lines = 1;
    ms.mlen = g.m1;
    ms.side_stride = 0;
    ms.march_stride = g.m0;
    ms.cm = g.cy;
    ms.cs = 0.0;
    ms.has_side = 0;
  }
  // automatic: one march chunk when that already gives 512 work-groups (the
  // lock-step march keeps side rows in L2), more chunks for smaller grids
  const uint32_t base = ms.lines * ms.nxs * ms.cc;
  uint32_t mc = mc_override > 0 ? (uint32_t)mc_override : (512u + base - 1) / base;
  if (mc < 1) mc = 1;
  if (mc > ms.mlen) mc = ms.mlen;
  ms.mchunk = (ms.mlen + mc - 1) / mc;
  ms.mc = (ms.mlen + ms.mchunk - 1) / ms.mchunk;
}

int64_t march_rows(const ope_ctx* c) {
  return (int64_t)c->ms.lines * c->ms.nxs * c->ms.mc;
}

hipError_t launch_apply_h(ope_ctx* c, const void* X, void* Yo) {
  ProfScope ps(c, OPE_KERNEL_STENCIL);
  return launch_march<SW_APPLY, false>(c, X, nullptr, Yo, nullptr, nullptr);
}

hipError_t launch_cg_pap(ope_ctx* c, const void* r, const void* pold, int first) {
  ProfScope ps(c, OPE_KERNEL_CG_SWEEP_A);
  if (first) return launch_march<SW_PAP, true>(c, r, pold, nullptr, nullptr, nullptr);
  return launch_march<SW_PAP, false>(c, r, pold, nullptr, nullptr, nullptr);
}

hipError_t launch_cg_update(ope_ctx* c, const void* r, const void* pold, void* rnew, void* pnew,
                            void* y, int first) {
  ProfScope ps(c, OPE_KERNEL_CG_SWEEP_B);
  if (first) return launch_march<SW_UPDATE, true>(c, r, pold, rnew, pnew, y);
  return launch_march<SW_UPDATE, false>(c, r, pold, rnew, pnew, y);
}

hipError_t launch_reduce_cols(ope_ctx* c, const double* part, int64_t nrows, int64_t ncols, double* out, int mode) {
  if (ncols <= 128 && nrows * ncols <= (int64_t)1 << 17) {
    const uint32_t nr = (uint32_t)nrows, nc = (uint32_t)ncols;
    switch (mode) {
      case RED_PLAIN:
        hipLaunchKernelGGL((k_reduce_few<RED_PLAIN>), dim3(1), dim3(OPE_WG), 0, c->stream, part, nr, nc, out, c->alpha,
                           c->beta, c->rho, c->target, c->active, c->sc);
        break;
      case RED_CG_ALPHA:
        hipLaunchKernelGGL((k_reduce_few<RED_CG_ALPHA>), dim3(1), dim3(OPE_WG), 0, c->stream, part, nr, nc, out,
                           c->alpha, c->beta, c->rho, c->target, c->active, c->sc);
        break;
      default:
        hipLaunchKernelGGL((k_reduce_few<RED_CG_BETA>), dim3(1), dim3(OPE_WG), 0, c->stream, part, nr, nc, out,
                           c->alpha, c->beta, c->rho, c->target, c->active, c->sc);
        break;
    }
    return hipGetLastError();
  }
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
