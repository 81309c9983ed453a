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
// k >= 1 with at most 64 nodes is solved exactly with a dense inverse
// (Cholesky on the host).  Transfers per coarsened axis: prolongation
// 3/4 e_I + 1/4 e_J (J = I - 1 for even fine nodes, I + 1 for odd ones,
// missing J = 0), restriction R = P^T / 2^d.  V-cycle, damped Jacobi
// (omega = 0.8) once on each side of the coarse correction:
//   x0 = omega b / d;  r1 = b - H x0;  e = B_{k+1}(R r1);  x1 = x0 + P e;
//   z = x1 + omega (b - H x1) / d.
// Kernels, per level: k_mg_tstencil<0> (r1, one stencil over x0 formed on the
// fly from b), k_mg_zrestrict (R r1), k_mg_dense (coarsest), k_mg_zprolong
// (x1 = x0 + P e), k_mg_tstencil<1> (z, one stencil over x1; on level 0 also
// the per-column partial sums of r^T z and r^T r that the PCG needs).  The
// stencil and transfer kernels march along z (see zmarch_shape, tshape); the
// smoother's factors omega / d are precomputed per level.
// Layout: every block is n x N row-major (a grid point's N values
// contiguous), x fastest, as everywhere in the library; a thread owns one
// 16-byte chunk (VW elements) or one element of a point's row, FP64, or
// FP32 for mixed-precision contexts (dot products accumulated in FP64).  Columns
// whose CG has converged are skipped.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "ope_internal.h"

namespace {

constexpr double MG_OMEGA = 0.8;
constexpr int64_t MG_COARSEST_MAX = 64;
constexpr uint32_t MG_WG = 256;

struct MgGeom {
  uint32_t m0, m1, m2;
  double cx, cy, cz;
};

// VW consecutive elements of a point's row (16 bytes or less), loaded and
// stored as one access.
template <typename T, int VW>
struct alignas(sizeof(T) * VW) Chunk {
  T v[VW];
};

template <typename T, int VW>
__device__ __forceinline__ void ldr(const T* __restrict__ a, uint64_t row, uint32_t N, uint32_t v, T (&o)[VW]) {
  const Chunk<T, VW> t = *reinterpret_cast<const Chunk<T, VW>*>(a + row * N + (uint64_t)VW * v);
#pragma unroll
  for (int k = 0; k < VW; ++k) o[k] = t.v[k];
}

template <typename T, int VW>
__device__ __forceinline__ void str(T* __restrict__ a, uint64_t row, uint32_t N, uint32_t v, const T (&o)[VW]) {
  Chunk<T, VW> t;
#pragma unroll
  for (int k = 0; k < VW; ++k) t.v[k] = o[k];
  *reinterpret_cast<Chunk<T, VW>*>(a + row * N + (uint64_t)VW * v) = t;
}

template <typename T, int VW>
__device__ __forceinline__ void zero(T (&a)[VW]) {
#pragma unroll
  for (int k = 0; k < VW; ++k) a[k] = T(0);
}

template <int VW>
__device__ __forceinline__ bool vec_active(const int32_t* __restrict__ active, uint32_t v) {
  if (!active) return true;
  bool a = false;
#pragma unroll
  for (int k = 0; k < VW; ++k) a |= active[v * VW + k] != 0;
  return a;
}

// x0 = (omega / d) b at point q, with wd = omega / d (zero outside the grid is
// the caller's job)
template <typename T, int VW>
__device__ __forceinline__ void jac0(const T* __restrict__ b, const double* __restrict__ wd, uint64_t q, uint32_t N,
                                     uint32_t v, T (&o)[VW]) {
  ldr<T, VW>(b, q, N, v, o);
  const T w = (T)wd[q];
#pragma unroll
  for (int k = 0; k < VW; ++k) o[k] = w * o[k];
}

// Fine nodes and weights of coarse node I along one axis: always four taps
// (2I - 1, 2I, 2I + 1, 2I + 2 with weights 1/8, 3/8, 3/8, 1/8, the factor 1/2
// of R = P^T / 2^d included), a missing node clamped into the grid with weight
// zero; an axis that is not coarsened has the one tap I with weight 1.  The
// fixed count lets every load of a gather be issued before the first is used.
__device__ __forceinline__ void restrict_taps(uint32_t I, uint32_t mf, uint32_t (&f)[4], double (&w)[4]) {
  if (mf == 1) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f[t] = I;
      w[t] = t == 1 ? 1.0 : 0.0;
    }
    return;
  }
  const double cw[4] = {0.125, 0.375, 0.375, 0.125};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t c = 2 * (int64_t)I - 1 + t;
    const bool in = c >= 0 && c < (int64_t)mf;
    f[t] = in ? (uint32_t)c : (uint32_t)(2 * I);
    w[t] = in ? cw[t] : 0.0;
  }
}

// coarsest level: E = A^{-1} B with the dense inverse (row-major nc x nc)
template <typename T, int VW>
__global__ __launch_bounds__(MG_WG) void k_mg_dense(const double* __restrict__ Ainv, const T* __restrict__ B,
                                                   T* __restrict__ E, uint32_t nc,
                                                   const int32_t* __restrict__ active, uint32_t N, uint32_t NV,
                                                   uint64_t total) {
  const uint64_t e = (uint64_t)blockIdx.x * MG_WG + threadIdx.x;
  if (e >= total) return;
  const uint32_t v = (uint32_t)(e % NV);
  const uint32_t i = (uint32_t)(e / NV);
  if (!vec_active<VW>(active, v)) return;
  T acc[VW];
#pragma unroll
  for (int k = 0; k < VW; ++k) acc[k] = 0.0;
  const double* a = Ainv + (uint64_t)i * nc;
  // four running sums over j = 4 u + s (their loads are issued together), added in order
  T part[4][VW];
#pragma unroll
  for (int s = 0; s < 4; ++s) zero(part[s]);
  uint32_t j = 0;
  for (; j + 4 <= nc; j += 4) {
    T t[4][VW];
#pragma unroll
    for (int s = 0; s < 4; ++s) ldr<T, VW>(B, j + s, N, v, t[s]);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const T w = (T)a[j + s];
#pragma unroll
      for (int k = 0; k < VW; ++k) part[s][k] += w * t[s][k];
    }
  }
  for (; j < nc; ++j) {
    T t[VW];
    ldr<T, VW>(B, j, N, v, t);
    const T w = (T)a[j];
#pragma unroll
    for (int k = 0; k < VW; ++k) part[0][k] += w * t[k];
  }
#pragma unroll
  for (int k = 0; k < VW; ++k) acc[k] = (part[0][k] + part[1][k]) + (part[2][k] + part[3][k]);
  str<T, VW>(E, i, N, v, acc);
}

// z-march decomposition of a level: a work-group owns PL = 256 / NV
// consecutive x nodes (thread t: vector t % NV of node t / NV) of one y row
// over ZC consecutive z planes, keeping the field of the planes below, at and
// above the current one in registers; work-groups are numbered x segment
// fastest, then y, then z range, and spread XCD-contiguously, so one XCD
// streams neighbouring rows of the same planes (their y neighbours hit L2).
struct ZMarch {
  uint32_t PL, nxs, nzc, ZC;
};

ZMarch zmarch_shape(uint32_t m0, uint32_t m1, uint32_t m2, uint32_t NV) {
  ZMarch s;
  s.PL = MG_WG / NV;
  s.nxs = (m0 + s.PL - 1) / s.PL;
  const uint64_t cols = (uint64_t)s.nxs * m1;
  uint64_t nzc = (2048 + cols - 1) / cols;          // at least 2048 work-groups when the grid allows
  if (nzc > m2) nzc = m2;
  if (nzc < 1) nzc = 1;
  s.ZC = (uint32_t)((m2 + nzc - 1) / nzc);
  s.nzc = (m2 + s.ZC - 1) / s.ZC;
  return s;
}

struct ZPos {
  uint32_t x, y, z0, z1, v;
  bool ok;
};

template <int VW>
__device__ __forceinline__ ZPos zpos(const MgGeom& g, const ZMarch& zs, const int32_t* __restrict__ active,
                                     uint32_t NV) {
  ZPos q;
  const uint32_t L = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t xs = L % zs.nxs, r = L / zs.nxs;
  q.y = r % g.m1;
  const uint32_t zc = r / g.m1;
  const uint32_t t = threadIdx.x;
  const bool lane_ok = t < zs.PL * NV;
  q.v = lane_ok ? t % NV : 0;
  q.x = xs * zs.PL + (lane_ok ? t / NV : 0);
  q.z0 = zc * zs.ZC;
  q.z1 = q.z0 + zs.ZC < g.m2 ? q.z0 + zs.ZC : g.m2;
  q.ok = lane_ok && q.x < g.m0 && vec_active<VW>(active, q.v);
  return q;
}

// x-y tiled form of the stencil sweeps: a work-group of TX TY NVS threads
// owns a TX x TY tile of grid columns over ZC planes, for one slice of NVS
// consecutive vector groups (of the NV = N / VW of a row; thread t: group
// t % NVS of the slice, column t / NVS).  At each plane the tile's field
// values and those of the one-column ring around it go to LDS, so the x and y
// neighbours come from LDS (each ring value is loaded once per work-group
// instead of by every neighbouring thread), and the z neighbours stay in
// registers.  Slicing the row lets the tile grow (the ring costs 2(TX + TY) + 4
// extra columns per TX TY) within the same threads and LDS.
struct TShape {
  uint32_t TX, TY, nxt, nyt, nzc, ZC, NS, NVS;
};

constexpr uint32_t MG_TWG = 1024;                 // threads of a tiled work-group (at most)
constexpr uint32_t MG_TLDS_BYTES = 36864;         // LDS of one plane's tile and ring

// Slices of a row: as many as keep a slice at least 8 vector groups wide (a
// 128-byte run of FP64 pairs), dividing NV.
uint32_t tslices(uint32_t NV) {
  uint32_t ns = 1;
  while (NV % (2 * ns) == 0 && NV / (2 * ns) >= 8) ns *= 2;
  return ns;
}

TShape tshape(uint32_t m0, uint32_t m1, uint32_t m2, uint32_t NV, uint32_t N, uint32_t esz) {
  TShape s;
  s.NS = tslices(NV);
  s.NVS = NV / s.NS;
  // columns per work-group: as many as MG_TWG threads hold (measured at 64^3,
  // N = 128: 1024 threads on 16 x 8 tiles beat 512 on 8 x 8 and 256 on 8 x 4,
  // whose rings cost more than the extra work-groups per compute unit gain)
  const uint32_t P = std::max(1u, MG_TWG / s.NVS);
  const uint64_t rowb = (uint64_t)(N / s.NS) * esz;      // LDS bytes of one column's slice
  uint32_t tx = 1;
  while ((tx * 2) * (tx * 2) <= P) tx *= 2;       // a square tile of powers of two, x side first
  if (tx * tx * 2 <= P) tx *= 2;
  s.TX = std::min(tx, m0);
  s.TY = std::max(1u, std::min(P / s.TX, m1));
  // fit the tile and its ring in the LDS array (a 1 x 1 tile always fits:
  // 9 columns of at most 4 KB)
  while ((uint64_t)(s.TX + 2) * (s.TY + 2) * rowb > MG_TLDS_BYTES && s.TX * s.TY > 1) {
    if (s.TY > 1) --s.TY;
    else --s.TX;
  }
  s.nxt = (m0 + s.TX - 1) / s.TX;
  s.nyt = (m1 + s.TY - 1) / s.TY;
  const uint64_t tiles = (uint64_t)s.nxt * s.nyt * s.NS;
  uint64_t nzc = (512 + tiles - 1) / tiles;       // at least 512 work-groups when the grid allows
  if (nzc > m2) nzc = m2;
  if (nzc < 1) nzc = 1;
  s.ZC = (uint32_t)((m2 + nzc - 1) / nzc);
  s.nzc = (m2 + s.ZC - 1) / s.ZC;
  return s;
}

// Ring columns per thread of a tiled sweep: ceil(2 (TX + TY) / (TX TY)) <= 4,
// as 1, 2 or 4.
int ring_per_thread(const TShape& ts) {
  const uint32_t P = ts.TX * ts.TY, need = (2 * (ts.TX + ts.TY) + P - 1) / P;
  return need <= 1 ? 1 : need <= 2 ? 2 : 4;
}

// Work-group L of a tiled sweep: tile (xt, yt), z chunk zc, slice sl; `row` is
// its partial-sum row (the tile and chunk; the slices of one tile share it).
struct TPos {
  uint32_t xt, yt, zc, sl, row;
};

__device__ __forceinline__ TPos tpos(const TShape& ts, uint32_t L) {
  TPos q;
  q.xt = L % ts.nxt;
  uint32_t r = L / ts.nxt;
  q.yt = r % ts.nyt;
  r /= ts.nyt;
  q.zc = r % ts.nzc;
  q.sl = r / ts.nzc;
  q.row = (q.zc * ts.nyt + q.yt) * ts.nxt + q.xt;
  return q;
}

// Ring column j of a tiled work-group (k = pt + j P, k < 2 (TX + TY): bottom
// row, top row, left column, right column): its grid x-y index (when inside
// the grid) and its LDS slot.
struct RingCol {
  uint64_t col;
  uint32_t slot;
  bool ok, in;
};

__device__ __forceinline__ RingCol ring_col(const MgGeom& g, const TShape& ts, uint32_t x0, uint32_t y0, uint32_t k,
                                            uint32_t NVS, uint32_t vl, uint32_t VW, bool act) {
  RingCol rc;
  const uint32_t RING = 2 * (ts.TX + ts.TY), W = ts.TX + 2;
  rc.ok = k < RING;
  rc.in = false;
  rc.col = 0;
  rc.slot = 0;
  if (!rc.ok) return rc;
  int64_t hx, hy;
  uint32_t cx, cy;
  if (k < ts.TX) {
    hx = (int64_t)x0 + k; hy = (int64_t)y0 - 1; cx = k + 1; cy = 0;
  } else if (k < 2 * ts.TX) {
    hx = (int64_t)x0 + (k - ts.TX); hy = (int64_t)y0 + ts.TY; cx = k - ts.TX + 1; cy = ts.TY + 1;
  } else if (k < 2 * ts.TX + ts.TY) {
    hx = (int64_t)x0 - 1; hy = (int64_t)y0 + (k - 2 * ts.TX); cx = 0; cy = k - 2 * ts.TX + 1;
  } else {
    hx = (int64_t)x0 + ts.TX; hy = (int64_t)y0 + (k - 2 * ts.TX - ts.TY); cx = ts.TX + 1;
    cy = k - 2 * ts.TX - ts.TY + 1;
  }
  rc.slot = ((cy * W + cx) * NVS + vl) * VW;
  rc.in = act && hx >= 0 && hx < (int64_t)g.m0 && hy >= 0 && hy < (int64_t)g.m1;
  if (rc.in) rc.col = (uint64_t)hy * g.m0 + (uint64_t)hx;
  return rc;
}

// Pre-smoothing residual r1 = b - H x0 with x0 = omega b / d formed on the fly,
// as an x-y tiled sweep (see TShape).  The loads are issued one plane ahead
// (the ring's b and omega/d of the next plane, the own column's two planes
// ahead), so a plane's wait finds them arrived; the two tile buffers
// alternate, one barrier per plane.
template <typename T, int VW, int R>
__global__ __launch_bounds__(MG_TWG) void k_mg_tstencil(const T* __restrict__ b, T* __restrict__ out, MgGeom g,
                                                       const double* __restrict__ diag, const double* __restrict__ wd,
                                                       const int32_t* __restrict__ active, uint32_t N, TShape ts) {
  __shared__ __align__(16) T tiles[2][MG_TLDS_BYTES / sizeof(T)];
  const uint32_t t = threadIdx.x;
  const uint32_t NVS = ts.NVS;
  const uint32_t vl = t % NVS, pt = t / NVS;
  const uint32_t tx = pt % ts.TX, ty = pt / ts.TX;
  const TPos wp = tpos(ts, xcd_remap(blockIdx.x, gridDim.x));
  const uint32_t v = wp.sl * NVS + vl;
  const uint32_t x0 = wp.xt * ts.TX, y0 = wp.yt * ts.TY;
  const uint32_t x = x0 + tx, y = y0 + ty;
  const bool inb = x < g.m0 && y < g.m1;
  const bool act = vec_active<VW>(active, v);
  if (!__syncthreads_or(act ? 1 : 0)) return;     // every column of the slice has stopped
  const bool own = inb && act;
  const uint32_t z0 = wp.zc * ts.ZC, z1 = z0 + ts.ZC < g.m2 ? z0 + ts.ZC : g.m2;
  const uint64_t s2 = (uint64_t)g.m0 * g.m1;
  const uint32_t W = ts.TX + 2, P = ts.TX * ts.TY;
  auto slot = [&](uint32_t cx, uint32_t cy) -> uint32_t { return ((cy * W + cx) * NVS + vl) * VW; };
  RingCol rc[R];
  T rb[R][VW], rw[R];
#pragma unroll
  for (int j = 0; j < R; ++j) rc[j] = ring_col(g, ts, x0, y0, pt + (uint32_t)j * P, NVS, vl, VW, act);
  auto ring_load = [&](uint32_t z) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      zero(rb[j]);
      rw[j] = T(0);
      if (rc[j].in) {
        const uint64_t q = (uint64_t)z * s2 + rc[j].col;
        ldr<T, VW>(b, q, N, v, rb[j]);
        rw[j] = (T)wd[q];
      }
    }
  };
  // own column: x0 at z - 1 and z, b and d at z, the raw b and omega/d of z + 1
  T fm[VW], fc[VW], bc[VW], bn[VW];
  T wn = T(0), dc = T(0);
  zero(fm);
  zero(fc);
  zero(bc);
  zero(bn);
  uint64_t p = ((uint64_t)z0 * g.m1 + (inb ? y : 0)) * g.m0 + (inb ? x : 0);
  if (own) {
    if (z0 > 0) jac0<T, VW>(b, wd, p - s2, N, v, fm);
    ldr<T, VW>(b, p, N, v, bc);
    const T w0 = (T)wd[p];
#pragma unroll
    for (int k = 0; k < VW; ++k) fc[k] = w0 * bc[k];
    dc = (T)diag[p];
    if (z0 + 1 < g.m2) {
      ldr<T, VW>(b, p + s2, N, v, bn);
      wn = (T)wd[p + s2];
    }
  }
  ring_load(z0);
  for (uint32_t z = z0; z < z1; ++z, p += s2) {
    T* tile = tiles[z & 1];
#pragma unroll
    for (int k = 0; k < VW; ++k) tile[slot(tx + 1, ty + 1) + k] = fc[k];
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (rc[j].ok) {
#pragma unroll
        for (int k = 0; k < VW; ++k) tile[rc[j].slot + k] = rw[j] * rb[j][k];
      }
    // the next plane's ring and the own column two planes ahead
    if (z + 1 < z1) ring_load(z + 1);
    T fp[VW], b2[VW];
    T w2 = T(0), d2 = T(0);
#pragma unroll
    for (int k = 0; k < VW; ++k) fp[k] = wn * bn[k];
    zero(b2);
    if (own && z + 1 < z1) {
      if (z + 2 < g.m2) {
        ldr<T, VW>(b, p + 2 * s2, N, v, b2);
        w2 = (T)wd[p + 2 * s2];
      }
      d2 = (T)diag[p + s2];
    }
    __syncthreads();
    if (own) {
      T o[VW];
      const uint32_t sxm = slot(tx, ty + 1), sxp = slot(tx + 2, ty + 1), sym = slot(tx + 1, ty),
                     syp = slot(tx + 1, ty + 2);
#pragma unroll
      for (int k = 0; k < VW; ++k) {
        const T hxv = dc * fc[k] - ((T)g.cx * (tile[sxm + k] + tile[sxp + k]) +
                                    (T)g.cy * (tile[sym + k] + tile[syp + k]) + (T)g.cz * (fm[k] + fp[k]));
        o[k] = bc[k] - hxv;
      }
      str<T, VW>(out, p, N, v, o);
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      fm[k] = fc[k];
      fc[k] = fp[k];
      bc[k] = bn[k];
      bn[k] = b2[k];
    }
    wn = w2;
    dc = d2;
  }
}

// Coarse nodes and weights of fine node f along one axis: always two taps,
// the parent f / 2 with 3/4 and the other neighbour (f / 2 - 1 for even f,
// f / 2 + 1 for odd f) with 1/4, or weight zero (clamped to the parent) when
// it is missing; an axis that is not coarsened has the tap f with weight 1.
__device__ __forceinline__ void prolong_taps(uint32_t f, uint32_t mf, uint32_t mc, uint32_t (&I)[2], double (&w)[2]) {
  if (mf == 1) {
    I[0] = I[1] = f;
    w[0] = 1.0;
    w[1] = 0.0;
    return;
  }
  I[0] = f / 2;
  w[0] = 0.75;
  const int64_t J = (f % 2 == 0) ? (int64_t)(f / 2) - 1 : (int64_t)(f / 2) + 1;
  const bool in = J >= 0 && J < (int64_t)mc;
  I[1] = in ? (uint32_t)J : f / 2;
  w[1] = in ? 0.25 : 0.0;
}


// Coarse x-y interpolation of coarse plane K at a fine column (fixed taps).
template <typename T, int VW>
__device__ __forceinline__ void coarse_xy(const T* __restrict__ E, const MgGeom& cg, const uint32_t (&Ix)[2],
                                          const double (&wx)[2], const uint32_t (&Iy)[2], const double (&wy)[2],
                                          uint32_t K, uint32_t N, uint32_t v, T (&o)[VW]) {
  zero(o);
#pragma unroll
  for (int bb = 0; bb < 2; ++bb) {
    T ax[VW];
    zero(ax);
    const uint64_t row = ((uint64_t)K * cg.m1 + Iy[bb]) * cg.m0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      T t[VW];
      ldr<T, VW>(E, row + Ix[a], N, v, t);
#pragma unroll
      for (int k = 0; k < VW; ++k) ax[k] += (T)wx[a] * t[k];
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) o[k] += (T)wy[bb] * ax[k];
  }
}

// The prolongation P e along one fine column, marched plane by plane: the
// x-y interpolations of the coarse planes K0 - 1, K0, K0 + 1 around the
// current plane's parent K0 stay in registers (each coarse plane read once).
template <typename T, int VW>
struct PeMarch {
  uint32_t Ix[2], Iy[2];
  double wx[2], wy[2];
  T lo[VW], mid[VW], hi[VW];
  uint32_t K0;
  bool flat;                                      // no z axis: the one coarse plane 0

  __device__ __forceinline__ void init(const T* __restrict__ E, const MgGeom& fg, const MgGeom& cg,
                                       uint32_t fx, uint32_t fy, uint32_t z, uint32_t N, uint32_t v) {
    prolong_taps(fx, fg.m0, cg.m0, Ix, wx);
    prolong_taps(fy, fg.m1, cg.m1, Iy, wy);
    flat = fg.m2 == 1;
    zero(lo);
    zero(hi);
    K0 = flat ? 0 : z / 2;
    coarse_xy<T, VW>(E, cg, Ix, wx, Iy, wy, K0, N, v, mid);
    if (!flat) {
      if (K0 >= 1) coarse_xy<T, VW>(E, cg, Ix, wx, Iy, wy, K0 - 1, N, v, lo);
      if (K0 + 1 < cg.m2) coarse_xy<T, VW>(E, cg, Ix, wx, Iy, wy, K0 + 1, N, v, hi);
    }
  }
  // move to plane z (the plane after the current one)
  __device__ __forceinline__ void step(const T* __restrict__ E, const MgGeom& cg, uint32_t z, uint32_t N,
                                       uint32_t v) {
    if (flat || z % 2 != 0) return;
    K0 = z / 2;
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      lo[k] = mid[k];
      mid[k] = hi[k];
    }
    zero(hi);
    if (K0 + 1 < cg.m2) coarse_xy<T, VW>(E, cg, Ix, wx, Iy, wy, K0 + 1, N, v, hi);
  }
  __device__ __forceinline__ void value(uint32_t z, T (&pe)[VW]) const {
#pragma unroll
    for (int k = 0; k < VW; ++k) pe[k] = flat ? mid[k] : T(0.75) * mid[k] + T(0.25) * (z % 2 == 0 ? lo[k] : hi[k]);
  }
};

// Prolongation and post-smoothing in one x-y tiled sweep (as k_mg_tstencil):
// x1 = omega b / d + P e is formed on the fly for the tile's columns and its
// ring, then z = x1 + omega (b - H x1) / d; with DOTS also the per-column
// sums of b z and b b (row blockIdx.x of part).  The ring columns are spread
// over the threads (at most two per thread), each with its own P e march.
template <typename T, int VW, bool DOTS, int R>
__global__ __launch_bounds__(MG_TWG) void k_mg_tpost(const T* __restrict__ b, const T* __restrict__ E,
                                                    T* __restrict__ out, MgGeom g, MgGeom cg,
                                                    const double* __restrict__ diag, const double* __restrict__ wd,
                                                    const int32_t* __restrict__ active, uint32_t N, TShape ts,
                                                    double* __restrict__ part) {
  // two tile buffers (planes alternate), so one barrier per plane suffices
  __shared__ __align__(16) T tiles[2][MG_TLDS_BYTES / sizeof(T)];
  const uint32_t t = threadIdx.x;
  const uint32_t NVS = ts.NVS;
  const uint32_t vl = t % NVS, pt = t / NVS;
  const uint32_t tx = pt % ts.TX, ty = pt / ts.TX;
  const TPos wp = tpos(ts, xcd_remap(blockIdx.x, gridDim.x));
  const uint32_t v = wp.sl * NVS + vl, zc = wp.zc;
  const uint32_t x0 = wp.xt * ts.TX, y0 = wp.yt * ts.TY;
  const uint32_t x = x0 + tx, y = y0 + ty;
  const bool inb = x < g.m0 && y < g.m1;
  const bool act = vec_active<VW>(active, v);
  if (!__syncthreads_or(act ? 1 : 0)) {          // every column of the slice has stopped
    if constexpr (DOTS) {
      const uint32_t SC = ts.NVS * VW, c0 = wp.sl * SC;
      for (uint32_t c = t; c < SC; c += blockDim.x) {
        part[(uint64_t)wp.row * 2 * N + c0 + c] = 0.0;
        part[(uint64_t)wp.row * 2 * N + N + c0 + c] = 0.0;
      }
    }
    return;
  }
  const bool own = inb && act;
  const uint32_t z0 = zc * ts.ZC, z1 = z0 + ts.ZC < g.m2 ? z0 + ts.ZC : g.m2;
  const uint64_t s2 = (uint64_t)g.m0 * g.m1;
  const uint32_t W = ts.TX + 2, RING = 2 * (ts.TX + ts.TY), P = ts.TX * ts.TY;
  auto slot = [&](uint32_t cx, uint32_t cy) -> uint32_t { return ((cy * W + cx) * NVS + vl) * VW; };
  // x1 at fine point `at` with the column's P e value pe
  auto x1 = [&](uint64_t at, const T(&pe)[VW], T(&f)[VW]) {
    jac0<T, VW>(b, wd, at, N, v, f);
#pragma unroll
    for (int k = 0; k < VW; ++k) f[k] = f[k] + pe[k];
  };
  // ring columns of this thread: k = pt + j P, j < R (R P at least the ring's
  // 2 (TX + TY) columns)
  uint32_t rk[R], rcx[R], rcy[R];
  int64_t rhx[R], rhy[R];
  bool rin[R];
  PeMarch<T, VW> rm[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const uint32_t k = pt + j * P;
    rk[j] = k;
    rin[j] = false;
    if (k >= RING) continue;
    if (k < ts.TX) {
      rhx[j] = (int64_t)x0 + k; rhy[j] = (int64_t)y0 - 1; rcx[j] = k + 1; rcy[j] = 0;
    } else if (k < 2 * ts.TX) {
      rhx[j] = (int64_t)x0 + (k - ts.TX); rhy[j] = (int64_t)y0 + ts.TY; rcx[j] = k - ts.TX + 1; rcy[j] = ts.TY + 1;
    } else if (k < 2 * ts.TX + ts.TY) {
      rhx[j] = (int64_t)x0 - 1; rhy[j] = (int64_t)y0 + (k - 2 * ts.TX); rcx[j] = 0; rcy[j] = k - 2 * ts.TX + 1;
    } else {
      rhx[j] = (int64_t)x0 + ts.TX; rhy[j] = (int64_t)y0 + (k - 2 * ts.TX - ts.TY); rcx[j] = ts.TX + 1;
      rcy[j] = k - 2 * ts.TX - ts.TY + 1;
    }
    rin[j] = act && rhx[j] >= 0 && rhx[j] < (int64_t)g.m0 && rhy[j] >= 0 && rhy[j] < (int64_t)g.m1;
    if (rin[j]) rm[j].init(E, g, cg, (uint32_t)rhx[j], (uint32_t)rhy[j], z0, N, v);
  }
  // own column: the march starts one plane below z0 when there is one
  PeMarch<T, VW> om;
  T fm[VW], fc[VW], fp[VW], pe[VW];
  zero(fm);
  zero(fc);
  uint64_t p = ((uint64_t)z0 * g.m1 + (inb ? y : 0)) * g.m0 + (inb ? x : 0);
  if (own) {
    if (z0 > 0) {
      om.init(E, g, cg, x, y, z0 - 1, N, v);
      om.value(z0 - 1, pe);
      x1(p - s2, pe, fm);
      om.step(E, cg, z0, N, v);
    } else {
      om.init(E, g, cg, x, y, z0, N, v);
    }
    om.value(z0, pe);
    x1(p, pe, fc);
  }
  double srz[VW], srr[VW];
  zero(srz);
  zero(srr);
  for (uint32_t z = z0; z < z1; ++z, p += s2) {
    T* tile = tiles[z & 1];
#pragma unroll
    for (int k = 0; k < VW; ++k) tile[slot(tx + 1, ty + 1) + k] = fc[k];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (rk[j] >= RING) continue;
      T hv[VW];
      zero(hv);
      if (rin[j]) {
        T rp[VW];
        rm[j].value(z, rp);
        x1(((uint64_t)z * g.m1 + (uint64_t)rhy[j]) * g.m0 + (uint64_t)rhx[j], rp, hv);
        if (z + 1 < z1) rm[j].step(E, cg, z + 1, N, v);
      }
#pragma unroll
      for (int kk = 0; kk < VW; ++kk) tile[slot(rcx[j], rcy[j]) + kk] = hv[kk];
    }
    zero(fp);
    T bc[VW];
    zero(bc);
    T d = T(0), w = T(0);
    if (own) {
      if (z + 1 < g.m2) {
        om.step(E, cg, z + 1, N, v);
        om.value(z + 1, pe);
        x1(p + s2, pe, fp);
      }
      ldr<T, VW>(b, p, N, v, bc);
      d = (T)diag[p];
      w = (T)wd[p];
    }
    __syncthreads();
    if (own) {
      T o[VW];
      const uint32_t sxm = slot(tx, ty + 1), sxp = slot(tx + 2, ty + 1), sym = slot(tx + 1, ty),
                     syp = slot(tx + 1, ty + 2);
#pragma unroll
      for (int k = 0; k < VW; ++k) {
        const T hxv = d * fc[k] - ((T)g.cx * (tile[sxm + k] + tile[sxp + k]) +
                                   (T)g.cy * (tile[sym + k] + tile[syp + k]) + (T)g.cz * (fm[k] + fp[k]));
        o[k] = fc[k] + w * (bc[k] - hxv);
      }
      str<T, VW>(out, p, N, v, o);
      if constexpr (DOTS) {
#pragma unroll
        for (int k = 0; k < VW; ++k) {
          srz[k] += (double)bc[k] * (double)o[k];
          srr[k] += (double)bc[k] * (double)bc[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      fm[k] = fc[k];
      fc[k] = fp[k];
    }
  }
  if constexpr (DOTS) {
    // per-column sums over the tile's columns in order, b z then b b (LDS
    // reused, one quantity at a time)
    double* red = reinterpret_cast<double*>(&tiles[0][0]);
    const uint32_t SC = NVS * VW, c0 = wp.sl * SC;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      __syncthreads();            // the last plane's (or the previous pass's) reads are done
#pragma unroll
      for (int k = 0; k < VW; ++k) red[t * VW + k] = q == 0 ? srz[k] : srr[k];
      __syncthreads();
      for (uint32_t c = t; c < SC; c += blockDim.x) {
        const uint32_t cv = c / VW, ck = c % VW;
        double a = 0.0;
        for (uint32_t l = 0; l < P; ++l) a += red[(l * NVS + cv) * VW + ck];
        part[(uint64_t)wp.row * 2 * N + (uint64_t)q * N + c0 + c] = a;
      }
    }
  }
}

// coarse B = R T, z-marched over the coarse planes of a coarse (I, J) column:
// the x-y restriction of each fine plane is formed once and added to the two
// coarse planes it feeds.
template <typename T, int VW>
__global__ __launch_bounds__(MG_WG) void k_mg_zrestrict(const T* __restrict__ R1, T* __restrict__ B,
                                                       MgGeom fg, MgGeom cg, const int32_t* __restrict__ active,
                                                       uint32_t N, uint32_t NV, ZMarch zs) {
  const ZPos q = zpos<VW>(cg, zs, active, NV);
  if (!q.ok) return;
  const uint32_t v = q.v;
  uint32_t fx[4], fy[4];
  double wx[4], wy[4];
  restrict_taps(q.x, fg.m0, fx, wx);
  restrict_taps(q.y, fg.m1, fy, wy);
  auto rxy = [&](uint32_t z, T(&o)[VW]) {
    zero(o);
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      T ax[VW];
      zero(ax);
      const uint64_t row = ((uint64_t)z * fg.m1 + fy[bb]) * fg.m0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        T t[VW];
        ldr<T, VW>(R1, row + fx[a], N, v, t);
#pragma unroll
        for (int k = 0; k < VW; ++k) ax[k] += (T)wx[a] * t[k];
      }
#pragma unroll
      for (int k = 0; k < VW; ++k) o[k] += (T)wy[bb] * ax[k];
    }
  };
  const uint64_t cs2 = (uint64_t)cg.m0 * cg.m1;
  uint64_t P = ((uint64_t)q.z0 * cg.m1 + q.y) * cg.m0 + q.x;
  if (fg.m2 == 1) {                 // no z axis
    T o[VW];
    rxy(0, o);
    str<T, VW>(B, P, N, v, o);
    return;
  }
  // fine planes 2K - 1, 2K, 2K + 1, 2K + 2 with weights 1/8, 3/8, 3/8, 1/8;
  // the last two are the first two of coarse plane K + 1
  T ra[VW], rb[VW];
  zero(ra);
  zero(rb);
  if (q.z0 >= 1) rxy(2 * q.z0 - 1, ra);
  rxy(2 * q.z0, rb);
  for (uint32_t K = q.z0; K < q.z1; ++K, P += cs2) {
    T rc[VW], rd[VW], o[VW];
    zero(rc);
    zero(rd);
    if (2 * K + 1 < fg.m2) rxy(2 * K + 1, rc);
    if (2 * K + 2 < fg.m2) rxy(2 * K + 2, rd);
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      o[k] = T(0.125) * ra[k] + T(0.375) * rb[k] + T(0.375) * rc[k] + T(0.125) * rd[k];
      ra[k] = rc[k];
      rb[k] = rd[k];
    }
    str<T, VW>(B, P, N, v, o);
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

// Storage type of the blocks (the context's: FP64, or FP32 for OPE_MIXED) and
// elements per thread (16 bytes when N allows).
inline uint32_t mg_esz(const ope_ctx* c) { return c->prec == OPE_FP64 ? 8u : 4u; }
inline uint32_t mg_vw(const ope_ctx* c) {
  if (c->prec == OPE_FP64) return c->N % 2 == 0 ? 2u : 1u;
  return c->N % 4 == 0 ? 4u : (c->N % 2 == 0 ? 2u : 1u);
}

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
  for (int k = 0; k < c->mg_levels; ++k) {
    if (k > 0 && c->mg[k].diag) (void)hipFree(c->mg[k].diag);
    if (c->mg[k].wd) (void)hipFree(c->mg[k].wd);
  }
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
  std::vector<std::vector<double>> diags;       // the diagonal of every level (level 0: the context's)
  diags.push_back(W);
  const double dsum0 = 2.0 * (c->g.cx + c->g.cy + c->g.cz);
  for (auto& w : W) w -= dsum0;
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
  const std::vector<double>& dc = diags[(size_t)nl - 1];
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
  const uint32_t esz = mg_esz(c);
  {
    const uint32_t NV = (uint32_t)N / mg_vw(c);
    const TShape ts = tshape(lv[0].m0, lv[0].m1, lv[0].m2, NV, (uint32_t)N, esz);
    c->mg_rows = (int64_t)ts.nxt * ts.nyt * ts.nzc;        // partial rows of the level-0 post-smoothing
  }
  bool ok = hipMalloc(&c->mg_mem, (size_t)esz * (size_t)elems) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->mg_inv, sizeof(double) * (size_t)nc * nc) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->mg_part, sizeof(double) * (size_t)c->mg_rows * 2 * N) == hipSuccess;
  ok = ok && hipMalloc((void**)&c->mg_dots, sizeof(double) * 2 * (size_t)N) == hipSuccess;
  for (int k = 1; k < nl && ok; ++k) ok = hipMalloc((void**)&lv[k].diag, sizeof(double) * lv[k].n) == hipSuccess;
  for (int k = 0; k < nl && ok; ++k) ok = hipMalloc((void**)&lv[k].wd, sizeof(double) * lv[k].n) == hipSuccess;
  c->mg_levels = nl;
  for (int k = 0; k < nl; ++k) c->mg[k] = lv[k];
  if (!ok) {
    mg_free(c);
    return OPE_ENOMEM;
  }
  char* mem = (char*)c->mg_mem;
  c->mg[0].T = mem;
  mem += (size_t)esz * c->n * N;
  c->mg_Z = mem;
  mem += (size_t)esz * c->n * N;
  for (int k = 1; k < nl; ++k) {
    c->mg[k].B = mem;
    mem += (size_t)esz * c->mg[k].n * N;
    c->mg[k].E = mem;
    mem += (size_t)esz * c->mg[k].n * N;
    c->mg[k].T = mem;
    mem += (size_t)esz * c->mg[k].n * N;
  }
  ok = hipMemcpy(c->mg_inv, A.data(), sizeof(double) * (size_t)nc * nc, hipMemcpyHostToDevice) == hipSuccess;
  for (int k = 1; k < nl && ok; ++k)
    ok = hipMemcpy(c->mg[k].diag, diags[(size_t)k].data(), sizeof(double) * c->mg[k].n, hipMemcpyHostToDevice) ==
         hipSuccess;
  for (int k = 0; k < nl && ok; ++k) {
    std::vector<double> w(diags[(size_t)k].size());
    for (size_t p = 0; p < w.size(); ++p) w[p] = MG_OMEGA / diags[(size_t)k][p];
    ok = hipMemcpy(c->mg[k].wd, w.data(), sizeof(double) * c->mg[k].n, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) {
    mg_free(c);
    return OPE_EHIP;
  }
  return OPE_OK;
}

template <typename T, int VW>
static hipError_t vcycle_t(ope_ctx* c, const T* r, T* z, const int32_t* active, bool dots) {
  const uint32_t N = (uint32_t)c->N, NV = N / VW;
  const int L = c->mg_levels;
  hipStream_t s = c->stream;
  for (int k = 0; k + 1 < L; ++k) {
    const MgLevel& f = c->mg[k];
    const MgLevel& q = c->mg[k + 1];
    const T* in = k == 0 ? r : (const T*)f.B;
    const TShape ts = tshape(f.m0, f.m1, f.m2, NV, N, sizeof(T));
    const ZMarch zq = zmarch_shape(q.m0, q.m1, q.m2, NV);
    const dim3 sgrid(ts.nxt * ts.nyt * ts.nzc * ts.NS), sblock(ts.TX * ts.TY * ts.NVS);
    switch (ring_per_thread(ts)) {
      case 1:
        hipLaunchKernelGGL((k_mg_tstencil<T, VW, 1>), sgrid, sblock, 0, s, in, (T*)f.T, geom(f), f.diag, f.wd, active,
                           N, ts);
        break;
      case 2:
        hipLaunchKernelGGL((k_mg_tstencil<T, VW, 2>), sgrid, sblock, 0, s, in, (T*)f.T, geom(f), f.diag, f.wd, active,
                           N, ts);
        break;
      default:
        hipLaunchKernelGGL((k_mg_tstencil<T, VW, 4>), sgrid, sblock, 0, s, in, (T*)f.T, geom(f), f.diag, f.wd, active,
                           N, ts);
    }
    hipLaunchKernelGGL((k_mg_zrestrict<T, VW>), dim3(zq.nxs * q.m1 * zq.nzc), dim3(MG_WG), 0, s, (const T*)f.T,
                       (T*)q.B, geom(f), geom(q), active, N, NV, zq);
  }
  const MgLevel& cl = c->mg[L - 1];
  const uint64_t tcl = (uint64_t)cl.n * NV;
  hipLaunchKernelGGL((k_mg_dense<T, VW>), dim3(grid_of(tcl)), dim3(MG_WG), 0, s, c->mg_inv, (const T*)cl.B, (T*)cl.E,
                     (uint32_t)cl.n, active, N, NV, tcl);
  for (int k = L - 2; k >= 0; --k) {
    const MgLevel& f = c->mg[k];
    const MgLevel& q = c->mg[k + 1];
    const T* in = k == 0 ? r : (const T*)f.B;
    T* out = k == 0 ? z : (T*)f.E;
    const T* qe = (const T*)q.E;
    const TShape ts = tshape(f.m0, f.m1, f.m2, NV, N, sizeof(T));
    const uint32_t rows = ts.nxt * ts.nyt * ts.nzc;
    const uint32_t P = ts.TX * ts.TY;
    const int R = ring_per_thread(ts);
    const dim3 grid(rows * ts.NS), block(P * ts.NVS);
    const bool d = k == 0 && dots;
    double* part = d ? c->mg_part : nullptr;
    auto post = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, block, 0, s, in, qe, out, geom(f), geom(q), f.diag, f.wd, active, N, ts, part);
    };
    {
      ProfScope ps(c, d ? OPE_KERNEL_MG_POST : OPE_KERNEL_COUNT);   // only the finest level is timed
      if (d) {
        if (R == 1) post(k_mg_tpost<T, VW, true, 1>);
        else if (R == 2) post(k_mg_tpost<T, VW, true, 2>);
        else post(k_mg_tpost<T, VW, true, 4>);
        c->mg_rows_used = rows;
      } else {
        if (R == 1) post(k_mg_tpost<T, VW, false, 1>);
        else if (R == 2) post(k_mg_tpost<T, VW, false, 2>);
        else post(k_mg_tpost<T, VW, false, 4>);
      }
    }
  }
  return hipGetLastError();
}

hipError_t mg_vcycle(ope_ctx* c, const void* r, void* z, const int32_t* active, bool dots) {
  ProfScope ps(c, OPE_KERNEL_MG);
  if (c->prec == OPE_FP64) {
    if (mg_vw(c) == 2) return vcycle_t<double, 2>(c, (const double*)r, (double*)z, active, dots);
    return vcycle_t<double, 1>(c, (const double*)r, (double*)z, active, dots);
  }
  switch (mg_vw(c)) {
    case 4: return vcycle_t<float, 4>(c, (const float*)r, (float*)z, active, dots);
    case 2: return vcycle_t<float, 2>(c, (const float*)r, (float*)z, active, dots);
    default: return vcycle_t<float, 1>(c, (const float*)r, (float*)z, active, dots);
  }
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
