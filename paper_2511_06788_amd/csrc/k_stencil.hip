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
//   sweep A (cg_pap):    p = r + beta p_old (formed on the fly, with its
//                        neighbours), sigma_j = p_j^T H p_j, and p is written out
//   sweep B (cg_update): r' = r - alpha H p, rho'_j = r'_j^T r'_j, and on odd
//                        iterations y += alpha_prev p_prev + alpha p
// B recomputes H p from p instead of reading a stored q = H p, so its neighbour
// rows come from one array.  The y update of an even iteration k is deferred to
// iteration k + 1 (p_k is still in the other p buffer then, and alpha keeps
// one array per iteration parity): per pair of iterations A moves 3 + 3 block
// passes (reads r, p_old, writes p) and B 3 + 6 (reads p, r, writes r'; then
// also reads y, p_prev and writes y), 15 instead of 16.  The two y terms are
// added in iteration order, so y equals that of updating it every iteration,
// bit for bit.  The per-column
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

// Whether any column is active, or (given `pending`) has a non-zero entry there.
__device__ __forceinline__ bool any_active(const int32_t* __restrict__ active, uint32_t N,
                                           const double* __restrict__ pending = nullptr) {
  int a = 0;
  for (uint32_t j = threadIdx.x; j < N; j += OPE_WG) a |= active[j] | (pending && pending[j] != 0.0 ? 1 : 0);
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
// x neighbours come from the current plane staged in LDS (and, at the ends of
// an x segment, from the neighbouring segment's rows), side neighbours from
// the rows the adjacent work-groups of the same XCD stream at the same time
// (L2 hits).
//
// Memory access is through buffer descriptors, one per array and plane (base
// = the plane's first row, range = one plane), with per-lane byte offsets
// that stay fixed over the march.  A lane without a row to touch (outside the
// grid or the column range) carries an offset beyond every range: its loads
// return zero and its stores are dropped by the range check, and a plane
// outside the march gets an empty range.  So no load or store sits under a
// branch.
//
// Software pipeline: at plane k the loads for plane k+2 (its side rows,
// x-segment ends, diagonal and y, and the centre row of plane k+3) are issued
// into one of two register sets, while the other set, issued one plane
// earlier, is taken in at the end of plane k.  Vector-memory counters retire
// in issue order, so a load has two plane steps to arrive; with every access
// unconditional the compiler's wait before taking a set in covers exactly the
// accesses issued before it.
// MODE selects the field and what is done with (H p) at each point:
//   SW_APPLY   field x (F0);          out = H x (O0)
//   SW_PAP     field p = r + beta p_old (F0, F1; r alone when FIRST);
//              sigma_j += p_j (H p)_j, p written (O1)
//   SW_UPDATE  field p (F1), r (F0) at the centre only;
//              r' = r - alpha H p (O0), rho'_j += r'_j^2
//   SW_UPDATE_Y  as SW_UPDATE, and y (Yv) += alpha_prev p_prev + alpha p, with
//              p_prev read from O1 and alpha_prev taken from the beta argument
enum { SW_APPLY = 0, SW_PAP = 1, SW_UPDATE = 2, SW_UPDATE_Y = 3 };

typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int RSRC_FLAGS = 0x00020000;        // raw (unformatted) 32-bit dword access
constexpr uint32_t NO_ROW = 0x80000000u;      // a byte offset beyond every plane's range
constexpr int AUX_NT = 2;                     // non-temporal (streamed, not kept in the caches)

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, RSRC_FLAGS);
}

typedef unsigned int BufU4 __attribute__((ext_vector_type(4)));
typedef unsigned int BufU2 __attribute__((ext_vector_type(2)));

// One row chunk (VW elements of T, 4, 8 or 16 bytes) through a descriptor
// (AUX: cache policy, AUX_NT for a stream read once).
template <typename T, int VW, int AUX = 0>
__device__ __forceinline__ void bld(Rsrc rs, uint32_t off, T (&v)[VW]) {
  constexpr int B = (int)sizeof(T) * VW;
  RowVec<T, VW> t;
  if constexpr (B == 16) t = __builtin_bit_cast(RowVec<T, VW>, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, AUX));
  else if constexpr (B == 8) t = __builtin_bit_cast(RowVec<T, VW>, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, AUX));
  else t = __builtin_bit_cast(RowVec<T, VW>, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, AUX));
#pragma unroll
  for (int k = 0; k < VW; ++k) v[k] = t.v[k];
}

template <typename T>
__device__ __forceinline__ T bld1(Rsrc rs, uint32_t off) {
  if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
}

template <typename T, int VW, int AUX>
__device__ __forceinline__ void bst(Rsrc rs, uint32_t off, const T (&v)[VW]) {
  constexpr int B = (int)sizeof(T) * VW;
  RowVec<T, VW> t;
#pragma unroll
  for (int k = 0; k < VW; ++k) t.v[k] = v[k];
  if constexpr (B == 16) __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(BufU4, t), rs, off, 0, AUX);
  else if constexpr (B == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufU2, t), rs, off, 0, AUX);
  else __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, t), rs, off, 0, AUX);
}

// A register move the compiler cannot fold away.  Taking a load set in
// through these leaves its load registers dead, so the loop keeps each set in
// the same registers; otherwise the combined values (r + beta p_old, formed in
// place) occupy them, the next load of the set lands elsewhere and is copied
// back at the loop edge, and the copy must wait for the load.
template <typename T>
__device__ __forceinline__ T vmove(T x) {
  T r;
  if constexpr (sizeof(T) == 8) asm volatile("v_mov_b64 %0, %1" : "=&v"(r) : "v"(x));
  else asm volatile("v_mov_b32 %0, %1" : "=&v"(r) : "v"(x));
  return r;
}

// The loads of one plane step, per pass q (raw field values: the two parts
// r and p_old apart in SW_PAP).
template <typename T, int VW, int Q>
struct MarchLoads {
  T cr[Q][VW], cp[Q][VW];      // field at the centre row of plane k+3
  T lr[Q][VW], lp[Q][VW];      // side row below, plane k+2
  T ur[Q][VW], up[Q][VW];      // side row above, plane k+2
  T hr[Q][VW], hp[Q][VW];      // the x-segment end's outer neighbour, plane k+2
  T d[Q];                      // diagonal, plane k+2
  T r[Q][VW], y[Q][VW];        // r and y at the centre row of plane k+2 (SW_UPDATE, y: SW_UPDATE_Y)
  T pp[Q][VW];                 // p_prev at the centre row of plane k+2 (SW_UPDATE_Y)
};

template <typename T, int VW, int Q, bool TWO, bool UPD, bool YUP, bool HALO, bool LN>
__device__ __forceinline__ void take_set(const MarchLoads<T, VW, Q>& a, MarchLoads<T, VW, Q>& b) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      b.cr[q][v] = vmove(a.cr[q][v]);
      if constexpr (TWO) b.cp[q][v] = vmove(a.cp[q][v]);
      if (!LN || q == 0) {
        b.lr[q][v] = vmove(a.lr[q][v]);
        if constexpr (TWO) b.lp[q][v] = vmove(a.lp[q][v]);
      }
      if (!LN || q == Q - 1) {
        b.ur[q][v] = vmove(a.ur[q][v]);
        if constexpr (TWO) b.up[q][v] = vmove(a.up[q][v]);
      }
      if constexpr (HALO) {
        b.hr[q][v] = vmove(a.hr[q][v]);
        if constexpr (TWO) b.hp[q][v] = vmove(a.hp[q][v]);
      }
      if constexpr (UPD) b.r[q][v] = vmove(a.r[q][v]);
      if constexpr (YUP) {
        b.y[q][v] = vmove(a.y[q][v]);
        b.pp[q][v] = vmove(a.pp[q][v]);
      }
    }
    b.d[q] = vmove(a.d[q]);
  }
}

// The march of work item t (0 <= t < lgroups * nxs * cc * mc) of one
// problem; shared by the single-problem kernel and the batched kernel below.
// HALO: the x line is split into several segments (nxs > 1).  LN: the
// work-group takes ly = Q lpp adjacent side lines, lpp per pass, each over one
// x segment (xseg = pp / lpp points), rather than Q parts of one line's x
// segment; the inner side neighbours come from the staged plane, and only the
// tile's outer lines load side rows.
// A plane of one array must be smaller than 2 GiB (checked when the context
// is created).
template <typename T, int VW, int Q, int MODE, bool FIRST, bool HALO, bool LN>
__device__ __forceinline__ void march_body(uint32_t t, const T* __restrict__ F0, const T* __restrict__ F1,
                                           T* __restrict__ O0, T* __restrict__ O1, T* __restrict__ Yv,
                                           const double* __restrict__ alpha, const double* __restrict__ beta,
                                           const int32_t* __restrict__ active, const T* __restrict__ diag,
                                           const OpeGrid& g, const MarchShape& ms, uint32_t N, uint32_t NV,
                                           double* __restrict__ part, OpeScalars* __restrict__ sc) {
  constexpr bool TWO = (MODE == SW_PAP) && !FIRST;   // field is r + beta p_old (two loads per value)
  constexpr bool UPD = (MODE == SW_UPDATE || MODE == SW_UPDATE_Y);
  constexpr bool YUP = (MODE == SW_UPDATE_Y);
  constexpr int AUX_OUT = 0;
  const T* __restrict__ FF = UPD ? F1 : F0;            // the field's (first) array
  __shared__ T lds[2 * Q * OPE_WG * VW];
  __shared__ double red[OPE_WG * VW];
  if (MODE != SW_APPLY) {
    if (!any_active(active, N)) {
      // every column has converged; SW_UPDATE_Y still adds the pending y term
      // of the previous iteration, y += alpha_prev p_prev (the arithmetic of
      // the full sweep with alpha = 0, and of the flush kernel), as a plain
      // stream over the block instead of a march
      if (YUP && any_active(active, N, beta)) {
        const uint64_t count = (uint64_t)g.m0 * g.m1 * g.m2 * N;
        const uint64_t stride = (uint64_t)ms.lgroups * ms.nxs * ms.cc * ms.mc * OPE_WG;
        for (uint64_t e = (uint64_t)t * OPE_WG + threadIdx.x; e < count; e += stride)
          Yv[e] = Yv[e] + (T)beta[e % N] * O1[e];
      }
      return;
    }
    if (MODE == SW_PAP && t == 0 && threadIdx.x == 0) sc->cg_iters += 1;
  }
  const uint32_t mchunk_id = t % ms.mc;
  t /= ms.mc;
  uint32_t cchunk, xs, lg;
  if (ms.order == 0) {           // ((group * nxs + xs) * cc + chunk) * mc + m
    cchunk = t % ms.cc;
    t /= ms.cc;
    xs = t % ms.nxs;
    lg = t / ms.nxs;
  } else {                       // ((chunk * lgroups + group) * nxs + xs) * mc + m
    xs = t % ms.nxs;
    t /= ms.nxs;
    lg = t % ms.lgroups;
    cchunk = t / ms.lgroups;
  }
  const uint32_t lpp = LN ? ms.lpp : 1u;                 // side lines per pass
  const uint32_t ly = LN ? (uint32_t)Q * lpp : 1u;       // side lines of the work-group
  const uint32_t line0 = lg * ly;
  const uint32_t cv = threadIdx.x % ms.ncv, slot = threadIdx.x / ms.ncv;
  const uint32_t used = LN ? lpp * ms.xseg : ms.pp;      // slots that hold points
  const uint32_t lip = LN ? slot / ms.xseg : 0u;         // line within the pass
  const uint32_t colv = cchunk * ms.ncv + cv;
  const bool lane_ok = slot < used && colv < NV;
  const uint32_t z0 = mchunk_id * ms.mchunk;
  const uint32_t z1 = min(ms.mlen, z0 + ms.mchunk);
  // one plane of an array: march_stride rows of N values
  const uint64_t plane_elems = (uint64_t)ms.march_stride * N;
  const uint32_t plane_bytes = (uint32_t)(plane_elems * sizeof(T));
  const uint32_t row_bytes = N * (uint32_t)sizeof(T);

  T b[VW], a[VW], ap[VW];
  double acc[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) {
    b[v] = (TWO && lane_ok) ? (T)beta[colv * VW + v] : T(0);
    a[v] = (UPD && lane_ok) ? (T)alpha[colv * VW + v] : T(0);
    ap[v] = (YUP && lane_ok) ? (T)beta[colv * VW + v] : T(0);     // alpha of the previous iteration
    acc[v] = 0.0;
  }
  const T cx = (T)g.cx, cs = (T)ms.cs, cm = (T)ms.cm;
  // per-pass byte offsets within a plane (NO_ROW where there is no row)
  uint32_t xq[Q], xiq[Q], ltq[Q], liq[Q], oc[Q], ol[Q], ou[Q], oh[Q], od[Q];
  bool okq[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const uint32_t lt = LN ? q * lpp + lip : 0u;               // line within the tile
    const uint32_t xi = LN ? slot - lip * ms.xseg : q * ms.pp + slot;   // position in the x segment
    const uint32_t line = line0 + lt;
    xiq[q] = xi;
    ltq[q] = lt;
    liq[q] = LN ? lt * ms.xseg + xi : q * ms.pp + slot;       // slot in the staged plane
    xq[q] = xs * ms.xseg + xi;
    okq[q] = lane_ok && xi < ms.xseg && xq[q] < g.m0 && line < ms.lines;
    const uint32_t p = xq[q] + line * ms.side_stride;     // point index within the plane
    oc[q] = okq[q] ? p * row_bytes + colv * VW * (uint32_t)sizeof(T) : NO_ROW;
    // side rows from memory: every pass, or in LN only the tile's outer lines
    const bool own_lo = !LN || lt == 0, own_hi = !LN || lt + 1 == ly;
    ol[q] = (okq[q] && own_lo && ms.has_side && line > 0) ? oc[q] - ms.side_stride * row_bytes : NO_ROW;
    ou[q] = (okq[q] && own_hi && ms.has_side && line + 1 < ms.lines) ? oc[q] + ms.side_stride * row_bytes : NO_ROW;
    oh[q] = NO_ROW;
    if (HALO && okq[q]) {
      if (xi == 0 && xq[q] > 0) oh[q] = oc[q] - row_bytes;
      else if (xi + 1 == ms.xseg && xq[q] + 1 < g.m0) oh[q] = oc[q] + row_bytes;
    }
    od[q] = okq[q] ? p * (uint32_t)sizeof(T) : NO_ROW;
  }
  // descriptors of plane z of an array and of the diagonal; empty unless `valid`
  // (an empty one points at plane 0, so no address is formed outside the array)
  auto prs = [&](const T* base, uint32_t z, bool valid) -> Rsrc {
    return make_rsrc(base + (valid ? (uint64_t)z * plane_elems : 0), valid ? plane_bytes : 0u);
  };
  auto drs = [&](uint32_t z, bool valid) -> Rsrc {
    return make_rsrc(diag + (valid ? (uint64_t)z * ms.march_stride : 0),
                     valid ? ms.march_stride * (uint32_t)sizeof(T) : 0u);
  };
  auto zero = [](T (&o)[VW]) {
#pragma unroll
    for (int v = 0; v < VW; ++v) o[v] = T(0);
  };
  auto comb = [&](const T (&r)[VW], const T (&po)[VW], T (&out)[VW]) {
#pragma unroll
    for (int v = 0; v < VW; ++v) out[v] = TWO ? r[v] + b[v] * po[v] : r[v];
  };

  // pipeline registers (per pass q)
  T pm[Q][VW], pz[Q][VW], p1[Q][VW];   // field at z-1, z, z+1
  T rz[Q][VW];                          // r at z (SW_UPDATE)
  T smz[Q][VW], spz[Q][VW], hz[Q][VW];  // side neighbours and segment-end neighbour at z
  T dz[Q], yz[Q][VW], ppz[Q][VW];       // diagonal, y and p_prev at z

  // loads for plane zs (side rows, segment ends, diagonal, r and y) and the
  // field's centre row of zs + 1
  auto issue = [&](uint32_t zs, MarchLoads<T, VW, Q>& L) {
    const bool vs = zs < z1, vc = vs && zs + 1 < ms.mlen;
    const Rsrc c0 = prs(FF, zs + 1, vc), s0 = prs(FF, zs, vs);
    const Rsrc c1 = prs(F1, zs + 1, vc && TWO), s1 = prs(F1, zs, vs && TWO);
    const Rsrc dr = drs(zs, vs), yr = prs(Yv, zs, vs && YUP), rr = prs(F0, zs, vs && UPD);
    const Rsrc qr = prs(O1, zs, vs && YUP);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      bld<T, VW>(c0, oc[q], L.cr[q]);
      if constexpr (TWO) bld<T, VW>(c1, oc[q], L.cp[q]);
      if (!LN || q == 0) {
        bld<T, VW>(s0, ol[q], L.lr[q]);
        if constexpr (TWO) bld<T, VW>(s1, ol[q], L.lp[q]);
      }
      if (!LN || q == Q - 1) {
        bld<T, VW>(s0, ou[q], L.ur[q]);
        if constexpr (TWO) bld<T, VW>(s1, ou[q], L.up[q]);
      }
      if constexpr (HALO) {
        bld<T, VW>(s0, oh[q], L.hr[q]);
        if constexpr (TWO) bld<T, VW>(s1, oh[q], L.hp[q]);
      }
      L.d[q] = bld1<T>(dr, od[q]);
      // single-use streams: non-temporal when the working set exceeds the
      // last-level cache (with it, they would hit there; measured slower)
      if constexpr (UPD) {
        if (ms.nt) bld<T, VW, AUX_NT>(rr, oc[q], L.r[q]);
        else bld<T, VW>(rr, oc[q], L.r[q]);
      }
      if constexpr (YUP) {
        if (ms.nt) {
          bld<T, VW, AUX_NT>(yr, oc[q], L.y[q]);
          bld<T, VW, AUX_NT>(qr, oc[q], L.pp[q]);
        } else {
          bld<T, VW>(yr, oc[q], L.y[q]);
          bld<T, VW>(qr, oc[q], L.pp[q]);
        }
      }
    }
  };
  // end of plane z: shift the planes and take in the set issued for plane z + 1
  // (moved out of its load registers first, so those stay free for the next
  // load of the same set)
  auto rotate = [&](const MarchLoads<T, VW, Q>& Lin) {
    MarchLoads<T, VW, Q> L;
    take_set<T, VW, Q, TWO, UPD, YUP, HALO, LN>(Lin, L);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        pm[q][v] = pz[q][v];
        pz[q][v] = p1[q][v];
        if constexpr (UPD) rz[q][v] = L.r[q][v];
        if constexpr (YUP) {
          yz[q][v] = L.y[q][v];
          ppz[q][v] = L.pp[q][v];
        }
      }
      comb(L.cr[q], L.cp[q], p1[q]);
      if (!LN || q == 0) comb(L.lr[q], L.lp[q], smz[q]);
      if (!LN || q == Q - 1) comb(L.ur[q], L.up[q], spz[q]);
      if constexpr (HALO) comb(L.hr[q], L.hp[q], hz[q]);
      dz[q] = L.d[q];
    }
  };

  // prologue: planes z0 - 1 and z0, then plane z0's set (its side rows etc.
  // and the centre of z0 + 1) through the same rotate
  {
    const uint32_t zm = z0 > 0 ? z0 - 1 : 0;
    const Rsrc m0r = prs(FF, zm, z0 > 0), m1r = prs(F1, zm, z0 > 0 && TWO);
    const Rsrc c0r = prs(FF, z0, true), c1r = prs(F1, z0, TWO);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T tr[VW], tp[VW];
      zero(tp);
      bld<T, VW>(m0r, oc[q], tr);
      if constexpr (TWO) bld<T, VW>(m1r, oc[q], tp);
      comb(tr, tp, pz[q]);                      // becomes pm
      bld<T, VW>(c0r, oc[q], tr);
      if constexpr (TWO) bld<T, VW>(c1r, oc[q], tp);
      comb(tr, tp, p1[q]);                      // becomes pz
    }
    MarchLoads<T, VW, Q> L0;
    issue(z0, L0);
    rotate(L0);
  }

  // plane z: stage it for the x neighbours, apply H, use the result
  auto compute = [&](uint32_t z, T* __restrict__ buf) {
    // lanes past the last used slot hold no point, and their index would
    // alias another pass's slot
    if (slot < used) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int v = 0; v < VW; ++v) buf[(liq[q] * ms.ncv + cv) * VW + v] = pz[q][v];
    }
    __syncthreads();
    const Rsrc o0 = prs(O0, z, MODE != SW_PAP);
    const Rsrc o1 = prs(O1, z, MODE == SW_PAP), yo = prs(Yv, z, YUP);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const uint32_t xi = xiq[q], li = liq[q];   // x position; slot in the staged plane
      // x neighbours: the staged plane, or the segment end's outer row (zero
      // where there is none: at the grid boundary, or a lane past the grid)
      const uint32_t im = xi > 0 ? li - 1 : li, ip = xi + 1 < ms.xseg ? li + 1 : li;
      T xm[VW], xp[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const T lm = buf[(im * ms.ncv + cv) * VW + v], lp = buf[(ip * ms.ncv + cv) * VW + v];
        const T hm = HALO ? hz[q][v] : T(0);
        xm[v] = xi > 0 ? lm : hm;
        xp[v] = xi + 1 < ms.xseg ? lp : hm;
      }
      // side neighbours: loaded rows, or in LN the staged plane's adjacent
      // lines inside the tile (zero beyond the grid: such a line loaded nothing)
      T sm[VW], sp[VW];
      const uint32_t lt = ltq[q];
      const uint32_t ym = (LN && lt > 0) ? li - ms.xseg : li, yp = (LN && lt + 1 < ly) ? li + ms.xseg : li;
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const T lm = buf[(ym * ms.ncv + cv) * VW + v], lp = buf[(yp * ms.ncv + cv) * VW + v];
        sm[v] = (LN && lt > 0) ? lm : ((!LN || q == 0) ? smz[q][v] : T(0));
        sp[v] = (LN && lt + 1 < ly) ? lp : ((!LN || q == Q - 1) ? spz[q][v] : T(0));
      }
      T hx[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v)
        hx[v] = dz[q] * pz[q][v] - (cx * (xm[v] + xp[v]) + cs * (sm[v] + sp[v]) + cm * (pm[q][v] + p1[q][v]));
      if constexpr (MODE == SW_APPLY) {
        if (ms.nt) bst<T, VW, AUX_NT>(o0, oc[q], hx);
        else bst<T, VW, AUX_OUT>(o0, oc[q], hx);
      } else if constexpr (MODE == SW_PAP) {
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] += okq[q] ? (double)pz[q][v] * (double)hx[v] : 0.0;
        if (ms.nt) bst<T, VW, AUX_NT>(o1, oc[q], pz[q]);
        else bst<T, VW, AUX_OUT>(o1, oc[q], pz[q]);
      } else {
        T yv[VW], rnew[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          rnew[v] = rz[q][v] - a[v] * hx[v];
          acc[v] += okq[q] ? (double)rnew[v] * (double)rnew[v] : 0.0;
          if constexpr (YUP) {
            const T y1 = yz[q][v] + ap[v] * ppz[q][v];      // the previous iteration's term first
            yv[v] = y1 + a[v] * pz[q][v];
          }
        }
        if (ms.nt) {
          if constexpr (YUP) bst<T, VW, AUX_NT>(yo, oc[q], yv);
          bst<T, VW, AUX_NT>(o0, oc[q], rnew);
        } else {
          if constexpr (YUP) bst<T, VW, AUX_OUT>(yo, oc[q], yv);
          bst<T, VW, AUX_OUT>(o0, oc[q], rnew);
        }
      }
    }
  };

  // the march, unrolled by two (a straight-line body, so that the two load
  // sets keep fixed registers across the loop edge), then an odd last plane
  MarchLoads<T, VW, Q> LA, LB;
  issue(z0 + 1, LA);      // z0 < z1 always (march chunks are never empty)
  uint32_t z = z0;
  for (; z + 1 < z1; z += 2) {
    issue(z + 2, LB);
    compute(z, lds);
    rotate(LA);
    issue(z + 3, LA);
    compute(z + 1, lds + Q * OPE_WG * VW);
    rotate(LB);
  }
  if (z < z1) compute(z, lds);
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
      const uint64_t row = ((uint64_t)lg * ms.nxs + xs) * ms.mc + mchunk_id;
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const uint64_t col = (uint64_t)colv * VW + v;
        if (col < N) part[row * N + col] = s[v];
      }
    }
  }
}

template <typename T, int VW, int Q, int MODE, bool FIRST, bool HALO, bool LN>
__global__ __launch_bounds__(OPE_WG) void k_march(const T* __restrict__ F0, const T* __restrict__ F1,
                                                  T* __restrict__ O0, T* __restrict__ O1,
                                                  T* __restrict__ Yv, const double* __restrict__ alpha,
                                                  const double* __restrict__ beta, const int32_t* __restrict__ active,
                                                  const T* __restrict__ diag, OpeGrid g, MarchShape ms,
                                                  uint32_t N, uint32_t NV, double* __restrict__ part,
                                                  OpeScalars* __restrict__ sc) {
  march_body<T, VW, Q, MODE, FIRST, HALO, LN>(xcd_remap(blockIdx.x, gridDim.x), F0, F1, O0, O1, Yv, alpha, beta, active,
                                          diag, g, ms, N, NV, part, sc);
}

// Batched form: one launch for the CG sweeps of many problems of the same
// storage type and shape class.  Problem j owns work-groups [wg_begin,
// wg_begin + wg_count rounded up to 8) (wg_begin a multiple of 8), remapped
// within the problem so that each XCD streams one contiguous eighth of every
// problem: a remap over the whole launch would give each XCD a range of
// whole problems, and their work per item differs widely (the work of the
// launch would not be spread evenly over the XCDs).
template <typename T, int VW, int Q, int MODE, bool FIRST, bool HALO, bool LN>
__global__ __launch_bounds__(OPE_WG) void k_march_batched(const MarchJob* __restrict__ jobs, uint32_t njobs) {
  const uint32_t b = blockIdx.x;
  uint32_t lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (jobs[mid].wg_begin <= b) lo = mid;
    else hi = mid;
  }
  const MarchJob& jb = jobs[lo];
  const uint32_t t = xcd_remap(b - jb.wg_begin, (jb.wg_count + 7u) & ~7u);
  if (t >= jb.wg_count) return;      // padding of the problem's range
  const OpeGrid g = jb.g;
  const MarchShape ms = jb.ms;
  march_body<T, VW, Q, MODE, FIRST, HALO, LN>(t, (const T*)jb.F0, (const T*)jb.F1, (T*)jb.O0, (T*)jb.O1,
                                    (T*)jb.Yv, jb.alpha, jb.beta, jb.active, (const T*)jb.diag, g, ms, jb.N, jb.NV,
                                    jb.part, jb.sc);
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

// First stage of the column sums of a [nrows][ncols] partial array: work-group
// (column group x, y) sums rows [y rps, (y + 1) rps) of its 64 columns into
// stage[y][col], in a fixed order.
__global__ __launch_bounds__(OPE_WG) void k_reduce_stage(const double* __restrict__ part, uint32_t nrows,
                                                         uint32_t ncols, uint32_t rps, double* __restrict__ stage) {
  __shared__ double red[OPE_WG];
  const uint32_t lc = threadIdx.x & 63u, grp = threadIdx.x >> 6;
  const uint32_t col = blockIdx.x * 64u + lc;
  const uint32_t w0 = blockIdx.y * rps, w1 = min(nrows, w0 + rps);
  double acc = 0.0;
  if (col < ncols)
    for (uint32_t w = w0 + grp; w < w1; w += 4) acc += part[(uint64_t)w * ncols + col];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (grp == 0 && col < ncols)
    stage[(uint64_t)blockIdx.y * ncols + col] = red[lc] + red[64 + lc] + red[128 + lc] + red[192 + lc];
}

// Column sums of a [nrows][ncols] partial array in a fixed order (one
// work-group per 64 columns), with an optional CG finalisation per column.
// Long partial arrays go through k_reduce_stage first.  (A last-block second
// stage inside one launch needs a device-scope fence per work-group, which
// writes back the XCD's dirty L2 lines; two launches need none.)
template <int MODE>
__global__ __launch_bounds__(OPE_WG) void k_reduce_cols(const double* __restrict__ part, uint32_t nrows,
                                                        uint32_t ncols, double* __restrict__ out,
                                                        double* __restrict__ alpha, double* __restrict__ beta,
                                                        double* __restrict__ rho, const double* __restrict__ target,
                                                        int32_t* __restrict__ active, OpeScalars* __restrict__ sc) {
  __shared__ double red[OPE_WG];
  // No early exit here even when every column has converged: the partials are
  // then stale, but inactive columns only ever receive alpha = beta = 0.
  const uint32_t lc = threadIdx.x & 63u, grp = threadIdx.x >> 6;
  const uint32_t col = blockIdx.x * 64u + lc;
  double acc = 0.0;
  if (col < ncols)
    for (uint32_t w = grp; w < nrows; w += 4) acc += part[(uint64_t)w * ncols + col];
  red[threadIdx.x] = acc;
  __syncthreads();
  double tot = 0.0;
  if (grp == 0) tot = red[lc] + red[64 + lc] + red[128 + lc] + red[192 + lc];
  if (grp != 0 || col >= ncols) return;
  if (MODE == RED_PLAIN) out[col] = tot;
  else cg_finalise<MODE>(col, tot, alpha, beta, rho, target, active, sc);
}

// The same column sums for few columns (ncols <= 128) by one 1024-thread
// work-group with no second stage: thread t sums column t % ncols over rows
// t / ncols, t / ncols + G, ... (G = 1024 / ncols row groups, 32 or eight
// loads in flight, eight running sums), then the groups are added in order (the single and the batched
// kernel share this order).  Avoids the cross-work-group fence of the split
// form, which writes back the L2 lines the preceding sweep left dirty.
constexpr uint32_t RED_WG = 1024;
// Largest partial array (rows x columns) summed by one work-group; longer ones
// take the two-launch split (measured: one work-group needs 10.5 us for the
// 512 x 128 partials of the FP32 sweeps at 64^3, N = 128).
constexpr int64_t FEW_MAX = (int64_t)1 << 15;

__device__ __forceinline__ double few_cols_sum(const double* __restrict__ part, uint32_t nrows, uint32_t ncols,
                                               double* red, uint32_t& col, bool& lead) {
  const uint32_t G = RED_WG / ncols;
  col = threadIdx.x % ncols;
  const uint32_t gi = threadIdx.x / ncols;
  double a = 0.0;
  if (gi < G) {
    double q[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    uint32_t w = gi;
    // 32 loads in flight, added in the order of the 8-wide loop below (so the
    // sums are the same bit for bit)
    for (; w + 31 * G < nrows; w += 32 * G) {
      double v[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) v[u] = part[(uint64_t)(w + u * G) * ncols + col];
#pragma unroll
      for (int u = 0; u < 32; ++u) q[u & 7] += v[u];
    }
    for (; w + 7 * G < nrows; w += 8 * G) {
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] += part[(uint64_t)(w + u * G) * ncols + col];
    }
    for (; w < nrows; w += G) q[0] += part[(uint64_t)w * ncols + col];
    a = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
  }
  red[threadIdx.x] = a;
  __syncthreads();
  lead = gi == 0;
  double tot = 0.0;
  if (lead)
    for (uint32_t k = 0; k < G; ++k) tot += red[k * ncols + col];
  return tot;
}

template <int MODE>
__global__ __launch_bounds__(RED_WG) void k_reduce_few(const double* __restrict__ part, uint32_t nrows,
                                                       uint32_t ncols, double* __restrict__ out,
                                                       double* __restrict__ alpha, double* __restrict__ beta,
                                                       double* __restrict__ rho, const double* __restrict__ target,
                                                       int32_t* __restrict__ active, OpeScalars* __restrict__ sc) {
  __shared__ double red[RED_WG];
  uint32_t col;
  bool lead;
  const double tot = few_cols_sum(part, nrows, ncols, red, col, lead);
  if (!lead) return;
  if (MODE == RED_PLAIN) out[col] = tot;
  else cg_finalise<MODE>(col, tot, alpha, beta, rho, target, active, sc);
}

// Batched one-work-group column reductions: work-group j reduces problem j.
// par: the CG iteration's parity, which selects the half of the problem's
// alpha array (2 ncols entries) the alpha reduction writes.
template <int MODE>
__global__ __launch_bounds__(RED_WG) void k_reduce_batched(const ReduceJob* __restrict__ jobs, uint32_t par) {
  __shared__ double red[RED_WG];
  const ReduceJob& jb = jobs[blockIdx.x];
  uint32_t col;
  bool lead;
  const double tot = few_cols_sum(jb.part, jb.nrows, jb.ncols, red, col, lead);
  if (!lead) return;
  cg_finalise<MODE>(col, tot, jb.alpha + (uint64_t)par * jb.ncols, jb.beta, jb.rho, jb.target, jb.active, jb.sc);
}

// y[i][j] += alpha[j] p[i][j] over n x N (a CG that stopped on an even
// iteration leaves that iteration's y term to add).
template <typename T>
__global__ __launch_bounds__(OPE_WG) void k_y_flush(T* __restrict__ y, const T* __restrict__ p,
                                                    const double* __restrict__ alpha, uint64_t count, uint32_t N) {
  for (uint64_t e = blockIdx.x * (uint64_t)OPE_WG + threadIdx.x; e < count; e += (uint64_t)gridDim.x * OPE_WG)
    y[e] = y[e] + (T)alpha[e % N] * p[e];
}

__global__ __launch_bounds__(OPE_WG) void k_gather_flags(const ReduceJob* __restrict__ jobs) {
  const ReduceJob& jb = jobs[blockIdx.x];
  for (uint32_t j = threadIdx.x; j < jb.ncols; j += OPE_WG) jb.flags_out[j] = jb.active[j];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// al, be: the kernel's alpha and beta arguments (their meaning per MODE is
// given at march_body).
template <typename T, int VW, int Q, int MODE, bool FIRST, bool LN>
static void launch_march_t(ope_ctx* c, const T* F0, const T* F1, T* O0, T* O1, T* Yv, const T* diag,
                           const double* al, const double* be) {
  const uint32_t N = (uint32_t)c->N, NV = N / VW;
  const MarchShape& ms = c->ms;
  const uint32_t grid = ms.lgroups * ms.nxs * ms.cc * ms.mc;
  if (ms.nxs > 1)
    hipLaunchKernelGGL((k_march<T, VW, Q, MODE, FIRST, true, LN>), dim3(grid), dim3(OPE_WG), 0, c->stream, F0, F1, O0,
                       O1, Yv, al, be, c->active, diag, c->g, ms, N, NV, c->part, c->sc);
  else
    hipLaunchKernelGGL((k_march<T, VW, Q, MODE, FIRST, false, LN>), dim3(grid), dim3(OPE_WG), 0, c->stream, F0, F1, O0,
                       O1, Yv, al, be, c->active, diag, c->g, ms, N, NV, c->part, c->sc);
}

template <typename T, int VW, int MODE, bool FIRST>
static void launch_march_q(ope_ctx* c, const T* F0, const T* F1, T* O0, T* O1, T* Yv, const T* diag,
                           const double* al, const double* be) {
  if (c->ms.ly > 1) {   // two side lines per work-group (q = 2)
    launch_march_t<T, VW, 2, MODE, FIRST, true>(c, F0, F1, O0, O1, Yv, diag, al, be);
    return;
  }
  switch (c->ms.q) {
    case 1: launch_march_t<T, VW, 1, MODE, FIRST, false>(c, F0, F1, O0, O1, Yv, diag, al, be); break;
    case 2: launch_march_t<T, VW, 2, MODE, FIRST, false>(c, F0, F1, O0, O1, Yv, diag, al, be); break;
    default: launch_march_t<T, VW, 4, MODE, FIRST, false>(c, F0, F1, O0, O1, Yv, diag, al, be); break;
  }
}

template <int MODE, bool FIRST>
static hipError_t launch_march(ope_ctx* c, const void* F0, const void* F1, void* O0, void* O1, void* Yv,
                               const double* al, const double* be) {
  if (c->prec == OPE_FP64) {
    using T = double;
    if (c->vw == 2)
      launch_march_q<T, 2, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag, al, be);
    else
      launch_march_q<T, 1, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag, al, be);
  } else {
    using T = float;
    if (c->vw == 4)
      launch_march_q<T, 4, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag32, al, be);
    else if (c->vw == 2)
      launch_march_q<T, 2, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag32, al, be);
    else
      launch_march_q<T, 1, MODE, FIRST>(c, (const T*)F0, (const T*)F1, (T*)O0, (T*)O1, (T*)Yv, c->diag32, al, be);
  }
  return hipGetLastError();
}

void march_shape(ope_ctx* c, int q_max, int mc_override, int order, int nt, int narrow, int lines) {
  MarchShape& ms = c->ms;
  ms.order = order ? 1u : 0u;
  ms.nt = nt ? 1u : 0u;
  const OpeGrid& g = c->g;
  const uint32_t NV = (uint32_t)(c->N / c->vw);
  // Column chunk of a work-group: whole rows when they have at most 32 vector
  // columns (one contiguous run of pp rows per pass, no partly idle chunk);
  // rows of up to 64 the widest of 32, 16 and 8 vector columns that divides
  // them (no idle lanes; a wide chunk streams long runs per grid point: at
  // N = 128 in FP64, 512-byte chunks sweep 1.17x faster than 128-byte ones);
  // else 8 vector columns, one 128-byte line of FP64 or FP32 per grid point
  // and work-group (at N = 512, 96^3, 32-vector chunks were 5% slower).
  // `narrow` asks for 8 vector columns at any row width.
  if (narrow) ms.ncv = NV < 8u ? NV : 8u;
  else if (NV <= 32u) ms.ncv = NV;
  else if (NV <= 64u) ms.ncv = NV % 32u == 0 ? 32u : (NV % 16u == 0 ? 16u : 8u);
  else ms.ncv = 8u;
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
  ms.ly = 1;
  ms.lpp = 1;
  const bool tile = lines && g.dim == 3 && g.m1 > 1;
  if (tile) q = 2;                 // side lines of the work-group: 2, 4 or 8 (1, 2 or 4 per pass)
  ms.q = q;
  ms.xseg = q * ms.pp;
  if (tile) {
    ms.lpp = (lines >= 3 && ms.pp >= 16) ? 4u : ((lines >= 2 && ms.pp >= 4) ? 2u : 1u);
    ms.ly = q * ms.lpp;
    ms.xseg = ms.pp / ms.lpp;
  }
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
  // automatic: at least 512 work-groups, and enough march chunks that about
  // 2.5 MB of plane data is in flight (a work-group with short rows moves
  // little per plane); one chunk when that already holds (the lock-step march
  // keeps side rows in L2)
  ms.lgroups = (ms.lines + ms.ly - 1) / ms.ly;
  const uint32_t base = ms.lgroups * ms.nxs * ms.cc;
  const double plane_bytes = (double)ms.q * ms.pp * ms.ncv * c->vw * (c->prec == OPE_FP64 ? 8.0 : 4.0);
  uint32_t mc_auto = (512u + base - 1) / base;
  const uint32_t mc_bytes = (uint32_t)(2.5 * 1048576.0 / ((double)base * plane_bytes) + 0.5);
  if (mc_bytes > mc_auto) mc_auto = mc_bytes;
  uint32_t mc = mc_override > 0 ? (uint32_t)mc_override : mc_auto;
  if (mc < 1) mc = 1;
  if (mc > ms.mlen) mc = ms.mlen;
  ms.mchunk = (ms.mlen + mc - 1) / mc;
  ms.mc = (ms.mlen + ms.mchunk - 1) / ms.mchunk;
}

int64_t march_rows(const ope_ctx* c) {
  return (int64_t)c->ms.lgroups * c->ms.nxs * c->ms.mc;
}

hipError_t launch_apply_h(ope_ctx* c, const void* X, void* Yo) {
  ProfScope ps(c, OPE_KERNEL_STENCIL);
  return launch_march<SW_APPLY, false>(c, X, nullptr, Yo, nullptr, nullptr, c->alpha, c->beta);
}

hipError_t launch_cg_pap(ope_ctx* c, const void* r, const void* pold, void* pnew, int first) {
  ProfScope ps(c, OPE_KERNEL_CG_SWEEP_A);
  if (first) return launch_march<SW_PAP, true>(c, r, pold, nullptr, pnew, nullptr, c->alpha, c->beta);
  return launch_march<SW_PAP, false>(c, r, pold, nullptr, pnew, nullptr, c->alpha, c->beta);
}

hipError_t launch_cg_update(ope_ctx* c, const void* r, const void* p, void* rnew, const double* alpha, void* y,
                            const void* pprev, const double* alpha_prev) {
  // profiled as sweep B (both forms), or the odd form alone
  ProfScope ps(c, (y && c->prof_kernel == OPE_KERNEL_CG_SWEEP_B_Y) ? OPE_KERNEL_CG_SWEEP_B_Y : OPE_KERNEL_CG_SWEEP_B);
  if (y) return launch_march<SW_UPDATE_Y, false>(c, r, p, rnew, const_cast<void*>(pprev), y, alpha, alpha_prev);
  return launch_march<SW_UPDATE, false>(c, r, p, rnew, nullptr, nullptr, alpha, c->beta);
}

hipError_t launch_y_flush(ope_ctx* c, hipStream_t s, void* y, const void* p, const double* alpha) {
  const uint64_t count = (uint64_t)c->n * (uint64_t)c->N;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((count + OPE_WG - 1) / OPE_WG, 8192);
  if (c->prec == OPE_FP64)
    hipLaunchKernelGGL((k_y_flush<double>), dim3(grid), dim3(OPE_WG), 0, s, (double*)y, (const double*)p, alpha, count,
                       (uint32_t)c->N);
  else
    hipLaunchKernelGGL((k_y_flush<float>), dim3(grid), dim3(OPE_WG), 0, s, (float*)y, (const float*)p, alpha, count,
                       (uint32_t)c->N);
  return hipGetLastError();
}

hipError_t launch_reduce_cols(ope_ctx* c, const double* part, int64_t nrows, int64_t ncols, double* out, int mode,
                              double* alpha) {
  if (!alpha) alpha = c->alpha;
  if (ncols <= 128 && nrows * ncols <= FEW_MAX) {
    const uint32_t nr = (uint32_t)nrows, nc = (uint32_t)ncols;
    switch (mode) {
      case RED_PLAIN:
        hipLaunchKernelGGL((k_reduce_few<RED_PLAIN>), dim3(1), dim3(RED_WG), 0, c->stream, part, nr, nc, out, alpha,
                           c->beta, c->rho, c->target, c->active, c->sc);
        break;
      case RED_CG_ALPHA:
        hipLaunchKernelGGL((k_reduce_few<RED_CG_ALPHA>), dim3(1), dim3(RED_WG), 0, c->stream, part, nr, nc, out,
                           alpha, c->beta, c->rho, c->target, c->active, c->sc);
        break;
      default:
        hipLaunchKernelGGL((k_reduce_few<RED_CG_BETA>), dim3(1), dim3(RED_WG), 0, c->stream, part, nr, nc, out,
                           alpha, c->beta, c->rho, c->target, c->active, c->sc);
        break;
    }
    return hipGetLastError();
  }
  const uint32_t ncg = (uint32_t)((ncols + 63) / 64);
  // first stage: about 32 rows per work-group, at most 64 work-groups per
  // column group (enough work-groups to keep HBM busy), within the stage buffer
  uint32_t S = (uint32_t)((nrows + 31) / 32);
  if (S > 64) S = 64;
  if ((int64_t)S * ncols > c->stage_cap) S = (uint32_t)(c->stage_cap / ncols);
  if (S > 1) {
    const uint32_t rps = (uint32_t)((nrows + S - 1) / S);
    S = (uint32_t)((nrows + rps - 1) / rps);
    hipLaunchKernelGGL(k_reduce_stage, dim3(ncg, S), dim3(OPE_WG), 0, c->stream, part, (uint32_t)nrows,
                       (uint32_t)ncols, rps, c->stage);
    part = c->stage;
    nrows = S;
  }
  const dim3 grid(ncg), blk(OPE_WG);
  switch (mode) {
    case RED_PLAIN:
      hipLaunchKernelGGL((k_reduce_cols<RED_PLAIN>), grid, blk, 0, c->stream, part, (uint32_t)nrows, (uint32_t)ncols,
                         out, alpha, c->beta, c->rho, c->target, c->active, c->sc);
      break;
    case RED_CG_ALPHA:
      hipLaunchKernelGGL((k_reduce_cols<RED_CG_ALPHA>), grid, blk, 0, c->stream, part, (uint32_t)nrows, (uint32_t)ncols,
                         out, alpha, c->beta, c->rho, c->target, c->active, c->sc);
      break;
    default:
      hipLaunchKernelGGL((k_reduce_cols<RED_CG_BETA>), grid, blk, 0, c->stream, part, (uint32_t)nrows, (uint32_t)ncols,
                         out, alpha, c->beta, c->rho, c->target, c->active, c->sc);
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

bool reduce_few_fits(const ope_ctx* c) {
  return c->N <= 128 && march_rows(c) * c->N <= FEW_MAX;
}

template <typename T, int VW, int Q, int MODE, bool FIRST, bool LN>
static void launch_mb(hipStream_t s, int halo, const MarchJob* jobs, uint32_t njobs, uint32_t total) {
  if (halo)
    hipLaunchKernelGGL((k_march_batched<T, VW, Q, MODE, FIRST, true, LN>), dim3(total), dim3(OPE_WG), 0, s, jobs,
                       njobs);
  else
    hipLaunchKernelGGL((k_march_batched<T, VW, Q, MODE, FIRST, false, LN>), dim3(total), dim3(OPE_WG), 0, s, jobs,
                       njobs);
}

template <typename T, int VW, int MODE, bool FIRST>
static void launch_mb_q(hipStream_t s, int q, int halo, int ln, const MarchJob* jobs, uint32_t njobs,
                        uint32_t total) {
  if (ln) {
    launch_mb<T, VW, 2, MODE, FIRST, true>(s, halo, jobs, njobs, total);
    return;
  }
  switch (q) {
    case 1: launch_mb<T, VW, 1, MODE, FIRST, false>(s, halo, jobs, njobs, total); break;
    case 2: launch_mb<T, VW, 2, MODE, FIRST, false>(s, halo, jobs, njobs, total); break;
    default: launch_mb<T, VW, 4, MODE, FIRST, false>(s, halo, jobs, njobs, total); break;
  }
}

template <int MODE, bool FIRST>
static void launch_mb_t(hipStream_t s, int prec, int vw, int q, int halo, int ln, const MarchJob* jobs,
                        uint32_t njobs, uint32_t total) {
  if (prec == OPE_FP64) {
    if (vw == 2) launch_mb_q<double, 2, MODE, FIRST>(s, q, halo, ln, jobs, njobs, total);
    else launch_mb_q<double, 1, MODE, FIRST>(s, q, halo, ln, jobs, njobs, total);
  } else {
    if (vw == 4) launch_mb_q<float, 4, MODE, FIRST>(s, q, halo, ln, jobs, njobs, total);
    else if (vw == 2) launch_mb_q<float, 2, MODE, FIRST>(s, q, halo, ln, jobs, njobs, total);
    else launch_mb_q<float, 1, MODE, FIRST>(s, q, halo, ln, jobs, njobs, total);
  }
}

hipError_t launch_march_batched(hipStream_t s, int prec, int vw, int q, int halo, int ln, int mode, int first,
                                const MarchJob* jobs, uint32_t njobs, uint32_t total_wgs) {
  if (njobs == 0 || total_wgs == 0) return hipSuccess;
  if (mode == SW_PAP) {
    if (first) launch_mb_t<SW_PAP, true>(s, prec, vw, q, halo, ln, jobs, njobs, total_wgs);
    else launch_mb_t<SW_PAP, false>(s, prec, vw, q, halo, ln, jobs, njobs, total_wgs);
  } else if (mode == SW_UPDATE_Y) {
    launch_mb_t<SW_UPDATE_Y, false>(s, prec, vw, q, halo, ln, jobs, njobs, total_wgs);
  } else {
    launch_mb_t<SW_UPDATE, false>(s, prec, vw, q, halo, ln, jobs, njobs, total_wgs);   // no first-iteration form
  }
  return hipGetLastError();
}

hipError_t launch_reduce_batched(hipStream_t s, int mode, int par, const ReduceJob* jobs, uint32_t njobs) {
  if (njobs == 0) return hipSuccess;
  if (mode == RED_CG_ALPHA)
    hipLaunchKernelGGL((k_reduce_batched<RED_CG_ALPHA>), dim3(njobs), dim3(RED_WG), 0, s, jobs, (uint32_t)par);
  else
    hipLaunchKernelGGL((k_reduce_batched<RED_CG_BETA>), dim3(njobs), dim3(RED_WG), 0, s, jobs, (uint32_t)par);
  return hipGetLastError();
}

hipError_t launch_gather_flags(hipStream_t s, const ReduceJob* jobs, uint32_t njobs) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_flags, dim3(njobs), dim3(OPE_WG), 0, s, jobs);
  return hipGetLastError();
}
