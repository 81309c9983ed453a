// Dense tall-skinny contractions of the step on the FP64 matrix cores (gfx950).
//
//  * Inner matrices <X, Y> = X^T Y over the n grid rows (the Grams
//    <U,U>, <U,HU>, <U,GU>, <GU,GU> used by Steps 2-3 of Section 4.1).
//  * Row-block products Out = beta C + X0 M0 + X1 M1 with small N x N
//    matrices (the residual HU - U Lam, the warm start U Lam^{-1}, and Step 4's
//    update U (I - tau A) + GU (tau B)).
//
// Both use v_mfma_f64_16x16x4f64.  Operand layout of that instruction for lane
// l of a wavefront: the A operand (16 x 4) supplies A[l % 16][l / 16], the B
// operand (4 x 16) supplies B[l / 16][l % 16], and the 16 x 16 accumulator
// holds D[l / 16 + 4 r][l % 16] in its r-th element.
//
// For the Gram the contraction index is the grid row, so a lane loads
// X[row0 + l/16][i0 + l%16]: four rows of 16 consecutive orbitals per load,
// straight from global memory with no LDS staging.  Split-K over rows writes
// one N x N partial per split; a fixed-order column reduction follows, so the
// result is bitwise reproducible.
#include "ope_internal.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Gram: work-group = 4 waves in a 2 x 2 arrangement over a 64 x 64 output
// tile; each wave owns a 32 x 32 sub-tile (2 x 2 MFMA blocks).
constexpr int GT = 64;      // work-group output tile edge
constexpr int GW = 32;      // wave output tile edge

__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A, uint64_t lda, uint32_t na,
                                              const double* __restrict__ B, uint64_t ldb, uint32_t nb,
                                              uint32_t rows, uint32_t rows_per_split, double* __restrict__ part) {
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t i_base = blockIdx.y * GT + (wave >> 1) * GW;
  const uint32_t j_base = blockIdx.x * GT + (wave & 1u) * GW;
  const uint32_t ks = blockIdx.z;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  const uint32_t r0 = ks * rows_per_split;
  const uint32_t r1 = min(rows, r0 + rows_per_split);
  const bool ia0 = i_base + ci < na, ia1 = i_base + 16 + ci < na;
  const bool jb0 = j_base + ci < nb, jb1 = j_base + 16 + ci < nb;
  if (i_base < na && j_base < nb) {
#pragma unroll 4
    for (uint32_t p = r0; p < r1; p += 4) {
      const uint32_t row = p + kr;
      const bool rok = row < r1;
      const double* ar = A + (uint64_t)row * lda + i_base + ci;
      const double* br = B + (uint64_t)row * ldb + j_base + ci;
      const double a0 = (rok && ia0) ? ar[0] : 0.0;
      const double a1 = (rok && ia1) ? ar[16] : 0.0;
      const double b0 = (rok && jb0) ? br[0] : 0.0;
      const double b1 = (rok && jb1) ? br[16] : 0.0;
      acc[0][0] = mfma16(a0, b0, acc[0][0]);
      acc[0][1] = mfma16(a0, b1, acc[0][1]);
      acc[1][0] = mfma16(a1, b0, acc[1][0]);
      acc[1][1] = mfma16(a1, b1, acc[1][1]);
    }
  }
  double* out = part + (uint64_t)ks * na * nb;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = i_base + a * 16 + kr + 4 * r;
        const uint32_t j = j_base + b * 16 + ci;
        if (i < na && j < nb) out[(uint64_t)i * nb + j] = acc[a][b][r];
      }
}

// Row-block products Out = cbeta Cm + ascale (X0 M0 + X1 M1): work-group = 4 waves, 2 (rows) x 2 (columns); a wave
// owns 32 rows x 64 columns (2 x 4 MFMA blocks), the work-group 64 x 128.
constexpr int RT = 64;      // rows per work-group tile
constexpr int CT = 128;     // columns per work-group tile

template <int NSRC>
__global__ __launch_bounds__(256) void k_rowmm(const double* X0, const double* __restrict__ M0,
                                               const double* X1, const double* __restrict__ M1,
                                               const double* Cm, double cbeta, double ascale, double* Out, uint32_t n,
                                               uint32_t N, int want_colsq, int predicated,
                                               const OpeScalars* __restrict__ sc, double* __restrict__ part) {
  __shared__ double colsq[2][CT];
  if (predicated && sc->err != 0) return;        // a failed small solve leaves the block untouched
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t wr = wave >> 1, wc = wave & 1u;
  const uint32_t row_base = blockIdx.x * RT + wr * 32;
  const uint32_t col_base = blockIdx.y * CT + wc * 64;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  v4d acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

#pragma unroll
  for (int s = 0; s < NSRC; ++s) {
    const double* X = s == 0 ? X0 : X1;
    const double* M = s == 0 ? M0 : M1;
    for (uint32_t k = 0; k < N; k += 4) {
      const uint32_t kk = k + kr;                  // B operand row / A operand column
      const bool kok = kk < N;
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const uint32_t row = row_base + a * 16 + ci;
        av[a] = (kok && row < n) ? X[(uint64_t)row * N + kk] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t col = col_base + b * 16 + ci;
        bv[b] = (kok && col < N) ? M[(uint64_t)kk * N + col] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
    }
  }
  // Out may alias X0 (in-place Step 4): every wave of the tile has finished
  // reading its rows before any wave writes.
  __syncthreads();
  double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t row = row_base + a * 16 + kr + 4 * r;
        const uint32_t col = col_base + b * 16 + ci;
        if (row < n && col < N) {
          const uint64_t o = (uint64_t)row * N + col;
          double v = ascale * acc[a][b][r];
          if (cbeta != 0.0) v += cbeta * Cm[o];
          Out[o] = v;
          sq[b] += v * v;
        }
      }
  if (!want_colsq) return;
  // per-column sums over the tile's rows: lanes l, l^16, l^32, l^48 share a column
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    sq[b] += __shfl_xor(sq[b], 16);
    sq[b] += __shfl_xor(sq[b], 32);
  }
  if (kr == 0) {
#pragma unroll
    for (int b = 0; b < 4; ++b) colsq[wr][wc * 64 + b * 16 + ci] = sq[b];
  }
  __syncthreads();
  if (threadIdx.x < CT) {
    const uint32_t col = blockIdx.y * CT + threadIdx.x;
    if (col < N) part[(uint64_t)blockIdx.x * N + col] = colsq[0][threadIdx.x] + colsq[1][threadIdx.x];
  }
}

}  // namespace

hipError_t launch_gram(ope_ctx* c, const double* A, int64_t lda, int na, const double* B, int64_t ldb, int nb,
                       int64_t rows, double* out) {
  const uint32_t ti = (uint32_t)((na + GT - 1) / GT), tj = (uint32_t)((nb + GT - 1) / GT);
  // about 1024 work-groups in total, within the partial buffer
  int64_t ks = 1024 / (int64_t)(ti * tj);
  if (ks < 1) ks = 1;
  const int64_t max_ks = c->part_cap / ((int64_t)na * nb);
  if (ks > max_ks) ks = max_ks;
  if (ks < 1) return hipErrorInvalidValue;
  int64_t rps = (rows + ks - 1) / ks;
  rps = (rps + 3) & ~int64_t(3);
  if (rps < 4) rps = 4;
  ks = (rows + rps - 1) / rps;
  if (ks < 1) ks = 1;
  {
    ProfScope ps(c, OPE_KERNEL_GRAM);
    hipLaunchKernelGGL(k_gram, dim3(tj, ti, (uint32_t)ks), dim3(256), 0, c->stream, A, (uint64_t)lda, (uint32_t)na, B,
                       (uint64_t)ldb, (uint32_t)nb, (uint32_t)rows, (uint32_t)rps, c->part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_cols(c, c->part, ks, (int64_t)na * nb, out, RED_PLAIN);
}

hipError_t launch_rowmm(ope_ctx* c, const double* X0, const double* M0, const double* X1, const double* M1,
                        const double* Cm, double cbeta, double ascale, double* Out, int want_colsq, int predicated,
                        int64_t* nparts) {
  const uint32_t n = (uint32_t)c->n, N = (uint32_t)c->N;
  const uint32_t gr = (n + RT - 1) / RT, gc = (N + CT - 1) / CT;
  if (gc != 1 && (Out == X0 || Out == X1)) return hipErrorInvalidValue;  // in place needs one column tile
  if (want_colsq && (int64_t)gr * N > c->part_cap) return hipErrorInvalidValue;
  ProfScope ps(c, OPE_KERNEL_ROWMM);
  if (X1)
    hipLaunchKernelGGL((k_rowmm<2>), dim3(gr, gc), dim3(256), 0, c->stream, X0, M0, X1, M1, Cm, cbeta, ascale, Out, n, N,
                       want_colsq, predicated, c->sc, c->part);
  else
    hipLaunchKernelGGL((k_rowmm<1>), dim3(gr, gc), dim3(256), 0, c->stream, X0, M0, X1, M1, Cm, cbeta, ascale, Out, n, N,
                       want_colsq, predicated, c->sc, c->part);
  if (nparts) *nparts = gr;
  return hipGetLastError();
}
