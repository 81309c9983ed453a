// Dense tall-skinny contractions of the step on the gfx950 matrix cores.
//
//  * Inner matrices <X, Y> = X^T Y over the n grid rows (the Grams
//    <U,U>, <U,HU>, <U,GU>, <GU,GU> used by Steps 2-3 of Section 4.1).
//  * Row-block products Out = cbeta C + ascale (X0 M0 + X1 M1) with small N x N
//    matrices (the residual HU - U Lam, the warm start U Lam^{-1}, Step 4's
//    update, and in mixed precision the projection Y - U <U,Y>).
//
// Three arithmetic kinds, chosen per call:
//   MK_F64   v_mfma_f64_16x16x4f64 on FP64 (inputs FP64, or FP32 widened)
//   MK_F32   v_mfma_f32_16x16x4f32 on FP32 inputs, FP32 accumulation
//   MK_BF16  v_mfma_f32_16x16x32_bf16: FP32 inputs rounded to BF16, FP32 accumulation
// Operand layout for lane l (checked on the device): the A operand supplies
// A[l % 16][k] and the B operand B[k][l % 16], with k = l / 16 (16x16x4) or
// k = 8 (l / 16) + e, e = 0..7 (16x16x32).  The 16 x 16 accumulator holds
// D[l / 16 + 4 r][l % 16] in element r for the FP64 instruction and
// D[4 (l / 16) + r][l % 16] for the FP32 and BF16 instructions.
//
// For the Gram the contraction index is the grid row, so a lane reads
// X[row0 + k][i0 + l%16]: rows of 16 consecutive orbitals.  Split-K over rows
// writes one partial per split (in FP64); a fixed-order column reduction
// follows, so results are bitwise reproducible.
//
// Kernels by shape: wide operands (>= 128 columns, 16-byte rows) stage
// panels in LDS with 128 x 128 work-group tiles (k_gram_lds, k_rowmm_lds);
// narrow blocks (<= 32 columns) use k_gram_narrow (the four waves split the
// rows of one 32 x 32 tile) and k_rowmm_narrow (128-row tiles through LDS);
// the rest read their operands straight from global memory (k_gram,
// k_gram_wide, k_rowmm).
#include "ope_internal.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int KIND> struct Mk;
template <> struct Mk<MK_F64> {
  using acc_t = v4d;
  static constexpr int KSTEP = 4;       // contraction length per instruction
  static constexpr int KPL = 1;         // contraction elements per lane
  __device__ static uint32_t drow(uint32_t kr, int r) { return kr + 4u * (uint32_t)r; }
};
template <> struct Mk<MK_F32> {
  using acc_t = v4f;
  static constexpr int KSTEP = 4;
  static constexpr int KPL = 1;
  __device__ static uint32_t drow(uint32_t kr, int r) { return 4u * kr + (uint32_t)r; }
};
template <> struct Mk<MK_BF16> {
  using acc_t = v4f;
  static constexpr int KSTEP = 32;
  static constexpr int KPL = 8;
  __device__ static uint32_t drow(uint32_t kr, int r) { return 4u * kr + (uint32_t)r; }
};

// Contraction indices per LDS panel of the staged kernels: at least 16, and a
// whole MFMA contraction step.
template <int KIND> struct PanelRows { static constexpr int KC = Mk<KIND>::KSTEP < 16 ? 16 : Mk<KIND>::KSTEP; };

// One MFMA with operands given as KPL values per lane (in the input type).
template <int KIND, typename TI>
__device__ __forceinline__ typename Mk<KIND>::acc_t mma(const TI (&a)[Mk<KIND>::KPL], const TI (&b)[Mk<KIND>::KPL],
                                                        typename Mk<KIND>::acc_t c) {
  if constexpr (KIND == MK_F64) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[0], (double)b[0], c, 0, 0, 0);
  } else if constexpr (KIND == MK_F32) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[0], (float)b[0], c, 0, 0, 0);
  } else {
    v8bf av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      av[e] = (__bf16)(float)a[e];
      bv[e] = (__bf16)(float)b[e];
    }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
}

template <typename V>
__device__ __forceinline__ V zero_acc() {
  V z;
#pragma unroll
  for (int r = 0; r < 4; ++r) z[r] = 0;
  return z;
}

// Gram: work-group = 4 waves in a 2 x 2 arrangement over a 64 x 64 output
// tile; each wave owns a 32 x 32 sub-tile (2 x 2 MFMA blocks).
constexpr int GT = 64;      // work-group output tile edge
constexpr int GW = 32;      // wave output tile edge

template <typename TI, int KIND>
__global__ __launch_bounds__(256) void k_gram(const TI* __restrict__ A, uint64_t lda, uint32_t na,
                                              const TI* __restrict__ B, uint64_t ldb, uint32_t nb,
                                              uint32_t rows, uint32_t rows_per_split, double* __restrict__ part) {
  using M = Mk<KIND>;
  using acc_t = typename M::acc_t;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t i_base = blockIdx.y * GT + (wave >> 1) * GW;
  const uint32_t j_base = blockIdx.x * GT + (wave & 1u) * GW;
  const uint32_t ks = blockIdx.z;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = zero_acc<acc_t>();
  const uint32_t r0 = ks * rows_per_split;
  const uint32_t r1 = min(rows, r0 + rows_per_split);
  const bool ia0 = i_base + ci < na, ia1 = i_base + 16 + ci < na;
  const bool jb0 = j_base + ci < nb, jb1 = j_base + 16 + ci < nb;
  if (i_base < na && j_base < nb) {
#pragma unroll 2
    for (uint32_t p = r0; p < r1; p += M::KSTEP) {
      TI a0[M::KPL], a1[M::KPL], b0[M::KPL], b1[M::KPL];
#pragma unroll
      for (int e = 0; e < M::KPL; ++e) {
        const uint32_t row = p + kr * M::KPL + e;
        const bool rok = row < r1;
        const TI* ar = A + (uint64_t)row * lda + i_base + ci;
        const TI* br = B + (uint64_t)row * ldb + j_base + ci;
        a0[e] = (rok && ia0) ? ar[0] : TI(0);
        a1[e] = (rok && ia1) ? ar[16] : TI(0);
        b0[e] = (rok && jb0) ? br[0] : TI(0);
        b1[e] = (rok && jb1) ? br[16] : TI(0);
      }
      acc[0][0] = mma<KIND, TI>(a0, b0, acc[0][0]);
      acc[0][1] = mma<KIND, TI>(a0, b1, acc[0][1]);
      acc[1][0] = mma<KIND, TI>(a1, b0, acc[1][0]);
      acc[1][1] = mma<KIND, TI>(a1, b1, acc[1][1]);
    }
  }
  double* out = part + (uint64_t)ks * na * nb;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = i_base + a * 16 + M::drow(kr, r);
        const uint32_t j = j_base + b * 16 + ci;
        if (i < na && j < nb) out[(uint64_t)i * nb + j] = (double)acc[a][b][r];
      }
}

// Wide Grams (both sides >= 128 columns, FP32 and BF16 kinds): work-group tile
// 128 x 128, each wave a 64 x 64 sub-tile (4 x 4 MFMA blocks), so every
// operand load feeds four MFMAs instead of two.
constexpr int GT2 = 128;
constexpr int GW2 = 64;

template <typename TI, int KIND>
__global__ __launch_bounds__(256) void k_gram_wide(const TI* __restrict__ A, uint64_t lda, uint32_t na,
                                                   const TI* __restrict__ B, uint64_t ldb, uint32_t nb,
                                                   uint32_t rows, uint32_t rows_per_split, double* __restrict__ part) {
  using M = Mk<KIND>;
  using acc_t = typename M::acc_t;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t i_base = blockIdx.y * GT2 + (wave >> 1) * GW2;
  const uint32_t j_base = blockIdx.x * GT2 + (wave & 1u) * GW2;
  const uint32_t ks = blockIdx.z;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero_acc<acc_t>();
  const uint32_t r0 = ks * rows_per_split;
  const uint32_t r1 = min(rows, r0 + rows_per_split);
  bool iok[4], jok[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    iok[a] = i_base + a * 16 + ci < na;
    jok[a] = j_base + a * 16 + ci < nb;
  }
  if (i_base < na && j_base < nb) {
    for (uint32_t p = r0; p < r1; p += M::KSTEP) {
      TI av[4][M::KPL], bv[4][M::KPL];
#pragma unroll
      for (int e = 0; e < M::KPL; ++e) {
        const uint32_t row = p + kr * M::KPL + e;
        const bool rok = row < r1;
        const TI* ar = A + (uint64_t)row * lda + i_base + ci;
        const TI* br = B + (uint64_t)row * ldb + j_base + ci;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          av[a][e] = (rok && iok[a]) ? ar[16 * a] : TI(0);
          bv[a][e] = (rok && jok[a]) ? br[16 * a] : TI(0);
        }
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mma<KIND, TI>(av[a], bv[b], acc[a][b]);
    }
  }
  double* out = part + (uint64_t)ks * na * nb;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = i_base + a * 16 + M::drow(kr, r);
        const uint32_t j = j_base + b * 16 + ci;
        if (i < na && j < nb) out[(uint64_t)i * nb + j] = (double)acc[a][b][r];
      }
}

// Narrow Grams (both sides at most 32 columns): one 32 x 32 output tile (2 x 2
// MFMA blocks) per work-group, and the four waves split the work-group's rows
// (wave w takes contraction steps w, w + 4, ...) instead of sharing a 64 x 64
// tile that such a Gram would leave three quarters idle.  The waves' tiles are
// summed in LDS in wave order.
template <typename TI, int KIND>
__global__ __launch_bounds__(256) void k_gram_narrow(const TI* __restrict__ A, uint64_t lda, uint32_t na,
                                                     const TI* __restrict__ B, uint64_t ldb, uint32_t nb,
                                                     uint32_t rows, uint32_t rows_per_split,
                                                     double* __restrict__ part) {
  using M = Mk<KIND>;
  using acc_t = typename M::acc_t;
  __shared__ double red[3][2][2][4][64];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t ks = blockIdx.x;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = zero_acc<acc_t>();
  const uint32_t r0 = ks * rows_per_split;
  const uint32_t r1 = min(rows, r0 + rows_per_split);
  const bool ia0 = ci < na, ia1 = 16 + ci < na;
  const bool jb0 = ci < nb, jb1 = 16 + ci < nb;
#pragma unroll 4
  for (uint32_t p = r0 + wave * M::KSTEP; p < r1; p += 4 * M::KSTEP) {
    TI a0[M::KPL], a1[M::KPL], b0[M::KPL], b1[M::KPL];
#pragma unroll
    for (int e = 0; e < M::KPL; ++e) {
      const uint32_t row = p + kr * M::KPL + e;
      const bool rok = row < r1;
      const TI* ar = A + (uint64_t)row * lda + ci;
      const TI* br = B + (uint64_t)row * ldb + ci;
      a0[e] = (rok && ia0) ? ar[0] : TI(0);
      a1[e] = (rok && ia1) ? ar[16] : TI(0);
      b0[e] = (rok && jb0) ? br[0] : TI(0);
      b1[e] = (rok && jb1) ? br[16] : TI(0);
    }
    acc[0][0] = mma<KIND, TI>(a0, b0, acc[0][0]);
    acc[0][1] = mma<KIND, TI>(a0, b1, acc[0][1]);
    acc[1][0] = mma<KIND, TI>(a1, b0, acc[1][0]);
    acc[1][1] = mma<KIND, TI>(a1, b1, acc[1][1]);
  }
  if (wave > 0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave - 1][a][b][r][lane] = (double)acc[a][b][r];
  }
  __syncthreads();
  if (wave != 0) return;
  double* out = part + (uint64_t)ks * na * nb;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = a * 16 + M::drow(kr, r);
        const uint32_t j = b * 16 + ci;
        const double v = (double)acc[a][b][r] + red[0][a][b][r][lane] + red[1][a][b][r][lane] + red[2][a][b][r][lane];
        if (i < na && j < nb) out[(uint64_t)i * nb + j] = v;
      }
}

// Row-block products Out = cbeta Cm + ascale (X0 M0 + X1 M1).  Work-group =
// 4 waves, 2 (rows) x 2 (columns); a wave owns 32 rows x 64 columns (2 x 4
// MFMA blocks), the work-group 64 x 128.  TI is the type of X, M, Cm and Out.
// Predication of the row-block products (bits of `predicated`): ROWMM_IF_OK
// skips the launch when the step's device error flag is set (a failed small
// solve leaves the block untouched), ROWMM_IF_RENORM unless the drift check
// asked for a re-normalisation.
__device__ __forceinline__ bool rowmm_skip(int predicated, const OpeScalars* __restrict__ sc) {
  return ((predicated & ROWMM_IF_OK) && sc->err != 0) || ((predicated & ROWMM_IF_RENORM) && sc->renorm == 0);
}

constexpr int RT = 64;      // rows per work-group tile
constexpr int CT = 128;     // columns per work-group tile

template <typename TI, int KIND, int NSRC>
__global__ __launch_bounds__(256) void k_rowmm(const TI* X0, const TI* __restrict__ M0, const TI* X1,
                                               const TI* __restrict__ M1, const TI* Cm, double cbeta, double ascale,
                                               TI* Out, uint32_t n, uint32_t N, int want_colsq, int predicated,
                                               const OpeScalars* __restrict__ sc, double* __restrict__ part) {
  using MK = Mk<KIND>;
  using acc_t = typename MK::acc_t;
  __shared__ double colsq[2][CT];
  if (rowmm_skip(predicated, sc)) return;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t wr = wave >> 1, wc = wave & 1u;
  const uint32_t row_base = blockIdx.x * RT + wr * 32;
  const uint32_t col_base = blockIdx.y * CT + wc * 64;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  acc_t acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero_acc<acc_t>();

#pragma unroll
  for (int s = 0; s < NSRC; ++s) {
    const TI* X = s == 0 ? X0 : X1;
    const TI* M = s == 0 ? M0 : M1;
    for (uint32_t k = 0; k < N; k += MK::KSTEP) {
      TI av[2][MK::KPL], bv[4][MK::KPL];
#pragma unroll
      for (int e = 0; e < MK::KPL; ++e) {
        const uint32_t kk = k + kr * MK::KPL + e;   // contraction index held by this lane
        const bool kok = kk < N;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const uint32_t row = row_base + a * 16 + ci;
          av[a][e] = (kok && row < n) ? X[(uint64_t)row * N + kk] : TI(0);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint32_t col = col_base + b * 16 + ci;
          bv[b][e] = (kok && col < N) ? M[(uint64_t)kk * N + col] : TI(0);
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mma<KIND, TI>(av[a], bv[b], acc[a][b]);
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
        const uint32_t row = row_base + a * 16 + MK::drow(kr, r);
        const uint32_t col = col_base + b * 16 + ci;
        if (row < n && col < N) {
          const uint64_t o = (uint64_t)row * N + col;
          TI v = (TI)(ascale * (double)acc[a][b][r]);
          if (cbeta != 0.0) v += (TI)cbeta * Cm[o];
          Out[o] = v;
          sq[b] += (double)v * (double)v;
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

// Narrow row-block products (N <= 32): work-group tile 128 rows x N columns,
// each wave 32 rows x 32 columns (2 x 2 MFMA blocks).  The tile's rows of X,
// of Cm and of the result are contiguous in memory, so they pass through LDS
// and every global access is a run of whole rows (the MFMA operand pattern
// itself reads 16 rows x 4 values per instruction, 16 cache lines).  Sources
// are staged one after the other; the LDS row stride is odd, so the 16 rows of
// an operand read fall in distinct banks.
constexpr int RTN = 128;    // rows per work-group tile
constexpr int LDXN = 33;    // LDS row stride of the staged tile

template <typename TI, int KIND, int NSRC>
__global__ __launch_bounds__(256) void k_rowmm_narrow(const TI* X0, const TI* __restrict__ M0, const TI* X1,
                                                      const TI* __restrict__ M1, const TI* Cm, double cbeta,
                                                      double ascale, TI* Out, uint32_t n, uint32_t N, int want_colsq,
                                                      int predicated, const OpeScalars* __restrict__ sc,
                                                      double* __restrict__ part) {
  using MK = Mk<KIND>;
  using acc_t = typename MK::acc_t;
  __shared__ TI xs[RTN * LDXN];
  __shared__ TI ms[32 * 32];
  __shared__ double colsq[8][32];
  if (rowmm_skip(predicated, sc)) return;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  const uint32_t row0 = blockIdx.x * RTN;
  const uint32_t tc = threadIdx.x & 31u, tg = threadIdx.x >> 5;    // column and row group of the copies
  const uint32_t wr = wave * 32u;                                  // the wave's first row in the tile
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = zero_acc<acc_t>();
#pragma unroll
  for (int s = 0; s < NSRC; ++s) {
    const TI* X = s == 0 ? X0 : X1;
    const TI* M = s == 0 ? M0 : M1;
    if (s > 0) __syncthreads();                  // the previous source's operands are consumed
#pragma unroll 4
    for (uint32_t u = 0; u < RTN / 8; ++u) {
      const uint32_t r = tg + 8u * u, gr = row0 + r;
      xs[r * LDXN + tc] = (gr < n && tc < N) ? X[(uint64_t)gr * N + tc] : TI(0);
    }
    for (uint32_t e = threadIdx.x; e < 32u * 32u; e += 256u) {
      const uint32_t kk = e >> 5, col = e & 31u;
      ms[e] = (kk < N && col < N) ? M[(uint64_t)kk * N + col] : TI(0);
    }
    __syncthreads();
    // contraction over the zero-padded 32 indices, in whole MFMA steps
    for (uint32_t k = 0; k < N; k += MK::KSTEP) {
      TI av[2][MK::KPL], bv[2][MK::KPL];
#pragma unroll
      for (int e = 0; e < MK::KPL; ++e) {
        const uint32_t kk = k + kr * MK::KPL + e;
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a][e] = xs[(wr + a * 16 + ci) * LDXN + kk];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b][e] = ms[kk * 32 + b * 16 + ci];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mma<KIND, TI>(av[a], bv[b], acc[a][b]);
    }
  }
  // every operand read of the tile is done before the result replaces it
  // (Out may alias X0: in-place Step 4)
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        xs[(wr + a * 16 + MK::drow(kr, r)) * LDXN + b * 16 + ci] = (TI)(ascale * (double)acc[a][b][r]);
  __syncthreads();
  double sq = 0.0;
#pragma unroll 4
  for (uint32_t u = 0; u < RTN / 8; ++u) {
    const uint32_t r = tg + 8u * u, gr = row0 + r;
    if (gr < n && tc < N) {
      const uint64_t o = (uint64_t)gr * N + tc;
      TI v = xs[r * LDXN + tc];
      if (cbeta != 0.0) v += (TI)cbeta * Cm[o];
      Out[o] = v;
      sq += (double)v * (double)v;
    }
  }
  if (!want_colsq) return;
  colsq[tg][tc] = sq;
  __syncthreads();
  if (threadIdx.x < N) {
    double t = 0.0;
#pragma unroll
    for (int g = 0; g < 8; ++g) t += colsq[g][threadIdx.x];
    part[(uint64_t)blockIdx.x * N + threadIdx.x] = t;
  }
}

// Row-block products from LDS (N a multiple of the 16-byte chunk, aligned
// blocks): work-group tile RTW rows x 128 columns, each wave RTW/2 x 64
// (RTW/32 x 4 MFMA blocks; RTW = 128, or 64 for the FP64 kind).  Panels of KC contraction indices are staged in LDS, double
// buffered: X's rows (read as 16-byte chunks) are stored transposed, Xt[k][row],
// so that the MFMA operand reads of both panels are contiguous across lanes,
// and the KC rows of M beside them.  M is read once per work-group instead of
// once per wave and 64-row tile.
constexpr int RT2 = 128;    // rows per work-group tile
constexpr int RT2H = 64;    // rows per work-group tile of the FP64 kind

template <typename TI, int KIND, int NSRC, int RTW>
__global__ __launch_bounds__(256, RTW == RT2H ? 3 : 2) void k_rowmm_lds(const TI* X0, const TI* __restrict__ M0, const TI* X1,
                                                   const TI* __restrict__ M1, const TI* Cm, double cbeta,
                                                   double ascale, TI* Out, uint32_t n, uint32_t N, int want_colsq,
                                                   int predicated, const OpeScalars* __restrict__ sc,
                                                   double* __restrict__ part) {
  using MK = Mk<KIND>;
  using acc_t = typename MK::acc_t;
  constexpr int KC = PanelRows<KIND>::KC;
  constexpr int VPC = 16 / (int)sizeof(TI);
  constexpr int XC = KC / VPC;                        // chunks per X row and panel
  constexpr int XCT = RTW * XC / 256;                 // X chunks per thread
  constexpr int AR = RTW / 32;                        // 16-row MFMA blocks per wave (a wave spans RTW / 2 rows)
  constexpr int MCR = CT / VPC;                       // chunks per M panel row
  constexpr int MCT = KC * MCR / 256;                 // M chunks per thread
  static_assert(XCT * 256 == RTW * XC && MCT * 256 == KC * MCR, "panel chunks must divide the work-group");
  typedef unsigned int Chunk __attribute__((ext_vector_type(4)));
  union ChunkV {
    Chunk c;
    TI v[VPC];
  };
  __shared__ __align__(16) TI xt[2][KC][RTW];
  __shared__ __align__(16) TI mp[2][KC][CT];
  __shared__ double colsq[2][CT];
  if (rowmm_skip(predicated, sc)) return;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t wr = wave >> 1, wc = wave & 1u;
  const uint32_t row0 = blockIdx.x * RTW, col0 = blockIdx.y * CT;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  acc_t acc[AR][4];
#pragma unroll
  for (int a = 0; a < AR; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero_acc<acc_t>();
  const uint32_t kpan = (N + KC - 1) / KC;          // panels per source
  const uint32_t npan = NSRC * kpan;
  ChunkV cx[XCT], cm[MCT];
  const Chunk z = {0u, 0u, 0u, 0u};
  auto load = [&](uint32_t t) {
    const TI* X = t < kpan ? X0 : X1;
    const TI* M = t < kpan ? M0 : M1;
    const uint32_t k0 = (t < kpan ? t : t - kpan) * KC;
#pragma unroll
    for (int u = 0; u < XCT; ++u) {
      const uint32_t c = threadIdx.x + 256u * u;
      const uint32_t r = c / XC, kc = (c % XC) * VPC;
      const uint32_t gr = row0 + r;
      cx[u].c = (gr < n && k0 + kc < N) ? *reinterpret_cast<const Chunk*>(X + (uint64_t)gr * N + k0 + kc) : z;
    }
#pragma unroll
    for (int u = 0; u < MCT; ++u) {
      const uint32_t c = threadIdx.x + 256u * u;
      const uint32_t kk = c / MCR, col = (c % MCR) * VPC;
      cm[u].c = (k0 + kk < N && col0 + col < N) ? *reinterpret_cast<const Chunk*>(M + (uint64_t)(k0 + kk) * N + col0 + col)
                                               : z;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < XCT; ++u) {
      const uint32_t c = threadIdx.x + 256u * u;
      const uint32_t r = c / XC, kc = (c % XC) * VPC;
#pragma unroll
      for (int e = 0; e < VPC; ++e) xt[buf][kc + e][r] = cx[u].v[e];
    }
#pragma unroll
    for (int u = 0; u < MCT; ++u) {
      const uint32_t c = threadIdx.x + 256u * u;
      const uint32_t kk = c / MCR, col = (c % MCR) * VPC;
      *reinterpret_cast<Chunk*>(&mp[buf][kk][col]) = cm[u].c;
    }
  };
  load(0);
  store(0);
  __syncthreads();
  for (uint32_t t = 0; t < npan; ++t) {
    const int buf = (int)(t & 1u);
    if (t + 1 < npan) load(t + 1);
#pragma unroll
    for (int kk = 0; kk < KC / MK::KSTEP; ++kk) {
      TI av[AR][MK::KPL], bv[4][MK::KPL];
#pragma unroll
      for (int e = 0; e < MK::KPL; ++e) {
        const uint32_t k = kk * MK::KSTEP + kr * MK::KPL + e;
#pragma unroll
        for (int a = 0; a < AR; ++a) av[a][e] = xt[buf][k][wr * (RTW / 2) + a * 16 + ci];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b][e] = mp[buf][k][wc * 64 + b * 16 + ci];
      }
#pragma unroll
      for (int a = 0; a < AR; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mma<KIND, TI>(av[a], bv[b], acc[a][b]);
    }
    if (t + 1 < npan) store(buf ^ 1);
    __syncthreads();
  }
  // every wave has read all of its rows (the last panel is in LDS) before any
  // wave writes: Out may alias X0 (in-place Step 4)
  double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < AR; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t row = row0 + wr * (RTW / 2) + a * 16 + MK::drow(kr, r);
        const uint32_t col = col0 + wc * 64 + b * 16 + ci;
        if (row < n && col < N) {
          const uint64_t o = (uint64_t)row * N + col;
          TI v = (TI)(ascale * (double)acc[a][b][r]);
          if (cbeta != 0.0) v += (TI)cbeta * Cm[o];
          Out[o] = v;
          sq[b] += (double)v * (double)v;
        }
      }
  if (!want_colsq) return;
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
    const uint32_t col = col0 + threadIdx.x;
    if (col < N) part[(uint64_t)blockIdx.x * N + col] = colsq[0][threadIdx.x] + colsq[1][threadIdx.x];
  }
}

// Square FP64 products of N x N matrices (the small solves for large N):
// D = alpha op(A) op(B) + beta C + gamma I, op = transpose when ta / tb is
// set.  Work-group tile 64 x 64 (4 waves of 32 x 32), operands straight from
// global memory (the matrices are L2-resident).  When res is given, the
// work-group adds sum over its tile of (delta_ij - D_ij)^2 into res[block]
// (the Newton-Schulz residual |I - M X|_F^2).  A non-zero *skip makes the
// launch a no-op (device-side convergence of an iteration).
__global__ __launch_bounds__(256) void k_sqmm(const double* __restrict__ A, int ta, const double* __restrict__ B,
                                              int tb, const double* __restrict__ C, double alpha, double beta,
                                              double gamma, double* __restrict__ D, uint32_t N,
                                              const int32_t* __restrict__ skip, double* __restrict__ res) {
  using MK = Mk<MK_F64>;
  __shared__ double red[256];
  if (skip && *skip) return;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t i_base = blockIdx.y * 64 + (wave >> 1) * 32;
  const uint32_t j_base = blockIdx.x * 64 + (wave & 1u) * 32;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = zero_acc<v4d>();
  for (uint32_t k0 = 0; k0 < N; k0 += 4) {
    const uint32_t k = k0 + kr;
    double av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const uint32_t i = i_base + a * 16 + ci;
      av[a] = (k < N && i < N) ? (ta ? A[(uint64_t)k * N + i] : A[(uint64_t)i * N + k]) : 0.0;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint32_t j = j_base + b * 16 + ci;
      bv[b] = (k < N && j < N) ? (tb ? B[(uint64_t)j * N + k] : B[(uint64_t)k * N + j]) : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
  double rs = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = i_base + a * 16 + MK::drow(kr, r);
        const uint32_t j = j_base + b * 16 + ci;
        if (i < N && j < N) {
          const uint64_t o = (uint64_t)i * N + j;
          double v = alpha * acc[a][b][r];
          if (beta != 0.0) v += beta * C[o];
          if (i == j) v += gamma;
          D[o] = v;
          const double e = (i == j ? 1.0 : 0.0) - v;
          rs += e * e;
        }
      }
  if (!res) return;
  red[threadIdx.x] = rs;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) res[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// Wide Grams from LDS (both sides >= 128 columns, 16-byte aligned rows):
// work-group tile 128 x 128, each wave a 64 x 64 sub-tile (4 x 4 MFMA blocks).
// The work-group stages KC-row panels of both operands in LDS (double
// buffered; the next panel's 16-byte loads are in flight while the current one
// is consumed), so each operand element crosses L2 once per work-group
// instead of once per wave: at the MFMA rate the 64 x 64-tile Gram needs more
// L1-to-L2 traffic than the chip sustains.
//
// A Gram of one block with itself (X^T X) that fits one tile (at most 128
// columns) runs as k_gram_lds_diag, which stages one panel and computes only
// the 36 MFMA blocks on or above the block diagonal (nine per wave, each
// block off the diagonal also written mirrored) instead of 64: the matrix
// cores do 36/64 of the work.

// Panel staging shared by the two kernels: the 16-byte chunks of KC rows
// starting at row p of columns c0 .. c0 + 127 of X (zero outside the rows
// [.., r1) and the columns [.., nc)).
template <typename TI, int KC>
struct PanelChunks {
  static constexpr int VPC = 16 / (int)sizeof(TI);      // values per 16-byte chunk
  static constexpr int CPR = GT2 / VPC;                  // chunks per panel row
  static constexpr int CPT = KC * CPR / 256;             // chunks per thread
  static_assert(CPT * 256 == KC * CPR, "panel chunks must divide the work-group");
  typedef unsigned int Chunk __attribute__((ext_vector_type(4)));
  Chunk ch[CPT];
  __device__ void load(const TI* __restrict__ X, uint64_t ld, uint32_t nc, uint32_t c0, uint32_t p, uint32_t r1) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const uint32_t c = threadIdx.x + 256u * u;
      const uint32_t row = c / CPR, col = (c % CPR) * VPC;
      const uint32_t gr = p + row;
      const Chunk z = {0u, 0u, 0u, 0u};
      ch[u] = (gr < r1 && c0 + col < nc) ? *reinterpret_cast<const Chunk*>(X + (uint64_t)gr * ld + c0 + col) : z;
    }
  }
  __device__ void store(TI (*panel)[GT2]) const {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const uint32_t c = threadIdx.x + 256u * u;
      const uint32_t row = c / CPR, col = (c % CPR) * VPC;
      *reinterpret_cast<Chunk*>(&panel[row][col]) = ch[u];
    }
  }
};

template <typename TI, int KIND>
__global__ __launch_bounds__(256) void k_gram_lds(const TI* __restrict__ A, uint64_t lda, uint32_t na,
                                                  const TI* __restrict__ B, uint64_t ldb, uint32_t nb,
                                                  uint32_t rows, uint32_t rows_per_split, double* __restrict__ part) {
  using M = Mk<KIND>;
  using acc_t = typename M::acc_t;
  constexpr int KC = PanelRows<KIND>::KC;
  __shared__ __align__(16) TI pa[2][KC][GT2];
  __shared__ __align__(16) TI pb[2][KC][GT2];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t wi = (wave >> 1) * GW2, wj = (wave & 1u) * GW2;     // the wave's sub-tile in the tile
  const uint32_t i0 = blockIdx.y * GT2, j0 = blockIdx.x * GT2;
  const uint32_t ks = blockIdx.z;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  const uint32_t r0 = ks * rows_per_split;
  const uint32_t r1 = min(rows, r0 + rows_per_split);
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = zero_acc<acc_t>();
  PanelChunks<TI, KC> ca, cb;
  const uint32_t npan = (r1 > r0) ? (r1 - r0 + KC - 1) / KC : 0;
  if (npan > 0) {
    ca.load(A, lda, na, i0, r0, r1);
    cb.load(B, ldb, nb, j0, r0, r1);
    ca.store(pa[0]);
    cb.store(pb[0]);
  }
  __syncthreads();
  for (uint32_t t = 0; t < npan; ++t) {
    const int buf = (int)(t & 1u);
    if (t + 1 < npan) {
      ca.load(A, lda, na, i0, r0 + (t + 1) * KC, r1);
      cb.load(B, ldb, nb, j0, r0 + (t + 1) * KC, r1);
    }
#pragma unroll
    for (int kk = 0; kk < KC / M::KSTEP; ++kk) {
      TI av[4][M::KPL], bv[4][M::KPL];
#pragma unroll
      for (int e = 0; e < M::KPL; ++e) {
        const uint32_t row = kk * M::KSTEP + kr * M::KPL + e;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          av[a][e] = pa[buf][row][wi + a * 16 + ci];
          bv[a][e] = pb[buf][row][wj + a * 16 + ci];
        }
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mma<KIND, TI>(av[a], bv[b], acc[a][b]);
    }
    if (t + 1 < npan) {
      ca.store(pa[buf ^ 1]);
      cb.store(pb[buf ^ 1]);
    }
    __syncthreads();
  }
  double* out = part + (uint64_t)ks * na * nb;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = i0 + wi + a * 16 + M::drow(kr, r);
        const uint32_t j = j0 + wj + b * 16 + ci;
        if (i < na && j < nb) out[(uint64_t)i * nb + j] = (double)acc[a][b][r];
      }
}

// The nine 16 x 16 blocks (a, b), a <= b, of a diagonal tile that wave w
// computes: together the 36 blocks of the upper block triangle of 8 x 8.
__device__ __forceinline__ void sym_blocks(uint32_t w, uint32_t (&oa)[9], uint32_t (&ob)[9]) {
  constexpr unsigned char T[4][9][2] = {
      {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {0, 4}, {0, 5}, {0, 6}, {0, 7}, {1, 1}},
      {{1, 2}, {1, 3}, {1, 4}, {1, 5}, {1, 6}, {1, 7}, {2, 2}, {2, 3}, {2, 4}},
      {{2, 5}, {2, 6}, {2, 7}, {3, 3}, {3, 4}, {3, 5}, {3, 6}, {3, 7}, {4, 4}},
      {{4, 5}, {4, 6}, {4, 7}, {5, 5}, {5, 6}, {5, 7}, {6, 6}, {6, 7}, {7, 7}}};
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    uint32_t a = T[0][p][0], b = T[0][p][1];
    if (w == 1u) a = T[1][p][0], b = T[1][p][1];
    if (w == 2u) a = T[2][p][0], b = T[2][p][1];
    if (w == 3u) a = T[3][p][0], b = T[3][p][1];
    oa[p] = 16u * a;
    ob[p] = 16u * b;
  }
}

// A symmetric A^T B for at most 128 columns (X^T X, or TWO: A != B known to
// give a symmetric product): the one tile, split blockIdx.z.
template <typename TI, int KIND, bool TWO>
__global__ __launch_bounds__(256) void k_gram_lds_diag(const TI* __restrict__ A, uint64_t lda, uint32_t na,
                                                       const TI* __restrict__ B, uint64_t ldb,
                                                       uint32_t rows, uint32_t rows_per_split,
                                                       double* __restrict__ part) {
  using M = Mk<KIND>;
  using acc_t = typename M::acc_t;
  constexpr int KC = PanelRows<KIND>::KC;
  __shared__ __align__(16) TI pa[2][KC][GT2];
  __shared__ __align__(16) TI pb[TWO ? 2 : 1][TWO ? KC : 1][TWO ? GT2 : 1];
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63u;
  const uint32_t i0 = blockIdx.x * GT2;
  const uint32_t ks = blockIdx.z;
  const uint32_t kr = lane >> 4, ci = lane & 15u;
  const uint32_t r0 = ks * rows_per_split;
  const uint32_t r1 = min(rows, r0 + rows_per_split);
  uint32_t oa[9], ob[9];
  sym_blocks(wave, oa, ob);
  acc_t acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = zero_acc<acc_t>();
  PanelChunks<TI, KC> ca, cb;
  const uint32_t npan = (r1 > r0) ? (r1 - r0 + KC - 1) / KC : 0;
  if (npan > 0) {
    ca.load(A, lda, na, i0, r0, r1);
    ca.store(pa[0]);
    if constexpr (TWO) {
      cb.load(B, ldb, na, i0, r0, r1);
      cb.store(pb[0]);
    }
  }
  __syncthreads();
  for (uint32_t t = 0; t < npan; ++t) {
    const int buf = (int)(t & 1u);
    if (t + 1 < npan) {
      ca.load(A, lda, na, i0, r0 + (t + 1) * KC, r1);
      if constexpr (TWO) cb.load(B, ldb, na, i0, r0 + (t + 1) * KC, r1);
    }
#pragma unroll
    for (int kk = 0; kk < KC / M::KSTEP; ++kk) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        TI av[M::KPL], bv[M::KPL];
#pragma unroll
        for (int e = 0; e < M::KPL; ++e) {
          const uint32_t row = kk * M::KSTEP + kr * M::KPL + e;
          av[e] = pa[buf][row][oa[q] + ci];
          if constexpr (TWO) bv[e] = pb[buf][row][ob[q] + ci];
          else bv[e] = pa[buf][row][ob[q] + ci];
        }
        acc[q] = mma<KIND, TI>(av, bv, acc[q]);
      }
    }
    if (t + 1 < npan) {
      ca.store(pa[buf ^ 1]);
      if constexpr (TWO) cb.store(pb[buf ^ 1]);
    }
    __syncthreads();
  }
  double* out = part + (uint64_t)ks * na * na;
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t i = i0 + oa[q] + M::drow(kr, r);
      const uint32_t j = i0 + ob[q] + ci;
      if (i < na && j < na) {
        out[(uint64_t)i * na + j] = (double)acc[q][r];
        if (oa[q] != ob[q]) out[(uint64_t)j * na + i] = (double)acc[q][r];
      }
    }
}

template <typename TI, int KIND>
hipError_t gram_t(ope_ctx* c, const TI* A, int64_t lda, int na, const TI* B, int64_t ldb, int nb, int64_t rows,
                  double* out, bool symmetric = false) {
  // 128 x 128 tiles from LDS when both sides are wide and rows split into
  // whole 16-byte chunks; else the wide tile from global memory (FP32 and
  // BF16 kinds), else 64 x 64 tiles
  constexpr int64_t VPC = 16 / (int64_t)sizeof(TI);
  const bool lds = na >= GT2 && nb >= GT2 && (reinterpret_cast<uintptr_t>(A) % 16) == 0 &&
                   (reinterpret_cast<uintptr_t>(B) % 16) == 0 && lda % VPC == 0 && ldb % VPC == 0 &&
                   na % VPC == 0 && nb % VPC == 0;
  const bool wide = lds || (KIND != MK_F64 && na >= GT2 && nb >= GT2);
  // a Gram of one block with itself in one tile: the MFMA blocks on and
  // above the block diagonal (with several tiles the two launches of fewer
  // work-groups each were measured slower than the full product)
  const bool same = A == B && lda == ldb;
  const bool sym = lds && (same || symmetric) && na == nb && na <= GT2;
  const int tile = wide ? GT2 : GT;
  const uint32_t ti = (uint32_t)((na + tile - 1) / tile), tj = (uint32_t)((nb + tile - 1) / tile);
  // about 1024 work-groups in total (512, two per CU, for the LDS kernels),
  // within the partial buffer
  int64_t ks = (lds ? 512 : 1024) / (int64_t)(ti * tj);
  if (ks < 1) ks = 1;
  const int64_t max_ks = c->part_cap / ((int64_t)na * nb);
  if (ks > max_ks) ks = max_ks;
  if (ks < 1) return hipErrorInvalidValue;
  const int64_t kstep = Mk<KIND>::KSTEP;
  int64_t rps = (rows + ks - 1) / ks;
  rps = ((rps + kstep - 1) / kstep) * kstep;
  if (rps < kstep) rps = kstep;
  ks = (rows + rps - 1) / rps;
  if (ks < 1) ks = 1;
  const bool narrow = na <= 32 && nb <= 32;    // one 32 x 32 tile; all four waves split the rows
  {
    ProfScope ps(c, OPE_KERNEL_GRAM);
    if (narrow)
      hipLaunchKernelGGL((k_gram_narrow<TI, KIND>), dim3((uint32_t)ks), dim3(256), 0, c->stream, A, (uint64_t)lda,
                         (uint32_t)na, B, (uint64_t)ldb, (uint32_t)nb, (uint32_t)rows, (uint32_t)rps, c->part);
    else if (sym && same)
      hipLaunchKernelGGL((k_gram_lds_diag<TI, KIND, false>), dim3(1, 1, (uint32_t)ks), dim3(256), 0, c->stream, A,
                         (uint64_t)lda, (uint32_t)na, A, (uint64_t)lda, (uint32_t)rows, (uint32_t)rps, c->part);
    else if (sym)
      hipLaunchKernelGGL((k_gram_lds_diag<TI, KIND, true>), dim3(1, 1, (uint32_t)ks), dim3(256), 0, c->stream, A,
                         (uint64_t)lda, (uint32_t)na, B, (uint64_t)ldb, (uint32_t)rows, (uint32_t)rps, c->part);
    else if (lds)
      hipLaunchKernelGGL((k_gram_lds<TI, KIND>), dim3(tj, ti, (uint32_t)ks), dim3(256), 0, c->stream, A,
                         (uint64_t)lda, (uint32_t)na, B, (uint64_t)ldb, (uint32_t)nb, (uint32_t)rows, (uint32_t)rps,
                         c->part);
    else if (wide)
      hipLaunchKernelGGL((k_gram_wide<TI, KIND>), dim3(tj, ti, (uint32_t)ks), dim3(256), 0, c->stream, A,
                         (uint64_t)lda, (uint32_t)na, B, (uint64_t)ldb, (uint32_t)nb, (uint32_t)rows, (uint32_t)rps,
                         c->part);
    else
      hipLaunchKernelGGL((k_gram<TI, KIND>), dim3(tj, ti, (uint32_t)ks), dim3(256), 0, c->stream, A, (uint64_t)lda,
                         (uint32_t)na, B, (uint64_t)ldb, (uint32_t)nb, (uint32_t)rows, (uint32_t)rps, c->part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_cols(c, c->part, ks, (int64_t)na * nb, out, RED_PLAIN);
}

template <typename TI, int KIND>
hipError_t rowmm_t(ope_ctx* c, const TI* X0, const TI* M0, const TI* X1, const TI* M1, const TI* Cm, double cbeta,
                   double ascale, TI* Out, int want_colsq, int predicated, int64_t* nparts) {
  const uint32_t n = (uint32_t)c->n, N = (uint32_t)c->N;
  // LDS-staged panels when every operand row splits into whole, aligned 16-byte chunks
  constexpr uint32_t VPC = 16 / (uint32_t)sizeof(TI);
  auto al16 = [](const void* q) { return q == nullptr || (reinterpret_cast<uintptr_t>(q) % 16) == 0; };
  const bool narrow = N <= 32;
  const bool lds = !narrow && N % VPC == 0 && al16(X0) && al16(M0) && al16(X1) && al16(M1);
  // FP64: 64-row tiles (132 VGPRs, three work-groups per compute unit, whose
  // output stores overlap the others' matrix-core work) measured 4% faster than
  // 128-row tiles (219 VGPRs, two) at 64^3, N = 128
  const bool half = lds && KIND == MK_F64;
  const uint32_t rt = narrow ? RTN : (lds ? (half ? RT2H : RT2) : RT);
  const uint32_t gr = (n + rt - 1) / rt, gc = (N + CT - 1) / CT;
  if (gc != 1 && (Out == X0 || Out == X1)) return hipErrorInvalidValue;  // in place needs one column tile
  if (want_colsq && (int64_t)gr * N > c->part_cap) return hipErrorInvalidValue;
  ProfScope ps(c, OPE_KERNEL_ROWMM);
  if (narrow) {
    if (X1)
      hipLaunchKernelGGL((k_rowmm_narrow<TI, KIND, 2>), dim3(gr), dim3(256), 0, c->stream, X0, M0, X1, M1, Cm, cbeta,
                         ascale, Out, n, N, want_colsq, predicated, c->sc, c->part);
    else
      hipLaunchKernelGGL((k_rowmm_narrow<TI, KIND, 1>), dim3(gr), dim3(256), 0, c->stream, X0, M0, X1, M1, Cm, cbeta,
                         ascale, Out, n, N, want_colsq, predicated, c->sc, c->part);
  } else if (lds) {
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(gr, gc), dim3(256), 0, c->stream, X0, M0, X1, M1, Cm, cbeta, ascale, Out, n, N,
                         want_colsq, predicated, c->sc, c->part);
    };
    if (half) {
      if (X1) go(k_rowmm_lds<TI, KIND, 2, RT2H>);
      else go(k_rowmm_lds<TI, KIND, 1, RT2H>);
    } else {
      if (X1) go(k_rowmm_lds<TI, KIND, 2, RT2>);
      else go(k_rowmm_lds<TI, KIND, 1, RT2>);
    }
  } else if (X1)
    hipLaunchKernelGGL((k_rowmm<TI, KIND, 2>), dim3(gr, gc), dim3(256), 0, c->stream, X0, M0, X1, M1, Cm, cbeta,
                       ascale, Out, n, N, want_colsq, predicated, c->sc, c->part);
  else
    hipLaunchKernelGGL((k_rowmm<TI, KIND, 1>), dim3(gr, gc), dim3(256), 0, c->stream, X0, M0, X1, M1, Cm, cbeta,
                       ascale, Out, n, N, want_colsq, predicated, c->sc, c->part);
  if (nparts) *nparts = gr;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gram(ope_ctx* c, const double* A, int64_t lda, int na, const double* B, int64_t ldb, int nb,
                       int64_t rows, double* out) {
  return gram_t<double, MK_F64>(c, A, lda, na, B, ldb, nb, rows, out);
}

hipError_t launch_gram_sym(ope_ctx* c, const double* A, int64_t lda, const double* B, int64_t ldb, int n,
                           int64_t rows, double* out) {
  return gram_t<double, MK_F64>(c, A, lda, n, B, ldb, n, rows, out, true);
}

hipError_t launch_gram_f32(ope_ctx* c, int kind, const float* A, int64_t lda, int na, const float* B, int64_t ldb,
                           int nb, int64_t rows, double* out) {
  switch (kind) {
    case MK_F64: return gram_t<float, MK_F64>(c, A, lda, na, B, ldb, nb, rows, out);
    case MK_F32: return gram_t<float, MK_F32>(c, A, lda, na, B, ldb, nb, rows, out);
    default: return gram_t<float, MK_BF16>(c, A, lda, na, B, ldb, nb, rows, out);
  }
}

hipError_t launch_rowmm(ope_ctx* c, const double* X0, const double* M0, const double* X1, const double* M1,
                        const double* Cm, double cbeta, double ascale, double* Out, int want_colsq, int predicated,
                        int64_t* nparts) {
  return rowmm_t<double, MK_F64>(c, X0, M0, X1, M1, Cm, cbeta, ascale, Out, want_colsq, predicated, nparts);
}

hipError_t launch_sqmm(ope_ctx* c, const double* A, int ta, const double* B, int tb, const double* C, double alpha,
                       double beta, double gamma, double* D, uint32_t N, const int32_t* skip, double* res) {
  const uint32_t t = (N + 63) / 64;
  ProfScope ps(c, OPE_KERNEL_SMALL);
  hipLaunchKernelGGL(k_sqmm, dim3(t, t), dim3(256), 0, c->stream, A, ta, B, tb, C, alpha, beta, gamma, D, N, skip,
                     res);
  return hipGetLastError();
}

hipError_t launch_rowmm_f32(ope_ctx* c, int kind, const float* X0, const float* M0, const float* X1, const float* M1,
                            const float* Cm, double cbeta, double ascale, float* Out, int want_colsq, int predicated,
                            int64_t* nparts) {
  if (kind == MK_BF16)
    return rowmm_t<float, MK_BF16>(c, X0, M0, X1, M1, Cm, cbeta, ascale, Out, want_colsq, predicated, nparts);
  return rowmm_t<float, MK_F32>(c, X0, M0, X1, M1, Cm, cbeta, ascale, Out, want_colsq, predicated, nparts);
}
