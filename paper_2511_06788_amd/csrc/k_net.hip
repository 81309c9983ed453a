// The conv-net preconditioner of the learned step (gradient form of the step,
// GU = (U - H^{-1} R) Lam^{-1}, with a network in place of H^{-1}), trained and
// applied on the gfx950 matrix cores.
//
// Network: four bias-free 3x3x3 cross-correlations with zero padding,
// channels 2 -> 16 -> 16 -> 16 -> 1, ReLU after the first three:
//   out[v, co] = sum_{tap, ci} W[tap][ci][co] in[v + tap, ci],
// taps (dz, dy, dx) with dx fastest.  Input channels: the normalised residual
// column and h^2 (V + shift); the output f is scaled back by |r| h^2.
//
// Layouts in HBM:
//   activations   [sample][z][y][x][channel] BF16 (32 bytes per voxel for 16
//                 channels, 4 for the input pair, 2 for one channel)
//   FP32 fields   [sample][z][y][x] (network output, training inputs/targets)
//   weights       FP32 masters W1 | W2 | W3 | W4, each [tap][ci][co]; BF16
//                 operand copies packed per layer as [row][k] (see pack_w)
//
// Convolution = implicit GEMM on v_mfma_f32_16x16x32_bf16 with the weights in
// the A operand (rows = output channels, k = (tap, input channel)) and the
// input tile in the B operand (columns = 16 voxels along x), so the
// accumulator gives each lane four consecutive output channels of one voxel
// and a wave stores 16 voxels x 32 bytes contiguously.  A work-group computes
// a 16 x 4 x 4 voxel tile from an LDS copy of the 18 x 6 x 6 input tile.
// The 16-channel layers march along z through a ring of LDS planes
// (k_conv16z, k_conv_out1: the last layer's one output channel puts the z
// and y offsets on the MFMA rows).
// Backward: the data gradient of a layer is the same convolution with the
// weights transposed in the channels and flipped in the taps, masked by the
// ReLU pattern of the forward activation; weight gradients are contractions
// over voxels on v_mfma_f32_16x16x4f32 (FP32 operands, split over voxel
// ranges, reduced in a fixed order).
#include <algorithm>
#include <cmath>
#include <new>

#include "ope_internal.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int TX = 16, TY = 4, TZ = 4;          // output tile of a work-group
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int HV = HX * HY * HZ;                // staged input voxels (with halo)
enum { EPI_RELU = 0, EPI_MASK = 1 };

// weight block offsets (FP32 masters) and packed BF16 operand offsets
constexpr int W1_OFF = 0, W2_OFF = 864, W3_OFF = 7776, W4_OFF = 14688;
constexpr int KS16 = 14, KS2 = 2, KS1 = 1;      // 32-wide k-steps for 16, 2, 1 input channels
constexpr int KSZ = 18;                         // 16 -> 16 layers: 9 (dz, dy) x 2 x-offset pairs
constexpr int PK_F1 = 0;                        // forward layer 1: 16 x 64
constexpr int PK_F2 = PK_F1 + 16 * 32 * KS2;    // forward layers 2, 3: 16 x 576 (see packed_value)
constexpr int PK_F3 = PK_F2 + 16 * 32 * KSZ;
constexpr int PK_F4 = PK_F3 + 16 * 32 * KSZ;    // forward layer 4: 16 x 448 (row 0 used)
constexpr int PK_B4 = PK_F4 + 16 * 32 * KS16;   // transposed layer 4: 16 x 32
constexpr int PK_B3 = PK_B4 + 16 * 32 * KS1;    // transposed layers 3, 2: 16 x 576
constexpr int PK_B2 = PK_B3 + 16 * 32 * KSZ;
constexpr int PK_TOTAL = PK_B2 + 16 * 32 * KSZ;
static_assert(W4_OFF + 432 == OPE_NET_PARAMS, "parameter count");

__device__ __forceinline__ uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float from_bf16(uint16_t u) { return (float)__builtin_bit_cast(__bf16, u); }

// LDS offset of tap t relative to the centre voxel of the staged tile
__host__ __device__ constexpr int tap_delta(int t) {
  return ((t / 9 - 1) * HY + ((t / 3) % 3 - 1)) * HX + (t % 3 - 1);
}

// ---------------------------------------------------------------------------
// convolution of a one-channel input (the data gradient of the last layer:
// its transposed weights, 1 -> 16 channels) on 16 x 4 x 4 voxel tiles
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wpk,
                                              const uint16_t* __restrict__ mask, void* __restrict__ out,
                                              uint32_t m0, uint32_t m1, uint32_t m2, uint32_t ntx, uint32_t nty,
                                              uint32_t ntz) {
  constexpr int KS = (27 * CIN + 31) / 32;
  static_assert(CIN == 1, "2- and 16-channel inputs take k_conv2z and k_conv16z");
  constexpr int LDS_WORDS = (HV + 1) / 2;
  __shared__ __align__(16) uint32_t tile[LDS_WORDS];
  const uint32_t tiles = ntx * nty * ntz;
  const uint32_t b = blockIdx.x / tiles;
  uint32_t t = blockIdx.x - b * tiles;
  const uint32_t tx = t % ntx;
  t /= ntx;
  const uint32_t ty = t % nty;
  const uint32_t tz = t / nty;
  const int x0 = (int)(tx * TX), y0 = (int)(ty * TY), z0 = (int)(tz * TZ);
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint16_t* src = in + (uint64_t)b * n * CIN;

  // stage the input tile with a one-voxel halo (zeros outside the grid)
  {
    uint16_t* t16 = reinterpret_cast<uint16_t*>(tile);
    for (int v = threadIdx.x; v < HV; v += 256) {
      const int lx = v % HX, ly = (v / HX) % HY, lz = v / (HX * HY);
      const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z0 + lz - 1;
      const bool inside = gx >= 0 && gx < (int)m0 && gy >= 0 && gy < (int)m1 && gz >= 0 && gz < (int)m2;
      const uint64_t gv = ((uint64_t)gz * m1 + gy) * m0 + gx;
      t16[v] = inside ? src[gv] : (uint16_t)0;
    }
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kq = lane >> 4;
  // A operand: packed weights, row = output channel j, k = 32 s + 8 kq + e
  v8bf wa[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    wa[s] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(wpk + j * (KS * 32) + 32 * s + 8 * kq));
  __syncthreads();

  v4f acc[TY];
#pragma unroll
  for (int yb = 0; yb < TY; ++yb) acc[yb] = v4f{0.f, 0.f, 0.f, 0.f};
  const int zc = wave + 1;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
#pragma unroll
    for (int yb = 0; yb < TY; ++yb) {
      const int base = (zc * HY + yb + 1) * HX + j + 1;
      v4u bw = {0u, 0u, 0u, 0u};
      {
        // k = 8 kq + e = tap
        const uint16_t* t16 = reinterpret_cast<const uint16_t*>(tile);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int t0 = 8 * kq + 2 * i, t1 = t0 + 1;
          const uint32_t lo = t0 < 27 ? t16[base + tap_delta(t0)] : 0u;
          const uint32_t hi = t1 < 27 ? t16[base + tap_delta(t1)] : 0u;
          bw[i] = lo | (hi << 16);
        }
      }
      acc[yb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s], __builtin_bit_cast(v8bf, bw), acc[yb], 0, 0, 0);
    }
  }

  // epilogue: lane holds output channels 4 kq + r of voxel (x0 + j, y0 + yb, z0 + wave)
  const int gx = x0 + j, gz = z0 + wave;
  if (gx >= (int)m0 || gz >= (int)m2) return;
#pragma unroll
  for (int yb = 0; yb < TY; ++yb) {
    const int gy = y0 + yb;
    if (gy >= (int)m1) break;
    const uint64_t v = ((uint64_t)gz * m1 + gy) * m0 + gx;
    const uint64_t o = ((uint64_t)b * n + v) * 16 + 4 * kq;
    float r[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = acc[yb][e];
    if constexpr (EPI == EPI_RELU) {
#pragma unroll
      for (int e = 0; e < 4; ++e) r[e] = r[e] > 0.f ? r[e] : 0.f;
    } else {
      const uint2 mk = *reinterpret_cast<const uint2*>(mask + o);
      const uint32_t mw[2] = {mk.x, mk.y};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint16_t mb = (uint16_t)(mw[e >> 1] >> (16 * (e & 1)));
        if (!(from_bf16(mb) > 0.f)) r[e] = 0.f;
      }
    }
    uint2 w;
    w.x = (uint32_t)to_bf16(r[0]) | ((uint32_t)to_bf16(r[1]) << 16);
    w.y = (uint32_t)to_bf16(r[2]) | ((uint32_t)to_bf16(r[3]) << 16);
    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(out) + o) = w;
  }
}

// ---------------------------------------------------------------------------
// 16 -> 16 channel convolution (layers 2-3 forward, and their data gradients)
// z-marched: a work-group owns a 16 x 16 x-y tile of one sample and OZ planes;
// the input planes pass through a ring of three 18 x 18 LDS planes (each
// staged once, halo 1.27x instead of the 2.5x of a 16 x 4 x 4 tile), and wave
// w computes output rows 4 w .. 4 w + 3 of the current plane (weights in the
// A operand, 16 voxels along x in B).  The contraction is packed per (dz, dy)
// in two 32-wide steps of x-offset pairs (dx 0, 1; dx 2 and zeros), so that
// one LDS read of an input row serves the up to three output rows that use
// it with different dy (36 reads and 72 MFMAs per wave and plane instead of
// 56 and 56).
// ---------------------------------------------------------------------------
constexpr int OX = 16, OY = 16, OZ = 16;        // x-y tile and z run of a work-group
constexpr int OHX = OX + 2, OHY = OY + 2, OPL = OHX * OHY;

template <int EPI>
__global__ __launch_bounds__(256) void k_conv16z(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wpk,
                                                 const uint16_t* __restrict__ mask, uint16_t* __restrict__ out,
                                                 uint32_t m0, uint32_t m1, uint32_t m2, uint32_t ntx, uint32_t nty,
                                                 uint32_t ntz) {
  __shared__ __align__(16) v4u ring[3][2][OPL];   // [plane slot][channel half][voxel of the 18 x 18 plane]
  const uint32_t tiles = ntx * nty * ntz;
  const uint32_t b = blockIdx.x / tiles;
  uint32_t t = blockIdx.x - b * tiles;
  const uint32_t tx = t % ntx;
  t /= ntx;
  const uint32_t ty = t % nty;
  const uint32_t tz = t / nty;
  const int x0 = (int)(tx * OX), y0 = (int)(ty * OY), z0 = (int)(tz * OZ);
  const int z1 = z0 + OZ < (int)m2 ? z0 + OZ : (int)m2;
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint16_t* src = in + (uint64_t)b * n * 16;
  // input plane z (zeros outside the grid) into ring slot (z + 1) mod 3
  auto stage = [&](int z) {
    v4u* dst = &ring[(z + 3 + 1) % 3][0][0];
    for (int idx = threadIdx.x; idx < 2 * OPL; idx += 256) {
      const int h = idx & 1, v = idx >> 1;
      const int gx = x0 + v % OHX - 1, gy = y0 + v / OHX - 1;
      v4u val = {0u, 0u, 0u, 0u};
      if (z >= 0 && z < (int)m2 && gx >= 0 && gx < (int)m0 && gy >= 0 && gy < (int)m1)
        val = *reinterpret_cast<const v4u*>(src + (((uint64_t)z * m1 + gy) * m0 + gx) * 16 + 8 * h);
      dst[h * OPL + v] = val;
    }
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kq = lane >> 4;
  // A operand: packed weights, row = output channel j, k = 32 s + 8 kq + e
  v8bf wa[KSZ];
#pragma unroll
  for (int s = 0; s < KSZ; ++s)
    wa[s] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(wpk + j * (KSZ * 32) + 32 * s + 8 * kq));
  stage(z0 - 1);
  stage(z0);
  const int gx = x0 + j;
  for (int z = z0; z < z1; ++z) {
    stage(z + 1);
    __syncthreads();
    v4f acc[4];
#pragma unroll
    for (int yb = 0; yb < 4; ++yb) acc[yb] = v4f{0.f, 0.f, 0.f, 0.f};
    // k-step 2 (3 dz + dy) + pair: lanes kq / 2 take x offset dx = 2 pair + kq / 2
    // (dx = 3: zero), kq % 2 the channel half.  Input row Y (frame row
    // 4 wave + Y) of plane z - 1 + dz feeds output rows yb = Y - dy, so each
    // LDS read serves up to three MFMAs.
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
      const v4u* pl = &ring[(z + dz) % 3][kq & 1][0];             // plane z - 1 + dz
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        const int dx = 2 * pr + (kq >> 1);
#pragma unroll
        for (int Y = 0; Y < 6; ++Y) {
          v4u bw = {0u, 0u, 0u, 0u};
          if (dx <= 2) bw = pl[(4 * wave + Y) * OHX + j + dx];
          const v8bf bv = __builtin_bit_cast(v8bf, bw);
#pragma unroll
          for (int dy = 0; dy < 3; ++dy) {
            const int yb = Y - dy;
            if (yb >= 0 && yb < 4)
              acc[yb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[2 * (3 * dz + dy) + pr], bv, acc[yb], 0, 0, 0);
          }
        }
      }
    }
    // epilogue: lane holds output channels 4 kq + r of voxel (x0 + j, y0 + 4 wave + yb, z)
    if (gx < (int)m0) {
#pragma unroll
      for (int yb = 0; yb < 4; ++yb) {
        const int gy = y0 + 4 * wave + yb;
        if (gy >= (int)m1) break;
        const uint64_t v = ((uint64_t)z * m1 + gy) * m0 + gx;
        const uint64_t o = ((uint64_t)b * n + v) * 16 + 4 * kq;
        float r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = acc[yb][e];
        if constexpr (EPI == EPI_RELU) {
#pragma unroll
          for (int e = 0; e < 4; ++e) r[e] = r[e] > 0.f ? r[e] : 0.f;
        } else {
          const uint2 mk = *reinterpret_cast<const uint2*>(mask + o);
          const uint32_t mw[2] = {mk.x, mk.y};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint16_t mb = (uint16_t)(mw[e >> 1] >> (16 * (e & 1)));
            if (!(from_bf16(mb) > 0.f)) r[e] = 0.f;
          }
        }
        uint2 w;
        w.x = (uint32_t)to_bf16(r[0]) | ((uint32_t)to_bf16(r[1]) << 16);
        w.y = (uint32_t)to_bf16(r[2]) | ((uint32_t)to_bf16(r[3]) << 16);
        *reinterpret_cast<uint2*>(out + o) = w;
      }
    }
    __syncthreads();                              // the slot of plane z - 1 is staged next
  }
}

// ---------------------------------------------------------------------------
// first layer (2 input channels -> 16) on the same z-march and 16 x 16 x-y
// tiles as k_conv16z, a plane ring of one 32-bit word (the two BF16 input
// channels) per voxel; the MFMA mapping is that of k_conv (k = 2 tap + ci:
// lane kq reads taps 16 s + 4 kq + i, i < 4).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv2z(const uint32_t* __restrict__ in, const uint16_t* __restrict__ wpk,
                                                uint16_t* __restrict__ out, uint32_t m0, uint32_t m1, uint32_t m2,
                                                uint32_t ntx, uint32_t nty, uint32_t ntz) {
  __shared__ uint32_t ring[3][OPL];               // [plane slot][voxel of the 18 x 18 plane]
  const uint32_t tiles = ntx * nty * ntz;
  const uint32_t b = blockIdx.x / tiles;
  uint32_t t = blockIdx.x - b * tiles;
  const uint32_t tx = t % ntx;
  t /= ntx;
  const uint32_t ty = t % nty;
  const uint32_t tz = t / nty;
  const int x0 = (int)(tx * OX), y0 = (int)(ty * OY), z0 = (int)(tz * OZ);
  const int z1 = z0 + OZ < (int)m2 ? z0 + OZ : (int)m2;
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint32_t* src = in + (uint64_t)b * n;
  // input plane z (zeros outside the grid) into ring slot (z + 1) mod 3
  auto stage = [&](int z) {
    uint32_t* dst = &ring[(z + 3 + 1) % 3][0];
    for (int v = threadIdx.x; v < OPL; v += 256) {
      const int gx = x0 + v % OHX - 1, gy = y0 + v / OHX - 1;
      uint32_t val = 0u;
      if (z >= 0 && z < (int)m2 && gx >= 0 && gx < (int)m0 && gy >= 0 && gy < (int)m1)
        val = src[((uint64_t)z * m1 + gy) * m0 + gx];
      dst[v] = val;
    }
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kq = lane >> 4;
  v8bf wa[KS2];
#pragma unroll
  for (int s = 0; s < KS2; ++s)
    wa[s] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4u*>(wpk + j * (KS2 * 32) + 32 * s + 8 * kq));
  stage(z0 - 1);
  stage(z0);
  const int gx = x0 + j;
  for (int z = z0; z < z1; ++z) {
    stage(z + 1);
    __syncthreads();
    v4f acc[4];
#pragma unroll
    for (int yb = 0; yb < 4; ++yb) acc[yb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS2; ++s) {
#pragma unroll
      for (int yb = 0; yb < 4; ++yb) {
        v4u bw = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int tap = 16 * s + 4 * kq + i;
          if (tap < 27) {
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // offsets + 1
            bw[i] = ring[(z + dz) % 3][(4 * wave + yb + dy) * OHX + j + dx];
          }
        }
        acc[yb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s], __builtin_bit_cast(v8bf, bw), acc[yb], 0, 0, 0);
      }
    }
    // epilogue: lane holds output channels 4 kq + r of voxel (x0 + j, y0 + 4 wave + yb, z), ReLU
    if (gx < (int)m0) {
#pragma unroll
      for (int yb = 0; yb < 4; ++yb) {
        const int gy = y0 + 4 * wave + yb;
        if (gy >= (int)m1) break;
        const uint64_t o = ((uint64_t)b * n + ((uint64_t)z * m1 + gy) * m0 + gx) * 16 + 4 * kq;
        float r[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = acc[yb][e] > 0.f ? acc[yb][e] : 0.f;
        uint2 w;
        w.x = (uint32_t)to_bf16(r[0]) | ((uint32_t)to_bf16(r[1]) << 16);
        w.y = (uint32_t)to_bf16(r[2]) | ((uint32_t)to_bf16(r[3]) << 16);
        *reinterpret_cast<uint2*>(out + o) = w;
      }
    }
    __syncthreads();                              // the slot of plane z - 1 is staged next
  }
}

// ---------------------------------------------------------------------------
// last forward layer (16 channels -> 1, FP32 output).  One output channel
// leaves no output-channel dimension for the matrix cores, so the MFMA rows
// carry the z and y offsets instead (row 4 dz + dy; 9 of 16 rows used, the
// matrix cores do 1.8x the algorithmic flops at 32x the FP32 vector rate):
// for input row Y of input plane P, a pair of MFMAs (x offsets 0, 1 and 2 in
// the contraction with the 16 channels, as in k_conv16z) gives in row
// 4 dz + dy the contribution of that row to output row Y - dy of output plane
// P + 1 - dz.  Each input plane is staged and multiplied once, right after it
// arrives; lane group dz (lanes 16 dz .. 16 dz + 15 hold rows 4 dz .. + 3)
// adds its rows into the three output planes in flight, and an output plane,
// complete once plane P = z + 1 is in, is summed over the lane groups.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv_out1(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wrow,
                                                   float* __restrict__ out, uint32_t m0, uint32_t m1, uint32_t m2,
                                                   uint32_t ntx, uint32_t nty, uint32_t ntz) {
  __shared__ __align__(16) v4u ring[2][2][OPL];   // [plane slot][channel half][voxel of the 18 x 18 plane]
  const uint32_t tiles = ntx * nty * ntz;
  const uint32_t b = blockIdx.x / tiles;
  uint32_t t = blockIdx.x - b * tiles;
  const uint32_t tx = t % ntx;
  t /= ntx;
  const uint32_t ty = t % nty;
  const uint32_t tz = t / nty;
  const int x0 = (int)(tx * OX), y0 = (int)(ty * OY), z0 = (int)(tz * OZ);
  const int z1 = z0 + OZ < (int)m2 ? z0 + OZ : (int)m2;
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint16_t* src = in + (uint64_t)b * n * 16;
  // input plane P (zeros outside the grid) into ring slot (P + 2) mod 2
  auto stage = [&](int P) {
    v4u* dst = &ring[(P + 2) & 1][0][0];
    for (int idx = threadIdx.x; idx < 2 * OPL; idx += 256) {
      const int h = idx & 1, v = idx >> 1;
      const int gx = x0 + v % OHX - 1, gy = y0 + v / OHX - 1;
      v4u val = {0u, 0u, 0u, 0u};
      if (P >= 0 && P < (int)m2 && gx >= 0 && gx < (int)m0 && gy >= 0 && gy < (int)m1)
        val = *reinterpret_cast<const v4u*>(src + (((uint64_t)P * m1 + gy) * m0 + gx) * 16 + 8 * h);
      dst[h * OPL + v] = val;
    }
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, kq = lane >> 4;
  // A operand of x-offset pair pr: row j = 4 dz + dy (dz, dy < 3, else zero),
  // k = 8 kq + e: dx = 2 pr + kq / 2 (dx = 3: zero), channel 8 (kq % 2) + e;
  // the packed row holds tap (dz, dy, dx) (dx fastest) at k = 16 tap + channel
  v8bf wa[2];
#pragma unroll
  for (int pr = 0; pr < 2; ++pr) {
    const int dz = j >> 2, dy = j & 3, dx = 2 * pr + (kq >> 1);
    v4u w = {0u, 0u, 0u, 0u};
    if (dz < 3 && dy < 3 && dx < 3) w = *reinterpret_cast<const v4u*>(wrow + 16 * (9 * dz + 3 * dy + dx) + 8 * (kq & 1));
    wa[pr] = __builtin_bit_cast(v8bf, w);
  }
  // output planes z, z + 1, z + 2 in flight: this lane's part (its dz = kq) of rows 4 wave + yb
  float acc[3][4];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int yb = 0; yb < 4; ++yb) acc[q][yb] = 0.f;
  // multiply input plane P (staged) into the planes in flight; z is the
  // output plane of acc[0], so lane group kq adds into plane offset P + 1 - kq - z
  auto process = [&](int P, int z) {
    const v4u* pl = &ring[(P + 2) & 1][kq & 1][0];
    const int qq = P + 1 - kq - z;
#pragma unroll
    for (int Y = 0; Y < 6; ++Y) {
      v4f d = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        const int dx = 2 * pr + (kq >> 1);
        v4u bw = {0u, 0u, 0u, 0u};
        if (dx <= 2) bw = pl[(4 * wave + Y) * OHX + j + dx];
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[pr], __builtin_bit_cast(v8bf, bw), d, 0, 0, 0);
      }
      // row 4 kq + r of column j: dz = kq, dy = r -> output row Y - r
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int yb = Y - r;
        if (yb >= 0 && yb < 4) {
#pragma unroll
          for (int q = 0; q < 3; ++q) acc[q][yb] += qq == q ? d[r] : 0.f;
        }
      }
    }
  };
  stage(z0 - 1);
  __syncthreads();
  process(z0 - 1, z0);
  stage(z0);
  __syncthreads();
  process(z0, z0);
  const int gx = x0 + j;
  for (int z = z0; z < z1; ++z) {
    stage(z + 1);                                 // the slot of plane z - 1 (its reads ended before the last wait)
    __syncthreads();
    process(z + 1, z);
    // output plane z is complete: sum the lane groups (kq = 3 holds zeros)
#pragma unroll
    for (int yb = 0; yb < 4; ++yb) {
      float v = acc[0][yb];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      const int gy = y0 + 4 * wave + yb;
      if (kq == 0 && gx < (int)m0 && gy < (int)m1) out[(uint64_t)b * n + ((uint64_t)z * m1 + gy) * m0 + gx] = v;
    }
#pragma unroll
    for (int yb = 0; yb < 4; ++yb) {
      acc[0][yb] = acc[1][yb];
      acc[1][yb] = acc[2][yb];
      acc[2][yb] = 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradients: dW[t][ca][cg] = sum over samples and voxels of
// a[v + tap_t][ca] g[v][cg]; one partial row per wave (a voxel range of one sample)
// ---------------------------------------------------------------------------
enum { WGR_16 = 0, WGR_W4 = 1, WGR_W1 = 2 };

struct Vox {
  int x, y, z;
};
__device__ __forceinline__ Vox vox_of(uint32_t v, uint32_t m0, uint32_t m1) {
  Vox r;
  r.x = (int)(v % m0);
  v /= m0;
  r.y = (int)(v % m1);
  r.z = (int)(v / m1);
  return r;
}
__device__ __forceinline__ bool inside(int x, int y, int z, uint32_t m0, uint32_t m1, uint32_t m2) {
  return x >= 0 && x < (int)m0 && y >= 0 && y < (int)m1 && z >= 0 && z < (int)m2;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ a, const uint16_t* __restrict__ g,
                                               float* __restrict__ part, uint32_t part_ld, uint32_t part_off,
                                               uint32_t rows, uint32_t rows_per_sample, uint32_t vox_per_row,
                                               uint32_t m0, uint32_t m1, uint32_t m2) {
  constexpr int NACC = MODE == WGR_16 ? 27 : (MODE == WGR_W4 ? 2 : 4);
  constexpr int CA = MODE == WGR_W1 ? 2 : 16;
  constexpr int CG = MODE == WGR_W4 ? 1 : 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t row = blockIdx.x * 4 + wave;
  if (row >= rows) return;
  const uint32_t b = row / rows_per_sample, ch = row - b * rows_per_sample;
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint32_t v0 = ch * vox_per_row;
  const uint32_t v1 = (uint32_t)min<uint64_t>(n, (uint64_t)v0 + vox_per_row);
  const uint16_t* as = a + (uint64_t)b * n * CA;
  const uint16_t* gs = g + (uint64_t)b * n * CG;
  const int j = lane & 15, kq = lane >> 4;
  v4f acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};

  for (uint32_t vb = v0; vb < v1; vb += 4) {
    const uint32_t v = vb + kq;
    const bool ok = v < v1;
    const Vox p = vox_of(ok ? v : v0, m0, m1);
    if constexpr (MODE == WGR_16) {
      // A[ca = j][k] = a[v_k + tap][j], B[k][cg = j] = g[v_k][j]
      const float gv = ok ? from_bf16(gs[(uint64_t)v * 16 + j]) : 0.f;
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int x = p.x + t % 3 - 1, y = p.y + (t / 3) % 3 - 1, z = p.z + t / 9 - 1;
        float av = 0.f;
        if (ok && inside(x, y, z, m0, m1, m2)) av = from_bf16(as[(((uint64_t)z * m1 + y) * m0 + x) * 16 + j]);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, gv, acc[t], 0, 0, 0);
      }
    } else if constexpr (MODE == WGR_W4) {
      // A[ca = j][k] = a[v_k][j], B[k][col] = g[v_k - tap_col], col = 16 cb + j
      const float av = ok ? from_bf16(as[(uint64_t)v * 16 + j]) : 0.f;
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int t = 16 * cb + j;
        float gv = 0.f;
        if (ok && t < 27) {
          const int x = p.x - (t % 3 - 1), y = p.y - ((t / 3) % 3 - 1), z = p.z - (t / 9 - 1);
          if (inside(x, y, z, m0, m1, m2)) gv = from_bf16(gs[((uint64_t)z * m1 + y) * m0 + x]);
        }
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, gv, acc[cb], 0, 0, 0);
      }
    } else {
      // A[row][k] = x[v_k + tap_t][ci], row = 16 rb + j = 2 t + ci; B[k][co = j] = g[v_k][j]
      const float gv = ok ? from_bf16(gs[(uint64_t)v * 16 + j]) : 0.f;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int r = 16 * rb + j, t = r >> 1, ci = r & 1;
        float av = 0.f;
        if (ok && t < 27) {
          const int x = p.x + t % 3 - 1, y = p.y + (t / 3) % 3 - 1, z = p.z + t / 9 - 1;
          if (inside(x, y, z, m0, m1, m2)) av = from_bf16(as[(((uint64_t)z * m1 + y) * m0 + x) * 2 + ci]);
        }
        acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, gv, acc[rb], 0, 0, 0);
      }
    }
  }

  // lane holds D[4 kq + r][j]
  float* out = part + (uint64_t)row * part_ld + part_off;
#pragma unroll
  for (int q = 0; q < NACC; ++q) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int dr = 4 * kq + r;
      if constexpr (MODE == WGR_16) {
        out[q * 256 + dr * 16 + j] = acc[q][r];                 // dW[t = q][ca = dr][cg = j]
      } else if constexpr (MODE == WGR_W4) {
        const int t = 16 * q + j;                               // dW4[t][ca = dr]
        if (t < 27) out[t * 16 + dr] = acc[q][r];
      } else {
        const int rr = 16 * q + dr;                             // dW1[t][ci][co = j], rr = 2 t + ci
        if (rr < 54) out[rr * 16 + j] = acc[q][r];
      }
    }
  }
}

// fixed-order sum of partial rows: stage[grp][p] over the rows of group grp
__global__ __launch_bounds__(256) void k_rows_sum(const float* __restrict__ part, uint32_t ld, uint32_t rows,
                                                  uint32_t rows_per_group, double* __restrict__ stage) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= ld) return;
  const uint32_t r0 = blockIdx.y * rows_per_group;
  const uint32_t r1 = min(rows, r0 + rows_per_group);
  double s = 0.0;
  for (uint32_t r = r0; r < r1; ++r) s += (double)part[(uint64_t)r * ld + p];
  stage[(uint64_t)blockIdx.y * ld + p] = s;
}

__global__ __launch_bounds__(256) void k_groups_sum(const double* __restrict__ stage, uint32_t ld, uint32_t groups,
                                                    float* __restrict__ grad) {
  const uint32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= ld) return;
  double s = 0.0;
  for (uint32_t q = 0; q < groups; ++q) s += stage[(uint64_t)q * ld + p];
  grad[p] = (float)s;
}

// ---------------------------------------------------------------------------
// loss: per sample, e = f - t, A e = h^2 H e = kin (6 e - sum of neighbours) + v2 e,
// L_b = e^T A e / (x . t); loss = mean_b L_b; dL/df_b = 2 A e / (x . t) / B
// ---------------------------------------------------------------------------
constexpr int LOSS_PTS = 1024;   // voxels per work-group

__device__ __forceinline__ float apply_a(const float* __restrict__ f, const float* __restrict__ t,
                                         const float* __restrict__ v2, uint32_t v, uint32_t m0, uint32_t m1,
                                         uint32_t m2, float kin) {
  const Vox p = vox_of(v, m0, m1);
  const float e = f[v] - t[v];
  float nb = 0.f;
  const uint32_t s1 = m0, s2 = m0 * m1;
  if (p.x > 0) nb += f[v - 1] - t[v - 1];
  if (p.x + 1 < (int)m0) nb += f[v + 1] - t[v + 1];
  if (p.y > 0) nb += f[v - s1] - t[v - s1];
  if (p.y + 1 < (int)m1) nb += f[v + s1] - t[v + s1];
  if (p.z > 0) nb += f[v - s2] - t[v - s2];
  if (p.z + 1 < (int)m2) nb += f[v + s2] - t[v + s2];
  return kin * (6.f * e - nb) + v2[v] * e;
}

__device__ __forceinline__ double wg_sum_d(double x, double* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_loss_part(const float* __restrict__ F, const float* __restrict__ T,
                                                   const float* __restrict__ X, const float* __restrict__ v2,
                                                   uint32_t m0, uint32_t m1, uint32_t m2, float kin,
                                                   double* __restrict__ part) {
  __shared__ double sh[256];
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint32_t b = blockIdx.y;
  const float* f = F + b * n;
  const float* t = T + b * n;
  const float* x = X + b * n;
  double num = 0.0, den = 0.0;
  const uint32_t p0 = blockIdx.x * LOSS_PTS;
  for (uint32_t q = threadIdx.x; q < LOSS_PTS; q += 256) {
    const uint32_t v = p0 + q;
    if (v >= n) break;
    const float ae = apply_a(f, t, v2, v, m0, m1, m2, kin);
    num += (double)(f[v] - t[v]) * (double)ae;
    den += (double)x[v] * (double)t[v];
  }
  num = wg_sum_d(num, sh);
  den = wg_sum_d(den, sh);
  if (threadIdx.x == 0) {
    part[((uint64_t)b * gridDim.x + blockIdx.x) * 2 + 0] = num;
    part[((uint64_t)b * gridDim.x + blockIdx.x) * 2 + 1] = den;
  }
}

// one work-group: per-sample sums, gradient coefficients and the batch loss
__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, uint32_t chunks, uint32_t B,
                                                    double* __restrict__ coef, double* __restrict__ loss) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (uint32_t b = 0; b < B; ++b) {
    double num = 0.0, den = 0.0;
    for (uint32_t c = threadIdx.x; c < chunks; c += 256) {
      num += part[((uint64_t)b * chunks + c) * 2 + 0];
      den += part[((uint64_t)b * chunks + c) * 2 + 1];
    }
    num = wg_sum_d(num, sh);
    den = wg_sum_d(den, sh);
    if (threadIdx.x == 0) {
      coef[b] = 2.0 / (den * (double)B);
      acc += num / den;
    }
  }
  if (threadIdx.x == 0) loss[0] = acc / (double)B;
}

__global__ __launch_bounds__(256) void k_loss_grad(const float* __restrict__ F, const float* __restrict__ T,
                                                   const float* __restrict__ v2, uint32_t m0, uint32_t m1,
                                                   uint32_t m2, float kin, const double* __restrict__ coef,
                                                   uint16_t* __restrict__ g) {
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint32_t b = blockIdx.y;
  const uint32_t v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  const float ae = apply_a(F + b * n, T + b * n, v2, v, m0, m1, m2, kin);
  g[b * n + v] = to_bf16((float)(coef[b] * (double)ae));
}

// residual-norm loss: e = A f - x, L_b = |e|^2 / |x|^2, dL/df_b = 2 A e / |x|^2 / B
__device__ __forceinline__ float apply_a1(const float* __restrict__ f, const float* __restrict__ v2, uint32_t v,
                                          uint32_t m0, uint32_t m1, uint32_t m2, float kin) {
  const Vox p = vox_of(v, m0, m1);
  float nb = 0.f;
  const uint32_t s1 = m0, s2 = m0 * m1;
  if (p.x > 0) nb += f[v - 1];
  if (p.x + 1 < (int)m0) nb += f[v + 1];
  if (p.y > 0) nb += f[v - s1];
  if (p.y + 1 < (int)m1) nb += f[v + s1];
  if (p.z > 0) nb += f[v - s2];
  if (p.z + 1 < (int)m2) nb += f[v + s2];
  return kin * (6.f * f[v] - nb) + v2[v] * f[v];
}

__global__ __launch_bounds__(256) void k_rloss_part(const float* __restrict__ F, const float* __restrict__ X,
                                                    const float* __restrict__ v2, uint32_t m0, uint32_t m1,
                                                    uint32_t m2, float kin, float* __restrict__ E,
                                                    double* __restrict__ part) {
  __shared__ double sh[256];
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint32_t b = blockIdx.y;
  const float* f = F + b * n;
  const float* x = X + b * n;
  double ee = 0.0, xx = 0.0;
  const uint32_t p0 = blockIdx.x * LOSS_PTS;
  for (uint32_t q = threadIdx.x; q < LOSS_PTS; q += 256) {
    const uint32_t v = p0 + q;
    if (v >= n) break;
    const float e = apply_a1(f, v2, v, m0, m1, m2, kin) - x[v];
    E[b * n + v] = e;
    ee += (double)e * (double)e;
    xx += (double)x[v] * (double)x[v];
  }
  ee = wg_sum_d(ee, sh);
  xx = wg_sum_d(xx, sh);
  if (threadIdx.x == 0) {
    part[((uint64_t)b * gridDim.x + blockIdx.x) * 2 + 0] = ee;
    part[((uint64_t)b * gridDim.x + blockIdx.x) * 2 + 1] = xx;
  }
}

// energy + residual losses: g = coefE A (f - t) + coefR A e
__global__ __launch_bounds__(256) void k_bloss_grad(const float* __restrict__ F, const float* __restrict__ T,
                                                    const float* __restrict__ E, const float* __restrict__ v2,
                                                    uint32_t m0, uint32_t m1, uint32_t m2, float kin,
                                                    const double* __restrict__ coefE, const double* __restrict__ coefR,
                                                    uint16_t* __restrict__ g) {
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint32_t b = blockIdx.y;
  const uint32_t v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  const float a1 = apply_a(F + b * n, T + b * n, v2, v, m0, m1, m2, kin);
  const float a2 = apply_a1(E + b * n, v2, v, m0, m1, m2, kin);
  g[b * n + v] = to_bf16((float)(coefE[b] * (double)a1 + coefR[b] * (double)a2));
}

__global__ __launch_bounds__(256) void k_rloss_grad(const float* __restrict__ E, const float* __restrict__ v2,
                                                    uint32_t m0, uint32_t m1, uint32_t m2, float kin,
                                                    const double* __restrict__ coef, uint16_t* __restrict__ g) {
  const uint64_t n = (uint64_t)m0 * m1 * m2;
  const uint32_t b = blockIdx.y;
  const uint32_t v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  const float ae = apply_a1(E + b * n, v2, v, m0, m1, m2, kin);
  g[b * n + v] = to_bf16((float)(coef[b] * (double)ae));
}

// ---------------------------------------------------------------------------
// input / output packing
// ---------------------------------------------------------------------------
// x[b][v] = (bf16 X[b][v], bf16 v2[v]) from column-major FP32 samples
__global__ __launch_bounds__(256) void k_pack_x(const float* __restrict__ X, const float* __restrict__ v2,
                                                uint64_t n, uint32_t B, uint32_t* __restrict__ x) {
  const uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n * B) return;
  const uint64_t v = q % n;
  x[q] = (uint32_t)to_bf16(X[q]) | ((uint32_t)to_bf16(v2[v]) << 16);
}

constexpr int TP = 64;           // grid points per transpose tile

// Point-major FP64 rows (n x ld, columns 0..B-1) to column-major values:
//   MODE 0: x[b][v] = (bf16 R[v][b] * scale_b, bf16 v2[v])     (network input)
//   MODE 1: out[b][v] = FP32 R[v][b] * scale_b                  (training samples)
// scale_b = mult / sqrt(colsq[b]), 0 for a zero column.  B <= 128.
template <int MODE>
__global__ __launch_bounds__(256) void k_rows_to_cols(const double* __restrict__ R, uint32_t ld, uint32_t B,
                                                      uint64_t n, const double* __restrict__ colsq, double mult,
                                                      const float* __restrict__ v2, void* __restrict__ out) {
  __shared__ float tl[TP][129];
  __shared__ float sc[128];
  const uint64_t p0 = (uint64_t)blockIdx.x * TP;
  if (threadIdx.x < B) {
    const double c2 = colsq[threadIdx.x];
    sc[threadIdx.x] = c2 > 0.0 ? (float)(mult / sqrt(c2)) : 0.f;
  }
  __syncthreads();
  const uint32_t tot = TP * B;
  for (uint32_t q = threadIdx.x; q < tot; q += 256) {
    const uint32_t p = q / B, c = q - p * B;
    tl[p][c] = p0 + p < n ? (float)R[(p0 + p) * ld + c] * sc[c] : 0.f;
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < tot; q += 256) {
    const uint32_t c = q / TP, p = q - c * TP;
    const uint64_t v = p0 + p;
    if (v >= n) continue;
    if constexpr (MODE == 0) {
      reinterpret_cast<uint32_t*>(out)[c * n + v] = (uint32_t)to_bf16(tl[p][c]) | ((uint32_t)to_bf16(v2[v]) << 16);
    } else {
      reinterpret_cast<float*>(out)[c * n + v] = tl[p][c];
    }
  }
}

// E[v][b] = U[v][b] - sqrt(colsq[b]) * hh * f[b][v]  (point-major FP64, B <= 128)
__global__ __launch_bounds__(256) void k_cols_to_rows(const float* __restrict__ f, const double* __restrict__ U,
                                                      uint32_t ld, uint32_t B, uint64_t n,
                                                      const double* __restrict__ colsq, double hh,
                                                      double* __restrict__ E) {
  __shared__ float tl[TP][129];
  __shared__ double sc[128];
  const uint64_t p0 = (uint64_t)blockIdx.x * TP;
  if (threadIdx.x < B) {
    const double c2 = colsq[threadIdx.x];
    sc[threadIdx.x] = c2 > 0.0 ? sqrt(c2) * hh : 0.0;
  }
  const uint32_t tot = TP * B;
  for (uint32_t q = threadIdx.x; q < tot; q += 256) {
    const uint32_t c = q / TP, p = q - c * TP;
    tl[p][c] = p0 + p < n ? f[c * n + p0 + p] : 0.f;
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < tot; q += 256) {
    const uint32_t p = q / B, c = q - p * B;
    const uint64_t v = p0 + p;
    if (v >= n) continue;
    E[v * ld + c] = U[v * ld + c] - sc[c] * (double)tl[p][c];
  }
}

// per-column sums of squares of point-major FP64 rows: part[w][c], one thread per column (B <= 256)
__global__ __launch_bounds__(256) void k_colsq(const double* __restrict__ R, uint32_t ld, uint32_t B, uint64_t n,
                                               uint64_t pts, double* __restrict__ part) {
  const uint32_t c = threadIdx.x;
  if (c >= B) return;
  const uint64_t p0 = (uint64_t)blockIdx.x * pts;
  const uint64_t p1 = min(n, p0 + pts);
  double s = 0.0;
  for (uint64_t p = p0; p < p1; ++p) {
    const double r = R[p * ld + c];
    s += r * r;
  }
  part[(uint64_t)blockIdx.x * B + c] = s;
}

// v2 = h^2 (V + shift) = hh * (diag - dsum)
__global__ __launch_bounds__(256) void k_make_v2(const double* __restrict__ diag, uint64_t n, double dsum, double hh,
                                                 float* __restrict__ v2) {
  const uint64_t v = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (v < n) v2[v] = (float)(hh * (diag[v] - dsum));
}

// ---------------------------------------------------------------------------
// weights: BF16 operand packing and Adam
// ---------------------------------------------------------------------------
__device__ float packed_value(const float* __restrict__ w, int q) {
  // forward layer: row co, k = tap * CIN + ci -> W[tap][ci][co]
  // transposed layer: row ci, k = tap' * COUT + co -> W[26 - tap'][ci][co]
  int off, ks, cin, cout, wo;
  bool tr;
  if (q < PK_F2) { off = PK_F1; ks = KS2; cin = 2; cout = 16; wo = W1_OFF; tr = false; }
  else if (q < PK_F3) { off = PK_F2; ks = KSZ; cin = 16; cout = 16; wo = W2_OFF; tr = false; }
  else if (q < PK_F4) { off = PK_F3; ks = KSZ; cin = 16; cout = 16; wo = W3_OFF; tr = false; }
  else if (q < PK_B4) { off = PK_F4; ks = KS16; cin = 16; cout = 1; wo = W4_OFF; tr = false; }
  else if (q < PK_B3) { off = PK_B4; ks = KS1; cin = 16; cout = 1; wo = W4_OFF; tr = true; }
  else if (q < PK_B2) { off = PK_B3; ks = KSZ; cin = 16; cout = 16; wo = W3_OFF; tr = true; }
  else { off = PK_B2; ks = KSZ; cin = 16; cout = 16; wo = W2_OFF; tr = true; }
  int r = (q - off) / (32 * ks), k = (q - off) % (32 * ks);
  if (ks == KSZ) {
    // 16 -> 16 layers: k-step s = 2 (3 dz + dy) + pair covers taps (dz, dy,
    // dx = 2 pair + half) for half 0, 1 (dx = 3 is zero), 16 channels each;
    // rewritten to the tap-major index k = 16 tap + channel used below
    const int st = k / 32, kk = k % 32;
    const int g = st / 2, dx = 2 * (st % 2) + kk / 16;
    if (dx > 2) return 0.f;
    k = 16 * (3 * g + dx) + kk % 16;
  }
  if (!tr) {
    const int tap = k / cin, ci = k % cin;
    if (r >= cout || tap >= 27) return 0.f;
    return w[wo + (tap * cin + ci) * cout + r];
  }
  const int tap = k / cout, co = k % cout;
  if (r >= cin || tap >= 27) return 0.f;
  return w[wo + ((26 - tap) * cin + r) * cout + co];
}

__global__ __launch_bounds__(256) void k_pack_w(const float* __restrict__ w, uint16_t* __restrict__ pk) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < PK_TOTAL) pk[q] = to_bf16(packed_value(w, q));
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int count, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= count) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  w[q] -= lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#define HIPCHK(x)                               \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return OPE_EHIP;      \
  } while (0)

namespace {

constexpr int WGRAD_ROWS = 2048;      // partial rows of the weight gradients (about 2 waves per SIMD)
constexpr int WGRAD_GROUPS = 32;      // first-stage groups of their fixed-order reduction

void free_net(ope_net* t) {
  if (!t) return;
  void* ptrs[] = {t->w, t->adam_m, t->adam_v, t->grad, t->wpk, t->v2, t->x, t->a1, t->a2, t->a3, t->g3, t->g4,
                  t->f, t->e, t->part, t->stage, t->lpart, t->coef, t->dloss, t->colsq};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (t->hloss) (void)hipHostFree(t->hloss);
  delete t;
}

template <int CIN, int COUT, int EPI>
hipError_t conv(ope_net* t, const uint16_t* in, int pk_off, const uint16_t* mask, void* out, uint32_t B) {
  if constexpr (CIN == 16 && COUT == 16) {
    const uint32_t ntx = (t->m0 + OX - 1) / OX, nty = (t->m1 + OY - 1) / OY, ntz = (t->m2 + OZ - 1) / OZ;
    const uint64_t blocks = (uint64_t)ntx * nty * ntz * B;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_conv16z<EPI>), dim3((uint32_t)blocks), dim3(256), 0, t->ctx->stream, in, t->wpk + pk_off,
                       mask, (uint16_t*)out, t->m0, t->m1, t->m2, ntx, nty, ntz);
    return hipGetLastError();
  } else {
    static_assert(CIN == 1, "2- and 16-channel inputs take the z-marched kernels");
    const uint32_t ntx = (t->m0 + TX - 1) / TX, nty = (t->m1 + TY - 1) / TY, ntz = (t->m2 + TZ - 1) / TZ;
    const uint64_t blocks = (uint64_t)ntx * nty * ntz * B;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_conv<CIN, COUT, EPI>), dim3((uint32_t)blocks), dim3(256), 0, t->ctx->stream, in,
                       t->wpk + pk_off, mask, out, t->m0, t->m1, t->m2, ntx, nty, ntz);
    return hipGetLastError();
  }
}

// layer 1..4 forward from the packed input pair in t->x; output f (FP32 [b][v])
hipError_t forward(ope_net* t, uint32_t B, float* f) {
  hipError_t e;
  {
    const uint32_t ntx = (t->m0 + OX - 1) / OX, nty = (t->m1 + OY - 1) / OY, ntz = (t->m2 + OZ - 1) / OZ;
    const uint64_t blocks = (uint64_t)ntx * nty * ntz * B;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    if (blocks > 0) {
      hipLaunchKernelGGL(k_conv2z, dim3((uint32_t)blocks), dim3(256), 0, t->ctx->stream, (const uint32_t*)t->x,
                         t->wpk + PK_F1, (uint16_t*)t->a1, t->m0, t->m1, t->m2, ntx, nty, ntz);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if ((e = conv<16, 16, EPI_RELU>(t, t->a1, PK_F2, nullptr, t->a2, B)) != hipSuccess) return e;
  if ((e = conv<16, 16, EPI_RELU>(t, t->a2, PK_F3, nullptr, t->a3, B)) != hipSuccess) return e;
  const uint32_t ntx = (t->m0 + OX - 1) / OX, nty = (t->m1 + OY - 1) / OY, ntz = (t->m2 + OZ - 1) / OZ;
  const uint64_t blocks = (uint64_t)ntx * nty * ntz * B;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_conv_out1, dim3((uint32_t)blocks), dim3(256), 0, t->ctx->stream, t->a3, t->wpk + PK_F4, f, t->m0,
                     t->m1, t->m2, ntx, nty, ntz);
  return hipGetLastError();
}

hipError_t pack_x(ope_net* t, const float* X, const float* v2, uint32_t B) {
  const uint64_t tot = (uint64_t)t->n * B;
  hipLaunchKernelGGL(k_pack_x, dim3((uint32_t)((tot + 255) / 256)), dim3(256), 0, t->ctx->stream, X, v2,
                     (uint64_t)t->n, B, (uint32_t*)t->x);
  return hipGetLastError();
}

template <int MODE>
hipError_t wgrad(ope_net* t, const uint16_t* a, const uint16_t* g, uint32_t off, uint32_t B, uint32_t rps,
                 uint32_t vpr) {
  const uint32_t rows = B * rps;
  hipLaunchKernelGGL(k_wgrad<MODE>, dim3((rows + 3) / 4), dim3(256), 0, t->ctx->stream, a, g, t->part,
                     (uint32_t)OPE_NET_PARAMS, off, rows, rps, vpr, t->m0, t->m1, t->m2);
  return hipGetLastError();
}

// forward + loss + backward: t->grad and t->dloss
ope_status grad_pass(ope_net* t, const float* X, const float* v2, const float* T, uint32_t B) {
  hipStream_t s = t->ctx->stream;
  const uint64_t n = t->n;
  HIPCHK(pack_x(t, X, v2, B));
  HIPCHK(forward(t, B, t->f));
  // loss and dL/df
  const uint32_t chunks = (uint32_t)((n + LOSS_PTS - 1) / LOSS_PTS);
  const int kind = t->loss_kind;
  const dim3 pgrid((uint32_t)((n + 255) / 256), B);
  double* lossE = t->dloss;
  double* lossR = kind == OPE_NET_LOSS_RESIDUAL ? t->dloss : t->dloss + 1;
  // per sample: coef = 2 / (den B), loss = mean(num / den); den = x . t (energy) or |x|^2 (residual)
  if (kind != OPE_NET_LOSS_RESIDUAL) {
    hipLaunchKernelGGL(k_loss_part, dim3(chunks, B), dim3(256), 0, s, t->f, T, X, v2, t->m0, t->m1, t->m2,
                       (float)t->kin, t->lpart);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, t->lpart, chunks, B, t->coef, lossE);
    HIPCHK(hipGetLastError());
  }
  if (kind != OPE_NET_LOSS_ENERGY) {
    hipLaunchKernelGGL(k_rloss_part, dim3(chunks, B), dim3(256), 0, s, t->f, X, v2, t->m0, t->m1, t->m2,
                       (float)t->kin, t->e, t->lpart);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, t->lpart, chunks, B, t->coef + t->max_batch, lossR);
    HIPCHK(hipGetLastError());
  }
  if (kind == OPE_NET_LOSS_ENERGY) {
    hipLaunchKernelGGL(k_loss_grad, pgrid, dim3(256), 0, s, t->f, T, v2, t->m0, t->m1, t->m2, (float)t->kin, t->coef,
                       t->g4);
  } else if (kind == OPE_NET_LOSS_RESIDUAL) {
    hipLaunchKernelGGL(k_rloss_grad, pgrid, dim3(256), 0, s, t->e, v2, t->m0, t->m1, t->m2, (float)t->kin,
                       t->coef + t->max_batch, t->g4);
  } else {
    hipLaunchKernelGGL(k_bloss_grad, pgrid, dim3(256), 0, s, t->f, T, t->e, v2, t->m0, t->m1, t->m2, (float)t->kin,
                       t->coef, t->coef + t->max_batch, t->g4);
  }
  HIPCHK(hipGetLastError());
  // voxel ranges of the weight-gradient partials
  uint32_t rps = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((int64_t)((n + 1023) / 1024), WGRAD_ROWS / B));
  uint32_t vpr = (uint32_t)((n + rps - 1) / rps);
  vpr = (vpr + 3) & ~3u;
  rps = (uint32_t)((n + vpr - 1) / vpr);
  const uint32_t rows = B * rps;
  // layer 4: g3 = conv^T(g4) masked by a3 > 0; dW4 from (a3, g4)
  HIPCHK((conv<1, 16, EPI_MASK>(t, t->g4, PK_B4, t->a3, t->g3, B)));
  HIPCHK(wgrad<WGR_W4>(t, t->a3, t->g4, W4_OFF, B, rps, vpr));
  // layer 3: dW3 from (a2, g3); g2 (into a3) = conv^T(g3) masked by a2
  HIPCHK(wgrad<WGR_16>(t, t->a2, t->g3, W3_OFF, B, rps, vpr));
  HIPCHK((conv<16, 16, EPI_MASK>(t, t->g3, PK_B3, t->a2, t->a3, B)));
  // layer 2: dW2 from (a1, g2); g1 (into g3) = conv^T(g2) masked by a1
  HIPCHK(wgrad<WGR_16>(t, t->a1, t->a3, W2_OFF, B, rps, vpr));
  HIPCHK((conv<16, 16, EPI_MASK>(t, t->a3, PK_B2, t->a1, t->g3, B)));
  // layer 1: dW1 from (x, g1)
  HIPCHK(wgrad<WGR_W1>(t, t->x, t->g3, W1_OFF, B, rps, vpr));
  // fixed-order reduction of the partial rows
  const uint32_t rpg = (rows + WGRAD_GROUPS - 1) / WGRAD_GROUPS;
  const uint32_t groups = (rows + rpg - 1) / rpg;
  hipLaunchKernelGGL(k_rows_sum, dim3((OPE_NET_PARAMS + 255) / 256, groups), dim3(256), 0, s, t->part,
                     (uint32_t)OPE_NET_PARAMS, rows, rpg, t->stage);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_groups_sum, dim3((OPE_NET_PARAMS + 255) / 256), dim3(256), 0, s, t->stage,
                     (uint32_t)OPE_NET_PARAMS, groups, t->grad);
  HIPCHK(hipGetLastError());
  return OPE_OK;
}

hipError_t pack_weights(ope_net* t) {
  hipLaunchKernelGGL(k_pack_w, dim3((PK_TOTAL + 255) / 256), dim3(256), 0, t->ctx->stream, t->w, t->wpk);
  return hipGetLastError();
}

// One Adam step (Kingma & Ba 2015, Algorithm 1: beta1 0.9, beta2 0.999,
// eps 1e-8, bias-corrected moments) on the FP32 masters from t->grad, then the
// BF16 operand copies.
hipError_t adam_update(ope_net* t, double lr) {
  t->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - std::pow(b1, (float)t->adam_t), bc2 = 1.f - std::pow(b2, (float)t->adam_t);
  hipLaunchKernelGGL(k_adam, dim3((OPE_NET_PARAMS + 255) / 256), dim3(256), 0, t->ctx->stream, t->w, t->adam_m,
                     t->adam_v, t->grad, (int)OPE_NET_PARAMS, (float)lr, b1, b2, 1e-8f, bc1, bc2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return pack_weights(t);
}

ope_status read_loss(ope_net* t, double* loss) {
  HIPCHK(hipMemcpyAsync(t->hloss, t->dloss, 2 * sizeof(double), hipMemcpyDeviceToHost, t->ctx->stream));
  HIPCHK(hipStreamSynchronize(t->ctx->stream));
  const double l = t->loss_kind == OPE_NET_LOSS_BOTH ? t->hloss[0] + t->hloss[1] : t->hloss[0];
  if (loss) *loss = l;
  return std::isfinite(l) ? OPE_OK : OPE_ENONFINITE;
}

ope_status check_batch(const ope_net* t, int64_t B) {
  if (B < 1 || B > t->max_batch) return OPE_EINVAL;
  return OPE_OK;
}

}  // namespace

// column sums of squares of point-major rows (B <= 256), reduced in a fixed order into out[B]
hipError_t launch_colsq(ope_ctx* c, const double* R, int64_t ld, int64_t B, double* out) {
  const int64_t pts = (c->n + 1023) / 1024;
  const int64_t wgs = (c->n + pts - 1) / pts;
  if (wgs * B > c->part_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_colsq, dim3((uint32_t)wgs), dim3(256), 0, c->stream, R, (uint32_t)ld, (uint32_t)B,
                     (uint64_t)c->n, (uint64_t)pts, c->part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_cols(c, c->part, wgs, B, out, RED_PLAIN);
}

// E = U - P(R) for the context's N columns: R point-major FP64 with column
// sums of squares colsq; P(r) = |r| h^2 f(r / |r|, h^2 (V + shift)).
hipError_t net_apply_residual(ope_net* t, const double* R, const double* colsq, const double* U, double* E) {
  ope_ctx* c = t->ctx;
  const uint32_t B = (uint32_t)c->N;
  const uint32_t tiles = (uint32_t)((c->n + TP - 1) / TP);
  hipLaunchKernelGGL(k_rows_to_cols<0>, dim3(tiles), dim3(256), 0, c->stream, R, B, B, (uint64_t)c->n, colsq, 1.0,
                     t->v2, (void*)t->x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = forward(t, B, t->f)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cols_to_rows, dim3(tiles), dim3(256), 0, c->stream, t->f, U, B, B, (uint64_t)c->n, colsq,
                     t->hh, E);
  return hipGetLastError();
}

extern "C" {

ope_status ope_net_create(ope_ctx* ctx, int64_t max_batch, ope_net** out) {
  if (!out) return OPE_EINVAL;
  *out = nullptr;
  if (!ctx || max_batch < 1 || max_batch > 4096) return OPE_EINVAL;
  if (ctx->g.dim != 3) return OPE_EUNSUPPORTED;
  const double h = ctx->h[0];
  if (std::fabs(ctx->h[1] - h) > 1e-12 * h || std::fabs(ctx->h[2] - h) > 1e-12 * h) return OPE_EUNSUPPORTED;
  ope_net* t = new (std::nothrow) ope_net();
  if (!t) return OPE_ENOMEM;
  t->ctx = ctx;
  t->max_batch = max_batch;
  t->n = ctx->n;
  t->m0 = ctx->g.m0;
  t->m1 = ctx->g.m1;
  t->m2 = ctx->g.m2;
  t->hh = h * h;
  t->kin = ctx->kinetic;
  t->adam_t = 0;
  t->loss_kind = OPE_NET_LOSS_ENERGY;
  const uint64_t nb = (uint64_t)t->n * (uint64_t)max_batch;
  const uint64_t chunks = (t->n + LOSS_PTS - 1) / LOSS_PTS;
  bool ok = true;
  auto al = [&](void** p, size_t bytes) { ok &= hipMalloc(p, bytes ? bytes : 1) == hipSuccess; };
  al((void**)&t->w, sizeof(float) * OPE_NET_PARAMS);
  al((void**)&t->adam_m, sizeof(float) * OPE_NET_PARAMS);
  al((void**)&t->adam_v, sizeof(float) * OPE_NET_PARAMS);
  al((void**)&t->grad, sizeof(float) * OPE_NET_PARAMS);
  al((void**)&t->wpk, sizeof(uint16_t) * PK_TOTAL);
  al((void**)&t->v2, sizeof(float) * t->n);
  al((void**)&t->x, sizeof(uint16_t) * 2 * nb);
  al((void**)&t->a1, sizeof(uint16_t) * 16 * nb);
  al((void**)&t->a2, sizeof(uint16_t) * 16 * nb);
  al((void**)&t->a3, sizeof(uint16_t) * 16 * nb);
  al((void**)&t->g3, sizeof(uint16_t) * 16 * nb);
  al((void**)&t->g4, sizeof(uint16_t) * nb);
  al((void**)&t->f, sizeof(float) * nb);
  al((void**)&t->e, sizeof(float) * nb);
  al((void**)&t->part, sizeof(float) * (size_t)std::max<int64_t>(WGRAD_ROWS, max_batch) * OPE_NET_PARAMS);
  al((void**)&t->stage, sizeof(double) * (size_t)WGRAD_GROUPS * OPE_NET_PARAMS);
  al((void**)&t->lpart, sizeof(double) * 2 * chunks * (uint64_t)max_batch);
  al((void**)&t->coef, sizeof(double) * 2 * (size_t)max_batch);
  al((void**)&t->dloss, sizeof(double) * 2);
  al((void**)&t->colsq, sizeof(double) * 256);
  ok &= hipHostMalloc((void**)&t->hloss, 2 * sizeof(double), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    free_net(t);
    return OPE_ENOMEM;
  }
  hipStream_t s = ctx->stream;
  bool hok = true;
  hok &= hipMemsetAsync(t->w, 0, sizeof(float) * OPE_NET_PARAMS, s) == hipSuccess;
  hok &= hipMemsetAsync(t->adam_m, 0, sizeof(float) * OPE_NET_PARAMS, s) == hipSuccess;
  hok &= hipMemsetAsync(t->adam_v, 0, sizeof(float) * OPE_NET_PARAMS, s) == hipSuccess;
  const double dsum = 2.0 * (ctx->g.cx + ctx->g.cy + ctx->g.cz);
  hipLaunchKernelGGL(k_make_v2, dim3((uint32_t)((t->n + 255) / 256)), dim3(256), 0, s, ctx->diag, (uint64_t)t->n,
                     dsum, t->hh, t->v2);
  hok &= hipGetLastError() == hipSuccess;
  hok &= pack_weights(t) == hipSuccess;
  hok &= hipStreamSynchronize(s) == hipSuccess;
  if (!hok) {
    free_net(t);
    return OPE_EHIP;
  }
  *out = t;
  return OPE_OK;
}

ope_status ope_net_destroy(ope_net* t) {
  if (!t) return OPE_OK;
  if (t->ctx->net == t) t->ctx->net = nullptr;
  (void)hipStreamSynchronize(t->ctx->stream);
  free_net(t);
  return OPE_OK;
}

ope_status ope_net_set_weights(ope_net* t, const float* w) {
  if (!t || !w) return OPE_EINVAL;
  hipStream_t s = t->ctx->stream;
  HIPCHK(hipMemcpyAsync(t->w, w, sizeof(float) * OPE_NET_PARAMS, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(t->adam_m, 0, sizeof(float) * OPE_NET_PARAMS, s));
  HIPCHK(hipMemsetAsync(t->adam_v, 0, sizeof(float) * OPE_NET_PARAMS, s));
  t->adam_t = 0;
  HIPCHK(pack_weights(t));
  HIPCHK(hipStreamSynchronize(s));
  return OPE_OK;
}

ope_status ope_net_get_weights(ope_net* t, float* w) {
  if (!t || !w) return OPE_EINVAL;
  HIPCHK(hipMemcpyAsync(w, t->w, sizeof(float) * OPE_NET_PARAMS, hipMemcpyDeviceToHost, t->ctx->stream));
  HIPCHK(hipStreamSynchronize(t->ctx->stream));
  return OPE_OK;
}

ope_status ope_net_forward(ope_net* t, const float* X, const float* V2, int64_t B, float* F) {
  if (!t || !X || !F) return OPE_EINVAL;
  ope_status st = check_batch(t, B);
  if (st != OPE_OK) return st;
  HIPCHK(pack_x(t, X, V2 ? V2 : t->v2, (uint32_t)B));
  HIPCHK(forward(t, (uint32_t)B, F));
  return OPE_OK;
}

ope_status ope_net_grad(ope_net* t, const float* X, const float* V2, const float* T, int64_t B, double* loss,
                        float* grad) {
  if (!t || !X || (!T && t->loss_kind != OPE_NET_LOSS_RESIDUAL)) return OPE_EINVAL;
  ope_status st = check_batch(t, B);
  if (st != OPE_OK) return st;
  st = grad_pass(t, X, V2 ? V2 : t->v2, T, (uint32_t)B);
  if (st != OPE_OK) return st;
  if (grad) HIPCHK(hipMemcpyAsync(grad, t->grad, sizeof(float) * OPE_NET_PARAMS, hipMemcpyDeviceToHost,
                                  t->ctx->stream));
  return read_loss(t, loss);
}

ope_status ope_net_train_step(ope_net* t, const float* X, const float* V2, const float* T, int64_t B, double lr,
                              double* loss) {
  if (!t || !X || (!T && t->loss_kind != OPE_NET_LOSS_RESIDUAL) || !(lr > 0.0)) return OPE_EINVAL;
  ope_status st = check_batch(t, B);
  if (st != OPE_OK) return st;
  st = grad_pass(t, X, V2 ? V2 : t->v2, T, (uint32_t)B);
  if (st != OPE_OK) return st;
  HIPCHK(adam_update(t, lr));
  return read_loss(t, loss);
}

ope_status ope_net_apply_grad(ope_net* t, const float* grad, double lr) {
  if (!t || !grad || !(lr > 0.0)) return OPE_EINVAL;
  HIPCHK(hipMemcpyAsync(t->grad, grad, sizeof(float) * OPE_NET_PARAMS, hipMemcpyHostToDevice, t->ctx->stream));
  HIPCHK(adam_update(t, lr));
  HIPCHK(hipStreamSynchronize(t->ctx->stream));
  return OPE_OK;
}

ope_status ope_net_samples(ope_net* t, const double* R, const double* S, int64_t ld, int64_t B, float* X,
                           float* T) {
  if (!t || !R || !S || !X || !T) return OPE_EINVAL;
  ope_ctx* c = t->ctx;
  if (B < 1 || B > 128 || B > c->N || ld < B) return OPE_EINVAL;
  HIPCHK(launch_colsq(c, R, ld, B, t->colsq));
  const uint32_t tiles = (uint32_t)((c->n + TP - 1) / TP);
  hipLaunchKernelGGL(k_rows_to_cols<1>, dim3(tiles), dim3(256), 0, c->stream, R, (uint32_t)ld, (uint32_t)B,
                     (uint64_t)c->n, t->colsq, 1.0, t->v2, (void*)X);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_rows_to_cols<1>, dim3(tiles), dim3(256), 0, c->stream, S, (uint32_t)ld, (uint32_t)B,
                     (uint64_t)c->n, t->colsq, 1.0 / t->hh, t->v2, (void*)T);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return OPE_OK;
}

ope_status ope_net_set_loss(ope_net* t, int32_t kind) {
  if (!t || kind < OPE_NET_LOSS_ENERGY || kind > OPE_NET_LOSS_BOTH) return OPE_EINVAL;
  t->loss_kind = kind;
  return OPE_OK;
}

ope_status ope_net_potential(ope_net* t, float* V2) {
  if (!t || !V2) return OPE_EINVAL;
  HIPCHK(hipMemcpyAsync(V2, t->v2, sizeof(float) * t->n, hipMemcpyDeviceToDevice, t->ctx->stream));
  HIPCHK(hipStreamSynchronize(t->ctx->stream));
  return OPE_OK;
}

}  // extern "C"
