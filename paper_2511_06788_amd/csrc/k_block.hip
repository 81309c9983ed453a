// Whole-block streaming operations of the step outside the sweeps: y += x over
// an n x N FP64 block (the recycled warm start of Step 1 adds its correction
// d to U Lam^{-1}).
#include <algorithm>

#include "ope_internal.h"

namespace {

__global__ __launch_bounds__(OPE_WG) void k_add_block(double2* __restrict__ y, const double2* __restrict__ x,
                                                      uint64_t count2) {
  for (uint64_t e = blockIdx.x * (uint64_t)OPE_WG + threadIdx.x; e < count2; e += (uint64_t)gridDim.x * OPE_WG) {
    double2 a = y[e];
    const double2 b = x[e];
    a.x += b.x;
    a.y += b.y;
    y[e] = a;
  }
}

__global__ __launch_bounds__(1) void k_add_tail(double* __restrict__ y, const double* __restrict__ x) {
  y[0] += x[0];
}

}  // namespace

hipError_t launch_add_block(ope_ctx* c, double* y, const double* x) {
  // 16-byte pairs (the blocks are 256-byte aligned), then an odd last element
  const uint64_t count = (uint64_t)c->n * c->N, count2 = count / 2;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((count2 + OPE_WG - 1) / OPE_WG, 8192);
  if (count2)
    hipLaunchKernelGGL(k_add_block, dim3(grid), dim3(OPE_WG), 0, c->stream, reinterpret_cast<double2*>(y),
                       reinterpret_cast<const double2*>(x), count2);
  if (count & 1) hipLaunchKernelGGL(k_add_tail, dim3(1), dim3(1), 0, c->stream, y + count - 1, x + count - 1);
  return hipGetLastError();
}
