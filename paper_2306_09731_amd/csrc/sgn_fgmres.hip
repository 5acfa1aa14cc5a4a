// Vector kernels of the flexible GMRES solve with a learned preconditioner
// (FP64 fields in physical space): block partials of several inner products,
// and linear combinations of basis fields.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sgn_launch.hpp"

namespace sgn {
namespace {

constexpr int kThreads = 256;

// partials[blk * nv + k] = sum over the block's points i of V_k[i] w[i],
// k < nv <= kFgMaxVecs, grid-stride over the n points.
__global__ void __launch_bounds__(kThreads) k_fg_dots(const double* __restrict__ V, size_t vstride, int nv,
                                                     const double* __restrict__ w, size_t n,
                                                     double* __restrict__ partials) {
  __shared__ double red[kFgMaxVecs][kThreads / 64];
  double acc[kFgMaxVecs];
#pragma unroll
  for (int k = 0; k < kFgMaxVecs; ++k) acc[k] = 0.0;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < kFgMaxVecs; ++k)
      if (k < nv) acc[k] += V[(size_t)k * vstride + i] * wi;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kFgMaxVecs; ++k) {
    if (k >= nv) break;
    double v = acc[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[k][wave] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    const int k = threadIdx.x;
    partials[(size_t)blockIdx.x * nv + k] = (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
  }
}

// out[i] = a y[i] + bx x[i] + sum_k c_k V_k[i] (y, x may be null; out may be y).
__global__ void __launch_bounds__(kThreads) k_fg_combine(double* out, const double* y, double a, const double* x,
                                                        double bx, const double* __restrict__ V, size_t vstride,
                                                        int nv, FgCoefs c, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    double s = y ? a * y[i] : 0.0;
    if (x) s += bx * x[i];
    for (int k = 0; k < nv; ++k) s += c.c[k] * V[(size_t)k * vstride + i];
    out[i] = s;
  }
}

int blocks_for(size_t n) {
  const size_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < (size_t)kFgBlocks ? b : (size_t)kFgBlocks);
}

}  // namespace

int fg_blocks(size_t n) { return blocks_for(n); }

hipError_t launch_fg_dots(const double* V, size_t vstride, int nv, const double* w, size_t n, double* partials,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_fg_dots, dim3(blocks_for(n)), dim3(kThreads), 0, s, V, vstride, nv, w, n, partials);
  return hipGetLastError();
}

hipError_t launch_fg_combine(double* out, const double* y, double a, const double* x, double bx, const double* V,
                             size_t vstride, int nv, const FgCoefs& c, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fg_combine, dim3(blocks_for(n)), dim3(kThreads), 0, s, out, y, a, x, bx, V, vstride, nv, c,
                     n);
  return hipGetLastError();
}

}  // namespace sgn
