// Mixed-precision iterative refinement of the elliptic solve: FP64 residuals
// of an FP64 solution, FP32 corrections (conversion and update passes).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sgn_launch.hpp"

namespace sgn {
namespace {

constexpr int kThreads = 256;

// out32[i] = (float) in64[i].
__global__ void __launch_bounds__(kThreads) k_to_f32(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// r[i] = b[i] - r[i] (r holds L sigma on entry), r32[i] = (float) r[i];
// partials[block] = (sum r^2, sum b^2) over the block's points.
__global__ void __launch_bounds__(kThreads) k_refine_resid(const double* __restrict__ b, double* __restrict__ r,
                                                           float* __restrict__ r32, size_t n, double* partials) {
  __shared__ double red[2][kThreads / 64];
  double sr = 0.0, sb = 0.0;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) {
    const double bi = b[i], ri = bi - r[i];
    r[i] = ri;
    r32[i] = (float)ri;
    sr += ri * ri;
    sb += bi * bi;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o, 64);
    sb += __shfl_xor(sb, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = sr;
    red[1][threadIdx.x >> 6] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) {
      a += red[0][w];
      c += red[1][w];
    }
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = c;
  }
}

// sigma[i] += (double) d32[i].
__global__ void __launch_bounds__(kThreads) k_refine_update(double* __restrict__ sigma, const float* __restrict__ d,
                                                            size_t n) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) sigma[i] += (double)d[i];
}

// out[i] = -(a[i] + c[i]) (the divergence from its two derivative terms).
__global__ void __launch_bounds__(kThreads) k_neg_sum(const double* __restrict__ a, const double* __restrict__ c,
                                                      double* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) out[i] = -(a[i] + c[i]);
}

unsigned blocks_for(size_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_to_f32(const double* in, float* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(n)), dim3(kThreads), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_refine_resid(const double* b, double* r, float* r32, size_t n, double* partials, int nblocks,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_refine_resid, dim3(nblocks), dim3(kThreads), 0, s, b, r, r32, n, partials);
  return hipGetLastError();
}

hipError_t launch_neg_sum(const double* a, const double* c, double* out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_neg_sum, dim3(blocks_for(n)), dim3(kThreads), 0, s, a, c, out, n);
  return hipGetLastError();
}

hipError_t launch_refine_update(double* sigma, const float* d, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_update, dim3(blocks_for(n)), dim3(kThreads), 0, s, sigma, d, n);
  return hipGetLastError();
}

}  // namespace sgn
