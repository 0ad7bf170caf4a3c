// Block reduction shared by the device kernels (FP64 sums).
#pragma once

#include <hip/hip_runtime.h>

namespace ndmg {

// Sum over the block: wavefront reduction by shuffles, then across the waves (sh holds
// one double per wave).  The result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  }
  __syncthreads();
  return t;
}

// Sum of v over the block, returned to every thread (sh: 17 doubles of LDS).
__device__ __forceinline__ double block_sum_all(double v, double* sh) {
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) sh[16] = t;
  __syncthreads();
  const double r = sh[16];
  __syncthreads();
  return r;
}

// Sum of the n per-block partials part[0 .. n) in a fixed order, returned to every
// thread of the block: every block that reduces the same partials gets the same value.
__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int n, double* sh) {
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) s += part[e];
  return block_sum_all(s, sh);
}

}  // namespace ndmg
