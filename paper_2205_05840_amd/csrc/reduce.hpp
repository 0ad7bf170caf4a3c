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

}  // namespace ndmg
