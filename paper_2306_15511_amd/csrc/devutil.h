// Device helpers shared by the vector-style kernels (HIP translation units only).
#pragma once

#include <hip/hip_runtime.h>

namespace crsht {

// fixed-order tree reduction over the block (blockDim.x a power of two, sh of blockDim.x doubles)
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// real-field inner product term of one stored coefficient: weight 1 for m = 0, 2 for m > 0
__device__ __forceinline__ double wdot(int m, double2 a, double2 c) {
  return (m == 0 ? 1.0 : 2.0) * fma(a.x, c.x, a.y * c.y);
}

}  // namespace crsht
