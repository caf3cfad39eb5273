// Deterministic FP64 block reductions (wavefront shuffle tree, then LDS).
#pragma once
#include <hip/hip_runtime.h>

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum over the workgroup (blockDim.x a multiple of 64, <= 1024); result valid in thread 0.
__device__ inline double block_sum(double v) {
  __shared__ double ws[16];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) ws[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < nw; ++k) r += ws[k];
  }
  return r;
}
