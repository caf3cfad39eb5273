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

// Compensated accumulation (Neumaier): value s with running error c.
struct Acc2 {
  double s = 0.0, c = 0.0;
  __device__ inline void add(double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v; else c += (v - t) + s;
    s = t;
  }
  __device__ inline void add(const Acc2& o) { add(o.s); c += o.c; }
  __device__ inline double value() const { return s + c; }
};

__device__ inline Acc2 wave_sum2(Acc2 a) {
  for (int o = 32; o > 0; o >>= 1) {
    Acc2 b;
    b.s = __shfl_xor(a.s, o);
    b.c = __shfl_xor(a.c, o);
    a.add(b);
  }
  return a;
}

// Compensated workgroup sum; result valid in thread 0.
__device__ inline double block_sum2(Acc2 a) {
  __shared__ double ws[16], wc[16];
  a = wave_sum2(a);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) { ws[w] = a.s; wc[w] = a.c; }
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    Acc2 t;
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < nw; ++k) { Acc2 u; u.s = ws[k]; u.c = wc[k]; t.add(u); }
    r = t.value();
  }
  return r;
}
